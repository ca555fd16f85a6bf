// dd_fold.hip -- the fold of the alpha = 1/p transform (Section 2, alpha < 1).
//
// With alpha N = N/p the kernel exp(-2 pi i m n / (N/p)) has period N' = N/p
// in n, so X_m = (T/N) sum_{r<N'} x'_r W_{N'}^{m r} with the folded sequence
// x'_r = sum_{k<p} x_{r + k N'}: one plain length-N' transform after this
// kernel.  The p-term sums are accumulated in double precision and rounded
// once to the input's type.
#include <hip/hip_runtime.h>

#include "../../include/dense_dft.h"
#include "dd_fft.hpp"

namespace dd {

namespace {

template <typename E> struct Wide;
template <> struct Wide<float> { using T = double; };
template <> struct Wide<double> { using T = double; };
template <> struct Wide<cx<float>> { using T = cx<double>; };
template <> struct Wide<cx<double>> { using T = cx<double>; };

__device__ __forceinline__ double widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ cx<double> widen(cx<float> v) { return {v.re, v.im}; }
__device__ __forceinline__ cx<double> widen(cx<double> v) { return v; }
__device__ __forceinline__ double acc_add(double a, double b) { return a + b; }
__device__ __forceinline__ cx<double> acc_add(cx<double> a, cx<double> b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ void narrow(double v, float* o) { *o = (float)v; }
__device__ __forceinline__ void narrow(double v, double* o) { *o = v; }
__device__ __forceinline__ void narrow(cx<double> v, cx<float>* o) { *o = {(float)v.re, (float)v.im}; }
__device__ __forceinline__ void narrow(cx<double> v, cx<double>* o) { *o = v; }

// y[b][r] = sum_{k<p} x[b][r + k Np]; consecutive threads take consecutive r,
// so each of the p loads is coalesced.
template <typename E>
__global__ __launch_bounds__(256) void k_fold(const E* __restrict__ x, E* __restrict__ y, int64_t batch, int64_t N,
                                             int64_t Np, int p) {
  const int64_t total = batch * Np;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t b = i / Np, r = i - b * Np;
    const E* src = x + b * N + r;
    typename Wide<E>::T s = widen(src[0]);
    for (int k = 1; k < p; ++k) s = acc_add(s, widen(src[(int64_t)k * Np]));
    narrow(s, y + i);
  }
}

template <typename E>
hipError_t launch_fold_t(const void* x, void* y, int64_t batch, int64_t N, int64_t Np, int p, hipStream_t s) {
  const int64_t total = batch * Np;
  const int64_t blocks = (total + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
  hipLaunchKernelGGL(k_fold<E>, dim3(grid), dim3(256), 0, s, static_cast<const E*>(x), static_cast<E*>(y), batch, N,
                     Np, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fold(dd_dtype dtype, const void* x, void* y, int64_t batch, int64_t N, int64_t Np, int p,
                       hipStream_t s) {
  switch (dtype) {
    case DD_F32:
      return launch_fold_t<float>(x, y, batch, N, Np, p, s);
    case DD_C64:
      return launch_fold_t<cx<float>>(x, y, batch, N, Np, p, s);
    case DD_F64:
      return launch_fold_t<double>(x, y, batch, N, Np, p, s);
    case DD_C128:
      return launch_fold_t<cx<double>>(x, y, batch, N, Np, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dd
