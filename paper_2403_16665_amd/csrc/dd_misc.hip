// Twiddle-table generation launchers and the length / geometry queries.
#include "dd_launch.hpp"

namespace dd {

template <typename R>
static hipError_t twiddle_impl(cx<R>* out, int64_t rows, int64_t cols, int64_t r0, int64_t den, int fp32,
                               hipStream_t s) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  const int B = 256;
  hipLaunchKernelGGL(k_twiddle<R>, dim3((unsigned)((n + B - 1) / B)), dim3(B), 0, s, out, rows, cols, r0,
                     den, fp32);
  return hipGetLastError();
}

hipError_t launch_twiddle(cx<float>* out, int64_t rows, int64_t cols, int64_t r0, int64_t den, int fp32,
                          hipStream_t s) {
  return twiddle_impl<float>(out, rows, cols, r0, den, fp32, s);
}
hipError_t launch_twiddle(cx<double>* out, int64_t rows, int64_t cols, int64_t r0, int64_t den, int fp32,
                          hipStream_t s) {
  return twiddle_impl<double>(out, rows, cols, r0, den, 0, s);
}

bool len_supported(int L) {
  switch (L) {
#define DD_CASE(LL) case LL:
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    return true;
    default:
      return false;
  }
}

bool pass2_len_supported(int L) {
  switch (L) {
#define DD_CASE(LL) case LL:
    DD_POW2_LENGTHS(DD_CASE)
#undef DD_CASE
    return true;
    default:
      return false;
  }
}

KGeom geom_single(int L, int rbytes) {
  switch (L) {
#define DD_CASE(LL)                                                                                   \
  case LL:                                                                                            \
    if (rbytes == 4)                                                                                  \
      return {Geom<LL, 4>::TLS, Geom<LL, 4>::lines_single(), Geom<LL, 4>::BLOCK_SINGLE};              \
    return {Geom<LL, 8>::TLS, Geom<LL, 8>::lines_single(), Geom<LL, 8>::BLOCK_SINGLE};
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return {0, 0, 0};
  }
}

KGeom geom_pass(int L, int rbytes) {
  switch (L) {
#define DD_CASE(LL)                                                                                   \
  case LL:                                                                                            \
    if (rbytes == 4) return {Geom<LL, 4>::TL, Geom<LL, 4>::lines_pass(), Geom<LL, 4>::BLOCK_PASS};    \
    return {Geom<LL, 8>::TL, Geom<LL, 8>::lines_pass(), Geom<LL, 8>::BLOCK_PASS};
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return {0, 0, 0};
  }
}

KGeom geom_pass2(int L, int rbytes) {
  switch (L) {
#define DD_CASE(LL)                                                                                   \
  case LL:                                                                                            \
    if (rbytes == 4) return {Geom<LL, 4>::TL, Geom<LL, 4>::lines_pass2(), Geom<LL, 4>::TL * Geom<LL, 4>::lines_pass2()}; \
    return {Geom<LL, 8>::TL, Geom<LL, 8>::lines_pass2(), Geom<LL, 8>::TL * Geom<LL, 8>::lines_pass2()};
    DD_POW2_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return {0, 0, 0};
  }
}

// Every instantiated length has a consistent radix plan.
#define DD_CASE(LL) static_assert(line_plan_ok(LL) && line_plan_ok(LL, single_narrow(LL)), "bad line plan");
DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE

}  // namespace dd
