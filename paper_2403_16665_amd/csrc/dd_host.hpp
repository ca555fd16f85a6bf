// dd_host.hpp -- host-side helpers shared by the plan and batch APIs.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>

#include "../../include/dense_dft.h"
#include "dd_launch.hpp"

namespace dd {

inline dd_status hip_status(hipError_t e) {
  if (e == hipSuccess) return DD_OK;
  if (e == hipErrorOutOfMemory) return DD_ERR_NOMEM;
  return DD_ERR_DEVICE;
}

inline bool is_smooth(int64_t n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

// A factor the kernels scale by (T/N forward, 1/(alpha T) inverse) must be a
// positive normal number in the arithmetic's precision (double, else float);
// otherwise every bin would come out infinite, NaN or flushed to zero.
inline bool scale_ok(double v, bool dbl) {
  if (!std::isnormal(v) || v < 0.0) return false;
  return dbl || (v >= (double)FLT_MIN && v <= (double)FLT_MAX);
}

inline int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t)1 << (r + 1) <= v) ++r;
  return r;
}

// Stage twiddle table of the line plan of L (narrow: the one-pass kernels'
// plan, single_narrow): for each stage st >= 1 the block
// [s][k] = W_{NS RAD}^{k s} (s < RAD, k < NS).  Allocates *out.
inline dd_status make_stage_table(void** out, int L, bool dbl, bool fp32, hipStream_t s, bool narrow = false) {
  const LinePlan lp = make_line_plan(L, narrow);
  const int n = line_tw_size(lp);
  const size_t cxb = dbl ? 16 : 8;
  hipError_t e = hipMalloc(out, (size_t)(n > 0 ? n : 1) * cxb);
  if (e != hipSuccess) return hip_status(e);
  for (int st = 1; st < lp.nst; ++st) {
    const int NS = line_ns(lp, st), RAD = lp.rad[st];
    const int off = line_tw_offset(lp, st);
    if (dbl)
      e = launch_twiddle(static_cast<cx<double>*>(*out) + off, RAD, NS, 0, (int64_t)NS * RAD, 0, s);
    else
      e = launch_twiddle(static_cast<cx<float>*>(*out) + off, RAD, NS, 0, (int64_t)NS * RAD, fp32, s);
    if (e != hipSuccess) return hip_status(e);
  }
  return DD_OK;
}

// out[r][c] = W_den^{(r c) mod den}.  Allocates *out.
inline dd_status make_table(void** out, int64_t rows, int64_t cols, int64_t den, bool dbl, bool fp32,
                            hipStream_t s) {
  hipError_t e = hipMalloc(out, (size_t)(rows * cols) * (dbl ? 16 : 8));
  if (e != hipSuccess) return hip_status(e);
  if (dbl)
    e = launch_twiddle(static_cast<cx<double>*>(*out), rows, cols, 0, den, 0, s);
  else
    e = launch_twiddle(static_cast<cx<float>*>(*out), rows, cols, 0, den, fp32, s);
  return hip_status(e);
}

}  // namespace dd
