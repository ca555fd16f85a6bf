// dd_inst.hpp -- instantiation bodies of the launchers; included by the
// per-precision translation units with DD_R set to float or double.
#pragma once

#include "dd_launch.hpp"

namespace dd {

template <typename R, typename In>
hipError_t launch_single_impl(int L, const LaunchCfg& c, const In* x, cx<R>* X, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                        \
  case LL: {                                                               \
    constexpr int B = Geom<LL, (int)sizeof(R)>::BLOCK_SINGLE;              \
    return launch_kernel(k_single<R, In, LL, B>, c, x, X, a);              \
  }
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Blocks of the one-pass kernel resident per CU for a block size and LDS
// size (registers, LDS and wavefront slots together); 0 if the runtime
// cannot tell (no device).
template <typename R, typename In>
int single_occupancy_impl(int L, int block, size_t lds) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (L) {
#define DD_CASE(LL)                                                                          \
  case LL: {                                                                                 \
    constexpr int B = Geom<LL, (int)sizeof(R)>::BLOCK_SINGLE;                                \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_single<R, In, LL, B>, block, lds); \
    break;                                                                                   \
  }
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      break;
  }
  return e == hipSuccess && n > 0 ? n : 0;
}

template <typename R, typename In>
hipError_t launch_pass1_impl(int L, const LaunchCfg& c, const In* x, cx<R>* Y, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                        \
  case LL: {                                                               \
    constexpr int C = Geom<LL, (int)sizeof(R)>::lines_pass();              \
    return launch_kernel(k_pass1<R, In, LL, C>, c, x, Y, a);               \
  }
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// HALF: blocks of RB rows that transform RB + 1 (real input, a.hrows > 0);
// otherwise the wider blocks of lines_pass2().
template <typename R, bool HALF = false>
hipError_t launch_pass2_impl(int L, const LaunchCfg& c, const cx<R>* Y, cx<R>* X, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                        \
  case LL: {                                                               \
    constexpr int RB = HALF ? Geom<LL, (int)sizeof(R)>::lines_pass()       \
                            : Geom<LL, (int)sizeof(R)>::lines_pass2();     \
    return launch_kernel(k_pass2<R, LL, RB, HALF ? RB + 1 : RB>, c, Y, X, a); \
  }
    DD_POW2_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace dd
