// Single-pass kernels, float arithmetic: real and complex input.
#include "dd_inst.hpp"

namespace dd {
hipError_t launch_single(int L, const LaunchCfg& c, const float* x, cx<float>* X, const DenseArgs<float>& a) {
  return launch_single_impl<float, float>(L, c, x, X, a);
}
hipError_t launch_single(int L, const LaunchCfg& c, const cx<float>* x, cx<float>* X, const DenseArgs<float>& a) {
  return launch_single_impl<float, cx<float>>(L, c, x, X, a);
}
int single_occupancy(int L, bool real, float /*tag*/, int block, size_t lds) {
  return real ? single_occupancy_impl<float, float>(L, block, lds)
              : single_occupancy_impl<float, cx<float>>(L, block, lds);
}
}  // namespace dd
