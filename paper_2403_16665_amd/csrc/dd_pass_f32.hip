// Two-pass kernels, float arithmetic: pass 1 for real and complex input, pass 2.
#include "dd_inst.hpp"

namespace dd {
hipError_t launch_pass1(int L, const LaunchCfg& c, const float* x, cx<float>* Y, const DenseArgs<float>& a) {
  return launch_pass1_impl<float, float>(L, c, x, Y, a);
}
hipError_t launch_pass1(int L, const LaunchCfg& c, const cx<float>* x, cx<float>* Y, const DenseArgs<float>& a) {
  return launch_pass1_impl<float, cx<float>>(L, c, x, Y, a);
}
hipError_t launch_pass2(int L, const LaunchCfg& c, const cx<float>* Y, cx<float>* X, const DenseArgs<float>& a) {
  return launch_pass2_impl<float>(L, c, Y, X, a);
}
hipError_t launch_pass2_half(int L, const LaunchCfg& c, const cx<float>* Y, cx<float>* X,
                             const DenseArgs<float>& a) {
  return launch_pass2_impl<float, true>(L, c, Y, X, a);
}
}  // namespace dd
