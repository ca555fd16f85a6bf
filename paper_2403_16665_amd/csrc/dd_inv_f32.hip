// Inverse transform kernels, float arithmetic.
#include "dd_inverse.hpp"

namespace dd {
hipError_t launch_single_inv(int L, const LaunchCfg& c, const cx<float>* X, cx<float>* x, const DenseArgs<float>& a) {
  return launch_single_inv_impl<float>(L, c, X, x, a);
}
hipError_t launch_passA(int L, const LaunchCfg& c, const cx<float>* X, cx<float>* G, const DenseArgs<float>& a) {
  return launch_passA_impl<float>(L, c, X, G, a);
}
hipError_t launch_passB(int L, const LaunchCfg& c, const cx<float>* G, cx<float>* x, const DenseArgs<float>& a) {
  return launch_passB_impl<float>(L, c, G, x, a);
}
}  // namespace dd
