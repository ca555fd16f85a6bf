// Inverse transform kernels, double arithmetic.
#include "dd_inverse.hpp"

namespace dd {
hipError_t launch_single_inv(int L, const LaunchCfg& c, const cx<double>* X, cx<double>* x, const DenseArgs<double>& a) {
  return launch_single_inv_impl<double>(L, c, X, x, a);
}
hipError_t launch_passA(int L, const LaunchCfg& c, const cx<double>* X, cx<double>* G, const DenseArgs<double>& a) {
  return launch_passA_impl<double>(L, c, X, G, a);
}
hipError_t launch_passB(int L, const LaunchCfg& c, const cx<double>* G, cx<double>* x, const DenseArgs<double>& a) {
  return launch_passB_impl<double>(L, c, G, x, a);
}
}  // namespace dd
