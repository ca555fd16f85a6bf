// Two-pass kernels, double arithmetic: pass 1 for real and complex input, pass 2.
#include "dd_inst.hpp"

namespace dd {
hipError_t launch_pass1(int L, const LaunchCfg& c, const double* x, cx<double>* Y, const DenseArgs<double>& a) {
  return launch_pass1_impl<double, double>(L, c, x, Y, a);
}
hipError_t launch_pass1(int L, const LaunchCfg& c, const cx<double>* x, cx<double>* Y, const DenseArgs<double>& a) {
  return launch_pass1_impl<double, cx<double>>(L, c, x, Y, a);
}
hipError_t launch_pass2(int L, const LaunchCfg& c, const cx<double>* Y, cx<double>* X, const DenseArgs<double>& a) {
  return launch_pass2_impl<double>(L, c, Y, X, a);
}
hipError_t launch_pass2_half(int L, const LaunchCfg& c, const cx<double>* Y, cx<double>* X,
                             const DenseArgs<double>& a) {
  return launch_pass2_impl<double, true>(L, c, Y, X, a);
}
}  // namespace dd
