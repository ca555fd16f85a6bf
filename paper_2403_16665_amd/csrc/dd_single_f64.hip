// Single-pass kernels, double arithmetic: real and complex input.
#include "dd_inst.hpp"

namespace dd {
hipError_t launch_single(int L, const LaunchCfg& c, const double* x, cx<double>* X, const DenseArgs<double>& a) {
  return launch_single_impl<double, double>(L, c, x, X, a);
}
hipError_t launch_single(int L, const LaunchCfg& c, const cx<double>* x, cx<double>* X, const DenseArgs<double>& a) {
  return launch_single_impl<double, cx<double>>(L, c, x, X, a);
}
int single_occupancy(int L, bool real, double /*tag*/, int block, size_t lds) {
  return real ? single_occupancy_impl<double, double>(L, block, lds)
              : single_occupancy_impl<double, cx<double>>(L, block, lds);
}
}  // namespace dd
