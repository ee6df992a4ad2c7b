// Row-pass kernels, double instantiation (compiled as its own unit).
#include "pass_kernels.hpp"

namespace ssfm {

template <>
hipError_t launch_row<double>(int kind, int n, int v, int nb, const PassArgs<double>& a,
                           hipStream_t s, const LaunchEv* ev) {
  switch (kind) {
    case ROW_FWD: return launch_row_kind<double, ROW_FWD>(n, v, nb, a, s, ev);
    case ROW_ADJ: return launch_row_kind<double, ROW_ADJ>(n, v, nb, a, s, ev);
    case ROW_INV: return launch_row_kind<double, ROW_INV>(n, v, nb, a, s, ev);
    case ROW_FD: return launch_row_kind<double, ROW_FD>(n, v, nb, a, s, ev);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssfm
