// Column-pass kernels, double instantiation (compiled as its own unit).
#include "pass_kernels.hpp"

namespace ssfm {

template <>
hipError_t launch_col<double>(int kind, int n, int v, int nb, const PassArgs<double>& a,
                           hipStream_t s, const LaunchEv* ev) {
  switch (kind) {
    case COL_FWD: return launch_col_kind<double, COL_FWD>(n, v, nb, a, s, ev);
    case COL_ADJ: return launch_col_kind<double, COL_ADJ>(n, v, nb, a, s, ev);
    case COL_INV: return launch_col_kind<double, COL_INV>(n, v, nb, a, s, ev);
    case COL_FD: return launch_col_kind<double, COL_FD>(n, v, nb, a, s, ev);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssfm
