// Column-pass kernels, float instantiation (compiled as its own unit).
#include "pass_kernels.hpp"

namespace ssfm {

template <>
hipError_t launch_col<float>(int kind, int n, int v, int nb, const PassArgs<float>& a,
                           hipStream_t s, const LaunchEv* ev) {
  switch (kind) {
    case COL_FWD: return launch_col_kind<float, COL_FWD>(n, v, nb, a, s, ev);
    case COL_ADJ: return launch_col_kind<float, COL_ADJ>(n, v, nb, a, s, ev);
    case COL_INV: return launch_col_kind<float, COL_INV>(n, v, nb, a, s, ev);
    case COL_FD: return launch_col_kind<float, COL_FD>(n, v, nb, a, s, ev);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssfm
