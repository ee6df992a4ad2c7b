// Row-pass kernels, float instantiation (compiled as its own unit).
#include "pass_kernels.hpp"

namespace ssfm {

template <>
hipError_t launch_row<float>(int kind, int n, int v, int nb, const PassArgs<float>& a,
                           hipStream_t s, const LaunchEv* ev) {
  switch (kind) {
    case ROW_FWD: return launch_row_kind<float, ROW_FWD>(n, v, nb, a, s, ev);
    case ROW_ADJ: return launch_row_kind<float, ROW_ADJ>(n, v, nb, a, s, ev);
    case ROW_INV: return launch_row_kind<float, ROW_INV>(n, v, nb, a, s, ev);
    case ROW_FD: return launch_row_kind<float, ROW_FD>(n, v, nb, a, s, ev);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ssfm
