// Half-exchange column-pass kernels, float instantiation (compiled as its
// own unit, so that the other column kernels are built without them).
#include "pass_col_hx.hpp"

namespace ssfm {

#define SSFM_HX_INST(NN, VV, ...)                                                               \
  template hipError_t launch_hx<float, ColPlanSel<NN, VV>::P, COL_FWD>(                         \
      int, const PassArgs<float>&, hipStream_t, const LaunchEv*);                               \
  template hipError_t launch_hx<float, ColPlanSel<NN, VV>::P, COL_ADJ>(                         \
      int, const PassArgs<float>&, hipStream_t, const LaunchEv*);                               \
  template hipError_t launch_hx<float, ColPlanSel<NN, VV>::P, COL_INV>(                         \
      int, const PassArgs<float>&, hipStream_t, const LaunchEv*);                               \
  template hipError_t launch_hx<float, ColPlanSel<NN, VV>::P, COL_FD>(                          \
      int, const PassArgs<float>&, hipStream_t, const LaunchEv*);
SSFM_COL_PLANS(SSFM_HX_INST)
#undef SSFM_HX_INST

}  // namespace ssfm
