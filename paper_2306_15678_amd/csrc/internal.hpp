// internal.hpp -- structures shared by the host plan and the kernels.
#pragma once

#include <cstdint>

namespace ssfm {

// Per-beam constants in device memory (one entry per instance).
struct InstDev {
  int32_t n;           // grid points per side
  int32_t K;           // multiphoton order
  uint32_t terms;      // screen-term mask
  int32_t n_screens;   // turbulence screens
  int64_t off;         // element offset of this beam in every field buffer
  int64_t screen_off;  // element offset of its screen plane 0
  int64_t prop_off;    // element offset of its propagator table (n entries)
  int64_t tw_off;      // element offset of the twiddle table for n
  int64_t steps_off;   // offset of its screen step list in the step table
  int64_t step_base;   // context step at which this beam's field was last set:
                       // its own step index (screens) is the context's minus this
  double cK;           // k0 n2 I_a dz
  double cM;           // (K-1) beta_K I_a^(K-1) dz
  double inv2k1;       // 1 / (2 (K-1))
  double theta[8];     // ansatz parameters
};

// One workgroup's share of a pass: LINES consecutive lines of one beam.
// widx is the position of this item in the beam-contiguous work order (the
// index its partial sums are written to); inst < 0 marks padding.
struct WorkItem {
  int32_t inst;
  int32_t line0;
  int32_t widx;
  int32_t pad;
};

}  // namespace ssfm
