// kernels.hpp -- host-visible interface of the HIP kernels (launch wrappers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "internal.hpp"

namespace ssfm {

template <typename R>
struct cx;

// Pass kinds.  A forward step is ROW_FWD (pending screen applied on load,
// then row diffraction) followed by COL_FWD (column diffraction, FP64 power
// partials, store of the pre-screen field).  An adjoint step is COL_ADJ
// followed by ROW_ADJ (adjoint screen of the previous step fused into the
// epilogue).  ROW_INV / COL_INV are plain inverse DFTs for screen synthesis.
// ROW_FD / COL_FD are the finite-difference reference scheme's passes: COL_FD
// applies the inverse of 1 - (i dz/4k0) Lap_h between a forward and an
// inverse column DFT (Lap_h diagonal in the 2-D DFT basis), ROW_FD inverts
// the row DFT, forms the next right-hand side pointwise (or finishes the
// step) and transforms the rows again.
enum PassKind {
  ROW_FWD = 0, ROW_ADJ = 1, ROW_INV = 2, COL_FWD = 3, COL_ADJ = 4, COL_INV = 5,
  ROW_FD = 6, COL_FD = 7
};
constexpr bool is_col_kind(int k) {
  return k == COL_FWD || k == COL_ADJ || k == COL_INV || k == COL_FD;
}

// ROW_FD flags: the input is row-transformed (else it is U itself), the pass
// finishes the step (U+ = 2 Ubar - U into the state, power partials), the
// finished step is the last one of the launch sequence (no next RHS).
enum : int32_t { FD_SPECTRAL = 2, FD_FINISH = 4, FD_LAST = 8 };

// Start/stop events carried by one pass launch (sampled timing).
struct LaunchEv {
  hipEvent_t start, stop;
};

template <typename R>
struct PassArgs {
  const void* src;            // cx<R> field buffer read
  void* dst;                  // cx<R> field buffer written
  const void* aux;            // ROW_ADJ: pre-screen field s_n (cx<R>)
  void* state;                // ROW_FD: U of the step (read; U+ written when finishing)
  const WorkItem* work;       // one entry per workgroup
  const InstDev* inst;        // beam table
  const void* tables;         // cx<R> twiddle and propagator tables
  const R* screens;           // turbulence planes (read)
  R* planes_out;              // COL_INV: screen planes (write)
  const int64_t* screen_steps;  // per-beam sorted step lists
  double* part;               // COL_FWD: [n_work][2] (sum x A^2, max x A^2)
                              // ROW_ADJ: [n_work][8] theta accumulators
  int64_t step;               // step whose screen is pending (-1: none)
  int32_t pair;               // COL_INV: screen pair index
  int32_t flags;              // COL_FWD: bit 0 = power partials without the screen's A^2;
                              // ROW_FD: FD_* bits
  int32_t n_work;             // entries of the work list (persistent passes; set at launch)
  int32_t precise;            // library sine/cosine in the screens: the pipelined row
                              // passes (which carry none) are replaced by k_row
};

struct PlanInfo {
  int threads;   // workgroup size
  int lines;     // lines per workgroup
  int t;         // threads per line
  size_t lds;    // static LDS bytes
};

// Number of variants and their shape for (kind is column?, n, precision).
int plan_count(bool column, int n);
bool plan_info(bool column, int n, int variant, bool fp64, PlanInfo* out);

template <typename R>
hipError_t launch_pass(int kind, int n, int variant, int n_blocks,
                       const PassArgs<R>& a, hipStream_t s, const LaunchEv* ev = nullptr);

// Pointwise helpers -------------------------------------------------------

// dst (cx<R> device state, beam b at off) = src (complex128 SI) * scale
template <typename R>
hipError_t launch_load_field(const double* src, void* dst, int64_t n_elem,
                             double scale, hipStream_t s);

// dst (complex128 SI) = sqrt(I_a) * [pending screen](state); optionally
// intensity only (float64 I = I_a |u|^2).
template <typename R>
hipError_t launch_store_field(const void* state, const InstDev* inst, int b,
                              int n, const R* screens,
                              const int64_t* screen_steps, int64_t pending_step,
                              double out_scale, double* dst, bool intensity,
                              hipStream_t s);

// Loss / cotangent seed.  For each point of beam b: u_N = screen(s_N);
// mode 0 (g_scale = I_a): I = I_a |u|^2, partial sums of (I - w)^2 and
// G_u = 4 (I - w) I_a u / sum w^2 (wsum[0] = sum w^2, SI);
// mode 1 (g_scale = sqrt(I_a)): G_u = sqrt(I_a) G_ext (G_ext in SI).
// Then the adjoint of the pending screen writes mu_N = S^*(G_u) into lam and
// the ansatz terms of that screen go to part_theta[row][8].
template <typename R>
hipError_t launch_seed(int mode, const void* state, const InstDev* inst, int b,
                       int n, const R* screens, const int64_t* screen_steps,
                       int64_t pending_step, const double* target,
                       const double* wsum, const double* g_ext,
                       double g_scale, void* lam, double* part_loss,
                       double* part_theta, int n_blocks, hipStream_t s);

template <typename R>
hipError_t launch_copy(const void* src, void* dst, int64_t n_elem, hipStream_t s);

// Reduce per-workgroup diag partials of `steps` consecutive steps:
// part[step][n_work][2] -> diag[b][(ring0 + step) % cap][2].
hipError_t launch_diag_finalize(const double* part, int n_work,
                                const int32_t* beam_work_begin, int n_beams,
                                int steps, double* diag, int64_t ring0,
                                int64_t cap, double power_scale_unused,
                                hipStream_t s);

// Fixed-order sum of rows of a [n_rows][width] FP64 array per beam range.
hipError_t launch_reduce_rows(const double* part, int width,
                              const int32_t* beam_begin, int n_beams,
                              double* out, hipStream_t s);

// Sum of squares of a float64 array divided by scale^2 (one value).
hipError_t launch_sumsq(const double* x, int64_t n, double inv_scale,
                        double* partial, double* out, hipStream_t s);

// White noise shaped by the screen spectrum: kind 0 Kolmogorov (amp0 (m^2)^(-11/12)),
// kind 1 step (amp0 where 0 < mx^2 + my^2 <= band_q2, integer mode indices).
template <typename R>
hipError_t launch_noise(const InstDev* inst, int b, int n, int pair,
                        uint64_t seed, double amp0, int kind, double band_q2,
                        void* dst, hipStream_t s);

template <typename R>
hipError_t launch_screen_to_f64(const R* plane, int64_t n_elem, double* dst,
                                hipStream_t s);

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

// Effective lens: FP64 parameters of one application (SI; segments
// {r_end, amplitude, frequency, phase}).
struct LensDev {
  double i_ref, w_l, c1, c2;
  int32_t n_re, n_im;
  double re[8][4];
  double im[8][4];
};
// wk[i] = (|s[i]|^2, 0) over all n_elem points (device units).
template <typename R>
hipError_t launch_lens_prep(const void* s, void* wk, int64_t n_elem, hipStream_t st);
// u[i] *= exp(i f(w_dif[i])) over one beam's n2 points where w_dif >= w_l.
template <typename R>
hipError_t launch_lens_apply(void* u, const void* wdif, int64_t n2, const LensDev& p,
                             hipStream_t st);

// Hot-area labelling of an n x n FP64 array (labels: n^2 ints, overflow:
// one int set if a union exceeded its retry cap) and the root count as
// n_part per-block partial sums; spatial moment partial sums.
hipError_t launch_hot_areas(const double* w, int n, double threshold, int periodic, int* labels,
                            int* overflow, double* part, int n_part, hipStream_t s);
hipError_t launch_moment(const double* w, int n, double dx, double p, int m, double* part,
                         int n_part, hipStream_t s);
// Measure-vector partials: n_part blocks x [sum w, sum w r^2, sum w^2,
// sum w^2 r^2, max w].
hipError_t launch_measure(const double* w, int n, double dx, double* part, int n_part,
                          hipStream_t s);

hipError_t launch_block_mean(const double* src, int n, int b, double* dst,
                             hipStream_t s);

// Allocation-free hot-area count: a file-scope device array (one per GPU)
// holds the labels of grids up to kStaticMaxN^2, the overflow flag at
// kStaticOverflowOff and kStaticParts partial counts at kStaticPartOff.
constexpr int kStaticMaxN = 2048;
constexpr int kStaticParts = 256;
constexpr size_t kStaticOverflowOff = size_t(kStaticMaxN) * kStaticMaxN * sizeof(int);
constexpr size_t kStaticPartOff = kStaticOverflowOff + 256;
constexpr size_t kStaticScratchBytes = kStaticPartOff + kStaticParts * sizeof(double);
// Device address of the current device's copy (looked up once per device).
hipError_t static_scratch(void** out);

}  // namespace ssfm
