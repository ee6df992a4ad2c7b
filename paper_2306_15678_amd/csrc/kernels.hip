// kernels.hip -- split-step march kernels for gfx950 (CDNA4).
//
// One z step of the march (Math and Equations, Eq. (1)-(3), (9)) is two
// passes over the field, each a batch of 1-D lines:
//   row pass     u <- F_x^-1 P_x F_x [S_{n-1}(u)]   (screen of the previous
//                                                     step fused on load)
//   column pass  u <- F_y^-1 P_y F_y u              (FP64 power partials)
// where P_x P_y = exp(-i (kx^2 + ky^2) dz / 2k0) is the separable
// diffraction factor and the 1/N of each inverse DFT is folded into P.
// The field between steps is therefore the pre-screen field V_n; its
// pending screen is applied by the next row pass, by the loss/cotangent
// kernel or when the field is read out.  This keeps the fields the adjoint
// needs (V_n) as the march's own state: recording them costs no extra
// traffic.
//
// Each workgroup owns whole lines: a row workgroup reads and writes LINES
// contiguous rows; a column workgroup reads W adjacent columns row by row
// (W * sizeof(complex) contiguous bytes per row).  Loads and stores are the
// only HBM traffic: 8 B read + 8 B written per point per pass (complex64).
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "screen.hpp"

namespace ssfm {

// --------------------------------------------------------------- plans
// Row plans (T threads per row, LINES rows per workgroup).
template <int N, int V>
struct RowPlanSel;
template <> struct RowPlanSel<128, 0> { using P = Plan<128, 8, 32, Radices<16, 8>>; };
template <> struct RowPlanSel<256, 0> { using P = Plan<256, 16, 16, Radices<16, 16>>; };
template <> struct RowPlanSel<512, 0> { using P = Plan<512, 64, 4, Radices<8, 8, 8>>; };
template <> struct RowPlanSel<768, 0> { using P = Plan<768, 32, 8, Radices<8, 8, 4, 3>>; };
template <> struct RowPlanSel<1024, 0> { using P = Plan<1024, 64, 4, Radices<16, 8, 8>>; };
template <> struct RowPlanSel<1024, 1> { using P = Plan<1024, 64, 2, Radices<16, 8, 8>>; };
template <> struct RowPlanSel<1024, 2> { using P = Plan<1024, 128, 2, Radices<8, 8, 4, 4>>; };
template <> struct RowPlanSel<2048, 0> { using P = Plan<2048, 128, 2, Radices<16, 16, 8>>; };
template <> struct RowPlanSel<4096, 0> { using P = Plan<4096, 256, 1, Radices<16, 16, 16>>; };

// Column plans (T threads per column, W = LINES columns per workgroup).
template <int N, int V>
struct ColPlanSel;
template <> struct ColPlanSel<128, 0> { using P = Plan<128, 8, 32, Radices<16, 8>>; };
template <> struct ColPlanSel<256, 0> { using P = Plan<256, 16, 16, Radices<16, 16>>; };
template <> struct ColPlanSel<512, 0> { using P = Plan<512, 64, 4, Radices<8, 8, 8>>; };
template <> struct ColPlanSel<512, 1> { using P = Plan<512, 32, 8, Radices<16, 16, 2>>; };
template <> struct ColPlanSel<768, 0> { using P = Plan<768, 32, 8, Radices<8, 8, 4, 3>>; };
template <> struct ColPlanSel<1024, 0> { using P = Plan<1024, 64, 4, Radices<16, 8, 8>>; };
template <> struct ColPlanSel<1024, 1> { using P = Plan<1024, 32, 8, Radices<16, 8, 8>>; };
template <> struct ColPlanSel<1024, 2> { using P = Plan<1024, 64, 8, Radices<16, 8, 8>>; };
template <> struct ColPlanSel<2048, 0> { using P = Plan<2048, 128, 2, Radices<16, 16, 8>>; };
template <> struct ColPlanSel<2048, 1> { using P = Plan<2048, 64, 4, Radices<16, 16, 8>>; };
template <> struct ColPlanSel<4096, 0> { using P = Plan<4096, 256, 2, Radices<16, 16, 16>>; };
template <> struct ColPlanSel<4096, 1> { using P = Plan<4096, 128, 2, Radices<16, 16, 16>>; };

static int row_variants(int n) {
  switch (n) {
    case 1024: return 3;
    case 128: case 256: case 512: case 768: case 2048: case 4096: return 1;
    default: return 0;
  }
}
static int col_variants(int n) {
  switch (n) {
    case 512: case 2048: case 4096: return 2;
    case 1024: return 3;
    case 128: case 256: case 768: return 1;
    default: return 0;
  }
}

#ifdef SSFM_INST_F32
int plan_count(bool column, int n) { return column ? col_variants(n) : row_variants(n); }
#endif

template <class P, bool COLUMN>
static size_t lds_bytes(bool fp64) {
  const size_t el = fp64 ? 16 : 8;
  if (COLUMN) return el * P::N * P::LINES;
  return el * P::LINES * LdsLineMajor<float, P::N>::LINE;
}

template <class P, bool COLUMN>
static void fill_info(bool fp64, PlanInfo* o) {
  o->threads = P::THREADS;
  o->lines = P::LINES;
  o->t = P::T;
  o->lds = lds_bytes<P, COLUMN>(fp64);
}

#ifdef SSFM_INST_F32
bool plan_info(bool column, int n, int v, bool fp64, PlanInfo* o) {
  if (v < 0 || v >= plan_count(column, n)) return false;
#define SSFM_ROWCASE(NN, VV) \
  if (!column && n == NN && v == VV) { fill_info<RowPlanSel<NN, VV>::P, false>(fp64, o); return true; }
#define SSFM_COLCASE(NN, VV) \
  if (column && n == NN && v == VV) { fill_info<ColPlanSel<NN, VV>::P, true>(fp64, o); return true; }
  SSFM_ROWCASE(128, 0) SSFM_ROWCASE(256, 0) SSFM_ROWCASE(512, 0) SSFM_ROWCASE(768, 0)
  SSFM_ROWCASE(1024, 0) SSFM_ROWCASE(1024, 1) SSFM_ROWCASE(1024, 2)
  SSFM_ROWCASE(2048, 0) SSFM_ROWCASE(4096, 0)
  SSFM_COLCASE(128, 0) SSFM_COLCASE(256, 0) SSFM_COLCASE(512, 0) SSFM_COLCASE(512, 1)
  SSFM_COLCASE(768, 0) SSFM_COLCASE(1024, 0) SSFM_COLCASE(1024, 1) SSFM_COLCASE(1024, 2)
  SSFM_COLCASE(2048, 0) SSFM_COLCASE(2048, 1) SSFM_COLCASE(4096, 0) SSFM_COLCASE(4096, 1)
#undef SSFM_ROWCASE
#undef SSFM_COLCASE
  return false;
}
#endif

// ------------------------------------------------------------ helpers
template <typename R>
__device__ __forceinline__ ScreenConst<R> screen_const(const InstDev& in) {
  ScreenConst<R> s;
  s.cK = R(in.cK);
  s.cM = R(in.cM);
  s.inv2k1 = R(in.inv2k1);
#pragma unroll
  for (int p = 0; p < 8; ++p) s.th[p] = R(in.theta[p]);
  s.K = in.K;
  s.terms = in.terms;
  return s;
}

// Turbulence plane applied after `step` (nullptr if none).
template <typename R>
__device__ __forceinline__ const R* find_plane(const R* screens,
                                               const int64_t* steps,
                                               const InstDev& in, int64_t step) {
  if (step < 0 || !(in.terms & T_TURB) || in.n_screens <= 0 || screens == nullptr)
    return nullptr;
  const int64_t* st = steps + in.steps_off;
  for (int s = 0; s < in.n_screens; ++s) {
    if (st[s] == step) return screens + in.screen_off + int64_t(s) * in.n * in.n;
  }
  return nullptr;
}

// Deterministic workgroup reduction of NV doubles (sum or max); the result
// is valid in thread 0.  red: shared [THREADS/64][NV].
template <int NV, int THREADS, bool MAX>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double o = __shfl_xor(v[k], off, 64);
      v[k] = MAX ? fmax(v[k], o) : v[k] + o;
    }
  }
  constexpr int NW = (THREADS + 63) / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = red[k];
      for (int w = 1; w < NW; ++w) s = MAX ? fmax(s, red[w * NV + k]) : s + red[w * NV + k];
      v[k] = s;
    }
  }
}

// ------------------------------------------------------------ row pass
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS) k_row(PassArgs<R> a) {
  constexpr int N = P::N, T = P::T, E = P::E;
  using L = LdsLineMajor<R, N>;
  __shared__ cx<R> lds_mem[P::LINES * L::LINE];
  __shared__ double red[((P::THREADS + 63) / 64) * 8];

  const WorkItem w = a.work[blockIdx.x];
  if (w.inst < 0) return;
  const InstDev& in = a.inst[w.inst];
  if constexpr (KIND == ROW_INV) {
    if (2 * a.pair >= in.n_screens || !(in.terms & T_TURB)) return;
  }
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int64_t row = w.line0 + line;
  const int64_t base = in.off + row * N;
  const L lds{lds_mem + line * L::LINE};
  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ tw = tables + in.tw_off;
  const cx<R>* __restrict__ prop = tables + in.prop_off;
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src) + base;
  cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst) + base;

  cx<R> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[t + T * e];

  if constexpr (KIND == ROW_FWD) {
    if (a.step >= 0) {
      const ScreenConst<R> sc = screen_const<R>(in);
      const R* plane = find_plane(a.screens, a.screen_steps, in, a.step);
      const R* prow = plane ? plane + row * N : nullptr;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const R pt = prow ? prow[t + T * e] : R(0);
        v[e] = screen_apply(sc, v[e], pt);
      }
    }
  }

  if constexpr (KIND == ROW_INV) {
    fft_line<R, P, +1>(v, t, lds, tw);
  } else {
    fft_line<R, P, -1>(v, t, lds, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> p = prop[t + T * e];
      v[e] = (KIND == ROW_ADJ) ? cmulc(v[e], p) : cmul(v[e], p);
    }
    fft_line<R, P, +1>(v, t, lds, tw);
  }

  if constexpr (KIND == ROW_ADJ) {
    if (a.step >= 0) {
      const ScreenConst<R> sc = screen_const<R>(in);
      const R* plane = find_plane(a.screens, a.screen_steps, in, a.step);
      const R* prow = plane ? plane + row * N : nullptr;
      const cx<R>* __restrict__ sv = static_cast<const cx<R>*>(a.aux) + base;
      double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const R pt = prow ? prow[t + T * e] : R(0);
        v[e] = screen_adjoint(sc, sv[t + T * e], v[e], pt, g);
      }
      if (in.terms & T_ANSATZ) {
        block_reduce<8, P::THREADS, false>(g, red);
        if (threadIdx.x == 0) {
          double* acc = a.part + int64_t(w.widx) * 8;
#pragma unroll
          for (int p = 0; p < 8; ++p) acc[p] += g[p];
        }
      }
    }
  }

#pragma unroll
  for (int e = 0; e < E; ++e) dst[t + T * e] = v[e];
}

// --------------------------------------------------------- column pass
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS) k_col(PassArgs<R> a) {
  constexpr int N = P::N, T = P::T, E = P::E, W = P::LINES;
  using L = LdsPointMajor<R, W>;
  __shared__ cx<R> lds_mem[N * W];
  __shared__ double red[((P::THREADS + 63) / 64) * 2];

  const WorkItem w = a.work[blockIdx.x];
  if (w.inst < 0) return;
  const InstDev& in = a.inst[w.inst];
  if constexpr (KIND == COL_INV) {
    if (2 * a.pair >= in.n_screens || !(in.terms & T_TURB)) return;
  }
  const int c = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int64_t col = w.line0 + c;
  const int64_t base = in.off + col;
  const L lds{lds_mem + c};
  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ tw = tables + in.tw_off;
  const cx<R>* __restrict__ prop = tables + in.prop_off;
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src) + base;

  cx<R> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[int64_t(t + T * e) * N];

  if constexpr (KIND == COL_INV) {
    fft_line<R, P, +1>(v, t, lds, tw);
  } else {
    fft_line<R, P, -1>(v, t, lds, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cx<R> p = prop[t + T * e];
      v[e] = (KIND == COL_ADJ) ? cmulc(v[e], p) : cmul(v[e], p);
    }
    fft_line<R, P, +1>(v, t, lds, tw);
  }

  if constexpr (KIND == COL_INV) {
    // screen pair: real part -> plane 2p, imaginary part -> plane 2p+1
    R* pre = a.planes_out + in.screen_off + int64_t(2 * a.pair) * N * N + col;
    const bool has_im = 2 * a.pair + 1 < in.n_screens;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      pre[int64_t(t + T * e) * N] = v[e].re;
      if (has_im) pre[int64_t(N) * N + int64_t(t + T * e) * N] = v[e].im;
    }
    return;
  } else {
    cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst) + base;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[int64_t(t + T * e) * N] = v[e];
  }

  if constexpr (KIND == COL_FWD) {
    if (a.part != nullptr) {
      const ScreenConst<R> sc = screen_const<R>(in);
      double s[1] = {0.0}, m[1] = {0.0};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const R x = v[e].re * v[e].re + v[e].im * v[e].im;
        const double xa = double(x) * double(screen_amp2(sc, x));
        s[0] += xa;
        m[0] = fmax(m[0], xa);
      }
      __syncthreads();  // red[] reuse is safe; keep LDS reads finished
      block_reduce<1, P::THREADS, false>(s, red);
      __syncthreads();
      block_reduce<1, P::THREADS, true>(m, red + ((P::THREADS + 63) / 64));
      if (threadIdx.x == 0) {
        a.part[int64_t(w.widx) * 2 + 0] = s[0];
        a.part[int64_t(w.widx) * 2 + 1] = m[0];
      }
    }
  }
}

// -------------------------------------------------------------- launch
template <typename R, class P, int KIND>
static hipError_t launch_one(int n_blocks, const PassArgs<R>& a, hipStream_t s) {
  if constexpr (KIND >= COL_FWD) {
    hipLaunchKernelGGL((k_col<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_row<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
  }
  return hipGetLastError();
}

template <typename R, int KIND>
static hipError_t launch_kind(int n, int v, int n_blocks, const PassArgs<R>& a,
                              hipStream_t s) {
  constexpr bool COL = KIND >= COL_FWD;
#define SSFM_CCASE(NN, VV) \
  if (n == NN && v == VV) return launch_one<R, typename ColPlanSel<NN, VV>::P, KIND>(n_blocks, a, s);
#define SSFM_RCASE(NN, VV) \
  if (n == NN && v == VV) return launch_one<R, typename RowPlanSel<NN, VV>::P, KIND>(n_blocks, a, s);
  if constexpr (COL) {
    SSFM_CCASE(128, 0) SSFM_CCASE(256, 0) SSFM_CCASE(512, 0) SSFM_CCASE(512, 1)
    SSFM_CCASE(768, 0) SSFM_CCASE(1024, 0) SSFM_CCASE(1024, 1) SSFM_CCASE(1024, 2)
    SSFM_CCASE(2048, 0) SSFM_CCASE(2048, 1) SSFM_CCASE(4096, 0) SSFM_CCASE(4096, 1)
  } else {
    SSFM_RCASE(128, 0) SSFM_RCASE(256, 0) SSFM_RCASE(512, 0) SSFM_RCASE(768, 0)
    SSFM_RCASE(1024, 0) SSFM_RCASE(1024, 1) SSFM_RCASE(1024, 2)
    SSFM_RCASE(2048, 0) SSFM_RCASE(4096, 0)
  }
#undef SSFM_CCASE
#undef SSFM_RCASE
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_pass(int kind, int n, int variant, int n_blocks,
                       const PassArgs<R>& a, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  switch (kind) {
    case ROW_FWD: return launch_kind<R, ROW_FWD>(n, variant, n_blocks, a, s);
    case ROW_ADJ: return launch_kind<R, ROW_ADJ>(n, variant, n_blocks, a, s);
    case ROW_INV: return launch_kind<R, ROW_INV>(n, variant, n_blocks, a, s);
    case COL_FWD: return launch_kind<R, COL_FWD>(n, variant, n_blocks, a, s);
    case COL_ADJ: return launch_kind<R, COL_ADJ>(n, variant, n_blocks, a, s);
    case COL_INV: return launch_kind<R, COL_INV>(n, variant, n_blocks, a, s);
    default: return hipErrorInvalidValue;
  }
}

#ifdef SSFM_INST_F32
template hipError_t launch_pass<float>(int, int, int, int, const PassArgs<float>&, hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_pass<double>(int, int, int, int, const PassArgs<double>&, hipStream_t);
#endif

// ----------------------------------------------------- pointwise kernels
template <typename R>
__global__ void k_load_field(const double* __restrict__ src, cx<R>* __restrict__ dst,
                             int64_t n_elem, double scale) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n_elem;
       i += int64_t(gridDim.x) * blockDim.x) {
    dst[i] = {R(src[2 * i] * scale), R(src[2 * i + 1] * scale)};
  }
}

static int grid_for(int64_t n_elem, int threads) {
  int64_t g = (n_elem + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return int(g);
}

template <typename R>
hipError_t launch_load_field(const double* src, void* dst, int64_t n_elem,
                             double scale, hipStream_t s) {
  hipLaunchKernelGGL((k_load_field<R>), dim3(grid_for(n_elem, 256)), dim3(256), 0, s,
                     src, static_cast<cx<R>*>(dst), n_elem, scale);
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_load_field<float>(const double*, void*, int64_t, double, hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_load_field<double>(const double*, void*, int64_t, double, hipStream_t);
#endif

template <typename R>
__global__ void k_store_field(const cx<R>* __restrict__ state, const InstDev* inst,
                              int b, const R* screens, const int64_t* steps,
                              int64_t pending, double out_scale,
                              double* __restrict__ dst, int intensity) {
  const InstDev& in = inst[b];
  const int64_t n2 = int64_t(in.n) * in.n;
  const ScreenConst<R> sc = screen_const<R>(in);
  const R* plane = find_plane(screens, steps, in, pending);
  const cx<R>* st = state + in.off;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    cx<R> u = st[i];
    if (pending >= 0) u = screen_apply(sc, u, plane ? plane[i] : R(0));
    if (intensity) {
      dst[i] = (double(u.re) * u.re + double(u.im) * u.im) * out_scale * out_scale;
    } else {
      dst[2 * i] = double(u.re) * out_scale;
      dst[2 * i + 1] = double(u.im) * out_scale;
    }
  }
}

template <typename R>
hipError_t launch_store_field(const void* state, const InstDev* inst, int b, int n,
                              const R* screens, const int64_t* screen_steps,
                              int64_t pending_step, double out_scale, double* dst,
                              bool intensity, hipStream_t s) {
  hipLaunchKernelGGL((k_store_field<R>), dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, s,
                     static_cast<const cx<R>*>(state), inst, b, screens, screen_steps,
                     pending_step, out_scale, dst, intensity ? 1 : 0);
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_store_field<float>(const void*, const InstDev*, int, int, const float*,
                                              const int64_t*, int64_t, double, double*, bool,
                                              hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_store_field<double>(const void*, const InstDev*, int, int,
                                               const double*, const int64_t*, int64_t, double,
                                               double*, bool, hipStream_t);
#endif

// Loss / cotangent seed: one workgroup per row of beam b (256 threads).
template <typename R>
__global__ void __launch_bounds__(256)
k_seed(int mode, const cx<R>* __restrict__ state, const InstDev* inst, int b,
       const R* screens, const int64_t* steps, int64_t pending,
       const double* __restrict__ target, const double* wsum,
       const double* __restrict__ g_ext, double g_scale, cx<R>* __restrict__ lam,
       double* part_loss, double* part_theta) {
  __shared__ double red[4 * 8];
  const InstDev& in = inst[b];
  const int n = in.n;
  const int64_t row = blockIdx.x;
  const ScreenConst<R> sc = screen_const<R>(in);
  const R* plane = find_plane(screens, steps, in, pending);
  // mode 0: g_scale = I_a; loss in SI, G_u = 4 (I - w) I_a u / sum w^2
  const double inv_w = (mode == 0) ? 1.0 / wsum[0] : 0.0;
  double loss[1] = {0.0};
  double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int x = threadIdx.x; x < n; x += 256) {
    const int64_t i = row * n + x;
    const cx<R> v = state[in.off + i];
    const R pt = plane ? plane[i] : R(0);
    const cx<R> u = (pending >= 0) ? screen_apply(sc, v, pt) : v;
    cx<R> gu;
    if (mode == 0) {
      const double xx = double(u.re) * u.re + double(u.im) * u.im;
      const double d = xx * g_scale - target[i];
      loss[0] += d * d;
      const double f = 4.0 * d * g_scale * inv_w;
      gu = {R(f * u.re), R(f * u.im)};
    } else {
      gu = {R(g_ext[2 * i] * g_scale), R(g_ext[2 * i + 1] * g_scale)};
    }
    const cx<R> out = (pending >= 0) ? screen_adjoint(sc, v, gu, pt, g) : gu;
    lam[in.off + i] = out;
  }
  block_reduce<1, 256, false>(loss, red);
  __syncthreads();
  block_reduce<8, 256, false>(g, red);
  if (threadIdx.x == 0) {
    part_loss[row] = loss[0];
#pragma unroll
    for (int p = 0; p < 8; ++p) part_theta[row * 8 + p] = g[p];
  }
}

template <typename R>
hipError_t launch_seed(int mode, const void* state, const InstDev* inst, int b, int n,
                       const R* screens, const int64_t* screen_steps, int64_t pending_step,
                       const double* target, const double* wsum, const double* g_ext,
                       double g_scale, void* lam, double* part_loss, double* part_theta,
                       int n_blocks, hipStream_t s) {
  (void)n;
  hipLaunchKernelGGL((k_seed<R>), dim3(n_blocks), dim3(256), 0, s, mode,
                     static_cast<const cx<R>*>(state), inst, b, screens, screen_steps,
                     pending_step, target, wsum, g_ext, g_scale, static_cast<cx<R>*>(lam),
                     part_loss, part_theta);
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_seed<float>(int, const void*, const InstDev*, int, int, const float*,
                                       const int64_t*, int64_t, const double*, const double*,
                                       const double*, double, void*, double*, double*, int,
                                       hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_seed<double>(int, const void*, const InstDev*, int, int,
                                        const double*, const int64_t*, int64_t, const double*,
                                        const double*, const double*, double, void*, double*,
                                        double*, int, hipStream_t);
#endif

template <typename R>
__global__ void k_copy(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

template <typename R>
hipError_t launch_copy(const void* src, void* dst, int64_t n_elem, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<R>), dim3(grid_for(n_elem, 256)), dim3(256), 0, s,
                     static_cast<const cx<R>*>(src), static_cast<cx<R>*>(dst), n_elem);
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_copy<float>(const void*, void*, int64_t, hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_copy<double>(const void*, void*, int64_t, hipStream_t);
#endif

// One workgroup per (beam, step): fixed-order sum / max over the beam's
// column work items.
#ifdef SSFM_INST_F32
__global__ void k_diag_finalize(const double* __restrict__ part, int n_work,
                                const int32_t* __restrict__ wbegin, int steps,
                                double* __restrict__ diag, int64_t ring0, int64_t cap) {
  const int b = blockIdx.y;
  const int step = blockIdx.x;
  if (step >= steps || threadIdx.x != 0) return;
  const double* p = part + int64_t(step) * n_work * 2;
  double s = 0.0, m = 0.0;
  for (int w = wbegin[b]; w < wbegin[b + 1]; ++w) {
    s += p[2 * w];
    m = fmax(m, p[2 * w + 1]);
  }
  const int64_t slot = (ring0 + step) % cap;
  diag[(int64_t(b) * cap + slot) * 2 + 0] = s;
  diag[(int64_t(b) * cap + slot) * 2 + 1] = m;
}
#endif

#ifdef SSFM_INST_F32
hipError_t launch_diag_finalize(const double* part, int n_work, const int32_t* wbegin,
                                int n_beams, int steps, double* diag, int64_t ring0,
                                int64_t cap, double, hipStream_t s) {
  if (steps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_finalize, dim3(steps, n_beams), dim3(64), 0, s, part, n_work,
                     wbegin, steps, diag, ring0, cap);
  return hipGetLastError();
}
#endif

#ifdef SSFM_INST_F32
__global__ void k_reduce_rows(const double* __restrict__ part, int width,
                              const int32_t* __restrict__ begin, double* __restrict__ out) {
  const int b = blockIdx.x;
  const int k = threadIdx.x;
  if (k >= width) return;
  double s = 0.0;
  for (int r = begin[b]; r < begin[b + 1]; ++r) s += part[int64_t(r) * width + k];
  out[int64_t(b) * width + k] = s;
}
#endif

#ifdef SSFM_INST_F32
hipError_t launch_reduce_rows(const double* part, int width, const int32_t* begin,
                              int n_beams, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_rows, dim3(n_beams), dim3(64), 0, s, part, width, begin, out);
  return hipGetLastError();
}
#endif

// sum of (x/scale)^2 in two fixed-order levels
#ifdef SSFM_INST_F32
__global__ void __launch_bounds__(256)
k_sumsq_part(const double* __restrict__ x, int64_t n, double inv_scale, double* part) {
  __shared__ double red[4];
  double s[1] = {0.0};
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double v = x[i] * inv_scale;
    s[0] += v * v;
  }
  block_reduce<1, 256, false>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
#endif

#ifdef SSFM_INST_F32
__global__ void k_sum_small(const double* part, int n, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] = s;
}
#endif

#ifdef SSFM_INST_F32
hipError_t launch_sumsq(const double* x, int64_t n, double inv_scale, double* partial,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_part, dim3(256), dim3(256), 0, s, x, n, inv_scale, partial);
  hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(64), 0, s, partial, 256, out);
  return hipGetLastError();
}
#endif

// ------------------------------------------------ turbulence white noise
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies, key advanced by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = uint64_t(M0) * c[0];
    const uint64_t p1 = uint64_t(M1) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Spectrum sample c * sqrt(Phi(f)) df at FFT index (row, col) of beam b:
// Phi(f) df^2 = amp0^2 * m^(-11/3) with m = |(signed col, signed row)|.
template <typename R>
__global__ void k_noise(const InstDev* inst, int b, int pair, uint32_t k0, uint32_t k1,
                        double amp0, cx<R>* __restrict__ dst) {
  const InstDev& in = inst[b];
  const int n = in.n;
  const int64_t n2 = int64_t(n) * n;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int row = int(i / n), col = int(i - int64_t(row) * n);
    uint32_t c[4] = {uint32_t(col), uint32_t(row), uint32_t(pair), 0u};
    philox4x32_10(c, k0, k1);
    const double u1 = (double(c[0]) + 0.5) * 2.3283064365386962890625e-10;
    const double u2 = (double(c[1]) + 0.5) * 2.3283064365386962890625e-10;
    const double rr = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    const int mx = (col <= n / 2) ? col : col - n;
    const int my = (row <= n / 2) ? row : row - n;
    const double m2 = double(mx) * mx + double(my) * my;
    const double a = (m2 > 0.0) ? amp0 * pow(m2, -11.0 / 12.0) : 0.0;
    dst[in.off + i] = {R(a * rr * cs), R(a * rr * sn)};
  }
}

template <typename R>
hipError_t launch_noise(const InstDev* inst, int b, int n, int pair, uint64_t seed,
                        double amp0, void* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_noise<R>), dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, s,
                     inst, b, pair, uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32), amp0,
                     static_cast<cx<R>*>(dst));
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_noise<float>(const InstDev*, int, int, int, uint64_t, double, void*,
                                        hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_noise<double>(const InstDev*, int, int, int, uint64_t, double, void*,
                                         hipStream_t);
#endif

template <typename R>
__global__ void k_plane_f64(const R* __restrict__ p, int64_t n, double* __restrict__ d) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    d[i] = double(p[i]);
}

template <typename R>
hipError_t launch_screen_to_f64(const R* plane, int64_t n_elem, double* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_plane_f64<R>), dim3(grid_for(n_elem, 256)), dim3(256), 0, s, plane,
                     n_elem, dst);
  return hipGetLastError();
}
#ifdef SSFM_INST_F32
template hipError_t launch_screen_to_f64<float>(const float*, int64_t, double*, hipStream_t);
#endif
#ifdef SSFM_INST_F64
template hipError_t launch_screen_to_f64<double>(const double*, int64_t, double*, hipStream_t);
#endif

#ifdef SSFM_INST_F32
__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
#endif

#ifdef SSFM_INST_F32
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
#endif

#ifdef SSFM_INST_F32
__global__ void k_block_mean(const double* __restrict__ src, int n, int b,
                             double* __restrict__ dst) {
  const int m = n / b;
  const int64_t total = int64_t(m) * m;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(i / m), c = int(i - int64_t(r) * m);
    double s = 0.0;
    for (int y = 0; y < b; ++y)
      for (int x = 0; x < b; ++x) s += src[int64_t(r * b + y) * n + c * b + x];
    dst[i] = s / (double(b) * b);
  }
}
#endif

#ifdef SSFM_INST_F32
hipError_t launch_block_mean(const double* src, int n, int b, double* dst, hipStream_t s) {
  const int64_t total = int64_t(n / b) * (n / b);
  hipLaunchKernelGGL(k_block_mean, dim3(grid_for(total, 256)), dim3(256), 0, s, src, n, b,
                     dst);
  return hipGetLastError();
}
#endif

}  // namespace ssfm
