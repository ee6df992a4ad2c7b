// kernels.hip -- plan tables, pass dispatch and the pointwise kernels of
// the march (field load/store with the pending screen, loss and cotangent
// seed, FP64 reductions, Philox turbulence noise, block means).  The row and
// column pass kernels live in pass_kernels.hpp and are compiled per
// precision in pass_{row,col}_{f32,f64}.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "pass_kernels.hpp"
#include "lens_vjp.hpp"
#include "subharmonics.hpp"

namespace ssfm {

// ------------------------------------------------------------- plans
int plan_count(bool column, int n) {
  int c = 0;
#define SSFM_COUNT(NN, VV, ...) \
  if (n == NN && VV + 1 > c) c = VV + 1;
  if (column) {
    SSFM_COL_PLANS(SSFM_COUNT)
  } else {
    SSFM_ROW_PLANS(SSFM_COUNT)
  }
#undef SSFM_COUNT
  return c;
}

// false when the plan is not built at this precision (its tile does not
// fit a workgroup's LDS, or a pipelined plan at complex128)
template <class P, bool COLUMN>
static bool fill_info(bool fp64, PlanInfo* o) {
  o->threads = P::THREADS;
  o->lines = P::LINES;
  o->t = P::T;
  o->lds = fp64 ? plan_lds_bytes<double, P>(COLUMN) : plan_lds_bytes<float, P>(COLUMN);
  return fp64 ? plan_fits<double, P>(COLUMN) : plan_fits<float, P>(COLUMN);
}

bool plan_info(bool column, int n, int v, bool fp64, PlanInfo* o) {
#define SSFM_RINFO(NN, VV, ...) \
  if (!column && n == NN && v == VV) return fill_info<RowPlanSel<NN, VV>::P, false>(fp64, o);
#define SSFM_CINFO(NN, VV, ...) \
  if (column && n == NN && v == VV) return fill_info<ColPlanSel<NN, VV>::P, true>(fp64, o);
  SSFM_ROW_PLANS(SSFM_RINFO)
  SSFM_COL_PLANS(SSFM_CINFO)
#undef SSFM_RINFO
#undef SSFM_CINFO
  return false;
}

template <typename R>
hipError_t launch_pass(int kind, int n, int variant, int n_blocks, const PassArgs<R>& a,
                       hipStream_t s, const LaunchEv* ev) {
  if (n_blocks <= 0) return hipSuccess;
  if (is_col_kind(kind)) return launch_col<R>(kind, n, variant, n_blocks, a, s, ev);
  return launch_row<R>(kind, n, variant, n_blocks, a, s, ev);
}
template hipError_t launch_pass<float>(int, int, int, int, const PassArgs<float>&, hipStream_t,
                                       const LaunchEv*);
template hipError_t launch_pass<double>(int, int, int, int, const PassArgs<double>&, hipStream_t,
                                        const LaunchEv*);

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
template hipError_t launch_load_field<float>(const double*, void*, int64_t, double, hipStream_t);
template hipError_t launch_load_field<double>(const double*, void*, int64_t, double, hipStream_t);

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
template hipError_t launch_store_field<float>(const void*, const InstDev*, int, int, const float*,
                                              const int64_t*, int64_t, double, double*, bool,
                                              hipStream_t);
template hipError_t launch_store_field<double>(const void*, const InstDev*, int, int,
                                               const double*, const int64_t*, int64_t, double,
                                               double*, bool, hipStream_t);

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
    if (lam) lam[in.off + i] = out;  // null: the loss alone (fitness evaluations)
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
template hipError_t launch_seed<float>(int, const void*, const InstDev*, int, int, const float*,
                                       const int64_t*, int64_t, const double*, const double*,
                                       const double*, double, void*, double*, double*, int,
                                       hipStream_t);
template hipError_t launch_seed<double>(int, const void*, const InstDev*, int, int,
                                        const double*, const int64_t*, int64_t, const double*,
                                        const double*, const double*, double, void*, double*,
                                        double*, int, hipStream_t);

// ---------------------------------------------------- effective lens
template <typename R>
__global__ void k_lens_prep(const cx<R>* __restrict__ s, cx<R>* __restrict__ wk, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const cx<R> v = s[i];
    wk[i] = cx<R>{v.re * v.re + v.im * v.im, R(0)};
  }
}

__device__ __forceinline__ double lens_profile(double r, const double (*seg)[4], int n) {
  double lo = 0.0;
  for (int j = 0; j < n; ++j) {
    if (r >= lo && r < seg[j][0]) return seg[j][1] * cos(seg[j][2] * r + seg[j][3]);
    lo = seg[j][0];
  }
  return 0.0;
}

template <typename R>
__global__ void k_lens_apply(cx<R>* __restrict__ u, const cx<R>* __restrict__ wd, int64_t n2,
                             LensDev p) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double w_dif = double(wd[i].re) * p.i_ref;
    if (!(w_dif >= p.w_l)) continue;
    const double r = cbrt(fmax(w_dif / p.c1 + p.c2, 0.0));
    const double f_re = lens_profile(r, p.re, p.n_re);
    const double f_im = lens_profile(r, p.im, p.n_im);
    const double a = exp(-f_im);
    const double c = a * cos(f_re), sn = a * sin(f_re);
    const double ur = double(u[i].re), ui = double(u[i].im);
    u[i] = cx<R>{R(ur * c - ui * sn), R(ur * sn + ui * c)};
  }
}

template <typename R>
hipError_t launch_lens_prep(const void* s, void* wk, int64_t n_elem, hipStream_t st) {
  hipLaunchKernelGGL((k_lens_prep<R>), dim3(grid_for(n_elem, 256)), dim3(256), 0, st,
                     static_cast<const cx<R>*>(s), static_cast<cx<R>*>(wk), n_elem);
  return hipGetLastError();
}
template <typename R>
hipError_t launch_lens_apply(void* u, const void* wdif, int64_t n2, const LensDev& p,
                             hipStream_t st) {
  hipLaunchKernelGGL((k_lens_apply<R>), dim3(grid_for(n2, 256)), dim3(256), 0, st,
                     static_cast<cx<R>*>(u), static_cast<const cx<R>*>(wdif), n2, p);
  return hipGetLastError();
}
template hipError_t launch_lens_prep<float>(const void*, void*, int64_t, hipStream_t);
template hipError_t launch_lens_prep<double>(const void*, void*, int64_t, hipStream_t);
template hipError_t launch_lens_apply<float>(void*, const void*, int64_t, const LensDev&,
                                             hipStream_t);
template hipError_t launch_lens_apply<double>(void*, const void*, int64_t, const LensDev&,
                                              hipStream_t);

// Vector-Jacobian product of the lens (G = dL/dRe U + i dL/dIm U).  With
// E = exp(i f(w_dif)) on the active points, z = conj(G_out) U E, q_re =
// -Im z, q_im = -Re z:
//   h    = q_re df_re/dw + q_im df_im/dw,   G_in = conj(E) G_out + 2 Gauss(h) U,
//   dL/dp = sum q_re df_re/dp + q_im df_im/dp  (c1, c2, each segment's
//           amplitude, frequency and phase).
// Fields u, g_out, g_in: complex128 SI of one beam; wk: that beam's slice of
// the work buffer (w_dif in, h I_a out, both real parts, device units).
template <typename R>
__global__ void k_lens_vjp_prep(const double* __restrict__ u, double inv_iref,
                                cx<R>* __restrict__ wk, int64_t n2) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double ur = u[2 * i], ui = u[2 * i + 1];
    wk[i] = cx<R>{R((ur * ur + ui * ui) * inv_iref), R(0)};
  }
}

// segment of r in one part (-1: beyond the last joining point)
__device__ __forceinline__ int lens_segment(double r, const double (*seg)[4], int n) {
  double lo = 0.0;
  for (int j = 0; j < n; ++j) {
    if (r >= lo && r < seg[j][0]) return j;
    lo = seg[j][0];
  }
  return -1;
}

template <typename R>
__global__ void __launch_bounds__(256)
k_lens_vjp_point(const double* __restrict__ u, const double* __restrict__ g_out,
                 cx<R>* __restrict__ wk, double* __restrict__ g_in, int64_t n2, LensDev p,
                 double* __restrict__ part) {
  __shared__ double red[4 * kLensGrads];
  double acc[kLensGrads];
#pragma unroll
  for (int k = 0; k < kLensGrads; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double gr = g_out[2 * i], gi = g_out[2 * i + 1];
    const double w_dif = double(wk[i].re) * p.i_ref;
    if (!(w_dif >= p.w_l)) {
      g_in[2 * i] = gr;
      g_in[2 * i + 1] = gi;
      wk[i] = cx<R>{R(0), R(0)};
      continue;
    }
    const double arg = w_dif / p.c1 + p.c2;
    const double r = cbrt(fmax(arg, 0.0));
    const int jr = lens_segment(r, p.re, p.n_re), ji = lens_segment(r, p.im, p.n_im);
    double cr = 0.0, sr = 0.0, ci = 0.0, si = 0.0;
    if (jr >= 0) sincos(p.re[jr][2] * r + p.re[jr][3], &sr, &cr);
    if (ji >= 0) sincos(p.im[ji][2] * r + p.im[ji][3], &si, &ci);
    const double f_re = (jr >= 0) ? p.re[jr][1] * cr : 0.0;
    const double f_im = (ji >= 0) ? p.im[ji][1] * ci : 0.0;
    const double a = exp(-f_im);
    const double er = a * cos(f_re), ei = a * sin(f_re);
    const double ur = u[2 * i], ui = u[2 * i + 1];
    // z = conj(G) U E
    const double xr = gr * ur + gi * ui, xi = gr * ui - gi * ur;
    const double zr = xr * er - xi * ei, zi = xr * ei + xi * er;
    const double q_re = -zi, q_im = -zr;
    double dp_dr = 0.0;
    if (jr >= 0) {
      const double amp = p.re[jr][1];
      dp_dr += q_re * (-amp * p.re[jr][2] * sr);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j == jr) {
          acc[2 + 3 * j] += q_re * cr;
          acc[3 + 3 * j] += q_re * (-amp * r * sr);
          acc[4 + 3 * j] += q_re * (-amp * sr);
        }
      }
    }
    if (ji >= 0) {
      const double amp = p.im[ji][1];
      dp_dr += q_im * (-amp * p.im[ji][2] * si);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j == ji) {
          acc[26 + 3 * j] += q_im * ci;
          acc[27 + 3 * j] += q_im * (-amp * r * si);
          acc[28 + 3 * j] += q_im * (-amp * si);
        }
      }
    }
    // r = cbrt(w / c1 + c2): dr/dw = 1 / (3 c1 r^2), dr/dc1 = -w / (3 c1^2 r^2),
    // dr/dc2 = 1 / (3 r^2) where the root's argument is positive
    const double inv3r2 = (arg > 0.0) ? 1.0 / (3.0 * r * r) : 0.0;
    acc[0] += dp_dr * inv3r2 * (-w_dif / (p.c1 * p.c1));
    acc[1] += dp_dr * inv3r2;
    const double h = dp_dr * inv3r2 / p.c1;
    g_in[2 * i] = er * gr + ei * gi;
    g_in[2 * i + 1] = er * gi - ei * gr;
    wk[i] = cx<R>{R(h * p.i_ref), R(0)};
  }
  block_reduce<kLensGrads, 256, false>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kLensGrads; ++k) part[int64_t(blockIdx.x) * kLensGrads + k] = acc[k];
  }
}

// G_in += 2 Gauss(h) U (wk: Gauss(h I_a) in its real parts)
template <typename R>
__global__ void k_lens_vjp_final(const double* __restrict__ u, const cx<R>* __restrict__ wk,
                                 double inv_iref, double* __restrict__ g_in, int64_t n2) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double t = 2.0 * double(wk[i].re) * inv_iref;
    g_in[2 * i] += t * u[2 * i];
    g_in[2 * i + 1] += t * u[2 * i + 1];
  }
}

// fixed-order sum of the per-block partials
__global__ void k_lens_vjp_reduce(const double* __restrict__ part, int blocks,
                                  double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= kLensGrads) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += part[int64_t(b) * kLensGrads + k];
  out[k] = s;
}

template <typename R>
hipError_t launch_lens_vjp_prep(const double* u, double i_ref, void* wk, int64_t n2,
                                hipStream_t st) {
  hipLaunchKernelGGL((k_lens_vjp_prep<R>), dim3(grid_for(n2, 256)), dim3(256), 0, st, u,
                     1.0 / i_ref, static_cast<cx<R>*>(wk), n2);
  return hipGetLastError();
}

int lens_vjp_blocks(int64_t n2) { return std::min(grid_for(n2, 256), 512); }

template <typename R>
hipError_t launch_lens_vjp_point(const double* u, const double* g_out, void* wk, double* g_in,
                                 int64_t n2, const LensDev& p, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_lens_vjp_point<R>), dim3(lens_vjp_blocks(n2)), dim3(256), 0, st, u,
                     g_out, static_cast<cx<R>*>(wk), g_in, n2, p, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_lens_vjp_final(const double* u, const void* wk, double i_ref, double* g_in,
                                 int64_t n2, double* part, double* grads, hipStream_t st) {
  hipLaunchKernelGGL((k_lens_vjp_final<R>), dim3(grid_for(n2, 256)), dim3(256), 0, st, u,
                     static_cast<const cx<R>*>(wk), 1.0 / i_ref, g_in, n2);
  hipLaunchKernelGGL(k_lens_vjp_reduce, dim3(1), dim3(64), 0, st, part, lens_vjp_blocks(n2),
                     grads);
  return hipGetLastError();
}
template hipError_t launch_lens_vjp_prep<float>(const double*, double, void*, int64_t,
                                                hipStream_t);
template hipError_t launch_lens_vjp_prep<double>(const double*, double, void*, int64_t,
                                                 hipStream_t);
template hipError_t launch_lens_vjp_point<float>(const double*, const double*, void*, double*,
                                                 int64_t, const LensDev&, double*, hipStream_t);
template hipError_t launch_lens_vjp_point<double>(const double*, const double*, void*, double*,
                                                  int64_t, const LensDev&, double*, hipStream_t);
template hipError_t launch_lens_vjp_final<float>(const double*, const void*, double, double*,
                                                 int64_t, double*, double*, hipStream_t);
template hipError_t launch_lens_vjp_final<double>(const double*, const void*, double, double*,
                                                  int64_t, double*, double*, hipStream_t);

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
template hipError_t launch_copy<float>(const void*, void*, int64_t, hipStream_t);
template hipError_t launch_copy<double>(const void*, void*, int64_t, hipStream_t);

// One thread per (beam, step): fixed-order sum / max over the beam's
// column work items.
// One workgroup per (beam, step): thread t sums the beam's work items
// t, t + 256, ... in order, then a fixed tree across the workgroup, so the
// result depends only on the beam's own item count (a beam in a batch sums
// exactly as it does alone).
__global__ void __launch_bounds__(256)
k_diag_finalize(const double* __restrict__ part, int n_work, const int32_t* __restrict__ wbegin,
                double* __restrict__ diag, int64_t ring0, int64_t cap) {
  __shared__ double red[8];
  const int b = blockIdx.x;
  const int step = blockIdx.y;
  const double* p = part + int64_t(step) * n_work * 2;
  double s[1] = {0.0}, m[1] = {0.0};
  for (int w = wbegin[b] + int(threadIdx.x); w < wbegin[b + 1]; w += 256) {
    s[0] += p[2 * w];
    m[0] = fmax(m[0], p[2 * w + 1]);
  }
  block_reduce<1, 256, false>(s, red);
  block_reduce<1, 256, true>(m, red + 4);
  if (threadIdx.x == 0) {
    const int64_t slot = (ring0 + step) % cap;
    diag[(int64_t(b) * cap + slot) * 2 + 0] = s[0];
    diag[(int64_t(b) * cap + slot) * 2 + 1] = m[0];
  }
}

hipError_t launch_diag_finalize(const double* part, int n_work, const int32_t* wbegin,
                                int n_beams, int steps, double* diag, int64_t ring0,
                                int64_t cap, double, hipStream_t s) {
  if (steps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_finalize, dim3(n_beams, steps), dim3(256), 0, s, part, n_work,
                     wbegin, diag, ring0, cap);
  return hipGetLastError();
}

// Per beam (one workgroup each), the column sums of its rows of a
// [rows][width] array, width <= 8: strided partial sums then a fixed tree.
__global__ void __launch_bounds__(256)
k_reduce_rows(const double* __restrict__ part, int width, const int32_t* __restrict__ begin,
              double* __restrict__ out) {
  __shared__ double red[4 * 8];
  const int b = blockIdx.x;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = begin[b] + int(threadIdx.x); r < begin[b + 1]; r += 256) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < width) s[k] += part[int64_t(r) * width + k];
  }
  block_reduce<8, 256, false>(s, red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < width; ++k) out[int64_t(b) * width + k] = s[k];
  }
}

hipError_t launch_reduce_rows(const double* part, int width, const int32_t* begin,
                              int n_beams, double* out, hipStream_t s) {
  if (width < 1 || width > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_rows, dim3(n_beams), dim3(256), 0, s, part, width, begin, out);
  return hipGetLastError();
}

// sum of (x/scale)^2 in two fixed-order levels
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

// Sum of n <= 256 partials: one per thread, then a fixed tree.
__global__ void __launch_bounds__(256) k_sum_small(const double* part, int n, double* out) {
  __shared__ double red[4];
  double s[1] = {int(threadIdx.x) < n ? part[threadIdx.x] : 0.0};
  block_reduce<1, 256, false>(s, red);
  if (threadIdx.x == 0) out[0] = s[0];
}

hipError_t launch_sumsq(const double* x, int64_t n, double inv_scale, double* partial,
                        double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_part, dim3(256), dim3(256), 0, s, x, n, inv_scale, partial);
  hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(256), 0, s, partial, 256, out);
  return hipGetLastError();
}

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
                        double amp0, int kind, double band_q2, cx<R>* __restrict__ dst) {
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
    // |m|^2 is an exact integer (at most n^2 / 2)
    const double m2 = double(int64_t(mx) * mx + int64_t(my) * my);
    double a;
    if (kind == 1) {
      // Eq. (10) band on the integer mode indices: 0 < |m|^2 <= q2
      a = (m2 > 0.0 && m2 <= band_q2) ? amp0 : 0.0;
    } else {
      a = (m2 > 0.0) ? amp0 * pow(m2, -11.0 / 12.0) : 0.0;
    }
    dst[in.off + i] = {R(a * rr * cs), R(a * rr * sn)};
  }
}

template <typename R>
hipError_t launch_noise(const InstDev* inst, int b, int n, int pair, uint64_t seed,
                        double amp0, int kind, double band_q2, void* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_noise<R>), dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, s,
                     inst, b, pair, uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32), amp0,
                     kind, band_q2, static_cast<cx<R>*>(dst));
  return hipGetLastError();
}
template hipError_t launch_noise<float>(const InstDev*, int, int, int, uint64_t, double, int,
                                        double, void*, hipStream_t);
template hipError_t launch_noise<double>(const InstDev*, int, int, int, uint64_t, double, int,
                                         double, void*, hipStream_t);

// Subharmonic part of the screens, for all beams at once.  Coefficients
// (grid: pairs x beams, one workgroup each): thread t < 8 levels draws mode t
// (level p = t / 8 + 1, cell q = the t % 8-th of the 3 x 3 cells around f = 0
// without the centre, (mx, my) = (q % 3 - 1, q / 3 - 1), spacing df =
// 1 / (3^p L)) from Philox counter (q, p, pair, 1) and stores w = c
// sqrt(density) df; the grid mean of sum w e^{2 pi i f.x} is formed from
// the w (the mean of exp(2 pi i m df x) over the cell-centred grid x_j =
// (j + 1/2 - n/2) L/n is g_p = sin(pi/3^p) / (n sin(pi/(3^p n))) for |m| = 1,
// 1 for m = 0), each mode's share by its own thread, summed in fixed order.
// Tables (grid: blocks x beams): e_p[j] = exp(2 pi i (j + 1/2 - n/2) /
// (3^p n)), the same for rows and columns of the square grid.  Apply (grid:
// blocks x beams, one launch per pair): every point adds Re / Im of
// sum w e_p[col]^mx e_p[row]^my - mean to its two planes, in FP64.
__global__ void __launch_bounds__(256) k_subharm_coef(const SubBeam* __restrict__ beams,
                                                     double* __restrict__ region) {
  __shared__ double sre[8 * kMaxSubharmonicLevels], sim[8 * kMaxSubharmonicLevels];
  const SubBeam sb = beams[blockIdx.y];
  const int pair = blockIdx.x;
  if (pair >= sb.pairs) return;
  const SubharmonicSpec& sp = sb.sp;
  const int n = sb.n;
  const int nm = 8 * sp.levels;
  const int t = threadIdx.x;
  double* blk = region + sb.coef_off + int64_t(kSubPair) * pair;
  if (t < nm) {
    const int p = t / 8 + 1, j = t % 8, q = (j < 4) ? j : j + 1;
    const int mx = q % 3 - 1, my = q / 3 - 1;
    uint32_t c[4] = {uint32_t(q), uint32_t(p), uint32_t(pair), 1u};
    philox4x32_10(c, sb.k0, sb.k1);
    const double u1 = (double(c[0]) + 0.5) * 2.3283064365386962890625e-10;
    const double u2 = (double(c[1]) + 0.5) * 2.3283064365386962890625e-10;
    const double rr = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    double pow3 = 1.0;
    for (int i = 0; i < p; ++i) pow3 *= 3.0;
    const double df = 1.0 / (pow3 * sp.length);
    double a;
    if (sp.kind == 1) {
      // f = m / (3^p L): kappa <= kappa_h reads |m|^2 <= 9^p q2 on the
      // integer indices (one correctly rounded product, 9^p exact)
      const double m2 = double(mx * mx + my * my);
      a = (m2 <= sp.band_q2 * (pow3 * pow3)) ? sqrt(sp.tau * sp.length * sp.length) * df : 0.0;
    } else {
      const double fx = double(mx) * df, fy = double(my) * df;
      a = sqrt(0.023 * pow(sp.r0, -5.0 / 3.0) * pow(hypot(fx, fy), -11.0 / 3.0)) * df;
    }
    const double wr = rr * cs * a, wi = rr * sn * a;
    blk[2 * t] = wr;
    blk[2 * t + 1] = wi;
    const double g = sinpi(1.0 / pow3) / (double(n) * sinpi(1.0 / (pow3 * n)));
    const double f = ((mx == 0) ? 1.0 : g) * ((my == 0) ? 1.0 : g);
    sre[t] = wr * f;
    sim[t] = wi * f;
  }
  __syncthreads();
  if (t == 0) {
    double mre = 0.0, mim = 0.0;
    for (int m = 0; m < nm; ++m) {
      mre += sre[m];
      mim += sim[m];
    }
    blk[128] = mre;
    blk[129] = mim;
  }
}

__global__ void __launch_bounds__(256) k_subharm_table(const SubBeam* __restrict__ beams,
                                                      double* __restrict__ region) {
  const SubBeam sb = beams[blockIdx.y];
  const int n = sb.n;
  const int64_t total = int64_t(sb.sp.levels) * n;
  double* tab = region + sb.tab_off;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < total;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int p = int(k / n), j = int(k - int64_t(p) * n);
    double pow3 = 3.0;
    for (int i = 0; i < p; ++i) pow3 *= 3.0;
    double sn, cs;
    sincospi(2.0 * (double(j) + 0.5 - 0.5 * n) / (pow3 * n), &sn, &cs);
    tab[2 * k] = cs;
    tab[2 * k + 1] = sn;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_subharm_apply(const SubBeam* __restrict__ beams,
                                                      const InstDev* __restrict__ inst, int pair,
                                                      const double* __restrict__ region,
                                                      R* __restrict__ planes) {
  __shared__ double w[kSubPair];
  const SubBeam sb = beams[blockIdx.y];
  if (pair >= sb.pairs) return;
  const InstDev& in = inst[sb.inst];
  const int n = sb.n;
  const int levels = sb.sp.levels;
  const double* blk = region + sb.coef_off + int64_t(kSubPair) * pair;
  for (int k = threadIdx.x; k < 16 * levels; k += blockDim.x) w[k] = blk[k];
  if (threadIdx.x < 2) w[128 + threadIdx.x] = blk[128 + threadIdx.x];
  __syncthreads();
  const double mre = w[128], mim = w[129];
  const double* __restrict__ tab = region + sb.tab_off;
  const int64_t n2 = int64_t(n) * n;
  R* pre = planes + in.screen_off + int64_t(2 * pair) * n2;
  R* pim = pre + n2;
  const bool has_im = 2 * pair + 1 < in.n_screens;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int row = int(i / n), col = int(i - int64_t(row) * n);
    double sre = 0.0, sim = 0.0;
    for (int p = 0; p < levels; ++p) {
      const double xr = tab[2 * (p * n + col)], xi = tab[2 * (p * n + col) + 1];
      const double yr = tab[2 * (p * n + row)], yi = tab[2 * (p * n + row) + 1];
      // e^{i a} for the x-exponents (-1, 0, 1) and y-exponents, combined per
      // cell; cells in the order q = 0..8 without q = 4
      const double exr[3] = {xr, 1.0, xr}, exi[3] = {-xi, 0.0, xi};
      const double eyr[3] = {yr, 1.0, yr}, eyi[3] = {-yi, 0.0, yi};
      const double* wp = w + 16 * p;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int q = (j < 4) ? j : j + 1, ix = q % 3, iy = q / 3;
        const double er = exr[ix] * eyr[iy] - exi[ix] * eyi[iy];
        const double ei = exr[ix] * eyi[iy] + exi[ix] * eyr[iy];
        const double wr = wp[2 * j], wi = wp[2 * j + 1];
        sre += wr * er - wi * ei;
        sim += wr * ei + wi * er;
      }
    }
    pre[i] = R(double(pre[i]) + (sre - mre));
    if (has_im) pim[i] = R(double(pim[i]) + (sim - mim));
  }
}

hipError_t launch_subharmonic_setup(const SubBeam* beams, int n_beams, int max_pairs,
                                    int64_t max_table, double* region, hipStream_t s) {
  if (n_beams <= 0 || max_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_subharm_coef, dim3(max_pairs, n_beams), dim3(256), 0, s, beams, region);
  hipLaunchKernelGGL(k_subharm_table, dim3(grid_for(max_table, 256), n_beams), dim3(256), 0, s,
                     beams, region);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_subharmonic_apply(const SubBeam* beams, int n_beams, const InstDev* inst,
                                    int pair, int64_t max_n2, const double* region, void* planes,
                                    hipStream_t s) {
  if (n_beams <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_subharm_apply<R>), dim3(std::min(grid_for(max_n2, 256), 4096), n_beams),
                     dim3(256), 0, s, beams, inst, pair, region, static_cast<R*>(planes));
  return hipGetLastError();
}
template hipError_t launch_subharmonic_apply<float>(const SubBeam*, int, const InstDev*, int,
                                                    int64_t, const double*, void*, hipStream_t);
template hipError_t launch_subharmonic_apply<double>(const SubBeam*, int, const InstDev*, int,
                                                     int64_t, const double*, void*, hipStream_t);

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
template hipError_t launch_screen_to_f64<float>(const float*, int64_t, double*, hipStream_t);
template hipError_t launch_screen_to_f64<double>(const double*, int64_t, double*, hipStream_t);

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

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

hipError_t launch_block_mean(const double* src, int n, int b, double* dst, hipStream_t s) {
  const int64_t total = int64_t(n / b) * (n / b);
  hipLaunchKernelGGL(k_block_mean, dim3(grid_for(total, 256)), dim3(256), 0, s, src, n, b,
                     dst);
  return hipGetLastError();
}

}  // namespace ssfm
