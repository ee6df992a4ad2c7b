// pass_kernels.hpp -- the row and column pass kernels of the march.
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
// kernel or when the field is read out, so the fields the adjoint needs
// are the march's own state and recording them costs no extra traffic.
//
// Each workgroup owns whole lines: a row workgroup reads and writes LINES
// contiguous rows; a column workgroup reads W = LINES adjacent columns row
// by row.  A thread first issues all of its loads (field points, propagator
// values, twiddles of every stage, turbulence phases) as one batch, then
// runs FFT -> multiply -> inverse FFT with LDS exchanges between radix
// stages only.  The field loads and stores are the only HBM traffic:
// 8 B read + 8 B written per point per pass (complex64).
#pragma once

#include <algorithm>
#include <atomic>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "plans.hpp"
#include "screen.hpp"

namespace ssfm {

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

// Turbulence plane applied after context step `step` (nullptr if none): the
// screen whose step equals the beam's own step index (the context step
// minus the step at which the beam's field was set), by lower-bound search
// of the beam's increasing step list (a workgroup-uniform chain of
// log2(n_screens) scalar loads instead of one per screen).
template <typename R>
__device__ __forceinline__ const R* find_plane(const R* screens, const int64_t* steps,
                                               const InstDev& in, int64_t step) {
  if (step < 0 || !(in.terms & T_TURB) || in.n_screens <= 0 || screens == nullptr)
    return nullptr;
  step -= in.step_base;
  const int64_t* st = steps + in.steps_off;
  int lo = 0, hi = in.n_screens - 1;
  if (step < st[lo] || step > st[hi]) return nullptr;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] < step)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (st[lo] != step) return nullptr;
  return screens + in.screen_off + int64_t(lo) * in.n * in.n;
}

// Uniform reads of the tables no kernel writes (work list, beam table,
// screen step lists) through the constant address space: scalar loads,
// counted apart from the vector loads, so waiting for them never waits for
// the field loads in flight.
template <typename T>
using const_as4 = const __attribute__((address_space(4))) T;
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  T out;
  const_as4<uint32_t>* src =
      reinterpret_cast<const_as4<uint32_t>*>(reinterpret_cast<uintptr_t>(p));
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) dst[i] = src[i];
  return out;
}

// find_plane with the step list read through scalar loads.
template <typename R>
__device__ __forceinline__ const R* find_plane_uniform(const R* screens, const int64_t* steps,
                                                       const InstDev& in, int64_t step) {
  if (step < 0 || !(in.terms & T_TURB) || in.n_screens <= 0 || screens == nullptr)
    return nullptr;
  step -= in.step_base;
  const int64_t* st = steps + in.steps_off;
  int lo = 0, hi = in.n_screens - 1;
  if (step < load_uniform(st + lo) || step > load_uniform(st + hi)) return nullptr;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (load_uniform(st + mid) < step)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (load_uniform(st + lo) != step) return nullptr;
  return screens + in.screen_off + int64_t(lo) * in.n * in.n;
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

// dz G(x) of the finite-difference scheme, x = |u|^2 / I_a: the generators
// of the Kerr, plasma and multiphoton terms (each split-step screen term is
// the exact solution of du/dz = G u over one step).
template <typename R>
__device__ __forceinline__ void fd_generator(const ScreenConst<R>& s, R x, R& gr, R& gi) {
  const unsigned tm = s.terms;
  R xk1 = R(0);
  if (tm & (T_MPA | T_PLASMA)) xk1 = ipow(x, s.K - 1);
  gr = R(0);
  gi = R(0);
  if (tm & T_KERR) gi += s.cK * x;
  if (tm & T_PLASMA) gi -= s.cK * x * (R(1) - rcp(R(1) + xk1));
  if (tm & T_MPA) gr -= s.cM * s.inv2k1 * xk1;
}

// A line transform of a row pass: twiddles from registers / the table, or
// (QTW plans) from the quarter table in LDS.
template <typename R, class P, int DIR, class Lds>
__device__ __forceinline__ void row_fft(cx<R>* v, int t, const Lds& lds, const cx<R>* wt,
                                        const cx<R>* __restrict__ tw, const cx<R>* twq) {
  if constexpr (P::QTW)
    fft_line_qtw<R, P, DIR>(v, t, lds, twq);
  else
    fft_line<R, P, DIR>(v, t, lds, wt, tw);
}

template <class P>
constexpr int tw_regs() {
  return TwCount<P>::value > 0 ? TwCount<P>::value : 1;
}

// ------------------------------------------------------------ row pass
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS)
    __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? P::WAVES_PER_EU : 1))) k_row(PassArgs<R> a) {
  constexpr int N = P::N, T = P::T, E = P::E;
  using L = LdsLineMajor<R, N>;
  __shared__ cx<R> lds_mem[P::LINES * L::LINE];
  __shared__ cx<R> twq[P::QTW ? qtw_entries<N>(typename P::radices{}) : 1];
  __shared__ double red[((P::THREADS + 63) / 64) * 8];

  const WorkItem w = a.work[blockIdx.x];
  if (w.inst < 0) return;
  const InstDev& in = a.inst[w.inst];
  if constexpr (KIND == ROW_INV) {
    if (2 * a.pair >= in.n_screens || !(in.terms & T_TURB)) return;
  }
  // screen constants fetched with the first loads, not after the FFT input
  const ScreenConst<R> sc = screen_const<R>(in);
  const int line = threadIdx.x / T;
  const int t = threadIdx.x - line * T;
  const int row = w.line0 + line;
  // uniform base of this workgroup's rows; per-thread 32-bit offsets
  const int64_t wbase = in.off + int64_t(w.line0) * N;
  const uint32_t toff = uint32_t(line) * N + uint32_t(t);
  const L lds{lds_mem + line * L::LINE};
  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ tw = tables + in.tw_off;
  const cx<R>* __restrict__ prop = tables + in.prop_off;
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src) + wbase;
  cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst) + wbase;

  // one batch of loads: field, propagator, twiddles (and, for the adjoint,
  // the stored pre-screen field and turbulence phases)
  cx<R> v[E];
  cx<R> pr[E];
  cx<R> wt[tw_regs<P>()];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[toff + uint32_t(T * e)];
  if constexpr (KIND != ROW_INV && KIND != ROW_FD && !P::LATE_PROP) {
#pragma unroll
    for (int e = 0; e < E; ++e) pr[e] = prop[t + T * e];
  }
  load_twiddles<R, P>(wt, t, tw);
  // quarter twiddle table (QTW plans); the first exchange's barrier orders
  // it before the first twiddle is read
  if constexpr (P::QTW)
    fill_qtw_tables<R, N, P::THREADS>(twq, int(threadIdx.x), tw, typename P::radices{});
  cx<R> sv[KIND == ROW_ADJ ? E : 1];
  R ph[(KIND == ROW_ADJ || KIND == ROW_FWD) ? E : 1];
  const R* plane = nullptr;
  if constexpr (KIND == ROW_ADJ || KIND == ROW_FWD)
    plane = find_plane(a.screens, a.screen_steps, in, a.step);
  // turbulence phases (forward and adjoint) and the stored pre-screen field
  // (adjoint) of points [e0, e1), needed by the screen on load (forward) or
  // by the adjoint screen after the inverse FFT (adjoint; with late loads
  // it reads them there, chunk by chunk, so they are not held through the
  // transforms)
  auto load_screen_inputs = [&](int e0, int e1) {
    if (plane) {
      const R* pw = plane + int64_t(w.line0) * N;
#pragma unroll
      for (int e = e0; e < e1; ++e) ph[e] = pw[toff + uint32_t(T * e)];
    } else {
#pragma unroll
      for (int e = e0; e < e1; ++e) ph[e] = R(0);
    }
    if constexpr (KIND == ROW_ADJ) {
      if (a.step >= 0) {
        const cx<R>* __restrict__ svp = static_cast<const cx<R>*>(a.aux) + wbase;
#pragma unroll
        for (int e = e0; e < e1; ++e) sv[e] = svp[toff + uint32_t(T * e)];
      }
    }
  };
  constexpr bool kLateScreenInputs = (KIND == ROW_ADJ) && P::LATE_PROP;
  if constexpr ((KIND == ROW_ADJ || KIND == ROW_FWD) && !kLateScreenInputs) load_screen_inputs(0, E);
  (void)row;

  if constexpr (KIND == ROW_FD) {
    // finite-difference iteration: v is Ubar row-transformed (the column pass
    // applied the solve and both 1/N), or U itself when the step starts
    cx<R>* __restrict__ st = static_cast<cx<R>*>(a.state) + wbase;
    cx<R> un[E];
#pragma unroll
    for (int e = 0; e < E; ++e) un[e] = st[toff + uint32_t(T * e)];
    if (a.flags & FD_SPECTRAL) row_fft<R, P, +1>(v, t, lds, wt, tw, twq);
    if (a.flags & FD_FINISH) {
      // U+ = 2 Ubar - U, its power partials; it is the next step's U and
      // its first Ubar
      double s[1] = {0.0}, m[1] = {0.0};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        v[e] = {R(2) * v[e].re - un[e].re, R(2) * v[e].im - un[e].im};
        st[toff + uint32_t(T * e)] = v[e];
        const double x = double(v[e].re) * double(v[e].re) + double(v[e].im) * double(v[e].im);
        s[0] += x;
        m[0] = fmax(m[0], x);
        un[e] = v[e];
      }
      if (a.part != nullptr) {
        block_reduce<1, P::THREADS, false>(s, red);
        __syncthreads();
        block_reduce<1, P::THREADS, true>(m, red + ((P::THREADS + 63) / 64));
        if (threadIdx.x == 0) {
          a.part[int64_t(w.widx) * 2 + 0] = s[0];
          a.part[int64_t(w.widx) * 2 + 1] = m[0];
        }
      }
      if (a.flags & FD_LAST) return;
    }
    // right-hand side U + (dz/2) G(J) Ubar, J = (|2 Ubar - U|^2 + |U|^2) / 2
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const R dr = R(2) * v[e].re - un[e].re, di = R(2) * v[e].im - un[e].im;
      const R j = R(0.5) * (dr * dr + di * di + un[e].re * un[e].re + un[e].im * un[e].im);
      R gr, gi;
      fd_generator<R>(sc, j, gr, gi);
      gr *= R(0.5);
      gi *= R(0.5);
      v[e] = {un[e].re + (gr * v[e].re - gi * v[e].im), un[e].im + (gr * v[e].im + gi * v[e].re)};
    }
    row_fft<R, P, -1>(v, t, lds, wt, tw, twq);
#pragma unroll
    for (int e = 0; e < E; ++e) dst[toff + uint32_t(T * e)] = v[e];
    return;
  }

  if constexpr (KIND == ROW_FWD) {
    if (a.step >= 0) screen_apply_n<R, E>(sc, v, ph);
  }

  if constexpr (KIND == ROW_INV) {
    row_fft<R, P, +1>(v, t, lds, wt, tw, twq);
  } else {
    row_fft<R, P, -1>(v, t, lds, wt, tw, twq);
    if constexpr (P::LATE_PROP) {
      // loaded after the forward FFT: not held in registers through it
#pragma unroll
      for (int e = 0; e < E; ++e) pr[e] = prop[t + T * e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = (KIND == ROW_ADJ) ? cmulc(v[e], pr[e]) : cmul(v[e], pr[e]);
    row_fft<R, P, +1>(v, t, lds, wt, tw, twq);
  }

  if constexpr (KIND == ROW_ADJ) {
    if (a.step >= 0) {
      double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      constexpr int AC = (E % P::ADJ_BATCH == 0) ? P::ADJ_BATCH : E;  // points per batch
      // late inputs: each batch's stored field and phases are requested one
      // batch ahead, so their latency overlaps the previous batch's screen
      if constexpr (kLateScreenInputs) load_screen_inputs(0, AC);
#pragma unroll
      for (int c = 0; c < E; c += AC) {
        if constexpr (kLateScreenInputs) {
          if (c + AC < E) load_screen_inputs(c + AC, c + 2 * AC);
        }
        screen_adjoint_n<R, AC>(sc, sv + c, v + c, ph + c, plane != nullptr, g);
        // the batch's cotangent is stored now, not held through the
        // reduction (offset laundered: formed here, not kept from the loads)
        uint32_t to = toff;
        asm volatile("" : "+v"(to));
#pragma unroll
        for (int e = c; e < c + AC; ++e) dst[to + uint32_t(T * e)] = v[e];
      }
      if (in.terms & T_ANSATZ) {
        block_reduce<8, P::THREADS, false>(g, red);
        if (threadIdx.x == 0) {
          double* acc = a.part + int64_t(w.widx) * 8;
#pragma unroll
          for (int p = 0; p < 8; ++p) acc[p] += g[p];
        }
      }
      return;
    }
  }

#pragma unroll
  for (int e = 0; e < E; ++e) dst[toff + uint32_t(T * e)] = v[e];
}

// ------------------------------------------------- pipelined row pass
// Forward and adjoint row passes of a pipelined plan.  The grid holds as
// many workgroups as are resident at once (a multiple of 8, so that every
// item a workgroup takes runs on its own XCD); workgroup g takes items g,
// g + gridDim.x, ... of the work list.  While it transforms one row, the
// field loads of its next row are in flight, so the memory latency of a
// row overlaps the arithmetic of the previous one.  The twiddles are copied
// into LDS once per workgroup (stage by stage in the order they are read)
// and the propagator is held in registers, reloaded only when the beam
// changes.  The next row's loads are issued on every iteration (after the
// last row, every lane reads that row's first point): loads issued on one
// path only would make the compiler wait for every load in flight before
// the transform.  The forward pass loads a row's turbulence phases when
// its iteration starts, ahead of the next row's field; the adjoint pass
// loads the stored pre-screen field and the phases after its inverse
// transform, when they are needed.  These kernels carry no library sine and
// cosine: with precise math on, the passes run k_row.  Per row the
// arithmetic and its order are those of k_row with the same radices and
// threads (screens run over batches of points, point by point in the same
// order); the two kernels agree to rounding (the compiler may fuse a
// multiply and an add in one and not the other).
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS)
    __attribute__((amdgpu_waves_per_eu(P::WAVES_PER_EU))) k_row_pipe(PassArgs<R> a) {
  static_assert(KIND == ROW_FWD || KIND == ROW_ADJ, "pipelined row pass: forward or adjoint");
  static_assert(P::LINES == 1, "one row per item");
  constexpr int N = P::N, T = P::T, E = P::E;
  constexpr bool ADJ = KIND == ROW_ADJ;
  constexpr int SB = (E % 4 == 0) ? 4 : E;  // forward screen batch
  using L = LdsLineMajor<R, N>;
  __shared__ cx<R> lds_mem[L::LINE];
  __shared__ cx<R> twl[lds_tw_entries<N>(typename P::radices{})];
  __shared__ double red[((P::THREADS + 63) / 64) * 8];
  const L lds{lds_mem};
  const int t0 = threadIdx.x;
  const int nb = a.n_work, G = gridDim.x;
  auto next_item = [&](int i) {
    while (i < nb && load_uniform(a.work + i).inst < 0) i += G;
    return i;
  };
  int it = next_item(int(blockIdx.x));
  if (it >= nb) return;

  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src);
  const cx<R>* __restrict__ aux = static_cast<const cx<R>*>(a.aux);
  cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst);

  WorkItem w = load_uniform(a.work + it);
  int64_t base = load_uniform(&a.inst[w.inst].off) + int64_t(w.line0) * N;
  cx<R> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[base + uint32_t(t0 + T * e)];
  int64_t prop_off = load_uniform(&a.inst[w.inst].prop_off);
  int64_t tw_off = load_uniform(&a.inst[w.inst].tw_off);
  cx<R> pr[E];
#pragma unroll
  for (int e = 0; e < E; ++e) pr[e] = tables[prop_off + t0 + T * e];
  fill_lds_twiddles<R, N, P::THREADS>(twl, t0, tables + tw_off, typename P::radices{});

  for (;;) {
    // the thread index laundered per iteration: addresses derived from it
    // are recomputed in the loop instead of held in registers across it
    int t = t0;
    asm volatile("" : "+v"(t));
    const InstDev in = load_uniform(a.inst + w.inst);
    ScreenConst<R> sc = screen_const<R>(in);
    sc.terms &= ~unsigned(T_PRECISE);
    const R* plane = find_plane_uniform(a.screens, a.screen_steps, in, a.step);
    // this row's turbulence phases and (adjoint) stored pre-screen field,
    // ahead of the next row's field
    R ph[E];
    if (plane) {
      const R* pw = plane + int64_t(w.line0) * N;
#pragma unroll
      for (int e = 0; e < E; ++e) ph[e] = pw[uint32_t(t + T * e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) ph[e] = R(0);
    }
    cx<R> sv[ADJ ? E : 1];
    if constexpr (ADJ) {
      if (a.step >= 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) sv[e] = aux[base + uint32_t(t + T * e)];
      }
    }
    // the next row's field
    const int nit = next_item(it + G);
    const bool more = nit < nb;
    const WorkItem wn = more ? load_uniform(a.work + nit) : w;
    const int64_t base_n =
        more ? load_uniform(&a.inst[wn.inst].off) + int64_t(wn.line0) * N : base;
    const uint32_t live = more ? 0xffffffffu : 0u;
    cx<R> vn[E];
#pragma unroll
    for (int e = 0; e < E; ++e) vn[e] = src[base_n + (uint32_t(t + T * e) & live)];

    if constexpr (!ADJ) {
      if (a.step >= 0) {
#pragma unroll
        for (int c = 0; c < E; c += SB) screen_apply_n<R, SB>(sc, v + c, ph + c);
      }
    }
    // every wave has read the previous row out of LDS (and the twiddles
    // are in place)
    __syncthreads();
    fft_line_ltw<R, P, -1>(v, t, lds, twl);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ADJ ? cmulc(v[e], pr[e]) : cmul(v[e], pr[e]);
    fft_line_ltw<R, P, +1>(v, t, lds, twl);
    bool stored = false;
    if constexpr (ADJ) {
      if (a.step >= 0) {
        double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        constexpr int AC = (E % P::ADJ_BATCH == 0) ? P::ADJ_BATCH : E;
#pragma unroll
        for (int c = 0; c < E; c += AC) {
          screen_adjoint_n<R, AC, true>(sc, sv + c, v + c, ph + c, plane != nullptr, g);
          // the batch's cotangent is stored now, not held through the
          // reduction
#pragma unroll
          for (int e = c; e < c + AC; ++e) dst[base + uint32_t(t + T * e)] = v[e];
          // one batch at a time: the scheduler does not interleave batches
          __builtin_amdgcn_sched_barrier(0);
        }
        stored = true;
        if (in.terms & T_ANSATZ) {
          // the scratch's address from a laundered zero, so its per-wave
          // slot addresses are not held in registers across the loop
          int z = 0;
          asm volatile("" : "+v"(z));
          block_reduce<8, P::THREADS, false>(g, red + z);
          if (threadIdx.x == 0) {
            double* acc = a.part + int64_t(w.widx) * 8;
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] += g[p];
          }
        }
      }
    }
    if (!stored) {
#pragma unroll
      for (int e = 0; e < E; ++e) dst[base + uint32_t(t + T * e)] = v[e];
    }
    if (!more) break;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vn[e];
    w = wn;
    base = base_n;
    it = nit;
    const int64_t po = load_uniform(&a.inst[w.inst].prop_off);
    if (po != prop_off) {
      prop_off = po;
#pragma unroll
      for (int e = 0; e < E; ++e) pr[e] = tables[prop_off + t + T * e];
    }
    const int64_t to = load_uniform(&a.inst[w.inst].tw_off);
    if (to != tw_off) {
      tw_off = to;
      __syncthreads();
      fill_lds_twiddles<R, N, P::THREADS>(twl, t, tables + tw_off, typename P::radices{});
    }
  }
}

// --------------------------------------------------------- column pass
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS)
    __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? P::WAVES_PER_EU : 1))) k_col(PassArgs<R> a) {
  constexpr int N = P::N, T = P::T, E = P::E, W = P::LINES;
  using L = LdsPointMajor<R, W, P::PA, P::PB>;
  __shared__ cx<R> lds_mem[L::size(N)];
  __shared__ double red[((P::THREADS + 63) / 64) * 2];

  const WorkItem w = a.work[blockIdx.x];
  if (w.inst < 0) return;
  const InstDev& in = a.inst[w.inst];
  if constexpr (KIND == COL_INV) {
    if (2 * a.pair >= in.n_screens || !(in.terms & T_TURB)) return;
  }
  const ScreenConst<R> sc = screen_const<R>(in);
  const int c = threadIdx.x % W;
  const int t = threadIdx.x / W;
  // uniform base (first column of the tile); per-thread 32-bit offsets
  const int64_t wbase = in.off + w.line0;
  const uint32_t toff = uint32_t(t) * N + uint32_t(c);
  constexpr uint32_t ESTRIDE = uint32_t(T) * N;
  const L lds{lds_mem + c};
  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ tw = tables + in.tw_off;
  const cx<R>* __restrict__ prop = tables + in.prop_off;
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src) + wbase;

  cx<R> v[E];
  cx<R> pr[E];
  cx<R> wt[tw_regs<P>()];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[toff + ESTRIDE * e];
  if constexpr (KIND != COL_INV && !P::LATE_PROP) {
#pragma unroll
    for (int e = 0; e < E; ++e) pr[e] = prop[t + T * e];
  }
  load_twiddles<R, P>(wt, t, tw);

  if constexpr (KIND == COL_INV) {
    fft_line<R, P, +1>(v, t, lds, wt, tw);
  } else {
    fft_line<R, P, -1>(v, t, lds, wt, tw);
    if constexpr (P::LATE_PROP) {
      // loaded after the forward FFT: not held in registers through it
#pragma unroll
      for (int e = 0; e < E; ++e) pr[e] = prop[t + T * e];
    }
    if constexpr (KIND == COL_FD) {
      // (1 - (i dz/4k0) Lap_h)^-1 = 1 / (1 + i (d[kx] + d[ky])) with the 1/N^2
      // of both inverse DFTs; the table holds d[m] = (dz/4k0)(4/dx^2)
      // sin^2(pi m / N) in its real parts
      const R dkx = prop[w.line0 + c].re;
      const R inv_n2 = R(1) / (R(N) * R(N));
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const R sm = dkx + pr[e].re;
        const R den = inv_n2 / (R(1) + sm * sm);
        v[e] = cmul(v[e], cx<R>{den, -sm * den});
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[e] = (KIND == COL_ADJ) ? cmulc(v[e], pr[e]) : cmul(v[e], pr[e]);
    }
    fft_line<R, P, +1>(v, t, lds, wt, tw);
  }

  if constexpr (KIND == COL_INV) {
    // screen pair: real part -> plane 2p, imaginary part -> plane 2p+1
    R* pre = a.planes_out + in.screen_off + int64_t(2 * a.pair) * N * N + w.line0;
    R* pim = pre + int64_t(N) * N;
    const bool has_im = 2 * a.pair + 1 < in.n_screens;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      pre[toff + ESTRIDE * e] = v[e].re;
      if (has_im) pim[toff + ESTRIDE * e] = v[e].im;
    }
    return;
  } else {
    cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst) + wbase;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[toff + ESTRIDE * e] = v[e];
  }

  if constexpr (KIND == COL_FWD) {
    if (a.part != nullptr) {
      double s[1] = {0.0}, m[1] = {0.0};
      R x[E], a2[E];
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = v[e].re * v[e].re + v[e].im * v[e].im;
      if (a.flags & 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) a2[e] = R(1);
      } else {
        screen_amp2_n<R, E>(sc, x, a2);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double xa = double(x[e]) * double(a2[e]);
        s[0] += xa;
        m[0] = fmax(m[0], xa);
      }
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

// ---------------------------------------------- pipelined column pass
// Forward and adjoint column passes of a pipelined plan, organised like
// k_row_pipe: a resident grid, workgroup g taking column tiles g,
// g + gridDim.x, ... (a multiple of 8: an XCD's workgroups hold adjacent
// tiles at any time, so the rows of neighbouring tiles meet in its L2),
// the next tile's field loads in flight while the current tile is
// transformed.  Twiddles come from LDS: the stage tables, or (QTW plans,
// whose tile fills the LDS) a quarter table; the propagator is held in
// registers, or (QTW) loaded after the forward transform.
template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS)
    __attribute__((amdgpu_waves_per_eu(P::WAVES_PER_EU))) k_col_pipe(PassArgs<R> a) {
  static_assert(KIND == COL_FWD || KIND == COL_ADJ, "pipelined column pass: forward or adjoint");
  constexpr int N = P::N, T = P::T, E = P::E, W = P::LINES;
  constexpr bool ADJ = KIND == COL_ADJ;
  constexpr bool QTW = P::QTW;
  constexpr int SB = (E % 4 == 0) ? 4 : E;  // power-partial batch
  constexpr uint32_t ESTRIDE = uint32_t(T) * N;
  using L = LdsPointMajor<R, W, P::PA, P::PB>;
  __shared__ cx<R> lds_mem[L::size(N)];
  __shared__ cx<R> twl[QTW ? qtw_entries<N>(typename P::radices{}) : lds_tw_entries<N>(typename P::radices{})];
  __shared__ double red[((P::THREADS + 63) / 64) * 2];
  const int nb = a.n_work, G = gridDim.x;
  auto next_item = [&](int i) {
    while (i < nb && load_uniform(a.work + i).inst < 0) i += G;
    return i;
  };
  int it = next_item(int(blockIdx.x));
  if (it >= nb) return;

  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src);
  cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst);
  const int c0 = threadIdx.x % W, t0 = threadIdx.x / W;
  const uint32_t toff0 = uint32_t(t0) * N + uint32_t(c0);
  auto fill_twiddles = [&](int64_t off) {
    if constexpr (QTW)
      fill_qtw_tables<R, N, P::THREADS>(twl, int(threadIdx.x), tables + off,
                                        typename P::radices{});
    else
      fill_lds_twiddles<R, N, P::THREADS>(twl, int(threadIdx.x), tables + off,
                                          typename P::radices{});
  };

  WorkItem w = load_uniform(a.work + it);
  int64_t base = load_uniform(&a.inst[w.inst].off) + w.line0;
  cx<R> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[base + toff0 + ESTRIDE * e];
  int64_t prop_off = load_uniform(&a.inst[w.inst].prop_off);
  int64_t tw_off = load_uniform(&a.inst[w.inst].tw_off);
  cx<R> pr[E];
  if constexpr (!QTW) {
#pragma unroll
    for (int e = 0; e < E; ++e) pr[e] = tables[prop_off + t0 + T * e];
  }
  fill_twiddles(tw_off);

  for (;;) {
    // thread coordinates laundered per iteration (addresses recomputed in
    // the loop instead of held across it)
    int c = c0, t = t0;
    asm volatile("" : "+v"(c), "+v"(t));
    const uint32_t toff = uint32_t(t) * N + uint32_t(c);
    const L lds{lds_mem + c};
    // the next tile's field
    const int nit = next_item(it + G);
    const bool more = nit < nb;
    const WorkItem wn = more ? load_uniform(a.work + nit) : w;
    const int64_t base_n = more ? load_uniform(&a.inst[wn.inst].off) + wn.line0 : base;
    const uint32_t live = more ? 0xffffffffu : 0u;
    cx<R> vn[E];
#pragma unroll
    for (int e = 0; e < E; ++e) vn[e] = src[base_n + ((toff + ESTRIDE * e) & live)];

    // every wave has read the previous tile out of LDS (and the twiddles
    // are in place)
    __syncthreads();
    if constexpr (QTW) {
      fft_line_qtw<R, P, -1>(v, t, lds, twl);
      // after the transform: not held through it (its wait also covers the
      // next tile's loads, issued a transform earlier)
#pragma unroll
      for (int e = 0; e < E; ++e) pr[e] = tables[prop_off + t + T * e];
    } else {
      fft_line_ltw<R, P, -1>(v, t, lds, twl);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ADJ ? cmulc(v[e], pr[e]) : cmul(v[e], pr[e]);
    if constexpr (QTW)
      fft_line_qtw<R, P, +1>(v, t, lds, twl);
    else
      fft_line_ltw<R, P, +1>(v, t, lds, twl);
#pragma unroll
    for (int e = 0; e < E; ++e) dst[base + toff + ESTRIDE * e] = v[e];

    if constexpr (!ADJ) {
      if (a.part != nullptr) {
        const InstDev in = load_uniform(a.inst + w.inst);
        ScreenConst<R> sc = screen_const<R>(in);
        double s[1] = {0.0}, m[1] = {0.0};
#pragma unroll
        for (int b = 0; b < E; b += SB) {
          R x[SB], a2[SB];
#pragma unroll
          for (int e = 0; e < SB; ++e) x[e] = v[b + e].re * v[b + e].re + v[b + e].im * v[b + e].im;
          if (a.flags & 1) {
#pragma unroll
            for (int e = 0; e < SB; ++e) a2[e] = R(1);
          } else {
            screen_amp2_n<R, SB>(sc, x, a2);
          }
#pragma unroll
          for (int e = 0; e < SB; ++e) {
            const double xa = double(x[e]) * double(a2[e]);
            s[0] += xa;
            m[0] = fmax(m[0], xa);
          }
        }
        int z = 0;
        asm volatile("" : "+v"(z));
        double* rp = red + z;
        block_reduce<1, P::THREADS, false>(s, rp);
        __syncthreads();
        block_reduce<1, P::THREADS, true>(m, rp + ((P::THREADS + 63) / 64));
        if (threadIdx.x == 0) {
          a.part[int64_t(w.widx) * 2 + 0] = s[0];
          a.part[int64_t(w.widx) * 2 + 1] = m[0];
        }
      }
    }
    if (!more) break;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = vn[e];
    w = wn;
    base = base_n;
    it = nit;
    const int64_t po = load_uniform(&a.inst[w.inst].prop_off);
    if (po != prop_off) {
      prop_off = po;
      if constexpr (!QTW) {
#pragma unroll
        for (int e = 0; e < E; ++e) pr[e] = tables[prop_off + t + T * e];
      }
    }
    const int64_t to = load_uniform(&a.inst[w.inst].tw_off);
    if (to != tw_off) {
      tw_off = to;
      __syncthreads();
      fill_twiddles(tw_off);
    }
  }
}

// -------------------------------------------------------------- launch
// With ev, the launch carries start/stop events on its own dispatch (timing
// of the kernel alone, no separate marker packets).  A plan whose LDS tile
// does not fit a workgroup at this precision is not built for it.
// Workgroups of a persistent launch: as many as are resident at once (the
// runtime's occupancy for the kernel times the compute units), rounded down
// to a multiple of 8, and no more than the items.
inline int resident_grid(int per_cu, int items) {
  // compute units of the current device, looked up once per device
  constexpr int kMaxDevices = 64;
  static std::atomic<int> cu_count[kMaxDevices] = {};
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) cus = cu_count[dev];
  if (cus < 1) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 1;
    else if (dev >= 0 && dev < kMaxDevices)
      cu_count[dev] = cus;
  }
  const int g = std::max(8, per_cu * cus / 8 * 8);
  return std::min(g, items);
}

// Column passes of half-exchange plans (their kernels are compiled in a
// unit of their own, pass_col_hx_f32.hip).
template <typename R, class P, int KIND>
hipError_t launch_hx(int n_blocks, const PassArgs<R>& a, hipStream_t s, const LaunchEv* ev);

template <typename R, class P, int KIND>
hipError_t launch_one(int n_blocks, const PassArgs<R>& a, hipStream_t s, const LaunchEv* ev) {
  if constexpr (!plan_fits<R, P>(is_col_kind(KIND))) {
    return hipErrorInvalidValue;
  } else if constexpr (P::HX) {
    return launch_hx<R, P, KIND>(n_blocks, a, s, ev);
  } else if constexpr (P::PIPE && (KIND == ROW_FWD || KIND == ROW_ADJ)) {
    if (a.precise) {
      if (ev)
        hipExtLaunchKernelGGL((k_row<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s,
                              ev->start, ev->stop, 0, a);
      else
        hipLaunchKernelGGL((k_row<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
      return hipGetLastError();
    }
    static const int per_cu = [] {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &b, reinterpret_cast<const void*>(k_row_pipe<R, P, KIND>), P::THREADS, 0) !=
              hipSuccess ||
          b < 1)
        b = 1;
      return b;
    }();
    PassArgs<R> b = a;
    b.n_work = n_blocks;
    const int grid = resident_grid(per_cu, n_blocks);
    if (ev)
      hipExtLaunchKernelGGL((k_row_pipe<R, P, KIND>), dim3(grid), dim3(P::THREADS), 0, s,
                            ev->start, ev->stop, 0, b);
    else
      hipLaunchKernelGGL((k_row_pipe<R, P, KIND>), dim3(grid), dim3(P::THREADS), 0, s, b);
  } else if constexpr (P::PIPE && (KIND == COL_FWD || KIND == COL_ADJ)) {
    static const int per_cu = [] {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &b, reinterpret_cast<const void*>(k_col_pipe<R, P, KIND>), P::THREADS, 0) !=
              hipSuccess ||
          b < 1)
        b = 1;
      return b;
    }();
    PassArgs<R> b = a;
    b.n_work = n_blocks;
    const int grid = resident_grid(per_cu, n_blocks);
    if (ev)
      hipExtLaunchKernelGGL((k_col_pipe<R, P, KIND>), dim3(grid), dim3(P::THREADS), 0, s,
                            ev->start, ev->stop, 0, b);
    else
      hipLaunchKernelGGL((k_col_pipe<R, P, KIND>), dim3(grid), dim3(P::THREADS), 0, s, b);
  } else if constexpr (is_col_kind(KIND)) {
    if (ev)
      hipExtLaunchKernelGGL((k_col<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s,
                            ev->start, ev->stop, 0, a);
    else
      hipLaunchKernelGGL((k_col<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
  } else {
    if (ev)
      hipExtLaunchKernelGGL((k_row<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s,
                            ev->start, ev->stop, 0, a);
    else
      hipLaunchKernelGGL((k_row<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
  }
  return hipGetLastError();
}

template <typename R, int KIND>
hipError_t launch_row_kind(int n, int v, int nb, const PassArgs<R>& a, hipStream_t s,
                           const LaunchEv* ev) {
#define SSFM_RCASE(NN, VV, ...) \
  if (n == NN && v == VV)       \
    return launch_one<R, typename RowPlanSel<NN, VV>::P, KIND>(nb, a, s, ev);
  SSFM_ROW_PLANS(SSFM_RCASE)
#undef SSFM_RCASE
  return hipErrorInvalidValue;
}

template <typename R, int KIND>
hipError_t launch_col_kind(int n, int v, int nb, const PassArgs<R>& a, hipStream_t s,
                           const LaunchEv* ev) {
#define SSFM_CCASE(NN, VV, ...) \
  if (n == NN && v == VV)       \
    return launch_one<R, typename ColPlanSel<NN, VV>::P, KIND>(nb, a, s, ev);
  SSFM_COL_PLANS(SSFM_CCASE)
#undef SSFM_CCASE
  return hipErrorInvalidValue;
}

// Per-unit entry points (defined in pass_{row,col}_{f32,f64}.hip).
template <typename R>
hipError_t launch_row(int kind, int n, int v, int nb, const PassArgs<R>& a, hipStream_t s,
                      const LaunchEv* ev);
template <typename R>
hipError_t launch_col(int kind, int n, int v, int nb, const PassArgs<R>& a, hipStream_t s,
                      const LaunchEv* ev);

}  // namespace ssfm
