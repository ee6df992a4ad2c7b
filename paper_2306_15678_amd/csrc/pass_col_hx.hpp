// pass_col_hx.hpp -- column passes whose tile exchanges through half the LDS.
//
// The same column pass as k_col (Eq. (1) split into its row and column
// factors; this is the column factor F_y^-1 P_y F_y, with the FP64 power
// partials of the forward pass), for tiles of W adjacent columns whose
// full LDS tile would leave room for one workgroup per compute unit only.
// The transforms exchange through N/2 points of the tile (fft_line_hx) and
// read their twiddles from a quarter table and the second stage's table in
// LDS, so the workgroup needs a little under half the LDS and two of them
// share a compute unit: the loads,
// LDS exchanges and arithmetic of one overlap those of the other.  The
// propagator is read after the forward transform; the inverse transform's
// outputs are stored (and, forward, summed into the power partials) one
// last-stage butterfly at a time.  Compiled in a unit of its own.
#pragma once

#include "pass_kernels.hpp"

namespace ssfm {

template <typename R, class P, int KIND>
__global__ void __launch_bounds__(P::THREADS)
    __attribute__((amdgpu_waves_per_eu(P::WAVES_PER_EU))) k_col_hx(PassArgs<R> a) {
  static_assert(P::HX && sizeof(R) == 4, "half-exchange column pass: complex64 HX plans");
  constexpr int N = P::N, T = P::T, E = P::E, W = P::LINES;
  constexpr int SB = 4;  // power-partial batch
  using L = LdsPointMajor<R, W, P::PA, P::PB>;
  __shared__ cx<R> lds_mem[L::size(N / 2)];
  __shared__ cx<R> twq[qtw_entries<N>(typename P::radices{})];
  __shared__ double red[((P::THREADS + 63) / 64) * 2];

  const WorkItem w = a.work[blockIdx.x];
  if (w.inst < 0) return;
  const InstDev& in = a.inst[w.inst];
  if constexpr (KIND == COL_INV) {
    if (2 * a.pair >= in.n_screens || !(in.terms & T_TURB)) return;
  }
  const int c = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int64_t wbase = in.off + w.line0;
  const uint32_t toff = uint32_t(t) * N + uint32_t(c);
  constexpr uint32_t ESTRIDE = uint32_t(T) * N;
  const L lds{lds_mem + c};
  const cx<R>* tables = static_cast<const cx<R>*>(a.tables);
  const cx<R>* __restrict__ prop = tables + in.prop_off;
  const cx<R>* __restrict__ src = static_cast<const cx<R>*>(a.src) + wbase;

  cx<R> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[toff + ESTRIDE * e];
  // twiddle tables; the first exchange's barrier orders them before use
  fill_qtw_tables<R, N, P::THREADS>(twq, int(threadIdx.x), tables + in.tw_off,
                                    typename P::radices{});

  // the last transform's outputs go out butterfly by butterfly (point
  // t + T (b + r NBL) of the last stage's butterfly b), so that they need
  // not all stay live; addresses formed from a laundered offset
  constexpr int RL = LastRadix<P>::value, NBL = E / RL;
  uint32_t to = toff;
  if constexpr (KIND == COL_INV) {
    R* pre = a.planes_out + in.screen_off + int64_t(2 * a.pair) * N * N + w.line0;
    R* pim = pre + int64_t(N) * N;
    const bool has_im = 2 * a.pair + 1 < in.n_screens;
    fft_line_hx<R, P, +1>(v, t, lds, twq, [&](int b, const cx<R>(&y)[RL]) {
      asm volatile("" : "+v"(to));
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const uint32_t e = uint32_t(b + r * NBL);
        pre[to + ESTRIDE * e] = y[r].re;
        if (has_im) pim[to + ESTRIDE * e] = y[r].im;
      }
    });
    return;
  } else {
    fft_line_hx<R, P, -1>(v, t, lds, twq);
    // thread index laundered: the addresses are formed here, not held from
    // the loads
    int tp = t;
    asm volatile("" : "+v"(tp));
    if constexpr (KIND == COL_FD) {
      // the Crank-Nicolson solve with both 1/N (as in k_col)
      const R dkx = prop[w.line0 + c].re;
      const R inv_n2 = R(1) / (R(N) * R(N));
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const R sm = dkx + prop[tp + T * e].re;
        const R den = inv_n2 / (R(1) + sm * sm);
        v[e] = cmul(v[e], cx<R>{den, -sm * den});
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const cx<R> pr = prop[tp + T * e];
        v[e] = (KIND == COL_ADJ) ? cmulc(v[e], pr) : cmul(v[e], pr);
      }
    }
    cx<R>* __restrict__ dst = static_cast<cx<R>*>(a.dst) + wbase;
    // stores, and (forward) the power partials of each point as it is
    // stored (per thread in the order of the last stage's outputs)
    const bool partials = KIND == COL_FWD && a.part != nullptr;
    const ScreenConst<R> sc = screen_const<R>(in);
    double s[1] = {0.0}, m[1] = {0.0};
    fft_line_hx<R, P, +1>(v, t, lds, twq, [&](int b, const cx<R>(&y)[RL]) {
      asm volatile("" : "+v"(to));
#pragma unroll
      for (int r = 0; r < RL; ++r) dst[to + ESTRIDE * uint32_t(b + r * NBL)] = y[r];
      if (partials) {
#pragma unroll
        for (int r0 = 0; r0 < RL; r0 += SB) {
          R x[SB], a2[SB];
#pragma unroll
          for (int q = 0; q < SB; ++q)
            x[q] = y[r0 + q].re * y[r0 + q].re + y[r0 + q].im * y[r0 + q].im;
          if (a.flags & 1) {
#pragma unroll
            for (int q = 0; q < SB; ++q) a2[q] = R(1);
          } else {
            screen_amp2_n<R, SB>(sc, x, a2);
          }
#pragma unroll
          for (int q = 0; q < SB; ++q) {
            const double xa = double(x[q]) * double(a2[q]);
            s[0] += xa;
            m[0] = fmax(m[0], xa);
          }
        }
      }
    });
    if (partials) {
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

template <typename R, class P, int KIND>
hipError_t launch_hx(int n_blocks, const PassArgs<R>& a, hipStream_t s, const LaunchEv* ev) {
  if constexpr (!(P::HX && sizeof(R) == 4)) {
    return hipErrorInvalidValue;
  } else {
    if (ev)
      hipExtLaunchKernelGGL((k_col_hx<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s,
                            ev->start, ev->stop, 0, a);
    else
      hipLaunchKernelGGL((k_col_hx<R, P, KIND>), dim3(n_blocks), dim3(P::THREADS), 0, s, a);
    return hipGetLastError();
  }
}

}  // namespace ssfm
