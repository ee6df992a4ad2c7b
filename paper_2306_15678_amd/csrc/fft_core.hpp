// fft_core.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A "line" is one row or one column of the transverse grid (the split-step
// diffraction operator of Eq. (1) factorises exactly into a row operator and
// a column operator, each diagonal in its own 1-D Fourier basis).  T threads
// cooperate on a line of N points; thread t holds the E = N/T points
// t + T*e (e = 0..E-1) in registers.  Each radix stage of the
// self-sorting (Stockham, decimation-in-time) FFT computes N/R butterflies
// of radix R; thread t owns butterflies j = t + T*b (b < E/R).
//
//   stage with span Ns (1, R0, R0*R1, ...):
//     inputs    x[j + r*N/R]                       r = 0..R-1
//     twiddle   w^(r * (j mod Ns) * N/(Ns*R)),     w = exp(dir 2 pi i / N)
//     DFT_R
//     outputs   y[(j div Ns)*Ns*R + (j mod Ns) + r*Ns]
//
// The inputs of the first stage and the outputs of the last stage are
// exactly the thread's own register points, so an FFT needs LDS only
// between stages, and FFT -> pointwise multiply -> inverse FFT needs no LDS
// traffic at the junction.  Twiddles come from a table
// tw[m] = exp(-2 pi i m / N) computed in FP64 on the host and rounded once;
// each thread loads the ones it needs once and keeps them in registers.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace ssfm {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> conjg(cx<R> a) {
  return {a.re, -a.im};
}
template <typename R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) {
  return {a.re * s, a.im * s};
}
// multiply by (dir * i): dir = -1 gives -i, dir = +1 gives +i
template <int DIR, typename R>
__device__ __forceinline__ cx<R> rot_q(cx<R> a) {
  if constexpr (DIR < 0) {
    return {a.im, -a.re};
  } else {
    return {-a.im, a.re};
  }
}
// multiply by exp(dir i pi/4) = (1 + dir i)/sqrt(2)
template <int DIR, typename R>
__device__ __forceinline__ cx<R> rot_8(cx<R> a) {
  const R h = R(0.70710678118654752440);
  if constexpr (DIR < 0) {
    return {(a.re + a.im) * h, (a.im - a.re) * h};
  } else {
    return {(a.re - a.im) * h, (a.im + a.re) * h};
  }
}
// multiply by exp(dir 3 i pi/4) = (-1 + dir i)/sqrt(2)
template <int DIR, typename R>
__device__ __forceinline__ cx<R> rot_38(cx<R> a) {
  const R h = R(0.70710678118654752440);
  if constexpr (DIR < 0) {
    return {(a.im - a.re) * h, -(a.re + a.im) * h};
  } else {
    return {-(a.re + a.im) * h, (a.re - a.im) * h};
  }
}
// multiply by exp(dir 2 pi i e / 16) for e = 1, 3, 9
template <int DIR, int EXP, typename R>
__device__ __forceinline__ cx<R> rot_16(cx<R> a) {
  constexpr double c1 = 0.92387953251128675613;  // cos(pi/8)
  constexpr double s1 = 0.38268343236508977173;  // sin(pi/8)
  double cr, ci;
  if constexpr (EXP == 1) {
    cr = c1;
    ci = DIR * s1;
  } else if constexpr (EXP == 3) {
    cr = s1;
    ci = DIR * c1;
  } else {  // EXP == 9
    cr = -c1;
    ci = -DIR * s1;
  }
  return cmul(a, cx<R>{R(cr), R(ci)});
}

// ---------------------------------------------------------------- DFTs
// In-place DFT of R points in natural order: y_k = sum_n x_n w^(nk),
// w = exp(dir 2 pi i / R).

template <int DIR, typename R>
__device__ __forceinline__ void dft2(cx<R>* v) {
  cx<R> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <int DIR, typename R>
__device__ __forceinline__ void dft3(cx<R>* v) {
  const R h = R(0.86602540378443864676);  // sqrt(3)/2
  cx<R> t = v[1] + v[2];
  cx<R> u = v[1] - v[2];
  cx<R> m = {v[0].re - R(0.5) * t.re, v[0].im - R(0.5) * t.im};
  cx<R> w = scale(rot_q<DIR>(u), h);
  v[0] = v[0] + t;
  v[1] = m + w;
  v[2] = m - w;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft4_(cx<R>& a0, cx<R>& a1, cx<R>& a2,
                                      cx<R>& a3) {
  cx<R> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3;
  cx<R> t3 = rot_q<DIR>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft4(cx<R>* v) {
  dft4_<DIR>(v[0], v[1], v[2], v[3]);
}

template <int DIR, typename R>
__device__ __forceinline__ void dft8(cx<R>* v) {
  cx<R> b0 = v[0] + v[4], c0 = v[0] - v[4];
  cx<R> b1 = v[1] + v[5], c1 = v[1] - v[5];
  cx<R> b2 = v[2] + v[6], c2 = v[2] - v[6];
  cx<R> b3 = v[3] + v[7], c3 = v[3] - v[7];
  c1 = rot_8<DIR>(c1);
  c2 = rot_q<DIR>(c2);
  c3 = rot_38<DIR>(c3);
  dft4_<DIR>(b0, b1, b2, b3);  // even outputs
  dft4_<DIR>(c0, c1, c2, c3);  // odd outputs
  v[0] = b0; v[2] = b1; v[4] = b2; v[6] = b3;
  v[1] = c0; v[3] = c1; v[5] = c2; v[7] = c3;
}

// 16 = 4 x 4: inner DFT4 over n2 (stride 4), twiddle w16^(n1 k2), outer
// DFT4 over n1; output index k2 + 4 k1.
template <int DIR, typename R>
__device__ __forceinline__ void dft16(cx<R>* v) {
  dft4_<DIR>(v[0], v[4], v[8], v[12]);
  dft4_<DIR>(v[1], v[5], v[9], v[13]);
  dft4_<DIR>(v[2], v[6], v[10], v[14]);
  dft4_<DIR>(v[3], v[7], v[11], v[15]);
  // v[n1 + 4 k2] *= w16^(n1 k2)
  v[5] = rot_16<DIR, 1>(v[5]);
  v[9] = rot_8<DIR>(v[9]);
  v[13] = rot_16<DIR, 3>(v[13]);
  v[6] = rot_8<DIR>(v[6]);
  v[10] = rot_q<DIR>(v[10]);
  v[14] = rot_38<DIR>(v[14]);
  v[7] = rot_16<DIR, 3>(v[7]);
  v[11] = rot_38<DIR>(v[11]);
  v[15] = rot_16<DIR, 9>(v[15]);
  dft4_<DIR>(v[0], v[1], v[2], v[3]);
  dft4_<DIR>(v[4], v[5], v[6], v[7]);
  dft4_<DIR>(v[8], v[9], v[10], v[11]);
  dft4_<DIR>(v[12], v[13], v[14], v[15]);
  // now v[4 k2 + k1] holds y[k2 + 4 k1]: transpose the 4x4 index
  cx<R> t;
#define SSFM_SWAP(a, b) t = v[a]; v[a] = v[b]; v[b] = t;
  SSFM_SWAP(1, 4) SSFM_SWAP(2, 8) SSFM_SWAP(3, 12)
  SSFM_SWAP(6, 9) SSFM_SWAP(7, 13) SSFM_SWAP(11, 14)
#undef SSFM_SWAP
}

// cos(e pi / 16) and sin(e pi / 16) for integer e (exact table of the
// first octant, extended by symmetry).
constexpr double kCos16[9] = {1.0,
                              0.98078528040323044913,
                              0.92387953251128675613,
                              0.83146961230254523708,
                              0.70710678118654752440,
                              0.55557023301960222474,
                              0.38268343236508977173,
                              0.19509032201612826785,
                              0.0};
constexpr double cos16(int e) {
  e = ((e % 32) + 32) % 32;
  if (e <= 8) return kCos16[e];
  if (e <= 16) return -kCos16[16 - e];
  if (e <= 24) return -kCos16[e - 16];
  return kCos16[32 - e];
}
constexpr double sin16(int e) { return cos16(8 - e); }

// multiply by exp(dir 2 pi i e / 32)
template <int DIR, int EXP, typename R>
__device__ __forceinline__ cx<R> rot_32(cx<R> a) {
  constexpr int e = ((EXP % 32) + 32) % 32;
  if constexpr (e == 0) return a;
  else if constexpr (e == 8) return rot_q<DIR>(a);
  else if constexpr (e == 16) return cx<R>{-a.re, -a.im};
  else if constexpr (e == 24) return rot_q<-DIR>(a);
  else if constexpr (e == 4) return rot_8<DIR>(a);
  else if constexpr (e == 12) return rot_38<DIR>(a);
  else return cmul(a, cx<R>{R(cos16(e)), R(DIR * sin16(e))});
}

// 32 = 4 x 8: inner DFT8 over n2 (points n1 + 4 n2), twiddle w32^(n1 k2),
// outer DFT4 over n1; output index k2 + 8 k1.
template <int DIR, int N1, int K2, typename R>
__device__ __forceinline__ void dft32_tw(cx<R>* v) {
  v[N1 + 4 * K2] = rot_32<DIR, N1 * K2>(v[N1 + 4 * K2]);
}

template <int DIR, typename R>
__device__ __forceinline__ void dft32(cx<R>* v) {
  cx<R> t[32];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cx<R> g[8];
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) g[n2] = v[n1 + 4 * n2];
    dft8<DIR>(g);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) t[n1 + 4 * k2] = g[k2];
  }
  [&]<int... I>(std::integer_sequence<int, I...>) {
    ((dft32_tw<DIR, I / 8, I % 8>(t)), ...);
  }(std::make_integer_sequence<int, 32>{});
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {
    dft4_<DIR>(t[4 * k2], t[4 * k2 + 1], t[4 * k2 + 2], t[4 * k2 + 3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) v[k2 + 8 * k1] = t[4 * k2 + k1];
  }
}

template <int RAD, int DIR, typename R>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (RAD == 2) dft2<DIR>(v);
  else if constexpr (RAD == 3) dft3<DIR>(v);
  else if constexpr (RAD == 4) dft4<DIR>(v);
  else if constexpr (RAD == 8) dft8<DIR>(v);
  else if constexpr (RAD == 16) dft16<DIR>(v);
  else if constexpr (RAD == 32) dft32<DIR>(v);
  else static_assert(RAD == 2, "unsupported radix");
}

// ------------------------------------------------------------ plans
template <int... Rs>
struct Radices {};

template <int R0, int... Rest>
constexpr int first_radix() {
  return R0;
}

// N points per line, T threads per line, LINES lines per workgroup; column
// tiles pad their LDS by B slots every A points (see LdsPointMajor).  OPT:
// bit 0 set loads each stage's twiddles just before that stage (fewer live
// registers) instead of all of them before the first; bit 1 loads the
// diffraction factors after the forward FFT instead of with the field (and,
// in the adjoint row pass, the stored field and the screen phases after
// the inverse FFT); bits 4-7 set the points per batch of the adjoint
// screen (0: 4); bits 8-11 give the wavefronts per SIMD the compiler must
// leave room for in the complex64 kernels (0: no target); bit 12 makes the
// forward and adjoint row passes persistent and pipelined (complex64 only:
// each workgroup loads its next row while it transforms the current one);
// bit 13 recomputes each stage's LDS and twiddle addresses within the stage
// (fewer registers held through the transform, a few more instructions);
// bit 14 gives a plain row pass or a pipelined column pass its twiddles
// from a quarter table in LDS (a pipelined column pass also loads its
// propagator after the forward transform: its tile leaves no LDS room for
// the stage tables); bit 15 makes a column pass
// exchange through half its tile (fft_line_hx), complex64 only.
template <int N_, int T_, int LINES_, class Rad, int PA_ = 32, int PB_ = 0, int OPT_ = 0>
struct Plan {
  static constexpr int N = N_;
  static constexpr int T = T_;
  static constexpr int LINES = LINES_;
  static constexpr int E = N_ / T_;
  static constexpr int THREADS = T_ * LINES_;
  static constexpr int PA = PA_;
  static constexpr int PB = PB_;
  static constexpr bool LATE_TW = (OPT_ & 1) != 0;
  static constexpr bool LATE_PROP = (OPT_ & 2) != 0;
  static constexpr int ADJ_BATCH = ((OPT_ >> 4) & 15) ? ((OPT_ >> 4) & 15) : 4;
  static constexpr int WAVES_PER_EU = ((OPT_ >> 8) & 15) ? ((OPT_ >> 8) & 15) : 1;
  static constexpr bool PIPE = (OPT_ & 0x1000) != 0;
  static constexpr bool LAUNDER = (OPT_ & 0x2000) != 0;
  static constexpr bool QTW = (OPT_ & 0x4000) != 0;
  static constexpr bool HX = (OPT_ & 0x8000) != 0;
  using radices = Rad;
  static_assert(N_ % T_ == 0, "T must divide N");
};

// --------------------------------------------------------- LDS layouts
// Row lines: line-major with one pad slot per 32 points.
template <typename R, int N>
struct LdsLineMajor {
  static constexpr int LINE = N + N / 32;
  static constexpr int SIZE_PER_LINE = LINE;
  cx<R>* base;
  __device__ __forceinline__ cx<R> get(int p) const { return base[p + (p >> 5)]; }
  __device__ __forceinline__ void put(int p, cx<R> v) const { base[p + (p >> 5)] = v; }
};

// Column tiles: point-major, the W columns of a point adjacent, B padding
// slots after every A points.
template <typename R, int W, int A, int B>
struct LdsPointMajor {
  static constexpr int size(int n) { return n * W + (n / A) * B; }
  cx<R>* base;  // already offset by the column index
  // unsigned (p >= 0): the division is a shift, and constant offsets of p
  // that are multiples of A fold into the instruction's offset
  __device__ __forceinline__ int idx(int p) const {
    const unsigned u = unsigned(p);
    return int(u * W + (u / A) * B);
  }
  __device__ __forceinline__ cx<R> get(int p) const { return base[idx(p)]; }
  __device__ __forceinline__ void put(int p, cx<R> v) const { base[idx(p)] = v; }
};

// ------------------------------------------------------------ twiddles
// A thread's twiddles for every stage are loaded once, before the first
// stage (one batch of independent loads), and reused conjugated by the
// inverse transform.  Stage s (span NS > 1, radix R) needs, for each of
// its E/R butterflies b and r = 1..R-1, tw[r * (j mod NS) * N/(NS R)]
// with j = t + T b.
template <int N, int T, int... Rs>
constexpr int twiddle_count() {
  int ns = 1, c = 0;
  ((c += (ns > 1 ? (N / T / Rs) * (Rs - 1) : 0), ns *= Rs), ...);
  return c;
}

template <class P>
struct TwCount;
template <int N, int T, int L, int... Rs, int A, int B, int O>
struct TwCount<Plan<N, T, L, Radices<Rs...>, A, B, O>> {
  // late twiddles are loaded stage by stage: nothing held up front
  static constexpr int value = (O & 1) ? 0 : twiddle_count<N, T, Rs...>();
};

template <typename R, int N, int T, int NS, int RAD>
__device__ __forceinline__ void load_stage_twiddles(cx<R>* w, int t,
                                                    const cx<R>* __restrict__ tw) {
  constexpr int E = N / T, NB = E / RAD, TWS = N / (NS * RAD);
  if constexpr (NS > 1) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (t + T * b) % NS;
#pragma unroll
      for (int r = 1; r < RAD; ++r) w[b * (RAD - 1) + r - 1] = tw[r * k * TWS];
    }
  }
}

template <typename R, int N, int T, int NS, int R0, int... Rest>
__device__ __forceinline__ void load_twiddles_rec(cx<R>* w, int t,
                                                  const cx<R>* __restrict__ tw) {
  load_stage_twiddles<R, N, T, NS, R0>(w, t, tw);
  if constexpr (sizeof...(Rest) > 0) {
    constexpr int used = (NS > 1) ? (N / T / R0) * (R0 - 1) : 0;
    load_twiddles_rec<R, N, T, NS * R0, Rest...>(w + used, t, tw);
  }
}

template <typename R, int N, int T, int... Rs>
__device__ __forceinline__ void load_twiddles_impl(cx<R>* w, int t,
                                                   const cx<R>* __restrict__ tw,
                                                   Radices<Rs...>) {
  load_twiddles_rec<R, N, T, 1, Rs...>(w, t, tw);
}

template <typename R, class P>
__device__ __forceinline__ void load_twiddles(cx<R>* w, int t, const cx<R>* __restrict__ tw) {
  if constexpr (!P::LATE_TW) load_twiddles_impl<R, P::N, P::T>(w, t, tw, typename P::radices{});
}

// ---------------------------------------------------------- one stage
// w: this stage's twiddles in registers (preloaded), or, with LATE, loaded
// here from the table before the stage's LDS reads so that their latency
// overlaps the exchange.
template <typename R, int N, int T, int RAD, int NS, int DIR, bool FIRST,
          bool LAST, bool LATE, class Lds, bool LAUNDER = false>
__device__ __forceinline__ void fft_stage(cx<R>* v, int t, const Lds& lds,
                                          const cx<R>* wpre, const cx<R>* __restrict__ tw) {
  // LAUNDER: the thread index made opaque per stage, so the stage's LDS
  // and twiddle addresses are computed where they are used instead of
  // held in registers from the kernel's start
  if constexpr (LAUNDER) asm volatile("" : "+v"(t));
  constexpr int E = N / T;
  constexpr int NB = E / RAD;
  constexpr int STRIDE = N / RAD;
  static_assert(E % RAD == 0, "radix must divide points per thread");
  cx<R> wl[(LATE && NS > 1) ? NB * (RAD - 1) : 1];
  if constexpr (LATE && NS > 1) load_stage_twiddles<R, N, T, NS, RAD>(wl, t, tw);
  const cx<R>* w = LATE ? wl : wpre;
  cx<R> a[NB][RAD];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      if constexpr (FIRST) {
        a[b][r] = v[b + r * NB];
      } else {
        a[b][r] = lds.get(t + T * b + r * STRIDE);
      }
    }
  }
  if constexpr (!FIRST) {
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + T * b;
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        const cx<R> ww = w[b * (RAD - 1) + r - 1];
        a[b][r] = (DIR > 0) ? cmulc(a[b][r], ww) : cmul(a[b][r], ww);
      }
    }
    dft<RAD, DIR>(a[b]);
    if constexpr (!LAST) {
      const int base = (j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds.put(base + r * NS, a[b][r]);
    } else {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b + r * NB] = a[b][r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
  }
}

template <typename R, int N, int T, int DIR, int NS, bool FIRST, bool LATE, bool LAUNDER,
          class Lds, int R0, int... Rest>
__device__ __forceinline__ void fft_stages(cx<R>* v, int t, const Lds& lds,
                                           const cx<R>* w, const cx<R>* __restrict__ tw) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  fft_stage<R, N, T, R0, NS, DIR, FIRST, LAST, LATE, Lds, LAUNDER>(v, t, lds, w, tw);
  if constexpr (!LAST) {
    constexpr int used = (!LATE && NS > 1) ? (N / T / R0) * (R0 - 1) : 0;
    fft_stages<R, N, T, DIR, NS * R0, false, LATE, LAUNDER, Lds, Rest...>(v, t, lds, w + used,
                                                                         tw);
  }
}

template <typename R, int N, int T, int DIR, bool LATE, bool LAUNDER, class Lds, int... Rs>
__device__ __forceinline__ void fft_line_impl(cx<R>* v, int t, const Lds& lds,
                                              const cx<R>* w, const cx<R>* __restrict__ tw,
                                              Radices<Rs...>) {
  fft_stages<R, N, T, DIR, 1, true, LATE, LAUNDER, Lds, Rs...>(v, t, lds, w, tw);
}

// In-register FFT of one line (DIR = -1 forward, +1 inverse, unscaled),
// with the thread's twiddles preloaded by load_twiddles<R, P> (w), or, for
// a late-twiddle plan, read stage by stage from the table tw.  On entry and
// exit v[e] holds point t + T*e.
template <typename R, class P, int DIR, class Lds>
__device__ __forceinline__ void fft_line(cx<R>* v, int t, const Lds& lds, const cx<R>* w,
                                         const cx<R>* __restrict__ tw) {
  fft_line_impl<R, P::N, P::T, DIR, P::LATE_TW, P::LAUNDER>(v, t, lds, w, tw,
                                                             typename P::radices{});
}

// ------------------------------------------- twiddles staged in LDS
// Persistent kernels copy the twiddles of every stage with span NS > 1 into
// LDS once, in the order the stage reads them: entry (r - 1) NS + k of the
// stage's block holds tw[r k N/(NS R)] for butterflies with j mod NS = k.
// Stage blocks follow each other; the block of span NS starts at NS - R0
// and they hold N - R0 entries together.  The lanes of a wave read
// consecutive k (or one broadcast value), so the reads are free of bank
// conflicts, and the values are those of the table.
template <int N, int R0, int... Rest>
constexpr int lds_tw_entries(Radices<R0, Rest...>) {
  return N - R0;
}

template <typename R, int N, int NS, int RAD, int... Rest>
__device__ __forceinline__ cx<R> lds_tw_value(int idx, const cx<R>* __restrict__ tw) {
  // idx counts from the start of this stage's block
  if (NS > 1 && idx < (RAD - 1) * NS) {
    const int r = idx / NS + 1, k = idx - (r - 1) * NS;
    return tw[r * k * (N / (NS * RAD))];
  }
  if constexpr (sizeof...(Rest) > 0) {
    return lds_tw_value<R, N, NS * RAD, Rest...>(NS > 1 ? idx - (RAD - 1) * NS : idx, tw);
  } else {
    return tw[0];
  }
}

template <typename R, int N, int THREADS, int... Rs>
__device__ __forceinline__ void fill_lds_twiddles(cx<R>* twl, int t, const cx<R>* __restrict__ tw,
                                                  Radices<Rs...> rad) {
  constexpr int M = lds_tw_entries<N>(rad);
  for (int i = t; i < M; i += THREADS) twl[i] = lds_tw_value<R, N, 1, Rs...>(i, tw);
}

template <typename R, int N, int T, int RAD, int NS, int R0, int DIR, bool FIRST, bool LAST,
          class Lds>
__device__ __forceinline__ void fft_stage_ltw(cx<R>* v, int t, const Lds& lds,
                                              const cx<R>* twl) {
  constexpr int E = N / T;
  constexpr int NB = E / RAD;
  constexpr int STRIDE = N / RAD;
  static_assert(E % RAD == 0, "radix must divide points per thread");
  const cx<R>* ws = twl + (NS - R0);
  cx<R> a[NB][RAD];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      if constexpr (FIRST) {
        a[b][r] = v[b + r * NB];
      } else {
        a[b][r] = lds.get(t + T * b + r * STRIDE);
      }
    }
  }
  if constexpr (!FIRST) {
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const unsigned j = unsigned(t + T * b);  // j >= 0: shifts and masks
    const int k = int(j % NS);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        const cx<R> ww = ws[(r - 1) * NS + k];
        a[b][r] = (DIR > 0) ? cmulc(a[b][r], ww) : cmul(a[b][r], ww);
      }
    }
    dft<RAD, DIR>(a[b]);
    if constexpr (!LAST) {
      const int base = int(j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds.put(base + r * NS, a[b][r]);
    } else {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b + r * NB] = a[b][r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
  }
}

template <typename R, int N, int T, int DIR, int NS, int R0, bool FIRST, class Lds, int RA,
          int... Rest>
__device__ __forceinline__ void fft_stages_ltw(cx<R>* v, int t, const Lds& lds,
                                               const cx<R>* twl) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  fft_stage_ltw<R, N, T, RA, NS, R0, DIR, FIRST, LAST>(v, t, lds, twl);
  if constexpr (!LAST) fft_stages_ltw<R, N, T, DIR, NS * RA, R0, false, Lds, Rest...>(v, t, lds, twl);
}

template <typename R, int N, int T, int DIR, class Lds, int R0, int... Rest>
__device__ __forceinline__ void fft_line_ltw_impl(cx<R>* v, int t, const Lds& lds,
                                                  const cx<R>* twl, Radices<R0, Rest...>) {
  fft_stages_ltw<R, N, T, DIR, 1, R0, true, Lds, R0, Rest...>(v, t, lds, twl);
}

// fft_line with the twiddles read from the LDS copy made by
// fill_lds_twiddles; same values and operation order as fft_line.
template <typename R, class P, int DIR, class Lds>
__device__ __forceinline__ void fft_line_ltw(cx<R>* v, int t, const Lds& lds, const cx<R>* twl) {
  fft_line_ltw_impl<R, P::N, P::T, DIR>(v, t, lds, twl, typename P::radices{});
}

// ----------------------------------- twiddles from a quarter table in LDS
// tw[m] = exp(-2 pi i m / N) for m < N/4 in LDS; the rest follow from
// exp(-2 pi i (m + q N/4) / N) = (-i)^q exp(-2 pi i m / N), a swap and sign
// changes.  For tiles that fill the LDS (N/4 entries instead of N - R0).
template <typename R, int N>
__device__ __forceinline__ cx<R> qtw(const cx<R>* twq, int m) {
  const unsigned u = unsigned(m);  // m >= 0
  const cx<R> a = twq[u & (N / 4 - 1)];
  const unsigned q = (u / (N / 4)) & 3;
  const cx<R> b = (q & 1) ? cx<R>{a.im, -a.re} : a;
  return (q & 2) ? cx<R>{-b.re, -b.im} : b;
}

template <typename R, int N, int THREADS>
__device__ __forceinline__ void fill_qtw(cx<R>* twq, int t, const cx<R>* __restrict__ tw) {
  for (int i = t; i < N / 4; i += THREADS) twq[i] = tw[i];
}

// The quarter table (N/4 entries) followed by the second stage's own
// table (span R0, radix R1: entry (r - 1) R0 + k holds tw[r k N/(R0 R1)]),
// which that stage reads without the quadrant rotation and by consecutive
// k across a wave.
template <int N, int R0, int R1, int... Rest>
constexpr int qtw_entries(Radices<R0, R1, Rest...>) {
  return N / 4 + (R1 - 1) * R0;
}

template <typename R, int N, int THREADS, int R0, int R1, int... Rest>
__device__ __forceinline__ void fill_qtw_tables(cx<R>* twl, int t, const cx<R>* __restrict__ tw,
                                                Radices<R0, R1, Rest...>) {
  fill_qtw<R, N, THREADS>(twl, t, tw);
  for (int i = t; i < (R1 - 1) * R0; i += THREADS) {
    const int r = i / R0 + 1, k = i % R0;
    twl[N / 4 + i] = tw[r * k * (N / (R0 * R1))];
  }
}

// A twiddle of stage (span NS, radix RAD) from the tables of fill_qtw_tables.
template <typename R, int N, int RAD, int NS, int R0>
__device__ __forceinline__ cx<R> qtw_stage(const cx<R>* twq, int r, int k) {
  if constexpr (NS == R0)
    return twq[N / 4 + (r - 1) * NS + k];
  else
    return qtw<R, N>(twq, r * k * (N / (NS * RAD)));
}

template <typename R, int N, int T, int RAD, int NS, int R0, int DIR, bool FIRST, bool LAST,
          class Lds>
__device__ __forceinline__ void fft_stage_qtw(cx<R>* v, int t, const Lds& lds,
                                              const cx<R>* twq) {
  // the thread index made opaque per stage (addresses computed in the stage)
  asm volatile("" : "+v"(t));
  constexpr int E = N / T;
  constexpr int NB = E / RAD;
  constexpr int STRIDE = N / RAD;
  constexpr int TWS = N / (NS * RAD);
  static_assert(E % RAD == 0, "radix must divide points per thread");
  cx<R> a[NB][RAD];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      if constexpr (FIRST) {
        a[b][r] = v[b + r * NB];
      } else {
        a[b][r] = lds.get(t + T * b + r * STRIDE);
      }
    }
  }
  if constexpr (!FIRST) {
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const unsigned j = unsigned(t + T * b);  // j >= 0: shifts and masks
    const int k = int(j % NS);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        const cx<R> ww = qtw_stage<R, N, RAD, NS, R0>(twq, r, k);
        a[b][r] = (DIR > 0) ? cmulc(a[b][r], ww) : cmul(a[b][r], ww);
      }
    }
    dft<RAD, DIR>(a[b]);
    if constexpr (!LAST) {
      const int base = int(j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds.put(base + r * NS, a[b][r]);
    } else {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b + r * NB] = a[b][r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
  }
}

template <typename R, int N, int T, int DIR, int NS, int R0, bool FIRST, class Lds, int RA,
          int... Rest>
__device__ __forceinline__ void fft_stages_qtw(cx<R>* v, int t, const Lds& lds,
                                               const cx<R>* twq) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  fft_stage_qtw<R, N, T, RA, NS, R0, DIR, FIRST, LAST>(v, t, lds, twq);
  if constexpr (!LAST)
    fft_stages_qtw<R, N, T, DIR, NS * RA, R0, false, Lds, Rest...>(v, t, lds, twq);
}

template <typename R, int N, int T, int DIR, class Lds, int R0, int... Rs>
__device__ __forceinline__ void fft_line_qtw_impl(cx<R>* v, int t, const Lds& lds,
                                                  const cx<R>* twq, Radices<R0, Rs...>) {
  fft_stages_qtw<R, N, T, DIR, 1, R0, true, Lds, R0, Rs...>(v, t, lds, twq);
}

// fft_line with the twiddles read from the tables made by fill_qtw_tables.
template <typename R, class P, int DIR, class Lds>
__device__ __forceinline__ void fft_line_qtw(cx<R>* v, int t, const Lds& lds, const cx<R>* twq) {
  fft_line_qtw_impl<R, P::N, P::T, DIR>(v, t, lds, twq, typename P::radices{});
}


// ------------------------------------ exchanges through half an LDS tile
// A tile that would fill the LDS can exchange through half of it, so that
// two workgroups fit one compute unit.  In a stage of radix R and span NS
// (not the last), butterfly j writes its outputs below N/2 exactly when
// j < N/(2R) (given N/(NS R) even), i.e. for b < NB/2 of every thread; the
// next stage (radix R') reads point t + T b' + r' N/R', below N/2 exactly
// when r' < R'/2.  So each exchange runs in two rounds over the same N/2
// slots: the lower outputs are written and the lower inputs read, then the
// upper ones, with a barrier between every write and read (four per
// exchange, the first guarding the previous exchange's last reads).  The
// butterflies, twiddles (quarter table) and their order are those of
// fft_line_qtw.
template <typename R, int N, int T, int RAD, int NS, int R0, int DIR>
__device__ __forceinline__ void hx_butterfly(cx<R> (&y)[RAD], int j, const cx<R>* twq) {
  if constexpr (NS > 1) {
    // unsigned (j >= 0): butterflies T apart share k when NS divides T,
    // and the compiler sees it
    const int k = int(unsigned(j) % unsigned(NS));
#pragma unroll
    for (int r = 1; r < RAD; ++r) {
      const cx<R> ww = qtw_stage<R, N, RAD, NS, R0>(twq, r, k);
      y[r] = (DIR > 0) ? cmulc(y[r], ww) : cmul(y[r], ww);
    }
  }
  dft<RAD, DIR>(y);
}

template <typename R, int N, int T, int RAD, int NS, int RB, class Lds>
__device__ __forceinline__ void hx_exchange(cx<R> (&a)[N / T / RAD][RAD],
                                            cx<R> (&nx)[N / T / RB][RB], int t, const Lds& lds) {
  constexpr int NB = N / T / RAD, NB2 = N / T / RB, H = N / 2;
  static_assert(NB % 2 == 0 && RB % 2 == 0 && (N / (NS * RAD)) % 2 == 0,
                "half exchange: even butterfly count, next radix and remaining span");
  asm volatile("" : "+v"(t));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
#pragma unroll
    for (int b = h * NB / 2; b < (h + 1) * NB / 2; ++b) {
      const unsigned j = unsigned(t + T * b);
      const int base = int((j / NS) * NS * RAD + j % NS) - h * H;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds.put(base + r * NS, a[b][r]);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB2; ++b) {
#pragma unroll
      for (int r = h * RB / 2; r < (h + 1) * RB / 2; ++r)
        nx[b][r] = lds.get(t + T * b + r * (N / RB) - h * H);
    }
  }
}

// The last stage hands each butterfly's outputs to sink(b, y) as soon as
// they are formed: y[r] is point t + T (b + r NB), NB = E / R_last.
template <typename R, int N, int T, int DIR, int NS, int R0, class Lds, class Sink, int RA,
          int... Rest>
__device__ __forceinline__ void hx_stages(cx<R> (&a)[N / T / RA][RA], int t, const Lds& lds,
                                          const cx<R>* twq, Sink&& sink) {
  constexpr int NB = N / T / RA;
  // the thread index made opaque per stage (addresses computed in the stage)
  asm volatile("" : "+v"(t));
  if constexpr (sizeof...(Rest) == 0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      hx_butterfly<R, N, T, RA, NS, R0, DIR>(a[b], t + T * b, twq);
      sink(b, a[b]);
    }
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) hx_butterfly<R, N, T, RA, NS, R0, DIR>(a[b], t + T * b, twq);
    constexpr int RB = first_radix<Rest...>();
    cx<R> nx[N / T / RB][RB];
    hx_exchange<R, N, T, RA, NS, RB>(a, nx, t, lds);
    hx_stages<R, N, T, DIR, NS * RA, R0, Lds, Sink, Rest...>(nx, t, lds, twq,
                                                             static_cast<Sink&&>(sink));
  }
}

template <int... Rs>
constexpr int last_radix() {
  int r = 0;
  ((r = Rs), ...);
  return r;
}

template <class P>
struct LastRadix;
template <int N, int T, int L, int... Rs, int A, int B, int O>
struct LastRadix<Plan<N, T, L, Radices<Rs...>, A, B, O>> {
  static constexpr int value = last_radix<Rs...>();
};

template <typename R, int N, int T, int DIR, class Lds, class Sink, int R0, int... Rest>
__device__ __forceinline__ void fft_line_hx_impl(cx<R>* v, int t, const Lds& lds,
                                                 const cx<R>* twq, Sink&& sink,
                                                 Radices<R0, Rest...>) {
  constexpr int NB = N / T / R0;
  cx<R> a[NB][R0];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int r = 0; r < R0; ++r) a[b][r] = v[b + r * NB];
  }
  hx_stages<R, N, T, DIR, 1, R0, Lds, Sink, R0, Rest...>(a, t, lds, twq,
                                                        static_cast<Sink&&>(sink));
}

// fft_line with half-tile exchanges and the twiddles of fill_qtw_tables
// (lds spans N/2 points of each line); the outputs go to sink(b, y)
// butterfly by butterfly of the last stage (y[r]: point t + T (b + r NB)).
template <typename R, class P, int DIR, class Lds, class Sink>
__device__ __forceinline__ void fft_line_hx(cx<R>* v, int t, const Lds& lds, const cx<R>* twq,
                                            Sink&& sink) {
  fft_line_hx_impl<R, P::N, P::T, DIR>(v, t, lds, twq, static_cast<Sink&&>(sink),
                                       typename P::radices{});
}

// the same with the outputs in place (v[e] = point t + T e)
template <typename R, class P, int DIR, class Lds>
__device__ __forceinline__ void fft_line_hx(cx<R>* v, int t, const Lds& lds, const cx<R>* twq) {
  [&]<int... Rs>(Radices<Rs...>) {
    constexpr int NB = P::E / last_radix<Rs...>();
    fft_line_hx<R, P, DIR>(v, t, lds, twq, [&](int b, const auto& y) {
#pragma unroll
      for (int r = 0; r < last_radix<Rs...>(); ++r) v[b + r * NB] = y[r];
    });
  }(typename P::radices{});
}

}  // namespace ssfm
