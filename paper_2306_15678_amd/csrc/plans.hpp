// plans.hpp -- compiled FFT tile variants of the row and column passes.
//
// Rows: X(N, variant, T, LINES, OPT, radices...); columns: X(N, variant,
// T, W, A, B, OPT, radices...).  OPT: 1 = late twiddles, 2 = late
// propagator, plus 0x100 times the wavefronts per SIMD the compiler must
// leave room for, 0x1000 = persistent pipelined passes (complex64),
// 0x2000 = per-stage address computation, 0x4000 = twiddles from a quarter
// table in LDS (plain row passes and pipelined columns; the latter also
// load the propagator late), 0x8000 = column exchanges through half the
// tile (two workgroups per compute unit; see Plan).  T
// threads per line, LINES lines per workgroup (rows:
// LINES consecutive rows; columns: W adjacent columns, read as
// W * sizeof(complex) contiguous bytes per row), radix plan in stage order.
// Column tiles keep point p of column c at LDS slot p W + c + (p / A) B:
// the padding (A, B) is chosen per plan to spread the stage exchanges over
// the LDS banks (64 banks of 4 bytes; a wave64 64-bit access served 32
// lanes at a time).  Variant 0 is the default; the autotuner picks among the
// others per grid size.  E = N/T points per thread: 16 keeps more work per
// thread, 8 and 4 give 2x / 4x more wavefronts for latency hiding.
#pragma once

#include "fft_core.hpp"

namespace ssfm {

#define SSFM_ROW_PLANS(X)              \
  X(128, 0, 8, 32, 0, 16, 8)              \
  X(128, 1, 16, 16, 0, 8, 4, 4)           \
  X(256, 0, 16, 16, 0, 16, 16)            \
  X(256, 1, 32, 8, 0, 8, 8, 4)            \
  X(512, 0, 64, 4, 0, 8, 8, 8)            \
  X(512, 1, 32, 8, 0, 16, 16, 2)          \
  X(512, 2, 64, 1, 0, 8, 8, 8)            \
  X(768, 0, 32, 8, 0, 8, 8, 4, 3)         \
  X(768, 1, 64, 4, 0, 4, 4, 4, 4, 3)      \
  X(1024, 0, 64, 4, 0, 16, 8, 8)          \
  X(1024, 1, 128, 2, 0, 8, 8, 4, 4)       \
  X(1024, 2, 256, 1, 0, 4, 4, 4, 4, 4)    \
  X(1024, 3, 64, 2, 0, 16, 8, 8)          \
  X(1024, 4, 64, 1, 0, 16, 8, 8)          \
  X(1024, 5, 128, 1, 0, 8, 8, 4, 4)       \
  X(1024, 6, 32, 2, 0, 32, 32)            \
  X(2048, 0, 128, 2, 0, 16, 16, 8)        \
  X(2048, 1, 256, 1, 0, 8, 8, 8, 4)       \
  X(2048, 2, 256, 1, 0x1000, 8, 8, 8, 4)  \
  X(4096, 0, 256, 1, 0, 16, 16, 16)       \
  X(4096, 1, 512, 1, 0, 8, 8, 8, 8)       \
  X(4096, 2, 256, 1, 0x201, 16, 16, 16)   \
  X(4096, 3, 256, 1, 0x203, 16, 16, 16)   \
  X(4096, 4, 256, 1, 0x323, 16, 16, 16)   \
  X(4096, 5, 256, 1, 0x303, 16, 16, 16)   \
  X(4096, 6, 512, 1, 0x1000, 8, 8, 8, 8)  \
  X(4096, 7, 512, 1, 0x1010, 8, 8, 8, 8)  \
  X(4096, 8, 256, 1, 0x4303, 16, 16, 16)

#define SSFM_COL_PLANS(X)              \
  X(128, 0, 8, 32, 1, 0, 0, 16, 8) \
  X(128, 1, 16, 16, 2, 4, 0, 8, 4, 4) \
  X(256, 0, 16, 16, 2, 2, 0, 16, 16) \
  X(256, 1, 32, 8, 4, 4, 0, 8, 8, 4) \
  X(512, 0, 64, 4, 8, 4, 0, 8, 8, 8) \
  X(512, 1, 32, 8, 4, 2, 0, 16, 16, 2) \
  X(768, 0, 32, 8, 4, 4, 0, 8, 8, 4, 3) \
  X(768, 1, 64, 4, 8, 4, 0, 4, 4, 4, 4, 3) \
  X(1024, 0, 64, 4, 8, 2, 0, 16, 8, 8) \
  X(1024, 1, 128, 2, 16, 2, 0, 8, 8, 4, 4) \
  X(1024, 2, 128, 4, 8, 4, 0, 8, 8, 4, 4) \
  X(1024, 3, 256, 2, 16, 6, 0, 4, 4, 4, 4, 4) \
  X(1024, 4, 64, 8, 4, 2, 0, 16, 8, 8) \
  X(1024, 5, 32, 8, 4, 1, 0, 32, 32) \
  X(1024, 6, 64, 16, 4, 4, 0x2403, 16, 8, 8) \
  X(2048, 0, 128, 2, 16, 2, 0, 16, 16, 8) \
  X(2048, 1, 256, 2, 16, 2, 0, 8, 8, 8, 4) \
  X(2048, 2, 256, 2, 16, 2, 0x1000, 8, 8, 8, 4) \
  X(2048, 3, 128, 8, 4, 2, 0x7403, 16, 16, 8) \
  X(4096, 0, 256, 2, 16, 2, 0, 16, 16, 16) \
  X(4096, 1, 512, 2, 16, 2, 0, 8, 8, 8, 8) \
  X(4096, 2, 256, 2, 16, 2, 0x203, 16, 16, 16) \
  X(4096, 3, 256, 4, 16, 2, 0x403, 16, 16, 16) \
  X(4096, 4, 128, 2, 16, 2, 0x203, 16, 16, 16) \
  X(4096, 5, 128, 4, 16, 2, 0x203, 16, 16, 16) \
  X(4096, 6, 512, 2, 16, 2, 0x1000, 8, 8, 8, 8) \
  X(4096, 7, 256, 2, 16, 2, 0x1000, 16, 16, 16) \
  X(4096, 8, 256, 4, 16, 2, 0x7403, 16, 16, 16) \
  X(4096, 9, 256, 4, 8, 2, 0x7403, 16, 16, 16) \
  X(4096, 10, 128, 4, 16, 2, 0x8400, 16, 16, 16)

// LDS of a pass workgroup (line tiles, plus the FP64 reduction scratch)
// against the 160 KiB a gfx950 workgroup may allocate.
constexpr size_t kMaxLdsBytes = 160 * 1024;
// (pipelined plans also hold the twiddles of every stage, N - R0 entries,
// or a quarter table of N / 4 and the second stage's (R1 - 1) R0 entries)
template <typename R, class P>
constexpr size_t plan_lds_bytes(bool column) {
  const size_t tile =
      column ? size_t(LdsPointMajor<R, P::LINES, P::PA, P::PB>::size(P::HX ? P::N / 2 : P::N))
             : size_t(P::LINES) * LdsLineMajor<R, P::N>::LINE;
  const size_t tw = (P::HX || P::QTW) ? size_t(qtw_entries<P::N>(typename P::radices{}))
                    : !P::PIPE         ? 0
                                       : size_t(lds_tw_entries<P::N>(typename P::radices{}));
  return (tile + tw) * sizeof(cx<R>) + sizeof(double) * 8 * ((P::THREADS + 63) / 64);
}
// Pipelined (persistent) plans are built for complex64 only, rows with one
// row per workgroup; half-exchange plans for complex64 columns only.
template <typename R, class P>
constexpr bool plan_fits(bool column) {
  return plan_lds_bytes<R, P>(column) <= kMaxLdsBytes &&
         !(P::PIPE && (sizeof(R) != 4 || (!column && P::LINES != 1))) &&
         !(P::HX && (sizeof(R) != 4 || !column));
}

template <int N, int V>
struct RowPlanSel;
template <int N, int V>
struct ColPlanSel;

#define SSFM_DEF_ROW(NN, VV, TT, LL, OO, ...) \
  template <> struct RowPlanSel<NN, VV> { using P = Plan<NN, TT, LL, Radices<__VA_ARGS__>, 32, 0, OO>; };
#define SSFM_DEF_COL(NN, VV, TT, LL, AA, BB, OO, ...) \
  template <> struct ColPlanSel<NN, VV> { using P = Plan<NN, TT, LL, Radices<__VA_ARGS__>, AA, BB, OO>; };
SSFM_ROW_PLANS(SSFM_DEF_ROW)
SSFM_COL_PLANS(SSFM_DEF_COL)
#undef SSFM_DEF_ROW
#undef SSFM_DEF_COL

}  // namespace ssfm
