// ssfm.cpp -- host plan, workspace layout and the C ABI of libssfm.
//
// The host side turns beam descriptions into device tables (twiddles and
// diffraction factors computed in FP64 and rounded once, per-beam screen
// constants), builds the per-pass work lists, and drives the march:
//
//   forward step n   ROW_FWD (pending screen n-1 applied on load) -> COL_FWD
//   adjoint step n   COL_ADJ -> ROW_ADJ (adjoint of screen n-1 fused)
//
// All beams of a context march in lock-step; beams of equal grid size share
// one launch per pass, so a batch of uneven beams costs one launch per
// distinct size per pass (captured once into a HIP graph and replayed).
#include "../../include/ssfm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "lens_vjp.hpp"
#include "subharmonics.hpp"

using namespace ssfm;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(SSFM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                             \
  } while (0)

constexpr int kDiagChunk = 64;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool supported_n(int n) {
  return n == 128 || n == 256 || n == 512 || n == 768 || n == 1024 || n == 2048 || n == 4096;
}

int validate_desc(const ssfm_instance_desc* d, int32_t n_inst, int32_t precision) {
  if (!d) return fail(SSFM_EINVAL, "desc is NULL");
  if (n_inst < 1 || n_inst > 65536) return fail(SSFM_EINVAL, "n_inst %d out of range", n_inst);
  if (precision != SSFM_FP32 && precision != SSFM_FP64)
    return fail(SSFM_EINVAL, "precision must be 32 or 64, got %d", precision);
  for (int i = 0; i < n_inst; ++i) {
    const ssfm_instance_desc& x = d[i];
    if (!supported_n(x.n))
      return fail(SSFM_EUNSUPPORTED, "instance %d: grid size %d not supported", i, x.n);
    if (!(x.length > 0) || !(x.dz > 0) || !(x.wavelength > 0) || !(x.i_ref > 0))
      return fail(SSFM_EINVAL, "instance %d: length, dz, wavelength, i_ref must be > 0", i);
    if (x.terms & ~31u) return fail(SSFM_EINVAL, "instance %d: unknown term bits", i);
    if ((x.terms & (SSFM_MPA | SSFM_PLASMA)) && x.mpa_order < 2)
      return fail(SSFM_EINVAL, "instance %d: mpa_order must be >= 2", i);
    if (x.mpa_order > 32) return fail(SSFM_EINVAL, "instance %d: mpa_order > 32", i);
    if (x.n_screens < 0 || x.n_screens > 4096)
      return fail(SSFM_EINVAL, "instance %d: n_screens out of range", i);
    if ((x.terms & SSFM_TURB) && x.n_screens > 0 && (!(x.screen_dz > 0) || !(x.cn2 >= 0)))
      return fail(SSFM_EINVAL, "instance %d: turbulence needs screen_dz > 0, cn2 >= 0", i);
    // closer screens could fall on one step (or before the first one)
    if ((x.terms & SSFM_TURB) && x.n_screens > 0 && !(x.screen_dz >= x.dz))
      return fail(SSFM_EINVAL, "instance %d: screen_dz %g below dz %g", i, x.screen_dz, x.dz);
  }
  return SSFM_OK;
}

// Device-side layout of everything a context keeps in the workspace.
struct Layout {
  size_t inst, steps, work, wbegin_row, wbegin_col, tables;
  size_t S, Wk, Lam, ckpt, stack, screens, stage, diag_part, diag, theta_acc,
      theta_out, seed_loss, seed_theta, scal, sumsq_part, lens_inst, half_inst, back_inst,
      fd_inst, subh, subh_beams;
  size_t total;
  int64_t field_elems;  // sum n^2
  int64_t table_elems;
  int64_t n_work_rows, n_work_cols;  // launch entries (with padding)
  int64_t n_widx_rows, n_widx_cols;  // real work items
  int64_t n_ckpt, n_stack, diag_cap, screen_elems, n_steps_total;
  // regions of n_stack segment slots: recompute banks (0, 1 or 2) and
  // segments kept whole by the forward record
  int64_t n_banks, n_kept;
  int max_n;
};

struct Group {
  int n;
  int row_var = 0, col_var = 0;
  // variants of the adjoint passes (-1: the forward ones); same lines per
  // workgroup as the forward variant, so the work lists are shared
  int row_adj_var = -1, col_adj_var = -1;
  std::vector<int> beams;
  // launch order (XCD-aware), offsets into the work array
  int64_t row_work_off = 0, col_work_off = 0;
  int row_blocks = 0, col_blocks = 0;
};

}  // namespace

struct ssfm_ctx {
  int precision = SSFM_FP32;
  size_t el = 8;  // bytes per complex element
  std::vector<ssfm_instance_desc> desc;
  std::vector<InstDev> inst;
  std::vector<int64_t> screen_steps;
  std::vector<int64_t> lens_off;  // element offset of each beam's lens filter table
  // Strang splitting: the state holds V = L(dz/2) U and every step applies
  // its own screen on load; half_off / back_off: tables of L(+-dz/2)
  bool strang = false;
  std::vector<int64_t> half_off, back_off;
  // finite-difference reference scheme (Crank-Nicolson, fixed-point
  // iterations per step); fd_off: each beam's table of
  // d[m] = (dz / (k0 dx^2)) sin^2(pi m / n)
  bool fd = false;
  int fd_iters = 4;
  std::vector<int64_t> fd_off;
  std::vector<SubBeam> sub_beams;  // host copy of the last uploaded subharmonic list
  struct Spectrum {
    int kind = SSFM_SPECTRUM_KOLMOGOROV;
    double tau = 0.0, kappa_h = 0.0;
    int subharmonics = 0;  // subharmonic levels added to each screen
  };
  std::vector<Spectrum> spectrum;  // per beam, for gen_screens
  std::vector<Group> groups;
  std::vector<WorkItem> work;  // all launch entries, group by group
  std::vector<int32_t> wbegin_row, wbegin_col;
  Layout L{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t max_steps = 0;
  int32_t ckpt_every = 1;
  int32_t stored_segments = 0;  // last segments of a record kept whole
  // march state
  int64_t step = 0;        // steps taken since the last set_field
  bool pending = false;    // state holds V with its screen still to apply
  int64_t diag_valid = 0;  // steps of diag kept from the last call
  // adjoint record
  int64_t rec_steps = 0, rec_step0 = 0;
  bool rec_valid = false, seeded = false, grads_valid = false;
  // backward sweep: recompute of the next segment on the second stream
  // beside the adjoint of the current one (else after it, on the stream)
  bool overlap_recompute = false;
  std::vector<char> seeded_beam;  // per beam: cotangent set since the record
  bool use_graphs = true;
  std::map<std::tuple<int, int64_t, int64_t, int64_t, int64_t>, hipGraphExec_t> graphs;
  // Sampled pass timing (0: off): with timing_every = m, step s of a
  // forward march with s % m == m / 2 runs outside the step graphs, each of
  // its pass kernels launched with start/stop events on its own dispatch;
  // samples holds those of the most recent forward march.  ev[2 * (p * G +
  // g) + {0, 1}]: start/stop of pass p (0 row, 1 column) for size group g.
  struct PassSample {
    std::vector<hipEvent_t> ev;
  };
  int32_t timing_every = 0;
  std::vector<PassSample> samples, free_samples;
  // samples of the most recent backward: adjoint steps s of its first
  // segment (which runs alone, not beside a recompute) with
  // s % timing_every == timing_every / 2; pass 0 the column pass, 1 the row
  // pass
  std::vector<PassSample> adj_samples;
  // second stream (default priority) and events for the overlapped backward
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // streams and events for running the grid-size groups of one pass
  // concurrently on the main chain (group g > 0 on gstream[g - 1])
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gjoin;
  hipEvent_t gfork = nullptr;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  void* field(size_t off, int64_t k = 0) const {
    return ws + off + size_t(k) * size_t(L.field_elems) * el;
  }
  static void destroy(std::vector<PassSample>& v) {
    for (auto& e : v)
      for (auto x : e.ev) (void)hipEventDestroy(x);
    v.clear();
  }
  ~ssfm_ctx() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    destroy(samples);
    destroy(free_samples);
    destroy(adj_samples);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
    for (auto s : gstream) (void)hipStreamDestroy(s);
    for (auto e : gjoin) (void)hipEventDestroy(e);
    if (gfork) (void)hipEventDestroy(gfork);
  }
};

namespace {

// Per-beam screen step list (turbulence): screen s (1-based) sits at
// z_s = (s - 1/2) dz_s and is applied after step floor(z_s / dz + 1/2) - 1
// (the step that reaches z_s; ties round up).
std::vector<int64_t> screen_step_list(const ssfm_instance_desc& d) {
  std::vector<int64_t> out;
  if (!(d.terms & SSFM_TURB)) return out;
  for (int s = 1; s <= d.n_screens; ++s) {
    const double zs = (s - 0.5) * d.screen_dz;
    out.push_back(int64_t(std::floor(zs / d.dz + 0.5)) - 1);
  }
  return out;
}

// Eq. (10) band in mode-index units: the Fourier mode m = (mx, my) of a
// window of side L has kappa = 2 pi |m| / L, so kappa <= kappa_h reads
// |m|^2 <= (kappa_h L / 2 pi)^2.  That bound is formed once here, with a
// relative slack of 2^-40 so that a kappa_h placed on a ring of modes keeps
// the ring whatever the rounding; the kernels then decide on the exact
// integer |m|^2.
double band_q2(double length, double kappa_h) {
#pragma clang fp contract(off)
  const double q = kappa_h * length / (2.0 * M_PI);
  return q * q * (1.0 + 0x1p-40);
}

// Groups by grid size in first-appearance order.
std::vector<Group> make_groups(const ssfm_instance_desc* d, int n_inst) {
  std::vector<Group> g;
  for (int i = 0; i < n_inst; ++i) {
    auto it = std::find_if(g.begin(), g.end(), [&](const Group& x) { return x.n == d[i].n; });
    if (it == g.end()) {
      Group ng;
      ng.n = d[i].n;
      ng.beams.push_back(i);
      g.push_back(ng);
    } else {
      it->beams.push_back(i);
    }
  }
  return g;
}

// XCD-aware launch order: workgroups are dispatched round-robin over the 8
// XCDs (blockIdx mod 8), so entry b runs on XCD b % 8.  Giving each XCD a
// contiguous run of work items keeps neighbouring lines (which share cache
// lines in the column pass) in one XCD's L2.
std::vector<WorkItem> xcd_order(const std::vector<WorkItem>& items) {
  const size_t n = items.size();
  const size_t m = (n + 7) / 8 * 8;
  const size_t chunk = m / 8;
  std::vector<WorkItem> out(m, WorkItem{-1, 0, -1, 0});
  for (size_t b = 0; b < m; ++b) {
    const size_t x = b % 8, q = b / 8;
    const size_t t = x * chunk + q;
    if (t < n) out[b] = items[t];
  }
  return out;
}

// Builds groups, work lists and the layout.  Pure host computation.
using VariantMap = std::map<int, std::pair<int, int>>;  // n -> (row, column)

// Largest number of work items any variant gives a beam of size n.
int64_t max_items(bool column, int n, bool fp64) {
  int64_t m = 0;
  for (int v = 0; v < plan_count(column, n); ++v) {
    PlanInfo pi;
    if (plan_info(column, n, v, fp64, &pi)) m = std::max<int64_t>(m, n / pi.lines);
  }
  return m;
}

int plan_layout(const ssfm_instance_desc* d, int n_inst, int precision, int64_t max_steps,
                int32_t ckpt_every, int32_t stored_segments, const VariantMap* variants,
                std::vector<Group>* groups_out,
                std::vector<WorkItem>* work_out, std::vector<int32_t>* wb_row,
                std::vector<int32_t>* wb_col, Layout* L) {
  const size_t el = precision == SSFM_FP64 ? 16 : 8;
  const size_t rel = el / 2;
  std::vector<Group> groups = make_groups(d, n_inst);
  if (variants) {
    for (auto& g : groups) {
      auto it = variants->find(g.n);
      if (it != variants->end()) {
        g.row_var = it->second.first;
        g.col_var = it->second.second;
      }
    }
  }
  // beam-contiguous work indices
  std::vector<int32_t> row_first(n_inst + 1), col_first(n_inst + 1);
  int64_t nr = 0, nc = 0;
  std::vector<PlanInfo> rinfo(n_inst), cinfo(n_inst);
  for (auto& g : groups) {
    PlanInfo ri, ci;
    if (!plan_info(false, g.n, g.row_var, precision == SSFM_FP64, &ri) ||
        !plan_info(true, g.n, g.col_var, precision == SSFM_FP64, &ci))
      return fail(SSFM_EUNSUPPORTED, "no kernel plan for n=%d", g.n);
    for (int b : g.beams) {
      rinfo[b] = ri;
      cinfo[b] = ci;
    }
  }
  for (int b = 0; b < n_inst; ++b) {
    row_first[b] = int32_t(nr);
    col_first[b] = int32_t(nc);
    nr += d[b].n / rinfo[b].lines;
    nc += d[b].n / cinfo[b].lines;
  }
  row_first[n_inst] = int32_t(nr);
  col_first[n_inst] = int32_t(nc);
  std::vector<WorkItem> work;
  for (auto& g : groups) {
    std::vector<WorkItem> rows, cols;
    for (int b : g.beams) {
      const int rl = rinfo[b].lines, cl = cinfo[b].lines;
      for (int k = 0; k < d[b].n / rl; ++k)
        rows.push_back(WorkItem{b, k * rl, row_first[b] + k, 0});
      for (int k = 0; k < d[b].n / cl; ++k)
        cols.push_back(WorkItem{b, k * cl, col_first[b] + k, 0});
    }
    auto ro = xcd_order(rows), co = xcd_order(cols);
    g.row_work_off = int64_t(work.size());
    g.row_blocks = int(ro.size());
    work.insert(work.end(), ro.begin(), ro.end());
    g.col_work_off = int64_t(work.size());
    g.col_blocks = int(co.size());
    work.insert(work.end(), co.begin(), co.end());
  }
  // partial-sum arrays are sized for the variant with the most work items
  int64_t nr_max = 0, nc_max = 0;
  for (int b = 0; b < n_inst; ++b) {
    nr_max += max_items(false, d[b].n, precision == SSFM_FP64);
    nc_max += max_items(true, d[b].n, precision == SSFM_FP64);
  }
  Layout l{};
  int64_t fe = 0, te = 0, se = 0, nsteps = 0, subh_doubles = 0;
  int max_n = 0;
  std::vector<int> tw_done;
  for (int b = 0; b < n_inst; ++b) {
    fe += int64_t(d[b].n) * d[b].n;
    max_n = std::max(max_n, d[b].n);
    if (std::find(tw_done.begin(), tw_done.end(), d[b].n) == tw_done.end()) {
      tw_done.push_back(d[b].n);
      te += d[b].n;
    }
    // propagator, lens filter, +/- half-step propagators, finite-difference table
    te += 5 * int64_t(d[b].n);
    if (d[b].terms & SSFM_TURB) {
      se += int64_t(d[b].n_screens) * d[b].n * d[b].n;
      nsteps += d[b].n_screens;
      subh_doubles += subharmonic_region_doubles(d[b].n, (d[b].n_screens + 1) / 2);
    }
  }
  l.field_elems = fe;
  l.table_elems = te;
  l.screen_elems = se;
  l.n_steps_total = nsteps;
  l.max_n = max_n;
  l.n_work_rows = nr;
  l.n_work_cols = nc;
  l.n_widx_rows = nr;
  l.n_widx_cols = nc;
  if (max_steps > 0) {
    const int64_t m = std::max<int64_t>(1, ckpt_every);
    const int64_t seg = std::min<int64_t>(m, max_steps);
    l.n_ckpt = (max_steps + seg - 1) / seg;
    l.n_stack = seg - 1;
    if (l.n_ckpt == 1) {
      l.n_banks = 0;  // a single segment is always kept whole
      l.n_kept = 1;
    } else {
      l.n_kept = std::min<int64_t>(stored_segments, l.n_ckpt);
      l.n_banks = std::min<int64_t>(2, l.n_ckpt - l.n_kept);
    }
  }
  l.diag_cap = std::max<int64_t>(max_steps, 4096);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  l.inst = take(sizeof(InstDev) * n_inst);
  l.steps = take(sizeof(int64_t) * std::max<int64_t>(nsteps, 1));
  // room for the work list of any variant choice (with XCD padding)
  l.work = take(sizeof(WorkItem) * size_t(nr_max + nc_max + 16 * groups.size()));
  l.wbegin_row = take(sizeof(int32_t) * (n_inst + 1));
  l.wbegin_col = take(sizeof(int32_t) * (n_inst + 1));
  l.tables = take(el * te);
  l.S = take(el * fe);
  l.Wk = take(el * fe);
  // (with more than one segment the recompute of the next segment runs
  // beside the adjoint of the current one, in its own bank of segment
  // slots; both work in place)
  l.Lam = take(max_steps > 0 ? el * fe : 0);
  l.ckpt = take(el * fe * l.n_ckpt);
  l.stack = take(el * fe * l.n_stack * (l.n_banks + l.n_kept));
  l.screens = take(rel * se);
  l.stage = take(16 * size_t(max_n) * max_n);
  // power partials of column work items (split-step) or row work items
  // (finite differences)
  l.diag_part = take(sizeof(double) * 2 * kDiagChunk * std::max(nr_max, nc_max));
  l.diag = take(sizeof(double) * 2 * l.diag_cap * n_inst);
  l.theta_acc = take(sizeof(double) * 8 * nr_max);
  l.theta_out = take(sizeof(double) * 8 * n_inst);
  l.seed_loss = take(sizeof(double) * max_n);
  l.seed_theta = take(sizeof(double) * 8 * max_n * n_inst);
  l.scal = take(sizeof(double) * 16);
  // 256 partials of a sum of squares, moment or hot-area count, then 256 x 5
  // measure-vector partials
  l.sumsq_part = take(sizeof(double) * 256 * 6);
  l.lens_inst = take(sizeof(InstDev) * n_inst);
  l.half_inst = take(sizeof(InstDev) * n_inst);
  l.back_inst = take(sizeof(InstDev) * n_inst);
  l.fd_inst = take(sizeof(InstDev) * n_inst);
  // subharmonic tables and coefficients of every turbulent beam, its beam list
  l.subh = take(sizeof(double) * size_t(subh_doubles));
  l.subh_beams = take(sizeof(SubBeam) * n_inst);
  l.total = off;
  if (groups_out) *groups_out = groups;
  if (work_out) *work_out = work;
  if (wb_row) *wb_row = row_first;
  if (wb_col) *wb_col = col_first;
  *L = l;
  return SSFM_OK;
}

// exp(-2 pi i m / n) in FP64, rounded to the working precision.
void twiddles(int n, std::vector<double>* out) {
  out->resize(2 * size_t(n));
  for (int m = 0; m < n; ++m) {
    const double a = 2.0 * M_PI * double(m) / double(n);
    (*out)[2 * m] = std::cos(a);
    (*out)[2 * m + 1] = -std::sin(a);
  }
}

// exp(-i k_m^2 dz / 2k0) / n, phase reduced modulo 2 pi in FP64.
void propagator(const ssfm_instance_desc& d, std::vector<double>* out) {
  const int n = d.n;
  const double k0 = 2.0 * M_PI / d.wavelength;
  out->resize(2 * size_t(n));
  for (int m = 0; m < n; ++m) {
    const int ms = (m <= n / 2) ? m : m - n;
    const double k = 2.0 * M_PI * double(ms) / d.length;
    double ph = std::fmod(k * k * d.dz / (2.0 * k0), 2.0 * M_PI);
    (*out)[2 * m] = std::cos(ph) / n;
    (*out)[2 * m + 1] = -std::sin(ph) / n;
  }
}

template <typename R>
void append_table(std::vector<unsigned char>* blob, const std::vector<double>& v) {
  const size_t n = v.size();
  const size_t o = blob->size();
  blob->resize(o + n * sizeof(R));
  R* p = reinterpret_cast<R*>(blob->data() + o);
  for (size_t i = 0; i < n; ++i) p[i] = R(v[i]);
}

int check_ctx(ssfm_ctx* c) {
  if (!c) return fail(SSFM_EINVAL, "ctx is NULL");
  return SSFM_OK;
}

int check_inst(ssfm_ctx* c, int32_t i) {
  if (int r = check_ctx(c)) return r;
  if (i < 0 || i >= int32_t(c->desc.size()))
    return fail(SSFM_EINVAL, "instance %d out of range [0, %zu)", i, c->desc.size());
  return SSFM_OK;
}

// Forget a recorded march, its cotangents and gradients (the fields or
// parameters it was recorded with have changed).
void drop_record(ssfm_ctx* c) {
  c->rec_valid = false;
  c->seeded = false;
  c->grads_valid = false;
  c->seeded_beam.assign(c->desc.size(), 0);
}

// Copy beam table entries [b0, b1) to the device (stream-ordered; waits,
// the host table may change right after).
int upload_inst(ssfm_ctx* c, size_t b0, size_t b1) {
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.inst + sizeof(InstDev) * b0, &c->inst[b0],
                         sizeof(InstDev) * (b1 - b0), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SSFM_OK;
}

// ---------------------------------------------------------------- passes
template <typename R>
PassArgs<R> base_args(ssfm_ctx* c) {
  PassArgs<R> a{};
  a.inst = c->at<InstDev>(c->L.inst);
  a.tables = c->ws + c->L.tables;
  a.screens = c->at<R>(c->L.screens);
  a.screen_steps = c->at<int64_t>(c->L.steps);
  a.step = -1;
  for (const auto& in : c->inst)
    if (in.terms & (1u << 8)) a.precise = 1;
  return a;
}

// One pass over every beam: one launch per grid-size group.  On the main
// chain (the context's stream, the primary stream of a graph capture) the
// groups run concurrently (group g > 0 on its own stream, forked from and
// joined back to st), so their ramps and tails overlap.  On the auxiliary
// chain (the checkpoint recompute, itself a fork of the main chain) they
// run in sequence on that stream: a stream capture must join every fork
// to its primary stream, and a fork of a fork would be joined to the
// auxiliary stream instead.
template <typename R>
int run_pass(ssfm_ctx* c, int kind, PassArgs<R> a, hipStream_t st = nullptr,
             const hipEvent_t* ev = nullptr) {
  const bool col = is_col_kind(kind);
  if (!st) st = c->stream;
  const size_t ng = c->groups.size();
  const bool fork = st != c->aux && ng > 1 && c->gstream.size() + 1 >= ng;
  if (fork) {
    HIP_TRY(hipEventRecord(c->gfork, st));
    for (size_t g = 1; g < ng; ++g) HIP_TRY(hipStreamWaitEvent(c->gstream[g - 1], c->gfork, 0));
  }
  for (size_t gi = 0; gi < ng; ++gi) {
    const Group& g = c->groups[gi];
    a.work = c->at<WorkItem>(c->L.work) + (col ? g.col_work_off : g.row_work_off);
    const int nb = col ? g.col_blocks : g.row_blocks;
    const int v = col ? ((kind == COL_ADJ && g.col_adj_var >= 0) ? g.col_adj_var : g.col_var)
                      : ((kind == ROW_ADJ && g.row_adj_var >= 0) ? g.row_adj_var : g.row_var);
    hipStream_t sg = (fork && gi > 0) ? c->gstream[gi - 1] : st;
    const LaunchEv le = ev ? LaunchEv{ev[2 * gi], ev[2 * gi + 1]} : LaunchEv{nullptr, nullptr};
    HIP_TRY(launch_pass<R>(kind, g.n, v, nb, a, sg, ev ? &le : nullptr));
  }
  if (fork) {
    for (size_t g = 1; g < ng; ++g) {
      HIP_TRY(hipEventRecord(c->gjoin[g - 1], c->gstream[g - 1]));
      HIP_TRY(hipStreamWaitEvent(st, c->gjoin[g - 1], 0));
    }
  }
  return SSFM_OK;
}

// One forward step: src (s_n) -> work -> dst (s_{n+1}), on stream st.
// A timing sample (a start/stop pair per pass and size group) from the
// pool; false if none could be made.
bool take_sample(ssfm_ctx* c, ssfm_ctx::PassSample* ps) {
  const size_t need = 4 * c->groups.size();
  if (!c->free_samples.empty()) {
    *ps = std::move(c->free_samples.back());
    c->free_samples.pop_back();
    if (ps->ev.size() == need) return true;
    for (auto x : ps->ev) (void)hipEventDestroy(x);
  }
  ps->ev.assign(need, nullptr);
  for (auto& x : ps->ev)
    if (hipEventCreate(&x) != hipSuccess) {
      for (auto y : ps->ev)
        if (y) (void)hipEventDestroy(y);
      ps->ev.clear();
      (void)hipGetLastError();  // timing is best effort: the march proceeds unsampled
      return false;
    }
  return true;
}

void clear_graphs(ssfm_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Whether steps into fresh slots of the stored trajectory go through the
// work buffer (see fwd_step): for beams whose field spans at least 64 MiB
// (4096^2 complex64 and up), where it measures faster; the 1024^2 march
// measures faster with the column pass in place on the slot.
bool fresh_via_work(const ssfm_ctx* c) {
  return int64_t(c->L.max_n) * c->L.max_n * int64_t(c->el) >= (int64_t(64) << 20);
}

template <typename R>
int fwd_step(ssfm_ctx* c, const void* src, void* dst, int64_t pending_step, double* part,
             void* work = nullptr, hipStream_t st = nullptr,
             const ssfm_ctx::PassSample* ts = nullptr) {
  // both passes transform whole lines, each read and written by one
  // workgroup, so the row pass can write straight into dst and the column
  // pass finish there in place.  For large beams a step into a fresh slot
  // of the stored trajectory goes through a work buffer instead (row pass
  // into it, column pass out of it): the column pass then reads a buffer
  // every step uses and only its stores touch the new slot, which measures
  // faster than column reads and writes on the freshly written slot there.
  if (!work) work = dst;
  if (!st) st = c->stream;
  PassArgs<R> a = base_args<R>(c);
  a.src = src;
  a.dst = work;
  a.step = pending_step;
  const size_t ng = c->groups.size();
  if (int r = run_pass<R>(c, ROW_FWD, a, st, ts ? ts->ev.data() : nullptr)) return r;
  PassArgs<R> b = base_args<R>(c);
  b.src = work;
  b.dst = dst;
  b.part = part;
  b.flags = c->strang ? 1 : 0;  // Strang: |U|^2 = |V|^2 summed as it is
  return run_pass<R>(c, COL_FWD, b, st, ts ? ts->ev.data() + 2 * ng : nullptr);
}

// One adjoint step: Lam -> Wk (columns) -> Lam (rows + adjoint screen with
// the pre-screen field `sv` of the screen applied after step pending_step).
// ts: timing events around the two passes (sampled steps only).
template <typename R>
int adj_step(ssfm_ctx* c, const void* sv, int64_t pending_step,
             const ssfm_ctx::PassSample* ts = nullptr) {
  const size_t ng = c->groups.size();
  // both passes in place on the cotangent (whole lines per workgroup)
  PassArgs<R> a = base_args<R>(c);
  a.src = c->field(c->L.Lam);
  a.dst = c->field(c->L.Lam);
  if (int r = run_pass<R>(c, COL_ADJ, a, nullptr, ts ? ts->ev.data() : nullptr)) return r;
  PassArgs<R> b = base_args<R>(c);
  b.src = c->field(c->L.Lam);
  b.dst = c->field(c->L.Lam);
  b.aux = sv;
  b.step = pending_step;
  b.part = c->at<double>(c->L.theta_acc);
  return run_pass<R>(c, ROW_ADJ, b, nullptr, ts ? ts->ev.data() + 2 * ng : nullptr);
}

template <typename R>
int diag_flush(ssfm_ctx* c, int steps, int64_t first_step) {
  HIP_TRY(launch_diag_finalize(c->at<double>(c->L.diag_part), int(c->L.n_widx_cols),
                               c->at<int32_t>(c->L.wbegin_col), int(c->desc.size()), steps,
                               c->at<double>(c->L.diag), first_step, c->L.diag_cap, 0.0,
                               c->stream));
  return SSFM_OK;
}

// Enqueue steps i0 <= i < i1 of a plain forward march from step0 (step
// step0 + i; pending0: the state holds V with the screen of step0 - 1 still
// to apply).  ts: timing events around the passes (single steps only).
template <typename R>
int enqueue_propagate(ssfm_ctx* c, int64_t step0, bool pending0, int64_t i0, int64_t i1,
                      const ssfm_ctx::PassSample* ts) {
  int64_t chunk_start = step0 + i0;
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t step = step0 + i;
    const int slot = int((i - i0) % kDiagChunk);
    double* part = c->at<double>(c->L.diag_part) + size_t(slot) * 2 * c->L.n_widx_cols;
    // Lie: the screen of the previous step, pending in the state; Strang:
    // the state is V = L(dz/2) U and this step's own screen acts first
    const int64_t pend = c->strang ? step : ((i == 0 && !pending0) ? -1 : step - 1);
    if (int r = fwd_step<R>(c, c->field(c->L.S), c->field(c->L.S), pend, part, nullptr, nullptr,
                            ts))
      return r;
    if (slot == kDiagChunk - 1 || i == i1 - 1) {
      if (int r = diag_flush<R>(c, slot + 1, chunk_start)) return r;
      chunk_start = step + 1;
    }
  }
  return SSFM_OK;
}

// Steps i0 <= i < i1 of a finite-difference march from step step0 + i0, on
// S (U) and Wk (the row-transformed right-hand side).  The first row pass
// forms U + (dz/2) G(|U|^2) U from S; each of the fd_iters iterations is a
// column pass (the solve) and a row pass (Ubar, then the next right-hand
// side); the last row pass of a step writes U+ = 2 Ubar - U and its power
// partials and, unless the range ends, starts the next step.
template <typename R>
int enqueue_fd(ssfm_ctx* c, int64_t step0, int64_t i0, int64_t i1) {
  PassArgs<R> a = base_args<R>(c);
  a.inst = c->at<InstDev>(c->L.fd_inst);
  a.state = c->field(c->L.S);
  a.src = c->field(c->L.S);
  a.dst = c->field(c->L.Wk);
  a.flags = 0;
  if (int r = run_pass<R>(c, ROW_FD, a)) return r;
  PassArgs<R> col = base_args<R>(c);
  col.inst = a.inst;
  col.src = c->field(c->L.Wk);
  col.dst = c->field(c->L.Wk);
  a.src = c->field(c->L.Wk);
  int64_t chunk_start = step0 + i0;
  for (int64_t i = i0; i < i1; ++i) {
    const int slot = int((i - i0) % kDiagChunk);
    for (int k = 1; k <= c->fd_iters; ++k) {
      if (int r = run_pass<R>(c, COL_FD, col)) return r;
      const bool fin = (k == c->fd_iters);
      a.flags = FD_SPECTRAL | (fin ? FD_FINISH : 0) | ((fin && i == i1 - 1) ? FD_LAST : 0);
      a.part = fin ? c->at<double>(c->L.diag_part) + size_t(slot) * 2 * c->L.n_widx_rows
                   : nullptr;
      if (int r = run_pass<R>(c, ROW_FD, a)) return r;
    }
    if (slot == kDiagChunk - 1 || i == i1 - 1) {
      HIP_TRY(launch_diag_finalize(c->at<double>(c->L.diag_part), int(c->L.n_widx_rows),
                                   c->at<int32_t>(c->L.wbegin_row), int(c->desc.size()),
                                   slot + 1, c->at<double>(c->L.diag), chunk_start,
                                   c->L.diag_cap, 0.0, c->stream));
      chunk_start = step0 + i + 1;
    }
  }
  return SSFM_OK;
}

// Runs `body` directly or through a cached graph keyed by (kind, a, b, i0, i1).
template <typename F>
int maybe_graph(ssfm_ctx* c, int kind, int64_t a, int64_t b, int64_t i0, int64_t i1, F body) {
  if (!c->use_graphs) return body();
  auto key = std::make_tuple(kind, a, b, i0, i1);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    // graphs are specific to their first step; a caller marching in many
    // small chunks would grow the cache without bound, so past a limit it
    // is emptied (after the stream drains, so no cached graph still runs)
    constexpr size_t kMaxGraphs = 128;
    if (c->graphs.size() >= kMaxGraphs) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      clear_graphs(c);
    }
    hipStream_t cap;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      c->stream = saved;
      (void)hipStreamDestroy(cap);
      return fail(SSFM_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    int r = body();
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    c->stream = saved;
    (void)hipStreamDestroy(cap);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e2 != hipSuccess) return fail(SSFM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(SSFM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e3));
    it = c->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, c->stream));
  return SSFM_OK;
}

// Steps [0, n) of a forward march from step0 through seg(i0, i1, ts): in
// captured graphs keyed by (kind, key, n, i0, i1) between the sampled steps,
// each sampled step launched directly between its timing events.
template <typename Seg>
int run_forward(ssfm_ctx* c, int kind, int64_t key, int64_t n, int64_t step0, Seg seg) {
  for (auto& e : c->samples) c->free_samples.push_back(e);
  c->samples.clear();
  int64_t i = 0;
  auto graph_to = [&](int64_t k) -> int {
    if (k <= i) return SSFM_OK;
    const int64_t i0 = i;
    return maybe_graph(c, kind, key, n, i0, k, [&] { return seg(i0, k, nullptr); });
  };
  const int64_t m = c->timing_every;
  if (m > 0) {
    int64_t first = (m / 2 - step0 % m) % m;  // first i with (step0 + i) % m == m / 2
    if (first < 0) first += m;
    for (int64_t k = first; k < n; k += m) {
      if (int r = graph_to(k)) return r;
      ssfm_ctx::PassSample ps;
      const bool have = take_sample(c, &ps);
      int r = seg(k, k + 1, have ? &ps : nullptr);
      if (have) c->samples.push_back(std::move(ps));
      if (r) return r;
      i = k + 1;
    }
  }
  return graph_to(n);
}

template <typename R>
int do_propagate(ssfm_ctx* c, int64_t n) {
  const int64_t step0 = c->step;
  const bool pend = c->pending;
  if (c->fd) {
    // one graph per (start step, length): the diagnostics ring slots depend
    // on the absolute step
    int r = maybe_graph(c, 3, step0, n, 0, n, [&] { return enqueue_fd<R>(c, step0, 0, n); });
    if (r) return r;
    c->step += n;
    c->pending = false;
    c->diag_valid = std::min<int64_t>(n, c->L.diag_cap);
    c->rec_valid = false;
    c->seeded = false;
    c->seeded_beam.assign(c->desc.size(), 0);
    return SSFM_OK;
  }
  int r = run_forward(c, 0, step0 * 2 + (pend ? 1 : 0), n, step0,
                      [&](int64_t i0, int64_t i1, const ssfm_ctx::PassSample* ts) {
                        return enqueue_propagate<R>(c, step0, pend, i0, i1, ts);
                      });
  if (r) return r;
  c->step += n;
  c->pending = !c->strang;
  c->diag_valid = std::min<int64_t>(n, c->L.diag_cap);
  c->rec_valid = false;
  c->seeded = false;
  c->seeded_beam.assign(c->desc.size(), 0);
  return SSFM_OK;
}

// Half-step diffraction L(+-dz/2) of every beam: S -> Wk through the pass
// kernels with the half-step tables (no screen).
template <typename R>
int half_steps(ssfm_ctx* c, bool forward) {
  HIP_TRY(launch_copy<R>(c->field(c->L.S), c->field(c->L.Wk), c->L.field_elems, c->stream));
  PassArgs<R> a = base_args<R>(c);
  a.inst = c->at<InstDev>(forward ? c->L.half_inst : c->L.back_inst);
  a.src = c->field(c->L.Wk);
  a.dst = c->field(c->L.Wk);
  if (int r = run_pass<R>(c, ROW_FWD, a)) return r;
  return run_pass<R>(c, COL_FWD, a);
}

// Lam <- L(+-dz/2) Lam in place (the half-step tables, no screen).
template <typename R>
int half_step_lam(ssfm_ctx* c, bool forward) {
  PassArgs<R> a = base_args<R>(c);
  a.inst = c->at<InstDev>(forward ? c->L.half_inst : c->L.back_inst);
  a.src = c->field(c->L.Lam);
  a.dst = c->field(c->L.Lam);
  if (int r = run_pass<R>(c, ROW_FWD, a)) return r;
  return run_pass<R>(c, COL_FWD, a);
}

// Apply the pending screen in place (state becomes U_n).
template <typename R>
int flush_pending(ssfm_ctx* c) {
  if (!c->pending) return SSFM_OK;
  // store_field into the stage buffer (complex128, device units) per beam,
  // then load it back: a pointwise round trip through the staging area.
  for (size_t b = 0; b < c->desc.size(); ++b) {
    const InstDev& in = c->inst[b];
    const int64_t n2 = int64_t(in.n) * in.n;
    double* stage = c->at<double>(c->L.stage);
    HIP_TRY(launch_store_field<R>(c->field(c->L.S), c->at<InstDev>(c->L.inst), int(b), in.n,
                                  c->at<R>(c->L.screens), c->at<int64_t>(c->L.steps),
                                  c->step - 1, 1.0, stage, false, c->stream));
    HIP_TRY(launch_load_field<R>(stage, static_cast<char*>(c->field(c->L.S)) + in.off * c->el,
                                 n2, 1.0, c->stream));
  }
  c->pending = false;
  return SSFM_OK;
}

// Screen applied on load by step `step` of a record starting at step0: Lie
// the previous step's (none for the first), Strang the step's own.
int64_t rec_pending(const ssfm_ctx* c, int64_t step0, int64_t step) {
  if (c->strang) return step;
  return (step == step0) ? -1 : step - 1;
}

// Segments of a record of n steps.  Segment k covers s_{kM} .. s_{kM+M-1}:
// s_{kM} is checkpoint k, the others sit in segment slots (a region of
// n_stack fields).  Segments k >= first_kept are written whole by the
// forward record, each in a region of its own after the recompute banks;
// the backward recomputes the others from their checkpoints, alternating
// between banks 0 and 1.  A single-segment record is kept whole in region 0.
struct Segments {
  int64_t M, n_seg, first_kept, banks;
  int64_t region(int64_t k) const { return k >= first_kept ? banks + (k - first_kept) : k % 2; }
  bool recomputed(int64_t k) const { return k < first_kept; }
};

Segments rec_segments(const ssfm_ctx* c, int64_t n) {
  Segments g;
  g.M = std::min<int64_t>(std::max<int32_t>(c->ckpt_every, 1), n);
  g.n_seg = (n + g.M - 1) / g.M;
  if (g.n_seg == 1) {
    g.first_kept = 0;
    g.banks = 0;
  } else {
    // never more kept segments than the layout has regions for (a record
    // shorter than max_steps has no more segments than the layout)
    g.first_kept = g.n_seg - std::min<int64_t>(c->L.n_kept, g.n_seg);
    g.banks = c->L.n_banks;
  }
  return g;
}

// Location of s_i during a record of n steps (i in [0, n]).
void* rec_slot(ssfm_ctx* c, const Segments& g, int64_t i, int64_t n) {
  if (i == n) return c->field(c->L.S);
  if (i % g.M == 0) return c->field(c->L.ckpt, i / g.M);
  const int64_t k = i / g.M;
  if (!g.recomputed(k)) return c->field(c->L.stack, g.region(k) * c->L.n_stack + i % g.M - 1);
  return c->field(c->L.S);
}

// Steps i0 <= i < i1 of an n-step record from step0 (the first range also
// copies s_0 into checkpoint 0).  ts: timing events (single steps only).
template <typename R>
int enqueue_record(ssfm_ctx* c, int64_t n, int64_t step0, int64_t i0, int64_t i1,
                   const ssfm_ctx::PassSample* ts) {
  if (i0 == 0)
    HIP_TRY(launch_copy<R>(c->field(c->L.S), c->field(c->L.ckpt, 0), c->L.field_elems,
                           c->stream));
  int64_t chunk_start = step0 + i0;
  const Segments g = rec_segments(c, n);
  for (int64_t i = i0; i < i1; ++i) {
    const int slot = int((i - i0) % kDiagChunk);
    double* part = c->at<double>(c->L.diag_part) + size_t(slot) * 2 * c->L.n_widx_cols;
    const int64_t pend = rec_pending(c, step0, step0 + i);
    // a step whose state is kept goes through the work buffer for large
    // beams (see fwd_step); the others run in place
    void* dsl = rec_slot(c, g, i + 1, n);
    void* wk = (fresh_via_work(c) && dsl != c->field(c->L.S)) ? c->field(c->L.Wk) : nullptr;
    if (int r = fwd_step<R>(c, rec_slot(c, g, i, n), dsl, pend, part, wk, nullptr, ts)) return r;
    if (slot == kDiagChunk - 1 || i == i1 - 1) {
      if (int r = diag_flush<R>(c, slot + 1, chunk_start)) return r;
      chunk_start = step0 + i + 1;
    }
  }
  return SSFM_OK;
}

template <typename R>
int do_record(ssfm_ctx* c, int64_t n) {
  if (c->max_steps <= 0 || n > c->max_steps)
    return fail(SSFM_EINVAL, "record of %lld steps exceeds max_steps %lld", (long long)n,
                (long long)c->max_steps);
  if (int r = flush_pending<R>(c)) return r;
  const int64_t step0 = c->step;
  int r = run_forward(c, 1, step0, n, step0,
                      [&](int64_t i0, int64_t i1, const ssfm_ctx::PassSample* ts) {
                        return enqueue_record<R>(c, n, step0, i0, i1, ts);
                      });
  if (r) return r;
  c->step += n;
  c->pending = !c->strang;
  c->diag_valid = std::min<int64_t>(n, c->L.diag_cap);
  c->rec_steps = n;
  c->rec_step0 = step0;
  drop_record(c);
  c->rec_valid = true;
  return SSFM_OK;
}

// Backward over the recorded march, segment by segment from the last.  A
// segment the forward did not keep whole is recomputed from its checkpoint
// (into the other bank, through the work buffer): segment k-1 after the
// adjoint of segment k on the same stream, or (overlap_recompute) on the
// auxiliary stream while the adjoint of segment k runs on the main stream,
// the two chains joining before the adjoint of segment k-1.
template <typename R>
int enqueue_backward(ssfm_ctx* c) {
  const int64_t n = c->rec_steps, step0 = c->rec_step0;
  const Segments g = rec_segments(c, n);
  const int64_t M = g.M, n_seg = g.n_seg;
  const int64_t bank = c->L.n_stack;
  auto slot = [&](int64_t k, int64_t i) -> void* {  // slot i of segment k's region
    return c->field(c->L.stack, g.region(k) * bank + i);
  };
  auto sv = [&](int64_t k, int64_t i) -> void* {  // s_{kM+i}
    if (i == 0) return c->field(c->L.ckpt, k);
    return slot(k, i - 1);
  };
  auto recompute = [&](int64_t k, hipStream_t st) -> int {
    const int64_t s0 = k * M;
    const int64_t len = std::min<int64_t>(M, n - s0);
    for (int64_t i = 0; i + 1 < len; ++i) {
      const int64_t g = s0 + i;
      const int64_t pend = rec_pending(c, step0, step0 + g);
      // large beams through the work buffer, which nothing else uses during
      // the backward sweep (the adjoint steps run in place on the cotangent)
      void* wk = fresh_via_work(c) ? c->field(c->L.Wk) : nullptr;
      if (int r = fwd_step<R>(c, sv(k, i), slot(k, i), pend, nullptr, wk, st)) return r;
    }
    return SSFM_OK;
  };
  HIP_TRY(launch_fill_f64(c->at<double>(c->L.theta_acc), 8 * c->L.n_widx_rows, 0.0, c->stream));
  // Strang: the seed is the cotangent of U_N = L(-dz/2) V_N, so the march's
  // adjoint starts from L(dz/2) of it (the adjoint of the read-out)
  if (c->strang)
    if (int r = half_step_lam<R>(c, true)) return r;
  if (g.recomputed(n_seg - 1)) {
    if (int r = recompute(n_seg - 1, c->stream)) return r;
  }
  for (int64_t k = n_seg - 1; k >= 0; --k) {
    const bool rec_prev = k >= 1 && g.recomputed(k - 1);
    const bool overlap = rec_prev && c->overlap_recompute;
    if (overlap) {
      HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
      HIP_TRY(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
      if (int r = recompute(k - 1, c->aux)) return r;
      HIP_TRY(hipEventRecord(c->ev_join, c->aux));
    }
    const int64_t s0 = k * M;
    const int64_t len = std::min<int64_t>(M, n - s0);
    const int64_t every = c->timing_every;
    for (int64_t i = len - 1; i >= 0; --i) {
      const int64_t g = s0 + i;
      const int64_t pend = rec_pending(c, step0, step0 + g);
      ssfm_ctx::PassSample ps;
      const bool sample = every > 0 && k == 0 && g % every == every / 2 && take_sample(c, &ps);
      if (int r = adj_step<R>(c, sv(k, i), pend, sample ? &ps : nullptr)) return r;
      if (sample) c->adj_samples.push_back(std::move(ps));
    }
    if (overlap) {
      HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    } else if (rec_prev) {
      if (int r = recompute(k - 1, c->stream)) return r;
    }
  }
  // Strang: V_0 = L(dz/2) U_0, so dL/dU_0 = L(-dz/2) dL/dV_0
  if (c->strang)
    if (int r = half_step_lam<R>(c, false)) return r;
  HIP_TRY(launch_reduce_rows(c->at<double>(c->L.theta_acc), 8, c->at<int32_t>(c->L.wbegin_row),
                             int(c->desc.size()), c->at<double>(c->L.theta_out), c->stream));
  return SSFM_OK;
}

template <typename R>
int do_backward(ssfm_ctx* c) {
  if (!c->rec_valid) return fail(SSFM_ESTATE, "backward needs a preceding ssfm_forward_record");
  if (!c->seeded) return fail(SSFM_ESTATE, "backward needs a cotangent (set_cotangent/fluence_loss)");
  for (auto& e : c->adj_samples) c->free_samples.push_back(std::move(e));
  c->adj_samples.clear();
  // a beam without a cotangent contributes nothing to the loss: its
  // cotangent and its seed-step theta partials are zero (else the adjoint
  // would march whatever an earlier backward left there)
  for (size_t b = 0; b < c->desc.size(); ++b) {
    if (c->seeded_beam[b]) continue;
    const int64_t n2 = int64_t(c->inst[b].n) * c->inst[b].n;
    HIP_TRY(launch_fill_f64(reinterpret_cast<double*>(static_cast<char*>(c->field(c->L.Lam)) +
                                                      c->inst[b].off * c->el),
                            n2 * int64_t(c->el / 8), 0.0, c->stream));
    HIP_TRY(launch_fill_f64(c->at<double>(c->L.seed_theta) + size_t(b) * 8 * c->L.max_n,
                            8 * int64_t(c->inst[b].n), 0.0, c->stream));
  }
  // sampled timing launches the backward directly (its sampled passes
  // carry events on their own dispatches)
  int r = c->timing_every > 0 ? enqueue_backward<R>(c)
                              : maybe_graph(c, 2, c->rec_step0, c->rec_steps, 0, 0,
                                            [&] { return enqueue_backward<R>(c); });
  if (r) return r;
  c->grads_valid = true;
  return SSFM_OK;
}

// Seed (mode 0: loss; mode 1: external cotangent) for one beam.
template <typename R>
int do_seed(ssfm_ctx* c, int b, int mode, const double* target_dev, const double* g_dev) {
  const InstDev& in = c->inst[b];
  const ssfm_instance_desc& d = c->desc[b];
  const int64_t pend = c->step - 1;  // rec: the last recorded step's screen
  double* loss = c->at<double>(c->L.seed_loss);
  double* th = c->at<double>(c->L.seed_theta) + size_t(b) * 8 * c->L.max_n;
  if (mode == 0) {
    HIP_TRY(launch_sumsq(target_dev, int64_t(in.n) * in.n, 1.0, c->at<double>(c->L.sumsq_part),
                         c->at<double>(c->L.scal), c->stream));
  }
  const double gs = (mode == 0) ? d.i_ref : std::sqrt(d.i_ref);
  const void* state = c->field(c->L.S);
  int64_t seed_pend = pend;
  if (c->strang) {
    // U_N = L(-dz/2) V_N into the work buffer; nothing pending
    seed_pend = -1;
    if (mode == 0) {
      if (int r = half_steps<R>(c, false)) return r;
      state = c->field(c->L.Wk);
    }
  }
  HIP_TRY(launch_seed<R>(mode, state, c->at<InstDev>(c->L.inst), b, in.n,
                         c->at<R>(c->L.screens), c->at<int64_t>(c->L.steps), seed_pend, target_dev,
                         c->at<double>(c->L.scal), g_dev, gs, c->field(c->L.Lam), loss, th,
                         in.n, c->stream));
  return SSFM_OK;
}


// Turbulence screens: for every screen pair p, Philox/Box-Muller white noise
// shaped by the Kolmogorov amplitude goes into the work buffer, then an
// unscaled inverse DFT (rows in place, columns into planes 2p and 2p+1).
template <typename R>
int do_gen_screens(ssfm_ctx* c) {
  int max_pairs = 0;
  for (auto& d : c->desc)
    if ((d.terms & SSFM_TURB) && d.n_screens > 0) max_pairs = std::max(max_pairs, (d.n_screens + 1) / 2);
  // beams with subharmonic levels: coefficients, means and axis tables for
  // all their pairs up front (the region is laid out over every turbulent
  // beam in order), then one apply launch per pair after its inverse DFT
  std::vector<SubBeam>& sub = c->sub_beams;
  // the previous list may still be in an asynchronous upload
  if (!sub.empty()) HIP_TRY(hipStreamSynchronize(c->stream));
  sub.clear();
  int64_t region_off = 0, max_table = 0, max_n2 = 0;
  int sub_pairs = 0;
  for (size_t b = 0; b < c->desc.size(); ++b) {
    const ssfm_instance_desc& d = c->desc[b];
    if (!(d.terms & SSFM_TURB) || d.n_screens <= 0) continue;
    const int pairs = (d.n_screens + 1) / 2;
    const int64_t off = region_off;
    region_off += subharmonic_region_doubles(d.n, pairs);
    const ssfm_ctx::Spectrum& sp = c->spectrum[b];
    if (sp.subharmonics == 0 || (sp.kind != SSFM_SPECTRUM_STEP && !(d.cn2 > 0))) continue;
    SubBeam e{};
    e.inst = int32_t(b);
    e.n = d.n;
    e.pairs = pairs;
    e.k0 = uint32_t(d.seed & 0xffffffffu);
    e.k1 = uint32_t(d.seed >> 32);
    e.sp.levels = sp.subharmonics;
    e.sp.kind = sp.kind;
    const double k0 = 2.0 * M_PI / d.wavelength;
    e.sp.r0 = (sp.kind == SSFM_SPECTRUM_STEP) ? 0.0
                                               : std::pow(0.423 * k0 * k0 * d.cn2 * d.screen_dz, -0.6);
    e.sp.tau = sp.tau;
    e.sp.band_q2 = band_q2(d.length, sp.kappa_h);
    e.sp.length = d.length;
    e.tab_off = off;
    e.coef_off = off + 2 * int64_t(kMaxSubharmonicLevels) * d.n;
    sub.push_back(e);
    max_table = std::max<int64_t>(max_table, int64_t(sp.subharmonics) * d.n);
    max_n2 = std::max<int64_t>(max_n2, int64_t(d.n) * d.n);
    sub_pairs = std::max(sub_pairs, pairs);
  }
  const int n_sub = int(sub.size());
  if (n_sub > 0) {
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.subh_beams, sub.data(), sizeof(SubBeam) * sub.size(),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_subharmonic_setup(c->at<SubBeam>(c->L.subh_beams), n_sub, sub_pairs, max_table,
                                     c->at<double>(c->L.subh), c->stream));
  }
  for (int p = 0; p < max_pairs; ++p) {
    for (size_t b = 0; b < c->desc.size(); ++b) {
      const ssfm_instance_desc& d = c->desc[b];
      if (!(d.terms & SSFM_TURB) || 2 * p >= d.n_screens) continue;
      const double k0 = 2.0 * M_PI / d.wavelength;
      const ssfm_ctx::Spectrum& sp = c->spectrum[b];
      double amp0 = 0.0;
      if (sp.kind == SSFM_SPECTRUM_STEP) {
        amp0 = std::sqrt(sp.tau);
      } else if (d.cn2 > 0) {
        // sqrt(Phi(f)) df with Phi(f) = 0.023 r0^(-5/3) f^(-11/3), f = m / L,
        // df = 1 / L:  amplitude = sqrt(0.023) (L / r0)^(5/6) m^(-11/6)
        const double r0 = std::pow(0.423 * k0 * k0 * d.cn2 * d.screen_dz, -0.6);
        amp0 = std::sqrt(0.023) * std::pow(d.length / r0, 5.0 / 6.0);
      }
      HIP_TRY(launch_noise<R>(c->at<InstDev>(c->L.inst), int(b), d.n, p, d.seed, amp0, sp.kind,
                              band_q2(d.length, sp.kappa_h), c->field(c->L.Wk), c->stream));
    }
    PassArgs<R> a = base_args<R>(c);
    a.src = c->field(c->L.Wk);
    a.dst = c->field(c->L.Wk);
    a.pair = p;
    if (int r = run_pass<R>(c, ROW_INV, a)) return r;
    PassArgs<R> b = base_args<R>(c);
    b.src = c->field(c->L.Wk);
    b.planes_out = c->at<R>(c->L.screens);
    b.pair = p;
    if (int r = run_pass<R>(c, COL_INV, b)) return r;
    if (n_sub > 0)
      HIP_TRY(launch_subharmonic_apply<R>(c->at<SubBeam>(c->L.subh_beams), n_sub,
                                          c->at<InstDev>(c->L.inst), p, max_n2,
                                          c->at<double>(c->L.subh), c->at<R>(c->L.screens),
                                          c->stream));
  }
  return SSFM_OK;
}

// Upload host tables, beam constants and work lists.
template <typename R>
int upload_plan(ssfm_ctx* c) {
  const int n_inst = int(c->desc.size());
  // tables: twiddles per distinct n, then one propagator per beam
  std::vector<unsigned char> blob;
  std::map<int, int64_t> tw_off;
  std::vector<double> tmp;
  c->inst.assign(n_inst, InstDev{});
  c->lens_off.assign(n_inst, 0);
  c->half_off.assign(n_inst, 0);
  c->back_off.assign(n_inst, 0);
  c->fd_off.assign(n_inst, 0);
  if (c->spectrum.size() != size_t(n_inst)) c->spectrum.assign(n_inst, ssfm_ctx::Spectrum{});
  c->screen_steps.clear();
  int64_t foff = 0, soff = 0;
  for (int b = 0; b < n_inst; ++b) {
    const ssfm_instance_desc& d = c->desc[b];
    InstDev& in = c->inst[b];
    if (!tw_off.count(d.n)) {
      tw_off[d.n] = int64_t(blob.size() / c->el);
      twiddles(d.n, &tmp);
      append_table<R>(&blob, tmp);
    }
    in.n = d.n;
    in.K = (d.mpa_order >= 2) ? d.mpa_order : 2;
    in.terms = d.terms;
    in.n_screens = (d.terms & SSFM_TURB) ? d.n_screens : 0;
    in.off = foff;
    foff += int64_t(d.n) * d.n;
    in.screen_off = soff;
    soff += int64_t(in.n_screens) * d.n * d.n;
    in.tw_off = tw_off[d.n];
    in.prop_off = int64_t(blob.size() / c->el);
    propagator(d, &tmp);
    append_table<R>(&blob, tmp);
    c->lens_off[b] = int64_t(blob.size() / c->el);
    tmp.assign(2 * size_t(d.n), 0.0);
    for (int m = 0; m < d.n; ++m) tmp[2 * m] = 1.0 / d.n;  // identity filter until set
    append_table<R>(&blob, tmp);
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      ssfm_instance_desc h = d;
      h.dz = sgn * 0.5 * d.dz;
      (sgn > 0 ? c->half_off : c->back_off)[b] = int64_t(blob.size() / c->el);
      propagator(h, &tmp);
      append_table<R>(&blob, tmp);
    }
    {
      // 1 - (i dz/4k0) Lap_h has eigenvalue 1 + i (d[mx] + d[my]) on the DFT
      // mode (mx, my) of the periodic 5-point Laplacian
      const double k0 = 2.0 * M_PI / d.wavelength;
      const double dx = d.length / d.n;
      const double coef = d.dz / (k0 * dx * dx);
      c->fd_off[b] = int64_t(blob.size() / c->el);
      tmp.assign(2 * size_t(d.n), 0.0);
      for (int m = 0; m < d.n; ++m) {
        const double sn = std::sin(M_PI * m / d.n);
        tmp[2 * m] = coef * sn * sn;
      }
      append_table<R>(&blob, tmp);
    }
    in.steps_off = int64_t(c->screen_steps.size());
    for (int64_t s : screen_step_list(d)) c->screen_steps.push_back(s);
    const double k0 = 2.0 * M_PI / d.wavelength;
    in.cK = k0 * d.n2 * d.i_ref * d.dz;
    in.cM = (d.terms & SSFM_MPA) ? (in.K - 1) * d.beta_k * std::pow(d.i_ref, in.K - 1) * d.dz : 0.0;
    in.inv2k1 = 1.0 / (2.0 * (in.K - 1));
    for (int p = 0; p < 8; ++p) in.theta[p] = 0.0;
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.tables, blob.data(), blob.size(), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.inst, c->inst.data(), sizeof(InstDev) * n_inst,
                         hipMemcpyHostToDevice, c->stream));
  // the lens filter runs the pass kernels on a copy of the beam table whose
  // propagator is the filter and whose screen is off
  std::vector<InstDev> lens_inst = c->inst;
  for (int b = 0; b < n_inst; ++b) {
    lens_inst[b].prop_off = c->lens_off[b];
    lens_inst[b].terms = 0;
    lens_inst[b].n_screens = 0;
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.lens_inst, lens_inst.data(), sizeof(InstDev) * n_inst,
                         hipMemcpyHostToDevice, c->stream));
  std::vector<InstDev> half_inst = lens_inst, back_inst = lens_inst;
  for (int b = 0; b < n_inst; ++b) {
    half_inst[b].prop_off = c->half_off[b];
    back_inst[b].prop_off = c->back_off[b];
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.half_inst, half_inst.data(), sizeof(InstDev) * n_inst,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.back_inst, back_inst.data(), sizeof(InstDev) * n_inst,
                         hipMemcpyHostToDevice, c->stream));
  // finite differences: the beam's own screen constants, the solve table
  std::vector<InstDev> fd_inst = c->inst;
  for (int b = 0; b < n_inst; ++b) {
    fd_inst[b].prop_off = c->fd_off[b];
    fd_inst[b].n_screens = 0;
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.fd_inst, fd_inst.data(), sizeof(InstDev) * n_inst,
                         hipMemcpyHostToDevice, c->stream));
  if (!c->screen_steps.empty())
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.steps, c->screen_steps.data(),
                           sizeof(int64_t) * c->screen_steps.size(), hipMemcpyHostToDevice,
                           c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.wbegin_row, c->wbegin_row.data(),
                         sizeof(int32_t) * c->wbegin_row.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.wbegin_col, c->wbegin_col.data(),
                         sizeof(int32_t) * c->wbegin_col.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->field(c->L.S), 0, c->el * c->L.field_elems, c->stream));
  HIP_TRY(hipMemsetAsync(c->ws + c->L.diag, 0, sizeof(double) * 2 * c->L.diag_cap * n_inst,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // host vectors above are temporaries
  return SSFM_OK;
}


// The lens filter exp(-l_dif k^2) of beam b (1/n per pass) into its filter
// table; *blob holds the host copy until the caller synchronises.
template <typename R>
int upload_lens_filter(ssfm_ctx* c, int b, double l_dif, std::vector<unsigned char>* blob) {
  const ssfm_instance_desc& d = c->desc[b];
  std::vector<double> tab(2 * size_t(d.n), 0.0);
  const double dk = 2.0 * M_PI / d.length;
  for (int m = 0; m < d.n; ++m) {
    const int f = (m <= (d.n - 1) / 2) ? m : m - d.n;  // fftfreq order
    const double k = dk * f;
    tab[2 * m] = std::exp(-l_dif * k * k) / d.n;
  }
  append_table<R>(blob, tab);
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.tables + c->lens_off[b] * c->el, blob->data(),
                         blob->size(), hipMemcpyHostToDevice, c->stream));
  return SSFM_OK;
}

// Wk <- the lens filter applied to Wk (row and column passes with the filter
// tables in place of the propagators, no screen).
template <typename R>
int lens_filter_passes(ssfm_ctx* c) {
  PassArgs<R> a = base_args<R>(c);
  a.inst = c->at<InstDev>(c->L.lens_inst);
  a.src = c->field(c->L.Wk);
  a.dst = c->field(c->L.Wk);
  if (int r = run_pass<R>(c, ROW_FWD, a)) return r;
  a.part = nullptr;
  return run_pass<R>(c, COL_FWD, a);
}

LensDev lens_dev(const ssfm_instance_desc& d, const ssfm_lens& l) {
  LensDev p{};
  p.i_ref = d.i_ref;
  p.w_l = l.w_l;
  p.c1 = l.c1;
  p.c2 = l.c2;
  p.n_re = l.n_re;
  p.n_im = l.n_im;
  for (int j = 0; j < 8; ++j)
    for (int k = 0; k < 4; ++k) {
      p.re[j][k] = l.re[j][k];
      p.im[j][k] = l.im[j][k];
    }
  return p;
}

// Vector-Jacobian product of the lens at u_in (device complex128 of beam b):
// filter |u|^2, pointwise cotangent and partials, filter h, final cotangent
// and the fixed-order parameter sums (partials and sums in the staging area).
template <typename R>
int do_lens_vjp(ssfm_ctx* c, int b, const ssfm_lens& l, const double* u, const double* g_out,
                double* g_in, double* grad) {
  const ssfm_instance_desc& d = c->desc[b];
  const int64_t n2 = int64_t(d.n) * d.n;
  void* wk = static_cast<char*>(c->field(c->L.Wk)) + c->inst[b].off * int64_t(c->el);
  double* part = c->at<double>(c->L.stage);
  double* sums = part + int64_t(lens_vjp_blocks(n2)) * kLensGrads;
  std::vector<unsigned char> blob;
  if (int r = upload_lens_filter<R>(c, b, l.l_dif, &blob)) return r;
  HIP_TRY(launch_lens_vjp_prep<R>(u, d.i_ref, wk, n2, c->stream));
  if (int r = lens_filter_passes<R>(c)) return r;
  HIP_TRY(launch_lens_vjp_point<R>(u, g_out, wk, g_in, n2, lens_dev(d, l), part, c->stream));
  if (int r = lens_filter_passes<R>(c)) return r;
  HIP_TRY(launch_lens_vjp_final<R>(u, wk, d.i_ref, g_in, n2, part, sums, c->stream));
  double all[kLensGrads];
  HIP_TRY(hipMemcpyAsync(all, sums, sizeof(all), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  // slots: c1, c2, real segments 0..7, imaginary segments 0..7 -> packed
  int k = 0;
  grad[k++] = all[0];
  grad[k++] = all[1];
  for (int j = 0; j < l.n_re; ++j)
    for (int q = 0; q < 3; ++q) grad[k++] = all[2 + 3 * j + q];
  for (int j = 0; j < l.n_im; ++j)
    for (int q = 0; q < 3; ++q) grad[k++] = all[26 + 3 * j + q];
  return SSFM_OK;
}

// Effective lens on beam b: filter |U|^2 through the pass kernels, then the
// pointwise lens where the filtered intensity reaches the trimming level.
template <typename R>
int do_apply_lens(ssfm_ctx* c, int b, const ssfm_lens& l) {
  const ssfm_instance_desc& d = c->desc[b];
  if (int r = flush_pending<R>(c)) return r;
  std::vector<unsigned char> blob;
  if (int r = upload_lens_filter<R>(c, b, l.l_dif, &blob)) return r;
  HIP_TRY(launch_lens_prep<R>(c->field(c->L.S), c->field(c->L.Wk), c->L.field_elems, c->stream));
  if (int r = lens_filter_passes<R>(c)) return r;
  const LensDev p = lens_dev(d, l);
  const int64_t off = c->inst[b].off;
  HIP_TRY(launch_lens_apply<R>(static_cast<char*>(c->field(c->L.S)) + off * c->el,
                               static_cast<const char*>(c->field(c->L.Wk)) + off * c->el,
                               int64_t(d.n) * d.n, p, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // the filter table above is a host temporary
  drop_record(c);
  return SSFM_OK;
}

#define SSFM_DISPATCH(ctx, fn, ...) \
  ((ctx)->precision == SSFM_FP64 ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

// Device pointer of a caller buffer, staging host data through the
// workspace's complex128 staging area (bytes <= 16 n_max^2).
int stage_in(ssfm_ctx* c, const void* src, int32_t where, size_t bytes, const double** out) {
  if (!src) return fail(SSFM_EINVAL, "source pointer is NULL");
  if (where == SSFM_DEVICE) {
    *out = static_cast<const double*>(src);
    return SSFM_OK;
  }
  if (where != SSFM_HOST) return fail(SSFM_EINVAL, "where must be SSFM_HOST or SSFM_DEVICE");
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.stage, src, bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // the caller may free src on return
  *out = c->at<double>(c->L.stage);
  return SSFM_OK;
}

template <typename R>
int store_out(ssfm_ctx* c, int b, const void* state, int64_t pending, double scale, void* dst,
              int32_t where, bool intensity) {
  if (!dst) return fail(SSFM_EINVAL, "destination pointer is NULL");
  if (where != SSFM_HOST && where != SSFM_DEVICE)
    return fail(SSFM_EINVAL, "where must be SSFM_HOST or SSFM_DEVICE");
  const int n = c->desc[b].n;
  const size_t bytes = (intensity ? 8 : 16) * size_t(n) * n;
  double* out = (where == SSFM_DEVICE) ? static_cast<double*>(dst) : c->at<double>(c->L.stage);
  HIP_TRY(launch_store_field<R>(state, c->at<InstDev>(c->L.inst), b, n, c->at<R>(c->L.screens),
                                c->at<int64_t>(c->L.steps), pending, scale, out, intensity,
                                c->stream));
  if (where == SSFM_HOST) {
    HIP_TRY(hipMemcpyAsync(dst, out, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return SSFM_OK;
}

template <typename R>
int do_set_field(ssfm_ctx* c, int b, const void* src, int32_t where) {
  if (c->step > 0 || c->pending) {
    // keep the other beams exact: apply their pending screen first
    if (int r = flush_pending<R>(c)) return r;
  }
  const int n = c->desc[b].n;
  const double* dsrc;
  if (int r = stage_in(c, src, where, 16 * size_t(n) * n, &dsrc)) return r;
  HIP_TRY(launch_load_field<R>(dsrc, static_cast<char*>(c->field(c->L.S)) + c->inst[b].off * c->el,
                               int64_t(n) * n, 1.0 / std::sqrt(c->desc[b].i_ref), c->stream));
  if (c->strang) {
    // the state of a Strang march is V = L(dz/2) U: half a step for beam b
    if (int r = half_steps<R>(c, true)) return r;
    const size_t off = size_t(c->inst[b].off) * c->el;
    HIP_TRY(launch_copy<R>(static_cast<char*>(c->field(c->L.Wk)) + off,
                           static_cast<char*>(c->field(c->L.S)) + off, int64_t(n) * n,
                           c->stream));
  }
  // beam b starts its own step count (its screen schedule) here; the other
  // beams keep theirs.  Once every beam has been set at the same step, the
  // context count restarts at 0 (so marches from fresh fields reuse their
  // captured graphs).
  c->pending = false;
  c->diag_valid = 0;
  drop_record(c);
  c->inst[b].step_base = c->step;
  bool same = true;
  for (const InstDev& in : c->inst) same = same && (in.step_base == c->step);
  if (same) {
    for (InstDev& in : c->inst) in.step_base = 0;
    c->step = 0;
    return upload_inst(c, 0, c->inst.size());
  }
  return upload_inst(c, b, b + 1);
}

// Lines per workgroup of a variant (0 if it does not exist).
int plan_lines(bool column, int n, int v) {
  PlanInfo pi{};
  plan_info(column, n, v, false, &pi);
  return pi.lines;
}

// Adjoint-pass variants of size n (-1: follow the forward variants).
int do_select_adjoint(ssfm_ctx* c, int32_t n, int32_t rv, int32_t cv) {
  const bool fp64 = c->precision == SSFM_FP64;
  const int rc = plan_count(false, n), cc = plan_count(true, n);
  if (rc == 0) return fail(SSFM_EUNSUPPORTED, "grid size %d not supported", n);
  if (rv < -1 || rv >= rc || cv < -1 || cv >= cc)
    return fail(SSFM_EINVAL, "variant (%d, %d) out of range [-1, %d) x [-1, %d)", rv, cv, rc, cc);
  Group* grp = nullptr;
  for (auto& g : c->groups)
    if (g.n == n) grp = &g;
  if (!grp) return fail(SSFM_EINVAL, "no instance with n=%d in this context", n);
  PlanInfo pi{};
  if (rv >= 0) {
    if (!plan_info(false, n, rv, fp64, &pi))
      return fail(SSFM_EUNSUPPORTED, "row variant %d of n=%d is not built at this precision", rv, n);
    if (pi.lines != plan_lines(false, n, grp->row_var))
      return fail(SSFM_EINVAL, "row variant %d has %d lines per workgroup, the forward one %d", rv,
                  pi.lines, plan_lines(false, n, grp->row_var));
  }
  if (cv >= 0) {
    if (!plan_info(true, n, cv, fp64, &pi))
      return fail(SSFM_EUNSUPPORTED, "column variant %d of n=%d is not built at this precision",
                  cv, n);
    if (pi.lines != plan_lines(true, n, grp->col_var))
      return fail(SSFM_EINVAL, "column variant %d has %d columns per workgroup, the forward one %d",
                  cv, pi.lines, plan_lines(true, n, grp->col_var));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  grp->row_adj_var = rv;
  grp->col_adj_var = cv;
  clear_graphs(c);
  return SSFM_OK;
}

int do_select(ssfm_ctx* c, int32_t n, int32_t rv, int32_t cv) {
  const int rc = plan_count(false, n), cc = plan_count(true, n);
  if (rc == 0) return fail(SSFM_EUNSUPPORTED, "grid size %d not supported", n);
  if (rv < 0 || rv >= rc || cv < 0 || cv >= cc)
    return fail(SSFM_EINVAL, "variant (%d, %d) out of range [0, %d) x [0, %d)", rv, cv, rc, cc);
  bool found = false;
  VariantMap vm;
  for (auto& g : c->groups) {
    vm[g.n] = {g.row_var, g.col_var};
    if (g.n == n) found = true;
  }
  if (!found) return fail(SSFM_EINVAL, "no instance with n=%d in this context", n);
  vm[n] = {rv, cv};
  // rebuild work lists; the layout's partial arrays are already sized for
  // the variant with the most work items, so offsets stay valid
  Layout L2;
  std::vector<Group> groups;
  std::vector<WorkItem> work;
  std::vector<int32_t> wr, wc;
  if (int r = plan_layout(c->desc.data(), int(c->desc.size()), c->precision, c->max_steps,
                          c->ckpt_every, c->stored_segments, &vm, &groups, &work, &wr, &wc, &L2))
    return r;
  if (L2.total != c->L.total) return fail(SSFM_EUNSUPPORTED, "variant changes the workspace layout");
  // keep each size's adjoint variants while their lines per workgroup still
  // match the forward ones
  for (auto& g : groups) {
    for (const auto& o : c->groups) {
      if (o.n != g.n) continue;
      g.row_adj_var = o.row_adj_var;
      g.col_adj_var = o.col_adj_var;
    }
    if (g.row_adj_var >= 0 && plan_lines(false, g.n, g.row_adj_var) != plan_lines(false, g.n, g.row_var))
      g.row_adj_var = -1;
    if (g.col_adj_var >= 0 && plan_lines(true, g.n, g.col_adj_var) != plan_lines(true, g.n, g.col_var))
      g.col_adj_var = -1;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->groups = groups;
  c->work = work;
  c->wbegin_row = wr;
  c->wbegin_col = wc;
  c->L = L2;
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.wbegin_row, c->wbegin_row.data(),
                         sizeof(int32_t) * c->wbegin_row.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.wbegin_col, c->wbegin_col.data(),
                         sizeof(int32_t) * c->wbegin_col.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  clear_graphs(c);
  return SSFM_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

int ssfm_version(void) { return SSFM_VERSION; }

const char* ssfm_strerror(int s) {
  switch (s) {
    case SSFM_OK: return "ok";
    case SSFM_EINVAL: return "invalid argument";
    case SSFM_EUNSUPPORTED: return "unsupported grid size or option";
    case SSFM_EHIP: return "HIP runtime error";
    case SSFM_ESTATE: return "call out of order";
    case SSFM_ENONFINITE: return "non-finite power or gradient";
    case SSFM_EWORKSPACE: return "workspace missing, misaligned or too small";
    default: return "unknown status";
  }
}

const char* ssfm_last_error(void) { return g_last_error.c_str(); }

int ssfm_workspace_bytes(const ssfm_instance_desc* desc, int32_t n_inst, int32_t precision,
                         int64_t max_steps, int32_t ckpt_every, int32_t stored_segments,
                         size_t* bytes) {
  g_last_error.clear();
  if (!bytes) return fail(SSFM_EINVAL, "bytes is NULL");
  if (int r = validate_desc(desc, n_inst, precision)) return r;
  if (max_steps < 0 || ckpt_every < 1 || stored_segments < 0)
    return fail(SSFM_EINVAL, "need max_steps >= 0, ckpt_every >= 1, stored_segments >= 0");
  Layout L;
  if (int r = plan_layout(desc, n_inst, precision, max_steps, ckpt_every, stored_segments,
                          nullptr, nullptr, nullptr, nullptr, nullptr, &L))
    return r;
  *bytes = L.total;
  return SSFM_OK;
}

int ssfm_checkpoint_plan(const ssfm_instance_desc* desc, int32_t n_inst, int32_t precision,
                         int64_t n_steps, size_t budget_bytes, int32_t* ckpt_every,
                         int32_t* stored_segments, int64_t* recomputed) {
  g_last_error.clear();
  if (!ckpt_every || !stored_segments) return fail(SSFM_EINVAL, "output pointer is NULL");
  if (int r = validate_desc(desc, n_inst, precision)) return r;
  if (n_steps < 1 || n_steps > INT32_MAX) return fail(SSFM_EINVAL, "need 1 <= n_steps < 2^31");
  Layout L;
  auto bytes_of = [&](int64_t m, int64_t k, size_t* out) {
    int r = plan_layout(desc, n_inst, precision, n_steps, int32_t(m), int32_t(k), nullptr,
                        nullptr, nullptr, nullptr, nullptr, &L);
    *out = L.total;
    return r;
  };
  size_t b = 0;
  // every pre-screen field kept: no recompute
  if (int r = bytes_of(n_steps, 0, &b)) return r;
  if (b <= budget_bytes) {
    *ckpt_every = int32_t(n_steps);
    *stored_segments = 0;
    if (recomputed) *recomputed = 0;
    return SSFM_OK;
  }
  if (n_steps < 3) return fail(SSFM_EWORKSPACE, "%zu bytes needed, budget %zu", b, budget_bytes);
  // With M < n_steps the layout is affine in its field slots (every field
  // array is a whole number of alignment units): bytes = A + F * slots,
  // slots = checkpoints + (M - 1) * (banks + kept segments).
  auto slots_of = [&](int64_t m, int64_t k) {
    const int64_t seg = (n_steps + m - 1) / m;
    const int64_t kept = std::min(k, seg);
    return seg + (m - 1) * (std::min<int64_t>(2, seg - kept) + kept);
  };
  size_t b2 = 0;
  if (int r = bytes_of(2, 0, &b2)) return r;
  const double F = double(L.field_elems) * (precision == SSFM_FP64 ? 16.0 : 8.0);
  const double A = double(b2) - F * double(slots_of(2, 0));
  const double cap = (double(budget_bytes) - A) / F;  // field slots that fit
  // Cost of (M, K): steps recomputed by the backward, plus one per segment
  // for its fork, join and checkpoint boundary; the cheapest that fits.
  int64_t best_m = -1, best_k = 0, best_rec = 0;
  double best_cost = 0.0;
  for (int64_t m = 2; m < n_steps; ++m) {
    const int64_t seg = (n_steps + m - 1) / m;
    if (double(slots_of(m, 0)) > cap) continue;
    // kept segments that fit (slots rise with K; K = seg - 1 costs what
    // K = seg costs, so it is never the choice)
    int64_t k = 0;
    if (double(slots_of(m, seg)) <= cap) {
      k = seg;
    } else {
      const double room = (cap - double(seg)) / double(m - 1) - 2.0;
      k = std::max<int64_t>(0, std::min<int64_t>(seg - 2, int64_t(std::floor(room))));
      while (k > 0 && double(slots_of(m, k)) > cap) --k;
    }
    const int64_t rec = (k == 0) ? n_steps - seg : (seg - std::min(k, seg)) * (m - 1);
    const double cost = double(rec) + double(seg);
    if (best_m < 0 || cost < best_cost) {
      best_m = m;
      best_k = k;
      best_rec = rec;
      best_cost = cost;
    }
  }
  if (best_m < 0) {
    // the smallest layout: M near sqrt(n_steps / 2), nothing kept
    size_t need = 0;
    bytes_of(std::max<int64_t>(2, int64_t(std::sqrt(0.5 * double(n_steps)))), 0, &need);
    return fail(SSFM_EWORKSPACE, "no checkpoint layout fits %zu bytes (at least %zu needed)",
                budget_bytes, need);
  }
  // the affine model is exact; confirm with the layout itself
  if (int r = bytes_of(best_m, best_k, &b)) return r;
  if (b > budget_bytes)
    return fail(SSFM_EWORKSPACE, "checkpoint layout of %zu bytes exceeds budget %zu", b,
                budget_bytes);
  *ckpt_every = int32_t(best_m);
  *stored_segments = int32_t(best_k);
  if (recomputed) *recomputed = best_rec;
  return SSFM_OK;
}

int ssfm_create(const ssfm_instance_desc* desc, int32_t n_inst, int32_t precision,
                int64_t max_steps, int32_t ckpt_every, int32_t stored_segments,
                void* workspace, size_t ws_bytes, void* stream, ssfm_ctx** out) {
  g_last_error.clear();
  if (!out) return fail(SSFM_EINVAL, "out is NULL");
  *out = nullptr;
  if (int r = validate_desc(desc, n_inst, precision)) return r;
  if (max_steps < 0 || ckpt_every < 1 || stored_segments < 0)
    return fail(SSFM_EINVAL, "need max_steps >= 0, ckpt_every >= 1, stored_segments >= 0");
  std::unique_ptr<ssfm_ctx> c(new ssfm_ctx);
  c->precision = precision;
  c->el = precision == SSFM_FP64 ? 16 : 8;
  c->desc.assign(desc, desc + n_inst);
  c->seeded_beam.assign(n_inst, 0);
  c->max_steps = max_steps;
  c->ckpt_every = ckpt_every;
  c->stored_segments = stored_segments;
  c->stream = static_cast<hipStream_t>(stream);
  if (int r = plan_layout(desc, n_inst, precision, max_steps, ckpt_every, stored_segments,
                          nullptr, &c->groups,
                          &c->work, &c->wbegin_row, &c->wbegin_col, &c->L))
    return r;
  if (!workspace) return fail(SSFM_EWORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(SSFM_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
  if (ws_bytes < c->L.total)
    return fail(SSFM_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, c->L.total);
  c->ws = static_cast<char*>(workspace);
  HIP_TRY(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->gfork, hipEventDisableTiming));
  for (size_t g = 1; g < c->groups.size(); ++g) {
    hipStream_t sg;
    hipEvent_t ej;
    HIP_TRY(hipStreamCreateWithFlags(&sg, hipStreamNonBlocking));
    c->gstream.push_back(sg);
    HIP_TRY(hipEventCreateWithFlags(&ej, hipEventDisableTiming));
    c->gjoin.push_back(ej);
  }
  int r = SSFM_DISPATCH(c, upload_plan, c.get());
  if (r) return r;
  *out = c.release();
  return SSFM_OK;
}

int ssfm_destroy(ssfm_ctx* ctx) {
  if (!ctx) return SSFM_OK;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return SSFM_OK;
}

int ssfm_set_field(ssfm_ctx* c, int32_t inst, const void* src, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  return SSFM_DISPATCH(c, do_set_field, c, inst, src, where);
}

int ssfm_set_theta(ssfm_ctx* c, int32_t inst, const double* theta) {
  if (int r = check_inst(c, inst)) return r;
  if (!theta) return fail(SSFM_EINVAL, "theta is NULL");
  for (int p = 0; p < 8; ++p) {
    if (!std::isfinite(theta[p])) return fail(SSFM_EINVAL, "theta[%d] not finite", p);
    c->inst[inst].theta[p] = theta[p];
  }
  // a recorded march (its stored fields, the screen its adjoint applies)
  // belongs to the old parameters
  drop_record(c);
  return upload_inst(c, inst, inst + 1);
}

int ssfm_gen_screens(ssfm_ctx* c) {
  if (int r = check_ctx(c)) return r;
  drop_record(c);  // the recorded march used the previous screens
  return SSFM_DISPATCH(c, do_gen_screens, c);
}

int ssfm_get_screen(ssfm_ctx* c, int32_t inst, int32_t s, void* dst, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  const InstDev& in = c->inst[inst];
  if (s < 0 || s >= in.n_screens) return fail(SSFM_EINVAL, "screen %d out of range", s);
  if (!dst) return fail(SSFM_EINVAL, "dst is NULL");
  const int64_t n2 = int64_t(in.n) * in.n;
  double* out = (where == SSFM_DEVICE) ? static_cast<double*>(dst) : c->at<double>(c->L.stage);
  const size_t rel = c->el / 2;
  const void* plane = c->ws + c->L.screens + rel * size_t(in.screen_off + int64_t(s) * n2);
  if (c->precision == SSFM_FP64)
    HIP_TRY(launch_screen_to_f64<double>(static_cast<const double*>(plane), n2, out, c->stream));
  else
    HIP_TRY(launch_screen_to_f64<float>(static_cast<const float*>(plane), n2, out, c->stream));
  if (where == SSFM_HOST) {
    HIP_TRY(hipMemcpyAsync(dst, out, 8 * n2, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return SSFM_OK;
}

int ssfm_propagate(ssfm_ctx* c, int64_t n_steps) {
  if (int r = check_ctx(c)) return r;
  if (n_steps < 0) return fail(SSFM_EINVAL, "n_steps < 0");
  if (n_steps == 0) return SSFM_OK;
  return SSFM_DISPATCH(c, do_propagate, c, n_steps);
}

extern "C++" {
// Read-out of beam b: Lie applies the pending screen; Strang diffracts the
// state V back by half a step (U = L(-dz/2) V) in the work buffer first.
template <typename R>
int read_out(ssfm_ctx* c, int b, void* dst, int32_t where, bool intensity) {
  const double sc = std::sqrt(c->desc[b].i_ref);
  if (c->strang) {
    if (int r = half_steps<R>(c, false)) return r;
    return store_out<R>(c, b, c->field(c->L.Wk), -1, sc, dst, where, intensity);
  }
  const int64_t pend = c->pending ? c->step - 1 : -1;
  return store_out<R>(c, b, c->field(c->L.S), pend, sc, dst, where, intensity);
}
}  // extern "C++"

int ssfm_get_field(ssfm_ctx* c, int32_t inst, void* dst, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  return SSFM_DISPATCH(c, read_out, c, inst, dst, where, false);
}

int ssfm_get_intensity(ssfm_ctx* c, int32_t inst, void* dst, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  return SSFM_DISPATCH(c, read_out, c, inst, dst, where, true);
}

int ssfm_set_splitting(ssfm_ctx* c, int32_t scheme) {
  if (int r = check_ctx(c)) return r;
  if (scheme != SSFM_LIE && scheme != SSFM_STRANG && scheme != SSFM_FD)
    return fail(SSFM_EINVAL, "unknown scheme %d", scheme);
  if (scheme == SSFM_FD) {
    for (size_t b = 0; b < c->desc.size(); ++b) {
      const ssfm_instance_desc& d = c->desc[b];
      if ((d.terms & SSFM_ANSATZ) || ((d.terms & SSFM_TURB) && d.n_screens > 0))
        return fail(SSFM_EUNSUPPORTED,
                    "the finite-difference scheme covers the Kerr, plasma and multiphoton "
                    "terms only (instance %zu has the ansatz or turbulence screens)", b);
    }
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  clear_graphs(c);
  c->strang = (scheme == SSFM_STRANG);
  c->fd = (scheme == SSFM_FD);
  HIP_TRY(hipMemsetAsync(c->field(c->L.S), 0, c->el * c->L.field_elems, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  c->pending = false;
  c->diag_valid = 0;
  drop_record(c);
  for (InstDev& in : c->inst) in.step_base = 0;
  return upload_inst(c, 0, c->inst.size());
}

namespace {
int split_step_only(ssfm_ctx* c, const char* what) {
  if (c->fd)
    return fail(SSFM_EUNSUPPORTED, "%s needs a split-step scheme (the finite-difference scheme "
                                   "marches forward only)", what);
  return SSFM_OK;
}

int lie_only(ssfm_ctx* c, const char* what) {
  if (c->strang || c->fd)
    return fail(SSFM_EUNSUPPORTED, "%s needs the Lie split-step scheme (%s marches forward only)",
                what, c->strang ? "Strang" : "the finite-difference scheme");
  return SSFM_OK;
}

}  // namespace

int ssfm_set_fd_iterations(ssfm_ctx* c, int32_t iterations) {
  if (int r = check_ctx(c)) return r;
  if (iterations < 1 || iterations > 64)
    return fail(SSFM_EINVAL, "finite-difference iterations must be in [1, 64], got %d",
                iterations);
  HIP_TRY(hipStreamSynchronize(c->stream));
  clear_graphs(c);
  c->fd_iters = iterations;
  return SSFM_OK;
}

namespace {
}  // namespace

int ssfm_get_diag(ssfm_ctx* c, int32_t inst, double* power, double* peak, int64_t n) {
  if (int r = check_inst(c, inst)) return r;
  if (n < 0 || n > c->diag_valid)
    return fail(SSFM_EINVAL, "n=%lld exceeds the %lld recorded diagnostic steps", (long long)n,
                (long long)c->diag_valid);
  if (n == 0) return SSFM_OK;
  std::vector<double> buf(2 * size_t(c->L.diag_cap));
  HIP_TRY(hipMemcpyAsync(buf.data(), c->ws + c->L.diag + sizeof(double) * 2 * c->L.diag_cap * inst,
                         sizeof(double) * 2 * c->L.diag_cap, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const ssfm_instance_desc& d = c->desc[inst];
  const double dx = d.length / d.n;
  int status = SSFM_OK;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t step = c->step - n + i;
    const int64_t slot = step % c->L.diag_cap;
    const double pw = buf[2 * slot] * d.i_ref * dx * dx;
    const double pk = buf[2 * slot + 1] * d.i_ref;
    if (power) power[i] = pw;
    if (peak) peak[i] = pk;
    if (!std::isfinite(pw)) status = SSFM_ENONFINITE;
  }
  if (status) return fail(status, "non-finite power in the diagnostics of instance %d", inst);
  return SSFM_OK;
}

int ssfm_forward_record(ssfm_ctx* c, int64_t n_steps) {
  if (int r = check_ctx(c)) return r;
  if (int r = split_step_only(c, "forward_record")) return r;
  if (n_steps < 1) return fail(SSFM_EINVAL, "n_steps must be >= 1");
  return SSFM_DISPATCH(c, do_record, c, n_steps);
}

int ssfm_set_cotangent(ssfm_ctx* c, int32_t inst, const void* g, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  if (int r = split_step_only(c, "set_cotangent")) return r;
  if (!c->rec_valid) return fail(SSFM_ESTATE, "set_cotangent needs a preceding forward_record");
  const int n = c->desc[inst].n;
  const double* dg;
  if (int r = stage_in(c, g, where, 16 * size_t(n) * n, &dg)) return r;
  int r = SSFM_DISPATCH(c, do_seed, c, inst, 1, nullptr, dg);
  if (r) return r;
  if (where == SSFM_HOST) HIP_TRY(hipStreamSynchronize(c->stream));
  c->seeded = true;
  c->seeded_beam[inst] = 1;
  return SSFM_OK;
}

int ssfm_fluence_loss(ssfm_ctx* c, int32_t inst, const void* target, int32_t where, double* loss) {
  if (int r = check_inst(c, inst)) return r;
  if (int r = split_step_only(c, "fluence_loss")) return r;
  if (!c->rec_valid) return fail(SSFM_ESTATE, "fluence_loss needs a preceding forward_record");
  const int n = c->desc[inst].n;
  const double* dt;
  if (int r = stage_in(c, target, where, 8 * size_t(n) * n, &dt)) return r;
  int r = SSFM_DISPATCH(c, do_seed, c, inst, 0, dt, nullptr);
  if (r) return r;
  std::vector<double> part(n);
  double wsum = 0.0;
  HIP_TRY(hipMemcpyAsync(part.data(), c->ws + c->L.seed_loss, sizeof(double) * n,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&wsum, c->ws + c->L.scal, sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  if (loss) *loss = s / wsum;
  c->seeded = true;
  c->seeded_beam[inst] = 1;
  return SSFM_OK;
}

int ssfm_fluence_mismatch(ssfm_ctx* c, int32_t inst, const void* target, int32_t where,
                          double* loss) {
  if (int r = check_inst(c, inst)) return r;
  if (!loss) return fail(SSFM_EINVAL, "loss is NULL");
  const int n = c->desc[inst].n;
  const double* dt;
  if (int r = stage_in(c, target, where, 8 * size_t(n) * n, &dt)) return r;
  // the seed kernel in loss mode without a cotangent output; its gradient
  // partials go to the staging area past the target
  double* scratch = c->at<double>(c->L.stage) + size_t(n) * n;
  double* th = scratch;
  double* part = scratch + 8 * size_t(n);
  const InstDev& in = c->inst[inst];
  const ssfm_instance_desc& d = c->desc[inst];
  auto run = [&]<typename R>(R*) -> int {
    // the field U: the state with its pending screen (Lie), the state itself
    // (finite differences), or L(-dz/2) of it in the work buffer (Strang)
    const void* state = c->field(c->L.S);
    int64_t pend = c->pending ? c->step - 1 : -1;
    if (c->strang) {
      if (int r = half_steps<R>(c, false)) return r;
      state = c->field(c->L.Wk);
      pend = -1;
    }
    HIP_TRY(launch_sumsq(dt, int64_t(n) * n, 1.0, c->at<double>(c->L.sumsq_part),
                         c->at<double>(c->L.scal), c->stream));
    HIP_TRY(launch_seed<R>(0, state, c->at<InstDev>(c->L.inst), inst, in.n,
                           c->at<R>(c->L.screens), c->at<int64_t>(c->L.steps), pend, dt,
                           c->at<double>(c->L.scal), nullptr, d.i_ref, nullptr, part, th, in.n,
                           c->stream));
    return SSFM_OK;
  };
  if (int r = (c->precision == SSFM_FP64) ? run((double*)nullptr) : run((float*)nullptr))
    return r;
  std::vector<double> h(n);
  double wsum = 0.0;
  HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&wsum, c->ws + c->L.scal, sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += h[i];
  *loss = s / wsum;
  return SSFM_OK;
}

int ssfm_backward(ssfm_ctx* c) {
  if (int r = check_ctx(c)) return r;
  if (int r = split_step_only(c, "backward")) return r;
  return SSFM_DISPATCH(c, do_backward, c);
}

int ssfm_get_grad_field(ssfm_ctx* c, int32_t inst, void* dst, int32_t where) {
  if (int r = check_inst(c, inst)) return r;
  if (!c->grads_valid) return fail(SSFM_ESTATE, "no gradient: call ssfm_backward first");
  const double sc = 1.0 / std::sqrt(c->desc[inst].i_ref);
  return SSFM_DISPATCH(c, store_out, c, inst, c->field(c->L.Lam), -1, sc, dst, where, false);
}

int ssfm_get_grad_theta(ssfm_ctx* c, int32_t inst, double* g) {
  if (int r = check_inst(c, inst)) return r;
  if (!c->grads_valid) return fail(SSFM_ESTATE, "no gradient: call ssfm_backward first");
  if (!g) return fail(SSFM_EINVAL, "g is NULL");
  double acc[8], seed_part[8];
  const int n = c->desc[inst].n;
  std::vector<double> sp(size_t(8) * n);
  HIP_TRY(hipMemcpyAsync(acc, c->ws + c->L.theta_out + sizeof(double) * 8 * inst,
                         sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(sp.data(), c->ws + c->L.seed_theta + sizeof(double) * 8 * c->L.max_n * inst,
                         sizeof(double) * 8 * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int p = 0; p < 8; ++p) {
    seed_part[p] = 0.0;
    for (int r = 0; r < n; ++r) seed_part[p] += sp[size_t(r) * 8 + p];
    g[p] = acc[p] + seed_part[p];
  }
  for (int p = 0; p < 8; ++p)
    if (!std::isfinite(g[p]))
      return fail(SSFM_ENONFINITE,
                  "theta gradient of instance %d is not finite: the linearised march "
                  "outgrew the precision's range", inst);
  return SSFM_OK;
}

int ssfm_block_mean(ssfm_ctx* c, const double* src, int32_t n, int32_t b, double* dst) {
  if (int r = check_ctx(c)) return r;
  if (!src || !dst) return fail(SSFM_EINVAL, "src/dst is NULL");
  if (n < 1 || b < 1 || n % b) return fail(SSFM_EINVAL, "block %d must divide n=%d", b, n);
  HIP_TRY(launch_block_mean(src, n, b, dst, c->stream));
  return SSFM_OK;
}

int ssfm_set_recompute_overlap(ssfm_ctx* c, int32_t enable) {
  if (int r = check_ctx(c)) return r;
  c->overlap_recompute = enable != 0;
  // captured backward sweeps hold the previous schedule
  clear_graphs(c);
  return SSFM_OK;
}

int ssfm_set_precise_math(ssfm_ctx* c, int32_t enable) {
  if (int r = check_ctx(c)) return r;
  for (auto& in : c->inst) {
    if (enable) in.terms |= (1u << 8);
    else in.terms &= ~(1u << 8);
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->L.inst, c->inst.data(), sizeof(InstDev) * c->inst.size(),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  // captured steps hold the kernels chosen for the previous setting
  clear_graphs(c);
  return SSFM_OK;
}

int ssfm_use_graphs(ssfm_ctx* c, int32_t enable) {
  if (int r = check_ctx(c)) return r;
  c->use_graphs = enable != 0;
  return SSFM_OK;
}

int ssfm_plan_variants(int32_t n, int32_t precision, int32_t* n_row, int32_t* n_col) {
  if (!n_row || !n_col) return fail(SSFM_EINVAL, "n_row/n_col is NULL");
  if (precision != SSFM_FP32 && precision != SSFM_FP64) return fail(SSFM_EINVAL, "precision");
  *n_row = plan_count(false, n);
  *n_col = plan_count(true, n);
  if (*n_row == 0 || *n_col == 0) return fail(SSFM_EUNSUPPORTED, "grid size %d not supported", n);
  return SSFM_OK;
}

int ssfm_select_plan(ssfm_ctx* c, int32_t n, int32_t row_variant, int32_t col_variant) {
  if (int r = check_ctx(c)) return r;
  return do_select(c, n, row_variant, col_variant);
}

int ssfm_select_adjoint_plan(ssfm_ctx* c, int32_t n, int32_t row_variant,
                             int32_t col_variant) {
  if (int r = check_ctx(c)) return r;
  return do_select_adjoint(c, n, row_variant, col_variant);
}

int ssfm_time_adjoint_passes(ssfm_ctx* c, int32_t reps, double* ms_col, double* ms_row) {
  if (int r = check_ctx(c)) return r;
  if (reps < 1) return fail(SSFM_EINVAL, "reps must be >= 1");
  if (c->max_steps <= 0)
    return fail(SSFM_ESTATE, "adjoint passes need a context created with max_steps > 0");
  struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  for (auto& x : ev.e) HIP_TRY(hipEventCreate(&x));
  // column pass: cotangent -> work buffer; row pass: work buffer in place,
  // the state standing in for the stored pre-screen field, at a step with
  // no turbulence screen (its ansatz partials go to the accumulators every
  // backward clears first).  Fields, cotangent and gradients are unchanged.
  auto body = [&]<typename R>(R*) -> int {
    PassArgs<R> a = base_args<R>(c);
    a.src = c->field(c->L.Lam);
    a.dst = c->field(c->L.Wk);
    PassArgs<R> b = base_args<R>(c);
    b.src = c->field(c->L.Wk);
    b.dst = c->field(c->L.Wk);
    b.aux = c->field(c->L.S);
    b.step = int64_t(1) << 60;
    b.part = c->at<double>(c->L.theta_acc);
    HIP_TRY(hipEventRecord(ev.e[0], c->stream));
    for (int i = 0; i < reps; ++i)
      if (int q = run_pass<R>(c, COL_ADJ, a)) return q;
    HIP_TRY(hipEventRecord(ev.e[1], c->stream));
    for (int i = 0; i < reps; ++i)
      if (int q = run_pass<R>(c, ROW_ADJ, b)) return q;
    HIP_TRY(hipEventRecord(ev.e[2], c->stream));
    return SSFM_OK;
  };
  int r = (c->precision == SSFM_FP64) ? body((double*)nullptr) : body((float*)nullptr);
  if (r) return r;
  HIP_TRY(hipEventSynchronize(ev.e[2]));
  float t1 = 0, t2 = 0;
  HIP_TRY(hipEventElapsedTime(&t1, ev.e[0], ev.e[1]));
  HIP_TRY(hipEventElapsedTime(&t2, ev.e[1], ev.e[2]));
  if (ms_col) *ms_col = double(t1) / reps;
  if (ms_row) *ms_row = double(t2) / reps;
  return SSFM_OK;
}

int ssfm_time_passes(ssfm_ctx* c, int32_t reps, double* ms_row, double* ms_col,
                     double* bytes_row, double* bytes_col) {
  if (int r = check_ctx(c)) return r;
  if (reps < 1) return fail(SSFM_EINVAL, "reps must be >= 1");
  // events released on every return path
  struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  for (auto& x : ev.e) HIP_TRY(hipEventCreate(&x));
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1], e2 = ev.e[2];
  int r = SSFM_OK;
  auto body = [&]<typename R>(R*) -> int {
    PassArgs<R> a = base_args<R>(c);
    a.src = c->field(c->L.S);
    a.dst = c->field(c->L.Wk);
    a.step = c->pending ? c->step - 1 : -1;
    PassArgs<R> b = base_args<R>(c);
    b.src = c->field(c->L.Wk);
    b.dst = c->field(c->L.Wk);
    b.part = c->at<double>(c->L.diag_part);
    HIP_TRY(hipEventRecord(e0, c->stream));
    for (int i = 0; i < reps; ++i)
      if (int q = run_pass<R>(c, ROW_FWD, a)) return q;
    HIP_TRY(hipEventRecord(e1, c->stream));
    for (int i = 0; i < reps; ++i)
      if (int q = run_pass<R>(c, COL_FWD, b)) return q;
    HIP_TRY(hipEventRecord(e2, c->stream));
    return SSFM_OK;
  };
  r = (c->precision == SSFM_FP64) ? body((double*)nullptr) : body((float*)nullptr);
  if (r == SSFM_OK) {
    HIP_TRY(hipEventSynchronize(e2));
    float t1 = 0, t2 = 0;
    HIP_TRY(hipEventElapsedTime(&t1, e0, e1));
    HIP_TRY(hipEventElapsedTime(&t2, e1, e2));
    if (ms_row) *ms_row = double(t1) / reps;
    if (ms_col) *ms_col = double(t2) / reps;
    const double b = 2.0 * double(c->el) * double(c->L.field_elems);
    if (bytes_row) *bytes_row = b;
    if (bytes_col) *bytes_col = b;
  }
  return r;
}

int ssfm_set_screen_spectrum(ssfm_ctx* c, int32_t inst, int32_t kind, double tau,
                             double kappa_h) {
  if (int r = check_inst(c, inst)) return r;
  if (kind != SSFM_SPECTRUM_KOLMOGOROV && kind != SSFM_SPECTRUM_STEP)
    return fail(SSFM_EINVAL, "unknown spectrum kind %d", kind);
  if (kind == SSFM_SPECTRUM_STEP &&
      (!(tau >= 0.0) || !std::isfinite(tau) || !(kappa_h > 0.0) || !std::isfinite(kappa_h)))
    return fail(SSFM_EINVAL, "step spectrum needs finite tau >= 0 and kappa_h > 0");
  ssfm_ctx::Spectrum& sp = c->spectrum[inst];
  sp.kind = kind;
  sp.tau = tau;
  sp.kappa_h = kappa_h;
  return SSFM_OK;
}

int ssfm_set_subharmonics(ssfm_ctx* c, int32_t inst, int32_t levels) {
  if (int r = check_inst(c, inst)) return r;
  if (levels < 0 || levels > kMaxSubharmonicLevels)
    return fail(SSFM_EINVAL, "subharmonic levels must be in [0, %d], got %d",
                kMaxSubharmonicLevels, levels);
  c->spectrum[inst].subharmonics = levels;
  return SSFM_OK;
}

namespace {
int check_lens(const ssfm_lens* lens) {
  if (!lens) return fail(SSFM_EINVAL, "lens is NULL");
  const ssfm_lens& l = *lens;
  if (!(l.l_dif >= 0.0) || !std::isfinite(l.l_dif) || !std::isfinite(l.w_l) ||
      !std::isfinite(l.c1) || l.c1 == 0.0 || !std::isfinite(l.c2))
    return fail(SSFM_EINVAL, "lens needs finite l_dif >= 0, w_l, c2 and c1 != 0");
  if (l.n_re < 0 || l.n_re > 8 || l.n_im < 0 || l.n_im > 8)
    return fail(SSFM_EINVAL, "lens segment counts must be in [0, 8]");
  for (int part = 0; part < 2; ++part) {
    const int n = part ? l.n_im : l.n_re;
    const double(*seg)[4] = part ? l.im : l.re;
    double lo = 0.0;
    for (int j = 0; j < n; ++j) {
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(seg[j][k])) return fail(SSFM_EINVAL, "lens segment not finite");
      if (!(seg[j][0] > lo))
        return fail(SSFM_EINVAL, "lens segment radii must increase from 0");
      lo = seg[j][0];
    }
  }
  return SSFM_OK;
}
}  // namespace

int ssfm_apply_lens(ssfm_ctx* c, int32_t inst, const ssfm_lens* lens) {
  if (int r = check_inst(c, inst)) return r;
  if (int r = lie_only(c, "the effective lens")) return r;
  if (int r = check_lens(lens)) return r;
  return SSFM_DISPATCH(c, do_apply_lens, c, inst, *lens);
}

int ssfm_lens_vjp(ssfm_ctx* c, int32_t inst, const ssfm_lens* lens, const void* u_in,
                  const void* g_out, void* g_in, double* grad, int32_t n_grad) {
  if (int r = check_inst(c, inst)) return r;
  if (int r = check_lens(lens)) return r;
  if (!u_in || !g_out || !g_in || !grad)
    return fail(SSFM_EINVAL, "u_in, g_out, g_in and grad must not be NULL");
  const int need = 2 + 3 * (lens->n_re + lens->n_im);
  if (n_grad < need)
    return fail(SSFM_EINVAL, "grad holds %d values, the lens has %d parameters", n_grad, need);
  return SSFM_DISPATCH(c, do_lens_vjp, c, inst, *lens, static_cast<const double*>(u_in),
                       static_cast<const double*>(g_out), static_cast<double*>(g_in), grad);
}

int ssfm_hot_areas(ssfm_ctx* c, const double* w, int32_t n, double threshold, int32_t periodic,
                   int64_t* count) {
  if (int r = check_ctx(c)) return r;
  if (!w || !count) return fail(SSFM_EINVAL, "w/count is NULL");
  if (n < 1 || n > c->L.max_n)
    return fail(SSFM_EINVAL, "n=%d must be in [1, %d] (the context's largest grid)", n,
                c->L.max_n);
  if (!std::isfinite(threshold)) return fail(SSFM_EINVAL, "threshold must be finite");
  // labels (n^2 ints) and the overflow flag live in the staging buffer
  int* labels = c->at<int>(c->L.stage);
  int* overflow = labels + int64_t(n) * n;
  double* part = c->at<double>(c->L.sumsq_part);
  constexpr int kParts = 256;
  HIP_TRY(launch_hot_areas(w, n, threshold, periodic ? 1 : 0, labels, overflow, part, kParts,
                           c->stream));
  double host[kParts];
  int ovf = 0;
  HIP_TRY(hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (ovf) return fail(SSFM_EHIP, "hot-area labelling: a union exceeded its retry cap");
  double total = 0.0;
  for (int k = 0; k < kParts; ++k) total += host[k];
  *count = int64_t(total);
  return SSFM_OK;
}

int ssfm_hot_areas_static(const double* w, int32_t n, double threshold, int32_t periodic,
                          void* stream, int64_t* count) {
  g_last_error.clear();
  if (!w || !count) return fail(SSFM_EINVAL, "w/count is NULL");
  if (n < 1 || n > kStaticMaxN)
    return fail(SSFM_EINVAL,
                "n=%d outside [1, %d], the static scratch's largest grid (larger grids: "
                "ssfm_hot_areas with a context)", n, kStaticMaxN);
  if (!std::isfinite(threshold)) return fail(SSFM_EINVAL, "threshold must be finite");
  void* base = nullptr;
  HIP_TRY(static_scratch(&base));
  char* sc = static_cast<char*>(base);
  int* labels = reinterpret_cast<int*>(sc);
  int* overflow = reinterpret_cast<int*>(sc + kStaticOverflowOff);
  double* part = reinterpret_cast<double*>(sc + kStaticPartOff);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_hot_areas(w, n, threshold, periodic ? 1 : 0, labels, overflow, part,
                           kStaticParts, st));
  double host[kStaticParts];
  int ovf = 0;
  HIP_TRY(hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ovf) return fail(SSFM_EHIP, "hot-area labelling: a union exceeded its retry cap");
  double total = 0.0;
  for (int k = 0; k < kStaticParts; ++k) total += host[k];
  *count = int64_t(total);
  return SSFM_OK;
}

namespace {
// The measure vector of an n x n device fluence w (see ssfm_measure_vector);
// the hot-area labels use the staging area's first half.
int measure(ssfm_ctx* c, const double* w, int32_t n, double length, double w_p,
            int32_t periodic, double* p) {
  constexpr int kParts = 256;
  const double dx = length / n;
  double* part = c->at<double>(c->L.sumsq_part) + kParts;
  HIP_TRY(launch_measure(w, n, dx, part, kParts, c->stream));
  std::vector<double> host(5 * kParts);
  HIP_TRY(hipMemcpyAsync(host.data(), part, sizeof(double) * host.size(), hipMemcpyDeviceToHost,
                         c->stream));
  int64_t count = 0;
  if (int r = ssfm_hot_areas(c, w, n, w_p, periodic, &count)) return r;  // synchronises
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, mx = 0.0;
  for (int b = 0; b < kParts; ++b) {
    for (int k = 0; k < 4; ++k) acc[k] += host[5 * b + k];
    mx = std::max(mx, host[5 * b + 4]);
  }
  p[0] = acc[0] * dx * dx;  // Q(1, 0)
  p[1] = acc[1] * dx * dx;  // Q(1, 1)
  p[2] = acc[2] * dx * dx;  // Q(2, 0)
  p[3] = acc[3] * dx * dx;  // Q(2, 1)
  p[4] = mx;
  p[5] = double(count);
  return SSFM_OK;
}
}  // namespace

int ssfm_measure_vector(ssfm_ctx* c, const double* w, int32_t n, double length, double w_p,
                        int32_t periodic, double* p) {
  if (int r = check_ctx(c)) return r;
  if (!w || !p) return fail(SSFM_EINVAL, "w/p is NULL");
  if (n < 1 || n > c->L.max_n || !(length > 0.0) || !std::isfinite(w_p))
    return fail(SSFM_EINVAL, "need 1 <= n <= %d, length > 0, finite w_p", c->L.max_n);
  return measure(c, w, n, length, w_p, periodic, p);
}

int ssfm_measure_distance(ssfm_ctx* c, int32_t inst, double w_p, int32_t periodic,
                          const double* p0, double* d, double* p) {
  if (int r = check_inst(c, inst)) return r;
  if (!p0 || !d) return fail(SSFM_EINVAL, "p0/d is NULL");
  if (!std::isfinite(w_p)) return fail(SSFM_EINVAL, "w_p must be finite");
  const ssfm_instance_desc& desc = c->desc[inst];
  const int n = desc.n;
  // the fluence into the staging area's second half (the labels use the first)
  double* w = c->at<double>(c->L.stage) + size_t(c->L.max_n) * c->L.max_n;
  if (int r = SSFM_DISPATCH(c, read_out, c, inst, w, SSFM_DEVICE, true)) return r;
  double pv[SSFM_MEASURE_LEN];
  if (int r = measure(c, w, n, desc.length, w_p, periodic, pv)) return r;
  double acc = 0.0;
  for (int k = 0; k < SSFM_MEASURE_LEN; ++k) {
    const double s = (p0[k] != 0.0) ? std::fabs(p0[k]) : 1.0;
    const double q = (pv[k] - p0[k]) / s;
    acc += q * q;
  }
  *d = std::sqrt(acc);
  if (p)
    for (int k = 0; k < SSFM_MEASURE_LEN; ++k) p[k] = pv[k];
  return SSFM_OK;
}

int ssfm_moment(ssfm_ctx* c, const double* w, int32_t n, double length, double p, int32_t m,
                double* q) {
  if (int r = check_ctx(c)) return r;
  if (!w || !q) return fail(SSFM_EINVAL, "w/q is NULL");
  if (n < 1 || !(length > 0.0) || m < 0 || !std::isfinite(p))
    return fail(SSFM_EINVAL, "need n >= 1, length > 0, m >= 0, finite p");
  double* part = c->at<double>(c->L.sumsq_part);
  constexpr int kParts = 256;
  const double dx = length / n;
  HIP_TRY(launch_moment(w, n, dx, p, m, part, kParts, c->stream));
  double host[kParts];
  HIP_TRY(hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (int k = 0; k < kParts; ++k) total += host[k];
  *q = total * dx * dx;
  return SSFM_OK;
}

int ssfm_set_pass_timing(ssfm_ctx* c, int32_t every) {
  if (int r = check_ctx(c)) return r;
  if (every < 0) return fail(SSFM_EINVAL, "every must be >= 0");
  if (every == c->timing_every) return SSFM_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  clear_graphs(c);  // the step graphs are cut at the sampled steps
  for (auto& e : c->samples) c->free_samples.push_back(e);
  c->samples.clear();
  c->timing_every = every;
  return SSFM_OK;
}

namespace {
// Mean span of pass 0 and pass 1 over samples: for each sample the earliest
// start to the latest stop over its size groups (group 0 launches first;
// the others run concurrently).
int mean_spans(ssfm_ctx* c, const std::vector<ssfm_ctx::PassSample>& samples, double* t0,
               double* t1, int32_t* count) {
  double acc[2] = {0.0, 0.0};
  int32_t n = 0;
  if (!samples.empty()) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t ng = c->groups.size();
    for (const auto& e : samples) {
      for (int p = 0; p < 2; ++p) {
        const hipEvent_t ref = e.ev[2 * (p * ng)];
        double lo = 0.0, hi = 0.0;
        for (size_t g = 0; g < ng; ++g) {
          float a = 0.f, b = 0.f;
          HIP_TRY(hipEventElapsedTime(&a, ref, e.ev[2 * (p * ng + g)]));
          HIP_TRY(hipEventElapsedTime(&b, ref, e.ev[2 * (p * ng + g) + 1]));
          lo = std::min(lo, double(a));
          hi = std::max(hi, double(b));
        }
        acc[p] += hi - lo;
      }
      ++n;
    }
  }
  if (t0) *t0 = n ? acc[0] / n : 0.0;
  if (t1) *t1 = n ? acc[1] / n : 0.0;
  if (count) *count = n;
  return SSFM_OK;
}
}  // namespace

int ssfm_pass_times(ssfm_ctx* c, double* ms_row, double* ms_col, int32_t* n_samples) {
  if (int r = check_ctx(c)) return r;
  return mean_spans(c, c->samples, ms_row, ms_col, n_samples);
}

int ssfm_adjoint_pass_times(ssfm_ctx* c, double* ms_col, double* ms_row, int32_t* n_samples) {
  if (int r = check_ctx(c)) return r;
  return mean_spans(c, c->adj_samples, ms_col, ms_row, n_samples);
}

int ssfm_synchronize(ssfm_ctx* c) {
  if (int r = check_ctx(c)) return r;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return SSFM_OK;
}

}  // extern "C"
