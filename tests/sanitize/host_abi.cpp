// Host-side driver of the C ABI for AddressSanitizer / UBSan builds.
//
// Runs every host-only path of libssfm: status strings, workspace sizing
// over grid sizes, precisions, checkpoint intervals and kept segments, the
// checkpoint planner over budgets and step counts, plan-variant counts, the
// argument checks of ssfm_create (which fail before any device call), and
// every context entry point with a NULL context.  None of these touch a GPU,
// so the driver runs on a host without one.  Exit status 0 when every
// status matches; the sanitizers abort on the first memory or UB error.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ssfm.h"

static int g_fail = 0;

static void expect(bool ok, const char* what, int line) {
  if (!ok) {
    std::fprintf(stderr, "host_abi: check failed at line %d: %s (last error: %s)\n", line,
                 what, ssfm_last_error());
    ++g_fail;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

static ssfm_instance_desc beam(int n, uint32_t terms, int n_screens, double dz) {
  ssfm_instance_desc d;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.mpa_order = 8;
  d.terms = terms;
  d.n_screens = n_screens;
  d.length = 8e-3;
  d.dz = dz;
  d.wavelength = 800e-9;
  d.n2 = 3.2e-23;
  d.beta_k = 1e-120;
  d.i_ref = 5e17;
  d.cn2 = 1e-14;
  d.screen_dz = 10 * dz;
  d.seed = 1234;
  return d;
}

int main() {
  EXPECT(ssfm_version() > 0);
  for (int s = -8; s <= 1; ++s) EXPECT(ssfm_strerror(s) != nullptr && ssfm_strerror(s)[0]);
  EXPECT(ssfm_last_error() != nullptr);

  const int sizes[] = {128, 256, 512, 768, 1024, 2048, 4096};
  const uint32_t all = SSFM_KERR | SSFM_MPA | SSFM_PLASMA | SSFM_ANSATZ | SSFM_TURB;
  // workspace sizes: every size alone, and an uneven batch
  std::vector<ssfm_instance_desc> batch;
  for (int n : sizes) {
    for (int prec : {SSFM_FP32, SSFM_FP64}) {
      ssfm_instance_desc d = beam(n, all, 3, 0.1);
      size_t b = 0;
      EXPECT(ssfm_workspace_bytes(&d, 1, prec, 0, 1, 0, &b) == SSFM_OK && b > 0);
      for (int64_t steps : {1, 2, 7, 60}) {
        for (int m : {1, 2, 5, 60, 1000}) {
          for (int k : {0, 1, 3, 100}) {
            size_t bk = 0;
            EXPECT(ssfm_workspace_bytes(&d, 1, prec, steps, m, k, &bk) == SSFM_OK && bk >= b);
          }
        }
      }
      int32_t nr = 0, nc = 0;
      EXPECT(ssfm_plan_variants(n, prec, &nr, &nc) == SSFM_OK && nr > 0 && nc > 0);
    }
    if (n <= 1024) batch.push_back(beam(n, all, 2, 0.05));
  }
  size_t bb = 0;
  EXPECT(ssfm_workspace_bytes(batch.data(), int32_t(batch.size()), SSFM_FP32, 40, 6, 2, &bb) ==
         SSFM_OK);

  // checkpoint planner: budgets from below the smallest layout to above the
  // whole trajectory; the plan always fits its budget
  for (int64_t steps : {1, 2, 3, 4, 17, 60, 500}) {
    size_t full = 0;
    EXPECT(ssfm_workspace_bytes(batch.data(), int32_t(batch.size()), SSFM_FP32, steps,
                                int32_t(steps), 0, &full) == SSFM_OK);
    for (double frac : {0.0, 0.05, 0.2, 0.5, 0.9, 1.0, 2.0}) {
      const size_t budget = size_t(double(full) * frac);
      int32_t m = 0, k = 0;
      int64_t rec = -1;
      const int st = ssfm_checkpoint_plan(batch.data(), int32_t(batch.size()), SSFM_FP32,
                                          steps, budget, &m, &k, &rec);
      EXPECT(st == SSFM_OK || st == SSFM_EWORKSPACE);
      if (st == SSFM_OK) {
        size_t b = 0;
        EXPECT(ssfm_workspace_bytes(batch.data(), int32_t(batch.size()), SSFM_FP32, steps, m, k,
                                    &b) == SSFM_OK);
        EXPECT(b <= budget && m >= 1 && k >= 0 && rec >= 0 && rec < steps);
      }
    }
  }
  int32_t m = 0, k = 0;
  EXPECT(ssfm_checkpoint_plan(batch.data(), 1, SSFM_FP32, 0, 1u << 30, &m, &k, nullptr) ==
         SSFM_EINVAL);
  EXPECT(ssfm_checkpoint_plan(batch.data(), 1, SSFM_FP32, 10, 1u << 30, nullptr, &k, nullptr) ==
         SSFM_EINVAL);

  // argument checks
  ssfm_instance_desc d = beam(128, all, 3, 0.1);
  size_t b = 0;
  EXPECT(ssfm_workspace_bytes(nullptr, 1, SSFM_FP32, 0, 1, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 0, SSFM_FP32, 0, 1, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 1, 48, 0, 1, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 1, SSFM_FP32, -1, 1, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 1, SSFM_FP32, 5, 0, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 1, SSFM_FP32, 5, 2, -1, &b) == SSFM_EINVAL);
  EXPECT(ssfm_workspace_bytes(&d, 1, SSFM_FP32, 0, 1, 0, nullptr) == SSFM_EINVAL);
  ssfm_instance_desc bad = d;
  bad.n = 100;
  EXPECT(ssfm_workspace_bytes(&bad, 1, SSFM_FP32, 0, 1, 0, &b) == SSFM_EUNSUPPORTED);
  bad = d;
  bad.screen_dz = 0.5 * d.dz;
  EXPECT(ssfm_workspace_bytes(&bad, 1, SSFM_FP32, 0, 1, 0, &b) == SSFM_EINVAL);
  bad = d;
  bad.dz = NAN;
  EXPECT(ssfm_workspace_bytes(&bad, 1, SSFM_FP32, 0, 1, 0, &b) == SSFM_EINVAL);
  EXPECT(ssfm_plan_variants(100, SSFM_FP32, &m, &k) == SSFM_EUNSUPPORTED);
  EXPECT(ssfm_plan_variants(128, 16, &m, &k) == SSFM_EINVAL);

  // create refuses a missing, misaligned or short workspace before any
  // device call
  ssfm_ctx* ctx = reinterpret_cast<ssfm_ctx*>(0x1);
  EXPECT(ssfm_create(&d, 1, SSFM_FP32, 0, 1, 0, nullptr, 0, nullptr, &ctx) == SSFM_EWORKSPACE);
  EXPECT(ctx == nullptr);
  EXPECT(ssfm_create(&d, 1, SSFM_FP32, 0, 1, 0, reinterpret_cast<void*>(257), size_t(1) << 30,
                     nullptr, &ctx) == SSFM_EWORKSPACE);
  EXPECT(ssfm_create(&d, 1, SSFM_FP32, 0, 1, 0, reinterpret_cast<void*>(256), 16, nullptr,
                     &ctx) == SSFM_EWORKSPACE);
  EXPECT(ssfm_create(&d, 1, SSFM_FP32, 0, 1, 0, nullptr, 0, nullptr, nullptr) == SSFM_EINVAL);

  // every context call refuses a NULL context
  double x = 0, y = 0, th[8] = {0};
  int32_t ns = 0;
  int64_t cnt = 0;
  ssfm_lens lens;
  std::memset(&lens, 0, sizeof(lens));
  EXPECT(ssfm_destroy(nullptr) == SSFM_OK);
  EXPECT(ssfm_set_field(nullptr, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_set_theta(nullptr, 0, th) == SSFM_EINVAL);
  EXPECT(ssfm_gen_screens(nullptr) == SSFM_EINVAL);
  EXPECT(ssfm_set_splitting(nullptr, 0) == SSFM_EINVAL);
  EXPECT(ssfm_set_fd_iterations(nullptr, 4) == SSFM_EINVAL);
  EXPECT(ssfm_set_screen_spectrum(nullptr, 0, 0, 1.0, 1.0) == SSFM_EINVAL);
  EXPECT(ssfm_set_subharmonics(nullptr, 0, 1) == SSFM_EINVAL);
  EXPECT(ssfm_get_screen(nullptr, 0, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_propagate(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_get_field(nullptr, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_get_intensity(nullptr, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_get_diag(nullptr, 0, &x, &y, 1) == SSFM_EINVAL);
  EXPECT(ssfm_forward_record(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_set_cotangent(nullptr, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_fluence_loss(nullptr, 0, &x, SSFM_HOST, &y) == SSFM_EINVAL);
  EXPECT(ssfm_fluence_mismatch(nullptr, 0, &x, SSFM_HOST, &y) == SSFM_EINVAL);
  EXPECT(ssfm_backward(nullptr) == SSFM_EINVAL);
  EXPECT(ssfm_get_grad_field(nullptr, 0, &x, SSFM_HOST) == SSFM_EINVAL);
  EXPECT(ssfm_get_grad_theta(nullptr, 0, th) == SSFM_EINVAL);
  EXPECT(ssfm_block_mean(nullptr, &x, 128, 8, &y) == SSFM_EINVAL);
  EXPECT(ssfm_apply_lens(nullptr, 0, &lens) == SSFM_EINVAL);
  EXPECT(ssfm_lens_vjp(nullptr, 0, &lens, &x, &x, &y, th, 8) == SSFM_EINVAL);
  EXPECT(ssfm_hot_areas(nullptr, &x, 128, 1.0, 0, &cnt) == SSFM_EINVAL);
  EXPECT(ssfm_hot_areas_static(nullptr, 128, 1.0, 0, nullptr, &cnt) == SSFM_EINVAL);
  EXPECT(ssfm_hot_areas_static(&x, 4096, 1.0, 0, nullptr, &cnt) == SSFM_EINVAL);
  EXPECT(ssfm_moment(nullptr, &x, 128, 1.0, 1.0, 0, &y) == SSFM_EINVAL);
  EXPECT(ssfm_measure_vector(nullptr, &x, 128, 1.0, 1.0, 0, th) == SSFM_EINVAL);
  EXPECT(ssfm_measure_distance(nullptr, 0, 1.0, 0, th, &y, th) == SSFM_EINVAL);
  EXPECT(ssfm_set_precise_math(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_set_recompute_overlap(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_use_graphs(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_select_plan(nullptr, 128, 0, 0) == SSFM_EINVAL);
  EXPECT(ssfm_select_adjoint_plan(nullptr, 128, 0, 0) == SSFM_EINVAL);
  EXPECT(ssfm_time_adjoint_passes(nullptr, 1, &x, &y) == SSFM_EINVAL);
  EXPECT(ssfm_time_passes(nullptr, 1, &x, &y, &x, &y) == SSFM_EINVAL);
  EXPECT(ssfm_set_pass_timing(nullptr, 1) == SSFM_EINVAL);
  EXPECT(ssfm_pass_times(nullptr, &x, &y, &ns) == SSFM_EINVAL);
  EXPECT(ssfm_adjoint_pass_times(nullptr, &x, &y, &ns) == SSFM_EINVAL);
  EXPECT(ssfm_synchronize(nullptr) == SSFM_EINVAL);

  if (g_fail) {
    std::fprintf(stderr, "host_abi: %d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host_abi: all checks passed\n");
  return 0;
}
