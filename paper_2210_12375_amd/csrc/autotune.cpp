// solver_autotune: times launch candidates on the caller's problem and keeps
// the fastest shape for later solver_init calls with the same configuration
// shape (and, when BATCHODE_TUNE_CACHE names a file, in that file).
//
// Candidates:
//  - analytic fields (the persistent per-lane solver): threads per workgroup
//    {64, 128, 256} x lanes launched per kind of instance {B, B/2, B/4};
//  - neural fields: wavefronts per 16-row tile {4, 8} (the default for the
//    width first) for the matrix-core kernels, and for the per-stage path
//    rounds per captured graph / running-count read-back {4, 8, 16}.
// Every candidate computes the same result bit for bit (the shapes change
// which lane or wavefront does a piece of work, never the order of any
// sum), so the search only picks the fastest.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/batchode.h"
#include "mlp_mfma.hpp"
#include "modular.hpp"

namespace bode {

namespace {

// One full solve (init + solve) with the given shape; returns the best of
// reps - 1 timed runs in milliseconds (the first warms up) or a negative
// value on failure.
float time_solve(bode_config c, const bode_problem* p, void* ws, size_t bytes,
                 hipStream_t s, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1.f;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1.f;
  }
  float best = -1.f;
  for (int r = 0; r < reps; ++r) {
    bode_solver* h = nullptr;
    if (hipEventRecord(a, s) != hipSuccess) break;
    if (solver_init(&c, p, ws, bytes, s, &h) != BODE_OK) break;
    const int rc = solver_solve(h);
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    solver_destroy(h);
    if (rc != BODE_OK) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) break;
    if (r > 0 && (best < 0.f || ms < best)) best = ms;  // first run warms up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace

int autotune(const bode_config* cfg, const bode_problem* p, void* workspace,
             size_t workspace_bytes, void* stream) {
  if (!cfg || !p) {
    set_thread_error("autotune: config or problem is NULL");
    return BODE_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Tune before = get_tune(*cfg);
  std::vector<Tune> cands;
  if (cfg->rhs == BODE_RHS_ANALYTIC) {
    for (int blk : {64, 128, 256})
      for (int f : {1, 2, 4}) {
        Tune t;
        t.block = blk;
        t.lanes_vdp = t.lanes_lin = (cfg->B + f - 1) / f;
        cands.push_back(t);
      }
  } else {
    const int din = cfg->rhs == BODE_RHS_CNF ? cfg->D - 1 : cfg->D;
    const bool mfma =
        cfg->precision == BODE_BF16 ||
        (cfg->precision == BODE_FP32 &&
         mfma_supported(din, cfg->mlp_hidden).empty());
    const bool fused = mfma && !cfg->keep_dense;
    std::vector<int> waves = {0};
    if (mfma && cfg->mlp_hidden > 64) {
      const int def = mfma_waves(cfg->mlp_hidden, cfg->rhs == BODE_RHS_CNF,
                                 cfg->B, 0);
      waves = {def, def == 8 ? 4 : 8};
    }
    std::vector<int> rounds = {0};
    if (!fused) rounds = {8, 4, 16};
    for (int w : waves)
      for (int r : rounds) {
        Tune t;
        t.waves = w;
        t.rounds = r;
        cands.push_back(t);
      }
  }
  float best = -1.f;
  Tune best_t;
  for (const Tune& t : cands) {
    set_tune_candidate(*cfg, t);
    bode_config c = *cfg;
    c.tune_block = t.block;
    c.tune_lanes = t.lanes_vdp;
    const float ms = time_solve(c, p, workspace, workspace_bytes, s, 3);
    if (ms < 0.f) {
      set_tune_candidate(*cfg, before);
      set_thread_error("autotune: a candidate solve failed");
      return BODE_EHIP;
    }
    if (best < 0.f || ms < best) {
      best = ms;
      best_t = t;
    }
  }
  set_tune(*cfg, best_t);
  return BODE_OK;
}

}  // namespace bode
