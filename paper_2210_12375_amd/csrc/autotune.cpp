// solver_autotune: times launch candidates on the caller's problem and keeps
// the fastest shape for later solver_init calls with the same configuration.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/batchode.h"
#include "modular.hpp"

namespace bode {

namespace {

// One full solve (init + solve) with the given shape; returns milliseconds or
// a negative value on failure.
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
  bode_config c = *cfg;
  float best = -1.f;
  int best_block = 0, best_lanes = 0, best_tile = 0;
  std::vector<int> blocks = {64, 128, 256};
  std::vector<int> lanes;
  if (c.rhs == BODE_RHS_ANALYTIC) {
    for (int f : {1, 2, 4}) lanes.push_back((c.B + f - 1) / f);
  } else {
    lanes.push_back(0);
  }
  std::vector<int> tiles = {0};
  for (int blk : blocks)
    for (int ln : lanes)
      for (int tile : tiles) {
        c.tune_block = blk;
        c.tune_lanes = ln;
        const float ms = time_solve(c, p, workspace, workspace_bytes, s, 3);
        if (ms < 0.f) {
          set_thread_error("autotune: a candidate solve failed");
          return BODE_EHIP;
        }
        if (best < 0.f || ms < best) {
          best = ms;
          best_block = blk;
          best_lanes = ln;
          best_tile = tile;
        }
      }
  set_tune(*cfg, best_block, best_lanes, best_lanes, best_tile);
  return BODE_OK;
}

}  // namespace bode
