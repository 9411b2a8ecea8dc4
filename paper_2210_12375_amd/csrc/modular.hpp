// Batched ("modular") solver for neural right-hand sides: the state lives in
// HBM as [B, D] arrays.  On the matrix cores a whole solve is one persistent
// launch; otherwise each step is a short sequence of kernels (stage
// combination fused into the MLP GEMM prologue, the error norm + controller +
// commit + dense output), eight steps of which are captured once into a HIP
// graph and replayed between the running-count read-backs.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/batchode.h"

namespace bode {

struct ModularPlan {
  bode_config cfg{};
  bode_problem p{};
  // per-instance state [B]
  double* t = nullptr;
  void* h = nullptr;
  void* err_prev = nullptr;
  int32_t *n_att = nullptr, *n_acc = nullptr, *n_rej = nullptr,
          *n_fe = nullptr, *status = nullptr, *cursor = nullptr,
          *prev_rej = nullptr;
  double* h_rec = nullptr;
  double* e_rec = nullptr;
  int32_t* n_running = nullptr;  // device counter (1 int) in the workspace
  void* impl = nullptr;          // kernel-side plan (owned)
};

size_t modular_layout(const bode_config& c, void* base, ModularPlan* mp);
std::string modular_supported(const bode_config& c);
hipError_t modular_init(ModularPlan& mp, const bode_config& c,
                        const bode_problem& p, hipStream_t s);
hipError_t modular_run(ModularPlan& mp, int budget, hipStream_t s);
hipError_t modular_eval(ModularPlan& mp, const double* t_query, void* y_out,
                        int32_t* qstatus, hipStream_t s);
hipError_t modular_backward(ModularPlan& mp, const void* g_y_eval,
                            const void* g_y_final, void* dy0, void* dtheta,
                            hipStream_t s);
// Continuous adjoint of the completed solve (joint 0: per instance, 1:
// joint); the workspace (modular_cadjoint_bytes) is the caller's.
size_t modular_cadjoint_bytes(const ModularPlan& mp, int joint);
hipError_t modular_cadjoint(ModularPlan& mp, int joint, const void* g_y_eval,
                            const void* g_y_final, void* workspace,
                            void* dy0, void* dtheta, int32_t* stats,
                            hipStream_t s);
void modular_release(ModularPlan& mp);

hipError_t launch_count_equal(const int32_t* a, int n, int32_t v, int32_t* out,
                              hipStream_t s);

// Launch shapes, per configuration shape, shared by the solver handle and
// the autotuner (0 in a field: the library default).
struct Tune {
  int block = 0;      // analytic: threads per workgroup of the solve kernel
  int lanes_vdp = 0;  // analytic: lanes launched for each kind of instance
  int lanes_lin = 0;
  int waves = 0;      // neural: wavefronts per 16-row tile (4 or 8)
  int rounds = 0;     // neural per-stage path: rounds per graph / read-back
};
// set_tune also rewrites the tune cache file; set_tune_candidate only
// changes the shape used by the next solves (the autotuner's trials).
void set_tune(const bode_config& c, const Tune& t);
void set_tune_candidate(const bode_config& c, const Tune& t);
Tune get_tune(const bode_config& c);
void set_thread_error(const std::string& m);
// The process's second stream on the current device (created on first use,
// default priority), shared by every handle: work on it is ordered against
// the caller's stream by each handle's own events.
hipError_t shared_aux_stream(hipStream_t* out);
hipError_t shared_aux_stream2(hipStream_t* out);  // a third one
int autotune(const bode_config* cfg, const bode_problem* p, void* workspace,
             size_t workspace_bytes, void* stream);

}  // namespace bode
