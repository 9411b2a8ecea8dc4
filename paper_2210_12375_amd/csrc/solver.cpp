// C ABI of the batchode library (declared in include/batchode.h).
//
// The host side validates arguments, lays out the caller's workspace,
// enqueues kernels on the caller's stream and copies statistics.  It owns no
// device memory.  Each entry point catches everything, so no C++ exception
// crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/batchode.h"
#include "analytic.hpp"
#include "common.hpp"
#include "modular.hpp"
#include "noalloc.hpp"
#include "tableau.hpp"

namespace {

thread_local std::string g_thread_error;

struct Layout {
  char* base;
  size_t off = 0;
  explicit Layout(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// Launch shapes chosen by solver_autotune, per device architecture and
// configuration shape (right-hand side, precision, method, B, D, E, hidden
// width, plain BF16).  When BATCHODE_TUNE_CACHE names a file, the shapes
// are read from it on first use and every autotune rewrites it: one JSON
// object per line.
using bode::Tune;
typedef std::tuple<std::string, int, int, int, int, int, int, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, Tune> g_tune;
bool g_tune_loaded = false;

// The current device's architecture name, asked of the runtime once per
// device (the query is slow, and every launch-shape lookup needs it).
std::mutex g_arch_mu;
std::map<int, std::string> g_arch;

std::string device_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(g_arch_mu);
  auto it = g_arch.find(dev);
  if (it != g_arch.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a = a.substr(0, colon);
  g_arch[dev] = a;
  return a;
}

TuneKey tune_key(const bode_config& c) {
  return TuneKey(device_arch(), c.rhs, c.precision, c.method, c.B, c.D, c.E,
                 c.rhs == BODE_RHS_ANALYTIC ? 0 : c.mlp_hidden,
                 c.precision == BODE_BF16 ? c.plain_bf16 : 0);
}

// The integer after "name": in a line of the cache (absent: fallback).
long json_int(const std::string& line, const char* name, long fallback) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return fallback;
  return std::strtol(line.c_str() + p + pat.size(), nullptr, 10);
}

std::string json_str(const std::string& line, const char* name) {
  const std::string pat = std::string("\"") + name + "\":\"";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return "";
  const size_t q = line.find('"', p + pat.size());
  return q == std::string::npos ? "" : line.substr(p + pat.size(),
                                                   q - p - pat.size());
}

const char* tune_cache_path() {
  const char* p = std::getenv("BATCHODE_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// Caller holds g_tune_mu.
void load_tune_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char buf[1024];
  while (std::fgets(buf, sizeof buf, f)) {
    const std::string line(buf);
    const std::string arch = json_str(line, "arch");
    if (arch.empty()) continue;
    TuneKey k(arch, (int)json_int(line, "rhs", -1),
              (int)json_int(line, "precision", -1),
              (int)json_int(line, "method", -1), (int)json_int(line, "B", -1),
              (int)json_int(line, "D", -1), (int)json_int(line, "E", -1),
              (int)json_int(line, "H", -1), (int)json_int(line, "plain", -1));
    Tune t;
    t.block = (int)json_int(line, "block", 0);
    t.lanes_vdp = (int)json_int(line, "lanes_vdp", 0);
    t.lanes_lin = (int)json_int(line, "lanes_lin", 0);
    t.waves = (int)json_int(line, "waves", 0);
    t.rounds = (int)json_int(line, "rounds", 0);
    g_tune[k] = t;
  }
  std::fclose(f);
}

// Caller holds g_tune_mu.  Rewrites the whole cache (temporary file, then
// rename), so a reader never sees a half-written line.
bool save_tune_cache() {
  const char* path = tune_cache_path();
  if (!path) return true;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  for (const auto& kv : g_tune) {
    const TuneKey& k = kv.first;
    const Tune& t = kv.second;
    std::fprintf(f,
                 "{\"arch\":\"%s\",\"rhs\":%d,\"precision\":%d,\"method\":%d,"
                 "\"B\":%d,\"D\":%d,\"E\":%d,\"H\":%d,\"plain\":%d,"
                 "\"block\":%d,\"lanes_vdp\":%d,\"lanes_lin\":%d,"
                 "\"waves\":%d,\"rounds\":%d}\n",
                 std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k),
                 std::get<6>(k), std::get<7>(k), std::get<8>(k), t.block,
                 t.lanes_vdp, t.lanes_lin, t.waves, t.rounds);
  }
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// One second stream per device for the linear-instance kernel, created on
// first use and kept for the life of the process (default priority).
std::mutex g_aux_mu;
std::map<int, hipStream_t> g_aux;

hipError_t aux_stream(hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  auto it = g_aux.find(dev);
  if (it != g_aux.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  g_aux[dev] = s;
  *out = s;
  return hipSuccess;
}

}  // namespace

namespace bode {
hipError_t shared_aux_stream(hipStream_t* out) { return aux_stream(out); }

// A third stream per device, created on first use (default priority).
std::mutex g_aux2_mu;
std::map<int, hipStream_t> g_aux2;

hipError_t shared_aux_stream2(hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_aux2_mu);
  auto it = g_aux2.find(dev);
  if (it != g_aux2.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  g_aux2[dev] = s;
  *out = s;
  return hipSuccess;
}
}  // namespace bode

struct bode_solver {
  bode_config cfg{};
  bode_problem p{};
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bode::AnalyticArgs<double> ad{};
  bode::AnalyticArgs<float> af{};
  bode::ModularPlan mp{};
  int32_t* counts = nullptr;
  int32_t* n_running_dev = nullptr;
  Tune tune{};
  bool stepped = false;
  std::string err;
};

namespace {

int fail(bode_solver* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  g_thread_error = msg;
  return code;
}

bool is64(const bode_config& c) { return c.precision == BODE_FP64; }

std::string check_config(const bode_config* c) {
  if (!c) return "config is NULL";
  if (c->method != BODE_DOPRI5 && c->method != BODE_TSIT5)
    return "method must be BODE_DOPRI5 or BODE_TSIT5";
  if (c->precision < BODE_FP64 || c->precision > BODE_BF16)
    return "precision must be BODE_FP64, BODE_FP32 or BODE_BF16";
  if (c->rhs != BODE_RHS_ANALYTIC && c->rhs != BODE_RHS_MLP &&
      c->rhs != BODE_RHS_CNF)
    return "rhs must be BODE_RHS_ANALYTIC, BODE_RHS_MLP or BODE_RHS_CNF";
  if (c->B < 1) return "B must be >= 1";
  if (c->D < 1) return "D must be >= 1";
  if (c->rhs == BODE_RHS_ANALYTIC && c->D > 8)
    return "analytic batches need D <= 8";
  if (c->rhs == BODE_RHS_CNF && c->D < 2) return "CNF needs D >= 2";
  if (c->E < 0) return "E must be >= 0";
  if (c->max_steps < 1) return "max_steps must be >= 1";
  if (!(c->safety > 0.0) || !(c->fac_min > 0.0) || !(c->fac_min <= 1.0) ||
      !(c->fac_max >= 1.0) || !(c->beta1 >= 0.0) ||
      !std::isfinite(c->beta1) || !std::isfinite(c->beta2) ||
      !std::isfinite(c->beta3) || !std::isfinite(c->fac_max) ||
      !std::isfinite(c->safety))
    return "controller needs safety > 0, 0 < fac_min <= 1 <= fac_max, "
           "finite beta1 >= 0, finite beta2 and beta3";
  if (c->joint != 0 && c->joint != 1) return "joint must be 0 or 1";
  if (c->joint && (c->rhs != BODE_RHS_ANALYTIC || c->keep_dense != 0))
    return "joint mode is built for analytic fields without keep_dense";
  if (c->fixed_step != 0 && c->fixed_step != 1)
    return "fixed_step must be 0 or 1";
  if (c->eager != 0 && c->eager != 1) return "eager must be 0 or 1";
  if (c->plain_bf16 != 0 && c->plain_bf16 != 1)
    return "plain_bf16 must be 0 or 1";
  if (c->fixed_step && c->joint)
    return "fixed_step is not built for joint mode";
  if (c->record_cap < 0) return "record_cap must be >= 0";
  if (c->ckpt_every < 0) return "ckpt_every must be >= 0";
  if (c->ckpt_every > 0 && c->record_cap < 1)
    return "checkpoints need record_cap > 0";
  if (c->rhs != BODE_RHS_ANALYTIC && c->mlp_hidden < 1)
    return "mlp_hidden must be >= 1 for neural right-hand sides";
  if ((long)c->B * (long)std::max(c->D, 1) * std::max(c->E, 1) > (1L << 40))
    return "problem too large";
  return "";
}

// Host-visible checks of the problem description (the device inputs are
// checked per instance by the initialisation kernels).
std::string check_problem(const bode_config& c, const bode_problem* p) {
  if (!p) return "problem is NULL";
  if (!p->y0 || !p->t0 || !p->t_end || !p->rtol || !p->atol || !p->y_final)
    return "y0, t0, t_end, rtol, atol and y_final are required";
  if (c.E > 0 && (!p->t_eval || !p->y_eval))
    return "E > 0 needs t_eval and y_eval";
  if (c.rhs == BODE_RHS_ANALYTIC && (!p->kind || !p->dim))
    return "analytic batches need kind and dim";
  if (c.rhs != BODE_RHS_ANALYTIC &&
      (!p->W1 || !p->b1 || !p->W2 || !p->b2 || !p->W3 || !p->b3))
    return "neural fields need W1..b3";
  if (c.rhs == BODE_RHS_CNF && !p->eps) return "CNF needs eps";
  if (c.fixed_step && !p->h0) return "fixed_step needs h0 (the step)";
  return "";
}

template <typename R>
size_t layout_analytic(const bode_config& c, void* base,
                       bode::AnalyticArgs<R>* a, int32_t** counts,
                       int32_t** n_running) {
  Layout L(base);
  const size_t B = c.B, D = c.D;
  bode::State<R> st;
  st.t = L.take<double>(B);
  st.h = L.take<R>(B);
  st.err_prev = L.take<R>(B);
  st.err_prev2 = L.take<R>(B);
  st.n_att = L.take<int32_t>(B);
  st.n_acc = L.take<int32_t>(B);
  st.n_rej = L.take<int32_t>(B);
  st.n_fe = L.take<int32_t>(B);
  st.status = L.take<int32_t>(B);
  st.cursor = L.take<int32_t>(B);
  st.prev_rej = L.take<int32_t>(B);
  st.y = L.take<R>(B * D);
  st.k1 = L.take<R>(B * D);
  st.yc = c.joint ? nullptr : L.take<R>(B * D);
  int32_t* list = L.take<int32_t>(B);
  int32_t* cnt = L.take<int32_t>(8);
  double* h_rec = c.record_cap > 0 ? L.take<double>(B * c.record_cap) : nullptr;
  double* e_rec = c.record_cap > 0 ? L.take<double>(B * c.record_cap) : nullptr;
  bode::DenseKeep<R> dk{};
  if (c.keep_dense) {
    dk.t_prev = L.take<double>(B);
    dk.h_last = L.take<R>(B);
    dk.y_prev = L.take<R>(B * D);
    dk.q = L.take<R>(4 * B * D);
  }
  bode::JointState* js = nullptr;
  R *jK = nullptr, *jY = nullptr;
  if (c.joint) {
    js = L.take<bode::JointState>(1);
    jK = L.take<R>(6 * B * D);
    jY = L.take<R>(B * D);
  }
  if (a) {
    a->js = js;
    a->jK = jK;
    a->jY = jY;
    a->st = st;
    a->list = list;
    a->counts = cnt;
    a->h_rec = h_rec;
    a->e_rec = e_rec;
    a->rec_cap = c.record_cap;
    a->dk = dk;
    a->keep_dense = c.keep_dense;
  }
  if (counts) *counts = cnt;
  if (n_running) *n_running = cnt + 4;
  return L.off + 256;
}

size_t workspace_bytes(const bode_config& c) {
  if (c.rhs == BODE_RHS_ANALYTIC)
    return is64(c) ? layout_analytic<double>(c, nullptr, nullptr, nullptr,
                                             nullptr)
                   : layout_analytic<float>(c, nullptr, nullptr, nullptr,
                                            nullptr);
  return bode::modular_layout(c, nullptr, nullptr);
}

template <typename R>
void fill_analytic_args(bode_solver* s, bode::AnalyticArgs<R>* a) {
  const bode_config& c = s->cfg;
  const bode_problem& p = s->p;
  a->B = c.B;
  a->D = c.D;
  a->E = c.E;
  a->y0 = static_cast<const R*>(p.y0);
  a->t0 = p.t0;
  a->t_end = p.t_end;
  a->rtol = p.rtol;
  a->atol = p.atol;
  a->t_eval = p.t_eval;
  a->h0 = p.h0;
  a->kind = p.kind;
  a->dim = p.dim;
  a->mu = static_cast<const R*>(p.mu);
  a->A = static_cast<const R*>(p.A);
  a->y_eval = static_cast<R*>(p.y_eval);
  a->y_final = static_cast<R*>(p.y_final);
  a->ctrl = bode::Ctrl{c.beta1, c.beta2, c.safety, c.fac_min, c.fac_max,
                       c.max_steps, c.beta3, c.fixed_step};
  a->budget = c.max_steps + 1;
}

// Launch shapes: the autotuned ones for this shape, overridden by the
// configuration's explicit tune fields.
void apply_tune(bode_solver* s) {
  const bode_config& c = s->cfg;
  s->tune = bode::get_tune(c);
  if (c.tune_block > 0) s->tune.block = c.tune_block;
  if (c.tune_lanes > 0) s->tune.lanes_vdp = s->tune.lanes_lin = c.tune_lanes;
}

// Per-device resources of solver_solve_noalloc, set up on its first call on
// a device (with that device current) and kept for the life of the process:
// the address of the device's copy of the static scratch array, the second
// stream of the analytic solve and the two events that fork and join it.
struct NoallocDevice {
  void* scratch = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_noalloc_mu;
std::map<int, NoallocDevice> g_noalloc;

hipError_t noalloc_device(NoallocDevice* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc.find(dev);
  if (it != g_noalloc.end()) {
    *out = it->second;
    return hipSuccess;
  }
  NoallocDevice d;
  e = bode::noalloc_scratch(&d.scratch);
  if (e != hipSuccess) return e;
  e = aux_stream(&d.aux);
  if (e != hipSuccess) return e;
  e = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventCreateWithFlags(&d.join, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipEventDestroy(d.fork);
    return e;
  }
  g_noalloc[dev] = d;
  *out = d;
  return hipSuccess;
}

// Lays out the analytic plan in s->ws and enqueues the initialisation (the
// work-queue counters are cleared by a fill kernel, not a memset).
template <typename R>
hipError_t start_analytic_t(bode_solver* s, bode::AnalyticArgs<R>* a) {
  const bode_config& c = s->cfg;
  layout_analytic<R>(c, s->ws, a, &s->counts, &s->n_running_dev);
  fill_analytic_args<R>(s, a);
  hipError_t e = bode::launch_fill_i32(s->counts, 8, 0, s->stream);
  if (e != hipSuccess) return e;
  return c.joint ? bode::launch_joint_init<R>(*a, c.method, s->stream)
                 : bode::launch_analytic_init<R>(*a, c.method, s->stream);
}

hipError_t start_analytic(bode_solver* s) {
  return is64(s->cfg) ? start_analytic_t<double>(s, &s->ad)
                      : start_analytic_t<float>(s, &s->af);
}

#define HIP_TRY(expr)                                                    \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess)                                                \
      return fail(s, BODE_EHIP, std::string(#expr) + ": " +             \
                                    hipGetErrorString(e_));              \
  } while (0)

// Van der Pol instances on the caller's stream, linear ones on a second
// stream, so the two kernels (each with its own register budget) overlap.
template <typename R>
int run_analytic(bode_solver* s, bode::AnalyticArgs<R>& a, int budget) {
  a.budget = budget;
  if (s->cfg.joint) {
    HIP_TRY(bode::launch_joint_solve<R>(a, s->cfg.method, s->stream));
    return BODE_OK;
  }
  HIP_TRY(bode::launch_fill_i32(s->counts + 2, 2, 0, s->stream));
  HIP_TRY(hipEventRecord(s->ev_fork, s->stream));
  HIP_TRY(hipStreamWaitEvent(s->aux, s->ev_fork, 0));
  const int lanes_v = s->tune.lanes_vdp > 0 ? s->tune.lanes_vdp : s->cfg.B;
  const int lanes_l = s->tune.lanes_lin > 0 ? s->tune.lanes_lin : s->cfg.B;
  const int block = s->tune.block > 0 ? s->tune.block : 64;
  HIP_TRY(bode::launch_analytic_solve<R>(a, s->cfg.method, bode::kKindVdp,
                                         std::min(lanes_v, s->cfg.B), block,
                                         s->stream));
  HIP_TRY(bode::launch_analytic_solve<R>(a, s->cfg.method, bode::kKindLinear,
                                         std::min(lanes_l, s->cfg.B), block,
                                         s->aux));
  HIP_TRY(hipEventRecord(s->ev_join, s->aux));
  HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_join, 0));
  return BODE_OK;
}

int run_steps(bode_solver* s, int budget) {
  if (s->cfg.rhs == BODE_RHS_ANALYTIC)
    return is64(s->cfg) ? run_analytic<double>(s, s->ad, budget)
                        : run_analytic<float>(s, s->af, budget);
  hipError_t e = bode::modular_run(s->mp, budget, s->stream);
  if (e != hipSuccess)
    return fail(s, BODE_EHIP, std::string("modular solve: ") +
                                  hipGetErrorString(e));
  return BODE_OK;
}

const int32_t* status_ptr(const bode_solver* s) {
  if (s->cfg.rhs == BODE_RHS_ANALYTIC)
    return is64(s->cfg) ? s->ad.st.status : s->af.st.status;
  return s->mp.status;
}

}  // namespace

extern "C" {

size_t solver_workspace_size(const bode_config* cfg) {
  try {
    if (!check_config(cfg).empty()) return 0;
    return workspace_bytes(*cfg);
  } catch (...) {
    return 0;
  }
}

int solver_init(const bode_config* cfg, const bode_problem* p, void* workspace,
                size_t workspace_bytes_, void* stream, bode_solver** out) {
  bode_solver* s = nullptr;
  try {
    if (!out) return fail(nullptr, BODE_EINVAL, "out is NULL");
    *out = nullptr;
    const std::string msg = check_config(cfg);
    if (!msg.empty()) return fail(nullptr, BODE_EINVAL, msg);
    const std::string pmsg = check_problem(*cfg, p);
    if (!pmsg.empty()) return fail(nullptr, BODE_EINVAL, pmsg);
    const size_t need = workspace_bytes(*cfg);
    if (!workspace) return fail(nullptr, BODE_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(nullptr, BODE_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes_ < need)
      return fail(nullptr, BODE_EINVAL,
                  "workspace too small: need " + std::to_string(need) +
                      " bytes");
    if (cfg->rhs != BODE_RHS_ANALYTIC) {
      std::string why = bode::modular_supported(*cfg);
      if (!why.empty()) return fail(nullptr, BODE_EUNSUPPORTED, why);
    }

    s = new bode_solver();
    s->cfg = *cfg;
    s->p = *p;
    s->ws = workspace;
    s->ws_bytes = workspace_bytes_;
    s->stream = static_cast<hipStream_t>(stream);
    apply_tune(s);

    if (cfg->rhs == BODE_RHS_ANALYTIC) {
      if (aux_stream(&s->aux) != hipSuccess ||
          hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) !=
              hipSuccess ||
          hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming) !=
              hipSuccess) {
        solver_destroy(s);
        return fail(nullptr, BODE_EHIP, "cannot create stream/events");
      }
      const hipError_t e = start_analytic(s);
      if (e != hipSuccess) {
        std::string m = std::string("init launch: ") + hipGetErrorString(e);
        solver_destroy(s);
        return fail(nullptr, BODE_EHIP, m);
      }
    } else {
      bode::modular_layout(*cfg, workspace, &s->mp);
      hipError_t e = bode::modular_init(s->mp, *cfg, *p, s->stream);
      if (e != hipSuccess) {
        std::string m = std::string("init: ") + hipGetErrorString(e);
        solver_destroy(s);
        return fail(nullptr, BODE_EHIP, m);
      }
      s->n_running_dev = s->mp.n_running;
    }
    *out = s;
    return BODE_OK;
  } catch (const std::exception& ex) {
    if (s) solver_destroy(s);
    return fail(nullptr, BODE_EHIP, ex.what());
  } catch (...) {
    if (s) solver_destroy(s);
    return fail(nullptr, BODE_EHIP, "unknown error in solver_init");
  }
}

int solver_step(bode_solver* s, int32_t n_attempts, int32_t* n_running_host) {
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (n_attempts < 1) return fail(s, BODE_EINVAL, "n_attempts must be >= 1");
    int rc = run_steps(s, n_attempts);
    if (rc != BODE_OK) return rc;
    s->stepped = true;
    if (n_running_host) {
      if (s->n_running_dev == nullptr)
        return fail(s, BODE_ESTATE, "no running-count buffer in this plan");
      HIP_TRY(bode::launch_fill_i32(s->n_running_dev, 1, 0, s->stream));
      HIP_TRY(bode::launch_count_equal(status_ptr(s), s->cfg.B, bode::kRunning,
                                       s->n_running_dev, s->stream));
      HIP_TRY(hipMemcpyAsync(n_running_host, s->n_running_dev, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_step");
  }
}

int solver_solve(bode_solver* s) {
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    int rc = run_steps(s, s->cfg.max_steps + 1);
    if (rc == BODE_OK) s->stepped = true;
    return rc;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_solve");
  }
}

int solver_solve_noalloc(const bode_config* cfg, const bode_problem* p,
                         int32_t* stats, void* stream) {
  try {
    const std::string msg = check_config(cfg);
    if (!msg.empty()) return fail(nullptr, BODE_EINVAL, msg);
    const std::string pmsg = check_problem(*cfg, p);
    if (!pmsg.empty()) return fail(nullptr, BODE_EINVAL, pmsg);
    if (cfg->rhs != BODE_RHS_ANALYTIC)
      return fail(nullptr, BODE_EUNSUPPORTED,
                  "solver_solve_noalloc is built for analytic fields");
    const size_t need = workspace_bytes(*cfg);
    if (need > bode::kNoallocBytes)
      return fail(nullptr, BODE_EINVAL,
                  "problem needs " + std::to_string(need) +
                      " bytes of workspace; solver_solve_noalloc holds " +
                      std::to_string(bode::kNoallocBytes));
    NoallocDevice dev;
    hipError_t e = noalloc_device(&dev);
    if (e != hipSuccess)
      return fail(nullptr, BODE_EHIP,
                  std::string("scratch set-up: ") + hipGetErrorString(e));
    // A handle that lives for this call only; it owns nothing (the events
    // and the second stream are the device's).
    bode_solver s;
    s.cfg = *cfg;
    s.p = *p;
    s.ws = dev.scratch;
    s.ws_bytes = bode::kNoallocBytes;
    s.stream = static_cast<hipStream_t>(stream);
    s.aux = dev.aux;
    s.ev_fork = dev.fork;
    s.ev_join = dev.join;
    apply_tune(&s);
    e = start_analytic(&s);
    if (e != hipSuccess)
      return fail(nullptr, BODE_EHIP,
                  std::string("init launch: ") + hipGetErrorString(e));
    const int rc = run_steps(&s, cfg->max_steps + 1);
    if (rc != BODE_OK) return fail(nullptr, rc, s.err);
    if (stats) {
      const auto copy = [&](const int32_t* src, int row) {
        return hipMemcpyAsync(stats + (size_t)row * cfg->B, src,
                              sizeof(int32_t) * cfg->B,
                              hipMemcpyDeviceToDevice, s.stream);
      };
      const int32_t* src[5];
      if (is64(*cfg)) {
        const auto& st = s.ad.st;
        src[0] = st.n_att, src[1] = st.n_acc, src[2] = st.n_rej,
        src[3] = st.n_fe, src[4] = st.status;
      } else {
        const auto& st = s.af.st;
        src[0] = st.n_att, src[1] = st.n_acc, src[2] = st.n_rej,
        src[3] = st.n_fe, src[4] = st.status;
      }
      for (int k = 0; k < 5; ++k) {
        e = copy(src[k], k);
        if (e != hipSuccess)
          return fail(nullptr, BODE_EHIP,
                      std::string("statistics copy: ") + hipGetErrorString(e));
      }
    }
    return BODE_OK;
  } catch (...) {
    return fail(nullptr, BODE_EHIP, "unknown error in solver_solve_noalloc");
  }
}

int solver_eval(bode_solver* s, const double* t_query, void* y_out,
                int32_t* qstatus) {
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (!t_query || !y_out || !qstatus)
      return fail(s, BODE_EINVAL, "t_query, y_out and qstatus are required");
    if (!s->cfg.keep_dense)
      return fail(s, BODE_ESTATE, "solver_eval needs cfg.keep_dense = 1");
    if (!s->stepped) return fail(s, BODE_ESTATE, "no step has been taken yet");
    hipError_t e;
    if (s->cfg.rhs != BODE_RHS_ANALYTIC)
      e = bode::modular_eval(s->mp, t_query, y_out, qstatus, s->stream);
    else if (is64(s->cfg))
      e = bode::launch_dense_eval<double>(s->ad.dk, s->ad.st, s->cfg.B,
                                          s->cfg.D, t_query,
                                          static_cast<double*>(y_out), qstatus,
                                          s->stream);
    else
      e = bode::launch_dense_eval<float>(s->af.dk, s->af.st, s->cfg.B,
                                         s->cfg.D, t_query,
                                         static_cast<float*>(y_out), qstatus,
                                         s->stream);
    HIP_TRY(e);
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_eval");
  }
}

int solver_backward(bode_solver* s, const void* g_y_eval,
                    const void* g_y_final, void* dy0, void* dtheta) {
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (!g_y_final || !dy0)
      return fail(s, BODE_EINVAL, "g_y_final and dy0 are required");
    if (s->cfg.E > 0 && !g_y_eval)
      return fail(s, BODE_EINVAL, "g_y_eval is required when E > 0");
    if (s->cfg.record_cap < 1)
      return fail(s, BODE_ESTATE, "backward needs cfg.record_cap > 0");
    if (!s->stepped) return fail(s, BODE_ESTATE, "no completed solve");
    if (s->cfg.rhs == BODE_RHS_ANALYTIC)
      return fail(s, BODE_EUNSUPPORTED,
                  "backward is built for MLP and CNF fields");
    if (!dtheta) return fail(s, BODE_EINVAL, "dtheta is required");
    if (s->cfg.precision == BODE_BF16 && s->cfg.plain_bf16)
      return fail(s, BODE_EUNSUPPORTED,
                  "plain BF16 is built for forward solves only");
    hipError_t e = bode::modular_backward(s->mp, g_y_eval, g_y_final, dy0,
                                          dtheta, s->stream);
    if (e == hipErrorInvalidValue)
      return fail(s, BODE_ESTATE,
                  "recorded steps exceed record_cap or the solve is not "
                  "complete");
    HIP_TRY(e);
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_backward");
  }
}

size_t solver_cadjoint_workspace_bytes(const bode_solver* s, int32_t joint) {
  if (!s || s->cfg.rhs == BODE_RHS_ANALYTIC || (joint != 0 && joint != 1))
    return 0;
  return bode::modular_cadjoint_bytes(s->mp, joint);
}

int solver_cadjoint(bode_solver* s, int32_t joint, const void* g_y_eval,
                    const void* g_y_final, void* workspace,
                    size_t workspace_bytes, void* dy0, void* dtheta,
                    int32_t* stats) {
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (joint != 0 && joint != 1)
      return fail(s, BODE_EINVAL, "joint must be 0 or 1");
    if (!g_y_final || !dy0 || !dtheta || !workspace)
      return fail(s, BODE_EINVAL,
                  "g_y_final, dy0, dtheta and workspace are required");
    if (s->cfg.E > 0 && !g_y_eval)
      return fail(s, BODE_EINVAL, "g_y_eval is required when E > 0");
    if (s->cfg.rhs == BODE_RHS_ANALYTIC)
      return fail(s, BODE_EUNSUPPORTED,
                  "the continuous adjoint is built for MLP and CNF fields");
    if (s->cfg.fixed_step)
      return fail(s, BODE_EUNSUPPORTED,
                  "the continuous adjoint is built for adaptive solves");
    if (s->cfg.precision == BODE_BF16 && s->cfg.plain_bf16)
      return fail(s, BODE_EUNSUPPORTED,
                  "plain BF16 is built for forward solves only");
    if (!s->stepped) return fail(s, BODE_ESTATE, "no completed solve");
    const size_t need = bode::modular_cadjoint_bytes(s->mp, joint);
    if (workspace_bytes < need)
      return fail(s, BODE_EINVAL,
                  "workspace too small: need " + std::to_string(need) +
                      " bytes");
    HIP_TRY(bode::modular_cadjoint(s->mp, joint, g_y_eval, g_y_final,
                                   workspace, dy0, dtheta, stats, s->stream));
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_cadjoint");
  }
}

int solver_get_stats(const bode_solver* cs, int32_t* n_attempted,
                     int32_t* n_accepted, int32_t* n_rejected,
                     int32_t* n_feval, int32_t* status) {
  bode_solver* s = const_cast<bode_solver*>(cs);
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    const int32_t* src[5];
    if (s->cfg.rhs == BODE_RHS_ANALYTIC) {
      if (is64(s->cfg)) {
        const auto& st = s->ad.st;
        src[0] = st.n_att, src[1] = st.n_acc, src[2] = st.n_rej,
        src[3] = st.n_fe, src[4] = st.status;
      } else {
        const auto& st = s->af.st;
        src[0] = st.n_att, src[1] = st.n_acc, src[2] = st.n_rej,
        src[3] = st.n_fe, src[4] = st.status;
      }
    } else {
      src[0] = s->mp.n_att, src[1] = s->mp.n_acc, src[2] = s->mp.n_rej,
      src[3] = s->mp.n_fe, src[4] = s->mp.status;
    }
    int32_t* dst[5] = {n_attempted, n_accepted, n_rejected, n_feval, status};
    for (int k = 0; k < 5; ++k)
      if (dst[k])
        HIP_TRY(hipMemcpyAsync(dst[k], src[k], sizeof(int32_t) * s->cfg.B,
                               hipMemcpyDeviceToDevice, s->stream));
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_get_stats");
  }
}

int solver_get_steps(const bode_solver* cs, double* h, int32_t* n) {
  bode_solver* s = const_cast<bode_solver*>(cs);
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (s->cfg.record_cap < 1)
      return fail(s, BODE_ESTATE, "steps are recorded only if record_cap > 0");
    const double* src_h;
    const int32_t* src_n;
    if (s->cfg.rhs == BODE_RHS_ANALYTIC) {
      src_h = is64(s->cfg) ? s->ad.h_rec : s->af.h_rec;
      src_n = is64(s->cfg) ? s->ad.st.n_att : s->af.st.n_att;
    } else {
      src_h = s->mp.h_rec;
      src_n = s->mp.n_att;
    }
    if (h)
      HIP_TRY(hipMemcpyAsync(h, src_h,
                             sizeof(double) * s->cfg.B * s->cfg.record_cap,
                             hipMemcpyDeviceToDevice, s->stream));
    if (n)
      HIP_TRY(hipMemcpyAsync(n, src_n, sizeof(int32_t) * s->cfg.B,
                             hipMemcpyDeviceToDevice, s->stream));
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_get_steps");
  }
}

int solver_get_errors(const bode_solver* cs, double* err) {
  bode_solver* s = const_cast<bode_solver*>(cs);
  try {
    if (!s) return fail(nullptr, BODE_EINVAL, "solver is NULL");
    if (!err) return fail(s, BODE_EINVAL, "err is NULL");
    if (s->cfg.record_cap < 1)
      return fail(s, BODE_ESTATE,
                  "error norms are recorded only if record_cap > 0");
    const double* src =
        s->cfg.rhs != BODE_RHS_ANALYTIC ? s->mp.e_rec
                                        : (is64(s->cfg) ? s->ad.e_rec
                                                        : s->af.e_rec);
    HIP_TRY(hipMemcpyAsync(err, src,
                           sizeof(double) * s->cfg.B * s->cfg.record_cap,
                           hipMemcpyDeviceToDevice, s->stream));
    return BODE_OK;
  } catch (...) {
    return fail(s, BODE_EHIP, "unknown error in solver_get_errors");
  }
}

void solver_destroy(bode_solver* s) {
  if (!s) return;
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  bode::modular_release(s->mp);
  delete s;
}

const char* solver_last_error(const bode_solver* s) {
  return s ? s->err.c_str() : g_thread_error.c_str();
}

int solver_tableau(int32_t method, double* c, double* a, double* b, double* e,
                   double* dense) {
  auto put = [&](auto M) {
    using T = decltype(M);
    for (int i = 0; i < 7; ++i) {
      if (c) c[i] = T::C[i];
      if (b) b[i] = T::A[6][i];
      if (e) e[i] = T::E[i];
      for (int j = 0; j < 7; ++j)
        if (a) a[i * 7 + j] = T::A[i][j];
      for (int m = 0; m < 4; ++m)
        if (dense) dense[i * 4 + m] = T::P[i][m];
    }
  };
  if (method == BODE_DOPRI5)
    put(bode::Dopri5{});
  else if (method == BODE_TSIT5)
    put(bode::Tsit5{});
  else
    return fail(nullptr, BODE_EINVAL, "unknown method");
  return BODE_OK;
}

int solver_autotune(const bode_config* cfg, const bode_problem* p,
                    void* workspace, size_t workspace_bytes_, void* stream) {
  return bode::autotune(cfg, p, workspace, workspace_bytes_, stream);
}

int solver_get_tune(const bode_config* cfg, int32_t* shape) {
  try {
    const std::string msg = check_config(cfg);
    if (!msg.empty()) return fail(nullptr, BODE_EINVAL, msg);
    if (!shape) return fail(nullptr, BODE_EINVAL, "shape is NULL");
    const Tune t = bode::get_tune(*cfg);
    shape[0] = t.block;
    shape[1] = t.lanes_vdp;
    shape[2] = t.lanes_lin;
    shape[3] = t.waves;
    shape[4] = t.rounds;
    return BODE_OK;
  } catch (...) {
    return fail(nullptr, BODE_EHIP, "unknown error in solver_get_tune");
  }
}

}  // extern "C"

namespace bode {

void set_tune(const bode_config& c, const Tune& t) {
  const TuneKey k = tune_key(c);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_cache();
  g_tune[k] = t;
  if (!save_tune_cache())
    std::fprintf(stderr, "batchode: cannot write the tune cache %s\n",
                 tune_cache_path());
}

void set_tune_candidate(const bode_config& c, const Tune& t) {
  const TuneKey k = tune_key(c);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_cache();
  g_tune[k] = t;
}

Tune get_tune(const bode_config& c) {
  const TuneKey k = tune_key(c);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_cache();
  auto it = g_tune.find(k);
  return it == g_tune.end() ? Tune() : it->second;
}

void set_thread_error(const std::string& m) { g_thread_error = m; }

}  // namespace bode
