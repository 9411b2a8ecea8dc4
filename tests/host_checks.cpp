// Host-side argument checks of the C ABI, for a build whose host code runs
// under AddressSanitizer and UndefinedBehaviorSanitizer (tests/
// test_sanitizers.py builds and runs it; no GPU is touched: every call here
// fails validation before any HIP call).  Prints each failed expectation and
// returns the number of failures.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "batchode.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}

static bode_config good() {
  bode_config c;
  std::memset(&c, 0, sizeof c);
  c.method = BODE_DOPRI5;
  c.precision = BODE_FP64;
  c.rhs = BODE_RHS_ANALYTIC;
  c.B = 64;
  c.D = 2;
  c.E = 8;
  c.max_steps = 1000;
  c.beta1 = 0.14;
  c.beta2 = 0.08;
  c.safety = 0.9;
  c.fac_min = 0.2;
  c.fac_max = 10.0;
  return c;
}

int main() {
  // workspace sizes: valid configurations > 0, each invalid field 0
  bode_config c = good();
  expect(solver_workspace_size(&c) > 0, "valid analytic size");
  c.record_cap = 4096;
  c.keep_dense = 1;
  expect(solver_workspace_size(&c) > 0, "record + keep size");
  expect(solver_workspace_size(nullptr) == 0, "null config size");
  struct Bad {
    const char* name;
    void (*set)(bode_config&);
  } bad[] = {
      {"B = 0", [](bode_config& x) { x.B = 0; }},
      {"D = 0", [](bode_config& x) { x.D = 0; }},
      {"D = 9 analytic", [](bode_config& x) { x.D = 9; }},
      {"E < 0", [](bode_config& x) { x.E = -1; }},
      {"method", [](bode_config& x) { x.method = 7; }},
      {"precision", [](bode_config& x) { x.precision = -1; }},
      {"rhs", [](bode_config& x) { x.rhs = 1; }},
      {"max_steps", [](bode_config& x) { x.max_steps = 0; }},
      {"fac_min", [](bode_config& x) { x.fac_min = 0.0; }},
      {"fac_max", [](bode_config& x) { x.fac_max = 0.5; }},
      {"safety", [](bode_config& x) { x.safety = -1.0; }},
      {"beta1 nan", [](bode_config& x) { x.beta1 = 0.0 / 0.0; }},
      {"beta3 inf", [](bode_config& x) { x.beta3 = 1.0 / 0.0; }},
      {"record_cap", [](bode_config& x) { x.record_cap = -2; }},
      {"ckpt without record", [](bode_config& x) { x.ckpt_every = 2; }},
      {"joint + keep_dense", [](bode_config& x) {
         x.joint = 1;
         x.keep_dense = 1;
       }},
      {"fixed + joint", [](bode_config& x) {
         x.fixed_step = 1;
         x.joint = 1;
       }},
      {"eager", [](bode_config& x) { x.eager = 2; }},
      {"plain_bf16", [](bode_config& x) { x.plain_bf16 = 3; }},
      {"neural without width", [](bode_config& x) {
         x.rhs = BODE_RHS_MLP;
         x.mlp_hidden = 0;
       }},
      {"cnf D = 1", [](bode_config& x) {
         x.rhs = BODE_RHS_CNF;
         x.D = 1;
         x.mlp_hidden = 64;
       }},
      {"huge", [](bode_config& x) {
         x.B = 1 << 30;
         x.D = 8;
         x.E = 1 << 20;
       }},
  };
  for (auto& b : bad) {
    bode_config x = good();
    b.set(x);
    expect(solver_workspace_size(&x) == 0, b.name);
    bode_solver* h = reinterpret_cast<bode_solver*>(1);
    bode_problem p;
    std::memset(&p, 0, sizeof p);
    expect(solver_init(&x, &p, reinterpret_cast<void*>(256), 1 << 20, nullptr,
                       &h) == BODE_EINVAL && h == nullptr,
           b.name);
    expect(std::strlen(solver_last_error(nullptr)) > 0, "error text");
  }

  // solver_init: problems and workspaces refused before any device work
  bode_problem p;
  std::memset(&p, 0, sizeof p);
  bode_solver* h = nullptr;
  void* ws = reinterpret_cast<void*>(256);
  expect(solver_init(&c, &p, ws, 1 << 20, nullptr, nullptr) == BODE_EINVAL,
         "null out");
  expect(solver_init(nullptr, &p, ws, 1 << 20, nullptr, &h) == BODE_EINVAL,
         "null config");
  expect(solver_init(&c, nullptr, ws, 1 << 20, nullptr, &h) == BODE_EINVAL,
         "null problem");
  expect(solver_init(&c, &p, ws, 1 << 20, nullptr, &h) == BODE_EINVAL,
         "missing inputs");
  const void* fake = reinterpret_cast<const void*>(256);
  p.y0 = fake;
  p.t0 = p.t_end = p.rtol = p.atol = p.t_eval =
      reinterpret_cast<const double*>(256);
  p.kind = p.dim = reinterpret_cast<const int32_t*>(256);
  p.y_eval = p.y_final = reinterpret_cast<void*>(256);
  expect(solver_init(&c, &p, ws, 16, nullptr, &h) == BODE_EINVAL,
         "workspace too small");
  expect(solver_init(&c, &p, reinterpret_cast<void*>(260), 1 << 20, nullptr,
                     &h) == BODE_EINVAL,
         "misaligned workspace");
  expect(solver_init(&c, &p, nullptr, 1 << 20, nullptr, &h) == BODE_EINVAL,
         "null workspace");
  bode_config f = good();
  f.fixed_step = 1;
  expect(solver_init(&f, &p, ws, 1 << 20, nullptr, &h) == BODE_EINVAL,
         "fixed step without h0");
  bode_config m = good();
  m.rhs = BODE_RHS_MLP;
  m.precision = BODE_BF16;
  m.D = 24;
  m.mlp_hidden = 64;
  p.W1 = p.b1 = p.W2 = p.b2 = p.W3 = p.b3 = fake;
  expect(solver_init(&m, &p, ws, (size_t)1 << 40, nullptr, &h) ==
             BODE_EUNSUPPORTED,
         "BF16 width 24 unsupported");

  // the no-allocation entry point refuses what its array cannot hold
  bode_config big = good();
  big.B = 1 << 20;
  big.D = 8;
  big.E = 16;
  expect(solver_solve_noalloc(&big, &p, nullptr, nullptr) == BODE_EINVAL,
         "noalloc too large");
  expect(solver_solve_noalloc(&m, &p, nullptr, nullptr) == BODE_EUNSUPPORTED,
         "noalloc neural");
  expect(solver_solve_noalloc(nullptr, &p, nullptr, nullptr) == BODE_EINVAL,
         "noalloc null config");

  // calls on a null handle
  expect(solver_step(nullptr, 1, nullptr) == BODE_EINVAL, "step null");
  expect(solver_solve(nullptr) == BODE_EINVAL, "solve null");
  expect(solver_eval(nullptr, nullptr, nullptr, nullptr) == BODE_EINVAL,
         "eval null");
  expect(solver_backward(nullptr, nullptr, nullptr, nullptr, nullptr) ==
             BODE_EINVAL,
         "backward null");
  expect(solver_cadjoint(nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr,
                         nullptr, nullptr) == BODE_EINVAL,
         "cadjoint null");
  expect(solver_cadjoint_workspace_bytes(nullptr, 0) == 0, "cadjoint bytes");
  expect(solver_get_stats(nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr) == BODE_EINVAL,
         "stats null");
  expect(solver_get_steps(nullptr, nullptr, nullptr) == BODE_EINVAL,
         "steps null");
  expect(solver_get_errors(nullptr, nullptr) == BODE_EINVAL, "errors null");
  solver_destroy(nullptr);

  // tableaux
  double cc[7], a[49], b[7], e[7], d[28];
  for (int meth = 0; meth < 2; ++meth) {
    expect(solver_tableau(meth, cc, a, b, e, d) == BODE_OK, "tableau");
    double sb = 0, se = 0;
    for (int j = 0; j < 7; ++j) {
      sb += b[j];
      se += e[j];
    }
    expect(sb > 1 - 1e-14 && sb < 1 + 1e-14, "sum b = 1");
    expect(se > -1e-14 && se < 1e-14, "sum e = 0");
  }
  expect(solver_tableau(5, cc, a, b, e, d) == BODE_EINVAL, "bad method");
  std::printf("host checks: %d failures\n", failures);
  return failures;
}
