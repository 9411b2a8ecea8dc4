#!/usr/bin/env python3
"""Benchmark of the batched adaptive Runge-Kutta hot path on one MI355X.

A step is one whole solve of the uneven batch: 65,536 independent instances,
half Van der Pol (mu log-uniform on [0.1, 20]) and half linear y' = A y in 8
dimensions, t_end ~ U[1, 50], 16 dense-output times each, rtol 1e-6,
atol 1e-8, PI controller: solver_init (first stage, starting step, queue) and
solver_solve (the persistent per-lane kernels) through the C ABI, inputs
resident in HBM.  The metric is accepted instance-steps per second.

The headline runs FP32 (state, norm and controller in float; time in
double) with Dormand-Prince; FP64 and Tsit5 variants are reported beside it,
each with its error at the stated tolerance against a tight FP64 solve.

Prints one JSON line.  --gpus above 1 is refused: the solver runs on one
GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="dopri5")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--variants", default="all",
                    help="'all' or 'headline' (skip the side variants)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time the library's default launch shapes instead "
                         "of the autotuned ones")
    ap.add_argument("--no-neural", action="store_true",
                    help="skip the neural-field workloads")
    ap.add_argument("--study", default="",
                    choices=["", "cadjoint", "neural", "ceilings", "hbm",
                             "paper", "fwdbwd", "fig1", "sweep",
                             "accuracy"],
                    help="only run one side study and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), "
                         "the reference kernel for HBM byte counters")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4,
                      "copy_calibration_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def ensure_built():
    from paper_2210_12375_amd import binding
    from paper_2210_12375_amd import build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    elif not os.path.exists(build.CEIL_LIB):
        build.build_ceilings()


def timed_solves(bd, dp, method, precision, steps, warmup, autotune=False,
                 **cfg_kw):
    """Runs warmup + steps whole solves; returns per-solve ms (init + solve),
    per-solve ms of solver_solve alone (HIP events on the solver's stream),
    and the statistics of the last solve."""
    import torch
    s = bd.Solver(dp, method=method, precision=precision, **cfg_kw)
    if autotune:
        bd.solver_autotune(s.cfg, s.prob, s.workspace.data_ptr(),
                           s.workspace.numel(), s.stream.cuda_stream)
        torch.cuda.synchronize()
    s.close()
    cfg, prob = s.cfg, s.prob
    shape = bd.solver_get_tune(cfg)
    ws_ptr, ws_bytes = s.workspace.data_ptr(), s.workspace.numel()
    stream = torch.cuda.current_stream()
    L = bd.lib()
    import ctypes as C
    evs = [(torch.cuda.Event(enable_timing=True),
            torch.cuda.Event(enable_timing=True)) for _ in range(steps)]

    def one(ev=None):
        h = C.c_void_p()
        rc = L.solver_init(C.byref(cfg), C.byref(prob), ws_ptr, ws_bytes,
                           stream.cuda_stream, C.byref(h))
        if rc != 0:
            raise bd.BodeError(rc, bd.solver_last_error())
        if ev is not None:
            ev[0].record(stream)
        rc = L.solver_solve(h)
        if ev is not None:
            ev[1].record(stream)
        if rc != 0:
            raise bd.BodeError(rc, bd.solver_last_error(h))
        L.solver_destroy(h)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        one(evs[k])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    solve_ms = [a.elapsed_time(b) for a, b in evs]
    # statistics of the (deterministic) solve
    s = bd.Solver(dp, method=method, precision=precision, **cfg_kw).solve()
    st = {k: v.cpu().numpy() for k, v in s.stats().items()}
    y_eval = s.y_eval.double().cpu().numpy()
    y_final = s.y_final.double().cpu().numpy()
    s.close()
    return wall, solve_ms, st, y_eval, y_final, shape


def error_at_tolerance(p, y_eval, y_final, ref, idx):
    """Global error over a sample against a tight FP64 solve, in units of
    the requested tolerance: max |y - ref| / (rtol |ref| + atol) over every
    output component (median and maximum over instances)."""
    a = np.concatenate([y_eval[idx].reshape(len(idx), -1),
                        y_final[idx].reshape(len(idx), -1)], axis=1)
    b = np.concatenate([ref[0].reshape(len(idx), -1),
                        ref[1].reshape(len(idx), -1)], axis=1)
    tol = p["rtol"][idx][:, None] * np.abs(b) + p["atol"][idx][:, None]
    e = (np.abs(a - b) / tol).max(axis=1)
    return float(np.median(e)), float(e.max())


PROFILE = os.path.join(ROOT, "profiles",
                       "analytic_persistent_uneven65536_fp32.md")
KERNEL_SOURCES = ["analytic.hip", "common.hpp", "tableau.hpp", "analytic.hpp"]


def measured_traffic():
    """HBM bytes per launch of the persistent solve from the committed
    rocprofv3 counter summary, or None if the kernel sources changed since
    the counters were taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines()
                  if ": " in l and l.split(": ", 1)[0].isidentifier())
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2210_12375_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256_16") != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_launch_pair"])


def ceilings():
    """Achievable ceilings beside the datasheet peaks: a streaming triad and
    a plain device copy for HBM, register-resident MFMA loops (BF16 16x16x32,
    FP32 16x16x4) and an FP32 FMA loop without packed instructions."""
    import ctypes as C
    import torch
    try:
        lib = C.CDLL(os.path.join(ROOT, "paper_2210_12375_amd",
                                  "libceilings.so"))
    except OSError as e:  # measurement only: the run goes on without it
        print(f"# ceilings skipped: {e}", file=sys.stderr, flush=True)
        return None
    vp = C.c_void_p
    lib.ceil_triad.argtypes = [vp, vp, vp, C.c_long, C.c_float, vp]
    for f in (lib.ceil_mfma_bf16, lib.ceil_mfma_f32, lib.ceil_fma_f32):
        f.argtypes = [vp, C.c_int, C.c_int, vp]
    st = torch.cuda.current_stream()

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(st)
            fn()
            b.record(st)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3

    def ok(rc):
        if rc != 0:
            raise RuntimeError(f"ceilings kernel failed: {rc}")

    n = 256 << 20  # 1 GiB per vector: far beyond every cache
    a = torch.ones(n, device="cuda")
    b = torch.ones(n, device="cuda")
    c = torch.empty(n, device="cuda")
    t_triad = timed(lambda: ok(lib.ceil_triad(a.data_ptr(), b.data_ptr(),
                                              c.data_ptr(), n, 0.5,
                                              st.cuda_stream)))
    # the streaming kernel's shape: vectors in flight per lane x grid
    lib.ceil_triad_shape.argtypes = [vp, vp, vp, C.c_long, C.c_float, C.c_int,
                                     C.c_int, vp]
    sweep = {}
    for unroll in (1, 2, 4, 8):
        for blocks in (1024, 4096, 8192, 32768):
            t = timed(lambda: ok(lib.ceil_triad_shape(
                a.data_ptr(), b.data_ptr(), c.data_ptr(), n, 0.5, unroll,
                blocks, st.cuda_stream)), 5)
            sweep[f"u{unroll}_b{blocks}"] = round(12 * n / t / 1e9, 1)
    t_triad = min(t_triad, 12 * n / max(sweep.values()) / 1e9)
    t_copy = timed(lambda: c.copy_(a))
    del a, b, c
    blocks, iters = 2048, 20000
    out = torch.empty(blocks * 256, device="cuda")
    res = {}
    for name, fn, fl in (
            ("mfma_bf16_tflops", lib.ceil_mfma_bf16, 16 * 16 * 32 * 2),
            ("mfma_f32_tflops", lib.ceil_mfma_f32, 16 * 16 * 4 * 2)):
        t = timed(lambda: ok(fn(out.data_ptr(), blocks, iters,
                                st.cuda_stream)), 5)
        res[name] = blocks * 4 * iters * 8 * fl / t / 1e12
    t = timed(lambda: ok(lib.ceil_fma_f32(out.data_ptr(), blocks, iters,
                                          st.cuda_stream)), 5)
    res["vector_fp32_fma_tflops"] = blocks * 256 * 16 * iters * 2 / t / 1e12
    res.update(hbm_triad_gbps=12 * n / t_triad / 1e9,
               hbm_triad_sweep_gbps=sweep,
               hbm_copy_gbps=8 * n / t_copy / 1e9,
               datasheet={"hbm_gbps": 8000, "mfma_bf16_tflops": 2500,
                          "mfma_f32_tflops": 157.3,
                          "vector_fp32_tflops_packed": 157.3,
                          "vector_fp64_tflops": 78.6})
    print("# ceilings: " + json.dumps({k: (round(v, 1)
                                          if isinstance(v, float) else v)
                                      for k, v in res.items()}),
          file=sys.stderr, flush=True)
    return res


def hbm_study(bd, W):
    """The scan-like commit kernel (error norm, controller, commit) out of
    cache: an MLP field with D = 64 state features on 2^20 instances in FP32
    on the per-stage path (hidden width 48 runs on the FMA field kernels),
    so every commit launch streams 10 D floats per instance (the six
    non-zero error stages, y and the candidate read; y and the FSAL stage
    written): 2.7 GB per launch.  Its duration comes from the kernel trace
    of this study."""
    import torch
    B = 1 << 20
    p = W.neural_ode(B=B, d=64, hidden=48)
    dp = bd.device_problem(p, "fp32")
    s = bd.Solver(dp, method="dopri5", precision="fp32", rhs=bd.RHS_MLP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    st = {k: v.cpu().numpy() for k, v in s.stats().items()}
    s.close()
    att = st["n_attempted"]
    return {"instances": B, "D": 64, "hidden": 48,
            "attempts_min": int(att.min()), "attempts_max": int(att.max()),
            "commit_bytes_per_launch_all_rows": 10 * 64 * 4 * B,
            "solve_ms": ms, "all_success": bool(np.all(st["status"] == 1))}


def cpu_baseline(p, method, seconds):
    """The FP64 oracle on the host cores over whole copies of a bounded
    sample of the same batch."""
    import oracle
    nt = os.cpu_count() or 1
    try:
        nt = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    from paper_2210_12375_amd import workloads as W
    n = 8192
    q = W.subset(p, np.arange(n))
    t0 = time.perf_counter()
    r = oracle.solve(q, method=method, n_threads=nt)
    dt = time.perf_counter() - t0
    reps = max(1, int(seconds / max(dt, 1e-3)))
    acc = int(r["n_accepted"].sum())
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.solve(q, method=method, n_threads=nt)
    dt = (time.perf_counter() - t0) / reps
    return {"value": acc / dt, "unit": "accepted instance-steps/s",
            "cores": nt, "kind": "oracle",
            "sample": f"first {n} of the 65,536 instances (FP64 oracle, "
                      f"{method}, PI), {reps} repetitions, "
                      f"{dt * 1e3:.1f} ms per pass"}


def cpu_configs(method="dopri5"):
    """The FP64 oracle on the host at one thread and at all threads on each
    workload's sample (the parity batch in full, the first 8192 uneven
    instances, the first 256 / 64 / 64 neural instances): accepted
    instance-steps/s for forward solves, instances/s for forward + discrete
    adjoint.  Context for the GPU figures, not a target."""
    import oracle
    from paper_2210_12375_amd import workloads as W
    nt = os.cpu_count() or 1
    try:
        nt = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    P = ("W1", "b1", "W2", "b2", "W3", "b3")

    def fwd(q, threads):
        t0 = time.perf_counter()
        r = oracle.solve(q, method=method, n_threads=threads)
        return int(r["n_accepted"].sum()) / (time.perf_counter() - t0)

    def fwdbwd(q, threads):
        t0 = time.perf_counter()
        r = oracle.solve(q, method=method, n_threads=threads, record_cap=512)
        h, n = oracle.accepted_steps(r["h_rec"], r["n_attempted"])
        B, D = q["y0"].shape
        E = q["t_eval"].shape[1]
        g_eval = np.ones((B, E, D)) if E else None
        oracle.adjoint(q, h, n, g_eval, np.ones((B, D)), method=method,
                       n_threads=threads)
        return B / (time.perf_counter() - t0)

    out = {"threads": nt}
    work = (("vdp_64_fp64", W.vdp_batch(), fwd, "accepted instance-steps/s"),
            ("uneven_first8192", W.subset(W.uneven_batch(), np.arange(8192)),
             fwd, "accepted instance-steps/s"),
            ("neural_fwd_first256", W.subset(W.neural_ode(), np.arange(256)),
             fwd, "accepted instance-steps/s"),
            ("neural_fwdbwd_first64",
             W.subset(W.neural_ode_fit(), np.arange(64)), fwdbwd,
             "fwd+bwd instances/s"),
            ("cnf_fwdbwd_first64", W.subset(W.cnf_density(), np.arange(64)),
             fwdbwd, "fwd+bwd instances/s"))
    for name, q, fn, unit in work:
        out[name] = {"unit": unit, "one_thread": fn(q, 1),
                     "all_threads": fn(q, nt)}
    print("# cpu oracle per workload: " + json.dumps(out), file=sys.stderr,
          flush=True)
    return out


def neural_suite(bd, W, rl, steps, warmup, only=None):
    """The neural-field workloads: forward solves (accepted instance-steps/s)
    and forward + discrete-adjoint backward passes (fwd+bwd/s)."""
    import torch
    out = {}

    def run(p, rhs, precision, backward, nsteps, **extra):
        dp = bd.device_problem(p, precision)
        opts = dict(method="dopri5", precision=precision, rhs=rhs, **extra)
        if backward:
            opts.update(record_cap=256, ckpt_every=2)
        P = sum(np.asarray(p["mlp"][k]).size
                for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
        sd = torch.float64 if precision == "fp64" else torch.float32
        g_final = torch.ones(p["y0"].shape, dtype=sd, device="cuda")
        E = p["t_eval"].shape[1]
        g_eval = (torch.ones((p["y0"].shape[0], E, p["y0"].shape[1]),
                             dtype=sd, device="cuda") if E else None)
        times = []
        st = None
        for k in range(warmup + nsteps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = bd.Solver(dp, **opts).solve()
            if backward:
                s.backward(g_eval, g_final, P)
            torch.cuda.synchronize()
            if k >= warmup:
                times.append(time.perf_counter() - t0)
            if k == warmup + nsteps - 1:
                st = {kk: v.cpu().numpy() for kk, v in s.stats().items()}
            s.close()
        ms = float(np.median(times)) * 1e3
        acc = int(st["n_accepted"].sum())
        rounds = int(st["n_attempted"].max())
        d = p["y0"].shape[1] - (1 if rhs == bd.RHS_CNF else 0)
        H = p["mlp"]["W1"].shape[1]
        evals = (2 + 6 * rounds) * p["y0"].shape[0]  # rows the kernels touch
        row = rl.mlp_flops_per_row(d, H) * (2 if rhs == bd.RHS_CNF else 1)
        fl = evals * row
        if backward:
            # per accepted step and stage: the vector-Jacobian product and
            # the parameter-gradient outer products, each one field's worth
            # of multiply-adds (the recomputation of checkpointed stages is
            # not counted)
            fl += acc * 7 * 2 * row
        na = st["n_accepted"]
        r = dict(ms=ms, accepted=acc, steps_mean=float(na.mean()),
                 steps_p50=float(np.median(na)),
                 steps_p90=float(np.quantile(na, 0.9)), steps_max=int(na.max()),
                 steps_hist={int(k): int(v) for k, v in
                             zip(*np.unique(na, return_counts=True))},
                 rounds=rounds, ok=bool(np.all(st["status"] == 1)),
                 model_tflops=fl / (ms * 1e-3) / 1e12)
        if backward:
            r["fwd_bwd_per_s"] = 1e3 / ms
        else:
            r["instance_steps_per_s"] = acc / (ms * 1e-3)
        return r

    if only == "fwdbwd":  # the 1024-instance MLP fwd+bwd workload alone
        out["neural_fwdbwd_1024_bf16"] = run(W.neural_ode_fit(), bd.RHS_MLP,
                                             "bf16", True, steps)
        return out
    p3 = W.neural_ode()
    out["neural_fwd_4096_bf16"] = run(p3, bd.RHS_MLP, "bf16", False, steps)
    out["neural_fwd_4096_bf16_plain"] = run(p3, bd.RHS_MLP, "bf16", False,
                                            steps, plain_bf16=1)
    out["neural_fwd_4096_fp64"] = run(p3, bd.RHS_MLP, "fp64", False,
                                      max(1, steps // 2))
    p4 = W.neural_ode_fit()
    out["neural_fwdbwd_1024_bf16"] = run(p4, bd.RHS_MLP, "bf16", True, steps)
    out["neural_fwdbwd_1024_fp32"] = run(p4, bd.RHS_MLP, "fp32", True, steps)
    p5 = W.cnf_density()
    out["cnf_fwdbwd_8192_bf16"] = run(p5, bd.RHS_CNF, "bf16", True,
                                      max(1, steps // 2))
    for k, v in out.items():
        print(f"# {k}: {v['ms']:.2f} ms, {v['steps_mean']:.2f} steps, "
              f"{v['model_tflops']:.1f} model TFLOP/s", file=sys.stderr,
              flush=True)
    return out


def vdp64_rate(bd, W):
    """The 64-instance Van der Pol batch (FP64 Dormand-Prince, rtol 1e-6,
    atol 1e-8, 8 evaluation times): accepted instance-steps/s of whole
    solves (init + solve), median of 20 after 3 warm-ups."""
    p = W.vdp_batch()
    dp = bd.device_problem(p, "fp64")
    wall, solve_ms, st, _, _, _ = timed_solves(bd, dp, "dopri5", "fp64", 20,
                                               3)
    acc = int(st["n_accepted"].sum())
    return {"instances": int(p["y0"].shape[0]), "ms_per_solve": wall,
            "solve_kernel_ms": float(np.median(solve_ms)), "accepted": acc,
            "instance_steps_per_s": acc / (wall * 1e-3),
            "steps_p50": float(np.median(st["n_accepted"])),
            "steps_max": int(st["n_accepted"].max()),
            "ok": bool(np.all(st["status"] == 1))}


def neural_accuracy(bd, W, n=256):
    """The neural forward workload's error at its stated tolerance (rtol
    1e-5, atol 1e-6) on its first n instances, per precision: max over the
    final state's components of |y - ref| / (rtol |ref| + atol) against the
    FP64 field solved at rtol 1e-11, atol 1e-13 (median and maximum over
    instances).  The BF16 modes are also held against the FP64 solve of
    their own model, whose weight matrices are rounded to BF16: the first
    figure is then the model's rounding, the second the solver's error."""
    p = W.subset(W.neural_ode(), np.arange(n))

    def reference(weights_bf16):
        q = W.subset(p, np.arange(n))
        q["rtol"][:] = 1e-11
        q["atol"][:] = 1e-13
        if weights_bf16:  # the BF16 modes' model: W1 (state rows), W2, W3
            q["mlp"] = dict(q["mlp"])  # rounded to the nearest BF16 value
            for k in ("W1", "W2", "W3"):
                w = np.array(q["mlp"][k], dtype=np.float32)
                keep = w[-1:].copy() if k == "W1" else None  # time row
                u = w.view(np.uint32).astype(np.uint64)
                u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(
                    np.uint32)
                w = u.view(np.float32)
                if keep is not None:
                    w[-1:] = keep
                q["mlp"][k] = w
        s = bd.Solver(bd.device_problem(q, "fp64"), method="dopri5",
                      precision="fp64", rhs=bd.RHS_MLP).solve()
        r = s.y_final.cpu().numpy()
        s.close()
        return r
    refs = {False: reference(False), True: reference(True)}
    out = {}
    for name, prec, kw in (("fp64", "fp64", {}), ("fp32", "fp32", {}),
                           ("bf16", "bf16", {}),
                           ("bf16_plain", "bf16", {"plain_bf16": 1})):
        s = bd.Solver(bd.device_problem(p, prec), method="dopri5",
                      precision=prec, rhs=bd.RHS_MLP, **kw).solve()
        y = s.y_final.cpu().numpy().astype(np.float64)
        na = s.stats()["n_accepted"].cpu().numpy()
        s.close()
        r = {"accepted_steps_p50": float(np.median(na))}
        for rounded, label in ((False, ""), (True, "_vs_bf16_weights")):
            if rounded and prec != "bf16":
                continue
            ref = refs[rounded]
            tol = p["rtol"][:, None] * np.abs(ref) + p["atol"][:, None]
            e = (np.abs(y - ref) / tol).max(axis=1)
            r["err_in_tol_units_median" + label] = float(np.median(e))
            r["err_in_tol_units_max" + label] = float(e.max())
        out[name] = r
    return out


def cadjoint_study(bd, W, reps=2):
    """Appendix A's adjoint-equation backward: the continuous adjoint solved
    per instance (b (f + p) variables) and jointly (b f + p), beside the
    discrete adjoint of the same forward solve.  Backward time, steps and
    time per step; the gradients of the three agree to O(tol)."""
    import torch
    out = {}
    for name, p, rhs, prec in (
            ("cnf_8192_bf16", W.cnf_density(), bd.RHS_CNF, "bf16"),
            ("mlp_1024_fp32", W.neural_ode_fit(), bd.RHS_MLP, "fp32")):
        dp = bd.device_problem(p, prec)
        P = sum(np.asarray(p["mlp"][k]).size
                for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
        s = bd.Solver(dp, method="dopri5", precision=prec, rhs=rhs,
                      record_cap=256, ckpt_every=2).solve()
        B, D = p["y0"].shape
        E = p["t_eval"].shape[1]
        g_final = torch.ones((B, D), dtype=torch.float32, device="cuda")
        g_eval = (torch.ones((B, E, D), dtype=torch.float32, device="cuda")
                  if E else None)
        r = {"instances": B, "params": P}
        grads = {}
        for mode in ("discrete", "per_instance", "joint"):
            times = []
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "discrete":
                    dy0, dth = s.backward(g_eval, g_final, P)
                    st = None
                else:
                    dy0, dth, st = s.cadjoint(g_eval, g_final, P,
                                              joint=mode == "joint")
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            ms = float(np.median(times[1:])) * 1e3
            grads[mode] = dth.double().cpu().numpy()
            m = {"ms": round(ms, 3)}
            if st is not None:
                att = st[0].cpu().numpy()
                ok = st[4].cpu().numpy() == 1
                m["steps"] = int(att.max())
                m["ms_per_step"] = round(ms / max(1, int(att.max())), 3)
                m["all_success"] = bool(ok.all())
            r[mode] = m
        ref = grads["discrete"]
        for mode in ("per_instance", "joint"):
            r[mode]["rel_diff_vs_discrete"] = float(
                np.linalg.norm(grads[mode] - ref) / np.linalg.norm(ref))
        s.close()
        out[name] = r
        print(f"# continuous adjoint {name}: " + json.dumps(r),
              file=sys.stderr, flush=True)
    return out


def paper_loop_study(bd, W, steps=50, warmup=5):
    """Appendix A's Van der Pol benchmark on this solver: 256 instances with
    mu = 2 over one cycle, atol = rtol = 1e-5, 200 evenly spaced evaluation
    times, Dormand-Prince with the integral controller.  The paper's loop
    time is the solver's time per step of the batch loop minus the model's
    time; here the model is fused into the step, so the figure is the whole
    solve (init + solve, host clock around synchronised solves) over the
    batch's loop steps, the largest attempted-step count of any instance.
    Independent and joint batching, FP32 and FP64."""
    p = W.paper_vdp()
    out = {"workload": "256 Van der Pol instances, mu = 2, one cycle "
                       "(t_end 7.6295), atol = rtol = 1e-5, 200 evaluation "
                       "times, dopri5, integral controller",
           "paper_ms_per_step_gtx1080ti": {"torchode": 3.21,
                                           "torchode_jit": 1.629,
                                           "torchdiffeq_joint": 3.58,
                                           "diffrax": 0.9014},
           "rows": []}
    for precision in ("fp32", "fp64"):
        dp = bd.device_problem(p, precision)
        for joint in (0, 1):
            wall, solve_ms, st, _, _, _ = timed_solves(
                bd, dp, "dopri5", precision, steps, warmup, joint=joint,
                **bd.I_CONTROLLER)
            loop = int(st["n_attempted"].max())
            ok = bool((st["status"] == bd.SUCCESS).all())
            out["rows"].append(dict(
                precision=precision, joint=joint, ok=ok, loop_steps=loop,
                accepted=int(st["n_accepted"].sum()),
                solve_ms=float(np.median(solve_ms)), wall_ms=wall,
                us_per_loop_step=1e3 * wall / loop,
                instance_steps_per_s=float(st["n_accepted"].sum()) /
                (wall * 1e-3)))
    print("# paper VdP loop time (us per loop step): " + ", ".join(
        f"{r['precision']}{'/joint' if r['joint'] else ''} "
        f"{r['us_per_loop_step']:.2f} ({r['loop_steps']} steps)"
        for r in out["rows"]), file=sys.stderr, flush=True)
    return out


def pid_study(bd, W):
    """Appendix C's controller study: accepted + rejected steps for one Van
    der Pol cycle per mu, integral controller against PI and PID laws on
    log err (Gustafsson's PI; Soderlind's H211PI and H312PID filters; a PID
    with gains 0.3, 0.4, 0.1), FP64 Dormand-Prince on the GPU."""
    import torch
    p = W.vdp_cycles()
    dp = bd.device_problem(p, "fp64")
    ctrls = {"I": bd.I_CONTROLLER, "PI": bd.PI_CONTROLLER,
             "H211PI": bd.pid_gains(1 / 3, -1 / 6, 0.0),
             "H312PID": bd.pid_gains(2 / 9, -2 / 9, 1 / 18),
             "PID_0.3_0.4_0.1": bd.pid_gains(0.3, 0.4, 0.1)}
    out = {"mu": [float(m) for m in p["mu"]], "steps": {},
           "workload": "one Van der Pol cycle per mu from (2, 0), "
                       "atol = rtol = 1e-6, FP64 dopri5"}
    for name, c in ctrls.items():
        s = bd.Solver(dp, method="dopri5", precision="fp64", **c).solve()
        st = {k: v.cpu().numpy() for k, v in s.stats().items()}
        s.close()
        out["steps"][name] = [int(v) for v in st["n_attempted"]]
    torch.cuda.synchronize()
    base = np.array(out["steps"]["I"], dtype=float)
    out["change_vs_I_pct"] = {
        k: [round(100.0 * (a / b - 1.0), 2) for a, b in zip(v, base)]
        for k, v in out["steps"].items() if k != "I"}
    print("# pid study (attempted steps per mu): " +
          json.dumps(out["steps"]), file=sys.stderr, flush=True)
    return out


def joint_study(bd, W):
    """Section 4.1: attempted steps of a joint (coupled) solve of B Van der
    Pol oscillators at different phases against the independent solve of
    the same batch (FP64 Dormand-Prince on the GPU)."""
    import torch
    rows = []
    for mu in (5.0, 10.0, 25.0, 50.0):
        for B in (4, 16, 64):
            p = W.vdp_phases(B=B, mu=mu)
            dp = bd.device_problem(p, "fp64")
            out = {}
            for joint in (0, 1):
                s = bd.Solver(dp, method="dopri5", precision="fp64",
                              joint=joint).solve()
                out[joint] = s.stats()["n_attempted"].cpu().numpy()
                s.close()
            torch.cuda.synchronize()
            rows.append(dict(mu=mu, B=B, joint=int(out[1][0]),
                             independent_mean=float(out[0].mean()),
                             independent_max=int(out[0].max()),
                             ratio=round(float(out[1][0] / out[0].mean()), 2)))
    print("# joint study (joint / independent attempted steps): " +
          ", ".join(f"mu={r['mu']:g} B={r['B']}: {r['ratio']}" for r in rows),
          file=sys.stderr, flush=True)
    return {"rows": rows, "workload": "B Van der Pol oscillators at uniformly "
            "drawn phases of one cycle, atol = rtol = 1e-6, FP64 dopri5"}


def batch_sweep(bd, W, rl, steps=3, warmup=1):
    """Matrix-core utilisation against batch size: the fused forward solve of
    the 65-256-256-64 MLP field (BF16, split activations) from 4,096 to
    65,536 instances and of the CNF field (17-512-512-16 with tangent rows)
    from 8,192 to 65,536, each timed whole (median of `steps`) with its
    model flops (6 evaluations per attempt round over every row)."""
    import torch
    out = {}
    for name, make, rhs, sizes in (
            ("mlp_bf16", W.neural_ode, bd.RHS_MLP, (4096, 16384, 65536)),
            ("cnf_bf16", W.cnf_density, bd.RHS_CNF, (8192, 32768, 65536))):
        rows = []
        for B in sizes:
            p = make(B=B)
            dp = bd.device_problem(p, "bf16")
            times, st = [], None
            for k in range(warmup + steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = bd.Solver(dp, method="dopri5", precision="bf16",
                              rhs=rhs).solve()
                torch.cuda.synchronize()
                if k >= warmup:
                    times.append(time.perf_counter() - t0)
                st = s.stats()
                s.close()
            ms = float(np.median(times)) * 1e3
            att = st["n_attempted"].cpu().numpy()
            d = p["y0"].shape[1] - (1 if rhs == bd.RHS_CNF else 0)
            H = p["mlp"]["W1"].shape[1]
            row = rl.mlp_flops_per_row(d, H) * (2 if rhs == bd.RHS_CNF else 1)
            fl = float((2 + 6 * att).sum()) * row
            rows.append(dict(B=B, ms=round(ms, 3), attempts_max=int(att.max()),
                             model_tflops=round(fl / (ms * 1e-3) / 1e12, 1)))
            print(f"# sweep {name} B={B}: {ms:.2f} ms, "
                  f"{rows[-1]['model_tflops']} model TFLOP/s", file=sys.stderr,
                  flush=True)
        out[name] = rows
    return out


def fig1_traces(bd, W, mu=25.0, B=16, grid=48):
    """Section 4.1, Figure 1: the step sizes of the joint (coupled) solve of
    B Van der Pol oscillators at different phases of one cycle, mu = 25,
    beside the step sizes each oscillator takes when solved independently
    (FP64 Dormand-Prince, atol = rtol = 1e-6): on a grid of times over the
    cycle, the joint step in force and the smallest, median and largest
    independent step in force."""
    import torch
    p = W.vdp_phases(B=B, mu=mu)
    dp = bd.device_problem(p, "fp64")
    rec = {}
    for joint in (0, 1):
        s = bd.Solver(dp, method="dopri5", precision="fp64", joint=joint,
                      record_cap=8192).solve()
        h, n = s.steps()
        rec[joint] = (h.cpu().numpy(), n.cpu().numpy())
        s.close()
    torch.cuda.synchronize()

    def accepted(h, n, i):
        a = h[i, :n[i]]
        a = a[a > 0]
        return np.concatenate([[p["t0"][i]], p["t0"][i] + np.cumsum(a)]), a

    tj, hj = accepted(*rec[1], 0)
    ind = [accepted(*rec[0], i) for i in range(B)]
    times = np.linspace(p["t0"][0], p["t_end"][0], grid, endpoint=False)
    rows = []
    for t in times:
        in_force = lambda tt, hh: float(hh[min(np.searchsorted(tt, t, "right")
                                             - 1, len(hh) - 1)])
        hi = [in_force(tt, hh) for tt, hh in ind]
        rows.append([round(float(t), 4), in_force(tj, hj), float(np.min(hi)),
                     float(np.median(hi)), float(np.max(hi))])
    return {"workload": f"{B} Van der Pol oscillators, mu = {mu}, uniformly "
                        "drawn phases of one cycle, atol = rtol = 1e-6, FP64 "
                        "dopri5",
            "joint_accepted_steps": int(len(hj)),
            "independent_accepted_steps": [int(len(hh)) for _, hh in ind],
            "columns": ["t", "h_joint", "h_independent_min",
                        "h_independent_median", "h_independent_max"],
            "rows": rows}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; "
                                   "--gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(3)
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    ensure_built()
    from paper_2210_12375_amd import binding as bd
    from paper_2210_12375_amd import roofline as rl
    from paper_2210_12375_amd import workloads as W
    if a.study == "cadjoint":
        print(json.dumps({"cadjoint_study": cadjoint_study(bd, W)}),
              flush=True)
        return
    if a.study == "paper":
        print(json.dumps({"paper_loop_study": paper_loop_study(bd, W)}),
              flush=True)
        return
    if a.study == "ceilings":
        print(json.dumps({"ceilings": ceilings()}), flush=True)
        return
    if a.study == "hbm":
        print(json.dumps({"hbm_study": hbm_study(bd, W)}), flush=True)
        return
    if a.study == "sweep":
        print(json.dumps({"batch_sweep": batch_sweep(bd, W, rl)}), flush=True)
        return
    if a.study == "fig1":
        print(json.dumps({"fig1_traces": fig1_traces(bd, W)}), flush=True)
        return
    if a.study == "accuracy":
        print(json.dumps({"vdp64_fp64": vdp64_rate(bd, W),
                          "neural_accuracy": neural_accuracy(bd, W)}),
              flush=True)
        return
    if a.study == "fwdbwd":
        print(json.dumps({"neural": neural_suite(bd, W, rl, a.steps, a.warmup,
                                                 only="fwdbwd")}), flush=True)
        return
    if a.study == "neural":
        print(json.dumps({"neural": neural_suite(bd, W, rl, 2, 1)}),
              flush=True)
        return

    p = W.uneven_batch()
    B = p["y0"].shape[0]
    variants = [(a.method, a.precision)]
    if a.variants == "all":
        for m in ("dopri5", "tsit5"):
            for pr in ("fp32", "fp64"):
                if (m, pr) not in variants:
                    variants.append((m, pr))
    # tight FP64 reference on a sample (GPU, parity-tested against the oracle)
    idx = np.random.default_rng(7).choice(B, 1024, replace=False)
    q = W.subset(p, idx)
    q["rtol"][:] = 1e-12
    q["atol"][:] = 1e-14
    sref = bd.Solver(bd.device_problem(q, "fp64"), method="dopri5",
                     precision="fp64").solve()
    ref = (sref.y_eval.cpu().numpy(), sref.y_final.cpu().numpy())
    sref.close()

    results = {}
    for (m, pr) in variants:
        dp = bd.device_problem(p, pr)
        wall, solve_ms, st, ye, yf, shape = timed_solves(
            bd, dp, m, pr, a.steps if (m, pr) == variants[0] else
            max(3, a.steps // 2), a.warmup, autotune=a.autotune)
        acc = int(st["n_accepted"].sum())
        att = int(st["n_attempted"].sum())
        emitted = np.full(B, p["t_eval"].shape[1])
        flops = rl.analytic_flops(m, p["kind"], p["dim"], st["n_attempted"],
                                  emitted)
        solve_avg = float(np.mean(solve_ms))
        crit = None
        if (m, pr) == variants[0]:
            # the critical path: the instance with the most attempts, alone
            top = int(np.argmax(st["n_attempted"]))
            dq = bd.device_problem(W.subset(p, [top]), pr)
            _, one_ms, _, _, _, _ = timed_solves(bd, dq, m, pr, 5, 2)
            crit = dict(instance=top, attempts=int(st["n_attempted"][top]),
                        alone_ms=float(np.median(one_ms)))
        results[(m, pr)] = dict(
            crit=crit, launch_shape=shape,
            ms_per_step=wall, solve_ms=solve_avg, accepted=acc,
            attempted=att, value=acc / (wall * 1e-3),
            flops=flops, ok=bool(np.all(st["status"] == 1)),
            steps_p50=int(np.median(st["n_accepted"])),
            steps_max=int(st["n_accepted"].max()),
            steps_hist=np.histogram(st["n_accepted"],
                                    bins=[0, 50, 100, 200, 400, 800, 1600,
                                          3200, 1 << 30])[0].tolist(),
            err_at_tol=error_at_tolerance(p, ye, yf, ref, idx))
        print(f"# {m} {pr}: {wall:.3f} ms/solve, solve kernel "
              f"{solve_avg:.3f} ms, {acc} accepted steps", file=sys.stderr,
              flush=True)

    head = results[variants[0]]
    peak = (rl.PEAK["fp64_vector_tflops"] if a.precision == "fp64"
            else rl.PEAK["fp32_vector_tflops"])
    achieved = head["flops"] / (head["solve_ms"] * 1e-3) / 1e12
    line = {
        "metric": "accepted instance-steps/sec",
        "value": head["value"],
        "unit": "instance-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": "uneven batch: 65,536 instances, half Van der "
                               "Pol (mu log-U[0.1,20], D=2), half linear "
                               "y'=Ay (D=8), t_end~U[1,50], 16 dense-output "
                               "times, rtol 1e-6 atol 1e-8, PI controller",
                   "method": variants[0][0], "precision": variants[0][1],
                   "instances": B, "parallelism": "1 GPU, instances over "
                                                  "lanes",
                   "launch_shape": dict(head["launch_shape"],
                                        source="autotuned" if a.autotune
                                        else "library default")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": (measured_traffic()
                                 if (a.method, a.precision) == ("dopri5", "fp32")
                                 else None),
                     "kernel": "persistent solve (Van der Pol + linear "
                               "kernels, concurrent)",
                     "critical_path_steps": head["steps_max"],
                     # the batch cannot finish before its longest instance:
                     # that instance solved alone is the latency floor
                     "critical_path": {
                         "longest_instance_attempts": head["crit"]["attempts"],
                         "longest_instance_alone_ms": head["crit"]["alone_ms"],
                         "batch_solve_ms": head["solve_ms"],
                         "frac": head["crit"]["alone_ms"] / head["solve_ms"]}},
        "accuracy": {f"{m}/{pr}": {"err_in_tol_units_median":
                                   r["err_at_tol"][0],
                                   "err_in_tol_units_max": r["err_at_tol"][1],
                                   "sample": 1024, "reference":
                                   "GPU FP64 dopri5 at rtol 1e-12"}
                     for (m, pr), r in results.items()},
        "variants": {f"{m}/{pr}": {k: r[k] for k in
                                   ("value", "ms_per_step", "solve_ms",
                                    "accepted", "attempted", "steps_p50",
                                    "steps_max", "steps_hist", "ok",
                                    "launch_shape")}
                     for (m, pr), r in results.items()},
    }
    line["vdp64_fp64"] = vdp64_rate(bd, W)
    if not a.no_neural:
        line["neural"] = neural_suite(bd, W, rl, max(2, a.steps // 4),
                                      min(a.warmup, 2))
        line["neural_accuracy"] = neural_accuracy(bd, W)
        line["cadjoint_study"] = cadjoint_study(bd, W)
    line["ceilings"] = ceilings()
    line["paper_loop_study"] = paper_loop_study(bd, W)
    line["pid_study"] = pid_study(bd, W)
    line["joint_study"] = joint_study(bd, W)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, a.method, a.cpu_seconds)
        line["cpu_oracle_per_workload"] = cpu_configs(a.method)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
