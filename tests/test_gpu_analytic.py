"""GPU parity of the analytic-field path (Van der Pol / linear batches)
against the FP64 oracle, through the C ABI.

FP64 mode: identical per-instance accepted / rejected / evaluation counts and
statuses, outputs within 1e-9 relative per instance.  FP32 mode: every decision
and step size of the GPU's attempt record follows from its recorded error
norms by the controller law, and the oracle's FP64 replay of the record agrees
within 1e-4 relative per instance.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import (TOL_FP32, as_float_inputs, assert_fp64_parity,
                         assert_linear_accuracy,
                         assert_uneven_parity, controller, norm_bias,
                         oracle_replay, per_instance_absdiff, per_instance_rel,
                         reduced_replay_check, replay_check, run_gpu)
from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W

pytestmark = pytest.mark.gpu

METHODS = ["dopri5", "tsit5"]


def flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("ctrl", ["PI", "I", "H312PID", "PID"])
def test_vdp64_fp64_parity(method, ctrl):
    flush(f"vdp64 fp64 {method} {ctrl}")
    p = W.vdp_batch()
    g, _ = run_gpu(p, method=method, **controller(ctrl))
    r = oracle.solve(p, method=method, **controller(ctrl))
    assert np.all(r["status"] == bd.SUCCESS)
    assert_fp64_parity(g, r)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("ctrl", ["PI", "I", "H211PI"])
def test_uneven_short_horizon_exact(method, ctrl):
    """The uneven batch over short horizons (t_end / 12.5), where every step
    is accuracy-limited: identical counts and statuses for every instance,
    outputs within 1e-9, and every decision and step-size proposal of the
    GPU's attempt record equal to the oracle's."""
    flush(f"uneven short fp64 {method} {ctrl}")
    p = W.uneven_batch(B=2000)
    p["t_end"] = p["t_end"] / 12.5
    p["t_eval"] = p["t_eval"] / 12.5
    c = controller(ctrl)
    g, _ = run_gpu(p, method=method, record_cap=2048, **c)
    r = oracle.solve(p, method=method, **c)
    assert np.all(r["status"] == bd.SUCCESS)
    assert_fp64_parity(g, r)
    replay_check(p, g, method, c)


@pytest.mark.parametrize("method", METHODS)
def test_uneven_fp64_parity_ragged(method):
    """Mixed Van der Pol (D=2 in an 8-wide row) and linear instances over the
    full horizons, some linear ones with a smaller true dimension; B not a
    multiple of 64."""
    flush(f"uneven fp64 {method}")
    p = W.uneven_batch(B=1500)
    lin = np.flatnonzero(p["kind"] == W.LINEAR)
    for j, i in enumerate(lin[:40]):
        d = 1 + j % 7
        p["dim"][i] = d
        p["A"][i, d:, :] = 0.0
        p["A"][i, :, d:] = 0.0
        p["y0"][i, d:] = 0.0
    g, _ = run_gpu(p, method=method, record_cap=4096)
    info = assert_uneven_parity(p, g, method)
    flush(f"  {info}")
    assert_linear_accuracy(p, g)


# Bound on the median relative deviation of the FP32 error norms from the
# FP64 oracle's on the same steps, over the attempts whose norm decides
# (0.1 <= err <= 10).  A unit norm at rtol = 1e-6 is an estimate
# h sum_j e_j k_j of about 1e-6 |y| formed from terms h e_j k_j of up to
# |e_j| |y| (sum_j e_j = 0 cancels them), each rounded to float, so the norm
# carries relative noise up to eps_f32 / rtol * sum_j |e_j| = 0.06 sum |e_j|
# (Dormand-Prince sum |e_j| = 0.16, Tsitouras 1.21); the bound is
# 0.1 sum_j |e_j|.  A wrong coefficient, scale or dimension shifts the
# median by O(1).  Checked
# on the Van der Pol attempts: the linear family's steps sit on the
# stability boundary, where its norm is rounding noise of the decayed stiff
# modes in either precision.
def norm_bias_bound(method):
    return 0.1 * np.abs(bd.solver_tableau(method)[3]).sum()


def check_uneven_fp32(p, g, method, ctrl=None):
    info = reduced_replay_check(p, g, method, "fp32", ctrl, phase=True)
    rel = info["rel"]
    b = norm_bias(info, p["kind"], W.VDP)
    assert b <= norm_bias_bound(method), b
    flush(f"  max rel {rel.max():.2e} (p99 {np.quantile(rel, 0.99):.2e}, "
          f"{info['n_phase']} outputs within the phase allowance), "
          f"proposals checked {info['n_ctl_checked']}, norm bias VdP "
          f"{norm_bias(info, p['kind'], W.VDP):.1e} linear "
          f"{norm_bias(info, p['kind'], W.LINEAR):.1e}")
    return info


@pytest.mark.parametrize("method", METHODS)
def test_uneven_fp32_replay_parity(method):
    """FP32 state, norm and controller (compensated summation of the state
    update): every decision and every proposed step size of the GPU's record
    follows from its recorded error norms by the controller law; the FP64
    oracle's replay of that record agrees within 1e-4 for every instance;
    the recorded norms agree with the oracle's without bias."""
    flush(f"uneven fp32 replay {method}")
    p = W.uneven_batch(B=1024)
    g, _ = run_gpu(p, method=method, precision="fp32", record_cap=4096)
    assert np.all(g["status"] == bd.SUCCESS)
    check_uneven_fp32(p, g, method)


@pytest.mark.parametrize("method", METHODS)
def test_headline_fp32_full_batch_sampled(method):
    """The benchmark's workload itself: all 65,536 instances of the uneven
    batch in FP32 with the step record, 2048 sampled instances checked
    attempt by attempt as above; the whole batch's outputs are bitwise those
    of the solve without the record (the benchmark's launch configuration)."""
    flush(f"uneven full 65536 fp32 {method}")
    p = W.uneven_batch()
    g, _ = run_gpu(p, method=method, precision="fp32", record_cap=2048)
    assert np.all(g["status"] == bd.SUCCESS)
    assert g["n_rec"].max() <= 2048
    plain, _ = run_gpu(p, method=method, precision="fp32")
    np.testing.assert_array_equal(plain["y_final"], g["y_final"])
    np.testing.assert_array_equal(plain["y_eval"], g["y_eval"])
    np.testing.assert_array_equal(plain["n_accepted"], g["n_accepted"])
    idx = np.random.default_rng(2048).choice(p["y0"].shape[0], 2048,
                                             replace=False)
    check_uneven_fp32(W.subset(p, idx), {k: v[idx] for k, v in g.items()},
                      method)


@pytest.mark.parametrize("method", METHODS)
def test_fp32_decisions_accuracy_limited(method):
    """Non-stiff Van der Pol (mu <= 2) and slowly decaying linear instances
    (rates <= 1) over short spans, where every step is accuracy-limited:
    every FP32 accept / reject decision equals the FP64 oracle's on the same
    step, except near-ties |err - 1| <= 2 eps_f32 / rtol * sum_j |e_j| (the
    float noise of the norm, see norm_bias_bound: 0.019 Dormand-Prince,
    0.145 Tsitouras at rtol 1e-6)."""
    flush(f"fp32 decisions, accuracy-limited {method}")
    p = W.uneven_batch(B=2000)
    p["mu"] = np.minimum(p["mu"], 2.0)
    p["A"] = p["A"] * 0.1
    p["t_end"] = p["t_end"] / 5.0
    p["t_eval"] = p["t_eval"] / 5.0
    g, _ = run_gpu(p, method=method, precision="fp32", record_cap=4096)
    assert np.all(g["status"] == bd.SUCCESS)
    band = 2.0 * np.finfo(np.float32).eps / 1e-6 * np.abs(
        bd.solver_tableau(method)[3]).sum()
    assert np.all(p["rtol"] == 1e-6)
    info = reduced_replay_check(p, g, method, "fp32", decision_band=band)
    flush(f"  max rel {info['rel'].max():.2e}, norm bias VdP "
          f"{norm_bias(info, p['kind'], W.VDP):.1e}")


@pytest.mark.parametrize("method", METHODS)
def test_full_uneven_batch_sampled(method):
    """The full 65,536-instance uneven batch in the benchmark's launch
    configuration; 384 sampled instances checked against the oracle."""
    flush(f"uneven full 65536 fp64 {method}")
    p = W.uneven_batch()
    g, _ = run_gpu(p, method=method, record_cap=2048)
    assert np.all(g["status"] == bd.SUCCESS)
    idx = np.random.default_rng(99).choice(p["y0"].shape[0], 384, replace=False)
    q = W.subset(p, idx)
    gs = {k: v[idx] for k, v in g.items()}
    info = assert_uneven_parity(q, gs, method)
    flush(f"  {info}")
    # whole-batch invariants hold at any size
    np.testing.assert_array_equal(g["n_attempted"],
                                  g["n_accepted"] + g["n_rejected"])
    np.testing.assert_array_equal(g["n_feval"], 2 + 6 * g["n_attempted"])
    assert np.isfinite(g["y_eval"]).all()


def test_step_calls_match_one_solve():
    """solver_step in slices of 7 attempts gives bitwise the same result as a
    single solver_solve, and reports the running count."""
    flush("step slices")
    p = W.uneven_batch(B=700)
    g, _ = run_gpu(p, method="tsit5")
    dp = bd.device_problem(p, "fp64")
    s = bd.Solver(dp, method="tsit5")
    running = []
    for _ in range(10000):
        n = s.step(7, want_running=True)
        running.append(n)
        if n == 0:
            break
    assert running[-1] == 0 and running[0] > 0
    assert all(a >= b for a, b in zip(running, running[1:]))
    np.testing.assert_array_equal(s.y_final.cpu().numpy(), g["y_final"])
    np.testing.assert_array_equal(s.y_eval.cpu().numpy(), g["y_eval"])
    st = s.stats()
    np.testing.assert_array_equal(st["n_accepted"].cpu().numpy(),
                                  g["n_accepted"])


def test_eval_last_step_dense_output():
    """solver_eval answers inside each instance's last accepted step with the
    same interpolant the oracle uses."""
    flush("solver_eval")
    p = W.vdp_batch(B=100)
    B = 100
    dp = bd.device_problem(p, "fp64")
    s = bd.Solver(dp, method="dopri5", keep_dense=1, record_cap=2048)
    s.step(20)
    h, n = s.steps()
    h = h.cpu().numpy()
    n = n.cpu().numpy()
    hacc, nacc = oracle.accepted_steps(h, n)
    t_prev = np.zeros(B)
    for i in range(B):  # sequential sums, as the kernel advances t
        t = p["t0"][i]
        for k in range(nacc[i] - 1):
            t = t + hacc[i, k]
        t_prev[i] = t
    t_cur = t_prev + hacc[np.arange(B), nacc - 1]
    tq = t_prev + 0.37 * (t_cur - t_prev)
    y, q = s.eval(torch.as_tensor(tq, device="cuda"))
    y = y.cpu().numpy()
    assert np.all(q.cpu().numpy() == 0)
    # oracle: replay the same steps with tq as the single evaluation time
    r = oracle.solve(dict(p, t_eval=tq[:, None]), method="dopri5",
                     h_replay=h[:, :n.max()], n_replay=n)
    err = np.abs(y - r["y_eval"][:, 0]).max(axis=1) / np.abs(r["y_eval"][:, 0]).max(axis=1)
    assert err.max() < 1e-9
    # outside the last step: flagged and NaN
    y2, q2 = s.eval(torch.as_tensor(t_prev - 1.0, device="cuda"))
    assert np.all(q2.cpu().numpy() == 1) and np.isnan(y2.cpu().numpy()).all()


def test_edge_cases():
    flush("edge cases")
    p = W.uneven_batch(B=130)
    p["t_end"][3] = p["t0"][3]
    p["t_eval"][3] = 0.0
    p["t_eval"][5, 0] = 0.0            # evaluation at t0
    p["t_eval"][6, -1] = p["t_end"][6]  # evaluation at t_end
    p["t_eval"][7, 4] = -1.0           # invalid: before t0 -> INVALID
    p["rtol"][8] = 0.0
    p["atol"][8] = 0.0                 # invalid tolerances
    p["y0"][9, 0] = np.nan             # invalid state
    g, _ = run_gpu(p, method="dopri5", record_cap=4096)
    r = oracle.solve(p, method="dopri5")
    np.testing.assert_array_equal(g["status"], r["status"])
    assert list(g["status"][[3, 7, 8, 9]]) == [1, 4, 4, 4]
    ok = r["status"] != bd.INVALID
    sub = {k: v[ok] for k, v in g.items()}
    assert_uneven_parity(W.subset(p, np.flatnonzero(ok)), sub, "dopri5")
    assert np.isnan(g["y_final"][7, :2]).all()
    # max_steps: every instance stops after 3 attempts
    g, _ = run_gpu(p, method="tsit5", max_steps=3, record_cap=8)
    r = oracle.solve(p, method="tsit5", max_steps=3)
    np.testing.assert_array_equal(g["status"], r["status"])
    running = r["status"] == bd.MAX_STEPS
    assert running.sum() > 100
    np.testing.assert_array_equal(g["n_attempted"][running], 3)
    np.testing.assert_array_equal(g["n_accepted"], r["n_accepted"])
    sub = {k: v[ok] for k, v in g.items()}
    replay_check(W.subset(p, np.flatnonzero(ok)), sub, "tsit5")


def test_single_instance_and_user_h0():
    flush("single instance, h0")
    p = W.subset(W.vdp_batch(), [5])
    p["h0"] = np.array([1e-3])
    g, _ = run_gpu(p, method="dopri5")
    r = oracle.solve(p, method="dopri5")
    assert_fp64_parity(g, r)
    assert g["n_feval"][0] == 1 + 6 * g["n_attempted"][0]


def autotune(p, precision, rhs=bd.RHS_ANALYTIC, **kw):
    dp = bd.device_problem(p, precision)
    s = bd.Solver(dp, method="dopri5", precision=precision, rhs=rhs, **kw)
    bd.solver_autotune(s.cfg, s.prob, s.workspace.data_ptr(),
                       s.workspace.numel(), s.stream.cuda_stream)
    torch.cuda.synchronize()
    shape = bd.solver_get_tune(s.cfg)
    s.close()
    return shape


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_keeps_results(precision):
    """The autotuner's shape (threads per workgroup, lanes) changes which
    lane solves which instance, never an instance's arithmetic: a solve
    with the tuned shape equals, bit for bit, solves with fixed shapes."""
    flush(f"autotune analytic {precision}")
    p = W.uneven_batch(B=4096)
    shape = autotune(p, precision)
    flush(f"  tuned {shape}")
    assert shape["block"] in (64, 128, 256) and shape["lanes_vdp"] > 0
    g1, _ = run_gpu(p, method="dopri5", precision=precision)
    for blk, lanes in ((64, 4096), (256, 1024)):
        g2, _ = run_gpu(p, method="dopri5", precision=precision,
                        tune_block=blk, tune_lanes=lanes)
        np.testing.assert_array_equal(g1["y_final"], g2["y_final"])
        np.testing.assert_array_equal(g1["y_eval"], g2["y_eval"])
        np.testing.assert_array_equal(g1["n_accepted"], g2["n_accepted"])
        np.testing.assert_array_equal(g1["n_rejected"], g2["n_rejected"])


@pytest.mark.parametrize("precision,keep", [("bf16", 0), ("fp32", 0),
                                            ("bf16", 1), ("fp64", 0)])
def test_autotune_neural_shapes_bitwise(precision, keep):
    """Neural fields: every candidate of the autotuner (4 or 8 wavefronts per
    16-row tile; 4, 8 or 16 rounds per graph on the per-stage path) gives
    bitwise the solve of the default shape, and the tuned one is kept."""
    from paper_2210_12375_amd import binding
    flush(f"autotune neural {precision} keep={keep}")
    p = W.neural_ode(B=512, hidden=256)
    ref, _ = run_gpu(p, method="dopri5", precision=precision, rhs=bd.RHS_MLP,
                     keep_dense=keep)
    shape = autotune(p, precision, rhs=bd.RHS_MLP, keep_dense=keep)
    flush(f"  tuned {shape}")
    got, _ = run_gpu(p, method="dopri5", precision=precision, rhs=bd.RHS_MLP,
                     keep_dense=keep)
    np.testing.assert_array_equal(got["y_final"], ref["y_final"])
    np.testing.assert_array_equal(got["n_attempted"], ref["n_attempted"])


def test_tune_cache_file_round_trip(tmp_path):
    """BATCHODE_TUNE_CACHE: a process that autotunes writes the kept shape to
    the file; a fresh process reads it back for the same configuration."""
    import json
    import os
    import subprocess
    import sys
    flush("tune cache file")
    cache = tmp_path / "tune.jsonl"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = f"""
import sys, json
sys.path.insert(0, {root!r}); sys.path.insert(0, {root + '/tests'!r})
import torch
from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W
p = W.uneven_batch(B=2048)
dp = bd.device_problem(p, "fp32")
s = bd.Solver(dp, method="dopri5", precision="fp32")
if sys.argv[1] == "tune":
    bd.solver_autotune(s.cfg, s.prob, s.workspace.data_ptr(),
                       s.workspace.numel(), s.stream.cuda_stream)
    torch.cuda.synchronize()
print(json.dumps(bd.solver_get_tune(s.cfg)), flush=True)
s.close()
"""
    env = dict(os.environ, BATCHODE_TUNE_CACHE=str(cache))
    outs = []
    for mode in ("tune", "read"):
        r = subprocess.run([sys.executable, "-c", code, mode], env=env,
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert outs[0] == outs[1] and outs[0]["block"] > 0, outs
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["B"] == 2048
    assert json.loads(lines[0])["arch"].startswith("gfx")


@pytest.mark.parametrize("ctrl", ["H312PID", "PID"])
def test_pid_fp32_replay(ctrl):
    """FP32 with a PID controller (one exp2 for the whole factor): the
    oracle replays the GPU's attempt record within the FP32 bound."""
    flush(f"vdp fp32 {ctrl}")
    p = W.vdp_batch(B=256)
    c = controller(ctrl)
    g, _ = run_gpu(p, method="dopri5", precision="fp32", record_cap=4096, **c)
    assert np.all(g["status"] == bd.SUCCESS)
    q = as_float_inputs(p)
    info = reduced_replay_check(p, g, "dopri5", "fp32", c)
    flush(f"  max rel {info['rel'].max():.2e}")
    f = oracle.solve(q, method="dopri5", **c)
    flush(f"  steps {g['n_accepted'].mean():.1f} vs FP64 "
          f"{f['n_accepted'].mean():.1f}")
    assert abs(g["n_accepted"].mean() / f["n_accepted"].mean() - 1) < 0.02


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("E", [200, 203])
def test_dense_outputs_many_per_step(method, E):
    """Appendix A's Van der Pol shape (mu = 2, one cycle, tol 1e-5) with E
    evaluation times, about four per accepted step (several emissions per
    step, each reading the prefetched next time), in FP64 against the
    oracle."""
    flush(f"paper vdp E={E} fp64 {method}")
    p = W.paper_vdp(B=64, E=E)
    g, _ = run_gpu(p, method=method, **controller("I"))
    r = oracle.solve(p, method=method, **controller("I"))
    assert np.all(r["status"] == bd.SUCCESS)
    assert_fp64_parity(g, r)
    assert np.median(E / g["n_accepted"]) > 2.0  # several outputs per step


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_slices_resume_inside_a_block(precision):
    """solver_step in slices of 3 attempts resumes each instance with its
    evaluation cursor mid-row (the prefetched next times reloaded): bitwise
    the result of one solve."""
    flush(f"paper vdp slices {precision}")
    p = W.paper_vdp(B=96, E=203)
    dp = bd.device_problem(p, precision)
    one = bd.Solver(dp, method="dopri5", precision=precision,
                    **bd.I_CONTROLLER).solve()
    s = bd.Solver(dp, method="dopri5", precision=precision,
                  **bd.I_CONTROLLER)
    for _ in range(2000):
        if s.step(3, want_running=True) == 0:
            break
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s.y_eval.cpu().numpy(),
                                  one.y_eval.cpu().numpy())
    np.testing.assert_array_equal(s.y_final.cpu().numpy(),
                                  one.y_final.cpu().numpy())
    st = s.stats()
    assert (st["status"].cpu().numpy() == bd.SUCCESS).all()
    one.close()
    s.close()
