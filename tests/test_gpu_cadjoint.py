"""GPU continuous adjoint (solver_cadjoint, appendix A) against the oracle's
continuous adjoint of the same forward result (the GPU's y_final and
statuses are handed to the oracle), per instance and joint.  FP64: the
backward step counts equal and the gradients agree to 1e-9; FP32 (matrix
cores where the shape is built): 1e-4; BF16: 1e-2."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import as_float_inputs, assert_grads
from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W

pytestmark = pytest.mark.gpu

PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")


def flush(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cotangents(p, seed=0):
    rng = np.random.default_rng(seed)
    B, D = p["y0"].shape
    E = p["t_eval"].shape[1]
    return (rng.standard_normal((B, E, D)) if E else None,
            rng.standard_normal((B, D)))


def run(p, precision, rhs, joint, g_eval, g_final, method="dopri5"):
    dp = bd.device_problem(p, precision)
    s = bd.Solver(dp, method=method, precision=precision, rhs=rhs)
    s.solve()
    dt = s.y_final.dtype
    ge = (None if g_eval is None
          else torch.as_tensor(g_eval, dtype=dt, device="cuda"))
    gf = torch.as_tensor(g_final, dtype=dt, device="cuda")
    P = sum(np.asarray(p["mlp"][k]).size for k in PARAMS)
    dy0, dth, st = s.cadjoint(ge, gf, P, joint)
    out = dict(y_final=s.y_final.double().cpu().numpy(),
               fwd=s.stats()["status"].cpu().numpy(),
               dy0=dy0.double().cpu().numpy(), dth=dth.double().cpu().numpy(),
               st=st.cpu().numpy(),
               ge=None if ge is None else ge.double().cpu().numpy(),
               gf=gf.double().cpu().numpy())
    s.close()
    return out


def reference(p, g, joint, method="dopri5"):
    return oracle.cadjoint(p, g["y_final"], g["fwd"], g["ge"], g["gf"],
                           joint=joint, method=method)


CASES = [("mlp", "dopri5"), ("mlp", "tsit5"), ("cnf", "dopri5")]


def problem(kind, B=6, d=8, hidden=16):
    if kind == "mlp":
        return W.neural_ode_fit(B=B, d=d, hidden=hidden, n_times=3), \
            bd.RHS_MLP
    return W.cnf_density(B=B, d=d, hidden=hidden), bd.RHS_CNF


@pytest.mark.parametrize("joint", [0, 1])
@pytest.mark.parametrize("kind,method", CASES)
def test_fp64_against_oracle(kind, method, joint):
    flush(f"cadjoint fp64 {kind} {method} joint={joint}")
    p, rhs = problem(kind)
    g_eval, g_final = cotangents(p)
    g = run(p, "fp64", rhs, joint, g_eval, g_final, method)
    assert np.all(g["fwd"] == bd.SUCCESS)
    r = reference(p, g, joint, method)
    assert np.all(g["st"][4] == bd.SUCCESS)
    assert np.array_equal(g["st"][0], r["n_attempted"]), (g["st"][0],
                                                          r["n_attempted"])
    assert np.array_equal(g["st"][1], r["n_accepted"])
    assert np.array_equal(g["st"][3], r["n_feval"])
    assert_grads(p, g, r["dy0"], r["dtheta"], 1e-9)


@pytest.mark.parametrize("joint", [0, 1])
@pytest.mark.parametrize("precision,kind,d,hidden", [
    ("fp32", "mlp", 32, 64),   # FP32 matrix cores
    ("fp32", "mlp", 24, 48),   # FMA kernels
    ("bf16", "mlp", 32, 64),
    ("fp32", "cnf", 16, 64),
    ("bf16", "cnf", 16, 64),
])
def test_reduced_precision_against_oracle(precision, kind, d, hidden, joint):
    flush(f"cadjoint {precision} {kind} d={d} H={hidden} joint={joint}")
    p, rhs = problem(kind, B=24, d=d, hidden=hidden)
    g_eval, g_final = cotangents(p, 1)
    g = run(p, precision, rhs, joint, g_eval, g_final)
    assert np.all(g["fwd"] == bd.SUCCESS)
    assert np.all(g["st"][4] == bd.SUCCESS)
    r = reference(as_float_inputs(p), g, joint)
    flush(f"  steps gpu {g['st'][0].sum()} oracle {r['n_attempted'].sum()}")
    assert_grads(p, g, r["dy0"], r["dtheta"],
                 1e-4 if precision == "fp32" else 1e-2)


def test_edges():
    """An instance with t0 = t_end (no backward steps: dy0 = the cotangents),
    evaluation times at t0 and at t_end, and joint membership (an instance
    with other evaluation times is left out of the joint system)."""
    flush("cadjoint edges")
    p, rhs = problem("mlp", B=5, d=8, hidden=16)
    p["t_eval"] = np.tile(np.array([0.0, 0.5, 0.5, 1.0]), (5, 1))
    p["t_end"][3] = 0.0
    p["t_eval"][3] = 0.0
    g_eval, g_final = cotangents(p, 2)
    for joint in (0, 1):
        g = run(p, "fp64", rhs, joint, g_eval, g_final)
        r = reference(p, g, joint)
        assert np.array_equal(g["st"][4], r["status"])
        ok = r["status"] != 4
        assert np.all(np.isnan(g["dy0"][~ok]))
        assert rel(g["dy0"][ok], r["dy0"][ok]) <= 1e-9
        assert rel(g["dth"], r["dtheta"]) <= 1e-9
        if joint:
            assert r["status"][3] == 4  # other span: not a member
        else:
            assert np.allclose(g["dy0"][3], g_final[3] + g_eval[3].sum(0),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("precision,kind,d,hidden,reps", [
    ("bf16", "cnf", 16, 512, 100),   # the CNF field of the benchmark
    ("fp32", "mlp", 32, 384, 200),   # FMA kernels, ragged entry blocks
])
def test_per_instance_at_scale_replicated(precision, kind, d, hidden, reps):
    """Per-instance parameter adjoints of 12 * reps instances (two [B, P]
    buffers of several GB): 12 distinct instances repeated, so every copy
    takes its original's steps and dtheta is reps times the oracle's."""
    flush(f"cadjoint replicated {precision} {kind} H={hidden} reps={reps}")
    base, rhs = problem(kind, B=12, d=d, hidden=hidden)
    idx = np.tile(np.arange(12), reps)
    p = W.subset(base, idx)
    g_eval0, g_final0 = cotangents(base, 4)
    g = run(p, precision, rhs, 0, None if g_eval0 is None else g_eval0[idx],
            g_final0[idx])
    assert np.all(g["st"][4] == bd.SUCCESS)
    for r in range(1, reps):
        assert np.array_equal(g["st"][0][12 * r:12 * r + 12], g["st"][0][:12])
    sub = dict(y_final=g["y_final"][:12], fwd=g["fwd"][:12],
               ge=None if g["ge"] is None else g["ge"][:12], gf=g["gf"][:12])
    r = reference(as_float_inputs(base), sub, 0)
    assert_grads(base, g, np.tile(r["dy0"], (reps, 1)), reps * r["dtheta"],
                 1e-4 if precision == "fp32" else 1e-2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("joint", [0, 1])
def test_graph_matches_eager(precision, joint):
    """The backward loop replays a captured graph of 4 attempts between its
    running-count checks; the eager loop gives bitwise the same result."""
    flush(f"cadjoint graph vs eager {precision} joint={joint}")
    p, rhs = problem("cnf", B=20, d=8, hidden=32)
    g_eval, g_final = cotangents(p, 6)
    out = []
    for eager in (0, 1):
        dp = bd.device_problem(p, precision)
        s = bd.Solver(dp, precision=precision, rhs=rhs, eager=eager)
        s.solve()
        dt = s.y_final.dtype
        gf = torch.as_tensor(g_final, dtype=dt, device="cuda")
        P = sum(np.asarray(p["mlp"][k]).size for k in PARAMS)
        dy0, dth, st = s.cadjoint(None, gf, P, joint)
        out.append((dy0.cpu().numpy(), dth.cpu().numpy(), st.cpu().numpy()))
        s.close()
    for x, y in zip(out[0], out[1]):
        np.testing.assert_array_equal(x, y)
    assert out[0][2][0].max() > 4  # more than one replay


@pytest.mark.parametrize("kind", ["cnf", "mlp"])
def test_full_size_continuous_agrees_with_discrete(kind):
    """The benchmark's continuous-adjoint workloads at full size: 8192 CNF
    instances with a 512-wide field in BF16 (the joint pass forms each
    attempt's parameter part with the 256 x 256-tile GEMM over all seven
    stages at once) and 1024 MLP instances in FP32.  The per-instance and
    joint continuous adjoints and the discrete adjoint of the same forward
    solve approximate one gradient: dtheta and dy0 agree to well within
    the solve's tolerance (rtol 1e-5; measured 1e-6), where a wrong stage,
    slot or tape offset gives an O(1) difference."""
    flush(f"full-size continuous vs discrete {kind}")
    if kind == "cnf":
        p, rhs, prec = W.cnf_density(), bd.RHS_CNF, "bf16"
    else:
        p, rhs, prec = W.neural_ode_fit(), bd.RHS_MLP, "fp32"
    dp = bd.device_problem(p, prec)
    P = sum(np.asarray(p["mlp"][k]).size for k in PARAMS)
    s = bd.Solver(dp, method="dopri5", precision=prec, rhs=rhs,
                  record_cap=256, ckpt_every=2).solve()
    B, D = p["y0"].shape
    E = p["t_eval"].shape[1]
    gf = torch.ones((B, D), dtype=torch.float32, device="cuda")
    ge = (torch.ones((B, E, D), dtype=torch.float32, device="cuda")
          if E else None)
    dy0_d, dth_d = s.backward(ge, gf, P)
    ref0, ref1 = dy0_d.double().cpu().numpy(), dth_d.double().cpu().numpy()
    for joint in (0, 1):
        dy0, dth, st = s.cadjoint(ge, gf, P, joint)
        assert np.all(st[4].cpu().numpy() == bd.SUCCESS)
        e0 = rel(dy0.double().cpu().numpy(), ref0)
        e1 = rel(dth.double().cpu().numpy(), ref1)
        flush(f"  joint={joint}: dy0 {e0:.2e} dtheta {e1:.2e}")
        assert e0 <= 1e-4 and e1 <= 1e-4, (joint, e0, e1)
    s.close()
