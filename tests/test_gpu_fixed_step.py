"""Fixed-step integration (bode_config.fixed_step) on the GPU against the
oracle's fixed-step mode: every instance steps with its own h0, every
attempt is accepted, the last step is clipped to t_end.  With no controller
in the loop the step sequence is the same on both sides, so FP64 counts are
identical and outputs agree to 1e-9; FP32 to 1e-4 and BF16 to 1e-2 (relative
to each instance's largest output)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import as_float_inputs, run_gpu
from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W

pytestmark = pytest.mark.gpu


def flush(msg):
    print(msg, flush=True)


def rel_rows(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1),
                                                  1e-300)


def compare(p, g, r, tol):
    assert np.array_equal(g["n_attempted"], r["n_attempted"])
    assert np.all(g["n_rejected"] == 0) and np.all(g["status"] == bd.SUCCESS)
    e = max(rel_rows(g["y_final"], r["y_final"]).max(),
            rel_rows(g["y_eval"], r["y_eval"]).max() if g["y_eval"].size
            else 0.0)
    flush(f"  max rel {e:.2e}, steps {int(g['n_attempted'].sum())}")
    assert e <= tol, e


@pytest.mark.parametrize("method", ["dopri5", "tsit5"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_analytic_fixed_steps(method, precision, tol):
    """Van der Pol and linear instances, h0 = 1/32 or 1/64 (exact in binary)
    over spans that are and are not multiples of it, 8 evaluation times."""
    flush(f"fixed step analytic {method} {precision}")
    p = W.subset(W.uneven_batch(B=256, E=8), np.arange(256))
    p["t_end"][:] = np.where(np.arange(256) % 2 == 0, 4.0, 3.3)
    p["t_eval"][:] = np.sort(np.random.default_rng(3).uniform(
        0, 1, (256, 8)) * p["t_end"][:, None], axis=1)
    p["h0"] = np.where(np.arange(256) % 3 == 0, 1 / 32, 1 / 64)
    g, _ = run_gpu(p, method=method, precision=precision, fixed_step=1)
    q = p if precision == "fp64" else as_float_inputs(p)
    r = oracle.solve(q, method=method, fixed_step=True)
    compare(p, g, r, tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4),
                                           ("bf16", 1e-2)])
def test_mlp_fixed_steps(precision, tol):
    """The neural path (per-stage FMA kernels in FP64, the fused matrix-core
    solve in FP32 and BF16) with 16 fixed steps and 8 evaluation times."""
    flush(f"fixed step mlp {precision}")
    p = W.neural_ode_fit(B=40, d=32, hidden=64, n_times=8)
    p["h0"] = np.full(40, 1 / 16)
    g, _ = run_gpu(p, precision=precision, rhs=bd.RHS_MLP, fixed_step=1)
    q = p if precision == "fp64" else as_float_inputs(p)
    r = oracle.solve(q, fixed_step=True)
    assert np.all(r["n_attempted"] == 16)
    compare(p, g, r, tol)
