"""Safety nets of the HIP path (through the C ABI):

* guard bands: every device buffer the library writes (the workspace, the
  outputs, the continuous adjoint's workspace, the gradients) is allocated
  with 4 KiB of a known byte pattern before and after it; after solves,
  backward passes and the continuous adjoint the bands must be untouched
  (an out-of-bounds write of any kernel shows up here, not as silent
  corruption elsewhere);
* determinism: the same solve and backward twice give bitwise the same
  outputs, statistics, step records and gradients (every reduction has a
  fixed order; no atomics decide a sum)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W

pytestmark = pytest.mark.gpu

GUARD = 4096
PATTERN = 0xA5


def flush(msg):
    print(msg, flush=True)


class Guarded:
    """A device buffer of nbytes between two guard bands."""

    def __init__(self, nbytes):
        self.nbytes = int(nbytes)
        self.raw = torch.full((self.nbytes + 2 * GUARD,), PATTERN,
                              dtype=torch.uint8, device="cuda")
        self.ptr = self.raw.data_ptr() + GUARD
        assert self.ptr % 256 == 0

    def view(self, shape, dtype):
        n = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
        assert n <= self.nbytes
        return self.raw[GUARD:GUARD + n].view(dtype).view(*shape)

    def intact(self):
        g = torch.cat([self.raw[:GUARD], self.raw[GUARD + self.nbytes:]])
        return bool((g == PATTERN).all().item())


def guarded_solve(p, precision, rhs=bd.RHS_ANALYTIC, backward=False,
                  cadjoint=None, **kw):
    dp = bd.device_problem(p, precision)
    B, D = dp["y0"].shape
    E = dp["t_eval"].shape[1]
    if rhs != bd.RHS_ANALYTIC:
        kw.setdefault("mlp_hidden", dp["W1"].shape[1])
    cfg = bd.make_config(B, D, E, precision=precision, rhs=rhs, **kw)
    sd = torch.float64 if precision == "fp64" else torch.float32
    esz = 8 if precision == "fp64" else 4
    ws = Guarded(bd.solver_workspace_size(cfg))
    ye = Guarded(max(1, B * E * D) * esz)
    yf = Guarded(B * D * esz)
    bufs = [ws, ye, yf]
    prob = bd.Problem()
    for k in bd._PROBLEM_FIELDS:
        t = dp.get(k)
        if k == "y_eval":
            setattr(prob, k, ye.ptr)
        elif k == "y_final":
            setattr(prob, k, yf.ptr)
        elif k == "t_eval" and E == 0:
            setattr(prob, k, None)
        else:
            setattr(prob, k, None if t is None else t.data_ptr())
    stream = torch.cuda.current_stream()
    h = bd.solver_init(cfg, prob, ws.ptr, ws.nbytes, stream.cuda_stream)
    bd.solver_solve(h)
    out = {"y_eval": ye.view((B, E, D), sd).clone(),
           "y_final": yf.view((B, D), sd).clone()}
    st = Guarded(5 * B * 4)
    bufs.append(st)
    ptrs = [st.ptr + q * B * 4 for q in range(5)]
    bd.solver_get_stats(h, *ptrs)
    out["stats"] = st.view((5, B), torch.int32).clone()
    if cfg.record_cap > 0:
        rec = Guarded(B * cfg.record_cap * 8)
        nn = Guarded(B * 4)
        er = Guarded(B * cfg.record_cap * 8)
        bufs += [rec, nn, er]
        bd.solver_get_steps(h, rec.ptr, nn.ptr)
        bd.solver_get_errors(h, er.ptr)
        out["h_rec"] = rec.view((B, cfg.record_cap), torch.float64).clone()
    if backward or cadjoint is not None:
        P = sum(np.asarray(p["mlp"][k]).size
                for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
        ge = torch.ones((B, E, D), dtype=sd, device="cuda") if E else None
        gf = torch.ones((B, D), dtype=sd, device="cuda")
        dy0 = Guarded(B * D * esz)
        dth = Guarded(P * esz)
        bufs += [dy0, dth]
        if backward:
            bd.solver_backward(h, None if ge is None else ge.data_ptr(),
                               gf.data_ptr(), dy0.ptr, dth.ptr)
        else:
            cws = Guarded(bd.solver_cadjoint_workspace_bytes(h, cadjoint))
            cst = Guarded(5 * B * 4)
            bufs += [cws, cst]
            bd.solver_cadjoint(h, cadjoint,
                               None if ge is None else ge.data_ptr(),
                               gf.data_ptr(), cws.ptr, cws.nbytes, dy0.ptr,
                               dth.ptr, cst.ptr)
        out["dy0"] = dy0.view((B, D), sd).clone()
        out["dth"] = dth.view((P,), sd).clone()
    torch.cuda.synchronize()
    bd.solver_destroy(h)
    assert all(b.intact() for b in bufs), [b.intact() for b in bufs]
    return {k: v.cpu().numpy() for k, v in out.items()}


CASES = [
    ("analytic fp64, record, keep", lambda: W.uneven_batch(B=777), "fp64",
     bd.RHS_ANALYTIC, dict(record_cap=4096, keep_dense=1)),
    ("analytic fp32", lambda: W.uneven_batch(B=3001), "fp32",
     bd.RHS_ANALYTIC, {}),
    ("joint fp64", lambda: W.vdp_phases(B=37, mu=5.0), "fp64",
     bd.RHS_ANALYTIC, dict(joint=1)),
    ("mlp bf16 fwd+bwd", lambda: W.neural_ode_fit(B=77), "bf16", bd.RHS_MLP,
     dict(record_cap=64, ckpt_every=2, backward=True)),
    ("mlp fp32 per-stage + keep", lambda: W.neural_ode(B=50, d=32,
                                                        hidden=64),
     "fp32", bd.RHS_MLP, dict(keep_dense=1, record_cap=64)),
    ("cnf bf16 fwd+bwd", lambda: W.cnf_density(B=45, hidden=128), "bf16",
     bd.RHS_CNF, dict(record_cap=64, ckpt_every=3, backward=True)),
    ("mlp fp64 fwd+bwd", lambda: W.neural_ode_fit(B=9, d=16, hidden=32),
     "fp64", bd.RHS_MLP, dict(record_cap=64, ckpt_every=0, backward=True)),
    ("mlp fp32 continuous adjoint per instance",
     lambda: W.neural_ode_fit(B=21, d=32, hidden=64), "fp32", bd.RHS_MLP,
     dict(cadjoint=0)),
    ("cnf bf16 continuous adjoint joint", lambda: W.cnf_density(B=24,
                                                                hidden=64),
     "bf16", bd.RHS_CNF, dict(cadjoint=1)),
]


@pytest.mark.parametrize("name,make,precision,rhs,kw", CASES,
                         ids=[c[0] for c in CASES])
def test_guard_bands_and_determinism(name, make, precision, rhs, kw):
    flush(name)
    p = make()
    a = guarded_solve(p, precision, rhs, **kw)
    b = guarded_solve(p, precision, rhs, **kw)
    assert a.keys() == b.keys()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    assert (a["stats"][4] == bd.SUCCESS).any()
