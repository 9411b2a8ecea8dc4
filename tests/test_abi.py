"""The C ABI without a GPU: the library loads, exports every entry point
declared in include/batchode.h, validates configurations on the host and
carries tableau constants that satisfy the order conditions (an independent
copy from the oracle's)."""
import re

import numpy as np
import pytest

import oracle
from paper_2210_12375_amd import binding as bd
from test_oracle_tableau import trees

HEADER = __import__("os").path.join(
    __import__("os").path.dirname(__import__("os").path.dirname(
        __import__("os").path.abspath(__file__))), "include", "batchode.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(solver_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(bd.EXPORTED)


def test_library_exports_every_symbol():
    L = bd.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("method", ["dopri5", "tsit5"])
def test_kernel_tableau_satisfies_order_conditions(method):
    c, A, b, e, P = bd.solver_tableau(method)
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-15)
    np.testing.assert_array_equal(A[6], b)
    bh = b - e
    for phi, order, gamma in trees(c, A):
        assert abs(b @ phi - 1.0 / gamma) < 2e-15
        if order <= 4:
            assert abs(bh @ phi - 1.0 / gamma) < 2e-15
    for theta in (0.2, 0.5, 0.9):
        w = P @ theta ** np.arange(1, 5)
        for phi, order, gamma in trees(c, A):
            if order <= 4:
                assert abs(w @ phi - theta ** order / gamma) < 1e-14
    np.testing.assert_allclose(P.sum(axis=1), b, atol=1e-14)  # w(1) = b


@pytest.mark.parametrize("method", ["dopri5", "tsit5"])
def test_kernel_interpolant_equals_oracle_interpolant(method):
    """Two independently written forms of the same continuous extension."""
    _, _, _, _, P = bd.solver_tableau(method)
    for theta in np.linspace(0, 1, 9):
        np.testing.assert_allclose(P @ theta ** np.arange(1, 5),
                                   oracle.dense_weights(method, theta),
                                   atol=1e-14)


def test_workspace_size_rejects_bad_configs():
    good = bd.make_config(64, 2, 8)
    assert bd.solver_workspace_size(good) > 0
    for field, value in [("B", 0), ("D", 0), ("D", 9), ("E", -1),
                         ("method", 5), ("precision", 7), ("rhs", 1),
                         ("max_steps", 0), ("fac_min", 0.0), ("fac_max", 0.5),
                         ("safety", -1.0), ("record_cap", -2),
                         ("fixed_step", 2), ("eager", 3)]:
        c = bd.make_config(64, 2, 8)
        setattr(c, field, value)
        assert bd.solver_workspace_size(c) == 0, field


def test_init_validates_before_touching_the_device():
    import ctypes as C
    cfg = bd.make_config(64, 2, 8)
    cfg.B = -3
    prob = bd.Problem()
    with pytest.raises(bd.BodeError) as ei:
        bd.solver_init(cfg, prob, 256, 1 << 20, None)
    assert ei.value.code == bd.EINVAL
    cfg = bd.make_config(64, 2, 8)
    with pytest.raises(bd.BodeError) as ei:  # missing y0 etc.
        bd.solver_init(cfg, prob, 256, 1 << 20, None)
    assert ei.value.code == bd.EINVAL
    assert "required" in bd.solver_last_error()
    for k in ("y0", "t0", "t_end", "rtol", "atol", "y_final", "t_eval",
              "y_eval", "kind", "dim"):
        setattr(prob, k, 256)
    with pytest.raises(bd.BodeError) as ei:  # workspace too small
        bd.solver_init(cfg, prob, 256, 16, None)
    assert ei.value.code == bd.EINVAL and "too small" in bd.solver_last_error()
    with pytest.raises(bd.BodeError) as ei:  # misaligned workspace
        bd.solver_init(cfg, prob, 260, 1 << 20, None)
    assert ei.value.code == bd.EINVAL
    cfg = bd.make_config(64, 2, 8, fixed_step=1)
    with pytest.raises(bd.BodeError) as ei:  # fixed steps need h0
        bd.solver_init(cfg, prob, 256, 1 << 20, None)
    assert ei.value.code == bd.EINVAL and "h0" in bd.solver_last_error()
    cfg = bd.make_config(64, 2, 8, fixed_step=1, joint=1)
    assert bd.solver_workspace_size(cfg) == 0  # not built for joint mode


def test_null_handles_are_rejected():
    assert bd.lib().solver_solve(None) == bd.EINVAL
    assert bd.lib().solver_step(None, 1, None) == bd.EINVAL
    assert bd.lib().solver_cadjoint(None, 0, None, None, None, 0, None, None,
                                    None) == bd.EINVAL
    assert bd.lib().solver_cadjoint_workspace_bytes(None, 0) == 0
    bd.lib().solver_destroy(None)


def test_ceilings_library_exports_its_kernels():
    """The measurement-only ceilings library (bench.py's achievable peaks)
    is built beside the solver library and exports its four launchers; its
    argument checks run on the host."""
    import ctypes as C
    from paper_2210_12375_amd import build
    L = C.CDLL(build.CEIL_LIB)
    for name in ("ceil_triad", "ceil_mfma_bf16", "ceil_mfma_f32",
                 "ceil_fma_f32"):
        assert hasattr(L, name), name
    L.ceil_mfma_bf16.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    assert L.ceil_mfma_bf16(None, 1, 1, None) != 0  # null output refused


def test_noalloc_solve_validates_before_touching_the_device():
    """The static-scratch entry point rejects, on the host, configurations
    whose workspace exceeds its 32 MiB array and right-hand sides it is not
    built for."""
    prob = bd.Problem()
    for k in ("y0", "t0", "t_end", "rtol", "atol", "y_final", "t_eval",
              "y_eval", "kind", "dim", "W1", "b1", "W2", "b2", "W3", "b3"):
        setattr(prob, k, 256)
    small = bd.make_config(64, 2, 8)
    assert bd.solver_workspace_size(small) <= 32 << 20
    big = bd.make_config(1 << 20, 8, 16, record_cap=8)
    assert bd.solver_workspace_size(big) > 32 << 20
    with pytest.raises(bd.BodeError) as ei:
        bd.solver_solve_noalloc(big, prob, None, None)
    assert ei.value.code == bd.EINVAL and "33554432" in bd.solver_last_error()
    mlp = bd.make_config(64, 64, 0, rhs=bd.RHS_MLP, mlp_hidden=256)
    with pytest.raises(bd.BodeError) as ei:
        bd.solver_solve_noalloc(mlp, prob, None, None)
    assert ei.value.code == bd.EUNSUPPORTED
    bad = bd.make_config(64, 2, 8)
    bad.B = 0
    with pytest.raises(bd.BodeError) as ei:
        bd.solver_solve_noalloc(bad, prob, None, None)
    assert ei.value.code == bd.EINVAL
    with pytest.raises(bd.BodeError) as ei:  # missing inputs
        bd.solver_solve_noalloc(small, bd.Problem(), None, None)
    assert ei.value.code == bd.EINVAL
