"""Pins of the oracle's stepping loop, controller and dense output.

Each test checks the oracle against something other than itself: a library
routine that implements the same algorithm (scipy's RK45 is the same
Dormand-Prince pair with the same weighted RMS norm and integral controller),
a closed form (matrix exponential, stability polynomial, harmonic-oscillator
energy, constant fields), a convergence rate, or an invariant of the paper's
design (instances solved independently, section 3).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.integrate._ivp.common import select_initial_step
from scipy.linalg import expm

import oracle
from oracle.oracle import I_CONTROLLER, PI_CONTROLLER, pid_gains
from paper_2210_12375_amd import workloads as W

METHODS = ["dopri5", "tsit5"]


def linear_problem(A, y0, t_end, t_eval=None, rtol=1e-6, atol=1e-8):
    B, D = y0.shape
    E = 0 if t_eval is None else t_eval.shape[1]
    return dict(kind=np.full(B, W.LINEAR, np.int32), dim=np.full(B, D, np.int32),
                y0=y0, t0=np.zeros(B), t_end=np.broadcast_to(t_end, (B,)).copy(),
                rtol=np.full(B, rtol), atol=np.full(B, atol),
                t_eval=np.zeros((B, 0)) if t_eval is None else t_eval, A=A)


def stability_matrix(method, Z):
    c, A, b, bh = oracle.tableau(method)
    R = np.eye(Z.shape[0])
    P = np.eye(Z.shape[0])
    for k in range(1, 8):
        P = P @ Z
        R = R + (b @ np.linalg.matrix_power(A, k - 1) @ np.ones(7)) * P
    return R


def fixed_steps(B, N, h):
    return np.full((B, N), h), np.full(B, N, np.int32)


@pytest.mark.parametrize("method", METHODS)
def test_fixed_steps_follow_stability_polynomial(method, rng):
    """y' = A y with N fixed steps gives y_N = R(hA)^N y0 exactly."""
    D, N, T = 5, 40, 2.0
    M = rng.standard_normal((2, D, D)) - 2 * np.eye(D)
    y0 = rng.standard_normal((2, D))
    p = linear_problem(M, y0, T)
    hr, nr = fixed_steps(2, N, T / N)
    r = oracle.solve(p, method=method, h_replay=hr, n_replay=nr)
    for i in range(2):
        R = stability_matrix(method, (T / N) * M[i])
        ref = np.linalg.matrix_power(R, N) @ y0[i]
        np.testing.assert_allclose(r["y_final"][i], ref, rtol=1e-12,
                                   atol=1e-14 * np.abs(ref).max())
    assert np.all(r["n_accepted"] == N) and np.all(r["n_rejected"] == 0)


@pytest.mark.parametrize("method", METHODS)
def test_fixed_step_mode_follows_stability_polynomial(method, rng):
    """The fixed-step mode (every attempt accepted, h = h0 kept) on y' = A y
    with h0 = T/N (exact in binary) takes N accepted steps and gives
    y_N = R(hA)^N y0; with h0 that does not divide T the last step is
    clipped: y = R(rA) R(hA)^(N-1) y0 with r = T - (N-1) h."""
    D, N, T = 5, 32, 2.0
    M = rng.standard_normal((2, D, D)) - 2 * np.eye(D)
    y0 = rng.standard_normal((2, D))
    p = linear_problem(M, y0, T)
    p["h0"] = np.full(2, T / N)
    p["rtol"][:] = 1e-12  # tolerances the adaptive mode could not meet
    p["atol"][:] = 1e-14
    r = oracle.solve(p, method=method, fixed_step=True)
    for i in range(2):
        R = stability_matrix(method, (T / N) * M[i])
        ref = np.linalg.matrix_power(R, N) @ y0[i]
        np.testing.assert_allclose(r["y_final"][i], ref, rtol=1e-12,
                                   atol=1e-14 * np.abs(ref).max())
    assert np.all(r["n_accepted"] == N) and np.all(r["n_rejected"] == 0)
    h = 0.07
    p["h0"] = np.full(2, h)
    r = oracle.solve(p, method=method, fixed_step=True)
    n = int(np.ceil(T / h))
    t_last = (n - 1) * h
    for i in range(2):
        ref = np.linalg.matrix_power(stability_matrix(method, h * M[i]),
                                     n - 1) @ y0[i]
        ref = stability_matrix(method, (T - t_last) * M[i]) @ ref
        np.testing.assert_allclose(r["y_final"][i], ref, rtol=1e-11,
                                   atol=1e-13 * np.abs(ref).max())
    assert np.all(r["n_accepted"] == n)


@pytest.mark.parametrize("method", METHODS)
def test_order_five_convergence_on_van_der_pol(method):
    """Global error of fixed-step solves of VdP (mu = 0.5, t in [0, 3])
    against a 30-digit Taylor-series reference (mpmath.odefun) falls at least
    like h^5.  Both pairs minimise their fifth-order error constants, so at
    these step sizes the observed slope sits between 5 and 7; any wrong
    coefficient drops it to 4 or below."""
    import mpmath
    mu, T, y = 0.5, 3.0, [1.0, 1.0]
    with mpmath.workdps(30):
        sol = mpmath.odefun(
            lambda t, z: [z[1], mu * (1 - z[0] ** 2) * z[1] - z[0]], 0, y)
        ref = np.array([float(v) for v in sol(T)])
    p = dict(kind=np.zeros(1, np.int32), dim=np.full(1, 2, np.int32),
             y0=np.array([y]), t0=np.zeros(1), t_end=np.full(1, T),
             rtol=np.full(1, 1e-6), atol=np.full(1, 1e-8), mu=np.full(1, mu))
    errs, hs = [], []
    for N in (8, 16, 32, 64, 128):
        hr, nr = fixed_steps(1, N, T / N)
        r = oracle.solve(p, method=method, h_replay=hr, n_replay=nr)
        errs.append(np.abs(r["y_final"][0] - ref).max())
        hs.append(T / N)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 4.7 < slope < 7.0, slope
    assert errs[-1] < 1e-10


@pytest.mark.parametrize("method", METHODS)
def test_error_estimate_is_order_five_locally(method, rng):
    """One step of size h: the embedded error estimate scales like h^5."""
    D = 3
    M = rng.standard_normal((1, D, D))
    y0 = rng.standard_normal((1, D))
    errs = []
    hs = [0.04, 0.02, 0.01, 0.005]
    c, A, b, bh = oracle.tableau(method)
    for h in hs:
        # err of a single step from the closed form of the linear problem
        Z = h * M[0]
        K = np.zeros((7, D))
        for s in range(7):
            Y = y0[0] + h * (A[s, :s] @ K[:s]) if s else y0[0]
            K[s] = M[0] @ Y
        errs.append(np.abs(h * (b - bh) @ K).max())
        # the oracle's accepted step reproduces y + h b^T K
        p = linear_problem(M, y0, h)
        hr, nr = fixed_steps(1, 1, h)
        r = oracle.solve(p, method=method, h_replay=hr, n_replay=nr)
        np.testing.assert_allclose(r["y_final"][0], y0[0] + h * b @ K,
                                   rtol=1e-14, atol=1e-15)
        assert np.allclose(stability_matrix(method, Z) @ y0[0], r["y_final"][0],
                           rtol=1e-13)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 4.7 < slope < 5.4, slope


@pytest.mark.parametrize("method", METHODS)
def test_adaptive_linear_matches_matrix_exponential(method):
    """The uneven batch's linear family against expm(A t) y0, at every
    evaluation time, to a small multiple of the requested tolerance."""
    p = W.uneven_batch(B=64)
    lin = np.flatnonzero(p["kind"] == W.LINEAR)[:12]
    q = W.subset(p, lin)
    r = oracle.solve(q, method=method, **PI_CONTROLLER)
    assert np.all(r["status"] == 1)
    for i in range(len(lin)):
        for e in range(q["t_eval"].shape[1]):
            ref = expm(q["A"][i] * q["t_eval"][i, e]) @ q["y0"][i]
            err = np.abs(r["y_eval"][i, e] - ref).max()
            assert err < 50 * (1e-6 * np.abs(ref).max() + 1e-8), (i, e, err)
        ref = expm(q["A"][i] * q["t_end"][i]) @ q["y0"][i]
        assert np.abs(r["y_final"][i] - ref).max() < 50 * 1e-8 + 1e-12


@pytest.mark.parametrize("method", METHODS)
def test_tolerance_proportionality(method):
    """Global error tracks the tolerance: slope of log err vs log tol in
    [0.6, 1.3] on the linear family."""
    p = W.uneven_batch(B=64)
    lin = np.flatnonzero(p["kind"] == W.LINEAR)[:8]
    q = W.subset(p, lin)
    errs = []
    tols = [1e-5, 1e-7, 1e-9]
    for tol in tols:
        q["rtol"][:] = tol
        q["atol"][:] = tol
        r = oracle.solve(q, method=method, **PI_CONTROLLER)
        e = 0.0
        for i in range(len(lin)):
            ref = expm(q["A"][i] * q["t_end"][i]) @ q["y0"][i]
            e = max(e, np.abs(r["y_final"][i] - ref).max())
            for k in range(q["t_eval"].shape[1]):
                ref = expm(q["A"][i] * q["t_eval"][i, k]) @ q["y0"][i]
                e = max(e, np.abs(r["y_eval"][i, k] - ref).max())
        errs.append(e)
    slope = np.polyfit(np.log(tols), np.log(errs), 1)[0]
    assert 0.6 < slope < 1.3, (slope, errs)


@pytest.mark.parametrize("method", METHODS)
def test_harmonic_oscillator_energy(method):
    """VdP with mu = 0 is x'' = -x.  Fixed steps scale the energy by exactly
    |R(i h)|^2 per step; adaptive solves follow cos / sin."""
    h, N = 0.1, 200
    y0 = np.array([[1.0, 0.0]])
    p = dict(kind=np.zeros(1, np.int32), dim=np.full(1, 2, np.int32), y0=y0,
             t0=np.zeros(1), t_end=np.full(1, h * N), rtol=np.full(1, 1e-6),
             atol=np.full(1, 1e-8), mu=np.zeros(1))
    hr, nr = fixed_steps(1, N, h)
    r = oracle.solve(p, method=method, h_replay=hr, n_replay=nr)
    c, A, b, bh = oracle.tableau(method)
    coeff = [1.0] + [b @ np.linalg.matrix_power(A, k - 1) @ np.ones(7)
                     for k in range(1, 8)]
    R = sum(ck * (1j * h) ** k for k, ck in enumerate(coeff))
    energy = (r["y_final"][0] ** 2).sum()
    assert abs(energy / abs(R) ** (2 * N) - 1.0) < 1e-12
    if method == "dopri5":
        # closed form |R(ih)|^2 for Dormand-Prince's stability polynomial
        Rd = sum(ck * (1j * h) ** k for k, ck in
                 enumerate([1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 120, 1 / 600]))
        assert abs(abs(R) - abs(Rd)) < 1e-15
    # adaptive: the solution is (cos t, -sin t) to the tolerance's order
    t_eval = np.linspace(0, 20, 41)[None, :]
    p2 = dict(p, t_end=np.full(1, 20.0), t_eval=t_eval)
    drift = []
    for tol in (1e-6, 1e-8):
        p2["rtol"], p2["atol"] = np.full(1, tol), np.full(1, tol)
        r2 = oracle.solve(p2, method=method, **PI_CONTROLLER)
        ref = np.stack([np.cos(t_eval[0]), -np.sin(t_eval[0])], axis=1)
        assert np.abs(r2["y_eval"][0] - ref).max() < 200 * tol
        drift.append(abs((r2["y_final"][0] ** 2).sum() - 1.0))
    assert drift[1] < drift[0] / 10


def test_matches_scipy_rk45_step_for_step():
    """Integral controller + Dopri5 is scipy's RK45: the same accepted and
    rejected step counts, step sizes, final states and dense outputs."""
    p = W.vdp_batch(B=16)
    r = oracle.solve(p, method="dopri5", record_cap=4000, **I_CONTROLLER)
    hacc, _ = oracle.accepted_steps(r["h_rec"], r["n_attempted"])
    for i in range(16):
        mu = p["mu"][i]
        f = lambda t, y: np.array([y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]])
        s = solve_ivp(f, (0.0, p["t_end"][i]), p["y0"][i], method="RK45",
                      rtol=1e-6, atol=1e-8, dense_output=True)
        n_acc = len(s.t) - 1
        n_att = (s.nfev - 2) // 6
        assert r["n_accepted"][i] == n_acc
        assert r["n_rejected"][i] == n_att - n_acc
        assert r["n_feval"][i] == s.nfev
        np.testing.assert_allclose(hacc[i, :n_acc], np.diff(s.t), rtol=1e-6)
        scale = np.abs(s.y).max()
        assert np.abs(r["y_final"][i] - s.y[:, -1]).max() < 1e-9 * scale
        ye = s.sol(p["t_eval"][i]).T
        assert np.abs(r["y_eval"][i] - ye).max() < 1e-9 * scale


def test_initial_step_is_hairers_rule():
    p = W.vdp_batch(B=8)
    for i in range(8):
        mu = p["mu"][i]
        f = lambda t, y: np.array([y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]])
        y0 = p["y0"][i]
        ref = select_initial_step(f, 0.0, y0, p["t_end"][i], np.inf, f(0, y0),
                                  1, 4, 1e-6, 1e-8)
        h, nfe = oracle.initial_step(p, i)
        assert nfe == 2
        assert abs(h - ref) <= 1e-14 * ref


_H211PI = pid_gains(1 / 3, -1 / 6, 0.0)
_H312PID = pid_gains(2 / 9, -2 / 9, 1 / 18)


@pytest.mark.parametrize("ctrl,beta", [
    ("I", (0.2, 0.0, 0.0)),
    ("PI", (0.7 / 5, 0.4 / 5, 0.0)),
    ("PI2", (0.15, 0.05, 0.0)),
    ("H211PI", tuple(_H211PI[k] for k in ("beta1", "beta2", "beta3"))),
    ("H312PID", tuple(_H312PID[k] for k in ("beta1", "beta2", "beta3"))),
    ("PID", (0.2, 0.1, -0.02)),
])
def test_controller_steady_state(ctrl, beta):
    """On y' = -y with atol = 0 the error of a step depends only on h, so the
    controller settles where safety * err^(beta2 + beta3 - beta1) = 1, i.e. at
    err* = safety^(1 / (beta1 - beta2 - beta3)).  A dropped or sign-flipped
    term moves this fixed point."""
    b1, b2, b3 = beta
    p = dict(kind=np.full(1, W.LINEAR, np.int32), dim=np.ones(1, np.int32),
             y0=np.ones((1, 1)), t0=np.zeros(1), t_end=np.full(1, 40.0),
             rtol=np.full(1, 1e-6), atol=np.zeros(1), A=-np.ones((1, 1, 1)))
    r = oracle.solve(p, method="dopri5", beta1=b1, beta2=b2, beta3=b3,
                     record_cap=20000)
    hacc, nacc = oracle.accepted_steps(r["h_rec"], r["n_attempted"])
    h = hacc[0, nacc[0] - 5]  # well before the clipped last step
    c, A, b, bh = oracle.tableau("dopri5")
    z = -h
    stage = np.linalg.solve(np.eye(7) - z * A, np.ones(7))  # k_j / (lam y_n)
    err = abs(z * (b - bh) @ stage) / 1e-6
    target = 0.9 ** (1.0 / (b1 - b2 - b3))
    assert abs(err / target - 1.0) < 0.02, (err, target)


def test_pid_gains_map_to_the_known_controllers():
    """The PID-on-log-error parametrisation gives the integral controller for
    gains (1, 0, 0) and Gustafsson's PI (exponents 0.7/5, 0.4/5) for
    (0.3, 0.4, 0); a derivative gain enters all three exponents."""
    for g, ref in (((1.0, 0.0, 0.0), I_CONTROLLER),
                   ((0.3, 0.4, 0.0), PI_CONTROLLER)):
        got = pid_gains(*g)
        for k in ("beta1", "beta2", "beta3"):
            assert abs(got[k] - ref[k]) < 1e-15, (g, k)
    d = pid_gains(0.0, 0.0, 1.0)
    assert (d["beta1"], d["beta2"], d["beta3"]) == (0.2, 0.4, -0.2)


def test_constant_field_grows_steps_by_fac_max():
    """MLP with W3 = 0 is the constant field b3: y(t) = y0 + b3 t exactly,
    the error estimate vanishes and every step grows by fac_max."""
    p = W.neural_ode(B=3, d=4, hidden=8)
    p["mlp"]["W3"][:] = 0.0
    p["h0"] = np.full(3, 1e-3)
    r = oracle.solve(p, method="dopri5", record_cap=64, **PI_CONTROLLER)
    assert np.all(r["status"] == 1)
    ref = p["y0"] + p["mlp"]["b3"][None, :] * 1.0
    np.testing.assert_allclose(r["y_final"], ref, rtol=1e-14, atol=1e-14)
    hacc, nacc = oracle.accepted_steps(r["h_rec"], r["n_attempted"])
    h = hacc[0, :nacc[0]]
    np.testing.assert_allclose(h[1:3] / h[:2], 10.0, rtol=1e-12)


def test_mlp_field_matches_numpy():
    p = W.neural_ode(B=4, d=6, hidden=16)
    m = p["mlp"]
    for i in range(4):
        y = p["y0"][i]
        x = np.append(y, 0.37)
        ref = np.tanh(np.tanh(x @ m["W1"] + m["b1"]) @ m["W2"] + m["b2"]) @ m["W3"] + m["b3"]
        np.testing.assert_allclose(oracle.rhs(p, i, 0.37, y), ref, rtol=1e-13,
                                   atol=1e-14)


def test_special_cases():
    p = W.vdp_batch(B=4)
    p["t_end"][1] = p["t0"][1]
    p["t_eval"][1] = 0.0
    r = oracle.solve(p, method="dopri5", max_steps=100000)
    assert r["status"][1] == 1 and r["n_attempted"][1] == 0
    assert r["n_feval"][1] == 1
    np.testing.assert_array_equal(r["y_final"][1], p["y0"][1])
    np.testing.assert_array_equal(r["y_eval"][1], np.tile(p["y0"][1], (8, 1)))
    r = oracle.solve(p, method="dopri5", max_steps=1)
    assert r["status"][0] == 2 and r["n_attempted"][0] == 1
    assert np.isnan(r["y_eval"][0, -1]).all()
    # a field that overflows: every attempt is rejected until h underflows
    q = W.subset(p, [0])
    q["y0"][:] = 1e200
    q["t0"][:] = 1.0
    q["t_eval"][:] = np.linspace(1.0, q["t_end"][0], 8)
    q["h0"] = np.ones(1)
    r = oracle.solve(q, method="dopri5")
    assert r["status"][0] == 3 and r["n_accepted"][0] == 0
    # invalid inputs are a per-instance status
    q = W.subset(p, [0, 2])
    q["t_eval"][0, 3] = -1.0
    q["rtol"][1] = -1.0
    r = oracle.solve(q, method="dopri5")
    assert list(r["status"]) == [4, 4]


@pytest.mark.parametrize("method", METHODS)
def test_statistics_identities(method):
    p = W.uneven_batch(B=128)
    r = oracle.solve(p, method=method, **PI_CONTROLLER)
    assert np.all(r["status"] == 1)
    np.testing.assert_array_equal(r["n_attempted"],
                                  r["n_accepted"] + r["n_rejected"])
    np.testing.assert_array_equal(r["n_feval"], 2 + 6 * r["n_attempted"])
    p["h0"] = np.full(128, 1e-3)
    r = oracle.solve(p, method=method, **PI_CONTROLLER)
    np.testing.assert_array_equal(r["n_feval"], 1 + 6 * r["n_attempted"])


def test_instances_are_independent():
    """Section 3: each instance is solved as if alone.  Solving a sub-batch,
    a permuted batch or one instance at a time gives bitwise equal results."""
    p = W.uneven_batch(B=96)
    full = oracle.solve(p, method="tsit5")
    perm = np.random.default_rng(0).permutation(96)
    r = oracle.solve(W.subset(p, perm), method="tsit5")
    for k in ("y_eval", "y_final", "n_accepted", "n_rejected"):
        np.testing.assert_array_equal(r[k], full[k][perm])
    for i in (0, 17, 95):
        r = oracle.solve(W.subset(p, [i]), method="tsit5")
        np.testing.assert_array_equal(r["y_eval"][0], full["y_eval"][i])
        np.testing.assert_array_equal(r["y_final"][0], full["y_final"][i])


def test_replay_reproduces_the_adaptive_solve():
    p = W.uneven_batch(B=32)
    r = oracle.solve(p, method="dopri5", record_cap=4000)
    cap = int(r["n_attempted"].max())
    q = oracle.solve(p, method="dopri5", h_replay=r["h_rec"][:, :cap],
                     n_replay=r["n_attempted"], replay_errors=True)
    np.testing.assert_array_equal(q["y_final"], r["y_final"])
    np.testing.assert_array_equal(q["y_eval"], r["y_eval"])
    # replaying the signed attempt record reproduces every decision: the
    # accepted attempts had err < 1, the rejected ones err >= 1, and each
    # attempt's size is the previous attempt's proposal (or the end clip)
    valid = np.arange(cap)[None, :] < r["n_attempted"][:, None]
    acc = r["h_rec"][:, :cap] > 0
    np.testing.assert_array_equal((q["err_rec"] < 1)[valid], acc[valid])
    prop = q["hprop_rec"][:, :-1]
    nxt = np.abs(r["h_rec"][:, 1:cap])
    ok = valid[:, 1:] & (nxt < prop * (1 - 1e-12))  # clipped final steps
    assert np.all((np.abs(nxt - prop) <= 1e-15 * prop)[valid[:, 1:] & ~ok])


def test_float_rounding_probe_is_float_sized():
    """The tests' rounding probe (state rounded to float after each accepted
    step) perturbs a well-conditioned replay by float-sized amounts and leaves
    the step sequence alone."""
    p = W.vdp_batch(B=16)
    r = oracle.solve(p, method="dopri5", record_cap=2048)
    n = r["n_attempted"]
    h = r["h_rec"][:, :n.max()]
    rr = oracle.solve(p, method="dopri5", h_replay=h, n_replay=n)
    rp = oracle.solve(p, method="dopri5", h_replay=h, n_replay=n,
                      round_state_f32=True)
    np.testing.assert_array_equal(rp["n_accepted"], rr["n_accepted"])
    rel = np.abs(rp["y_final"] - rr["y_final"]).max(axis=1) / \
        np.abs(rr["y_final"]).max(axis=1)
    assert np.all(rel > 1e-12) and np.all(rel < 1e-4), rel


def test_pid_study_shape_of_appendix_c():
    """Appendix C: over one Van der Pol cycle, PID-family controllers take
    more steps than the integral controller when the step size varies
    little (small mu) and save steps once the cycle is stiff (mu > 25)."""
    p = W.vdp_cycles(mus=(0.0, 5.0, 10.0, 30.0, 40.0, 50.0))
    i = oracle.solve(p, method="dopri5", **I_CONTROLLER)["n_attempted"]
    for c in (PI_CONTROLLER, pid_gains(0.3, 0.4, 0.1)):
        n = oracle.solve(p, method="dopri5", **c)["n_attempted"]
        assert np.all(n[:3] > i[:3]), (n, i)
        saving = 1.0 - n[3:] / i[3:]
        assert np.all(saving > 0.02), (n, i)
