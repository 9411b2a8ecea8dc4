"""Seeded synthetic workloads shaped like the paper's benchmarks.

This module only draws inputs.  It holds none of the solver's arithmetic and
is the one piece of Python that the HIP path's tests and the CPU oracle
share.  Every generator returns a dict of float64 / int32 numpy arrays in the
layout the C ABI and the oracle both read:

  kind[B], dim[B]            RHS kind per instance and its true dimension
  y0[B, D]                   padded initial states (padding is zero)
  t0[B], t_end[B]            integration bounds per instance
  rtol[B], atol[B]           tolerances per instance (paper section 3 allows
                             per-problem tolerances)
  t_eval[B, E]               sorted evaluation times per instance
  mu[B], A[B, D, D]          Van der Pol damping, linear systems
  mlp{W1,b1,W2,b2,W3,b3}     shared MLP, W_l stored [fan_in, fan_out]
  eps[B, D]                  Rademacher probes for the CNF

The paper's own data (the Black Sea graph data, MNIST) is not used: these
generators stand in for those workloads with the shapes described below.
"""
import numpy as np

VDP, LINEAR, MLP, CNF, CNF_DIAG = 0, 1, 2, 3, 4


def _base(B, D, E):
    return dict(kind=np.zeros(B, np.int32), dim=np.zeros(B, np.int32),
                y0=np.zeros((B, D)), t0=np.zeros(B), t_end=np.zeros(B),
                rtol=np.zeros(B), atol=np.zeros(B), t_eval=np.zeros((B, E)))


def vdp_batch(seed=1, B=64, E=8, rtol=1e-6, atol=1e-8):
    """Van der Pol batch (section 4.1, Eq. eq:vdp): mu ~ U[0.5, 5],
    y0 ~ N(0, 1)^2, t0 = 0, t_end ~ U[5, 10], E sorted times ~ U[0, t_end]."""
    rng = np.random.default_rng(seed)
    p = _base(B, 2, E)
    p["mu"] = rng.uniform(0.5, 5.0, B)
    p["y0"][:] = rng.standard_normal((B, 2))
    p["t_end"][:] = rng.uniform(5.0, 10.0, B)
    p["t_eval"][:] = np.sort(rng.uniform(0.0, 1.0, (B, E)) * p["t_end"][:, None],
                             axis=1)
    p["kind"][:] = VDP
    p["dim"][:] = 2
    p["rtol"][:] = rtol
    p["atol"][:] = atol
    return p


def uneven_batch(seed=2, B=65536, E=16, rtol=1e-6, atol=1e-8):
    """Uneven batch: half Van der Pol (mu log-uniform on [0.1, 20]), half
    linear y' = A y in 8 dimensions with A = -Q diag(lam) Q^T, lam ~ U[0.1, 10]
    and Q a Haar-random orthogonal matrix; t_end ~ U[1, 50]; E sorted times.
    Kinds are interleaved by a seeded permutation; rows are padded to D = 8.
    """
    rng = np.random.default_rng(seed)
    D = 8
    p = _base(B, D, E)
    kind = rng.permutation(np.repeat(np.array([VDP, LINEAR], np.int32),
                                     [B - B // 2, B // 2]))
    p["kind"][:] = kind
    p["dim"][:] = np.where(kind == VDP, 2, 8)
    p["mu"] = np.exp(rng.uniform(np.log(0.1), np.log(20.0), B))
    y0v = rng.standard_normal((B, 2))
    lin = np.flatnonzero(kind == LINEAR)
    n_lin = lin.size
    G = rng.standard_normal((n_lin, D, D))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    lam = rng.uniform(0.1, 10.0, (n_lin, D))
    A = np.zeros((B, D, D))
    A[lin] = -np.einsum("nij,nj,nkj->nik", Q, lam, Q)
    p["A"] = A
    y0l = rng.standard_normal((n_lin, D))
    vd = np.flatnonzero(kind == VDP)
    p["y0"][vd, :2] = y0v[vd]
    p["y0"][lin] = y0l
    p["t_end"][:] = rng.uniform(1.0, 50.0, B)
    p["t_eval"][:] = np.sort(rng.uniform(0.0, 1.0, (B, E)) * p["t_end"][:, None],
                             axis=1)
    p["rtol"][:] = rtol
    p["atol"][:] = atol
    return p


def subset(p, idx):
    """The instances idx of a batch (per-instance arrays sliced, MLP shared)."""
    idx = np.asarray(idx)
    out = {}
    for k, v in p.items():
        if k == "mlp" or v is None or np.ndim(v) == 0:
            out[k] = v
        else:
            out[k] = np.ascontiguousarray(np.asarray(v)[idx])
    return out


def mlp_weights(seed, sizes):
    """Weights W_l ~ N(0, 1/fan_in) stored [fan_in, fan_out], biases likewise."""
    rng = np.random.default_rng(seed)
    w = {}
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        w[f"W{l + 1}"] = rng.standard_normal((fi, fo)) / np.sqrt(fi)
        w[f"b{l + 1}"] = rng.standard_normal(fo) / np.sqrt(fi)
    return w


def neural_ode(seed=3, B=4096, d=64, hidden=256, rtol=1e-5, atol=1e-6,
               weight_seed=3):
    """Neural-ODE forward: y' = MLP([y, t]) with d+1 -> hidden -> hidden -> d
    and tanh hidden layers, y0 ~ N(0, 1), t in [0, 1], final state only."""
    p = _base(B, d, 0)
    p["mlp"] = mlp_weights(weight_seed, [d + 1, hidden, hidden, d])
    rng = np.random.default_rng(seed)
    p["y0"][:] = rng.standard_normal((B, d))
    p["kind"][:] = MLP
    p["dim"][:] = d
    p["t_end"][:] = 1.0
    p["rtol"][:] = rtol
    p["atol"][:] = atol
    return p


def neural_ode_fit(seed=4, B=1024, d=64, hidden=256, n_times=8, rtol=1e-5,
                   atol=1e-6):
    """Neural-ODE fwd+bwd: the MLP of neural_ode (weight seed 3), batch B,
    evaluation at n_times fixed times j / n_times, N(0, 1) targets there."""
    p = neural_ode(seed=seed, B=B, d=d, hidden=hidden, rtol=rtol, atol=atol)
    rng = np.random.default_rng(seed + 1000)
    times = np.arange(1, n_times + 1) / n_times
    p["t_eval"] = np.tile(times, (B, 1))
    p["target"] = rng.standard_normal((B, n_times, d))
    return p


def cnf_density(seed=5, B=8192, d=16, hidden=512, n_comp=8, rtol=1e-5,
                atol=1e-6):
    """CNF-style density: samples x of an n_comp Gaussian mixture in d dims
    (weights 1/n_comp, means 2 N(0, I), isotropic sd 0.5), state [x, 0],
    Rademacher probes, field d+1 -> hidden -> hidden -> d, t in [0, 1]."""
    rng = np.random.default_rng(seed)
    D = d + 1
    p = _base(B, D, 0)
    means = 2.0 * rng.standard_normal((n_comp, d))
    comp = rng.integers(0, n_comp, B)
    x = means[comp] + 0.5 * rng.standard_normal((B, d))
    eps = np.zeros((B, D))
    eps[:, :d] = rng.choice(np.array([-1.0, 1.0]), (B, d))
    p["y0"][:, :d] = x
    p["eps"] = eps
    p["mlp"] = mlp_weights(seed + 1000, [d + 1, hidden, hidden, d])
    p["kind"][:] = CNF
    p["dim"][:] = D
    p["t_end"][:] = 1.0
    p["rtol"][:] = rtol
    p["atol"][:] = atol
    return p


def paper_vdp(seed=6, B=256, mu=2.0, E=200, tol=1e-5, period=7.6295):
    """The paper's Van der Pol loop-time benchmark shape (appendix A): B
    instances with mu = 2 over one cycle, atol = rtol = 1e-5, E evenly spaced
    evaluation times.  Initial states scatter around (2, 0)."""
    rng = np.random.default_rng(seed)
    p = _base(B, 2, E)
    p["mu"] = np.full(B, mu)
    p["y0"][:] = np.array([2.0, 0.0]) + 0.1 * rng.standard_normal((B, 2))
    p["t_end"][:] = period
    p["t_eval"][:] = np.linspace(0.0, period, E)[None, :]
    p["kind"][:] = VDP
    p["dim"][:] = 2
    p["rtol"][:] = tol
    p["atol"][:] = tol
    return p


def vdp_period(mu):
    """Approximate period of Van der Pol's limit cycle: 2 pi (1 + mu^2/16)
    for mu < 1, else the leading relaxation terms (3 - 2 ln 2) mu +
    7.014 mu^(-1/3)."""
    mu = np.asarray(mu, dtype=np.float64)
    small = 2 * np.pi * (1 + mu ** 2 / 16)
    large = (3 - 2 * np.log(2)) * mu + 7.014 * np.maximum(mu, 1e-12) ** (-1 / 3)
    return np.where(mu < 1, small, large)


def vdp_cycles(mus=(0.0, 1.0, 2.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0, 40.0,
                    50.0), tol=1e-6):
    """One cycle of Van der Pol's oscillator per damping strength mu (the
    controller study of appendix C): state (2, 0) near the limit cycle,
    t in [0, vdp_period(mu)], atol = rtol = tol, final state only."""
    mus = np.asarray(mus, dtype=np.float64)
    B = mus.size
    p = _base(B, 2, 0)
    p["mu"] = mus.copy()
    p["y0"][:] = np.array([2.0, 0.0])
    p["t_end"][:] = vdp_period(mus)
    p["kind"][:] = VDP
    p["dim"][:] = 2
    p["rtol"][:] = tol
    p["atol"][:] = tol
    return p


def vdp_phases(seed=7, B=64, mu=25.0, tol=1e-6, E=0):
    """Section 4.1's batch: B Van der Pol oscillators with the same damping
    mu, each started at a different phase of its limit cycle (the state
    after a uniformly drawn fraction of a cycle from (2, 0)), integrated over
    one cycle; atol = rtol = tol.  The phase points come from marching (2, 0)
    along the cycle with small forward-Euler steps (they only need to be
    spread over the cycle, not exact)."""
    rng = np.random.default_rng(seed)
    T = float(vdp_period(mu))
    frac = rng.uniform(0.0, 1.0, B)
    # march (2, 0) along the cycle with small explicit steps to the phases
    n = 200000
    dt = T / n
    x, v = 2.0, 0.0
    marks = np.sort(frac) * T
    order = np.argsort(frac)
    y0 = np.zeros((B, 2))
    t, m = 0.0, 0
    for step in range(n + 1):
        while m < B and marks[m] <= t + 0.5 * dt:
            y0[order[m]] = (x, v)
            m += 1
        if m == B:
            break
        a = mu * (1 - x * x) * v - x
        x, v = x + dt * v, v + dt * a
        t += dt
    p = _base(B, 2, E)
    p["mu"] = np.full(B, mu)
    p["y0"][:] = y0
    p["t_end"][:] = T
    if E:
        p["t_eval"][:] = np.linspace(0.0, T, E)[None, :]
    p["kind"][:] = VDP
    p["dim"][:] = 2
    p["rtol"][:] = tol
    p["atol"][:] = tol
    return p
