"""Shared helpers of the GPU parity tests (they call the HIP path only
through the C ABI, via paper_2210_12375_amd.binding)."""
import numpy as np

import oracle
from paper_2210_12375_amd import binding as bd
from paper_2210_12375_amd import workloads as W

# FP64 mode must match the FP64 oracle to this relative error per instance
# with identical accepted / rejected counts.
TOL_FP64 = 1e-9
# FP32 state (and the FP32 controller): the oracle replays the GPU's accepted
# steps in FP64; per-instance relative error bound.
TOL_FP32 = 1e-4
# BF16 MFMA right-hand side, same replay.
TOL_BF16 = 1e-2


def per_instance_absdiff(a_eval, a_final, b_eval, b_final):
    """(max |a - b|, max |b|) per instance over evaluation outputs and final
    state."""
    B = a_final.shape[0]
    a = np.concatenate([a_eval.reshape(B, -1), a_final.reshape(B, -1)], axis=1)
    b = np.concatenate([b_eval.reshape(B, -1), b_final.reshape(B, -1)], axis=1)
    nan_a, nan_b = np.isnan(a), np.isnan(b)
    assert np.array_equal(nan_a, nan_b), "NaN pattern differs"
    a = np.where(nan_a, 0.0, a)
    b = np.where(nan_b, 0.0, b)
    return np.abs(a - b).max(axis=1), np.abs(b).max(axis=1)


def per_instance_rel(a_eval, a_final, b_eval, b_final):
    """max |a - b| / max |b| per instance over evaluation outputs and final
    state (robust at zero crossings of single components)."""
    B = a_final.shape[0]
    a = np.concatenate([a_eval.reshape(B, -1), a_final.reshape(B, -1)], axis=1)
    b = np.concatenate([b_eval.reshape(B, -1), b_final.reshape(B, -1)], axis=1)
    nan_a, nan_b = np.isnan(a), np.isnan(b)
    assert np.array_equal(nan_a, nan_b), "NaN pattern differs"
    a = np.where(nan_a, 0.0, a)
    b = np.where(nan_b, 0.0, b)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / scale


def run_gpu(p, method="dopri5", precision="fp64", rhs=bd.RHS_ANALYTIC, **kw):
    import torch
    dp = bd.device_problem(p, precision)
    s = bd.Solver(dp, method=method, precision=precision, rhs=rhs, **kw)
    s.solve()
    st = s.stats()
    out = dict(y_eval=s.y_eval.double().cpu().numpy(),
               y_final=s.y_final.double().cpu().numpy(),
               **{k: v.cpu().numpy() for k, v in st.items()})
    if s.cfg.record_cap > 0:
        h, n = s.steps()
        out["h_rec"] = h.cpu().numpy()
        out["n_rec"] = n.cpu().numpy()
        out["e_rec"] = s.errors().cpu().numpy()
    torch.cuda.synchronize()
    return out, s


# PID presets on log err: Soderlind's H211PI and H312PID digital filters
# (2003) in gain form, and a PID with a positive derivative gain.
PID_CONTROLLERS = {
    "H211PI": bd.pid_gains(1 / 3, -1 / 6, 0.0),
    "H312PID": bd.pid_gains(2 / 9, -2 / 9, 1 / 18),
    "PID": bd.pid_gains(0.3, 0.4, 0.1),
}


def controller(ctrl):
    if ctrl in PID_CONTROLLERS:
        return PID_CONTROLLERS[ctrl]
    return bd.I_CONTROLLER if ctrl == "I" else bd.PI_CONTROLLER


def assert_fp64_parity(g, r, max_mismatch=0):
    """Identical counters and statuses, outputs within TOL_FP64.  Instances
    whose step sequence split at a near-tie accept decision (error norm within
    rounding of 1) are allowed up to max_mismatch, and must still agree to the
    tolerance level of the solve."""
    same = ((g["n_accepted"] == r["n_accepted"])
            & (g["n_rejected"] == r["n_rejected"]))
    np.testing.assert_array_equal(g["status"], r["status"])
    bad = np.flatnonzero(~same)
    assert bad.size <= max_mismatch, (bad, g["n_accepted"][bad],
                                      r["n_accepted"][bad])
    rel = per_instance_rel(g["y_eval"], g["y_final"], r["y_eval"], r["y_final"])
    ok = np.flatnonzero(same)
    assert rel[ok].max(initial=0.0) <= TOL_FP64, (rel[ok].max(),
                                                  ok[np.argmax(rel[ok])])
    if bad.size:
        assert rel[bad].max() <= 1e-4, rel[bad]
    np.testing.assert_array_equal(g["n_feval"][ok], r["n_feval"][ok])
    return rel


def as_float_inputs(p):
    """The problem as the FP32 path sees it: state-typed inputs (initial
    states and field parameters) rounded to float; times stay double."""
    q = dict(p)
    for k in ("y0", "mu", "A", "eps"):
        if q.get(k) is not None:
            q[k] = np.asarray(q[k]).astype(np.float32).astype(np.float64)
    if q.get("mlp") is not None:
        q["mlp"] = {k: np.asarray(v).astype(np.float32).astype(np.float64)
                    for k, v in q["mlp"].items()}
    return q


def oracle_replay(p, g, method):
    """The oracle's FP64 replay of the GPU's accepted step sequence."""
    n = g["n_rec"]
    cap = int(n.max()) if n.size else 0
    assert cap <= g["h_rec"].shape[1], "record_cap too small for the replay"
    return oracle.solve(p, method=method, h_replay=g["h_rec"][:, :max(cap, 1)],
                        n_replay=n)


def conditioned_counts(p, method, ctrl=None, eps=1e-12):
    """The oracle's solve plus a mask of instances whose accepted / rejected
    counts are a well-conditioned function of the input: unchanged when
    rtol and atol are scaled by 1 +- eps.  Instances whose step size sits at
    the stability boundary (the linear family at h * lambda_max ~ 3.3) flip
    accept decisions under any 1-ulp perturbation, including the oracle's own
    compilation with or without fused multiply-add, so only their solutions,
    not their exact step counts, are defined.  The probes: tolerances scaled
    by 1 +- eps, and the oracle's source compiled with contracted
    multiply-adds."""
    kw = ctrl or {}
    r0 = oracle.solve(p, method=method, **kw)
    ok = np.ones(p["y0"].shape[0], bool)
    probes = [(dict(p, rtol=p["rtol"] * s, atol=p["atol"] * s), None)
              for s in (1 + eps, 1 - eps)] + [(p, "fma")]
    for q, variant in probes:
        r = oracle.solve(q, method=method, variant=variant, **kw)
        ok &= ((r["n_accepted"] == r0["n_accepted"])
               & (r["n_rejected"] == r0["n_rejected"]))
    return r0, ok


def replay_check(p, g, method, ctrl=None, tol=TOL_FP64, decisions=True,
                 decision_kinds=(0, 1)):
    """Decision-by-decision check of the GPU's attempt record (every attempted
    step size, negated when rejected) against the FP64 oracle:
      - replaying exactly that sequence reproduces every output within tol;
      - the first attempt is Hairer's starting step (clipped to the span);
      - every accept / reject decision agrees with the oracle's FP64 error
        test, except near-ties |err - 1| < 1e-4;
      - every later attempt's size is the oracle controller's proposal from
        the replayed history (or the clip to t_end), within 1e-4 (the error
        estimate of a tiny step carries ~1e-5 relative rounding noise).
    Every valid instance is replayed (those that stopped early, e.g. at
    max_steps, without the final clip to t_end); decisions and
    proposals are checked for the kinds in decision_kinds (at the stability
    boundary the linear family's error norm is rounding noise at the atol
    level, so its decisions are not defined beyond that noise)."""
    kw = ctrl or {}
    n = g["n_rec"]
    H = g["h_rec"]
    assert n.max() <= H.shape[1], "record_cap too small"
    idx = np.flatnonzero((g["status"] != 4) & (n > 0))
    q = W.subset(p, idx)
    cap = int(max(1, n[idx].max()))
    Hs = H[idx, :cap]
    fin = (g["status"][idx] == 1).astype(np.int32)
    if "e_rec" in g:  # the record's own decisions and controller steps
        controller_record_check(q, Hs, g["e_rec"][idx, :cap], n[idx], ctrl,
                                "fp64")
    rr = oracle.solve(q, method=method, h_replay=Hs, n_replay=n[idx],
                      replay_errors=True, replay_final=fin, **kw)
    np.testing.assert_array_equal(rr["status"] == 1, fin == 1)
    # the instance's own rounding sensitivity on this step sequence: the same
    # replay by the oracle's source compiled with contracted multiply-adds
    rf = oracle.solve(q, method=method, h_replay=Hs, n_replay=n[idx],
                      variant="fma", replay_errors=True, replay_final=fin,
                      **kw)
    sens, _ = per_instance_absdiff(rf["y_eval"], rf["y_final"], rr["y_eval"],
                                   rr["y_final"])
    diff, scale = per_instance_absdiff(g["y_eval"][idx], g["y_final"][idx],
                                       rr["y_eval"], rr["y_final"])
    allowed = np.maximum(tol * scale, 1000.0 * sens)
    worst = np.argmax(diff / np.maximum(allowed, 1e-300))
    assert np.all(diff <= allowed), (idx[worst], diff[worst], scale[worst],
                                     sens[worst])
    rel = diff / np.maximum(scale, 1e-300)
    if not decisions:
        return rel
    valid = np.arange(cap)[None, :] < n[idx][:, None]
    err = rr["err_rec"]
    acc = Hs > 0
    # a decision is a near-tie when err sits within its own rounding noise of
    # 1: the embedded estimate cancels (sum e_j = 0), so on very small steps
    # it carries relative noise up to ~1e-5; also ten times the norm's change
    # under contracted multiply-adds
    err_sens = np.abs(err - rf["err_rec"])
    tie = np.abs(err - 1.0) < np.maximum(1e-4, 10.0 * err_sens)
    dk = np.isin(q["kind"], decision_kinds)[:, None]
    wrong = valid & dk & (acc != (err < 1.0)) & ~tie
    assert not wrong.any(), (np.argwhere(wrong)[:5], err[wrong][:5])
    # start times of every attempt (sequential sums, as the kernel forms t)
    hacc = np.where(acc & valid, np.abs(Hs), 0.0)
    t_start = np.empty_like(Hs)
    t = q["t0"].astype(np.float64).copy()
    for k in range(cap):
        t_start[:, k] = t
        t = t + hacc[:, k]
    te = q["t_end"][:, None]
    prop = rr["hprop_rec"][:, :-1]
    prop_sens = np.abs(prop - rf["hprop_rec"][:, :-1])
    nxt = np.abs(Hs[:, 1:])
    ts = t_start[:, 1:]
    clip = ts + prop >= te
    expect = np.where(clip, te - ts, prop)
    ambiguous = np.abs(ts + prop - te) <= 1e-6 * prop
    chk = valid[:, 1:] & ~ambiguous & dk
    bad = chk & (np.abs(nxt - expect)
                 > np.maximum(1e-4 * expect, 10.0 * prop_sens))
    assert not bad.any(), (np.argwhere(bad)[:5], nxt[bad][:5], expect[bad][:5])
    if q.get("h0") is None:
        for j in range(min(len(idx), 64)):
            if q["t_end"][j] == q["t0"][j]:
                continue
            h0, _ = oracle.initial_step(q, j)
            assert abs(abs(Hs[j, 0]) - h0) <= 1e-9 * h0, (j, Hs[j, 0], h0)
    return rel


def free_check(p, g, method, ctrl=None, exact_kinds=(0,), loose=1e-4,
               mismatch_frac=0.005):
    """The GPU's free-running solve against the oracle's: identical statuses;
    identical counts for well-conditioned instances of exact_kinds (a
    near-tie share of mismatch_frac allowed); counts within 5 % (or 3) for
    the rest; outputs within `loose` (both are valid solutions at the stated
    tolerance once their step sequences have parted).  The linear family is
    not in exact_kinds: its steps settle on the method's stability boundary
    (h * lambda_max ~ 3.3 for Dormand-Prince) where any rounding change flips
    accept decisions, so its exact counts are not defined."""
    r0, ok = conditioned_counts(p, method, ctrl)
    ok &= np.isin(p["kind"], exact_kinds)
    np.testing.assert_array_equal(g["status"], r0["status"])
    same = ((g["n_accepted"] == r0["n_accepted"])
            & (g["n_rejected"] == r0["n_rejected"]))
    cond = np.flatnonzero(ok)
    bad = cond[~same[cond]]
    assert bad.size <= max(1, int(mismatch_frac * cond.size)), bad
    ill = np.flatnonzero(~ok)
    d = np.abs(g["n_accepted"][ill] - r0["n_accepted"][ill])
    assert np.all(d <= np.maximum(3, 0.05 * r0["n_accepted"][ill])), d.max()
    diff, scale = per_instance_absdiff(g["y_eval"], g["y_final"],
                                       r0["y_eval"], r0["y_final"])
    # decayed instances are atol-level noise: an absolute floor of 100 atol
    allowed = loose * scale + 100.0 * p["atol"]
    worst = np.argmax(diff / allowed)
    assert np.all(diff <= allowed), (worst, diff[worst], scale[worst])
    return dict(n_exact=cond.size, n_mismatch=bad.size, n_ill=ill.size,
                max_rel=float((diff / np.maximum(scale, 1e-300)).max()))


def assert_uneven_parity(p, g, method, ctrl=None):
    rel = replay_check(p, g, method, ctrl, decision_kinds=(0,))
    info = free_check(p, g, method, ctrl)
    info["replay_max_rel"] = float(rel.max(initial=0.0))
    return info


def assert_linear_accuracy(p, g, n_max=64, factor=50.0):
    """Linear instances against the matrix exponential at every output."""
    from scipy.linalg import expm
    lin = np.flatnonzero(p["kind"] == 1)[:n_max]
    for i in lin:
        A = p["A"][i]
        for e in range(p["t_eval"].shape[1]):
            ref = expm(A * (p["t_eval"][i, e] - p["t0"][i])) @ p["y0"][i]
            bound = factor * (p["rtol"][i] * np.abs(ref).max() + p["atol"][i])
            assert np.abs(g["y_eval"][i, e] - ref).max() <= bound, (i, e)
        ref = expm(A * (p["t_end"][i] - p["t0"][i])) @ p["y0"][i]
        bound = factor * (p["rtol"][i] * np.abs(ref).max() + p["atol"][i])
        assert np.abs(g["y_final"][i] - ref).max() <= bound, i


# Relative agreement of a recorded step size with the controller law applied
# to the recorded error norms.  FP64: pow and products correctly rounded to a
# few ulps.  FP32 / BF16: the exponent of the factor is formed in float from
# terms up to ~60 in magnitude (log2 of squared norms) and the hardware
# log2 / exp2 are ~1 ulp, so the factor carries ~1e-6 relative rounding;
# 1e-5 leaves a margin of ten.
CTL_RTOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-5}


def controller_record_check(p, h_rec, e_rec, n, ctrl=None, precision="fp64",
                            fixed=False):
    """The GPU's step record against its own recorded error norms and the
    controller law declared in include/batchode.h (paper section 3: each
    instance accepts or rejects on its own error norm and sizes its next step
    from its own error history; appendix C for the PID family):
      - an attempt is accepted exactly when its recorded norm is below 1
        (every attempt in fixed-step mode);
      - the next attempt's size is hs * fac, fac the law of the header
        evaluated in FP64 on the recorded norms (err_prev, err_prev2 the
        norms of the two previous accepted attempts clamped below at 1e-4, 1
        before any), clipped to t_end - t when t + hs * fac reaches t_end,
        within CTL_RTOL[precision].
    Returns the number of checked proposals."""
    c = dict(beta1=0.14, beta2=0.08, beta3=0.0, safety=0.9, fac_min=0.2,
             fac_max=10.0)
    c.update(ctrl or {})
    B, cap = h_rec.shape
    n = np.minimum(n, cap)
    k_idx = np.arange(cap)[None, :]
    valid = k_idx < n[:, None]
    acc = h_rec > 0
    if fixed:
        assert np.all(acc[valid]), "a fixed-step attempt was rejected"
    else:
        dec = e_rec < 1.0
        wrong = valid & (acc != dec)
        assert not wrong.any(), (np.argwhere(wrong)[:5], e_rec[wrong][:5])
    rtol = CTL_RTOL[precision]
    t = np.asarray(p["t0"], np.float64).copy()
    te = np.asarray(p["t_end"], np.float64)
    ep1 = np.ones(B)
    ep2 = np.ones(B)
    prev_rej = np.zeros(B, bool)
    checked = 0
    for k in range(cap - 1):
        live = n > k + 1
        if not live.any():
            break
        hk = np.abs(h_rec[:, k])
        e = e_rec[:, k]
        a = acc[:, k]
        with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
            fa = (c["safety"] * e ** -c["beta1"] * ep1 ** c["beta2"]
                  * ep2 ** c["beta3"])
            fr = c["safety"] * e ** -0.2
        fa = np.where(e == 0.0, c["fac_max"], fa)
        fa = np.clip(fa, c["fac_min"], c["fac_max"])
        fa = np.where(prev_rej, np.minimum(1.0, fa), fa)
        fr = np.maximum(c["fac_min"], fr)
        fac = np.where(a, fa, fr)
        fac = np.where(np.isfinite(e), fac, c["fac_min"])
        if fixed:
            fac = np.ones(B)
        t = np.where(a, t + hk, t)
        ep2 = np.where(a, ep1, ep2)
        ep1 = np.where(a, np.maximum(e, 1e-4), ep1)
        prev_rej = ~a
        with np.errstate(invalid="ignore"):  # attempts past n are unset
            prop = hk * fac
        clip = t + prop >= te
        expect = np.where(clip, te - t, prop)
        ambiguous = np.abs(t + prop - te) <= 10 * rtol * prop
        chk = live & ~ambiguous
        nxt = np.abs(h_rec[:, k + 1])
        bad = chk & (np.abs(nxt - expect) > rtol * expect)
        assert not bad.any(), (k, np.flatnonzero(bad)[:5], nxt[bad][:5],
                               expect[bad][:5])
        checked += int(chk.sum())
    return checked


# FP32 phase allowance of the analytic replay check, as a fraction of the
# time an output lies after t0: 2^-20, eight float ulps of the elapsed time.
# The FP32 state is rounded to float at every stage; on the slow branch of a
# stiff relaxation oscillation (Van der Pol, mu up to 20) a state
# perturbation dy moves the phase by about mu dy, and at the fast jump that
# follows a phase error dt moves the state by |y'| dt ~ mu dt, so float
# rounding alone gives errors up to ~mu^2 eps_f32 ~ 1e-4 at outputs that
# fall inside a jump while the final state agrees to ~1e-7.  Such an output
# counts as agreeing when it is within tol of the oracle's solution at a time
# at most 2^-20 (t_e - t0) away: |a - b| <= tol scale + 2^-20 (t_e - t0) |f|.
PHASE_REL = 2.0 ** -20


def phase_allowance(p, kinds_ok, r_eval, diff_eval, bound):
    """For outputs of analytic instances whose difference exceeds bound
    (per instance), the phase allowance 2^-20 (t_e - t0) max |f(t_e, b)|
    with f evaluated by the oracle at its own output b; zero elsewhere."""
    B, E = diff_eval.shape
    allow = np.zeros((B, E))
    for i, e in zip(*np.nonzero(diff_eval > bound[:, None])):
        if not kinds_ok[i]:
            continue
        dim = int(p["dim"][i])
        te = p["t_eval"][i, e]
        f = oracle.rhs(p, i, te, r_eval[i, e, :dim])
        allow[i, e] = PHASE_REL * (te - p["t0"][i]) * np.abs(f).max()
    return allow


def reduced_replay_check(p, g, method, precision, ctrl=None,
                         decision_band=None, decision_kinds=(0, 1, 2, 3),
                         tol=None, phase=False):
    """Reduced-precision (FP32 / BF16) solve against the FP64 oracle, attempt
    by attempt:
      - controller_record_check: every decision equals its own recorded norm
        test and every next step size is the controller law applied to the
        recorded norms (CTL_RTOL);
      - the oracle replays the recorded attempts in FP64 on the inputs the
        GPU received (state-typed inputs rounded to float); every instance's
        outputs agree within tol (1e-4 FP32, 1e-2 BF16) of the instance's
        scale, the largest magnitude among its outputs and its initial
        state (an instance that decays far below its start is measured
        against where it started);
      - if decision_band is given, every decision of the kinds in
        decision_kinds agrees with the oracle's FP64 norm test, except
        near-ties |err - 1| <= decision_band.
    Returns the per-instance relative errors and the attempts' recorded and
    oracle norms."""
    tol = tol if tol is not None else (TOL_BF16 if precision == "bf16"
                                       else TOL_FP32)
    kw = ctrl or {}
    n = g["n_rec"]
    H, E = g["h_rec"], g["e_rec"]
    assert n.max() <= H.shape[1], "record_cap too small"
    checked = controller_record_check(p, H, E, n, ctrl, precision)
    q = as_float_inputs(p)
    cap = int(max(1, n.max()))
    fin = (g["status"] == bd.SUCCESS).astype(np.int32)
    rr = oracle.solve(q, method=method, h_replay=H[:, :cap], n_replay=n,
                      replay_errors=True, replay_final=fin, **kw)
    diff, scale = per_instance_absdiff(g["y_eval"], g["y_final"], rr["y_eval"],
                                       rr["y_final"])
    scale = np.maximum(scale, np.abs(q["y0"]).max(axis=1))
    rel = diff / np.maximum(scale, 1e-300)
    n_phase = 0
    if phase and rel.max() > tol:
        B = scale.size
        de = np.abs(np.nan_to_num(g["y_eval"]) - np.nan_to_num(rr["y_eval"]))
        de = de.reshape(B, g["y_eval"].shape[1], -1).max(axis=2)
        df = np.abs(np.nan_to_num(g["y_final"]) - np.nan_to_num(rr["y_final"]))
        df = df.max(axis=1)
        bound = tol * scale
        allow = phase_allowance(q, q["kind"] <= 1, rr["y_eval"], de, bound)
        n_phase = int(np.sum((de > bound[:, None]) & (de <= bound[:, None]
                                                      + allow)))
        bad = np.flatnonzero((de > bound[:, None] + allow).any(axis=1)
                             | (df > bound))
        assert bad.size == 0, (bad[:5], rel[bad[:5]])
    else:
        worst = int(np.argmax(rel))
        assert rel.max() <= tol, (worst, rel[worst], int(n[worst]))
    valid = np.arange(cap)[None, :] < n[:, None]
    eo, eg = rr["err_rec"], E[:, :cap]
    if decision_band is not None:
        dk = np.isin(q["kind"], decision_kinds)[:, None]
        acc = H[:, :cap] > 0
        wrong = (valid & dk & (acc != (eo < 1.0))
                 & (np.abs(eo - 1.0) > decision_band))
        assert not wrong.any(), (np.argwhere(wrong)[:5], eo[wrong][:5],
                                 eg[wrong][:5])
    return dict(rel=rel, e_gpu=eg, e_oracle=eo, valid=valid,
                n_ctl_checked=checked, n_phase=n_phase)


def norm_bias(info, kinds, kind, lo=0.1, hi=10.0):
    """Median relative deviation of the recorded norms from the oracle's over
    the attempts of one kind whose oracle norm lies in [lo, hi] (the norms
    that decide steps)."""
    eo, eg, v = info["e_oracle"], info["e_gpu"], info["valid"]
    m = v & (kinds[:, None] == kind) & (eo >= lo) & (eo <= hi)
    if not m.any():
        return 0.0
    return float(np.median(np.abs(eg[m] - eo[m]) / eo[m]))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grad_errors(p, g, dy0, dth):
    """Relative L2 errors of every parameter tensor (W1 ... b3) separately
    and of every instance's dy0 row, so a wrong small block (a bias, the
    time row of W1, one instance) cannot hide under the norm of the whole
    vector."""
    errs, off = {}, 0
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        size = np.asarray(p["mlp"][k]).size
        errs[k] = rel_l2(g["dth"][off:off + size], dth[off:off + size])
        off += size
    assert off == dth.size
    n_in = np.asarray(p["mlp"]["W1"]).shape[0]  # the time row is the last
    W1g = g["dth"][:np.asarray(p["mlp"]["W1"]).size].reshape(n_in, -1)
    W1r = dth[:W1g.size].reshape(n_in, -1)
    errs["W1_time_row"] = rel_l2(W1g[-1], W1r[-1])
    rows = np.linalg.norm(g["dy0"] - dy0, axis=1) / np.maximum(
        np.linalg.norm(dy0, axis=1), 1e-300)
    errs["dy0_rows"] = float(rows.max())
    errs["dy0"] = rel_l2(g["dy0"], dy0)
    errs["dtheta"] = rel_l2(g["dth"], dth)
    return errs


def assert_grads(p, g, dy0, dth, tol):
    errs = grad_errors(p, g, dy0, dth)
    print("  " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    return errs
