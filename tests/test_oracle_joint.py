"""Pins of the oracle's joint (coupled) batch solve, the comparison mode of
paper section 4.1: one step size, one error norm over the stacked vector,
all-or-nothing acceptance."""
import numpy as np
import pytest

import oracle
from paper_2210_12375_amd import workloads as W


@pytest.mark.parametrize("method", ["dopri5", "tsit5"])
def test_one_member_is_the_independent_solve(method):
    """A batch of one is solved exactly as the independent solve solves it
    (bitwise: the stacked norm of one instance is its own norm)."""
    p = W.vdp_batch(B=6)
    for i in range(6):
        q = W.subset(p, np.array([i]))
        a = oracle.solve(q, method=method)
        b = oracle.solve_joint(q, method=method)
        for k in ("n_attempted", "n_accepted", "n_feval", "status"):
            np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a["y_eval"], b["y_eval"])
        np.testing.assert_array_equal(a["y_final"], b["y_final"])


def test_stacked_norm_is_the_rms_over_all_components():
    """Stacking a Van der Pol instance with a zero field of the same size
    (y = 0, f = 0) halves the mean of the squared scaled errors, which is the
    Van der Pol solve with both tolerances scaled by sqrt(2): same steps,
    same solution.  A per-instance norm or a sum instead of a mean would not
    give this."""
    p = W.vdp_batch(B=1)
    D = 8
    pair = W._base(2, D, p["t_eval"].shape[1])
    pair["kind"][:] = [W.VDP, W.LINEAR]
    pair["dim"][:] = [2, 2]
    pair["mu"] = np.full(2, p["mu"][0])
    pair["A"] = np.zeros((2, D, D))
    pair["y0"][0, :2] = p["y0"][0]
    pair["t_end"][:] = p["t_end"][0]
    pair["t_eval"][:] = p["t_eval"][0]
    pair["rtol"][:] = p["rtol"][0]
    pair["atol"][:] = p["atol"][0]
    j = oracle.solve_joint(pair, method="dopri5")
    s = W.subset(p, np.array([0]))
    s["rtol"] = s["rtol"] * np.sqrt(2.0)
    s["atol"] = s["atol"] * np.sqrt(2.0)
    r = oracle.solve(s, method="dopri5")
    assert np.all(j["status"] == 1)
    assert j["n_accepted"][0] == r["n_accepted"][0]
    assert j["n_rejected"][0] == r["n_rejected"][0]
    np.testing.assert_allclose(j["y_eval"][0, :, :2], r["y_eval"][0],
                               rtol=1e-9, atol=1e-12)
    assert np.all(j["y_final"][1, :2] == 0.0)


def test_identical_copies_take_the_single_instance_steps():
    p = W.vdp_batch(B=1)
    four = W.subset(p, np.zeros(4, dtype=np.int64))
    a = oracle.solve(p, method="dopri5")
    b = oracle.solve_joint(four, method="dopri5")
    assert np.all(b["n_accepted"] == a["n_accepted"][0])
    np.testing.assert_allclose(b["y_final"], np.repeat(a["y_final"], 4, 0),
                               rtol=1e-12, atol=1e-14)


def test_members_share_the_span():
    """Instances whose span or evaluation times differ from the first valid
    instance's, and invalid ones, are left out of the joint system."""
    p = W.paper_vdp(B=5, E=4)
    p["t_end"][2] = p["t_end"][2] * 0.5
    p["rtol"][4] = -1.0
    j = oracle.solve_joint(p, method="dopri5")
    np.testing.assert_array_equal(j["status"], [1, 1, 4, 1, 4])
    assert len(set(j["n_attempted"][[0, 1, 3]])) == 1
    assert np.all(np.isnan(j["y_final"][[2, 4], :2]))


def test_stacked_oscillators_need_more_steps():
    """Section 4.1: stacked Van der Pol oscillators at mu = 25 started at
    different phases share the smallest step of the batch at every time, so
    the joint solve needs several times the steps of an independent one."""
    p = W.vdp_phases(B=16, mu=25.0)
    ind = oracle.solve(p, method="dopri5")
    j = oracle.solve_joint(p, method="dopri5")
    assert np.all(ind["status"] == 1) and np.all(j["status"] == 1)
    ratio = j["n_attempted"][0] / ind["n_attempted"].mean()
    assert ratio > 2.0, ratio


def test_joint_record_of_one_member_is_the_independent_record():
    """The joint attempt record (every member's row) of a batch of one is the
    independent solve's record, and every member of a larger joint batch
    carries the same record, whose length is the joint attempt count."""
    p = W.vdp_batch(B=5)
    q = W.subset(p, np.array([2]))
    a = oracle.solve(q, method="dopri5", record_cap=512)
    b = oracle.solve_joint(q, method="dopri5", record_cap=512)
    n = int(a["n_attempted"][0])
    np.testing.assert_array_equal(a["h_rec"][0, :n], b["h_rec"][0, :n])
    r = oracle.solve_joint(W.vdp_phases(B=6, mu=5.0), method="dopri5",
                           record_cap=4096)
    n = int(r["n_attempted"][0])
    assert np.all(r["n_attempted"] == n)
    for i in range(1, 6):
        np.testing.assert_array_equal(r["h_rec"][i, :n], r["h_rec"][0, :n])
    assert np.sum(r["h_rec"][0, :n] > 0) == r["n_accepted"][0]
