"""Pins of the oracle's tableaux and continuous extensions.

The paper names the methods (appendix A: dopri5 and tsit5) but prints no
coefficients, so the pins are the Runge-Kutta order conditions themselves
(Butcher trees up to order 5), which a wrong digit, sign or index in any
coefficient breaks, plus scipy's independent copy of the Dormand-Prince
dense-output matrix.
"""
import numpy as np
import pytest

import oracle

METHODS = ["dopri5", "tsit5"]


def trees(c, A):
    """(Phi(tree) vector over stages, order, density gamma) for all rooted
    trees of order <= 5."""
    one = np.ones(7)
    Ac = A @ c
    Ac2 = A @ (c * c)
    AAc = A @ Ac
    return [
        (one, 1, 1),
        (c, 2, 2),
        (c**2, 3, 3), (Ac, 3, 6),
        (c**3, 4, 4), (c * Ac, 4, 8), (Ac2, 4, 12), (AAc, 4, 24),
        (c**4, 5, 5), (c**2 * Ac, 5, 10), (c * Ac2, 5, 15), (c * AAc, 5, 30),
        (Ac * Ac, 5, 20), (A @ c**3, 5, 20), (A @ (c * Ac), 5, 40),
        (A @ Ac2, 5, 60), (A @ AAc, 5, 120),
    ]


@pytest.mark.parametrize("method", METHODS)
def test_row_sums_and_fsal(method):
    c, A, b, bh = oracle.tableau(method)
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-15)
    assert np.all(np.triu(A) == 0.0)  # explicit
    np.testing.assert_array_equal(A[6], b)  # FSAL / SSAL
    assert c[6] == 1.0 and c[0] == 0.0 and b[6] == 0.0


@pytest.mark.parametrize("method", METHODS)
def test_order_conditions(method):
    c, A, b, bh = oracle.tableau(method)
    for phi, order, gamma in trees(c, A):
        assert abs(b @ phi - 1.0 / gamma) < 2e-15, (order, gamma)
        if order <= 4:
            assert abs(bh @ phi - 1.0 / gamma) < 2e-15, (order, gamma)
    # the embedded method is genuinely only of order 4
    worst = max(abs(bh @ phi - 1.0 / g) for phi, o, g in trees(c, A) if o == 5)
    assert worst > 1e-4
    assert abs((b - bh).sum()) < 1e-15


def test_dopri5_stability_polynomial_closed_form():
    """R(z) = 1 + sum_k (b^T A^(k-1) 1) z^k: Dormand-Prince has
    1, 1, 1/2, 1/6, 1/24, 1/120, 1/600 and no z^7 term."""
    c, A, b, bh = oracle.tableau("dopri5")
    coeff = [b @ np.linalg.matrix_power(A, k - 1) @ np.ones(7)
             for k in range(1, 8)]
    expect = [1, 1 / 2, 1 / 6, 1 / 24, 1 / 120, 1 / 600, 0.0]
    np.testing.assert_allclose(coeff, expect, rtol=0, atol=2e-15)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("theta", [0.1, 1 / 3, 0.5, 0.7, 0.95])
def test_dense_output_order_conditions(method, theta):
    c, A, b, bh = oracle.tableau(method)
    w = oracle.dense_weights(method, theta)
    for phi, order, gamma in trees(c, A):
        if order <= 4:
            assert abs(w @ phi - theta**order / gamma) < 5e-15, (order, gamma)


@pytest.mark.parametrize("method", METHODS)
def test_dense_output_ends(method):
    c, A, b, bh = oracle.tableau(method)
    np.testing.assert_allclose(oracle.dense_weights(method, 0.0), 0.0, atol=0)
    np.testing.assert_allclose(oracle.dense_weights(method, 1.0), b,
                               atol=1e-15)
    # derivative at theta = 0 is the first stage (y'(t_n) = k_1)
    d = 1e-7
    w0 = (oracle.dense_weights(method, d) - oracle.dense_weights(method, -d))
    np.testing.assert_allclose(w0 / (2 * d), np.eye(7)[0], atol=1e-7)


def test_dopri5_dense_is_hermite_at_the_end():
    d = 1e-7
    w1 = (oracle.dense_weights("dopri5", 1 + d)
          - oracle.dense_weights("dopri5", 1 - d))
    np.testing.assert_allclose(w1 / (2 * d), np.eye(7)[6], atol=1e-7)


def test_dopri5_dense_matches_scipy_P():
    """scipy's RK45 stores the same continuous extension as a 7x4 matrix P
    with w_j(theta) = sum_m P[j, m] theta^(m+1)."""
    from scipy.integrate._ivp.rk import RK45
    P = RK45.P
    for theta in np.linspace(0, 1, 11):
        w_scipy = P @ (theta ** np.arange(1, 5))
        np.testing.assert_allclose(oracle.dense_weights("dopri5", theta),
                                   w_scipy, atol=2e-15)


def test_dopri5_matches_scipy_tableau():
    from scipy.integrate._ivp.rk import RK45
    c, A, b, bh = oracle.tableau("dopri5")
    np.testing.assert_allclose(c[:6], RK45.C, atol=0)
    np.testing.assert_allclose(A[:6, :5], RK45.A, atol=0)
    np.testing.assert_allclose(b[:6], RK45.B, atol=0)
    # scipy's error weights are bhat - b
    np.testing.assert_allclose(bh - b, RK45.E, atol=2e-17)
