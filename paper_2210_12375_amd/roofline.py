"""Algorithmic work of the solver, for roofline fractions.

Counts follow the arithmetic each step needs, independent of how a kernel
schedules it: a fused multiply-add is 2 flops, every other add, multiply,
divide, square root, max or power is 1.  Coefficients that are zero in a
tableau (Dormand-Prince's b_2, e_2, ...) are not counted.

Per attempted step of an instance of true dimension n, with nnz(a) nonzero
stage coefficients a_sj (s = 2..7), nnz(e) nonzero error weights:
  stage combination   n * (2 nnz(a) + 2 * 6)        (acc, then y + h acc)
  right-hand side     6 * f(n)                      (6 new stages, FSAL)
  error estimate      n * (2 nnz(e) + 1)
  weighted RMS norm   n * 6 + 2                     (scale, divide, square,
                                                     accumulate; mean, sqrt)
  controller          6                             (power, products, clamp)
Right-hand sides: Van der Pol f = 5 flops; linear f = 2 n^2; the MLP
2 (65*256 + 256*256 + 256*64) + tanh per hidden unit (as 1 flop).
Dense output per emitted point: 4 * 2 * 7 (Horner weights) + n (2 * 7 + 2).
"""
import numpy as np

from .binding import solver_tableau

VDP_FLOPS = 5


def _nnz(method):
    c, a, b, e, P = solver_tableau(method)
    return int(np.count_nonzero(a[1:])), int(np.count_nonzero(e))


def flops_per_attempt(method, n, rhs_flops):
    nnz_a, nnz_e = _nnz(method)
    return (n * (2 * nnz_a + 12) + 6 * rhs_flops + n * (2 * nnz_e + 1)
            + 6 * n + 2 + 6)


def dense_flops(n):
    return 4 * 2 * 7 + n * (2 * 7 + 2)


def analytic_flops(method, kind, dim, n_attempted, n_emitted):
    """Total algorithmic flops of an analytic batch (per-instance arrays)."""
    kind = np.asarray(kind)
    dim = np.asarray(dim)
    n_attempted = np.asarray(n_attempted, dtype=np.float64)
    rhs = np.where(kind == 0, VDP_FLOPS, 2 * dim * dim)
    per = np.zeros(kind.shape, dtype=np.float64)
    dns = np.zeros(kind.shape, dtype=np.float64)
    for d, f in set(zip(dim.tolist(), rhs.tolist())):
        m = (dim == d) & (rhs == f)
        per[m] = flops_per_attempt(method, d, f)
        dns[m] = dense_flops(d)
    return float((per * n_attempted).sum()
                 + (np.asarray(n_emitted, dtype=np.float64) * dns).sum())


def mlp_flops_per_row(d, hidden):
    macs = (d + 1) * hidden + hidden * hidden + hidden * d
    return 2 * macs + 2 * hidden


# MI355X published peaks.
PEAK = {"fp64_vector_tflops": 78.6, "fp32_vector_tflops": 157.3,
        "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0}
