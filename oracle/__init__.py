"""FP64 CPU oracle for the batched adaptive Runge-Kutta solver.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.
"""
from .oracle import (accepted_steps, adjoint, cadjoint,  # noqa: F401
                     dense_weights, initial_step, rhs, solve, solve_joint,
                     tableau)
