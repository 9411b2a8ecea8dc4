"""torch.autograd.Function over the C ABI: forward = solver_init +
solver_solve, backward = solver_backward (the discrete adjoint through the
accepted steps, section 4.2 of the paper: training through the solver).

Differentiates with respect to the initial states and the six MLP / CNF
parameter tensors; times, tolerances and probes get no gradient.
"""
import torch

from . import binding as bd

PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")


class ODESolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, W1, b1, W2, b2, W3, b3, fixed, opts):
        dp = dict(fixed)
        dp.update(y0=y0.contiguous(), W1=W1.contiguous(), b1=b1.contiguous(),
                  W2=W2.contiguous(), b2=b2.contiguous(), W3=W3.contiguous(),
                  b3=b3.contiguous())
        s = bd.Solver(dp, **opts)
        s.solve()
        ctx.solver = s
        # The handle borrows these tensors and solver_backward re-reads them;
        # saving them lets torch refuse a backward after an in-place change.
        ctx.save_for_backward(y0, W1, b1, W2, b2, W3, b3)
        ctx.shapes = [t.shape for t in (W1, b1, W2, b2, W3, b3)]
        return s.y_eval.clone(), s.y_final.clone()

    @staticmethod
    def backward(ctx, g_eval, g_final):
        ctx.saved_tensors  # raises if an input was modified in place
        s = ctx.solver
        n = sum(int(torch.Size(sh).numel()) for sh in ctx.shapes)
        if g_eval is None:
            g_eval = torch.zeros_like(s.y_eval)
        if g_final is None:
            g_final = torch.zeros_like(s.y_final)
        dy0, dth = s.backward(g_eval.contiguous() if s.E > 0 else None,
                              g_final.contiguous(), n)
        grads, off = [], 0
        for sh in ctx.shapes:
            k = int(torch.Size(sh).numel())
            grads.append(dth[off:off + k].view(sh))
            off += k
        s.close()
        return (dy0, *grads, None, None)


def odesolve(y0, params, fixed, method="dopri5", precision="fp32",
             rhs=bd.RHS_MLP, record_cap=1024, ckpt_every=2, **kw):
    """(y_eval, y_final) with gradients to y0 and params (a dict W1..b3).

    `fixed` holds the non-differentiable device tensors: t0, t_end, rtol,
    atol, t_eval (and eps for a CNF)."""
    opts = dict(method=method, precision=precision, rhs=rhs,
                record_cap=record_cap, ckpt_every=ckpt_every, **kw)
    return ODESolve.apply(y0, *[params[k] for k in PARAMS], fixed, opts)
