"""ctypes binding of libbatchode (include/batchode.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module turns torch
tensors into the C structs, keeps them alive for the handle's lifetime and
forwards the calls with the same names as the C ABI.  There is no fallback:
if the library is missing, `lib()` raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbatchode.so")

DOPRI5, TSIT5 = 0, 1
FP64, FP32, BF16 = 0, 1, 2
RHS_ANALYTIC, RHS_MLP, RHS_CNF = 0, 2, 3
KIND_VDP, KIND_LINEAR = 0, 1
RUNNING, SUCCESS, MAX_STEPS, DT_UNDERFLOW, INVALID = 0, 1, 2, 3, 4
OK, EINVAL, EUNSUPPORTED, EHIP, ESTATE = 0, -1, -2, -3, -4

METHODS = {"dopri5": DOPRI5, "tsit5": TSIT5}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
# Controller presets: integral (the paper's benchmarks, appendix A) and
# Gustafsson's PI controller.
I_CONTROLLER = dict(beta1=0.2, beta2=0.0, beta3=0.0)
PI_CONTROLLER = dict(beta1=0.7 / 5, beta2=0.4 / 5, beta3=0.0)


def pid_gains(k_i, k_p, k_d, order=5):
    """Controller exponents (beta1, beta2, beta3) of a PID law on the log of
    the error norm with gains (k_i, k_p, k_d)."""
    return dict(beta1=(k_i + k_p + k_d) / order, beta2=(k_p + 2 * k_d) / order,
                beta3=-k_d / order)

EXPORTED = ["solver_workspace_size", "solver_init", "solver_step",
            "solver_solve", "solver_eval", "solver_backward",
            "solver_cadjoint_workspace_bytes", "solver_cadjoint",
            "solver_get_stats", "solver_get_steps", "solver_autotune",
            "solver_destroy", "solver_last_error", "solver_tableau",
            "solver_solve_noalloc", "solver_get_errors", "solver_get_tune"]


class Config(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32),
                ("rhs", C.c_int32), ("B", C.c_int32), ("D", C.c_int32),
                ("E", C.c_int32), ("max_steps", C.c_int32),
                ("beta1", C.c_double), ("beta2", C.c_double),
                ("safety", C.c_double), ("fac_min", C.c_double),
                ("fac_max", C.c_double), ("record_cap", C.c_int32),
                ("keep_dense", C.c_int32), ("mlp_hidden", C.c_int32),
                ("tune_block", C.c_int32), ("tune_lanes", C.c_int32),
                ("ckpt_every", C.c_int32), ("beta3", C.c_double),
                ("joint", C.c_int32), ("eager", C.c_int32),
                ("fixed_step", C.c_int32), ("plain_bf16", C.c_int32)]


_PROBLEM_FIELDS = ["y0", "t0", "t_end", "rtol", "atol", "t_eval", "h0", "kind",
                   "dim", "mu", "A", "W1", "b1", "W2", "b2", "W3", "b3", "eps",
                   "y_eval", "y_final"]


class Problem(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _PROBLEM_FIELDS]


class BodeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"batchode error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, cp, ip, dp = C.c_void_p, C.POINTER(Config), C.c_void_p, C.c_void_p
        L.solver_workspace_size.restype = C.c_size_t
        L.solver_workspace_size.argtypes = [cp]
        L.solver_init.restype = C.c_int
        L.solver_init.argtypes = [cp, C.POINTER(Problem), vp, C.c_size_t, vp,
                                  C.POINTER(vp)]
        L.solver_step.restype = C.c_int
        L.solver_step.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        L.solver_solve.restype = C.c_int
        L.solver_solve.argtypes = [vp]
        L.solver_eval.restype = C.c_int
        L.solver_eval.argtypes = [vp, dp, vp, ip]
        L.solver_backward.restype = C.c_int
        L.solver_backward.argtypes = [vp, vp, vp, vp, vp]
        L.solver_cadjoint_workspace_bytes.restype = C.c_size_t
        L.solver_cadjoint_workspace_bytes.argtypes = [vp, C.c_int32]
        L.solver_cadjoint.restype = C.c_int
        L.solver_cadjoint.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_size_t,
                                      vp, vp, vp]
        L.solver_get_stats.restype = C.c_int
        L.solver_get_stats.argtypes = [vp, ip, ip, ip, ip, ip]
        L.solver_get_steps.restype = C.c_int
        L.solver_get_steps.argtypes = [vp, dp, ip]
        L.solver_get_tune.restype = C.c_int
        L.solver_get_tune.argtypes = [cp, vp]
        L.solver_get_errors.restype = C.c_int
        L.solver_get_errors.argtypes = [vp, dp]
        L.solver_autotune.restype = C.c_int
        L.solver_autotune.argtypes = [cp, C.POINTER(Problem), vp, C.c_size_t,
                                      vp]
        L.solver_destroy.restype = None
        L.solver_destroy.argtypes = [vp]
        L.solver_last_error.restype = C.c_char_p
        L.solver_last_error.argtypes = [vp]
        L.solver_solve_noalloc.restype = C.c_int
        L.solver_solve_noalloc.argtypes = [cp, C.POINTER(Problem), ip, vp]
        L.solver_tableau.restype = C.c_int
        L.solver_tableau.argtypes = [C.c_int32, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != OK:
        msg = lib().solver_last_error(handle).decode(errors="replace")
        raise BodeError(rc, msg)


def make_config(B, D, E=0, method="dopri5", precision="fp64",
                rhs=RHS_ANALYTIC, max_steps=100000, beta1=PI_CONTROLLER["beta1"],
                beta2=PI_CONTROLLER["beta2"], safety=0.9, fac_min=0.2,
                fac_max=10.0, record_cap=0, keep_dense=0, mlp_hidden=0,
                tune_block=0, tune_lanes=0, ckpt_every=0, beta3=0.0,
                joint=0, eager=0, fixed_step=0, plain_bf16=0):
    c = Config()
    c.method = METHODS[method] if isinstance(method, str) else method
    c.precision = (PRECISIONS[precision] if isinstance(precision, str)
                   else precision)
    c.rhs, c.B, c.D, c.E, c.max_steps = rhs, B, D, E, max_steps
    c.beta1, c.beta2, c.safety = beta1, beta2, safety
    c.fac_min, c.fac_max = fac_min, fac_max
    c.record_cap, c.keep_dense, c.mlp_hidden = record_cap, keep_dense, mlp_hidden
    c.tune_block, c.tune_lanes = tune_block, tune_lanes
    c.ckpt_every = ckpt_every
    c.beta3 = beta3
    c.joint = joint
    c.eager = eager
    c.fixed_step = fixed_step
    c.plain_bf16 = plain_bf16
    return c


# ---- thin wrappers with the C names ----------------------------------------

def solver_workspace_size(cfg):
    return lib().solver_workspace_size(C.byref(cfg))


def solver_init(cfg, prob, workspace_ptr, workspace_bytes, stream_ptr):
    h = C.c_void_p()
    rc = lib().solver_init(C.byref(cfg), C.byref(prob), workspace_ptr,
                           workspace_bytes, stream_ptr, C.byref(h))
    _check(rc)
    return h


def solver_step(h, n_attempts, want_running=False):
    n = C.c_int32(-1)
    rc = lib().solver_step(h, n_attempts, C.byref(n) if want_running else None)
    _check(rc, h)
    return n.value if want_running else None


def solver_solve(h):
    _check(lib().solver_solve(h), h)


def solver_solve_noalloc(cfg, prob, stats_ptr, stream_ptr):
    _check(lib().solver_solve_noalloc(C.byref(cfg), C.byref(prob), stats_ptr,
                                      stream_ptr))


def solver_eval(h, t_query_ptr, y_out_ptr, qstatus_ptr):
    _check(lib().solver_eval(h, t_query_ptr, y_out_ptr, qstatus_ptr), h)


def solver_backward(h, g_eval_ptr, g_final_ptr, dy0_ptr, dtheta_ptr):
    _check(lib().solver_backward(h, g_eval_ptr, g_final_ptr, dy0_ptr,
                                 dtheta_ptr), h)


def solver_cadjoint_workspace_bytes(h, joint):
    return int(lib().solver_cadjoint_workspace_bytes(h, int(joint)))


def solver_cadjoint(h, joint, g_eval_ptr, g_final_ptr, ws_ptr, ws_bytes,
                    dy0_ptr, dtheta_ptr, stats_ptr):
    _check(lib().solver_cadjoint(h, int(joint), g_eval_ptr, g_final_ptr,
                                 ws_ptr, ws_bytes, dy0_ptr, dtheta_ptr,
                                 stats_ptr), h)


def solver_get_stats(h, *ptrs):
    _check(lib().solver_get_stats(h, *ptrs), h)


def solver_get_steps(h, h_ptr, n_ptr):
    _check(lib().solver_get_steps(h, h_ptr, n_ptr), h)


def solver_get_errors(h, err_ptr):
    _check(lib().solver_get_errors(h, err_ptr), h)


def solver_autotune(cfg, prob, workspace_ptr, workspace_bytes, stream_ptr):
    _check(lib().solver_autotune(C.byref(cfg), C.byref(prob), workspace_ptr,
                                 workspace_bytes, stream_ptr))


TUNE_FIELDS = ("block", "lanes_vdp", "lanes_lin", "waves", "rounds")


def solver_get_tune(cfg):
    """The launch shape solver_init would use for cfg (0: default)."""
    out = (C.c_int32 * 5)()
    _check(lib().solver_get_tune(C.byref(cfg), C.cast(out, C.c_void_p)))
    return dict(zip(TUNE_FIELDS, list(out)))


def solver_destroy(h):
    lib().solver_destroy(h)


def solver_last_error(h=None):
    return lib().solver_last_error(h).decode(errors="replace")


def solver_tableau(method):
    """(c[7], a[7,7], b[7], e[7], dense[7,4]) exactly as the kernels use them."""
    c, a, b, e, d = (np.zeros(7), np.zeros(49), np.zeros(7), np.zeros(7),
                     np.zeros(28))
    m = METHODS[method] if isinstance(method, str) else method
    rc = lib().solver_tableau(m, c.ctypes.data, a.ctypes.data, b.ctypes.data,
                              e.ctypes.data, d.ctypes.data)
    _check(rc)
    return c, a.reshape(7, 7), b, e, d.reshape(7, 4)


# ---- torch-facing helper -----------------------------------------------------

def _state_dtype(precision):
    import torch
    return torch.float64 if precision == "fp64" else torch.float32


def device_problem(p, precision="fp64", device="cuda"):
    """Moves a workload dict (numpy, see workloads.py) to device tensors in
    the layout and dtypes the ABI expects."""
    import torch
    sd = _state_dtype(precision)
    out = {}
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64),
                                    device=device)
    st = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=device).to(sd)
    i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32),
                                    device=device)
    out["y0"] = st(p["y0"])
    for k in ("t0", "t_end", "rtol", "atol"):
        out[k] = f64(np.broadcast_to(p[k], (p["y0"].shape[0],)))
    t_eval = p.get("t_eval")
    out["t_eval"] = f64(t_eval if t_eval is not None
                        else np.zeros((p["y0"].shape[0], 0)))
    if p.get("h0") is not None:
        out["h0"] = f64(p["h0"])
    out["kind"] = i32(p["kind"])
    out["dim"] = i32(p["dim"])
    for k in ("mu", "A", "eps"):
        if p.get(k) is not None:
            out[k] = st(p[k])
    if p.get("mlp") is not None:
        for k, v in p["mlp"].items():
            out[k] = st(v)
    return out


class Solver:
    """One solve: owns the workspace tensor and the C handle."""

    def __init__(self, dp, method="dopri5", precision="fp64", rhs=RHS_ANALYTIC,
                 stream=None, **cfg_kw):
        import torch
        self.torch = torch
        y0 = dp["y0"]
        B, D = y0.shape
        E = dp["t_eval"].shape[1] if dp.get("t_eval") is not None else 0
        if rhs != RHS_ANALYTIC and "mlp_hidden" not in cfg_kw:
            cfg_kw["mlp_hidden"] = dp["W1"].shape[1]
        self.cfg = make_config(B, D, E, method=method, precision=precision,
                               rhs=rhs, **cfg_kw)
        self.B, self.D, self.E = B, D, E
        sd = _state_dtype(precision)
        dev = y0.device
        self.y_eval = torch.empty((B, E, D), dtype=sd, device=dev)
        self.y_final = torch.empty((B, D), dtype=sd, device=dev)
        nbytes = solver_workspace_size(self.cfg)
        if nbytes == 0:
            raise BodeError(EINVAL, "invalid configuration")
        # torch's caching allocator hands out 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.inputs = dict(dp)
        self.prob = Problem()
        for k in _PROBLEM_FIELDS:
            t = self.inputs.get(k)
            if k == "y_eval":
                t = self.y_eval
            elif k == "y_final":
                t = self.y_final
            if k == "t_eval" and E == 0:
                t = None
            setattr(self.prob, k, None if t is None else t.data_ptr())
        self.stream = (stream if stream is not None
                       else torch.cuda.current_stream(dev))
        self.handle = solver_init(self.cfg, self.prob,
                                  self.workspace.data_ptr(), nbytes,
                                  self.stream.cuda_stream)

    def solve(self):
        solver_solve(self.handle)
        return self

    def step(self, n_attempts, want_running=False):
        return solver_step(self.handle, n_attempts, want_running)

    def stats(self):
        torch = self.torch
        out = {k: torch.empty(self.B, dtype=torch.int32,
                              device=self.y_final.device)
               for k in ("n_attempted", "n_accepted", "n_rejected", "n_feval",
                         "status")}
        solver_get_stats(self.handle, *[out[k].data_ptr() for k in
                                        ("n_attempted", "n_accepted",
                                         "n_rejected", "n_feval", "status")])
        return out

    def steps(self):
        torch = self.torch
        cap = self.cfg.record_cap
        h = torch.empty((self.B, cap), dtype=torch.float64,
                        device=self.y_final.device)
        n = torch.empty(self.B, dtype=torch.int32, device=self.y_final.device)
        solver_get_steps(self.handle, h.data_ptr(), n.data_ptr())
        return h, n

    def errors(self):
        """[B, record_cap] error norm of every recorded attempt."""
        torch = self.torch
        e = torch.empty((self.B, self.cfg.record_cap), dtype=torch.float64,
                        device=self.y_final.device)
        solver_get_errors(self.handle, e.data_ptr())
        return e

    def eval(self, t_query):
        torch = self.torch
        y = torch.empty((self.B, self.D), dtype=self.y_final.dtype,
                        device=self.y_final.device)
        q = torch.empty(self.B, dtype=torch.int32, device=self.y_final.device)
        solver_eval(self.handle, t_query.data_ptr(), y.data_ptr(), q.data_ptr())
        return y, q

    def backward(self, g_eval, g_final, n_params):
        torch = self.torch
        dy0 = torch.empty_like(self.y_final)
        dth = torch.empty(n_params, dtype=self.y_final.dtype,
                          device=self.y_final.device)
        solver_backward(self.handle,
                        None if g_eval is None else g_eval.data_ptr(),
                        g_final.data_ptr(), dy0.data_ptr(), dth.data_ptr())
        return dy0, dth

    def cadjoint(self, g_eval, g_final, n_params, joint=False):
        """Continuous adjoint of the completed solve; returns (dy0, dtheta,
        stats [5, B]).  The workspace is allocated here for the call."""
        torch = self.torch
        dev = self.y_final.device
        nb = solver_cadjoint_workspace_bytes(self.handle, joint)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        dy0 = torch.empty_like(self.y_final)
        dth = torch.empty(n_params, dtype=self.y_final.dtype, device=dev)
        st = torch.empty((5, self.B), dtype=torch.int32, device=dev)
        solver_cadjoint(self.handle, joint,
                        None if g_eval is None else g_eval.data_ptr(),
                        g_final.data_ptr(), ws.data_ptr(), nb,
                        dy0.data_ptr(), dth.data_ptr(), st.data_ptr())
        self.stream.synchronize()  # the workspace is freed on return
        return dy0, dth, st

    def close(self):
        if getattr(self, "handle", None) is not None:
            solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
