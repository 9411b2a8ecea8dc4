"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's C sources are built a third time with -fsanitize=address,
undefined and -fno-sanitize-recover=all; a child process with the
sanitizer runtimes preloaded runs its entry points (solves of every
right-hand side, replays with diagnostics, the joint mode, both adjoints,
edge cases and invalid instances), so any out-of-bounds access, use of
freed memory, signed overflow or misaligned load aborts the child.  Its
results must equal the plain build's bitwise (the sanitizers change no
floating-point operation: both builds keep every multiply-add as written).
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent('''
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    from oracle import oracle as O
    from paper_2210_12375_amd import workloads as W
    if MODE == "san":
        O._lib = O._load("san")  # every entry point below uses it
    out = {}
    def keep(tag, r):
        for k, v in r.items():
            if isinstance(v, np.ndarray):
                out[tag + "/" + k] = v
    p = W.vdp_batch()
    keep("vdp", oracle.solve(p, method="dopri5", record_cap=512))
    q = W.uneven_batch(B=300)
    q["t_end"][3] = q["t0"][3]
    q["t_eval"][3] = 0.0
    q["t_eval"][7, 4] = -1.0          # invalid instance
    q["y0"][9, 0] = np.nan           # invalid instance
    r = oracle.solve(q, method="tsit5", record_cap=2048)
    keep("uneven", r)
    n = r["n_attempted"]
    h = np.nan_to_num(r["h_rec"][:, :max(1, int(n.max()))])
    keep("replay", oracle.solve(q, method="tsit5", h_replay=h, n_replay=n,
                                replay_errors=True))
    keep("maxsteps", oracle.solve(q, method="dopri5", max_steps=3))
    keep("probe", oracle.solve(q, method="dopri5", h_replay=h, n_replay=n,
                               round_state_f32="stages"))
    keep("joint", oracle.solve_joint(W.vdp_phases(B=8, mu=5.0),
                                     method="dopri5"))
    m = W.neural_ode_fit(B=6, d=16, hidden=32, n_times=3)
    rm = oracle.solve(m, method="dopri5", record_cap=64)
    keep("mlp", rm)
    hh, nn = oracle.accepted_steps(rm["h_rec"], rm["n_attempted"])
    rng = np.random.default_rng(0)
    ge = rng.standard_normal(rm["y_eval"].shape)
    gf = rng.standard_normal(rm["y_final"].shape)
    dy0, dth = oracle.adjoint(m, hh, nn, ge, gf, method="dopri5")
    out["adj/dy0"], out["adj/dth"] = dy0, dth
    for joint in (False, True):
        ca = oracle.cadjoint(m, rm["y_final"], rm["status"], ge, gf,
                             joint=joint, method="dopri5")
        keep(f"cadj{int(joint)}", ca)
    c = W.cnf_density(B=5, d=8, hidden=16)
    rc = oracle.solve(c, method="tsit5", record_cap=64)
    keep("cnf", rc)
    hh, nn = oracle.accepted_steps(rc["h_rec"], rc["n_attempted"])
    dy0, dth = oracle.adjoint(c, hh, nn, None, np.ones_like(rc["y_final"]),
                              method="tsit5")
    out["cnfadj/dy0"], out["cnfadj/dth"] = dy0, dth
    np.savez(OUT, **out)
    print("child done", len(out), flush=True)
''')


def run_child(mode, out, env):
    code = f"ROOT = {ROOT!r}\nMODE = {mode!r}\nOUT = {out!r}\n" + CHILD
    return subprocess.run([sys.executable, "-c", code], env=env,
                          capture_output=True, text=True, timeout=600)


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    from oracle import build
    build.build_sanitized()
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["gcc", f"-print-file-name={name}"],
                              capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(path) or not os.path.exists(path):
            pytest.skip(f"{name} is not installed")
        libs.append(path)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    plain = run_child("plain", str(tmp_path / "plain.npz"), env)
    assert plain.returncode == 0, plain.stderr[-3000:]
    senv = dict(env, LD_PRELOAD=":".join(libs),
                ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    san = run_child("san", str(tmp_path / "san.npz"), senv)
    assert san.returncode == 0, san.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in san.stderr
    assert "runtime error" not in san.stderr
    a = np.load(tmp_path / "plain.npz")
    b = np.load(tmp_path / "san.npz")
    assert sorted(a.files) == sorted(b.files) and len(a.files) > 30
    for k in a.files:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_host_argument_checks_under_sanitizers(tmp_path):
    """The library's host code (argument and configuration checks of every
    entry point) built with AddressSanitizer and UndefinedBehaviorSanitizer
    on the host side only (device code as usual) and linked with
    tests/host_checks.cpp, whose calls all fail validation before any HIP
    call: no sanitizer report, every expected error code."""
    import concurrent.futures as cf
    import shlex
    csrc = os.path.join(ROOT, "paper_2210_12375_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc)
                  if f.endswith((".hip", ".cpp")))
    srcs.append(os.path.join(ROOT, "tests", "host_checks.cpp"))
    base = shlex.split(
        "/opt/rocm/bin/hipcc -std=c++17 -O1 --offload-arch=gfx950 "
        "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
        "-Xarch_host -fno-sanitize-recover=all "
        "-Xarch_host -fno-omit-frame-pointer -Wno-unused-command-line-argument")
    inc = ["-I" + os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run(base + inc + ["-c", src, "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_checks")
    r = subprocess.run(base + objs + ["-o", exe], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    run = subprocess.run([exe], capture_output=True, text=True, env=env,
                         timeout=300)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-2000:])
    assert "host checks: 0 failures" in run.stdout
    assert "runtime error" not in run.stderr
