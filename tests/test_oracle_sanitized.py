"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code), run
over its entry points in a child process with the ASan runtime preloaded: every
integration mode (difference-form, complex-step and literal finite-difference JVPs,
fixed steps, forcing, carried steps), the conservative form, the explicit pair, the
quad-precision difference, the projected solve and the linear model problems.  Any
out-of-bounds access, use of freed memory or undefined behaviour aborts the child."""
import os
import subprocess
import sys
import textwrap

import pytest

from conftest import ROOT

CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_1712_00953_amd import synth
    w = synth.workload(1, a_scale=1e-8, n_cells=24)
    st = w.states
    for mode in (O.JVP_FD, O.JVP_COMPLEX, O.JVP_FD_LITERAL):
        r = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, jvp=mode, nthreads=1)
        assert np.all(r[4] == 0)
    O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, fixed_steps=3, nthreads=1)
    dY, dT = O.rhs(w.mech, st.Y, st.T, st.p)
    S = -np.vstack([dY, dT[None]])
    h = np.full(st.n_cells, w.dt / 3)
    O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, S=S, h_io=h, nthreads=1)
    O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, 16, nthreads=1)
    O.integrate_rkdp(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, nthreads=1)
    u = np.concatenate([st.Y[:, 0], [st.T[0]]])
    v = np.linspace(-1.0, 1.0, u.size) / u.size
    O.cell_fdiff(w.mech, u, st.p[0], 1e-7 * v)
    O.cell_fdiff(w.mech, u, st.p[0], 1e-7 * v, quad=True)
    O.cell_arnoldi(w.mech, u, st.p[0], w.M)
    w2 = synth.workload(2, a_scale=1e-8, n_cells=3)
    r = O.integrate(w2.mech, w2.states.Y, w2.states.T, w2.states.p, w2.dt, w2.rtol, w2.atol, w2.M, nthreads=1)
    assert np.all(r[4] == 0)
    vel = np.zeros((3, w2.states.n_cells))
    U = O.cons_state(w2.mech, w2.states.Y, w2.states.T, w2.states.p, vel)
    O.integrate_cons(w2.mech, U, w2.dt, w2.rtol, w2.atol, w2.M, nthreads=1)
    A = np.array([[-3.0, 1.0, 0.5], [0.2, -2.0, 0.1], [0.0, 0.4, -1.5]])
    O.lu_solve(A, np.ones(3))
    O.integrate_linear(A, None, np.ones(3), 1.0, 1e-8, 1e-12, M=2, trace_cap=64)
    O.row_dense_linear(A, None, np.ones(3), 0.1, 4)
    O.rkdp_linear(A, None, np.ones(3), 1.0)
    print("sanitized oracle ok", flush=True)
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    from oracle import oracle as O
    try:
        lib = O.build_sanitized()
        asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no sanitizer toolchain: {e}")
    if not os.path.isabs(asan):
        pytest.skip("libasan not found")
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="1")
    script = tmp_path / "child.py"
    script.write_text(f"ROOT = {ROOT!r}\n" + CHILD)
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
