"""Python binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark import
this module.  The product path (the HIP library and its binding) never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rok4e_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with fused multiply-adds: a second, equally valid rounding of
# every expression.  Comparing the two builds measures how far rounding alone moves the
# method's result (the envelope that GPU-vs-oracle differences are held to).
_LIB_FMA = os.path.join(_HERE, "liboracle_fma.so")
# The same source built with AddressSanitizer and UndefinedBehaviorSanitizer (host code
# only), for the sanitizer test; loaded in place of the plain build when ORACLE_LIB names
# it (the process must have the ASan runtime preloaded).
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")

CXXFLAGS = ["-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
            "-shared", "-fPIC"]
CXXFLAGS_FMA = ["-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=fast", "-mfma", "-fopenmp",
                "-shared", "-fPIC"]
LIBS = ["-lquadmath"]
CXXFLAGS_SAN = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
                "-fopenmp", "-shared", "-fPIC", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

# finite difference (difference form), complex step, exact (linear), finite difference
# evaluated literally as the difference of two rounded right-hand sides
JVP_FD, JVP_COMPLEX, JVP_EXACT, JVP_FD_LITERAL = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile the oracle and its FMA twin with g++ (always recompiles)."""
    for flags, out in ((CXXFLAGS, _LIB), (CXXFLAGS_FMA, _LIB_FMA)):
        cmd = ["g++", *flags, "-o", out + ".tmp", _SRC, *LIBS]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return _LIB


class OrcMech(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("W", C.c_void_p), ("cp", C.c_void_p), ("hf", C.c_void_p),
                ("reac", C.c_void_p), ("prod", C.c_void_p),
                ("lnAf", C.c_void_p), ("bf", C.c_void_p), ("Ef", C.c_void_p),
                ("lnAr", C.c_void_p), ("br", C.c_void_p), ("Er", C.c_void_p)]


class OrcOpts(C.Structure):
    _fields_ = [("M", C.c_int32), ("jvp", C.c_int32), ("fixed_steps", C.c_int32),
                ("max_attempts", C.c_int32), ("eps_fd", C.c_double), ("h0", C.c_double)]


def build_sanitized(verbose: bool = False) -> str:
    """Compile the sanitizer build of the oracle (g++, host code; rebuilt when stale)."""
    if os.path.exists(_LIB_SAN) and os.path.getmtime(_LIB_SAN) >= os.path.getmtime(_SRC):
        return _LIB_SAN
    cmd = ["g++", *CXXFLAGS_SAN, "-o", _LIB_SAN + ".tmp", _SRC, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB_SAN + ".tmp", _LIB_SAN)
    return _LIB_SAN


_lib = None
_lib_fma = None


def lib(fma: bool = False):
    global _lib, _lib_fma
    if _lib is None:
        override = os.environ.get("ORACLE_LIB")
        if override:
            _lib = _lib_fma = C.CDLL(override)
            return _lib
        stale = [p for p in (_LIB, _LIB_FMA)
                 if not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC)]
        if stale:
            build()
        _lib = C.CDLL(_LIB)
        _lib_fma = C.CDLL(_LIB_FMA)
    return _lib_fma if fma else _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class MechHandle:
    """Keeps contiguous copies of the mechanism arrays alive for the C struct."""

    def __init__(self, mech):
        self.arrays = dict(
            W=np.ascontiguousarray(mech.W, np.float64), cp=np.ascontiguousarray(mech.cp, np.float64),
            hf=np.ascontiguousarray(mech.hf, np.float64),
            reac=np.ascontiguousarray(mech.reac, np.int32).reshape(-1),
            prod=np.ascontiguousarray(mech.prod, np.int32).reshape(-1),
            lnAf=np.ascontiguousarray(mech.lnAf, np.float64), bf=np.ascontiguousarray(mech.bf, np.float64),
            Ef=np.ascontiguousarray(mech.Ef, np.float64), lnAr=np.ascontiguousarray(mech.lnAr, np.float64),
            br=np.ascontiguousarray(mech.br, np.float64), Er=np.ascontiguousarray(mech.Er, np.float64))
        self.n_species = int(mech.n_species)
        self.n_reactions = int(mech.n_reactions)
        self.s = OrcMech(self.n_species, self.n_reactions,
                         *[self.arrays[k].ctypes.data for k in
                           ("W", "cp", "hf", "reac", "prod", "lnAf", "bf", "Ef", "lnAr", "br", "Er")])


def coefficients() -> dict:
    out = np.zeros(21)
    lib().orc_coefficients(_p(out), 21)
    names = ["gamma", "g21", "g31", "g32", "g41", "g42", "g43", "a21", "a31", "a32", "a41",
             "a42", "a43", "b1", "b2", "b3", "b4", "bh1", "bh2", "bh3", "bh4"]
    return dict(zip(names, out.tolist()))


def rhs(mech, Y, T, p, S=None):
    """f(u) for every cell; Y [ns, n], T [n], p [n], S [(ns+1), n] or None."""
    h = MechHandle(mech)
    Y = np.ascontiguousarray(Y, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    n = T.shape[0]
    dY = np.zeros_like(Y)
    dT = np.zeros_like(T)
    S = None if S is None else np.ascontiguousarray(S, np.float64)
    lib().orc_rhs(C.byref(h.s), C.c_int64(n), _p(Y), _p(T), _p(p), _p(S), _p(dY), _p(dT))
    return dY, dT


def cell_jvp(mech, u, p, v, mode=JVP_FD, eps_fd=0.0):
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros_like(u)
    rc = lib().orc_cell_jvp(C.byref(h.s), _p(u), C.c_double(p), _p(v), C.c_int(mode),
                            C.c_double(eps_fd), _p(out))
    if rc != 0:
        raise RuntimeError("jvp mode not available")
    return out


def cell_fdiff(mech, u, p, du, quad=False):
    """f(u + du) - f(u) of one cell: difference form, or the quad-precision reference."""
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    du = np.ascontiguousarray(du, np.float64)
    out = np.zeros_like(u)
    fn = lib().orc_cell_fdiff_quad if quad else lib().orc_cell_fdiff
    fn(C.byref(h.s), _p(u), C.c_double(p), _p(du), _p(out))
    return out


def cell_arnoldi(mech, u, p, M, mode=JVP_FD, eps_fd=0.0, fma=False):
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    n = u.shape[0]
    Q = np.zeros((M, n))
    H = np.zeros((M, M))
    meff = lib(fma).orc_cell_arnoldi(C.byref(h.s), _p(u), C.c_double(p), C.c_int(M), C.c_int(mode),
                                  C.c_double(eps_fd), _p(Q), _p(H))
    return Q.T.copy(), H, meff


def make_opts(M, jvp=JVP_FD, fixed_steps=0, max_attempts=0, eps_fd=0.0, h0=0.0):
    return OrcOpts(int(M), int(jvp), int(fixed_steps), int(max_attempts), float(eps_fd), float(h0))


def integrate(mech, Y, T, p, dt, rtol, atol, M, S=None, jvp=JVP_FD, fixed_steps=0,
              max_attempts=0, eps_fd=0.0, h0=0.0, nthreads=0, fma=False, h_io=None):
    """Integrate every cell over [0, dt]; returns (Y, T, accepted, rejected, status)
    as new arrays (inputs untouched).  fma=True runs the FMA-contracted twin build.
    h_io (float64 [n], updated in place): per-cell first trial steps (<= 0: h0 or dt),
    replaced by the step to start the next call from."""
    h = MechHandle(mech)
    Y = np.array(Y, np.float64, order="C", copy=True)
    T = np.array(T, np.float64, copy=True)
    p = np.ascontiguousarray(p, np.float64)
    S = None if S is None else np.ascontiguousarray(S, np.float64)
    n = T.shape[0]
    acc = np.zeros(n, np.int32)
    rej = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    o = make_opts(M, jvp, fixed_steps, max_attempts, eps_fd, h0)
    if h_io is None:
        lib(fma).orc_integrate(C.byref(h.s), C.byref(o), C.c_int64(n), _p(Y), _p(T), _p(p), _p(S),
                               C.c_double(dt), C.c_double(rtol), C.c_double(atol), _p(acc), _p(rej),
                               _p(st), C.c_int(nthreads))
    else:
        assert h_io.dtype == np.float64 and h_io.shape == (n,) and h_io.flags.c_contiguous
        lib(fma).orc_integrate_h(C.byref(h.s), C.byref(o), C.c_int64(n), _p(Y), _p(T), _p(p), _p(S),
                                 C.c_double(dt), C.c_double(rtol), C.c_double(atol), _p(h_io), _p(acc),
                                 _p(rej), _p(st), C.c_int(nthreads))
    return Y, T, acc, rej, st


def integrate_rkdp(mech, Y, T, p, dt, rtol, atol, S=None, fixed_steps=0, max_attempts=0, h0=0.0,
                   nthreads=0, fma=False):
    """The explicit Dormand-Prince 5(4) reference integrator on every cell over [0, dt];
    returns (Y, T, accepted, rejected, status) as new arrays."""
    h = MechHandle(mech)
    Y = np.array(Y, np.float64, order="C", copy=True)
    T = np.array(T, np.float64, copy=True)
    p = np.ascontiguousarray(p, np.float64)
    S = None if S is None else np.ascontiguousarray(S, np.float64)
    n = T.shape[0]
    acc = np.zeros(n, np.int32)
    rej = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    o = make_opts(1, JVP_FD, fixed_steps, max_attempts, 0.0, h0)
    lib(fma).orc_integrate_rkdp(C.byref(h.s), C.byref(o), C.c_int64(n), _p(Y), _p(T), _p(p), _p(S),
                             C.c_double(dt), C.c_double(rtol), C.c_double(atol), _p(acc), _p(rej),
                             _p(st), C.c_int(nthreads))
    return Y, T, acc, rej, st


def rkdp_linear(A, c, u, dt, rtol=1e-6, atol=1e-12, fixed_steps=0):
    """RKDP 5(4) on u' = A u + c; returns (u, accepted, rejected, status)."""
    A = np.ascontiguousarray(A, np.float64)
    c = None if c is None else np.ascontiguousarray(c, np.float64)
    u = np.array(u, np.float64, copy=True)
    acc, rej, st = C.c_int32(), C.c_int32(), C.c_int32()
    o = make_opts(1, JVP_EXACT, fixed_steps, 0, 0.0, 0.0)
    lib().orc_rkdp_linear(C.c_int(A.shape[0]), _p(A), _p(c), C.byref(o), _p(u), C.c_double(dt),
                          C.c_double(rtol), C.c_double(atol), C.byref(acc), C.byref(rej), C.byref(st))
    return u, acc.value, rej.value, st.value


def lu_solve(A, b):
    """A^{-1} b through the oracle's LU with partial pivoting; returns (x, piv)."""
    A = np.ascontiguousarray(A, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    m = A.shape[0]
    x = np.zeros(m)
    piv = np.zeros(m, np.int32)
    rc = lib().orc_lu_solve(C.c_int(m), _p(A), _p(b), _p(x), piv.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != 0:
        raise ZeroDivisionError("zero pivot")
    return x, piv


def rkdp_coefficients() -> dict:
    out = np.zeros(30)
    lib().orc_rkdp_coefficients(_p(out))
    names = ["c2", "c3", "c4", "c5", "a21", "a31", "a32", "a41", "a42", "a43", "a51", "a52", "a53", "a54",
             "a61", "a62", "a63", "a64", "a65", "b1", "b3", "b4", "b5", "b6", "bh1", "bh3", "bh4", "bh5",
             "bh6", "bh7"]
    return dict(zip(names, out.tolist()))


def integrate_linear(A, c, u, dt, rtol, atol, M, jvp=JVP_EXACT, fixed_steps=0, max_attempts=0,
                     h0=0.0, trace_cap=0):
    """ROK4E on u' = A u + c.  Returns (u, accepted, rejected, status) and, when
    ``trace_cap`` > 0, a fifth item: the [attempts, 4] trace (t, h, err, accepted)."""
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    c = None if c is None else np.ascontiguousarray(c, np.float64)
    u = np.array(u, np.float64, copy=True)
    acc, rej, st, ntr = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    o = make_opts(M, jvp, fixed_steps, max_attempts, 0.0, h0)
    tr = np.zeros((max(trace_cap, 1), 4))
    lib().orc_integrate_linear(C.c_int(n), _p(A), _p(c), C.byref(o), _p(u), C.c_double(dt),
                               C.c_double(rtol), C.c_double(atol), C.byref(acc), C.byref(rej),
                               C.byref(st), _p(tr) if trace_cap > 0 else None, C.c_int(trace_cap),
                               C.byref(ntr))
    if trace_cap > 0:
        return u, acc.value, rej.value, st.value, tr[:min(ntr.value, trace_cap)].copy()
    return u, acc.value, rej.value, st.value


def row_dense_linear(A, c, u, dt, nsteps, jvp=JVP_EXACT):
    A = np.ascontiguousarray(A, np.float64)
    c = None if c is None else np.ascontiguousarray(c, np.float64)
    u = np.array(u, np.float64, copy=True)
    rc = lib().orc_row_dense_linear(C.c_int(A.shape[0]), _p(A), _p(c), _p(u), C.c_double(dt),
                                    C.c_int(nsteps), C.c_int(jvp))
    if rc != 0:
        raise RuntimeError(f"row_dense_linear failed: {rc}")
    return u


def row_dense_cell(mech, u, p, dt, nsteps, jvp=JVP_COMPLEX):
    h = MechHandle(mech)
    u = np.array(u, np.float64, copy=True)
    rc = lib().orc_row_dense_cell(C.byref(h.s), _p(u), C.c_double(p), C.c_double(dt),
                                  C.c_int(nsteps), C.c_int(jvp))
    if rc != 0:
        raise RuntimeError(f"row_dense_cell failed: {rc}")
    return u


# ------------------------------------------------ conservative variables (Sec. 5) ----

def cons_state(mech, Y, T, p, vel):
    """Conservative variables [(ns+5), n] (rho Y_k, rho, rho u_x, rho u_y, rho u_z, rho E)
    of the states (Y, T, p) moving with velocity vel [3, n]: ideal gas rho = p / (Ru T
    sum Y_k/W_k), internal energy e = sum_k Y_k (h_k - Ru T / W_k) with
    h_k = h_f,k + c_p,k (T - 298.15), E = e + |vel|^2 / 2."""
    Ru = 8.314462618
    W = np.asarray(mech.W, np.float64)[:, None]
    cp = np.asarray(mech.cp, np.float64)[:, None]
    hf = np.asarray(mech.hf, np.float64)[:, None]
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.float64)
    vel = np.asarray(vel, np.float64)
    rho = np.asarray(p, np.float64) / (Ru * T * (Y / W).sum(0))
    e = (Y * (hf + cp * (T - 298.15) - Ru * T / W)).sum(0)
    E = e + 0.5 * (vel * vel).sum(0)
    return np.ascontiguousarray(np.vstack([rho * Y, rho[None], rho * vel, (rho * E)[None]]))


def cons_temperature(mech, U):
    """Temperature of the conservative variables of every cell (NaN where rho c_v <= 0)."""
    h = MechHandle(mech)
    U = np.ascontiguousarray(U, np.float64)
    n = U.shape[1]
    T = np.zeros(n)
    lib().orc_cons_temperature(C.byref(h.s), C.c_int64(n), _p(U), _p(T))
    return T


def cons_f(mech, u, s=None):
    """f of one cell in the auxiliary-temperature state u (length ns+6)."""
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    s = None if s is None else np.ascontiguousarray(s, np.float64)
    out = np.zeros_like(u)
    lib().orc_cons_f(C.byref(h.s), _p(u), _p(s), _p(out))
    return out


def cons_fdiff(mech, u, du, s=None, quad=False):
    """f(u + du) - f(u) of one auxiliary-temperature cell: difference form, or the
    quad-precision reference."""
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    du = np.ascontiguousarray(du, np.float64)
    s = None if s is None else np.ascontiguousarray(s, np.float64)
    out = np.zeros_like(u)
    lib().orc_cons_fdiff(C.byref(h.s), _p(u), _p(s), _p(du), C.c_int(1 if quad else 0), _p(out))
    return out


def cons_jvp(mech, u, v, s=None, mode=JVP_FD):
    """J(u) v of one auxiliary-temperature cell (FD in difference form, or complex step)."""
    h = MechHandle(mech)
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    s = None if s is None else np.ascontiguousarray(s, np.float64)
    out = np.zeros_like(u)
    if lib().orc_cons_jvp(C.byref(h.s), _p(u), _p(s), _p(v), C.c_int(mode), _p(out)) != 0:
        raise RuntimeError("jvp mode not available")
    return out


def integrate_cons(mech, U, dt, rtol, atol, M, S=None, jvp=JVP_FD, fixed_steps=0,
                   max_attempts=0, nthreads=0, fma=False):
    """Reaction substep in conservative variables with the auxiliary temperature over
    [0, dt]; returns (U, T_aux, accepted, rejected, status) as new arrays.  T_aux is NaN
    for cells with invalid input."""
    h = MechHandle(mech)
    U = np.array(U, np.float64, order="C", copy=True)
    S = None if S is None else np.ascontiguousarray(S, np.float64)
    n = U.shape[1]
    Ta = np.full(n, np.nan)
    acc = np.zeros(n, np.int32)
    rej = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    o = make_opts(M, jvp, fixed_steps, max_attempts, 0.0, 0.0)
    lib(fma).orc_integrate_cons(C.byref(h.s), C.byref(o), C.c_int64(n), _p(U), _p(S), C.c_double(dt),
                                C.c_double(rtol), C.c_double(atol), _p(Ta), _p(acc), _p(rej), _p(st),
                                C.c_int(nthreads))
    return U, Ta, acc, rej, st
