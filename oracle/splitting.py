"""Splitting drivers around the oracle's ROK4E (test infrastructure only).

The Simpler balanced splitting, Sec. 3.3 eq. e:simpler_balanced, for a system
u' = T(u) + R(u): with c_n = -T(u_n), integrate u' = R(u) - c_n over h with ROK4E
(the stiff reaction substep), then u' = T(u) + c_n over h/2 with an explicit
Runge-Kutta method (the non-stiff transport substep; the first transport half step of
the balanced form is identically at rest and is dropped).  Strang splitting,
e:strang_t1..e:strang_t3, is the control that does not preserve steady states.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import oracle as O

_FN = C.CFUNCTYPE(None, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


def rok4e(f, u0, h, rtol=1e-10, atol=1e-14, M=None):
    """ROK4E (finite-difference JVPs) on u' = f(u) over [0, h]."""
    u = np.array(u0, np.float64, copy=True)
    n = u.shape[0]

    def cb(nn, up, outp, ctx):
        uu = np.ctypeslib.as_array(up, shape=(nn,))
        out = np.ctypeslib.as_array(outp, shape=(nn,))
        out[:] = f(uu.copy())

    fn = _FN(cb)
    acc, rej, st = C.c_int32(), C.c_int32(), C.c_int32()
    o = O.make_opts(M if M is not None else n)
    O.lib().orc_integrate_callback(C.c_int(n), fn, None, C.byref(o), O._p(u), C.c_double(h),
                                   C.c_double(rtol), C.c_double(atol), C.byref(acc),
                                   C.byref(rej), C.byref(st))
    if st.value != 0:
        raise RuntimeError(f"ROK4E substep failed with status {st.value}")
    return u


def rk4(f, u0, h, nsub=8):
    """Classical 4th-order Runge-Kutta with nsub equal steps (transport substeps)."""
    u = np.array(u0, np.float64, copy=True)
    dt = h / nsub
    for _ in range(nsub):
        k1 = f(u)
        k2 = f(u + 0.5 * dt * k1)
        k3 = f(u + 0.5 * dt * k2)
        k4 = f(u + dt * k3)
        u = u + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u


def simpler_step(T, R, u, h, reaction=rok4e, transport=rk4):
    c = -T(u)                                            # c_n = -T(U_n)
    u1 = reaction(lambda v: R(v) - c, u, h)              # reaction substep over h
    return transport(lambda v: T(v) + c, u1, 0.5 * h)    # transport over h/2


def strang_step(T, R, u, h, reaction=rok4e, transport=rk4):
    u1 = transport(T, u, 0.5 * h)
    u2 = reaction(R, u1, h)
    return transport(T, u2, 0.5 * h)


# ---- grid form: the reaction substep per cell, the model transport operator on a grid ----

def transport_grid(U, nx, ny, nz, dx, vel, diff, inflow=None):
    """The model transport operator on an nx x ny x nz grid (cell c = x + nx (y + ny z)):
    advection with velocity vel along x and isotropic diffusion, second-order central
    differences, for every row of U [N, n].  y and z are periodic.  x is periodic when
    inflow is None; otherwise the x-neighbour before the first cell is the ghost value
    inflow[r] of row r and the x-neighbour after the last cell is that cell (zero-gradient
    outflow)."""
    N = U.shape[0]
    V = U.reshape(N, nz, ny, nx)
    if inflow is None:
        xp, xm = np.roll(V, -1, axis=3), np.roll(V, 1, axis=3)
    else:
        ghost = np.broadcast_to(np.asarray(inflow, np.float64).reshape(N, 1, 1, 1), (N, nz, ny, 1))
        xm = np.concatenate([ghost, V[..., :-1]], axis=3)
        xp = np.concatenate([V[..., 1:], V[..., -1:]], axis=3)
    yp, ym = np.roll(V, -1, axis=2), np.roll(V, 1, axis=2)
    zp, zm = np.roll(V, -1, axis=1), np.roll(V, 1, axis=1)
    adv = -vel * (xp - xm) / (2.0 * dx)
    dif = diff * (xm + xp + ym + yp + zm + zp - 6.0 * V) / (dx * dx)
    return (adv + dif).reshape(N, -1)


def _rows(Y, T):
    return np.vstack([np.asarray(Y, np.float64), np.asarray(T, np.float64)[None, :]])


def _transport_substep(U, grid, h, nsub, s0=None):
    """u' = T(u) - s0 over h with nsub classical Runge-Kutta steps (s0 = None: 0)."""
    N, n = U.shape

    def f(v):
        t = transport_grid(v.reshape(N, n), *grid)
        return (t if s0 is None else t - s0).reshape(-1)

    return rk4(f, U.reshape(-1), h, nsub).reshape(N, n)


def simpler_step_grid(mech, Y, T, p, grid, h, rtol, atol, M, src=None, nsub=1, **kw):
    """One Simpler balanced splitting step on the grid (e:simpler_balanced): c_n = -T(U_n);
    the reaction substep u' = R(u) + src - c_n over h, cell by cell with the oracle's
    ROK4E; the transport substep u' = T(u) + c_n over h/2.  grid = (nx, ny, nz, dx, vel,
    diff) for a periodic grid, or with a seventh entry, the inflow ghost state, for a grid
    open along x.  Returns (Y, T, accepted, rejected, status)."""
    U = _rows(Y, T)
    s0 = transport_grid(U, *grid)
    F = s0 if src is None else s0 + src
    Yr, Tr, acc, rej, st = O.integrate(mech, U[:-1], U[-1], p, h, rtol, atol, M, S=F, **kw)
    U2 = _transport_substep(_rows(Yr, Tr), grid, 0.5 * h, nsub, s0)
    return U2[:-1], U2[-1], acc, rej, st


def strang_step_grid(mech, Y, T, p, grid, h, rtol, atol, M, src=None, nsub=1, **kw):
    """Strang splitting on the grid (e:strang_t1..e:strang_t3): transport over h/2,
    reaction u' = R(u) + src over h, transport over h/2."""
    U1 = _transport_substep(_rows(Y, T), grid, 0.5 * h, nsub)
    Yr, Tr, acc, rej, st = O.integrate(mech, U1[:-1], U1[-1], p, h, rtol, atol, M, S=src, **kw)
    U2 = _transport_substep(_rows(Yr, Tr), grid, 0.5 * h, nsub)
    return U2[:-1], U2[-1], acc, rej, st
