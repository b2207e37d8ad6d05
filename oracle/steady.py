"""Discrete steady states of the model reacting flow on a grid open along x.

Test infrastructure only: it computes inputs for the splitting tests and is never imported
by the product path.

Sec. 3.3 calls a splitting steady-state preserving (definition d:steady_state_preserving)
when a state at which the full right-hand side vanishes is mapped to itself for every step
size.  On the grid problem u' = T(u) + R(u) that needs a state U_s with
T(U_s) + R(U_s) = 0.  On a periodic grid with uniform advection the only such states of a
reacting mixture are uniform, but on a grid open along x (a premixed stream entering
through an inflow ghost cell and leaving through a zero-gradient outflow, the open
boundary of the model transport operator) the stream reacts as it flows and the steady
state is a profile along x.  It is found here by Newton's method on the nx (ns + 1)
unknowns of one x line,

    G(U) = T_x(U) + R(U) = 0,

where T_x is the x part of the transport operator (the y and z parts vanish on a state
that is uniform in y and z) and R the oracle's cell right-hand side (Sec. 4.4,
e:cv_reactor).  T_x(U)_i = a_m U_{i-1} + a_c U_i + a_p U_{i+1} with
a_m = vel / (2 dx) + diff / dx^2, a_c = -2 diff / dx^2, a_p = -vel / (2 dx) + diff / dx^2,
U_{-1} the inflow state and U_{nx} = U_{nx-1}.  The Jacobian of G is block tridiagonal:
the stencil weights times the identity off the diagonal, and on the diagonal each cell's
(ns + 1)^2 Jacobian of R, assembled column by column from the oracle's exact
(complex-step) Jacobian-vector products, plus a_c (and a_p in the last cell).  The
starting guess is the plug-flow profile: the inflow state carried through each cell for
its residence time dx / vel by the oracle's ROK4E.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spl

from . import oracle as O


def stencil(dx, vel, diff):
    """Weights (a_m, a_c, a_p) of the x part of the transport operator."""
    return vel / (2.0 * dx) + diff / dx**2, -2.0 * diff / dx**2, -vel / (2.0 * dx) + diff / dx**2


def line_transport(U, inflow, dx, vel, diff):
    """T_x(U) on one open x line: U [N, nx], inflow [N]."""
    a_m, a_c, a_p = stencil(dx, vel, diff)
    Um = np.concatenate([np.asarray(inflow, np.float64)[:, None], U[:, :-1]], axis=1)
    Up = np.concatenate([U[:, 1:], U[:, -1:]], axis=1)
    return a_m * Um + a_c * U + a_p * Up


def line_transport_matrix(N, nx, dx, vel, diff):
    """Sparse matrix of U -> T_x(U) with the inflow held at zero, unknowns ordered
    k = c N + r (cell-major)."""
    a_m, a_c, a_p = stencil(dx, vel, diff)
    n = N * nx
    main = np.full(n, a_c)
    main[(nx - 1) * N:] += a_p          # the outflow ghost repeats the last cell
    return sps.diags([np.full(n - N, a_m), main, np.full(n - N, a_p)], [-N, 0, N], format="csr")


def newton_line(R, JR, U0, inflow, dx, vel, diff, tol=1e-14, max_iter=40):
    """Newton's method on T_x(U) + R(U) = 0 from U0 [N, nx].  R(U) -> [N, nx]; JR(U) -> the
    nx diagonal Jacobian blocks [nx, N, N] of R.  Stops when the largest Newton step, relative
    to max(|U|, 1e-14) entry by entry, is at most tol.  Returns (U, steps taken, history of
    the largest relative step)."""
    U = np.array(U0, np.float64, copy=True)
    N, nx = U.shape
    A = line_transport_matrix(N, nx, dx, vel, diff)
    hist = []
    for it in range(max_iter):
        g = line_transport(U, inflow, dx, vel, diff) + R(U)
        J = (sps.block_diag(list(JR(U)), format="csr") + A).tocsc()
        d = spl.spsolve(J, -g.T.reshape(-1)).reshape(nx, N).T
        U = U + d
        hist.append(float((np.abs(d) / np.maximum(np.abs(U), 1e-14)).max()))
        if hist[-1] <= tol:
            return U, it + 1, hist
    raise RuntimeError(f"Newton did not converge: relative steps {hist}")


def cell_jacobian(mech, u, p):
    """Jacobian of the cell right-hand side at u = (Y, T), column by column from the
    complex-step Jacobian-vector product."""
    N = u.shape[0]
    J = np.empty((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        J[:, j] = O.cell_jvp(mech, u, p, e, O.JVP_COMPLEX)
    return J


def plug_flow(mech, inflow, p, nx, dx, vel, M, rtol=1e-10, atol=1e-16):
    """The inflow state integrated over the residence time dx / vel of each cell in turn:
    column c is the state after c + 1 residence times."""
    N = inflow.shape[0]
    U = np.empty((N, nx))
    u = np.array(inflow, np.float64, copy=True)
    for c in range(nx):
        Y, T, _, _, st = O.integrate(mech, u[:-1, None], u[-1:], np.array([p]), dx / vel, rtol, atol, M)
        if st[0] != 0:
            raise RuntimeError(f"plug-flow integration failed at cell {c} (status {st[0]})")
        u = np.concatenate([Y[:, 0], T])
        U[:, c] = u
    return U


def steady_premixed_line(mech, inflow, p, nx, dx, vel, diff, M, tol=1e-14):
    """The discrete steady state of T + R on an open x line of nx cells with the given
    inflow state (Y_1..Y_ns, T) at pressure p.  Returns (U [ns + 1, nx], Newton steps,
    history of the largest relative step)."""
    inflow = np.asarray(inflow, np.float64)
    pv = np.full(nx, float(p))

    def R(U):
        dY, dT = O.rhs(mech, U[:-1], U[-1], pv)
        return np.vstack([dY, dT[None, :]])

    def JR(U):
        return [cell_jacobian(mech, U[:, c], float(p)) for c in range(U.shape[1])]

    U0 = plug_flow(mech, inflow, float(p), nx, dx, vel, M)
    return newton_line(R, JR, U0, inflow, dx, vel, diff, tol=tol)
