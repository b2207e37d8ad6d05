"""Pins of the open x boundary of the oracle's transport operator and of the discrete
steady premixed profile the splitting tests start from (Sec. 3.3, definition
d:steady_state_preserving).

* A state equal to the inflow state everywhere is at rest.
* With a constant source s and no reaction, the discrete steady state of the central
  stencil with an inflow ghost cell and a zero-gradient outflow has the closed form
  U_i = A + B rho^i + C i: rho = a_m / a_p is the second root of the stencil's
  characteristic polynomial (the first is 1), C = s dx / vel balances the source, and
  A, B follow from the two boundary conditions.  The operator and the Newton solver both
  reproduce it.
* For the 53-species mechanism the Newton solution is a steady state of the full 3-D
  operator plus the oracle right-hand side to rounding, it is not uniform, and 100 Simpler
  steps of the oracle keep it while two Strang steps move it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import splitting as SP
from oracle import steady as ST
from paper_1712_00953_amd import synth

DX, VEL, DIFF = 1e-4, 10.0, 2e-5
A_SCALE = 1e-8


def closed_form(nx, U_in, s, dx, vel, diff):
    a_m, a_c, a_p = ST.stencil(dx, vel, diff)
    rho = a_m / a_p
    C = s * dx / vel
    B = -C / (rho ** (nx - 1) * (rho - 1.0))
    A = U_in + C - B / rho
    i = np.arange(nx, dtype=np.float64)
    return A[:, None] + B[:, None] * rho ** i[None, :] + C[:, None] * i[None, :]


def test_inflow_state_everywhere_is_at_rest():
    rng = np.random.default_rng(5)
    inflow = rng.uniform(0.1, 2.0, 3)
    nx, ny, nz = 7, 3, 2
    U = np.repeat(inflow[:, None], nx * ny * nz, axis=1)
    out = SP.transport_grid(U, nx, ny, nz, DX, VEL, DIFF, inflow=inflow)
    assert np.abs(out).max() <= 1e-11 * DIFF / DX**2 * inflow.max()


@pytest.mark.parametrize("vel,diff", [(VEL, DIFF), (VEL, 0.0), (2.0, DIFF)])
def test_open_line_steady_state_with_a_source_has_the_closed_form(vel, diff):
    nx, ny, nz = 16, 2, 3
    U_in = np.array([0.3, 1.2, -0.7])
    s = np.array([2.0e3, -5.0e2, 1.0e1])
    Ux = closed_form(nx, U_in, s, DX, vel, diff)
    # the 3-D operator on the profile repeated along y and z: T(U) + s = 0
    U = np.tile(Ux, ny * nz)
    res = SP.transport_grid(U, nx, ny, nz, DX, vel, diff, inflow=U_in) + s[:, None]
    scale = (vel / DX + diff / DX**2) * np.abs(U).max()
    assert np.abs(res).max() <= 1e-12 * scale
    # Newton on T_x(U) + s = 0 from a uniform guess: the problem is linear, one step lands
    # and the next is rounding
    U0 = np.repeat(U_in[:, None], nx, axis=1)
    got, steps, hist = ST.newton_line(lambda V: np.repeat(s[:, None], nx, axis=1),
                                      lambda V: np.zeros((nx, 3, 3)), U0, U_in, DX, vel, diff, tol=1e-12)
    assert steps <= 2
    np.testing.assert_allclose(got, Ux, rtol=1e-11, atol=1e-13 * np.abs(Ux).max())


@pytest.fixture(scope="module")
def premixed():
    w = synth.workload(2, a_scale=A_SCALE, n_cells=4)
    inflow = synth.premixed_inflow(w.mech, 4600)
    nx = 128
    U, steps, hist = ST.steady_premixed_line(w.mech, inflow, synth.P_ATM, nx, DX, VEL, DIFF, w.M)
    return w, inflow, U, steps, hist


def test_newton_finds_a_steady_premixed_profile(premixed):
    w, inflow, U, steps, hist = premixed
    nx = U.shape[1]
    print(f"\n[premixed] Newton steps {steps}, largest relative steps {hist}, T {U[-1, 0]:.2f} .. "
          f"{U[-1, -1]:.2f} K", flush=True)
    assert steps <= 10
    # a genuine profile: the stream reacts as it flows (T changes by more than 10 K) and
    # transport and reaction balance without vanishing
    assert abs(U[-1, 0] - U[-1, -1]) > 10.0
    ny = nz = 2
    U3 = np.tile(U, ny * nz)
    p = np.full(nx * ny * nz, synth.P_ATM)
    Tr = SP.transport_grid(U3, nx, ny, nz, DX, VEL, DIFF, inflow=inflow)
    dY, dT = O.rhs(w.mech, U3[:-1], U3[-1], p)
    Rr = np.vstack([dY, dT[None, :]])
    assert np.abs(Tr[-1]).max() > 1e3          # K/s: transport is far from zero
    # the residual of the 3-D operator plus the right-hand side is rounding: relative to the
    # size of the terms that cancel in each entry
    scale = np.abs(Tr) + np.abs(Rr) + (VEL / DX) * np.abs(U3)
    assert (np.abs(Tr + Rr) / scale).max() <= 1e-11


def test_simpler_keeps_the_steady_premixed_profile_and_strang_moves_it(premixed):
    w, inflow, U, _, _ = premixed
    nx = U.shape[1]
    grid = (nx, 1, 1, DX, VEL, DIFF, inflow)
    p = np.full(nx, synth.P_ATM)
    h = 0.5 * DX / VEL                           # CFL 0.5
    g = np.abs(U) >= 1e-14
    dev = {}
    for name, step, n in (("simpler", SP.simpler_step_grid, 100), ("strang", SP.strang_step_grid, 2)):
        Y, T = U[:-1].copy(), U[-1].copy()
        for _ in range(n):
            Y, T, acc, rej, st = step(w.mech, Y, T, p, grid, h, 1e-8, 1e-14, w.M)
            assert np.all(st == 0)
        V = np.vstack([Y, T[None, :]])
        dev[name] = float((np.abs(V - U)[g] / np.abs(U)[g]).max())
    print(f"\n[premixed] 100 Simpler steps {dev['simpler']:.3e}, 2 Strang steps {dev['strang']:.3e}",
          flush=True)
    assert dev["simpler"] <= 1e-12
    assert dev["strang"] >= 1e-4
