"""Pins of the oracle's grid transport operator and grid splitting steps (Sec. 3.3).

* The central-difference operator on a Fourier mode exp(i theta x) has the closed-form
  eigenvalue lambda = -i vel sin(theta)/dx + diff (2 cos(theta) - 2)/dx^2 per direction.
* The classical Runge-Kutta substep multiplies that mode by the stability polynomial
  R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 at z = lambda dt per step.
* The Simpler balanced splitting keeps a steady state of T + R + src; Strang splitting
  moves it (the property that motivates the balanced form).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import splitting as SP
from paper_1712_00953_amd import synth

DX, VEL, DIFF = 1e-4, 10.0, 2e-5


def _cells(nx, ny, nz):
    c = np.arange(nx * ny * nz)
    return c % nx, (c // nx) % ny, c // (nx * ny)


def test_constant_field_is_at_rest():
    U = np.full((3, 6 * 4 * 5), 1.7)
    np.testing.assert_array_equal(SP.transport_grid(U, 6, 4, 5, DX, VEL, DIFF), 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fourier_mode_eigenvalue(axis):
    nx, ny, nz = 16, 12, 10
    x, y, z = _cells(nx, ny, nz)
    coord, nn = ((x, nx), (y, ny), (z, nz))[axis]
    k = 3
    th = 2 * np.pi * k / nn
    U = np.vstack([np.cos(th * coord), np.sin(th * coord)])
    out = SP.transport_grid(U, nx, ny, nz, DX, VEL, DIFF)
    lam = DIFF * (2 * np.cos(th) - 2) / DX**2 + (-1j * VEL * np.sin(th) / DX if axis == 0 else 0.0)
    w = lam * (U[0] + 1j * U[1])
    scale = abs(lam)
    assert np.max(np.abs(out[0] - w.real)) <= 1e-12 * scale
    assert np.max(np.abs(out[1] - w.imag)) <= 1e-12 * scale


def test_rk4_substep_is_the_stability_polynomial():
    nx, ny, nz = 16, 2, 2
    x, _, _ = _cells(nx, ny, nz)
    th = 2 * np.pi * 2 / nx
    U = np.vstack([np.cos(th * x), np.sin(th * x)])
    h, nsub = 4e-6, 3
    out = SP._transport_substep(U, (nx, ny, nz, DX, VEL, DIFF), h, nsub)
    lam = DIFF * (2 * np.cos(th) - 2) / DX**2 - 1j * VEL * np.sin(th) / DX
    z = lam * h / nsub
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    w = R**nsub * (U[0] + 1j * U[1])
    np.testing.assert_allclose(out[0], w.real, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out[1], w.imag, rtol=0, atol=1e-13)


def _steady_setup(nx=8, ny=2, nz=2):
    w = synth.workload(1, a_scale=1e-8, n_cells=4)
    st = synth.states_flame(w.mech, nx, ny * nz, 4001)
    grid = (nx, ny, nz, DX, VEL, DIFF)
    U = np.vstack([st.Y, st.T[None, :]])
    Ry, Rt = O.rhs(w.mech, st.Y, st.T, st.p)
    src = -(np.vstack([Ry, Rt[None, :]]) + SP.transport_grid(U, *grid))
    return w, st, grid, U, src


def test_simpler_keeps_a_steady_state_and_strang_moves_it():
    w, st, grid, U, src = _steady_setup()
    h, steps = 1e-7, 10
    scale = 1e-12 + 1e-6 * np.abs(U)
    dev = {}
    for name, step in (("simpler", SP.simpler_step_grid), ("strang", SP.strang_step_grid)):
        Y, T = st.Y.copy(), st.T.copy()
        for _ in range(steps):
            Y, T, acc, rej, sta = step(w.mech, Y, T, st.p, grid, h, 1e-8, 1e-14, w.M, src=src)
            assert np.all(sta == 0)
        dev[name] = float(np.max(np.abs(np.vstack([Y, T[None, :]]) - U) / scale))
    # the balanced form moves the state only by the rounding of f(u_n) = R + T + src;
    # Strang's transport substeps leave the steady state by O(h) per step
    assert dev["simpler"] <= 1e-4
    assert dev["strang"] >= 1e3 * max(dev["simpler"], 1e-6)
