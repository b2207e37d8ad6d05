"""Pins for the oracle's integrator on linear problems u' = A u + c.

* one step on the scalar problem equals the stability function R(h lambda) of
  e:stability_exact_jac (stages, Woodbury solve with M = N = 1);
* fixed-step convergence against the matrix exponential shows order 4 for M = 4 < N
  and M = N (Rosenbrock-Krylov order conditions, e:krylov_jac_cond);
* M = N reduces ROK4E to the classical ROW method with the full Jacobian
  (e:jac_proj: A_n = J_n when M = N);
* the adaptive controller follows the PI rule of Sec. 4.3 with the embedded estimate,
  re-derived here from the stability functions of the two weight vectors.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from conftest import stability_R, stability_R_gap


@pytest.mark.parametrize("z", [-0.1, -1.0, -10.0, -1e3, 0.5])
def test_scalar_step_equals_stability_function(orc, coeffs, z):
    lam = -3.0 if z < 0 else 3.0
    h = z / lam
    u, acc, rej, st = orc.integrate_linear(np.array([[lam]]), None, np.array([1.0]), h, 1e-6, 1e-12,
                                           M=1, jvp=orc.JVP_EXACT, fixed_steps=1)
    R = stability_R(coeffs, z)
    assert st == 0 and acc == 1
    assert abs(u[0] - R) <= 1e-14 * max(1.0, abs(R))


def test_stability_function_is_fourth_order_and_L_stable(coeffs):
    # R(z) - exp(z) = O(z^5): halving z divides the defect by ~32
    d1 = abs(stability_R(coeffs, -0.02) - np.exp(-0.02))
    d2 = abs(stability_R(coeffs, -0.01) - np.exp(-0.01))
    assert 4.7 < np.log2(d1 / d2) < 5.3
    assert abs(stability_R(coeffs, -1e8)) < 1e-7


def _stable_matrix(n, seed, lam_lo=0.5, lam_hi=5.0):
    rng = np.random.default_rng(seed)
    V = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    lam = -np.geomspace(lam_lo, lam_hi, n)
    A = V @ np.diag(lam) @ np.linalg.inv(V)
    c = rng.standard_normal(n)
    u0 = rng.standard_normal(n)
    return A, c, u0


def _exact(A, c, u0, t):
    uinf = -np.linalg.solve(A, c)
    return uinf + expm(t * A) @ (u0 - uinf)


@pytest.mark.parametrize("M", [4, 10])
def test_fourth_order_convergence_linear(orc, M):
    A, c, u0 = _stable_matrix(10, 11)
    T = 1.0
    ref = _exact(A, c, u0, T)
    errs = []
    steps = [8, 16, 32, 64, 128, 256]
    for n in steps:
        u, acc, rej, st = orc.integrate_linear(A, c, u0, T, 1e-6, 1e-12, M=M, jvp=orc.JVP_EXACT,
                                               fixed_steps=n)
        assert st == 0 and acc == n
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1) if errs[i + 1] > 1e-13]
    assert len(orders) >= 4
    for o in orders[-2:]:                   # asymptotic range
        assert 3.8 <= o <= 4.2, (orders, errs)
    assert all(o > 3.3 for o in orders), orders


def test_full_krylov_equals_dense_row_linear(orc):
    # a spectrum narrow enough that the Krylov space fills R^10 without breakdown
    A, c, u0 = _stable_matrix(10, 5, 2.0, 20.0)
    for n in (1, 3):
        u_rok, *_ = orc.integrate_linear(A, c, u0, 0.2, 1e-6, 1e-12, M=10, jvp=orc.JVP_EXACT, fixed_steps=n)
        u_row = orc.row_dense_linear(A, c, u0, 0.2, n, jvp=orc.JVP_EXACT)
        assert np.max(np.abs(u_rok - u_row)) <= 1e-12 * np.max(np.abs(u_row))


def test_krylov_m4_differs_from_dense_row(orc):
    # M < N uses a rank-M Jacobian, so it is a different (still 4th-order) method
    A, c, u0 = _stable_matrix(10, 5, 0.5, 80.0)
    u_rok, *_ = orc.integrate_linear(A, c, u0, 0.2, 1e-6, 1e-12, M=4, jvp=orc.JVP_EXACT, fixed_steps=1)
    u_row = orc.row_dense_linear(A, c, u0, 0.2, 1, jvp=orc.JVP_EXACT)
    assert np.max(np.abs(u_rok - u_row)) > 1e-8


def _controller_sequence(coeffs, lam, y0, dt, rtol, atol, max_att=20000):
    """Expected (t, h, err, accepted) of the adaptive loop on y' = lam y, from the
    stability functions of b and b-hat and the PI rule h* = h min(5, max(0.2,
    0.8 err_n^0.1 / err^0.175)), first err_n = 1, last step clipped to the end."""
    out = []
    t, h, y, err_prev = 0.0, dt, y0, 1.0
    while t < dt and len(out) < max_att:
        last = False
        if h >= (dt - t) * (1 - 1e-12):
            h, last = dt - t, True
        z = h * lam
        ys = stability_R(coeffs, z) * y
        err = abs(stability_R_gap(coeffs, z) * y) / (atol + rtol * abs(ys))
        fac = min(5.0, max(0.2, 0.8 * max(err_prev, 1e-10) ** 0.1 / max(err, 1e-10) ** 0.175))
        out.append((t, h, err, err <= 1.0))
        if err <= 1.0:
            y, t, err_prev = ys, (dt if last else t + h), err
        h = h * fac
    return np.array(out, dtype=float), y


@pytest.mark.parametrize("lam,rtol", [(-50.0, 1e-6), (-2.0, 1e-9), (-1e4, 1e-4)])
def test_pi_controller_trace(orc, coeffs, lam, rtol):
    dt, atol = 1.0, 1e-12
    u, acc, rej, st, tr = orc.integrate_linear(np.array([[lam]]), None, np.array([1.0]), dt, rtol, atol,
                                               M=1, jvp=orc.JVP_EXACT, trace_cap=20000)
    exp_tr, y_end = _controller_sequence(coeffs, lam, 1.0, dt, rtol, atol)
    assert st == 0
    assert tr.shape == exp_tr.shape
    assert rej >= 1                         # h0 = dt is always rejected on these problems
    np.testing.assert_array_equal(tr[:, 3], exp_tr[:, 3])
    # stage arithmetic and the closed form round differently; over hundreds of
    # attempts the controller feeds that back into h
    np.testing.assert_allclose(tr[:-1, 1], exp_tr[:-1, 1], rtol=1e-8)
    # the clipped last step is dt - t: the accumulated t carries the rounding of all steps
    np.testing.assert_allclose(tr[-1, 1], exp_tr[-1, 1], rtol=1e-6)
    np.testing.assert_allclose(tr[:-1, 2], exp_tr[:-1, 2], rtol=1e-7, atol=1e-14)
    np.testing.assert_allclose(tr[-1, 2], exp_tr[-1, 2], rtol=1e-5)
    assert abs(u[0] - y_end) <= 1e-8 * abs(y_end) + 1e-300
    # every rejection shrinks the step by at least 0.8 (first err_n = 1, err > 1)
    for i in range(len(tr) - 1):
        if tr[i, 3] == 0:
            assert tr[i + 1, 1] <= 0.8 * tr[i, 1] * (1 + 1e-12)


def test_adaptive_accuracy_linear(orc):
    A, c, u0 = _stable_matrix(10, 3, 0.5, 200.0)
    ref = _exact(A, c, u0, 1.0)
    for rtol in (1e-4, 1e-6, 1e-8):
        u, acc, rej, st = orc.integrate_linear(A, c, u0, 1.0, rtol, 1e-12, M=4, jvp=orc.JVP_FD)
        assert st == 0
        assert np.max(np.abs(u - ref) / (np.abs(ref) + 1e-3)) <= 20 * rtol
