"""Pins of the oracle's explicit Dormand-Prince 5(4) reference integrator (the explicit
method of the efficiency study in Sec. 5).

* The tableau satisfies the Runge-Kutta order conditions (the 17 rooted-tree conditions
  through order 5 for the propagated weights b, through order 4 for the embedded weights
  with the first-same-as-last stage), and the embedded weights fail an order-5 condition.
* Fixed steps converge at order 5 against the matrix exponential.
* Adaptive steps meet the tolerance on a linear system and agree with ROK4E on reactor
  cells at tight tolerances.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from paper_1712_00953_amd import synth


def _tableau():
    k = O.rkdp_coefficients()
    A = np.zeros((7, 7))
    A[1, 0] = k["a21"]
    A[2, :2] = k["a31"], k["a32"]
    A[3, :3] = k["a41"], k["a42"], k["a43"]
    A[4, :4] = k["a51"], k["a52"], k["a53"], k["a54"]
    A[5, :5] = k["a61"], k["a62"], k["a63"], k["a64"], k["a65"]
    b = np.array([k["b1"], 0.0, k["b3"], k["b4"], k["b5"], k["b6"], 0.0])
    A[6, :] = b                               # first-same-as-last: stage 7 at u_{n+1}
    bh = np.array([k["bh1"], 0.0, k["bh3"], k["bh4"], k["bh5"], k["bh6"], k["bh7"]])
    c = np.array([0.0, k["c2"], k["c3"], k["c4"], k["c5"], 1.0, 1.0])
    return A, b, bh, c


def _conditions(A, b, c):
    """Residuals of the rooted-tree order conditions of orders 1..5, grouped by order."""
    Ac, Ac2, Ac3 = A @ c, A @ c**2, A @ c**3
    AAc, AAc2 = A @ Ac, A @ Ac2
    AAAc = A @ AAc
    return {
        1: [b.sum() - 1],
        2: [b @ c - 1 / 2],
        3: [b @ c**2 - 1 / 3, b @ Ac - 1 / 6],
        4: [b @ c**3 - 1 / 4, b @ (c * Ac) - 1 / 8, b @ Ac2 - 1 / 12, b @ AAc - 1 / 24],
        5: [b @ c**4 - 1 / 5, b @ (c**2 * Ac) - 1 / 10, b @ (Ac**2) - 1 / 20, b @ (c * Ac2) - 1 / 15,
            b @ Ac3 - 1 / 20, b @ (c * AAc) - 1 / 30, b @ (A @ (c * Ac)) - 1 / 40, b @ AAc2 - 1 / 60,
            b @ AAAc - 1 / 120],
    }


def test_tableau_consistency_and_order_conditions():
    A, b, bh, c = _tableau()
    np.testing.assert_allclose(A[:6].sum(axis=1), c[:6], atol=1e-15)
    for order, res in _conditions(A, b, c).items():
        assert max(abs(r) for r in res) <= 1e-14, (order, res)
    emb = _conditions(A, bh, c)
    for order in (1, 2, 3, 4):
        assert max(abs(r) for r in emb[order]) <= 1e-14, (order, emb[order])
    assert max(abs(r) for r in emb[5]) >= 1e-4     # the embedded solution is order 4


def _linear(seed=3, n=6):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) - 2.0 * np.eye(n)
    return A, rng.standard_normal(n), rng.standard_normal(n)


def test_fixed_steps_converge_at_order_5():
    A, c, u0 = _linear()
    dt = 0.5
    n = len(u0)
    E = sla.expm(np.block([[A, c[:, None]], [np.zeros((1, n + 1))]]) * dt)
    exact = E[:n, :n] @ u0 + E[:n, n]
    errs = []
    for steps in (8, 16, 32):
        u, acc, rej, st = O.rkdp_linear(A, c, u0, dt, fixed_steps=steps)
        assert st == 0 and acc == steps
        errs.append(np.max(np.abs(u - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 4.7) and np.all(rates < 5.5), rates


def test_adaptive_meets_tolerance_on_linear_system():
    A, c, u0 = _linear(5)
    dt = 2.0
    n = len(u0)
    E = sla.expm(np.block([[A, c[:, None]], [np.zeros((1, n + 1))]]) * dt)
    exact = E[:n, :n] @ u0 + E[:n, n]
    for rtol in (1e-6, 1e-9):
        u, acc, rej, st = O.rkdp_linear(A, c, u0, dt, rtol=rtol, atol=rtol * 1e-3)
        assert st == 0 and acc > 3
        assert np.max(np.abs(u - exact) / (np.abs(exact) + 1e-3)) <= 100 * rtol


def test_agrees_with_rok4e_on_reactor_cells():
    w = synth.workload(1, a_scale=1e-8, n_cells=16)
    st = w.states
    dt = 2e-7
    a = O.integrate_rkdp(w.mech, st.Y, st.T, st.p, dt, 1e-10, 1e-16, max_attempts=200000)
    b = O.integrate(w.mech, st.Y, st.T, st.p, dt, 1e-10, 1e-16, w.M, max_attempts=200000)
    assert np.all(a[4] == 0) and np.all(b[4] == 0)
    big = np.abs(b[0]) > 1e-8
    assert np.max(np.abs(a[0] - b[0])[big] / np.abs(b[0])[big]) <= 1e-6
    assert np.max(np.abs(a[1] - b[1]) / b[1]) <= 1e-9
