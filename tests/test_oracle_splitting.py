"""Pins for the Simpler balanced splitting around the oracle's ROK4E (Sec. 3).

* steady-state preservation (definition d:steady_state_preserving) of the Simpler
  splitting on the linear model e:ode_linear and on the scalar PSR e:scalar_psr, with
  Strang splitting drifting as the paper states;
* the Simpler recurrence u_{n+1} = R u_n + alpha B* (a + b) with
  R = alpha beta alpha + [alpha B* - (alpha beta + I) A*] A, reproduced by exact
  substeps, and its limits R -> I (h -> inf) and R -> I - alpha (|B| -> inf);
* the PSR S-curve turning points printed in Sec. 3.4 (golden fixture).
"""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.optimize import brentq

from conftest import read_golden
from oracle import splitting as S


def _linear_model(seed=3):
    rng = np.random.default_rng(seed)
    n = 4
    QA = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = QA @ np.diag(-rng.uniform(0.5, 2.0, n)) @ QA.T           # non-stiff transport
    QB = np.linalg.qr(rng.standard_normal((n, n)))[0]
    B = QB @ np.diag(-np.geomspace(10.0, 400.0, n)) @ QB.T       # stiff reaction
    a = rng.standard_normal(n)
    b = rng.standard_normal(n)
    return A, a, B, b


def test_simpler_preserves_linear_steady_state_strang_drifts():
    A, a, B, b = _linear_model()
    uinf = -np.linalg.solve(A + B, a + b)
    T = lambda u: A @ u + a
    R = lambda u: B @ u + b
    h = 0.5
    u_simpler = uinf.copy()
    for _ in range(100):
        u_simpler = S.simpler_step(T, R, u_simpler, h)
    drift = np.max(np.abs(u_simpler - uinf)) / np.max(np.abs(uinf))
    assert drift <= 1e-13, drift
    u_strang = S.strang_step(T, R, uinf.copy(), h)
    assert np.max(np.abs(u_strang - uinf)) / np.max(np.abs(uinf)) > 1e-4


def _simpler_exact_step(A, a, B, b, u, h):
    """One Simpler step with exact substeps (matrix exponentials)."""
    c = -(A @ u + a)
    g = b - c
    beta = expm(B * h)
    u1 = beta @ u + (beta - np.eye(len(u))) @ np.linalg.solve(B, g)
    alpha = expm(A * h / 2)
    # u' = A u + a + c = A (u - u_n): exact solution
    return u + alpha @ (u1 - u)


@pytest.mark.parametrize("h", [0.1, 1.0, 7.0])
def test_simpler_recurrence_matrix(h):
    A, a, B, b = _linear_model(5)
    n = len(a)
    I = np.eye(n)
    alpha, beta = expm(A * h / 2), expm(B * h)
    As = (alpha - I) @ np.linalg.inv(A)
    Bs = (beta - I) @ np.linalg.inv(B)
    R = alpha @ beta @ alpha + (alpha @ Bs - (alpha @ beta + I) @ As) @ A
    # columns of the recurrence from exact substeps with a = b = 0
    Rsim = np.stack([_simpler_exact_step(A, 0 * a, B, 0 * b, I[:, j], h) for j in range(n)], axis=1)
    assert np.max(np.abs(R - Rsim)) <= 1e-12
    # affine part: + alpha B* (a + b)  (the printed "- Q (a + b)" carries the opposite sign)
    u0 = np.random.default_rng(1).standard_normal(n)
    un = _simpler_exact_step(A, a, B, b, u0, h)
    assert np.max(np.abs(un - (R @ u0 + alpha @ Bs @ (a + b)))) <= 1e-12


def test_simpler_recurrence_limits():
    # scalar case, A = -1: R -> 1 for h -> inf; R -> 1 - alpha for |B| -> inf
    A = -1.0
    for h in (0.7, 2.0):
        alpha = np.exp(A * h / 2)
        for B in (-1e3, -1e6):
            beta = np.exp(B * h)
            R = alpha * beta * alpha + (alpha * (beta - 1) / B - (alpha * beta + 1) * (alpha - 1) / A) * A
            assert abs(R - (1 - alpha)) <= 2e-3
    h = 60.0
    alpha, beta = np.exp(A * h / 2), np.exp(-5.0 * h)
    R = alpha * beta * alpha + (alpha * (beta - 1) / -5.0 - (alpha * beta + 1) * (alpha - 1) / A) * A
    assert abs(R - 1.0) <= 1e-12


def _psr(g):
    Tin, Tad, Ta = g["T_in"], g["T_ad"], g["T_a"]
    R = lambda T, Da: (Tad - T) * np.exp(-Ta / T)
    Tr = lambda T, Da: (Tin - T) / Da
    Da_of_T = lambda T: (T - Tin) / ((Tad - T) * np.exp(-Ta / T))
    return R, Tr, Da_of_T


def test_psr_turning_points_match_paper():
    g = read_golden("psr_turning_points.txt")
    _, _, Da_of_T = _psr(g)
    dDa = lambda T: (Da_of_T(T * (1 + 1e-7)) - Da_of_T(T * (1 - 1e-7))) / (2e-7 * T)
    Ts = np.linspace(g["T_in"] + 1e-3, g["T_ad"] - 1e-3, 4000)
    d = dDa(Ts)
    roots = [brentq(dDa, Ts[i], Ts[i + 1]) for i in range(len(Ts) - 1) if d[i] * d[i + 1] < 0]
    assert len(roots) == 2
    das = sorted(Da_of_T(np.array(roots)))
    assert round(das[0], 2) == g["Da_E"]
    assert round(das[1], 2) == g["Da_I"]


def test_simpler_preserves_psr_steady_states():
    g = read_golden("psr_turning_points.txt")
    R, Tr, Da_of_T = _psr(g)
    Da = 100.0                            # between the turning points: three steady states
    F = lambda T: R(T, Da) + Tr(T, Da)
    grid = np.linspace(g["T_in"] + 1e-4, g["T_ad"] - 1e-4, 20000)
    fv = F(grid)
    roots = [brentq(F, grid[i], grid[i + 1], xtol=1e-16, rtol=1e-15)
             for i in range(len(grid) - 1) if fv[i] * fv[i + 1] < 0]
    assert len(roots) == 3
    for Tinf in roots:
        u = np.array([Tinf])
        Rf = lambda v: R(v, Da)
        Tf = lambda v: Tr(v, Da)
        for _ in range(100):
            u = S.simpler_step(Tf, Rf, u, 1.0)
        assert abs(u[0] - Tinf) <= 1e-12, (Tinf, u[0])
    # Strang moves off the (upper, stable) steady state by far more than roundoff
    Tinf = roots[-1]
    u = S.strang_step(lambda v: Tr(v, Da), lambda v: R(v, Da), np.array([Tinf]), 1.0)
    assert abs(u[0] - Tinf) > 1e-6
