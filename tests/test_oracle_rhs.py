"""Pins for the oracle's reactor right-hand side (Sec. 4.4, e:cv_reactor, read as the
adiabatic constant-pressure reactor with mass-action kinetics and CHEMKIN units).

Special cases with closed forms fix the rate law, the unit conversions and the sign
of every term; conservation identities fix the stoichiometry and the energy equation
on the synthetic mechanisms.
"""
import math

import numpy as np
import pytest

from mechs import NO_RATE, tiny_mech
from paper_1712_00953_amd import synth

RU = 8.314462618


def _cell(Y, T, p=101325.0):
    return np.asarray(Y, float)[:, None], np.array([T]), np.array([p])


def test_unimolecular_arrhenius_rate(orc):
    # A -> B + C with B, C absent: dY_A/dt = -k_f Y_A, k_f = A T^b exp(-E/(R T)) (1/s)
    lnA, b, E, T = math.log(3.0e5), 0.7, 8.0e4, 1400.0
    m = tiny_mech([0.03, 0.01, 0.02], [1000, 1200, 1400], [0, 0, 0],
                  [([0], [1, 2], (lnA, b, E), (NO_RATE, 0, 0))])
    dY, dT = orc.rhs(m, *_cell([1.0, 0.0, 0.0], T))
    kf = 3.0e5 * T**b * math.exp(-E / (RU * T))
    assert abs(dY[0, 0] - (-kf * 1.0)) <= 1e-14 * kf
    # products appear in proportion to their weights: W_k * (moles made) / rho
    assert abs(dY[1, 0] - kf * 0.01 / 0.03) <= 1e-14 * kf
    assert abs(dY[2, 0] - kf * 0.02 / 0.03) <= 1e-14 * kf


def test_bimolecular_rate_uses_mol_per_cm3(orc):
    # 2A -> B: omega_A = -2 k c_A^2 with c in mol/cm^3 and k in cm^3/(mol s)
    Wa, T, p, Ya = 0.002, 1500.0, 2.0e5, 0.6
    m = tiny_mech([Wa, 2 * Wa], [1500, 1500], [0, 0],
                  [([0, 0], [1], (math.log(2.0e12), 0, 0), (NO_RATE, 0, 0))])
    dY, _ = orc.rhs(m, *_cell([Ya, 1 - Ya], T, p))
    sigma = Ya / Wa + (1 - Ya) / (2 * Wa)
    rho = p / (RU * T * sigma)
    cA = 1e-6 * rho * Ya / Wa
    want = Wa * 1e6 * (-2.0 * 2.0e12 * cA * cA) / rho
    assert abs(dY[0, 0] - want) <= 1e-14 * abs(want)
    assert abs(dY[1, 0] + want) <= 1e-14 * abs(want)


def test_isomerisation_is_linear_and_isothermal(orc):
    kf, kr = 2.0e3, 5.0e2
    m = tiny_mech([0.028, 0.028], [1500, 1500], [1e5, 1e5],
                  [([0], [1], (math.log(kf), 0, 0), (math.log(kr), 0, 0))])
    for ya in (0.9, 0.3, 0.2):
        dY, dT = orc.rhs(m, *_cell([ya, 1 - ya], 1200.0))
        want = -kf * ya + kr * (1 - ya)
        assert abs(dY[0, 0] - want) <= 1e-13 * kf
        assert abs(dY[1, 0] + want) <= 1e-13 * kf
        assert abs(dT[0]) <= 1e-9
    # equilibrium: c_B / c_A = kf / kr makes f vanish
    ya = kr / (kf + kr)
    dY, _ = orc.rhs(m, *_cell([ya, 1 - ya], 1200.0))
    assert np.max(np.abs(dY)) <= 1e-12 * kf


def test_heat_release_sign(orc):
    # A -> B with h_f(B) < h_f(A): exothermic, T rises at rate -(h_B - h_A) * dY_B/dt / cp
    kf = 1.0e3
    m = tiny_mech([0.03, 0.03], [2000, 2000], [1.0e6, -5.0e5],
                  [([0], [1], (math.log(kf), 0, 0), (NO_RATE, 0, 0))])
    dY, dT = orc.rhs(m, *_cell([1.0, 0.0], 1000.0))
    want = -((-5.0e5 + 2000 * (1000 - 298.15)) - (1.0e6 + 2000 * (1000 - 298.15))) * kf / 2000.0
    assert dT[0] > 0
    assert abs(dT[0] - want) <= 1e-13 * abs(want)


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_conservation_identities_of_f(orc, cfg):
    w = synth.workload(cfg, a_scale=1e-8, n_cells=64)
    m, st = w.mech, w.states
    dY, dT = orc.rhs(m, st.Y, st.T, st.p)
    scale = np.abs(dY).max(axis=0)                         # per cell
    # mass: sum_k dY_k/dt = 0
    assert np.all(np.abs(dY.sum(axis=0)) <= 1e-13 * scale)
    # elements: sum_k a_ke dY_k/dt / W_k = 0
    el = m.elem.T.astype(float) @ (dY / m.W[:, None])
    el_scale = (m.elem.T.astype(float) @ (np.abs(dY) / m.W[:, None])) + 1e-300
    assert np.all(np.abs(el) <= 1e-13 * el_scale)
    # energy (adiabatic, constant p): sum_k h_k(T) dY_k/dt + cp_mix dT/dt = 0
    h = m.hf[:, None] + m.cp[:, None] * (st.T[None, :] - 298.15)
    cpm = (m.cp[:, None] * st.Y).sum(axis=0)
    terms = np.abs(h * dY).sum(axis=0)
    assert np.all(np.abs((h * dY).sum(axis=0) + cpm * dT) <= 1e-12 * terms)


def test_forcing_adds_to_f(orc):
    w = synth.workload(1, a_scale=1e-8, n_cells=8)
    m, st = w.mech, w.states
    dY, dT = orc.rhs(m, st.Y, st.T, st.p)
    S = np.random.default_rng(0).standard_normal((m.n_species + 1, 8))
    dY2, dT2 = orc.rhs(m, st.Y, st.T, st.p, S)
    np.testing.assert_array_equal(dY2, dY + S[:-1])
    np.testing.assert_array_equal(dT2, dT + S[-1])


def test_complex_step_jvp_matches_finite_difference(orc):
    w = synth.workload(2, a_scale=1e-8, n_cells=4)
    m, st = w.mech, w.states
    rng = np.random.default_rng(1)
    for c in range(4):
        u = np.concatenate([st.Y[:, c], [st.T[c]]])
        v = rng.standard_normal(u.shape[0])
        v /= np.linalg.norm(v)
        jc = orc.cell_jvp(m, u, st.p[c], v, orc.JVP_COMPLEX)
        # central differences with a step well above roundoff, as an independent check
        eps = 1e-5
        up = u + eps * v
        um = u - eps * v
        fp = np.concatenate(orc.rhs(m, up[:-1, None], up[-1:], st.p[c:c + 1]), axis=None)
        fm = np.concatenate(orc.rhs(m, um[:-1, None], um[-1:], st.p[c:c + 1]), axis=None)
        jcd = (fp - fm) / (2 * eps)
        assert np.max(np.abs(jc - jcd)) <= 1e-6 * np.max(np.abs(jc))
        jfd = orc.cell_jvp(m, u, st.p[c], v, orc.JVP_FD)
        assert np.max(np.abs(jc - jfd)) <= 1e-5 * np.max(np.abs(jc))
