"""Pins for the reaction substep in conservative variables with the auxiliary
temperature equation (Sec. 5, e:chemical_source_balanced, e:aux_t_equation).

* Thermodynamics: the conservative state built from (Y, T, p, velocity) gives back T,
  and the ideal-gas pressure, through the oracle's inversion.
* The paper's stated property: integrated exactly, the auxiliary temperature equals the
  temperature of the conservative variables.  With balancing constants on every row and
  non-zero velocities, each term of the temperature source (species energies, kinetic
  energy, momentum, total energy) moves T by far more than the tolerance, so a dropped
  or mis-signed term, or the enthalpy in place of the internal energy, breaks the
  agreement.  The gap shrinks with the tolerance.
* rho, rho u and rho E only receive their constants: they end at U + dt s.
* Difference-form JVP numerator against quadruple precision; the FD JVP against the
  complex-step derivative of the same f.
"""
import numpy as np
import pytest

from paper_1712_00953_amd import synth

RU = 8.314462618


def cons_case(orc, cfg, n, seed=5, a=1e3, v_scale=50.0):
    w = synth.workload(cfg, a_scale=1e-8, n_cells=n)
    st = w.states
    rng = np.random.default_rng(seed)
    vel = v_scale * rng.standard_normal((3, n))
    U = orc.cons_state(w.mech, st.Y, st.T, st.p, vel)
    S = a * np.abs(U) * rng.standard_normal(U.shape)
    return w, st, U, S


def aux_state(U, T, ns):
    return np.concatenate([U[:ns], [T], U[ns:]])


@pytest.mark.parametrize("cfg", [2, 4])
def test_conservative_state_round_trip(orc, cfg):
    w, st, U, _ = cons_case(orc, cfg, 64)
    ns = w.mech.n_species
    T = orc.cons_temperature(w.mech, U)
    np.testing.assert_allclose(T, st.T, rtol=1e-11)
    # ideal gas: p = rho Ru T sum Y_k / W_k with Y_k = rho Y_k / rho
    rho = U[ns]
    p = (U[:ns] / np.asarray(w.mech.W)[:, None]).sum(0) * RU * T
    np.testing.assert_allclose(p, st.p, rtol=1e-11)
    np.testing.assert_allclose(U[:ns].sum(0), rho, rtol=1e-12)


@pytest.mark.parametrize("cfg", [2, 4])
def test_auxiliary_temperature_tracks_the_conservative_one(orc, cfg):
    n = 24
    w, st, U, S = cons_case(orc, cfg, n)
    ns = w.mech.n_species
    gaps = []
    for rtol in (1e-6, 1e-9):
        U1, Ta, acc, rej, sta = orc.integrate_cons(w.mech, U, w.dt, rtol, rtol * 1e-6, w.M, S=S)
        assert np.all(sta == 0)
        Tc = orc.cons_temperature(w.mech, U1)
        gaps.append(np.abs(Ta - Tc).max() / Tc.max())
    # the forcing moves T by kelvins over the step
    _, Ta0, *_ = orc.integrate_cons(w.mech, U, w.dt, 1e-9, 1e-15, w.M)
    moved = np.abs(Ta - Ta0).max()
    print(f"\n[aux T cfg{cfg}] gap rtol 1e-6 {gaps[0]:.2e}, rtol 1e-9 {gaps[1]:.2e}, "
          f"forcing moves T by {moved:.2f} K")
    assert moved > 1.0
    assert gaps[0] <= 1e-6 and gaps[1] <= 1e-9
    assert gaps[1] < gaps[0]


def test_each_term_of_the_temperature_source_matters(orc):
    # f_T of the oracle against the derivative of T(U) along f, computed from the
    # conservative rows alone by a central difference of the inversion
    w, st, U, S = cons_case(orc, 2, 6)
    ns = w.mech.n_species
    for c in range(6):
        u = aux_state(U[:, c], st.T[c], ns)
        s = aux_state(S[:, c], 0.0, ns)
        f = orc.cons_f(w.mech, u, s)
        fU = np.concatenate([f[:ns], f[ns + 1:]])
        eps = 1e-7
        Tp = orc.cons_temperature(w.mech, (U[:, c] + eps * fU)[:, None])[0]
        Tm = orc.cons_temperature(w.mech, (U[:, c] - eps * fU)[:, None])[0]
        dTdt = (Tp - Tm) / (2 * eps)
        assert abs(f[ns] - dTdt) <= 1e-6 * abs(dTdt) + 1e-6, (c, f[ns], dTdt)
        # the rows other than the species only carry their constants
        np.testing.assert_array_equal(f[ns + 1:], s[ns + 1:])


def test_flow_rows_advance_linearly(orc):
    w, st, U, S = cons_case(orc, 2, 16)
    ns = w.mech.n_species
    U1, Ta, acc, rej, sta = orc.integrate_cons(w.mech, U, w.dt, 1e-6, 1e-12, w.M, S=S)
    assert np.all(sta == 0)
    np.testing.assert_allclose(U1[ns:], U[ns:] + w.dt * S[ns:], rtol=1e-13)


@pytest.mark.parametrize("cfg", [2, 4])
def test_cons_difference_form_matches_quad_precision(orc, cfg):
    w, st, U, S = cons_case(orc, cfg, 8)
    ns = w.mech.n_species
    rng = np.random.default_rng(cfg + 50)
    worst = 0.0
    for c in range(8):
        u = aux_state(U[:, c], st.T[c], ns)
        s = aux_state(S[:, c], 0.0, ns)
        v = rng.standard_normal(u.size)
        v /= np.linalg.norm(v)
        du = np.sqrt(2.0**-52 * (1 + np.linalg.norm(u))) * v
        d = orc.cons_fdiff(w.mech, u, du, s)
        q = orc.cons_fdiff(w.mech, u, du, s, quad=True)
        np.testing.assert_array_equal(d[ns + 1:], 0.0)
        worst = max(worst, np.abs(d - q).max() / np.abs(q).max())
        # the temperature row on its own scale
        assert abs(d[ns] - q[ns]) <= 1e-11 * abs(q[ns]) + 1e-300
    assert worst <= 1e-12, worst


def test_cons_fd_jvp_matches_complex_step(orc):
    # the integrator's FD Jacobian-vector product against Im f(u + i h v) / h of the same
    # f: they differ by the O(delta) truncation of the first-order difference only (delta
    # ~ 1e-8 sqrt(|u|) is ~1e-5 here, |u| being dominated by rho E; measured ~3e-5 of the
    # largest entry), while a wrong or missing term of the increment is an O(1) error
    w, st, U, S = cons_case(orc, 2, 6)
    ns = w.mech.n_species
    rng = np.random.default_rng(11)
    for c in range(6):
        u = aux_state(U[:, c], st.T[c], ns)
        s = aux_state(S[:, c], 0.0, ns)
        v = rng.standard_normal(u.size)
        v /= np.linalg.norm(v)
        fd = orc.cons_jvp(w.mech, u, v, s, orc.JVP_FD)
        cs = orc.cons_jvp(w.mech, u, v, s, orc.JVP_COMPLEX)
        scale = np.abs(cs).max()
        assert np.abs(fd - cs).max() <= 1e-3 * scale, (c, np.abs(fd - cs).max() / scale)
        assert abs(fd[ns] - cs[ns]) <= 1e-3 * abs(cs[ns])
