"""Pins for the finite-difference Jacobian-vector product (Sec. 4.3) and for the
rounding envelope of the method.

* The difference-form numerator f(u + du) - f(u) equals the same difference computed in
  quadruple precision to ~1e-13 of its size; the literal difference of two FP64
  evaluations carries absolute noise eps |f| (relative noise up to ~1e-6 here).
* Two builds of the same oracle that round differently (with and without fused
  multiply-adds) agree on the adaptive result to ~1e-13 relative on every species above
  1e-14 and take the same step sequence on every cell.  This holds only because the
  Arnoldi basis stays orthonormal to rounding (Eq. e:solve_kry_jac needs V^T V = I):
  with modified Gram-Schmidt alone the basis of a stiff cell loses orthogonality at
  M = 8, the stage solves then differ by ~1e-7 between the two builds and a third of
  the cells change their step count.  The twin's difference is the rounding floor the
  GPU bar is scaled from.
"""
import numpy as np
import pytest

from paper_1712_00953_amd import synth


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_difference_form_matches_quad_precision(orc, cfg):
    w = synth.workload(cfg, a_scale=1e-8, n_cells=12)
    st = w.states
    rng = np.random.default_rng(cfg)
    worst, worst_lit = 0.0, 0.0
    for c in range(12):
        u = np.concatenate([st.Y[:, c], [st.T[c]]])
        v = rng.standard_normal(u.size)
        v /= np.linalg.norm(v)
        delta = np.sqrt(2.0**-52 * (1 + np.linalg.norm(u)))
        du = delta * v
        d = orc.cell_fdiff(w.mech, u, st.p[c], du)
        q = orc.cell_fdiff(w.mech, u, st.p[c], du, quad=True)
        lit = orc.cell_jvp(w.mech, u, st.p[c], v, orc.JVP_FD_LITERAL) * delta
        # the FD JVP of the integrator is the difference form divided by delta (delta
        # recomputed here with a differently ordered norm: equal to rounding)
        np.testing.assert_allclose(orc.cell_jvp(w.mech, u, st.p[c], v, orc.JVP_FD), d / delta,
                                   rtol=1e-13, atol=1e-13 * np.abs(d / delta).max())
        worst = max(worst, np.abs(d - q).max() / np.abs(q).max())
        worst_lit = max(worst_lit, np.abs(lit - q).max() / np.abs(q).max())
    assert worst <= 1e-12, worst
    assert worst_lit > 100 * worst


def test_difference_form_on_a_linear_problem_is_exact(orc):
    # affine f: the difference is A du exactly (no truncation error)
    A = np.array([[-2.0, 1.0], [0.5, -3.0]])
    u, acc, rej, st = orc.integrate_linear(A, np.array([1.0, 2.0]), np.array([0.3, 0.1]), 1.0, 1e-8,
                                           1e-12, M=2, jvp=orc.JVP_FD)
    ue, *_ = orc.integrate_linear(A, np.array([1.0, 2.0]), np.array([0.3, 0.1]), 1.0, 1e-8,
                                  1e-12, M=2, jvp=orc.JVP_EXACT)
    np.testing.assert_allclose(u, ue, rtol=1e-14, atol=1e-15)


def normalized_error(a, b, rtol, atol):
    """max over cells and rows of |a - b| / (atol + rtol |b|) for (Y, T) tuples."""
    eY = np.abs(a[0] - b[0]) / (atol + rtol * np.abs(b[0]))
    eT = np.abs(a[1] - b[1]) / (atol + rtol * np.abs(b[1]))
    return float(max(eY.max(), eT.max()))


@pytest.mark.parametrize("cfg,n", [(1, 256), (2, 96)])
def test_rounding_envelope_is_within_tolerance(orc, cfg, n):
    w = synth.workload(cfg, a_scale=1e-8)
    st = w.states.subset(synth.stratified_sample(w.states.T, n, 9))
    a = orc.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M)
    b = orc.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, fma=True)
    e = normalized_error(b, a, w.rtol, w.atol)
    match = np.mean((a[2] == b[2]) & (a[3] == b[3]))
    rel = np.abs(a[0] - b[0]) / np.maximum(np.abs(a[0]), 1e-14)
    print(f"\n[envelope cfg{cfg}] normalized {e:.3e} relative {rel.max():.3e} count match {match:.3f}")
    # the same step sequence everywhere, and a rounding-level difference in the result
    assert match == 1.0
    assert rel.max() <= 1e-12
    assert e <= 1e-6
