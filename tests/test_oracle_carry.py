"""Pins of the per-cell first trial step (the h_0 input of Algorithm a:ROK4E) and of the
step handed to the next call (carried between reaction substeps of a splitting run).

* h_io <= 0 reproduces the plain call bitwise; h_io = c reproduces the scalar option
  h0 = c bitwise.
* A cell already at a steady state of its forced system (forcing s = -f(u0) in the same
  order, so f(u0) = 0 exactly) takes one attempt with error 0, where the controller's
  factor is capped at 5: the next call starts from exactly 5 dt.
* The second of two consecutive substeps started from the carried steps agrees with the
  same substep restarted from dt to within a few tolerance units.
"""
import numpy as np

from oracle import oracle as O
from paper_1712_00953_amd import synth


def test_nonpositive_or_constant_first_step_reproduces_plain_calls():
    w = synth.workload(1, a_scale=1e-8, n_cells=32)
    st = w.states
    a = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M)
    h = np.zeros(st.n_cells)
    b = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, h_io=h)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert np.all(h > 0) and np.all(np.isfinite(h))
    c = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, h0=w.dt / 7)
    d = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, h_io=np.full(st.n_cells, w.dt / 7))
    for x, y in zip(c, d):
        np.testing.assert_array_equal(x, y)


def test_steady_cell_hands_on_five_dt():
    w = synth.workload(1, a_scale=1e-8, n_cells=8)
    st = w.states
    dY, dT = O.rhs(w.mech, st.Y, st.T, st.p)
    S = -np.vstack([dY, dT[None, :]])
    h = np.zeros(st.n_cells)
    Y, T, acc, rej, sta = O.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, S=S, h_io=h)
    np.testing.assert_array_equal(Y, st.Y)
    np.testing.assert_array_equal(T, st.T)
    assert np.all(acc == 1) and np.all(rej == 0)
    np.testing.assert_array_equal(h, 5.0 * w.dt)


def test_carried_step_gives_a_solution_of_the_next_substep():
    """Two consecutive substeps on the stiffer mechanism: the second started from the
    carried steps and the second restarted from dt are both solutions to the tolerance
    (they agree to a few tolerance units); on these cells the carried start saves no
    attempts (the controller recovers from h0 = dt within a few rejections)."""
    w = synth.workload(1, a_scale=1e-5, n_cells=64)
    st = w.states
    dt = 1e-7
    h = np.zeros(st.n_cells)
    Y1, T1, *_ = O.integrate(w.mech, st.Y, st.T, st.p, dt, w.rtol, w.atol, w.M, h_io=h)
    assert np.all(h > 0) and np.all(h < 5 * dt)
    carry = O.integrate(w.mech, Y1, T1, st.p, dt, w.rtol, w.atol, w.M, h_io=h.copy())
    restart = O.integrate(w.mech, Y1, T1, st.p, dt, w.rtol, w.atol, w.M)
    assert np.all(carry[4] == 0) and np.all(restart[4] == 0)
    sc = w.atol + w.rtol * np.abs(restart[0])
    assert np.max(np.abs(carry[0] - restart[0]) / sc) <= 10.0
    assert np.max(np.abs(carry[1] - restart[1]) / (w.atol + w.rtol * restart[1])) <= 10.0
