"""GPU parity on the literal draw of the synthetic mechanism generator (pre-exponential
factors log-uniform in [1e6, 1e14], no multiplier), through the C ABI.

These cells take thousands to tens of thousands of ROK4E attempts over dt (1.5e3 to
1.2e4 on the 9-species batch, 1.9e3 to 7.8e4 on the 53-species flame slice), so the
result is the end of a long chain of accepted and rejected steps.  The checks are those
of the other FP64 parity tests: relative error at most max(1e-10, 4x the oracle's FMA
twin's) on every species above 1e-14 and on T, the tolerance-normalised difference
within 4x the twin's (+1e-6), and accept/reject counts matching at the twin's rate up to
binomial noise.  Over so many attempts rounding decides accept/reject at some step of
most cells: the oracle and its twin take the same step sequence on only 31 % (9 species)
and 47 % (53 species) of the cells and end up to 2.3 and 1.4 tolerance units apart, so
on this draw the bar is the method's own rounding envelope, not 1e-10.  The GPU stays
inside it (measured 2.2 and 1.2 tolerance units, count match 31 % and 47 %).  The large
relative spreads sit on species below 1e-8, whose error control is atol = 1e-12; on the
species above 1e-8 and on T the twin's spread is 2.3e-8 (9 species) and 3.9e-5 (53
species), and the GPU is held to 4x the twin's spread on those entries as well (measured
2.5e-8 and 2.0e-5).
"""
import numpy as np
import pytest

from gpu_util import envelope, gpu_integrate, normalized, parity, relative
from paper_1712_00953_amd import synth

pytestmark = pytest.mark.gpu

MAX_ATT = 1 << 22


def match_floor(env_match, n):
    """Lowest acceptable accept/reject count-match rate for an n-cell sample."""
    return env_match - 3.0 * np.sqrt(max(env_match * (1 - env_match), 1e-4) / n) - 0.02


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    from paper_1712_00953_amd import rok4e as R
    R.load()
    return R


def _check(name, g, o, env, w, twin):
    mx, p99 = normalized(g, o, w.rtol, w.atol)
    d = dict(norm_max=mx, norm_p99=p99, **env, **parity(g, o), rel=relative(g, o),
             attempts_median=float(np.median(o[2] + o[3])), attempts_max=int((o[2] + o[3]).max()))
    # the species that the relative tolerance governs: above 1e-8 (the rounding spread of
    # the species below it is set by atol = 1e-12, up to tens of percent of their value)
    d.update(rel_above_1e8=relative(g, o, floor=1e-8), twin_rel_above_1e8=relative(twin, o, floor=1e-8))
    print(f"\n[{name}] " + " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                     for k, v in d.items()), flush=True)
    assert np.all(g[4] == 0) and np.all(o[4] == 0)
    assert mx <= 4 * env["env_max"] + 1e-6
    assert d["rel"] <= max(1e-10, 4 * env["env_rel"])
    assert d["rel_above_1e8"] <= max(1e-10, 4 * d["twin_rel_above_1e8"])
    assert d["match_frac"] >= match_floor(env["env_match"], g[0].shape[1])


def test_literal_draw_9_species_every_cell(R, orc):
    w = synth.workload(1, a_scale=1.0)
    st = w.states
    m = R.Mech(w.mech, M=w.M, max_attempts=MAX_ATT)
    g = gpu_integrate(m, st, w.dt, w.rtol, w.atol)
    o, env = envelope(orc, w, st, w.dt, w.rtol, w.atol, max_attempts=MAX_ATT)
    twin = orc.integrate(w.mech, st.Y, st.T, st.p, w.dt, w.rtol, w.atol, w.M, max_attempts=MAX_ATT, fma=True)
    _check("literal 9sp, 1,024 cells", g, o, env, w, twin)
    assert (o[2] + o[3]).min() > 1000
    m.close()


def test_literal_draw_53_species_full_batch_sampled(R, orc):
    """The whole 65,536-cell flame slice in one launch; the oracle recomputes a stratified
    sample of 32 cells."""
    w = synth.workload(2, a_scale=1.0)
    st = w.states
    m = R.Mech(w.mech, M=w.M, max_attempts=MAX_ATT)
    g = gpu_integrate(m, st, w.dt, w.rtol, w.atol)
    assert np.all(g[4] == 0)
    idx = synth.stratified_sample(st.T, 32, 700)
    sub = st.subset(idx)
    o, env = envelope(orc, w, sub, w.dt, w.rtol, w.atol, max_attempts=MAX_ATT)
    twin = orc.integrate(w.mech, sub.Y, sub.T, sub.p, w.dt, w.rtol, w.atol, w.M, max_attempts=MAX_ATT, fma=True)
    gs = (g[0][:, idx], g[1][idx], g[2][idx], g[3][idx], g[4][idx])
    _check("literal 53sp, 32 of 65,536 cells", gs, o, env, w, twin)
    # whole batch: mass fractions keep their totals
    assert np.abs(g[0].sum(0) - st.Y.sum(0)).max() <= 1e-9
    m.close()


@pytest.mark.parametrize("cfg,n", [(1, None), (2, 2048)])
def test_literal_draw_mixed_form_stays_within_tolerance_units(R, cfg, n):
    """The mixed FP32/FP64 form on the literal draw, against the FP64 GPU result of the same
    cells.  Over thousands of attempts FP32 rates of progress change the step sequence of
    every cell, so the two runs are different solutions of the same tolerance: the check is
    that every cell finishes and that the results agree to a few tolerance units (measured
    1.9 on the 9-species batch, 7.1 at most and 1.4 at the 99th percentile on the 53-species
    sample; relative 1.5e-6 and 4.1e-4 on species above 1e-8).  The 1e-5 relative bar of the
    mixed form holds on the calibrated workloads (test_gpu_parity.py), not here."""
    w = synth.workload(cfg, a_scale=1.0)
    st = w.states if n is None else w.states.subset(synth.stratified_sample(w.states.T, n, 5))
    res = {}
    for prec in (R.FP64, R.MIXED):
        m = R.Mech(w.mech, M=w.M, precision=prec, max_attempts=MAX_ATT)
        res[prec] = gpu_integrate(m, st, w.dt, w.rtol, w.atol)
        m.close()
    a, b = res[R.FP64], res[R.MIXED]
    mx, p99 = normalized(b, a, w.rtol, w.atol)
    print(f"\n[literal mixed cfg{cfg}] normalized max {mx:.3e} p99 {p99:.3e} relative above 1e-8 "
          f"{relative(b, a, floor=1e-8):.3e}", flush=True)
    assert np.all(b[4] == 0) and np.all(a[4] == 0)
    assert mx <= 20.0 and p99 <= 3.0
