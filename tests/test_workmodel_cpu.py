"""The algorithmic work model behind the roofline (paper_1712_00953_amd/workmodel.py).

Pins: the per-unit figures the benchmark's roofline is built from (53 species, 325
reactions, M = 8), a rough count of one right-hand side (about 21 R + 13 N_S operations
plus 2 R exponentials), the launch total of the benchmark batch (6,045,553
new-basis attempts and 164,308 retries give 7.40e11 operations), the cell-state bytes
(872 per cell at 53 species), and the monotone growth of an attempt with M.
"""
import pytest

from paper_1712_00953_amd import synth, workmodel as wm


@pytest.fixture(scope="module")
def mech53():
    return synth.workload(2, a_scale=1e-8, n_cells=2).mech


def test_per_unit_figures(mech53):
    a = wm.attempt_ops(mech53, 8)
    assert (a["new"], a["retry"], a["rhs"], a["basis"]) == (121624, 27428, 8270, 94196)
    ops, trans = wm.rhs_ops(mech53)
    R, ns = mech53.n_reactions, mech53.n_species
    assert abs(ops - (21 * R + 13 * ns)) <= 0.15 * ops
    assert trans == 2 * R + 1


def test_launch_total_and_state_bytes(mech53):
    b = wm.batch_ops(mech53, 8, 6045553, 164308)
    assert abs(b["flops"] - 7.398e11) <= 1e-3 * 7.398e11
    assert wm.state_bytes(mech53, 1) == 872
    assert wm.state_bytes(mech53, 65536) == 57147392


def test_attempt_grows_with_M(mech53):
    prev = None
    for M in (4, 6, 8, 12):
        a = wm.attempt_ops(mech53, M)
        assert a["new"] > a["retry"] > 2 * a["rhs"]
        if prev is not None:
            assert a["new"] > prev["new"] and a["basis"] > prev["basis"]
        prev = a
