"""Pin of the projected solve of the stages (Sec. 4.1, the M x M system with I - h gamma H
in Eq. e:solve_kry_jac): the oracle's LU with partial pivoting against numpy's solver
(LAPACK) on upper-Hessenberg matrices whose factorisation interchanges rows at several
consecutive steps, where a solve that ignored the interchanges' effect on the stored
multipliers would be wrong by O(1)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1712_00953_amd import synth

G = 0.572816062482135


@pytest.mark.parametrize("m", [2, 4, 8, 12])
def test_hessenberg_solve_with_interchanges(m):
    rng = np.random.default_rng(m)
    worst, pivoting = 0.0, 0
    for _ in range(200):
        H = np.triu(rng.standard_normal((m, m)), -1)
        A = np.eye(m) - rng.uniform(0.5, 5.0) * H
        b = rng.standard_normal(m)
        x, piv = O.lu_solve(A, b)
        ref = np.linalg.solve(A, b)
        # backward-stable solves of the same system differ by cond(A) eps at most
        worst = max(worst, np.max(np.abs(x - ref)) / (np.linalg.cond(A) * np.max(np.abs(ref))))
        assert np.all((piv == np.arange(m)) | (piv == np.arange(m) + 1))   # Hessenberg: k or k+1
        pivoting += int(np.sum(piv[1:] != np.arange(1, m)) >= 2)
    assert worst <= 1e-14
    if m >= 4:
        assert pivoting >= 20


def test_arnoldi_matrices_of_stiff_cells_pivot():
    """The reactor cells' own projected matrices interchange rows after the first
    step for large h on the stiffer mechanism, so the GPU solve is exercised there."""
    w = synth.workload(1, a_scale=1e-5, n_cells=16)
    st = w.states
    hits = 0
    for c in range(16):
        u = np.concatenate([st.Y[:, c], [st.T[c]]])
        Q, H, meff = O.cell_arnoldi(w.mech, u, st.p[c], w.M, O.JVP_FD)
        A = np.eye(meff) - 1e-6 * G * H[:meff, :meff]
        b = np.arange(1.0, meff + 1)
        x, piv = O.lu_solve(A, b)
        np.testing.assert_allclose(A @ x, b, rtol=0, atol=1e-12 * np.linalg.cond(A))
        hits += int(np.any(piv[1:] != np.arange(1, meff)))
    assert hits >= 3
