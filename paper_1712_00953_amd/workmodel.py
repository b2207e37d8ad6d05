"""Algorithmic operation counts of the ROK4E reaction substep (for the roofline).

Counts follow the formulas, not the kernels: every +, -, *, / is one operation, a fused
multiply-add is two, and each exp, log, expm1, sqrt or pow is one operation (also
reported on its own as a transcendental count).  Bytes are the cell state that must
cross HBM: Y, T and p read, Y and T written.

Per attempt (Algorithm a:ROK4E, Sec. 4.3):
* a new basis (after an accepted step, and at the start) costs f(u_n), M finite-
  difference Jacobian-vector products (one f each, the cost Sec. 4.3 assigns to the
  basis), the Arnoldi process (modified Gram-Schmidt and one re-orthogonalisation
  pass), the M x M factorisation, the four stages with two further evaluations of f
  (stage 4 reuses the stage-3 argument), the solution, the embedded error and the
  controller;
* a retry after a rejection reuses the basis of the same u_n: two evaluations of f, the
  factorisation, the stages, the error and the controller.
"""
from __future__ import annotations

import numpy as np


def rhs_ops(mech) -> tuple[int, int]:
    """(arithmetic ops, transcendentals) of one reactor right-hand side (Sec. 4.4)."""
    ns = int(mech.n_species)
    ops = 8 + 16 * ns          # per cell: rho, 1/(Ru T), dT/dt; per species: sums, c, f, h
    for j in range(int(mech.n_reactions)):
        nf = int(np.sum(mech.reac[j] >= 0))
        nr = int(np.sum(mech.prod[j] >= 0))
        sp = set(int(x) for x in mech.reac[j] if x >= 0) | set(int(x) for x in mech.prod[j] if x >= 0)
        nnz = len(sp)
        # two exponents (4 each), two exps, concentration products, q, nu q scatter
        ops += 8 + 2 + (nf - 1) + (nr - 1) + 3 + 2 * nnz
    trans = 2 * int(mech.n_reactions) + 1
    return ops, trans


def attempt_ops(mech, M: int) -> dict:
    """Operation counts of an attempt with a new basis and of a retry."""
    N = int(mech.n_species) + 1
    Me = min(M, N)
    cf, tf = rhs_ops(mech)
    jvp = cf + 4 * N                        # perturbation and difference quotient
    arnoldi = 3 * N + 2 * N + 4             # |f_n|, first vector, |u| and delta
    for j in range(Me):
        # |w|, modified Gram-Schmidt, the re-orthogonalisation pass (projections, removal,
        # coefficients added to H), |w| and normalise
        arnoldi += 2 * N + 4 * N * (j + 1) + 4 * N * (j + 1) + (j + 1) + 3 * N + 2
    lu = 3 * Me * Me + Me * Me + Me          # build I - h g H, Hessenberg LU
    solve = Me * Me + 2 * Me
    stage = 4 * N * Me + solve + Me + 2 * N  # Q^T F, solve, z - y, Q w, k
    stages = 4 * stage + 25 * N             # + stage arguments and gamma corrections
    finish = 7 * N + 22 * N + 12            # u*, error norm, controller
    new = (3 * cf) + Me * jvp + arnoldi + lu + stages + finish
    retry = 2 * cf + lu + stages + finish
    trans_new = (Me + 3) * tf + 2 + Me
    trans_retry = 2 * tf + 2
    # the basis alone: f(u_n), the M_eff Jacobian-vector products and the Gram-Schmidt work
    basis = cf + Me * jvp + arnoldi
    return dict(new=new, retry=retry, trans_new=trans_new, trans_retry=trans_retry, rhs=cf,
                basis=basis)


def batch_ops(mech, M: int, accepted: int, rejected: int) -> dict:
    """Algorithmic ops of a batch whose cells took `accepted` and `rejected` attempts in
    total (every accepted attempt builds the basis it used; retries reuse one)."""
    a = attempt_ops(mech, M)
    flops = accepted * a["new"] + rejected * a["retry"]
    trans = accepted * a["trans_new"] + rejected * a["trans_retry"]
    return dict(flops=float(flops), transcendentals=float(trans))


def state_bytes(mech, n_cells: int) -> int:
    """HBM bytes of the cell state: read Y, T, p; write Y, T (FP64)."""
    ns = int(mech.n_species)
    return 8 * n_cells * (2 * ns + 3)
