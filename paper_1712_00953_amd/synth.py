"""Seeded synthetic inputs for the batched reaction substep: mechanisms and cell states.

This module is shared by the HIP path's callers (tests, benchmark) and by the CPU
oracle's callers.  It holds only random draws, the combinatorics of atom balance and
the preparation of an element-consistent burnt mixture; none of the integration
method's arithmetic (no rate law, no right-hand side, no integrator) lives here.

Mechanism recipe (a synthetic stand-in for the paper's detailed mechanisms, e.g. the
53-species, 325-reaction methane mechanism used for the 0-D reactor tests of the
ROK4E section):

* species are element-count vectors over E elements with counts 0..2 each
  (3**E - 1 non-empty compositions); molecular weight = sum(count * w_e) with
  w = (1, 16, 12, 14) g/mol; when more species than compositions are asked for,
  the extra species are isomers (duplicate compositions);
* reactions are atom-balanced elementary swaps with 1-2 reactants and 1-2
  products that share no species between the two sides;
* forward and reverse Arrhenius parameters are drawn independently:
  A log-uniform in [1e6, 1e14] (cm-mol-s units), b uniform in [-1, 1],
  Ea uniform in [0, 1.5e5] J/mol;
* species heat capacity is constant, uniform in [1, 3] kJ/kg/K, and formation
  enthalpy at 298.15 K is uniform in [-2e6, 2e6] J/kg.

The optional ``a_scale`` multiplies every pre-exponential factor (forward and reverse)
by one global constant.  It is the single knob of the *calibrated* variant; the literal
recipe is ``a_scale = 1``.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

R_U = 8.314462618          # J/(mol K)
P_ATM = 101325.0           # Pa
ELEMENT_WEIGHTS_G = (1.0, 16.0, 12.0, 14.0)   # g/mol, element order H, O, C, N
T_BURNT = 2200.0           # K, temperature of the equilibrium-like burnt mixture


@dataclasses.dataclass
class Mechanism:
    """A reversible mass-action mechanism (host arrays, float64 / int32)."""
    n_species: int
    n_reactions: int
    n_elements: int
    elem: np.ndarray      # int8  [n_species, n_elements] element counts
    W: np.ndarray         # f64   [n_species] molecular weight, kg/mol
    cp: np.ndarray        # f64   [n_species] heat capacity, J/(kg K)
    hf: np.ndarray        # f64   [n_species] formation enthalpy at 298.15 K, J/kg
    reac: np.ndarray      # int32 [n_reactions, 2] reactant species, -1 if absent
    prod: np.ndarray      # int32 [n_reactions, 2] product species, -1 if absent
    lnAf: np.ndarray      # f64   [n_reactions] ln of forward A (cm-mol-s)
    bf: np.ndarray        # f64   [n_reactions] forward temperature exponent
    Ef: np.ndarray        # f64   [n_reactions] forward activation energy, J/mol
    lnAr: np.ndarray      # f64   [n_reactions] ln of reverse A (cm-mol-s)
    br: np.ndarray
    Er: np.ndarray
    a_scale: float = 1.0
    seed: int = 0

    @property
    def n_state(self) -> int:
        return self.n_species + 1


@dataclasses.dataclass
class States:
    """Cell states in the structure-of-arrays layout the boundary takes."""
    Y: np.ndarray         # f64 [n_species, n_cells] mass fractions (species-major)
    T: np.ndarray         # f64 [n_cells] temperature, K
    p: np.ndarray         # f64 [n_cells] pressure, Pa

    @property
    def n_cells(self) -> int:
        return int(self.T.shape[0])

    def subset(self, idx) -> "States":
        idx = np.asarray(idx)
        return States(np.ascontiguousarray(self.Y[:, idx]),
                      np.ascontiguousarray(self.T[idx]),
                      np.ascontiguousarray(self.p[idx]))


def _compositions(n_elements: int) -> np.ndarray:
    combos = [c for c in itertools.product(range(3), repeat=n_elements) if any(c)]
    return np.array(combos, dtype=np.int8)


def _candidate_reactions(elem: np.ndarray):
    """All atom-balanced swaps {side_a <-> side_b}; a side is a multiset of 1-2 species.

    Returned in a canonical order (by composition, then by side) so that a seeded
    choice among them is reproducible.
    """
    ns = elem.shape[0]
    sides = [(i,) for i in range(ns)] + [(i, j) for i in range(ns) for j in range(i, ns)]
    groups: dict = {}
    for s in sides:
        comp = tuple(int(v) for v in elem[list(s)].sum(axis=0))
        groups.setdefault(comp, []).append(s)
    cands = []
    for comp in sorted(groups):
        g = sorted(groups[comp], key=lambda s: (len(s), s))
        for a_i in range(len(g)):
            for b_i in range(a_i + 1, len(g)):
                a, b = g[a_i], g[b_i]
                if set(a) & set(b):
                    continue            # spectators: not an elementary swap
                cands.append((a, b))
    return cands


def make_mechanism(n_species: int, n_reactions: int, n_elements: int, seed: int,
                   a_scale: float = 1.0) -> Mechanism:
    """Draw a synthetic mechanism.  Draw order: compositions, isomers, cp, hf,
    reaction choice, orientation, then forward and reverse Arrhenius triples."""
    rng = np.random.default_rng(seed)
    comps = _compositions(n_elements)
    perm = rng.permutation(len(comps))
    if n_species <= len(comps):
        elem = comps[perm[:n_species]]
    else:
        extra = n_species - len(comps)
        if extra > len(comps):
            raise ValueError("too many species for the composition space")
        iso = rng.choice(len(comps), size=extra, replace=False)
        elem = np.concatenate([comps[perm], comps[iso]], axis=0)
    w = np.array(ELEMENT_WEIGHTS_G[:n_elements])
    W = (elem.astype(np.float64) @ w) * 1e-3
    cp = rng.uniform(1000.0, 3000.0, n_species)
    hf = rng.uniform(-2.0e6, 2.0e6, n_species)

    cands = _candidate_reactions(elem)
    if len(cands) < n_reactions:
        raise ValueError(f"only {len(cands)} atom-balanced candidates for {n_reactions} reactions")
    pick = rng.choice(len(cands), size=n_reactions, replace=False)
    flip = rng.random(n_reactions) < 0.5
    reac = -np.ones((n_reactions, 2), dtype=np.int32)
    prod = -np.ones((n_reactions, 2), dtype=np.int32)
    for r, (ci, fl) in enumerate(zip(pick, flip)):
        a, b = cands[ci]
        if fl:
            a, b = b, a
        reac[r, :len(a)] = a
        prod[r, :len(b)] = b

    ln10 = math.log(10.0)
    lnAf = rng.uniform(6.0, 14.0, n_reactions) * ln10 + math.log(a_scale)
    bf = rng.uniform(-1.0, 1.0, n_reactions)
    Ef = rng.uniform(0.0, 1.5e5, n_reactions)
    lnAr = rng.uniform(6.0, 14.0, n_reactions) * ln10 + math.log(a_scale)
    br = rng.uniform(-1.0, 1.0, n_reactions)
    Er = rng.uniform(0.0, 1.5e5, n_reactions)
    return Mechanism(n_species, n_reactions, n_elements, elem, W, cp, hf, reac, prod,
                     lnAf, bf, Ef, lnAr, br, Er, float(a_scale), seed)


def element_moles(mech: Mechanism, Y: np.ndarray) -> np.ndarray:
    """Moles of each element per kg of mixture; Y is [n_species] or [n_species, n]."""
    return mech.elem.T.astype(np.float64) @ (Y / (mech.W[:, None] if Y.ndim == 2 else mech.W))


def burnt_mixture(mech: Mechanism, Y_u: np.ndarray, T_b: float = T_BURNT) -> np.ndarray:
    """Equilibrium-like product mixture with the same element totals as ``Y_u``.

    Mole numbers follow the element-constrained Boltzmann distribution
    n_k = exp(-h_k W_k / (R T_b) + a_k . lam), with lam chosen so that the element
    totals of Y_u are met (the convex dual is minimised by damped Newton).  This is a
    preparation of input data only; it uses no reaction rate.
    """
    b = element_moles(mech, Y_u)
    A = mech.elem.astype(np.float64)                  # [ns, E]
    g = mech.hf * mech.W / (R_U * T_b)
    lam = np.zeros(mech.n_elements)

    def phi(l):
        return np.exp(-g + A @ l).sum() - b @ l

    for _ in range(200):
        n = np.exp(-g + A @ lam)
        grad = A.T @ n - b
        if np.max(np.abs(grad) / b) < 1e-14:
            break
        H = (A * n[:, None]).T @ A
        step = np.linalg.solve(H, -grad)
        t, f0 = 1.0, phi(lam)
        while phi(lam + t * step) > f0 + 1e-4 * t * (grad @ step) and t > 1e-12:
            t *= 0.5
        lam = lam + t * step
    n = np.exp(-g + A @ lam)
    Y_b = n * mech.W
    return Y_b / Y_b.sum()


def _tanh_profile(nx: int, ny: int, width: float = 8.0) -> np.ndarray:
    x = np.tile(np.arange(nx, dtype=np.float64), ny)        # cell = y*nx + x
    return 0.5 * (1.0 + np.tanh((x - nx / 2) / width))


def states_uniform(mech: Mechanism, n_cells: int, seed: int,
                   T_lo: float = 1000.0, T_hi: float = 2000.0, alpha: float = 1.0) -> States:
    """T uniform in [T_lo, T_hi], p = 1 atm, Y ~ Dirichlet(alpha) per cell."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(T_lo, T_hi, n_cells)
    Y = rng.dirichlet(np.full(mech.n_species, alpha), n_cells).T
    return States(np.ascontiguousarray(Y), T, np.full(n_cells, P_ATM))


def states_flame(mech: Mechanism, nx: int, ny: int, seed: int) -> States:
    """A tanh flame profile along x: T = (800 + 1400 s)(1 + 0.05 xi), clipped to
    [250, 3500] K, Y = (1 - s) Y_u + s Y_b with Y_u ~ Dirichlet(0.2)."""
    rng = np.random.default_rng(seed)
    Y_u = rng.dirichlet(np.full(mech.n_species, 0.2))
    Y_b = burnt_mixture(mech, Y_u)
    s = _tanh_profile(nx, ny)
    xi = rng.standard_normal(nx * ny)
    T = np.clip((800.0 + 1400.0 * s) * (1.0 + 0.05 * xi), 250.0, 3500.0)
    Y = (1.0 - s)[None, :] * Y_u[:, None] + s[None, :] * Y_b[:, None]
    return States(np.ascontiguousarray(Y), T, np.full(nx * ny, P_ATM))


def premixed_inflow(mech: Mechanism, seed: int, s: float = 0.5) -> np.ndarray:
    """The inflow state (Y_1..Y_ns, T) of a premixed stream: the mixture of the flame
    profile of ``states_flame`` (same seed) at progress s, Y = (1 - s) Y_u + s Y_b, at
    T = 800 + 1400 s K, without the temperature noise."""
    rng = np.random.default_rng(seed)
    Y_u = rng.dirichlet(np.full(mech.n_species, 0.2))
    Y_b = burnt_mixture(mech, Y_u)
    return np.concatenate([(1.0 - s) * Y_u + s * Y_b, [800.0 + 1400.0 * s]])


def states_bimodal(mech: Mechanism, n_cells: int, seed: int) -> States:
    """70 % cold cells (300-600 K, unburnt), 25 % burnt (1900-2300 K), 5 % flame front
    (1000-1600 K, s = (T - 800)/1400); cell order shuffled."""
    rng = np.random.default_rng(seed)
    Y_u = rng.dirichlet(np.full(mech.n_species, 0.2))
    Y_b = burnt_mixture(mech, Y_u)
    n_cold = int(round(0.70 * n_cells))
    n_burnt = int(round(0.25 * n_cells))
    n_front = n_cells - n_cold - n_burnt
    T = np.concatenate([rng.uniform(300.0, 600.0, n_cold),
                        rng.uniform(1900.0, 2300.0, n_burnt),
                        rng.uniform(1000.0, 1600.0, n_front)])
    s = np.concatenate([np.zeros(n_cold), np.ones(n_burnt), (T[n_cold + n_burnt:] - 800.0) / 1400.0])
    order = rng.permutation(n_cells)
    T, s = T[order], s[order]
    Y = (1.0 - s)[None, :] * Y_u[:, None] + s[None, :] * Y_b[:, None]
    return States(np.ascontiguousarray(Y), T, np.full(n_cells, P_ATM))


@dataclasses.dataclass
class Workload:
    name: str
    mech: Mechanism
    states: States
    M: int
    dt: float
    rtol: float
    atol: float


# Mechanism sizes and integration settings of the four single-GPU workloads.
WORKLOADS = {
    1: dict(ns=9, nr=24, ne=2, M=4, dt=1e-6, rtol=1e-6, atol=1e-12),
    2: dict(ns=53, nr=325, ne=4, M=8, dt=1e-5, rtol=1e-6, atol=1e-12),
    3: dict(ns=53, nr=325, ne=4, M=8, dt=1e-5, rtol=1e-6, atol=1e-12),
    4: dict(ns=111, nr=784, ne=4, M=12, dt=1e-5, rtol=1e-6, atol=1e-12),
}
WORKLOAD_NAMES = {1: "rok4e-9sp-24rx-1024cells", 2: "rok4e-53sp-325rx-65536cells-flame",
                  3: "rok4e-53sp-325rx-262144cells-bimodal", 4: "rok4e-111sp-784rx-131072cells-flame"}


def workload(cfg: int, a_scale: float = 1.0, n_cells: int | None = None) -> Workload:
    """Build workload ``cfg`` (1..4).  ``n_cells`` truncates the cell batch (the first
    cells of the full batch, same seeds) for small test runs."""
    p = WORKLOADS[cfg]
    mech_seed = 1000 + (2 if cfg == 3 else cfg)
    mech = make_mechanism(p["ns"], p["nr"], p["ne"], mech_seed, a_scale)
    st_seed = 2000 + cfg
    if cfg == 1:
        st = states_uniform(mech, 1024, st_seed)
    elif cfg == 2:
        st = states_flame(mech, 256, 256, st_seed)
    elif cfg == 3:
        st = states_bimodal(mech, 262144, st_seed)
    else:
        st = states_flame(mech, 512, 256, st_seed)
    if n_cells is not None:
        st = st.subset(np.arange(min(n_cells, st.n_cells)))
    name = WORKLOAD_NAMES[cfg] + ("" if a_scale == 1.0 else f"-ascale{a_scale:g}")
    return Workload(name, mech, st, p["M"], p["dt"], p["rtol"], p["atol"])


def stratified_sample(T: np.ndarray, n: int, seed: int, bands=(0, 700, 1200, 1700, 1e9)) -> np.ndarray:
    """Seeded sample of ``n`` cell indices, stratified by temperature band (equal share
    per non-empty band, sorted)."""
    rng = np.random.default_rng(seed)
    groups = [np.nonzero((T >= lo) & (T < hi))[0] for lo, hi in zip(bands[:-1], bands[1:])]
    groups = [g for g in groups if len(g)]
    per = max(1, n // len(groups))
    out = []
    for g in groups:
        out.append(rng.choice(g, size=min(per, len(g)), replace=False))
    idx = np.concatenate(out)
    if len(idx) < n:
        rest = np.setdiff1d(np.arange(len(T)), idx)
        idx = np.concatenate([idx, rng.choice(rest, size=min(n - len(idx), len(rest)), replace=False)])
    return np.sort(idx[:n])
