"""Hand-built tiny mechanisms for the right-hand-side pins (test helper)."""
import numpy as np

from paper_1712_00953_amd.synth import Mechanism

NO_RATE = -1.0e3       # ln A of a direction that must not react: exp(-1000) = 0


def tiny_mech(W, cp, hf, reactions, elem=None):
    """reactions: list of (reactants, products, (lnAf, bf, Ef), (lnAr, br, Er))."""
    ns, nr = len(W), len(reactions)
    reac = -np.ones((nr, 2), np.int32)
    prod = -np.ones((nr, 2), np.int32)
    arr = np.zeros((6, nr))
    for j, (r, p, fw, rv) in enumerate(reactions):
        reac[j, :len(r)] = r
        prod[j, :len(p)] = p
        arr[0:3, j] = fw
        arr[3:6, j] = rv
    if elem is None:
        elem = np.zeros((ns, 1), np.int8)
    return Mechanism(ns, nr, elem.shape[1], elem, np.asarray(W, float), np.asarray(cp, float),
                     np.asarray(hf, float), reac, prod, arr[0], arr[1], arr[2], arr[3], arr[4], arr[5])
