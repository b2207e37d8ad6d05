import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def read_golden(name):
    """Reads a 'name value' text fixture (comments start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def coeffs():
    return read_golden("rok4e_coefficients.txt")


def stability_matrices(c):
    """b, b-hat and the lower-triangular beta matrix (beta_ii = gamma,
    beta_ij = alpha_ij + gamma_ij) of the stability function e:stability_exact_jac."""
    b = np.array([c["b1"], c["b2"], c["b3"], c["b4"]])
    bh = np.array([c["bh1"], c["bh2"], c["bh3"], c["bh4"]])
    al = np.zeros((4, 4))
    ga = np.zeros((4, 4))
    for i in range(1, 4):
        for j in range(i):
            al[i, j] = c[f"a{i+1}{j+1}"]
            ga[i, j] = c[f"g{i+1}{j+1}"]
    beta = al + ga + np.eye(4) * c["gamma"]
    return b, bh, al, ga, beta


def stability_R(c, z, weights="b"):
    b, bh, _, _, beta = stability_matrices(c)
    w = b if weights == "b" else bh
    return 1.0 + z * w @ np.linalg.solve(np.eye(4) - z * beta, np.ones(4))


def stability_R_gap(c, z):
    """R_hat(z) - R(z) = z (bh - b)^T (I - z beta)^{-1} 1, formed without cancellation."""
    b, bh, _, _, beta = stability_matrices(c)
    return z * (bh - b) @ np.linalg.solve(np.eye(4) - z * beta, np.ones(4))
