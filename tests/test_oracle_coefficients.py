"""Pins for the oracle's ROK4E coefficient table (Sec. 4.2, table t:coeff_rok4e).

The oracle's constants must equal the printed table (golden fixture), and the printed
table, read as documented in the fixture, must satisfy the fourth-order Rosenbrock-Krylov
conditions e:order_cond_ros_k, L-stability R(inf) = 0 of e:stability_exact_jac, and the
embedded third-order conditions.  A mistyped digit in the oracle fails the equality; a
misread row label fails an order condition.
"""
import numpy as np
import pytest

from conftest import stability_matrices


def _conditions(c, w=None):
    b, bh, al, ga, beta_full = stability_matrices(c)
    if w is not None:
        b = w
    g = c["gamma"]
    be = al + ga                                  # beta_ij = alpha_ij + gamma_ij (i > j)
    alpha_i = al.sum(axis=1)                      # alpha_i = sum_j alpha_ij
    betap = be.sum(axis=1)                        # beta'_i = sum_j beta_ij
    a2, a3, a4 = alpha_i[1], alpha_i[2], alpha_i[3]
    bp2, bp3, bp4 = betap[1], betap[2], betap[3]
    b1, b2, b3, b4 = b
    res = {
        "a": b1 + b2 + b3 + b4 - 1.0,
        "b": b2 * bp2 + b3 * bp3 + b4 * bp4 - (0.5 - g),
        "c": b2 * a2**2 + b3 * a3**2 + b4 * a4**2 - 1.0 / 3.0,
        "d": b3 * be[2, 1] * bp2 + b4 * (be[3, 1] * bp2 + be[3, 2] * bp3) - (1.0 / 6.0 - g + g * g),
        "e": b2 * a2**3 + b3 * a3**3 + b4 * a4**3 - 0.25,
        "f": b3 * a3 * al[2, 1] * bp2 + b4 * a4 * (al[3, 1] * bp2 + al[3, 2] * bp3) - (1.0 / 8.0 - g / 3.0),
        "g": b3 * al[2, 1] * a2**2 + b4 * (al[3, 1] * a2**2 + al[3, 2] * a3**2) - 1.0 / 12.0,
        "h": b3 * ga[2, 1] * a2**2 + b4 * (ga[3, 1] * a2**2 + ga[3, 2] * a3**2) - (-g / 3.0),
        # condition (i): the printed b_2' is read as beta'_2
        "i": b4 * be[3, 2] * be[2, 1] * bp2 - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g**3),
    }
    return res


def test_oracle_constants_equal_printed_table(orc, coeffs):
    got = orc.coefficients()
    for k, v in coeffs.items():
        assert got[k] == v, k


def test_fourth_order_conditions(coeffs):
    res = _conditions(coeffs)
    for k, r in res.items():
        assert abs(r) <= 1e-14, (k, r)


def test_embedded_third_order_conditions(coeffs):
    _, bh, *_ = stability_matrices(coeffs)
    res = _conditions(coeffs, w=bh)
    # the printed b-hat_2 carries one digit fewer than the others: sum(bh) = 1 - 4e-15
    for k in "abcd":
        assert abs(res[k]) <= 1e-14, (k, res[k])
    # and b-hat is a genuinely different (lower-order) formula
    assert abs(res["e"]) > 1e-3


def test_literal_row_labels_fail_condition_b(coeffs):
    c = dict(coeffs)
    # literal labels: the second b row assigns 0 to b2 and 0.3224.. to b3
    c["b2"], c["b3"], c["b4"] = 0.0, coeffs["b4"], 0.0
    assert abs(_conditions(c)["b"]) > 0.1


def test_L_stability_and_gamma_root(coeffs):
    b, _, _, _, beta = stability_matrices(coeffs)
    r_inf = 1.0 - b @ np.linalg.solve(beta, np.ones(4))
    assert abs(r_inf) <= 1e-14
    # gamma is 1/x for a root x of the Laguerre polynomial L4 (R(inf) = 0 for 4 stages)
    x = 1.0 / coeffs["gamma"]
    L4 = (x**4 - 16 * x**3 + 72 * x**2 - 96 * x + 24) / 24.0
    assert abs(L4) <= 1e-13
    # the text's rounded value
    assert round(coeffs["gamma"], 3) == 0.573


def test_stage3_and_stage4_share_the_f_argument(coeffs):
    assert coeffs["a43"] == 0.0
    assert coeffs["a41"] == coeffs["a31"] and coeffs["a42"] == coeffs["a32"]
    assert coeffs["b3"] == 0.0


@pytest.mark.parametrize("y", [0.5, 2.0, 10.0, 100.0, 1e4])
def test_A_stable_on_imaginary_axis(coeffs, y):
    from conftest import stability_R
    assert abs(stability_R(coeffs, 1j * y)) <= 1.0 + 1e-12
