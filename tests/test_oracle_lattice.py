"""Pins of the oracle's lattice constants against the paper's Appendix B and Gauss-Hermite theory."""
import math
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")


def _weight(text):
    # a printed decimal, or a closed form a+b*sqrt(193) over an integer (Tab. d2q17)
    m = re.fullmatch(r"\((\d+)([+-]\d+)\*sqrt\(193\)\)/(\d+)", text)
    if m:
        return (int(m.group(1)) + int(m.group(2)) * math.sqrt(193.0)) / int(m.group(3))
    return float(text)


def _paper_table(stencil):
    rows = []
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if len(line) == 5 and int(line[0]) == stencil:
            rows.append(((int(line[1]), int(line[2])), int(line[3]), _weight(line[4])))
    return rows


@pytest.mark.parametrize("stencil", [9, 17, 37])
def test_weights_match_paper_table(stencil):
    # Appendix B, Tab. d2q9 / d2q17 / d2q37: group (a,b) lists every sign/axis permutation
    cs2, w, cx, cy, M = O.lattice(stencil)
    table = _paper_table(stencil)
    assert len(w) == sum(n for _, n, _ in table) == stencil
    for (a, b), count, wp in table:
        members = [i for i in range(len(w)) if sorted((abs(cx[i]), abs(cy[i]))) == sorted((a, b))]
        assert len(members) == count
        for i in members:
            # D2Q37 weights are printed with 14 digits; the others exactly
            assert abs(w[i] - wp) < (2e-14 if stencil == 37 else 1e-16), (a, b, w[i], wp)
    assert M == (1 if stencil == 9 else 3)  # maximum displacement (Sec. 3.3, multi-speed LBM)
    assert max(np.abs(cx).max(), np.abs(cy).max()) == M


def test_d2q9_sound_speed():
    cs2 = O.lattice(9)[0]
    assert abs(cs2 - 1.0 / 3.0) < 1e-15  # Tab. d2q9 caption: cs = 1/sqrt(3)


def test_d2q37_sound_speed_closed_form():
    # Tab. d2q37 caption prints (1/6) sqrt(49 - (119 + a^(2/3)) / a^(1/3)), a = 469 + 252 sqrt(30).
    # That value (0.8665) fails the isotropy conditions; with the sign of a^(2/3) flipped the
    # expression equals 1/cs of the 9th-order rule (reading of a garbled caption).
    cs2 = O.lattice(37)[0]
    a = 469.0 + 252.0 * math.sqrt(30.0)
    inv_cs = (1.0 / 6.0) * math.sqrt(49.0 - (119.0 - a ** (2.0 / 3.0)) / a ** (1.0 / 3.0))
    assert abs(1.0 / math.sqrt(cs2) - inv_cs) < 1e-13
    # cs^2 is also the real root of 35 s^3 - 70 s^2 + 49 s - 12 (elimination of the weights)
    assert abs(35 * cs2 ** 3 - 70 * cs2 ** 2 + 49 * cs2 - 12) < 1e-13


def _gauss_moment(n):
    return 0.0 if n % 2 else float(np.prod(np.arange(n - 1, 0, -2))) if n > 0 else 1.0


def test_d2q17_sound_speed_closed_form():
    # Tab. d2q17 caption prints sqrt(5 (25 + sqrt 193) / 72) = 1.6434; as for D2Q37 the printed
    # expression is 1 / cs of the rule (cs = 0.608 makes the weights of the table isotropic)
    cs2 = O.lattice(17)[0]
    assert abs(1.0 / math.sqrt(cs2) - math.sqrt(5.0 * (25.0 + math.sqrt(193.0)) / 72.0)) < 1e-14


@pytest.mark.parametrize("stencil,order", [(9, 5), (17, 7), (37, 9)])
def test_quadrature_isotropy(stencil, order):
    # Gauss-Hermite quadrature (Sec. 2): sum_i w_i xi_x^a xi_y^b equals the unit Gaussian moments
    # for every a + b <= order (D2Q9: 5th order, D2Q17: 7th order, D2Q37: 9th order).
    cs2, w, cx, cy, _ = O.lattice(stencil)
    xi_x, xi_y = cx / math.sqrt(cs2), cy / math.sqrt(cs2)
    for a in range(order + 1):
        for b in range(order + 1 - a):
            m = np.sum(w * xi_x ** a * xi_y ** b)
            ref = _gauss_moment(a) * _gauss_moment(b)
            assert abs(m - ref) < 1e-12 * max(1.0, abs(ref)), (a, b, m, ref)
    assert abs(w.sum() - 1.0) < 4e-16


@pytest.mark.parametrize("stencil,degree,gauss", [(37, 10, 945.0), (17, 8, 105.0)])
def test_rule_order_is_exact(stencil, degree, gauss):
    # a 9th-order (7th-order) rule: degree-10 (degree-8) moments are not Gaussian
    cs2, w, cx, cy, _ = O.lattice(stencil)
    m = np.sum(w * (cx / math.sqrt(cs2)) ** degree)
    assert abs(m - gauss) > 1.0
