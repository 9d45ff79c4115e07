"""Pins of the oracle's equilibrium (eq. feq-3 / feq-4) and moments (eq. macro)."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _states(n, seed=7):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = 1.0 + 0.1 * rng.uniform(-1, 1)
        ux, uy = 0.3 * rng.uniform(-1, 1, 2)
        T = 1.0 + 0.1 * rng.uniform(-1, 1)
        yield rho, ux, uy, T


def test_d2q37_equilibrium_moments():
    # 4th-order Hermite equilibrium on a 9th-order rule reproduces the Maxwellian moments up to
    # 4th order: rho, rho u, T (eq. macro), zero 3rd central moment, 4th central moments
    # 3 rho T~^2 and rho T~^2 with T~ = cs^2 T.
    cs2, w, cx, cy, _ = O.lattice(37)
    for rho, ux, uy, T in _states(20):
        f = O.feq(37, rho, ux, uy, T)
        dx, dy = cx - ux, cy - uy
        Tt = cs2 * T
        assert abs(f.sum() - rho) < 1e-14
        assert abs((f * cx).sum() - rho * ux) < 1e-14
        assert abs((f * cy).sum() - rho * uy) < 1e-14
        assert abs((f * (dx * dx + dy * dy)).sum() - 2 * rho * Tt) < 1e-13
        for a, b in [(3, 0), (2, 1), (1, 2), (0, 3)]:
            assert abs((f * dx ** a * dy ** b).sum()) < 1e-13
        assert abs((f * dx ** 4).sum() - 3 * rho * Tt ** 2) < 1e-13
        assert abs((f * dx ** 2 * dy ** 2).sum() - rho * Tt ** 2) < 1e-13
        assert abs((f * dy ** 4).sum() - 3 * rho * Tt ** 2) < 1e-13
        r, mx, my, mT = O.moments(37, f)
        assert max(abs(r - rho), abs(mx - ux), abs(my - uy), abs(mT - T)) < 1e-13


def test_d2q17_equilibrium_moments_third_order():
    # eq. feq-3 on the 7th-order D2Q17 rule: the moments of the Maxwellian up to 3rd order are
    # exact (rho, rho u, T, zero 3rd central moment), and the equilibrium has no 4th-order
    # Hermite component (sum_i f_i He4(xi_i) = 0 for every 4th-order tensor Hermite polynomial)
    cs2, w, cx, cy, _ = O.lattice(17)
    cs = math.sqrt(cs2)
    xx, xy = cx / cs, cy / cs
    he4 = [xx ** 4 - 6 * xx ** 2 + 3, xx ** 3 * xy - 3 * xx * xy, xx ** 2 * xy ** 2 - xx ** 2 - xy ** 2 + 1,
           xx * xy ** 3 - 3 * xx * xy, xy ** 4 - 6 * xy ** 2 + 3]
    for rho, ux, uy, T in _states(20, seed=5):
        f = O.feq(17, rho, ux, uy, T)
        dx, dy = cx - ux, cy - uy
        assert abs(f.sum() - rho) < 1e-14
        assert abs((f * cx).sum() - rho * ux) < 1e-14
        assert abs((f * cy).sum() - rho * uy) < 1e-14
        assert abs((f * (dx * dx + dy * dy)).sum() - 2 * rho * cs2 * T) < 1e-14
        for a, b in [(3, 0), (2, 1), (1, 2), (0, 3)]:
            assert abs((f * dx ** a * dy ** b).sum()) < 1e-14
        for h in he4:
            assert abs((f * h).sum()) < 1e-13
        r, mx, my, mT = O.moments(17, f)
        assert max(abs(r - rho), abs(mx - ux), abs(my - uy), abs(mT - T)) < 1e-14
    # but the 4th central moment is not the Maxwellian's 3 rho T~^2 away from rest
    f = O.feq(17, 1.0, 0.2, 0.1, 1.05)
    assert abs((f * (cx - 0.2) ** 4).sum() - 3 * (cs2 * 1.05) ** 2) > 1e-4


def _paper_feq4(w, cx, cy, cs2, rho, ux, uy, T, k):
    # eq. feq-3 + feq-4 written in the scaled variables xi = c / cs, u / cs (every printed cs
    # factor equals 1 there); k is the constant of the (u.c)^2 (T-1) term (printed: 4)
    cs = math.sqrt(cs2)
    Xx, Xy = cx / cs, cy / cs
    a = Xx * ux / cs + Xy * uy / cs
    u2 = (ux * ux + uy * uy) / cs2
    x2 = Xx * Xx + Xy * Xy
    th = T - 1.0
    h = (1 + a + 0.5 * (a * a - u2 + th * (x2 - 2)) + a / 6 * (a * a - 3 * u2 + 3 * th * (x2 - 4))
         + (a ** 4 - 6 * a * a * u2 + 3 * u2 * u2 + 6 * th * (a * a * (x2 - k) + u2 * (4 - x2))
            + 3 * th * th * (x2 * x2 - 8 * x2 + 8)) / 24)
    return w * rho * h


def test_d2q37_equilibrium_matches_expanded_formula():
    # The oracle builds f^eq from the Hermite tensor definition; the expanded formula of
    # eq. feq-4 (with (xi^2 - 6) in place of the printed (c^2 - 4)) must agree term by term.
    cs2, w, cx, cy, _ = O.lattice(37)
    for rho, ux, uy, T in _states(20, seed=3):
        f = O.feq(37, rho, ux, uy, T)
        g = _paper_feq4(w, cx, cy, cs2, rho, ux, uy, T, 6.0)
        assert np.abs(f - g).max() < 1e-15


def test_printed_feq4_constant_breaks_mass():
    # with the printed constant 4 the zeroth moment is wrong at T != 1 (erratum of eq. feq-4)
    cs2, w, cx, cy, _ = O.lattice(37)
    g = _paper_feq4(w, cx, cy, cs2, 1.02, 0.08, -0.03, 1.03, 4.0)
    assert abs(g.sum() - 1.02) > 1e-5


def test_d2q9_equilibrium_textbook():
    # 2nd-order isothermal truncation: w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
    cs2, w, cx, cy, _ = O.lattice(9)
    for rho, ux, uy, _T in _states(10):
        f = O.feq(9, rho, ux, uy, 1.0)
        cu = cx * ux + cy * uy
        g = w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
        assert np.abs(f - g).max() < 1e-15
        assert abs(f.sum() - rho) < 1e-14
        assert abs((f * cx).sum() - rho * ux) < 1e-14


@pytest.mark.parametrize("stencil", [9, 17, 37])
def test_collision_conserves(stencil):
    # BGK (eq. bgk) conserves mass and momentum; the thermal stencils also energy, for any f
    cs2, w, cx, cy, _ = O.lattice(stencil)
    rng = np.random.default_rng(11)
    tau = 0.8
    for _ in range(10):
        f = w * (1 + 0.05 * rng.standard_normal(len(w)))
        r, ux, uy, T = O.moments(stencil, f)
        fe = O.feq(stencil, r, ux, uy, T)
        fs = f - (f - fe) / tau
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert abs((fs * cx).sum() - (f * cx).sum()) < 1e-15
        assert abs((fs * cy).sum() - (f * cy).sum()) < 1e-15
        if stencil != 9:
            e = cx * cx + cy * cy
            assert abs((fs * e).sum() - (f * e).sum()) < 1e-14
