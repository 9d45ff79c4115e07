"""Pins of the oracle's boundary time integration, transverse terms and corner coupling.

* Time integration (Sec. 3.3, "Time integration"): one classic RK4 step of the layers' evolution
  with the bulk values interpolated linearly in time.  Near a uniform state the layers' system is
  linear, dz/dt = J z + g0 + g1 t (g1 from the bulk values' change over the step), and RK4
  reproduces the degree-4 Taylor polynomial of its exact solution,
      z(1) = g0 + (J g0 + g1)/2 + (J^2 g0 + J g1)/6 + (J^3 g0 + J^2 g1)/24,
  which the tests build from J, g0 and g1 measured through the oracle's right-hand-side probe
  (bulk values interpolated here, not by the oracle) and compare with the oracle's step.  Wrong
  stage weights or offsets, or bulk values held at t during the half-step stages, change the
  coefficients of this polynomial.
* Transverse terms (eq. NSF-CHAR): T = -B d_s U (s the coordinate along the side) with B the
  tangential flux Jacobian of the inviscid NSF system in the side's local variables, derived
  here independently.
* Corner coupling (Sec. 3.3, corner treatment): the end rows of a side take the corner block's
  value as the neighbour beyond the end, at time t and t + dt interpolated like bulk values (the
  RK4 pins run with corners), so a field whose corner value continues it smoothly has the same
  transverse terms at the end rows as at any other row.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O

CHAR = ("lodi", "lodi_relax", "cbc", "cbc_relax")


def _tau(stencil):
    return {9: 0.8, 17: 0.9, 37: 0.5 + 0.1 / O.lattice(37)[0]}[stencil]


def _layer_nodes(nx, ny, bc, side, M):
    """(x, y) of layer j (1..M), row r of a side, as the oracle orders its rows."""
    nax = 0 if side < 2 else 1
    sn = -1 if side % 2 == 0 else 1
    Nn, Nt = (nx, ny) if nax == 0 else (ny, nx)
    tper = (bc[2] == "periodic") if nax == 0 else (bc[0] == "periodic")
    r0 = 0 if tper else M
    length = Nt if tper else Nt - 2 * M
    xf = Nn - 1 - M if sn > 0 else M
    out = np.zeros((M, length, 2), dtype=int)
    for j in range(1, M + 1):
        for r in range(length):
            n, t = xf + sn * j, r0 + r
            out[j - 1, r] = (n, t) if nax == 0 else (t, n)
    return out


def _near_uniform(nx, ny, u, eps, seed):
    rng = np.random.default_rng(seed)
    base = np.array([1.0, u[0], u[1], 1.0])[:, None, None] * np.ones((4, ny, nx))
    return base + eps * rng.standard_normal((4, ny, nx))


def _taylor_rk4(J, g0, g1):
    Jg0, Jg1 = J @ g0, J @ g1
    J2g0, J2g1 = J @ Jg0, J @ Jg1
    return g0 + 0.5 * (Jg0 + g1) + (J2g0 + Jg1) / 6.0 + (J @ J2g0 + J2g1) / 24.0


SIDE_CASES = [
    # stencil, nx, ny, bc, tested side, outflow velocity (global), viscous mode
    (37, 14, 6, ["lodi", "lodi_relax", "periodic", "periodic"], 1, (0.05, 0.02), None),
    (37, 14, 12, ["lodi_relax", "cbc_relax", "lodi_relax", "cbc"], 1, (0.05, 0.02), None),
    (37, 14, 12, ["lodi_relax", "cbc_relax", "lodi_relax", "cbc"], 3, (0.02, 0.05), None),
    (37, 12, 12, ["cbc", "cbc_relax", "lodi", "lodi"], 1, (0.05, -0.03), "fd"),
    (37, 12, 12, ["cbc_relax", "lodi", "cbc_relax", "lodi_relax"], 0, (-0.05, 0.03), None),
    (17, 12, 10, ["lodi_relax", "cbc_relax", "lodi", "lodi"], 1, (0.05, 0.02), None),
    (9, 10, 8, ["lodi_relax", "lodi_relax", "periodic", "periodic"], 1, (0.05, 0.02), None),
    (9, 10, 8, ["lodi_relax", "lodi", "lodi_relax", "lodi"], 2, (0.02, -0.05), None),
]


@pytest.mark.parametrize("case", SIDE_CASES, ids=lambda c: f"q{c[0]}-{'-'.join(c[3])}-side{c[4]}-{c[6]}")
def test_side_rk4_step_is_the_taylor_polynomial(case):
    stencil, nx, ny, bc, side, u, visc = case
    M = O.lattice(stencil)[4]
    o = O.Oracle(stencil, nx, ny, _tau(stencil), bc)
    o.set_relax(-1, sigma=0.3, alpha=0.4, mach=0.1)
    if visc:
        o.set_viscous(side, visc)
    eps = 1e-6
    # the pre-collision populations (frozen mesoscopic viscous terms) of a perturbed state
    o.init(*_near_uniform(nx, ny, u, eps, 1))
    Ut = _near_uniform(nx, ny, u, eps, 2)
    Unp1 = Ut + eps * np.random.default_rng(3).standard_normal(Ut.shape)
    nodes = _layer_nodes(nx, ny, bc, side, M)
    xs, ys = nodes[..., 0], nodes[..., 1]
    Y0 = np.moveaxis(Ut[:, ys, xs], 0, -1)          # [M][len][4]

    def field(theta):
        F = (1 - theta) * Ut + theta * Unp1
        F[:, ys, xs] = np.moveaxis(Y0, -1, 0)       # wave directions from the layers at t
        return F

    F0, F1 = field(0.0), field(1.0)
    g0 = o.side_rhs_probe(side, F0, Y0).ravel()
    g1 = o.side_rhs_probe(side, F1, Y0).ravel() - g0
    n = g0.size
    J = np.zeros((n, n))
    h = 1e-5
    for k in range(n):
        d = np.zeros(n)
        d[k] = h
        J[:, k] = (o.side_rhs_probe(side, F0, (Y0.ravel() + d).reshape(Y0.shape)).ravel()
                   - o.side_rhs_probe(side, F0, (Y0.ravel() - d).reshape(Y0.shape)).ravel()) / (2 * h)
    want = _taylor_rk4(J, g0, g1)
    got = (o.side_step_probe(side, Ut, Unp1) - Y0).ravel()
    scale = np.abs(want).max()
    assert scale > 1e-8
    assert np.abs(got - want).max() < 1e-4 * scale, (np.abs(got - want).max(), scale)
    # the bulk values' change and the layers' own coupling both matter in this setup
    assert np.abs(0.5 * g1).max() > 0.05 * scale
    assert np.abs(0.5 * J @ g0).max() > 0.05 * scale


@pytest.mark.parametrize("stencil,cidx", [(37, 0), (37, 3), (17, 1), (9, 2)])
def test_corner_rk4_step_is_the_taylor_polynomial(stencil, cidx):
    M = O.lattice(stencil)[4]
    nx, ny = 12, 10
    bc = ["lodi_relax", "lodi", "lodi", "lodi_relax"]
    o = O.Oracle(stencil, nx, ny, _tau(stencil), bc)
    o.set_relax(-1, sigma=0.3, alpha=0.4, mach=0.1)
    eps = 1e-6
    sx, sy = cidx & 1, cidx >> 1
    # flow out through the corner along its diagonal
    u = (0.04 * (1 if sx else -1), 0.03 * (1 if sy else -1))
    o.init(*_near_uniform(nx, ny, u, eps, 1))
    Ut = _near_uniform(nx, ny, u, eps, 4)
    Unp1 = Ut + eps * np.random.default_rng(5).standard_normal(Ut.shape)
    # innermost corner node and the two inward diagonal bulk nodes
    x = nx - M if sx else M - 1
    y = ny - M if sy else M - 1
    vx, vy = (-1 if sx else 1), (-1 if sy else 1)
    U0 = Ut[:, y, x]
    B = [(Ut[:, y + k * vy, x + k * vx], Unp1[:, y + k * vy, x + k * vx]) for k in (1, 2)]

    def rhs(Uc, theta):
        b1 = (1 - theta) * B[0][0] + theta * B[0][1]
        b2 = (1 - theta) * B[1][0] + theta * B[1][1]
        return o.corner_rhs_probe(cidx, Uc, U0, b1, b2)

    nc = 4 if stencil != 9 else 3
    g0 = rhs(U0, 0.0)[:nc]
    g1 = rhs(U0, 1.0)[:nc] - g0
    J = np.zeros((nc, nc))
    h = 1e-5
    for k in range(nc):
        d = np.zeros(4)
        d[k] = h
        J[:, k] = (rhs(U0 + d, 0.0)[:nc] - rhs(U0 - d, 0.0)[:nc]) / (2 * h)
    want = _taylor_rk4(J, g0, g1)
    got = (o.corner_step_probe(cidx, Ut, Unp1) - U0)[:nc]
    scale = np.abs(want).max()
    assert scale > 1e-8
    assert np.abs(got - want).max() < 1e-4 * scale, (got, want)
    assert np.abs(0.5 * g1).max() > 0.05 * scale


def _tangential_jacobian(cs2, U, thermal=True):
    # d_t U + B d_s U = 0 with s the coordinate along the side: the tangential flux Jacobian of
    # the inviscid NSF system (eq. NSF with P = rho cs^2 T, c_v = 1 in d = 2) in the local
    # variables (rho, u_n, u_t, T), derived here from
    #   d_t rho + u_t d_s rho + rho d_s u_t = 0
    #   d_t u_n + u_t d_s u_n = 0
    #   d_t u_t + u_t d_s u_t + (cs^2 T / rho) d_s rho + cs^2 d_s T = 0
    #   d_t T   + u_t d_s T + T d_s u_t = 0
    # (isothermal: T = 1 fixed and no energy row)
    rho, un, ut, T = U
    B = np.diag([ut] * 4)
    B[0, 2] = rho
    B[2, 0] = cs2 * T / rho
    if thermal:
        B[2, 3] = cs2
        B[3, 2] = T
    else:
        B[3, 3] = 0.0
    return B


def _smooth_along(nx, ny, along_x, k, A=2e-3):
    """Fields that vary along one axis only (x if along_x, else y), with every component's
    derivative comparable, plus a non-zero normal and tangential base velocity."""
    X, Y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    s = X if along_x else Y
    a, b = np.sin(k * s + 0.4), np.cos(k * s + 1.1)
    ut0, un0 = 0.1, 0.05
    tang = ut0 + A * (a - b)
    norm = un0 + A * (a + 0.5 * b)
    ux, uy = (tang, norm) if along_x else (norm, tang)
    return [1 + A * (a + 0.5 * b), ux, uy, 1 + A * (b - 0.3 * a)]


def _local_analytic(side, along_x, k, t, thermal=True, A=2e-3):
    # exact values and tangential derivatives of _smooth_along at tangential coordinate t, in
    # the local frame of the side (u_n = sn * normal component); T = 1 on the isothermal stencil
    sn = -1 if side % 2 == 0 else 1

    def loc(tt):
        a, b = math.sin(k * tt + 0.4), math.cos(k * tt + 1.1)
        return np.array([1 + A * (a + 0.5 * b), sn * (0.05 + A * (a + 0.5 * b)), 0.1 + A * (a - b),
                         1 + A * (b - 0.3 * a) if thermal else 1.0])

    h = 1e-5
    return loc(t), (loc(t + h) - loc(t - h)) / (2 * h)


@pytest.mark.parametrize("stencil,side", [(37, 0), (37, 1), (37, 2), (37, 3), (17, 1), (9, 1), (9, 2)])
def test_transverse_terms_are_the_tangential_fluxes(stencil, side):
    # periodic tangent, field varying along the side only: -B d_s U to O(k^2) on every layer
    cs2, *_, M = O.lattice(stencil)
    thermal = stencil != 9
    n_t, k = 48, 2 * math.pi / 48
    along_x = side >= 2
    nx, ny = (n_t, 14) if along_x else (14, n_t)
    bc = ["periodic", "periodic", "cbc", "lodi"] if along_x else ["cbc", "lodi", "periodic", "periodic"]
    if not thermal:
        bc = [b if b == "periodic" else "lodi" for b in bc]
    o = O.Oracle(stencil, nx, ny, _tau(stencil), bc)
    o.init(*_smooth_along(nx, ny, along_x, k))
    for j, r in itertools.product(range(1, M + 1), (3, 17, 40)):
        U, dU = _local_analytic(side, along_x, k, r, thermal)
        ref = -_tangential_jacobian(cs2, U, thermal) @ dU
        got = o.transverse_probe(side, j, r)
        n = 4 if thermal else 3
        for m in range(n):
            # central differences: relative O(k^2 / 6) = 0.3 % apart from the product-rule form
            assert abs(got[m] - ref[m]) <= 0.01 * abs(ref[m]) + 1e-12, (side, j, r, m, got, ref)


@pytest.mark.parametrize("stencil,side", [(37, 0), (37, 1), (37, 2), (37, 3), (17, 2), (9, 1)])
def test_end_rows_see_the_corner_block(stencil, side):
    # all four sides characteristic: the rows of a side run over [M, Nt - 1 - M] and the
    # neighbour of an end row beyond the end is the corner block, whose value is that of its
    # innermost node (x_{b,1}, y_{b,1}).  With a field that varies along the side only, that
    # value continues the field smoothly, so the end rows' transverse terms equal -B d_s U to
    # O(k^2) like those of any other row (a one-sided difference at the ends is off by O(k),
    # the wrong corner or a corner at the wrong row by O(1)).
    cs2, *_, M = O.lattice(stencil)
    thermal = stencil != 9
    n_t, k = 30, 2 * math.pi / 60
    along_x = side >= 2
    nx, ny = (n_t, 14) if along_x else (14, n_t)
    bc = ["lodi", "cbc", "lodi_relax", "cbc_relax"] if thermal else ["lodi", "lodi_relax", "lodi", "lodi"]
    o = O.Oracle(stencil, nx, ny, _tau(stencil), bc)
    o.init(*_smooth_along(nx, ny, along_x, k))
    length = o.side_len(side)
    assert length == n_t - 2 * M
    n = 4 if thermal else 3
    for j, r in itertools.product(range(1, M + 1), (0, length - 1)):
        t = M + r                                   # tangential coordinate of the row
        U, dU = _local_analytic(side, along_x, k, t, thermal)
        ref = -_tangential_jacobian(cs2, U, thermal) @ dU
        got = o.transverse_probe(side, j, r)
        for m in range(n):
            assert abs(got[m] - ref[m]) <= 0.01 * abs(ref[m]) + 1e-12, (side, j, r, m, got, ref)
