"""Pins of the oracle's characteristic matrices (Sec. 3.1: A = S^-1 Lambda S)."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _euler_A(cs2, rho, u, T):
    # primitive-variable Jacobian of the 1D inviscid NSF system in the normal direction, derived
    # from eq. NSF with P = rho cs^2 T, c_v = 1 (d = 2):
    #   d_t rho + u d rho + rho d u = 0
    #   d_t u   + u d u   + (cs^2 T / rho) d rho + cs^2 d T = 0
    #   d_t v   + u d v   = 0
    #   d_t T   + u d T   + T d u = 0
    return np.array([[u, rho, 0, 0],
                     [cs2 * T / rho, u, 0, cs2],
                     [0, 0, u, 0],
                     [0, T, 0, u]])


def _states():
    rng = np.random.default_rng(5)
    for _ in range(10):
        yield np.array([1 + 0.1 * rng.uniform(-1, 1), 0.2 * rng.uniform(-1, 1),
                        0.2 * rng.uniform(-1, 1), 1 + 0.1 * rng.uniform(-1, 1)])


def test_thermal_diagonalisation():
    cs2 = O.lattice(37)[0]
    for U in _states():
        A, S, Si, lam = O.char_matrices(37, U)
        assert np.abs(S @ Si - np.eye(4)).max() < 1e-14
        assert np.abs(Si @ np.diag(lam) @ S - _euler_A(cs2, *U[[0, 1]], U[3])).max() < 1e-14
        assert np.abs(A - _euler_A(cs2, U[0], U[1], U[3])).max() < 1e-15
        s = math.sqrt(2 * cs2 * U[3])  # adiabatic sound speed, gamma = c_p / c_v = 2
        assert np.allclose(lam, [U[1], U[1], U[1] - s, U[1] + s], atol=1e-15)


def test_printed_S41_is_an_erratum():
    # with S_41 = T~/(4 rho cs) as printed, S S^-1 != I
    cs2 = O.lattice(37)[0]
    U = np.array([1.01, 0.05, 0.02, 1.02])
    A, S, Si, lam = O.char_matrices(37, U)
    S2 = S.copy()
    S2[3, 0] = cs2 * U[3] / (4 * U[0] * math.sqrt(cs2))
    assert np.abs(S2 @ Si - np.eye(4)).max() > 1e-3


def test_isothermal_diagonalisation():
    cs2 = O.lattice(9)[0]
    cs = math.sqrt(cs2)
    for U in _states():
        rho, u = U[0], U[1]
        A, S, Si, lam = O.char_matrices(9, U)
        Aref = np.array([[u, rho, 0], [cs2 / rho, u, 0], [0, 0, u]])
        assert np.abs(S @ Si - np.eye(3)).max() < 1e-14
        assert np.abs(Si @ np.diag(lam) @ S - Aref).max() < 1e-14
        assert np.allclose(lam, [u, u - cs, u + cs], atol=1e-15)


def test_wave_amplitudes_match_printed_form():
    # eq. thermal_WAV, written with T~ = cs^2 T, against Lambda S dU/dx from the matrices
    cs2 = O.lattice(37)[0]
    rng = np.random.default_rng(2)
    for U in _states():
        dU = rng.standard_normal(4)
        A, S, Si, lam = O.char_matrices(37, U)
        L = lam * (S @ dU)
        rho, u, _, T = U
        Tt = cs2 * T
        dr, du, dv, dT = dU
        dTt = cs2 * dT
        ref = [u * (-Tt / (2 * rho * cs2) * dr + dTt / (2 * cs2)),
               u * dv,
               (u - math.sqrt(2 * Tt)) * (Tt / (4 * rho * cs2) * dr - math.sqrt(Tt / (8 * cs2 ** 2)) * du + dTt / (4 * cs2)),
               (u + math.sqrt(2 * Tt)) * (Tt / (4 * rho * cs2) * dr + math.sqrt(Tt / (8 * cs2 ** 2)) * du + dTt / (4 * cs2))]
        assert np.abs(L - np.array(ref)).max() < 1e-14


def _lodi_rate_by_eigenprojection(cs2, n, Uc, U0, B1, B2):
    """LODI rate of the corner's diagonal analysis, computed independently: local frame along the
    outward diagonal n, one-sided difference over the two inward diagonal nodes (spacing sqrt 2),
    the Euler Jacobian's eigenspaces from a numerical eigendecomposition, outgoing families (by
    the eigenvalue at U0) kept, incoming ones zero; back to global components."""
    t = np.array([-n[1], n[0]])

    def loc(U):
        return np.array([U[0], U[1] * n[0] + U[2] * n[1], U[1] * t[0] + U[2] * t[1], U[3]])

    l0, l1, l2, ln = loc(Uc), loc(B1), loc(B2), loc(U0)
    dn = (3 * l0 - 4 * l1 + l2) / (2 * math.sqrt(2))
    A = _euler_A(cs2, l0[0], l0[1], l0[3])
    w, V = np.linalg.eig(A)
    w, V = w.real, V.real
    Vi = np.linalg.inv(V)
    s0 = math.sqrt(2 * cs2 * ln[3])
    u, s = l0[1], math.sqrt(2 * cs2 * l0[3])
    rate = np.zeros(4)
    # eigenvalue families u (entropy, shear), u - s, u + s and their frozen counterparts at U0
    for lam, lam0 in ((u, ln[1]), (u - s, ln[1] - s0), (u + s, ln[1] + s0)):
        sel = np.abs(w - lam) < 1e-9
        if lam0 >= 0.0:
            P = V[:, sel] @ Vi[sel, :]            # projector onto the family's eigenspace
            rate -= lam * (P @ dn)
    return np.array([rate[0], rate[1] * n[0] + rate[2] * t[0], rate[1] * n[1] + rate[2] * t[1], rate[3]])


@pytest.mark.parametrize("cidx", [0, 1, 2, 3])
def test_corner_diagonal_lodi_rate(cidx):
    # Sec. 3.3, corner treatment: the oracle's corner right-hand side equals a LODI analysis along
    # the outward diagonal built from a numerical eigendecomposition of the Euler Jacobian (no
    # use of the printed S, S^-1), for states with either sign of the diagonal velocity
    cs2 = O.lattice(37)[0]
    o = O.Oracle(37, 12, 12, 0.8, ["lodi"] * 4)
    sx = -1 if cidx in (0, 2) else 1
    sy = -1 if cidx in (0, 1) else 1
    n = np.array([sx, sy]) / math.sqrt(2)
    rng = np.random.default_rng(40 + cidx)
    for _ in range(12):
        Uc = np.array([1 + 0.05 * rng.uniform(-1, 1), 0.1 * rng.uniform(-1, 1), 0.1 * rng.uniform(-1, 1),
                       1 + 0.05 * rng.uniform(-1, 1)])
        U0 = Uc + 0.01 * rng.uniform(-1, 1, 4)
        B1 = Uc + 0.02 * rng.uniform(-1, 1, 4)
        B2 = Uc + 0.02 * rng.uniform(-1, 1, 4)
        got = o.corner_rhs_probe(cidx, Uc, U0, B1, B2)
        ref = _lodi_rate_by_eigenprojection(cs2, n, Uc, U0, B1, B2)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), (cidx, got, ref)
    o.close()
