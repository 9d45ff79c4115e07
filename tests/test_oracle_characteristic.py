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
