"""ctypes wrapper of the FP64 CPU oracle (lbm_oracle.cpp).

TEST INFRASTRUCTURE: only the tests, the package smoke check and the CPU-baseline leg of the
benchmark use this module.  Arrays are float64, row-major [ny][nx] with x fastest.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

BC = {"periodic": 0, "lodi": 1, "lodi_relax": 2, "cbc": 3, "cbc_relax": 4, "zg": 5, "dirichlet": 6}
NTAN = 3

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_error.restype = ctypes.c_char_p
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_lattice.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _ip, _ip]
        L.oracle_feq.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [_dp]
        L.oracle_moments.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle_char_matrices.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_side_len.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_set_relax.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.oracle_set_inlet.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.oracle_set_recon.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.oracle_set_viscous.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.oracle_visc_fd_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_macro.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        L.oracle_pops.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_diag.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_visc_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_corner_rhs_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.oracle_side_rhs_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_side_step_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_corner_step_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_transverse_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_loss.restype = ctypes.c_double
        L.oracle_loss.argtypes = [ctypes.c_void_p]
        L.oracle_tangent_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip,
                                         _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_tangent_run_fields.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip,
                                                _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_tangent_run_fields_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip,
                                                   _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _ip, ctypes.c_int, _dp]
        _LIB = L
    return _LIB


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return lib().oracle_num_threads()


def set_threads(n):
    """Threads for the oracle's OpenMP loops from now on."""
    lib().oracle_set_threads(int(n))


def lattice(stencil):
    """(cs2, w[q], cx[q], cy[q], M) as derived by the oracle."""
    L = lib()
    q, M = ctypes.c_int(), ctypes.c_int()
    cs2 = ctypes.c_double()
    w = np.zeros(64)
    cx = np.zeros(64, dtype=np.int32)
    cy = np.zeros(64, dtype=np.int32)
    rc = L.oracle_lattice(stencil, ctypes.byref(q), ctypes.byref(M), ctypes.byref(cs2), _ptr(w),
                          cx.ctypes.data_as(_ip), cy.ctypes.data_as(_ip))
    if rc != 0:
        raise ValueError("unknown stencil")
    n = q.value
    return cs2.value, w[:n].copy(), cx[:n].copy(), cy[:n].copy(), M.value


def feq(stencil, rho, ux, uy, T):
    cs2, w, *_ = lattice(stencil)
    out = np.zeros(len(w))
    lib().oracle_feq(stencil, rho, ux, uy, T, _ptr(out))
    return out


def moments(stencil, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(4)
    lib().oracle_moments(stencil, _ptr(f), _ptr(out))
    return out


def char_matrices(stencil, U):
    """A, S, S^-1, Lambda at the local-frame state U = (rho, u_n, u_t, T)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    A, S, Si = np.zeros(16), np.zeros(16), np.zeros(16)
    lam = np.zeros(4)
    n = lib().oracle_char_matrices(stencil, _ptr(U), _ptr(A), _ptr(S), _ptr(Si), _ptr(lam))
    return A[:n * n].reshape(n, n), S[:n * n].reshape(n, n), Si[:n * n].reshape(n, n), lam[:n]


def _bc_codes(bc):
    return [BC[b] if isinstance(b, str) else int(b) for b in bc]


class Oracle:
    """One oracle simulation.  bc = [x0, x1, y0, y1] names or codes."""

    def __init__(self, stencil, nx, ny, tau, bc):
        self.stencil, self.nx, self.ny, self.tau = stencil, nx, ny, tau
        self.bc = _bc_codes(bc)
        arr = (ctypes.c_int * 4)(*self.bc)
        h = lib().oracle_create(stencil, nx, ny, tau, arr)
        if not h:
            raise ValueError(lib().oracle_error().decode())
        self.h = ctypes.c_void_p(h)

    def close(self):
        if self.h:
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def side_len(self, side):
        return lib().oracle_side_len(self.h, side)

    def set_relax(self, side, sigma=0.0, alpha=0.0, rho_inf=1.0, T_inf=1.0, mach=0.0, length=0.0):
        sides = range(4) if side < 0 else [side]
        p = np.array([sigma, alpha, rho_inf, T_inf, mach, length], dtype=np.float64)
        for s in sides:
            lib().oracle_set_relax(self.h, s, _ptr(p))

    def set_inlet(self, side, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        if lib().oracle_set_inlet(self.h, side, _ptr(U)) != 0:
            raise ValueError("side is not a Dirichlet side")

    def corner_rhs_probe(self, cidx, Uc, Ucn, B1, B2):
        """Corner LODI right-hand side (Sec. 3.3, corner treatment) for given states."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (Uc, Ucn, B1, B2)]
        out = np.zeros(4)
        if lib().oracle_corner_rhs_probe(self.h, cidx, *[_ptr(a) for a in arrs], _ptr(out)) != 0:
            raise ValueError("no characteristic corner there")
        return out

    def _field(self, F):
        return np.ascontiguousarray(np.broadcast_to(np.asarray(F, dtype=np.float64), (4, self.ny, self.nx)))

    def side_rhs_probe(self, side, Uv, Y):
        """Right-hand side of a characteristic side's layers at stage values Y [M][len][4]; bulk
        nodes, corner blocks and the wave directions are read from the field Uv [4][ny][nx]."""
        Uv = self._field(Uv)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        K = np.zeros_like(Y)
        if lib().oracle_side_rhs_probe(self.h, side, _ptr(Uv), _ptr(Y), _ptr(K)) != 0:
            raise ValueError("not a characteristic side")
        return K

    def side_step_probe(self, side, Ut, Unp1):
        """One RK4 boundary step of a side from field Ut to t + dt (bulk/corners at t + dt from
        Unp1); returns the layers' new values [M][len][4]."""
        Ut, Unp1 = self._field(Ut), self._field(Unp1)
        M = lattice(self.stencil)[4]
        Y1 = np.zeros((M, self.side_len(side), 4))
        if lib().oracle_side_step_probe(self.h, side, _ptr(Ut), _ptr(Unp1), _ptr(Y1)) != 0:
            raise ValueError("not a characteristic side")
        return Y1

    def corner_step_probe(self, cidx, Ut, Unp1):
        """One RK4 step of a corner's diagonal LODI analysis; returns the corner value at t + dt."""
        Ut, Unp1 = self._field(Ut), self._field(Unp1)
        out = np.zeros(4)
        if lib().oracle_corner_step_probe(self.h, cidx, _ptr(Ut), _ptr(Unp1), _ptr(out)) != 0:
            raise ValueError("no characteristic corner there")
        return out

    def transverse_probe(self, side, j, r):
        """Transverse terms (local components rho, u_n, u_t, T) at layer j, row r of a side."""
        out = np.zeros(4)
        if lib().oracle_transverse_probe(self.h, side, j, r, _ptr(out)) != 0:
            raise ValueError("bad probe position")
        return out

    def set_recon(self, side, mode):
        """Mesoscopic BC of a characteristic side: "equilibrium" or "neep" (eq. NEEP)."""
        m = {"equilibrium": 0, "neep": 1}[mode]
        if lib().oracle_set_recon(self.h, side, m) != 0:
            raise ValueError("NEEP needs a characteristic side")

    def visc_fd_probe(self, side, j, r):
        """V (local components) of the -FD variant at layer j, row r of a side, at the current time."""
        out = np.zeros(4)
        if lib().oracle_visc_fd_probe(self.h, side, j, r, _ptr(out)) != 0:
            raise ValueError("bad probe position")
        return out

    def set_viscous(self, side, mode):
        """Viscous terms of a CBC side: "meso" (eq. LaplaceU / LaplaceT) or "fd" (Sec. 4.2)."""
        m = {"meso": 0, "fd": 1}[mode]
        if lib().oracle_set_viscous(self.h, side, m) != 0:
            raise ValueError("finite-difference viscous terms need a CBC side")

    def init(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.ny, self.nx)))
                for a in (rho, ux, uy, T)]
        self._keep = arrs
        lib().oracle_init(self.h, *[_ptr(a) for a in arrs])

    def step(self, n=1):
        lib().oracle_step(self.h, n)

    def macro(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(4)]
        lib().oracle_macro(self.h, *[_ptr(a) for a in out])
        return out

    def pops(self):
        q = lattice(self.stencil)[1].size
        f = np.zeros((q, self.ny, self.nx))
        lib().oracle_pops(self.h, _ptr(f))
        return f

    def diag(self):
        out = np.zeros(8)
        lib().oracle_diag(self.h, _ptr(out))
        return out

    def loss(self):
        return lib().oracle_loss(self.h)

    def visc_probe(self, nax, sn, x, y):
        """Viscous terms (0, V_n, V_t, V_T) in the local frame of a would-be side (see C source)."""
        out = np.zeros(4)
        if lib().oracle_visc_probe(self.h, nax, sn, x, y, _ptr(out)) != 0:
            raise ValueError("probe stencil leaves the domain")
        return out


def tangent_run(stencil, nx, ny, tau, bc, relax, dsigma, dalpha, fields, dT, nsteps):
    """Loss and its NTAN directional derivatives (forward mode, dual numbers).

    relax: [4][6] per-side (sigma, alpha, rho_inf, T_inf, mach, length); dsigma, dalpha: [NTAN];
    fields: (rho, ux, uy, T) [ny][nx]; dT: [NTAN][ny][nx].
    """
    codes = (ctypes.c_int * 4)(*_bc_codes(bc))
    relax = np.ascontiguousarray(relax, dtype=np.float64).reshape(4, 6)
    ds = np.ascontiguousarray(dsigma, dtype=np.float64).reshape(NTAN)
    da = np.ascontiguousarray(dalpha, dtype=np.float64).reshape(NTAN)
    fl = [np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx) for a in fields]
    dT = np.ascontiguousarray(dT, dtype=np.float64).reshape(NTAN, ny, nx)
    out = np.zeros(1 + NTAN)
    rc = lib().oracle_tangent_run(stencil, nx, ny, tau, codes, _ptr(relax), _ptr(ds), _ptr(da),
                                  *[_ptr(a) for a in fl], _ptr(dT), nsteps, _ptr(out))
    if rc != 0:
        raise ValueError(lib().oracle_error().decode())
    return out[0], out[1:].copy()


def tangent_run_fields(stencil, nx, ny, tau, bc, relax, dsigma, dalpha, fields, dF, nsteps, wlin=None, visc=None,
                       recon=None):
    """Loss and its NTAN directional derivatives with tangents on all four initial fields.

    dF: [NTAN][4][ny][nx] perturbation of (rho0, ux0, uy0, T0) per direction.  wlin: None for
    the pressure loss, or [4][ny][nx] weights of the linear loss sum w . (rho, ux, uy, T) of the
    final fields over every node.  visc: None, or the viscous terms of each side ("meso" or "fd",
    CBC sides).  recon: None, or the mesoscopic BC of each side ("equilibrium" or "neep").
    """
    codes = (ctypes.c_int * 4)(*_bc_codes(bc))
    relax = np.ascontiguousarray(relax, dtype=np.float64).reshape(4, 6)
    ds = np.ascontiguousarray(dsigma, dtype=np.float64).reshape(NTAN)
    da = np.ascontiguousarray(dalpha, dtype=np.float64).reshape(NTAN)
    fl = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx))) for a in fields]
    dF = np.ascontiguousarray(dF, dtype=np.float64).reshape(NTAN, 4, ny, nx)
    w = None if wlin is None else np.ascontiguousarray(wlin, dtype=np.float64).reshape(4, ny, nx)
    out = np.zeros(1 + NTAN)
    vm = None if visc is None else (ctypes.c_int * 4)(*[{"meso": 0, "fd": 1}[v] for v in visc])
    rm = None if recon is None else (ctypes.c_int * 4)(*[{"equilibrium": 0, "neep": 1}[v] for v in recon])
    rc = lib().oracle_tangent_run_fields_ex(stencil, nx, ny, tau, codes, _ptr(relax), _ptr(ds), _ptr(da),
                                            *[_ptr(a) for a in fl], _ptr(dF), _ptr(w) if w is not None else None,
                                            vm, rm, nsteps, _ptr(out))
    if rc != 0:
        raise ValueError(lib().oracle_error().decode())
    return out[0], out[1:].copy()
