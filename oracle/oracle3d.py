"""ctypes wrapper of the three-dimensional FP64 CPU oracle (lbm3d_oracle.cpp, Appendix A).

TEST INFRASTRUCTURE: only the tests, the package smoke check and the CPU-baseline leg of the
benchmark use this module.  Fields are float64 [nz][ny][nx] with x fastest; the box is periodic in
y and z, boundaries sit on the two x-faces.
"""
import ctypes

import numpy as np

from . import oracle as _o2

BC = {"periodic": 0, "lodi": 1, "lodi_relax": 2, "cbc": 3, "cbc_relax": 4, "zg": 5}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_ready = False


def _ptr(a):
    return a.ctypes.data_as(_dp)


def lib():
    global _ready
    L = _o2.lib()
    if not _ready:
        L.oracle3d_last_error.restype = ctypes.c_char_p
        L.oracle3d_lattice.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _ip, _ip, _ip]
        L.oracle3d_feq.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5 + [_dp]
        L.oracle3d_moments.argtypes = [ctypes.c_int, _dp, _dp]
        L.oracle3d_char_matrices.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.oracle3d_create.restype = ctypes.c_void_p
        L.oracle3d_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip]
        L.oracle3d_create_axis.restype = ctypes.c_void_p
        L.oracle3d_create_axis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip,
                                           ctypes.c_int]
        L.oracle3d_destroy.argtypes = [ctypes.c_void_p]
        L.oracle3d_set_relax.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_double] * 6
        L.oracle3d_set_recon.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.oracle3d_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.oracle3d_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle3d_macro.argtypes = [ctypes.c_void_p, _dp]
        L.oracle3d_pops.argtypes = [ctypes.c_void_p, _dp]
        L.oracle3d_diag.argtypes = [ctypes.c_void_p, _dp]
        L.oracle3d_transverse_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle3d_visc_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        _ready = True
    return L


def lattice(stencil=39):
    """(cs2, w[q], cx[q], cy[q], cz[q], M) as derived by the oracle."""
    q, M, cs2 = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    w = np.zeros(128)
    c = [np.zeros(128, dtype=np.int32) for _ in range(3)]
    if lib().oracle3d_lattice(stencil, ctypes.byref(q), ctypes.byref(M), ctypes.byref(cs2), _ptr(w),
                              *[a.ctypes.data_as(_ip) for a in c]) != 0:
        raise ValueError("unknown stencil")
    n = q.value
    return cs2.value, w[:n].copy(), c[0][:n].copy(), c[1][:n].copy(), c[2][:n].copy(), M.value


def feq(rho, ux, uy, uz, T, stencil=39):
    q = lattice(stencil)[1].size
    out = np.zeros(q)
    lib().oracle3d_feq(stencil, rho, ux, uy, uz, T, _ptr(out))
    return out


def moments(f, stencil=39):
    out = np.zeros(5)
    lib().oracle3d_moments(stencil, _ptr(np.ascontiguousarray(f, dtype=np.float64)), _ptr(out))
    return out


def char_matrices(U, stencil=39):
    """A, S, S^-1 (5 x 5) and Lambda at the local state U = (rho, u_n, u_t1, u_t2, T)."""
    A, S, Si, lam = np.zeros(25), np.zeros(25), np.zeros(25), np.zeros(5)
    lib().oracle3d_char_matrices(stencil, _ptr(np.asarray(U, dtype=np.float64)), _ptr(A), _ptr(S), _ptr(Si), _ptr(lam))
    return A.reshape(5, 5), S.reshape(5, 5), Si.reshape(5, 5), lam


class Oracle3D:
    """One 3D simulation: D3Q39, bc = [low face, high face] of the axis `axis` (0 = x, 1 = y,
    2 = z), periodic along the other two axes."""

    def __init__(self, nx, ny, nz, tau, bc, stencil=39, axis=0):
        self.nx, self.ny, self.nz, self.tau, self.axis = nx, ny, nz, tau, axis
        codes = (ctypes.c_int * 2)(*[BC[b] for b in bc])
        h = lib().oracle3d_create_axis(stencil, nx, ny, nz, tau, codes, axis)
        if not h:
            raise ValueError(lib().oracle3d_last_error().decode())
        self.h = h
        self.q = lattice(stencil)[1].size

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle3d_destroy(self.h)
            self.h = None

    def set_relax(self, side, sigma=0.0, alpha=0.0, rho_inf=1.0, T_inf=1.0, mach=0.0, length=0.0):
        lib().oracle3d_set_relax(self.h, side, sigma, alpha, rho_inf, T_inf, mach, length)

    def set_recon(self, side, mode):
        if lib().oracle3d_set_recon(self.h, side, {"equilibrium": 0, "neep": 1}[mode]) != 0:
            raise ValueError("NEEP needs a characteristic face")

    def init(self, rho, ux, uy, uz, T):
        shape = (self.nz, self.ny, self.nx)
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape)) for a in (rho, ux, uy, uz, T)]
        lib().oracle3d_init(self.h, *[_ptr(a) for a in arrs])

    def step(self, n=1):
        lib().oracle3d_step(self.h, n)

    def macro(self):
        out = np.zeros((5, self.nz, self.ny, self.nx))
        lib().oracle3d_macro(self.h, _ptr(out))
        return out

    def pops(self):
        out = np.zeros((self.q, self.nz, self.ny, self.nx))
        lib().oracle3d_pops(self.h, _ptr(out))
        return out

    def diag(self):
        out = np.zeros(8)
        lib().oracle3d_diag(self.h, _ptr(out))
        return out

    def transverse_probe(self, side, j, y, z):
        """Transverse terms (local components) at layer j of row (t1, t2) = (y, z) of a face (for
        faces normal to y: (z, x); to z: (x, y)), current state."""
        out = np.zeros(5)
        if lib().oracle3d_transverse_probe(self.h, side, j, y, z, _ptr(out)) != 0:
            raise ValueError("bad probe")
        return out

    def visc_probe(self, g, x, y, z):
        """V (local frame of the outward normal g e_axis) at bulk node (x, y, z) = (normal, t1, t2)
        coordinates, as a face evaluates it there."""
        out = np.zeros(5)
        if lib().oracle3d_visc_probe(self.h, g, x, y, z, _ptr(out)) != 0:
            raise ValueError("bad probe")
        return out
