"""Thin ctypes binding of the three-dimensional C ABI (include/lbm3d.h) of liblbm_hip.so.

Argument marshalling only: every step runs in the HIP kernels of the library; PyTorch provides the
device memory (workspace, fields) and the stream.  Fields are [nz][ny][nx] arrays with x fastest.
"""
import ctypes

import numpy as np

from . import lbm as _lbm

D3Q39 = 39
BC3 = {"periodic": 0, "lodi": 1, "lodi_relax": 2, "cbc": 3, "cbc_relax": 4, "zg": 5}

SYMBOLS = ["lbm3d_workspace_bytes", "lbm3d_init", "lbm3d_cbc_params", "lbm3d_reconstruction", "lbm3d_step",
           "lbm3d_macroscopic", "lbm3d_populations", "lbm3d_diagnostics", "lbm3d_set_kernel_timing",
           "lbm3d_bulk_kernel_time", "lbm3d_lattice_info", "lbm3d_last_error", "lbm3d_destroy"]

_vp = ctypes.c_void_p
_ready = False


class Config3(ctypes.Structure):
    _fields_ = [("stencil", ctypes.c_int), ("precision", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("tau", ctypes.c_double), ("bc", ctypes.c_int * 2), ("axis", ctypes.c_int)]


def load():
    global _ready
    L = _lbm.load()
    if not _ready:
        L.lbm3d_workspace_bytes.restype = ctypes.c_size_t
        L.lbm3d_workspace_bytes.argtypes = [ctypes.POINTER(Config3)]
        L.lbm3d_init.argtypes = [ctypes.POINTER(Config3), _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp, _vp,
                                 ctypes.POINTER(_vp)]
        L.lbm3d_cbc_params.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_lbm.Relax)]
        L.lbm3d_reconstruction.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
        L.lbm3d_step.argtypes = [_vp, ctypes.c_int]
        L.lbm3d_macroscopic.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.lbm3d_populations.argtypes = [_vp, _vp]
        L.lbm3d_diagnostics.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.lbm3d_set_kernel_timing.argtypes = [_vp, ctypes.c_int]
        L.lbm3d_bulk_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
        L.lbm3d_lattice_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.lbm3d_last_error.restype = ctypes.c_char_p
        L.lbm3d_last_error.argtypes = [_vp]
        L.lbm3d_destroy.argtypes = [_vp]
        _ready = True
    return L


def lattice_info(stencil=D3Q39):
    """(cs2, w[q], cx[q], cy[q], cz[q], M) used by the library."""
    L = load()
    M, cs2 = ctypes.c_int(), ctypes.c_double()
    w = (ctypes.c_double * 128)()
    c = [(ctypes.c_int * 128)() for _ in range(3)]
    q = L.lbm3d_lattice_info(stencil, ctypes.byref(M), ctypes.byref(cs2), w, *c)
    if q < 0:
        raise _lbm.LBMError(q, L.lbm3d_last_error(None).decode())
    return cs2.value, np.array(w[:q]), np.array(c[0][:q]), np.array(c[1][:q]), np.array(c[2][:q]), M.value


def make_config(nx, ny, nz, tau, bc, precision="fp64", stencil=D3Q39, axis=0):
    codes = [BC3[b] if isinstance(b, str) else int(b) for b in bc]
    prec = _lbm.PRECISION[precision] if isinstance(precision, str) else int(precision)
    return Config3(stencil, prec, nx, ny, nz, tau, (ctypes.c_int * 2)(*codes), axis)


class LBM3D:
    """One 3D simulation on the current HIP device: bc = [low face, high face] of the face axis
    `axis` (0 = x, 1 = y, 2 = z); the other two axes are periodic."""

    def __init__(self, nx, ny, nz, tau, bc, fields, precision="fp64", stream=None, axis=0):
        import torch
        L = load()
        self.torch = torch
        self.cfg = make_config(nx, ny, nz, tau, bc, precision, axis=axis)
        self.nx, self.ny, self.nz = nx, ny, nz
        nbytes = L.lbm3d_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise _lbm.LBMError(_lbm.LBM_E_ARG, L.lbm3d_last_error(None).decode())
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        dev = [self._as_device(a) for a in fields]
        ctx = _vp()
        rc = L.lbm3d_init(ctypes.byref(self.cfg), _vp(self.workspace.data_ptr()), nbytes, _vp(self.stream.cuda_stream),
                          *[_vp(a.data_ptr()) for a in dev], ctypes.byref(ctx))
        if rc != _lbm.LBM_OK:
            raise _lbm.LBMError(rc, L.lbm3d_last_error(None).decode())
        self._fields = dev
        self.ctx = ctx

    def _as_device(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=torch.float64).contiguous()
        arr = np.array(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.nz, self.ny, self.nx)))
        return torch.from_numpy(arr).to(self.device).contiguous()

    def _check(self, rc):
        if rc != _lbm.LBM_OK:
            raise _lbm.LBMError(rc, load().lbm3d_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.torch.cuda.synchronize(self.device)
            load().lbm3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_relax(self, face, sigma=0.0, alpha=0.0, rho_inf=1.0, T_inf=1.0, mach=0.0, length=0.0):
        p = _lbm.Relax(sigma, alpha, rho_inf, T_inf, mach, length)
        self._check(load().lbm3d_cbc_params(self.ctx, face, ctypes.byref(p)))

    def set_reconstruction(self, face, mode):
        self._check(load().lbm3d_reconstruction(self.ctx, face, _lbm.RECON[mode]))

    def step(self, n=1):
        self._check(load().lbm3d_step(self.ctx, n))

    def macroscopic(self):
        torch = self.torch
        out = [torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(5)]
        self._check(load().lbm3d_macroscopic(self.ctx, *[_vp(t.data_ptr()) for t in out]))
        return out

    def macro_numpy(self):
        out = self.macroscopic()
        self.torch.cuda.synchronize(self.device)
        return np.stack([t.cpu().numpy() for t in out])

    def populations(self):
        """Full populations f_i (library velocity order), numpy [q][nz][ny][nx]."""
        q = lattice_info()[1].size
        t = self.torch.empty((q, self.nz, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
        self._check(load().lbm3d_populations(self.ctx, _vp(t.data_ptr())))
        self.torch.cuda.synchronize(self.device)
        return t.cpu().numpy()

    def diagnostics(self, allow_nonfinite=False):
        out = (ctypes.c_double * 8)()
        rc = load().lbm3d_diagnostics(self.ctx, out)
        if rc != _lbm.LBM_OK and not (allow_nonfinite and rc == _lbm.LBM_E_NONFINITE):
            self._check(rc)
        return np.array(out[:8])

    def set_kernel_timing(self, enable, every=1):
        """Time every `every`-th bulk kernel launch with HIP events (enable False: off)."""
        self._check(load().lbm3d_set_kernel_timing(self.ctx, int(every) if enable else 0))

    def bulk_kernel_time(self):
        ms, n = ctypes.c_double(), ctypes.c_long()
        self._check(load().lbm3d_bulk_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
