"""Thin ctypes binding of liblbm_hip.so (C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the library.
PyTorch provides the device memory (workspace, fields) and the stream.  The library must have
been built (``python -m paper_2307_16766_amd.build`` or ``__graft_entry__.build()``); loading
fails loudly otherwise.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm_hip.so")

LBM_OK, LBM_E_ARG, LBM_E_HIP, LBM_E_NONFINITE, LBM_E_STATE, LBM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
D2Q9, D2Q17, D2Q37 = 9, 17, 37
FP64, FP32DEV = 0, 1
BC = {"periodic": 0, "lodi": 1, "lodi_relax": 2, "cbc": 3, "cbc_relax": 4, "zg": 5, "dirichlet": 6}
PRECISION = {"fp64": FP64, "fp32dev": FP32DEV}
RECON = {"equilibrium": 0, "neep": 1}
VISC = {"meso": 0, "fd": 1}

# exported symbols, as declared in include/lbm.h
SYMBOLS = ["lbm_workspace_bytes", "lbm_init", "lbm_cbc_params", "lbm_reconstruction", "lbm_viscous", "lbm_dirichlet_profile", "lbm_step",
           "lbm_macroscopic", "lbm_boundary_state", "lbm_diagnostics", "lbm_diagnostics_noalloc", "lbm_diag_every", "lbm_state_bytes", "lbm_save",
           "lbm_restore", "lbm_steps_done", "lbm_set_kernel_timing", "lbm_bulk_kernel_time",
           "lbm_tape_bytes", "lbm_record", "lbm_adjoint", "lbm_lattice_info", "lbm_last_error", "lbm_destroy"]


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("stencil", ctypes.c_int), ("precision", ctypes.c_int), ("nx", ctypes.c_int),
                ("ny", ctypes.c_int), ("tau", ctypes.c_double), ("bc", ctypes.c_int * 4)]


class Relax(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("alpha", ctypes.c_double), ("rho_inf", ctypes.c_double),
                ("T_inf", ctypes.c_double), ("mach", ctypes.c_double), ("length", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p


def load():
    """Load the library (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime that the library links against)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.lbm_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_workspace_bytes.argtypes = [ctypes.POINTER(Config)]
    L.lbm_init.argtypes = [ctypes.POINTER(Config), _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp,
                           ctypes.POINTER(_vp)]
    L.lbm_cbc_params.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(Relax)]
    L.lbm_reconstruction.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    L.lbm_viscous.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    L.lbm_dirichlet_profile.argtypes = [_vp, ctypes.c_int, _vp]
    L.lbm_step.argtypes = [_vp, ctypes.c_int]
    L.lbm_macroscopic.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.lbm_boundary_state.argtypes = [_vp, ctypes.c_int, _vp]
    L.lbm_diagnostics.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
    L.lbm_diag_every.argtypes = [_vp, ctypes.c_int]
    L.lbm_diagnostics_noalloc.argtypes = [_vp, _vp]
    L.lbm_state_bytes.restype = ctypes.c_size_t
    L.lbm_state_bytes.argtypes = [_vp]
    L.lbm_save.argtypes = [_vp, _vp]
    L.lbm_restore.argtypes = [_vp, _vp]
    L.lbm_steps_done.restype = ctypes.c_long
    L.lbm_steps_done.argtypes = [_vp]
    L.lbm_set_kernel_timing.argtypes = [_vp, ctypes.c_int]
    L.lbm_bulk_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
    L.lbm_tape_bytes.restype = ctypes.c_size_t
    L.lbm_tape_bytes.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    L.lbm_record.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t]
    L.lbm_adjoint.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
    L.lbm_lattice_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = [_vp]
    L.lbm_destroy.argtypes = [_vp]
    _lib = L
    return L


def lattice_info(stencil):
    """(cs2, w[q], cx[q], cy[q], M) used by the library."""
    L = load()
    M = ctypes.c_int()
    cs2 = ctypes.c_double()
    w = (ctypes.c_double * 64)()
    cx = (ctypes.c_int * 64)()
    cy = (ctypes.c_int * 64)()
    q = L.lbm_lattice_info(stencil, ctypes.byref(M), ctypes.byref(cs2), w, cx, cy)
    if q < 0:
        raise LBMError(q, L.lbm_last_error(None).decode())
    return cs2.value, np.array(w[:q]), np.array(cx[:q]), np.array(cy[:q]), M.value


def make_config(stencil, nx, ny, tau, bc, precision="fp64"):
    codes = [BC[b] if isinstance(b, str) else int(b) for b in bc]
    prec = PRECISION[precision] if isinstance(precision, str) else int(precision)
    return Config(stencil, prec, nx, ny, tau, (ctypes.c_int * 4)(*codes))


def workspace_bytes(cfg):
    return load().lbm_workspace_bytes(ctypes.byref(cfg))


class LBM:
    """One simulation on the current HIP device (torch.cuda.current_device())."""

    def __init__(self, stencil, nx, ny, tau, bc, fields, precision="fp64", stream=None):
        import torch
        L = load()
        self.torch = torch
        self.cfg = make_config(stencil, nx, ny, tau, bc, precision)
        self.nx, self.ny, self.stencil = nx, ny, stencil
        nbytes = L.lbm_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise LBMError(LBM_E_ARG, L.lbm_last_error(None).decode())
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        dev = [self._as_device(a) for a in fields]
        ctx = _vp()
        rc = L.lbm_init(ctypes.byref(self.cfg), _vp(self.workspace.data_ptr()), nbytes, _vp(self.stream.cuda_stream),
                        *[_vp(a.data_ptr()) if a is not None else None for a in dev], ctypes.byref(ctx))
        if rc != LBM_OK:
            raise LBMError(rc, L.lbm_last_error(None).decode())
        self._fields = dev   # kept alive until the init kernels have run
        self.ctx = ctx

    def _as_device(self, a):
        torch = self.torch
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            t = a.to(device=self.device, dtype=torch.float64)
        else:
            arr = np.array(np.broadcast_to(np.asarray(a, dtype=np.float64), (self.ny, self.nx)))
            t = torch.from_numpy(arr).to(self.device)
        return t.contiguous()

    def _check(self, rc):
        if rc != LBM_OK:
            raise LBMError(rc, load().lbm_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.torch.cuda.synchronize(self.device)
            load().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_relax(self, side, sigma=0.0, alpha=0.0, rho_inf=1.0, T_inf=1.0, mach=0.0, length=0.0):
        p = Relax(sigma, alpha, rho_inf, T_inf, mach, length)
        self._check(load().lbm_cbc_params(self.ctx, side, ctypes.byref(p)))

    def set_reconstruction(self, side, mode):
        """Mesoscopic BC of characteristic side(s): "equilibrium" or "neep" (side -1: all)."""
        self._check(load().lbm_reconstruction(self.ctx, side, RECON[mode]))

    def set_viscous(self, side, mode):
        """Viscous terms of CBC side(s): "meso" (eq. LaplaceU / LaplaceT) or "fd" (side -1: all)."""
        self._check(load().lbm_viscous(self.ctx, side, VISC[mode]))

    def set_inlet(self, side, U):
        t = self.torch.as_tensor(np.asarray(U, dtype=np.float64)).to(self.device).contiguous()
        self._keep_inlet = t
        self._check(load().lbm_dirichlet_profile(self.ctx, side, _vp(t.data_ptr())))

    def step(self, n=1):
        self._check(load().lbm_step(self.ctx, n))

    def macroscopic(self):
        torch = self.torch
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(4)]
        self._check(load().lbm_macroscopic(self.ctx, *[_vp(t.data_ptr()) for t in out]))
        return out

    def macro_numpy(self):
        out = self.macroscopic()
        self.torch.cuda.synchronize(self.device)
        return [t.cpu().numpy() for t in out]

    def boundary_state(self, side, M, length):
        t = self.torch.empty((M, length, 4), dtype=self.torch.float64, device=self.device)
        self._check(load().lbm_boundary_state(self.ctx, side, _vp(t.data_ptr())))
        return t

    def diagnostics(self, allow_nonfinite=False):
        out = (ctypes.c_double * 8)()
        rc = load().lbm_diagnostics(self.ctx, out)
        if rc == LBM_E_NONFINITE and allow_nonfinite:
            return np.array(out[:])
        self._check(rc)
        return np.array(out[:])

    def diagnostics_noalloc(self, out):
        """Enqueue the diagnostics into the float64 device tensor out[8] without allocating or
        synchronising (lbm_diagnostics_noalloc)."""
        if out.dtype != self.torch.float64 or out.numel() < 8 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of 8 elements")
        self._check(load().lbm_diagnostics_noalloc(self.ctx, _vp(out.data_ptr())))

    def set_diag_every(self, n):
        """Check for non-finite populations every n steps inside step() (0: off); step() then
        raises LBMError with code LBM_E_NONFINITE at the first check that finds one."""
        self._check(load().lbm_diag_every(self.ctx, int(n)))

    def state_bytes(self):
        return load().lbm_state_bytes(self.ctx)

    def save(self):
        buf = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device=self.device)
        self._check(load().lbm_save(self.ctx, _vp(buf.data_ptr())))
        return buf

    def restore(self, buf):
        self._check(load().lbm_restore(self.ctx, _vp(buf.data_ptr())))

    def steps_done(self):
        return load().lbm_steps_done(self.ctx)

    def set_kernel_timing(self, enable=True, every=1):
        """Time every `every`-th step kernel launch with HIP events (enable False: off)."""
        self._check(load().lbm_set_kernel_timing(self.ctx, int(every) if enable else 0))

    def bulk_kernel_time(self):
        """(summed milliseconds, launches) of the timed bulk kernel launches."""
        ms = ctypes.c_double()
        n = ctypes.c_long()
        self._check(load().lbm_bulk_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ---------------------------------------------------------------- discrete adjoint
    def tape_bytes(self, nsteps, every):
        return load().lbm_tape_bytes(self.ctx, nsteps, every)

    def record(self, nsteps, every=50):
        """Advance nsteps steps from the initial state, keeping a checkpoint every `every` steps
        in a device tape (owned here) for adjoint()."""
        nbytes = self.tape_bytes(nsteps, every)
        if nbytes == 0:
            raise LBMError(LBM_E_ARG, "invalid nsteps / every")
        self.tape = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        self._check(load().lbm_record(self.ctx, nsteps, every, _vp(self.tape.data_ptr()), nbytes))

    def adjoint(self, seed=None):
        """Gradient of a loss of the final fields (seed = dL/d(rho, ux, uy, T), shape (4, ny, nx);
        None: the pressure loss of diagnostics()[4]).  Returns (dL/d(rho0, ux0, uy0, T0) as a
        (4, ny, nx) float64 device tensor, dL/d(sigma, alpha) per side as a (4, 2) array)."""
        torch = self.torch
        grad = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=self.device)
        sd = None
        if seed is not None:
            sd = torch.as_tensor(seed).to(device=self.device, dtype=torch.float64).contiguous()
            if tuple(sd.shape) != (4, self.ny, self.nx):
                raise LBMError(LBM_E_ARG, "seed must have shape (4, ny, nx)")
        rel = (ctypes.c_double * 8)()
        self._check(load().lbm_adjoint(self.ctx, _vp(sd.data_ptr()) if sd is not None else None,
                                       _vp(grad.data_ptr()), rel))
        return grad, np.array(rel[:]).reshape(4, 2)
