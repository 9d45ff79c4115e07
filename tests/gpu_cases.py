"""Shared helpers of the GPU parity tests: run the HIP library and the oracle on the same seeded
inputs and compare macroscopic fields node by node."""
import json
import math
import os
import sys

import numpy as np

from oracle import oracle as O
from paper_2307_16766_amd import workloads as W

CS2_37 = O.lattice(37)[0]
CS_37 = math.sqrt(CS2_37)
TAU_37 = 0.5 + W.NU_D2Q37 / CS2_37
CS2_17 = O.lattice(17)[0]
CS_17 = math.sqrt(CS2_17)
TAU_17 = 0.9   # the D2Q17 runs of Sec. 4.1

# Tolerances: relative L2 error bound on rho, u and T.  In FP64, where the fluid is at rest apart
# from a pulse (rms |u| of the reference below U_FLOOR_BELOW, i.e. u ~ 1e-6..1e-4), u alone also
# gets an absolute rounding floor of one ulp of 1 per step: u is then a moment of O(w_i)
# populations that the oracle stores as f itself, rounded to ~2.2e-16 per step, so a relative
# bound of 1e-12 on u ~ 1e-5 would measure the oracle's own rounding (measured: 5e-11 .. 8e-10
# relative on the at-rest cases).  Flows with a background velocity, and FP32 deviation storage
# everywhere, take the plain relative bound.  Every comparison's achieved errors are appended as
# a JSON line to the file named by the environment variable PARITY_LOG, when set.
TOL = {"fp64": (1e-12, 2.2e-16), "fp32dev": (2e-5, 0.0)}
U_FLOOR_BELOW = 1e-3


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_errors(gpu, ref):
    """Relative L2 errors of (rho, u, T) over all nodes (u as a vector field)."""
    r, ux, uy, T = gpu
    R, UX, UY, TT = ref
    e_rho = np.linalg.norm(r - R) / np.linalg.norm(R)
    nu = math.sqrt(np.sum(UX ** 2 + UY ** 2))
    e_u = math.sqrt(np.sum((ux - UX) ** 2 + (uy - UY) ** 2)) / max(nu, 1e-300)
    e_T = np.linalg.norm(T - TT) / np.linalg.norm(TT)
    return e_rho, e_u, e_T


CHAR_BCS = ("lodi", "lodi_relax", "cbc", "cbc_relax")


def make_pair(stencil, nx, ny, tau, bc, fields, precision, relax=None, inlet=None, recon=None, visc=None):
    from paper_2307_16766_amd import lbm
    g = lbm.LBM(stencil, nx, ny, tau, bc, fields, precision=precision)
    o = O.Oracle(stencil, nx, ny, tau, bc)
    o.init(*fields)
    if relax is not None:
        g.set_relax(-1, **relax)
        o.set_relax(-1, **relax)
    if recon is not None:
        g.set_reconstruction(-1, recon)
        for s, b in enumerate(bc):
            if b in CHAR_BCS:
                o.set_recon(s, recon)
    if visc is not None:
        g.set_viscous(-1, visc)
        for s, b in enumerate(bc):
            if b in ("cbc", "cbc_relax"):
                o.set_viscous(s, visc)
    if inlet is not None:
        side, U = inlet
        g.set_inlet(side, U)
        o.set_inlet(side, U)
    return g, o


def record(entry):
    path = os.environ.get("PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(entry) + "\n")


def check_fields(name, precision, n, gpu, ref, tol=None):
    """Assert parity of (rho, u, T) after n steps; returns the relative errors."""
    rel, floor = TOL[precision] if tol is None else tol
    errs = rel_errors(gpu, ref)
    du = math.sqrt(np.mean((gpu[1] - ref[1]) ** 2 + (gpu[2] - ref[2]) ** 2))
    uref = math.sqrt(np.mean(ref[1] ** 2 + ref[2] ** 2))
    at_rest = uref < U_FLOOR_BELOW and floor > 0
    record({"case": name, "precision": precision, "step": n, "rel_rho": errs[0], "rel_u": errs[1], "rel_T": errs[2],
            "rms_u": uref, "u_floor": at_rest})
    assert all(np.isfinite(errs)), (name, n, errs)
    assert errs[0] <= rel and errs[2] <= rel, f"{name} {precision} step {n}: rel errors rho/u/T = {errs}"
    if at_rest:
        assert du <= rel * uref + floor * (n + 1), f"{name} {precision} step {n}: rms du {du:.3e}, rms u {uref:.3e}"
    else:
        assert errs[1] <= rel, f"{name} {precision} step {n}: relative u error {errs[1]:.3e} (rms u {uref:.3e})"
    return errs


def gpu_pops(g):
    """Full populations (q, ny, nx) of the GPU state in the oracle's velocity order, decoded from
    a checkpoint (populations are stored as f - w_i in row-interleaved planes [y][i][x])."""
    from paper_2307_16766_amd import lbm
    _, w, cx, cy, _ = lbm.lattice_info(g.stencil)
    q = len(w)
    dt = np.float64 if g.cfg.precision == lbm.FP64 else np.float32
    pitch = (g.nx + 63) // 64 * 64
    raw = g.save().cpu().numpy()
    d = raw[256:256 + q * pitch * g.ny * np.dtype(dt).itemsize].view(dt).reshape(g.ny, q, pitch)[:, :, :g.nx]
    f = d.transpose(1, 0, 2).astype(np.float64) + w[:, None, None]
    _, _, ocx, ocy, _ = O.lattice(g.stencil)
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(cx, cy))}
    return np.stack([f[index[(int(a), int(b))]] for a, b in zip(ocx, ocy)])


def compare_run(name, stencil, nx, ny, tau, bc, fields, precision, steps, relax=None, inlet=None, tol=None,
                recon=None, pops_tol=None, visc=None):
    """Step both implementations, comparing after every listed step count (and the populations
    of every node at the end, absolute tolerance pops_tol, when given).  Returns worst errors."""
    log(f"[gpu-case] {name} {precision} {nx}x{ny} D2Q{stencil} bc={bc} recon={recon} visc={visc} steps={steps}")
    g, o = make_pair(stencil, nx, ny, tau, bc, fields, precision, relax, inlet, recon, visc)
    worst = [0.0, 0.0, 0.0]
    done = 0
    for n in steps:
        g.step(n - done)
        o.step(n - done)
        done = n
        errs = check_fields(name, precision, n, g.macro_numpy(), o.macro(), tol)
        worst = [max(a, b) for a, b in zip(worst, errs)]
    if pops_tol is not None:
        dmax = float(np.abs(gpu_pops(g) - o.pops()).max())
        log(f"[gpu-case] {name} {precision} max |f_gpu - f_oracle| = {dmax:.3e}")
        assert dmax <= pops_tol, (name, dmax)
    g.close()
    log(f"[gpu-case] {name} {precision} ok worst rel errors rho/u/T = {worst}")
    return worst


def smooth_random(nx, ny, seed, amp):
    rng = np.random.default_rng(seed)
    X, Y = W.grid(nx, ny)
    out = np.zeros((ny, nx))
    for _ in range(4):
        kx, ky = rng.integers(1, 3, 2)
        out += amp * rng.uniform(-1, 1) * np.sin(2 * np.pi * (kx * X / nx + ky * Y / ny) + rng.uniform(0, 6))
    return out
