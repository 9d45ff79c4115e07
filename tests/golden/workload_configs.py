"""Definitions of the five workload configurations and of the nodes sampled from their long runs.

Shared by the oracle-only script that writes the stored expected values
(`make_workload_goldens.py`) and by the GPU tests that compare against them.  Holds sizes,
boundary kinds, relaxation settings, step counts and sample positions only: none of the
method's arithmetic.  Initial fields come from `paper_2307_16766_amd.workloads`.
"""
import math

import numpy as np

from paper_2307_16766_amd import workloads as W


def _span(a, b):
    return list(range(a, b))


def _tau(cs2):
    return 0.5 + W.NU_D2Q37 / cs2


# Each function takes the D2Q37 sound speed squared (from the oracle's lattice solve) and returns
# the configuration; tau gives nu = 0.1 as in Sec. 4.
def c2(cs2):
    """D2Q37 temperature (pressure) pulse, 512 x 512, LODI-RELAX on all four sides and corners."""
    n = 512
    return dict(
        name="c2", stencil=37, nx=n, ny=n, tau=_tau(cs2), bc=["lodi_relax"] * 4,
        relax=dict(sigma=0.25, alpha=0.0, mach=0.0), inlet=None,
        fields=lambda: W.temperature_pulse(n, n, amp=1e-3, width=12.0),
        # the pulse reaches the sides at ~200 steps and the corners at ~300
        snapshots=[300, 5000],
        cols=_span(0, 6) + [128, 255, 256] + _span(n - 6, n),
        rows=_span(0, 6) + [255, 256] + _span(n - 6, n),
        workload="D2Q37 512x512 pressure + temperature pulse (amplitude 1e-3, width 12), LODI-RELAX "
                 "on four sides and corners (sigma 0.25), 5000 steps",
    )


def c3(cs2, alpha=0.2):
    """D2Q37 convected isentropic vortex, 1024 x 512, CBC-RELAX outflow, periodic y."""
    nx, ny = 1024, 512
    mach = 0.2
    return dict(
        name="c3" if alpha == mach else f"c3_alpha{alpha:g}", stencil=37, nx=nx, ny=ny, tau=_tau(cs2),
        bc=["lodi_relax", "cbc_relax", "periodic", "periodic"],
        relax=dict(sigma=0.25, alpha=alpha, mach=mach), inlet=None,
        fields=lambda: W.isentropic_vortex(nx, ny, math.sqrt(cs2), mach=mach, radius=20.0, strength=0.05,
                                           center=(256.0, None)),
        # the vortex core reaches the outflow at ~4600 steps
        snapshots=[4600, 6000],
        cols=_span(0, 6) + [256, 512, 768] + _span(nx - 6, nx),
        rows=[0, 127, 255, 256, 383, 511],
        workload=f"D2Q37 1024x512 isentropic vortex (Ma 0.2, R 20, U_v 0.05), LODI-RELAX inflow, "
                 f"CBC-RELAX outflow (sigma 0.25, alpha {alpha:g}), periodic y, 6000 steps",
    )


def c5(cs2):
    """D2Q37 shear layer, 4096 x 2048, Dirichlet inlet, LODI-RELAX outflow, periodic y."""
    nx, ny = 4096, 2048
    fields, prof = W.shear_layer(nx, ny, u0=0.1, thickness=10.0, noise=1e-3, seed=16766)
    return dict(
        name="c5", stencil=37, nx=nx, ny=ny, tau=_tau(cs2), bc=["dirichlet", "lodi_relax", "periodic", "periodic"],
        relax=dict(sigma=0.25, alpha=0.0, mach=0.1 / math.sqrt(2 * cs2)), inlet=(0, prof),
        fields=lambda: fields,
        snapshots=[500, 1000],
        cols=_span(0, 6) + [2048] + _span(nx - 7, nx),
        rows=[0, 1024, 1034, ny - 1],
        workload="D2Q37 4096x2048 shear layer (u0 0.1, thickness 10, noise 1e-3, seed 16766), Dirichlet "
                 "inlet, LODI-RELAX outflow (sigma 0.25), periodic y, 1000 steps",
    )


CONFIGS = {"c2": c2, "c3": c3, "c5": c5}


def sample(fields4, cfg):
    """Rows and columns of (rho, ux, uy, T): arrays [4][len(rows)][nx] and [4][ny][len(cols)]."""
    F = np.stack([np.asarray(a, dtype=np.float64) for a in fields4])
    return F[:, cfg["rows"], :].copy(), F[:, :, cfg["cols"]].copy()
