"""Seeded synthetic initial fields for the benchmark and test workloads.

This module only builds input arrays (numpy float64, [ny][nx], x fastest); it holds none of the
method's arithmetic.  Lattice constants it needs (the sound speed) are passed in by the caller.
The fields follow the initial-value problems of Sec. 4 of the paper (pulses, vortex) at the sizes
of the workloads named below.
"""
import math

import numpy as np

# tau giving kinematic viscosity nu = (tau - 1/2) cs^2 = 0.1 on D2Q37 (Sec. 4 uses nu = 0.1)
NU_D2Q37 = 0.1


def grid(nx, ny):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    return np.meshgrid(x, y)


def gaussian_density_pulse(nx, ny, amp=1e-3, width=8.0, center=None):
    """rho = 1 + amp exp(-r^2 / (2 width^2)), u = 0, T = 1 (D2Q9 pulse, 256 x 128)."""
    X, Y = grid(nx, ny)
    cx, cy = center if center is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0)
    r2 = (X - cx) ** 2 + (Y - cy) ** 2
    rho = 1.0 + amp * np.exp(-r2 / (2.0 * width ** 2))
    z = np.zeros_like(rho)
    return rho, z.copy(), z.copy(), np.ones_like(rho)


def temperature_pulse(nx, ny, amp=1e-3, width=12.0, center=None):
    """rho = 1, u = 0, T = 1 + amp exp(-r^2 / (2 width^2)): pressure and temperature pulse."""
    X, Y = grid(nx, ny)
    cx, cy = center if center is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0)
    r2 = (X - cx) ** 2 + (Y - cy) ** 2
    T = 1.0 + amp * np.exp(-r2 / (2.0 * width ** 2))
    z = np.zeros_like(T)
    return np.ones_like(T), z.copy(), z.copy(), T


def planar_temperature_pulse(nx, ny, amp=1e-3, width=10.0, x0=None):
    """Pulse that depends on x only (a 1D problem on a y-periodic strip)."""
    X, _ = grid(nx, ny)
    x0 = (nx - 1) / 2.0 if x0 is None else x0
    T = 1.0 + amp * np.exp(-((X - x0) ** 2) / (2.0 * width ** 2))
    z = np.zeros_like(T)
    return np.ones_like(T), z.copy(), z.copy(), T


def isentropic_vortex(nx, ny, cs, mach=0.2, radius=20.0, strength=0.05, center=(256.0, None)):
    """Vortex convected by a uniform flow u0 = (mach cs, 0).

    du = U_v exp((1 - r^2/R^2)/2) (-(y - y0), x - x0) / R,
    T = 1 - U_v^2 / (4 cs^2) exp(1 - r^2/R^2), rho = T (isentropic for cp/cv = 2).
    """
    X, Y = grid(nx, ny)
    x0 = center[0]
    y0 = (ny - 1) / 2.0 if center[1] is None else center[1]
    dx, dy = X - x0, Y - y0
    g = np.exp(1.0 - (dx ** 2 + dy ** 2) / radius ** 2)
    amp = strength * np.sqrt(g) / radius
    ux = mach * cs - amp * dy
    uy = amp * dx
    T = 1.0 - strength ** 2 / (4.0 * cs * cs) * g
    return T.copy(), ux, uy, T


def random_temperature(nx, ny, std=1e-4, seed=2307):
    """rho = 1, u = 0, T = 1 + std N(0, 1) per node (numpy default_rng, PCG64)."""
    rng = np.random.default_rng(seed)
    T = 1.0 + std * rng.standard_normal((ny, nx))
    z = np.zeros_like(T)
    return np.ones_like(T), z.copy(), z.copy(), T


def shear_layer(nx, ny, u0=0.1, thickness=10.0, noise=1e-3, seed=16766):
    """u_x = u0 tanh((y - ny/2) / thickness) + noise U(-1, 1), u_y = noise U(-1, 1), rho = T = 1.

    Returns the fields and the unperturbed inlet profile [ny][4] = (rho, u_x, u_y, T) at x = 0.
    """
    rng = np.random.default_rng(seed)
    X, Y = grid(nx, ny)
    base = u0 * np.tanh((Y - ny / 2.0) / thickness)
    ux = base + noise * rng.uniform(-1.0, 1.0, (ny, nx))
    uy = noise * rng.uniform(-1.0, 1.0, (ny, nx))
    one = np.ones((ny, nx))
    prof = np.zeros((ny, 4))
    prof[:, 0] = 1.0
    prof[:, 1] = base[:, 0]
    prof[:, 3] = 1.0
    return (one.copy(), ux, uy, one.copy()), prof


def temperature_step(nx, ny, cs, mach=0.1, T0=1.0, T1=1.0005, s=0.5, length=None, offset=0.0):
    """Smooth temperature step T0 -> T1 -> T0 across x in a uniform stream u = (mach cs, 0), rho = 1
    (Sec. 4.1): tanh fronts of steepness s at length/4 and 3 length/4, length = nx by default.
    The printed second branch has (tanh - 1); (tanh + 1) is the one that returns to T0, which
    the text and the figure describe.  offset shifts the fronts (a window of a wider grid)."""
    L = float(nx if length is None else length)
    x = np.arange(nx, dtype=np.float64)[None, :] - offset
    left = T1 + 0.5 * (T1 - T0) * (np.tanh(s * (x - L / 4)) - 1.0)
    right = T1 - 0.5 * (T1 - T0) * (np.tanh(s * (x - 3 * L / 4)) + 1.0)
    T = np.broadcast_to(np.where(x <= L / 2, left, right), (ny, nx)).copy()
    one = np.ones((ny, nx))
    return one.copy(), mach * cs * one, 0.0 * one, T


def uniform_flow(nx, ny, ux=0.0, uy=0.0, rho=1.0, T=1.0):
    one = np.ones((ny, nx))
    return rho * one, ux * one, uy * one, T * one


def random_directions(n, nx, ny, seed):
    """n seeded standard-normal perturbation fields [n][ny][nx] (directional-derivative checks)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, ny, nx))


def config(name, cs2, alpha_c3=None):
    """The five workload configurations C1..C5: stencil, grid, tau, boundary kinds (x0, x1, y0,
    y1), relaxation settings, Dirichlet inlet (side, profile) or None, a callable returning the
    initial fields, the step count and a description.  cs2: the stencil's sound speed squared
    (D2Q37 unless C1), which sets tau for nu = 0.1 and the Mach numbers."""
    cs = math.sqrt(cs2)
    tau37 = 0.5 + NU_D2Q37 / cs2
    if name == "c1":
        return dict(stencil=9, nx=256, ny=128, tau=0.6, bc=["lodi_relax", "lodi_relax", "periodic", "periodic"],
                    relax=dict(sigma=0.25, alpha=0.0, mach=0.0), inlet=None, steps=1000,
                    fields=lambda: gaussian_density_pulse(256, 128, amp=1e-3, width=8.0),
                    workload="D2Q9 256x128 density pulse, tau 0.6, LODI-RELAX x-sides, periodic y, FP64, 1000 steps")
    if name == "c2":
        return dict(stencil=37, nx=512, ny=512, tau=tau37, bc=["lodi_relax"] * 4,
                    relax=dict(sigma=0.25, alpha=0.0, mach=0.0), inlet=None, steps=5000,
                    fields=lambda: temperature_pulse(512, 512, amp=1e-3, width=12.0),
                    workload="D2Q37 512x512 pressure + temperature pulse (amplitude 1e-3, width 12), LODI-RELAX "
                             "on four sides and corners (sigma 0.25), 5000 steps")
    if name == "c3":
        a = 0.2 if alpha_c3 is None else alpha_c3
        return dict(stencil=37, nx=1024, ny=512, tau=tau37, bc=["lodi_relax", "cbc_relax", "periodic", "periodic"],
                    relax=dict(sigma=0.25, alpha=a, mach=0.2), inlet=None, steps=6000,
                    fields=lambda: isentropic_vortex(1024, 512, cs, mach=0.2, radius=20.0, strength=0.05,
                                                     center=(256.0, None)),
                    workload=f"D2Q37 1024x512 isentropic vortex (Ma 0.2, R 20, U_v 0.05), LODI-RELAX inflow, "
                             f"CBC-RELAX outflow (sigma 0.25, alpha {a:g}), periodic y, 6000 steps")
    if name == "c4":
        return dict(stencil=37, nx=256, ny=256, tau=tau37, bc=["lodi_relax"] * 4,
                    relax=dict(sigma=0.25, alpha=0.0, mach=0.0), inlet=None, steps=2000,
                    fields=lambda: random_temperature(256, 256, std=1e-4, seed=2307),
                    workload="D2Q37 256x256 random temperature (std 1e-4, seed 2307), LODI-RELAX on four sides "
                             "and corners (sigma 0.25, alpha = Ma = 0), 2000 steps")
    if name == "c5":
        fields, prof = shear_layer(4096, 2048, u0=0.1, thickness=10.0, noise=1e-3, seed=16766)
        return dict(stencil=37, nx=4096, ny=2048, tau=tau37, bc=["dirichlet", "lodi_relax", "periodic", "periodic"],
                    relax=dict(sigma=0.25, alpha=0.0, mach=0.1 / math.sqrt(2 * cs2)), inlet=(0, prof), steps=1000,
                    fields=lambda: fields,
                    workload="D2Q37 4096x2048 shear layer (u0 0.1, thickness 10, noise 1e-3, seed 16766), Dirichlet "
                             "inlet, LODI-RELAX outflow (sigma 0.25), periodic y, 1000 steps")
    raise ValueError(f"unknown workload {name}")
