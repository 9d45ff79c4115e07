"""GPU parity of the three-dimensional path (Appendix A; D3Q39, characteristic faces normal to x, y
or z, the other two axes periodic) against the FP64 3D oracle, node by node on seeded inputs."""
import math

import numpy as np
import pytest

from gpu_cases import TOL, log
from oracle import oracle3d as O3

pytestmark = pytest.mark.gpu

TAU = 0.9
CS2 = O3.lattice()[0]
RELAX = dict(sigma=0.25, alpha=0.1, mach=0.05)
EARLY = [1, 2, 3, 5, 10, 30]


def _grid(nx, ny, nz):
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return X.astype(float), Y.astype(float), Z.astype(float)


def drifting_pulse(nx, ny, nz, center, amp=1e-3, width=3.0, u=(0.01, -0.004, 0.006)):
    X, Y, Z = _grid(nx, ny, nz)
    g = amp * np.exp(-((X - center[0]) ** 2 + (Y - center[1]) ** 2 + (Z - center[2]) ** 2) / (2 * width ** 2))
    one = np.ones_like(X)
    return [one, u[0] * one, u[1] * one, u[2] * one, 1 + g]


def smooth_random(nx, ny, nz, seed, amp):
    rng = np.random.default_rng(seed)
    X, Y, Z = _grid(nx, ny, nz)
    out = np.zeros_like(X)
    for _ in range(4):
        k = rng.integers(1, 3, 3)
        out += amp * rng.uniform(-1, 1) * np.sin(2 * np.pi * (k[0] * X / nx + k[1] * Y / ny + k[2] * Z / nz) + rng.uniform(0, 6))
    return out


def rel_errors(g, o):
    e_rho = np.linalg.norm(g[0] - o[0]) / np.linalg.norm(o[0])
    du = math.sqrt(sum(np.sum((g[k] - o[k]) ** 2) for k in (1, 2, 3)))
    nu = math.sqrt(sum(np.sum(o[k] ** 2) for k in (1, 2, 3)))
    e_T = np.linalg.norm(g[4] - o[4]) / np.linalg.norm(o[4])
    return e_rho, du / max(nu, 1e-300), e_T, du


def compare3(name, nx, ny, nz, bc, fields, precision, steps, relax=None, recon=None, pops_tol=None, axis=0):
    from paper_2307_16766_amd import lbm3d
    log(f"[gpu-case] 3d {name} {precision} {nx}x{ny}x{nz} axis={axis} bc={bc} recon={recon} steps={steps}")
    g = lbm3d.LBM3D(nx, ny, nz, TAU, bc, fields, precision=precision, axis=axis)
    o = O3.Oracle3D(nx, ny, nz, TAU, bc, axis=axis)
    o.init(*fields)
    if relax:
        g.set_relax(-1, **relax)
        o.set_relax(-1, **relax)
    if recon:
        g.set_reconstruction(-1, recon)
        for s, b in enumerate(bc):
            if b not in ("periodic", "zg"):
                o.set_recon(s, recon)
    rel, floor = TOL[precision]
    done, worst = 0, [0.0, 0.0, 0.0]
    for n in steps:
        g.step(n - done)
        o.step(n - done)
        done = n
        gm, om = g.macro_numpy(), o.macro()
        e_rho, e_u, e_T, du = rel_errors(gm, om)
        assert all(np.isfinite([e_rho, e_u, e_T])), (name, n)
        assert e_rho <= rel and e_T <= rel, f"{name} {precision} step {n}: rho {e_rho:.3e} T {e_T:.3e}"
        uref = math.sqrt(sum(np.sum(om[k] ** 2) for k in (1, 2, 3)))
        assert du <= rel * uref + floor * (n + 1) * math.sqrt(nx * ny * nz), f"{name} {precision} step {n}: du {du:.3e}"
        worst = [max(a, b) for a, b in zip(worst, (e_rho, e_u, e_T))]
    if pops_tol is not None:
        _, w, cx, cy, cz, _ = lbm3d.lattice_info()
        fg = g.populations()
        _, _, ocx, ocy, ocz, _ = O3.lattice()
        index = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(cx, cy, cz))}
        fg = np.stack([fg[index[(int(a), int(b), int(c))]] for a, b, c in zip(ocx, ocy, ocz)])
        dmax = float(np.abs(fg - o.pops()).max())
        log(f"[gpu-case] 3d {name} max |f_gpu - f_oracle| = {dmax:.3e}")
        assert dmax <= pops_tol, (name, dmax)
    d_g, d_o = g.diagnostics(), o.diag()
    f = 1 if precision == "fp64" else 1e5
    assert abs(d_g[0] - d_o[0]) < 1e-12 * d_o[0] * f
    for k in (1, 2, 3):   # momenta, in the caller's axes
        assert abs(d_g[k] - d_o[k]) < 1e-12 * d_o[0] * f, (k, d_g[k], d_o[k])
    g.close()
    log(f"[gpu-case] 3d {name} {precision} ok worst rel errors rho/u/T = {worst}")
    return worst


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_3d_periodic_box(precision):
    nx, ny, nz = 20, 12, 10
    f = [1 + smooth_random(nx, ny, nz, 1, 0.01), smooth_random(nx, ny, nz, 2, 0.03), smooth_random(nx, ny, nz, 3, 0.03),
         smooth_random(nx, ny, nz, 4, 0.03), 1 + smooth_random(nx, ny, nz, 5, 0.01)]
    compare3("periodic", nx, ny, nz, ["periodic", "periodic"], f, precision, EARLY)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_3d_relax_faces(precision):
    nx, ny, nz = 28, 10, 8
    compare3("lodi_relax|cbc_relax", nx, ny, nz, ["lodi_relax", "cbc_relax"], drifting_pulse(nx, ny, nz, (14, 4, 3)),
             precision, EARLY, relax=RELAX)


@pytest.mark.parametrize("bc", ["lodi", "cbc", "zg"])
def test_3d_schemes(bc):
    nx, ny, nz = 24, 9, 7
    compare3(bc, nx, ny, nz, [bc, bc], drifting_pulse(nx, ny, nz, (10, 4, 3)), "fp64", EARLY, relax=RELAX)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_3d_neep(precision):
    nx, ny, nz = 26, 8, 9
    compare3("neep", nx, ny, nz, ["cbc_relax", "lodi"], drifting_pulse(nx, ny, nz, (12, 3, 4)), precision, EARLY,
             relax=RELAX, recon="neep", pops_tol=1e-14 if precision == "fp64" else 2e-8)


def test_3d_multi_tile():
    # 300 nodes along x: two bulk tiles per row with a ragged tail; 30 rows
    nx, ny, nz = 300, 6, 5
    compare3("multitile", nx, ny, nz, ["lodi_relax", "cbc_relax"], drifting_pulse(nx, ny, nz, (280, 2, 2), width=4.0),
             "fp64", [1, 5, 20], relax=RELAX)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("nx,bc", [(9, ["lodi", "lodi_relax"]), (12, ["cbc_relax", "lodi_relax"])])
def test_3d_minimum_grid(precision, nx, bc):
    # the smallest accepted boxes: nx = 2M + 3 = 9 with two faces (the strips of both faces share
    # the three bulk columns), 3M + 3 = 12 with a CBC face (its viscous moments come from x_f - M ..
    # x_f - M - 2, here the other face's strip column among them); ny = nz = M + 1 = 4 (every
    # periodic wrap of a 3-step pull)
    from paper_2307_16766_amd import lbm3d
    ny, nz = 4, 4
    compare3("minimum", nx, ny, nz, bc, drifting_pulse(nx, ny, nz, (nx // 2, 1.5, 2.0), width=1.5),
             precision, [1, 2, 5, 20], relax=RELAX)
    if bc[0] == "cbc_relax":
        with pytest.raises(lbm3d._lbm.LBMError):
            lbm3d.LBM3D(nx - 1, ny, nz, TAU, bc, drifting_pulse(nx - 1, ny, nz, (5, 1.5, 2.0)))


def test_3d_zero_steps_and_errors():
    from paper_2307_16766_amd import lbm, lbm3d
    nx, ny, nz = 12, 5, 4
    f = drifting_pulse(nx, ny, nz, (6, 2, 2))
    g = lbm3d.LBM3D(nx, ny, nz, TAU, ["lodi", "zg"], f)
    before = g.macro_numpy()
    g.step(0)
    assert np.array_equal(g.macro_numpy(), before)
    with pytest.raises(lbm.LBMError):
        g.step(-1)
    with pytest.raises(lbm.LBMError):
        g.set_reconstruction(1, "neep")      # NEEP on a zero-gradient face
    with pytest.raises(lbm.LBMError):
        g.set_relax(0, sigma=0.1, rho_inf=-1.0)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("axis", [1, 2])
def test_3d_faces_normal_to_y_and_z(axis, precision):
    # faces normal to y (z): the library runs the rotated problem on its internal grid, the oracle
    # solves the faces along that axis directly; fields, outputs and populations in the caller's
    # [nz][ny][nx] layout and axes
    dims = {1: (9, 28, 8), 2: (8, 9, 28)}[axis]
    c = [d / 2 for d in dims]
    compare3(f"faces-axis{axis}", *dims, ["lodi_relax", "cbc_relax"], drifting_pulse(*dims, c), precision, EARLY,
             relax=RELAX, axis=axis)


@pytest.mark.parametrize("axis", [1, 2])
def test_3d_faces_normal_to_y_and_z_neep_populations(axis):
    # NEEP on the CBC face, and every population compared (the library's output maps its internal
    # velocity order back to the caller's axes)
    dims = {1: (7, 26, 9), 2: (9, 8, 26)}[axis]
    c = [d / 2 for d in dims]
    compare3(f"faces-axis{axis}-neep", *dims, ["cbc_relax", "lodi"], drifting_pulse(*dims, c), "fp64", EARLY,
             relax=RELAX, recon="neep", pops_tol=1e-14, axis=axis)
