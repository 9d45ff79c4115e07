"""Parity at the benchmark sizes, in the launch configuration bench.py times.

A state that varies only along x stays independent of y (and z) under periodic y (and z): every
row of the full-size GPU run must then equal the oracle's run of the same x-profile on a grid with
four rows, which the oracle finishes in seconds.  Any tile the bulk launch skipped or visited
twice, or any row mixed into another, breaks the equality."""
import math

import numpy as np
import pytest

from gpu_cases import CS_37, TAU_37, TOL, log
from oracle import oracle as O
from oracle import oracle3d as O3

pytestmark = pytest.mark.gpu
STEPS = 20


def _profile(nx, x0, width, u0):
    x = np.arange(nx, dtype=np.float64)
    T = 1 + 1e-3 * np.exp(-((x - x0) ** 2) / (2 * width ** 2))
    return np.ones(nx), np.full(nx, u0), np.zeros(nx), T


def _check_rows(name, precision, got_rows, ref):
    rel, floor = TOL[precision]
    for row in got_rows:
        for k, z in ((0, "rho"), (-1, "T")):
            err = np.linalg.norm(row[k] - ref[k]) / np.linalg.norm(ref[k])
            assert err <= rel, (name, precision, z, err)
        du = math.sqrt(np.mean((row[1] - ref[1]) ** 2))
        assert du <= rel * math.sqrt(np.mean(ref[1] ** 2)) + floor * (STEPS + 1), (name, precision, du)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_2d_benchmark_size_rows_match_oracle(precision):
    # 4096 x 2048 D2Q37, Dirichlet inlet + LODI-RELAX outflow, periodic y: the bench.py launch
    from paper_2307_16766_amd import lbm
    nx, ny = 4096, 2048
    log(f"[gpu-case] full-size 2d {precision} {nx}x{ny}")
    r, ux, uy, T = _profile(nx, 4070.0, 6.0, 0.1 * CS_37)
    fields = [np.broadcast_to(a, (ny, nx)) for a in (r, ux, uy, T)]
    bc = ["dirichlet", "lodi_relax", "periodic", "periodic"]
    relax = dict(sigma=0.25, mach=0.05)
    g = lbm.LBM(37, nx, ny, TAU_37, bc, fields, precision=precision)
    g.set_relax(-1, **relax)
    g.step(STEPS)
    m = g.macro_numpy()
    g.close()
    o = O.Oracle(37, nx, 4, TAU_37, bc)
    o.set_relax(-1, **relax)
    o.init(*[np.broadcast_to(a, (4, nx)) for a in (r, ux, uy, T)])
    o.step(STEPS)
    ref = [a[0] for a in o.macro()]
    rows = [[m[k][y] for k in range(4)] for y in (0, 1, 1023, 2047)]
    _check_rows("2d", precision, rows, ref)
    # and the rows agree with each other to rounding
    for k in range(4):
        assert np.abs(m[k] - m[k][0]).max() <= (1e-15 if precision == "fp64" else 1e-7)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_3d_benchmark_size_rows_match_oracle(precision):
    # 512 x 256 x 256 D3Q39, LODI-RELAX / CBC-RELAX x-faces, periodic y and z: the bench.py launch
    from paper_2307_16766_amd import lbm3d
    nx, ny, nz = 512, 256, 256
    log(f"[gpu-case] full-size 3d {precision} {nx}x{ny}x{nz}")
    cs = math.sqrt(O3.lattice()[0])
    r, ux, uy, T = _profile(nx, 490.0, 5.0, 0.05 * cs)
    shape = (nz, ny, nx)
    fields = [np.broadcast_to(a, shape) for a in (r, ux, uy, np.zeros(nx), T)]
    bc = ["lodi_relax", "cbc_relax"]
    relax = dict(sigma=0.25, alpha=0.05, mach=0.05)
    g = lbm3d.LBM3D(nx, ny, nz, 0.9, bc, fields, precision=precision)
    g.set_relax(-1, **relax)
    g.step(STEPS)
    m = g.macro_numpy()
    g.close()
    o = O3.Oracle3D(nx, 4, 4, 0.9, bc)
    o.set_relax(-1, **relax)
    o.init(*[np.broadcast_to(a, (4, 4, nx)) for a in (r, ux, uy, np.zeros(nx), T)])
    o.step(STEPS)
    ref = [o.macro()[k][0, 0] for k in (0, 1, 4)]
    rows = [[m[k][z, y] for k in (0, 1, 4)] for z, y in ((0, 0), (17, 200), (255, 255), (128, 3))]
    _check_rows("3d", precision, rows, ref)
    for k in range(5):
        assert np.abs(m[k] - m[k][0, 0]).max() <= (1e-15 if precision == "fp64" else 1e-7)


@pytest.mark.parametrize("precision,nx,ny", [("fp32dev", 32768, 16384), ("fp64", 16384, 16384)])
def test_2d_maximum_size_rows_match_oracle(precision, nx, ny):
    # grids that fill most of the 288 GB of one GPU (159 GB of populations): the element offsets
    # of the population planes pass 2^32, so any 32-bit index arithmetic would show; every
    # sampled row must equal the oracle's four-row run of the same x-profile
    import torch
    from paper_2307_16766_amd import lbm
    log(f"[gpu-case] maximum-size 2d {precision} {nx}x{ny}")
    dev = torch.device("cuda", 0)
    r, ux, uy, T = _profile(nx, nx - 26.0, 6.0, 0.1 * CS_37)
    fields = [torch.tensor(a, device=dev).expand(ny, nx) for a in (r, ux, uy, T)]
    bc = ["dirichlet", "lodi_relax", "periodic", "periodic"]
    relax = dict(sigma=0.25, mach=0.05)
    g = lbm.LBM(37, nx, ny, TAU_37, bc, fields, precision=precision)
    del fields
    g.set_relax(-1, **relax)
    g.step(STEPS)
    m = g.macroscopic()
    sample = (0, 1, ny // 2 - 1, ny - 1)
    rows = [[m[k][y].cpu().numpy() for k in range(4)] for y in sample]
    spread = max(float((m[k] - m[k][0:1]).abs().max()) for k in range(4))
    g.close()
    del m, g
    torch.cuda.empty_cache()
    o = O.Oracle(37, nx, 4, TAU_37, bc)
    o.set_relax(-1, **relax)
    o.init(*[np.broadcast_to(a, (4, nx)) for a in (r, ux, uy, T)])
    o.step(STEPS)
    ref = [a[0] for a in o.macro()]
    _check_rows("2d-max", precision, rows, ref)
    assert spread <= (1e-15 if precision == "fp64" else 1e-7)


@pytest.mark.parametrize("precision,nx,ny,nz", [("fp32dev", 1024, 512, 512), ("fp64", 1024, 512, 256)])
def test_3d_maximum_size_rows_match_oracle(precision, nx, ny, nz):
    # D3Q39 boxes of 84 GB of populations: element offsets past 2^32, every sampled row equal to
    # the oracle's 4 x 4 run of the same x-profile
    import torch
    from paper_2307_16766_amd import lbm3d
    log(f"[gpu-case] maximum-size 3d {precision} {nx}x{ny}x{nz}")
    dev = torch.device("cuda", 0)
    cs = math.sqrt(O3.lattice()[0])
    r, ux, uy, T = _profile(nx, nx - 22.0, 5.0, 0.05 * cs)
    fields = [torch.tensor(a, device=dev).expand(nz, ny, nx) for a in (r, ux, uy, np.zeros(nx), T)]
    bc = ["lodi_relax", "cbc_relax"]
    relax = dict(sigma=0.25, alpha=0.05, mach=0.05)
    g = lbm3d.LBM3D(nx, ny, nz, 0.9, bc, fields, precision=precision)
    del fields
    g.set_relax(-1, **relax)
    g.step(STEPS)
    m = g.macroscopic()
    sample = ((0, 0), (nz // 2, ny - 1), (nz - 1, 3), (nz - 1, ny - 1))
    rows = [[m[k][z, y].cpu().numpy() for k in (0, 1, 4)] for z, y in sample]
    spread = max(float((m[k] - m[k][0:1, 0:1]).abs().max()) for k in range(5))
    g.close()
    del m, g
    torch.cuda.empty_cache()
    o = O3.Oracle3D(nx, 4, 4, 0.9, bc)
    o.set_relax(-1, **relax)
    o.init(*[np.broadcast_to(a, (4, 4, nx)) for a in (r, ux, uy, np.zeros(nx), T)])
    o.step(STEPS)
    ref = [o.macro()[k][0, 0] for k in (0, 1, 4)]
    _check_rows("3d-max", precision, rows, ref)
    assert spread <= (1e-15 if precision == "fp64" else 1e-7)
