"""The allocation-free diagnostics entry point against lbm_diagnostics (GPU)."""
import numpy as np
import pytest

from gpu_cases import TAU_37, log
from paper_2307_16766_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

BC = ["lodi_relax", "cbc_relax", "lodi_relax", "lodi_relax"]
RELAX = dict(sigma=0.25, alpha=0.1, mach=0.05)


def _compare(got, ref, exact):
    # sums: equal bit for bit where every work-group takes one row tile, else to rounding of the
    # FP64 sums (folding order); max |u|, the non-finite count and the step count are exact
    assert got[5] == ref[5] and got[6] == ref[6] and got[7] == ref[7]
    if exact:
        assert np.array_equal(got, ref), (got, ref)
    else:
        for k in (0, 3):
            assert abs(got[k] - ref[k]) <= 1e-13 * abs(ref[k]), (k, got[k], ref[k])
        for k in (1, 2):
            assert abs(got[k] - ref[k]) <= 1e-13 * abs(ref[0]), (k, got[k], ref[k])
        assert abs(got[4] - ref[4]) <= 1e-12 * abs(ref[4]), (got[4], ref[4])


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_noalloc_diagnostics_match_lbm_diagnostics(precision):
    import torch
    # two calls in a row on the shared scratch: 4100 x 1030 (17 tiles per row, 17510 > 16384
    # tiles: two tiles per work-group), then a smaller grid (one tile per work-group)
    for nx, ny, steps, exact in ((4100, 1030, 3, False), (300, 70, 5, True)):
        log(f"[gpu-case] diagnostics_noalloc {precision} {nx}x{ny}")
        f = W.temperature_pulse(nx, ny, amp=1e-3, width=20.0)
        g = lbm.LBM(37, nx, ny, TAU_37, BC, f, precision=precision)
        g.set_relax(-1, **RELAX)
        g.step(steps)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device=g.device)
        g.diagnostics_noalloc(out)
        torch.cuda.synchronize(g.device)
        got = out.cpu().numpy()
        ref = g.diagnostics()
        assert ref[7] == steps
        _compare(got, ref, exact)
        g.close()
