"""Whole-run parity of the long workloads against the oracle: C2 (5000 steps), C3 (6000 steps)
and C5 (1000 steps) on the GPU, FP64 and FP32 deviation storage, compared node by node on the
rows and columns that `tests/golden/make_workload_goldens.py` stored from the oracle's run
(through the boundary layers, the corners, the outflow strip and the interior), at the step of
strongest boundary interaction and at the last step, and on whole-field sums of squares (of rho, T and |u|).

Bounds: the relative L2 error over the sampled nodes of rho, u (as a vector) and T is at most
1e-12 in FP64 and 2e-5 in FP32 deviation storage, and every node's rho and T error relative to the
field's largest sampled magnitude is within the same bound; in FP64, where the fluid is at rest
apart from the pulse (rms |u| below 1e-3: C2), u also gets the rounding floor per step of the other
parity tests.  The node-wise u errors are logged, not bounded: where the pulse has left (C2 after
5000 steps, rms |u| ~ 2e-8) single nodes carry the storage rounding at several times the mean.  The
achieved errors are appended to the file named by PARITY_LOG, when set."""
import math
import os
import sys

import numpy as np
import pytest

from gpu_cases import CS2_37, TOL, U_FLOOR_BELOW, log, record

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import workload_configs as WC  # noqa: E402

pytestmark = pytest.mark.gpu


def _golden(name):
    path = os.path.join(HERE, "golden", f"{name}_samples.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_workload_goldens.py)")
    return np.load(path, allow_pickle=False)


def _compare(name, precision, n, got_rows, got_cols, ref_rows, ref_cols, sumsq_got, sumsq_ref):
    rel, floor = TOL[precision]
    g = np.concatenate([got_rows.reshape(4, -1), got_cols.reshape(4, -1)], axis=1)
    r = np.concatenate([ref_rows.reshape(4, -1), ref_cols.reshape(4, -1)], axis=1)
    e_rho = np.linalg.norm(g[0] - r[0]) / np.linalg.norm(r[0])
    e_T = np.linalg.norm(g[3] - r[3]) / np.linalg.norm(r[3])
    du = np.sqrt((g[1] - r[1]) ** 2 + (g[2] - r[2]) ** 2)
    umag = np.sqrt(r[1] ** 2 + r[2] ** 2)
    e_u = np.linalg.norm(du) / np.linalg.norm(umag)
    rms_u = float(np.sqrt(np.mean(umag ** 2)))
    at_rest = rms_u < U_FLOOR_BELOW and floor > 0
    node_rho = np.abs(g[0] - r[0]).max() / np.abs(r[0]).max()
    node_T = np.abs(g[3] - r[3]).max() / np.abs(r[3]).max()
    node_u = du.max() / umag.max()
    e_sq = [abs(a - b) / b for a, b in zip(sumsq_got, sumsq_ref)]
    # u as a vector, as e_u: the component sums' errors over the sum of |u|^2 (after the vortex of
    # C3 has left, u_y is a small part of |u| and its own sum is no scale for the error)
    e_sq_u = (abs(sumsq_got[1] - sumsq_ref[1]) + abs(sumsq_got[2] - sumsq_ref[2])) / (sumsq_ref[1] + sumsq_ref[2])
    entry = {"case": f"{name} whole run (sampled)", "precision": precision, "step": int(n), "rel_rho": e_rho,
             "rel_u": e_u, "rel_T": e_T, "node_rho": node_rho, "node_u": node_u, "node_T": node_T, "rms_u": rms_u,
             "u_floor": at_rest, "sumsq_rel": e_sq, "sumsq_u_rel": e_sq_u}
    record(entry)
    log(f"[gpu-case] {name} {precision} step {n}: {entry}")
    assert max(e_rho, e_T, node_rho, node_T) <= rel, entry
    assert e_sq[0] <= 2 * rel and e_sq[3] <= 2 * rel, entry
    if at_rest:
        assert np.sqrt(np.mean(du ** 2)) <= rel * rms_u + floor * (n + 1), entry
    else:
        assert e_u <= rel and e_sq_u <= 2 * rel, entry


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_whole_run_against_oracle_samples(name, precision):
    from paper_2307_16766_amd import lbm
    G = _golden(name)
    cfg = WC.CONFIGS[name](CS2_37)
    assert abs(cfg["tau"] - float(G["tau"])) < 1e-15
    assert list(G["rows"]) == cfg["rows"] and list(G["cols"]) == cfg["cols"]
    log(f"[gpu-case] {name} {precision} whole run to step {max(cfg['snapshots'])}")
    g = lbm.LBM(37, cfg["nx"], cfg["ny"], cfg["tau"], cfg["bc"], cfg["fields"](), precision=precision)
    g.set_relax(-1, **cfg["relax"])
    if cfg["inlet"] is not None:
        g.set_inlet(*cfg["inlet"])
    done = 0
    for n in cfg["snapshots"]:
        g.step(n - done)
        done = n
        F = g.macro_numpy()
        rows, cols = WC.sample(F, cfg)
        sumsq = [float(np.sum(z * z)) for z in F]
        _compare(name, precision, n, rows, cols, G[f"rows_{n}"], G[f"cols_{n}"], sumsq, G[f"sumsq_{n}"])
    assert g.diagnostics()[6] == 0
    g.close()
