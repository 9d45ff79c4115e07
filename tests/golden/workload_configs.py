"""Nodes and step counts sampled from the long workload runs C2, C3 and C5.

Shared by the oracle-only script that writes the stored expected values
(`make_workload_goldens.py`) and by the GPU tests that compare against them.  The workloads
themselves (sizes, boundary kinds, relaxation settings, initial fields) come from
`paper_2307_16766_amd.workloads.config`; this module adds the snapshot steps and the sampled rows
and columns, and holds none of the method's arithmetic.
"""
import numpy as np

from paper_2307_16766_amd import workloads as W


def _span(a, b):
    return list(range(a, b))


# per workload: snapshot steps (strongest boundary interaction, last step) and sampled rows and
# columns (through the boundary layers, the corners, the outflow strip and the interior)
SAMPLES = {
    # the pulse reaches the sides at ~200 steps and the corners at ~300
    "c2": dict(snapshots=[300, 5000], cols=_span(0, 6) + [128, 255, 256] + _span(506, 512),
               rows=_span(0, 6) + [255, 256] + _span(506, 512)),
    # the vortex core reaches the outflow at ~4600 steps
    "c3": dict(snapshots=[4600, 6000], cols=_span(0, 6) + [256, 512, 768] + _span(1018, 1024),
               rows=[0, 127, 255, 256, 383, 511]),
    "c5": dict(snapshots=[500, 1000], cols=_span(0, 6) + [2048] + _span(4089, 4096), rows=[0, 1024, 1034, 2047]),
}


def config(name, cs2, alpha_c3=None):
    """Workload `name` (W.config) with its snapshot steps and sampled rows and columns; C3 with a
    transverse relaxation other than Ma is named c3_alpha<value>."""
    cfg = dict(W.config(name, cs2, alpha_c3))
    cfg.update(SAMPLES[name])
    cfg["name"] = name if (name != "c3" or alpha_c3 is None or alpha_c3 == 0.2) else f"c3_alpha{alpha_c3:g}"
    return cfg


CONFIGS = {k: (lambda cs2, k=k: config(k, cs2)) for k in SAMPLES}


def sample(fields4, cfg):
    """Rows and columns of (rho, ux, uy, T): arrays [4][len(rows)][nx] and [4][ny][len(cols)]."""
    F = np.stack([np.asarray(a, dtype=np.float64) for a in fields4])
    return F[:, cfg["rows"], :].copy(), F[:, :, cfg["cols"]].copy()
