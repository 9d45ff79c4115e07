"""Write <name>_samples.npz: sampled rows and columns of the oracle's macroscopic fields for the
long runs of the workloads C2 (5000 steps), C3 (6000 steps) and C5 (1000 steps), at the step
counts listed in `workload_configs.py`, for the GPU tests that compare whole runs against the
oracle.  Calls only the oracle (and the seeded input generators).

Stored per snapshot step n: rows_n [4][len(rows)][nx] and cols_n [4][ny][len(cols)] of
(rho, ux, uy, T), and the whole-field sums and sums of squares sum_n, sumsq_n [4].

Run from the repository root, one configuration per call:
    python tests/golden/make_workload_goldens.py c5 --threads 6   (about 2.1 hours)
    python tests/golden/make_workload_goldens.py c2 --threads 2   (about 25 minutes)
    python tests/golden/make_workload_goldens.py c3 --threads 2   (about 1 hour)
Optional: --alpha A (C3's transverse relaxation), --threads N.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from oracle import oracle as O  # noqa: E402
import workload_configs as WC  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=sorted(WC.CONFIGS))
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads:
        O.set_threads(a.threads)
    cs2 = O.lattice(37)[0]
    cfg = WC.config(a.config, cs2, a.alpha if a.config == "c3" else None)
    o = O.Oracle(cfg["stencil"], cfg["nx"], cfg["ny"], cfg["tau"], cfg["bc"])
    o.set_relax(-1, **cfg["relax"])
    o.init(*cfg["fields"]())
    if cfg["inlet"] is not None:
        o.set_inlet(*cfg["inlet"])
    out = {"rows": np.array(cfg["rows"]), "cols": np.array(cfg["cols"]), "tau": cfg["tau"],
           "snapshots": np.array(cfg["snapshots"])}
    t0 = time.time()
    done = 0
    for n in cfg["snapshots"]:
        while done < n:
            k = min(100, n - done)
            o.step(k)
            done += k
            print(f"{cfg['name']}: step {done} ({time.time() - t0:.0f} s)", flush=True)
        F = o.macro()
        d = o.diag()
        if d[6] != 0:
            raise SystemExit(f"{cfg['name']}: non-finite populations at step {n}")
        rows, cols = WC.sample(F, cfg)
        out[f"rows_{n}"] = rows
        out[f"cols_{n}"] = cols
        out[f"sum_{n}"] = np.array([np.sum(z) for z in F])
        out[f"sumsq_{n}"] = np.array([np.sum(z * z) for z in F])
    meta = {"workload": cfg["workload"], "relax": cfg["relax"], "bc": cfg["bc"],
            "oracle_threads": O.num_threads(), "seconds": round(time.time() - t0, 1),
            "command": "python tests/golden/make_workload_goldens.py " + " ".join(sys.argv[1:])}
    out["meta"] = np.array(json.dumps(meta))
    path = os.path.join(HERE, f"{cfg['name']}_samples.npz")
    np.savez_compressed(path, **out)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
