#!/usr/bin/env python
"""Throughput benchmark of the thermal LBM with characteristic boundaries on one MI355X.

Workload (the throughput configuration): D2Q37, 4096 x 2048 nodes, FP32 deviation storage,
shear layer u_x = 0.1 tanh((y - ny/2)/10) plus seeded noise (amplitude 1e-3, seed 16766),
equilibrium Dirichlet inlet at x = 0 with the unperturbed profile, LODI-RELAX outflow at
x = nx-1 (sigma = 0.25), periodic in y, nu = 0.1.  One step = bulk stream + collide over every
bulk node plus the characteristic boundary solve and reconstruction (lbm_step).

Prints one JSON line: MLUPS of the FP32 deviation path over all nx*ny nodes, the roofline of the
step kernel k_step (one launch per step: bulk stream + collide and the boundary chunks), with
algorithmic bytes per launch = 2 q s per bulk node (read q populations, write q) + q s per
written boundary-layer node + q s per re-pulled strip node (s = 4 or 8 bytes), over its
HIP-event-timed duration, against 8 TB/s; the FP64 path on the same workload; the adjoint, D2Q17
and D3Q39 lines; the workloads C1..C4 at full size (whole-step and step-kernel MLUPS, both
precisions); and the FP64 CPU oracle timed on a bounded slab of the throughput workload and on
the C1..C5 inputs (all host threads and one).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TIMED_EVERY = 10        # kernel-timing stride inside the timed region (see run_gpu)
NX, NY = 4096, 2048
Q = 37
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_d2q37_fp32_4096x2048_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2307_16766_amd", "csrc", n) for n in ("kernels.h", "lattice.h")]


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(nx, ny):
    from paper_2307_16766_amd import workloads as W
    fields, prof = W.shear_layer(nx, ny, u0=0.1, thickness=10.0, noise=1e-3, seed=16766)
    return fields, prof


def relax_params(cs2):
    # reference Mach number of the outflow: peak shear-layer speed over the adiabatic sound speed
    return dict(sigma=0.25, alpha=0.0, mach=0.1 / math.sqrt(2.0 * cs2))


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def run_gpu(precision, steps, warmup, q=Q, tau=None):
    import torch
    from paper_2307_16766_amd import lbm
    cs2 = lbm.lattice_info(q)[0]
    if tau is None:
        tau = 0.5 + 0.1 / cs2
    fields, prof = workload(NX, NY)
    g = lbm.LBM(q, NX, NY, tau, ["dirichlet", "lodi_relax", "periodic", "periodic"], fields, precision=precision)
    g.set_relax(1, **relax_params(cs2))
    g.set_inlet(0, prof)
    del fields
    g.step(warmup)
    torch.cuda.synchronize()
    # every TIMED_EVERY-th step kernel of the timed region is bracketed by HIP events (each pair
    # adds ~7 us of event work to the stream, which would otherwise inflate the step time)
    g.set_kernel_timing(True, every=TIMED_EVERY)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(g.stream)
    g.step(steps)
    e1.record(g.stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    kms, launches = g.bulk_kernel_time()
    g.set_kernel_timing(False)
    diag = g.diagnostics()
    g.close()
    del g
    torch.cuda.empty_cache()
    bytes_per_launch = algorithmic_bytes(4 if precision == "fp32dev" else 8, q)
    # one step is one launch of k_step: the event-bracketed launches read ~1 us above the step
    # time (event work on the stream), so the smaller of the two is the kernel's duration
    bracketed_ms = kms / max(launches, 1)
    kernel_ms = min(bracketed_ms, step_ms)
    gbps = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    return {
        "ms_per_step": step_ms,
        "mlups": NX * NY / (step_ms * 1e-3) / 1e6,
        "bulk_kernel_ms": kernel_ms,
        "bulk_kernel_ms_bracketed": bracketed_ms,
        "bulk_launches": launches,
        "bulk_bytes_per_launch": bytes_per_launch,
        "bulk_GBps": gbps,
        "bulk_frac": gbps / HBM_PEAK_GBPS,
        "mass": diag[0],
        "finite": bool(diag[6] == 0),
    }


def run_adjoint_c4(steps=2000, every=50):
    """Adjoint workload: D2Q37 256 x 256, FP64, random initial temperature (std 1e-4, seed 2307),
    LODI-RELAX on all four sides and corners (sigma 0.25, alpha = Ma = 0), pressure loss at the
    final step.  Times a plain forward run of `steps` steps, the recording forward run (with a
    checkpoint every `every` steps) and the adjoint sweep (recomputation included)."""
    import torch
    from paper_2307_16766_amd import lbm
    from paper_2307_16766_amd import workloads as W
    cs2 = lbm.lattice_info(Q)[0]
    tau = 0.5 + 0.1 / cs2
    fields = W.random_temperature(256, 256, std=1e-4, seed=2307)
    bc = ["lodi_relax"] * 4
    relax = dict(sigma=0.25, alpha=0.0, mach=0.0)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    g = lbm.LBM(Q, 256, 256, tau, bc, fields, precision="fp64")
    g.set_relax(-1, **relax)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(g.stream)
    g.step(steps)
    e1.record(g.stream)
    torch.cuda.synchronize()
    fwd = e0.elapsed_time(e1)
    loss_fwd = g.diagnostics()[4]
    g.close()
    g = lbm.LBM(Q, 256, 256, tau, bc, fields, precision="fp64")
    g.set_relax(-1, **relax)
    torch.cuda.synchronize()
    e0, e1, e2 = ev(), ev(), ev()
    e0.record(g.stream)
    g.record(steps, every)
    e1.record(g.stream)
    grad, grel = g.adjoint()
    e2.record(g.stream)
    torch.cuda.synchronize()
    rec, adj = e0.elapsed_time(e1), e1.elapsed_time(e2)
    loss = g.diagnostics()[4]
    g.close()
    return {
        "workload": f"D2Q37 256x256 FP64, random temperature std 1e-4, LODI-RELAX x4 with corners, "
                    f"{steps} steps, checkpoint every {every}, pressure loss",
        "forward_ms": fwd, "record_ms": rec, "adjoint_ms": adj,
        "adjoint_over_forward": adj / fwd,
        "record_plus_adjoint_over_forward": (rec + adj) / fwd,
        "forward_us_per_step": fwd / steps * 1e3, "adjoint_us_per_step": adj / steps * 1e3,
        "loss": loss, "loss_plain_forward": loss_fwd,
        "dL_dsigma": float(grel[:, 0].sum()), "dL_dalpha": float(grel[:, 1].sum()),
    }


def run_3d(precision, steps, warmup, n=(512, 256, 256)):
    """D3Q39 (Appendix A) on 512 x 256 x 256: LODI-RELAX and CBC-RELAX x-faces, periodic y and z,
    a temperature blob in a uniform stream.  MLUPS over all nodes and the bulk kernel's fraction
    of HBM bandwidth (2 q s bytes per bulk node per launch, HIP events on the stream)."""
    import torch
    from paper_2307_16766_amd import lbm3d
    nx, ny, nz = n
    dev = torch.device("cuda", 0)
    z = torch.arange(nz, device=dev, dtype=torch.float64)[:, None, None]
    y = torch.arange(ny, device=dev, dtype=torch.float64)[None, :, None]
    x = torch.arange(nx, device=dev, dtype=torch.float64)[None, None, :]
    one = torch.ones((nz, ny, nx), device=dev, dtype=torch.float64)
    T = one + 1e-3 * torch.exp(-((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2) / (2 * 20.0 ** 2))
    cs = math.sqrt(2.0 / 3.0)
    g = lbm3d.LBM3D(nx, ny, nz, 0.9, ["lodi_relax", "cbc_relax"], [one, 0.05 * cs * one, 0 * one, 0 * one, T],
                    precision=precision)
    del one, T
    g.set_relax(-1, sigma=0.25, alpha=0.05, mach=0.05)
    g.step(warmup)
    torch.cuda.synchronize()
    g.set_kernel_timing(True, every=TIMED_EVERY)
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ms, launches = g.bulk_kernel_time()
    d = g.diagnostics(allow_nonfinite=True)
    g.close()
    del g
    torch.cuda.empty_cache()
    esz = 4 if precision == "fp32dev" else 8
    bulk_bytes = 2 * 39 * esz * (nx - 6) * ny * nz
    gbps = bulk_bytes / (ms / launches * 1e-3) / 1e9
    return {"workload": f"D3Q39 {nx}x{ny}x{nz}, LODI-RELAX / CBC-RELAX x-faces, periodic y and z",
            "precision": precision, "mlups": nx * ny * nz / dt / 1e6, "ms_per_step": dt * 1e3,
            "bulk_kernel_ms": ms / launches, "bulk_GBps": gbps, "bulk_frac": gbps / HBM_PEAK_GBPS,
            "finite": bool(d[7] == 0)}


def run_diag_every_cost(steps=500, every=100):
    """Cost of lbm_step's non-finite check on the throughput workload (FP32 deviation storage):
    the same `steps` steps with and without a check every `every` steps, event-timed."""
    import torch
    from paper_2307_16766_amd import lbm
    cs2 = lbm.lattice_info(Q)[0]
    fields, prof = workload(NX, NY)
    g = lbm.LBM(Q, NX, NY, 0.5 + 0.1 / cs2, ["dirichlet", "lodi_relax", "periodic", "periodic"], fields,
                precision="fp32dev")
    del fields
    g.set_relax(1, **relax_params(cs2))
    g.set_inlet(0, prof)
    g.step(20)
    out = {}
    for n in (0, every, 0, every):
        g.set_diag_every(n)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.step(steps)
        e1.record(g.stream)
        torch.cuda.synchronize()
        out.setdefault(n, []).append(e0.elapsed_time(e1) / steps)
    g.close()
    torch.cuda.empty_cache()
    base, chk = min(out[0]), min(out[every])
    return {"workload": f"D2Q37 {NX}x{NY} FP32 deviation throughput run, {steps} steps",
            "every": every, "ms_per_step_off": base, "ms_per_step_on": chk, "overhead": chk / base - 1.0}


def run_config_gpu(name, precision, steps, warmup=20):
    """Whole-step and step-kernel MLUPS of workload C1..C4 (paper_2307_16766_amd.workloads) at its
    full size: one untimed pass of `steps` steps between two events for the step rate, then the
    same number of steps with every step kernel bracketed by events for the kernel rate."""
    import torch
    from paper_2307_16766_amd import lbm
    from paper_2307_16766_amd import workloads as W
    c = W.config(name, lbm.lattice_info(37)[0])
    g = lbm.LBM(c["stencil"], c["nx"], c["ny"], c["tau"], c["bc"], c["fields"](), precision=precision)
    g.set_relax(-1, **c["relax"])
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(steps)
    e1.record(g.stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    g.set_kernel_timing(True, every=1)
    g.step(steps)
    kms, launches = g.bulk_kernel_time()
    g.set_kernel_timing(False)
    finite = bool(g.diagnostics(allow_nonfinite=True)[6] == 0)
    g.close()
    n = c["nx"] * c["ny"]
    kernel_ms = kms / max(launches, 1)
    esz = 4 if precision == "fp32dev" else 8
    M = 1 if c["stencil"] == 9 else 3
    xb = c["nx"] - (0 if c["bc"][0] == "periodic" else 2 * M)
    yb = c["ny"] - (0 if c["bc"][2] == "periodic" else 2 * M)
    bulk_bytes = 2 * c["stencil"] * esz * xb * yb
    return {"workload": c["workload"], "precision": precision, "steps": steps,
            "ms_per_step": step_ms, "mlups": n / (step_ms * 1e-3) / 1e6,
            "kernel_ms": kernel_ms, "kernel_mlups": n / (kernel_ms * 1e-3) / 1e6,
            "bulk_bytes_GBps": bulk_bytes / (kernel_ms * 1e-3) / 1e9, "finite": finite}


def oracle_configs(budget_s=2.0):
    """The FP64 oracle on the inputs of C1..C5 at their full sizes: MLUPS with all host threads and
    with one, each timed over enough steps for about budget_s seconds (at least one step).  C5's
    single-thread figure is not taken (one step there takes about a minute); its multi-thread
    figure is extrapolated from the few steps timed."""
    from oracle import oracle as O
    from paper_2307_16766_amd import workloads as W
    cores = O.num_threads()
    out = {"cores": cores}
    for name in ("c1", "c2", "c3", "c4", "c5"):
        c = W.config(name, O.lattice(37)[0])
        o = O.Oracle(c["stencil"], c["nx"], c["ny"], c["tau"], c["bc"])
        o.set_relax(-1, **c["relax"])
        o.init(*c["fields"]())
        if c["inlet"] is not None:
            o.set_inlet(*c["inlet"])
        n = c["nx"] * c["ny"]
        res = {"workload": c["workload"]}
        for threads in ((cores, 1) if name != "c5" else (cores,)):
            O.set_threads(threads)
            t = time.perf_counter()
            o.step(1)
            per = time.perf_counter() - t
            k = max(1, min(200, int(budget_s / max(per, 1e-6))))
            t = time.perf_counter()
            o.step(k)
            dt = time.perf_counter() - t
            res["mlups_all_threads" if threads == cores else "mlups_one_thread"] = n * k / dt / 1e6
            res["steps_all_threads" if threads == cores else "steps_one_thread"] = k
        O.set_threads(cores)
        if name == "c5":
            res["note"] = f"extrapolated from {res['steps_all_threads']} timed steps; one thread: see cpu_baseline"
        o.close()
        out[name] = res
    return out


def algorithmic_bytes(esz, q=Q):
    """Bytes one step kernel must move: bulk nodes read and write q populations; the outflow
    side's M layers are written (equilibrium reconstruction) and its x_f column re-pulled (q
    reads); the Dirichlet inlet layers are static and cost nothing per step."""
    M = 3
    bulk_nodes = (NX - 2 * M) * NY
    layer_nodes = M * NY
    strip_nodes = NY
    return (2 * bulk_nodes + layer_nodes + strip_nodes) * q * esz


def cpu_baseline(steps=None):
    """FP64 oracle on a 512 x 256 slab of the same workload (same BCs, same fields recipe)."""
    from oracle import oracle as O
    nx, ny = 512, 256
    cs2 = O.lattice(Q)[0]
    tau = 0.5 + 0.1 / cs2
    fields, prof = workload(nx, ny)
    o = O.Oracle(Q, nx, ny, tau, ["dirichlet", "lodi_relax", "periodic", "periodic"])
    o.init(*fields)
    o.set_relax(1, **relax_params(cs2))
    o.set_inlet(0, prof)
    o.step(1)
    if steps is None:   # size the sample to about 15 s of CPU work
        t = time.perf_counter()
        o.step(2)
        per = (time.perf_counter() - t) / 2
        steps = max(3, min(400, int(15.0 / max(per, 1e-6))))
    t = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t
    cores = O.num_threads()
    # the same oracle on one core, over a quarter of the steps
    O.set_threads(1)
    s1 = max(2, steps // 4)
    t = time.perf_counter()
    o.step(s1)
    dt1 = time.perf_counter() - t
    O.set_threads(cores)
    return {
        "value": nx * ny * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{nx}x{ny} slab of the same workload (D2Q37, Dirichlet inlet + LODI-RELAX outflow, periodic y), "
                  f"{steps} steps, {dt:.1f} s; one core: {s1} steps, {dt1:.1f} s",
        "value_one_core": nx * ny * s1 / dt1 / 1e6,
    }


def traffic_from_profile():
    """HBM bytes per bulk launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(gib):
    """Plain device copy of known size (calibration of the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    eprint(f"copy probe: 5 copies of {n * 4} bytes")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-d2q17", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1..C4 GPU lines and the oracle on C1..C5")
    ap.add_argument("--cpu-steps", type=int, default=None)
    ap.add_argument("--copy-probe", type=float, default=None, metavar="GIB",
                    help="only run a plain copy of GIB gibibytes (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (sharding is a design note)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe is not None:
        copy_probe(args.copy_probe)
        return
    import torch
    if not torch.cuda.is_available():
        eprint("bench.py needs a GPU")
        sys.exit(1)
    torch.cuda.set_device(0)
    eprint(f"[bench] fp32dev {NX}x{NY}: warmup {args.warmup}, steps {args.steps}")
    r32 = run_gpu("fp32dev", args.steps, args.warmup)
    eprint(f"[bench] fp32dev: {r32['ms_per_step']:.3f} ms/step, bulk {r32['bulk_kernel_ms']:.3f} ms, "
           f"{r32['bulk_GBps']:.0f} GB/s")
    r64 = None
    if not args.no_fp64:
        s64 = max(10, args.steps // 2)
        eprint(f"[bench] fp64 {NX}x{NY}: steps {s64}")
        r64 = run_gpu("fp64", s64, max(5, args.warmup // 2))
        eprint(f"[bench] fp64: {r64['ms_per_step']:.3f} ms/step, bulk {r64['bulk_GBps']:.0f} GB/s")
    adj = None
    if not args.no_adjoint:
        eprint("[bench] adjoint workload (D2Q37 256x256, 2000 steps)")
        adj = run_adjoint_c4()
        eprint(f"[bench] adjoint: forward {adj['forward_ms']:.1f} ms, adjoint {adj['adjoint_ms']:.1f} ms, "
               f"ratio {adj['adjoint_over_forward']:.2f}")
    d17 = None
    if not args.no_d2q17:
        # the same workload on D2Q17 (3rd-order equilibrium, M = 3), tau = 0.9
        eprint(f"[bench] D2Q17 {NX}x{NY} (fp32dev, fp64)")
        d17 = {}
        for p in ("fp32dev", "fp64"):
            r = run_gpu(p, 300 if p == "fp32dev" else 150, 20, q=17, tau=0.9)
            d17[p] = {"workload": f"D2Q17 shear-layer run {NX}x{NY}, tau 0.9, Dirichlet inlet + LODI-RELAX outflow, periodic y",
                      "mlups": r["mlups"], "ms_per_step": r["ms_per_step"], "bulk_kernel_ms": r["bulk_kernel_ms"],
                      "bulk_GBps": r["bulk_GBps"], "bulk_frac": r["bulk_frac"], "finite": r["finite"]}
        eprint(f"[bench] d2q17: fp32 {d17['fp32dev']['ms_per_step']:.3f} ms/step, fp64 {d17['fp64']['ms_per_step']:.3f}")
    d3 = None
    if not args.no_3d:
        eprint("[bench] D3Q39 512x256x256 (fp32dev, fp64)")
        d3 = {p: run_3d(p, 50 if p == "fp32dev" else 25, 5) for p in ("fp32dev", "fp64")}
        eprint(f"[bench] d3q39: fp32 {d3['fp32dev']['ms_per_step']:.3f} ms/step, fp64 {d3['fp64']['ms_per_step']:.3f}")
    dchk = None
    if not args.no_configs:
        eprint("[bench] non-finite check every 100 steps (throughput run)")
        dchk = run_diag_every_cost()
        eprint(f"[bench] check every 100: {dchk['ms_per_step_on']:.4f} vs {dchk['ms_per_step_off']:.4f} ms/step "
               f"({100 * dchk['overhead']:.2f} %)")
    cfgs = None
    if not args.no_configs:
        eprint("[bench] workloads C1..C4 at full size (GPU)")
        cfgs = {"c1": {"fp64": run_config_gpu("c1", "fp64", 1000)}}
        for name, steps in (("c2", 300), ("c3", 300), ("c4", 1000)):
            cfgs[name] = {p: run_config_gpu(name, p, steps) for p in ("fp64", "fp32dev")}
        for name, d in cfgs.items():
            eprint(f"[bench] {name}: " + ", ".join(f"{p} {r['mlups']:.0f} MLUPS ({r['kernel_mlups']:.0f} kernel)"
                                                   for p, r in d.items()))
    cpu = None
    if not args.no_cpu_baseline:
        eprint("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(args.cpu_steps)
        eprint(f"[bench] cpu baseline: {cpu['value']:.3f} MLUPS on {cpu['cores']} threads")
        if not args.no_configs:
            eprint("[bench] oracle on the C1..C5 inputs")
            cpu["configs"] = oracle_configs()
    traffic = traffic_from_profile()
    out = {
        "metric": "MLUPS, D2Q37 FP32 deviation storage (HBM roofline fraction; FP64 path alongside)",
        "value": r32["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "D2Q37 shear-layer throughput run 4096x2048, FP32 deviation storage, "
                        "Dirichlet inlet + LODI-RELAX outflow, periodic y, 1 GPU",
            "nx": NX, "ny": NY, "stencil": "D2Q37", "precision": "fp32dev", "nu": 0.1,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": r32["bulk_GBps"],
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": r32["bulk_frac"],
            "traffic": traffic,
            "kernel": "k_step<37,float> (bulk tiles + boundary chunks, one launch per step)",
            "kernel_ms": r32["bulk_kernel_ms"],
            "kernel_ms_bracketed": r32["bulk_kernel_ms_bracketed"],
            "bytes_per_launch": r32["bulk_bytes_per_launch"],
        },
        "fp64": None if r64 is None else {
            "mlups": r64["mlups"], "ms_per_step": r64["ms_per_step"], "bulk_GBps": r64["bulk_GBps"],
            "bulk_frac": r64["bulk_frac"], "fp32dev_over_fp64": r32["mlups"] / r64["mlups"],
        },
        "adjoint": adj,
        "d2q17": d17,
        "d3q39": d3,
        "workloads": cfgs,
        "nonfinite_check": dchk,
        "cpu_baseline": cpu,
        "finite": r32["finite"] and (r64 is None or r64["finite"]),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
