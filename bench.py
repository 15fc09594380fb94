#!/usr/bin/env python3
"""Benchmark of the SAP-preconditioned FGMRES-DR Wilson-Dirac solver on one
MI355X.

A step is one complete solve D x = b to a true FP64 relative residual of
1e-10 (every row of the method: SAP sweeps, FP64 operator, Arnoldi,
least squares, deflated restarts, explicit residuals). The default
workload is the 32^3 x 64 lattice with eps = 0.7 links at a near-critical
mass, FP16-storage SAP (4^4 blocks, 2 cycles, 5 MR steps) inside FP64
FGMRES-DR(30, 12). The same solve with all-FP64 SAP is timed beside it, the
Wilson-Dirac operator alone is timed at each storage precision, and the
FP64 CPU oracle is timed on a bounded sample of the same work.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop x 2.4 GHz, packed FP32 disabled
FP64_VALU_PEAK_TFLOPS = 78.6

WORKLOADS = {
    # name: lattice, eps, gauge seed, mass spec, SAP, solver
    "32^3x64": dict(L=(32, 32, 32, 64), eps=0.7, seed=0, mass=(("16^3x32_eps0.7", "12^4_eps0.7"), 0.01),
                    block=(4, 4, 4, 4), ncycles=2, nmr=5, storage="f16", m=30, k=12),
    "16^3x32": dict(L=(16, 16, 16, 32), eps=0.6, seed=0, mass=(("16^3x32_eps0.6", "12^4_eps0.6"), 0.001),
                    block=(4, 4, 4, 4), ncycles=2, nmr=5, storage="f32", m=30, k=10),
    "8^4": dict(L=(8, 8, 8, 8), eps=0.3, seed=0, mass=(None, -0.1),
                block=(4, 4, 4, 4), ncycles=1, nmr=4, storage="f16", m=20, k=5),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mass_for(spec):
    """m0 = m_c + delta with m_c = -Re(leftmost eigenvalue of D(0)), computed
    by the oracle for the largest lattice of the same link distribution that
    has been tuned (tests/golden/critical_mass.json). Returns (m0, source)."""
    names, delta = spec
    if names is None:
        return delta, "fixed"
    with open(os.path.join(ROOT, "tests", "golden", "critical_mass.json")) as f:
        data = json.load(f)
    for name in names:
        if name in data:
            return data[name]["m_c"] + delta, f"m_c({name}) + {delta}"
    raise KeyError(f"no critical mass for {names}")


def source_sha(files):
    import hashlib
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(ROOT, "paper_1204_5463_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of the kernel class `key` (class/workload/storage)
    from the committed counter summary (two rocprofv3 --pmc passes,
    FETCH_SIZE then WRITE_SIZE, scaled by what the counters read for a plain
    copy), or None if absent or if the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    ent = prof.get("kernels", {}).get(key)
    if not ent:
        return None
    if ent.get("source_sha") != source_sha(ent.get("sources", [])):
        return None
    return ent["bytes_per_launch"]


def time_dslash(P, torch, f, m0, prec, reps=50, warm=10):
    """Average kernel time of D at storage precision prec (events on the launch stream)."""
    V = f.volume
    x = torch.randn((V * 12, 2), dtype=torch.float64, device="cuda")
    xc = torch.view_as_complex(x)
    xi = f.pack(prec, xc)
    yi = torch.empty_like(xi)
    del x, xc
    for _ in range(warm):
        f.apply_ex(m0, prec, xi, yi)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        f.apply_ex(m0, prec, xi, yi)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = V * 60 * P.PAIR_BYTES[prec]
    del xi, yi
    return ms, nbytes / ms / 1e6


def copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / ms / 1e6


def cpu_baseline(L, eps, seed, m0, wl, iterations, cycles):
    """Times the oracle as it stands on a bounded sample of the workload and
    projects solves/s: one whole-lattice operator application, one block-
    operator application and one Gram-Schmidt update (vdot + axpy) at the
    full lattice size, combined with the per-iteration operation counts of
    the GPU solve (SAP: ncycles x 2 colours x (D + nmr block-D); one FP64 D;
    modified GS over j+1 vectors, j averaged over a cycle)."""
    import numpy as np

    import synth
    from oracle import sap as S
    from oracle import wilson as W

    U = synth.gauge_field(L, eps, seed)
    x = synth.gaussian_spinor(L, 1000)
    t0 = time.perf_counter()
    y = W.apply_D(U, m0, x)
    t_d = time.perf_counter() - t0
    t0 = time.perf_counter()
    y = W.apply_D_blocks(U, m0, x, wl["block"])
    S.block_sum(np.abs(y) ** 2, L, wl["block"])
    t_db = time.perf_counter() - t0
    a, b = x.reshape(-1), y.reshape(-1)
    t0 = time.perf_counter()
    h = np.vdot(a, b)
    b = b - h * a
    t_gs = time.perf_counter() - t0
    sample_s = t_d + t_db + t_gs
    m, k = wl["m"], wl["k"]
    j_avg = (k + m) / 2.0
    per_iter = wl["ncycles"] * 2 * (t_d + wl["nmr"] * t_db) + t_d + (j_avg + 1) * t_gs
    per_solve = iterations * per_iter + cycles * (2 * t_d + m * t_gs)
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle timed on the full {'x'.join(map(str, L))} lattice: one D ({t_d:.2f} s), one block D + "
                   f"block sums ({t_db:.2f} s), one GS update ({t_gs:.3f} s); {sample_s:.1f} s total; projected to "
                   f"{iterations} iterations / {cycles} cycles of the GPU solve ({per_solve:.0f} s per solve); "
                   f"NumPy single-threaded on {platform.processor() or platform.machine()}, os.cpu_count()="
                   f"{os.cpu_count()}"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--workload", default="32^3x64", choices=sorted(WORKLOADS))
    ap.add_argument("--skip-fp64", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--skip-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--skip-dslash", action="store_true", help="skip the per-precision operator timings")
    ap.add_argument("--m0", type=float, default=None, help="override the workload's mass (exploration only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU volume split is a design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1204_5463_amd as P
    import synth

    wl = WORKLOADS[args.workload]
    L = wl["L"]
    if args.m0 is None:
        m0, mass_src = mass_for(wl["mass"])
    else:
        m0, mass_src = args.m0, "command line"
    prec = P.PREC_NAMES[wl["storage"]]
    log(f"[bench] workload {args.workload}: L={L} eps={wl['eps']} m0={m0:.6f}; generating inputs")
    t0 = time.time()
    U = synth.gauge_field(L, wl["eps"], wl["seed"])
    b = synth.gaussian_spinor(L, 1000)
    log(f"[bench] inputs ready in {time.time() - t0:.1f} s")
    ctx = P.Context(0)
    f = P.Field(ctx, L, wl["block"], P.to_device(U))
    del U
    bt = P.to_device(b)
    sap = P.SapParams(block=wl["block"], ncycles=wl["ncycles"], nmr=wl["nmr"], storage=prec)
    params = P.SolverParams(m=wl["m"], k=wl["k"], tol=1e-10, restart_t=5.0, max_iter=20000, sap=sap)

    for i in range(args.warmup):
        _, st = f.solve(m0, params, bt)
        log(f"[bench] warmup solve {i}: {st[0].iterations} it, {st[0].seconds:.3f} s, relres {st[0].true_relres:.2e}")

    # ---- timed region: K complete solves
    ctx.profile_reset()
    ctx.profile(True)
    torch.cuda.synchronize()
    lat, stats = [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        x, st = f.solve(m0, params, bt)
        lat.append(time.perf_counter() - ts)
        stats.append(st[0])
        log(f"[bench] solve {i}: {st[0].iterations} it, {lat[-1]:.3f} s, relres {st[0].true_relres:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ctx.profile(False)
    kern = ctx.profile_stats()
    value = args.steps / elapsed
    st0 = stats[-1]

    # independent FP64 residual check of the last solution (library FP64 operator)
    r = bt - f.apply(m0, x)
    relres_check = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(bt))
    del r

    # dominant kernel class in the timed region
    dom = max(kern, key=lambda k: kern[k]["ms"])
    kd = kern[dom]
    avg_ms = kd["ms"] / max(1, kd["launches"])
    if dom == "sap":
        peak = FP64_VALU_PEAK_TFLOPS if prec == P.DW_PREC_F64 else FP32_VALU_PEAK_TFLOPS
        achieved = kd["flops"] / kd["ms"] / 1e9
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": None}
    else:
        achieved = kd["bytes"] / kd["ms"] / 1e6
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
    roofline["traffic"] = measured_traffic(f"{dom}/{args.workload}/{wl['storage']}")
    roofline.update({"kernel_class": dom, "avg_launch_ms": round(avg_ms, 4), "launches": kd["launches"],
                     "algorithmic_bytes_per_launch": kd["bytes"] / max(1, kd["launches"]),
                     "algorithmic_flops_per_launch": kd["flops"] / max(1, kd["launches"])})
    kernels = {}
    for k, v in kern.items():
        if v["launches"] == 0:
            continue
        kernels[k] = {"ms_per_solve": round(v["ms"] / args.steps, 3), "launches": v["launches"],
                      "avg_us": round(1000 * v["ms"] / v["launches"], 2),
                      "GB/s": round(v["bytes"] / v["ms"] / 1e6, 1) if v["ms"] > 0 else None,
                      "TFLOP/s": round(v["flops"] / v["ms"] / 1e9, 2) if v["ms"] > 0 and v["flops"] else None}

    out_extra = {}
    # ---- all-FP64 comparison solve
    if not args.skip_fp64:
        p64 = P.SolverParams(m=wl["m"], k=wl["k"], tol=1e-10, restart_t=5.0, max_iter=20000,
                             sap=P.SapParams(block=wl["block"], ncycles=wl["ncycles"], nmr=wl["nmr"],
                                             storage=P.DW_PREC_F64))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, s64 = f.solve(m0, p64, bt)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - ts
        log(f"[bench] FP64 solve: {s64[0].iterations} it, {t64:.3f} s, relres {s64[0].true_relres:.2e}")
        out_extra.update({"fp64_solves_per_s": round(1.0 / t64, 4), "fp64_iterations": s64[0].iterations,
                          "speedup_vs_fp64": round(value * t64, 3)})

    # ---- Wilson-Dirac operator alone, each storage precision
    if not args.skip_dslash:
        ds = {}
        for name in ("f64", "f32", "f16", "bf16"):
            ms, gbs = time_dslash(P, torch, f, m0, P.PREC_NAMES[name])
            ds[name] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 3)}
            log(f"[bench] D at {name}: {ms:.4f} ms, {gbs:.0f} GB/s")
        out_extra["dslash"] = ds
        out_extra["copy_GB/s"] = round(copy_bandwidth(torch), 1)

    f.close()
    del bt
    torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(L, wl["eps"], wl["seed"], m0, wl, st0.iterations, st0.cycles)

    lat_ms = sorted(1000 * t for t in lat)
    line = {
        "metric": "solves/s to 1e-10 true residual, mixed-precision SAP+FGMRES-DR (Dslash HBM GB/s and "
                  "all-FP64 GPU solver alongside)",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec != P.DW_PREC_F64 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} lattice, eps={wl['eps']} SU(3) links (seed 0), m0={m0:.6f} "
                               f"near-critical, Gaussian RHS, SAP {wl['storage']} storage "
                               f"{'x'.join(map(str, wl['block']))} blocks s={wl['ncycles']} nMR={wl['nmr']}, "
                               f"FGMRES-DR({wl['m']},{wl['k']}) FP64 outer, tol 1e-10",
                   "lattice": list(L), "m0": m0, "m0_from": mass_src, "sap_storage": wl["storage"],
                   "parallelism": "single GPU"},
        "iterations": st0.iterations,
        "cycles": st0.cycles,
        "clean_restarts": st0.clean_restarts,
        "true_relres": st0.true_relres,
        "true_relres_check": relres_check,
        "p50_ms": round(lat_ms[len(lat_ms) // 2], 2),
        "p99_ms": round(lat_ms[min(len(lat_ms) - 1, int(math.ceil(0.99 * len(lat_ms))) - 1)], 2),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    line.update(out_extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
