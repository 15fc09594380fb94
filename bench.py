#!/usr/bin/env python3
"""Benchmark of the SAP-preconditioned FGMRES-DR Wilson-Dirac solver on one
MI355X.

A step is one complete solve D x = b to a true FP64 relative residual of
1e-10 (every row of the method: SAP sweeps, FP64 operator, Arnoldi,
least squares, deflated restarts, explicit residuals). The default
workload is the 32^3 x 64 lattice with eps = 0.7 links at a near-critical
mass, FP16-storage SAP (4^4 blocks, 13 cycles, 8 MR steps, as tuned) inside
FP64 FGMRES-DR(30, 12). The same solve with all-FP64 SAP is timed beside it, the
Wilson-Dirac operator alone is timed at each storage precision, and the
FP64 CPU oracle is timed on a bounded sample of the same work.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X published FP64 vector peak

WORKLOADS = {
    # name: lattice, eps, gauge seed, mass spec, SAP, solver
    # FGMRES-DR(30, 12) as specified for this lattice; the SAP parameters
    # (4^4 blocks, 13 cycles, 8 MR steps) are the time-to-solution optimum
    # found by dw_autotune on this system (4^4 blocks, nMR 6..14, s 4..16;
    # an earlier search over all block shapes with extents 2/4/8 picked 4^4);
    # at m0 = m_c(12^4) + 0.01, s = 8, nMR = 9, the optimum of a search capped
    # at s = 8, needed 37 iterations and 6% more time; the starting point
    # s = 2, nMR = 5 needed 152 iterations and 2.5x the time
    # The mass: 0.005 above the critical mass estimated on the 16^3x32 field of
    # the same eps (no estimate converges on 32^3x64 itself); at this distance
    # the solve makes one deflated restart (0.01 above: 25 iterations in one
    # cycle; 0.002: 45; 0: 64)
    "32^3x64": dict(L=(32, 32, 32, 64), eps=0.7, seed=0,
                    mass=(("32^3x64_eps0.7", "16^3x32_eps0.7", "12^4_eps0.7"), 0.005),
                    block=(4, 4, 4, 4), ncycles=13, nmr=8, storage="f16", m=30, k=12),
    "16^3x32": dict(L=(16, 16, 16, 32), eps=0.6, seed=0, mass=(("16^3x32_eps0.6", "12^4_eps0.6"), 0.001),
                    block=(4, 4, 4, 4), ncycles=2, nmr=5, storage="f32", m=30, k=10),
    "8^4": dict(L=(8, 8, 8, 8), eps=0.3, seed=0, mass=(None, -0.1),
                block=(4, 4, 4, 4), ncycles=1, nmr=4, storage="f16", m=20, k=5),
    # 12 point-source + noise RHS in lock-step (one SAP / operator launch for
    # all of them); m, k reduced from (30, 12) so that the 12 FP64 Krylov
    # bases fit in one GPU's memory; block shape, cycles and MR steps from the
    # tuning (the starting point 8x4x4x4, s = 2, nMR = 5 takes 168 iterations
    # and 2.6x the time)
    "32^3x64x12": dict(L=(32, 32, 32, 64), eps=0.7, seed=0,
                       mass=(("32^3x64_eps0.7", "16^3x32_eps0.7", "12^4_eps0.7"), 0.005),
                       block=(4, 4, 4, 4), ncycles=13, nmr=8, storage="f16", m=20, k=8, nrhs=12, rhs="point"),
    # the same lattice with the clover term (c_sw = 1.9, as in the paper's
    # experiments), near the critical mass of the clover operator; the SAP
    # parameters re-tuned for the plain workload (s = 8, nMR = 9 takes 29
    # iterations and 6% more time)
    "32^3x64_clover": dict(L=(32, 32, 32, 64), eps=0.7, seed=0, csw=1.9,
                           mass=(("12^4_eps0.7_csw1.9", "8^4_eps0.7_csw1.9"), 0.01),
                           block=(4, 4, 4, 4), ncycles=13, nmr=8, storage="f16", m=30, k=12),
    "48^3x96": dict(L=(48, 48, 48, 96), eps=0.7, seed=0, mass=(("16^3x32_eps0.7", "12^4_eps0.7"), 0.01),
                    block=(8, 4, 4, 4), ncycles=2, nmr=5, storage="f16", m=30, k=12),
}

# serving stream: lattice sizes of the request mix (eps 0.6 links, gauge seed 0)
SERVE_LATTICES = {"8^4": (8, 8, 8, 8), "16^3x32": (16, 16, 16, 32), "24^3x48": (24, 24, 24, 48),
                  "32^3x64": (32, 32, 32, 64)}
SERVE_MASS = {"8^4": ("8^4_eps0.6",), "16^3x32": ("16^3x32_eps0.6", "12^4_eps0.6"),
              "24^3x48": ("24^3x48_eps0.6", "16^3x32_eps0.6", "12^4_eps0.6"),
              "32^3x64": ("32^3x64_eps0.6", "16^3x32_eps0.6", "12^4_eps0.6")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mass_for(spec):
    """m0 = m_c + delta with m_c = -Re(leftmost eigenvalue of D(0)), computed
    by the oracle's ARPACK run on the workload's own lattice where available,
    else on the largest lattice of the same link distribution that has been
    tuned (tests/golden/critical_mass.json). Returns (m0, source)."""
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


def time_dslash(P, torch, f, m0, prec, reps=50, warm=10, nrhs=1):
    """Average kernel time of D at storage precision prec (events on the launch
    stream) for nrhs right-hand sides in one launch."""
    V = f.volume
    x = torch.randn((nrhs * V * 12, 2), dtype=torch.float64, device="cuda")
    xc = torch.view_as_complex(x)
    xi = f.pack(prec, xc)
    yi = torch.empty_like(xi)
    del x, xc
    for _ in range(warm):
        f.apply_ex(m0, prec, xi, yi, nrhs=nrhs)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        f.apply_ex(m0, prec, xi, yi, nrhs=nrhs)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # links read once (36 pairs, + the clover term's 36), x read and y written
    # once per right-hand side (24 pairs)
    nbytes = V * ((36 + (36 if getattr(f, "csw", 0.0) else 0)) + 24 * nrhs) * P.PAIR_BYTES[prec]
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


def csw_requested(args, wl):
    return bool(args.csw or wl.get("csw", 0.0))


def solver_params(P, wl, prec, tuned=None):
    if tuned is not None:
        return tuned
    sap = P.SapParams(block=wl["block"], ncycles=wl["ncycles"], nmr=wl["nmr"], storage=prec)
    return P.SolverParams(m=wl["m"], k=wl["k"], tol=1e-10, restart_t=5.0, max_iter=20000, sap=sap)


def describe(params, P):
    inv = {v: k for k, v in P.PREC_NAMES.items()}
    sp = params.sap
    return (f"SAP {inv[sp.storage]} storage {'x'.join(map(str, sp.block))} blocks s={sp.ncycles} nMR={sp.nmr}, "
            f"FGMRES-DR({params.m},{params.k}) FP64 outer, tol {params.tol:g}")


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, max(0, int(math.ceil(q * len(xs))) - 1))]


def serve(args):
    """Serving stream: exponential inter-arrivals, a mix of lattice sizes
    and RHS counts near the critical mass, solved by the library's server
    (continuous batching on concurrent streams, FP16 SAP) and, for
    comparison, one request at a time with all-FP64 SAP (same SAP
    parameters) in the same order
    (its latencies follow from the measured service times and the same
    arrival times). Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1204_5463_amd as P
    import synth

    rng = np.random.default_rng(20)
    names = sorted(SERVE_LATTICES, key=lambda n: math.prod(SERVE_LATTICES[n]))
    log(f"[serve] generating gauge fields for {names}")
    fields = {n: P.to_device(synth.gauge_field(SERVE_LATTICES[n], 0.6, 0)) for n in names}
    mc = {}
    with open(os.path.join(ROOT, "tests", "golden", "critical_mass.json")) as fh:
        crit = json.load(fh)
    for n in names:
        src = next(s for s in SERVE_MASS[n] if s in crit)
        mc[n] = (crit[src]["m_c"], src)
    # SAP parameters from the time-to-solution tuning at 32^3x64 (the flat
    # optimum s = 6..8, nMR = 7..10), the same for every request
    def params(storage, graphs=False):
        return P.SolverParams(m=30, k=12, tol=1e-10, restart_t=5.0, max_iter=20000,
                              flags=P.SOLVE_GRAPHS if graphs else 0,
                              sap=P.SapParams(block=(4, 4, 4, 4), ncycles=args.serve_cycles, nmr=8,
                                              storage=storage))

    # RHS per request: 1..max_rhs, capped per lattice so that two requests
    # of the largest count fit the server's budget (0.8 of free memory)
    # side by side, by the footprint the server itself charges
    free = torch.cuda.mem_get_info()[0]
    cap = {}
    for n in names:
        L = SERVE_LATTICES[n]
        bmax = torch.empty((args.max_rhs,) + synth.lattice_shape(L) + (4, 3), dtype=torch.complex128, device="cuda")
        c = 1
        for k in range(1, args.max_rhs + 1):
            fp = P.Server.footprint(L, (4, 4, 4, 4), mc[n][0], fields[n], bmax[:k], params(P.DW_PREC_F16))
            if 2 * fp <= 0.8 * free:
                c = k
        cap[n] = c
        del bmax
    torch.cuda.empty_cache()
    log(f"[serve] RHS caps per lattice: {cap}")
    reqs, t = [], 0.0
    for i in range(args.requests):
        t += rng.exponential(args.mean_gap)
        n = names[int(rng.integers(len(names)))]
        nrhs = min(int(rng.integers(1, args.max_rhs + 1)), cap[n])
        delta = float(np.exp(rng.uniform(np.log(2e-3), np.log(2e-2))))
        reqs.append(dict(arrival=t, lattice=n, nrhs=nrhs, m0=mc[n][0] + delta, seed=3000 + 100 * i))
    log(f"[serve] {len(reqs)} requests over {t:.2f} s of arrivals, {sum(r['nrhs'] for r in reqs)} RHS")

    # The client's request buffers (right-hand sides and solutions) come from
    # one preallocated pool of slots + 2 buffer pairs, each large enough for the
    # largest request, so that the client's device memory stays fixed (a
    # caching allocator fed requests of many sizes would keep growing into the
    # memory the server's budget counts on).
    shp_of = {n: synth.lattice_shape(SERVE_LATTICES[n]) + (4, 3) for n in names}
    big = max(cap[n] * math.prod(shp_of[n]) for n in names)
    nbuf = args.slots + 2
    pool = torch.empty((nbuf, 2, big), dtype=torch.complex128, device="cuda") if args.serve_part != "fp64" else None
    free_bufs = list(range(nbuf))

    def rhs_into(r, out):
        # the request's right-hand sides, made on the device when it is sent:
        # seeded Gaussian real and imaginary parts of variance 1/2 (the serial
        # baseline draws the same)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(r["seed"])
        torch.view_as_real(out).normal_(0.0, math.sqrt(0.5), generator=gen)
        return out

    def rhs_of(r):
        shp = (r["nrhs"],) + shp_of[r["lattice"]]
        return rhs_into(r, torch.empty(shp, dtype=torch.complex128, device="cuda"))

    ctx = P.Context(0)
    # warm the kernels of every lattice once (untimed)
    for n in names:
        L = SERVE_LATTICES[n]
        f = P.Field(ctx, L, (4, 4, 4, 4), fields[n])
        f.solve(mc[n][0] + 0.05, params(P.DW_PREC_F16), P.to_device(synth.gaussian_spinors(L, 1, seed0=1)),
                raise_on_notconv=False)
        f.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    line = {
        "metric": "serving throughput (requests/s) of a Poisson stream of solve requests, continuous batching",
        "value": None,
        "unit": "requests/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, exponential gaps mean {args.mean_gap * 1e3:.0f} ms (seed 20), "
                               f"lattices {names} uniform, nrhs 1..{args.max_rhs} capped per lattice {cap}, "
                               f"eps=0.6 links, m0 = m_c + logU[2e-3, 2e-2], FP16 SAP 4^4 s={args.serve_cycles} nMR=8, "
                               f"FGMRES-DR(30,12), tol 1e-10, {args.slots} slots, restart cycles replayed as HIP graphs",
                   "m_c_from": {n: mc[n][1] for n in names}},
        "requests": len(reqs),
        "rhs_total": sum(r["nrhs"] for r in reqs),
        "offered_requests_per_s": round(len(reqs) / reqs[-1]["arrival"], 4),
    }
    rhs_total = line["rhs_total"]
    if args.serve_part in ("both", "mixed"):
        # Requests wait on the host until the server holds fewer than
        # slots + 2 unfinished ones (their inputs and outputs then go to
        # device memory), as a client would queue them; latency runs from
        # the arrival time.
        srv = P.Server(ctx, slots=args.slots, queue_capacity=nbuf)
        pending, done, lat, buf_of = {}, {}, [0.0] * len(reqs), {}
        t0 = time.perf_counter()
        i = 0
        while i < len(reqs) or pending:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["arrival"] <= now and free_bufs:
                r = reqs[i]
                shp = (r["nrhs"],) + shp_of[r["lattice"]]
                nel = math.prod(shp)
                q = free_bufs.pop()
                b = rhs_into(r, pool[q, 0, :nel].view(shp))
                tk = srv.submit(SERVE_LATTICES[r["lattice"]], (4, 4, 4, 4), r["m0"], fields[r["lattice"]], b,
                                params(P.DW_PREC_F16, graphs=True), x=pool[q, 1, :nel].view(shp))
                pending[tk] = i
                buf_of[tk] = q
                i += 1
            for tk in list(pending):
                out = srv.poll(tk)
                if out is not None:
                    x, st, tm = out
                    free_bufs.append(buf_of.pop(tk))
                    k = pending.pop(tk)
                    fin = time.perf_counter() - t0
                    done[k] = (st, tm, fin)
                    lat[k] = fin - reqs[k]["arrival"]
                    r = reqs[k]
                    log(f"[serve] request {k} {r['lattice']} nrhs={r['nrhs']} done: "
                        f"{max(s.iterations for s in st)} it (per RHS {[s.iterations for s in st]}), "
                        f"service {tm['running']:.3f} s, latency {lat[k]:.3f} s")
                    del x
            time.sleep(2e-4)
        makespan = time.perf_counter() - t0
        srv.close()
        # service time (admitted to done) per lattice: the sum over requests
        # against slots x makespan gives the slots' occupancy
        svc = {}
        for k in range(len(reqs)):
            n = reqs[k]["lattice"]
            svc.setdefault(n, []).append(done[k][1]["running"])
        line.update({
            "service_s_per_lattice": {n: {"requests": len(v), "mean": round(sum(v) / len(v), 4),
                                          "sum": round(sum(v), 2)} for n, v in svc.items()},
            "slot_occupancy": round(sum(sum(v) for v in svc.values()) / (args.slots * makespan), 3),
        })
        line.update({
            "value": round(len(reqs) / makespan, 4),
            "makespan_s": round(makespan, 3),
            "rhs_solves_per_s": round(rhs_total / makespan, 4),
            "p50_latency_ms": round(1e3 * pct(lat, 0.5), 1),
            "p99_latency_ms": round(1e3 * pct(lat, 0.99), 1),
            "all_converged": all(s.converged for k in range(len(reqs)) for s in done[k][0]),
        })

    if args.serve_part in ("both", "fp64"):
        # serial all-FP64 baseline: same order, one request at a time
        log("[serve] serial FP64 baseline")
        svc = []
        conv64 = True
        for k, r in enumerate(reqs):
            L = SERVE_LATTICES[r["lattice"]]
            b = rhs_of(r)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            f = P.Field(ctx, L, (4, 4, 4, 4), fields[r["lattice"]])
            _, st = f.solve(r["m0"], params(P.DW_PREC_F64, graphs=False), b, raise_on_notconv=False)
            f.close()
            torch.cuda.synchronize()
            svc.append(time.perf_counter() - ts)
            conv64 = conv64 and all(x.converged for x in st)
            log(f"[serve] serial {k} {r['lattice']} nrhs={r['nrhs']}: {svc[-1]:.3f} s")
        svc64 = {}
        for r, sv in zip(reqs, svc):
            svc64.setdefault(r["lattice"], []).append(sv)
        fin, lat64 = 0.0, []
        for r, sv in zip(reqs, svc):
            fin = max(fin, r["arrival"]) + sv
            lat64.append(fin - r["arrival"])
        line["serial_fp64"] = {"requests_per_s": round(len(reqs) / fin, 4) if fin > 0 else None,
                               "rhs_solves_per_s": round(rhs_total / fin, 4) if fin > 0 else None,
                               "busy_s": round(sum(svc), 3),
                               "service_s_per_lattice": {n: {"requests": len(v), "mean": round(sum(v) / len(v), 4),
                                                             "sum": round(sum(v), 2)} for n, v in svc64.items()},
                               "p50_latency_ms": round(1e3 * pct(lat64, 0.5), 1),
                               "p99_latency_ms": round(1e3 * pct(lat64, 0.99), 1),
                               "all_converged": conv64}
    print(json.dumps(line), flush=True)


def sap_study(args):
    """SAP iterated on its own, x_{k+1} = x_k + M (b - D x_k) with one SAP
    cycle per iteration (Section 3, Fig. 5), on the workload's lattice and
    block solves, at masses from well above to just below the critical one;
    once with the workload's fixed MR step count and once with the adaptive
    0.1 block-residual reduction (capped at twice that count). Prints one
    JSON line with the residual histories and asymptotic rates."""
    import numpy as np
    import torch

    import paper_1204_5463_amd as P
    import synth

    wl = WORKLOADS[args.workload]
    L = wl["L"]
    names, _ = wl["mass"]
    m_c, src = mass_for((names, 0.0)) if names is not None else (None, None)
    if m_c is None:
        raise SystemExit("the study needs a workload with a known critical mass")
    csw = args.csw or wl.get("csw", 0.0)
    log(f"[study] {args.workload}: L={L} eps={wl['eps']} m_c={m_c:.6f} ({src}); generating inputs")
    U = synth.gauge_field(L, wl["eps"], wl["seed"])
    b = synth.gaussian_spinor(L, 1000)
    ctx = P.Context(0)
    f = P.Field(ctx, L, wl["block"], P.to_device(U))
    del U
    if csw:
        f.set_clover(csw)
    bt = P.to_device(b)
    prec = P.PREC_NAMES[wl["storage"]]
    deltas = [0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 0.0, -0.02]
    variants = {"fixed": P.SapParams(block=wl["block"], ncycles=1, nmr=wl["nmr"], storage=prec),
                "adaptive": P.SapParams(block=wl["block"], ncycles=1, nmr=2 * wl["nmr"], storage=prec,
                                        mr_reduction=0.1)}
    out = {}
    for vname, sp in variants.items():
        rows = []
        for d in deltas:
            m0 = m_c + d
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, hist = f.sap_solve(m0, sp, bt, args.study_iters)
            sec = time.perf_counter() - t0
            n = len(hist) - 1
            # asymptotic rate: the last 20 iterations before the residual
            # reaches the FP64 floor
            e = next((k for k, h in enumerate(hist) if h < 1e-12), n)
            j = min(20, e)
            rate = (hist[e] / hist[e - j]) ** (1.0 / j) if j > 0 and hist[e - j] > 0 else None
            rows.append({"delta_m": d, "m0": round(m0, 6), "final_relres": hist[n], "rate": rate,
                         "converges": bool(rate is not None and rate < 1.0),
                         "ms_per_iteration": 1e3 * sec / max(n, 1),
                         "history": [float(f"{h:.4g}") for h in hist]})
            log(f"[study] {vname:8s} m0 = m_c {d:+.3f}: relres {hist[n]:.3e} after {n} iterations, "
                f"rate {rate:.4f}, {1e3 * sec / max(n, 1):.2f} ms/iteration")
        out[vname] = rows
    print(json.dumps({"metric": "sap_standalone_study", "workload": args.workload, "lattice": list(L),
                      "eps": wl["eps"], "csw": csw, "m_c": m_c, "m_c_source": src, "block": list(wl["block"]),
                      "nmr": wl["nmr"], "storage": wl["storage"], "cycles_per_iteration": 1,
                      "adaptive_reduction": 0.1, "iterations": args.study_iters, "data": "synthetic",
                      "variants": out}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--workload", default="32^3x64", choices=sorted(WORKLOADS))
    ap.add_argument("--skip-fp64", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--skip-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--skip-dslash", action="store_true", help="skip the per-precision operator timings")
    ap.add_argument("--skip-v32", action="store_true",
                    help="skip the FP32-basis and single-precision-Arnoldi comparison solves")
    ap.add_argument("--all-precisions", action="store_true",
                    help="also time the solve with FP16, BF16, FP32 and FP64 SAP storage")
    ap.add_argument("--m0", type=float, default=None, help="override the workload's mass (exploration only)")
    ap.add_argument("--csw", type=float, default=0.0, help="clover coefficient (0: plain Wilson operator)")
    ap.add_argument("--params", default=None,
                    help="override solver parameters, e.g. s=3,nmr=7,m=30,k=6,block=4x4x4x4,shared=1,red=0.1 "
                         "(exploration)")
    ap.add_argument("--also-k0", action="store_true", help="also run FGMRES(m) (k = 0) on the same system")
    ap.add_argument("--sequential", action="store_true",
                    help="multi-RHS workloads: also time the RHS one after another")
    ap.add_argument("--autotune", default=None, metavar="CACHE.json",
                    help="tune (block, nMR, s, m, k) by time to solution before timing (cached in this file)")
    ap.add_argument("--serve", action="store_true", help="run the serving stream instead of the solve benchmark")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--mean-gap", type=float, default=0.05, help="mean inter-arrival time (s)")
    ap.add_argument("--max-rhs", type=int, default=12)
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--serve-cycles", type=int, default=6, help="serving: SAP cycles per application")
    ap.add_argument("--serve-part", choices=("both", "mixed", "fp64"), default="both",
                    help="serving: run the server stream, the serial all-FP64 baseline, or both")
    ap.add_argument("--sap-study", action="store_true",
                    help="SAP as a stand-alone solver at masses around the critical one, fixed and adaptive "
                         "MR block solves, instead of the solve benchmark")
    ap.add_argument("--study-iters", type=int, default=60)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU volume split is a design, not built", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve(args)
    if args.sap_study:
        return sap_study(args)

    import numpy as np
    import torch

    import paper_1204_5463_amd as P
    import synth

    # all work on one non-default stream (HIP graph capture needs one)
    torch.cuda.set_stream(torch.cuda.Stream())
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
    nrhs = wl.get("nrhs", 1)
    if wl.get("rhs") == "point":
        b = np.stack([synth.point_source_noise(L, j, 1000 + j) for j in range(nrhs)])
    else:
        b = synth.gaussian_spinors(L, nrhs, seed0=1000)
    log(f"[bench] inputs ready in {time.time() - t0:.1f} s")
    ctx = P.Context(0)
    Ud = P.to_device(U)
    del U
    bt = P.to_device(b)
    params = solver_params(P, wl, prec)
    if args.params:
        for kv in args.params.split(","):
            key, val = kv.split("=")
            if key == "s":
                params.sap.ncycles = int(val)
            elif key == "nmr":
                params.sap.nmr = int(val)
            elif key == "block":
                params.sap.block = tuple(int(t) for t in val.split("x"))
            elif key in ("m", "k"):
                setattr(params, key, int(val))
            elif key == "shared":
                params.shared_defl = int(val)
            elif key == "graphs":
                params.flags = (params.flags & ~P.SOLVE_GRAPHS) | (P.SOLVE_GRAPHS if int(val) else 0)
            elif key == "v32":
                params.flags = (params.flags & ~P.SOLVE_V32) | (P.SOLVE_V32 if int(val) else 0)
            elif key == "inject":
                params.flags = (params.flags & ~P.SOLVE_INJECT) | (P.SOLVE_INJECT if int(val) else 0)
            elif key == "red":
                params.sap.mr_reduction = float(val)
            else:
                raise SystemExit(f"unknown parameter {key}")
    tune = None
    if args.autotune:
        log("[bench] autotuning (untimed)")
        ts = time.perf_counter()
        # the workload fixes FGMRES-DR(m, k); the SAP parameters are tuned
        space = P.TuneSpace(nmr=(4, 14), s=(2, 16), passes=2, iter_cap=2.0)
        params, trials = P.autotune(ctx, L, Ud, m0, params, bt, space=space, cache=P.TuneCache(args.autotune),
                                    csw=args.csw or wl.get("csw", 0.0))
        for t in trials:
            log(f"[bench]   trial {t}")
        tune = {"trials": len(trials), "tuning_s": round(time.perf_counter() - ts, 1)}
        torch.cuda.empty_cache()
    csw = args.csw or wl.get("csw", 0.0)
    f = P.Field(ctx, L, params.sap.block, Ud)
    if csw:
        f.set_clover(csw)
    del Ud

    def summary(st):
        return (f"{max(s.iterations for s in st)} it, relres <= {max(s.true_relres for s in st):.2e}, "
                f"converged {all(s.converged for s in st)}")

    for i in range(args.warmup):
        _, st = f.solve(m0, params, bt)
        log(f"[bench] warmup solve {i}: {summary(st)}, {st[0].seconds:.3f} s")

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
        stats.append(st)
        log(f"[bench] solve {i}: {summary(st)}, {lat[-1]:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ctx.profile(False)
    kern = ctx.profile_stats()
    value = nrhs * args.steps / elapsed
    stl = stats[-1]
    st0 = max(stl, key=lambda s: s.iterations)

    # the same solve without per-launch event timing (wall clock only)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    f.solve(m0, params, bt)
    torch.cuda.synchronize()
    unprofiled_ms = 1000 * (time.perf_counter() - ts)
    log(f"[bench] solve without event timing: {unprofiled_ms:.1f} ms")

    # the same solve replayed from captured restart cycles (DW_SOLVE_GRAPHS;
    # no per-launch event timing), wall clock over a few solves
    graph_fig = None
    if not (params.flags & P.SOLVE_GRAPHS):
        pg = dataclasses.replace(params, flags=params.flags | P.SOLVE_GRAPHS)
        f.solve(m0, pg, bt)  # captures
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        ts = time.perf_counter()
        for _ in range(reps):
            _, sg = f.solve(m0, pg, bt)
        torch.cuda.synchronize()
        tg = (time.perf_counter() - ts) / reps
        graph_fig = {"solves_per_s": round(nrhs / tg, 4), "ms_per_solve": round(1000 * tg, 2),
                     "iterations": max(s.iterations for s in sg)}
        log(f"[bench] solve replayed from captured cycles: {1000 * tg:.1f} ms")

    # FP64 residual check of the last solutions by the oracle's operator (eq. 1)
    # on the host, outside the timed region
    relres_oracle = None
    if not csw_requested(args, wl):
        from oracle import wilson as W
        log("[bench] oracle residual of the final solution")
        xh = x.cpu().numpy()
        Uh = synth.gauge_field(L, wl["eps"], wl["seed"])
        relres_oracle = 0.0
        for j in range(nrhs):
            r = b[j] - W.apply_D(Uh, m0, xh[j])
            relres_oracle = max(relres_oracle, float(np.linalg.norm(r) / np.linalg.norm(b[j])))
        del Uh, xh, r

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
    alg_bytes = kd["bytes"] / max(1, kd["launches"])
    roofline.update({"kernel_class": dom, "avg_launch_ms": round(avg_ms, 4), "launches": kd["launches"],
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "algorithmic_flops_per_launch": kd["flops"] / max(1, kd["launches"]),
                     "traffic_over_algorithmic": (round(roofline["traffic"] / alg_bytes, 3)
                                                  if roofline["traffic"] else None)})
    kernels = {}
    for k, v in kern.items():
        if v["launches"] == 0:
            continue
        kernels[k] = {"ms_per_solve": round(v["ms"] / args.steps, 3), "launches": v["launches"],
                      "avg_us": round(1000 * v["ms"] / v["launches"], 2),
                      "GB/s": round(v["bytes"] / v["ms"] / 1e6, 1) if v["ms"] > 0 else None,
                      "TFLOP/s": round(v["flops"] / v["ms"] / 1e9, 2) if v["ms"] > 0 and v["flops"] else None}

    out_extra = {}
    if graph_fig is not None:
        out_extra["captured_cycles"] = graph_fig
    if tune is not None:
        out_extra["autotune"] = tune
    del x
    # ---- all-FP64 comparison solve
    if not args.skip_fp64:
        p64 = P.SolverParams(m=params.m, k=params.k, tol=params.tol, restart_t=params.restart_t,
                             max_iter=params.max_iter, flags=params.flags,
                             sap=dataclasses.replace(params.sap, storage=P.DW_PREC_F64))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        ts = time.perf_counter()
        _, s64 = f.solve(m0, p64, bt)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - ts
        log(f"[bench] FP64 solve: {summary(s64)}, {t64:.3f} s")
        out_extra.update({"fp64_solves_per_s": round(nrhs / t64, 4),
                          "fp64_iterations": max(s.iterations for s in s64),
                          "speedup_vs_fp64": round(value * t64 / nrhs, 3)})
    # ---- the same solve with the Krylov basis stored in FP32 (the paper's
    # single-precision Arnoldi storage, FP64 arithmetic and explicit FP64
    # residual at restarts); reported beside the FP64-basis value
    if not args.skip_v32 and not (params.flags & (P.SOLVE_V32 | P.SOLVE_A32)):
        # FP32 storage of the basis V (FP64 arithmetic), and the single-precision
        # Arnoldi of Section 4.7 (FP32 V, Z, w = D z and Gram-Schmidt, explicit
        # FP64 residual injected at restarts): the same tolerance on the true
        # FP64 residual
        for key, extra, label in (("fp32_basis", P.SOLVE_V32, "FP32-basis"),
                                  ("fp32_arnoldi", P.SOLVE_A32 | P.SOLVE_INJECT, "single-precision Arnoldi")):
            p32 = P.SolverParams(m=params.m, k=params.k, tol=params.tol, restart_t=params.restart_t,
                                 max_iter=params.max_iter, flags=params.flags | extra, sap=params.sap,
                                 shared_defl=params.shared_defl)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            f.solve(m0, p32, bt)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, s32 = f.solve(m0, p32, bt)
            torch.cuda.synchronize()
            t32 = time.perf_counter() - ts
            log(f"[bench] {label} solve: {summary(s32)}, {t32:.3f} s")
            out_extra[key] = {"solves_per_s": round(nrhs / t32, 4),
                              "iterations": max(s.iterations for s in s32),
                              "cycles": max(s.cycles for s in s32),
                              "clean_restarts": max(s.clean_restarts for s in s32),
                              "true_relres": max(s.true_relres for s in s32)}
    # ---- the same solve with each SAP storage precision
    if args.all_precisions:
        sp = {}
        for name in ("f16", "bf16", "f32", "f64"):
            pp = P.SolverParams(m=params.m, k=params.k, tol=params.tol, restart_t=params.restart_t,
                                max_iter=params.max_iter, flags=params.flags,
                                sap=dataclasses.replace(params.sap, storage=P.PREC_NAMES[name]))
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            f.solve(m0, pp, bt)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, sx = f.solve(m0, pp, bt)
            torch.cuda.synchronize()
            tx = time.perf_counter() - ts
            log(f"[bench] SAP {name}: {summary(sx)}, {tx:.3f} s")
            sp[name] = {"solves_per_s": round(nrhs / tx, 4), "iterations": max(s.iterations for s in sx),
                        "true_relres": max(s.true_relres for s in sx)}
        out_extra["sap_precisions"] = sp
    # ---- FGMRES(m): the same solve without deflation
    if args.also_k0:
        pk0 = P.SolverParams(m=params.m, k=0, tol=params.tol, restart_t=params.restart_t,
                             max_iter=max(4 * st0.iterations, 2000), sap=params.sap)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        ts = time.perf_counter()
        _, sk0 = f.solve(m0, pk0, bt, raise_on_notconv=False)
        torch.cuda.synchronize()
        tk0 = time.perf_counter() - ts
        log(f"[bench] FGMRES({params.m}) solve: {summary(sk0)}, {tk0:.3f} s")
        out_extra["fgmres_k0"] = {"iterations": max(s.iterations for s in sk0),
                                  "converged": all(s.converged for s in sk0),
                                  "relres": max(s.true_relres for s in sk0), "seconds": round(tk0, 3),
                                  "max_iter": pk0.max_iter}
    # ---- the RHS one after another (multi-RHS workloads)
    if args.sequential and nrhs > 1:
        torch.cuda.synchronize()
        ts = time.perf_counter()
        its = []
        for j in range(nrhs):
            _, sj = f.solve(m0, params, bt[j:j + 1].contiguous())
            its.append(sj[0].iterations)
        torch.cuda.synchronize()
        tseq = time.perf_counter() - ts
        log(f"[bench] {nrhs} sequential solves: {tseq:.3f} s")
        out_extra["sequential"] = {"rhs_solves_per_s": round(nrhs / tseq, 4), "iterations": its,
                                   "lockstep_speedup": round(value * tseq / nrhs, 3)}
    if nrhs > 1:
        out_extra["iterations_per_rhs"] = [s.iterations for s in stl]

    # ---- Wilson-Dirac operator alone, each storage precision
    if not args.skip_dslash:
        ds = {}
        for name in ("f64", "f32", "f16", "bf16"):
            ms, gbs = time_dslash(P, torch, f, m0, P.PREC_NAMES[name])
            ds[name] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 3)}
            log(f"[bench] D at {name}: {ms:.4f} ms, {gbs:.0f} GB/s")
        if nrhs > 1:
            # one launch for all right-hand sides (RHS fastest in the launch
            # order, so the workgroups that read a block's links run together
            # and the links are read from memory once): the storage precision
            # of the SAP and the FP64 of the outer operator
            for name in dict.fromkeys((wl["storage"], "f64")):
                pr = P.PREC_NAMES[name]
                ms, gbs = time_dslash(P, torch, f, m0, pr, nrhs=nrhs, reps=20)
                ds[f"{name}_x{nrhs}"] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 3),
                                         "bytes_per_site": (36 + 24 * nrhs) * P.PAIR_BYTES[pr],
                                         "ms_per_rhs": round(ms / nrhs, 4),
                                         "per_rhs_speedup_vs_1": round(ds[name]["ms"] * nrhs / ms, 3)}
                log(f"[bench] D at {name} x {nrhs} RHS: {ms:.4f} ms ({ms / nrhs:.4f} per RHS), {gbs:.0f} GB/s")
        out_extra["dslash"] = ds
        out_extra["copy_GB/s"] = round(copy_bandwidth(torch), 1)

    f.close()
    del bt
    torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu and not csw:  # the oracle sample times the plain Wilson operator
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(L, wl["eps"], wl["seed"], m0, wl, st0.iterations, st0.cycles)
        if nrhs > 1:
            cpu["unit"] = "RHS solves/s"  # the oracle solves the RHS one after another

    lat_ms = sorted(1000 * t for t in lat)
    line = {
        "metric": "solves/s to 1e-10 true residual, mixed-precision SAP+FGMRES-DR (Dslash HBM GB/s and "
                  "all-FP64 GPU solver alongside)",
        "value": round(value, 4),
        "unit": "solves/s" if nrhs == 1 else "RHS solves/s",
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
                               + (f"clover c_sw={csw}, " if csw else "") + "near-critical, "
                               + (f"{nrhs} point-source+noise RHS in lock-step, " if wl.get("rhs") == "point"
                                  else f"{nrhs} Gaussian RHS, ")
                               + describe(params, P) + (" (autotuned)" if tune is not None else ""),
                   "lattice": list(L), "m0": m0, "m0_from": mass_src, "sap_storage": wl["storage"], "nrhs": nrhs,
                   "csw": csw,
                   "parallelism": "single GPU"},
        "iterations": st0.iterations,
        "cycles": st0.cycles,
        "clean_restarts": st0.clean_restarts,
        "true_relres": st0.true_relres,
        "true_relres_oracle": relres_oracle,
        "ms_per_step_without_event_timing": round(unprofiled_ms, 2),
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
