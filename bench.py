"""Benchmark of the MI355X linearized Poisson-Boltzmann grid solve.

Default workload: the serving stream -- 512 synthetic molecules (200-20,000 atoms,
log-uniform), grids 65^3-257^3 at h in {0.5, 0.75, 1.0} A, all in the mixed form (FP32 CG,
FP64 reliable updates and energies).  One step = the whole stream through the
continuous-batching server with every request present at t=0 (closed loop); value = solves/s
of that step.  Also reported: p50/p99 latency of the same stream with Poisson arrivals at
0.8x that rate (open loop), the same 512 requests solved one at a time in plain FP64
(throughput, and latency under the same arrivals), the energy error of every served result,
PCG Gnode-iter/s of the 385^3 single solve in FP64 and mixed form, the roofline of the
dominant kernel, and the CPU oracle on a bounded sample.

Other workloads (--workload c1|c2|c4) time single solves (build + solve + energy).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import replace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2502_09323_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "PBE solves/s + p99 latency at 1e-6 energy err; PCG Gnode-iter/s vs FP64 plain"

# Residual tolerance that keeps |dE/E| <= 1e-6 (both forms use it, so they are compared at
# equal energy error), and the reliable-update factor of the mixed form.
RTOL = 1e-8
# algorithmic bytes per unknown of one FP32 CG iteration kernel: read z, w, p, x and the
# node code, write z, w, p and x (4 bytes each)
ITER_BYTES_FP32 = 36

# HBM traffic per launch relative to the algorithmic bytes, from rocprofv3 FETCH_SIZE (x2.0)
# and WRITE_SIZE (x1.0) passes (the copy kernel's own counters give the factors), with the
# fingerprint of the kernel sources they were taken on; a kernel changed since then reports
# null.  The summaries with the commands are in profiles/.
COUNTER_TRAFFIC = {
    # the 385^3 single solve (multigrid_385_counters)
    "kb_rb_apply<float>@385": {"sources": "mg", "fingerprint": "39febc3c1145bdbc", "ratio": 1.325},
    "kb_rb_sweep<float>@385": {"sources": "mg", "fingerprint": "39febc3c1145bdbc", "ratio": 1.185},
    "k_cg_iter<float>@385": {"sources": "solve", "fingerprint": "1245bd79cc9547d8", "ratio": 1.148},
    # the serving stream's batched launches (serving_stream_512_counters); the sampled
    # half-sweeps are a subset of the launches the counters see, so no ratio for them
    "kb_rb_apply<float>@stream": {"sources": "mg", "fingerprint": "39febc3c1145bdbc", "ratio": 1.353},
    "kb_rb_sweep<float>@stream": {"sources": "mg", "fingerprint": None, "ratio": None},
}


def kernel_fingerprint(which):
    """sha256 (first 16 hex digits) of a kernel family's sources: "solve" = the Jacobi iteration
    kernel (pb_solve.hip and pb_stencil.h), "mg" = the multigrid kernels (pb_mg.hip and
    pb_stencil.h); with the shared types of pb_internal.h (the text before its kernel
    declarations)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2502_09323_amd", "csrc")
    for f in ({"solve": "pb_solve.hip", "mg": "pb_mg.hip"}[which], "pb_stencil.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "pb_internal.h"), "rb") as fh:
        b = fh.read()
    h.update(b[:b.index(b"// ---- build kernels (pb_build.hip)")])
    return h.hexdigest()[:16]


def counter_traffic(key, bytes_per_launch):
    t = COUNTER_TRAFFIC.get(key)
    if not t or not t["ratio"] or t["fingerprint"] != kernel_fingerprint(t["sources"]):
        return None
    return round(t["ratio"] * bytes_per_launch)
DELTA = 1e-2
DELTA_MG = 1e-4   # reliable-update factor of the multigrid-preconditioned mixed solve
MG_MIN_N = 65     # serving: grids from this many nodes per axis use the multigrid preconditioner (all of
                  # the stream's; batched, the multigrid requests share every launch)
BIND_COMPLEXES, BIND_DISP, BIND_H = 6, 30, 0.5   # binding workload: complexes, displacements, spacing
N_REQ = 512
SEED = 2505
MAX_RESIDENT = 64
OPEN_LOOP_LOAD = 0.8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def relerr(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def pct(x, q):
    return float(np.percentile(np.asarray(x), q))


# ---- serving stream ---------------------------------------------------------------------------

def stream(n, precond="auto", mg_min_n=None):
    """The serving stream; with precond "auto" the requests on grids of at least MG_MIN_N nodes
    per axis take the multigrid preconditioner (Jacobi-CG needs hundreds of iterations there),
    the smaller ones Jacobi-CG in the batched launches."""
    reqs = I.serving_stream_c5(n_req=n, seed=SEED, rate_hz=1.0, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA)
    unit_arrivals = np.array([r[0] for r in reqs])  # Poisson process at 1 request/s
    mg_min_n = MG_MIN_N if mg_min_n is None else mg_min_n
    out = []
    for _, m, g in reqs:
        if precond == "mg" or (precond == "auto" and min(g.n) >= mg_min_n):
            g = replace(g, precond=I.MG, inner_rtol=DELTA_MG)
        out.append((m, g))
    return out, unit_arrivals


def serve(B, main, side, reqs, arrivals=None, max_resident=MAX_RESIDENT, progress=0):
    """Run requests through a fresh server; returns (results by id, wall seconds, server).
    With progress > 0 a line is logged each time that many more requests have completed."""
    srv = B.Server(main, side, max_resident=max_resident)
    t0 = srv.now()
    for i, (mol, g) in enumerate(reqs):
        srv.submit(mol, g, i, t0 if arrivals is None else t0 + float(arrivals[i]))
    out = {}
    while len(out) < len(reqs):
        srv.step()
        for r in srv.poll():
            r["latency_s"] = r["done_s"] - (t0 if arrivals is None else t0 + float(arrivals[r["id"]]))
            out[r["id"]] = r
            if progress and len(out) % progress == 0:
                log(f"{len(out)} of {len(reqs)} requests served")
    wall = srv.now() - t0
    return out, wall, srv


class NbodyTimes:
    """The energy N-body kernel of every read-back of a run, timed with HIP events (profiling
    on in every context): standalone solves report theirs, servers their totals."""

    def __init__(self):
        self.ms = 0.0
        self.pairs = 0.0
        self.calls = 0

    def add_solve(self, r):
        if r.get("nbody_pairs", 0) > 0:
            self.ms += r["nbody_ms"]
            self.pairs += r["nbody_pairs"]
            self.calls += 1

    def add_server(self, p):
        self.ms += p["nbody_ms"]
        self.pairs += p["nbody_pairs"]
        self.calls += p["nbody_calls"]

    def roofline(self, scope):
        if self.calls == 0 or self.ms <= 0:
            return None
        tf = self.pairs * NBODY_FLOPS_PER_PAIR / (self.ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP64_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": "k_nbody (energy read-back: atoms x cut points, FP64)",
                "flops_per_launch": round(self.pairs * NBODY_FLOPS_PER_PAIR / self.calls),
                "flops_per_pair": NBODY_FLOPS_PER_PAIR, "avg_launch_ms": round(self.ms / self.calls, 4),
                "launches_timed": self.calls, "total_ms": round(self.ms, 1), "scope": scope}


def fifo_latency(arrivals, service):
    """Latency of a single FIFO server with the given arrivals and service times."""
    free = 0.0
    lat = []
    for a, s in zip(arrivals, service):
        start = max(a, free)
        free = start + s
        lat.append(free - a)
    return np.array(lat)


SERVE_BUDGET = 96 << 30   # HBM budget of the serving loop (a third of the device)
ERR_BAR = 1e-6            # relative energy error every served result must meet


def rf_hbm(kernel, ms_total, bytes_total, launches, scope, traffic_key=None):
    """An HBM roofline record from timed launches and their algorithmic bytes."""
    if not launches or ms_total <= 0:
        return None
    ach = bytes_total / (ms_total * 1e-3) / 1e9
    bpl = bytes_total / launches
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(traffic_key, bpl) if traffic_key else None,
            "kernel": kernel, "bytes_per_launch": round(bpl), "avg_launch_ms": round(ms_total / launches, 5),
            "launches_timed": launches, "total_ms": round(ms_total, 1), "scope": scope}


def bench_serving(args, B, torch):
    main = B.Context(0, hbm_budget_bytes=SERVE_BUDGET)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    reqs, unit_arr = stream(N_REQ, args.serve_precond, args.mg_min_n)
    nu = np.array([g.unknowns for _, g in reqs], dtype=np.float64)
    n_mg = sum(1 for _, g in reqs if g.precond == I.MG)
    log(f"generated {N_REQ} requests")

    # Every batched launch of the run (warm-up, closed and open loop) is timed with HIP events
    # on the serving streams, so that the averages agree with a kernel trace of the command.
    main.set_profiling(True)
    side.set_profiling(True)
    prof = dict(stencil_ms=0.0, stencil_bytes=0.0, launches=0, mg_sweep_ms=0.0, mg_sweep_bytes=0.0,
                mg_vcycle_ms=0.0, mg_samples=0, mg_apply_ms=0.0, mg_apply_bytes=0.0, mg_apply_launches=0)
    nbt = NbodyTimes()
    mem_peak = [0]

    def close(srv):
        p = srv.profile()
        for k in prof:
            prof[k] += p[k]
        nbt.add_server(p)
        mem_peak[0] = max(mem_peak[0], srv.memory()["peak"])
        srv.close()

    # warmup: the first requests through a server (untimed)
    for _ in range(args.warmup):
        close(serve(B, main, side, reqs[:32], max_resident=args.max_resident)[2])
        log("warm-up done")

    # timed: the whole stream, closed loop
    walls, res = [], None
    for _ in range(args.steps):
        torch.cuda.synchronize()
        res, wall, srv = serve(B, main, side, reqs, max_resident=args.max_resident,
                               progress=64 if args.counters_run else 0)
        torch.cuda.synchronize()
        close(srv)
        walls.append(wall)
    value = N_REQ / float(np.mean(walls))
    codes = sorted({r["code"] for r in res.values()})
    log(f"closed loop: {value:.2f} solves/s")
    if args.counters_run:
        # the launches of a hardware-counter pass (which serializes them): the algorithmic
        # bytes of the batched solver launches beside the counters
        main.set_profiling(False)
        side.set_profiling(False)
        scope = "every batched launch of the run (warm-up and closed loop)"
        out = {"metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "counters_run": True,
               "roofline_solver_kernels": [
                   rf_hbm("kb_rb_apply<float>", prof["mg_apply_ms"], prof["mg_apply_bytes"], prof["mg_apply_launches"],
                          scope),
                   rf_hbm("kb_rb_sweep<float>", prof["mg_sweep_ms"], prof["mg_sweep_bytes"], prof["mg_samples"],
                          "the first black half-sweep of every batched iteration (warm-up and closed loop)")],
               # the copy kernel that scales the counters (1 GiB read and written per launch)
               "stream_copy_GBs": round(main.stream_copy_gbps(1 << 30, 4), 1)}
        main.close()
        side.close()
        return out

    # open loop: Poisson arrivals at OPEN_LOOP_LOAD x the closed-loop rate
    rate = OPEN_LOOP_LOAD * value
    arr = unit_arr / rate
    res_open, wall_open, srv = serve(B, main, side, reqs, arr, max_resident=args.max_resident)
    close(srv)
    lat_open = [res_open[i]["latency_s"] for i in range(N_REQ)]
    log(f"open loop at {rate:.2f}/s done")
    # the same at half and at the full closed-loop rate
    sweep = {}
    for load in (0.5, 1.0):
        r_s, w_s, srv = serve(B, main, side, reqs, unit_arr / (load * value), max_resident=args.max_resident)
        close(srv)
        l_s = [r_s[i]["latency_s"] for i in range(N_REQ)]
        sweep[f"{load:.1f}x"] = {"arrival_rate_hz": round(load * value, 3), "solves_per_s": round(N_REQ / w_s, 3),
                                 "p50_ms": round(1e3 * pct(l_s, 50), 1), "p99_ms": round(1e3 * pct(l_s, 99), 1)}
    log("open-loop sweep done")

    # baselines, one request at a time in plain FP64 at the same tolerance (the same energy
    # error): with Jacobi-CG, and with the served stream's own preconditioner policy
    def one_at_a_time(precond=None):
        svc, out = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for mol, g in reqs:
            t = time.perf_counter()
            r = B.solve(mol, replace(g, precision=I.FP64, precond=g.precond if precond is None else precond), main)
            svc.append(time.perf_counter() - t)
            out.append(r)
            nbt.add_solve(r)
        return time.perf_counter() - t0, svc, out

    t_fp64, svc, e64 = one_at_a_time(I.JACOBI)
    log(f"fp64 Jacobi one at a time: {N_REQ / t_fp64:.2f} solves/s")
    t_fp64p, svc_p, _ = one_at_a_time()
    log(f"fp64 same preconditioners one at a time: {N_REQ / t_fp64p:.2f} solves/s")
    lat64 = fifo_latency(arr, svc)
    lat64p = fifo_latency(arr, svc_p)
    err_mix_vs_64 = max(max(relerr(res[i][k], e64[i][k]) for k in ("e_pol", "e_ion")) for i in range(N_REQ))

    # every served result against a tight FP64 solve of the same request (multigrid, rtol
    # 1e-12), and against the stored oracle values of 16 requests of the stream
    err_tight = []
    for i, (mol, g) in enumerate(reqs):
        ref = B.solve(mol, replace(g, precision=I.FP64, rtol=1e-12, precond=I.MG), main)
        err_tight.append(max(relerr(res[i][k], ref[k]) for k in ("e_pol", "e_ion")))
    err_tight = np.array(err_tight)
    with open(os.path.join(ROOT, "tests", "golden", "c5_sample_oracle.json")) as fh:
        gold = json.load(fh)
    gold_reqs = [r for r in gold["requests"] if r["request"] < N_REQ]
    err_oracle = max((relerr(res[r["request"]][k], r["energy"][k]) for r in gold_reqs for k in ("e_pol", "e_ion",
                                                                                               "e_coul")),
                     default=None)
    log("energy errors done")

    # the 385^3 single solve: PCG node-iterations per second in FP64 and mixed (Jacobi-CG)
    mol4, g4 = I.large_c4()
    c4 = {}
    for name, prec in (("mixed", I.MIXED), ("fp64", I.FP64)):
        g = replace(g4, precision=prec, rtol=RTOL, inner_rtol=DELTA)
        nbt.add_solve(B.solve(mol4, g, main))  # warm
        r = B.solve(mol4, g, main)
        nbt.add_solve(r)
        c4[name] = dict(gnode_iter_per_s=round(g4.unknowns * r["iters"] / r["t_solve_s"] / 1e9, 3),
                        iters=r["iters"], t_solve_ms=round(1e3 * r["t_solve_s"], 2))
    log("precision comparison done")
    main.set_profiling(False)
    side.set_profiling(False)

    # Rooflines.  Every served launch of the batched multigrid operator pass is timed; the
    # level-0 black half-sweep once per batched iteration (and per chunk of a request run alone);
    # the batched Jacobi iteration kernel (requests below the multigrid threshold) on every
    # launch; the energy N-body sum on every read-back of the run.  The kernel with the most
    # timed GPU time is `roofline`, the others follow.
    scope = "every batched launch of the run (warm-up, closed and open loop)"
    rf_apply = rf_hbm("kb_rb_apply<float> (batched multigrid CG operator pass, level 0, red-black layout)",
                      prof["mg_apply_ms"], prof["mg_apply_bytes"], prof["mg_apply_launches"], scope,
                      "kb_rb_apply<float>@stream")
    rf_sweep = rf_hbm("kb_rb_sweep<float> (batched level-0 black half-sweep of the V-cycle, red-black layout)",
                      prof["mg_sweep_ms"], prof["mg_sweep_bytes"], prof["mg_samples"],
                      "the first black half-sweep of every batched iteration (warm-up, closed and open loop)",
                      "kb_rb_sweep<float>@stream")
    if rf_sweep is not None:
        rf_sweep["avg_vcycle_ms"] = round(prof["mg_vcycle_ms"] / prof["mg_samples"], 5)
    rf_jacobi = rf_hbm("kb_iter<float> (batched FP32 Jacobi-CG iteration)", prof["stencil_ms"],
                       prof["stencil_bytes"], prof["launches"], scope)
    rf_nb = nbt.roofline("every energy read-back of the run (served, FP64 baselines, 385^3 comparison)")
    ranked = sorted([r for r in (rf_nb, rf_apply, rf_sweep, rf_jacobi) if r is not None],
                    key=lambda r: -r["total_ms"])
    roofline, others = ranked[0], ranked[1:]

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_stream(reqs)

    lat_closed = [r["latency_s"] for r in res.values()]
    n_bad = int((err_tight > ERR_BAR).sum()) + int(err_oracle is not None and err_oracle > ERR_BAR)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * float(np.mean(walls)), 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 CG + f64 reliable updates/energy",
        "data": "synthetic",
        "config": {"workload": f"serving stream: {N_REQ} synthetic molecules (200-20000 atoms, log-uniform), "
                               f"grids 65^3-257^3, h in {{0.5,0.75,1.0}} A, mixed precision",
                   "n_requests": N_REQ, "seed": SEED, "rtol": RTOL,
                   "reliable_update_factor": {"jacobi": DELTA, "multigrid": DELTA_MG},
                   "preconditioner": {"auto": f"multigrid V-cycle on grids >= {args.mg_min_n}^3, Jacobi below",
                                      "mg": "multigrid V-cycle", "jacobi": "Jacobi"}[args.serve_precond],
                   "multigrid_requests": n_mg, "max_resident": args.max_resident,
                   "hbm_budget_bytes": SERVE_BUDGET, "unknowns_total": float(nu.sum()),
                   "atoms_total": int(sum(m.n for m, _ in reqs))},
        "served_closed_loop": {"solves_per_s": round(value, 3), "p50_s": round(pct(lat_closed, 50), 3),
                               "p99_s": round(pct(lat_closed, 99), 3), "codes": codes,
                               "hbm_accounted_peak_bytes": mem_peak[0]},
        "served_open_loop": {"arrival_rate_hz": round(rate, 3), "solves_per_s": round(N_REQ / wall_open, 3),
                             "p50_ms": round(1e3 * pct(lat_open, 50), 1), "p99_ms": round(1e3 * pct(lat_open, 99), 1)},
        "served_open_loop_sweep": {"0.5x": sweep["0.5x"], "0.8x": {"arrival_rate_hz": round(rate, 3),
                                                                  "solves_per_s": round(N_REQ / wall_open, 3),
                                                                  "p50_ms": round(1e3 * pct(lat_open, 50), 1),
                                                                  "p99_ms": round(1e3 * pct(lat_open, 99), 1)},
                                   "1.0x": sweep["1.0x"]},
        "fp64_one_at_a_time": {"solves_per_s": round(N_REQ / t_fp64, 3), "preconditioner": "Jacobi",
                               "mean_service_ms": round(1e3 * float(np.mean(svc)), 2),
                               "p50_ms_same_arrivals": round(1e3 * pct(lat64, 50), 1),
                               "p99_ms_same_arrivals": round(1e3 * pct(lat64, 99), 1)},
        "fp64_one_at_a_time_same_preconditioners": {
            "solves_per_s": round(N_REQ / t_fp64p, 3), "preconditioner": "as served (multigrid)",
            "mean_service_ms": round(1e3 * float(np.mean(svc_p)), 2),
            "p50_ms_same_arrivals": round(1e3 * pct(lat64p, 50), 1),
            "p99_ms_same_arrivals": round(1e3 * pct(lat64p, 99), 1)},
        "speedup_vs_fp64_one_at_a_time": round(value / (N_REQ / t_fp64), 3),
        "speedup_decomposed": {
            "preconditioner (fp64 multigrid vs fp64 Jacobi, one at a time)": round(t_fp64 / t_fp64p, 3),
            "mixed precision and batching (served vs fp64 multigrid one at a time)": round(value / (N_REQ / t_fp64p), 3)},
        "energy_relerr": {"bar": ERR_BAR, "requests_over_bar": n_bad,
                          "served_vs_fp64_rtol1e-12_all_max": float(err_tight.max()),
                          "served_vs_fp64_rtol1e-12_all_p50": float(np.median(err_tight)),
                          "served_vs_fp64_same_rtol_max": err_mix_vs_64,
                          "vs_oracle": {"max": err_oracle, "requests": len(gold_reqs),
                                        "reference": "stored FP64 CPU-oracle energies (rtol 1e-12) of requests "
                                                     + ",".join(str(r["request"]) for r in gold_reqs)}},
        "pcg_gnode_iter_per_s": {"workload": "385^3 single solve (60000 atoms, h=0.5 A), Jacobi-CG",
                                 "mixed": c4["mixed"], "fp64": c4["fp64"]},
        "roofline": roofline,
        "roofline_solver_kernels": [r for r in others if r["bound"] == "hbm"],
        "roofline_other": [r for r in others if r["bound"] != "hbm"],
        "stream_copy_GBs": round(main.stream_copy_gbps(1 << 30, 20), 1),
        "cpu_baseline": cpu,
    }
    main.close()
    side.close()
    return out


def host_cpu():
    """The host's CPU model and logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def oracle_single_thread(mol, g, timeout_s=90.0):
    """Seconds the oracle takes for one request in a child process with one OpenMP thread."""
    import subprocess
    import tempfile

    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "req.npz")
        np.savez(path, xyz=mol.xyz, radius=mol.radius, charge=mol.charge, n=np.array(g.n), h=g.h,
                 origin=np.array(g.origin), temp=g.temp_K, ionic=g.ionic_M, eps_in=g.eps_in, eps_out=g.eps_out,
                 bc=g.bc)
        code = (
            "import sys, time, numpy as np\n"
            f"sys.path.insert(0, {ROOT!r})\n"
            "from paper_2502_09323_amd import inputs as I\n"
            "from oracle import oracle as O\n"
            f"z = np.load({path!r})\n"
            "m = I.Molecule(z['xyz'], z['radius'], z['charge'])\n"
            "g = I.GridSpec(n=tuple(int(v) for v in z['n']), h=float(z['h']), origin=tuple(float(v) for v in z['origin']),"
            " eps_in=float(z['eps_in']), eps_out=float(z['eps_out']), ionic_M=float(z['ionic']),"
            " temp_K=float(z['temp']), bc=int(z['bc']))\n"
            "t = time.perf_counter()\n"
            f"O.run(m, g, rtol={RTOL})\n"
            "print(time.perf_counter() - t, O.num_threads())\n")
        env = dict(os.environ, OMP_NUM_THREADS="1")
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout_s)
        dt, nt = out.stdout.split()[-2:]
        return float(dt), int(nt)


def cpu_baseline_stream(reqs, budget_s=15.0):
    """The oracle (FP64, all host threads) on the first requests of the same stream, and on the
    smallest of them with one thread."""
    from oracle import oracle as O

    t0 = time.perf_counter()
    n = 0
    for mol, g in reqs:
        O.run(mol, replace(g, precision=I.FP64), rtol=RTOL)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": round(n / dt, 4), "unit": "solves/s", "cores": O.num_threads(), "kind": "oracle",
           "sample": f"the first {n} requests of the same stream solved by the FP64 CPU oracle at rtol {RTOL} "
                     f"({dt:.1f} s)", "host": host_cpu()}
    k = min(range(n), key=lambda i: reqs[i][1].unknowns)
    try:
        t1, nt = oracle_single_thread(reqs[k][0], reqs[k][1])
        out["single_thread"] = {"seconds": round(t1, 2), "threads": nt,
                                "sample": f"request {k} of the stream ({reqs[k][1].n[0]}^3 nodes, {reqs[k][0].n} atoms)"}
    except Exception as e:   # the single-thread figure is context only
        out["single_thread"] = {"error": str(e)[:200]}
    return out


# ---- single solves (c1, c2, c4) ---------------------------------------------------------------

def workload(name: str):
    if name == "c1":
        return I.kirkwood_c1() + ("kirkwood sphere R=2A q=+1e, 65^3 nodes, h=0.25A",)
    if name == "c2":
        return I.protein_c2() + ("synthetic 2000-atom molecule in a 20A ball, 161^3 nodes, h=0.5A",)
    if name == "c4":
        return I.large_c4() + ("synthetic 60000-atom molecule in a 65A ball, 385^3 nodes, h=0.5A",)
    if name == "c3":
        return I.refined_c3() + ("synthetic 20000-atom molecule in a 45A ball, 193^3 coarse nodes at h=1.0A, "
                                 "refined to 0.5A within 3A of the surface (4^3-cell bricks)",)
    raise SystemExit(f"unknown workload {name}")


# algorithmic bytes per grid node (coarse and fine arrays, FP64) of one composite CG iteration
# on a refined problem: apply (K x3 and the lumped term, role, p; q), dot (role, p, q),
# update (role, x, r rw; p, q, D^-1; z), direction (role, z, p rw)
# FP64 flops per atom x cut-point pair of the energy N-body sum (a fused multiply-add counts
# two), in the direct form: the three differences, the squared distance (5), the Newton step
# on the hardware reciprocal square root estimate (6; the estimate itself is not counted),
# the dot product with the weighted normal (5), F/r into its sum (2) and the r^-3 term (4).
# The kernel's expanded form (squared distance and dot product from per-point and per-atom
# terms) performs the same 25 in 15 instructions instead of 17.
NBODY_FLOPS_PER_PAIR = 25
FP64_PEAK_TFLOPS = 78.6
# algorithmic bytes per interior unknown of one level-0 red-black half-sweep of the V-cycle
# (FP32, red-black layout): read x of the other colour, b, 1/D and the node codes of the swept
# colour, write x of the swept colour (20 B per node of the swept colour; the codes of the
# other colour are read only by waves with a cut edge)
MG_SWEEP_BYTES_FP32 = (4 + 4 + 4 + 4 + 4) / 2
REFINED_ITER_BYTES = 49 + 17 + 65 + 25
# ... and with FP32 coefficients and vectors (mixed precision)
REFINED_ITER_BYTES_FP32 = 25 + 9 + 33 + 13


def bench_refined(args, B, torch):
    ctx = B.Context(0)
    mol, grid, desc = workload("c3")
    ref = None

    def run(g):
        nonlocal ref
        lat, res = [], []
        for s in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb = B.Problem(ctx, mol, g)
            t1 = time.perf_counter()
            st = pb.solve()
            en = pb.energy()
            info = pb.refine_info()
            pb.close()
            torch.cuda.synchronize()
            if s >= args.warmup:
                lat.append(time.perf_counter() - t0)
                res.append((st, en, info, t1 - t0))
        st, en, info, t_build = res[-1]
        if ref is None:
            ref = en
        t_solve = float(np.mean([r[0]["t_solve_s"] for r in res]))
        iters = float(np.mean([r[0]["iters"] for r in res]))
        return dict(lat=lat, st=st, en=en, info=info, t_build=t_build, t_solve=t_solve, iters=iters,
                    err=max(relerr(en[k], ref[k]) for k in ("e_pol", "e_ion")))

    p64 = run(replace(grid, rtol=RTOL, precision=I.FP64))
    mx = run(replace(grid, rtol=RTOL, precision=I.MIXED, inner_rtol=DELTA))
    tl = run(replace(grid, rtol=RTOL, precision=I.FP64, precond=I.MG))
    tlm = run(replace(grid, rtol=RTOL, precision=I.MIXED, inner_rtol=DELTA_MG, precond=I.MG))
    info = mx["info"]
    nunk = info["unknowns_coarse"] + info["unknowns_fine"]
    nc = np.prod([int(v) for v in grid.n])
    nf = np.prod(info["fine_n"])
    nodes = float(nc + nf)
    t_iter = mx["t_solve"] / max(mx["iters"], 1.0)
    ach = nodes * REFINED_ITER_BYTES_FP32 / t_iter / 1e9
    # value: the mixed solve with the two-level preconditioner (the fastest form); the
    # Jacobi-preconditioned mixed solve beside it, whose iteration gives the roofline
    lat = tlm["lat"]
    out = {
        "metric": METRIC, "value": round(len(lat) / sum(lat), 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * float(np.mean(lat)), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 CG + f64 reliable updates/energy", "data": "synthetic",
        "config": {"workload": desc, "n_atoms": mol.n, "rtol": RTOL, "reliable_update_factor": DELTA_MG,
                   "preconditioner": "damped Jacobi + coarse-grid multigrid V-cycle (symmetric two-level)",
                   "unknowns": int(nunk), "refined_cells": int(info["refined_cells"]),
                   "hanging_nodes": int(info["hanging_nodes"]), "fine_lattice": list(info["fine_n"])},
        "iters": tlm["iters"], "reliable_updates": tlm["st"]["outer_iters"],
        "t_solve_ms": round(1e3 * tlm["t_solve"], 2), "t_build_ms": round(1e3 * tlm["t_build"], 2),
        "energy_relerr_vs_fp64": tlm["err"],
        "jacobi_mixed": {"solves_per_s": round(len(mx["lat"]) / sum(mx["lat"]), 4), "iters": mx["iters"],
                         "reliable_updates": mx["st"]["outer_iters"], "reliable_update_factor": DELTA,
                         "t_solve_ms": round(1e3 * mx["t_solve"], 2), "energy_relerr_vs_fp64": mx["err"]},
        "pcg_gnode_iter_per_s": {"mixed": round(nunk * mx["iters"] / mx["t_solve"] / 1e9, 3),
                                 "fp64": round(nunk * p64["iters"] / p64["t_solve"] / 1e9, 3)},
        "fp64_plain": {"solves_per_s": round(len(p64["lat"]) / sum(p64["lat"]), 4), "iters": p64["iters"],
                       "t_solve_ms": round(1e3 * p64["t_solve"], 2),
                       "iteration_GBs": round(nodes * REFINED_ITER_BYTES * p64["iters"] / p64["t_solve"] / 1e9, 1)},
        "fp64_two_level": {"solves_per_s": round(len(tl["lat"]) / sum(tl["lat"]), 4), "iters": tl["iters"],
                           "t_solve_ms": round(1e3 * tl["t_solve"], 2), "energy_relerr_vs_fp64": tl["err"],
                           "preconditioner": "damped Jacobi + coarse-grid multigrid V-cycle (symmetric two-level)"},
        "energies_kT": {k: tlm["en"][k] for k in ("e_pol", "e_ion", "e_coul")},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "composite CG iteration in FP32 of the Jacobi-preconditioned mixed solve (all "
                               "kernels of one iteration, reliable updates included)",
                     "bytes_per_launch": round(nodes * REFINED_ITER_BYTES_FP32), "avg_launch_ms": round(1e3 * t_iter, 4)},
        "stream_copy_GBs": round(ctx.stream_copy_gbps(1 << 30, 20), 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import oracle as O
        from oracle import refined as R

        # the oracle's refined path on a reduced molecule and grid of the same recipe
        mol_s = I.random_molecule(1500, 18.0, 2503)
        g_s = I.cubic_grid(65, 1.0, refine=1, refine_shell=3.0, refine_brick=4)
        t0 = time.perf_counter()
        run_o = R.refined_run(mol_s, g_s, delta=3.0, brick=4, rtol=RTOL)
        dt = time.perf_counter() - t0
        rate = run_o.free.size * run_o.iters / run_o.times["solve"] / 1e9
        out["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": O.num_threads(),
                               "kind": "oracle",
                               "gnode_iter_per_s": round(rate, 5),
                               "sample": f"the refined-grid oracle on a reduced case of the same recipe (1500 atoms in "
                                         f"an 18 A ball, 65^3 coarse nodes at 1.0 A, {run_o.free.size} unknowns): "
                                         f"{dt:.1f} s, {run_o.iters} CG iterations"}
    ctx.close()
    return out


def mg_smooth_single(grid) -> int:
    """Red-black sweeps before and after the coarse correction for a single large solve: on
    385^3, V(2,2) takes 13 iterations and 47 ms against 22 and 51 ms for V(1,1) (V(3,3): 10
    iterations, 50 ms).  The serving stream's grids (65^3 ... 257^3, batched only with equal
    smoothing counts) run faster with V(1,1)."""
    return 2 if min(grid.n) > 257 else 1


def bench_single(args, B, torch):
    ctx = B.Context(0)
    mol, grid, desc = workload(args.workload)
    grid = replace(grid, mg_smooth=mg_smooth_single(grid))
    nu = grid.unknowns
    ref = B.solve(mol, replace(grid, rtol=1e-12, precision=I.FP64), ctx)
    log("tight FP64 reference solved")

    def run(g):
        lat, res = [], []
        for s in range(args.warmup + args.steps):
            timed = s >= args.warmup
            ctx.set_profiling(timed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb = B.Problem(ctx, mol, g)
            st = pb.solve()
            en = pb.energy()
            prof = pb.profile() if timed else None
            if timed:
                en.update(pb.energy_profile())
            pb.close()
            torch.cuda.synchronize()
            if timed:
                lat.append(time.perf_counter() - t0)
                res.append((st, en, prof))
        ctx.set_profiling(False)
        st, en, _ = res[-1]
        t_solve = np.mean([r[0]["t_solve_s"] for r in res])
        iters = np.mean([r[0]["iters"] for r in res])
        stencil_ms = float(np.mean([r[2]["stencil_ms"] for r in res if r[2]["samples"]]))
        update_ms = float(np.mean([r[2]["update_ms"] for r in res if r[2]["samples"]]))
        for r in res:
            nbt.add_solve(r[1])
        return dict(solves_per_s=len(lat) / sum(lat), ms=1e3 * float(np.mean(lat)), p50=1e3 * pct(lat, 50),
                    p99=1e3 * pct(lat, 99), iters=float(iters), gnode=nu * iters / t_solve / 1e9,
                    stencil_ms=stencil_ms, update_ms=update_ms, vcycles=float(iters) + st["outer_iters"] + 1,
                    err=max(relerr(en[k], ref[k]) for k in ("e_pol", "e_ion")), en=en)

    nbt = NbodyTimes()

    mg = run(replace(grid, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA_MG, precond=I.MG))
    log("mixed multigrid done")
    mg64 = run(replace(grid, precision=I.FP64, rtol=RTOL, precond=I.MG))
    log("FP64 multigrid done")
    mx = run(replace(grid, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA))
    log("mixed Jacobi done")
    p64 = run(replace(grid, precision=I.FP64, rtol=RTOL))
    log("FP64 Jacobi done")
    # the two-run salt term: grid energies of multigrid mixed solves at the actual and at zero
    # ionic strength, against the same change of the surface read-back's solvation energy
    two_run = None
    if grid.ionic_M > 0:
        two = {}
        for ion in (grid.ionic_M, 0.0):
            pb = B.Problem(ctx, mol, replace(grid, ionic_M=ion, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA_MG,
                                             precond=I.MG))
            pb.solve()
            en = pb.energy()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ge = pb.grid_energy()
            two[ion] = (ge, en["e_pol"] + en["e_ion"], time.perf_counter() - t0)
            pb.close()
        hi, lo = two[grid.ionic_M], two[0.0]
        two_run = {"ionic_M": grid.ionic_M, "grid_energy_two_run_kT": round(hi[0] - lo[0], 6),
                   "surface_solvation_change_kT": round(hi[1] - lo[1], 6),
                   "grid_energy_call_ms": round(1e3 * min(hi[2], lo[2]), 3)}
    ach = nu * MG_SWEEP_BYTES_FP32 / (mg["stencil_ms"] * 1e-3) / 1e9
    ach_j = nu * ITER_BYTES_FP32 / (mx["stencil_ms"] * 1e-3) / 1e9
    nu_tag = f"{grid.n[0]}" if grid.n[0] == grid.n[1] == grid.n[2] else "x".join(map(str, grid.n))
    out = {
        "metric": METRIC, "value": round(mg["solves_per_s"], 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(mg["ms"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 CG + f64 reliable updates/energy", "data": "synthetic",
        "config": {"workload": desc, "unknowns": nu, "n_atoms": mol.n, "rtol": RTOL,
                   "preconditioner": f"multigrid V({grid.mg_smooth},{grid.mg_smooth}) cycle, red-black Gauss-Seidel "
                                     "smoothing",
                   "reliable_update_factor": DELTA_MG},
        "p50_ms": round(mg["p50"], 3), "p99_ms": round(mg["p99"], 3), "energy_relerr_vs_fp64": mg["err"],
        "iters": mg["iters"],
        "pcg_gnode_iter_per_s": {"mixed": round(mx["gnode"], 3), "fp64": round(p64["gnode"], 3)},
        "multigrid_fp64": {"solves_per_s": round(mg64["solves_per_s"], 3), "p50_ms": round(mg64["p50"], 3),
                           "iters": mg64["iters"], "energy_relerr_vs_fp64": mg64["err"]},
        "jacobi_mixed": {"solves_per_s": round(mx["solves_per_s"], 3), "p50_ms": round(mx["p50"], 3),
                         "iters": mx["iters"], "energy_relerr_vs_fp64": mx["err"],
                         "iteration_kernel": {"kernel": "k_cg_iter<float>", "achieved_GBs": round(ach_j, 1),
                                              "avg_launch_ms": round(mx["stencil_ms"], 5),
                                              "traffic": counter_traffic(f"k_cg_iter<float>@{nu_tag}",
                                                                         nu * ITER_BYTES_FP32)}},
        "fp64_plain": {"solves_per_s": round(p64["solves_per_s"], 3), "p50_ms": round(p64["p50"], 3),
                       "p99_ms": round(p64["p99"], 3), "iters": p64["iters"], "energy_relerr_vs_fp64": p64["err"]},
        "two_run_salt": two_run,
        "roofline": None,
        "stream_copy_GBs": round(ctx.stream_copy_gbps(1 << 30, 20), 1),
        "cpu_baseline": None,
    }
    # the dominant kernel of the multigrid solve's step: the level-0 half-sweep (4 nu - 2 per
    # V(nu, nu) cycle besides its first smoothing step) or the energy N-body sum, whichever
    # takes longer per step; the Jacobi iteration kernel of the mixed Jacobi-CG solve beside them
    rf_sweep = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": counter_traffic(f"kb_rb_sweep<float>@{nu_tag}", nu * MG_SWEEP_BYTES_FP32),
                "kernel": "kb_rb_sweep<float> (level-0 black half-sweep of the V-cycle, red-black layout)",
                "bytes_per_launch": nu * MG_SWEEP_BYTES_FP32, "avg_launch_ms": round(mg["stencil_ms"], 5),
                "v_cycle_ms": round(mg["update_ms"], 5), "per_step_ms": round((4 * grid.mg_smooth - 2) * mg["vcycles"] * mg["stencil_ms"], 3)}
    rf_nb = nbt.roofline("every energy read-back of the timed solves (all four configurations)")
    if rf_nb is not None:
        rf_nb["per_step_ms"] = rf_nb["avg_launch_ms"]
    if rf_nb is not None and rf_nb["per_step_ms"] > rf_sweep["per_step_ms"]:
        out["roofline"], out["roofline_other"] = rf_nb, rf_sweep
    else:
        out["roofline"], out["roofline_other"] = rf_sweep, rf_nb
    out["roofline_solver_kernels"] = [
        rf_sweep,
        {"bound": "hbm", "achieved": round(ach_j, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(ach_j / HBM_PEAK_GBS, 4),
         "traffic": counter_traffic(f"k_cg_iter<float>@{nu_tag}", nu * ITER_BYTES_FP32),
         "kernel": "k_cg_iter<float> (whole Jacobi-CG iteration in one pass, mixed form)",
         "bytes_per_launch": nu * ITER_BYTES_FP32, "avg_launch_ms": round(mx["stencil_ms"], 5)}]
    # energy error of every configuration against the oracle: the stored FP64 oracle values of
    # this workload (rtol 1e-12) where they exist, and the oracle solve of the CPU baseline
    gold_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.json")
    vs = {}
    if os.path.exists(gold_path):
        with open(gold_path) as fh:
            gold = json.load(fh)["energy"]
        vs["stored_oracle_rtol1e-12"] = {name: max(relerr(r["en"][k], gold[k]) for k in ("e_pol", "e_ion", "e_coul"))
                                         for name, r in (("multigrid_mixed", mg), ("multigrid_fp64", mg64),
                                                         ("jacobi_mixed", mx), ("jacobi_fp64", p64))}
    if not args.no_cpu:
        from oracle import oracle as O

        t0 = time.perf_counter()
        run_o = O.run(mol, replace(grid, precision=I.FP64), rtol=RTOL)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": O.num_threads(),
                               "kind": "oracle", "sample": f"one full FP64 oracle solve of the same workload at rtol "
                                                           f"{RTOL}: {dt:.1f} s, {run_o.iters} CG iterations"}
        vs[f"oracle_rtol{RTOL:g}"] = {name: max(relerr(r["en"][k], run_o.energy[k]) for k in ("e_pol", "e_ion"))
                                      for name, r in (("multigrid_mixed", mg), ("multigrid_fp64", mg64),
                                                      ("jacobi_mixed", mx), ("jacobi_fp64", p64))}
    out["energy_relerr_vs_oracle"] = vs or None
    ctx.close()
    return out


def bench_binding(args, B, torch):
    """Binding energies of synthetic complexes by the paper's protocol (30 displacements of
    the solute within a cube of half the grid spacing, three solves each: complex, receptor,
    ligand, all on one grid per complex), served through the serving loop."""
    main = B.Context(0)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    w = I.binding_workload(n_complex=BIND_COMPLEXES, n_disp=BIND_DISP, h=BIND_H, precision=I.MIXED, rtol=RTOL,
                           inner_rtol=DELTA_MG, precond=I.MG)
    reqs = [(m, g) for _, _, _, m, g in w]
    main.set_profiling(True)
    side.set_profiling(True)
    for _ in range(args.warmup):
        serve(B, main, side, reqs[:3 * 6], max_resident=args.max_resident)[2].close()
    walls, res = [], None
    for _ in range(args.steps):
        torch.cuda.synchronize()
        res, wall, srv = serve(B, main, side, reqs, max_resident=args.max_resident)
        torch.cuda.synchronize()
        prof = srv.profile()
        srv.close()
        walls.append(wall)
    main.set_profiling(False)
    side.set_profiling(False)
    nbt = NbodyTimes()
    nbt.add_server(prof)
    value = len(reqs) / float(np.mean(walls))
    # ddG per complex over the displacements
    per = {}
    for idx, (c, k, part, _, _) in enumerate(w):
        per.setdefault(c, {}).setdefault(k, {})[part] = res[idx]
    table = []
    for c in sorted(per):
        dd = [B.binding_ddg(v["c"], v["1"], v["2"]) for v in per[c].values()]
        row = {"complex": c}
        for key in ("ddg_total", "ddg_coul", "ddg_pol", "ddg_ion"):
            xs = np.array([d[key] for d in dd])
            row[key] = [round(float(xs.mean()), 4), round(float(xs.std()), 4)]
        table.append(row)
    # accuracy: the first displacement of the first complex against tight FP64 Jacobi solves
    ref = [B.solve(m, replace(g, precision=I.FP64, precond=I.JACOBI, rtol=1e-12), main) for _, _, _, m, g in w[:3]]
    d_srv = B.binding_ddg(res[0], res[1], res[2])
    d_ref = B.binding_ddg(ref[0], ref[1], ref[2])
    n = max(prof["mg_samples"], 1)
    a_mg = prof["mg_sweep_bytes"] / (prof["mg_sweep_ms"] * 1e-3) / 1e9 if prof["mg_sweep_ms"] > 0 else None
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * float(np.mean(walls)), 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 CG + f64 reliable updates/energy", "data": "synthetic",
        "config": {"workload": f"binding energies: {BIND_COMPLEXES} synthetic complexes (1500 + 250 atoms) x "
                               f"{BIND_DISP} displacements x 3 solves (complex, receptor, ligand), "
                               f"h = {BIND_H} A, one grid per complex",
                   "requests": len(reqs), "grid": list(w[0][4].n), "rtol": RTOL,
                   "preconditioner": "multigrid V-cycle", "max_resident": args.max_resident},
        "ddg_kT_mean_std_per_complex": table,
        "ddg_served_vs_fp64_rtol1e-12": {k: abs(d_srv[k] - d_ref[k]) for k in d_ref},
        "roofline": {"bound": "hbm", "achieved": round(a_mg, 1) if a_mg else None, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(a_mg / HBM_PEAK_GBS, 4) if a_mg else None, "traffic": None,
                     "kernel": "k_sweep<float, true> (level-0 red-black half-sweep of the multigrid V-cycle)",
                     "bytes_per_launch": round(prof["mg_sweep_bytes"] / n),
                     "avg_launch_ms": round(prof["mg_sweep_ms"] / n, 5), "launches_timed": prof["mg_samples"],
                     "avg_vcycle_ms": round(prof["mg_vcycle_ms"] / n, 5),
                     "scope": "the first iteration of every chunk of every request (timed run)"},
        "roofline_other": nbt.roofline("every energy read-back of the timed run"),
        "stream_copy_GBs": round(main.stream_copy_gbps(1 << 30, 20), 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        from oracle import oracle as O

        _, _, _, m, g = w[0]
        t0 = time.perf_counter()
        run_o = O.run(m, replace(g, precision=I.FP64), rtol=RTOL)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": O.num_threads(),
                               "kind": "oracle",
                               "sample": f"one FP64 oracle solve (Jacobi-CG) of the first complex on its grid at rtol "
                                         f"{RTOL}: {dt:.1f} s, {run_o.iters} CG iterations"}
    main.close()
    side.close()
    return out


def bench_derefine(args, B, torch):
    """The paper's treatment of the box with one de-refinement level: the 2000-atom molecule
    with null Dirichlet values on a 160 A box, 0.5 A cells around the solute (its extent
    widened by 2 A) and 1 A cells beyond, against the tight uniform 161^3 grid at 0.5 A with
    Debye-Hueckel box values."""
    ctx = B.Context(0)
    mol, g_dh = I.protein_c2()
    g_dr = I.cubic_grid(161, 1.0, bc=I.BC_ZERO, refine=2, refine_shell=2.0, refine_brick=4)
    ref_dh = B.solve(mol, replace(g_dh, precision=I.FP64, rtol=1e-10), ctx)

    def run(g):
        lat, out = [], None
        for s_ in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb = B.Problem(ctx, mol, g)
            st = pb.solve()
            en = pb.energy()
            info = pb.refine_info() if g.refine else None
            pb.close()
            torch.cuda.synchronize()
            if s_ >= args.warmup:
                lat.append(time.perf_counter() - t0)
                out = (st, en, info)
        return len(lat) / sum(lat), out

    v_dr, (st, en, info) = run(replace(g_dr, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA))
    v_tl, (st_tl, en_tl, _) = run(replace(g_dr, precision=I.FP64, rtol=RTOL, precond=I.MG))
    v_tm, (st_tm, en_tm, _) = run(replace(g_dr, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA_MG, precond=I.MG))
    v_dh, (st_dh, en_dh, _) = run(replace(g_dh, precision=I.MIXED, rtol=RTOL, inner_rtol=DELTA, precond=I.MG))
    nunk = info["unknowns_coarse"] + info["unknowns_fine"]
    # value: the mixed solve with the two-level preconditioner (the fastest form), the
    # Jacobi-preconditioned mixed and the two-level FP64 solves beside it
    out = {
        "metric": METRIC, "value": round(v_tm, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 / v_tm, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 CG + f64 reliable updates/energy", "data": "synthetic",
        "config": {"workload": "2000-atom molecule, null Dirichlet values on a 160 A box, 0.5 A cells within 2 A of the "
                               "solute's extent (4^3-cell bricks), 1 A cells beyond (one de-refinement level)",
                   "preconditioner": "damped Jacobi + coarse-grid multigrid V-cycle (symmetric two-level)",
                   "reliable_update_factor": DELTA_MG,
                   "unknowns": int(nunk), "refined_cells": int(info["refined_cells"]),
                   "hanging_nodes": int(info["hanging_nodes"]), "fine_lattice": list(info["fine_n"]), "rtol": RTOL},
        "iters": st_tm["iters"],
        "fp64_two_level": {"solves_per_s": round(v_tl, 3), "iters": st_tl["iters"],
                           "energy_relerr_vs_mixed": max(abs(en_tl[k] / en_tm[k] - 1.0) for k in ("e_pol", "e_ion"))},
        "jacobi_mixed": {"solves_per_s": round(v_dr, 3), "iters": st["iters"], "reliable_update_factor": DELTA,
                         "energy_relerr_vs_mixed": max(abs(en[k] / en_tm[k] - 1.0) for k in ("e_pol", "e_ion"))},
        "energies_kT": {k: en_tm[k] for k in ("e_pol", "e_ion", "e_coul")},
        "vs_tight_uniform_debye_hueckel": {
            "grid": "161^3 at 0.5 A (80 A box), Debye-Hueckel box values, FP64 rtol 1e-10",
            "e_pol_relerr": abs(en_tm["e_pol"] / ref_dh["e_pol"] - 1.0),
            "e_ion_relerr": abs(en_tm["e_ion"] / ref_dh["e_ion"] - 1.0),
            "uniform_mixed_multigrid_solves_per_s": round(v_dh, 3)},
        "roofline": None,
        "stream_copy_GBs": round(ctx.stream_copy_gbps(1 << 30, 20), 1),
        "cpu_baseline": None,
    }
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c5", "c1", "c2", "c3", "c4", "binding", "derefine"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--counters-run", action="store_true",
                    help="serving stream: warm-up and closed loop only, with progress lines, for hardware-counter "
                         "passes (prints the algorithmic bytes of the batched solver launches)")
    ap.add_argument("--max-resident", type=int, default=MAX_RESIDENT,
                    help="serving stream: problems resident at once")
    ap.add_argument("--serve-precond", default="auto", choices=["auto", "mg", "jacobi"],
                    help="serving stream: preconditioner policy")
    ap.add_argument("--mg-min-n", type=int, default=MG_MIN_N,
                    help="serving stream, policy auto: smallest grid (nodes per axis) given the multigrid preconditioner")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): running the solver over "
              "several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_09323_amd import binding as B

    B.load()
    torch.cuda.set_device(0)
    if args.workload == "c5":
        out = bench_serving(args, B, torch)
    elif args.workload == "c3":
        out = bench_refined(args, B, torch)
    elif args.workload == "binding":
        out = bench_binding(args, B, torch)
    elif args.workload == "derefine":
        out = bench_derefine(args, B, torch)
    else:
        out = bench_single(args, B, torch)
    print(json.dumps(out), flush=True)
    bad = (out.get("energy_relerr") or {}).get("requests_over_bar", 0)
    if bad:
        print(f"[bench] {bad} served results exceed the {ERR_BAR:g} energy-error bar", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
