"""Throughput of the fused LBM-RANS step on one MI355X.

Default workload: the 3-D turbulent channel, D3Q19, 512 x 256 x 256 cells
(streamwise x wall-normal x spanwise), FP32 storage and arithmetic, Re_tau =
5000 with 128 cells per half channel, Ma = 0.05, BGK collision with the local
tau from nu + nu_t (Spalart-Allmaras), slip-velocity bounce-back with
Reichardt's law, started from Dean's bulk velocity as in the paper's channel
runs (--amp adds a seeded random perturbation).  A step is the whole hot path:
the fused stream-collide-SA kernel, the wall-function kernel and, every 100
steps, the FP64 residual reduction.

--calibrate-copy times a plain device-to-device copy of known size instead;
its hardware byte counters give the scale factor for the kernel's counters.

The default run also measures the serving half of the metric on a bounded
sample (the first 64 requests of the seeded serving workload, step cap 5000;
--serving-requests, --serving-cap): seeded Poisson arrivals of 2-D channel
and flat-plate solves (70/30, log-uniform Ny in [32, 1024] and Re_tau in
[500, 20000], wall scheme drawn per request), each retired on an L2 velocity
residual below 1e-8, on a relative change of the mean u_tau below 1e-4
between reductions (Sec. 4.1.1), on divergence or at the cap, through the
batched pool and then one at a time through the plain per-lattice path:
solves/s, p50/p99 time-to-result and time-to-converged, and the same-result
check.  --serving runs the whole 512-request workload alone instead.

Kernel durations come from HIP events around the launches of two steps in
every ten inside the timed region (both step parities), so the timed steps
run back to back.

Prints one JSON line: the metric, its value and unit, the timing contract
fields, the workload, the roofline of the fused step kernel (algorithmic bytes
per launch over its measured duration, against 8 TB/s, and the HBM traffic
measured by the hardware counters when available), the serving figures and
the oracle's rate on the host's cores, one thread and all of them.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# HBM bytes per k_step launch from the FETCH_SIZE / WRITE_SIZE counters of the
# default workload (void once the kernel sources change)
TRAFFIC_PROFILE = "k_step_d3q19_512x256x256_f32_traffic.md"


def bytes_per_lup(q: int, precision: str, sa: bool = True) -> int:
    """Algorithmic bytes per lattice update: every population read and written
    once, nu_tilde read and written once, the velocity written once and read
    once through the SA stencil (without SA: populations and the velocity
    written once)."""
    sb = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[precision]
    tb = 8 if precision == "f64" else 4
    D = 2 if q == 9 else 3
    if not sa:
        return 2 * q * sb + D * tb
    return 2 * q * sb + 2 * tb + 2 * D * tb


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(nx, ny, nz, lat, steps, collision, amp, threads):
    import oracle as O
    from paper_2506_03905_amd import inputs

    O.set_threads(threads)
    u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], amp)
    p = O.params(q=19, nx=nx, ny=ny, nz=nz, nu=lat["nu"], force=(lat["force"], 0, 0),
                 scheme=O.BB_SLIP, collision={"bgk": O.BGK, "cm": O.CM}[collision])
    o = O.Oracle(p, u0)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return nx * ny * nz * steps / dt / 1e6, dt


def cpu_baseline(nx: int, ny: int, lat: dict, steps: int, collision: str, amp: float) -> dict:
    """The oracle on slabs of the same channel (same resolution, Re_tau and
    start; full x and y extent, a few z planes): one thread, then every
    thread the host gives it (OpenMP over lattice rows)."""
    import oracle as O

    threads = O.get_threads()  # OMP_NUM_THREADS or all cores
    v1, dt1 = _oracle_rate(nx, ny, 4, lat, steps, collision, amp, 1)
    nz_all = 4 * max(1, min(threads, 16))
    vn, dtn = _oracle_rate(nx, ny, nz_all, lat, steps, collision, amp, threads)
    O.set_threads(threads)
    return {"value": round(vn, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle on a {nx}x{ny}x{nz_all} slab of the same channel (same "
                      f"resolution, Re_tau, start), {steps} steps, {threads} threads, {dtn:.1f} s",
            "one_thread": {"value": round(v1, 3), "unit": "MLUPS",
                           "sample": f"{nx}x{ny}x4 slab, {steps} steps, 1 thread, {dt1:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def timed_steps(g, steps: int, warmup: int):
    """(ms for `steps` steps between HIP events on the lattice's stream, timing dict)."""
    import torch

    g.lbm_step(warmup)
    torch.cuda.synchronize()
    g.lbm_set_timing(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    g.lbm_step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    tm = g.lbm_get_timing()
    g.lbm_set_timing(False)
    return e0.elapsed_time(e1), tm


def plate_bench(args):
    """The flat-plate workload: D2Q9 2048 x 256, U = 0.1, Re = 5e6 per L_ref
    (992 cells), plate from column 64, CM + SA, slip BB or HRFD."""
    import paper_2506_03905_amd.lbm as L

    nx, ny = args.nx or 2048, args.ny or 256
    ps, U = 64, 0.1
    nu = U * ((nx - ps) / 2.0) / 5e6
    p = L.lbm_params_default(precision=L.PRECISION[args.precision], flow=L.LBM_FLOW_PLATE,
                             scheme=L.SCHEME[args.scheme], collision=L.LBM_COLL_CM, nu=nu,
                             u_init=(U, 0, 0), u_inlet=U, u_ref=U, plate_start=ps, reduce_every=100)
    g = L.Lattice(L.LBM_D2Q9, nx, ny, 1, p, device="cuda:0")
    ms, tm = timed_steps(g, args.steps, args.warmup)
    ncell = nx * ny
    bpl = bytes_per_lup(9, args.precision)
    k_ms = tm["step_ms"] / max(tm["step_launches"], 1)
    achieved = bpl * ncell / (k_ms * 1e-3) / 1e9
    out = {"metric": "MLUPS (D2Q9 flat plate)", "value": round(ncell * args.steps / (ms * 1e-3) / 1e6, 1),
           "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": f"2-D flat plate D2Q9 {nx}x{ny}, Re 5e6 per L_ref, CM + SA, "
                                  f"{args.scheme}", "cells": ncell},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                        "kernel": "k_step", "bytes_per_lup": bpl, "kernel_ms": round(k_ms, 4),
                        "wall_kernel_ms": round(tm["wall_ms"] / max(tm["wall_launches"], 1), 4)}}
    print(json.dumps(out), flush=True)


def serving_bench(args):
    import torch

    from paper_2506_03905_amd import inputs, serving

    reqs = inputs.requests(0, args.requests, args.rate)
    need = sum(serving.footprint(r) for r in reqs)
    pool_bytes = min(int(need * 1.05) + (64 << 20), 128 << 30)

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    print(f"# serving: {len(reqs)} requests, total footprint {need / 1e9:.2f} GB, "
          f"pool {pool_bytes / 1e9:.2f} GB", file=sys.stderr, flush=True)
    res_b, sum_b = serving.run_batched(reqs, pool_bytes, chunk=args.chunk, tol=args.tol,
                                       tol_utau=args.tol_utau, max_steps=args.max_steps, log=log)
    torch.cuda.synchronize()
    nseq = len(reqs) if args.seq_requests < 0 else min(args.seq_requests, len(reqs))
    seq = reqs[:nseq]
    res_s, sum_s = serving.run_sequential(seq, tol=args.tol, tol_utau=args.tol_utau,
                                          max_steps=args.max_steps, log=log)
    # same requests, same result: step counts and end status must agree, and
    # the mean u_tau at the end (FP32 fields; the two paths differ only in the
    # order of FP64 sums and in FMA contraction)
    agree = all(res_b[r["id"]]["status"] == res_s[r["id"]]["status"] and
                res_b[r["id"]]["steps"] == res_s[r["id"]]["steps"] and
                res_b[r["id"]]["converged_by"] == res_s[r["id"]]["converged_by"] for r in seq)
    dut = [abs(res_b[r["id"]]["mean_u_tau"] - res_s[r["id"]]["mean_u_tau"]) /
           max(abs(res_s[r["id"]]["mean_u_tau"]), 1e-300) for r in seq
           if res_s[r["id"]]["status"] != 4 and res_b[r["id"]]["status"] != 4]
    out = {
        "metric": "batched solves/s (p99 time-to-result reported) vs sequential plain solves",
        "value": round(sum_b["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.max_steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving: {len(reqs)} Poisson requests at {args.rate:g}/s, 70% "
                               f"2-D channel (4 x Ny) / 30% flat plate (8Ny x Ny), Ny log-uniform "
                               f"[32, 1024], Re_tau log-uniform [500, 20000], retired on residual < "
                               f"{args.tol:g} or d(u_tau)/u_tau < {args.tol_utau:g} per 100 steps, "
                               f"step cap {args.max_steps}, D2Q9 FP32 CM + SA",
                   "chunk": args.chunk, "parallelism": "single GPU"},
        "batched": sum_b,
        "sequential": sum_s,
        "sequential_requests": nseq,
        "speedup_solves_per_s": sum_b["solves_per_s"] / sum_s["solves_per_s"]
                                if nseq and sum_s["solves_per_s"] > 0 else None,
        "same_steps_and_status": agree,
        "max_rel_diff_mean_u_tau": max(dut) if dut else None,
    }
    print(json.dumps(out), flush=True)


def serving_sample(n_requests: int, cap: int, rate: float, chunk: int, tol: float,
                   tol_utau: float) -> dict:
    """The serving half of the metric on the first n_requests of the seeded
    workload: batched pool vs the same requests one at a time."""
    import torch

    from paper_2506_03905_amd import inputs, serving

    reqs = inputs.requests(0, n_requests, rate)
    need = sum(serving.footprint(r) for r in reqs)
    pool_bytes = min(int(need * 1.05) + (64 << 20), 64 << 30)
    kw = dict(tol=tol, tol_utau=tol_utau, max_steps=cap)
    res_b, sum_b = serving.run_batched(reqs, pool_bytes, chunk=chunk, **kw)
    torch.cuda.synchronize()
    res_s, sum_s = serving.run_sequential(reqs, **kw)
    same = [res_b[r["id"]]["status"] == res_s[r["id"]]["status"] and
            res_b[r["id"]]["steps"] == res_s[r["id"]]["steps"] and
            res_b[r["id"]]["converged_by"] == res_s[r["id"]]["converged_by"] for r in reqs]
    dut = [abs(res_b[r["id"]]["mean_u_tau"] - res_s[r["id"]]["mean_u_tau"]) /
           max(abs(res_s[r["id"]]["mean_u_tau"]), 1e-300) for r in reqs
           if res_s[r["id"]]["status"] != 4 and res_b[r["id"]]["status"] != 4]
    keep = ("solves_per_s", "makespan_s", "p50_s", "p99_s", "p50_converged_s", "p99_converged_s",
            "converged", "converged_by_residual", "converged_by_u_tau", "capped", "diverged",
            "lattice_updates")
    return {"workload": f"first {n_requests} requests of the serving workload (Poisson "
                        f"{rate:g}/s, 70% channel 4 x Ny / 30% plate 8Ny x Ny, Ny in [32, 1024], "
                        f"Re_tau in [500, 20000]), D2Q9 FP32 CM + SA, retired on residual < "
                        f"{tol:g} or d(u_tau)/u_tau < {tol_utau:g} per 100 steps, cap {cap} steps",
            "unit": "solves/s",
            "batched": {k: sum_b[k] for k in keep},
            "sequential": {k: sum_s[k] for k in keep},
            "speedup_solves_per_s": sum_b["solves_per_s"] / sum_s["solves_per_s"]
                                    if sum_s["solves_per_s"] > 0 else None,
            "same_steps_status_criterion": f"{sum(same)}/{len(same)}",
            "max_rel_diff_mean_u_tau": max(dut) if dut else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="f32", choices=["f32", "f16", "bf16", "f64"])
    ap.add_argument("--plate", action="store_true",
                    help="the 2-D flat plate (D2Q9 2048 x 256, CM) instead of the 3-D channel")
    ap.add_argument("--scheme", default="slip_bb", choices=["slip_bb", "hrfd"])
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--nz", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--collision", default="bgk", choices=["bgk", "cm"])
    ap.add_argument("--amp", type=float, default=0.0)
    ap.add_argument("--store-shift", type=float, default=0.0,
                    help="store f - f_eq(rho0, (s U_b, 0, 0)) (s = this value; 0 stores f - w rho0)")
    ap.add_argument("--sa", default="on", choices=["on", "off"])
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB")
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--seq-requests", type=int, default=-1,
                    help="requests run sequentially (default: all)")
    ap.add_argument("--tol-utau", type=float, default=1e-4)
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-cap", type=int, default=5000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--timing-every", type=int, default=10,
                    help="kernel events around 2 steps in every k (1: every launch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the lattice is not sharded across GPUs here "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20)
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        a.fill_(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(json.dumps({"copy_bytes": n, "ms": ms, "GBs_read_plus_write": 2 * n / ms / 1e6}))
        return

    if args.serving:
        serving_bench(args)
        return

    import paper_2506_03905_amd.lbm as L
    from paper_2506_03905_amd import inputs, units

    if args.plate:
        return plate_bench(args)
    nx, ny, nz = args.nx or 512, args.ny or 256, args.nz or 256
    lat = units.channel(5000.0, ny // 2, 0.05)
    coll = {"bgk": L.LBM_COLL_BGK, "cm": L.LBM_COLL_CM}[args.collision]
    p = L.lbm_params_default(precision=L.PRECISION[args.precision], scheme=L.LBM_WALL_SLIP_BB,
                             nu=lat["nu"], force=(lat["force"], 0, 0), u_ref=lat["u_bulk"],
                             reduce_every=100, collision=coll, sa_on=1 if args.sa == "on" else 0,
                             store_shift_u=args.store_shift * lat["u_bulk"])
    g = L.Lattice(L.LBM_D3Q19, nx, ny, nz, p, device="cuda:0")
    u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], args.amp)
    g.lbm_set_velocity(u0)
    del u0
    print(f"# lattice {nx}x{ny}x{nz} D3Q19 {args.precision}, nu={lat['nu']:.4e}, "
          f"tau-1/2={3 * lat['nu']:.3e}, footprint {g.bytes / 1e9:.2f} GB", file=sys.stderr, flush=True)
    g.lbm_step(args.warmup)
    torch.cuda.synchronize()
    # sampled events need a window of several periods; short runs time every launch
    every = args.timing_every if args.steps >= 2 * args.timing_every else 1
    g.lbm_set_timing(True, every=every)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    t0 = time.perf_counter()
    g.lbm_step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    tm = g.lbm_get_timing()
    g.lbm_set_timing(False)
    res = g.lbm_residual()
    ncell = nx * ny * nz
    mlups = ncell * args.steps / (ms * 1e-3) / 1e6
    bpl = bytes_per_lup(19, args.precision, args.sa == "on")
    k_ms = tm["step_ms"] / max(tm["step_launches"], 1)
    achieved = bpl * ncell / (k_ms * 1e-3) / 1e9
    traffic = None
    if (nx, ny, nz, args.precision, args.collision, args.sa, args.amp, args.store_shift) == \
            (512, 256, 256, "f32", "bgk", "on", 0.0, 0.0):
        from paper_2506_03905_amd import profile_summary
        t = profile_summary.read_traffic(os.path.join(ROOT, "profiles", TRAFFIC_PROFILE))
        traffic = None if t is None else round(t["traffic_bytes"])
    out = {
        "metric": "MLUPS & % HBM peak (D3Q19 fp32); batched solves/s + p99 latency vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32",
                  "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"3-D channel D3Q19 {nx}x{ny}x{nz}, Re_tau 5000, "
                               f"{args.collision.upper()}" + (" + SA" if args.sa == "on" else
                                                               " (no SA)") + ", slip-velocity bounce-back "
                               f"(Reichardt), Dean start" + (f" + {args.amp:g} perturbation"
                                                             if args.amp else "")
                               + (f", stored f - f_eq(rho0, {args.store_shift:g} U_b)" if args.store_shift
                                  else ""),
                   "cells": ncell, "collision": args.collision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "k_step", "bytes_per_lup": bpl,
                     "algorithmic_bytes_per_launch": bpl * ncell,
                     "kernel_ms": round(k_ms, 4),
                     "kernel_launches_timed": tm["step_launches"],
                     # HBM bytes the counters measured per launch over the launch time
                     "measured_gbs": None if traffic is None else round(traffic / (k_ms * 1e-3) / 1e9, 1),
                     # the populations alone (read and written once), the figure LBM codes quote
                     "pops_only_gbs": round(2 * 19 * {"f64": 8, "f32": 4}.get(args.precision, 2) * ncell
                                            / (k_ms * 1e-3) / 1e9, 1),
                     "wall_kernel_ms": round(tm["wall_ms"] / max(tm["wall_launches"], 1), 4)},
        "residual": {"l2_du_rel": res["l2_du_rel"], "mean_u_tau": res["mean_u_tau"],
                     "nan_flag": res["nan_flag"]},
        "host_wall_s": round(wall_s, 3),
    }
    del g
    torch.cuda.synchronize()
    if not args.no_serving:
        print(f"# serving sample: {args.serving_requests} requests, cap {args.serving_cap}",
              file=sys.stderr, flush=True)
        out["serving"] = serving_sample(args.serving_requests, args.serving_cap, args.rate,
                                        args.chunk, args.tol, args.tol_utau)
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(nx, ny, lat, args.cpu_steps, args.collision, args.amp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
