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

--serving runs the serving workload instead: seeded Poisson arrivals of 2-D
channel and flat-plate solves (70/30, log-uniform Ny in [32, 1024] and Re_tau
in [500, 20000], wall scheme drawn per request), each run to an L2 velocity
residual below 1e-8 or to the step cap, through the batched pool and then one
at a time through the plain per-lattice path; it prints solves/s and p50/p99
time-to-result for both.

Prints one JSON line: the metric, its value and unit, the timing contract
fields, the workload, the roofline of the fused step kernel (algorithmic bytes
per launch over its measured duration, against 8 TB/s, and the HBM traffic
measured by the hardware counters when available) and the oracle's rate on
the host for scale.
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


def cpu_baseline(nx: int, ny: int, nz: int, lat: dict, steps: int, collision: str,
                 amp: float) -> dict:
    import numpy as np

    import oracle as O
    from paper_2506_03905_amd import inputs

    u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], amp)
    p = O.params(q=19, nx=nx, ny=ny, nz=nz, nu=lat["nu"], force=(lat["force"], 0, 0),
                 scheme=O.BB_SLIP, collision={"bgk": O.BGK, "cm": O.CM}[collision])
    o = O.Oracle(p, u0)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    del o, u0
    _ = np
    return {"value": nx * ny * nz * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{nx}x{ny}x{nz} slab of the same channel (same resolution, Re_tau, start), "
                      f"{steps} steps, FP64, 1 thread, {dt:.1f} s"}


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
                                       max_steps=args.max_steps, log=log)
    torch.cuda.synchronize()
    nseq = len(reqs) if args.seq_requests < 0 else min(args.seq_requests, len(reqs))
    seq = reqs[:nseq]
    res_s, sum_s = serving.run_sequential(seq, tol=args.tol, max_steps=args.max_steps, log=log)
    # same requests, same result: step counts and end status must agree, and
    # the mean u_tau at the end (FP32 fields; the two paths differ only in the
    # order of FP64 sums and in FMA contraction)
    agree = all(res_b[r["id"]]["status"] == res_s[r["id"]]["status"] and
                res_b[r["id"]]["steps"] == res_s[r["id"]]["steps"] for r in seq)
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
                               f"[32, 1024], Re_tau log-uniform [500, 20000], tol {args.tol:g}, "
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
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--collision", default="bgk", choices=["bgk", "cm"])
    ap.add_argument("--amp", type=float, default=0.0)
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the lattice is not sharded across GPUs here "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
                             reduce_every=100, collision=coll, sa_on=1 if args.sa == "on" else 0)
    g = L.Lattice(L.LBM_D3Q19, nx, ny, nz, p, device="cuda:0")
    u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], args.amp)
    g.lbm_set_velocity(u0)
    del u0
    print(f"# lattice {nx}x{ny}x{nz} D3Q19 {args.precision}, nu={lat['nu']:.4e}, "
          f"tau-1/2={3 * lat['nu']:.3e}, footprint {g.bytes / 1e9:.2f} GB", file=sys.stderr, flush=True)
    g.lbm_step(args.warmup)
    torch.cuda.synchronize()
    g.lbm_set_timing(True)
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
    if (nx, ny, nz, args.precision, args.collision, args.sa, args.amp) == \
            (512, 256, 256, "f32", "bgk", "on", 0.0):
        from paper_2506_03905_amd import profile_summary
        t = profile_summary.read_traffic(os.path.join(ROOT, "profiles", TRAFFIC_PROFILE))
        traffic = None if t is None else round(t["traffic_bytes"])
    out = {
        "metric": "MLUPS & % HBM peak (D3Q19 fp32)",
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
                                                             if args.amp else ""),
                   "cells": ncell, "collision": args.collision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "k_step", "bytes_per_lup": bpl,
                     "algorithmic_bytes_per_launch": bpl * ncell,
                     "kernel_ms": round(k_ms, 4),
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
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(nx, ny, 4, lat, args.cpu_steps, args.collision,
                                           args.amp)
    _ = np
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
