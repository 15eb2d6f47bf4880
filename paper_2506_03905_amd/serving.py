"""Serving: many channel and flat-plate solves arriving over time.

Continuous batching over the C ABI's pool (lbm_pool_*): requests are
admitted in arrival order as soon as a slot and a block of their footprint
are free; all resident lattices advance together in two groups that run
concurrently (small lattices in persistent launches, the others in
multi-lattice launches on a second stream), each group relaunched as soon as
its previous chunk of steps ends (lbm_pool_pump); a lattice leaves the pool
when its residual ||u^n - u^(n-K)|| / (K ||u^n||) falls below `tol`, when the
mean friction velocity changes by less than `tol_utau` (relative) between two
reductions K steps apart (the paper's criterion, Sec. 4.1.1), when it
diverges or when it reaches the step cap; the result says which.  The
sequential baseline runs the same requests one at a time with the plain
per-lattice path and the same criteria.

Request -> lattice (Sec. 4.1.1 and 4.2.1 of the paper, sizes from the
serving workload): channel 4 x Ny, Re_tau from Dean's correlation at Ma 0.05;
flat plate 8Ny x Ny with a slip leading section of nx/32 columns, plate
length 2 L_ref, Re per L_ref = 2500 Re_tau, U = 0.1.  All use FP32 storage,
the central-moment collision and the Spalart-Allmaras model.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm as L
from . import units


def request_lattice(req: dict, reduce_every: int = 100):
    """(lattice, nx, ny, nz, params, u0) for one request."""
    ny, nx = int(req["ny"]), int(req["nx"])
    scheme = L.SCHEME[req["scheme"]]
    if req["kind"] == "channel":
        lat = units.channel(float(req["re_tau"]), ny // 2, 0.05)
        p = L.lbm_params_default(precision=L.LBM_F32, flow=L.LBM_FLOW_CHANNEL, scheme=scheme,
                                 collision=L.LBM_COLL_CM, nu=lat["nu"],
                                 force=(lat["force"], 0, 0), u_init=(lat["u_bulk"], 0, 0),
                                 u_ref=lat["u_bulk"], reduce_every=reduce_every)
    else:
        plate_start = max(nx // 32, 2)
        lref = (nx - plate_start) / 2.0
        pl = units.plate(0.1, 2500.0 * float(req["re_tau"]), lref)
        p = L.lbm_params_default(precision=L.LBM_F32, flow=L.LBM_FLOW_PLATE, scheme=scheme,
                                 collision=L.LBM_COLL_CM, nu=pl["nu"], u_init=(0.1, 0, 0),
                                 u_inlet=0.1, u_ref=0.1, plate_start=plate_start,
                                 reduce_every=reduce_every)
    return L.LBM_D2Q9, nx, ny, 1, p, None


def footprint(req: dict) -> int:
    lat, nx, ny, nz, p, _ = request_lattice(req)
    return L.lbm_footprint(lat, nx, ny, nz, p)


def _summary(results: dict, makespan: float) -> dict:
    lat = np.array([r["latency"] for r in results.values()])
    st = [r["status"] for r in results.values()]
    by = [r.get("converged_by", 0) for r in results.values()]
    conv = np.array([r["latency"] for r in results.values() if r["status"] == L.LBM_SLOT_CONVERGED])
    return {
        "solves": len(results),
        "solves_per_s": len(results) / makespan if makespan > 0 else 0.0,
        "makespan_s": makespan,
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        # time-to-converged over the requests that converged
        "p50_converged_s": float(np.percentile(conv, 50)) if len(conv) else None,
        "p99_converged_s": float(np.percentile(conv, 99)) if len(conv) else None,
        "converged": sum(s == L.LBM_SLOT_CONVERGED for s in st),
        "converged_by_residual": sum(b == 1 for b in by),
        "converged_by_u_tau": sum(b == 2 for b in by),
        "capped": sum(s == L.LBM_SLOT_CAPPED for s in st),
        "diverged": sum(s == L.LBM_SLOT_DIVERGED for s in st),
        "lattice_updates": int(sum(r["steps"] * r["cells"] for r in results.values())),
    }


def run_batched(requests: list, pool_bytes: int, chunk: int = 200, tol: float = 1e-8,
                max_steps: int = 20000, max_slots: int = 1024, keep_fields: set = frozenset(),
                device="cuda:0", log=None, tol_utau: float = 0.0) -> tuple:
    """Continuous batching in one pool.  Returns (results by id, summary)."""
    pool = L.Pool(pool_bytes, max_slots=max_slots, device=device)
    reqs = sorted(requests, key=lambda r: r["t_arrival"])
    results, active = {}, {}
    i = 0
    t0 = time.perf_counter()
    while i < len(reqs) or active:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i]["t_arrival"] <= now:
            lat, nx, ny, nz, p, u0 = request_lattice(reqs[i])
            slot = pool.lbm_pool_admit(lat, nx, ny, nz, p, u0, tol, max_steps, tol_utau=tol_utau)
            if slot is None:
                break  # wait for memory / a slot to free up (arrival order is kept)
            active[slot] = (reqs[i], now)
            i += 1
        if not active:
            time.sleep(max(0.0, min(reqs[i]["t_arrival"] - now, 0.05)))
            continue
        busy = pool.lbm_pool_pump(chunk)
        now = time.perf_counter() - t0
        finished = 0
        for slot in list(active):
            st = pool.lbm_pool_poll(slot)
            if st["status"] == L.LBM_SLOT_RUNNING:
                continue
            req, t_adm = active.pop(slot)
            res = {"latency": now - req["t_arrival"], "queued": t_adm - req["t_arrival"],
                   "steps": st["steps"], "status": st["status"], "batched": st["batched"],
                   "residual": st["residual"], "mean_u_tau": st["mean_u_tau"],
                   "d_u_tau_rel": st["d_u_tau_rel"], "converged_by": st["converged_by"],
                   "cells": req["nx"] * req["ny"]}
            if req["id"] in keep_fields:
                v = pool.lbm_pool_lattice(slot)
                res["u"] = v.lbm_moments()[1]
                res["utau"] = v.lbm_wall()["utau"]
            results[req["id"]] = res
            pool.lbm_pool_release(slot)
            finished += 1
            if log:
                log(f"done {req['id']} {req['kind']} {req['nx']}x{req['ny']} steps={st['steps']} "
                    f"status={st['status']} latency={res['latency']:.3f}s")
        if not finished and busy:
            time.sleep(2e-4)
    makespan = time.perf_counter() - t0
    pool.close()
    return results, _summary(results, makespan)


def run_sequential(requests: list, tol: float = 1e-8, max_steps: int = 20000, check_every: int = 100,
                   keep_fields: set = frozenset(), device="cuda:0", honor_arrivals: bool = True,
                   log=None, tol_utau: float = 0.0) -> tuple:
    """The same requests one at a time through the plain per-lattice path
    (checks every `check_every` steps, the lattices' reduction period)."""
    reqs = sorted(requests, key=lambda r: r["t_arrival"])
    results = {}
    t0 = time.perf_counter()
    for req in reqs:
        now = time.perf_counter() - t0
        if honor_arrivals and now < req["t_arrival"]:
            time.sleep(req["t_arrival"] - now)
        lat, nx, ny, nz, p, u0 = request_lattice(req)
        g = L.Lattice(lat, nx, ny, nz, p, device=device)
        status, steps, r, by = L.LBM_SLOT_CAPPED, 0, {}, 0
        while steps < max_steps:
            n = min(check_every, max_steps - steps)
            try:
                g.lbm_step(n)
            except L.LbmError as e:
                if e.code != L.LBM_EDIVERGED:
                    raise
                status = L.LBM_SLOT_DIVERGED
                break
            steps += n
            r = g.lbm_residual()
            if r["rc"] == L.LBM_EDIVERGED:
                status = L.LBM_SLOT_DIVERGED
                break
            if steps % check_every:
                continue  # only reduction steps decide convergence
            if r["l2_du_rel"] < tol:
                status, by = L.LBM_SLOT_CONVERGED, 1
                break
            if tol_utau > 0 and 0 <= r["d_u_tau_rel"] < tol_utau:
                status, by = L.LBM_SLOT_CONVERGED, 2
                break
        res = {"latency": time.perf_counter() - t0 - req["t_arrival"], "steps": steps,
               "status": status, "batched": False, "residual": r.get("l2_du_rel"),
               "mean_u_tau": r.get("mean_u_tau"), "d_u_tau_rel": r.get("d_u_tau_rel"),
               "converged_by": by, "cells": nx * ny}
        if req["id"] in keep_fields:
            res["u"] = g.lbm_moments()[1]
            res["utau"] = g.lbm_wall()["utau"]
        results[req["id"]] = res
        g.close()
        if log:
            log(f"seq done {req['id']} steps={steps} status={status}")
    makespan = time.perf_counter() - t0
    return results, _summary(results, makespan)
