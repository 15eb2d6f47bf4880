"""Channel studies of Sec. 4.1 run to convergence in the serving pool.

Every case is a 2-D channel (D2Q9, 4 x 2N cells, walls at y = 0 and y = 2N
(halfway) or q from the first nodes, body force rho0 u_tau^2 / h, Dean's bulk
velocity as the start, Ma = 0.05) with the central-moment collision and the
Spalart-Allmaras model, FP64 storage.  Reported per case: the wall-function
friction velocity at convergence over the target one (the force fixes the
target: u_tau^2 = F h / rho0), the bulk velocity over Dean's, and the bulk
friction coefficient 2 (u_tau / U_b)^2.

Studies (only formulas of the paper are needed):
  grid      Re_tau = 4200, N = 5 ... 40 (Table 3), every wall treatment
  reynolds  N = 20, Re_tau = 2000 ... 20000 (Table 2)
  beta      N = 20, Re_tau = 4200: HRFD beta sweep next to Cai-Degrigny
            (Sec. 4.1.2.2: beta = 0.25 reproduces Cai-Degrigny)
  wall      N = 20, Re_tau = 4200: wall q from the first node with Bouzidi's
            interpolated bounce-back (Sec. 4.1.2.5)

    python -m paper_2506_03905_amd.replicate [--studies grid,beta] [--max-steps N]
        [--tol R] [--tol-utau T] [--out table.md]

A case retires when the residual falls below --tol or, with --tol-utau > 0,
when the mean u_tau changes by less than that (relative) between two
reductions (100 steps apart), the criterion of Sec. 4.1.1; the table says
which fired.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


from . import lbm as L
from . import units

SCHEMES = {
    "slip_bb": dict(scheme=L.LBM_WALL_SLIP_BB),
    "hrfd_0.28": dict(scheme=L.LBM_WALL_HRFD, beta=0.28),
    "hrfd_0.25": dict(scheme=L.LBM_WALL_HRFD, beta=0.25),
    "hrfd_0": dict(scheme=L.LBM_WALL_HRFD, beta=0.0),
    "hrfd_1": dict(scheme=L.LBM_WALL_HRFD, beta=1.0),
    "cai_degrigny": dict(scheme=L.LBM_WALL_CAI_DEGRIGNY),
}


def cases(studies) -> list:
    out = []
    if "grid" in studies:
        for n in (5, 10, 20, 30, 40):
            for s in SCHEMES:
                out.append({"study": "grid", "re_tau": 4200.0, "n": n, "wall": s, "q": 0.5})
    if "reynolds" in studies:
        for re_tau in (2000.0, 4200.0, 8000.0, 20000.0):
            for s in ("slip_bb", "hrfd_0.28", "cai_degrigny"):
                out.append({"study": "reynolds", "re_tau": re_tau, "n": 20, "wall": s, "q": 0.5})
    if "beta" in studies:
        for s in ("hrfd_0", "hrfd_0.25", "hrfd_0.28", "hrfd_1", "cai_degrigny"):
            out.append({"study": "beta", "re_tau": 4200.0, "n": 20, "wall": s, "q": 0.5})
    if "wall" in studies:
        for q in (0.25, 0.5, 0.75, 1.0):
            out.append({"study": "wall", "re_tau": 4200.0, "n": 20, "wall": "slip_bb", "q": q,
                        "interp": L.LBM_IBB_BOUZIDI})
    return out


def lattice_of(case: dict):
    """(ny, h, U_b, u_tau, params): 2N nodes across, the walls q from the first
    and last nodes, so the half height is h = (2N - 1 + 2q) / 2 cells."""
    n, q = case["n"], case["q"]
    ny = 2 * n
    h = (ny - 1 + 2 * q) / 2.0
    lat = units.channel(case["re_tau"], 1, 0.05)  # velocities only (Ma scaling)
    u_b, u_tau = lat["u_bulk"], lat["u_tau"]
    nu = u_tau * h / case["re_tau"]
    kw = dict(SCHEMES[case["wall"]])
    kw.update(precision=L.LBM_F64, collision=L.LBM_COLL_CM, nu=nu, force=(u_tau * u_tau / h, 0, 0),
              u_init=(u_b, 0, 0), u_ref=u_b, reduce_every=100)
    if case.get("interp"):
        kw.update(bb_interp=case["interp"], wall_dist=q)
    return ny, h, u_b, u_tau, L.lbm_params_default(**kw)


def run(case_list: list, tol: float = 1e-9, max_steps: int = 600000, chunk: int = 2000,
        log=None, keep_fields: bool = False, tol_utau: float = 0.0) -> list:
    """Runs every case to convergence (residual below tol, or, with tol_utau >
    0, the relative change of the mean u_tau between reductions below
    tol_utau, the criterion of Sec. 4.1.1) or max_steps in one pool;
    keep_fields adds each case's final velocity field and u_tau."""
    pool = L.Pool(1 << 30, max_slots=max(len(case_list), 1))
    slots = []
    for c in case_list:
        ny, h, u_b, u_tau, p = lattice_of(c)
        slots.append((pool.lbm_pool_admit(L.LBM_D2Q9, 4, ny, 1, p, None, tol, max_steps, tol_utau=tol_utau),
                      ny, h, u_b, u_tau))
    t0 = time.perf_counter()
    while True:
        pool.lbm_pool_step(chunk)
        st = [pool.lbm_pool_poll(s[0]) for s in slots]
        running = sum(x["status"] == L.LBM_SLOT_RUNNING for x in st)
        if log:
            log(f"t={time.perf_counter() - t0:6.1f}s running={running}")
        if not running:
            break
    rows = []
    for c, (slot, ny, h, u_b, u_tau), s in zip(case_list, slots, st):
        v = pool.lbm_pool_lattice(slot)
        _, u, _ = v.lbm_moments()
        ub = float(u[0].mean())
        ut = float(v.lbm_wall()["utau"].mean())
        extra = {"u": u, "utau": v.lbm_wall()["utau"]} if keep_fields else {}
        rows.append({**c, **extra, "ny": ny, "steps": s["steps"],
                     "status": {2: "converged", 3: "capped", 4: "diverged"}.get(s["status"], "?"),
                     "converged_by": {1: "residual", 2: "u_tau"}.get(s.get("converged_by", 0), ""),
                     "residual": s["residual"], "u_tau/target": ut / u_tau,
                     "U_b/dean": ub / u_b, "cf_b/dean": (ut / ub) ** 2 / (u_tau / u_b) ** 2,
                     "y_b_plus": c["q"] * c["re_tau"] / h})
    pool.close()
    return rows


def table(rows: list) -> str:
    out = ["| study | Re_tau | N | wall | q | steps | status | residual | u_tau/target | U_b/Dean |",
           "|---|---:|---:|---|---:|---:|---|---:|---:|---:|"]
    for r in rows:
        st = r["status"] + (f" ({r['converged_by']})" if r.get("converged_by") else "")
        out.append(f"| {r['study']} | {r['re_tau']:.0f} | {r['n']} | {r['wall']} | {r['q']:g} | "
                   f"{r['steps']} | {st} | {r['residual']:.1e} | {r['u_tau/target']:.4f} | "
                   f"{r['U_b/dean']:.4f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--studies", default="grid,reynolds,beta,wall")
    ap.add_argument("--max-steps", type=int, default=600000)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--tol-utau", type=float, default=0.0,
                    help="also retire a case once its mean u_tau changes by less than this "
                         "(relative) between reductions (Sec. 4.1.1 uses 1e-4)")
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--out", default=None, help="also write the table (markdown) to this file")
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    rows = run(cases(a.studies.split(",")), tol=a.tol, max_steps=a.max_steps, tol_utau=a.tol_utau,
               log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    text = json.dumps(rows) if a.json else table(rows)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write("# Channel studies of Sec. 4.1 (written by paper_2506_03905_amd.replicate)\n\n"
                     f"Command: `python -m paper_2506_03905_amd.replicate --studies {a.studies} "
                     f"--max-steps {a.max_steps} --tol {a.tol:g} --tol-utau {a.tol_utau:g} --out <file>`; "
                     f"{len(rows)} channels in one serving pool, {time.perf_counter() - t0:.1f} s on one "
                     "MI355X.  D2Q9 4 x 2N, FP64, central-moment collision + SA, Dean start; "
                     "u_tau/target = the wall function's mean friction velocity over the one the "
                     "body force imposes, U_b/Dean = the bulk velocity over Dean's.\n\n" + table(rows) + "\n")


if __name__ == "__main__":
    main()
