"""Seeded synthetic inputs shared by the tests, the benchmark and the serving
loop.  Only random numbers and shapes live here -- no step of the method.

* ``perturbation(seed, D, nz, ny, nx, amp)``: velocity perturbation
  amp * xi with xi uniform in [-1, 1), drawn from numpy's PCG64 seeded with
  ``seed``, SoA layout (D, nz, ny, nx).
* ``channel_velocity(...)``: a uniform streamwise velocity plus that
  perturbation.
* ``requests(...)``: the serving workload's arrival times and request mix.
"""
from __future__ import annotations

import numpy as np


def perturbation(seed: int, D: int, nz: int, ny: int, nx: int, amp: float) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return amp * (2.0 * rng.random((D, nz, ny, nx)) - 1.0)


def channel_velocity(seed: int, D: int, nz: int, ny: int, nx: int, u0: float,
                     amp: float) -> np.ndarray:
    u = perturbation(seed, D, nz, ny, nx, amp) if amp > 0 else np.zeros((D, nz, ny, nx))
    u[0] += u0
    return u


def requests(seed: int, n: int, rate_per_s: float, frac_channel: float = 0.7,
             ny_range=(32, 1024), re_tau_range=(500.0, 20000.0)) -> list:
    """Poisson arrivals with the request mix of the serving workload: channel
    (nx = 4) or flat plate (nx = 8 ny), log-uniform ny and Re_tau, and a wall
    scheme drawn uniformly from {slip bounce-back, HRFD}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
    out = []
    for k in range(n):
        kind = "channel" if rng.random() < frac_channel else "plate"
        ny = int(round(np.exp(rng.uniform(np.log(ny_range[0]), np.log(ny_range[1])))))
        re_tau = float(np.exp(rng.uniform(np.log(re_tau_range[0]), np.log(re_tau_range[1]))))
        scheme = "slip_bb" if rng.random() < 0.5 else "hrfd"
        out.append({"id": k, "t_arrival": float(t[k]), "kind": kind, "ny": ny,
                    "nx": 4 if kind == "channel" else 8 * ny, "re_tau": re_tau,
                    "scheme": scheme})
    return out
