"""The oracle's row loops run on several threads (OpenMP): the result must be
bitwise the same as with one thread, on every path of the step (streaming,
wall links, interpolated links, HRFD, plate edges, SA, wall function)."""
import numpy as np
import pytest

import oracle as O
from paper_2506_03905_amd import inputs


def _run(p, u0, steps, threads):
    O.set_threads(threads)
    o = O.Oracle(p, u0)
    o.step(steps)
    w = o.wall()
    return o.f(), o.u(), o.nt(), w["utau"], w["uw"]


CASES = {
    "d3q19_channel_slip": (dict(q=19, nx=6, ny=12, nz=5, scheme=O.BB_SLIP, nu=2e-4,
                                force=(1e-6, 0, 0)), 3),
    "d3q19_channel_cm_yu": (dict(q=19, nx=5, ny=10, nz=4, scheme=O.BB_SLIP, nu=2e-4,
                                 force=(1e-6, 2e-7, 0), collision=O.CM, bb_interp=O.IBB_YU,
                                 wall_dist=0.3), 3),
    "d2q9_channel_hrfd": (dict(q=9, nx=8, ny=16, scheme=O.HRFD, nu=1e-4, force=(1e-6, 0, 0)), 2),
    "d2q9_plate_bouzidi": (dict(q=9, nx=40, ny=12, flow=O.PLATE, plate_start=6, scheme=O.BB_SLIP,
                                nu=1e-3, u_inlet=0.05, collision=O.CM, bb_interp=O.IBB_BOUZIDI,
                                wall_dist=0.7), 2),
    "d2q9_plate_cd": (dict(q=9, nx=40, ny=12, flow=O.PLATE, plate_start=6,
                           scheme=O.CAI_DEGRIGNY, nu=1e-3, u_inlet=0.05, collision=O.CM), 2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_threads_bitwise_equal(name):
    kw, D = CASES[name]
    p = O.params(**kw)
    u0 = inputs.channel_velocity(7, D, kw.get("nz", 1), kw["ny"], kw["nx"], 0.03, 1e-3)
    n0 = O.get_threads()
    try:
        one = _run(p, u0, 23, 1)
        many = _run(p, u0, 23, 7)
    finally:
        O.set_threads(n0)
    for a, b in zip(one, many):
        assert np.array_equal(a, b, equal_nan=True)
