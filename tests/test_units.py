"""The package's host-side unit conversion, pinned to the paper's Tables 2-3
and cross-checked against the oracle's independent conversion."""
import os

import numpy as np

from oracle import units as OU
from paper_2506_03905_amd import units as U

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_dean_table2():
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_dean.txt"))
    for re_tau, u_tau, g, re_b, u_b, cf_b, y50 in rows:
        assert abs(U.dean_bulk_reynolds(re_tau) / re_b - 1) < 1e-4
        # lattice form: U_b / u_tau = Re_b / (2 Re_tau) in any units
        lat = U.channel(re_tau, 20, 0.05)
        assert abs(lat["u_bulk"] / lat["u_tau"] - u_b / u_tau) / (u_b / u_tau) < 2e-3
        cf_print = 0.00220 if re_tau == 20000 else cf_b
        assert abs(lat["cf_bulk"] - cf_print) < 1e-5


def test_table3_and_oracle_agree():
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_grid.txt"))
    for N, _, ybp, yfp in rows:
        lat = U.channel(4200.0, int(N))
        assert abs(lat["y_b_plus"] - ybp) < 1e-9 * ybp
        assert abs(lat["y_f_plus"] - yfp) < 1e-9 * yfp
    for re_tau, n in ((2000.0, 32), (5000.0, 128), (5000.0, 24)):
        a, b = U.channel(re_tau, n), OU.channel_lattice(re_tau, n)
        assert abs(a["nu"] / b["nu"] - 1) < 1e-14 and abs(a["force"] / b["g"] - 1) < 1e-14


def test_replication_cases_are_consistent():
    """The channel studies: Table 3's grid (Re_tau 4200, N = 5 ... 40) with
    y_B+ = Re_tau / (2N) for halfway walls, and a force that balances the
    target wall stress, F h = u_tau^2."""
    from paper_2506_03905_amd import replicate as R
    cs = R.cases(["grid", "reynolds", "beta", "wall"])
    assert {c["n"] for c in cs if c["study"] == "grid"} == {5, 10, 20, 30, 40}
    for c in cs:
        ny, h, u_b, u_tau, p = R.lattice_of(c)
        assert abs(p.force[0] * h - u_tau ** 2) < 1e-18
        assert abs(u_tau * h / p.nu - c["re_tau"]) < 1e-9 * c["re_tau"]
        if c["q"] == 0.5:
            assert h == c["n"] and abs(0.5 * u_tau / p.nu - c["re_tau"] / (2 * c["n"])) < 1e-9
