"""Host-side unit conversion for the oracle's runs -- TEST INFRASTRUCTURE ONLY.

Written independently of the product package's own conversion; the tests pin
both against the paper's Table 2 and Table 3.

* Channel (Sec. 4.1.1): the body force is rho0 u_tau^2 / h along x; the bulk
  velocity follows Dean's correlation Re_b = (8/0.073)^(4/7) Re_tau^(8/7) with
  Re_b = U_b 2h / nu; the acoustic time step makes the lattice reference
  velocity Ma / sqrt(3) (Sec. 3.2, the relation for tau).
* Flat plate (Sec. 4.2.1): Re = U L_ref / nu per unit reference length.
"""
import math


def dean_re_b(re_tau: float) -> float:
    return (8.0 / 0.073) ** (4.0 / 7.0) * re_tau ** (8.0 / 7.0)


def table2_row(re_tau: float, nu: float = 1.5e-5, h: float = 1.0) -> dict:
    """Physical-unit quantities of Table 2 (rho0 = 1, nu = 1.5e-5, h = 1)."""
    u_tau = re_tau * nu / h
    re_b = dean_re_b(re_tau)
    u_b = re_b * nu / (2.0 * h)
    return {"u_tau": u_tau, "g": u_tau * u_tau / h, "re_b": re_b, "u_b": u_b,
            "cf_b": 2.0 * (u_tau / u_b) ** 2, "y50": 50.0 * nu / u_tau}


def channel_lattice(re_tau: float, n_half: int, ma: float = 0.05) -> dict:
    """Lattice parameters of a channel with n_half cells per half height."""
    u_b = ma / math.sqrt(3.0)
    ub_over_ut = dean_re_b(re_tau) / (2.0 * re_tau)
    u_tau = u_b / ub_over_ut
    nu = u_tau * n_half / re_tau
    return {"u_b": u_b, "u_tau": u_tau, "nu": nu, "g": u_tau * u_tau / n_half,
            "y_b_plus": 0.5 * u_tau / nu, "y_f_plus": 1.5 * u_tau / nu}


def plate_lattice(u_inf: float, re_per_lref: float, lref_cells: float) -> dict:
    return {"u_inf": u_inf, "nu": u_inf * lref_cells / re_per_lref}
