"""Host-side set-up: lattice parameters of the paper's two flows.

Channel (Sec. 4.1.1): the driving force is rho0 u_tau^2 / h in x; Dean's
correlation Re_b = (8/0.073)^(4/7) Re_tau^(8/7), Re_b = 2 U_b h / nu, gives the
bulk velocity; with an acoustic time step the lattice bulk velocity is
Ma / sqrt(3) (the relation for tau in Sec. 3.2).  h is the number of cells
per half channel.

Flat plate (Sec. 4.2.1): Re per unit reference length, U the inlet velocity,
L_ref in cells.
"""
import math


def dean_bulk_reynolds(re_tau: float) -> float:
    return (8.0 / 0.073) ** (4.0 / 7.0) * re_tau ** (8.0 / 7.0)


def channel(re_tau: float, cells_per_half: int, mach: float = 0.05) -> dict:
    """Lattice viscosity, body force and reference velocities of a channel."""
    u_bulk = mach / math.sqrt(3.0)
    re_b = dean_bulk_reynolds(re_tau)
    u_tau = u_bulk * 2.0 * re_tau / re_b
    h = float(cells_per_half)
    nu = u_tau * h / re_tau
    return {
        "nu": nu,
        "force": u_tau * u_tau / h,
        "u_bulk": u_bulk,
        "u_tau": u_tau,
        "tau": 0.5 + 3.0 * nu,
        "y_b_plus": 0.5 * u_tau / nu,
        "y_f_plus": 1.5 * u_tau / nu,
        "cf_bulk": 2.0 * (u_tau / u_bulk) ** 2,
    }


def plate(u_inf: float, re_per_lref: float, lref_cells: float) -> dict:
    nu = u_inf * lref_cells / re_per_lref
    return {"nu": nu, "u_inf": u_inf, "tau": 0.5 + 3.0 * nu}
