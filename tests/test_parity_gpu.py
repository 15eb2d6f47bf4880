"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP64 storage is compared element by element; FP32 / FP16 / BF16 storage by
relative L2 error.  Inputs come from the seeded generators in
paper_2506_03905_amd.inputs and are handed to both sides.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2506_03905_amd import inputs, units

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2506_03905_amd.lbm")


def _torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(q, nx, ny, nz, *, scheme, u0, nu, force=(0, 0, 0), flow=O.CHANNEL, plate_start=0,
          u_inlet=0.0, sa_on=1, law=O.REICHARDT, beta=0.28, precision="f64",
          wall_u_top=(0, 0, 0), collision=O.BGK, oracle_shape=None, oracle_u0=None,
          store_shift_u=0.0, bb_interp=0, wall_dist=0.5):
    _torch_gpu()
    oq = dict(nx=nx, ny=ny, nz=nz)
    if oracle_shape is not None:
        oq = dict(zip(("nx", "ny", "nz"), oracle_shape))
    op = O.params(q=q, **oq, flow=flow, scheme=scheme, law=law, sa_on=sa_on,
                  plate_start=plate_start, nu=nu, force=force, u_inlet=u_inlet, beta=beta,
                  wall_u_top=wall_u_top, collision=collision, bb_interp=bb_interp,
                  wall_dist=wall_dist)
    o = O.Oracle(op, u0 if oracle_u0 is None else oracle_u0)
    gp = L.lbm_params_default(precision=L.PRECISION[precision], flow=flow, scheme=scheme,
                              law=law, sa_on=sa_on, plate_start=plate_start, nu=nu,
                              force=force, u_inlet=u_inlet, beta=beta, wall_u_top=wall_u_top,
                              reduce_every=0, collision=collision, store_shift_u=store_shift_u,
                              bb_interp=bb_interp, wall_dist=wall_dist)
    g = L.Lattice(q, nx, ny, nz, gp)
    g.lbm_set_velocity(u0)
    return o, g


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _compare_f64(o, g, tol=1e-11):
    rho_g, u_g, nut_g = g.lbm_moments()
    assert _rel(u_g, o.u()) < tol, _rel(u_g, o.u())
    assert np.abs(rho_g - o.rho()).max() < tol
    if o.p.sa_on:
        assert _rel(g.lbm_nu_tilde(), o.nt()) < tol
        assert _rel(nut_g, o.nut()) < tol
    wg, wo = g.lbm_wall(), o.wall()
    if o.nwall:
        assert _rel(wg["utau"], wo["utau"]) < tol
        assert _rel(wg["uw"], wo["uw"]) < max(tol, 1e-12)


def _channel_u0(q, nx, ny, nz, ub, amp=1e-3, seed=0):
    D = 2 if q == 9 else 3
    return inputs.channel_velocity(seed, D, nz, ny, nx, ub, amp)


@pytest.mark.parametrize("steps", [1, 2, 3, 10, 51])
def test_d2q9_channel_slip_bb_f64(steps):
    lat = units.channel(2000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 20, 0, 0))
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


@pytest.mark.parametrize("scheme", [O.HRFD, O.CAI_DEGRIGNY])
@pytest.mark.parametrize("law", [O.REICHARDT, O.SA_LAW])
def test_d2q9_channel_hrfd_f64(law, scheme):
    lat = units.channel(4200.0, 10)
    nx, ny = 6, 20
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=lat["nu"], law=law,
                 force=(lat["force"], 0, 0))
    o.step(40)
    g.lbm_step(40)
    _compare_f64(o, g)


def test_d2q9_poiseuille_fixed_bb_f64():
    tau, H = 0.8, 16
    nu = (tau - 0.5) / 3
    g_ = 8 * nu * 1e-3 / H ** 2
    u0 = np.zeros((2, 1, H, 3))
    o, g = _pair(9, 3, H, 1, scheme=O.BB_FIXED, u0=u0, nu=nu, force=(g_, 0, 0), sa_on=0,
                 wall_u_top=(0.002, 0, 0))
    o.step(333)
    g.lbm_step(333)
    _compare_f64(o, g)


@pytest.mark.parametrize("steps", [1, 2, 25])
def test_d3q19_channel_slip_bb_f64(steps):
    lat = units.channel(5000.0, 6)
    nx, ny, nz = 5, 12, 4
    u0 = _channel_u0(19, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0))
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("collision", [O.BGK, O.CM])
def test_oblique_body_force_f64(q, collision):
    """A body force with components along every axis: the Guo term of every
    direction (Sec. 2.1) and the half-force shift of u (eq. 5), element-wise
    against the oracle; the row mapping (nx = 256) and a ragged tail (nx = 37)."""
    lat = units.channel(2000.0, 8)
    g0 = lat["force"] * 10
    for nx in (37, 256):
        ny, nz = 16, (1 if q == 9 else 3)
        force = (g0, 0.3 * g0, 0.0) if q == 9 else (g0, 0.3 * g0, -0.2 * g0)
        u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"])
        o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"], force=force,
                     collision=collision)
        o.step(15)
        g.lbm_step(15)
        _compare_f64(o, g)


@pytest.mark.parametrize("q", [9, 19])
def test_storage_shift_f64(q):
    """FP64 storage of f - f_eq(rho0, (U, 0, 0)) reproduces the oracle (which
    stores f): the offsets of the gather, the store, the initialisation and
    the exports agree, across both step parities and a row-mapped lattice."""
    lat = units.channel(2000.0, 8)
    nx, ny, nz = 256, 16, (1 if q == 9 else 3)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), store_shift_u=lat["u_bulk"])
    for n in (1, 1, 9):
        o.step(n)
        g.lbm_step(n)
        _compare_f64(o, g)
        assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


@pytest.mark.parametrize("interp,q", [(O.IBB_BOUZIDI, 0.3), (O.IBB_BOUZIDI, 0.7),
                                      (O.IBB_YU, 0.5), (O.IBB_YU, 0.25)])
@pytest.mark.parametrize("steps", [1, 2, 41])
def test_d2q9_interpolated_bounce_back_f64(interp, q, steps):
    """Slip-velocity bounce-back with the walls q from the first nodes:
    Bouzidi's rule (eq. 36, both branches) and Yu's (eq. 37)."""
    lat = units.channel(3000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 20, 0, 0), collision=O.CM, bb_interp=interp, wall_dist=q)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)
    assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


@pytest.mark.parametrize("interp,q", [(O.IBB_BOUZIDI, 0.2), (O.IBB_YU, 0.8)])
def test_interpolated_couette_fixed_walls_f64(interp, q):
    """Laminar Couette flow with a moving top wall off the halfway position."""
    ny, U = 10, 0.01
    nu = 0.1
    u0 = np.zeros((2, 1, ny, 3))
    o, g = _pair(9, 3, ny, 1, scheme=O.BB_FIXED, u0=u0, nu=nu, sa_on=0,
                 wall_u_top=(U, 0, 0), bb_interp=interp, wall_dist=q)
    o.step(500)
    g.lbm_step(500)
    _compare_f64(o, g)


@pytest.mark.parametrize("interp", [O.IBB_BOUZIDI, O.IBB_YU])
def test_d3q19_interpolated_row_block_f64(interp):
    """D3Q19 with interpolated links on the row-mapped, LDS-staged kernel."""
    lat = units.channel(5000.0, 8)
    nx, ny, nz = 128, 16, 4
    u0 = _channel_u0(19, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), collision=O.CM, bb_interp=interp, wall_dist=0.35)
    o.step(9)
    g.lbm_step(9)
    _compare_f64(o, g)


@pytest.mark.parametrize("q", [0.5, 0.3])
@pytest.mark.parametrize("steps", [1, 2, 60])
def test_d2q9_plate_yu_f64(q, steps):
    """The flat plate with Yu's rule (the paper's choice there), including the
    leading-edge links and the outlet corner."""
    nx, ny, U = 300, 12, 0.05
    u0 = inputs.channel_velocity(3, 2, 1, ny, nx, U, 1e-3)
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=0.03, flow=O.PLATE, plate_start=40,
                 u_inlet=U, bb_interp=O.IBB_YU, wall_dist=q)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


@pytest.mark.parametrize("collision", [O.BGK, O.CM])
@pytest.mark.parametrize("steps", [1, 2, 25])
def test_d3q19_row_block_odd_step_f64(steps, collision):
    """Channel rows that fit one block (nx % 64 == 0, ny % 8 == 0): the odd
    steps run one block per row with the x-shifted populations exchanged
    through LDS."""
    lat = units.channel(5000.0, 8)
    nx, ny, nz = 128, 16, 4
    u0 = _channel_u0(19, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), collision=collision)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)
    assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD, O.CAI_DEGRIGNY])
def test_d2q9_row_block_odd_step_f64(scheme):
    lat = units.channel(4200.0, 8)
    nx, ny = 192, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=lat["nu"], force=(lat["force"], 0, 0),
                 collision=O.CM)
    o.step(31)
    g.lbm_step(31)
    _compare_f64(o, g)


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD, O.CAI_DEGRIGNY])
@pytest.mark.parametrize("steps", [1, 2, 60])
def test_d2q9_plate_f64(scheme, steps):
    nx, ny, U = 300, 12, 0.05
    u0 = inputs.channel_velocity(3, 2, 1, ny, nx, U, 1e-3)
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=0.03, flow=O.PLATE, plate_start=40,
                 u_inlet=U)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


def test_populations_export_matches_oracle():
    lat = units.channel(2000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"])
    for n in (1, 1, 5):  # odd layout, even layout, odd layout
        o.step(n)
        g.lbm_step(n)
        assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


def test_residual_reduction_matches_oracle_definition():
    lat = units.channel(2000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"])
    r0 = g.lbm_residual()
    o.step(20)
    g.lbm_step(20)
    r = g.lbm_residual()
    uo0 = u0.reshape(2, -1)
    uo = o.u().reshape(2, -1)
    tot = o.totals()
    assert abs(r["mass"] - tot[0]) < 1e-12 * tot[0]
    assert np.allclose(r["momentum"][:2], tot[1:3], rtol=1e-11, atol=1e-18)
    l2 = np.linalg.norm(uo - uo0) / (20 * np.linalg.norm(uo))
    assert abs(r["l2_du_rel"] / l2 - 1) < 1e-9
    assert abs(r["mean_u_tau"] / o.wall()["utau"].mean() - 1) < 1e-12
    assert r["nan_flag"] == 0.0 and r0["step"] == 0 and r["steps_since_previous"] == 20


@pytest.mark.parametrize("precision,shift,tol,guard", [("f64", 1.0, 1e-11, None)] + [v[:4] for v in [
    ("f32", 0.0, 1e-4, None), ("f16", 1.0, 1e-3, None), ("f16", 0.0, None, 2e-2),
    ("bf16", 1.0, None, 2e-2), ("bf16", 0.0, None, 2e-1)]])
def test_d3q19_channel_reduced_precision(precision, shift, tol, guard):
    """A small perturbed D3Q19 channel (16 x 24 x 8, 100 steps) in every
    storage type against the FP64 oracle: relative L2 of u, u_tau and Cf
    (targets as above; FP64 storage with the shift as a control)."""
    lat = units.channel(5000.0, 12)
    nx, ny, nz = 16, 24, 8
    u0 = _channel_u0(19, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"], 0, 0), precision=precision,
                 store_shift_u=shift * lat["u_bulk"])
    o.step(100)
    g.lbm_step(100)
    _, ug, _ = g.lbm_moments()
    uo = o.u()
    ut_g, ut_o = g.lbm_wall()["utau"], o.wall()["utau"]
    errs = {"u_rel_l2": float(np.linalg.norm(ug - uo) / np.linalg.norm(uo)),
            "u_tau_rel_l2": float(np.linalg.norm(ut_g - ut_o) / np.linalg.norm(ut_o)),
            "cf_rel_l2": float(np.linalg.norm(ut_g ** 2 - ut_o ** 2) / np.linalg.norm(ut_o ** 2))}
    _report(f"16x24x8 3-d-perturbed {precision} shift={shift:g} steps=100", errs)
    _check_precision(errs, tol, guard)


@pytest.mark.parametrize("interp,q", [(O.IBB_HALFWAY, 0.5), (O.IBB_YU, 0.3)])
def test_checkpoint_roundtrip_bitwise(interp, q):
    """Save, continue, load into a second lattice, continue: bitwise equal
    (the wall cells' kept populations of the interpolated links included)."""
    lat = units.channel(2000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    kw = dict(scheme=O.BB_SLIP, u0=u0, nu=lat["nu"], precision="f32", bb_interp=interp,
              wall_dist=q)
    _, g = _pair(9, nx, ny, 1, **kw)
    _, h = _pair(9, nx, ny, 1, **kw)
    g.lbm_step(7)
    blob = g.lbm_save()
    g.lbm_step(9)
    h.lbm_load(blob)
    h.lbm_step(9)
    assert np.array_equal(g.lbm_moments()[1], h.lbm_moments()[1])
    assert np.array_equal(g.lbm_populations(), h.lbm_populations())


def test_divergence_is_reported():
    _torch_gpu()
    p = L.lbm_params_default(precision=L.LBM_F64, scheme=L.LBM_WALL_FIXED_BB, sa_on=0, nu=1e-3,
                             reduce_every=0)
    g = L.Lattice(9, 4, 8, 1, p)
    u = np.zeros((2, 1, 8, 4))
    u[0, 0, 3, 1] = np.nan
    g.lbm_set_velocity(u)
    g.lbm_step(2)
    r = g.lbm_residual()
    assert r["rc"] == L.LBM_EDIVERGED and r["nan_flag"] == 1.0
    with pytest.raises(L.LbmError):
        g.lbm_step(1)


# ------------------------------------------------- central-moment collision ---
@pytest.mark.parametrize("steps", [1, 2, 31])
def test_d2q9_channel_cm_f64(steps):
    lat = units.channel(2000.0, 8)
    nx, ny = 4, 16
    u0 = _channel_u0(9, nx, ny, 1, lat["u_bulk"])
    o, g = _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 20, 0, 0), collision=O.CM)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


@pytest.mark.parametrize("steps", [1, 2, 20])
def test_d3q19_channel_cm_f64(steps):
    lat = units.channel(5000.0, 6)
    nx, ny, nz = 5, 12, 4
    u0 = _channel_u0(19, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), collision=O.CM)
    o.step(steps)
    g.lbm_step(steps)
    _compare_f64(o, g)


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD])
def test_d2q9_plate_cm_low_viscosity_f64(scheme):
    """The plate at the viscosity of the 2048 x 256 workload (tau - 1/2 = 6e-5)."""
    nx, ny, U = 260, 24, 0.1
    u0 = inputs.channel_velocity(5, 2, 1, ny, nx, U, 0.0)
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=1.984e-5, flow=O.PLATE,
                 plate_start=16, u_inlet=U, collision=O.CM)
    o.step(150)
    g.lbm_step(150)
    _compare_f64(o, g, tol=1e-10)


# ------------------------------------------------------ configuration cases ---
def _cfg1(collision):
    lat = units.channel(2000.0, 32, 0.05)
    nx, ny = 4, 64
    u0 = inputs.channel_velocity(0, 2, 1, ny, nx, 0.0, 1e-3)
    return _pair(9, nx, ny, 1, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"], 0, 0), collision=collision)


def test_config1_bgk_parity_then_divergence():
    """D2Q9 4 x 64 channel, FP64, BGK, rest + seeded 1e-3 perturbation: parity
    element-wise while the run is finite; BGK with slip-velocity bounce-back
    then diverges near step 1450 on both sides, and the GPU reduction says so."""
    o, g = _cfg1(O.BGK)
    o.step(1000)
    g.lbm_step(1000)
    _compare_f64(o, g, tol=1e-9)
    o.step(2000)
    g.lbm_step(2000)
    assert not np.all(np.isfinite(o.u()))
    assert g.lbm_residual()["rc"] == L.LBM_EDIVERGED


def test_config1_cm_full_run_parity():
    """The same workload with the paper's central-moment collision: 20000
    steps, element-wise FP64 parity at the end."""
    o, g = _cfg1(O.CM)
    for _ in range(4):
        o.step(5000)
        g.lbm_step(5000)
    _compare_f64(o, g, tol=1e-9)
    assert g.lbm_residual()["nan_flag"] == 0.0


# ------------------------------------------------------------------ precision --
# Targets (relative L2 against the FP64 oracle, on u, u_tau and Cf alike):
# 1e-4 for FP32 storage and arithmetic, 1e-3 for FP16 storage with FP32
# arithmetic.  The FP16 layout that carries the target stores the deviation
# from the bulk equilibrium, f - f_eq(rho0, (U_b, 0, 0)); FP16 with f - w rho0
# and BF16 are reported (the report records every case) with a regression
# guard only: FP16's 11-bit significand applied to the velocity-carrying part
# of f - w rho0 cannot hold 1e-3 on Cf (measured 2e-3 after 100 steps).
TARGET = {"f32": 1e-4, "f16": 1e-3}
# (precision, storage shift in units of U_b, tolerance or None, regression guard)
VARIANTS = [("f32", 0.0, TARGET["f32"], None), ("f16", 1.0, TARGET["f16"], None),
            ("f16", 0.0, None, 2e-2), ("bf16", 1.0, None, 2e-2), ("bf16", 0.0, None, 2e-1)]


def _report(key, vals):
    """Append the measured errors to $LBM_REPORT_DIR/precision_report.jsonl
    when that directory is given."""
    import json
    import os
    d = os.environ.get("LBM_REPORT_DIR")
    if d and os.path.isdir(d):
        with open(os.path.join(d, "precision_report.jsonl"), "a") as fh:
            fh.write(json.dumps({"case": key, **vals}) + "\n")


def _check_precision(errs, tol, guard):
    assert all(np.isfinite(v) for v in errs.values()), errs
    if tol is not None:
        assert max(errs["u_rel_l2"], errs["u_tau_rel_l2"], errs["cf_rel_l2"]) < tol, errs
    else:
        assert max(errs["u_rel_l2"], errs["u_tau_rel_l2"], errs["cf_rel_l2"]) < guard, errs


def _column_oracle(ny, steps, amp, seed=0):
    """The oracle's single column (1 x ny x 1) of the x/z-invariant channel
    at Re_tau 5000 (ny/2 cells per half channel) from Dean's bulk velocity
    plus, when amp > 0, a seeded perturbation that varies along y only."""
    lat = units.channel(5000.0, ny // 2, 0.05)
    u0c = inputs.channel_velocity(0, 3, 1, ny, 1, lat["u_bulk"], 0.0)
    if amp > 0:
        u0c += inputs.perturbation(seed, 3, 1, ny, 1, amp)
    op = O.params(q=19, nx=1, ny=ny, nz=1, scheme=O.BB_SLIP, nu=lat["nu"],
                  force=(lat["force"], 0, 0))
    o = O.Oracle(op, u0c)
    o.step(steps)
    return lat, u0c, o


def _invariant_channel(nx, ny, nz, precision, steps, shift=0.0, amp=0.0, label=""):
    """The GPU on the full nx x ny x nz lattice against the oracle column:
    every (x, z) column must be bitwise identical (the same arithmetic), and
    the column is compared with the oracle's."""
    lat, u0c, o = _column_oracle(ny, steps, amp)
    u0 = np.broadcast_to(u0c, (3, nz, ny, nx))
    gp = L.lbm_params_default(precision=L.PRECISION[precision], scheme=L.LBM_WALL_SLIP_BB,
                              nu=lat["nu"], force=(lat["force"], 0, 0), reduce_every=0,
                              store_shift_u=shift * lat["u_bulk"], u_ref=lat["u_bulk"])
    g = L.Lattice(L.LBM_D3Q19, nx, ny, nz, gp)
    g.lbm_set_velocity(u0)
    del u0
    g.lbm_step(steps)
    _, ug, _ = g.lbm_moments("f64" if precision == "f64" else "f32")
    col = ug[:, 0, :, 0].astype(np.float64)
    assert np.array_equal(ug, np.broadcast_to(ug[:, :1, :, :1], ug.shape))
    del ug
    uo = o.u()[:, 0, :, 0]
    w = g.lbm_wall()
    ut_o = o.wall()["utau"]                      # bottom cell, top cell
    ref = np.repeat(ut_o, w["utau"].size // 2)   # wall cells: bottom row, then top row
    cf_o = 2.0 * (ref / lat["u_bulk"]) ** 2
    errs = {"u_rel_l2": float(np.linalg.norm(col - uo) / np.linalg.norm(uo)),
            "u_tau_rel_l2": float(np.linalg.norm(w["utau"] - ref) / np.linalg.norm(ref)),
            "cf_rel_l2": float(np.linalg.norm(w["cf"] - cf_o) / np.linalg.norm(cf_o))}
    _report(f"{nx}x{ny}x{nz} {label}{precision} shift={shift:g} steps={steps}", errs)
    return errs


def test_config3_full_size_invariance_f32():
    """512 x 256 x 256 D3Q19 FP32 (the benchmark's lattice and launch) from the
    Dean start, 1000 steps: x/z-invariant, and equal to the oracle's single
    column within the FP32 target on u, u_tau and Cf."""
    _torch_gpu()
    _check_precision(_invariant_channel(512, 256, 256, "f32", 1000), TARGET["f32"], None)


@pytest.mark.parametrize("precision,shift,tol,guard", VARIANTS)
def test_config4_full_size_precision(precision, shift, tol, guard):
    """768 x 384 x 384 D3Q19 with FP32/FP16/BF16 storage over 1000 steps
    against the FP64 oracle column: relative L2 of u, of u_tau per wall cell
    and of Cf = 2 (u_tau / U_b)^2."""
    _torch_gpu()
    _check_precision(_invariant_channel(768, 384, 384, precision, 1000, shift=shift), tol, guard)


# Over 20 000 steps the FP32 arithmetic drifts linearly in time (2.2e-5 at
# 2000 steps, 1.9e-4 at 20 000 before the momentum compensation of the
# collision; 3.5e-4 / Cf 6e-4 after it): the body force (9e-8 per step here)
# is a few ulp of the momentum, and the rounding of the FP32 momentum sums
# leaves about 1 % of it per step.  The targets are not met over that window.
_LONG_XFAIL = pytest.mark.xfail(strict=True, reason=(
    "measured over 20 000 steps: FP32 u 3.5e-4, Cf 6.0e-4 (target 1e-4); FP16 with the "
    "storage shift Cf 1.4e-3 (target 1e-3): linear drift from the FP32 momentum sums"))


@pytest.mark.parametrize("steps", [1000, 20000])
@pytest.mark.parametrize("precision,shift,tol,guard", VARIANTS)
def test_config4_subsample_long_window(precision, shift, tol, guard, steps, request):
    """The 96 x 48 x 48 subsample (24 cells per half channel, y_B+ = 104) from
    Dean's velocity with a seeded +-1e-3 perturbation along y, over 1000 and
    20 000 steps, against the FP64 oracle column."""
    _torch_gpu()
    if steps == 20000 and tol is not None:
        request.applymarker(_LONG_XFAIL)
    errs = _invariant_channel(96, 48, 48, precision, steps, shift=shift, amp=1e-3,
                              label="y-perturbed ")
    _check_precision(errs, tol, guard)


_SUB = {}


def _subsample_oracle(steps):
    """The oracle on the 96 x 48 x 48 subsample with a seeded 3-D +-1e-3
    perturbation (Re_tau 5000, 24 cells per half channel).  With nu_tilde
    starting at 3 nu the transverse velocity grows in this flow (1e-3 to 0.1
    within ~750 steps, NaN by 1000 in the oracle itself), so this case is
    compared over 60 steps, before the growth."""
    if steps not in _SUB:
        lat = units.channel(5000.0, 24, 0.05)
        nx, ny, nz = 96, 48, 48
        u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], 1e-3)
        op = O.params(q=19, nx=nx, ny=ny, nz=nz, nu=lat["nu"], force=(lat["force"], 0, 0),
                      scheme=O.BB_SLIP)
        o = O.Oracle(op, u0)
        o.step(steps)
        _SUB[steps] = (lat, u0, o.u(), o.wall()["utau"])
    return _SUB[steps]


@pytest.mark.parametrize("precision,shift,tol,guard", VARIANTS)
def test_config4_subsample_3d_perturbed(precision, shift, tol, guard):
    """96 x 48 x 48 D3Q19 with a seeded 3-D perturbation (a full field, no
    symmetry used) against the FP64 oracle over 60 steps: relative L2 of u,
    of u_tau per wall cell and of Cf = 2 (u_tau / U_b)^2."""
    _torch_gpu()
    steps = 60
    lat, u0, uo, ut_o = _subsample_oracle(steps)
    gp = L.lbm_params_default(precision=L.PRECISION[precision], scheme=L.LBM_WALL_SLIP_BB,
                              nu=lat["nu"], force=(lat["force"], 0, 0), reduce_every=0,
                              store_shift_u=shift * lat["u_bulk"], u_ref=lat["u_bulk"])
    g = L.Lattice(L.LBM_D3Q19, 96, 48, 48, gp)
    g.lbm_set_velocity(u0)
    g.lbm_step(steps)
    _, ug, _ = g.lbm_moments()
    w = g.lbm_wall()
    cf_o = 2.0 * (ut_o / lat["u_bulk"]) ** 2
    errs = {"u_rel_l2": float(np.linalg.norm(ug - uo) / np.linalg.norm(uo)),
            "u_tau_rel_l2": float(np.linalg.norm(w["utau"] - ut_o) / np.linalg.norm(ut_o)),
            "cf_rel_l2": float(np.linalg.norm(w["cf"] - cf_o) / np.linalg.norm(cf_o))}
    _report(f"96x48x48 3-d-perturbed {precision} shift={shift:g} steps={steps}", errs)
    _check_precision(errs, tol, guard)


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD])
def test_config2_plate_cf_profile_f32(scheme):
    """Flat plate at the plate workload's viscosity (tau - 1/2 = 6e-5, U = 0.1,
    CM collision) on a 256 x 32 lattice, FP32 storage and arithmetic against
    the FP64 oracle after 2000 steps: relative L2 of u and of the skin
    friction profile Cf(x) = 2 (u_tau / U)^2, and the integrated error of the
    plate's second half, int |Cf - Cf_ref| dx / int Cf_ref dx (trapezoid)."""
    nx, ny, U, ps = 256, 32, 0.1, 8
    nu = U * 992 / 5e6
    u0 = inputs.channel_velocity(0, 2, 1, ny, nx, U, 0.0)
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=nu, flow=O.PLATE, plate_start=ps,
                 u_inlet=U, collision=O.CM, precision="f32")
    o.step(2000)
    g.lbm_step(2000)
    _, ug, _ = g.lbm_moments()
    uo = o.u()
    err_u = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    cf_g = 2 * (g.lbm_wall()["utau"] / U) ** 2
    cf_o = 2 * (o.wall()["utau"] / U) ** 2
    err_cf = np.linalg.norm(cf_g - cf_o) / np.linalg.norm(cf_o)
    half = (nx - ps) // 2
    eps = np.trapezoid(np.abs(cf_g - cf_o)[half:]) / np.trapezoid(cf_o[half:])
    _report(f"plate 256x32 f32 {'hrfd' if scheme == O.HRFD else 'slip_bb'} steps=2000",
            {"u_rel_l2": err_u, "cf_rel_l2": err_cf, "cf_integrated": eps})
    assert err_u < 1e-4 and err_cf < 1e-4 and eps < 1e-4, (err_u, err_cf, eps)


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD])
def test_config2_full_size_plate_f64(scheme):
    """2048 x 256 flat plate, CM collision, 64-cell slip leading section,
    U = 0.1, Re = 5e6 per L_ref = 992 cells: FP64 parity after 40 steps."""
    nx, ny, U = 2048, 256, 0.1
    nu = U * 992 / 5e6
    u0 = inputs.channel_velocity(0, 2, 1, ny, nx, U, 0.0)
    o, g = _pair(9, nx, ny, 1, scheme=scheme, u0=u0, nu=nu, flow=O.PLATE, plate_start=64,
                 u_inlet=U, collision=O.CM)
    o.step(40)
    g.lbm_step(40)
    _compare_f64(o, g, tol=1e-10)


@pytest.mark.parametrize("q,nx,ny,nz", [(9, 4, 16, 1), (19, 256, 16, 3), (9, 384, 16, 1)])
def test_fused_reduction_matches_oracle(q, nx, ny, nz):
    """The reduction carried by the even channel step (reduce_every = 10:
    steps 10 and 20, on a flat and on row-mapped lattices): mass, momentum,
    mean u_tau and the residual ||u^20 - u^10|| / (10 ||u^20||) against the
    oracle's fields."""
    lat = units.channel(2000.0, 8)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"])
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0))
    gp = L.lbm_params_default(precision=L.LBM_F64, scheme=L.LBM_WALL_SLIP_BB, nu=lat["nu"],
                              force=(lat["force"] * 10, 0, 0), reduce_every=10)
    g = L.Lattice(q, nx, ny, nz, gp)
    g.lbm_set_velocity(u0)
    o.step(10)
    u10 = o.u().reshape(o.D, -1).copy()
    o.step(10)
    g.lbm_step(20)
    r = g.lbm_residual()  # the step-20 reduction, not a new one
    u20 = o.u().reshape(o.D, -1)
    tot = o.totals()
    assert r["step"] == 20 and r["steps_since_previous"] == 10 and r["nan_flag"] == 0.0
    assert abs(r["mass"] - tot[0]) < 1e-12 * tot[0]
    D = o.D
    assert np.allclose(r["momentum"][:D], tot[1:1 + D], rtol=1e-11, atol=1e-16)
    l2 = np.linalg.norm(u20 - u10) / (10 * np.linalg.norm(u20))
    assert abs(r["l2_du_rel"] / l2 - 1) < 1e-9
    ut = o.wall()["utau"]
    assert abs(r["mean_u_tau"] / ut.mean() - 1) < 1e-12
    assert r["d_u_tau_rel"] >= 0.0


@pytest.mark.parametrize("flow,reduce_every", [("channel", 2), ("channel", 3), ("plate", 2)])
def test_lbm_step_reports_divergence_by_itself(flow, reduce_every):
    """A NaN in the start field: lbm_step's own periodic reductions (fused
    in the channel's even steps, standalone otherwise) raise the divergence
    flag, which a later lbm_step call returns as LBM_EDIVERGED without
    lbm_residual ever being called."""
    torch = _torch_gpu()
    kw = dict(precision=L.LBM_F64, scheme=L.LBM_WALL_SLIP_BB, sa_on=1, nu=1e-3,
              reduce_every=reduce_every)
    nx, ny = (4, 16) if flow == "channel" else (40, 12)
    if flow == "plate":
        kw.update(flow=L.LBM_FLOW_PLATE, plate_start=6, u_inlet=0.05, collision=L.LBM_COLL_CM)
    g = L.Lattice(9, nx, ny, 1, L.lbm_params_default(**kw))
    u = np.full((2, 1, ny, nx), 0.01)
    u[0, 0, 5, 2] = np.nan
    g.lbm_set_velocity(u)
    try:
        g.lbm_step(6)  # may already see an earlier reduction's flag
    except L.LbmError as e:
        assert e.code == L.LBM_EDIVERGED
    torch.cuda.synchronize()
    with pytest.raises(L.LbmError) as ei:
        g.lbm_step(1)
    assert ei.value.code == L.LBM_EDIVERGED
    # a healthy lattice with the same reductions keeps stepping
    h = L.Lattice(9, nx, ny, 1, L.lbm_params_default(**kw))
    h.lbm_set_velocity(np.full((2, 1, ny, nx), 0.01))
    h.lbm_step(6)
    torch.cuda.synchronize()
    h.lbm_step(6)
    assert h.steps == 12


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("q,nx,ny,nz,collision", [(19, 512, 16, 4, O.BGK), (19, 512, 16, 4, O.CM),
                                                  (9, 768, 16, 1, O.BGK), (19, 768, 8, 2, O.BGK)])
def test_row_map_multi_block_perturbed_f64(q, nx, ny, nz, collision):
    """Rows spanning two or three 256-thread blocks (as at 512 x 256 x 256),
    with a seeded +-1e-3 perturbation so that every column differs: the
    staged odd step's pushes across block edges and the even step, element-
    wise against the oracle after 1, 2 and 9 more steps (both parities):
    u, nu_tilde, nu_t, u_tau, u_w and the populations."""
    lat = units.channel(5000.0, ny // 2)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"], amp=1e-3, seed=11)
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), collision=collision)
    for n in (1, 1, 9):
        o.step(n)
        g.lbm_step(n)
        _compare_f64(o, g)
        assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


@pytest.mark.parametrize("q,nx,ny,nz", [(19, 320, 16, 4), (9, 448, 16, 1)])
def test_row_map_ragged_last_block_f64(q, nx, ny, nz):
    """Rows of two blocks whose second block is partly beyond the row (64 and
    192 active columns of 256): the staged odd step's pushes inside that
    block, across its edge and through the periodic wrap, element-wise
    against the oracle after 1, 2 and 9 more steps."""
    lat = units.channel(5000.0, ny // 2)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"], amp=1e-3, seed=13)
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0))
    for n in (1, 1, 9):
        o.step(n)
        g.lbm_step(n)
        _compare_f64(o, g)
        assert np.abs(g.lbm_populations() - o.f()).max() < 1e-13


def test_zero_steps_leave_the_state_alone():
    """lbm_step(0) takes no step: the step count, populations and moments stay
    bitwise the same."""
    lat = units.channel(5000.0, 8)
    u0 = _channel_u0(19, 128, 16, 4, lat["u_bulk"], amp=1e-3, seed=5)
    _, g = _pair(19, 128, 16, 4, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"], force=(lat["force"], 0, 0))
    g.lbm_step(3)
    f0, (_, u0g, _) = g.lbm_populations(), g.lbm_moments()
    g.lbm_step(0)
    assert g.lbm_steps() == 3
    assert np.array_equal(g.lbm_populations(), f0)
    assert np.array_equal(g.lbm_moments()[1], u0g)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_rest_state_stays_at_rest(precision):
    """No flow and no force on the row-mapped D3Q19 channel: the populations
    stay at equilibrium, so u stays exactly 0 and the wall function returns
    u_tau = 0 (a zero velocity at F gives a zero friction velocity); nu_tilde
    decays by destruction alone, as in the oracle."""
    nx, ny, nz = 128, 16, 4
    lat = units.channel(5000.0, ny // 2)
    u0 = np.zeros((3, nz, ny, nx))
    o, g = _pair(19, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"], precision=precision)
    for n in (1, 1, 8):
        o.step(n)
        g.lbm_step(n)
        _, ug, _ = g.lbm_moments()
        assert not np.any(ug), np.abs(ug).max()
        assert not np.any(g.lbm_wall()["utau"])
        tol = 1e-12 if precision == "f64" else 1e-6
        assert _rel_l2(g.lbm_nu_tilde(), o.nt()) < tol

@pytest.mark.parametrize("q,nx,ny,nz", [(19, 512, 16, 4), (9, 768, 16, 1)])
def test_row_map_multi_block_perturbed_f32(q, nx, ny, nz):
    """The same lattices with FP32 storage and arithmetic (the benchmark's
    kernel instantiation) against the FP64 oracle: relative L2 of u, nu_tilde,
    u_tau and the populations after 1, 2 and 30 more steps."""
    lat = units.channel(5000.0, ny // 2)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"], amp=1e-3, seed=12)
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), precision="f32")
    for n in (1, 1, 30):
        o.step(n)
        g.lbm_step(n)
        _, ug, _ = g.lbm_moments()
        errs = (_rel_l2(ug, o.u()), _rel_l2(g.lbm_nu_tilde(), o.nt()),
                _rel_l2(g.lbm_wall()["utau"], o.wall()["utau"]),
                _rel_l2(g.lbm_populations(), o.f()))
        assert max(errs) < 1e-5, errs



@pytest.mark.parametrize("precision,tol", [("f16", 1e-3), ("bf16", 1e-2)])
@pytest.mark.parametrize("q,nx,ny,nz", [(19, 512, 16, 4), (9, 768, 16, 1)])
def test_row_map_multi_block_perturbed_16bit(q, nx, ny, nz, precision, tol):
    """16-bit storage of the deviation from the bulk equilibrium (the layout
    whose interior rows run the collision on the stored values) on the same
    perturbed row-mapped lattices, against the FP64 oracle after 1, 2 and 30
    more steps: u, nu_tilde, u_tau and the populations within the FP16
    target (BF16: a guard ten times wider)."""
    lat = units.channel(5000.0, ny // 2)
    u0 = _channel_u0(q, nx, ny, nz, lat["u_bulk"], amp=1e-3, seed=12)
    o, g = _pair(q, nx, ny, nz, scheme=O.BB_SLIP, u0=u0, nu=lat["nu"],
                 force=(lat["force"] * 10, 0, 0), precision=precision,
                 store_shift_u=lat["u_bulk"])
    for n in (1, 1, 30):
        o.step(n)
        g.lbm_step(n)
        _, ug, _ = g.lbm_moments()
        errs = (_rel_l2(ug, o.u()), _rel_l2(g.lbm_nu_tilde(), o.nt()),
                _rel_l2(g.lbm_wall()["utau"], o.wall()["utau"]),
                _rel_l2(g.lbm_populations(), o.f()))
        _report(f"{q} {nx}x{ny}x{nz} row-map perturbed {precision} shift=1 steps+={n}",
                {"u_rel_l2": errs[0], "nt_rel_l2": errs[1], "u_tau_rel_l2": errs[2], "f_rel_l2": errs[3]})
        assert max(errs) < tol, errs

# ------------------------------------------------------------- plate, 50 000 steps --
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")
_PLATE = dict(nx=2048, ny=256, U=0.1, plate_start=64, lref=992)


def _plate_golden(scheme):
    path = __import__("os").path.join(GOLDEN, f"plate_2048x256_{scheme}.txt")
    if not __import__("os").path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_plate_reference.py {scheme})")
    rows = np.atleast_2d(np.loadtxt(path))
    return {int(r[0]): r[1:] for r in rows}


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["slip_bb", "hrfd"])
def test_config2_plate_50000_steps(scheme, precision):
    """The 2048 x 256 flat-plate workload (U = 0.1, Re = 5e6 per L_ref = 992
    cells, 64-column slip section, CM + SA) over 50 000 steps (~2.4
    flow-throughs), against the FP64 oracle's friction velocity stored at
    1000, 5000, 20 000 and 50 000 steps (tests/golden, written by
    make_plate_reference.py): relative L2 of Cf(x) = 2 (u_tau / U)^2 and the
    integrated error of the plate's second half (trapezoid)."""
    _torch_gpu()
    P = _PLATE
    gold = _plate_golden(scheme)
    gp = L.lbm_params_default(precision=L.PRECISION[precision], flow=L.LBM_FLOW_PLATE,
                              scheme=L.SCHEME[scheme], collision=L.LBM_COLL_CM,
                              nu=P["U"] * P["lref"] / 5e6, u_inlet=P["U"], u_ref=P["U"],
                              plate_start=P["plate_start"], reduce_every=0)
    g = L.Lattice(9, P["nx"], P["ny"], 1, gp)
    g.lbm_set_velocity(inputs.channel_velocity(0, 2, 1, P["ny"], P["nx"], P["U"], 0.0))
    done = 0
    tol = {"f64": 1e-9, "f32": 1e-4}[precision]
    for step in sorted(gold):
        g.lbm_step(step - done)
        done = step
        cf_g = g.lbm_wall()["cf"]  # 2 (u_tau / u_ref)^2 with u_ref = U
        cf_o = 2.0 * (gold[step] / P["U"]) ** 2
        err = float(np.linalg.norm(cf_g - cf_o) / np.linalg.norm(cf_o))
        half = cf_o.size // 2
        eps = float(np.trapezoid(np.abs(cf_g - cf_o)[half:]) / np.trapezoid(cf_o[half:]))
        _report(f"plate 2048x256 {precision} {scheme} steps={step}", {"cf_rel_l2": err, "cf_integrated": eps})
        assert err < tol and eps < tol, (step, err, eps)
