"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle (``oracle/``) against something other than
itself: exact lattice identities, closed-form steady states of the lattice
Boltzmann scheme, the paper's printed constants and tables, and limits of the
wall laws.  None of them re-types the formula under test.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import units as OU

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dims(q):
    return 2 if q == 9 else 3


# --------------------------------------------------------------------- P1 -----
@pytest.mark.parametrize("q", [9, 19])
def test_lattice_isotropy(q):
    """Lattice tables: weights sum to 1, odd moments vanish, second moment is
    c_s^2 I and the fourth is c_s^4 (dd + dd + dd) (Sec. 2.1, c_s^2 = 1/3)."""
    c, w, opp = O.lattice(q)
    D = _dims(q)
    c = c[:, :D].astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.abs(M2 - np.eye(D) / 3).max() < 1e-15
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-16
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(D)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(M4 - iso).max() < 1e-15
    assert np.all(c[opp] == -c)


# --------------------------------------------------------------------- P2 -----
@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    """f_eq reproduces rho, rho u and rho (c_s^2 I + u u) (eq. 4-6 at equilibrium)."""
    rng = np.random.default_rng(1)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    for _ in range(5):
        rho = 1.0 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(D)
        fe = O.feq(q, rho, u)
        cc = c[:, :D].astype(float)
        assert abs(fe.sum() - rho) < 1e-15
        assert np.abs(fe @ cc - rho * u).max() < 1e-16
        P = np.einsum("i,ia,ib->ab", fe, cc, cc)
        assert np.abs(P - rho * (np.eye(D) / 3 + np.outer(u, u))).max() < 1e-15


# --------------------------------------------------------------------- P3 -----
@pytest.mark.parametrize("q", [9, 19])
def test_collision_conserves_mass_and_adds_force(q):
    """BGK + Guo forcing: sum f* = sum f and sum c f* = sum c f + F exactly."""
    rng = np.random.default_rng(2)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    cc = c[:, :D].astype(float)
    for tau in (0.5 + 1e-5, 0.7, 1.3):
        u = 0.05 * rng.standard_normal(3)
        if D == 2:
            u[2] = 0.0
        f = O.feq(q, 1.02, u) * (1 + 0.01 * rng.standard_normal(q))
        F = 1e-3 * rng.standard_normal(3)
        if D == 2:
            F[2] = 0.0
        fp, rho, um = O.collide(q, f, tau, F)
        assert abs(fp.sum() - f.sum()) < 1e-15
        assert np.abs(fp @ cc - (f @ cc + F[:D])).max() < 1e-16
        # the returned velocity is the half-force-shifted first moment (eq. 5)
        assert np.abs(um[:D] - (f @ cc + 0.5 * F[:D]) / f.sum()).max() < 1e-16


def _run_steady(o, chunk=2000, tol=1e-15, max_steps=400000):
    prev = o.u().copy()
    done = 0
    while done < max_steps:
        o.step(chunk)
        done += chunk
        cur = o.u()
        if np.abs(cur - prev).max() <= tol * max(np.abs(cur).max(), 1e-30):
            break
        prev = cur.copy()
    return o


def _poiseuille_exact(H, nu, g, tau, uw=0.0):
    """Steady BGK + halfway bounce-back channel: the parabola plus the
    tau-dependent slip whose (2/3) Lambda part is eq. 34's numerical slip."""
    y = np.arange(H) + 0.5
    L = (tau - 0.5) ** 2
    return uw + g / (2 * nu) * y * (H - y) + g / nu * (16 * L - 3) / 24


# --------------------------------------------------------------------- P4 -----
@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2, 1.5, 0.5 + math.sqrt(3) / 4])
def test_poiseuille_closed_form(tau):
    """Laminar Poiseuille with no-slip halfway bounce-back (eq. 31, u_w = 0)
    and Guo forcing matches the closed-form discrete steady state pointwise."""
    H = 16
    nu = (tau - 0.5) / 3
    g = 8 * nu * 1e-3 / H ** 2
    p = O.params(q=9, nx=1, ny=H, nu=nu, force=(g, 0, 0), scheme=O.BB_FIXED, sa_on=0)
    o = _run_steady(O.Oracle(p))
    u = o.u()[0, 0, :, 0]
    ex = _poiseuille_exact(H, nu, g, tau)
    # round-off floor of the iterated steady state grows like 1/nu
    assert np.abs(u - ex).max() / ex.max() < 1e-10
    assert np.abs(o.u()[1]).max() / ex.max() < 1e-10


def test_poiseuille_second_order():
    """At fixed tau the error against the continuous parabola falls as H^-2."""
    tau = 0.8
    nu = (tau - 0.5) / 3
    errs = []
    for H in (8, 16, 32):
        g = 8 * nu * 1e-3 / H ** 2
        p = O.params(q=9, nx=1, ny=H, nu=nu, force=(g, 0, 0), scheme=O.BB_FIXED, sa_on=0)
        o = _run_steady(O.Oracle(p), chunk=4000, tol=1e-13)
        y = np.arange(H) + 0.5
        cont = g / (2 * nu) * y * (H - y)
        u = o.u()[0, 0, :, 0]
        errs.append(np.linalg.norm(u - cont) / np.linalg.norm(cont))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(o_ - 2.0) < 0.02 for o_ in orders), orders


def test_poiseuille_3d_channel():
    """D3Q19 with periodic x and z reproduces the same discrete steady state."""
    tau, H = 0.8, 8
    nu = (tau - 0.5) / 3
    g = 8 * nu * 1e-3 / H ** 2
    p = O.params(q=19, nx=2, ny=H, nz=2, nu=nu, force=(g, 0, 0), scheme=O.BB_FIXED, sa_on=0)
    o = _run_steady(O.Oracle(p), chunk=2000, tol=1e-14)
    u = o.u()
    ex = _poiseuille_exact(H, nu, g, tau)
    assert np.abs(u[0] - ex[None, :, None]).max() / ex.max() < 1e-10
    assert np.abs(u[1:]).max() / ex.max() < 1e-10


# --------------------------------------------------------------------- P5 -----
@pytest.mark.parametrize("tau", [0.55, 0.9, 1.4])
def test_couette_exact(tau):
    """Moving-wall bounce-back (eq. 31): plane Couette flow is linear with the
    wall velocity met exactly halfway (the second-derivative term of eq. 34
    vanishes)."""
    H, U = 10, 0.02
    nu = (tau - 0.5) / 3
    p = O.params(q=9, nx=1, ny=H, nu=nu, scheme=O.BB_FIXED, sa_on=0, wall_u_top=(U, 0, 0))
    o = _run_steady(O.Oracle(p), chunk=2000, tol=1e-15)
    y = np.arange(H) + 0.5
    assert np.abs(o.u()[0, 0, :, 0] - U * y / H).max() < 1e-14


# ------------------------------------------------------------------ P6/P7 -----
@pytest.mark.parametrize("law", [O.REICHARDT, O.SA_LAW])
def test_slip_bounce_back_laminar_steady_state(law):
    """Slip-velocity bounce-back (eq. 31 + eq. 35) with the wall function at F.

    Laminar (nu_t = 0 in the bulk) so the flow is the moving-wall Poiseuille
    state of P4 shifted by the slip u_w.  At steady state eq. 35 with
    nu_t|B = nu kappa y_B+ and Delta_w = 1/2 reads
    u_tau^2 / (2 (nu + kappa u_tau / 2)) = A_0 (the parabola's value at B),
    a quadratic in u_tau; u_F then follows from the wall law and fixes u_w.
    """
    H, tau = 12, 0.9
    nu = (tau - 0.5) / 3
    g = 8 * nu * 2e-3 / H ** 2
    kappa = 0.41
    p = O.params(q=9, nx=1, ny=H, nu=nu, force=(g, 0, 0), scheme=O.BB_SLIP, sa_on=0, law=law)
    o = _run_steady(O.Oracle(p), chunk=2000, tol=1e-15)
    A = _poiseuille_exact(H, nu, g, tau)
    A0, A1 = A[0], A[1]
    yB = 0.5
    ut = (kappa * yB * A0 + math.sqrt((kappa * yB * A0) ** 2 + 4 * yB * nu * A0)) / (2 * yB)
    uF = ut * O.uplus(law, 1.5 * ut / nu)
    uw = uF - A1
    u = o.u()[0, 0, :, 0]
    assert np.abs(u - (uw + A)).max() / np.abs(u).max() < 1e-11
    wall = o.wall()
    assert np.allclose(wall["utau"], ut, rtol=1e-11, atol=0)
    assert np.allclose(wall["uw"][:, 0], uw, rtol=1e-10, atol=0)


def _perturbed_u0(D, nz, ny, nx, amp, seed):
    rng = np.random.default_rng(seed)
    return amp * (2 * rng.random((D, nz, ny, nx)) - 1)


@pytest.mark.parametrize("q", [9, 19])
def test_slip_bounce_back_conserves_mass(q):
    """The slip-velocity correction is tangential, so its link terms sum to
    zero over each wall cell: total mass is constant to round-off."""
    nz = 1 if q == 9 else 3
    D = _dims(q)
    u0 = _perturbed_u0(D, nz, 12, 5, 0.02, 3)
    u0[0] += 0.03
    p = O.params(q=q, nx=5, ny=12, nz=nz, nu=2e-3, force=(1e-6, 0, 0), scheme=O.BB_SLIP, sa_on=1)
    o = O.Oracle(p, u0)
    m0 = o.rho().sum()
    o.step(300)
    assert abs(o.rho().sum() - m0) / m0 < 1e-13


# --------------------------------------------------------------------- P8 -----
@pytest.mark.parametrize("q", [9, 19])
def test_regularized_moments(q):
    """eq. 17-19/26: the reconstruction has density rho, momentum rho u and
    momentum flux rho (c_s^2 I + u u) - 2 rho tau c_s^2 S."""
    rng = np.random.default_rng(4)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    cc = c[:, :D].astype(float)
    rho, tau = 1.03, 0.93
    u = 0.05 * rng.standard_normal(D)
    S = np.zeros((3, 3))
    A = 1e-3 * rng.standard_normal((D, D))
    S[:D, :D] = 0.5 * (A + A.T)
    f = O.regularized(q, rho, u, S, tau)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(f @ cc - rho * u).max() < 1e-16
    P = np.einsum("i,ia,ib->ab", f, cc, cc)
    ex = rho * (np.eye(D) / 3 + np.outer(u, u)) - 2 * rho * tau / 3 * S[:D, :D]
    assert np.abs(P - ex).max() < 1e-15


# --------------------------------------------------------------------- P9 -----
@pytest.mark.parametrize("side", [-1, 1])
def test_boundary_density_closure(side):
    """eq. 23: with the streamed populations at equilibrium and u_B . n = 0,
    f_par + 2 f_perp returns the density exactly."""
    p = O.params(q=9, nu=1e-3, beta=0.28, sa_on=1)
    for rho, ux in ((1.0, 0.03), (0.97, -0.05), (1.04, 0.0)):
        f = O.feq(9, rho, (ux, 0.0))
        out = O.hrfd_cell(p, f, side, (1.0, 0.0), utau=2e-3, uF_t=0.01, uFF_t=0.012,
                          dudx=0.0, ntB=3e-3)
        assert abs(out.sum() - rho) < 2e-15


# ---------------------------------------------------------------- HRFD cell ---
@pytest.mark.parametrize("law", [O.REICHARDT, O.SA_LAW])
@pytest.mark.parametrize("side", [-1, 1])
def test_hrfd_cell_gradient_and_velocity(law, side):
    """HRFD at one wall cell (Sec. 3.1): the reconstruction's first moment is
    rho_B u_tau u+(y_B+) t; with beta = 0 a linear profile along the inward
    normal gives the exact FD gradient of eq. 28, with beta = 1 the analytic
    derivative of the law; S enters with the inward normal's sign."""
    c, w, _ = O.lattice(9)
    cc = c[:, :2].astype(float)
    nu, utau, ntB = 1e-4, 3e-3, 2e-3
    f = O.feq(9, 1.01, (0.04, 0.0))
    rhoB = O.hrfd_cell(O.params(q=9, nu=nu, law=law, beta=0.0), f, side, (1, 0), utau,
                       0, 0, 0, ntB).sum()
    uBwf = utau * O.uplus(law, 0.5 * utau / nu)
    b = 0.004  # slope of the tangential velocity along the inward normal
    tau = 0.5 + 3 * (nu + O.nut(O.params(q=9, nu=nu), ntB))
    for beta in (0.0, 1.0, 0.28):
        p = O.params(q=9, nu=nu, law=law, beta=beta, sa_on=1)
        out = O.hrfd_cell(p, f, side, (1, 0), utau, uBwf + b, uBwf + 2 * b, 0.0, ntB)
        assert abs(out.sum() - rhoB) < 1e-15
        assert abs(out @ cc[:, 0] - rhoB * uBwf) < 1e-16
        assert abs(out @ cc[:, 1]) < 1e-16
        G = beta * utau ** 2 / nu * O.duplus(law, 0.5 * utau / nu) + (1 - beta) * b
        dudy = -side * G  # inward normal is -side * y
        Pxy = out @ (cc[:, 0] * cc[:, 1])
        assert abs(Pxy - (-2 * rhoB * tau / 3 * 0.5 * dudy)) < 1e-15
    # tangential derivative enters S_xx = -S_yy
    p = O.params(q=9, nu=nu, law=law, beta=0.0, sa_on=1)
    dudx = 2e-4
    out = O.hrfd_cell(p, f, side, (1, 0), utau, uBwf, uBwf, dudx, ntB)
    Pxx = out @ (cc[:, 0] ** 2)
    Pyy = out @ (cc[:, 1] ** 2)
    assert abs(Pxx - rhoB * (1 / 3 + uBwf ** 2) - (-2 * rhoB * tau / 3 * dudx)) < 1e-15
    assert abs(Pyy - rhoB / 3 - (2 * rhoB * tau / 3 * dudx)) < 1e-15


# -------------------------------------------------------------------- P10 -----
def test_reichardt_limits_and_inverse():
    """Reichardt's law: u+ ~ y+ at the wall, log law with intercept B far out;
    the bisection inverse recovers u_tau from (y, u) to 1e-12."""
    k, B = 0.41, 5.2
    for yp in (1e-6, 1e-4):
        assert abs(O.uplus(O.REICHARDT, yp) / yp - 1) < 1e-3
    for yp in (1e7, 1e9):
        assert abs(O.uplus(O.REICHARDT, yp) - (math.log(yp) / k + B)) < 1e-5
    # derivative consistent with the law (central differences)
    for yp in (0.3, 3.0, 30.0, 300.0, 3e4):
        h = 1e-5 * yp
        nd = (O.uplus(O.REICHARDT, yp + h) - O.uplus(O.REICHARDT, yp - h)) / (2 * h)
        assert abs(nd / O.duplus(O.REICHARDT, yp) - 1) < 1e-8
    nu, y = 1.7e-5, 1.5
    for yp in np.logspace(-2, 5, 200):
        ut = yp * nu / y
        u = ut * O.uplus(O.REICHARDT, yp)
        got = O.solve_utau(O.REICHARDT, u, y, nu)
        assert abs(got / ut - 1) < 1e-12
    assert O.solve_utau(O.REICHARDT, 0.0, y, nu) == 0.0


# -------------------------------------------------------------------- P11 -----
def test_sa_law_eq16_consistent_with_eq15():
    """eq. 16 is the integral of eq. 15 with u+(0) = 0 and a log law with
    slope 1/kappa; the readings (atan2 branch, B-bar digit) are what make
    these hold."""
    assert abs(O.uplus(O.SA_LAW, 0.0)) < 1e-11
    for yp in (1e-2, 0.5, 6.0, 6.9287093849022945, 8.0, 60.0, 1e3, 1e5):
        h = 1e-6 * max(1.0, yp)
        nd = (O.uplus(O.SA_LAW, yp + h) - O.uplus(O.SA_LAW, yp - h)) / (2 * h)
        ex = (7.1 ** 3 + (0.41 * yp) ** 3) / (7.1 ** 3 + (1 + 0.41 * yp) * (0.41 * yp) ** 3)
        assert abs(nd / ex - 1) < 1e-7
        assert abs(O.duplus(O.SA_LAW, yp) / ex - 1) < 1e-14
    # log law far from the wall
    d = O.uplus(O.SA_LAW, 1e8) - math.log(1e8) / 0.41
    assert abs(d - 5.0334) < 1e-3
    # inverse
    nu, y = 2e-5, 1.5
    for yp in np.logspace(-2, 5, 60):
        ut = yp * nu / y
        got = O.solve_utau(O.SA_LAW, ut * O.uplus(O.SA_LAW, yp), y, nu)
        assert abs(got / ut - 1) < 1e-12


# -------------------------------------------------------------------- P12 -----
def test_cai_degrigny_ratio_fig5():
    """eq. 29 over eq. 15 at y_B = Delta/2 (Fig. 5): a near-constant factor
    around 0.76-0.77; its log-law limit is (3 ln3 - 1.5 ln5 + ln7/3)/2."""
    lim = (3 * math.log(3) - 1.5 * math.log(5) + math.log(7) / 3) / 2
    nu = 1.0
    for re_tau in (4000, 20000):
        for N in (5, 10, 20, 40):
            utau = re_tau * nu  # h = 1
            delta = 1.0 / N
            num = O.cai_degrigny_grad(O.SA_LAW, utau, nu, delta / 2, delta)
            ana = utau ** 2 / nu * O.duplus(O.SA_LAW, 0.5 * delta * utau / nu)
            r = num / ana
            assert 0.755 < r < 0.775, (re_tau, N, r)
    utau, delta = 1e9, 1.0
    num = O.cai_degrigny_grad(O.SA_LAW, utau, 1.0, 0.5, delta)
    ana = utau ** 2 * O.duplus(O.SA_LAW, 0.5 * utau)
    assert abs(num / ana - lim) < 1e-6


@pytest.mark.parametrize("law", [O.REICHARDT, O.SA_LAW])
def test_cai_degrigny_stencil_third_order(law):
    """eq. 29 is a one-sided third-order difference: at a fixed y_B its error
    against the law's derivative falls by 2^3 when Delta halves."""
    nu, utau, yB = 1.0, 1.0, 8.0
    ana = utau ** 2 / nu * O.duplus(law, yB * utau / nu)
    errs = [O.cai_degrigny_grad(law, utau, nu, yB, d) - ana for d in (0.1, 0.05, 0.025)]
    for e0, e1 in zip(errs, errs[1:]):
        assert 7.0 < e0 / e1 < 9.0, errs


@pytest.mark.parametrize("side", [-1, 1])
def test_cai_degrigny_cell(side):
    """The Cai-Degrigny scheme (Sec. 3.1.2, eq. 30) is the regularized cell of
    eq. 26 with the wall-normal gradient of eq. 29 at Delta = 1, y_B = 1/2:
    the flow at F, FF and beta do not enter, and in the log layer that
    gradient is 0.76-0.77 of the law's derivative (Fig. 5)."""
    c, w, _ = O.lattice(9)
    cc = c[:, :2].astype(float)
    nu, utau, ntB = 1e-5, 4e-3, 2e-3  # y_B+ = 200
    f = O.feq(9, 1.01, (0.04, 0.0))
    tau = 0.5 + 3 * (nu + O.nut(O.params(q=9, nu=nu), ntB))
    outs = []
    for beta, uF, uFF in ((0.28, 0.05, 0.06), (0.0, 0.01, 0.0), (1.0, 0.0, 0.3)):
        p = O.params(q=9, nu=nu, law=O.SA_LAW, beta=beta, sa_on=1, scheme=O.CAI_DEGRIGNY)
        outs.append(O.hrfd_cell(p, f, side, (1, 0), utau, uF, uFF, 0.0, ntB))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    out = outs[0]
    rhoB = out.sum()
    G = O.cai_degrigny_grad(O.SA_LAW, utau, nu, 0.5, 1.0)
    Pxy = out @ (cc[:, 0] * cc[:, 1])
    assert abs(Pxy - (-2 * rhoB * tau / 3 * 0.5 * (-side * G))) < 1e-15
    ana = utau ** 2 / nu * O.duplus(O.SA_LAW, 0.5 * utau / nu)
    assert 0.755 < G / ana < 0.775


# -------------------------------------------------------------------- P13 -----
def _loglayer_rhs(y, utau=0.05, nu=1e-9):
    p = O.params(q=9, nu=nu)
    k = 0.41
    u = lambda yy: utau / k * math.log(yy)
    nt = lambda yy: k * utau * yy
    ntm = [nt(y), nt(y - 1)]
    ntp = [nt(y), nt(y + 1)]
    u0 = [u(y), 0.0, 0.0]
    um = [u(y), 0, 0, u(y - 1), 0, 0, 0, 0, 0]
    up = [u(y), 0, 0, u(y + 1), 0, 0, 0, 0, 0]
    return O.sa_rhs(p, 2, nt(y), ntm, ntp, u0, um, up, y) / (0.1355 * utau ** 2)


def test_sa_rhs_vanishes_in_log_layer():
    """In the log layer (u = u_tau ln y / kappa, nu_tilde = kappa u_tau y,
    chi -> infinity) production, destruction and diffusion of eq. 11 cancel
    because of the definition of c_w1; the discrete residual falls at second
    order in 1/y."""
    r1, r2, r3 = (abs(_loglayer_rhs(y)) for y in (50.0, 100.0, 200.0))
    assert r1 < 2e-3
    assert 3.5 < r1 / r2 < 4.5 and 3.5 < r2 / r3 < 4.5


def test_sa_rhs_terms():
    """Convection is first-order upwind: with a curved nu_tilde profile the
    convective change depends only on the upstream neighbour (Sec. 2.2, the
    text after eq. 14); f_v1 = 1/2 at chi = c_v1 (eq. 10)."""
    p = O.params(q=9, nu=1e-3)
    assert abs(O.nut(p, 7.1e-3) - 7.1e-3 / 2) < 1e-18
    base = dict(D=2, nt0=2e-3, ntm=[1.9e-3, 2e-3], ntp=[2.3e-3, 2e-3], d=1e9)
    zero = [0.0] * 9
    r0 = O.sa_rhs(p, base["D"], base["nt0"], base["ntm"], base["ntp"], [0, 0, 0], zero, zero,
                  base["d"])
    for U in (0.03, -0.03):
        uu = [U, 0, 0]
        um = [U, 0, 0, U, 0, 0, 0, 0, 0]
        r = O.sa_rhs(p, base["D"], base["nt0"], base["ntm"], base["ntp"], uu, um, um, base["d"])
        upstream_diff = 1e-4 if U > 0 else 3e-4  # (nt0 - ntm) or (ntp - nt0)
        assert abs((r - r0) - (-U * upstream_diff)) < 1e-15


# SA constants printed after eq. 14 and the definition of c_w1 there
_K, _CB1, _CB2, _SIG, _CW2, _CW3, _CV1 = 0.41, 0.1355, 0.622, 2.0 / 3.0, 0.3, 2.0, 7.1
_CW1 = _CB1 / _K ** 2 + (1.0 + _CB2) / _SIG


def test_sa_constants_are_the_papers():
    """The oracle's default SA constants are the values printed after eq. 14
    (c_w1 follows from them: 3.2390678...)."""
    p = O.params(q=9)
    assert (p.kappa, p.cb1, p.cb2, p.cw2, p.cw3, p.cv1, p.rlim) == (0.41, 0.1355, 0.622, 0.3,
                                                                      2.0, 7.1, 10.0)
    assert abs(p.sigma - 2.0 / 3.0) < 1e-16
    assert abs(_CW1 - 3.2390678167757287) < 1e-15


def _eq15(yp):
    """du+/dy+ of the SA constant-stress layer as printed (eq. 15)."""
    ky = _K * yp
    return (_CV1 ** 3 + ky ** 3) / (_CV1 ** 3 + (1.0 + ky) * ky ** 3)


def _const_stress_rhs(yplus, y, utau=1e-3):
    """Discrete SA right-hand side at the node y (lattice units, wall distance
    d = y) of the constant-stress layer: nu_tilde = kappa u_tau y and u(y) the
    integral of eq. 15 (taken by quadrature, independently of eq. 16), with
    nu set so that y+ = yplus at the node.  Scaled by c_b1 u_tau^2."""
    from scipy.integrate import quad
    nu = y * utau / yplus
    s = utau / nu
    du_p = utau * quad(_eq15, yplus, (y + 1) * s, epsabs=0, epsrel=1e-13, limit=200)[0]
    du_m = utau * quad(_eq15, (y - 1) * s, yplus, epsabs=0, epsrel=1e-13, limit=200)[0]
    nt = lambda yy: _K * utau * yy
    p = O.params(q=9, nu=nu)
    um = [0.0, 0, 0, -du_m, 0, 0, 0, 0, 0]
    up = [0.0, 0, 0, du_p, 0, 0, 0, 0, 0]
    r = O.sa_rhs(p, 2, nt(y), [nt(y), nt(y - 1)], [nt(y), nt(y + 1)], [0.0, 0, 0], um, up, y)
    return r / (_CB1 * utau ** 2)


@pytest.mark.parametrize("yplus", [1.0, 3.0, 10.0, 30.0, 100.0])
def test_sa_rhs_vanishes_in_constant_stress_layer(yplus):
    """Constant total stress at finite chi = kappa y+ (eq. 15 is that layer's
    profile): with nu_tilde = kappa u_tau y, eq. 13 gives S_tilde = u_tau /
    (kappa y) exactly, because f_v2 = 1 - chi du+/dy+; so r = 1, f_w = 1, and
    production c_b1 u_tau^2, destruction c_w1 kappa^2 u_tau^2 and diffusion
    (1 + c_b2) kappa^2 u_tau^2 / sigma cancel by the definition of c_w1.
    The discrete right-hand side vanishes at second order under refinement
    at every y+ (this pins f_v1 and f_v2 where chi is finite)."""
    r = [_const_stress_rhs(yplus, y) for y in (20.0, 40.0, 80.0, 160.0)]
    assert abs(r[-1]) < 5e-4, r
    for a, b in zip(r, r[1:]):
        assert 3.8 < a / b < 4.2, r


@pytest.mark.parametrize("chi", [2.0, 3.0])
def test_sa_rhs_at_rest_with_negative_s_tilde(chi):
    """At rest (S = 0) with a uniform nu_tilde at chi = 2 or 3, f_v2 < 0 and
    S_tilde <= 0: the reading for that case switches production off and sets
    r = r_lim = 10, where g = r + c_w2 (r^6 - r) ~ 3e5 and f_w (eq. 14) is its
    large-g limit (1 + c_w3^6)^(1/6).  Only destruction remains:
    -c_w1 (1 + c_w3^6)^(1/6) (nu_tilde / d)^2."""
    nu = 1e-3
    nt = chi * nu
    p = O.params(q=9, nu=nu)
    z3, z9 = [0.0] * 3, [0.0] * 9
    for d in (0.5, 2.5, 7.0, 30.0, 1e3):
        r = O.sa_rhs(p, 2, nt, [nt] * 3, [nt] * 3, z3, z9, z9, d)
        ex = -_CW1 * (1.0 + _CW3 ** 6) ** (1.0 / 6.0) * (nt / d) ** 2
        assert abs(r / ex - 1.0) < 1e-13, (d, r, ex)


def _loglayer_rhs_a(a, y, utau=0.05, nu=1e-9):
    """Log layer (chi -> infinity, so S_tilde = S) with nu_tilde = a kappa
    u_tau y: r = a exactly, scaled right-hand side."""
    p = O.params(q=9, nu=nu)
    u = lambda yy: utau / _K * math.log(yy)
    nt = lambda yy: a * _K * utau * yy
    um = [u(y), 0, 0, u(y - 1), 0, 0, 0, 0, 0]
    up = [u(y), 0, 0, u(y + 1), 0, 0, 0, 0, 0]
    return O.sa_rhs(p, 2, nt(y), [nt(y), nt(y - 1)], [nt(y), nt(y + 1)], [u(y), 0, 0], um, up,
                    y) / utau ** 2


def test_sa_destruction_slope_at_r_equal_one():
    """In the log layer with nu_tilde = a kappa u_tau y the right-hand side per
    u_tau^2 is a c_b1 + a^2 (c_w1 kappa^2 - c_b1) - a^2 c_w1 kappa^2 f_w(a), so
    its slope at a = 1 is -(c_b1 + c_w1 kappa^2 f_w'(1)); differentiating eq. 14
    gives f_w'(1) = (1 + 5 c_w2) c_w3^6 / (1 + c_w3^6) (this pins the shape of
    g and f_w between r = 1 and r_lim).  The discrete slope converges to it at
    second order."""
    ex = -(_CB1 + _CW1 * _K ** 2 * (1.0 + 5.0 * _CW2) * _CW3 ** 6 / (1.0 + _CW3 ** 6))
    h = 1e-4
    err = []
    for y in (100.0, 200.0, 400.0):
        sl = (_loglayer_rhs_a(1 + h, y) - _loglayer_rhs_a(1 - h, y)) / (2 * h)
        err.append(abs(sl / ex - 1.0))
    assert err[-1] < 3e-5, err
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5, err


def test_sa_diffusion_second_order():
    """Diffusion and the c_b2 term of eq. 11 for nu_tilde = A y^2 at rest, far
    from walls (d large, so production and destruction are negligible): the
    exact value is (1/sigma)[(nu + nu_tilde) nu_tilde'' + (1 + c_b2) nu_tilde'^2]
    = (1/sigma)[2 A nu + (6 + 4 c_b2) A^2 y^2]; the discrete value approaches it
    at second order in 1/y."""
    nu, A = 1e-3, 1e-4
    p = O.params(q=9, nu=nu)
    z3, z9 = [0.0] * 3, [0.0] * 9
    err = []
    for y in (10.0, 20.0, 40.0):
        nt = lambda yy: A * yy * yy
        r = O.sa_rhs(p, 2, nt(y), [nt(y), nt(y - 1)], [nt(y), nt(y + 1)], z3, z9, z9, 1e12)
        ex = (2 * A * nu + (6 + 4 * _CB2) * A * A * y * y) / _SIG
        err.append(abs(r / ex - 1.0))
    assert err[-1] < 2e-4, err
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5, err


# ------------------------------------------------------------------ P14/15 ---
def test_table2_dean():
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_dean.txt"))
    for re_tau, u_tau, g, re_b, u_b, cf_b, y50 in rows:
        r = OU.table2_row(re_tau)
        assert abs(r["u_tau"] - u_tau) < 5e-5
        assert abs(r["g"] / g - 1) < 0.01
        assert abs(r["re_b"] / re_b - 1) < 1e-4
        assert abs(r["u_b"] - u_b) < 1e-4
        cf_print = 0.00220 if re_tau == 20000 else cf_b
        assert abs(r["cf_b"] - cf_print) < 1e-5
        assert abs(r["y50"] - y50) < 1e-4


def test_table3_geometry():
    """B at Delta/2, F at 1.5 Delta: y_B+ = Re_tau/(2N), y_F+ = 3 y_B+."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_grid.txt"))
    for N, yb_h, ybp, yfp in rows:
        lat = OU.channel_lattice(4200.0, int(N))
        assert abs(0.5 / N - yb_h) < 5e-4
        assert abs(lat["y_b_plus"] - ybp) < 1e-9 * ybp
        assert abs(lat["y_f_plus"] - yfp) < 1e-9 * yfp


# -------------------------------------------------------------------- P16 -----
@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD])
def test_channel_mirror_symmetry_and_x_invariance(scheme):
    """Without a perturbation the coupled SA/wall-function channel stays
    mirror-symmetric about the centre-line and x-invariant; a 4-wide run
    equals a 1-wide run."""
    lat = OU.channel_lattice(2000.0, 8)
    ny = 16
    res = []
    for nx in (1, 4):
        p = O.params(q=9, nx=nx, ny=ny, nu=lat["nu"], force=(lat["g"] * 50, 0, 0), scheme=scheme)
        u0 = np.zeros((2, 1, ny, nx))
        u0[0] = lat["u_b"]
        o = O.Oracle(p, u0)
        o.step(400)
        res.append((o.u(), o.nt(), o.wall()["utau"]))
    u, nt, ut = res[1]
    ub = lat["u_b"]
    assert np.abs(u - u[..., :1]).max() == 0.0
    assert np.abs(u[0, 0] - u[0, 0, ::-1]).max() < 1e-12 * ub
    assert np.abs(u[1, 0] + u[1, 0, ::-1]).max() < 1e-12 * ub
    assert np.abs(nt[0] - nt[0, ::-1]).max() < 1e-12 * nt.max()
    assert np.abs(u[..., 0] - res[0][0][..., 0]).max() == 0.0
    assert np.abs(ut[:4] - ut[4:]).max() < 1e-12 * ut.max()


def test_channel_3d_matches_2d_when_z_invariant():
    """A z-invariant D3Q19 channel with slip BB follows the D2Q9 one closely
    (same wall function and SA model; different lattice)."""
    lat = OU.channel_lattice(2000.0, 8)
    ny = 16
    out = {}
    for q, nz in ((9, 1), (19, 2)):
        p = O.params(q=q, nx=2, ny=ny, nz=nz, nu=lat["nu"], force=(lat["g"] * 50, 0, 0))
        D = _dims(q)
        u0 = np.zeros((D, nz, ny, 2))
        u0[0] = lat["u_b"]
        o = O.Oracle(p, u0)
        o.step(200)
        out[q] = o.u()
    u3 = out[19]
    assert np.abs(u3 - u3[:, :1]).max() == 0.0
    assert np.abs(u3[2]).max() < 1e-18
    rel = np.abs(u3[0, 0, :, 0] - out[9][0, 0, :, 0]).max() / lat["u_b"]
    assert rel < 2e-3


# ----------------------------------------------------------- plate edges -----
def test_zou_he_moments():
    rng = np.random.default_rng(5)
    c, w, _ = O.lattice(9)
    for U in (0.05, 0.1):
        f = O.feq(9, 1.0, (0.07, 0.01)) * (1 + 0.02 * rng.standard_normal(9))
        g = O.zou_he_west(f, U)
        rho = g.sum()
        assert abs(g @ c[:, 0] - rho * U) < 1e-16
        assert abs(g @ c[:, 1]) < 1e-17
        known = [0, 2, 3, 4, 6, 8]
        assert np.all(g[known] == f[known])


def test_plate_domain_free_stream_is_preserved():
    """With no wall (plate_start = nx) the inlet, outlet and symmetry planes
    keep a uniform stream exactly uniform."""
    nx, ny, U = 24, 10, 0.1
    p = O.params(q=9, nx=nx, ny=ny, flow=O.PLATE, plate_start=nx, nu=2e-5, u_inlet=U, sa_on=1)
    u0 = np.zeros((2, 1, ny, nx))
    u0[0] = U
    o = O.Oracle(p, u0)
    o.step(150)
    assert np.abs(o.u()[0] - U).max() < 1e-15
    assert np.abs(o.u()[1]).max() < 1e-16
    assert np.abs(o.rho() - 1.0).max() < 1e-15


@pytest.mark.parametrize("scheme", [O.BB_SLIP, O.HRFD])
def test_plate_runs_and_stays_finite(scheme):
    """The plate with a wall develops a boundary layer: velocity drops near
    the wall downstream, u_tau is positive along the plate."""
    # BGK with the Zou-He inlet needs tau - 1/2 above ~0.05 to stay stable
    nx, ny, U = 64, 16, 0.05
    p = O.params(q=9, nx=nx, ny=ny, flow=O.PLATE, plate_start=8, nu=0.03, u_inlet=U,
                 scheme=scheme)
    u0 = np.zeros((2, 1, ny, nx))
    u0[0] = U
    o = O.Oracle(p, u0)
    o.step(300)
    u = o.u()
    assert np.all(np.isfinite(u))
    assert u[0, 0, 0, 40] < 0.97 * U
    assert np.all(o.wall()["utau"] > 0)


# ------------------------------------------------------------ CM collision ---
def _basis(q):
    D = _dims(q)
    import itertools
    out = []
    for e in itertools.product(range(3), repeat=D):
        out.append(tuple(e) + (0,) * (3 - D))
    return out


@pytest.mark.parametrize("q", [9, 19])
def test_cm_conserves_mass_and_adds_force(q):
    rng = np.random.default_rng(7)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    cc = c[:, :D].astype(float)
    for tau in (0.5 + 1e-4, 0.8, 1.7):
        u = 0.05 * rng.standard_normal(3)
        u[D:] = 0
        f = O.feq(q, 1.01, u) * (1 + 0.03 * rng.standard_normal(q))
        F = 1e-3 * rng.standard_normal(3)
        F[D:] = 0
        fp, rho, um = O.collide_cm(q, f, tau, F)
        assert abs(fp.sum() - f.sum()) < 1e-15
        assert np.abs(fp @ cc - (f @ cc + F[:D])).max() < 1e-16


@pytest.mark.parametrize("q", [9, 19])
def test_cm_unit_relaxation_gives_maxwellian_moments(q):
    """With omega = 1 and no force, eq. 7 sends every central moment to its
    equilibrium, so each supported raw moment of f* equals that of a
    Maxwellian, rho prod_a M_pa(u_a) with M_0 = 1, M_1 = u, M_2 = cs2 + u^2."""
    rng = np.random.default_rng(8)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    for _ in range(4):
        u = 0.08 * rng.standard_normal(3)
        u[D:] = 0
        f = O.feq(q, 0.98, u) * (1 + 0.05 * rng.standard_normal(q))
        fp, rho, um = O.collide_cm(q, f, 1.0)
        M = lambda p, ua: (1.0, ua, 1 / 3 + ua * ua)[p]
        for e in _basis(q):
            mono = np.prod([c[:, a].astype(float) ** e[a] for a in range(3)], axis=0)
            # monomials that vanish identically on the lattice are not moments of it
            if not np.any(mono) or (q == 19 and sum(x > 0 for x in e) == 3):
                continue
            ex = rho * np.prod([M(e[a], um[a]) for a in range(3)])
            assert abs(fp @ mono - ex) < 1e-15, e


@pytest.mark.parametrize("q", [9, 19])
def test_cm_relaxes_deviatoric_stress_only(q):
    """Shear (off-diagonal) and deviatoric normal central moments relax with
    omega; their trace is reset to D rho cs2 (relaxation rate 1)."""
    rng = np.random.default_rng(9)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    cc = c[:, :D].astype(float)
    tau = 0.74
    om = 1 / tau
    u = 0.05 * rng.standard_normal(3)
    u[D:] = 0
    f = O.feq(q, 1.0, u) * (1 + 0.05 * rng.standard_normal(q))
    fp, rho, um = O.collide_cm(q, f, tau)
    ud = um[:D]

    def central2(g):
        cb = cc - ud
        return np.einsum("i,ia,ib->ab", g, cb, cb)

    k, ks = central2(f), central2(fp)
    dev = lambda m: m - np.eye(D) * np.trace(m) / D
    assert np.abs(dev(ks) - (1 - om) * dev(k)).max() < 1e-15
    assert abs(np.trace(ks) - D * rho / 3) < 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_cm_forcing_gives_shifted_maxwellian(q):
    """With omega = 1 and a body force, eq. 7 returns the Maxwellian moments at
    the post-collision velocity v = u + F/(2 rho), up to O(F^2): the forcing
    central moments (first order F, third order cs2 F) are that Maxwellian's
    central moments about u to first order in F."""
    rng = np.random.default_rng(10)
    c, w, _ = O.lattice(q)
    D = _dims(q)
    M = lambda p, ua: (1.0, ua, 1 / 3 + ua * ua)[p]
    for _ in range(3):
        u = 0.06 * rng.standard_normal(3)
        u[D:] = 0
        f = O.feq(q, 1.0, u) * (1 + 0.05 * rng.standard_normal(q))
        F = 2e-3 * rng.standard_normal(3)
        F[D:] = 0
        fp, rho, um = O.collide_cm(q, f, 1.0, F)
        v = um + F / (2 * rho)
        for e in _basis(q):
            mono = np.prod([c[:, a].astype(float) ** e[a] for a in range(3)], axis=0)
            if not np.any(mono) or (q == 19 and sum(x > 0 for x in e) == 3):
                continue
            ex = rho * np.prod([M(e[a], v[a]) for a in range(3)])
            assert abs(fp @ mono - ex) < 2e-6, (e, fp @ mono - ex)


# ----------------------------------------------- interpolated bounce-back -----
def _ibb_run(ny, q, interp, force=0.0, u_top=0.0, tau=0.8, steps=None):
    nu = (tau - 0.5) / 3
    H = ny - 1 + 2 * q
    p = O.params(q=9, nx=3, ny=ny, nz=1, nu=nu, force=(force, 0, 0), sa_on=0,
                 scheme=O.BB_FIXED, bb_interp=interp, wall_dist=q, wall_u_top=(u_top, 0, 0))
    o = O.Oracle(p, np.zeros((2, 1, ny, 3)))
    o.step(steps or int(4 * H * H / nu))
    return o.u()[0, 0, :, 1], np.arange(ny) + q, H, nu


@pytest.mark.parametrize("interp", [O.IBB_BOUZIDI, O.IBB_YU])
@pytest.mark.parametrize("q", [0.2, 0.5, 0.7])
def test_ibb_couette_exact(interp, q):
    """eq. 36 and eq. 37 interpolate linearly along the link, so plane Couette
    flow with the walls at distance q from the first and last nodes is
    reproduced exactly: u = U (y + q) / (ny - 1 + 2q)."""
    U = 0.01
    u, y, H, _ = _ibb_run(8, q, interp, u_top=U)
    assert np.abs(u - U * y / H).max() < 1e-11 * U


@pytest.mark.parametrize("interp", [O.IBB_BOUZIDI, O.IBB_YU])
@pytest.mark.parametrize("q", [0.2, 0.7])
def test_ibb_poiseuille_second_order(interp, q):
    """Poiseuille flow between walls placed off the halfway position converges
    to g/(2 nu) y (H - y) at second order in the lattice spacing."""
    errs = []
    for ny in (8, 16, 32):
        H = ny - 1 + 2 * q
        nu = 0.1
        g = 8 * nu * 1e-3 / H ** 2
        u, y, H, nu = _ibb_run(ny, q, interp, force=g)
        ex = g / (2 * nu) * y * (H - y)
        errs.append(np.linalg.norm(u - ex) / np.linalg.norm(ex))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.7) & (orders < 2.3)), (errs, orders)


def test_bouzidi_at_half_is_halfway_bounce_back():
    """At q = 1/2 eq. 36 reduces to the halfway rule of eq. 31 (both
    branches): a turbulent slip-velocity channel is bitwise the same."""
    lat = OU.channel_lattice(2000.0, 8, 0.05)
    rng = np.random.Generator(np.random.PCG64(0))
    u0 = np.zeros((2, 1, 16, 4))
    u0[0] = lat["u_b"]
    u0 += 1e-3 * (2 * rng.random(u0.shape) - 1)
    out = []
    for interp in (O.IBB_HALFWAY, O.IBB_BOUZIDI):
        p = O.params(q=9, nx=4, ny=16, nu=lat["nu"], force=(lat["g"] * 20, 0, 0),
                     scheme=O.BB_SLIP, bb_interp=interp, wall_dist=0.5)
        o = O.Oracle(p, u0)
        o.step(60)
        out.append((o.u(), o.f()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_yu_keeps_the_f_node_at_half():
    """Unlike eq. 36, eq. 37 at q = 1/2 is not the halfway rule (the reflected
    population keeps a share of the one at F), yet it still converges."""
    ny, q = 16, 0.5
    H = ny - 1 + 2 * q
    g = 8 * 0.1 * 1e-3 / H ** 2
    ub, y, H, nu = _ibb_run(ny, q, O.IBB_BOUZIDI, force=g)
    uy, _, _, _ = _ibb_run(ny, q, O.IBB_YU, force=g)
    ex = g / (2 * nu) * y * (H - y)
    assert np.abs(uy - ub).max() > 1e-6 * ex.max()
    assert np.linalg.norm(uy - ex) / np.linalg.norm(ex) < 5e-3


@pytest.mark.parametrize("q", [0.5, 0.3, 0.8])
def test_sa_wall_distance_follows_the_wall_position(q):
    """With the walls q from the first and last nodes, node y sits y + q from
    the bottom wall.  From rest with a uniform nu_tilde at chi = 3 (f_v2 < 0,
    so S_tilde <= 0: no production, r = r_lim) the first lattice step changes
    nu_tilde at the interior nodes by destruction alone,
    -c_w1 (1 + c_w3^6)^(1/6) (nu_tilde / d)^2 with d that distance."""
    ny, nu, nt0 = 12, 1e-3, 3e-3
    p = O.params(q=9, nx=3, ny=ny, nz=1, nu=nu, sa_on=1, scheme=O.BB_FIXED,
                 bb_interp=O.IBB_BOUZIDI if q != 0.5 else O.IBB_HALFWAY, wall_dist=q,
                 nut_init_ratio=nt0 / nu)
    o = O.Oracle(p, np.zeros((2, 1, ny, 3)))
    o.step(1)
    nt = o.nt()[0, :, 1]
    for y in range(2, ny - 2):  # neighbours away from the Dirichlet wall nodes
        d = min(y + q, ny - 1 - y + q)
        ex = nt0 - _CW1 * (1.0 + _CW3 ** 6) ** (1.0 / 6.0) * (nt0 / d) ** 2
        assert abs(nt[y] - ex) < 1e-15 * nt0, (y, nt[y], ex)


@pytest.mark.parametrize("q", [0.5, 0.3, 0.8])
def test_wall_function_reference_node_follows_the_wall_position(q):
    """A uniform shear u = S (y + q) measured from a wall q below the first
    node: with the SA law (u+ = y+ to O(y+^5) near the wall) the wall function,
    reading u at the second node (y_F = 1 + q), returns the exact friction
    velocity sqrt(nu S) at every wall cell."""
    ny, nu, S = 12, 1e-2, 1e-8
    y = np.arange(ny) + q
    u0 = np.zeros((2, 1, ny, 3))
    u0[0, 0] = (S * np.minimum(y, ny - 1 + 2 * q - y))[:, None]
    p = O.params(q=9, nx=3, ny=ny, nz=1, nu=nu, sa_on=1, scheme=O.BB_SLIP, law=O.SA_LAW,
                 bb_interp=O.IBB_BOUZIDI if q != 0.5 else O.IBB_HALFWAY, wall_dist=q)
    o = O.Oracle(p, u0)
    ut = o.wall()["utau"]
    assert np.abs(ut / math.sqrt(nu * S) - 1).max() < 1e-9, ut
