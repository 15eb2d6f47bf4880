"""Plain FP64 CPU oracle of the LBM-RANS hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never touches it,
and it shares no code with the HIP path.  The arithmetic lives in
``lbm_oracle.c`` (plain C, double precision); this module only marshals
arguments through ctypes.

Method: Ponsin & Lozano, "Lattice Boltzmann wall boundary conditions for
RANS-based simulations with wall functions", arXiv 2506.03905.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_HDR = os.path.join(_HERE, "lbm_oracle.h")
# A different build of the oracle (the planted-mistake test loads mutated
# copies through this variable; nothing else sets it).
_LIB_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")

CHANNEL, PLATE = 0, 1
BB_FIXED, BB_SLIP, HRFD, CAI_DEGRIGNY = 0, 1, 2, 3
REICHARDT, SA_LAW = 0, 1
BGK, CM = 0, 1
IBB_HALFWAY, IBB_BOUZIDI, IBB_YU = 0, 1, 2


def compile_oracle(src: str, out: str) -> str:
    """gcc, no fast-math, no FMA contraction; OpenMP over lattice rows."""
    tmp = out + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-Wall", "-Wno-unused-function", "-I", _HERE, src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def _stale() -> bool:
    if not os.path.exists(LIB_PATH):
        return True
    t = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(f) > t for f in (_SRC, _HDR))


def build(force: bool = True) -> str:
    """Compile the oracle (always with force=True; otherwise only when the
    library is missing or older than its sources)."""
    if force or _stale():
        compile_oracle(_SRC, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("flow", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("law", ctypes.c_int32), ("sa_on", ctypes.c_int32), ("plate_start", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("nu", ctypes.c_double), ("rho0", ctypes.c_double), ("force", ctypes.c_double * 3),
        ("u_inlet", ctypes.c_double), ("wall_u_bottom", ctypes.c_double * 3),
        ("wall_u_top", ctypes.c_double * 3), ("nut_init_ratio", ctypes.c_double),
        ("kappa", ctypes.c_double), ("B", ctypes.c_double), ("beta", ctypes.c_double),
        ("cb1", ctypes.c_double), ("cb2", ctypes.c_double), ("sigma", ctypes.c_double),
        ("cw2", ctypes.c_double), ("cw3", ctypes.c_double), ("cv1", ctypes.c_double),
        ("rlim", ctypes.c_double), ("bb_interp", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("wall_dist", ctypes.c_double),
    ]


def params(q=9, nx=4, ny=64, nz=1, flow=CHANNEL, scheme=BB_SLIP, law=REICHARDT, sa_on=1,
           plate_start=0, nu=1e-3, rho0=1.0, force=(0.0, 0.0, 0.0), u_inlet=0.0,
           wall_u_bottom=(0.0, 0.0, 0.0), wall_u_top=(0.0, 0.0, 0.0), nut_init_ratio=3.0,
           kappa=0.41, B=5.2, beta=0.28, collision=BGK, bb_interp=0,
           wall_dist=0.5) -> Params:
    """Parameters with the SA constants listed after eq. 14."""
    p = Params()
    p.q, p.nx, p.ny, p.nz = q, nx, ny, nz
    p.flow, p.scheme, p.law, p.sa_on, p.plate_start = flow, scheme, law, sa_on, plate_start
    p.collision = collision
    p.nu, p.rho0, p.u_inlet = nu, rho0, u_inlet
    p.force[:] = list(force)
    p.wall_u_bottom[:] = list(wall_u_bottom)
    p.wall_u_top[:] = list(wall_u_top)
    p.nut_init_ratio, p.kappa, p.B, p.beta = nut_init_ratio, kappa, B, beta
    p.cb1, p.cb2, p.sigma = 0.1355, 0.622, 2.0 / 3.0
    p.cw2, p.cw3, p.cv1, p.rlim = 0.3, 2.0, 7.1, 10.0
    p.bb_interp, p.wall_dist = bb_interp, wall_dist
    return p


_lib_handle = None


def lib():
    global _lib_handle
    if _lib_handle is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build(force=False)
            L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.POINTER(Params), vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_step.argtypes = [vp, ctypes.c_int64]
        for name in ("orc_ncell", "orc_nwall", "orc_steps"):
            getattr(L, name).restype = ctypes.c_int64
            getattr(L, name).argtypes = [vp]
        for name in ("orc_get_u", "orc_get_rho", "orc_get_nt", "orc_get_nut", "orc_get_f",
                     "orc_totals"):
            getattr(L, name).argtypes = [vp, vp]
        L.orc_get_wall.argtypes = [vp, vp, vp, vp, vp]
        L.orc_lattice.argtypes = [ctypes.c_int, vp, vp, vp]
        L.orc_feq.argtypes = [ctypes.c_int, ctypes.c_double, vp, vp]
        L.orc_collide.argtypes = [ctypes.c_int, vp, ctypes.c_double, vp, vp, vp, vp]
        L.orc_collide_cm.argtypes = [ctypes.c_int, vp, ctypes.c_double, vp, vp, vp, vp]
        for name in ("orc_uplus", "orc_duplus"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double]
        L.orc_solve_utau.restype = ctypes.c_double
        L.orc_solve_utau.argtypes = [ctypes.c_int] + [ctypes.c_double] * 5
        L.orc_sa_rhs.restype = ctypes.c_double
        L.orc_sa_rhs.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_double, vp, vp,
                                 vp, vp, vp, ctypes.c_double]
        L.orc_nut.restype = ctypes.c_double
        L.orc_nut.argtypes = [ctypes.POINTER(Params), ctypes.c_double]
        L.orc_zou_he_west.argtypes = [vp, ctypes.c_double]
        L.orc_regularized.argtypes = [ctypes.c_int, ctypes.c_double, vp, vp, ctypes.c_double, vp]
        L.orc_hrfd_cell.argtypes = [ctypes.POINTER(Params), vp, ctypes.c_int, vp] + \
            [ctypes.c_double] * 5
        L.orc_cai_degrigny_grad.restype = ctypes.c_double
        L.orc_cai_degrigny_grad.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    """Threads of the oracle's row loops (results do not depend on them)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# --- per-cell building blocks ------------------------------------------------
def lattice(q: int):
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    if lib().orc_lattice(q, _ptr(c), _ptr(w), _ptr(opp)) != 0:
        raise ValueError("unknown lattice")
    return c, w, opp


def feq(q: int, rho: float, u) -> np.ndarray:
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.zeros(q)
    lib().orc_feq(q, rho, _ptr(u3), _ptr(out))
    return out


def collide(q: int, f, tau: float, force=(0.0, 0.0, 0.0)):
    f = _f64(f)
    F = np.zeros(3)
    F[: len(force)] = force
    out = np.zeros(q)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib().orc_collide(q, _ptr(f), tau, _ptr(F), _ptr(out), _ptr(rho), _ptr(u))
    return out, float(rho[0]), u


def collide_cm(q: int, f, tau: float, force=(0.0, 0.0, 0.0)):
    f = _f64(f)
    F = np.zeros(3)
    F[: len(force)] = force
    out = np.zeros(q)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib().orc_collide_cm(q, _ptr(f), tau, _ptr(F), _ptr(out), _ptr(rho), _ptr(u))
    return out, float(rho[0]), u


def uplus(law: int, yp: float, kappa=0.41, B=5.2) -> float:
    return lib().orc_uplus(law, yp, kappa, B)


def duplus(law: int, yp: float, kappa=0.41, B=5.2) -> float:
    return lib().orc_duplus(law, yp, kappa, B)


def solve_utau(law: int, ut: float, y: float, nu: float, kappa=0.41, B=5.2) -> float:
    return lib().orc_solve_utau(law, ut, y, nu, kappa, B)


def sa_rhs(p: Params, D: int, nt0, ntm, ntp, u0, um, up, d) -> float:
    a = [_f64(x) for x in (ntm, ntp, u0, um, up)]
    return lib().orc_sa_rhs(ctypes.byref(p), D, nt0, *[_ptr(x) for x in a], d)


def nut(p: Params, nt: float) -> float:
    return lib().orc_nut(ctypes.byref(p), nt)


def zou_he_west(f, U: float) -> np.ndarray:
    f = _f64(f).copy()
    lib().orc_zou_he_west(_ptr(f), U)
    return f


def regularized(q: int, rho: float, u, S, tau: float) -> np.ndarray:
    u3 = np.zeros(3)
    u3[: len(u)] = u
    S = _f64(S).reshape(9)
    out = np.zeros(q)
    lib().orc_regularized(q, rho, _ptr(u3), _ptr(S), tau, _ptr(out))
    return out


def hrfd_cell(p: Params, f, side: int, t, utau: float, uF_t: float, uFF_t: float,
              dudx: float, ntB: float) -> np.ndarray:
    f = _f64(f).copy()
    t3 = np.zeros(3)
    t3[: len(t)] = t
    lib().orc_hrfd_cell(ctypes.byref(p), _ptr(f), side, _ptr(t3), utau, uF_t, uFF_t, dudx, ntB)
    return f


def cai_degrigny_grad(law: int, utau: float, nu: float, yB: float, delta: float,
                      kappa=0.41, B=5.2) -> float:
    return lib().orc_cai_degrigny_grad(law, utau, nu, yB, delta, kappa, B)


# --- whole lattice -------------------------------------------------------------
class Oracle:
    """One lattice advanced by the oracle.  Fields are returned as
    (D, nz, ny, nx) for vectors and (nz, ny, nx) for scalars."""

    def __init__(self, p: Params, u0: np.ndarray | None = None):
        self.p = p
        self.D = 2 if p.q == 9 else 3
        self.shape = (p.nz, p.ny, p.nx)
        u0p = None
        if u0 is not None:
            self._u0 = _f64(u0).reshape(self.D, -1)
            u0p = _ptr(self._u0)
        self.h = lib().orc_create(ctypes.byref(p), u0p)
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.ncell = lib().orc_ncell(self.h)
        self.nwall = lib().orc_nwall(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def step(self, n: int = 1):
        lib().orc_step(self.h, n)

    @property
    def steps(self) -> int:
        return lib().orc_steps(self.h)

    def _get(self, name, n):
        out = np.zeros(n)
        getattr(lib(), name)(self.h, _ptr(out))
        return out

    def u(self):
        return self._get("orc_get_u", self.D * self.ncell).reshape((self.D,) + self.shape)

    def rho(self):
        return self._get("orc_get_rho", self.ncell).reshape(self.shape)

    def nt(self):
        return self._get("orc_get_nt", self.ncell).reshape(self.shape)

    def nut(self):
        return self._get("orc_get_nut", self.ncell).reshape(self.shape)

    def f(self):
        return self._get("orc_get_f", self.p.q * self.ncell).reshape((self.p.q,) + self.shape)

    def totals(self):
        return self._get("orc_totals", 4)

    def wall(self):
        nw = self.nwall
        utau = np.zeros(nw)
        uw = np.zeros((nw, 3))
        t = np.zeros((nw, 3))
        cell = np.zeros(nw, np.int64)
        lib().orc_get_wall(self.h, _ptr(utau), _ptr(uw), _ptr(t), _ptr(cell))
        return {"utau": utau, "uw": uw, "t": t, "cell": cell}
