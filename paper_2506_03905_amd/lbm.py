"""ctypes binding of ``liblbm.so`` (C ABI: ``include/lbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies the device buffer and the stream.  The library is loaded on
first use; if it is missing the call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_D2Q9, LBM_D3Q19 = 9, 19
LBM_F64, LBM_F32, LBM_F16, LBM_BF16 = 0, 1, 2, 3
LBM_FLOW_CHANNEL, LBM_FLOW_PLATE = 0, 1
LBM_WALL_FIXED_BB, LBM_WALL_SLIP_BB, LBM_WALL_HRFD, LBM_WALL_CAI_DEGRIGNY = 0, 1, 2, 3
LBM_IBB_HALFWAY, LBM_IBB_BOUZIDI, LBM_IBB_YU = 0, 1, 2
LBM_LAW_REICHARDT, LBM_LAW_SA = 0, 1
LBM_COLL_BGK, LBM_COLL_CM = 0, 1
LBM_OUT_F64, LBM_OUT_F32 = 0, 1
LBM_ON_HOST, LBM_ON_DEVICE = 0, 1
OUT_DTYPE = {"f64": (LBM_OUT_F64, np.float64), "f32": (LBM_OUT_F32, np.float32)}

PRECISION = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16, "bf16": LBM_BF16}
SCHEME = {"fixed_bb": LBM_WALL_FIXED_BB, "slip_bb": LBM_WALL_SLIP_BB, "hrfd": LBM_WALL_HRFD,
          "cai_degrigny": LBM_WALL_CAI_DEGRIGNY}


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_params_t(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_int32), ("version", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("scheme", ctypes.c_int32), ("law", ctypes.c_int32),
        ("sa_on", ctypes.c_int32), ("plate_start", ctypes.c_int32),
        ("reduce_every", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("nu", ctypes.c_double), ("rho0", ctypes.c_double), ("force", ctypes.c_double * 3),
        ("u_init", ctypes.c_double * 3), ("u_inlet", ctypes.c_double), ("u_ref", ctypes.c_double),
        ("wall_u_bottom", ctypes.c_double * 3), ("wall_u_top", ctypes.c_double * 3),
        ("nut_init_ratio", ctypes.c_double), ("kappa", ctypes.c_double), ("B", ctypes.c_double),
        ("beta", ctypes.c_double), ("cb1", ctypes.c_double), ("cb2", ctypes.c_double),
        ("sigma", ctypes.c_double), ("cw2", ctypes.c_double), ("cw3", ctypes.c_double),
        ("cv1", ctypes.c_double), ("rlim", ctypes.c_double), ("store_shift_u", ctypes.c_double),
        ("bb_interp", ctypes.c_int32), ("pad_", ctypes.c_int32), ("wall_dist", ctypes.c_double),
    ]


class lbm_residual_t(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("steps_since_previous", ctypes.c_int64),
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
        ("l2_du_rel", ctypes.c_double), ("mean_u_tau", ctypes.c_double),
        ("d_u_tau_rel", ctypes.c_double), ("nan_flag", ctypes.c_double),
    ]


class lbm_pool_status_t(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("batched", ctypes.c_int32), ("steps", ctypes.c_int64),
        ("residual", ctypes.c_double), ("mean_u_tau", ctypes.c_double),
        ("footprint", ctypes.c_int64), ("d_u_tau_rel", ctypes.c_double),
        ("converged_by", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


LBM_SLOT_IDLE, LBM_SLOT_RUNNING, LBM_SLOT_CONVERGED, LBM_SLOT_CAPPED, LBM_SLOT_DIVERGED = range(5)


class lbm_timing_t(ctypes.Structure):
    _fields_ = [
        ("step_launches", ctypes.c_int64), ("step_ms", ctypes.c_double),
        ("wall_launches", ctypes.c_int64), ("wall_ms", ctypes.c_double),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -m paper_2506_03905_amd.build)")
    # torch ships its own HIP runtime with the same soname as the system one
    # the library links; the process must use one runtime for both (torch's
    # streams and buffers are handed to the library), and it works when
    # torch's is loaded first, so load torch before the library.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    P = ctypes.POINTER(lbm_params_t)
    sig = {
        "lbm_params_default": (None, [P]),
        "lbm_footprint": (i64, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]),
        "lbm_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                                      vp, i64, vp, ctypes.POINTER(vp)]),
        "lbm_set_velocity": (ctypes.c_int, [vp, vp, ctypes.c_int]),
        "lbm_set_wall_bc": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_double]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_moments": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_moments_noalloc": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_nu_tilde": (ctypes.c_int, [vp, vp, ctypes.c_int]),
        "lbm_populations": (ctypes.c_int, [vp, vp]),
        "lbm_wall": (ctypes.c_int, [vp, vp, vp, vp, vp, i64]),
        "lbm_ncell": (i64, [vp]),
        "lbm_nwall": (i64, [vp]),
        "lbm_steps": (i64, [vp]),
        "lbm_residual": (ctypes.c_int, [vp, ctypes.POINTER(lbm_residual_t)]),
        "lbm_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "lbm_get_timing": (ctypes.c_int, [vp, ctypes.POINTER(lbm_timing_t)]),
        "lbm_checkpoint_bytes": (i64, [vp]),
        "lbm_save": (ctypes.c_int, [vp, vp, i64]),
        "lbm_load": (ctypes.c_int, [vp, vp, i64]),
        "lbm_destroy": (ctypes.c_int, [vp]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_pool_create": (ctypes.c_int, [vp, i64, ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "lbm_pool_free_bytes": (i64, [vp]),
        "lbm_pool_admit": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          P, vp, ctypes.c_double, ctypes.c_double, i64,
                                          ctypes.POINTER(ctypes.c_int)]),
        "lbm_pool_step": (ctypes.c_int, [vp, i64]),
        "lbm_pool_pump": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_int)]),
        "lbm_pool_poll": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(lbm_pool_status_t)]),
        "lbm_pool_lattice": (vp, [vp, ctypes.c_int]),
        "lbm_pool_release": (ctypes.c_int, [vp, ctypes.c_int]),
        "lbm_pool_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())


def lbm_params_default(**overrides) -> lbm_params_t:
    p = lbm_params_t()
    lib().lbm_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k in ("force", "u_init", "wall_u_bottom", "wall_u_top"):
            arr = getattr(p, k)
            for a in range(3):
                arr[a] = float(v[a]) if a < len(v) else 0.0
        else:
            if not hasattr(p, k):
                raise AttributeError(k)
            setattr(p, k, v)
    return p


def lbm_footprint(lattice: int, nx: int, ny: int, nz: int, p: lbm_params_t) -> int:
    n = lib().lbm_footprint(lattice, nx, ny, nz, ctypes.byref(p))
    if n < 0:
        _check(int(n))
    return int(n)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Lattice:
    """One lattice resident in a caller-owned device buffer (a torch tensor)."""

    def __init__(self, lattice: int, nx: int, ny: int, nz: int, p: lbm_params_t,
                 device="cuda", stream=None, buffer=None):
        import torch

        self.lattice, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.D = 2 if lattice == LBM_D2Q9 else 3
        self.p = p
        self.bytes = lbm_footprint(lattice, nx, ny, nz, p)
        if buffer is None:
            buffer = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        self.buffer = buffer  # keeps the device memory alive
        base = buffer.data_ptr()
        aligned = (base + 255) & ~255
        avail = buffer.numel() - (aligned - base)
        self.stream = stream if stream is not None else torch.cuda.current_stream(buffer.device)
        h = ctypes.c_void_p()
        _check(lib().lbm_create(lattice, nx, ny, nz, ctypes.byref(p), ctypes.c_void_p(aligned),
                                avail, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.ncell = int(lib().lbm_ncell(h))
        self.nwall = int(lib().lbm_nwall(h))
        self.shape = (nz, ny, nx)

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- C ABI with the same names -----------------------------------------
    def lbm_set_velocity(self, u: np.ndarray):
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.D, -1))
        if u.shape[1] != self.ncell:
            raise ValueError("velocity field has the wrong size")
        _check(lib().lbm_set_velocity(self.h, _ptr(u), 0))

    def lbm_set_wall_bc(self, scheme: int, beta: float = 0.28):
        _check(lib().lbm_set_wall_bc(self.h, scheme, beta))

    def lbm_step(self, n: int = 1):
        _check(lib().lbm_step(self.h, n))

    def lbm_moments(self, dtype: str = "f64"):
        """(rho, u, nu_t) of the last step as host arrays of the given dtype."""
        code, npt = OUT_DTYPE[dtype]
        rho = np.zeros(self.ncell, npt)
        u = np.zeros(self.D * self.ncell, npt)
        nut = np.zeros(self.ncell, npt)
        _check(lib().lbm_moments(self.h, _ptr(rho), _ptr(u), _ptr(nut), code, LBM_ON_HOST))
        return (rho.reshape(self.shape), u.reshape((self.D,) + self.shape),
                nut.reshape(self.shape))

    def lbm_moments_noalloc(self, dtype: str = "f64", fields=("rho", "u", "nut")):
        """lbm_moments to host arrays staged through the library's static
        scratch (no device allocation); skipped fields come back as None."""
        code, npt = OUT_DTYPE[dtype]
        out = {"rho": np.zeros(self.ncell, npt) if "rho" in fields else None,
               "u": np.zeros(self.D * self.ncell, npt) if "u" in fields else None,
               "nut": np.zeros(self.ncell, npt) if "nut" in fields else None}
        ptr = lambda a: _ptr(a) if a is not None else None
        _check(lib().lbm_moments_noalloc(self.h, ptr(out["rho"]), ptr(out["u"]), ptr(out["nut"]), code,
                                         LBM_ON_HOST))
        return (None if out["rho"] is None else out["rho"].reshape(self.shape),
                None if out["u"] is None else out["u"].reshape((self.D,) + self.shape),
                None if out["nut"] is None else out["nut"].reshape(self.shape))

    def lbm_moments_device(self, rho=None, u=None, nut=None, dtype: str = "f64"):
        """The same into caller device tensors (None skips a field); asynchronous
        on the lattice's stream."""
        code, _ = OUT_DTYPE[dtype]
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _check(lib().lbm_moments(self.h, ptr(rho), ptr(u), ptr(nut), code, LBM_ON_DEVICE))

    def lbm_nu_tilde(self):
        nt = np.zeros(self.ncell)
        _check(lib().lbm_nu_tilde(self.h, _ptr(nt), 0))
        return nt.reshape(self.shape)

    def lbm_populations(self):
        f = np.zeros(self.lattice * self.ncell)
        _check(lib().lbm_populations(self.h, _ptr(f)))
        return f.reshape((self.lattice,) + self.shape)

    def lbm_wall(self):
        nw = self.nwall
        ut, cf = np.zeros(nw), np.zeros(nw)
        t, uw = np.zeros((nw, 3)), np.zeros((nw, 3))
        _check(lib().lbm_wall(self.h, _ptr(ut), _ptr(cf), _ptr(t), _ptr(uw), nw))
        return {"utau": ut, "cf": cf, "t": t, "uw": uw}

    def lbm_residual(self) -> dict:
        r = lbm_residual_t()
        rc = lib().lbm_residual(self.h, ctypes.byref(r))
        out = {"step": r.step, "steps_since_previous": r.steps_since_previous, "mass": r.mass,
               "momentum": list(r.momentum), "l2_du_rel": r.l2_du_rel,
               "mean_u_tau": r.mean_u_tau, "d_u_tau_rel": r.d_u_tau_rel, "nan_flag": r.nan_flag,
               "rc": rc}
        if rc not in (LBM_OK, LBM_EDIVERGED):
            _check(rc)
        return out

    def lbm_set_timing(self, on: bool, every: int = 1):
        """Per-launch kernel timing; every > 1 times 2 consecutive steps in
        every `every` steps (both step parities, fewer events on the stream)."""
        _check(lib().lbm_set_timing(self.h, (every if every > 1 else 1) if on else 0))

    def lbm_get_timing(self) -> dict:
        t = lbm_timing_t()
        _check(lib().lbm_get_timing(self.h, ctypes.byref(t)))
        return {"step_launches": t.step_launches, "step_ms": t.step_ms,
                "wall_launches": t.wall_launches, "wall_ms": t.wall_ms}

    def lbm_save(self) -> bytes:
        n = int(lib().lbm_checkpoint_bytes(self.h))
        buf = ctypes.create_string_buffer(n)
        _check(lib().lbm_save(self.h, buf, n))
        return buf.raw

    def lbm_load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().lbm_load(self.h, buf, len(blob)))

    @property
    def steps(self) -> int:
        return int(lib().lbm_steps(self.h))

    def lbm_steps(self) -> int:
        return int(lib().lbm_steps(self.h))

    def lbm_ncell(self) -> int:
        return int(lib().lbm_ncell(self.h))

    def lbm_nwall(self) -> int:
        return int(lib().lbm_nwall(self.h))


class _View(Lattice):
    """A lattice handle owned by a pool slot (exports only)."""

    def __init__(self, h, lattice, nx, ny, nz):
        self.h = ctypes.c_void_p(h)
        self.lattice, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.D = 2 if lattice == LBM_D2Q9 else 3
        self.ncell = int(lib().lbm_ncell(self.h))
        self.nwall = int(lib().lbm_nwall(self.h))
        self.shape = (nz, ny, nx)

    def close(self):
        self.h = None  # the pool owns the handle


class Pool:
    """The serving pool of the C ABI (lbm_pool_*) in one torch device buffer."""

    def __init__(self, nbytes: int, max_slots: int = 1024, device="cuda", stream=None):
        import torch

        self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buffer.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.buffer.device)
        h = ctypes.c_void_p()
        _check(lib().lbm_pool_create(ctypes.c_void_p(aligned), nbytes, max_slots,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.dims = {}

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lbm_pool_free_bytes(self) -> int:
        return int(lib().lbm_pool_free_bytes(self.h))

    def lbm_pool_admit(self, lattice, nx, ny, nz, p, u0=None, tol=1e-8, max_steps=10 ** 6,
                       tol_utau=0.0):
        """Returns the slot index, or None when the pool cannot hold it (LBM_ENOMEM)."""
        slot = ctypes.c_int(-1)
        ptr = None
        if u0 is not None:
            u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.float64))
            ptr = _ptr(u0)
        rc = lib().lbm_pool_admit(self.h, lattice, nx, ny, nz, ctypes.byref(p), ptr, tol,
                                  tol_utau, int(max_steps), ctypes.byref(slot))
        if rc == LBM_ENOMEM:
            return None
        _check(rc)
        self.dims[slot.value] = (lattice, nx, ny, nz)
        return slot.value

    def lbm_pool_step(self, steps: int):
        _check(lib().lbm_pool_step(self.h, int(steps)))

    def lbm_pool_pump(self, steps: int) -> int:
        """Non-blocking: harvest finished chunks, launch the next ones; returns
        the number of groups (0-2) with work on the device."""
        n = ctypes.c_int(0)
        _check(lib().lbm_pool_pump(self.h, int(steps), ctypes.byref(n)))
        return n.value

    def lbm_pool_poll(self, slot: int) -> dict:
        st = lbm_pool_status_t()
        _check(lib().lbm_pool_poll(self.h, slot, ctypes.byref(st)))
        return {"status": st.status, "batched": bool(st.batched), "steps": st.steps,
                "residual": st.residual, "mean_u_tau": st.mean_u_tau,
                "footprint": st.footprint, "d_u_tau_rel": st.d_u_tau_rel,
                "converged_by": st.converged_by}

    def lbm_pool_lattice(self, slot: int) -> Lattice:
        h = lib().lbm_pool_lattice(self.h, slot)
        if not h:
            raise LbmError(LBM_EINVAL, f"bad slot {slot}")
        return _View(h, *self.dims[slot])

    def lbm_pool_release(self, slot: int):
        _check(lib().lbm_pool_release(self.h, slot))
        self.dims.pop(slot, None)
