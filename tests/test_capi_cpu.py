"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/lbm.h declares, and rejects bad input before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2506_03905_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2506_03905_amd import build
        build.build()
    return lbm


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "lbm_step" in names and "lbm_create" in names and "lbm_pool_admit" in names
    assert len(names) >= 28
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(lbm_[a-z_0-9]+)$", out, flags=re.M))
    assert set(names) <= exported


def test_params_default_and_struct_size(L):
    p = L.lbm_params_default()
    assert p.size == ctypes.sizeof(L.lbm_params_t)
    assert (p.kappa, p.B, p.beta, p.cb1, p.cb2, p.cv1, p.rlim) == (0.41, 5.2, 0.28, 0.1355,
                                                                   0.622, 7.1, 10.0)
    assert abs(p.sigma - 2.0 / 3.0) < 1e-16 and p.nut_init_ratio == 3.0


def test_footprint_scales_with_storage(L):
    f32 = L.lbm_footprint(L.LBM_D3Q19, 64, 32, 16, L.lbm_params_default(precision=L.LBM_F32))
    f16 = L.lbm_footprint(L.LBM_D3Q19, 64, 32, 16, L.lbm_params_default(precision=L.LBM_F16))
    f64 = L.lbm_footprint(L.LBM_D3Q19, 64, 32, 16, L.lbm_params_default(precision=L.LBM_F64))
    n = 64 * 32 * 16
    assert f32 - f16 >= 19 * n * 2
    assert f64 > f32 > f16 >= 19 * n * 2
    # one population buffer (single-buffer streaming): f32 populations + fields
    assert f32 < (19 * 4 + 3 * 3 * 4 + 2 * 4) * n + 2 ** 20


@pytest.mark.parametrize("args,msg", [
    ((9, 4, 64, 2), "nz == 1"),
    ((9, 4, 2, 1), "bad dimensions"),
    ((7, 4, 64, 1), "unknown lattice"),
    ((19, 8, 16, 8), None),
])
def test_footprint_validation(L, args, msg):
    p = L.lbm_params_default()
    if msg is None:
        assert L.lbm_footprint(*args, p) > 0
    else:
        with pytest.raises(L.LbmError, match=msg):
            L.lbm_footprint(*args, p)


def test_invalid_parameters_rejected(L):
    for kw, msg in (({"nu": 0.0}, "nu"), ({"scheme": 7}, "scheme"), ({"law": 3}, "law"),
                    ({"precision": 9}, "precision")):
        p = L.lbm_params_default(**kw)
        with pytest.raises(L.LbmError, match=msg):
            L.lbm_footprint(L.LBM_D2Q9, 4, 16, 1, p)
    p = L.lbm_params_default(flow=L.LBM_FLOW_PLATE)
    with pytest.raises(L.LbmError, match="plate"):
        L.lbm_footprint(L.LBM_D3Q19, 16, 16, 4, p)
    p = L.lbm_params_default(scheme=L.LBM_WALL_HRFD)
    with pytest.raises(L.LbmError, match="HRFD"):
        L.lbm_footprint(L.LBM_D3Q19, 16, 16, 4, p)
    # interpolated links: bounce-back schemes only, the wall within one link;
    # halfway links need the wall at 1/2
    for kw in ({"bb_interp": 3}, {"bb_interp": L.LBM_IBB_BOUZIDI, "wall_dist": 0.0},
               {"bb_interp": L.LBM_IBB_YU, "wall_dist": 1.5}, {"wall_dist": 0.3},
               {"bb_interp": L.LBM_IBB_YU, "wall_dist": 0.3, "scheme": L.LBM_WALL_HRFD}):
        p = L.lbm_params_default(**kw)
        with pytest.raises(L.LbmError, match="bb_interp|wall_dist|interpolated"):
            L.lbm_footprint(L.LBM_D2Q9, 4, 16, 1, p)
    # the wall cells' populations are kept for interpolated links
    base = L.lbm_footprint(L.LBM_D2Q9, 4, 16, 1, L.lbm_params_default())
    ibb = L.lbm_footprint(L.LBM_D2Q9, 4, 16, 1,
                          L.lbm_params_default(bb_interp=L.LBM_IBB_YU, wall_dist=0.3))
    assert ibb >= base + 9 * 8 * 8


def test_create_rejects_small_buffer_without_device(L):
    p = L.lbm_params_default()
    h = ctypes.c_void_p()
    rc = L.lib().lbm_create(9, 4, 16, 1, ctypes.byref(p), None, 0, None, ctypes.byref(h))
    assert rc == L.LBM_EINVAL and not h.value
    assert b"too small" in L.lib().lbm_last_error()
    bad = L.lbm_params_default()
    bad.size = 12
    rc = L.lib().lbm_create(9, 4, 16, 1, ctypes.byref(bad), None, 0, None, ctypes.byref(h))
    assert rc == L.LBM_EINVAL


def test_null_handle_calls_fail_cleanly(L):
    lib = L.lib()
    assert lib.lbm_step(None, 1) == L.LBM_ESTATE
    assert lib.lbm_destroy(None) == L.LBM_ESTATE
    assert lib.lbm_ncell(None) == -1
