"""Serving pool on the GPU: the batched paths agree with the oracle and with
the plain path, and a request's result does not depend on what else is
resident."""
import numpy as np
import pytest

import oracle as O
from paper_2506_03905_amd import inputs, serving, units

pytestmark = pytest.mark.gpu
L = pytest.importorskip("paper_2506_03905_amd.lbm")


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _req(i, kind, ny, re_tau, scheme):
    return {"id": i, "t_arrival": 0.0, "kind": kind, "ny": ny,
            "nx": 4 if kind == "channel" else 8 * ny, "re_tau": re_tau, "scheme": scheme}


def _oracle_for(req, steps):
    lat, nx, ny, nz, p, _ = serving.request_lattice(req)
    op = O.params(q=9, nx=nx, ny=ny, nz=1, flow=p.flow, scheme=p.scheme, law=p.law,
                  sa_on=p.sa_on, plate_start=p.plate_start, nu=p.nu, force=tuple(p.force),
                  u_inlet=p.u_inlet, beta=p.beta, collision=p.collision)
    u0 = np.zeros((2, 1, ny, nx))
    u0[0] = p.u_init[0]
    o = O.Oracle(op, u0)
    o.step(steps)
    return o


@pytest.mark.parametrize("req", [_req(0, "channel", 64, 2000.0, "slip_bb"),
                                 _req(1, "channel", 48, 900.0, "hrfd"),
                                 _req(2, "plate", 16, 800.0, "slip_bb"),
                                 _req(3, "plate", 16, 3000.0, "hrfd")])
def test_batched_fp64_matches_oracle(req):
    """The persistent small-lattice kernel (FP64 storage) against the oracle."""
    _gpu()
    lat, nx, ny, nz, p, _ = serving.request_lattice(req)
    p.precision = L.LBM_F64
    pool = L.Pool(64 << 20, max_slots=8)
    slot = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 0.0, 300)
    pool.lbm_pool_step(300)
    st = pool.lbm_pool_poll(slot)
    assert st["batched"] and st["steps"] == 300 and st["status"] == L.LBM_SLOT_CAPPED
    v = pool.lbm_pool_lattice(slot)
    _, ug, _ = v.lbm_moments()
    o = _oracle_for(req, 300)
    assert np.abs(ug - o.u()).max() / np.abs(o.u()).max() < 1e-10
    ut = v.lbm_wall()["utau"]
    assert np.abs(ut - o.wall()["utau"]).max() / o.wall()["utau"].max() < 1e-10
    pool.close()


@pytest.mark.parametrize("req", [_req(0, "plate", 40, 800.0, "slip_bb"),
                                 _req(1, "plate", 48, 3000.0, "hrfd"),
                                 _req(2, "plate", 40, 1500.0, "cai_degrigny")])
def test_multi_lattice_fp64_matches_oracle(req):
    """The multi-lattice launches of the large-lattice group (FP64 storage)
    against the oracle, through a cap that is not a multiple of the chunk."""
    _gpu()
    lat, nx, ny, nz, p, _ = serving.request_lattice(req)
    p.precision = L.LBM_F64
    pool = L.Pool(256 << 20, max_slots=8)
    slot = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 0.0, 250)
    pool.lbm_pool_step(100)
    pool.lbm_pool_step(100)
    pool.lbm_pool_step(100)
    st = pool.lbm_pool_poll(slot)
    assert not st["batched"] and st["steps"] == 250 and st["status"] == L.LBM_SLOT_CAPPED
    v = pool.lbm_pool_lattice(slot)
    _, ug, _ = v.lbm_moments()
    o = _oracle_for(req, 250)
    assert np.abs(ug - o.u()).max() / np.abs(o.u()).max() < 1e-10
    ut = v.lbm_wall()["utau"]
    assert np.abs(ut - o.wall()["utau"]).max() / o.wall()["utau"].max() < 1e-10
    pool.close()


def test_pool_interpolated_links_fp64_matches_oracle():
    """Yu's rule on a plate and Bouzidi's on a channel, in both pool groups."""
    _gpu()
    cases = [("plate", 48, 1500.0, L.LBM_IBB_YU, 0.3), ("channel", 32, 2000.0, L.LBM_IBB_BOUZIDI, 0.7)]
    pool = L.Pool(256 << 20, max_slots=8)
    slots = []
    for kind, ny, rt, interp, q in cases:
        req = _req(0, kind, ny, rt, "slip_bb")
        lat, nx, ny_, nz, p, _ = serving.request_lattice(req)
        p.precision, p.bb_interp, p.wall_dist = L.LBM_F64, interp, q
        slots.append((pool.lbm_pool_admit(lat, nx, ny_, nz, p, None, 0.0, 220), p, nx, ny_))
    pool.lbm_pool_step(220)
    for (slot, p, nx, ny), (kind, *_rest) in zip(slots, cases):
        st = pool.lbm_pool_poll(slot)
        assert st["steps"] == 220 and st["batched"] == (kind == "channel")
        op = O.params(q=9, nx=nx, ny=ny, nz=1, flow=p.flow, scheme=p.scheme, law=p.law,
                      sa_on=p.sa_on, plate_start=p.plate_start, nu=p.nu, force=tuple(p.force),
                      u_inlet=p.u_inlet, beta=p.beta, collision=p.collision,
                      bb_interp=p.bb_interp, wall_dist=p.wall_dist)
        u0 = np.zeros((2, 1, ny, nx))
        u0[0] = p.u_init[0]
        o = O.Oracle(op, u0)
        o.step(220)
        ug = pool.lbm_pool_lattice(slot).lbm_moments()[1]
        assert np.abs(ug - o.u()).max() / np.abs(o.u()).max() < 1e-10
    pool.close()


def test_multi_lattice_d3q19_fp64_matches_oracle():
    """A D3Q19 channel in the pool (large-lattice group) against the oracle."""
    _gpu()
    lat = units.channel(5000.0, 6)
    nx, ny, nz = 5, 12, 4
    u0 = inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], 1e-3)
    p = L.lbm_params_default(precision=L.LBM_F64, scheme=L.LBM_WALL_SLIP_BB, nu=lat["nu"],
                             force=(lat["force"] * 10, 0, 0), reduce_every=10)
    pool = L.Pool(64 << 20, max_slots=4)
    slot = pool.lbm_pool_admit(L.LBM_D3Q19, nx, ny, nz, p, u0, 0.0, 25)
    pool.lbm_pool_step(40)
    st = pool.lbm_pool_poll(slot)
    assert not st["batched"] and st["steps"] == 25
    _, ug, _ = pool.lbm_pool_lattice(slot).lbm_moments()
    op = O.params(q=19, nx=nx, ny=ny, nz=nz, nu=lat["nu"], force=(lat["force"] * 10, 0, 0),
                  scheme=O.BB_SLIP)
    o = O.Oracle(op, u0)
    o.step(25)
    assert np.abs(ug - o.u()).max() / np.abs(o.u()).max() < 1e-11
    pool.close()


def test_pump_staggered_admission_equals_alone():
    """Continuous batching: requests admitted while others are on the device
    (staggered through lbm_pool_pump) end with the same fields, steps and
    status as each request run alone."""
    _gpu()
    reqs = [_req(0, "channel", 64, 2000.0, "slip_bb"), _req(1, "plate", 64, 1200.0, "hrfd"),
            _req(2, "channel", 200, 6000.0, "hrfd"), _req(3, "plate", 24, 900.0, "slip_bb")]
    cap = 700

    def run(subset, stagger):
        pool = L.Pool(1 << 30, max_slots=16)
        pending = list(subset)
        slots, done = {}, {}
        while pending or len(done) < len(slots):
            if pending:
                r = pending.pop(0)
                lat, nx, ny, nz, p, _ = serving.request_lattice(r)
                slots[r["id"]] = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 0.0, cap)
            for _ in range(stagger if pending else 1):
                pool.lbm_pool_pump(100)
            for i, sl in slots.items():
                st = pool.lbm_pool_poll(sl)
                if i not in done and st["status"] != L.LBM_SLOT_RUNNING:
                    done[i] = (st["steps"], st["status"], pool.lbm_pool_lattice(sl).lbm_moments()[1])
        pool.close()
        return done

    mixed = run(reqs, 3)
    for r in reqs:
        alone = run([r], 1)[r["id"]]
        got = mixed[r["id"]]
        assert got[0] == alone[0] == cap and got[1] == alone[1] == L.LBM_SLOT_CAPPED
        assert np.array_equal(got[2], alone[2]), r


def test_alone_equals_mixed_bitwise():
    """Each request's fields after the same number of steps are bitwise equal
    whether it runs alone or together with others (small and large tiers)."""
    _gpu()
    reqs = [_req(0, "channel", 64, 2000.0, "slip_bb"), _req(1, "plate", 16, 1200.0, "hrfd"),
            _req(2, "plate", 320, 5000.0, "slip_bb"), _req(3, "channel", 128, 9000.0, "hrfd")]
    steps = 400

    def run(subset):
        pool = L.Pool(2 << 30, max_slots=16)
        slots = {}
        for r in subset:
            lat, nx, ny, nz, p, _ = serving.request_lattice(r)
            slots[r["id"]] = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 0.0, steps)
        pool.lbm_pool_step(150)
        pool.lbm_pool_step(250)
        out = {}
        for i, s in slots.items():
            st = pool.lbm_pool_poll(s)
            assert st["steps"] == steps
            out[i] = (pool.lbm_pool_lattice(s).lbm_moments()[1], st["batched"])
        pool.close()
        return out

    mixed = run(reqs)
    assert mixed[0][1] and mixed[1][1] and not mixed[2][1]
    for r in reqs:
        alone = run([r])
        assert np.array_equal(alone[r["id"]][0], mixed[r["id"]][0]), r


def test_batched_matches_plain_path():
    """Persistent batched kernel vs the per-lattice kernels, FP32."""
    _gpu()
    req = _req(0, "channel", 96, 4000.0, "slip_bb")
    lat, nx, ny, nz, p, _ = serving.request_lattice(req)
    pool = L.Pool(64 << 20, max_slots=4)
    slot = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 0.0, 1000)
    pool.lbm_pool_step(1000)
    ub = pool.lbm_pool_lattice(slot).lbm_moments()[1]
    g = L.Lattice(lat, nx, ny, nz, p)
    g.lbm_step(1000)
    up = g.lbm_moments()[1]
    assert np.abs(ub - up).max() / np.abs(up).max() < 1e-5
    pool.close()


def test_admission_by_footprint_and_release():
    _gpu()
    req = _req(0, "channel", 256, 2000.0, "slip_bb")
    need = serving.footprint(req)
    # room for the slot descriptors and exactly two lattices
    pool = L.Pool(2 * need + 16384, max_slots=8)
    lat, nx, ny, nz, p, _ = serving.request_lattice(req)
    a = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 1e-8, 100)
    b = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 1e-8, 100)
    assert a is not None and b is not None
    assert pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 1e-8, 100) is None  # full
    pool.lbm_pool_release(a)
    c = pool.lbm_pool_admit(lat, nx, ny, nz, p, None, 1e-8, 100)
    assert c is not None
    pool.lbm_pool_release(b)
    pool.lbm_pool_release(c)
    assert pool.lbm_pool_free_bytes() >= 2 * need
    pool.close()


def test_converged_requests_stop():
    """A loose tolerance stops every request early, at a reduction step."""
    _gpu()
    reqs = [_req(i, k, ny, rt, s) for i, (k, ny, rt, s) in
            enumerate([("channel", 32, 800.0, "slip_bb"), ("channel", 64, 3000.0, "hrfd"),
                       ("plate", 32, 1000.0, "slip_bb")])]
    res, summ = serving.run_batched(reqs, 256 << 20, chunk=300, tol=1e-4, max_steps=20000)
    assert summ["solves"] == 3 and summ["diverged"] == 0
    for r in res.values():
        assert r["status"] == L.LBM_SLOT_CONVERGED and r["steps"] % 100 == 0
        assert r["residual"] < 1e-4


@pytest.mark.parametrize("kind,ny", [("channel", 64), ("plate", 40)])
def test_diverging_request_is_evicted_others_unchanged(kind, ny):
    """One request starts from a field with a NaN (small persistent group for
    the channel, multi-lattice group for the plate): the pool reports it
    diverged at its first reduction and it can be released, while the two
    requests resident beside it end bitwise equal to their runs alone."""
    _gpu()
    reqs = [_req(0, kind, ny, 2000.0, "slip_bb"), _req(1, kind, ny, 3000.0, "hrfd"),
            _req(2, kind, ny, 1500.0, "slip_bb")]
    cap = 300

    def admit(pool, r, poison):
        lat, nx, ny_, nz, p, _ = serving.request_lattice(r)
        u0 = None
        if poison:
            u0 = np.zeros((2, 1, ny_, nx))
            u0[0] = p.u_init[0]
            u0[0, 0, ny_ // 2, nx // 2] = np.nan
        return pool.lbm_pool_admit(lat, nx, ny_, nz, p, u0, 0.0, cap)

    def run(ids, poison_id=None):
        pool = L.Pool(512 << 20, max_slots=8)
        slots = {i: admit(pool, reqs[i], i == poison_id) for i in ids}
        pool.lbm_pool_step(150)
        out = {}
        if poison_id is not None:
            st = pool.lbm_pool_poll(slots[poison_id])
            assert st["status"] == L.LBM_SLOT_DIVERGED and st["steps"] == 100, st
            pool.lbm_pool_release(slots[poison_id])
        pool.lbm_pool_step(200)
        for i in ids:
            if i == poison_id:
                continue
            st = pool.lbm_pool_poll(slots[i])
            assert st["status"] == L.LBM_SLOT_CAPPED and st["steps"] == cap
            out[i] = (pool.lbm_pool_lattice(slots[i]).lbm_moments()[1], st["mean_u_tau"],
                      st["batched"])
        pool.close()
        return out

    mixed = run([0, 1, 2], poison_id=1)
    assert mixed[0][2] == (kind == "channel")
    for i in (0, 2):
        alone = run([i])[i]
        assert np.array_equal(alone[0], mixed[i][0]) and alone[1] == mixed[i][1], i


def test_u_tau_criterion_batched_and_sequential():
    """The paper's criterion (relative change of u_tau between reductions
    below tol_utau, Sec. 4.1.1) retires requests at a reduction step; the
    batched pool and the one-at-a-time path stop the same requests at the same
    step and say which criterion fired."""
    _gpu()
    reqs = [_req(i, k, ny, rt, s) for i, (k, ny, rt, s) in
            enumerate([("channel", 32, 800.0, "slip_bb"), ("channel", 48, 3000.0, "hrfd"),
                       ("plate", 24, 1000.0, "slip_bb"), ("channel", 300, 5000.0, "slip_bb")])]
    kw = dict(tol=0.0, tol_utau=1e-4, max_steps=20000)
    rb, sb = serving.run_batched(reqs, 512 << 20, chunk=300, **kw)
    rs, ss = serving.run_sequential(reqs, honor_arrivals=False, **kw)
    assert sb["converged_by_u_tau"] >= 1 and sb["converged_by_residual"] == 0
    for r in reqs:
        b, q = rb[r["id"]], rs[r["id"]]
        assert (b["status"], b["steps"], b["converged_by"]) == (q["status"], q["steps"], q["converged_by"]), r
        if b["status"] == L.LBM_SLOT_CONVERGED:
            assert b["steps"] % 100 == 0 and 0 <= b["d_u_tau_rel"] < 1e-4


@pytest.mark.parametrize("wall", ["slip_bb", "hrfd_0.28", "cai_degrigny", "bouzidi_0.75"])
def test_replication_cases_match_oracle(wall):
    """Channel cases of the Sec. 4.1 study harness (Table 3 grid, N = 5 and
    20 at Re_tau 4200, FP64, CM + SA, Dean start), run through the serving
    pool for 300 steps, against the oracle element-wise (u and u_tau)."""
    _gpu()
    from paper_2506_03905_amd import replicate as R
    if wall == "bouzidi_0.75":
        cases = [c for c in R.cases(["wall"]) if c["q"] == 0.75]
    else:
        cases = [c for c in R.cases(["grid"]) if c["wall"] == wall and c["n"] in (5, 20)]
    assert cases
    rows = R.run(cases, tol=0.0, max_steps=300, chunk=150, keep_fields=True)
    for c, row in zip(cases, rows):
        ny, h, u_b, u_tau, p = R.lattice_of(c)
        assert row["steps"] == 300
        op = O.params(q=9, nx=4, ny=ny, nz=1, scheme=p.scheme, law=p.law, sa_on=p.sa_on, nu=p.nu,
                      force=tuple(p.force), beta=p.beta, collision=p.collision,
                      bb_interp=p.bb_interp, wall_dist=p.wall_dist)
        u0 = np.zeros((2, 1, ny, 4))
        u0[0] = u_b
        o = O.Oracle(op, u0)
        o.step(300)
        assert np.abs(row["u"] - o.u()).max() / np.abs(o.u()).max() < 1e-10, c
        ut = o.wall()["utau"]
        assert np.abs(row["utau"] - ut).max() / ut.max() < 1e-10, c
