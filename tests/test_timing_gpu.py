"""Per-launch kernel timing (lbm_set_timing / lbm_get_timing) on the GPU: every
k_step and k_wall launch is counted once, across several lbm_step calls, a
residual reduction and a flush in the middle of a long call, and the timed
launches fit inside the stream time around them."""
import pytest

from paper_2506_03905_amd import inputs, units

pytestmark = pytest.mark.gpu
L = pytest.importorskip("paper_2506_03905_amd.lbm")


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("calls", [(7,), (3, 1, 5), (4100,)])
def test_timing_counts_every_launch(calls):
    _gpu()
    import torch
    nx, ny, nz = 64, 32, 8
    lat = units.channel(2000.0, ny // 2, 0.05)
    p = L.lbm_params_default(precision=L.LBM_F32, scheme=L.LBM_WALL_SLIP_BB, nu=lat["nu"],
                             force=(lat["force"], 0, 0), u_ref=lat["u_bulk"], reduce_every=2)
    g = L.Lattice(L.LBM_D3Q19, nx, ny, nz, p, device="cuda:0")
    # the unperturbed bulk-velocity start: a perturbed BGK channel at this
    # tau - 1/2 diverges within the 4100 steps (and lbm_step says so)
    g.lbm_set_velocity(inputs.channel_velocity(0, 3, nz, ny, nx, lat["u_bulk"], 0.0))
    g.lbm_step(2)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    g.lbm_set_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for n in calls:
        g.lbm_step(n)
    e1.record(s)
    torch.cuda.synchronize()
    tm = g.lbm_get_timing()
    g.lbm_set_timing(False)
    total = sum(calls)
    assert tm["step_launches"] == total and tm["wall_launches"] == total
    assert tm["step_ms"] > 0 and tm["wall_ms"] > 0
    # the timed intervals are disjoint pieces of the stream time
    assert tm["step_ms"] + tm["wall_ms"] <= e0.elapsed_time(e1) * 1.001 + 1e-3
    # timing off: nothing more is counted
    g.lbm_step(3)
    g.lbm_set_timing(True)
    t2 = g.lbm_get_timing()
    assert t2["step_launches"] == 0 and t2["wall_launches"] == 0
    g.lbm_set_timing(False)
    assert g.steps == 2 + total + 3


def test_sampled_timing_counts():
    """lbm_set_timing(every = 10) times the launches of the two steps that
    start at a multiple of 10 (both parities), and nothing else."""
    _gpu()
    import torch
    nx, ny, nz = 64, 32, 8
    lat = units.channel(2000.0, ny // 2, 0.05)
    p = L.lbm_params_default(precision=L.LBM_F32, scheme=L.LBM_WALL_SLIP_BB, nu=lat["nu"],
                             force=(lat["force"], 0, 0), reduce_every=5)
    g = L.Lattice(L.LBM_D3Q19, nx, ny, nz, p, device="cuda:0")
    g.lbm_step(3)
    g.lbm_set_timing(True, every=10)
    g.lbm_step(17)
    g.lbm_step(25)   # steps 3 .. 44
    torch.cuda.synchronize()
    tm = g.lbm_get_timing()
    g.lbm_set_timing(False)
    timed = sum(1 for s in range(3, 45) if s % 10 < 2)
    assert tm["step_launches"] == timed and tm["wall_launches"] == timed
    assert tm["step_ms"] > 0
