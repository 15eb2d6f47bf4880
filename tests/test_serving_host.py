"""CPU tests of the serving workload's host side: the seeded request stream
(arrivals, mix, ranges) and the summary statistics the benchmark reports."""
import numpy as np
import pytest

from paper_2506_03905_amd import inputs


def test_requests_are_seeded_and_follow_the_mix():
    a = inputs.requests(0, 4000, 50.0)
    assert a == inputs.requests(0, 4000, 50.0)
    assert a != inputs.requests(1, 4000, 50.0)
    t = np.array([r["t_arrival"] for r in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert (gaps > 0).all()
    # exponential gaps of mean 1/50 s: the sample mean within 5 standard errors
    assert abs(gaps.mean() - 0.02) < 5 * 0.02 / np.sqrt(len(gaps))
    kinds = [r["kind"] for r in a]
    frac = kinds.count("channel") / len(kinds)
    assert abs(frac - 0.7) < 5 * np.sqrt(0.7 * 0.3 / len(kinds))
    for r in a:
        assert 32 <= r["ny"] <= 1024 and 500.0 <= r["re_tau"] <= 20000.0
        assert r["nx"] == (4 if r["kind"] == "channel" else 8 * r["ny"])
        assert r["scheme"] in ("slip_bb", "hrfd")
    # log-uniform: log ny and log Re_tau have their medians near mid-range
    ln = np.log([r["ny"] for r in a])
    assert abs(np.median(ln) - 0.5 * (np.log(32) + np.log(1024))) < 0.15
    lr = np.log([r["re_tau"] for r in a])
    assert abs(np.median(lr) - 0.5 * (np.log(500) + np.log(20000))) < 0.15


def test_summary_counts_and_percentiles():
    from paper_2506_03905_amd import lbm as L
    from paper_2506_03905_amd import serving

    res = {}
    for k in range(100):
        st = L.LBM_SLOT_CONVERGED if k < 30 else (L.LBM_SLOT_DIVERGED if k == 99 else L.LBM_SLOT_CAPPED)
        res[k] = {"latency": float(k + 1), "status": st, "steps": 10 * (k + 1), "cells": 256,
                  "converged_by": (1 if k < 10 else 2) if k < 30 else 0}
    s = serving._summary(res, makespan=20.0)
    assert s["solves"] == 100 and s["solves_per_s"] == pytest.approx(5.0)
    assert s["converged"] == 30 and s["capped"] == 69 and s["diverged"] == 1
    assert s["converged_by_residual"] == 10 and s["converged_by_u_tau"] == 20
    assert s["p50_s"] == pytest.approx(np.percentile(np.arange(1, 101), 50))
    assert s["p99_s"] == pytest.approx(np.percentile(np.arange(1, 101), 99))
    assert s["p99_converged_s"] == pytest.approx(np.percentile(np.arange(1, 31), 99))
    assert s["lattice_updates"] == sum(10 * (k + 1) * 256 for k in range(100))
