"""Host-side logic of the learned-guess workflow (no GPU): sample points, the
time-to-accuracy bookkeeping, weight files, and the evaluation summary."""
import os

import numpy as np
import pytest

from paper_0911_4348_amd import learned_guess as LG


def test_sample_points_shape_order_and_seed():
    x = np.linspace(-40.0, 40.0, 199)
    ii, jj, qq = LG.sample_points(7, x, 1025, count=4096)
    assert ii.dtype == np.int32 and len(ii) == len(jj) == len(qq) == 4096
    assert np.all(ii <= jj) and ii.min() >= 0 and jj.max() < 199
    assert qq.min() >= 0 and qq.max() < 1025
    # about half of the index draws come from the nodes with |x| < 10
    core = np.abs(x) < 10.0
    frac_core = np.mean(core[ii]) / 2 + np.mean(core[jj]) / 2
    assert 0.5 < frac_core < 0.8
    # about half of the tau draws lie within 64 points of either end
    near_end = (qq < 64) | (qq > 1024 - 64)
    assert 0.45 < near_end.mean() < 0.65
    # seeded: same seed, same points; another seed, other points
    again = LG.sample_points(7, x, 1025, count=4096)
    assert all(np.array_equal(a, b) for a, b in zip((ii, jj, qq), again))
    assert not np.array_equal(LG.sample_points(8, x, 1025, count=4096)[2], qq)


def _log(energies, ms=10.0):
    rows, prev = [], None
    for E in energies:
        rows.append({"E": E, "dE": (E - prev) if prev is not None else float("inf"), "ms": ms})
        prev = E
    return rows


def test_time_to_reference_accuracy():
    E = [-1.0, -1.2, -1.25, -1.2501, -1.250101, -1.2501011]
    rows = _log(E, ms=10.0)
    wall = 1.0                                   # 0.94 s of set-up before the first record
    k, t = LG._time_to(rows, wall, 1e-6, -1.2501011)   # |E - E_ref| < 1e-6 first at step 4
    assert k == 4 and t == pytest.approx(0.94 + 0.05)
    k, t = LG._time_to(rows, wall, 1e-3, -1.2501011)   # |E_2 - E_ref| = 1.0e-4 < 1e-3 first
    assert k == 2 and t == pytest.approx(0.94 + 0.03)
    k, t = LG._time_to(rows, wall, 1e-12, 0.0)          # never: the whole run
    assert k == len(E) - 1 and t == wall


def test_weights_round_trip_without_pickle(tmp_path):
    p = str(tmp_path / "w.npz")
    params = np.arange(10, dtype=np.float64) * 0.5
    LG.save(p, params, 2.5e-3, {"epochs": 3, "note": "test"})
    got, scale, info = LG.load(p)
    assert got.dtype == np.float32 and np.array_equal(got, params.astype(np.float32))
    assert scale == 2.5e-3 and info == {"epochs": 3, "note": "test"}


def test_shipped_weights_load():
    params, scale, info = LG.load()
    n = sum(i * o + o for i, o in LG.LAYERS)
    assert params.shape == (n,) and np.all(np.isfinite(params)) and scale > 0


def test_summarize():
    rows = [
        {"seed": 1, "iters_hf_start": 30, "iters_learned": 20, "s_hf_start": 3.0, "s_learned": 2.0,
         "err_hf_start": 1e-7, "err_learned": 2e-7, "iters_to_acc_hf_start": 32, "iters_to_acc_learned": 22,
         "s_to_acc_hf_start": 3.2, "s_to_acc_learned": 2.2},
        {"seed": 2, "iters_hf_start": 40, "iters_learned": 41, "s_hf_start": 4.0, "s_learned": 4.2,
         "err_hf_start": 1e-7, "err_learned": 3e-6, "iters_to_acc_hf_start": 42, "iters_to_acc_learned": 40,
         "s_to_acc_hf_start": 4.2, "s_to_acc_learned": 4.0},
        {"seed": 3, "skipped": True, "status": -4},
    ]
    s = LG.summarize(rows)
    assert s["systems"] == 2 and s["skipped_seeds"] == [3]
    r = s["stopping_rule"]
    assert r["mean_iters_hf_start"] == 35 and r["mean_iters_learned"] == 30.5
    assert r["speedup"] == pytest.approx(7.0 / 6.2) and r["systems_with_fewer_iters"] == 1
    assert r["systems_learned_err_above_tol"] == 1
    assert s["to_accuracy"]["speedup"] == pytest.approx(7.4 / 6.2)
