"""Host logic of the serving form (no GPU): request mix, parameter mapping
with the viscosity floor, first-fit arena, nearest-rank percentiles."""
import math

import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import lbm, serve


def test_serving_requests_deterministic_and_in_range():
    a = lbm_inputs.serving_requests(64, seed=4)
    b = lbm_inputs.serving_requests(64, seed=4)
    assert a == b
    assert a != lbm_inputs.serving_requests(64, seed=5)
    for r in a:
        assert 128 <= r["nx"] <= 1024 and r["ny"] in (r["nx"], 2 * r["nx"])
        assert 8 <= r["d"] <= 24 and 500 <= r["steps"] <= 5000
        assert 1e5 <= r["Ra"] <= 1e8
        fill = r["n"] * math.pi * r["d"] ** 2 / 4 / (r["nx"] * r["ny"])
        assert fill <= 0.2 + 1e-12 and r["n"] <= 400


def test_poisson_arrivals_mean_gap():
    t = lbm_inputs.poisson_arrivals(20000, rate=4.0, seed=9)
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.25) < 0.01          # mean 1/rate
    assert abs(gaps.std() - 0.25) < 0.015          # exponential: std = mean


def test_request_params_viscosity_floor():
    low = dict(nx=128, ny=128, d=10.0, n=5, Ra=1e8, steps=10, seed=1)
    p, capped = serve.request_params(low)
    assert capped and p.nu == pytest.approx(serve.NU_MIN) and p.alpha == pytest.approx(serve.NU_MIN / 0.7)
    high = dict(low, Ra=1e5)
    p, capped = serve.request_params(high)
    assert not capped and p.nu > serve.NU_MIN
    assert p.storage == lbm.STORE["shift_bf16"] and p.max_particles == 5 and lbm.lbm_bytes_required(p) > 0


def test_first_fit_alloc_release_merge():
    a = serve.FirstFit(10 * serve.ALIGN)
    x = a.alloc(1)
    y = a.alloc(3 * serve.ALIGN)
    z = a.alloc(2 * serve.ALIGN + 5)
    assert x == (0, serve.ALIGN) and y == (serve.ALIGN, 3 * serve.ALIGN)
    assert z == (4 * serve.ALIGN, 3 * serve.ALIGN)
    assert a.alloc(4 * serve.ALIGN) is None
    a.release(*y)
    assert a.alloc(3 * serve.ALIGN) == y          # the freed hole is reused first
    a.release(*x)
    a.release(*y)
    a.release(*z)
    assert a.free == [(0, 10 * serve.ALIGN)] and a.used() == 0


def test_nearest_rank_percentiles():
    v = list(range(1, 257))
    assert serve.percentile_nearest_rank(v, 0.5) == 128
    assert serve.percentile_nearest_rank(v, 0.99) == 254
    assert serve.percentile_nearest_rank([3.0], 0.99) == 3.0


def test_summary_splits_capped_and_uncapped_requests():
    recs = [dict(status="ok", latency=float(i + 1), nodes=100, steps=10, ra_capped=(i % 3 == 0))
            for i in range(9)]
    recs.append(dict(status="rejected: over budget", arrival=0.0))
    s = serve.summarize(recs, wall=2.0)
    assert s["requests"] == 10 and s["failed"] == 1 and s["completed"] == 9
    assert s["ra_capped"] == 3 and s["capped"]["completed"] == 3 and s["uncapped"]["completed"] == 6
    # capped latencies 1, 4, 7; uncapped 2, 3, 5, 6, 8, 9 (nearest rank)
    assert s["capped"]["p50_s"] == 4.0 and s["capped"]["p99_s"] == 7.0
    assert s["uncapped"]["p50_s"] == 5.0 and s["uncapped"]["p99_s"] == 9.0
    assert s["mlups"] == pytest.approx(9 * 1000 / 2.0 / 1e6)
    assert s["capped"]["mlups"] + s["uncapped"]["mlups"] == pytest.approx(s["mlups"])
