"""Pins for oracle.post (windows, integration, Kendall tau-b) and oracle.quant."""
import numpy as np
import pytest
import scipy.stats
import torch

import oracle
from oracle.post import n_windows


def test_integrate_three_ways():
    p = np.random.default_rng(0).standard_normal(300)
    W = 16
    I = oracle.integrate(p, W)
    c = np.concatenate([[0.0], np.cumsum(p)])
    np.testing.assert_allclose(I, (c[W:] - c[:-W]) / W, atol=1e-12)
    np.testing.assert_allclose(I, np.convolve(p, np.ones(W) / W, mode="valid"), atol=1e-12)
    assert len(oracle.integrate(p[:10], W)) == 0
    np.testing.assert_allclose(oracle.integrate(p, 1), p)


def test_kendall_matches_scipy():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(200)
    b = a + 0.3 * rng.standard_normal(200)
    assert oracle.kendall_tau_b(a, b) == pytest.approx(scipy.stats.kendalltau(a, b).statistic, abs=1e-12)
    a2 = np.round(a, 1)
    b2 = np.round(b, 1)                      # ties in both
    assert oracle.kendall_tau_b(a2, b2) == pytest.approx(scipy.stats.kendalltau(a2, b2).statistic, abs=1e-12)
    assert oracle.kendall_tau_b(a, a) == pytest.approx(1.0)
    assert oracle.kendall_tau_b(a, -a) == pytest.approx(-1.0)


def test_window_count_and_content():
    assert n_windows(30720, 3072, 128) == 217          # 16 s, 0.5 s cropped per edge, 16 Hz
    assert n_windows(32768, 3072, 128) == 233          # uncropped
    assert n_windows(3071, 3072, 128) == 0
    y = np.arange(2 * 1000, dtype=float).reshape(2, 1000)
    w = oracle.unfold_windows(y, 100, 37)
    assert w.shape == (n_windows(1000, 100, 37), 2, 100)
    np.testing.assert_array_equal(w[5, 1], y[1, 185:285])
    ws = oracle.unfold_windows(y, 100, 300, shifts=np.array([0, 950]), wrap=1000)
    np.testing.assert_array_equal(ws[1, 1], y[1, (300 + 950 + np.arange(100)) % 1000])


def test_bf16_matches_torch_cast():
    x = np.random.default_rng(2).standard_normal(100000).astype(np.float32) * np.float32(3.0) ** np.random.default_rng(3).integers(-30, 30, 100000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(x.astype(np.float64)), ref)


def test_e4m3_matches_torch_cast_in_range():
    x = np.random.default_rng(4).uniform(-448, 448, 200000).astype(np.float32)
    x[:1000] *= np.float32(1e-3)             # subnormal range
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.e4m3_round(x.astype(np.float64)), ref)


def test_e4m3_format_extremes():
    # values listed in the OCP 8-bit floating point specification for E4M3
    fix = {}
    for line in open(__file__.replace("test_oracle_post.py", "golden/e4m3_points.txt")):
        if line.strip() and not line.startswith("#"):
            a, b = line.split()
            fix[float.fromhex(a)] = float.fromhex(b)
    for v, r in fix.items():
        assert oracle.e4m3_round(v) == r, (v, r)
        assert oracle.e4m3_round(-v) == -r
