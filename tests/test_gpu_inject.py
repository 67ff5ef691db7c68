"""GPU parity: projection onto detectors (af_project) and network SNR with
rescaling (af_snr_rescale) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from synth.detectors import ligo_detectors, polarisation_pairs, sky_draws
from synth.noise import analytic_psd
from tests.gpu_util import banner, dev, need_gpu

pytestmark = pytest.mark.gpu
FS = 2048.0


def _psd(df, n_freq, n_det=2):
    f = np.arange(n_freq) * df
    S = analytic_psd(np.maximum(f, 1.0)) * 1e42           # strain x 1e21 units
    return np.repeat(S[None, :], n_det, axis=0)


@pytest.mark.parametrize("n", [64, 1000])
def test_projection_matches_oracle(n):
    P = need_gpu()
    banner(f"project len={n}")
    rng = np.random.default_rng(n)
    hp = rng.standard_normal((6, n)).astype(np.float32)
    hc = rng.standard_normal((6, n)).astype(np.float32)
    sky = sky_draws(6, seed=n)
    det = ligo_detectors()
    got = P.project(dev(hp), dev(hc), dev(sky), det, FS).cpu().numpy()
    ref = oracle.project(hp, hc, sky, det, FS)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())


def test_snr_and_rescale_match_oracle():
    P = need_gpu()
    banner("snr rescale")
    n, n_inj = 4096, 12
    hp, hc = polarisation_pairs(n_inj, n, FS, seed=3)
    sig = P.project(dev(hp), dev(hc), dev(sky_draws(n_inj, seed=4)), ligo_detectors(), FS)
    before = sig.cpu().numpy().astype(np.float64)
    df = FS / 4096
    psd = _psd(df, 2049)
    snr = P.snr_rescale(sig, dev(psd), df, FS, 20.0).cpu().numpy()
    ref = oracle.network_snr(before, psd, df, FS, 20.0)
    np.testing.assert_allclose(snr, ref, rtol=1e-9)
    np.testing.assert_array_equal(sig.cpu().numpy(), before.astype(np.float32))   # no target: untouched
    target = np.linspace(4.0, 20.0, n_inj)
    P.snr_rescale(sig, dev(psd), df, FS, 20.0, target=dev(target))
    after = oracle.network_snr(sig.cpu().numpy(), psd, df, FS, 20.0)
    np.testing.assert_allclose(after, target, rtol=1e-6)


def test_snr_sizes_and_errors():
    P = need_gpu()
    rng = np.random.default_rng(9)
    df = FS / 8192
    psd = _psd(df, 4097, n_det=1)
    for n in (2, 256, 8192):                 # smallest, small, largest length
        sig = dev(rng.standard_normal((3, 1, n)).astype(np.float32))
        got = P.snr_rescale(sig, dev(psd), df, FS, 0.0).cpu().numpy()
        np.testing.assert_allclose(got, oracle.network_snr(sig.cpu().numpy(), psd, df, FS, 0.0), rtol=1e-9)
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.snr_rescale(dev(np.zeros((1, 1, 1000), np.float32)), dev(psd), df)   # not a power of two
    with pytest.raises(P.AframeError, match="EINVAL"):
        P.project(dev(np.zeros((1, 8), np.float32)), dev(np.zeros((1, 8), np.float32)),
                  dev(np.zeros((1, 4))), np.zeros((5, 9)))                       # five detectors
