"""Checks of the seeded input generators (no SRP arithmetic involved).

The far-field scene generator stands in for a reverberant room with diffuse
noise; these tests check that its noise field has the spherically isotropic
coherence sinc(2 f d / c) it is built to have, and that the direct and
reverberant parts carry the requested energy ratio.
"""
import numpy as np

import workloads as WL


def _coherence(x, a, b, nfft=256):
    seg = x[:, : (x.shape[1] // nfft) * nfft].reshape(x.shape[0], -1, nfft) * np.hanning(nfft)
    X = np.fft.rfft(seg, axis=2)
    sab = np.mean(X[a] * X[b].conj(), axis=0)
    return (sab / np.sqrt(np.mean(abs(X[a]) ** 2, 0) * np.mean(abs(X[b]) ** 2, 0))).real


def test_hemisphere_directions_unit_and_upper():
    d = WL.hemisphere_direction(np.random.default_rng(0), 500)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    assert d[:, 2].min() >= 0.0
    # uniform on the half sphere: mean r_z is 1/2
    assert abs(d[:, 2].mean() - 0.5) < 0.05


def test_diffuse_noise_coherence_is_isotropic_sinc():
    mic = WL.uniform_circular_array(6, 0.1)
    fs, c = 16000.0, 340.0
    # noise only: SNR -80 dB
    fr = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], fs, 2048, 64, c, -80.0,
                            np.random.default_rng(3))
    x = fr.transpose(1, 0, 2).reshape(6, -1).astype(np.float64)
    f = np.fft.rfftfreq(256, 1.0 / fs)
    for a, b in ((0, 1), (0, 3)):
        d = np.linalg.norm(mic[a] - mic[b])
        want = np.sinc(2.0 * f * d / c)
        got = _coherence(x, a, b)
        assert np.abs(got[1:-1] - want[1:-1]).max() < 0.12, (a, b)
    # white sensor noise: incoherent
    fr = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], fs, 2048, 64, c, -80.0,
                            np.random.default_rng(3), noise="white")
    x = fr.transpose(1, 0, 2).reshape(6, -1).astype(np.float64)
    assert np.abs(_coherence(x, 0, 3)[1:-1]).max() < 0.12


def test_reverberant_energy_ratio():
    """drr_db = 0: the reverberant tail has the direct path's energy, so the
    mic signal has about twice the power of the unit-gain direct path."""
    mic = WL.uniform_circular_array(6, 0.1)
    fr = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], 16000.0, 2048, 16, 340.0, 200.0,
                            np.random.default_rng(7), drr_db=0.0)
    p = float(np.mean(fr.astype(np.float64) ** 2))
    assert 1.6 < p < 2.4, p
    fr = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], 16000.0, 2048, 16, 340.0, 200.0,
                            np.random.default_rng(7), drr_db=200.0)
    assert abs(float(np.mean(fr.astype(np.float64) ** 2)) - 1.0) < 0.1


def test_snr_list_shares_signal_and_noise():
    mic = WL.uniform_circular_array(4, 0.1)
    a, b = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], 16000.0, 512, 4, 340.0, [0.0, 6.0],
                              np.random.default_rng(1))
    # same signal, noise scaled by 10^(-6/20) between the two
    n_a = a.astype(np.float64) - b.astype(np.float64)
    assert np.isfinite(n_a).all() and float(np.std(n_a)) > 0.0
    single = WL.synth_far_scene(mic, [0.0, 0.0, 1.0], 16000.0, 512, 4, 340.0, 0.0,
                                np.random.default_rng(1))
    np.testing.assert_array_equal(single, a)
