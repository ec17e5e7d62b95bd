"""Pins of the oracle's windowed-segment Fourier coefficients (the X_i(f, n)
of Section II.B, Eq. 12) and of the coherence over segments built on them,
to facts other than their own formulas:

- the windows against numpy's hamming / hanning and the Hamming window's
  closed-form gain 0.54 L - 0.46;
- the bins against numpy's FFT of the windowed segments (an independent
  library routine), including the segment count and hop;
- an on-bin tone with the rectangular window: X_k0 = (L/2) e^{ia}, 0 on the
  other bins; a constant with the Hamming window: X_0 = its gain;
- Parseval over every bin of a real segment;
- magnitude-squared coherence against scipy.signal.coherence (Welch's
  method: the same segments, window and overlap, no detrending);
- a row and a scaled copy of it: coherence 1, C = conj(c)/|c|.
"""
import numpy as np
import pytest

import oracle


def test_windows_match_numpy_and_the_hamming_gain():
    for L in (2, 5, 64, 400, 1001):
        assert np.allclose(oracle.window("hamming", L), np.hamming(L), atol=1e-15, rtol=0)
        assert np.allclose(oracle.window("hann", L), np.hanning(L), atol=1e-15, rtol=0)
        assert np.array_equal(oracle.window("rect", L), np.ones(L))
        if L >= 3:  # sum_m cos(2 pi m / (L-1)) over m < L is 1: a whole period plus m = L-1
            assert abs(oracle.window("hamming", L).sum() - (0.54 * L - 0.46)) < 1e-12


@pytest.mark.parametrize("L,H", [(64, 32), (100, 37), (256, 256), (400, 200)])
def test_bins_equal_numpy_fft_of_windowed_segments(L, H):
    rng = np.random.default_rng(L + H)
    x = rng.standard_normal((3, 2000))
    z = oracle.stft_bins(x, L, H, 0, L // 2, "hamming")
    S = (2000 - L) // H + 1
    assert z.shape == (L // 2 + 1, 3, S)
    w = np.hamming(L)
    for s in (0, S // 2, S - 1):
        ref = np.fft.rfft(x[:, s * H: s * H + L] * w, axis=1)   # [3][L//2 + 1]
        assert np.abs(z[:, :, s].T - ref).max() < 1e-10


def test_span_selects_the_segments():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 900))
    z = oracle.stft_bins(x, 50, 25, 3, 7, "hann", span=(100, 700))
    ref = oracle.stft_bins(x[:, 100:700], 50, 25, 3, 7, "hann")
    assert z.shape == ref.shape == (5, 2, (600 - 50) // 25 + 1)
    assert np.array_equal(z, ref)


def test_on_bin_tone_and_dc_gain():
    L, k0, a = 128, 9, 0.7
    m = np.arange(4 * L)
    x = np.cos(2 * np.pi * k0 * m / L + a)[None]
    z = oracle.stft_bins(x, L, L, 0, L // 2, "rect")
    for s in range(4):
        assert abs(z[k0, 0, s] - (L / 2) * np.exp(1j * a)) < 1e-10
        others = np.delete(z[:, 0, s], k0)
        assert np.abs(others).max() < 1e-10
    c = np.ones((1, 1000))
    zd = oracle.stft_bins(c, 400, 200, 0, 0, "hamming")
    assert np.abs(zd - (0.54 * 400 - 0.46)).max() < 1e-10


def test_parseval_over_every_bin():
    rng = np.random.default_rng(4)
    L = 200
    x = rng.standard_normal((1, L))
    z = oracle.stft_bins(x, L, L, 0, L - 1, "hamming")[:, 0, 0]
    assert abs(np.sum(np.abs(z) ** 2) - L * np.sum((x[0] * np.hamming(L)) ** 2)) < 1e-9


def test_coherence_matches_scipy_welch():
    signal = pytest.importorskip("scipy.signal")
    rng = np.random.default_rng(5)
    T, L, H = 6000, 400, 200
    src = rng.standard_normal(T + 10)
    x = np.stack([src[:T] + 0.5 * rng.standard_normal(T), src[3:T + 3] + 0.8 * rng.standard_normal(T),
                  rng.standard_normal(T)])
    res = oracle.full_coherence_stft(x, L, H, 0, L // 2, "hamming")
    for a, b in ((0, 1), (0, 2), (1, 2)):
        f, cxy = signal.coherence(x[a], x[b], fs=1.0, window=np.hamming(L), nperseg=L, noverlap=L - H,
                                  detrend=False)
        mine = np.array([r["coh"][a, b] ** 2 for r in res])
        assert np.abs(mine - cxy).max() < 1e-10


def test_scaled_copy_is_fully_coherent():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((1, 3000))
    x = np.concatenate([x, -2.5 * x])
    res = oracle.full_coherence_stft(x, 300, 150, 2, 20, "hamming")
    for r in res:
        assert abs(r["coh"][0, 1] - 1.0) < 1e-12
        assert abs(r["c"][0, 1] + 1.0) < 1e-12  # C = conj(c)/|c| for c = -2.5
        assert r["icoh"][0, 1] < 1e-12
