"""Pins of the oracle's FIR band-pass (the forward-backward filter the paper
names before the Hilbert transform, Section III, with the build's own design:
Hamming-windowed ideal band-pass of even order L, unit gain at the band
centre).  Checked against scipy's window-method design and its forward-
backward filter, and against closed forms for tones."""
import math

import numpy as np
import pytest

import oracle

scipy_signal = pytest.importorskip("scipy.signal")


@pytest.mark.parametrize("order,fs,band", [(100, 1000.0, (8.0, 12.0)), (2000, 1000.0, (8.0, 12.0)),
                                           (256, 256.0, (4.0, 6.5)), (64, 100.0, (10.0, 30.0))])
def test_taps_match_window_method_design(order, fs, band):
    h = oracle.fir_taps(order, fs, *band)
    ref = scipy_signal.firwin(order + 1, list(band), pass_zero=False, window="hamming", fs=fs)
    assert np.abs(h - ref).max() <= 1e-15 * max(1.0, np.abs(ref).max()) * 10


def test_odd_order_is_refused():
    with pytest.raises(ValueError):
        oracle.fir_taps(101, 1000.0, 8.0, 12.0)


@pytest.mark.parametrize("order,t", [(200, 1200), (600, 2500)])
def test_zero_phase_equals_forward_backward_filtering_away_from_the_ends(order, t):
    fs, band = 1000.0, (30.0, 60.0)
    x = np.random.default_rng(order).standard_normal((3, t))
    y = oracle.fir_zero_phase(x, fs, band + (order,))
    ref = scipy_signal.filtfilt(oracle.fir_taps(order, fs, *band), [1.0], x, axis=-1, padtype=None)
    inner = slice(order, t - order)
    err = np.abs(y[:, inner] - ref[:, inner]).max()
    assert err <= 1e-11 * np.abs(ref).max()


def test_power_unit_at_the_centre_small_in_the_stop_band_and_even():
    t, fs, band, order = 2000, 1000.0, (8.0, 12.0), 2000
    p = oracle.fir_power(t, fs, *band, order)
    hz = fs / t
    assert abs(p[int(round(10.0 / hz))] - 1.0) <= 1e-12          # centre 10 Hz
    # Hamming-window sidelobes lie below -53 dB: |H|^2 <= 10^-5.3 outside the band
    assert p[int(round(100.0 / hz))] <= 10 ** -5.3               # 90 Hz away
    assert p[0] <= 10 ** -5.3                                    # DC
    assert np.allclose(p[1:], p[1:][::-1], rtol=0, atol=1e-15)   # real taps: |H(-f)| = |H(f)|


def test_analytic_signal_of_an_in_band_tone():
    """A bin-centred tone at the band centre comes out as exp(i(w n + phi))."""
    t, fs = 2000, 1000.0
    n = np.arange(t)
    w, phi = 2 * math.pi * 10.0 / fs, 0.3
    z = oracle.analytic(np.cos(w * n + phi)[None], fs, (8.0, 12.0, 2000))[0]
    assert np.abs(z - np.exp(1j * (w * n + phi))).max() <= 1e-9


def test_plv_of_lagged_in_band_tones_with_out_of_band_interference():
    """In-band tones at a constant lag plus strong out-of-band tones at
    unrelated phases: after the FIR band PLV = 1 and iPLV = |sin lag|."""
    t, fs, lag = 2000, 1000.0, 0.7
    n = np.arange(t)
    w, w2 = 2 * math.pi * 10.0 / fs, 2 * math.pi * 60.0 / fs
    x = np.stack([np.cos(w * n) + 3.0 * np.cos(w2 * n + 1.1),
                  np.cos(w * n - lag) + 3.0 * np.cos(w2 * n - 2.0)])
    out = oracle.full_from_real(x, fs, (8.0, 12.0, 1000))
    assert abs(out["plv"][0, 1] - 1.0) <= 1e-6
    assert abs(out["iplv"][0, 1] - abs(math.sin(lag))) <= 1e-6
