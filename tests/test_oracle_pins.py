"""Pins for the CPU oracle: it is checked against what the paper and the
mathematics fix, never against the GPU path.

Each test names the property it pins and the passage it comes from.  The
combination is chosen so that a dropped term, a wrong sign or index, or a
transposed operand anywhere in the oracle fails at least one of them:

* spectral weights / analytic signal: Marple's weights by hand, scipy's
  ``hilbert`` (an independent library routine of the same construction),
  closed forms for on-bin sinusoids, the band mask's inclusive edges;
* per-pair means: a numpy matrix product of the normalised phasors (the
  paper's own identity, Eqs. 5-7, with the orientation of the Appendix's third
  listing), a hand-derived worked case, closed forms for constant-lag and
  zero-lag signals, Rayleigh statistics of independent phases;
* metrics: closed forms of |G|, |Im G| and the corrected ratio;
* gradient: central finite differences of the oracle's own forward map.
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
import synth
from tests.golden.fixtures import quarter_turns

RNG = np.random.default_rng(20240611)


# ----------------------------------------------------------------- weights ---

@pytest.mark.parametrize("t,expect", [
    (1, [1]),
    (2, [1, 1]),
    (3, [1, 2, 0]),
    (4, [1, 2, 1, 0]),
    (5, [1, 2, 2, 0, 0]),
    (8, [1, 2, 2, 2, 1, 0, 0, 0]),
])
def test_plain_mask_is_marples_one_sided_weights(t, expect):
    # Marple (1999): h0 = 1, h_k = 2 below Nyquist, h_{T/2} = 1 for even T.
    assert oracle.mask_plain(t).tolist() == expect


def test_band_mask_inclusive_edges_and_no_dc_or_nyquist():
    # fs = 100 Hz, T = 100 -> bin k is k Hz.  Band [8, 12] keeps bins 8..12.
    h = oracle.mask_band(100, 100.0, 8.0, 12.0)
    assert np.flatnonzero(h).tolist() == [8, 9, 10, 11, 12]
    assert set(h[h != 0].tolist()) == {2.0}
    # a band reaching DC and Nyquist keeps neither
    h = oracle.mask_band(100, 100.0, 0.0, 50.0)
    assert h[0] == 0 and h[50] == 0 and h[1] == 2 and h[49] == 2
    assert np.all(h[51:] == 0)


# -------------------------------------------------------- analytic signal ---

@pytest.mark.parametrize("t", [16, 17, 64, 101, 128])
def test_analytic_matches_scipy_hilbert(t):
    x = RNG.standard_normal((5, t))
    z = oracle.analytic(x)
    assert np.abs(z - scipy.signal.hilbert(x, axis=-1)).max() < 1e-12
    # the real part of the analytic signal is the signal itself (Eq. 3)
    assert np.abs(z.real - x).max() < 1e-12


@pytest.mark.parametrize("t,k", [(64, 5), (63, 7), (2048, 80)])
def test_analytic_of_on_bin_sinusoids(t, k):
    # cos(w t + a) -> exp(i(w t + a)); sin(w t + a) -> -i exp(i(w t + a))
    a = 0.7
    n = np.arange(t)
    w = 2 * math.pi * k * n / t
    z = oracle.analytic(np.stack([np.cos(w + a), np.sin(w + a)]))
    assert np.abs(z[0] - np.exp(1j * (w + a))).max() < 1e-11
    assert np.abs(z[1] - (-1j) * np.exp(1j * (w + a))).max() < 1e-11


def test_band_analytic_keeps_only_in_band_components():
    fs, t = 1000.0, 1000
    n = np.arange(t)
    inside = np.cos(2 * math.pi * 10 * n / fs + 0.3)
    outside = 0.8 * np.cos(2 * math.pi * 30 * n / fs - 1.1) + 0.5
    z = oracle.analytic((inside + outside)[None], fs=fs, band=(8.0, 12.0))[0]
    assert np.abs(z - np.exp(1j * (2 * math.pi * 10 * n / fs + 0.3))).max() < 1e-11


def test_spectral_filter_complex_input_is_linear_in_real_and_imag():
    x = RNG.standard_normal((3, 40)) + 1j * RNG.standard_normal((3, 40))
    h = oracle.mask_plain(40)
    lhs = oracle.spectral_filter(x, h)
    rhs = oracle.spectral_filter(x.real, h) + 1j * oracle.spectral_filter(x.imag, h)
    assert np.abs(lhs - rhs).max() < 1e-12
    ref = np.fft.ifft(h * np.fft.fft(x, axis=-1), axis=-1)
    assert np.abs(lhs - ref).max() < 1e-12


# ------------------------------------------------------------------ phase ---

def test_phase_is_angle_and_zero_rule():
    z = np.array([1 + 1j, -1 + 0j, -1 - 0j, 1e-300 - 2e-300j, 0j, complex(-0.0, 0.0),
                  complex(0.0, -0.0), complex(-0.0, -0.0)])
    phi = oracle.phase(z)
    assert np.allclose(phi[:4], np.angle(z[:4]), atol=0, rtol=1e-15)
    assert np.all(phi[4:] == 0.0)


# ------------------------------------------------------------- pair means ---

def test_pair_means_equal_normalised_gram_product():
    # Eqs. 5-7 / Appendix third listing: abs(ndat*ndat')/ns with ndat = z/|z|;
    # the complex product fixes the orientation G = U U^H / T.
    n, t = 9, 37
    z = RNG.standard_normal((n, t)) + 1j * RNG.standard_normal((n, t))
    u = z / np.abs(z)
    ref = u @ u.conj().T / t
    got = oracle.full_from_analytic(z)["g"]
    assert np.abs(got - ref).max() < 1e-14
    # G is not symmetric: the imaginary part flips sign under transposition
    assert np.abs(ref.imag).max() > 0.05


def test_hand_derived_quarter_turns():
    z, pairs = quarter_turns()
    full = oracle.full_from_analytic(z)
    for (i, j), (gr, gi, p, ip, cp) in pairs.items():
        assert full["g"][i, j].real == pytest.approx(gr, abs=1e-15)
        assert full["g"][i, j].imag == pytest.approx(gi, abs=1e-15)
        assert full["plv"][i, j] == pytest.approx(p, abs=1e-15)
        assert full["iplv"][i, j] == pytest.approx(ip, abs=1e-15)
        assert full["ciplv"][i, j] == pytest.approx(cp, abs=1e-15)


def test_self_plv_and_hermitian_assembly():
    z = synth.glag_analytic(12, 300, 1000.0, 4, (8, 12), seed=5)
    full = oracle.full_from_analytic(z)
    g = full["g"]
    assert np.all(np.diag(g) == 1.0)
    assert np.all(g == g.conj().T)
    for k in ("plv", "iplv", "ciplv"):
        assert np.all(full[k] == full[k].T)
    assert np.all(np.diag(full["plv"]) == 1.0)
    assert np.all(np.diag(full["iplv"]) == 0.0) and np.all(np.diag(full["ciplv"]) == 0.0)
    # a signal paired with an exact copy of itself: PLV 1, iPLV 0
    z2 = np.concatenate([z[:1], z[:1] * 3.5], axis=0)
    f2 = oracle.full_from_analytic(z2)
    assert f2["plv"][0, 1] == pytest.approx(1.0, abs=1e-15)
    assert f2["iplv"][0, 1] == pytest.approx(0.0, abs=1e-15)


def test_constant_lag_on_bin_sinusoids():
    # x_i = cos(w t + a_i) -> PLV = 1, iPLV = |sin(a_i - a_j)| (Section II.C,
    # the bound sin(phi)), ciPLV = 1 when the lag is nonzero.
    t, k = 512, 20
    a = np.array([0.0, 0.4, math.pi / 2, 2.5, -1.0])
    n = np.arange(t)
    x = np.cos(2 * math.pi * k * n[None] / t + a[:, None])
    full = oracle.full_from_real(x)
    for i in range(len(a)):
        for j in range(i + 1, len(a)):
            assert full["plv"][i, j] == pytest.approx(1.0, abs=1e-12)
            assert full["iplv"][i, j] == pytest.approx(abs(math.sin(a[i] - a[j])), abs=1e-12)
            assert full["ciplv"][i, j] == pytest.approx(1.0, abs=1e-9)
            assert full["g"][i, j] == pytest.approx(np.exp(1j * (a[i] - a[j])), abs=1e-12)


def test_zero_lag_scaled_copies():
    # x_j = c x_i: same phase (c > 0) or opposite (c < 0); G = sign(c), iPLV =
    # ciPLV = 0 (radicand 0 -> ciPLV 0).
    x = synth.glag_real(1, 256, 256.0, 3, 10.0, seed=11)[0]
    xs = np.stack([x, 2.0 * x, -0.5 * x])
    full = oracle.full_from_real(xs)
    assert full["g"][0, 1] == pytest.approx(1.0, abs=1e-13)
    assert full["g"][0, 2] == pytest.approx(-1.0, abs=1e-13)
    assert full["iplv"][0, 1] == pytest.approx(0.0, abs=1e-13)
    assert full["ciplv"][0, 1] == 0.0 and full["ciplv"][0, 2] == 0.0


def test_independent_phases_rayleigh_statistics():
    # Independent uniform phases: E|G|^2 = 1/T exactly, E[PLV] ~ sqrt(pi/(4T)).
    n, t = 48, 1024
    u = synth.uniform_phasors(n, t, seed=17)
    full = oracle.full_from_analytic(u)
    iu = np.triu_indices(n, 1)
    m = len(iu[0])
    g2 = np.abs(full["g"][iu]) ** 2
    assert abs(g2.mean() * t - 1.0) < 4 * math.sqrt(1.0 / m)     # |G|^2 T ~ Exp(1)
    plv = full["plv"][iu]
    sd = math.sqrt((4 - math.pi) / (4 * t * m))
    assert abs(plv.mean() - math.sqrt(math.pi / (4 * t))) < 4 * sd


def test_planted_lag_with_jitter():
    # phi_b = phi_a - lag + eta, eta ~ N(0, s^2): E G_ab = exp(i lag) exp(-s^2/2)
    u, pairs, lags = synth.phasors_planted(40, 20000, 6, seed=23, jitter=0.1)
    g = oracle.pairs_from_analytic(u, pairs)
    expect = np.exp(1j * lags) * math.exp(-0.005)
    assert np.abs(g - expect).max() < 5 * 0.1 / math.sqrt(20000) + 1e-3


def test_invariances():
    n, t = 6, 200
    z = synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=29)
    base = oracle.full_from_analytic(z)["g"]
    # a global phase rotation and positive per-sample amplitudes change nothing
    amp = np.exp(RNG.standard_normal(t))
    assert np.abs(oracle.full_from_analytic(z * np.exp(0.9j) * amp)["g"] - base).max() < 1e-13
    # a common permutation of samples changes nothing
    perm = RNG.permutation(t)
    assert np.abs(oracle.full_from_analytic(z[:, perm])["g"] - base).max() < 1e-13
    # permuting signals permutes G
    ps = RNG.permutation(n)
    assert np.abs(oracle.full_from_analytic(z[ps])["g"] - base[np.ix_(ps, ps)]).max() < 1e-13
    # conjugating every signal conjugates G
    assert np.abs(oracle.full_from_analytic(z.conj())["g"] - base.conj()).max() < 1e-13


def test_window_is_a_slice_after_the_analytic_signal():
    x = synth.glag_real(4, 300, 1000.0, 2, (8, 12), seed=31)
    z = oracle.analytic(x)
    full = oracle.full_from_real(x, window=(50, 250))
    ref = oracle.full_from_analytic(z[:, 50:250])
    assert np.abs(full["g"] - ref["g"]).max() == 0.0


# ---------------------------------------------------------------- metrics ---

@pytest.mark.parametrize("r,th", [(0.3, 0.2), (0.9, 1.3), (1.0, 0.7), (0.5, math.pi), (1.0, 0.0)])
def test_metric_closed_forms(r, th):
    g = np.array([r * np.exp(1j * th)])
    p, i_, c = oracle.metrics(g)
    assert p[0] == pytest.approx(r, abs=1e-15)
    assert i_[0] == pytest.approx(r * abs(math.sin(th)), abs=1e-15)
    d = 1 - (r * math.cos(th)) ** 2
    expect = r * abs(math.sin(th)) / math.sqrt(d) if d > 1e-15 else 0.0
    assert c[0] == pytest.approx(expect, abs=1e-12)


def test_ciplv_zero_when_radicand_vanishes():
    _, _, c = oracle.metrics(np.array([1.0 + 0j, -1.0 + 0j, 1.0 + 1e-9j]))
    assert c[0] == 0.0 and c[1] == 0.0
    assert c[2] == 0.0   # (1 - 1)(1 + 1) = 0 exactly


# --------------------------------------------------------------- gradient ---

def _loss_from_real(x, wp, wi, wc):
    f = oracle.full_from_real(x, nthreads=1)
    iu = np.triu_indices(x.shape[0], 1)
    return (wp[iu] * f["plv"][iu]).sum() + (wi[iu] * f["iplv"][iu]).sum() + (wc[iu] * f["ciplv"][iu]).sum()


def test_gradient_matches_central_finite_differences():
    n, t = 5, 24
    x = synth.glag_real(n, t, 100.0, 2, 10.0, seed=37, noise_var=0.3)
    wp, wi, wc = (RNG.standard_normal((n, n)) for _ in range(3))
    # upstream gradients as full matrices; the upper triangle carries the loss
    up = [np.triu(w, 1) for w in (wp, wi, wc)]
    g = oracle.grad_from_real(x, gp=up[0], gi=up[1], gc=up[2], nthreads=1)
    eps = 1e-6
    fd = np.zeros_like(x)
    for a in range(n):
        for b in range(t):
            xp = x.copy()
            xm = x.copy()
            xp[a, b] += eps
            xm[a, b] -= eps
            fd[a, b] = (_loss_from_real(xp, wp, wi, wc) - _loss_from_real(xm, wp, wi, wc)) / (2 * eps)
    assert np.abs(g - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())


def test_gradient_upstream_is_symmetrised():
    # dL/d(output) is given as a full matrix: (i,j) and (j,i) both feed pair i<j
    n, t = 4, 32
    z = synth.glag_analytic(n, t, 100.0, 2, 10.0, seed=41)
    w = RNG.standard_normal((n, n))
    a = oracle.grad_from_analytic(z, gp=w)
    b = oracle.grad_from_analytic(z, gp=np.triu(w + w.T, 1))
    assert np.abs(a - b).max() < 1e-14


# ------------------------------------------------- large-size helper paths ---

@pytest.mark.parametrize("t,band", [(64, None), (101, None), (1000, (8.0, 12.0))])
def test_fft_analytic_equals_plain_dft_sums(t, band):
    x = RNG.standard_normal((4, t))
    a = oracle.analytic(x, 1000.0, band)
    b = oracle.analytic_fft(x, 1000.0, band)
    assert np.abs(a - b).max() < 1e-11


def test_row_subset_gradient_equals_full_gradient():
    n, t = 9, 40
    x = synth.glag_real(n, t, 100.0, 3, 10.0, seed=43, noise_var=0.3)
    w = [RNG.standard_normal((n, n)) for _ in range(3)]
    full = oracle.grad_from_real(x, gp=w[0], gi=w[1], gc=w[2], window=(3, 37), nthreads=2)
    rows = [0, 4, 8]
    sub = oracle.grad_from_real_rows(x, rows, gp=w[0], gi=w[1], gc=w[2], window=(3, 37), nthreads=2)
    assert np.abs(sub - full[rows]).max() < 1e-12 * max(1.0, np.abs(full).max())
