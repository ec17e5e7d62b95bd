"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the method's arithmetic: it makes signals, it never
normalises them, never forms a Hilbert transform and never contracts them.  The
oracle (``oracle/``) and the HIP path (``paper_1710_08037_amd``) both receive
the arrays made here and nothing else from each other.

Generators
----------
``glag_real``      lagged-oscillator mixture, real signals (the band-pass signal
                   of Eq. 3 in the paper, before the Hilbert transform).
``glag_analytic``  the same latent model written directly as complex phasor
                   mixtures, i.e. an analytic-signal stand-in given as complex.
``phasors_planted`` unit phasors with uniform i.i.d. phases plus planted
                   constant-lag pairs with Gaussian jitter.
``batch_shapes``   (N, T) per trial for the uneven grouped workload.
``sparse_target``  the seeded sparse ciPLV target C* of the differentiable case.
``coefficients_mixed`` complex coefficients with amplitude modulation and
                   lagged mixtures of shared sources (coherency inputs).

The paper's recordings (MEG source space, 1 kHz, 4 s trials, alpha band,
Section III.A) are not available; these stand in for them with the same shapes.
Volume conduction follows the instantaneous linear mixing of Eq. 16 applied to
channel pairs (2m, 2m+1).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 171008037


def seed_for(config: int, rep: int = 0) -> int:
    """Seed for workload ``config`` (1-based) and repetition ``rep``."""
    return BASE_SEED + 1000 * int(config) + int(rep)


def _latent_phases(rng, k, t, fs, freq, sigma):
    """Phases theta_k(t) of K latent oscillators with random-walk phase noise."""
    if isinstance(freq, (tuple, list)):
        f = rng.uniform(freq[0], freq[1], size=k)
    else:
        f = np.full(k, float(freq))
    theta0 = rng.uniform(0.0, 2.0 * math.pi, size=k)
    step = (2.0 * math.pi * f / fs)[:, None] + sigma * rng.standard_normal((k, t))
    theta = theta0[:, None] + np.cumsum(step, axis=1)
    return theta


def _mixing(rng, n, k):
    w = rng.dirichlet(0.5 * np.ones(k), size=n)          # [n, k]
    lag = rng.uniform(0.0, math.pi, size=(n, k))         # [n, k]
    return w, lag


def _zero_lag_mix(s, v):
    """Eq. 16 on pairs (2m, 2m+1): x~ = x + V*y, y~ = y + V*x."""
    out = s.copy()
    m = (s.shape[0] // 2) * 2
    out[0:m:2] = s[0:m:2] + v * s[1:m:2]
    out[1:m:2] = s[1:m:2] + v * s[0:m:2]
    return out


def glag_real(n: int, t: int, fs: float, k: int, freq, seed: int,
              sigma: float = 0.05, v: float = 0.3, noise_var: float = 0.5,
              dtype=np.float64) -> np.ndarray:
    """Real lagged-oscillator signals, shape [n, t].

    s_i(t) = sum_k w_ik cos(theta_k(t) - lag_ik); zero-lag mixing with weight v
    on pairs (2m, 2m+1); plus white Gaussian noise of variance ``noise_var``.
    ``freq`` is a fixed frequency in Hz or a (lo, hi) range drawn per latent.
    """
    rng = np.random.default_rng(seed)
    theta = _latent_phases(rng, k, t, fs, freq, sigma)
    w, lag = _mixing(rng, n, k)
    a = w * np.cos(lag)
    b = w * np.sin(lag)
    s = a @ np.cos(theta) + b @ np.sin(theta)            # cos(th - l) expanded
    s = _zero_lag_mix(s, v)
    x = s + math.sqrt(noise_var) * rng.standard_normal((n, t))
    return x.astype(dtype, copy=False)


def glag_analytic(n: int, t: int, fs: float, k: int, freq, seed: int,
                  sigma: float = 0.05, v: float = 0.3, noise_var: float = 0.5,
                  dtype=np.complex128) -> np.ndarray:
    """Complex lagged-oscillator signals, shape [n, t].

    The same latent model as ``glag_real`` with each cosine replaced by its
    complex exponential: s_i(t) = sum_k w_ik exp(i(theta_k(t) - lag_ik)),
    mixed as in Eq. 16, plus complex white noise whose real and imaginary parts
    each have variance ``noise_var``.  It stands in for an analytic signal that
    the caller computed elsewhere.
    """
    rng = np.random.default_rng(seed)
    theta = _latent_phases(rng, k, t, fs, freq, sigma)
    w, lag = _mixing(rng, n, k)
    a = w * np.cos(lag)
    b = w * np.sin(lag)
    ct, st = np.cos(theta), np.sin(theta)
    # sum_k w_ik exp(i(theta_k - lag_ik)) with real products only
    re = _zero_lag_mix(a @ ct + b @ st, v)
    im = _zero_lag_mix(a @ st - b @ ct, v)
    sd = math.sqrt(noise_var)
    re += sd * rng.standard_normal((n, t))
    im += sd * rng.standard_normal((n, t))
    s = np.empty((n, t), dtype=dtype)
    s.real = re
    s.imag = im
    return s


def phasors_planted(n: int, t: int, npairs: int, seed: int, jitter: float = 0.1,
                    dtype=np.complex128):
    """Unit phasors with i.i.d. uniform phases plus planted lagged pairs.

    Returns (u, pairs, lags): u is [n, t]; pairs is an int64 array [npairs, 2]
    of (a, b) with phi_b(t) = phi_a(t) - lag + eta(t), eta ~ N(0, jitter^2);
    lags are uniform in [0, pi).
    """
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n, t))
    verts = rng.permutation(n)[: 2 * npairs]
    pairs = verts.reshape(npairs, 2).astype(np.int64)
    lags = rng.uniform(0.0, math.pi, size=npairs)
    for p in range(npairs):
        a, b = pairs[p]
        phi[b] = phi[a] - lags[p] + jitter * rng.standard_normal(t)
    u = np.exp(1j * phi)
    return u.astype(dtype, copy=False), pairs, lags


def uniform_phasors(n: int, t: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Unit phasors with i.i.d. uniform phases, shape [n, t]."""
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, size=(n, t))).astype(dtype, copy=False)


BATCH_NS = (68, 148, 360, 1000)
BATCH_CENTRES_HZ = (4.0, 8.0, 12.0, 20.0, 40.0)


def batch_shapes(ntrials: int, seed: int, t_lo: int = 500, t_hi: int = 4000, ns=BATCH_NS):
    """(N, T) per trial for the uneven batch: T ~ U{t_lo..t_hi}, N ~ U(ns)."""
    rng = np.random.default_rng(seed)
    ts = rng.integers(t_lo, t_hi + 1, size=ntrials)
    nn = rng.choice(np.asarray(ns), size=ntrials)
    return [(int(a), int(b)) for a, b in zip(nn, ts)]


def bands_hz(half_width: float = 2.0, centres=BATCH_CENTRES_HZ):
    """Band edges (lo, hi) in Hz, centre +- half_width."""
    return [(c - half_width, c + half_width) for c in centres]


def sparse_target(n: int, seed: int, frac: float = 0.01, lo: float = 0.2, hi: float = 0.8):
    """Symmetric [n, n] target with zero diagonal: round(frac * n(n-1)/2)
    distinct upper-triangle entries drawn U(lo, hi), the rest 0."""
    rng = np.random.default_rng(seed)
    npair = n * (n - 1) // 2
    m = int(round(frac * npair))
    pick = rng.choice(npair, size=m, replace=False)
    iu, ju = np.triu_indices(n, k=1)
    c = np.zeros((n, n), dtype=np.float64)
    vals = rng.uniform(lo, hi, size=m)
    c[iu[pick], ju[pick]] = vals
    c[ju[pick], iu[pick]] = vals
    return c


def coefficients_mixed(n: int, t: int, seed: int, k: int = 4, noise: float = 0.5,
                       dtype=np.complex128) -> np.ndarray:
    """Complex rows [n, t] standing in for Fourier coefficients over trials:
    K latent complex Gaussian sources whose amplitude is modulated per sample
    (log-normal, sigma 0.7, so samples carry very different weights), mixed
    into each row with Dirichlet(0.5) weights and uniform lags in [0, pi),
    plus complex white noise of variance `noise` per component."""
    rng = np.random.default_rng(seed)
    src = (rng.standard_normal((k, t)) + 1j * rng.standard_normal((k, t))) / math.sqrt(2.0)
    src *= np.exp(0.7 * rng.standard_normal((1, t)))
    w = rng.dirichlet(0.5 * np.ones(k), size=n)
    lag = rng.uniform(0.0, math.pi, size=(n, k))
    x = (w * np.exp(1j * lag)) @ src
    x += math.sqrt(noise) * (rng.standard_normal((n, t)) + 1j * rng.standard_normal((n, t)))
    return x.astype(dtype, copy=False)

