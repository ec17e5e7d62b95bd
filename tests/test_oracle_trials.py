"""Pins of the oracle's PLV across trials (Eq. 1; its matrix form Eq. 8).

- Trials that are time-shifted copies of one recording: the PLV across
  trials at time t equals the PLV over time (Eq. 2) of that recording's
  window [t, t + ntr), computed by the oracle's time-axis path on differently
  arranged data (catches any mix-up of the trial and time axes).
- Phase differences that are the same in every trial: PLV(t) = 1, with
  iPLV(t) = |sin(difference)|.
- Independent trials: E|G(t)|^2 = 1/ntr.
"""
import math

import numpy as np

import oracle


def test_shifted_trials_equal_the_time_plv_of_windows():
    rng = np.random.default_rng(1)
    n, ntr, tt = 5, 30, 12
    w = np.exp(1j * np.cumsum(rng.standard_normal((n, ntr + tt)), axis=1))
    w[3] = w[1] * np.exp(0.7j) * rng.uniform(0.5, 2.0, size=ntr + tt)
    z = np.stack([w[:, k:k + tt] for k in range(ntr)])        # [ntr, n, tt]: trial k starts at k
    tr = oracle.full_over_trials(z)
    for t in range(tt):
        ref = oracle.full_from_analytic(w[:, t:t + ntr])
        for key in ("g", "plv", "iplv", "ciplv"):
            assert np.abs(tr[key][t] - ref[key]).max() < 1e-13, (t, key)


def test_locked_trials_give_one():
    rng = np.random.default_rng(2)
    ntr, tt = 40, 6
    base = rng.uniform(0, 2 * np.pi, size=(ntr, tt))
    d = 0.9
    z = np.stack([np.exp(1j * base), np.exp(1j * (base - d))], axis=1)   # [ntr, 2, tt]
    out = oracle.full_over_trials(z)
    assert np.abs(out["plv"][:, 0, 1] - 1).max() < 1e-13
    assert np.abs(out["iplv"][:, 0, 1] - abs(math.sin(d))).max() < 1e-13


def test_independent_trials_mean_square():
    rng = np.random.default_rng(3)
    ntr, n, tt = 50, 24, 20
    z = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(ntr, n, tt)))
    out = oracle.full_over_trials(z)
    iu = np.triu_indices(n, 1)
    ms = np.mean(np.abs(out["g"][:, iu[0], iu[1]]) ** 2)
    assert abs(ms * ntr - 1.0) < 0.1
