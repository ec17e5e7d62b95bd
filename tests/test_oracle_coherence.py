"""Pins of the oracle's coherency (Section II.B, Eq. 12) to facts other than
its own formula.

- A two-sample case worked by hand.
- Eq. 12's second form: coherence is the amplitude-weighted mean of unit
  phase vectors, so with a constant amplitude per row it must equal the PLV
  the oracle computes through its separate angle / exp / mean path.
- Cauchy-Schwarz: |C| <= 1, with equality (and C = conj(c)/|c|) exactly for
  proportional rows X_b = c X_a.
- Invariance under positive scaling of each row and a common phase rotation;
  Hermitian symmetry C_ab = conj(C_ba).
- Independent complex Gaussian rows: E|C|^2 = 1/T.
- An all-zero row has no defined coherency and gets 0.
"""
import math

import numpy as np
import pytest

import oracle


def test_two_sample_case_by_hand():
    # X1 = [1, i], X2 = [1, 1]: sum X1 conj(X2) = 1 + i, powers 2 and 2,
    # C = (1 + i) / 2: coherence 1/sqrt(2), imaginary part 1/2,
    # corrected imaginary coherency (1/2) / sqrt(1 - 1/4) = 1/sqrt(3).
    z = np.array([[1.0, 1j], [1.0, 1.0]])
    c = oracle.coherency(z, np.array([[0, 1]]))[0]
    assert abs(c - (0.5 + 0.5j)) < 1e-15
    coh, icoh, cicoh = oracle.metrics(np.array([c]))
    assert abs(coh[0] - 1 / math.sqrt(2)) < 1e-15
    assert abs(icoh[0] - 0.5) < 1e-15
    assert abs(cicoh[0] - 1 / math.sqrt(3)) < 1e-15


def test_constant_amplitude_rows_give_the_plv():
    rng = np.random.default_rng(1)
    n, t = 7, 500
    phi = rng.uniform(0, 2 * np.pi, size=(n, t))
    phi[3] = phi[1] - 0.8 + 0.2 * rng.standard_normal(t)
    amp = rng.uniform(0.1, 10.0, size=(n, 1))
    z = amp * np.exp(1j * phi)
    pr = oracle.upper_pairs(n)
    c = oracle.coherency(z, pr)
    g = oracle.pair_means(phi, pr)
    assert np.abs(c - g).max() < 1e-12


def test_proportional_rows_reach_the_bound():
    rng = np.random.default_rng(2)
    t = 300
    a = rng.standard_normal(t) + 1j * rng.standard_normal(t)
    cst = 0.3 - 1.7j
    z = np.stack([a, cst * a, rng.standard_normal(t) + 1j * rng.standard_normal(t)])
    c = oracle.coherency(z, np.array([[0, 1], [0, 2], [1, 2]]))
    assert abs(c[0] - np.conj(cst) / abs(cst)) < 1e-13
    assert np.all(np.abs(c) <= 1 + 1e-15)
    assert abs(c[1]) < 1 and abs(c[2]) < 1


def test_invariances_and_hermitian_symmetry():
    rng = np.random.default_rng(3)
    n, t = 6, 400
    z = rng.standard_normal((n, t)) + 1j * rng.standard_normal((n, t))
    z[2] += 0.8 * z[4] * np.exp(0.6j)
    pr = oracle.upper_pairs(n)
    c = oracle.coherency(z, pr)
    s = rng.uniform(0.01, 100.0, size=(n, 1))
    assert np.abs(oracle.coherency(s * z, pr) - c).max() < 1e-13
    assert np.abs(oracle.coherency(z * np.exp(1.1j), pr) - c).max() < 1e-13
    assert np.abs(oracle.coherency(z, pr[:, ::-1]) - np.conj(c)).max() < 1e-15


def test_independent_rows_have_mean_square_one_over_t():
    rng = np.random.default_rng(4)
    n, t = 64, 256
    z = rng.standard_normal((n, t)) + 1j * rng.standard_normal((n, t))
    c = oracle.coherency(z, oracle.upper_pairs(n))
    ms = float(np.mean(np.abs(c) ** 2))
    # 2016 pairs: the mean of |C|^2 (an exponential-like variable of mean 1/T)
    # lies within a few standard errors of 1/T
    assert abs(ms * t - 1.0) < 0.15


def test_zero_row_gets_zero_and_full_matrix_conventions():
    rng = np.random.default_rng(5)
    z = rng.standard_normal((4, 50)) + 1j * rng.standard_normal((4, 50))
    z[2] = 0
    full = oracle.full_coherence(z)
    assert np.all(full["c"][2, [0, 1, 3]] == 0) and full["c"][2, 2] == 0
    assert np.all(np.diag(full["coh"])[[0, 1, 3]] == 1.0)
    assert np.array_equal(full["coh"], full["coh"].T)
    assert np.allclose(full["c"], np.conj(full["c"].T))
