"""GPU parity of plv_coherence (coherency, Section II.B, Eq. 12) against the
FP64 oracle, element by element on the same seeded inputs.

Tolerances (absolute on coherence, |Im C| and the components of C; the
corrected imaginary coherency gets the same bound times its condition number):
  f64          1e-12
  f32          1e-5
  split_bf16   1e-5
  bf16         1.1e-2 = 4 eps, eps = sqrt(2) 2^-9: every rounded (scaled)
               sample lies within eps|z| of the exact one, which moves the
               cross sum by at most (2 eps + eps^2) sqrt(P_a P_b) (Cauchy-
               Schwarz) and each root power by at most a factor (1 +- eps)
  f16          1.4e-3, the same with eps = sqrt(2) 2^-12
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import cond_ciplv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "split_bf16", "bf16", "f16"]
TOLC = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-5, "bf16": 1.1e-2, "f16": 1.4e-3}


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


def to_dev(z, prec):
    dt = np.complex128 if prec == "f64" else np.complex64
    return torch.from_numpy(np.ascontiguousarray(z.astype(dt))).cuda()


def exact(z, prec):
    return z.astype(np.complex128 if prec == "f64" else np.complex64).astype(np.complex128)


def gpu_coh(z, prec, window=None):
    out = plv_mod().coherence(to_dev(z, prec), prec=prec, window=window, want_g=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.complex128 if k == "c" else np.float64) for k, v in out.items()}


def compare(got, ref, tol, where=""):
    n = ref["coh"].shape[0]
    for k in ("coh", "icoh"):
        e = np.abs(got[k] - ref[k]).max()
        assert e <= tol, "%s %s max err %.3g > %.3g" % (where, k, e, tol)
    e = max(np.abs(got["c"].real - ref["c"].real).max(), np.abs(got["c"].imag - ref["c"].imag).max())
    assert e <= tol, "%s C max err %.3g > %.3g" % (where, e, tol)
    cnd = cond_ciplv(ref["c"])
    np.fill_diagonal(cnd, 1.0)
    assert np.all(np.abs(got["cicoh"] - ref["cicoh"]) <= tol * cnd + 1e-15), where
    assert np.all(np.diag(got["coh"]) == 1.0) and np.all(np.diag(got["icoh"]) == 0.0)
    for k in ("coh", "icoh", "cicoh"):
        assert np.array_equal(got[k], got[k].T), k
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(got["c"][off], np.conj(got["c"].T)[off])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,t", [(37, 300), (130, 1000), (5, 1)])
def test_ragged_shapes_against_oracle(prec, n, t):
    z = synth.coefficients_mixed(n, t, seed=synth.seed_for(6, n + t))
    got = gpu_coh(z, prec)
    ref = oracle.full_coherence(exact(z, prec))
    compare(got, ref, TOLC[prec], "n=%d t=%d %s" % (n, t, prec))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16"])
def test_zero_row_tiny_and_huge_rows_and_window(prec):
    """A row that is zero over the window (C = 0 with every other row), rows
    scaled by 2^-60 and 2^+60 (FP32 range; the row scale makes them O(1)),
    and a window."""
    n, t = 24, 700
    z = synth.coefficients_mixed(n, t, seed=synth.seed_for(6, 99))
    z[3, 100:650] = 0
    z[5] *= 2.0 ** -60
    z[9] *= 2.0 ** 60
    win = (100, 650)
    got = gpu_coh(z, prec, window=win)
    ref = oracle.full_coherence(exact(z, prec)[:, win[0]:win[1]])
    compare(got, ref, TOLC[prec], "edge cases %s" % prec)
    assert np.all(got["c"][3, np.arange(n) != 3] == 0)


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_grouped_equals_single(prec):
    shapes = [(40, 256), (7, 999), (150, 3000)]
    zs = [synth.coefficients_mixed(n, t, seed=synth.seed_for(6, 200 + k)) for k, (n, t) in enumerate(shapes)]
    outs = plv_mod().coherence_batch([to_dev(z, prec) for z in zs], prec=prec, want_g=True)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        got = {kk: v.cpu().numpy().astype(np.complex128 if kk == "c" else np.float64) for kk, v in outs[k].items()}
        compare(got, oracle.full_coherence(exact(z, prec)), TOLC[prec], "grouped %d" % k)


def test_constant_amplitude_rows_give_the_plv():
    """Eq. 12's weighted form on the GPU: rows of constant amplitude make
    coherency and the PLV's G the same matrix, computed by the two entry
    points through different kernels."""
    z = synth.glag_analytic(48, 5000, 1000.0, 4, (8, 12), seed=31)
    u = (z / np.abs(z)) * np.linspace(0.5, 3.0, 48)[:, None]
    zd = to_dev(u, "f32")
    c = plv_mod().coherence(zd, prec="f32", want_g=True)["c"]
    g = plv_mod().from_analytic(zd, prec="f32", want_g=True)["g"]
    torch.cuda.synchronize()
    assert torch.abs(c - g).max().item() <= 2e-6


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
def test_sensor_scale_sampled_pairs(prec):
    """N = 1024 rows of T = 60000 samples (several K-chunks), checked on all
    pairs among 24 sampled rows."""
    n, t = 1024, 60000
    z = synth.coefficients_mixed(n, t, seed=synth.seed_for(6, 1), dtype=np.complex64)
    got = gpu_coh(z, prec)
    rows = np.sort(np.random.default_rng(3).choice(n, size=24, replace=False))
    ref = oracle.full_coherence(exact(z[rows], prec))
    sub = {k: v[np.ix_(rows, rows)] for k, v in got.items()}
    compare(sub, ref, TOLC[prec], "sensor scale %s" % prec)
