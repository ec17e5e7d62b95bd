"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs, element by element.

Tolerances (absolute, on PLV, iPLV and the components of G; ciPLV gets the
same bound times its first-order condition number from the oracle's G):
  f64          1e-12
  f32          1e-5
  split_bf16   1e-5 on the lagged-oscillator workloads
  bf16         5.6e-3 = 2*sqrt(2)*2^-9: each rounded phasor is within
               sqrt(2)*2^-9 of the exact one, so every term of the mean, and
               the mean itself, is within twice that
  f16          7.0e-4 = 2*sqrt(2)*2^-12, the same argument for FP16
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.golden.fixtures import quarter_turns

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "split_bf16", "bf16", "f16"]
TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-5, "bf16": 5.6e-3, "f16": 7.0e-4}


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


def to_dev(z, prec):
    dt = np.complex128 if prec == "f64" else np.complex64
    return torch.from_numpy(np.ascontiguousarray(z.astype(dt))).cuda()


def gpu_full(z, prec, window=None):
    """Run plv_from_analytic on z (numpy) and return float64 / complex128 numpy results."""
    out = plv_mod().from_analytic(to_dev(z, prec), prec=prec, window=window, want_g=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in out.items()}


def exact_input(z, prec):
    """The values the GPU actually receives, widened exactly to complex128."""
    return z.astype(np.complex128 if prec == "f64" else np.complex64).astype(np.complex128)


def cond_ciplv(g):
    r, m = g.real, g.imag
    s2 = np.maximum((1 - r) * (1 + r), 1e-200)
    s = np.sqrt(s2)
    return 1.0 / s + np.abs(m) * np.abs(r) / (s2 * s)


def compare(got, ref, tol, where=""):
    n = ref["plv"].shape[0]
    errs = {}
    for k in ("plv", "iplv"):
        errs[k] = np.abs(got[k] - ref[k]).max()
        assert errs[k] <= tol, "%s %s max err %.3g > %.3g" % (where, k, errs[k], tol)
    eg = np.abs(got["g"] - ref["g"])
    eg = np.maximum(np.abs(got["g"].real - ref["g"].real), np.abs(got["g"].imag - ref["g"].imag))
    errs["g"] = eg.max()
    assert errs["g"] <= tol, "%s G max err %.3g > %.3g" % (where, errs["g"], tol)
    c = cond_ciplv(ref["g"])
    ec = np.abs(got["ciplv"] - ref["ciplv"])
    np.fill_diagonal(c, 1.0)
    ok = ec <= tol * c + 1e-15
    assert ok.all(), "%s ciplv err %.3g at cond %.3g" % (where, ec[~ok].max(), c[~ok][np.argmax(ec[~ok])])
    # exact conventions
    assert np.all(np.diag(got["plv"]) == 1.0)
    assert np.all(np.diag(got["iplv"]) == 0.0) and np.all(np.diag(got["ciplv"]) == 0.0)
    for k in ("plv", "iplv", "ciplv"):
        assert np.array_equal(got[k], got[k].T), k
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(got["g"][off], np.conj(got["g"].T)[off])
    return errs


@pytest.mark.parametrize("prec", PRECS)
def test_hand_derived_quarter_turns(prec):
    z, pairs = quarter_turns()
    got = gpu_full(z, prec)
    for (i, j), (gr, gi, p, ip, cp) in pairs.items():
        tol = TOL[prec]
        assert abs(got["g"][i, j].real - gr) <= tol
        assert abs(got["g"][i, j].imag - gi) <= tol
        assert abs(got["plv"][i, j] - p) <= tol
        assert abs(got["iplv"][i, j] - ip) <= tol
        assert abs(got["ciplv"][i, j] - cp) <= 2 * tol


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,t", [(1, 1), (2, 3), (17, 31), (127, 200), (129, 1000), (300, 4097), (64, 2048)])
def test_ragged_shapes_against_oracle(prec, n, t):
    z = synth.glag_analytic(n, t, 1000.0, 4, (8, 12), seed=synth.seed_for(2, n * 7 + t))
    ref = oracle.full_from_analytic(exact_input(z, prec))
    got = gpu_full(z, prec)
    compare(got, ref, TOL[prec], "n=%d t=%d %s" % (n, t, prec))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
def test_window_and_row_stride(prec):
    n, t = 70, 3000
    z = synth.glag_analytic(n, t + 37, 1000.0, 3, (8, 12), seed=101)
    big = np.zeros((n, t + 100), dtype=z.dtype)
    big[:, : t + 37] = z
    dev = to_dev(big, prec)[:, : t + 37]          # row stride t + 100 > t
    out = plv_mod().from_analytic(dev, prec=prec, window=(37, 37 + 2900), want_g=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in out.items()}
    ref = oracle.full_from_analytic(exact_input(z, prec), window=(37, 37 + 2900))
    compare(got, ref, TOL[prec], "window")


@pytest.mark.parametrize("prec", PRECS)
def test_exact_zero_samples_take_unit_phasor(prec):
    z = synth.glag_analytic(5, 64, 1000.0, 2, (8, 12), seed=7)
    z[1, ::3] = 0.0
    z[2, 5] = complex(-0.0, -0.0)
    got = gpu_full(z, prec)
    ref = oracle.full_from_analytic(exact_input(z, prec))
    compare(got, ref, TOL[prec], "zeros")


@pytest.mark.parametrize("prec", ["f32", "split_bf16", "bf16"])
def test_tiny_and_huge_magnitudes(prec):
    z = synth.glag_analytic(6, 128, 1000.0, 2, (8, 12), seed=9)
    z[0] *= 1e-30
    z[1] *= 1e30
    z[2] *= 1e-42          # denormal in FP32
    got = gpu_full(z, prec)
    ref = oracle.full_from_analytic(exact_input(z, prec))
    compare(got, ref, TOL[prec], "scale")


@pytest.mark.parametrize("prec", ["f32", "split_bf16", "bf16"])
def test_deterministic(prec):
    z = to_dev(synth.glag_analytic(300, 5000, 1000.0, 4, (8, 12), seed=3), prec)
    a = plv_mod().from_analytic(z, prec=prec, want_g=True)
    b = plv_mod().from_analytic(z, prec=prec, want_g=True)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["f32", "split_bf16", "f64"])
def test_grouped_batch_equals_single_calls(prec):
    shapes = [(68, 700), (148, 1500), (360, 2500), (5, 40), (129, 4001)]
    zs = [to_dev(synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=200 + k), prec) for k, (n, t) in enumerate(shapes)]
    batch = plv_mod().from_analytic_batch(zs, prec=prec, want_g=True)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        zn = z.cpu().numpy().astype(np.complex128)
        ref = oracle.full_from_analytic(zn)
        got = {kk: v.cpu().numpy().astype(np.complex128 if kk == "g" else np.float64) for kk, v in batch[k].items()}
        compare(got, ref, TOL[prec], "batch %d" % k)


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
def test_grouped_multichunk_problems(prec):
    """A grouped call whose long problems span two K-chunks (T = 20000 past
    the 16384-sample chunk cap), so their sums go through the epilogue over
    the launch's tile list with both tile edges present (68 rows on 64-wide
    tiles, 360 on 128-wide), next to a single-chunk problem; every element
    against the oracle."""
    shapes = [(68, 20000), (360, 20000), (148, 900)]
    zs = [synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=synth.seed_for(2, 60 + k))
          for k, (n, t) in enumerate(shapes)]
    batch = plv_mod().from_analytic_batch([to_dev(z, prec) for z in zs], prec=prec, want_g=True)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        ref = oracle.full_from_analytic(exact_input(z, prec))
        got = {kk: v.cpu().numpy().astype(np.complex128 if kk == "g" else np.float64) for kk, v in batch[k].items()}
        compare(got, ref, TOL[prec], "grouped multi-chunk %d %s" % (k, prec))


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
def test_sensor_scale_workload_sampled_pairs(prec):
    """N = 1024 analytic signals of T = 60000 samples (1 kHz, 60 s), 32 latent
    8-12 Hz oscillators: the full-size workload, in the launch configuration
    the benchmark times.  Every pair among 256 rows -- four from each 16-row
    block, so every 16 x 16 MFMA block of every 128 x 128 tile holds 16
    checked entries -- against the oracle (which computes pairs one by one),
    plus every zero-lag-mixed neighbour pair (2m, 2m+1) of the first 200
    rows; then a bilinear probe per tile and properties of every entry."""
    n, t = 1024, 60000
    z = synth.glag_analytic(n, t, 1000.0, 32, (8.0, 12.0), seed=synth.seed_for(2), dtype=np.complex64)
    got = gpu_full(z, prec)
    rng = np.random.default_rng(5)
    rows = np.sort(np.concatenate([16 * q + rng.choice(16, size=4, replace=False) for q in range(n // 16)]))
    ii, jj = np.triu_indices(len(rows), 1)
    pr = np.concatenate([np.stack([rows[ii], rows[jj]], 1),
                         np.stack([np.arange(0, 200, 2), np.arange(1, 200, 2)], 1)])
    g = oracle.pairs_from_analytic(z.astype(np.complex128), pr)
    p, ip, cp = oracle.metrics(g)
    a, b = pr[:, 0], pr[:, 1]
    tol = TOL[prec]
    gg = got["g"][a, b]
    assert np.abs(gg.real - g.real).max() <= tol
    assert np.abs(gg.imag - g.imag).max() <= tol
    assert np.abs(got["plv"][a, b] - p).max() <= tol
    assert np.abs(got["iplv"][a, b] - ip).max() <= tol
    c = cond_ciplv(g)
    assert np.all(np.abs(got["ciplv"][a, b] - cp) <= tol * c + 1e-15)
    # every entry: symmetric, bounded, diagonal conventions, trace of G = N
    assert np.array_equal(got["plv"], got["plv"].T)
    assert got["plv"].max() <= 1.0 + 1e-5 and got["plv"].min() >= 0.0
    assert abs(np.trace(got["g"]).real - n) <= n * tol
    # per tile (I, J): with unit-modulus weights w on the rows of panel I and
    # v on those of panel J, sum_ij conj(w_i) G_ij v_j = (1/T) sum_t a(t) b(t),
    # a = sum_i conj(w_i) u_i, b = sum_j v_j conj(u_j) over the exact phasors;
    # each of the tile's 128^2 entries is within tol, hence the bound
    u = z.astype(np.complex128)
    u = u / np.abs(u)
    bm = 128
    for I in range(n // bm):
        for J in range(I, n // bm):
            w = np.exp(2j * np.pi * rng.random(bm))
            v = np.exp(2j * np.pi * rng.random(bm))
            ra, rb = slice(I * bm, (I + 1) * bm), slice(J * bm, (J + 1) * bm)
            lhs = np.conj(w) @ got["g"][ra, rb] @ v
            rhs = np.sum((np.conj(w) @ u[ra]) * (v @ np.conj(u[rb]))) / t
            assert abs(lhs - rhs) <= 2 * tol * bm * bm, (I, J)


def test_input_rows_off_a_16_byte_boundary():
    """A z[:, 1:] view: every row starts 8 bytes past a 16-byte boundary, so
    the normalisation must take its per-sample loads, with the same result
    as a contiguous copy and the oracle."""
    n, t = 70, 1001
    z = synth.glag_analytic(n, t + 1, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(2, 40), dtype=np.complex64)
    zd = torch.from_numpy(z).cuda()
    view = zd[:, 1:]
    assert view.data_ptr() % 16 == 8 and view.stride(0) == t + 1
    for prec in ("split_bf16", "f32"):
        got = plv_mod().from_analytic(view, prec=prec, want_g=True)
        ref = plv_mod().from_analytic(view.contiguous(), prec=prec, want_g=True)
        torch.cuda.synchronize()
        for k in ("plv", "iplv", "ciplv", "g"):
            assert torch.equal(got[k], ref[k]), (prec, k)
        o = oracle.full_from_analytic(exact_input(z[:, 1:], prec))
        h = {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in got.items()}
        compare(h, o, TOL[prec], "offset view %s" % prec)


@pytest.mark.parametrize("t", [200, 3000])
def test_outputs_off_a_16_byte_boundary(t):
    """Outputs 4 bytes (G 8 bytes) past a 16-byte boundary, given through the
    C ABI: the measures are then written entry by entry instead of four
    entries per 16-byte store -- by the Gram kernel's fused store (T = 200,
    one K-chunk) or by the epilogue (T = 3000, several chunks) -- with
    bit-identical results."""
    import ctypes as C

    from paper_1710_08037_amd import _abi, api
    n = 148   # a multiple of 4, so aligned outputs take the four-entry stores
    z = synth.glag_analytic(n, t, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(2, 41 + t), dtype=np.complex64)
    zd = torch.from_numpy(z).cuda()
    for prec in ("split_bf16", "f32"):
        ref = plv_mod().from_analytic(zd, prec=prec, want_g=True)
        outs = {k: torch.zeros(n * n + 4, dtype=torch.float32, device="cuda")[1:1 + n * n]
                for k in ("plv", "iplv", "ciplv")}
        outs["g"] = torch.zeros(n * n + 2, dtype=torch.complex64, device="cuda")[1:1 + n * n]
        assert all(o.data_ptr() % 16 != 0 for o in outs.values())
        p = _abi.PREC[prec]
        arr = _abi.problems([_abi.Problem(n, t, t, 0, 0, zd.data_ptr(),
                                          *(outs[k].data_ptr() for k in ("plv", "iplv", "ciplv", "g")))])
        ctx = api.context(zd.device)
        ws = api._workspace(ctx, _abi.OP_FROM_ANALYTIC, p, arr, None, 1, zd.device)
        _abi.check(_abi.lib().plv_from_analytic(ctx.handle, p, arr, 1, C.c_void_p(ws.data_ptr()), ws.numel(),
                                                api._stream(zd.device)), ctx.handle)
        torch.cuda.synchronize()
        for k in ("plv", "iplv", "ciplv", "g"):
            assert torch.equal(outs[k].view(n, n), ref[k]), (prec, k)
        o = oracle.full_from_analytic(exact_input(z, prec))
        h = {k: v.view(n, n).cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in outs.items()}
        compare(h, o, TOL[prec], "offset outputs %s" % prec)


@pytest.mark.parametrize("prec", ["f32", "split_bf16", "f64"])
def test_many_tiles_many_chunks_sampled_pairs(prec):
    """N = 2000 signals (16 tiles a side, 8 for FP64's smaller tiles: the
    launch order of the tiles is blocked, not row-major) over T = 40000
    samples (several K-chunks, so chunk sums go through the partial slots and
    the epilogue): every pair among 40 sampled rows, which land in many
    different tiles, against the oracle."""
    n, t = 2000, 40000
    z = synth.uniform_phasors(n, t, seed=synth.seed_for(2, 7), dtype=np.complex64)
    lagged = synth.glag_analytic(200, t, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(2, 8), dtype=np.complex64)
    z[::10] = lagged  # some structure spread over all tiles
    got = gpu_full(z, prec)
    rows = np.sort(np.random.default_rng(9).choice(n, size=40, replace=False))
    ref = oracle.full_from_analytic(exact_input(z[rows], prec))
    sub = {k: v[np.ix_(rows, rows)] for k, v in got.items()}
    compare(sub, ref, TOL[prec], "N=2000 T=40000 %s" % prec)


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
@pytest.mark.parametrize("t", [16384, 60000])
def test_coherent_signals_keep_fp32_accuracy(prec, t):
    """The worst case for the FP32 accumulation inside a K-chunk: pure tones
    of one frequency, so every pair is perfectly locked (|G| = 1,
    G_ij = exp(i(a_i - a_j))) and every term of a sum is the same number, so
    rounding errors cannot cancel.  Every entry against the oracle at the FP32
    tolerance (measured: max |dG| about 1.3e-7 in FP32 and 1.9e-6 in the split
    form, at any T, with K-chunks of up to 16384 samples)."""
    n = 48
    rng = np.random.default_rng(21)
    a = rng.uniform(0, 2 * np.pi, size=n)
    s = np.arange(t)
    z = np.exp(1j * (0.0731 * s[None, :] + a[:, None])) * rng.uniform(0.5, 2.0, size=(n, 1))
    z = z.astype(np.complex64)
    got = gpu_full(z, prec)
    ref = oracle.full_from_analytic(exact_input(z, prec))
    compare(got, ref, TOL[prec], "coherent t=%d %s" % (t, prec))
