"""GPU parity of the FIR band-pass (fir_order > 0: the forward-backward FIR
the paper applies before the Hilbert transform, with the build's own
design) against the FP64 oracle, element by element on the same seeded real
inputs: forward metrics on padded rows trimmed by the window, the adjoint
through the FIR band, a mix with DFT-bin bands in one call, and the
argument checks.  Tolerances are those of the other parity tests."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, compare
from tests.test_gpu_real import real_dev, exact_real, to_np
from tests.test_gpu_backward import upstream, rel, GTOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
@pytest.mark.parametrize("t", [2048, 1999])
def test_fir_bands_forward(prec, t):
    """N = 20 rows at 1 kHz, padded by the filter order on each side and
    trimmed: FIR bands of orders 200 and 400, a DFT-bin band and the plain
    analytic signal in one call (power-of-two and Bluestein lengths)."""
    n, fs = 20, 1000.0
    bands = [(8.0, 12.0, 200), (18.0, 22.0, 400), (8.0, 12.0), (0.0, 0.0)]
    win = (400, t - 400)
    x = synth.glag_real(n, t, fs, 4, (8, 22), seed=700 + t)
    out = plv_mod().from_real(real_dev(x, prec), fs, bands=bands, prec=prec, window=win, want_g=True)
    torch.cuda.synchronize()
    xr = exact_real(x, prec)
    for b, band in enumerate(bands):
        ref = oracle.full_from_real(xr, fs, None if band == (0.0, 0.0) else band, window=win)
        compare(to_np(out, b), ref, TOL[prec], "t=%d band %s %s" % (t, band, prec))


@pytest.mark.parametrize("prec", ["f64", "split_bf16"])
def test_short_fir_orders(prec):
    """Orders 2, 6 and 14 (1, 3 and 7 taps past the centre: fewer than the
    weight kernel's lanes per bin, so most lanes sum nothing) and 18 (9
    taps: two per lane, the last lane one), in one call, against the oracle."""
    n, t, fs = 12, 1024, 1000.0
    bands = [(80.0, 160.0, 2), (80.0, 160.0, 6), (80.0, 160.0, 14), (80.0, 160.0, 18)]
    win = (32, t - 32)
    x = synth.glag_real(n, t, fs, 4, (90, 150), seed=731)
    out = plv_mod().from_real(real_dev(x, prec), fs, bands=bands, prec=prec, window=win, want_g=True)
    torch.cuda.synchronize()
    xr = exact_real(x, prec)
    for b, band in enumerate(bands):
        ref = oracle.full_from_real(xr, fs, band, window=win)
        compare(to_np(out, b), ref, TOL[prec], "short FIR band %s %s" % (band, prec))


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_fir_batch_of_uneven_rows(prec):
    """Several problems of different lengths, each with an FIR band: one
    weight table per (length, band)."""
    fs = 1000.0
    bands = [(4.0, 8.0, 300), (30.0, 45.0, 120)]
    shapes = [(12, 900), (30, 1500), (9, 2100), (16, 1024)]
    xs = [synth.glag_real(n, t, fs, 4, (3, 45), seed=720 + k) for k, (n, t) in enumerate(shapes)]
    outs = plv_mod().from_real_batch([real_dev(x, prec) for x in xs], fs, bands=bands, prec=prec, want_g=True)
    torch.cuda.synchronize()
    for k, x in enumerate(xs):
        xr = exact_real(x, prec)
        for b, band in enumerate(bands):
            compare(to_np(outs[k], b), oracle.full_from_real(xr, fs, band), TOL[prec],
                    "problem %d band %d" % (k, b))


@pytest.mark.parametrize("prec", ["f64", "split_bf16"])
def test_fir_backward(prec):
    """The adjoint through the FIR band (its weights are real, so the same
    table serves the transposed map)."""
    n, t, fs = 8, 900, 1000.0
    bands = [(8.0, 12.0, 160), (18.0, 22.0)]
    win = (160, 740)
    x = synth.glag_real(n, t, fs, 4, (8, 22), seed=83)
    dt = np.float64 if prec == "f64" else np.float32
    xd = torch.from_numpy(x.astype(dt)).cuda()
    out = plv_mod().from_real(xd, fs, bands=bands, prec=prec, window=win, want_g=True)
    ups = upstream(n, prec, nb=2, seed=5)
    din = plv_mod().backward_batch([xd], [out["g"]], [tuple(ups)], fs=fs, bands=bands, prec=prec,
                                   windows=[win])[0]
    torch.cuda.synchronize()
    xx = xd.cpu().numpy().astype(np.float64)
    ref = sum(oracle.grad_from_real(xx, fs, band, *(u[b].cpu().numpy().astype(np.float64) for u in ups),
                                    window=win) for b, band in enumerate(bands))
    assert rel(din.cpu().numpy().astype(np.float64), ref) <= GTOL[prec]


@pytest.mark.parametrize("band,fs", [((8.0, 12.0, 201), 1000.0), ((8.0, 12.0, -2), 1000.0),
                                     ((12.0, 12.0, 100), 1000.0), ((8.0, 600.0, 100), 1000.0),
                                     ((8.0, 12.0, 100000), 1000.0)])
def test_fir_band_arguments_refused(band, fs):
    from paper_1710_08037_amd._abi import PLVError
    x = real_dev(synth.glag_real(4, 512, fs, 2, 10.0, seed=1), "f32")
    with pytest.raises(PLVError, match="INVALID_ARG"):
        plv_mod().from_real(x, fs, bands=[band], prec="f32")


def test_fir_bench_size_sampled_rows():
    """The FIR workload bench.py times, at its size: N = 2048 real rows of
    T = 8192 at 1 kHz (4096-sample epoch with 2048 samples of padding each
    side), 8-12 Hz FIR of order 2000, split-BF16; all pairs among sampled
    rows against the oracle, and the global conventions."""
    n, t, fs, order, pad = 2048, 8192, 1000.0, 2000, 2048
    x = synth.glag_real(n, t, fs, 32, (8.0, 12.0), seed=synth.seed_for(7), dtype=np.float32)
    win = (pad, t - pad)
    band = (8.0, 12.0, order)
    out = plv_mod().from_real(real_dev(x, "split_bf16"), fs, bands=[band], prec="split_bf16", window=win,
                              want_g=True)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(9).choice(n, size=14, replace=False)]))
    got = {k: v[np.ix_(rows, rows)] for k, v in to_np(out, 0).items()}
    compare(got, oracle.full_from_real(exact_real(x[rows], "split_bf16"), fs, band, window=win),
            TOL["split_bf16"], "FIR bench size")
