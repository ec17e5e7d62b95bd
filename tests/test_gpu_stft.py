"""GPU parity of plv_coherence_stft -- coherency of real signals over
windowed segments (Section II.B, Eq. 12 with X_i(f, n) the DFT bins of
segments n; Section III.B's Hamming-windowed, overlapping segments) --
against the FP64 oracle (oracle.stft_bins + oracle.full_coherence), element
by element per bin, on the same seeded real inputs.

Tolerances as for plv_coherence (absolute on coherence, |Im C| and C; the
corrected imaginary coherency times its condition number): 1e-12 in F64,
1e-5 in F32 and split-BF16.  The segment spectra are summed in FP32 (FP64 in
F64 mode) from FP32 samples: each coefficient carries a relative error of a
few FP32 ulps times sqrt(L), far below 1e-5 on the coherency, whose value
does not depend on the scale of a row."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_coherence import compare

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "split_bf16": 1e-5}


def _gpu(xs, seg, hop, bins, win, prec, spans=None):
    import paper_1710_08037_amd as plv
    dt = np.float64 if prec == "f64" else np.float32
    outs = plv.coherence_stft_batch([torch.from_numpy(np.ascontiguousarray(x.astype(dt))).cuda() for x in xs],
                                    seg, hop, bins, win, prec=prec, windows=spans, want_g=True)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy().astype(np.complex128 if k == "c" else np.float64) for k, v in o.items()}
            for o in outs]


def _check(got, x, seg, hop, bins, win, prec, span=None, where=""):
    dt = np.float64 if prec == "f64" else np.float32
    ref = oracle.full_coherence_stft(x.astype(dt).astype(np.float64), seg, hop, bins[0], bins[1], win, span)
    assert got["coh"].shape[0] == len(ref)
    for b, r in enumerate(ref):
        compare({k: v[b] for k, v in got.items()}, r, TOL[prec], "%s bin %d" % (where, bins[0] + b))


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
@pytest.mark.parametrize("win", ["hamming", "hann", "rect"])
def test_segment_coherence_against_oracle(prec, win):
    # lagged oscillators at 8-12 Hz, 1 kHz: 1 Hz bins with 1000-sample
    # segments, 50% overlap (the paper's Hamming / half-overlap recipe)
    x = synth.glag_real(70, 12000, 1000.0, 6, (8.0, 12.0), seed=synth.seed_for(6, 500))
    got = _gpu([x], 1000, 500, (7, 13), win, prec)[0]
    _check(got, x, 1000, 500, (7, 13), win, prec, where="%s %s" % (prec, win))


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_ragged_segmentation_and_spans(prec):
    """Odd segment length and hop, a hop longer than the segment, a span
    [t0, t1) that does not hold a whole number of hops, DC and Nyquist bins,
    and two problems of different shapes in one grouped call."""
    xs = [synth.glag_real(37, 3001, 500.0, 4, (5.0, 40.0), seed=synth.seed_for(6, 501)),
          synth.glag_real(130, 2500, 500.0, 4, (5.0, 40.0), seed=synth.seed_for(6, 502))]
    spans = [(13, 2990), (0, 2500)]
    got = _gpu(xs, 101, 37, (0, 50), "hamming", prec, spans)
    for k, x in enumerate(xs):
        _check(got[k], x, 101, 37, (0, 50), "hamming", prec, spans[k], "problem %d" % k)
    got = _gpu([xs[1]], 64, 100, (30, 32), "hann", prec)[0]   # hop > seg: gaps between segments
    _check(got, xs[1], 64, 100, (30, 32), "hann", prec, where="gaps")


def test_sensor_scale_sampled_rows():
    """N = 1024 signals x 60 s at 1 kHz, 1000-sample Hamming segments with
    500 of overlap, 8-12 Hz (the bench workload): all pairs among 32 sampled
    rows, every bin."""
    n, t = 1024, 60000
    x = synth.glag_real(n, t, 1000.0, 32, (8.0, 12.0), seed=synth.seed_for(6, 7), dtype=np.float32)
    got = _gpu([x], 1000, 500, (8, 12), "hamming", "split_bf16")[0]
    rows = np.sort(np.random.default_rng(11).choice(n, size=32, replace=False))
    sub = {k: v[:, rows][:, :, rows] for k, v in got.items()}
    _check(sub, x[rows], 1000, 500, (8, 12), "hamming", "split_bf16", where="sensor")


def test_bad_segmentation_is_rejected():
    import paper_1710_08037_amd as plv
    from paper_1710_08037_amd._abi import PLVError
    x = torch.zeros((4, 100), dtype=torch.float32, device="cuda")
    for seg, hop, bins in ((1, 1, (0, 0)), (200, 10, (0, 1)), (64, 0, (0, 1)), (64, 8, (5, 40)), (64, 8, (3, 2))):
        with pytest.raises(PLVError):
            plv.coherence_stft(x, seg, hop, bins)
