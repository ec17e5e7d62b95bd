"""The uneven batch at its full size, in the launch configuration bench.py
times: 512 trials (N in {68, 148, 360, 1000}, T uniform in [500, 4000] at
1 kHz), five 4 Hz bands, real FP32 input, split-BF16 and plain BF16 -- one
call, one grouped Gram launch.  The same seeded inputs as the benchmark.

Checked against the FP64 oracle on sampled outputs: for trials chosen to
cover every N and every transform size class (plain and Bluestein lengths up
to M = 8192), all pairs among sampled rows (first, last and random rows) in
every band, to each precision's tolerance in the other parity tests.  The
analytic signal is per row, so the oracle needs only those rows.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, cond_ciplv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def compare_metrics(got, ref, tol, where):
    """PLV and iPLV to tol, ciPLV to tol times its condition number (from the
    oracle's G), the diagonal conventions and symmetry (the call asks for no
    G, as the benchmark's does not)."""
    for k in ("plv", "iplv"):
        err = np.abs(got[k] - ref[k]).max()
        assert err <= tol, "%s %s max err %.3g > %.3g" % (where, k, err, tol)
    c = cond_ciplv(ref["g"])
    np.fill_diagonal(c, 1.0)
    ec = np.abs(got["ciplv"] - ref["ciplv"])
    assert np.all(ec <= tol * c + 1e-15), "%s ciplv err %.3g" % (where, ec.max())
    assert np.all(np.diag(got["plv"]) == 1.0)
    assert np.all(np.diag(got["iplv"]) == 0.0) and np.all(np.diag(got["ciplv"]) == 0.0)
    for k in ("plv", "iplv", "ciplv"):
        assert np.array_equal(got[k], got[k].T), k


@pytest.mark.parametrize("prec", ["split_bf16", "bf16"])
def test_uneven_batch_full_size_sampled(prec):
    import paper_1710_08037_amd as plv
    fs = 1000.0
    seed = synth.seed_for(4)
    shapes = synth.batch_shapes(512, seed)
    xs = [synth.glag_real(n, t, fs, 32, (2.0, 42.0), seed=seed + 1 + k, dtype=np.float32)
          for k, (n, t) in enumerate(shapes)]
    bands = synth.bands_hz()
    print("uneven batch: 512 trials, from_real_batch", prec, flush=True)
    outs = plv.from_real_batch([torch.from_numpy(x).cuda() for x in xs], fs, bands=bands, prec=prec)
    torch.cuda.synchronize()

    # trials: for each N, the shortest, median and longest T
    pick = set()
    for n in synth.BATCH_NS:
        ks = [k for k, (nn, _) in enumerate(shapes) if nn == n]
        ks.sort(key=lambda k: shapes[k][1])
        pick.update([ks[0], ks[len(ks) // 2], ks[-1]])
    # every transform size class: 2t - 1 <= 1024, 2048, 4096, 8192
    for lo, hi in ((0, 512), (513, 1024), (1025, 2048), (2049, 4096)):
        ks = [k for k, (_, t) in enumerate(shapes) if lo <= t <= hi]
        if ks:
            pick.add(ks[0])
    rng = np.random.default_rng(41)
    for k in sorted(pick):
        n, t = shapes[k]
        rows = np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=min(n, 10), replace=False)]))
        xr = xs[k][rows].astype(np.float64)
        for b, band in enumerate(bands):
            ref = oracle.full_from_real(xr, fs, band)
            got = {m: outs[k][m][b].cpu().numpy().astype(np.float64)[np.ix_(rows, rows)]
                   for m in ("plv", "iplv", "ciplv")}
            compare_metrics(got, ref, TOL[prec], "trial %d (N=%d T=%d) band %d" % (k, n, t, b))
