"""Tile edges of the grouped Gram launch (the per-trial loop of the paper's
Appendix, batched): every row-count bucket of the uneven workload
(N in {68, 148, 360, 1000}) with the 64- and the 128-wide output tile, alone
and mixed in one call (one launch per edge), element by element against the
FP64 oracle; and plv_autotune's per-row-count choice for a grouped call.

Analytic input (the tile choice is a property of the Gram stage); T short
enough for the oracle's all-pairs sums, ragged in T and in N against both
tile edges."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, compare, exact_input, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BUCKETS = [(68, 777), (148, 1000), (360, 603), (1000, 430)]


def _inputs(prec):
    zs = [synth.glag_analytic(n, t, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(4, 300 + k), dtype=np.complex64)
          for k, (n, t) in enumerate(BUCKETS)]
    return zs


def _run(zs, prec):
    import paper_1710_08037_amd as plv
    outs = plv.from_analytic_batch([to_dev(z, prec) for z in zs], prec=prec, want_g=True)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in o.items()}
            for o in outs]


@pytest.fixture(scope="module")
def refs():
    zs = _inputs("split_bf16")
    return zs, [oracle.full_from_analytic(exact_input(z, "split_bf16")) for z in zs]


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
@pytest.mark.parametrize("edges", [(64, 64, 64, 64), (128, 128, 128, 128), (64, 64, 128, 128)])
def test_every_bucket_with_each_tile_edge(refs, prec, edges):
    import paper_1710_08037_amd as plv
    zs, ref = refs
    try:
        for (n, _), bm in zip(BUCKETS, edges):
            plv.set_tile_edge(n, bm, prec)
            assert plv.tile_edge(n, prec) == bm
        print("tiles", prec, edges, flush=True)
        got = _run(zs, prec)
    finally:
        for n, _ in BUCKETS:
            plv.set_tile_edge(n, 0, prec)
    for (n, t), g, r, bm in zip(BUCKETS, got, ref, edges):
        compare(g, r, TOL[prec], "n=%d t=%d bm=%d %s" % (n, t, bm, prec))


def test_tile_edges_give_the_same_measures(refs):
    """Both edges sum the same products over the same K-chunk: the results
    agree to the split form's rounding, far inside the tolerance."""
    import paper_1710_08037_amd as plv
    zs, _ = refs
    res = {}
    for bm in (64, 128):
        for n, _ in BUCKETS:
            plv.set_tile_edge(n, bm)
        res[bm] = _run(zs, "split_bf16")
    for n, _ in BUCKETS:
        plv.set_tile_edge(n, 0)
    for a, b in zip(res[64], res[128]):
        assert np.abs(a["g"] - b["g"]).max() <= 1e-6


def test_autotune_picks_an_edge_per_row_count(refs):
    import paper_1710_08037_amd as plv
    zs, ref = refs
    xs = [to_dev(z, "split_bf16") for z in zs]
    try:
        chosen = plv.autotune_batch(xs, prec="split_bf16")
        print("autotuned edges", chosen, flush=True)
        assert set(chosen) == {n for n, _ in BUCKETS}
        assert all(bm in (64, 128) for bm in chosen.values())
        got = _run(zs, "split_bf16")
    finally:
        for n, _ in BUCKETS:
            plv.set_tile_edge(n, 0)
    for (n, t), g, r in zip(BUCKETS, got, ref):
        compare(g, r, TOL["split_bf16"], "autotuned n=%d" % n)
