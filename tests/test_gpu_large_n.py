"""A single problem of many tiles in the 16-bit modes: N = 4100 signals (33
tile rows, the last one ragged) over one K-chunk (the fused store) and over
several (partial sums and the epilogue), against the FP64 oracle on every
pair among sampled rows that reach many tiles on and off the diagonal and
the ragged end."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, compare, exact_input

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def sampled_rows(n, seed):
    rng = np.random.default_rng(seed)
    rows = set(range(n - 4, n))                      # the ragged last tile
    for tile in range(0, (n + 127) // 128, 3):       # rows in many tiles
        rows.update(int(r) for r in tile * 128 + rng.choice(128, size=2, replace=False) if r < n)
    rows.update(int(r) for r in rng.choice(n, size=24, replace=False))
    return np.array(sorted(rows))


@pytest.mark.parametrize("prec", ["split_bf16", "bf16", "f16"])
@pytest.mark.parametrize("t", [640, 20000])
def test_large_n_16bit_against_oracle(prec, t):
    import paper_1710_08037_amd as plv
    n = 4100
    z = synth.uniform_phasors(n, t, seed=synth.seed_for(2, 11), dtype=np.complex64)
    lagged = synth.glag_analytic(410, t, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(2, 12), dtype=np.complex64)
    z[::10] = lagged  # structure spread over every tile
    print("large N: N=%d T=%d %s" % (n, t, prec), flush=True)
    out = plv.from_analytic(torch.from_numpy(z).cuda(), prec=prec, want_g=True)
    rows = sampled_rows(n, seed=t)
    ri = torch.from_numpy(rows).cuda()
    got = {k: v.index_select(0, ri).index_select(1, ri).cpu().numpy().astype(
        np.complex128 if k == "g" else np.float64) for k, v in out.items()}
    torch.cuda.synchronize()
    ref = oracle.full_from_analytic(exact_input(z[rows], prec))
    compare(got, ref, TOL[prec], "N=%d T=%d %s" % (n, t, prec))
