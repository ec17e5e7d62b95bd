"""Long-T parity: T = 1.2e6 unit phasors, where the contraction runs as FP32
MFMA accumulation inside K-chunks of at most 16384 samples and FP64 sums
across the chunks (several launches when the partial slots cannot hold every
chunk at once).

The phasors come from the device generator (torch's seeded generator on the
GPU: 144 GB at full size cannot be built on the host); the rows a check needs
are copied to the host and handed to the FP64 oracle.  Tolerances are those
of the other parity tests.  The planted pairs are also checked against what
their construction fixes: PLV = exp(-jitter^2 / 2) and iPLV = |sin lag| PLV up
to sampling noise of order 1 / sqrt(T).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, cond_ciplv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

T_LONG = 1_200_000


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


def check_pairs(out, z, pairs, extra_rows, prec, where):
    """GPU results on the planted pairs and on all pairs among extra_rows
    against the oracle on those rows; returns the oracle's G of the planted pairs."""
    planted = np.unique(pairs.reshape(-1))
    rows = np.unique(np.concatenate([planted, extra_rows]))
    pos = {int(v): k for k, v in enumerate(rows)}
    zz = z[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.complex128)
    loc = [[pos[int(a)], pos[int(b)]] for a, b in pairs]
    ex = [pos[int(v)] for v in extra_rows]
    loc += [[ex[i], ex[j]] for i in range(len(ex)) for j in range(i + 1, len(ex))]
    loc = np.array(loc, dtype=np.int64)
    loc = np.stack([loc.min(1), loc.max(1)], 1)
    g = oracle.pair_means(oracle.phase(zz), loc)
    p, ip, cp = oracle.metrics(g)
    ia = torch.from_numpy(rows[loc[:, 0]]).cuda()
    ib = torch.from_numpy(rows[loc[:, 1]]).cuda()
    tol = TOL[prec]
    for k, ref in (("plv", p), ("iplv", ip)):
        got = out[k][ia, ib].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref).max()
        assert err <= tol, "%s %s max err %.3g > %.3g" % (where, k, err, tol)
        # mirrored entry is the same value
        assert np.array_equal(got, out[k][ib, ia].cpu().numpy().astype(np.float64))
    got = out["ciplv"][ia, ib].cpu().numpy().astype(np.float64)
    c = cond_ciplv(g)
    assert np.all(np.abs(got - cp) <= tol * c + 1e-15), where
    if out.get("g") is not None:
        gg = out["g"][ia, ib].cpu().numpy().astype(np.complex128)
        e = max(np.abs(gg.real - g.real).max(), np.abs(gg.imag - g.imag).max())
        assert e <= tol, "%s G max err %.3g" % (where, e)
    # G_ab of each planted pair in its own (a, b) order
    gp = g[: len(pairs)]
    return np.where(pairs[:, 0] < pairs[:, 1], gp, np.conj(gp))


def check_planted(g, lags, jitter, t):
    """PLV -> exp(-jitter^2/2) and the signed lag: G_ab -> exp(i lag) exp(-jitter^2/2)
    for phi_b = phi_a - lag + eta."""
    amp = math.exp(-jitter ** 2 / 2)
    noise = 6.0 / math.sqrt(t)
    assert np.all(np.abs(np.abs(g) - amp) <= noise)
    assert np.all(np.abs(g - amp * np.exp(1j * lags)) <= noise)


@pytest.mark.parametrize("prec", ["bf16", "f16", "split_bf16", "f32"])
def test_long_t_reduced_n(prec):
    """N = 256 signals of T = 1.2e6 samples, 8 planted pairs: the pairs and
    all pairs among 24 other random signals against the oracle."""
    from synth.device import phasors_planted_device
    n, npairs = 256, 8
    z, pairs, lags = phasors_planted_device(n, T_LONG, npairs, synth.seed_for(3, 1))
    out = plv_mod().from_analytic(z, prec=prec, want_g=True)
    torch.cuda.synchronize()
    rest = np.setdiff1d(np.arange(n), pairs.reshape(-1))
    extra = np.random.default_rng(31).choice(rest, size=24, replace=False)
    g = check_pairs(out, z, pairs, extra, prec, "N=256 T=1.2e6 %s" % prec)
    check_planted(g, lags, 0.1, T_LONG)
    del z, out
    torch.cuda.empty_cache()


def test_whole_brain_scale_sampled_pairs():
    """The whole-brain case at its real shape: N = 15000 unit phasors of
    T = 1.2e6 samples (144 GB complex64), 200 planted pairs, BF16 MFMA.  The
    FP64 partial sums of one K-chunk pass fill the slot budget, so T runs as
    many passes.  Checked: every planted pair and all pairs among 32 other
    random signals against the oracle, the planted pairs against their
    construction, and a random sample of unplanted pairs against the
    independent-phase scale sqrt(pi / (4 T))."""
    from synth.device import phasors_planted_device
    torch.cuda.empty_cache()
    n, npairs = 15000, 200
    print("whole-brain case: generating N=%d x T=%d" % (n, T_LONG), flush=True)
    z, pairs, lags = phasors_planted_device(n, T_LONG, npairs, synth.seed_for(3))
    print("whole-brain case: plv_from_analytic bf16", flush=True)
    out = plv_mod().from_analytic(z, prec="bf16")
    torch.cuda.synchronize()
    rest = np.setdiff1d(np.arange(n), pairs.reshape(-1))
    extra = np.random.default_rng(32).choice(rest, size=32, replace=False)
    g = check_pairs(out, z, pairs, extra, "bf16", "N=15000 T=1.2e6 bf16")
    check_planted(g, lags, 0.1, T_LONG)
    # unplanted pairs: mean PLV of independent phases is sqrt(pi / (4 T))
    rng = np.random.default_rng(33)
    a = rng.choice(rest, size=4096)
    b = rng.choice(rest, size=4096)
    keep = a != b
    vals = out["plv"][torch.from_numpy(a[keep]).cuda(), torch.from_numpy(b[keep]).cuda()].double().cpu().numpy()
    expect = math.sqrt(math.pi / (4 * T_LONG))
    assert abs(vals.mean() - expect) <= 0.1 * expect
    del z, out
    torch.cuda.empty_cache()
