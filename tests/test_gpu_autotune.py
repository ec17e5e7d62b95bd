"""plv_autotune: the measured K-chunk count is kept in the context and later
calls of the same shape use it; their results match the FP64 oracle as the
untuned calls do (the chunking reorders only FP32 partial sums)."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import TOL, compare, exact_input, gpu_full, plv_mod, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_autotune_analytic_then_compute(prec):
    n, t = 200, 12000
    z = synth.glag_analytic(n, t, 1000.0, 6, (8, 12), seed=synth.seed_for(11, 1))
    k = plv_mod().autotune(to_dev(z, prec), prec=prec)
    torch.cuda.synchronize()
    assert k >= 1
    got = gpu_full(z, prec)
    compare(got, oracle.full_from_analytic(exact_input(z, prec)), TOL[prec], "tuned %s" % prec)
    # tuning again keeps a count of the same candidate kind and stays correct
    k2 = plv_mod().autotune(to_dev(z, prec), prec=prec)
    assert k2 >= 1
    compare(gpu_full(z, prec), oracle.full_from_analytic(exact_input(z, prec)), TOL[prec], "retuned %s" % prec)


def test_autotune_window():
    n, t, win = 90, 9000, (500, 8300)
    z = synth.glag_analytic(n, t, 1000.0, 4, (8, 12), seed=synth.seed_for(11, 2))
    assert plv_mod().autotune(to_dev(z, "split_bf16"), prec="split_bf16", window=win) >= 1
    got = gpu_full(z, "split_bf16", window=win)
    compare(got, oracle.full_from_analytic(exact_input(z, "split_bf16"), window=win), TOL["split_bf16"], "window")


def test_autotune_real_one_band():
    n, t, fs = 64, 8192, 1000.0
    x = synth.glag_real(n, t, fs, 8, (8.0, 12.0), seed=synth.seed_for(11, 3), dtype=np.float32)
    xd = torch.from_numpy(x).cuda()
    assert plv_mod().autotune(xd, prec="split_bf16", fs=fs, bands=[(8.0, 12.0)]) >= 1
    out = plv_mod().from_real(xd, fs, bands=[(8.0, 12.0)], prec="split_bf16", want_g=True)
    torch.cuda.synchronize()
    got = {k: v[0].cpu().numpy().astype(np.complex128 if k == "g" else np.float64) for k, v in out.items()}
    ref = oracle.full_from_real(x.astype(np.float64), fs, (8.0, 12.0))
    compare(got, ref, TOL["split_bf16"], "real band")


def test_autotune_coherence():
    n, t = 48, 6000
    z = synth.glag_analytic(n, t, 1000.0, 4, (8, 12), seed=synth.seed_for(11, 4))
    zd = to_dev(z, "f32")
    assert plv_mod().autotune(zd, prec="f32", coherence=True) >= 1
    got = plv_mod().coherence(zd, prec="f32")
    torch.cuda.synchronize()
    ref = oracle.full_coherence(exact_input(z, "f32"))
    assert np.abs(got["coh"].cpu().numpy() - ref["coh"]).max() <= 1e-5


def test_autotune_grouped_call_has_nothing_to_choose():
    n, t, fs = 32, 4000, 1000.0
    x = synth.glag_real(n, t, fs, 4, (8.0, 12.0), seed=synth.seed_for(11, 5), dtype=np.float32)
    k = plv_mod().autotune(torch.from_numpy(x).cuda(), prec="split_bf16", fs=fs, bands=[(8.0, 12.0), (13.0, 30.0)])
    assert k == 0
