"""GPU adjoint (plv_backward) against the FP64 oracle's angle-space gradient
and against finite differences of the GPU's own FP64 forward.

Tolerance: relative L2 error of the whole gradient, 1e-9 in FP64 and 1e-4
for the FP32 and split-BF16 paths (the gradient carries 1/|z| and the ciPLV
derivative's 1/s^3, so it is judged as a vector, not entry by entry).  The
plain BF16 / FP16 modes run their adjoint product in split form, but the
adjoint is evaluated at their own forward G, whose error (up to 5.6e-3 and
7.0e-4 absolute) enters through the metric derivatives' 1/|G| and 1/s^3:
2e-3 (BF16) and 5e-4 (FP16, 8x finer rounding) relative.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GTOL = {"f64": 1e-9, "f32": 1e-4, "split_bf16": 1e-4, "bf16": 2e-3, "f16": 5e-4}
RNG = np.random.default_rng(99)


def plv_mod():
    import paper_1710_08037_amd as plv
    return plv


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a, prec, real):
    if real:
        dt = np.float64 if prec == "f64" else np.float32
    else:
        dt = np.complex128 if prec == "f64" else np.complex64
    return torch.from_numpy(np.ascontiguousarray(a.astype(dt))).cuda()


def rdt(prec):
    return torch.float64 if prec == "f64" else torch.float32


def upstream(n, prec, nb=None, seed=0):
    rng = np.random.default_rng(seed)
    shape = (n, n) if nb is None else (nb, n, n)
    return [torch.from_numpy(rng.standard_normal(shape)).to(rdt(prec)).cuda() for _ in range(3)]


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16", "bf16", "f16"])
@pytest.mark.parametrize("n,t", [(9, 60), (33, 300)])
def test_backward_analytic_against_oracle(prec, n, t):
    z = synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=700 + n)
    zd = dev(z, prec, False)
    out = plv_mod().from_analytic(zd, prec=prec, want_g=True)
    ups = upstream(n, prec, seed=n)
    din = plv_mod().backward_batch([zd], [out["g"]], [tuple(ups)], prec=prec)[0]
    torch.cuda.synchronize()
    zx = zd.cpu().numpy().astype(np.complex128)
    ref = oracle.grad_from_analytic(zx, *(u.cpu().numpy().astype(np.float64) for u in ups))
    assert rel(din.cpu().numpy().astype(np.complex128), ref) <= GTOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
def test_backward_analytic_window_and_stride(prec):
    n, t = 12, 400
    z = synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=71)
    big = np.zeros((n, t + 24), dtype=np.complex128)
    big[:, :t] = z
    zd = dev(big, prec, False)[:, :t]
    win = (30, 370)
    out = plv_mod().from_analytic(zd, prec=prec, window=win, want_g=True)
    ups = upstream(n, prec, seed=5)
    din = plv_mod().backward_batch([zd], [out["g"]], [tuple(ups)], prec=prec, windows=[win])[0]
    torch.cuda.synchronize()
    zx = zd.cpu().numpy().astype(np.complex128)
    ref = oracle.grad_from_analytic(zx, *(u.cpu().numpy().astype(np.float64) for u in ups), window=win)
    got = din.cpu().numpy().astype(np.complex128)
    assert rel(got, ref) <= GTOL[prec]
    assert np.all(got[:, :30] == 0) and np.all(got[:, 370:] == 0)


@pytest.mark.parametrize("prec", ["f64", "f32", "split_bf16"])
@pytest.mark.parametrize("t", [256, 200])
def test_backward_real_against_oracle(prec, t):
    n, fs = 10, 1000.0
    x = synth.glag_real(n, t, fs, 3, (8, 12), seed=800 + t)
    xd = dev(x, prec, True)
    out = plv_mod().from_real(xd, fs, prec=prec, want_g=True)
    ups = upstream(n, prec, nb=1, seed=t)
    din = plv_mod().backward_batch([xd], [out["g"]], [tuple(ups)], fs=fs, prec=prec)[0]
    torch.cuda.synchronize()
    xx = xd.cpu().numpy().astype(np.float64)
    ref = oracle.grad_from_real(xx, gp=ups[0][0].cpu().numpy().astype(np.float64),
                                gi=ups[1][0].cpu().numpy().astype(np.float64),
                                gc=ups[2][0].cpu().numpy().astype(np.float64))
    assert rel(din.cpu().numpy().astype(np.float64), ref) <= GTOL[prec]


@pytest.mark.parametrize("prec", ["f64", "split_bf16"])
@pytest.mark.parametrize("t", [600, 3001, 8192])
def test_backward_real_bands_window(prec, t):
    """Two bands (their band sum kept in the work-group's spectrum slot),
    Bluestein lengths of M = 2048 and 8192 and a plain 8192-point one."""
    n, fs = 8, 1000.0
    bands = [(8.0, 12.0), (18.0, 22.0)]
    win = (50, t - 40)
    x = synth.glag_real(n, t, fs, 4, (8, 22), seed=81)
    xd = dev(x, prec, True)
    out = plv_mod().from_real(xd, fs, bands=bands, prec=prec, window=win, want_g=True)
    ups = upstream(n, prec, nb=2, seed=3)
    din = plv_mod().backward_batch([xd], [out["g"]], [tuple(ups)], fs=fs, bands=bands, prec=prec,
                                   windows=[win])[0]
    torch.cuda.synchronize()
    xx = xd.cpu().numpy().astype(np.float64)
    ref = sum(oracle.grad_from_real(xx, fs, band, *(u[b].cpu().numpy().astype(np.float64) for u in ups),
                                    window=win) for b, band in enumerate(bands))
    assert rel(din.cpu().numpy().astype(np.float64), ref) <= GTOL[prec]


@pytest.mark.parametrize("prec", ["f32", "split_bf16"])
def test_backward_grouped_problems(prec):
    shapes = [(7, 90), (20, 128), (5, 333)]
    zs = [synth.glag_analytic(n, t, 1000.0, 3, (8, 12), seed=900 + k) for k, (n, t) in enumerate(shapes)]
    zds = [dev(z, prec, False) for z in zs]
    outs = plv_mod().from_analytic_batch(zds, prec=prec, want_g=True)
    ups = [tuple(upstream(n, prec, seed=k)) for k, (n, _) in enumerate(shapes)]
    dins = plv_mod().backward_batch(zds, [o["g"] for o in outs], ups, prec=prec)
    torch.cuda.synchronize()
    for k, zd in enumerate(zds):
        ref = oracle.grad_from_analytic(zd.cpu().numpy().astype(np.complex128),
                                        *(u.cpu().numpy().astype(np.float64) for u in ups[k]))
        assert rel(dins[k].cpu().numpy().astype(np.complex128), ref) <= GTOL[prec]


def test_autograd_function_matches_direct_call():
    n, t = 16, 128
    x = dev(synth.glag_real(n, t, 100.0, 2, 10.0, seed=4), "f32", True).requires_grad_(True)
    plv, iplv, ciplv = plv_mod().plv_metrics(x, fs=100.0, prec="split_bf16")
    w = torch.from_numpy(RNG.standard_normal((1, n, n))).float().cuda()
    loss = (w * ciplv).sum() + plv.sum()
    loss.backward()
    out = plv_mod().from_real(x.detach(), 100.0, prec="split_bf16", want_g=True)
    din = plv_mod().backward_batch([x.detach()], [out["g"]], [(torch.ones_like(plv), None, w)], fs=100.0,
                                   prec="split_bf16")[0]
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, din, rtol=0, atol=0)


def test_f64_directional_finite_differences():
    """N = 256, T = 4096 real signals in FP64: the adjoint's directional
    derivative against central differences of the GPU FP64 forward, for the
    ciPLV target loss L = sum_{i<j} (ciPLV_ij - C*_ij)^2, in 16 random
    directions."""
    n, t, fs = 256, 4096, 1000.0
    x = dev(synth.glag_real(n, t, fs, 16, (8, 12), seed=11), "f64", True)
    cstar = torch.from_numpy(synth.sparse_target(n, seed=12)).cuda()
    upper = torch.triu(torch.ones(n, n, dtype=torch.float64, device="cuda"), 1)

    def loss(xx):
        c = plv_mod().from_real(xx, fs, prec="f64", want=("ciplv",))["ciplv"][0]
        return float((((c - cstar) ** 2) * upper).sum())

    out = plv_mod().from_real(x, fs, prec="f64", want_g=True)
    dc = (2 * (out["ciplv"][0] - cstar) * upper)[None]
    g = plv_mod().backward_batch([x], [out["g"]], [(None, None, dc)], fs=fs, prec="f64")[0]
    rng = np.random.default_rng(13)
    for k in range(16):
        d = torch.from_numpy(rng.standard_normal((n, t))).cuda()
        d /= d.norm()
        eps = 1e-5 * float(x.abs().max())
        fd = (loss(x + eps * d) - loss(x - eps * d)) / (2 * eps)
        an = float((g * d).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (k, fd, an)


def test_f64_directional_finite_differences_full_size():
    """The differentiable case at its own size, N = 2048 real signals of
    T = 8192 samples, in FP64 (8192-point transforms): the adjoint's
    directional derivative of L = sum_{i<j} (ciPLV_ij - C*_ij)^2 against
    central differences of the GPU FP64 forward in 16 random directions.

    A unit direction in N T = 1.7e7 coordinates sees only about |g| / 4096 of
    the gradient (about 2e-3 here), so the differences take a large step,
    h = 1e-3 max|x|, with Richardson's extrapolation from h and 2h (error
    O(h^4)); what is left is the rounding of L itself, about 12 ulp of L per
    evaluation as measured, bounded here by 32 ulp over the step."""
    n, t, fs = 2048, 8192, 1000.0
    x = dev(synth.glag_real(n, t, fs, 32, (8, 12), seed=synth.seed_for(5)), "f64", True)
    cstar = torch.from_numpy(synth.sparse_target(n, seed=synth.seed_for(5, 1))).cuda()
    upper = torch.triu(torch.ones(n, n, dtype=torch.float64, device="cuda"), 1)

    def loss(xx):
        c = plv_mod().from_real(xx, fs, prec="f64", want=("ciplv",))["ciplv"][0]
        return float((((c - cstar) ** 2) * upper).sum())

    print("f64 finite differences: N=2048 T=8192, 16 directions", flush=True)
    out = plv_mod().from_real(x, fs, prec="f64", want_g=True)
    dc = (2 * (out["ciplv"][0] - cstar) * upper)[None]
    g = plv_mod().backward_batch([x], [out["g"]], [(None, None, dc)], fs=fs, prec="f64")[0]
    lval = loss(x)
    h = 1e-3 * float(x.abs().max())
    noise = 32 * 2.0 ** -53 * lval / h
    rng = np.random.default_rng(15)
    for k in range(16):
        d = torch.from_numpy(rng.standard_normal((n, t))).cuda()
        d /= d.norm()
        f1 = (loss(x + h * d) - loss(x - h * d)) / (2 * h)
        f2 = (loss(x + 2 * h * d) - loss(x - 2 * h * d)) / (4 * h)
        fd = (4 * f1 - f2) / 3
        an = float((g * d).sum())
        print("direction %d: fd %.12e analytic %.12e" % (k, fd, an), flush=True)
        assert abs(fd - an) <= 2e-6 * abs(an) + noise, (k, fd, an, noise)


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
def test_differentiable_case_sampled_rows(prec):
    """N = 2048 real signals of T = 8192 samples, loss = sum_{i<j} (ciPLV -
    C*)^2 with a 1%-sparse target: the full forward and adjoint on the GPU,
    the gradient of sampled rows against the FP64 oracle (its analytic signal
    by FFT, its pair sums restricted to pairs that touch the rows)."""
    n, t, fs = 2048, 8192, 1000.0
    x = synth.glag_real(n, t, fs, 32, (8, 12), seed=synth.seed_for(5))
    cstar = synth.sparse_target(n, seed=synth.seed_for(5, 1))
    xd = dev(x, prec, True)
    out = plv_mod().from_real(xd, fs, prec=prec, want_g=True)
    upper = torch.triu(torch.ones(n, n, device="cuda"), 1)
    dc = (2 * (out["ciplv"][0] - torch.from_numpy(cstar).float().cuda()) * upper)[None]
    g = plv_mod().backward_batch([xd], [out["g"]], [(None, None, dc)], fs=fs, prec=prec)[0]
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(14).choice(n, size=14, replace=False)]))
    xx = xd.cpu().numpy().astype(np.float64)
    # the oracle's own ciPLV for the upstream gradient of the rows' pairs
    z = oracle.analytic_fft(xx)
    phi = oracle.phase(z)
    a_idx, b_idx = np.triu_indices(n, 1)
    sel = np.isin(a_idx, rows) | np.isin(b_idx, rows)
    pr = np.stack([a_idx[sel], b_idx[sel]], 1)
    _, _, c = oracle.metrics(oracle.pair_means(phi, pr))
    dcs = np.zeros((n, n))
    dcs[pr[:, 0], pr[:, 1]] = 2 * (c - cstar[pr[:, 0], pr[:, 1]])
    ref = oracle.grad_from_real_rows(xx, rows, gc=dcs)
    got = g.cpu().numpy().astype(np.float64)[rows]
    assert rel(got, ref) <= GTOL[prec]
