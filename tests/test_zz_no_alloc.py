"""plv_from_analytic_noalloc (the allocation-free variant for callers that
cannot allocate device memory) against plv_from_analytic on the same inputs:
two calls in a row on one device, the second smaller, then the size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1710_08037_amd import _abi

gpu = pytest.mark.gpu


def _noalloc(z, prec, want_g=True):
    """Through the C ABI directly: outputs allocated here, no workspace."""
    from paper_1710_08037_amd import api
    p = _abi.PREC[prec]
    cd = torch.complex128 if p == 0 else torch.complex64
    rd = torch.float64 if p == 0 else torch.float32
    n, t = z.shape
    out = {k: torch.full((n, n), float("nan"), dtype=rd, device=z.device) for k in ("plv", "iplv", "ciplv")}
    out["g"] = torch.full((n, n), float("nan"), dtype=cd, device=z.device) if want_g else None
    prob = _abi.Problem(n, t, z.stride(0), 0, 0, z.data_ptr(), out["plv"].data_ptr(), out["iplv"].data_ptr(),
                        out["ciplv"].data_ptr(), out["g"].data_ptr() if want_g else None)
    arr = _abi.problems([prob])
    ctx = api.context(z.device)
    st = _abi.lib().plv_from_analytic_noalloc(ctx.handle, p, arr, 1, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out, ctx


def _ws_bytes(n, t, prec):
    h = C.c_void_p()
    assert _abi.lib().plv_create(C.byref(h), -1) == 0
    arr = _abi.problems([_abi.Problem(n, t, t, 0, 0, 4096, 4096, 4096, 4096, 4096)])
    out = C.c_size_t(0)
    assert _abi.lib().plv_workspace_size(h, _abi.OP_FROM_ANALYTIC, _abi.PREC[prec], arr, 1, None, 1,
                                         C.byref(out)) == 0
    _abi.lib().plv_destroy(h)
    return out.value


@gpu
@pytest.mark.parametrize("prec", ["split_bf16", "f32", "f64"])
def test_noalloc_equals_from_analytic_on_two_calls(prec):
    import paper_1710_08037_amd as plv

    cd = np.complex128 if prec == "f64" else np.complex64
    shapes = [(300, 6000), (96, 777)] if prec == "f64" else [(200, 3000), (96, 777)]
    for k, (n, t) in enumerate(shapes):
        assert _ws_bytes(n, t, prec) <= _abi.NOALLOC_MAX_BYTES
        print("noalloc", prec, "call", k, "n", n, "t", t, flush=True)
        z = torch.from_numpy(synth.glag_analytic(n, t, 1000.0, 8, (8.0, 12.0), seed=synth.seed_for(2, 50 + k),
                                                 dtype=cd)).cuda()
        st, got, ctx = _noalloc(z, prec)
        assert st == 0, _abi.lib().plv_last_error(ctx.handle)
        ref = plv.from_analytic(z, prec=prec, want_g=True)
        torch.cuda.synchronize()
        for key in ("plv", "iplv", "ciplv", "g"):
            # the same plan and the same kernels: identical results
            assert torch.equal(got[key], ref[key]), (prec, k, key)
        if k == 1:
            # and the oracle's bar on the second, smaller call
            o = oracle.full_from_analytic(z.cpu().numpy().astype(np.complex128))
            tol = 1e-12 if prec == "f64" else 1e-5
            assert np.abs(got["plv"].cpu().numpy().astype(np.float64) - o["plv"]).max() <= tol
            assert np.abs(got["g"].cpu().numpy().astype(np.complex128) - o["g"]).max() <= 2 * tol


@gpu
def test_noalloc_rejects_problems_beyond_its_scratch():
    n, t = 1024, 2000
    assert _ws_bytes(n, t, "split_bf16") > _abi.NOALLOC_MAX_BYTES
    z = torch.ones((n, t), dtype=torch.complex64, device="cuda")
    st, out, ctx = _noalloc(z, "split_bf16")
    torch.cuda.synchronize()
    assert st == 4  # PLV_ERR_UNSUPPORTED
    msg = _abi.lib().plv_last_error(ctx.handle).decode()
    assert "scratch" in msg and "bytes" in msg
    assert torch.isnan(out["plv"]).all()  # nothing was written


@gpu
def test_noalloc_takes_one_problem():
    from paper_1710_08037_amd import api
    z = torch.ones((8, 64), dtype=torch.complex64, device="cuda")
    o = torch.empty((8, 8), dtype=torch.float32, device="cuda")
    p = _abi.Problem(8, 64, 64, 0, 0, z.data_ptr(), o.data_ptr(), None, None, None)
    arr = _abi.problems([p, p])
    ctx = api.context(z.device)
    assert _abi.lib().plv_from_analytic_noalloc(ctx.handle, 2, arr, 2, None) == 4
