"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/plv.h declares, and rejects bad arguments before it
would touch a device."""
import ctypes as C
import os
import re

import pytest

from paper_1710_08037_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "plv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(plv_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(_abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _abi.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert lib.plv_version() >= 10000


def test_status_strings():
    lib = _abi.lib()
    for s in range(5):
        assert lib.plv_status_str(s)
    assert lib.plv_status_str(99) == b"unknown status"


@pytest.fixture(scope="module")
def host_ctx():
    h = C.c_void_p()
    assert _abi.lib().plv_create(C.byref(h), -1) == 0
    yield h
    assert _abi.lib().plv_destroy(h) == 0


def _prob(n=64, t=2048, ld=None, t0=0, t1=0, ptr=4096):
    return _abi.Problem(n, t, ld if ld is not None else t, t0, t1, ptr, ptr, ptr, ptr, ptr)


def _ws(ctx, probs, op=_abi.OP_FROM_ANALYTIC, prec=2, bands=None, nb=1):
    arr = _abi.problems(probs)
    out = C.c_size_t(0)
    st = _abi.lib().plv_workspace_size(ctx, op, prec, arr, len(probs), bands, nb, C.byref(out))
    return st, out.value


def test_workspace_size_single_problem(host_ctx):
    st, nbytes = _ws(host_ctx, [_prob(1024, 60000)])
    assert st == 0
    # split planes: 2 x 1024 x 60000 x 4 B, plus FP64 partial slots
    assert nbytes > 2 * 1024 * 60000 * 4
    assert nbytes % 256 == 0


def test_workspace_grows_with_precision_width(host_ctx):
    sizes = {p: _ws(host_ctx, [_prob(256, 4096)], prec=_abi.PREC[p])[1] for p in _abi.PREC}
    assert sizes["bf16"] < sizes["split_bf16"] <= sizes["f32"] or sizes["bf16"] < sizes["f32"]
    assert sizes["bf16"] == sizes["f16"]


@pytest.mark.parametrize("kw", [dict(n=0), dict(t=0), dict(ld=10, t=20), dict(t0=-1), dict(t0=5, t1=5),
                                dict(t1=3000, t=2048), dict(ptr=0), dict(ptr=4097)])
def test_invalid_problems_rejected(host_ctx, kw):
    st, _ = _ws(host_ctx, [_prob(**kw)])
    assert st == 1
    assert _abi.lib().plv_last_error(host_ctx)


def test_invalid_enums_and_counts(host_ctx):
    assert _ws(host_ctx, [_prob()], prec=7)[0] == 1
    assert _ws(host_ctx, [_prob()], op=9)[0] == 1
    arr = _abi.problems([_prob()])
    out = C.c_size_t(0)
    assert _abi.lib().plv_workspace_size(host_ctx, 0, 2, arr, 0, None, 1, C.byref(out)) == 1
    assert _abi.lib().plv_workspace_size(host_ctx, 0, 2, None, 1, None, 1, C.byref(out)) == 1
    assert _abi.lib().plv_workspace_size(host_ctx, 0, 2, arr, 1, None, 1, None) == 1


def test_real_input_band_checks(host_ctx):
    bad, _ = _abi.bands([(10.0, 5.0)])
    assert _ws(host_ctx, [_prob()], op=_abi.OP_FROM_REAL, bands=bad, nb=1)[0] == 1
    good, nb = _abi.bands([(8.0, 12.0), (0.0, 0.0)])
    assert _ws(host_ctx, [_prob()], op=_abi.OP_FROM_REAL, bands=good, nb=nb)[0] == 0
    assert _ws(host_ctx, [_prob()], op=_abi.OP_FROM_REAL, bands=None, nb=2)[0] == 1


def test_backward_needs_forward_g(host_ctx):
    p = _prob()
    p.g = None
    assert _ws(host_ctx, [p], op=_abi.OP_BACKWARD_ANALYTIC)[0] == 1


def test_compute_on_host_only_context_is_rejected(host_ctx):
    arr = _abi.problems([_prob()])
    st = _abi.lib().plv_from_analytic(host_ctx, 2, arr, 1, C.c_void_p(256), 1 << 30, None)
    assert st == 1
    assert b"host-only" in _abi.lib().plv_last_error(host_ctx)


def test_autotune_checks_before_any_launch(host_ctx):
    arr = _abi.problems([_prob()])
    got = C.c_int32(-1)
    # a backward op is not tunable; a host-only context cannot run the trials
    st = _abi.lib().plv_autotune(host_ctx, _abi.OP_BACKWARD_ANALYTIC, 2, arr, 1, None, 1, 0.0, C.c_void_p(256),
                                 1 << 30, None, C.byref(got))
    assert st == 1 and got.value == 0
    assert b"forward op" in _abi.lib().plv_last_error(host_ctx)
    st = _abi.lib().plv_autotune(host_ctx, _abi.OP_FROM_ANALYTIC, 2, arr, 1, None, 1, 0.0, C.c_void_p(256),
                                 1 << 30, None, C.byref(got))
    assert st == 1 and got.value == 0
    assert b"host-only" in _abi.lib().plv_last_error(host_ctx)


def test_null_context_rejected():
    arr = _abi.problems([_prob()])
    assert _abi.lib().plv_from_analytic(None, 2, arr, 1, None, 0, None) == 1
    assert _abi.lib().plv_destroy(None) == 1


def test_tile_edge_model_and_overrides(host_ctx):
    L = _abi.lib()
    bm = C.c_int32(0)

    def edge(ctx, prec, n):
        assert L.plv_tile_edge(ctx, prec, n, C.byref(bm)) == 0
        return bm.value

    # whole-tile MFMA work over the upper triangle, the 64-wide tile's
    # counted 1/0.85 times: small row counts take the 64-wide tile
    for n, want in ((1, 64), (68, 64), (148, 64), (360, 128), (1000, 128), (1024, 128), (15000, 128)):
        assert edge(None, 2, n) == want, n
    assert edge(None, 0, 1000) == 64  # FP64 has only the 64-wide tile
    assert L.plv_set_tile_edge(host_ctx, 2, 1000, 64) == 0
    assert edge(host_ctx, 2, 1000) == 64
    assert edge(host_ctx, 1, 1000) == 128  # per precision
    assert L.plv_set_tile_edge(host_ctx, 2, 1000, 0) == 0
    assert edge(host_ctx, 2, 1000) == 128
    assert L.plv_set_tile_edge(host_ctx, 2, 1000, 96) == 1
    assert L.plv_set_tile_edge(host_ctx, 0, 1000, 128) == 1
    assert L.plv_tile_edge(None, 2, 0, C.byref(bm)) == 1


def test_workspace_follows_the_tile_edge(host_ctx):
    L = _abi.lib()
    # n = 148, one chunk: phasor planes of npad rows x tpad samples x 8 B (split),
    # npad = 192 with the 64-wide tile and 256 with the 128-wide one
    st, a = _ws(host_ctx, [_prob(148, 1000), _prob(148, 1000)])
    assert st == 0
    assert L.plv_set_tile_edge(host_ctx, 2, 148, 128) == 0
    st, b = _ws(host_ctx, [_prob(148, 1000), _prob(148, 1000)])
    assert L.plv_set_tile_edge(host_ctx, 2, 148, 0) == 0
    assert st == 0
    planes = 2 * 64 * 1024 * 8  # 64 more padded rows per problem
    assert planes - 4096 <= b - a <= planes  # less the smaller item table


def _trials_ws(ctx, prec, n, ntr, ntp=100):
    t = _abi.Trials(n, ntr, ntp, ntp, n * ntp, 1, 0, 0, 4096, 4096, 4096, 4096, 0)
    out = C.c_size_t(0)
    assert _abi.lib().plv_trials_workspace_size(ctx, _abi.PREC[prec], C.byref(t), C.byref(out)) == 0
    return out.value


def test_trials_pad_k_to_the_mode_unit(host_ctx):
    """Across trials the contracted length is the trial count (Eq. 8), a few
    dozen: the planes are padded only to the Gram kernel's K-unit of the mode
    (split BF16 16 samples, BF16 and FP16 32, FP32 8, FP64 4), so a count
    shares its workspace with the next multiple of that unit and needs less
    than the next multiple of 32 where the unit is smaller."""
    ws = lambda prec, ntr: _trials_ws(host_ctx, prec, 148, ntr)
    assert ws("split_bf16", 40) == ws("split_bf16", 48) < ws("split_bf16", 64)
    assert ws("split_bf16", 33) == ws("split_bf16", 48)
    assert ws("bf16", 40) == ws("bf16", 64) == ws("bf16", 33)
    assert ws("f16", 40) == ws("f16", 64)
    assert ws("f32", 40) < ws("f32", 48) < ws("f32", 64)
    assert ws("f64", 40) < ws("f64", 44) < ws("f64", 64)
    assert ws("f64", 41) == ws("f64", 44)
