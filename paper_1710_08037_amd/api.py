"""Torch-facing calls into libplv: allocate outputs and workspace with torch,
pass raw device pointers and the current HIP stream.  Every step of the
computation runs in the library's kernels; this module only marshals.
"""
from __future__ import annotations

import ctypes as C
import threading

import torch

from . import _abi

_CTX = {}
_CTX_LOCK = threading.Lock()


class Context:
    """A libplv context bound to one GPU."""

    def __init__(self, device: int):
        self.device = device
        h = C.c_void_p()
        _abi.check(_abi.lib().plv_create(C.byref(h), int(device)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _abi.lib().plv_destroy(h)
            except Exception:
                pass


def context(device=None) -> Context:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    with _CTX_LOCK:
        if idx not in _CTX:
            _CTX[idx] = Context(idx)
        return _CTX[idx]


def _prec_id(prec) -> int:
    if isinstance(prec, int):
        return prec
    try:
        return _abi.PREC[prec]
    except KeyError:
        raise ValueError("prec must be one of %s" % sorted(_abi.PREC)) from None


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _rows(x: torch.Tensor):
    if x.dim() != 2:
        raise ValueError("expected a 2-D [n, t] tensor, got shape %s" % (tuple(x.shape),))
    if x.stride(1) != 1:
        raise ValueError("samples must be contiguous (stride 1 along t)")
    if not x.is_cuda:
        raise ValueError("input must be a GPU tensor")
    return x.shape[0], x.shape[1], x.stride(0)


def _outputs(n, nb, real_dtype, cplx_dtype, dev, want, want_g):
    o = {}
    for k in ("plv", "iplv", "ciplv"):
        o[k] = torch.empty((nb, n, n), dtype=real_dtype, device=dev) if k in want else None
    o["g"] = torch.empty((nb, n, n), dtype=cplx_dtype, device=dev) if want_g else None
    return o


def _problem(x, window, outs):
    n, t, ld = _rows(x)
    t0, t1 = (0, 0) if window is None else (int(window[0]), int(window[1]))
    return _abi.Problem(n, t, ld, t0, t1, x.data_ptr(), *(_ptr(outs[k]) for k in ("plv", "iplv", "ciplv", "g")))


def _workspace(ctx, op, prec, probs, bands, nb, dev):
    nbytes = C.c_size_t(0)
    _abi.check(_abi.lib().plv_workspace_size(ctx.handle, op, prec, probs, len(probs), bands, nb, C.byref(nbytes)),
               ctx.handle)
    return torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)


ALL = ("plv", "iplv", "ciplv")


def from_analytic_noalloc(z, prec="split_bf16", window=None, want=ALL, want_g=False):
    """from_analytic for one problem through plv_from_analytic_noalloc: no
    workspace, the library's per-device scratch array instead (problems whose
    intermediate buffers exceed its size are rejected).  The outputs are still
    allocated here, by torch."""
    p = _prec_id(prec)
    dev = z.device
    cd = torch.complex128 if p == 0 else torch.complex64
    rd = torch.float64 if p == 0 else torch.float32
    if z.dtype != cd:
        raise TypeError("prec %s needs %s input, got %s" % (prec, cd, z.dtype))
    o = _outputs(z.shape[0], 1, rd, cd, dev, want, want_g)
    arr = _abi.problems([_problem(z, window, o)])
    ctx = context(dev)
    _abi.check(_abi.lib().plv_from_analytic_noalloc(ctx.handle, p, arr, 1, _stream(dev)), ctx.handle)
    return {k: (v[0] if v is not None else None) for k, v in o.items()}


def from_analytic_batch(zs, prec="split_bf16", windows=None, want=ALL, want_g=False):
    """PLV/iPLV/ciPLV of several analytic-signal problems in one grouped call.

    zs: list of complex GPU tensors [n_k, t_k] (complex64; complex128 for f64).
    Returns a list of dicts with [n_k, n_k] tensors plv, iplv, ciplv and g.
    """
    p = _prec_id(prec)
    dev = zs[0].device
    cd = torch.complex128 if p == 0 else torch.complex64
    rd = torch.float64 if p == 0 else torch.float32
    outs, probs = [], []
    for k, z in enumerate(zs):
        if z.dtype != cd:
            raise TypeError("prec %s needs %s input, got %s" % (prec, cd, z.dtype))
        o = _outputs(z.shape[0], 1, rd, cd, dev, want, want_g)
        outs.append(o)
        probs.append(_problem(z, None if windows is None else windows[k], o))
    arr = _abi.problems(probs)
    ctx = context(dev)
    ws = _workspace(ctx, _abi.OP_FROM_ANALYTIC, p, arr, None, 1, dev)
    _abi.check(_abi.lib().plv_from_analytic(ctx.handle, p, arr, len(probs), C.c_void_p(ws.data_ptr()), ws.numel(),
                                            _stream(dev)), ctx.handle)
    return [{k: (v[0] if v is not None else None) for k, v in o.items()} for o in outs]


def from_analytic(z, prec="split_bf16", window=None, want=ALL, want_g=False):
    """PLV/iPLV/ciPLV of one problem of analytic signals z [n, t]."""
    return from_analytic_batch([z], prec, None if window is None else [window], want, want_g)[0]


def coherence_batch(zs, prec="split_bf16", windows=None, want=ALL, want_g=False):
    """Coherency (Section II.B, Eq. 12) of several problems of complex rows in
    one call: Fourier coefficients over trials or windows, or analytic signals.

    zs: list of complex GPU tensors [n_k, t_k] (complex64; complex128 for f64).
    Returns a list of dicts of [n_k, n_k] tensors: 'coh' (coherence |C|),
    'icoh' (|Im C|), 'cicoh' (|Im C| / sqrt(1 - Re C^2)) and 'c' (complex C).
    `want` names the real outputs by their PLV-field names (plv, iplv, ciplv).
    """
    p = _prec_id(prec)
    dev = zs[0].device
    cd = torch.complex128 if p == 0 else torch.complex64
    rd = torch.float64 if p == 0 else torch.float32
    outs, probs = [], []
    for k, z in enumerate(zs):
        if z.dtype != cd:
            raise TypeError("prec %s needs %s input, got %s" % (prec, cd, z.dtype))
        o = _outputs(z.shape[0], 1, rd, cd, dev, want, want_g)
        outs.append(o)
        probs.append(_problem(z, None if windows is None else windows[k], o))
    arr = _abi.problems(probs)
    ctx = context(dev)
    ws = _workspace(ctx, _abi.OP_COHERENCE, p, arr, None, 1, dev)
    _abi.check(_abi.lib().plv_coherence(ctx.handle, p, arr, len(probs), C.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream(dev)), ctx.handle)
    names = {"plv": "coh", "iplv": "icoh", "ciplv": "cicoh", "g": "c"}
    return [{names[k]: (v[0] if v is not None else None) for k, v in o.items()} for o in outs]


def coherence(z, prec="split_bf16", window=None, want=ALL, want_g=False):
    """Coherency of one problem of complex rows z [n, t]; see coherence_batch."""
    return coherence_batch([z], prec, None if window is None else [window], want, want_g)[0]


def over_trials(z, prec="split_bf16", window=None, want=ALL, want_g=False):
    """Lachaux's PLV across trials (Eq. 1; matrix form Eq. 8): z is a complex
    GPU tensor [ntr, n, t] of analytic signals (any strides: trial-major data
    or a permuted view of signals x samples x trials).  For every time point
    of `window` (default all), PLV / iPLV / ciPLV over the trials.
    Returns a dict of [t1 - t0, n, n] tensors (and 'g' when want_g)."""
    p = _prec_id(prec)
    cd = torch.complex128 if p == 0 else torch.complex64
    rd = torch.float64 if p == 0 else torch.float32
    if z.dtype != cd:
        raise TypeError("prec %s needs %s input, got %s" % (prec, cd, z.dtype))
    if z.dim() != 3:
        raise ValueError("z must be [ntr, n, t]")
    ntr, n, t = z.shape
    t0, t1 = (0, t) if window is None else (int(window[0]), int(window[1]))
    dev = z.device
    o = _outputs(n, t1 - t0, rd, cd, dev, want, want_g)
    st = z.stride()
    d = _abi.Trials(n, ntr, t, st[1], st[0], st[2], t0, t1, z.data_ptr(),
                    *(_ptr(o[k]) for k in ("plv", "iplv", "ciplv", "g")))
    ctx = context(dev)
    nbytes = C.c_size_t(0)
    _abi.check(_abi.lib().plv_trials_workspace_size(ctx.handle, p, C.byref(d), C.byref(nbytes)), ctx.handle)
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
    _abi.check(_abi.lib().plv_over_trials(ctx.handle, p, C.byref(d), C.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream(dev)), ctx.handle)
    return o


def from_real_batch(xs, fs, bands=None, prec="split_bf16", windows=None, want=ALL, want_g=False):
    """PLV/iPLV/ciPLV of real signals, the analytic signal formed on the GPU.

    xs: list of real GPU tensors [n_k, t_k] (float32; float64 for f64).
    bands: list of (f_lo, f_hi) in Hz (a DFT-bin band), (f_lo, f_hi, order) (the
    forward-backward FIR band-pass of that even order), or None for the plain
    analytic signal.
    Returns a list of dicts with [nbands, n_k, n_k] tensors.
    """
    p = _prec_id(prec)
    dev = xs[0].device
    rd = torch.float64 if p == 0 else torch.float32
    cd = torch.complex128 if p == 0 else torch.complex64
    barr, nb = _abi.bands(bands)
    outs, probs = [], []
    for k, x in enumerate(xs):
        if x.dtype != rd:
            raise TypeError("prec %s needs %s input, got %s" % (prec, rd, x.dtype))
        o = _outputs(x.shape[0], nb, rd, cd, dev, want, want_g)
        outs.append(o)
        probs.append(_problem(x, None if windows is None else windows[k], o))
    arr = _abi.problems(probs)
    ctx = context(dev)
    ws = _workspace(ctx, _abi.OP_FROM_REAL, p, arr, barr, nb, dev)
    _abi.check(_abi.lib().plv_from_real(ctx.handle, p, arr, len(probs), barr, nb, float(fs),
                                        C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)), ctx.handle)
    return outs


def from_real(x, fs, bands=None, prec="split_bf16", window=None, want=ALL, want_g=False):
    return from_real_batch([x], fs, bands, prec, None if window is None else [window], want, want_g)[0]


def autotune(x, prec="split_bf16", window=None, fs=None, bands=None, coherence=False):
    """Measure the K-chunk count of one problem's forward call through
    plv_autotune and keep it for later calls of the same shape on this device.

    x: complex rows (analytic signals; Fourier coefficients with coherence=True)
    or real rows (then fs and at most one band).  Returns the count kept, or 0
    when there is nothing to choose.  Blocks until the trial runs finish.
    """
    p = _prec_id(prec)
    dev = x.device
    real = not x.is_complex()
    barr, nb = _abi.bands(bands) if real else (None, 1)
    rd = torch.float64 if p == 0 else torch.float32
    cd = torch.complex128 if p == 0 else torch.complex64
    o = _outputs(x.shape[0], nb, rd, cd, dev, ALL, False)
    arr = _abi.problems([_problem(x, window, o)])
    op = _abi.OP_FROM_REAL if real else (_abi.OP_COHERENCE if coherence else _abi.OP_FROM_ANALYTIC)
    ctx = context(dev)
    ws = _workspace(ctx, op, p, arr, barr, nb, dev)
    chosen = C.c_int32(0)
    _abi.check(_abi.lib().plv_autotune(ctx.handle, op, p, arr, 1, barr, nb, float(fs or 0.0),
                                       C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev), C.byref(chosen)),
               ctx.handle)
    return chosen.value


def coherence_stft_batch(xs, seg, hop, bins, window="hamming", prec="split_bf16", windows=None, want=ALL,
                         want_g=False):
    """Coherency of real rows over windowed segments (Section II.B, Eq. 12,
    the coefficients of segments of `seg` samples, `hop` apart) at the DFT
    bins bins = (k_lo, k_hi) of the segment length, through
    plv_coherence_stft: one call, every problem and bin in one grouped launch.

    xs: list of real GPU tensors [n_k, t_k] (float32; float64 for f64);
    windows: optional [t0, t1) per problem (segments start at t0).
    Returns a list of dicts of [nbins, n_k, n_k] tensors: 'coh' (coherence),
    'icoh' (|Im C|), 'cicoh' (corrected imaginary coherency), 'c' (C).
    `want` names the real outputs by their PLV-field names (plv, iplv, ciplv).
    """
    p = _prec_id(prec)
    dev = xs[0].device
    rd = torch.float64 if p == 0 else torch.float32
    cd = torch.complex128 if p == 0 else torch.complex64
    st = _abi.Stft(int(seg), int(hop), int(bins[0]), int(bins[1]), _abi.WINDOW[window], 0)
    nb = int(bins[1]) - int(bins[0]) + 1
    outs, probs = [], []
    for k, x in enumerate(xs):
        if x.dtype != rd:
            raise TypeError("prec %s needs %s input, got %s" % (prec, rd, x.dtype))
        o = _outputs(x.shape[0], nb, rd, cd, dev, want, want_g)
        outs.append(o)
        probs.append(_problem(x, None if windows is None else windows[k], o))
    arr = _abi.problems(probs)
    ctx = context(dev)
    nbytes = C.c_size_t(0)
    _abi.check(_abi.lib().plv_coherence_stft_workspace_size(ctx.handle, p, arr, len(probs), C.byref(st),
                                                            C.byref(nbytes)), ctx.handle)
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=dev)
    _abi.check(_abi.lib().plv_coherence_stft(ctx.handle, p, arr, len(probs), C.byref(st), C.c_void_p(ws.data_ptr()),
                                             ws.numel(), _stream(dev)), ctx.handle)
    names = {"plv": "coh", "iplv": "icoh", "ciplv": "cicoh", "g": "c"}
    return [{names[k]: v for k, v in o.items()} for o in outs]


def coherence_stft(x, seg, hop, bins, window="hamming", prec="split_bf16", span=None, want=ALL, want_g=False):
    """coherence_stft_batch for one problem."""
    return coherence_stft_batch([x], seg, hop, bins, window, prec, None if span is None else [span], want,
                                want_g)[0]


def autotune_batch(xs, prec="split_bf16", fs=None, bands=None, windows=None, coherence=False):
    """Measure the tile edge of every distinct row count of a grouped forward
    call (several problems, or real rows with several bands) through
    plv_autotune, and keep the choices for later calls on this device.

    xs: the call's inputs, as for from_analytic_batch / from_real_batch /
    coherence_batch.  Returns {n: tile edge} for the row counts of xs.
    Blocks until the trial runs finish.
    """
    p = _prec_id(prec)
    dev = xs[0].device
    real = not xs[0].is_complex()
    barr, nb = _abi.bands(bands) if real else (None, 1)
    rd = torch.float64 if p == 0 else torch.float32
    cd = torch.complex128 if p == 0 else torch.complex64
    outs, probs = [], []
    for k, x in enumerate(xs):
        o = _outputs(x.shape[0], nb, rd, cd, dev, ALL, False)
        outs.append(o)
        probs.append(_problem(x, None if windows is None else windows[k], o))
    arr = _abi.problems(probs)
    op = _abi.OP_FROM_REAL if real else (_abi.OP_COHERENCE if coherence else _abi.OP_FROM_ANALYTIC)
    ctx = context(dev)
    ws = _workspace(ctx, op, p, arr, barr, nb, dev)
    _abi.check(_abi.lib().plv_autotune(ctx.handle, op, p, arr, len(probs), barr, nb, float(fs or 0.0),
                                       C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev), None), ctx.handle)
    return {int(x.shape[0]): tile_edge(int(x.shape[0]), prec, dev) for x in xs}


def tile_edge(n, prec="split_bf16", device=None):
    """Tile edge (64 or 128) of a forward problem of n rows on this device."""
    ctx = context(device)
    bm = C.c_int32(0)
    _abi.check(_abi.lib().plv_tile_edge(ctx.handle, _prec_id(prec), int(n), C.byref(bm)), ctx.handle)
    return bm.value


def set_tile_edge(n, bm, prec="split_bf16", device=None):
    """Force the tile edge of forward problems of n rows (bm 64 or 128), or
    return them to the planner's model (bm = 0)."""
    ctx = context(device)
    _abi.check(_abi.lib().plv_set_tile_edge(ctx.handle, _prec_id(prec), int(n), int(bm)), ctx.handle)


def timing_enable(on=True, device=None):
    """Turn per-stage GPU timing (HIP events on the call's stream) on or off."""
    ctx = context(device)
    _abi.check(_abi.lib().plv_timing_enable(ctx.handle, 1 if on else 0), ctx.handle)


def timing_read(reset=True, device=None):
    """{stage: (ms, calls, launches)} summed since the last reset."""
    ctx = context(device)
    t = _abi.Timing()
    _abi.check(_abi.lib().plv_timing_read(ctx.handle, C.byref(t), 1 if reset else 0), ctx.handle)
    return {name: (t.ms[k], t.calls[k], t.launches[k]) for k, name in enumerate(_abi.STAGES)}


def timing_list(stage, device=None):
    """[(ms, launches)] of every recorded execution of `stage` (a name from
    timing_read's keys), in call order, without resetting."""
    ctx = context(device)
    k = _abi.STAGES.index(stage)
    cnt = C.c_int64(0)
    _abi.check(_abi.lib().plv_timing_list(ctx.handle, k, None, None, 0, C.byref(cnt)), ctx.handle)
    n = cnt.value
    ms = (C.c_double * max(n, 1))()
    ln = (C.c_int32 * max(n, 1))()
    _abi.check(_abi.lib().plv_timing_list(ctx.handle, k, ms, ln, n, C.byref(cnt)), ctx.handle)
    return [(ms[i], ln[i]) for i in range(n)]


def backward_batch(xs, gs, upstream, fs=None, bands=None, prec="split_bf16", windows=None):
    """dL/d(input) for each problem through plv_backward.

    xs: the forward inputs (complex analytic or real rows); gs: the forward's
    complex G per problem ([n, n] or [nbands, n, n]); upstream: per problem a
    tuple (dL/dplv, dL/diplv, dL/dciplv), each a tensor shaped like the
    outputs or None.  Returns tensors shaped like xs.
    """
    p = _prec_id(prec)
    dev = xs[0].device
    real = not xs[0].is_complex()
    barr, nb = _abi.bands(bands) if real else (None, 1)
    probs, grads, dins, keep = [], [], [], []
    for k, x in enumerate(xs):
        n, t, ld = _rows(x)
        w = None if windows is None else windows[k]
        t0, t1 = (0, 0) if w is None else (int(w[0]), int(w[1]))
        g = gs[k].contiguous()
        ups = [None if u is None else u.contiguous() for u in upstream[k]]
        # same layout and row stride as the input (the ABI writes din with in's ld)
        din = torch.empty_strided(x.size(), x.stride(), dtype=x.dtype, device=x.device)
        keep += [g, din] + ups
        probs.append(_abi.Problem(n, t, ld, t0, t1, x.data_ptr(), None, None, None, g.data_ptr()))
        grads.append(_abi.Grad(*(_ptr(u) for u in ups), din.data_ptr()))
        dins.append(din)
    arr = _abi.problems(probs)
    garr = (_abi.Grad * len(grads))(*grads)
    ctx = context(dev)
    op = _abi.OP_BACKWARD_REAL if real else _abi.OP_BACKWARD_ANALYTIC
    ws = _workspace(ctx, op, p, arr, barr, nb, dev)
    kind = _abi.INPUT_REAL if real else _abi.INPUT_ANALYTIC
    _abi.check(_abi.lib().plv_backward(ctx.handle, p, kind, arr, garr, len(probs), barr, nb,
                                       float(fs or 0.0), C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)),
               ctx.handle)
    return dins


class PLVFunction(torch.autograd.Function):
    """(plv, iplv, ciplv) of one problem with the library's adjoint as backward.

    Analytic (complex) input gives [n, n] outputs; real input gives
    [nbands, n, n] (one plain band when `bands` is None)."""

    @staticmethod
    def forward(ctx, x, fs, bands, prec, window):
        if x.is_complex():
            out = from_analytic(x, prec=prec, window=window, want_g=True)
        else:
            out = from_real(x, fs, bands=bands, prec=prec, window=window, want_g=True)
        ctx.save_for_backward(x, out["g"])
        ctx.cfg = (fs, bands, prec, window)
        return out["plv"], out["iplv"], out["ciplv"]

    @staticmethod
    def backward(ctx, gp, gi, gc):
        x, g = ctx.saved_tensors
        fs, bands, prec, window = ctx.cfg
        din = backward_batch([x], [g], [(gp, gi, gc)], fs=fs, bands=bands, prec=prec,
                             windows=None if window is None else [window])[0]
        return din, None, None, None, None


def plv_metrics(x, fs=None, bands=None, prec="split_bf16", window=None):
    """Differentiable (plv, iplv, ciplv) of x (complex analytic or real rows)."""
    return PLVFunction.apply(x, fs, bands, prec, window)
