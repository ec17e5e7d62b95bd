"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU reference for the PLV hot path, used by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``, and by
nothing else.  It shares no code with the HIP library: the arithmetic lives in
``plv_oracle.c`` (built with gcc, no fast-math) and this module only marshals
numpy arrays.

What is computed, and where it comes from in the paper (Bruna, Maestu, Pereda,
"Phase Locking Value revisited"):

* ``analytic``      Eq. 3: the (band-pass) analytic signal, as the DFT-domain
                    construction with one-sided weights, by plain DFT sums; the
                    band-pass a DFT-bin mask or a forward-backward FIR
                    (``fir_taps``, ``fir_power``: the build's own design, since
                    the paper names an FIR without giving it).
* ``phase``         Eq. 3 / Appendix, first listing: angle of z (0 at z = 0).
* ``pair_means``    Eq. 2 per pair, the original formulation: the mean over
                    samples of exp(i * phase difference).
* ``metrics``       PLV = |G| (Eq. 2), iPLV = |Im G| (Eq. 13) and
                    ciPLV = |Im G| / sqrt(1 - Re^2) (Eq. 14).
* ``full_*``        all pairs assembled into N x N matrices (mirror, diagonal
                    PLV = 1, iPLV = ciPLV = 0), as the Appendix's matrix forms
                    return them.
* ``grad_*``        gradient of a loss on the metrics, in angle space (not in
                    the paper; it checks the library's adjoint).
* ``coherency``     Section II.B, Eq. 12: amplitude-weighted cross sums over the
                    rows' powers (coherence = |C|); ``full_coherence``.
* ``full_over_trials`` Eq. 1 (matrix form Eq. 8): Lachaux's PLV(t), the mean
                    over trials at each time point.
* ``stft_bins``     Section II.B, Eq. 12's X_i(f, n): DFT bins of windowed
                    segments (``window``: symmetric Hamming, Hann or
                    rectangular), by plain DFT sums; ``full_coherence_stft``
                    the coherency over segments at each bin.

Readings of the paper that the oracle takes (orientation of G, absolute
iPLV/ciPLV, the 1/T normaliser, the z = 0 rule, the ciPLV radicand) are listed
in the repository's design notes.  Every function here is pinned by the
``-m "not gpu"`` tests to closed forms, library routines or brute force.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plv_oracle.c")
_SO = os.path.join(_HERE, "_plv_oracle.so")
_LIB = None
_LOCK = threading.Lock()

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle's C source into ``oracle/_plv_oracle.so`` with gcc."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_SO)
            L.oracle_mask_plain.argtypes = [C.c_int64, _D]
            L.oracle_mask_band.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, _D]
            L.oracle_fir_taps.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, _D]
            L.oracle_fir_taps.restype = C.c_int
            L.oracle_fir_power.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int64, _D]
            L.oracle_fir_power.restype = C.c_int
            L.oracle_mask_fir.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int64, _D]
            L.oracle_mask_fir.restype = C.c_int
            L.oracle_spectral_filter.argtypes = [_D, _D, C.c_int64, C.c_int64, C.c_int64, _D, _D, _D,
                                                 C.c_int64, C.c_int]
            L.oracle_spectral_filter.restype = C.c_int
            L.oracle_phase.argtypes = [_D, _D, C.c_int64, _D]
            L.oracle_pair_means.argtypes = [_D, C.c_int64, C.c_int64, _I, _I, C.c_int64, _D, _D, C.c_int]
            L.oracle_metrics.argtypes = [_D, _D, C.c_int64, _D, _D, _D]
            L.oracle_coherency.argtypes = [_D, _D, C.c_int64, C.c_int64, _I, _I, C.c_int64, _D, _D, C.c_int]
            L.oracle_metric_adjoint.argtypes = [_D, _D, _D, _D, _D, C.c_int64, _D, _D]
            L.oracle_phase_grad.argtypes = [_D, C.c_int64, C.c_int64, C.c_int64, _D, _D, _D, C.c_int64,
                                            C.c_int]
            L.oracle_phase_to_z.argtypes = [_D, _D, _D, C.c_int64, _D, _D]
            L.oracle_phase_grad_rows.argtypes = [_D, C.c_int64, C.c_int64, C.c_int64, _D, _D, _I, C.c_int64, _D,
                                                 C.c_int64, C.c_int]
            _LIB = L
    return _LIB


def threads() -> int:
    """Host threads the oracle uses: the cores this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# spectral weights and the analytic signal (Eq. 3)
# --------------------------------------------------------------------------

def mask_plain(t: int) -> np.ndarray:
    h = np.empty(int(t), dtype=np.float64)
    lib().oracle_mask_plain(int(t), _p(h))
    return h


def mask_band(t: int, fs: float, flo: float, fhi: float) -> np.ndarray:
    h = np.empty(int(t), dtype=np.float64)
    lib().oracle_mask_band(int(t), float(fs), float(flo), float(fhi), _p(h))
    return h


def fir_taps(order: int, fs: float, flo: float, fhi: float) -> np.ndarray:
    """Taps of the band-pass FIR (even order L, L + 1 taps): windowed ideal
    band-pass, Hamming window, unit gain at the band centre."""
    h = np.empty(int(order) + 1, dtype=np.float64)
    if lib().oracle_fir_taps(int(order), float(fs), float(flo), float(fhi), _p(h)):
        raise ValueError("FIR order must be even and positive")
    return h


def fir_power(t: int, fs: float, flo: float, fhi: float, order: int) -> np.ndarray:
    """|H|^2 on the T-point DFT grid: the gain of forward-backward filtering."""
    p = np.empty(int(t), dtype=np.float64)
    if lib().oracle_fir_power(int(t), float(fs), float(flo), float(fhi), int(order), _p(p)):
        raise ValueError("FIR order must be even and positive")
    return p


def mask_fir(t: int, fs: float, flo: float, fhi: float, order: int) -> np.ndarray:
    h = np.empty(int(t), dtype=np.float64)
    if lib().oracle_mask_fir(int(t), float(fs), float(flo), float(fhi), int(order), _p(h)):
        raise ValueError("FIR order must be even and positive")
    return h


def mask(t: int, fs: float | None, band) -> np.ndarray:
    """Spectrum weights of the analytic signal: plain (band None), a DFT-bin
    band (flo, fhi), or a forward-backward FIR band (flo, fhi, order)."""
    if band is None:
        return mask_plain(t)
    if len(band) > 2 and band[2]:
        return mask_fir(t, fs, band[0], band[1], int(band[2]))
    return mask_band(t, fs, band[0], band[1])


def fir_zero_phase(x: np.ndarray, fs: float, band) -> np.ndarray:
    """The real rows after forward-backward FIR filtering, as the DFT-domain
    product with |H|^2 (circular over the row)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return spectral_filter(x, fir_power(x.shape[1], fs, band[0], band[1], int(band[2]))).real


def spectral_filter(x: np.ndarray, h: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """IDFT(h .* DFT(x)) for every row of x (real or complex), by plain DFT sums."""
    x = np.atleast_2d(x)
    n, t = x.shape
    h = _f64(h)
    assert h.shape == (t,)
    if np.iscomplexobj(x):
        xr, xi = _f64(x.real), _f64(x.imag)
        pxi = _p(xi)
    else:
        xr, xi = _f64(x), None
        pxi = None
    zr = np.empty((n, t), dtype=np.float64)
    zi = np.empty((n, t), dtype=np.float64)
    rc = lib().oracle_spectral_filter(_p(xr), pxi, t, n, t, _p(h), _p(zr), _p(zi), t,
                                      int(nthreads or threads()))
    if rc:
        raise MemoryError("oracle_spectral_filter failed")
    return zr + 1j * zi


def analytic(x: np.ndarray, fs: float | None = None, band=None, nthreads=None) -> np.ndarray:
    """Analytic signal of each real row: plain one-sided weights, the
    band-pass weights of ``band = (flo, fhi)`` in Hz (needs ``fs``), or the
    forward-backward FIR of ``band = (flo, fhi, order)``."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    t = x.shape[1]
    h = mask(t, fs, band)
    return spectral_filter(x, h, nthreads)


def analytic_fft(x: np.ndarray, fs: float | None = None, band=None) -> np.ndarray:
    """The same analytic signal as ``analytic`` with numpy's FFT as the DFT
    (a library primitive; pinned against the plain-DFT sums), for rows too
    long or too many for O(T^2) sums."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    t = x.shape[1]
    h = mask(t, fs, band)
    return np.fft.ifft(h * np.fft.fft(x, axis=-1), axis=-1)


# --------------------------------------------------------------------------
# phase, per-pair means (Eq. 2) and metrics (Eqs. 13, 14)
# --------------------------------------------------------------------------

def phase(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z)
    zr, zi = _f64(z.real), _f64(z.imag)
    phi = np.empty(zr.shape, dtype=np.float64)
    lib().oracle_phase(_p(zr), _p(zi), zr.size, _p(phi))
    return phi


def pair_means(phi: np.ndarray, pairs: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """G_p = (1/T) sum_t exp(i(phi_a(t) - phi_b(t))) for (a, b) = pairs[p]."""
    phi = _f64(phi)
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    n, t = phi.shape
    assert pairs.size == 0 or (pairs.min() >= 0 and pairs.max() < n)
    gre = np.empty(len(pairs))
    gim = np.empty(len(pairs))
    lib().oracle_pair_means(_p(phi), t, t, pi.ctypes.data_as(_I), pj.ctypes.data_as(_I), len(pairs),
                            _p(gre), _p(gim), int(nthreads or threads()))
    return gre + 1j * gim


def coherency(z: np.ndarray, pairs: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """Complex coherency C_p = sum_t z_a conj(z_b) / sqrt(sum|z_a|^2 sum|z_b|^2)
    for (a, b) = pairs[p] (Section II.B, Eq. 12; 0 where a row is all zero).
    Coherence is |C|; imaginary and corrected imaginary coherency are
    metrics(C)[1:] (the iPLV / ciPLV forms)."""
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    zr = np.ascontiguousarray(z.real)
    zi = np.ascontiguousarray(z.imag)
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    n, t = z.shape
    assert pairs.size == 0 or (pairs.min() >= 0 and pairs.max() < n)
    cre = np.empty(len(pairs))
    cim = np.empty(len(pairs))
    lib().oracle_coherency(_p(zr), _p(zi), t, t, pi.ctypes.data_as(_I), pj.ctypes.data_as(_I), len(pairs),
                           _p(cre), _p(cim), int(nthreads or threads()))
    return cre + 1j * cim


def full_coherence(z: np.ndarray, nthreads=None) -> dict:
    """Every pair of rows of z: {'coh', 'icoh', 'cicoh' [n, n] and 'c' [n, n]
    complex coherency}, with coherence 1 and the others 0 on the diagonal."""
    n = z.shape[0]
    pr = upper_pairs(n)
    c = coherency(z, pr, nthreads)
    coh, icoh, cicoh = metrics(c)
    out = {k: np.zeros((n, n)) for k in ("coh", "icoh", "cicoh")}
    cc = np.zeros((n, n), dtype=np.complex128)
    a, b = pr[:, 0], pr[:, 1]
    for k, v in (("coh", coh), ("icoh", icoh), ("cicoh", cicoh)):
        out[k][a, b] = v
        out[k][b, a] = v
    cc[a, b] = c
    cc[b, a] = np.conj(c)
    d = np.arange(n)
    out["coh"][d, d] = 1.0
    cc[d, d] = coherency(z, np.stack([d, d], 1), nthreads)
    out["c"] = cc
    return out


WINDOWS = ("hamming", "hann", "rect")


def window(name: str, seg: int) -> np.ndarray:
    """Segment window of length seg, symmetric (the last sample repeats the
    first): Hamming 0.54 - 0.46 cos(2 pi m / (seg - 1)), Hann
    0.5 - 0.5 cos(2 pi m / (seg - 1)), or rectangular (all 1).  The paper's
    coherence segments are Hamming-windowed (Section III.B, Figure 2)."""
    m = np.arange(seg, dtype=np.float64)
    if name == "rect" or seg == 1:
        return np.ones(seg)
    c = np.cos(2.0 * np.pi * m / (seg - 1))
    if name == "hamming":
        return 0.54 - 0.46 * c
    if name == "hann":
        return 0.5 - 0.5 * c
    raise ValueError("window must be one of %s" % (WINDOWS,))


def stft_bins(x: np.ndarray, seg: int, hop: int, k_lo: int, k_hi: int, win: str = "hamming",
              span=None) -> np.ndarray:
    """Fourier coefficients of windowed segments, the X_i(f, n) of Section
    II.B, Eq. 12: segment n of row i covers samples s0 + n*hop + m,
    m = 0..seg-1, of the span [s0, s1) (the whole row by default), and
        X_i(k, n) = sum_m w[m] x_i(s0 + n*hop + m) exp(-2 pi i (k m mod seg) / seg)
    for the DFT bins k = k_lo..k_hi of the segment length; the number of
    segments is floor((s1 - s0 - seg) / hop) + 1.  A plain DFT (a matrix
    product with the twiddle matrix), FP64.  Returns [k_hi - k_lo + 1][n][S]."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[None]
    s0, s1 = (0, x.shape[1]) if span is None else (int(span[0]), int(span[1]))
    nseg = (s1 - s0 - seg) // hop + 1
    assert nseg >= 1 and 0 <= k_lo <= k_hi
    w = window(win, seg)
    idx = s0 + np.arange(nseg)[:, None] * hop + np.arange(seg)[None, :]   # [S][seg]
    segs = x[:, idx] * w[None, None, :]                                    # [n][S][seg]
    k = np.arange(k_lo, k_hi + 1)
    m = np.arange(seg)
    tw = np.exp(-2j * np.pi * ((k[:, None] * m[None, :]) % seg) / seg)     # [nbins][seg]
    return np.einsum("nsm,km->kns", segs, tw)


def full_coherence_stft(x: np.ndarray, seg: int, hop: int, k_lo: int, k_hi: int, win: str = "hamming",
                        span=None, nthreads=None) -> list:
    """Coherency between every pair of rows at each bin k_lo..k_hi over the
    windowed segments (Eq. 12 with n running over segments): one
    full_coherence dict per bin."""
    z = stft_bins(x, seg, hop, k_lo, k_hi, win, span)
    return [full_coherence(zk, nthreads) for zk in z]


def metrics(g: np.ndarray):
    """(plv, iplv, ciplv) from complex G values, element-wise."""
    g = np.asarray(g)
    gr, gi = _f64(g.real), _f64(g.imag)
    p = np.empty(gr.shape)
    i_ = np.empty(gr.shape)
    c = np.empty(gr.shape)
    lib().oracle_metrics(_p(gr), _p(gi), gr.size, _p(p), _p(i_), _p(c))
    return p, i_, c


def upper_pairs(n: int) -> np.ndarray:
    iu, ju = np.triu_indices(n, k=1)
    return np.stack([iu, ju], axis=1).astype(np.int64)


def full_from_phase(phi: np.ndarray, nthreads=None) -> dict:
    """All pairs of [N, T] phases assembled into N x N matrices.

    G_ij for i < j from Eq. 2, G_ji = conj(G_ij), G_ii = 1; PLV, iPLV and ciPLV
    symmetric with diagonal 1, 0, 0.
    """
    n = phi.shape[0]
    pr = upper_pairs(n)
    g = pair_means(phi, pr, nthreads)
    p, i_, c = metrics(g)
    G = np.eye(n, dtype=np.complex128)
    P = np.eye(n)
    I = np.zeros((n, n))
    Cc = np.zeros((n, n))
    a, b = pr[:, 0], pr[:, 1]
    G[a, b] = g
    G[b, a] = np.conj(g)
    for M, v in ((P, p), (I, i_), (Cc, c)):
        M[a, b] = v
        M[b, a] = v
    return {"g": G, "plv": P, "iplv": I, "ciplv": Cc}


def full_over_trials(z: np.ndarray, window=None, nthreads=None) -> dict:
    """Lachaux's time-resolved PLV across trials (Eq. 1): z is [ntr, N, T]
    analytic signals; for each time point t in the window, every pair's mean
    over the trials n of exp(i(phi_i(t, n) - phi_j(t, n))), assembled like
    full_from_phase.  Returns [T', N, N] arrays."""
    z = np.asarray(z)
    t0, t1 = (0, z.shape[2]) if window is None else window
    outs = []
    for t in range(t0, t1):
        phi = phase(np.ascontiguousarray(z[:, :, t].T))   # [N, ntr]: trials are the samples
        outs.append(full_from_phase(phi, nthreads))
    return {k: np.stack([o[k] for o in outs]) for k in outs[0]}


def full_from_analytic(z: np.ndarray, window=None, nthreads=None) -> dict:
    z = np.atleast_2d(z)
    if window is not None:
        z = z[:, window[0]:window[1]]
    return full_from_phase(phase(z), nthreads)


def full_from_real(x: np.ndarray, fs: float | None = None, band=None, window=None, nthreads=None) -> dict:
    return full_from_analytic(analytic(x, fs, band, nthreads), window, nthreads)


def pairs_from_analytic(z: np.ndarray, pairs: np.ndarray, window=None, nthreads=None) -> np.ndarray:
    """G for selected pairs only (rows are independent, so only the rows the
    pairs touch are needed)."""
    z = np.atleast_2d(z)
    if window is not None:
        z = z[:, window[0]:window[1]]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    rows, inv = np.unique(pairs.reshape(-1), return_inverse=True)
    phi = phase(np.asarray(z[rows]))
    return pair_means(phi, inv.reshape(-1, 2), nthreads)


# --------------------------------------------------------------------------
# gradient (angle space)
# --------------------------------------------------------------------------

def _pair_upstream(gp, gi, gc, n):
    """Combine dL/d(output) given as full N x N matrices over (i, j) and (j, i);
    the diagonal is ignored.  Returns upper-triangle arrays (zero elsewhere)."""
    out = []
    mask = np.triu(np.ones((n, n), dtype=bool), k=1)
    for gmat in (gp, gi, gc):
        if gmat is None:
            out.append(None)
            continue
        gmat = _f64(gmat).reshape(n, n)
        s = gmat + gmat.T
        out.append(np.where(mask, s, 0.0))
    return out


def grad_phase(phi: np.ndarray, gp=None, gi=None, gc=None, g_full=None, nthreads=None) -> np.ndarray:
    """dL/dphi [N, T] for upstream gradients on the N x N metric matrices."""
    phi = _f64(phi)
    n, t = phi.shape
    G = g_full if g_full is not None else full_from_phase(phi, nthreads)["g"]
    upp, upi, upc = _pair_upstream(gp, gi, gc, n)
    gr, gim = _f64(G.real), _f64(G.imag)
    dre = np.zeros((n, n))
    dim = np.zeros((n, n))
    z = np.zeros((n, n))
    lib().oracle_metric_adjoint(_p(gr), _p(gim), _p(upp if upp is not None else z),
                                _p(upi if upi is not None else z), _p(upc if upc is not None else z),
                                n * n, _p(dre), _p(dim))
    dphi = np.empty((n, t))
    lib().oracle_phase_grad(_p(phi), t, n, t, _p(dre), _p(dim), _p(dphi), t, int(nthreads or threads()))
    return dphi


def grad_from_analytic(z: np.ndarray, gp=None, gi=None, gc=None, window=None, nthreads=None) -> np.ndarray:
    """dL/dRe z + i dL/dIm z, [N, T]."""
    z = np.atleast_2d(np.asarray(z, dtype=np.complex128))
    n, t = z.shape
    w0, w1 = (0, t) if window is None else window
    zw = np.ascontiguousarray(z[:, w0:w1])
    dphi = grad_phase(phase(zw), gp, gi, gc, nthreads=nthreads)
    zr, zi = _f64(zw.real), _f64(zw.imag)
    dzr = np.empty(zr.shape)
    dzi = np.empty(zr.shape)
    lib().oracle_phase_to_z(_p(zr), _p(zi), _p(dphi), zr.size, _p(dzr), _p(dzi))
    out = np.zeros((n, t), dtype=np.complex128)
    out[:, w0:w1] = dzr + 1j * dzi
    return out


def grad_from_real(x: np.ndarray, fs=None, band=None, gp=None, gi=None, gc=None, window=None,
                   nthreads=None) -> np.ndarray:
    """dL/dx [N, T] through the analytic-signal map z = M x.

    M = IDFT diag(h) DFT is Hermitian for real h, so dL/dx = Re(M zbar) with
    zbar = dL/dRe z + i dL/dIm z.
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    t = x.shape[1]
    h = mask(t, fs, band)
    z = spectral_filter(x, h, nthreads)
    zbar = grad_from_analytic(z, gp, gi, gc, window, nthreads)
    return spectral_filter(zbar, h, nthreads).real


def grad_from_real_rows(x: np.ndarray, rows, fs=None, band=None, gp=None, gi=None, gc=None, window=None,
                        nthreads=None) -> np.ndarray:
    """dL/dx for the listed rows only, [len(rows), T], same chain as
    ``grad_from_real``.  The analytic signal of every row comes from
    ``analytic_fft``; the pair sums run only over pairs that touch the rows."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n, t = x.shape
    rows = np.asarray(rows, dtype=np.int64)
    w0, w1 = (0, t) if window is None else window
    z = analytic_fft(x, fs, band)
    zw = np.ascontiguousarray(z[:, w0:w1])
    tw = w1 - w0
    phi = phase(zw)
    # G and the metric adjoint for every pair that touches a listed row
    sel = np.zeros(n, dtype=bool)
    sel[rows] = True
    a_idx, b_idx = np.triu_indices(n, 1)
    keep = sel[a_idx] | sel[b_idx]
    pr = np.stack([a_idx[keep], b_idx[keep]], 1)
    g = pair_means(phi, pr, nthreads)
    upp, upi, upc = _pair_upstream(gp, gi, gc, n)
    dre = np.zeros((n, n))
    dim = np.zeros((n, n))
    zz = np.zeros(len(pr))
    gr_, gi_ = _f64(g.real), _f64(g.imag)
    vals = [(_f64(u[pr[:, 0], pr[:, 1]]) if u is not None else zz) for u in (upp, upi, upc)]
    ore = np.empty(len(pr))
    oim = np.empty(len(pr))
    lib().oracle_metric_adjoint(_p(gr_), _p(gi_), _p(vals[0]), _p(vals[1]), _p(vals[2]), len(pr), _p(ore),
                                _p(oim))
    dre[pr[:, 0], pr[:, 1]] = ore
    dim[pr[:, 0], pr[:, 1]] = oim
    dphi = np.empty((len(rows), tw))
    lib().oracle_phase_grad_rows(_p(phi), tw, n, tw, _p(dre), _p(dim), rows.ctypes.data_as(_I), len(rows), _p(dphi),
                                 tw, int(nthreads or threads()))
    zr, zi = _f64(zw[rows].real), _f64(zw[rows].imag)
    dzr = np.empty(zr.shape)
    dzi = np.empty(zr.shape)
    lib().oracle_phase_to_z(_p(zr), _p(zi), _p(dphi), zr.size, _p(dzr), _p(dzi))
    zbar = np.zeros((len(rows), t), dtype=np.complex128)
    zbar[:, w0:w1] = dzr + 1j * dzi
    h = mask(t, fs, band)
    return spectral_filter(zbar, h, nthreads).real
