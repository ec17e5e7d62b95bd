// fft.hip -- analytic signal of real rows by FFT (Section II.A, Eq. 3), fused
// with the window, the phasor normalisation (Eq. 4) and the store of the
// Gram kernel's phasor planes.
//
// For a row x of length t and each band b:
//   X = DFT_t(x);  z_b = IDFT_t(h_b .* X);  u_b(s) = z_b(t0 + s) / |z_b(t0 + s)|
// with h the one-sided weights of the discrete analytic signal (1 at DC, 2
// below Nyquist, 1 at Nyquist for even t, 0 above) or a band mask (2 on the
// positive-frequency bins [klo, khi], 0 elsewhere).  The transforms run at the
// exact length t: radix-2 when t is a power of two, otherwise Bluestein's
// chirp-z form, DFT_t(x)_k = conj(c_k) * (a (*) b)_k with c_m = exp(i pi m^2/t),
// a = x .* conj(c) zero-padded to M >= 2t - 1 and b the circular chirp, the
// circular convolution taken by length-M FFTs with FFT_M(b) precomputed once
// per length.  The inverse uses IDFT(Y) = conj(DFT(conj(Y))) / t.
//
// One work-group per row at a time (grid-stride over the rows of one FFT
// size): the row's spectrum X and a work buffer live in LDS with the twiddle
// table.  Forward transforms are decimation-in-time from a bit-reversed load
// (natural-order output); inverse transforms are decimation-in-frequency
// (natural-order input, bit-reversed output), so no permutation passes are
// needed between them.  Chirp angles are reduced exactly in integers
// (m^2 mod 2t) and evaluated in FP64.
#include "phasor.h"

namespace plv {
namespace {

template <class R>
struct cx {
    R x, y;
};
template <class R>
__device__ inline cx<R> cmul(cx<R> a, cx<R> b)
{
    return cx<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ inline cx<R> cconj(cx<R> a)
{
    return cx<R>{a.x, -a.y};
}
template <class R>
__device__ inline cx<R> cadd(cx<R> a, cx<R> b)
{
    return cx<R>{a.x + b.x, a.y + b.y};
}
template <class R>
__device__ inline cx<R> csub(cx<R> a, cx<R> b)
{
    return cx<R>{a.x - b.x, a.y - b.y};
}
template <class R>
__device__ inline cx<R> cscale(cx<R> a, R s)
{
    return cx<R>{a.x * s, a.y * s};
}

__device__ inline int brev(int n, int logm) { return (int)(__brev((unsigned)n) >> (32 - logm)); }

constexpr int NT = 256;  // threads per work-group

// In-place radix-2 DIT, forward (exp(-)), bit-reversed input -> natural output.
template <class R>
__device__ void fft_dit(cx<R> *W, const cx<R> *TW, int logm)
{
    const int M = 1 << logm;
    for (int s = 1; s <= logm; ++s) {
        const int h = 1 << (s - 1), ts = M >> s;
        for (int b = threadIdx.x; b < M / 2; b += NT) {
            const int j = b & (h - 1);
            const int i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + h;
            const cx<R> u = W[i0], v = cmul(W[i1], TW[j * ts]);
            W[i0] = cadd(u, v);
            W[i1] = csub(u, v);
        }
        __syncthreads();
    }
}

// In-place radix-2 DIF, inverse (exp(+)), natural input -> bit-reversed
// output, unscaled.
template <class R>
__device__ void ifft_dif(cx<R> *W, const cx<R> *TW, int logm)
{
    const int M = 1 << logm;
    for (int s = logm; s >= 1; --s) {
        const int h = 1 << (s - 1), ts = M >> s;
        for (int b = threadIdx.x; b < M / 2; b += NT) {
            const int j = b & (h - 1);
            const int i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + h;
            const cx<R> u = W[i0], v = W[i1];
            W[i0] = cadd(u, v);
            W[i1] = cmul(csub(u, v), cconj(TW[j * ts]));
        }
        __syncthreads();
    }
}

// TW[k] = exp(-2 pi i k / M), k < M/2, evaluated in FP64.
template <class R>
__global__ __launch_bounds__(NT) void twiddle_kernel(cx<R> *tab, int logm)
{
    const int M = 1 << logm;
    for (int k = blockIdx.x * NT + threadIdx.x; k < M / 2; k += gridDim.x * NT) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)M, &sn, &cs);
        tab[k] = cx<R>{(R)cs, (R)sn};
    }
}

// Chirp c_m = exp(i pi m^2 / t) for m < t and the circular chirp b of length
// M: b_m = c_m (m < t), b_{M-m} = c_m (0 < m < t), 0 elsewhere; then
// FFT_M(b) in place.  One work-group per job.
template <class R, int MAXLOG>
__global__ __launch_bounds__(NT) void chirp_kernel(const ChirpJob *jobs)
{
    __shared__ cx<R> W[1 << MAXLOG];
    __shared__ cx<R> TW[(1 << MAXLOG) / 2];
    const ChirpJob jb = jobs[blockIdx.x];
    const int t = jb.t, logm = jb.logm, M = 1 << logm;
    cx<R> *chirp = (cx<R> *)jb.chirp, *bh = (cx<R> *)jb.bhat;
    for (int k = threadIdx.x; k < M / 2; k += NT) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)M, &sn, &cs);
        TW[k] = cx<R>{(R)cs, (R)sn};
    }
    for (int m = threadIdx.x; m < M; m += NT) {
        const int src = m < t ? m : (M - m < t ? M - m : -1);
        cx<R> v{0, 0};
        if (src >= 0) {
            const int64_t r = ((int64_t)src * src) % (2 * (int64_t)t);  // m^2 mod 2t, exact
            double sn, cs;
            sincospi((double)r / (double)t, &sn, &cs);
            v = cx<R>{(R)cs, (R)sn};
            if (m < t)
                chirp[m] = v;
        }
        W[brev(m, logm)] = v;
    }
    __syncthreads();
    fft_dit(W, TW, logm);
    for (int k = threadIdx.x; k < M; k += NT)
        bh[k] = W[k];
}

template <int MODE>
__global__ __launch_bounds__(NT) void hilbert_kernel(HilbertArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type R;
    constexpr int MAXLOG = MODE == M_F64 ? FFT_MAXLOG_F64 : FFT_MAXLOG_F32;
    __shared__ cx<R> X[1 << MAXLOG];   // spectrum of the current row
    __shared__ cx<R> W[1 << MAXLOG];   // work buffer
    __shared__ cx<R> TW[(1 << MAXLOG) / 2];

    const int logm = a.logm, M = 1 << logm;
    bool tw_loaded = false;
    for (int ri = blockIdx.x; ri < a.nrows; ri += gridDim.x) {
        const RowRef rr = a.rows[ri];
        const HilbertProb hp = a.hp[rr.prob];
        if (!tw_loaded) {
            const cx<R> *tg = (const cx<R> *)hp.tw_tab;
            for (int k = threadIdx.x; k < M / 2; k += NT)
                TW[k] = tg[k];
            tw_loaded = true;
        }
        const int t = hp.t;
        const R *x = (const R *)hp.x + (int64_t)rr.row * hp.ld;
        const cx<R> *ch = (const cx<R> *)hp.chirp;
        const cx<R> *bh = (const cx<R> *)hp.bhat;
        __syncthreads();  // TW visible; previous row done with X and W

        // ---- X = DFT_t(x), natural order, k < t
        if (!hp.blue) {
            for (int n = threadIdx.x; n < M; n += NT)
                W[brev(n, logm)] = cx<R>{x[n], (R)0};
            __syncthreads();
            fft_dit(W, TW, logm);
            for (int k = threadIdx.x; k < M; k += NT)
                X[k] = W[k];
        } else {
            for (int n = threadIdx.x; n < M; n += NT) {
                cx<R> v{0, 0};
                if (n < t)
                    v = cscale(cconj(ch[n]), x[n]);
                W[brev(n, logm)] = v;
            }
            __syncthreads();
            fft_dit(W, TW, logm);
            for (int k = threadIdx.x; k < M; k += NT)
                W[k] = cmul(W[k], bh[k]);
            __syncthreads();
            ifft_dif(W, TW, logm);
            const R invm = (R)1 / (R)M;
            for (int k = threadIdx.x; k < t; k += NT)
                X[k] = cscale(cmul(cconj(ch[k]), W[brev(k, logm)]), invm);
        }
        __syncthreads();

        // ---- each band: z = IDFT_t(h .* X), window, normalise, store planes
        for (int b = 0; b < hp.nbands; ++b) {
            const BandBins bb = a.bins[hp.bin0 + b];
            auto weight = [&](int k) -> R {
                if (bb.klo < 0)
                    return k == 0 ? (R)1 : (2 * k < t ? (R)2 : (2 * k == t ? (R)1 : (R)0));
                return (k >= bb.klo && k <= bb.khi) ? (R)2 : (R)0;
            };
            R zscale;
            if (!hp.blue) {
                for (int k = threadIdx.x; k < M; k += NT)
                    W[k] = cscale(X[k], weight(k));
                __syncthreads();
                ifft_dif(W, TW, logm);  // z_n = W[brev(n)] / t
                zscale = (R)1 / (R)t;
            } else {
                // v = conj(Y) with Y = h .* X; Bluestein DFT of v; z = conj(DFT(v)) / t
                for (int n = threadIdx.x; n < M; n += NT) {
                    cx<R> v{0, 0};
                    if (n < t)
                        v = cconj(cmul(cscale(X[n], weight(n)), ch[n]));
                    W[brev(n, logm)] = v;
                }
                __syncthreads();
                fft_dit(W, TW, logm);
                for (int k = threadIdx.x; k < M; k += NT)
                    W[k] = cmul(W[k], bh[k]);
                __syncthreads();
                ifft_dif(W, TW, logm);  // z_n = c_n conj(W[brev(n)]) / (M t)
                zscale = (R)1 / ((R)M * (R)t);
            }
            const GramDesc g = a.gd[hp.gram0 + b];
            if (g.zbuf) {
                // backward: keep the analytic signal itself on the window
                cx<R> *zr = (cx<R> *)g.zbuf + (int64_t)rr.row * g.ldz;
                for (int s = threadIdx.x; s < hp.tw; s += NT) {
                    const int n = hp.t0 + s;
                    cx<R> z = W[brev(n, logm)];
                    if (hp.blue)
                        z = cmul(ch[n], cconj(z));
                    zr[s] = cscale(z, zscale);
                }
                __syncthreads();
                continue;
            }
            uint8_t *urow = (uint8_t *)g.u + (int64_t)rr.row * g.ldu * cbytes_of(MODE);
            for (int s0 = threadIdx.x * 4; s0 < g.tpad; s0 += NT * 4) {
                R ur[4], ui[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = s0 + v;
                    ur[v] = 0;
                    ui[v] = 0;
                    if (s < hp.tw) {
                        const int n = hp.t0 + s;
                        cx<R> z = W[brev(n, logm)];
                        if (hp.blue)
                            z = cmul(ch[n], cconj(z));
                        unit_phasor(z.x * zscale, z.y * zscale, ur[v], ui[v]);
                    }
                }
                store4<MODE>(urow + (int64_t)s0 * cbytes_of(MODE), g.plane_bytes, ur, ui);
            }
            __syncthreads();  // W is rewritten by the next band
        }
    }
}

// dL/dx of one row: z_b = M_b x with M_b = IDFT diag(h_b) DFT Hermitian
// (h_b real), so dL/dx = Re(sum_b M_b zbar_b) = Re(IDFT(sum_b h_b .*
// DFT(zbar_b))), zbar_b being 0 outside the window.
template <class R, int MAXLOG>
__global__ __launch_bounds__(NT) void hilbert_adjoint_kernel(HilbertArgs a)
{
    __shared__ cx<R> X[1 << MAXLOG];   // sum over bands of h_b .* DFT(zbar_b)
    __shared__ cx<R> W[1 << MAXLOG];
    __shared__ cx<R> TW[(1 << MAXLOG) / 2];
    const int logm = a.logm, M = 1 << logm;
    bool tw_loaded = false;
    for (int ri = blockIdx.x; ri < a.nrows; ri += gridDim.x) {
        const RowRef rr = a.rows[ri];
        const HilbertProb hp = a.hp[rr.prob];
        if (!tw_loaded) {
            const cx<R> *tg = (const cx<R> *)hp.tw_tab;
            for (int k = threadIdx.x; k < M / 2; k += NT)
                TW[k] = tg[k];
            tw_loaded = true;
        }
        const int t = hp.t;
        const cx<R> *ch = (const cx<R> *)hp.chirp;
        const cx<R> *bh = (const cx<R> *)hp.bhat;
        for (int k = threadIdx.x; k < M; k += NT)
            X[k] = cx<R>{0, 0};
        __syncthreads();
        for (int b = 0; b < hp.nbands; ++b) {
            const BandBins bb = a.bins[hp.bin0 + b];
            auto weight = [&](int k) -> R {
                if (bb.klo < 0)
                    return k == 0 ? (R)1 : (2 * k < t ? (R)2 : (2 * k == t ? (R)1 : (R)0));
                return (k >= bb.klo && k <= bb.khi) ? (R)2 : (R)0;
            };
            const GramDesc g = a.gd[hp.gram0 + b];
            const cx<R> *zb = (const cx<R> *)g.zbuf + (int64_t)rr.row * g.ldz;
            auto v_at = [&](int n) -> cx<R> {  // zbar on the full row, 0 off the window
                const int s = n - hp.t0;
                return (s >= 0 && s < hp.tw) ? zb[s] : cx<R>{0, 0};
            };
            if (!hp.blue) {
                for (int n = threadIdx.x; n < M; n += NT)
                    W[brev(n, logm)] = v_at(n);
                __syncthreads();
                fft_dit(W, TW, logm);
                for (int k = threadIdx.x; k < M; k += NT)
                    X[k] = cadd(X[k], cscale(W[k], weight(k)));
            } else {
                for (int n = threadIdx.x; n < M; n += NT) {
                    cx<R> v{0, 0};
                    if (n < t)
                        v = cmul(v_at(n), cconj(ch[n]));
                    W[brev(n, logm)] = v;
                }
                __syncthreads();
                fft_dit(W, TW, logm);
                for (int k = threadIdx.x; k < M; k += NT)
                    W[k] = cmul(W[k], bh[k]);
                __syncthreads();
                ifft_dif(W, TW, logm);
                const R invm = (R)1 / (R)M;
                for (int k = threadIdx.x; k < t; k += NT)
                    X[k] = cadd(X[k], cscale(cmul(cconj(ch[k]), W[brev(k, logm)]), weight(k) * invm));
            }
            __syncthreads();
        }
        // x_bar = Re(IDFT_t(X))
        R *xb = (R *)hp.xbar + (int64_t)rr.row * hp.ld;
        if (!hp.blue) {
            for (int k = threadIdx.x; k < M; k += NT)
                W[k] = X[k];
            __syncthreads();
            ifft_dif(W, TW, logm);
            const R inv_t = (R)1 / (R)t;
            for (int n = threadIdx.x; n < t; n += NT)
                xb[n] = W[brev(n, logm)].x * inv_t;
        } else {
            // IDFT(X) = conj(DFT(conj X)) / t; only its real part is needed
            for (int n = threadIdx.x; n < M; n += NT) {
                cx<R> v{0, 0};
                if (n < t)
                    v = cconj(cmul(X[n], ch[n]));
                W[brev(n, logm)] = v;
            }
            __syncthreads();
            fft_dit(W, TW, logm);
            for (int k = threadIdx.x; k < M; k += NT)
                W[k] = cmul(W[k], bh[k]);
            __syncthreads();
            ifft_dif(W, TW, logm);
            const R scale = (R)1 / ((R)M * (R)t);
            for (int n = threadIdx.x; n < t; n += NT)
                xb[n] = cmul(cconj(ch[n]), W[brev(n, logm)]).x * scale;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_hilbert_adjoint(bool f64, const HilbertArgs &a, int nwg, hipStream_t s)
{
    if (nwg <= 0 || a.nrows <= 0)
        return hipSuccess;
    if (f64)
        hilbert_adjoint_kernel<double, FFT_MAXLOG_F64><<<nwg, NT, 0, s>>>(a);
    else
        hilbert_adjoint_kernel<float, FFT_MAXLOG_F32><<<nwg, NT, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_twiddles(bool f64, void *tab, int logm, hipStream_t s)
{
    const int half = (1 << logm) / 2;
    const int grid = std::max(1, std::min(64, (half + NT - 1) / NT));
    if (f64)
        twiddle_kernel<double><<<grid, NT, 0, s>>>((cx<double> *)tab, logm);
    else
        twiddle_kernel<float><<<grid, NT, 0, s>>>((cx<float> *)tab, logm);
    return hipGetLastError();
}

hipError_t launch_chirps(bool f64, const ChirpJob *jobs, int njobs, hipStream_t s)
{
    if (njobs <= 0)
        return hipSuccess;
    if (f64)
        chirp_kernel<double, FFT_MAXLOG_F64><<<njobs, NT, 0, s>>>(jobs);
    else
        chirp_kernel<float, FFT_MAXLOG_F32><<<njobs, NT, 0, s>>>(jobs);
    return hipGetLastError();
}

hipError_t launch_hilbert(int mode, const HilbertArgs &a, int nwg, hipStream_t s)
{
    if (nwg <= 0 || a.nrows <= 0)
        return hipSuccess;
    switch (mode) {
    case M_F64: hilbert_kernel<M_F64><<<nwg, NT, 0, s>>>(a); break;
    case M_F32: hilbert_kernel<M_F32><<<nwg, NT, 0, s>>>(a); break;
    case M_SPLIT: hilbert_kernel<M_SPLIT><<<nwg, NT, 0, s>>>(a); break;
    case M_BF16: hilbert_kernel<M_BF16><<<nwg, NT, 0, s>>>(a); break;
    case M_F16: hilbert_kernel<M_F16><<<nwg, NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace plv
