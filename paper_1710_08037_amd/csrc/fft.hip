// fft.hip -- analytic signal of real rows by FFT (Section II.A, Eq. 3), fused
// with the window, the phasor normalisation (Eq. 4) and the store of the
// Gram kernel's phasor planes; and its adjoint for the backward.
//
// For a row x of length t and each band b:
//   X = DFT_t(x);  z_b = IDFT_t(h_b .* X);  u_b(s) = z_b(t0 + s) / |z_b(t0 + s)|
// with h the one-sided weights of the discrete analytic signal (1 at DC, 2
// below Nyquist, 1 at Nyquist for even t, 0 above) or a band mask (2 on the
// positive-frequency bins [klo, khi], 0 elsewhere).  The transforms run at the
// exact length t: an FFT of size M = t when t is a power of two, otherwise
// Bluestein's chirp-z form, DFT_t(x)_k = conj(c_k) * (a (*) b)_k / M-scaled,
// with c_m = exp(i pi m^2 / t), a = x .* conj(c) zero-padded to M >= 2t - 1
// and b the circular chirp; the circular convolution is taken by length-M FFTs
// with FFT_M(b) prepared once per length.  The inverse uses
// IDFT(Y) = conj(DFT(conj(Y))) / t.
//
// Transforms: Stockham autosort passes of radix 8 (one smaller radix pass
// when log2 M is not a multiple of 3), in natural order throughout.  Each
// active thread holds PER = 8 elements (16 at M = 8192) in registers --
// element tid + e * (M / PER) of the sequence -- and does whole radix-R
// butterflies on them; between passes the sequence goes through LDS (one hole every 16
// elements against bank conflicts).  Twiddles come from per-pass tables in
// LDS, built once per work-group from the quarter-wave table
// exp(-2 pi i m / M), m < M/4, by exact rotations.
//
// Bands: X stays in LDS after the forward transform; the first band taking the
// inverse transform reads it there, and when more follow (which overwrite
// the LDS) X is first copied to a slot of the work-group in global memory, so
// that no second M-element array is held in registers.  A band whose bin
// count K is small relative to the FFT cost is synthesised
// directly, z(n) = (2/t) sum_{k=klo..khi} X_k exp(2 pi i k n / t), as
// exp(2 pi i klo n / t) times a Horner polynomial in exp(2 pi i n / t) read
// from a per-length root table; other bands (and the plain analytic signal)
// take the inverse transform.
//
// One work-group per row at a time, grid-stride over the rows of one FFT
// size; one kernel instance per size, so LDS and the work-group shape fit M.
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

// Global-memory access of complex elements as native 2-vectors (loads and
// stores through global-address-space pointers).
template <class R>
using v2_t = typename std::conditional<sizeof(R) == 8, vd2, vf2>::type;
template <class R>
__device__ inline cx<R> gld(const cx<R> *p, int64_t i)
{
    const v2_t<R> a = gptr((const v2_t<R> *)p)[i];
    return cx<R>{a.x, a.y};
}
template <class R>
__device__ inline void gst(cx<R> *p, int64_t i, cx<R> a)
{
    gptr((v2_t<R> *)p)[i] = v2_t<R>{a.x, a.y};
}

// The same pointer (one value in every lane), opaque to the optimiser and
// held in scalar registers: addresses formed from it are recomputed where
// they are used instead of being hoisted out of the row and band loops and
// held in vector registers across the transforms.
template <class T>
__device__ inline T *fresh(T *p)
{
    const uint64_t u = (uint64_t)(uintptr_t)p;
    uint64_t w = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    asm volatile("" : "+s"(w));
    return (T *)(uintptr_t)w;
}

// ------------------------------------------------------------ shapes --
#ifndef PLV_FFT_LP
#define PLV_FFT_LP 3
#endif
constexpr int LP = PLV_FFT_LP;  // log2 of the main radix
// Elements per thread: one radix-8 butterfly's worth, except at M = 8192
// where 16 (two butterflies per pass) keep the work-group at 512 threads and
// its registers within a 2-waves-per-SIMD budget (1024 threads would spill).
__host__ __device__ constexpr int per_of(int logm) { return logm >= 13 ? 16 : 1 << (logm < LP ? logm : LP); }
__host__ __device__ constexpr int nta_of(int logm) { return (1 << logm) / per_of(logm); }  // active threads
__host__ __device__ constexpr int nt_of(int logm) { return nta_of(logm) < 64 ? 64 : nta_of(logm); }
__host__ __device__ constexpr int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int buf_elems(int logm) { return lpad((1 << logm) - 1) + 1; }
__host__ __device__ constexpr int npass_of(int logm) { return logm <= LP ? 1 : logm / LP + (logm % LP ? 1 : 0); }
// log2 of pass p's radix; the full-radix passes come first
__host__ __device__ constexpr int lrad_of(int logm, int p) { return logm <= LP ? logm : (p < logm / LP ? LP : logm % LP); }
// Per-pass twiddle tables: pass p >= 1 needs W^(r kk) for kk < NS = 2^(LP p)
// and 1 <= r < radix, stored at ptab_off(p) + kk (radix - 1) + r - 1.
__host__ __device__ constexpr int ptab_len(int logm, int p) { return (1 << (LP * p)) * ((1 << lrad_of(logm, p)) - 1); }
__host__ __device__ constexpr int ptab_off(int logm, int p) { return p <= 1 ? 0 : ptab_off(logm, p - 1) + ptab_len(logm, p - 1); }
__host__ __device__ constexpr int ptab_elems(int logm)
{
    return npass_of(logm) <= 1 ? 1 : ptab_off(logm, npass_of(logm) - 1) + ptab_len(logm, npass_of(logm) - 1);
}
// FP64 at M = 8192: the sequence alone takes 136 KB of LDS, so the passes read
// their twiddles straight from the quarter-wave table in global memory (32 KB,
// cache-resident; the same values the LDS tables would hold).
template <class R>
__host__ __device__ constexpr bool gtw_of(int logm) { return sizeof(R) == 8 && logm >= 13; }
template <class R>
__host__ __device__ constexpr int ptab_lds_elems(int logm) { return gtw_of<R>(logm) ? 1 : ptab_elems(logm); }

// a * exp(-+2 pi i m / 16) (forward: minus), m a constant after unrolling.
template <class R, bool INV>
__device__ inline cx<R> rot16(cx<R> a, int m)
{
    m &= 15;
    if (m == 0)
        return a;
    if (m == 8)
        return cx<R>{-a.x, -a.y};
    if (m == 4)  // forward: * (-i)
        return INV ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
    if (m == 12)  // forward: * (+i)
        return INV ? cx<R>{a.y, -a.x} : cx<R>{-a.y, a.x};
    // cos and sin of 2 pi m / 16
    constexpr R C1 = (R)0.92387953251128675613;  // cos(pi / 8)
    constexpr R S1 = (R)0.38268343236508977173;  // sin(pi / 8)
    constexpr R H = (R)0.70710678118654752440;   // sqrt(1/2)
    R c, s;
    switch (m) {
    case 1: c = C1; s = S1; break;
    case 2: c = H; s = H; break;
    case 3: c = S1; s = C1; break;
    case 5: c = -S1; s = C1; break;
    case 6: c = -H; s = H; break;
    case 7: c = -C1; s = S1; break;
    case 9: c = -C1; s = -S1; break;
    case 10: c = -H; s = -H; break;
    case 11: c = -S1; s = -C1; break;
    case 13: c = S1; s = -C1; break;
    case 14: c = H; s = -H; break;
    default: c = C1; s = -S1; break;  // 15
    }
    const R sg = INV ? s : -s;
    return cx<R>{a.x * c - a.y * sg, a.x * sg + a.y * c};
}

// In-register DFT of N = 1, 2, 4, 8, 16 points, natural order in and out
// (forward exp(-), inverse exp(+), unscaled).  N = 4 N2 splits as
// n = N2 n1 + n2, k = k1 + 4 k2: length-4 DFTs over n1, twiddles
// W_N^(n2 k1), length-N2 DFTs over n2.
template <class R, bool INV, int N>
__device__ inline void dft(cx<R> (&v)[N])
{
    if constexpr (N == 1) {
        return;
    } else if constexpr (N == 2) {
        const cx<R> a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (N == 4) {
        const cx<R> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const cx<R> a2 = cadd(v[1], v[3]), a3 = rot16<R, INV>(csub(v[1], v[3]), 4);
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    } else {
        constexpr int N2 = N / 4;
        cx<R> a[N2][4];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
            cx<R> s[4] = {v[n2], v[N2 + n2], v[2 * N2 + n2], v[3 * N2 + n2]};
            dft<R, INV, 4>(s);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1)
                a[n2][k1] = rot16<R, INV>(s[k1], n2 * k1 * (16 / N));
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cx<R> s[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2)
                s[n2] = a[n2][k1];
            dft<R, INV, N2>(s);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2)
                v[k1 + 4 * k2] = s[k2];
        }
    }
}

// exp(-+2 pi i idx / M) for 0 <= idx < M from the quarter-wave table.
template <class R, bool INV, int LOGM>
__device__ inline cx<R> twiddle(const cx<R> *twq, int idx)
{
    constexpr int Q = LOGM - 2;
    const int q = idx >> Q;
    const cx<R> w = twq[idx & ((1 << Q) - 1)];
    cx<R> o = (q & 1) ? cx<R>{w.y, -w.x} : w;  // times -i
    if (q & 2)
        o = cx<R>{-o.x, -o.y};                  // times -1
    if (INV)
        o.y = -o.y;
    return o;
}

// The same from the quarter-wave table in global memory.
template <class R, int LOGM>
__device__ inline cx<R> gtwiddle(const cx<R> *twq, int idx)
{
    constexpr int Q = LOGM - 2;
    const int q = idx >> Q;
    const cx<R> w = gld(twq, idx & ((1 << Q) - 1));
    cx<R> o = (q & 1) ? cx<R>{w.y, -w.x} : w;
    if (q & 2)
        o = cx<R>{-o.x, -o.y};
    return o;
}

// LDS index of element tid + e NTA (the natural register pattern); a base
// plus constants when NTA is a multiple of 16.
template <int LOGM>
__device__ inline int pat_addr(int tid, int e)
{
    constexpr int NTA = nta_of(LOGM);
    if constexpr (NTA % 16 == 0)
        return lpad(tid) + e * (NTA + NTA / 16);
    else
        return lpad(tid + e * NTA);
}

// Stockham pass P: butterflies j = tid + q NTA (q < PER / RR) read elements
// j + r M / RR -- registers e = q + r PER / RR of the natural pattern --, are
// twiddled by W_(NS RR)^(r (j mod NS)) and transformed, and land at
// (j - j mod NS) RR + j mod NS + r NS.
template <class R, int LOGM, bool INV, int P>
__device__ inline void fft_pass(cx<R> (&v)[per_of(LOGM)], cx<R> *buf, const cx<R> *ptab, bool act)
{
    constexpr int PER = per_of(LOGM), NTA = nta_of(LOGM);
    constexpr int LR = lrad_of(LOGM, P), RR = 1 << LR, NS = 1 << (LP * P), BPT = PER / RR;
    const int tid = threadIdx.x;
    if constexpr (P > 0) {
        __syncthreads();  // the previous pass is in LDS
        if (act) {
#pragma unroll
            for (int e = 0; e < PER; ++e)
                v[e] = buf[pat_addr<LOGM>(tid, e)];
        }
    }
    if (act) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            cx<R> b[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r)
                b[r] = v[q + r * BPT];
            if constexpr (NS > 1) {
                const int kk = (tid + q * NTA) & (NS - 1);
                const cx<R> *tw = ptab + ptab_off(LOGM, P) + kk * (RR - 1) - 1;
#pragma unroll
                for (int r = 1; r < RR; ++r) {
                    // W_(NS RR)^(r kk) = W_M^((r kk) M / (NS RR))
                    const cx<R> w = gtw_of<R>(LOGM) ? gtwiddle<R, LOGM>(ptab, (r * kk) << (LOGM - LP * P - LR))
                                                    : tw[r];
                    b[r] = cmul(b[r], INV ? cconj(w) : w);
                }
            }
            dft<R, INV, RR>(b);
#pragma unroll
            for (int r = 0; r < RR; ++r)
                v[q + r * BPT] = b[r];
            // one butterfly at a time: interleaving them only raises register use
            if constexpr (BPT > 1)
                __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();  // every thread has read this pass's input
    if (act) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int j = tid + q * NTA, kk = j & (NS - 1);
            const int d = ((j - kk) << LR) + kk;
            // lpad(d + r NS) as a base plus constants where that is exact:
            // NS >= 16 adds whole 16-groups; NS = 1 stays inside d's group
            const int base = lpad(d);
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const int adr = NS >= 16 ? base + r * (NS + NS / 16) : (NS == 1 ? base + r : lpad(d + r * NS));
                buf[adr] = v[q + r * BPT];
            }
        }
    }
    if constexpr (P + 1 < npass_of(LOGM))
        fft_pass<R, LOGM, INV, P + 1>(v, buf, ptab, act);
}

// Transform of the sequence held in v (natural pattern); the result is left
// in buf in natural order (index lpad(k)), visible to the whole work-group.
// ptab: the LDS pass tables, or the global quarter-wave table when
// gtw_of<R>(LOGM).  Every thread of the work-group must call it.
template <class R, int LOGM, bool INV>
__device__ inline void fft_lds(cx<R> (&v)[per_of(LOGM)], cx<R> *buf, const cx<R> *ptab, bool act)
{
    fft_pass<R, LOGM, INV, 0>(v, buf, ptab, act);
    __syncthreads();
}

// ------------------------------------------------------- set-up kernels --
// TW[k] = exp(-2 pi i k / M), k < M/2, evaluated in FP64.
template <class R>
__global__ __launch_bounds__(256) void twiddle_kernel(cx<R> *tab, int logm)
{
    const int M = 1 << logm;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < M / 2; k += gridDim.x * 256) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)M, &sn, &cs);
        tab[k] = cx<R>{(R)cs, (R)sn};
    }
}

// Builds the per-pass twiddle tables of the work-group: the quarter-wave
// table exp(-2 pi i m / M), m < M/4, is staged in `scratch` (the transform
// buffer, free at this point) and each entry W^(r kk) of pass p is read off it
// with an exact rotation by a power of -i.  Ends with a barrier.
template <class R, int LOGM>
__device__ inline void build_tables(cx<R> *ptab, cx<R> *scratch, const void *tw_tab)
{
    constexpr int M = 1 << LOGM, NP = npass_of(LOGM);
    if constexpr (NP > 1 && !gtw_of<R>(LOGM)) {
        for (int k = threadIdx.x; k < M / 4; k += blockDim.x)
            scratch[k] = gld((const cx<R> *)tw_tab, k);
        __syncthreads();
        for (int p = 1; p < NP; ++p) {
            const int lr = lrad_of(LOGM, p), rr = 1 << lr, len = ptab_len(LOGM, p), off = ptab_off(LOGM, p);
            for (int e = threadIdx.x; e < len; e += blockDim.x) {
                const int kk = e / (rr - 1), r = e - kk * (rr - 1) + 1;
                ptab[off + e] = twiddle<R, false, LOGM>(scratch, (r * kk) << (LOGM - LP * p - lr));
            }
        }
    }
    __syncthreads();
}

// The twiddle source the passes take: the LDS tables, or the global table.
template <class R, int LOGM>
__device__ inline const cx<R> *pass_tables(const cx<R> *ptab, const void *tw_tab)
{
    return gtw_of<R>(LOGM) ? (const cx<R> *)tw_tab : ptab;
}

// Per distinct row length t (one work-group per job): the root table
// exp(2 pi i m / t), m < t; for Bluestein lengths also the chirp
// c_m = exp(i pi m^2 / t), m < t, and FFT_M of the circular chirp
// b_m = c_m (m < t), b_{M-m} = c_m (0 < m < t), 0 elsewhere.  Angles are
// reduced exactly in integers (m^2 mod 2t) and evaluated in FP64.
template <class R, int LOGM>
__global__ __launch_bounds__(nt_of(LOGM)) void chirp_kernel(const ChirpJob *jobs)
{
    constexpr int M = 1 << LOGM, PER = per_of(LOGM), NTA = nta_of(LOGM);
    __shared__ cx<R> buf[buf_elems(LOGM)];
    __shared__ cx<R> ptab_lds[ptab_lds_elems<R>(LOGM)];
    const ChirpJob jb = jobs[blockIdx.x];
    const int t = jb.t, tid = threadIdx.x;
    cx<R> *roots = (cx<R> *)jb.roots;
    for (int m = tid; m < t; m += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)t, &sn, &cs);
        gst(roots, m, cx<R>{(R)cs, (R)sn});
    }
    if (!jb.blue)
        return;
    build_tables<R, LOGM>(ptab_lds, buf, jb.tw_tab);
    const cx<R> *ptab = pass_tables<R, LOGM>(ptab_lds, jb.tw_tab);
    cx<R> *chirp = (cx<R> *)jb.chirp, *bh = (cx<R> *)jb.bhat;
    const bool act = tid < NTA;
    cx<R> v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int m = tid + e * NTA;
        const int src = m < t ? m : (M - m < t ? M - m : -1);
        cx<R> c{0, 0};
        if (act && src >= 0) {
            const int64_t r2 = ((int64_t)src * src) % (2 * (int64_t)t);  // m^2 mod 2t, exact
            double sn, cs;
            sincospi((double)r2 / (double)t, &sn, &cs);
            c = cx<R>{(R)cs, (R)sn};
            if (m < t)
                gst(chirp, m, c);
        }
        v[e] = c;
    }
    fft_lds<R, LOGM, false>(v, buf, ptab, act);
    for (int k = tid; k < M; k += blockDim.x)
        gst(bh, k, buf[lpad(k)]);
}

// ------------------------------------------------------------- forward --
template <class R, bool FIR>
__device__ inline R band_weight(BandBins bb, int k, int t)
{
    if (FIR && bb.fir) {  // one-sided weights times the FIR's zero-phase gain |H|^2
        if (2 * k > t)
            return (R)0;
        const R one_sided = (k == 0 || 2 * k == t) ? (R)1 : (R)2;
        return one_sided * ((const R *)bb.w)[k];
    }
    if (bb.klo < 0)
        return k == 0 ? (R)1 : (2 * k < t ? (R)2 : (2 * k == t ? (R)1 : (R)0));
    return (k >= bb.klo && k <= bb.khi) ? (R)2 : (R)0;
}

template <class R>
__device__ inline void store4_mode(int mode, uint8_t *dst, int64_t plane_bytes, const R (&ur)[4], const R (&ui)[4])
{
    if constexpr (sizeof(R) == 8) {
        store4<M_F64>(dst, plane_bytes, ur, ui);
    } else {
        switch (mode) {
        case M_F32: store4<M_F32>(dst, plane_bytes, ur, ui); break;
        case M_SPLIT: store4<M_SPLIT>(dst, plane_bytes, ur, ui); break;
        case M_BF16: store4<M_BF16>(dst, plane_bytes, ur, ui); break;
        default: store4<M_F16>(dst, plane_bytes, ur, ui); break;
        }
    }
}

// Window samples of one band from z_n = zf(n) (a functor on the full-row
// index n = t0 + s): phasor planes, or z itself for the backward.
template <class R, class ZF>
__device__ inline void store_band(int mode, const GramDesc &g, const HilbertProb &hp, int row, ZF zf)
{
    const int nt = blockDim.x;
    if (g.zbuf) {
        cx<R> *zr = (cx<R> *)g.zbuf + (int64_t)row * g.ldz;
        for (int s = threadIdx.x; s < hp.tw; s += nt)
            gst(zr, s, zf(hp.t0 + s));
        return;
    }
    for (int s0 = threadIdx.x * 4; s0 < g.tpad; s0 += nt * 4) {
        R ur[4], ui[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int s = s0 + v;
            ur[v] = 0;
            ui[v] = 0;
            if (s < hp.tw) {
                const cx<R> z = zf(hp.t0 + s);
                unit_phasor(z.x, z.y, ur[v], ui[v]);
            }
        }
        store4_mode<R>(mode, plane_at((uint8_t *)g.u, g.cstride, g.chunk, g.npad, cbytes_of(mode), row, s0),
                       g.plane_bytes, ur, ui);
    }
}

// ------------------------------------------------------- band synthesis --
// Direct synthesis of a narrow band from its bins X_k, klo <= k <= khi:
// z(n) = (2/t) exp(2 pi i klo n / t) sum_{m < K} X_{klo+m} w^m, w = exp(2 pi i n / t)
// (Horner in w).  One work-group takes SYNTH_S consecutive window samples of one
// (problem, band) for SYNTH_R rows, 16 rows at a time: lane (quad q, row rr)
// holds four samples of row rr, so a wave stores one contiguous stage-major
// run of 16 rows.  The roots w and the base exp(2 pi i klo n / t) of a lane's
// samples are loaded once and serve every row; the bins of the 16 rows pass
// through LDS.
// Work-groups of problem q: nbands x ceil(L / SYNTH_S) x ceil(n / SYNTH_R), L the
// samples written per row (tpad for phasor planes, the window for the backward's
// complex z); the host stores the running sums in a table of nprob + 1 entries.
// FP64 mode; the FP32 modes take the matrix-product form below.
template <class R>
__global__ __launch_bounds__(256) void band_synth_kernel(HilbertArgs a, int mode)
{
    static_assert(SYNTH_S == 64 && SYNTH_R % 16 == 0, "16 quads of 4 samples, rows in groups of 16");
    __shared__ cx<R> xs[16][DIRECT_KMAX];
    // ---- which (problem, band, sample block, row chunk): scalar binary search
    const int job = blockIdx.x;
    int lo = 0, hi = a.nprob;  // prefix[lo] <= job < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.synth_prefix[mid] <= job)
            lo = mid;
        else
            hi = mid;
    }
    const int q = lo;
    const HilbertProb hp = a.hp[q];
    const GramDesc g0 = a.gd[hp.gram0];
    const int len0 = g0.zbuf ? hp.tw : g0.tpad;  // samples synthesised per row (host counts the same)
    const int nsb = (len0 + SYNTH_S - 1) / SYNTH_S;
    int rest = job - a.synth_prefix[q];
    const int b = rest % hp.nbands;
    rest /= hp.nbands;
    const int sb = rest % nsb, rc = rest / nsb;
    const BandBins bb = a.bins[hp.bin0 + b];
    if (!bb.direct)
        return;
    const GramDesc g = a.gd[hp.gram0 + b];
    const int t = hp.t, klo = bb.klo, khi = bb.khi;
    const int nk = khi >= klo ? khi - klo + 1 : 0;  // <= DIRECT_KMAX (host rule)
    const int kl = nk ? klo : 0;
    const int limit = g.zbuf ? hp.tw : g.tpad;
    const int tid = threadIdx.x, qd = tid >> 4, rr = tid & 15;
    const int s0 = sb * SYNTH_S + qd * 4;
    const cx<R> *roots = (const cx<R> *)hp.roots;
    const R scale = (R)2 / (R)t;
    cx<R> w[4], base[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int n = min(hp.t0 + s0 + v, t - 1);  // clamped: samples past the window are discarded
        w[v] = gld(roots, n);
        base[v] = gld(roots, (int)(((int64_t)kl * n) % t));
    }
    const cx<R> *xsrc = (const cx<R> *)hp.xbins + (int64_t)b * DIRECT_KMAX;
    const int64_t xrow = (int64_t)hp.nbands * DIRECT_KMAX;  // bins of one row to the next
    cx<R> *zrow0 = (cx<R> *)g.zbuf;
    const int r_end = min(hp.n, (rc + 1) * SYNTH_R);
    for (int r0 = rc * SYNTH_R; r0 < r_end; r0 += 16) {
        __syncthreads();  // the previous group's bins are no longer read
        for (int e = tid; e < 16 * nk; e += 256) {
            const int r = r0 + e / nk, k = e % nk;
            xs[e / nk][k] = r < hp.n ? gld(xsrc, r * xrow + k) : cx<R>{0, 0};
        }
        __syncthreads();
        const int row = r0 + rr;
        if (row >= r_end || s0 >= limit)
            continue;
        cx<R> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int k = nk - 1; k >= 0; --k) {
            const cx<R> xk = xs[rr][k];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[v] = cadd(cmul(acc[v], w[v]), xk);
        }
        cx<R> z[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            z[v] = cscale(cmul(base[v], acc[v]), scale);  // 0 for an empty band
        if (g.zbuf) {
            cx<R> *zrow = zrow0 + (int64_t)row * g.ldz;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (s0 + v < hp.tw)
                    gst(zrow, s0 + v, z[v]);
        } else {
            R ur[4], ui[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                ur[v] = 0;
                ui[v] = 0;
                if (s0 + v < hp.tw)
                    unit_phasor(z[v].x, z[v].y, ur[v], ui[v]);
            }
            store4_mode<R>(mode, plane_at((uint8_t *)g.u, g.cstride, g.chunk, g.npad, cbytes_of(mode), row, s0),
                           g.plane_bytes, ur, ui);
        }
    }
}

// FP32 modes: the same sums as a matrix product on MFMA.  With nb = t0 +
// sb SYNTH_S the full-row index of the block's first sample and n = nb + j:
//   z(n) = sum_{m<K} R[j][m] Y[m],   R[j][m] = exp(2 pi i (klo+m) j / t),
//   Y[m] = (2/t) exp(2 pi i (klo+m) nb / t) X_{klo+m}.
// R is one table for every row of the work-group (SYNTH_S x K, from the root
// table, in LDS); each row's Y is its B operand, formed as the row's bins
// times the block's rotations.  v_mfma_f32_16x16x4f32 with the samples as
// the row index and the signal rows as the column index: a wave takes 16
// rows at a time, and afterwards lane l holds samples 4 (l / 16) .. + 3 of
// every 16-sample column block for row l % 16, the store pattern of the
// Horner kernel (16 rows x 64 bytes of one plane stage per wave and store).
// Complex: Re z = Rr.Yr - Ri.Yi, Im z = Rr.Yi + Ri.Yr, four real products.
template <int MODE>
__global__ __launch_bounds__(256, 4) void band_synth_mfma_kernel(HilbertArgs a)
{
    static_assert(SYNTH_S == 64 && SYNTH_R % 64 == 0, "4 column blocks of 16 samples; 4 waves of 16 rows");
    constexpr int RS = SYNTH_S + 16;  // R row stride: the 4 K-rows one MFMA step reads land in distinct banks
    constexpr int KS = DIRECT_KMAX / 4;  // MFMA steps of 4 bins, at most
    __shared__ float rre[DIRECT_KMAX * RS], rim[DIRECT_KMAX * RS];
    __shared__ cx<float> pk[DIRECT_KMAX];
    const int job = blockIdx.x;
    int lo = 0, hi = a.nprob;  // prefix[lo] <= job < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.synth_prefix[mid] <= job)
            lo = mid;
        else
            hi = mid;
    }
    const int q = lo;
    const HilbertProb hp = a.hp[q];
    const GramDesc g0 = a.gd[hp.gram0];
    const int len0 = g0.zbuf ? hp.tw : g0.tpad;  // samples synthesised per row (host counts the same)
    const int nsb = (len0 + SYNTH_S - 1) / SYNTH_S;
    int rest = job - a.synth_prefix[q];
    const int b = rest % hp.nbands;
    rest /= hp.nbands;
    const int sb = rest % nsb, rc = rest / nsb;
    const BandBins bb = a.bins[hp.bin0 + b];
    if (!bb.direct)
        return;
    const GramDesc g = a.gd[hp.gram0 + b];
    const int t = hp.t, klo = bb.klo, khi = bb.khi;
    const int nk = khi >= klo ? khi - klo + 1 : 0;  // <= DIRECT_KMAX (host rule)
    const int kl = nk ? klo : 0, kp = max(4, (nk + 3) & ~3);  // an empty band: one step of zeros
    const int limit = g.zbuf ? hp.tw : g.tpad;
    const int tid = threadIdx.x;
    const cx<float> *roots = (const cx<float> *)hp.roots;
    const int nb = hp.t0 + sb * SYNTH_S;  // < t + SYNTH_S; (kl + m) nb < 2^31 for t <= 8192

    const int lane = tid & 63, wv = tid >> 6, lr = lane & 15, lk = lane >> 4;
    const cx<float> *xsrc = (const cx<float> *)hp.xbins + (int64_t)b * DIRECT_KMAX;
    const int64_t xrow = (int64_t)hp.nbands * DIRECT_KMAX;  // bins of one row to the next
    const int r_end = min(hp.n, (rc + 1) * SYNTH_R);
    const int rfirst = rc * SYNTH_R + wv * 16;
    // The bins of a 16-row group, raw (m < kp <= DIRECT_KMAX stays inside
    // each row's slot; bins past nk and rows past the end are selected away
    // where used).  Each group's loads are issued one group ahead.
    auto load_bins = [&](int r0, cx<float> (&y)[KS]) {
        const cx<float> *xr = xsrc + (int64_t)min(r0 + lr, r_end - 1) * xrow + lk;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (s * 4 < kp)
                y[s] = gld(xr, s * 4);
    };
    cx<float> ya[KS], yb[KS];
    if (rfirst < r_end)
        load_bins(rfirst, ya);

    // ---- R (zero rows up to kp): four threads per bin, 16 consecutive j
    // each, the root index stepped by kl + m (< t) from one remainder
    for (int e = tid; e < kp * 4; e += 256) {
        const int m = e >> 2, j0 = (e & 3) * 16, step = kl + m;
        int idx = m < nk ? (step * j0) % t : 0;
#pragma unroll
        for (int j = j0; j < j0 + 16; ++j) {
            const cx<float> r = m < nk ? gld(roots, idx) : cx<float>{0.0f, 0.0f};
            rre[m * RS + j] = r.x;
            rim[m * RS + j] = r.y;
            idx += step;
            idx = idx >= t ? idx - t : idx;
        }
    }
    if (tid < kp)
        pk[tid] = tid < nk ? cscale(gld(roots, ((kl + tid) * nb) % t), 2.0f / (float)t) : cx<float>{0.0f, 0.0f};
    __syncthreads();

    // the column blocks' plane offsets: a 16-sample block lies in one K-chunk
    // (chunks are whole granules) and its 4-sample runs in one plane stage;
    // the uniform part per block here, the lane's part (row, its 4 samples)
    // per row group
    constexpr int CB = cbytes_of(MODE), LSPS = CB == 4 ? 4 : 3;  // log2 samples per stage
    int64_t boff[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int sbk = sb * SYNTH_S + c * 16;
        const int ch = sbk < g.chunk ? 0 : sbk / g.chunk, k = sbk - ch * g.chunk;
        boff[c] = ch * g.cstride + ((int64_t)(k >> LSPS) * g.npad) * 64;
    }

    // one 16-row group: its product from y (the group's bins), the next
    // group's bins into yn, then the normalisation and store
    auto group = [&](int r0, const cx<float> (&y)[KS], cx<float> (&yn)[KS]) {
        const int row = r0 + lr;
        const bool rok = row < r_end;
        if (r0 + 64 < r_end)
            load_bins(r0 + 64, yn);
        vf4 zr[4], zi[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            zr[c] = vf4{0.0f, 0.0f, 0.0f, 0.0f};
            zi[c] = vf4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s > 0 && s * 4 >= kp)  // kp >= 4: the first step always runs
                break;
            const int m = s * 4 + lk;
            const cx<float> x = (rok && m < nk) ? y[s] : cx<float>{0.0f, 0.0f};
            const cx<float> yv = cmul(x, pk[m]);
            const float *ar = rre + m * RS + lr, *ai = rim + m * RS + lr;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float rr_ = ar[c * 16], ri_ = ai[c * 16];
                zr[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(rr_, yv.x, zr[c], 0, 0, 0);
                zr[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ri_, -yv.y, zr[c], 0, 0, 0);
                zi[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(rr_, yv.y, zi[c], 0, 0, 0);
                zi[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ri_, yv.x, zi[c], 0, 0, 0);
            }
        }
        if (!rok)
            return;
        if (g.zbuf) {
            cx<float> *zrow = (cx<float> *)g.zbuf + (int64_t)row * g.ldz;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int s0 = sb * SYNTH_S + c * 16 + lk * 4;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (s0 + v < hp.tw)
                        gst(zrow, s0 + v, cx<float>{zr[c][v], zi[c][v]});
            }
            return;
        }
        const int64_t lane_off = ((int64_t)((lk * 4) >> LSPS) * g.npad + row) * 64 + ((lk * 4) & ((1 << LSPS) - 1)) * CB;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int sbk = sb * SYNTH_S + c * 16;  // wave-uniform
            if (sbk >= limit)
                continue;
            const float re[4] = {zr[c][0], zr[c][1], zr[c][2], zr[c][3]};
            const float im[4] = {zi[c][0], zi[c][1], zi[c][2], zi[c][3]};
            float ur[4], ui[4];
            unit_phasor4(re, im, ur, ui);
            if (sbk + 16 > hp.tw) {  // zero phasors past the window
                const int s0 = sbk + lk * 4;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const bool in = s0 + v < hp.tw;
                    ur[v] = in ? ur[v] : 0.0f;
                    ui[v] = in ? ui[v] : 0.0f;
                }
            }
            store4<MODE, float, true>((uint8_t *)g.u + boff[c] + lane_off, g.plane_bytes, ur, ui);
        }
    };
    for (int r0 = rfirst; r0 < r_end; r0 += 64) {  // wave-uniform bounds
        group(r0, ya, yb);
#pragma unroll
        for (int s = 0; s < KS; ++s)
            ya[s] = yb[s];
    }
}

// FIR: the call has forward-backward FIR bands (weights from tables); the
// variant without them keeps the mask path's registers.
template <class R, int LOGM, bool FIR>
__global__ __launch_bounds__(nt_of(LOGM)) void hilbert_kernel(HilbertArgs a, int mode)
{
    constexpr int M = 1 << LOGM, PER = per_of(LOGM), NTA = nta_of(LOGM);
    __shared__ cx<R> buf[buf_elems(LOGM)];
    __shared__ cx<R> ptab_lds[ptab_lds_elems<R>(LOGM)];
    const int tid = threadIdx.x;
    const bool act = tid < NTA;
    build_tables<R, LOGM>(ptab_lds, buf, a.hp[a.rows[0].prob].tw_tab);  // one set per launch (one M)
    const cx<R> *ptab = pass_tables<R, LOGM>(ptab_lds, a.hp[a.rows[0].prob].tw_tab);

    // the spectrum X of a row with two or more inverse-transform bands is kept
    // in this work-group's slot of M elements (natural register pattern, each
    // thread reading back only what it wrote), not in registers
    cx<R> *xs = a.xs ? (cx<R> *)a.xs + (int64_t)blockIdx.x * M : nullptr;

    for (int ri = blockIdx.x; ri < a.nrows; ri += gridDim.x) {
        const RowRef rr = a.rows[ri];
        const HilbertProb hp = a.hp[rr.prob];
        const int t = hp.t;
        auto x = gptr((const R *)hp.x + (int64_t)rr.row * hp.ld);
        const cx<R> *ch = (const cx<R> *)hp.chirp;
        const cx<R> *bh = (const cx<R> *)hp.bhat;
        cx<R> v[PER];
        // loads are unconditional at clamped indices, then selected
        const int tid0 = act ? tid : 0;

        // ---- X = DFT_t(x), natural order in buf (k < t)
        if (!hp.blue) {
#pragma unroll
            for (int e = 0; e < PER; ++e)
                v[e] = cx<R>{x[tid0 + e * NTA], (R)0};
            fft_lds<R, LOGM, false>(v, buf, ptab, act);
        } else {
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int n = tid0 + e * NTA, nc = min(n, t - 1);
                const cx<R> a = cscale(cconj(gld(fresh(ch), nc)), x[nc]);
                v[e] = n < t ? a : cx<R>{0, 0};
            }
            fft_lds<R, LOGM, false>(v, buf, ptab, act);
#pragma unroll
            for (int e = 0; e < PER; ++e)
                v[e] = cmul(buf[pat_addr<LOGM>(tid0, e)], gld(fresh(bh), tid0 + e * NTA));
            fft_lds<R, LOGM, true>(v, buf, ptab, act);
            const R invm = (R)1 / (R)M;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int k = tid0 + e * NTA;
                const cx<R> a = cscale(cmul(cconj(gld(fresh(ch), min(k, t - 1))), buf[pat_addr<LOGM>(tid0, e)]), invm);
                v[e] = k < t ? a : cx<R>{0, 0};
            }
            __syncthreads();  // buf fully read
            if (act) {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    buf[pat_addr<LOGM>(tid, e)] = v[e];
            }
            __syncthreads();
        }

        // ---- narrow bands: their bins to xbins, synthesised by band_synth_kernel
        int ninv = 0;
        for (int b = 0; b < hp.nbands; ++b) {
            const BandBins bb = a.bins[hp.bin0 + b];
            if (bb.direct) {
                cx<R> *dst = (cx<R> *)hp.xbins + ((int64_t)rr.row * hp.nbands + b) * DIRECT_KMAX;
                for (int k = bb.klo + tid; k <= bb.khi; k += (int)blockDim.x)
                    gst(dst, k - bb.klo, buf[lpad(k)]);
            } else {
                ++ninv;
            }
        }
        if (ninv >= 2 && act) {
#pragma unroll
            for (int e = 0; e < PER; ++e)
                gst(fresh(xs), tid + e * NTA, buf[pat_addr<LOGM>(tid, e)]);
        }
        // ---- the other bands by inverse transform (each overwrites buf); the
        // first takes X from buf, the later ones from the slot
        int done = 0;
        for (int b = 0; b < hp.nbands; ++b) {
            const BandBins bb = a.bins[hp.bin0 + b];
            if (bb.direct)
                continue;
            const GramDesc g = a.gd[hp.gram0 + b];
            if (done++ == 0) {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = buf[pat_addr<LOGM>(tid0, e)];
            } else {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = gld(fresh(xs), tid0 + e * NTA);
            }
            if (!hp.blue) {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = cscale(v[e], band_weight<R, FIR>(bb, tid0 + e * NTA, t));
                fft_lds<R, LOGM, true>(v, buf, ptab, act);
                const R inv_t = (R)1 / (R)t;
                store_band<R>(mode, g, hp, rr.row, [&](int n) { return cscale(buf[lpad(n)], inv_t); });
            } else {
                // v = conj(Y), Y = h .* X; z = conj(DFT_t(v)) / t by Bluestein
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    const int n = tid0 + e * NTA;
                    // X is 0 at n >= t, so the clamped chirp index changes nothing
                    v[e] = cconj(cmul(cscale(v[e], band_weight<R, FIR>(bb, n, t)), gld(fresh(ch), min(n, t - 1))));
                }
                fft_lds<R, LOGM, false>(v, buf, ptab, act);
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = cmul(buf[pat_addr<LOGM>(tid0, e)], gld(fresh(bh), tid0 + e * NTA));
                fft_lds<R, LOGM, true>(v, buf, ptab, act);
                const R zs = (R)1 / ((R)M * (R)t);
                store_band<R>(mode, g, hp, rr.row,
                              [&](int n) { return cscale(cmul(gld(fresh(ch), n), cconj(buf[lpad(n)])), zs); });
            }
        }
    }
}

// -------------------------------------------------------------- adjoint --
// dL/dx of one row: z_b = M_b x with M_b = IDFT diag(h_b) DFT Hermitian
// (h_b real), so dL/dx = Re(sum_b M_b zbar_b) = Re(IDFT(sum_b h_b .*
// DFT(zbar_b))), zbar_b being 0 outside the window.  With several bands the
// running spectrum sum is kept in the work-group's slot of M elements (each
// thread reading back only what it wrote), not in registers.  ONE: calls
// with a single band (no sum, no slot code).
template <class R, int LOGM, bool ONE, bool FIR>
__global__ __launch_bounds__(nt_of(LOGM)) void hilbert_adjoint_kernel(HilbertArgs a)
{
    constexpr int M = 1 << LOGM, PER = per_of(LOGM), NTA = nta_of(LOGM);
    __shared__ cx<R> buf[buf_elems(LOGM)];
    __shared__ cx<R> ptab_lds[ptab_lds_elems<R>(LOGM)];
    const int tid = threadIdx.x;
    const bool act = tid < NTA;
    build_tables<R, LOGM>(ptab_lds, buf, a.hp[a.rows[0].prob].tw_tab);
    const cx<R> *ptab = pass_tables<R, LOGM>(ptab_lds, a.hp[a.rows[0].prob].tw_tab);
    cx<R> *xs = a.xs ? (cx<R> *)a.xs + (int64_t)blockIdx.x * M : nullptr;

    for (int ri = blockIdx.x; ri < a.nrows; ri += gridDim.x) {
        const RowRef rr = a.rows[ri];
        const HilbertProb hp = a.hp[rr.prob];
        const int t = hp.t, nb = ONE ? 1 : hp.nbands;
        const cx<R> *ch = (const cx<R> *)hp.chirp;
        const cx<R> *bh = (const cx<R> *)hp.bhat;
        const int tid0 = act ? tid : 0;
        cx<R> v[PER];
        for (int b = 0; b < nb; ++b) {
            const BandBins bb = a.bins[hp.bin0 + b];
            const GramDesc g = a.gd[hp.gram0 + b];
            const cx<R> *zb = (const cx<R> *)g.zbuf + (int64_t)rr.row * g.ldz;
            auto v_at = [&](int n) -> cx<R> {  // zbar on the full row, 0 off the window
                const int s = n - hp.t0;
                const cx<R> z = gld(fresh(zb), min(max(s, 0), hp.tw - 1));
                return (s >= 0 && s < hp.tw) ? z : cx<R>{0, 0};
            };
            // v <- h_b .* DFT_t(zbar_b)
            if (!hp.blue) {
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = v_at(tid0 + e * NTA);
                fft_lds<R, LOGM, false>(v, buf, ptab, act);
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = cscale(buf[pat_addr<LOGM>(tid0, e)], band_weight<R, FIR>(bb, tid0 + e * NTA, t));
            } else {
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    const int n = tid0 + e * NTA;
                    v[e] = cmul(v_at(n), cconj(gld(fresh(ch), min(n, t - 1))));  // v_at is 0 at n >= t
                }
                fft_lds<R, LOGM, false>(v, buf, ptab, act);
#pragma unroll
                for (int e = 0; e < PER; ++e)
                    v[e] = cmul(buf[pat_addr<LOGM>(tid0, e)], gld(fresh(bh), tid0 + e * NTA));
                fft_lds<R, LOGM, true>(v, buf, ptab, act);
                const R invm = (R)1 / (R)M;
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    const int k = tid0 + e * NTA;
                    const cx<R> d = cmul(cconj(gld(fresh(ch), min(k, t - 1))), buf[pat_addr<LOGM>(tid0, e)]);
                    v[e] = cscale(d, k < t ? band_weight<R, FIR>(bb, k, t) * invm : (R)0);
                }
            }
            // the band sum: bands 0 .. nb - 2 into the slot, the last one added to it in v
            if (!ONE && nb > 1 && act) {
                if (b == 0) {
#pragma unroll
                    for (int e = 0; e < PER; ++e)
                        gst(fresh(xs), tid + e * NTA, v[e]);
                } else if (b < nb - 1) {
#pragma unroll
                    for (int e = 0; e < PER; ++e)
                        gst(fresh(xs), tid + e * NTA, cadd(gld(fresh(xs), tid + e * NTA), v[e]));
                } else {
#pragma unroll
                    for (int e = 0; e < PER; ++e)
                        v[e] = cadd(gld(fresh(xs), tid + e * NTA), v[e]);
                }
            }
        }
        // x_bar = Re(IDFT_t(S)), S in v
        auto xb = gptr((R *)hp.xbar + (int64_t)rr.row * hp.ld);
        if (!hp.blue) {
            fft_lds<R, LOGM, true>(v, buf, ptab, act);
            const R inv_t = (R)1 / (R)t;
            for (int n = tid; n < t; n += blockDim.x)
                xb[n] = buf[lpad(n)].x * inv_t;
        } else {
            // IDFT(S) = conj(DFT(conj S)) / t; only its real part is needed
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int n = tid0 + e * NTA;
                v[e] = cconj(cmul(v[e], gld(fresh(ch), min(n, t - 1))));  // S is 0 at n >= t
            }
            fft_lds<R, LOGM, false>(v, buf, ptab, act);
#pragma unroll
            for (int e = 0; e < PER; ++e)
                v[e] = cmul(buf[pat_addr<LOGM>(tid0, e)], gld(fresh(bh), tid0 + e * NTA));
            fft_lds<R, LOGM, true>(v, buf, ptab, act);
            const R scale = (R)1 / ((R)M * (R)t);
            for (int n = tid; n < t; n += blockDim.x)
                xb[n] = cmul(cconj(gld(fresh(ch), n)), buf[lpad(n)]).x * scale;
        }
    }
}

// ------------------------------------------------------------ dispatch --
// Work-groups of a grid-stride transform launch: every one resident at once,
// and no more than the spectrum slots the host reserved (when it did).
template <class K>
int grid_for(K kernel, int nt, int rows, int cus, const HilbertArgs *ha)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, nt, 0) != hipSuccess || occ < 1)
        occ = 1;
    int n = std::min(rows, cus * occ);
    if (ha->xs)
        n = std::min(n, ha->xslots);
    return std::max(1, n);
}

template <class R, int LOGM>
hipError_t launch_sized(int kind, int mode, const HilbertArgs *ha, const ChirpJob *jobs, int n, int cus,
                        hipStream_t s)
{
    constexpr int NT = nt_of(LOGM);
    if (kind == 0) {
        chirp_kernel<R, LOGM><<<n, NT, 0, s>>>(jobs);
    } else if (kind == 1) {
        if (ha->fir) {
            const int nwg = grid_for(hilbert_kernel<R, LOGM, true>, NT, ha->nrows, cus, ha);
            hilbert_kernel<R, LOGM, true><<<nwg, NT, 0, s>>>(*ha, mode);
        } else {
            const int nwg = grid_for(hilbert_kernel<R, LOGM, false>, NT, ha->nrows, cus, ha);
            hilbert_kernel<R, LOGM, false><<<nwg, NT, 0, s>>>(*ha, mode);
        }
    } else {
        if (ha->nbands == 1 && !ha->fir) {
            const int nwg = grid_for(hilbert_adjoint_kernel<R, LOGM, true, false>, NT, ha->nrows, cus, ha);
            hilbert_adjoint_kernel<R, LOGM, true, false><<<nwg, NT, 0, s>>>(*ha);
        } else if (ha->nbands == 1) {
            const int nwg = grid_for(hilbert_adjoint_kernel<R, LOGM, true, true>, NT, ha->nrows, cus, ha);
            hilbert_adjoint_kernel<R, LOGM, true, true><<<nwg, NT, 0, s>>>(*ha);
        } else if (!ha->fir) {
            const int nwg = grid_for(hilbert_adjoint_kernel<R, LOGM, false, false>, NT, ha->nrows, cus, ha);
            hilbert_adjoint_kernel<R, LOGM, false, false><<<nwg, NT, 0, s>>>(*ha);
        } else {
            const int nwg = grid_for(hilbert_adjoint_kernel<R, LOGM, false, true>, NT, ha->nrows, cus, ha);
            hilbert_adjoint_kernel<R, LOGM, false, true><<<nwg, NT, 0, s>>>(*ha);
        }
    }
    return hipGetLastError();
}

template <class R, int LOGM, int MAXLOG>
hipError_t dispatch(int logm, int kind, int mode, const HilbertArgs *ha, const ChirpJob *jobs, int n, int cus,
                    hipStream_t s)
{
    if (logm == LOGM)
        return launch_sized<R, LOGM>(kind, mode, ha, jobs, n, cus, s);
    if constexpr (LOGM < MAXLOG)
        return dispatch<R, LOGM + 1, MAXLOG>(logm, kind, mode, ha, jobs, n, cus, s);
    return hipErrorInvalidValue;
}

hipError_t dispatch_any(bool f64, int logm, int kind, int mode, const HilbertArgs *ha, const ChirpJob *jobs, int n,
                        int cus, hipStream_t s)
{
    if (f64) {
        if (logm < 1 || logm > FFT_MAXLOG_F64)
            return hipErrorInvalidValue;
        return dispatch<double, 1, FFT_MAXLOG_F64>(logm, kind, mode, ha, jobs, n, cus, s);
    }
    if (logm < 1 || logm > FFT_MAXLOG_F32)
        return hipErrorInvalidValue;
    return dispatch<float, 1, FFT_MAXLOG_F32>(logm, kind, mode, ha, jobs, n, cus, s);
}

}  // namespace

hipError_t launch_twiddles(bool f64, void *tab, int logm, hipStream_t s)
{
    const int half = (1 << logm) / 2;
    const int grid = std::max(1, std::min(64, (half + 255) / 256));
    if (f64)
        twiddle_kernel<double><<<grid, 256, 0, s>>>((cx<double> *)tab, logm);
    else
        twiddle_kernel<float><<<grid, 256, 0, s>>>((cx<float> *)tab, logm);
    return hipGetLastError();
}

namespace {

// |H(e^{i theta})|^2 = A(theta)^2, A = c_0 + 2 sum_{j=1..half} c_j cos(j theta),
// theta = 2 pi k / t, in FP64.  FIR_LANES consecutive lanes share a bin, each
// summing one run of the taps with cos(j theta) stepped by the three-term
// recurrence cos((j+1) theta) = 2 cos(theta) cos(j theta) - cos((j-1) theta)
// from two cosines of exactly reduced angles (2 k j mod 2t over t), then a
// shuffle reduction: the 2000th-order band at t = 8192 is 4097 bins, and one
// lane per bin (a 1000-step dependent chain) took 46 us in 17 work-groups.
constexpr int FIR_LANES = 8;
template <class R>
__global__ __launch_bounds__(256) void fir_weights_kernel(const FirJob *jobs)
{
    const FirJob j = jobs[blockIdx.y];
    const int k = (blockIdx.x * 256 + threadIdx.x) / FIR_LANES, part = threadIdx.x % FIR_LANES;
    if (2 * k > j.t)
        return;  // past t / 2: the bin's FIR_LANES lanes all leave (the reduction stays within a bin)
    const int per = (j.half + FIR_LANES - 1) / FIR_LANES;
    const int lo = 1 + part * per, hi = min(j.half, lo + per - 1);
    const int64_t t2 = 2 * (int64_t)j.t;
    double acc = 0.0;
    if (lo <= hi) {
        double cm = cospi((double)((2 * (int64_t)k * lo) % t2) / (double)j.t);         // cos(lo theta)
        double cp = cospi((double)((2 * (int64_t)k * (lo - 1)) % t2) / (double)j.t);   // cos((lo - 1) theta)
        const double c2 = 2.0 * cospi((double)((2 * (int64_t)k) % t2) / (double)j.t);
        for (int m = lo; m <= hi; ++m) {
            acc = fma(j.c[m], cm, acc);
            const double cn = fma(c2, cm, -cp);
            cp = cm;
            cm = cn;
        }
    }
#pragma unroll
    for (int off = FIR_LANES / 2; off >= 1; off >>= 1)
        acc += __shfl_xor(acc, off, FIR_LANES);
    if (part == 0) {
        const double amp = j.c[0] + 2.0 * acc;
        ((R *)j.w)[k] = (R)(amp * amp);
    }
}

}  // namespace

hipError_t launch_fir_weights(bool f64, const FirJob *jobs, int njobs, int max_t, hipStream_t s)
{
    if (njobs <= 0)
        return hipSuccess;
    if (njobs > 65535 || max_t < 1)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)(((int64_t)(max_t / 2 + 1) * FIR_LANES + 255) / 256), (unsigned)njobs);
    if (f64)
        fir_weights_kernel<double><<<grid, 256, 0, s>>>(jobs);
    else
        fir_weights_kernel<float><<<grid, 256, 0, s>>>(jobs);
    return hipGetLastError();
}

hipError_t launch_chirps(bool f64, int logm, const ChirpJob *jobs, int njobs, hipStream_t s)
{
    if (njobs <= 0)
        return hipSuccess;
    return dispatch_any(f64, logm, 0, 0, nullptr, jobs, njobs, 0, s);
}

hipError_t launch_band_synth(int mode, const HilbertArgs &a, int njobs, hipStream_t s)
{
    if (njobs <= 0)
        return hipSuccess;
    if (mode < M_F64 || mode > M_F16 || a.nprob <= 0 || !a.synth_prefix)
        return hipErrorInvalidValue;
    switch (mode) {
    case M_F64: band_synth_kernel<double><<<njobs, 256, 0, s>>>(a, mode); break;
    case M_F32: band_synth_mfma_kernel<M_F32><<<njobs, 256, 0, s>>>(a); break;
    case M_SPLIT: band_synth_mfma_kernel<M_SPLIT><<<njobs, 256, 0, s>>>(a); break;
    case M_BF16: band_synth_mfma_kernel<M_BF16><<<njobs, 256, 0, s>>>(a); break;
    default: band_synth_mfma_kernel<M_F16><<<njobs, 256, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

int fft_wg_per_cu(bool f64, int logm)
{
    const size_t lds = f64 ? (size_t)(buf_elems(logm) + ptab_lds_elems<double>(logm)) * 16
                           : (size_t)(buf_elems(logm) + ptab_lds_elems<float>(logm)) * 8;
    return (int)std::max<size_t>(1, std::min<size_t>(16, (size_t)160 * 1024 / lds));
}

hipError_t launch_hilbert(int mode, const HilbertArgs &a, int cus, hipStream_t s)
{
    if (a.nrows <= 0)
        return hipSuccess;
    if (mode < M_F64 || mode > M_F16)
        return hipErrorInvalidValue;
    return dispatch_any(mode == M_F64, a.logm, 1, mode, &a, nullptr, 0, cus, s);
}

hipError_t launch_hilbert_adjoint(bool f64, const HilbertArgs &a, int cus, hipStream_t s)
{
    if (a.nrows <= 0)
        return hipSuccess;
    return dispatch_any(f64, a.logm, 2, f64 ? M_F64 : M_F32, &a, nullptr, 0, cus, s);
}

}  // namespace plv
