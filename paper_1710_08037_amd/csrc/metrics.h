// metrics.h -- the three phase-synchrony measures of one entry of G and their
// symmetric store.  Shared by the epilogue kernel (multi-chunk problems) and
// the Gram kernel's fused store (single-chunk problems), so both write
// bit-identical results.
//
//   PLV   = |G|                             (Eq. 2 / Eq. 7)
//   iPLV  = |Im G|                          (Section II.C, Eq. 13)
//   ciPLV = |Im G| / sqrt((1-Re)(1+Re))     (Eq. 14; FP64 radicand, 0 if <= 0)
//
// The ciPLV radicand is always formed in FP64.  For FP32 outputs the roots
// are taken in FP32 with the hardware square root and reciprocal square root
// (about 1 ulp each): the FP64 root and division cost the single-chunk Gram
// kernel a sixth of its time when K is short.
//
// Each is written at (i, j) and (j, i); the diagonal gets PLV = 1, iPLV = ciPLV = 0
// and the computed G_ii.  G is written as G_ij and G_ji = conj(G_ij), so every
// output is exactly symmetric (Hermitian for G).
#pragma once

#include "plv_internal.h"

namespace plv {

template <int MODE>
struct OutT {
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
};

// The three measures of an off-diagonal entry from r, m = Re and Im of G_ij
// (already divided by T).
template <int MODE>
__device__ inline void measures(double r, double m, typename OutT<MODE>::real_t &vp, typename OutT<MODE>::real_t &vi,
                                typename OutT<MODE>::real_t &vc)
{
    const double dd = (1.0 - r) * (1.0 + r);  // FP64: 1 - Re cancels
    if constexpr (MODE == M_F64) {
        const double am = fabs(m);
        vp = sqrt(r * r + m * m);
        vi = am;
        vc = dd > 0.0 ? am / sqrt(dd) : 0.0;
    } else {
        // FP32 outputs: the roots in FP32.  Components below 2^-60 are scaled
        // by 2^64 first (exact both ways), so no square underflows.  A
        // positive dd is at least about 2^-54 (1 +- Re of an FP64 Re), a
        // normal FP32 number.
        const float rf = (float)r, mf = (float)m;
        const float am = fabsf(mf);
        const bool tiny = fmaxf(fabsf(rf), am) < 0x1p-60f;
        const float sc = tiny ? 0x1p64f : 1.0f, isc = tiny ? 0x1p-64f : 1.0f;
        const float a = rf * sc, b = mf * sc;
        vp = __builtin_amdgcn_sqrtf(fmaf(a, a, b * b)) * isc;
        vi = am;
        vc = dd > 0.0 ? (am * sc) * __builtin_amdgcn_rsqf((float)dd) * isc : 0.0f;
    }
}

// Off-diagonal entry: r, m are Re and Im of G_ij (already divided by T),
// ij and ji the flat indices of (i, j) and (j, i).
template <int MODE>
__device__ inline void store_pair(const GramDesc &d, int64_t ij, int64_t ji, double r, double m)
{
    typedef typename OutT<MODE>::real_t real_t;
    typedef typename OutT<MODE>::cplx_t cplx_t;
    auto plv = gptr((real_t *)d.plv), iplv = gptr((real_t *)d.iplv), ciplv = gptr((real_t *)d.ciplv);
    auto g = gptr((cplx_t *)d.g);
    real_t vp, vi, vc;
    measures<MODE>(r, m, vp, vi, vc);
    if (plv) {
        plv[ij] = vp;
        plv[ji] = vp;
    }
    if (iplv) {
        iplv[ij] = vi;
        iplv[ji] = vi;
    }
    if (ciplv) {
        ciplv[ij] = vc;
        ciplv[ji] = vc;
    }
    if (g) {
        cplx_t v;
        v.x = (real_t)r;
        v.y = (real_t)m;
        g[ij] = v;
        v.y = (real_t)(-m);
        g[ji] = v;
    }
}

// One entry only, no mirror: the measures of G (r, m = Re and Im of the
// upper-triangle entry, already divided by T), or the diagonal's 1 / 0 / 0;
// G as given, or its conjugate when `conj` (the mirrored entry).  The
// measures never see the sign of m, so an entry and its mirror get
// bit-identical values from the same (r, m).
template <int MODE>
__device__ inline void store_one(const GramDesc &d, int64_t idx, bool diag, bool conj, double r, double m)
{
    typedef typename OutT<MODE>::real_t real_t;
    typedef typename OutT<MODE>::cplx_t cplx_t;
    auto plv = gptr((real_t *)d.plv), iplv = gptr((real_t *)d.iplv), ciplv = gptr((real_t *)d.ciplv);
    auto g = gptr((cplx_t *)d.g);
    real_t vp = (real_t)1, vi = (real_t)0, vc = (real_t)0;
    if (!diag)
        measures<MODE>(r, m, vp, vi, vc);
    if (plv)
        plv[idx] = vp;
    if (iplv)
        iplv[idx] = vi;
    if (ciplv)
        ciplv[idx] = vc;
    if (g) {
        cplx_t v;
        v.x = (real_t)r;
        v.y = conj ? (real_t)(-m) : (real_t)m;
        g[idx] = v;
    }
}

// One entry's outputs as store_one writes them, for a four-entry store: the
// measures (diagonal: 1, 0, 0) and G's components (Im negated for a
// mirrored entry), placed at position q of each vector.
template <int MODE>
__device__ inline void entry_of(bool diag, bool conj, double r, double m, int q, vf4 &vp, vf4 &vi, vf4 &vc,
                                vf4 &g01, vf4 &g23)
{
    static_assert(MODE != M_F64, "FP32 outputs only");
    float p = 1.0f, i = 0.0f, c = 0.0f;
    if (!diag)
        measures<MODE>(r, m, p, i, c);
    vp[q] = p;
    vi[q] = i;
    vc[q] = c;
    const float gr = (float)r, gi = conj ? (float)(-m) : (float)m;
    vf4 &g = q < 2 ? g01 : g23;
    g[2 * (q & 1)] = gr;
    g[2 * (q & 1) + 1] = gi;
}

// Four consecutive entries idx .. idx + 3 of one output row (entry_of):
// idx a multiple of 4 and every output 16-byte aligned, so each output takes
// one 16-byte store (G two) in place of four 4-byte ones -- the vector-memory
// path takes a 64-lane store in about the same time whether a lane writes 4
// or 16 bytes.
__device__ inline void store_four(const GramDesc &d, int64_t idx, const vf4 &vp, const vf4 &vi, const vf4 &vc,
                                  const vf4 &g01, const vf4 &g23)
{
    if (d.plv)
        *(PLV_GLOBAL vf4 *)(gptr((float *)d.plv) + idx) = vp;
    if (d.iplv)
        *(PLV_GLOBAL vf4 *)(gptr((float *)d.iplv) + idx) = vi;
    if (d.ciplv)
        *(PLV_GLOBAL vf4 *)(gptr((float *)d.ciplv) + idx) = vc;
    if (d.g) {
        auto g = (PLV_GLOBAL vf4 *)(gptr((float *)d.g) + 2 * idx);
        g[0] = g01;
        g[1] = g23;
    }
}

// r, m: Re and Im of G_ij (already divided by T); gi <= gj < d.n.
template <int MODE>
__device__ inline void store_entry(const GramDesc &d, int64_t gi, int64_t gj, double r, double m)
{
    typedef typename OutT<MODE>::real_t real_t;
    typedef typename OutT<MODE>::cplx_t cplx_t;
    const int64_t n = d.n;
    const int64_t ij = gi * n + gj;
    if (gi == gj) {
        auto plv = gptr((real_t *)d.plv), iplv = gptr((real_t *)d.iplv), ciplv = gptr((real_t *)d.ciplv);
        auto g = gptr((cplx_t *)d.g);
        if (plv) plv[ij] = (real_t)1;
        if (iplv) iplv[ij] = (real_t)0;
        if (ciplv) ciplv[ij] = (real_t)0;
        if (g) {
            cplx_t v;
            v.x = (real_t)r;
            v.y = (real_t)m;
            g[ij] = v;
        }
        return;
    }
    store_pair<MODE>(d, ij, gj * n + gi, r, m);
}

}  // namespace plv
