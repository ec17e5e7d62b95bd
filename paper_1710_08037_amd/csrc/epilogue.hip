// epilogue.hip -- chunk sum + metrics + mirrored store.
//
// For each upper-triangle tile: G_ij = (1/T) sum_s partial_s(i, j), the slots
// added in index order in FP64 (deterministic; no float atomics), T the true
// window length.  Then
//   PLV = |G|                               (Eq. 2 / Eq. 7)
//   iPLV = |Im G|                           (Section II.C, Eq. 13)
//   ciPLV = |Im G| / sqrt((1-Re)(1+Re))     (Eq. 14; FP64 radicand, 0 if <= 0)
// written at (i, j) and (j, i); the diagonal gets PLV = 1, iPLV = ciPLV = 0
// and the computed G_ii.  G is written as G_ij and G_ji = conj(G_ij), so every
// output is exactly symmetric (Hermitian for G).
//
// Each work-group covers 1024 elements (8 rows) of one tile so that even a
// small problem spreads over many CUs; reads of the partial sums are
// contiguous along j.
#include "plv_internal.h"

namespace plv {
namespace {

template <int MODE>
__global__ __launch_bounds__(256) void epilogue_kernel(EpiArgs args)
{
    constexpr int BM = tile_of(MODE);
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;

    GramDesc d;
    int tile;
    if (args.tiles) {
        const TileRef tr = args.tiles[blockIdx.x];
        d = args.gd[tr.gram];
        tile = tr.tile;
    } else {
        d = args.g;
        tile = blockIdx.x;
    }
    int I = 0, base = 0;
    while (tile >= base + (d.ntile - I)) {
        base += d.ntile - I;
        ++I;
    }
    const int J = I + (tile - base);

    auto part = gptr((const double *)d.partial + (int64_t)tile * 2 * BM * BM);
    const int64_t cstride = (int64_t)d.nupper * 2 * BM * BM;
    const double inv_t = 1.0 / (double)d.t;
    const int64_t n = d.n;
    auto plv = gptr((real_t *)d.plv), iplv = gptr((real_t *)d.iplv), ciplv = gptr((real_t *)d.ciplv);
    auto g = gptr((cplx_t *)d.g);

#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = blockIdx.y * 1024 + k * 256 + threadIdx.x;
        const int i = e / BM, j = e - (e / BM) * BM;
        const int64_t gi = (int64_t)I * BM + i, gj = (int64_t)J * BM + j;
        if (gi >= n || gj >= n || gi > gj)
            continue;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < d.nslot; ++c) {
            sr += part[c * cstride + e];
            si += part[c * cstride + BM * BM + e];
        }
        const double r = sr * inv_t, m = si * inv_t;
        const int64_t ij = gi * n + gj, ji = gj * n + gi;
        if (gi == gj) {
            if (plv) plv[ij] = (real_t)1;
            if (iplv) iplv[ij] = (real_t)0;
            if (ciplv) ciplv[ij] = (real_t)0;
            if (g) {
                cplx_t v;
                v.x = (real_t)r;
                v.y = (real_t)m;
                g[ij] = v;
            }
            continue;
        }
        const double am = fabs(m);
        const double dd = (1.0 - r) * (1.0 + r);
        const real_t vp = (real_t)sqrt(r * r + m * m);
        const real_t vi = (real_t)am;
        const real_t vc = (real_t)(dd > 0.0 ? am / sqrt(dd) : 0.0);
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
}

}  // namespace

hipError_t launch_epilogue(int mode, const EpiArgs &a, int ntiles, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    const int bm = tile_of(mode);
    dim3 grid(ntiles, bm * bm / 1024);
    switch (mode) {
    case M_F64: epilogue_kernel<M_F64><<<grid, 256, 0, s>>>(a); break;
    case M_F32: epilogue_kernel<M_F32><<<grid, 256, 0, s>>>(a); break;
    case M_SPLIT: epilogue_kernel<M_SPLIT><<<grid, 256, 0, s>>>(a); break;
    case M_BF16: epilogue_kernel<M_BF16><<<grid, 256, 0, s>>>(a); break;
    case M_F16: epilogue_kernel<M_F16><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace plv
