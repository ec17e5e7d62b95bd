// epilogue.hip -- chunk sum + metrics + mirrored store for problems whose T
// spans several K-chunks (single-chunk problems get the same store fused into
// the Gram kernel).
//
// For each upper-triangle tile: G_ij = (1/T) sum_s partial_s(i, j), the slots
// added in index order in FP64 (deterministic; no float atomics), T the true
// window length; then the measures of Eqs. 2, 13 and 14 at (i, j) and (j, i)
// (metrics.h).
//
// Each work-group covers EPB = 256 elements (two rows) of one tile, one per
// thread, so that every thread has all its slot loads in flight at once and
// even a small problem spreads over many CUs; reads of the partial sums are
// contiguous along j.  Where the rows allow 16-byte stores the row-wise
// variant below takes over (same sums, same measures).
#include "metrics.h"

namespace plv {
namespace {

constexpr int EPB = 256;  // tile elements per work-group (one per thread)

template <int MODE>
__global__ __launch_bounds__(256) void epilogue_kernel(EpiArgs args)
{
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
    const int BM = d.bm;
    if ((int)blockIdx.y * EPB >= BM * BM)
        return;  // the grid covers the largest tile of the launch

    auto part = gptr((const double *)d.partial + (int64_t)tile * 2 * BM * BM);
    const int64_t cstride = (int64_t)d.nupper * 2 * BM * BM;
    const double inv_t = 1.0 / (double)d.t;
    const int64_t n = d.n;

    {
        const int e = blockIdx.y * EPB + threadIdx.x;
        const int lbm = BM == 64 ? 6 : 7;  // the tile edges are 64 and 128
        const int i = e >> lbm, j = e & (BM - 1);
        const int64_t gi = (int64_t)I * BM + i, gj = (int64_t)J * BM + j;
        if (gi >= n || gj >= n || gi > gj)
            return;
        // slots added in index order; loads issued eight at a time so the
        // sum is not a chain of dependent memory latencies
        double sr = 0.0, si = 0.0;
        int c = 0;
        for (; c + 8 <= d.nslot; c += 8) {
            double vr[8], vi[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                vr[k] = part[(c + k) * cstride + e];
                vi[k] = part[(c + k) * cstride + BM * BM + e];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sr += vr[k];
                si += vi[k];
            }
        }
        for (; c < d.nslot; ++c) {
            sr += part[c * cstride + e];
            si += part[c * cstride + BM * BM + e];
        }
        if (args.coherence) {
            // C = S_ij / sqrt(S_ii S_jj) with the same fixed-order sums on the
            // diagonal (so C_ii = 1 exactly); 0 where a row is all zero
            const double den = sqrt(d.diag[gi]) * sqrt(d.diag[gj]);
            store_entry<MODE>(d, gi, gj, den > 0.0 ? sr / den : 0.0, den > 0.0 ? si / den : 0.0);
        } else {
            store_entry<MODE>(d, gi, gj, sr * inv_t, si * inv_t);
        }
    }
}

// Row-wise variant, for FP32 outputs with n a multiple of 4 and 16-byte
// aligned outputs: a work-group takes an ESB x ESB sub-block
// of an upper tile, sums its slots into LDS (in index order, as
// epilogue_kernel does, so the values are the same), then writes the
// sub-block and its mirror row by row, four entries per 16-byte store
// (store_four) -- epilogue_kernel writes each mirrored entry with a 4-byte
// store down a column.  A sub-block on the tile's diagonal is one pass over
// its square, the entries below the diagonal from the conjugate of their
// mirror; the sub-blocks below it are left to their mirrors.
constexpr int ESB = 32;  // sub-block edge: 32 rows x 8 four-entry groups = 256 threads
template <int MODE>
__global__ __launch_bounds__(256) void epilogue_rows_kernel(EpiArgs args)
{
    __shared__ double lr[ESB][ESB + 1], li[ESB][ESB + 1];  // padded: column reads spread over the banks
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
    const int BM = d.bm, nsub = BM / ESB;
    if ((int)blockIdx.y >= nsub * nsub)
        return;  // the grid covers the largest tile of the launch
    const int sa = blockIdx.y / nsub, sb = blockIdx.y % nsub;
    if (I == J && sa > sb)
        return;  // below the diagonal: written as the mirror of (sb, sa)
    const int64_t n = d.n;
    const int64_t gi0 = (int64_t)I * BM + sa * ESB, gj0 = (int64_t)J * BM + sb * ESB;
    if (gi0 >= n || gj0 >= n)
        return;  // every entry past n

    auto part = gptr((const double *)d.partial + (int64_t)tile * 2 * BM * BM);
    const int64_t cstride = (int64_t)d.nupper * 2 * BM * BM;
    const double inv_t = 1.0 / (double)d.t;
    for (int e = threadIdx.x; e < ESB * ESB; e += 256) {
        const int a = e / ESB, b = e % ESB;
        const int64_t idx = (int64_t)(sa * ESB + a) * BM + sb * ESB + b;
        double sr = 0.0, si = 0.0;
        int c = 0;
        for (; c + 8 <= d.nslot; c += 8) {
            double vr[8], vi[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                vr[k] = part[(c + k) * cstride + idx];
                vi[k] = part[(c + k) * cstride + BM * BM + idx];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sr += vr[k];
                si += vi[k];
            }
        }
        for (; c < d.nslot; ++c) {
            sr += part[c * cstride + idx];
            si += part[c * cstride + BM * BM + idx];
        }
        if (args.coherence) {  // as epilogue_kernel: S_ij / sqrt(S_ii S_jj), 0 where a row is all zero
            const double den = sqrt(d.diag[gi0 + a]) * sqrt(d.diag[gj0 + b]);
            lr[a][b] = den > 0.0 ? sr / den : 0.0;
            li[a][b] = den > 0.0 ? si / den : 0.0;
        } else {
            lr[a][b] = sr * inv_t;
            li[a][b] = si * inv_t;
        }
    }
    __syncthreads();

    const int a = threadIdx.x / (ESB / 4), b = (threadIdx.x % (ESB / 4)) * 4;
    const bool dsub = I == J && sa == sb;
    {  // the sub-block's rows (a diagonal sub-block: its whole square)
        const int64_t gr = gi0 + a, gc = gj0 + b;
        if (gr < n && gc < n) {  // n and gc multiples of 4: all four entries inside
            vf4 vp, vi, vc, g01, g23;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool lower = dsub && b + q < a;
                entry_of<MODE>(gr == gc + q, lower, lower ? lr[b + q][a] : lr[a][b + q],
                               lower ? li[b + q][a] : li[a][b + q], q, vp, vi, vc, g01, g23);
            }
            store_four(d, gr * n + gc, vp, vi, vc, g01, g23);
        }
    }
    if (!dsub) {  // the mirror: row gj0 + a, entry q the conjugate of (b + q, a); never diagonal
        const int64_t gr = gj0 + a, gc = gi0 + b;
        if (gr < n && gc < n) {
            vf4 vp, vi, vc, g01, g23;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                entry_of<MODE>(false, true, lr[b + q][a], li[b + q][a], q, vp, vi, vc, g01, g23);
            store_four(d, gr * n + gc, vp, vi, vc, g01, g23);
        }
    }
}

// d[i] = sum over slots (in index order) of Re G(i, i), read from the
// partials of diagonal tile (I, I), I = i / BM: the same sums the epilogue
// forms for the diagonal entry.
template <int MODE>
__global__ __launch_bounds__(256) void diag_kernel(GramDesc d)
{
    const int BM = d.bm;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= d.n)
        return;
    const int I = i / BM, r = i - I * BM;
    const int tile = I * d.ntile - I * (I - 1) / 2;  // row-major upper index of (I, I)
    auto part = gptr((const double *)d.partial + (int64_t)tile * 2 * BM * BM + (int64_t)r * BM + r);
    const int64_t cstride = (int64_t)d.nupper * 2 * BM * BM;
    double s = 0.0;
    for (int c = 0; c < d.nslot; ++c)
        s += part[c * cstride];
    gptr(d.diag)[i] = s;
}

}  // namespace

hipError_t launch_diag(int mode, const GramDesc &g, hipStream_t s)
{
    const int grid = (g.n + 255) / 256;
    switch (mode) {
    case M_F64: diag_kernel<M_F64><<<grid, 256, 0, s>>>(g); break;
    case M_F32: diag_kernel<M_F32><<<grid, 256, 0, s>>>(g); break;
    case M_SPLIT: diag_kernel<M_SPLIT><<<grid, 256, 0, s>>>(g); break;
    case M_BF16: diag_kernel<M_BF16><<<grid, 256, 0, s>>>(g); break;
    case M_F16: diag_kernel<M_F16><<<grid, 256, 0, s>>>(g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_epilogue(int mode, const EpiArgs &a, int ntiles, int bm_max, bool rows, hipStream_t s)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (rows) {
        if (mode == M_F64)
            return hipErrorInvalidValue;
        dim3 grid(ntiles, (bm_max / ESB) * (bm_max / ESB));
        switch (mode) {
        case M_F32: epilogue_rows_kernel<M_F32><<<grid, 256, 0, s>>>(a); break;
        case M_SPLIT: epilogue_rows_kernel<M_SPLIT><<<grid, 256, 0, s>>>(a); break;
        case M_BF16: epilogue_rows_kernel<M_BF16><<<grid, 256, 0, s>>>(a); break;
        case M_F16: epilogue_rows_kernel<M_F16><<<grid, 256, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 grid(ntiles, bm_max * bm_max / EPB);
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
