// dft.hip -- the DFT bins of narrow bands as a matrix product on MFMA
// (Section II.A, Eq. 3: the analytic signal of a band needs only the row's
// DFT at the band's bins).
//
// For a problem whose bands are all narrow (each a few dozen bins, the
// uneven-batch case), the bins of every band come straight from
//   X_k = sum_{t < T} x_t exp(-2 pi i k t / T),
// a product X [rows x bins] = x [rows x T] . W [T x bins], instead of a whole
// FFT of the row (for T not a power of two a Bluestein transform of size
// M >= 2T - 1: two size-M FFTs for the few bins kept).  Real arithmetic: the
// columns of W are cos and -sin of 2 pi (k t mod T) / T, i.e. the root table
// exp(2 pi i m / T) of the row length, conjugated.  FP32 products and sums on
// v_mfma_f32_16x16x4f32; the bins then go to the band synthesis as the
// transform kernel's bins do.
//
// One work-group: 64 rows of one problem (a 16-row block per wave) and every
// column (2 per bin, at most 12 blocks of 16).  T runs in chunks of 64
// samples: the work-group writes the chunk's W columns into LDS ([column]
// [sample], each thread a run of 16 samples of one bin, the root index
// stepped by k mod T), then each wave contracts its rows' 64 samples against
// every column block.  A lane holds 4 consecutive samples of one row as its A
// operand of 4 MFMA steps; the K index of a step is (lane / 16) -> sample
// 4 (lane / 16) + step of the 16-sample group, and B is read with the same map.
#include "phasor.h"

namespace plv {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DFT_ROWS = 64;              // rows per work-group
constexpr int DFT_TC = 64;                // samples per table chunk
constexpr int DFT_CB = DFT_MAX_BINS / 8;  // column blocks of 16 (two columns per bin)
constexpr int DFT_PITCH = DFT_TC + 4;     // LDS row of one column (floats)

__global__ __launch_bounds__(256) void dft_bins_kernel(HilbertArgs a)
{
    __shared__ __attribute__((aligned(16))) float wt[DFT_CB * 16][DFT_PITCH];
    __shared__ int kv[DFT_MAX_BINS];   // bin k of column pair j
    __shared__ int dst[DFT_MAX_BINS];  // its slot b * DIRECT_KMAX + m in the row's bins

    // ---- which (problem, row block): scalar binary search of the running counts
    const int job = blockIdx.x;
    int lo = 0, hi = a.nprob;  // prefix[lo] <= job < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.dft_prefix[mid] <= job)
            lo = mid;
        else
            hi = mid;
    }
    const int q = lo;
    const HilbertProb hp = a.hp[q];
    const int r0 = (job - a.dft_prefix[q]) * DFT_ROWS;
    const int t = hp.t;
    const int tid = threadIdx.x;

    // ---- the bins of every band (the host admits problems with at most
    // DFT_MAX_BINS of them, every band narrow)
    int nkt = 0;
    for (int b = 0; b < hp.nbands; ++b) {
        const BandBins bb = a.bins[hp.bin0 + b];
        const int nk = bb.khi >= bb.klo ? bb.khi - bb.klo + 1 : 0;
        for (int m = tid; m < nk; m += 256) {
            kv[nkt + m] = bb.klo + m;
            dst[nkt + m] = b * DIRECT_KMAX + m;
        }
        nkt += nk;
    }
    const int ncb = (2 * nkt + 15) / 16;  // column blocks in use (<= DFT_CB)
    for (int e = tid; e < DFT_CB * 16 * DFT_PITCH; e += 256)
        (&wt[0][0])[e] = 0.0f;  // padding columns stay 0
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int row = r0 + wave * 16 + (lane & 15);
    const bool live = row < hp.n;
    auto xr = gptr((const float *)hp.x) + (int64_t)(live ? row : 0) * hp.ld;
    const vf2 *roots = (const vf2 *)hp.roots;
    // table writers: thread (pair j, quarter qq) writes samples 16 qq .. 16 qq + 15
    const int wj = tid % DFT_MAX_BINS, wq = tid / DFT_MAX_BINS;  // wq < 256 / DFT_MAX_BINS
    constexpr int NQ = 256 / DFT_MAX_BINS;                      // writer threads per bin
    constexpr int RUN = DFT_TC / NQ;                            // samples per writer per chunk
    static_assert(256 % DFT_MAX_BINS == 0 && DFT_TC % NQ == 0, "writer split");
    const int kj = wj < nkt ? kv[wj] : 0;

    f32x4 acc[DFT_CB];
#pragma unroll
    for (int c = 0; c < DFT_CB; ++c)
        acc[c] = f32x4{0, 0, 0, 0};

    for (int c0 = 0; c0 < t; c0 += DFT_TC) {
        __syncthreads();  // the previous chunk's columns are read
        if (wj < nkt) {
            // all RUN gathers in flight at once, then the LDS writes
            const int s0 = c0 + wq * RUN;
            uint32_t idx = ((uint32_t)kj * (uint32_t)s0) % (uint32_t)t;  // < 2^31: k <= t/2, s0 < t
            vf2 rv[RUN];
#pragma unroll
            for (int u = 0; u < RUN; ++u) {
                rv[u] = gptr(roots)[idx];
                idx += (uint32_t)kj;
                idx = idx >= (uint32_t)t ? idx - (uint32_t)t : idx;
            }
#pragma unroll
            for (int u = 0; u < RUN; ++u) {
                const bool in = s0 + u < t;
                wt[2 * wj][wq * RUN + u] = in ? rv[u].x : 0.0f;        // Re W = cos
                wt[2 * wj + 1][wq * RUN + u] = in ? -rv[u].y : 0.0f;   // Im W = -sin
            }
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < DFT_TC / 16; ++g) {
            const int sl = g * 16 + 4 * (lane >> 4);  // this lane's 4 samples in the chunk
            float xv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int ts = c0 + sl + s;
                xv[s] = (live && ts < t) ? xr[ts] : 0.0f;
            }
#pragma unroll
            for (int c = 0; c < DFT_CB; ++c) {
                if (c < ncb) {
                    const vf4 wv = *(const vf4 *)&wt[c * 16 + (lane & 15)][sl];
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[s], wv[s], acc[c], 0, 0, 0);
                }
            }
        }
    }

    // ---- lane l, register r: row 4 (l / 16) + r of the wave's block, column
    // 16 c + l % 16 = bin pair (re, im)
    auto out = gptr((float *)hp.xbins);
    const int64_t xrow = (int64_t)hp.nbands * DIRECT_KMAX;  // complex bins per row
#pragma unroll
    for (int c = 0; c < DFT_CB; ++c) {
        if (c >= ncb)
            continue;
        const int col = c * 16 + (lane & 15), j = col >> 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = r0 + wave * 16 + 4 * (lane >> 4) + r;
            if (j < nkt && rr < hp.n)
                out[((int64_t)rr * xrow + dst[j]) * 2 + (col & 1)] = acc[c][r];
        }
    }
}

}  // namespace

hipError_t launch_dft_bins(const HilbertArgs &a, int njobs, hipStream_t s)
{
    if (njobs <= 0)
        return hipSuccess;
    dft_bins_kernel<<<njobs, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace plv
