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
// bin.  T runs in chunks of 64 samples, and with c0 the chunk's first sample
//   X_k = sum_c0 exp(-2 pi i k c0 / T) S_k(c0),
//   S_k(c0) = sum_{j < 64} x_{c0 + j} exp(-2 pi i k j / T),
// so one table C[j][k] = exp(-2 pi i k j / T) (64 samples x the bins, cos and
// -sin as two columns, in LDS) serves every chunk: it is written once per
// work-group from the row length's root table.  Per chunk each wave forms
// S for its 16 rows on MFMA and adds it into X rotated by the chunk's factor
// (VALU).  Column blocks come in pairs per 16 bins, the cos block then the
// -sin block, so a lane holds Re and Im of the same bin in two
// accumulators.  A lane holds 4 consecutive samples of one row as its A
// operand of 4 MFMA steps; the K index of a step is (lane / 16) -> sample
// 4 (lane / 16) + step of the 16-sample group, and B is read with the same
// map.  The samples reach that layout through LDS: each wave loads its 16
// rows one row per instruction (64 consecutive samples, coalesced) into its
// own LDS tile, and the next chunk's loads are in flight while the current
// one is contracted.
#include "phasor.h"

namespace plv {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DFT_ROWS = 64;              // rows per work-group
constexpr int DFT_TC = 64;                // samples per chunk
constexpr int DFT_BB = DFT_MAX_BINS / 16; // blocks of 16 bins (two column blocks each)
constexpr int DFT_PITCH = DFT_TC + 4;     // LDS row of one column (floats)

__global__ __launch_bounds__(256) void dft_bins_kernel(HilbertArgs a)
{
    __shared__ __attribute__((aligned(16))) float wt[DFT_BB * 32][DFT_PITCH];  // column 32 p + 16 h + u
    __shared__ __attribute__((aligned(16))) float xs[4][16][DFT_PITCH];        // each wave's rows of a chunk
    __shared__ int kv[DFT_MAX_BINS];   // bin k of bin slot j
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
    const int nbb = (nkt + 15) / 16;  // bin blocks in use (<= DFT_BB)
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int rw = r0 + wave * 16;  // the wave's first row
    const vf2 *roots = (const vf2 *)hp.roots;
    const int sl0 = 4 * (lane >> 4);  // this lane's first sample in each 16-sample group

    // chunk loads: instruction i takes row rw + i, lane l its sample c0 + l
    // (clamped addresses, values selected); the first chunk is in flight
    // while the table is written
    // Loads are unconditional (raw values, no control flow between a load
    // and the stage that consumes it, so they stay in flight across the
    // contraction); the mask is applied when the chunk is staged.
    auto xbase = gptr((const float *)hp.x);
    float xn[16];
    int cn = 0;  // first sample of the chunk in xn
    auto load_chunk = [&](int c0) {
        const int ts = min(c0 + lane, t - 1);
        cn = c0;
#pragma unroll
        for (int i = 0; i < 16; ++i)  // read once: streaming loads
            xn[i] = __builtin_nontemporal_load(&xbase[(int64_t)min(rw + i, hp.n - 1) * hp.ld + ts]);
    };
    auto stage_chunk = [&]() {  // this wave's tile; its own later reads see it
        const bool tin = cn + lane < t;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            xs[wave][i][lane] = (tin && rw + i < hp.n) ? xn[i] : 0.0f;
        __builtin_amdgcn_wave_barrier();
    };
    load_chunk(0);

    // ---- C: thread (bin slot j, quarter qq) writes samples 16 qq .. 16 qq + 15
    // of both columns of bin j (zero columns for unused slots)
    {
        constexpr int NQ = 256 / DFT_MAX_BINS;                      // writer threads per bin
        constexpr int RUN = DFT_TC / NQ;                            // samples per writer
        static_assert(NQ >= 1 && DFT_TC % NQ == 0, "writer split");
        const int wj = tid % DFT_MAX_BINS, wq = tid / DFT_MAX_BINS;  // wq < NQ for the writers
        const int colr = 32 * (wj >> 4) + (wj & 15);               // the cos column; -sin is 16 further
        if (wq < NQ && wj < nbb * 16) {
            const uint32_t kj = wj < nkt ? (uint32_t)kv[wj] : 0u;
            uint32_t idx = (kj * (uint32_t)(wq * RUN)) % (uint32_t)t;  // < 2^31: k <= t/2, j < 64
            vf2 rv[RUN];
#pragma unroll
            for (int u = 0; u < RUN; ++u) {
                rv[u] = gptr(roots)[idx];
                idx += kj;
                idx = idx >= (uint32_t)t ? idx - (uint32_t)t : idx;
            }
#pragma unroll
            for (int u = 0; u < RUN; ++u) {
                const bool in = wj < nkt;
                wt[colr][wq * RUN + u] = in ? rv[u].x : 0.0f;        // Re C = cos
                wt[colr + 16][wq * RUN + u] = in ? -rv[u].y : 0.0f;  // Im C = -sin
            }
        }
    }
    __syncthreads();

    // per bin block p: this lane's bin (lane % 16) and its chunk rotation index
    // k c0 mod T, stepped by k DFT_TC mod T per chunk (rix: the next chunk's)
    uint32_t kb[DFT_BB], rix[DFT_BB], rstep[DFT_BB];
#pragma unroll
    for (int p = 0; p < DFT_BB; ++p) {
        const int j = p * 16 + (lane & 15);
        kb[p] = j < nkt ? (uint32_t)kv[j] : 0u;
        rix[p] = 0;
        rstep[p] = (kb[p] * (uint32_t)DFT_TC) % (uint32_t)t;
    }
    f32x4 xre[DFT_BB], xim[DFT_BB];
#pragma unroll
    for (int p = 0; p < DFT_BB; ++p) {
        xre[p] = f32x4{0, 0, 0, 0};
        xim[p] = f32x4{0, 0, 0, 0};
    }

    // the chunk's rotation factors are loaded one chunk ahead, like its samples
    vf2 w[DFT_BB], wn[DFT_BB];
#pragma unroll
    for (int p = 0; p < DFT_BB; ++p)
        w[p] = vf2{1.0f, 0.0f};  // c0 = 0
    stage_chunk();
    float xv[DFT_TC / 16][4];
    for (int c0 = 0; c0 < t; c0 += DFT_TC) {
        // this lane's A operands of the chunk: row lane % 16, samples
        // 16 g + 4 (lane / 16) + s
#pragma unroll
        for (int g = 0; g < DFT_TC / 16; ++g) {
            const vf4 v = *(const vf4 *)&xs[wave][lane & 15][g * 16 + sl0];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                xv[g][s] = v[s];
        }
        __builtin_amdgcn_wave_barrier();
        if (c0 + DFT_TC < t) {
            load_chunk(c0 + DFT_TC);
#pragma unroll
            for (int p = 0; p < DFT_BB; ++p) {
                if (p < nbb) {
                    rix[p] += rstep[p];
                    rix[p] = rix[p] >= (uint32_t)t ? rix[p] - (uint32_t)t : rix[p];
                    wn[p] = gptr(roots)[rix[p]];
                }
            }
        }
#pragma unroll
        for (int p = 0; p < DFT_BB; ++p) {
            if (p >= nbb)
                break;
            f32x4 sr = f32x4{0, 0, 0, 0}, si = f32x4{0, 0, 0, 0};
#pragma unroll
            for (int g = 0; g < DFT_TC / 16; ++g) {
                const int sl = g * 16 + sl0;
                const vf4 wr = *(const vf4 *)&wt[32 * p + (lane & 15)][sl];
                const vf4 wi = *(const vf4 *)&wt[32 * p + 16 + (lane & 15)][sl];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    sr = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[g][s], wr[s], sr, 0, 0, 0);
                    si = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[g][s], wi[s], si, 0, 0, 0);
                }
            }
            // X += S exp(-2 pi i k c0 / T) = S conj(root[k c0 mod T])
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                xre[p][r] = fmaf(sr[r], w[p].x, fmaf(si[r], w[p].y, xre[p][r]));
                xim[p][r] = fmaf(si[r], w[p].x, fmaf(-sr[r], w[p].y, xim[p][r]));
            }
        }
        if (c0 + DFT_TC < t) {  // the next chunk's loads are waited for only here
            stage_chunk();
#pragma unroll
            for (int p = 0; p < DFT_BB; ++p)
                w[p] = wn[p];
        }
    }

    // ---- lane l, register r: row 4 (l / 16) + r of the wave's block, bin
    // slot 16 p + l % 16
    auto out = gptr((vf2 *)hp.xbins);
    const int64_t xrow = (int64_t)hp.nbands * DIRECT_KMAX;  // complex bins per row
#pragma unroll
    for (int p = 0; p < DFT_BB; ++p) {
        if (p >= nbb)
            break;
        const int j = p * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rr = r0 + wave * 16 + 4 * (lane >> 4) + r;
            if (j < nkt && rr < hp.n)
                out[(int64_t)rr * xrow + dst[j]] = vf2{xre[p][r], xim[p][r]};
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
