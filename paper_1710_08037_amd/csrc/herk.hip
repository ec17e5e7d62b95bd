// herk.hip -- the Gram contraction G = U U^H (Section II.A, Eqs. 5-7) on MFMA.
//
// One work-group computes one BM x BM tile (I, J), I <= J, of the upper
// triangle over one K-chunk of samples, and writes the tile's chunk sum
// (Re, Im as two BM x BM FP64 planes) to a slot of the partial buffer; the
// epilogue kernel adds the slots in a fixed order.  When T has more chunks
// than slots, the host launches several passes and pass p > 0 adds chunk
// p * nslot + s into slot s.  Only the upper triangle is computed:
// G_ji = conj(G_ij).
//
// Complex arithmetic on real MFMA.  Per sample the phasor is stored
// interleaved, p(t) = (Re u, Im u).  With q(t) = (Im u, -Re u):
//   Re G_ij = sum_t p_i(t) . p_j(t),   Im G_ij = sum_t q_i(t) . p_j(t)
// so a tile needs two real products that share the column operand, and q is
// made in registers from p (swap halves of each (re, im) pair, flip one sign).
// The 16-bit modes contract K' = 2T interleaved values with
// v_mfma_f32_16x16x32_{bf16,f16} (16 samples per instruction); the split mode
// adds the hi.lo and lo.hi cross products (three products; lo.lo dropped).
// FP32 and FP64 use v_mfma_{f32_16x16x4f32,f64_16x16x4f64} on the re and im
// lanes separately (4 samples per instruction, 4 products).
//
// Tiling (all modes): 256 threads = 4 waves in 2 x 2, each wave a
// (BM/2) x (BM/2) sub-tile made of 16 x 16 MFMA blocks.  Each K-stage stages
// 128 bytes per row (32 / 16 / 8 samples for 16-bit / f32 / f64) of the row
// panel I and the column panel J into LDS (row pitch 144 B: the 16 B pad makes
// the 16-lane fragment reads conflict-free), double-buffered with one barrier
// per stage and the next stage's global loads in flight during the MFMAs.
// A diagonal tile (I == J) loads one panel and uses it as both operands.
//
// Work-groups are handed out XCD-aware: the hardware deals work-group ids
// round-robin over the 8 XCDs, so ids are remapped to give each XCD a
// contiguous range of items (same chunk, neighbouring tiles), which keeps the
// shared row panels in that XCD's L2.
#include "plv_internal.h"

namespace plv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int ROWB = 128;  // bytes per row per K-stage
constexpr int LROW = 144;  // LDS row pitch

template <int MODE>
struct AccOf {
    typedef f32x4 type;
    typedef float scalar;
};
template <>
struct AccOf<M_F64> {
    typedef f64x4 type;
    typedef double scalar;
};

__device__ inline int xcd_remap(int wg, int nwg)
{
    constexpr int X = 8;
    const int q = nwg / X, r = nwg % X;
    const int x = wg % X, l = wg / X;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Upper-triangle tile index -> (I, J), row-major over I <= J.
__device__ inline void tile_ij(int tile, int nt, int &I, int &J)
{
    int i = 0, base = 0;
    while (tile >= base + (nt - i)) {
        base += nt - i;
        ++i;
    }
    I = i;
    J = i + (tile - base);
}

// (re, im) -> (im, -re) for each packed 16-bit pair.
__device__ inline u32x4 swap_neg(u32x4 v)
{
    u32x4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r[k] = __builtin_amdgcn_alignbit(v[k], v[k], 16) ^ 0x80000000u;
    return r;
}

template <int MODE>
__device__ inline f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c)
{
    if constexpr (MODE == M_F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                      c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <int MODE>
__global__ __launch_bounds__(256) void herk_kernel(HerkArgs args)
{
    constexpr int BM = tile_of(MODE);
    constexpr int NB = BM / 32;            // 16x16 blocks per wave side
    constexpr int CB = cbytes_of(MODE);
    constexpr int PL = planes_of(MODE);
    constexpr int BKC = ROWB / CB;         // samples per K-stage
    constexpr int PANEL = BM * LROW;       // one panel of one plane in LDS
    constexpr int STAGE = PL * 2 * PANEL;  // A and B panels of every plane
    constexpr int SEGS = BM * (ROWB / 16) / 256;  // 16-byte global loads per thread per panel
    typedef typename AccOf<MODE>::type acc_t;

    __shared__ __attribute__((aligned(16))) uint8_t smem[2 * STAGE];

    // ---- which item
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    GramDesc d;
    int tile, slot;
    if (args.items) {
        const Item it = args.items[item];
        d = args.gd[it.gram];
        tile = it.tile;
        slot = it.chunk;
    } else {
        d = args.g;
        slot = item / d.nupper;
        tile = item - slot * d.nupper;
    }
    const int chunk = args.pass * d.nslot + slot;
    int I, J;
    tile_ij(tile, d.ntile, I, J);
    const bool diag = (I == J);
    const int k0 = chunk * d.chunk;
    const int k1 = min(k0 + d.chunk, d.tpad);
    const int nst = (k1 - k0) / BKC;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // ---- global -> LDS staging
    const int64_t pitch = d.ldu * CB;
    const uint8_t *ga = d.u + (int64_t)I * BM * pitch + (int64_t)k0 * CB;
    const uint8_t *gb = d.u + (int64_t)J * BM * pitch + (int64_t)k0 * CB;
    const int lrow = tid >> 3, lseg = (tid & 7) * 16;

    u32x4 ra[PL][SEGS], rb[PL][SEGS];
    auto gload = [&](int st) {
        const int64_t off = (int64_t)st * ROWB + lseg;
#pragma unroll
        for (int p = 0; p < PL; ++p)
#pragma unroll
            for (int s = 0; s < SEGS; ++s)
                ra[p][s] = *(const u32x4 *)(ga + p * d.plane_bytes + (int64_t)(lrow + 32 * s) * pitch + off);
        if (!diag) {
#pragma unroll
            for (int p = 0; p < PL; ++p)
#pragma unroll
                for (int s = 0; s < SEGS; ++s)
                    rb[p][s] = *(const u32x4 *)(gb + p * d.plane_bytes + (int64_t)(lrow + 32 * s) * pitch + off);
        }
    };
    auto lstore = [&](int buf) {
        uint8_t *base = smem + buf * STAGE;
#pragma unroll
        for (int p = 0; p < PL; ++p)
#pragma unroll
            for (int s = 0; s < SEGS; ++s)
                *(u32x4 *)(base + p * 2 * PANEL + (lrow + 32 * s) * LROW + lseg) = ra[p][s];
        if (!diag) {
#pragma unroll
            for (int p = 0; p < PL; ++p)
#pragma unroll
                for (int s = 0; s < SEGS; ++s)
                    *(u32x4 *)(base + p * 2 * PANEL + PANEL + (lrow + 32 * s) * LROW + lseg) = rb[p][s];
        }
    };

    acc_t re[NB][NB], im[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            re[a][b] = acc_t{0, 0, 0, 0};
            im[a][b] = acc_t{0, 0, 0, 0};
        }

    const int arow = (wm * (BM / 2) + (lane & 15)) * LROW;
    const int brow = (wn * (BM / 2) + (lane & 15)) * LROW;
    const int bpanel = diag ? 0 : PANEL;

    auto compute = [&](int buf) {
        const uint8_t *As = smem + buf * STAGE;
        const uint8_t *Bs = As + bpanel;
        if constexpr (CB == 4) {
            // 16-bit modes: 2 sub-steps of 16 samples (K' = 32 values)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int off = ks * 64 + (lane >> 4) * 16;
                u32x4 vb[PL][NB];
#pragma unroll
                for (int p = 0; p < PL; ++p)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        vb[p][b] = *(const u32x4 *)(Bs + p * 2 * PANEL + brow + b * 16 * LROW + off);
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    u32x4 va[PL], vq[PL];
#pragma unroll
                    for (int p = 0; p < PL; ++p) {
                        va[p] = *(const u32x4 *)(As + p * 2 * PANEL + arow + a * 16 * LROW + off);
                        vq[p] = swap_neg(va[p]);
                    }
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        re[a][b] = mfma16<MODE>(va[0], vb[0][b], re[a][b]);
                        im[a][b] = mfma16<MODE>(vq[0], vb[0][b], im[a][b]);
                        if constexpr (PL == 2) {
                            re[a][b] = mfma16<MODE>(va[0], vb[1][b], re[a][b]);
                            im[a][b] = mfma16<MODE>(vq[0], vb[1][b], im[a][b]);
                            re[a][b] = mfma16<MODE>(va[1], vb[0][b], re[a][b]);
                            im[a][b] = mfma16<MODE>(vq[1], vb[0][b], im[a][b]);
                        }
                    }
                }
            }
        } else if constexpr (CB == 8) {
            // FP32: 4 sub-steps of 4 samples; one sample (re, im) per lane
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int off = ks * 32 + (lane >> 4) * 8;
                float2 vb[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    vb[b] = *(const float2 *)(Bs + brow + b * 16 * LROW + off);
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    const float2 va = *(const float2 *)(As + arow + a * 16 * LROW + off);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.x, vb[b].x, re[a][b], 0, 0, 0);
                        re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb[b].y, re[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb[b].x, im[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-va.x, vb[b].y, im[a][b], 0, 0, 0);
                    }
                }
            }
        } else {
            // FP64: 2 sub-steps of 4 samples; one sample (re, im) per lane
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int off = ks * 64 + (lane >> 4) * 16;
                double2 vb[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    vb[b] = *(const double2 *)(Bs + brow + b * 16 * LROW + off);
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    const double2 va = *(const double2 *)(As + arow + a * 16 * LROW + off);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.x, vb[b].x, re[a][b], 0, 0, 0);
                        re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.y, vb[b].y, re[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.y, vb[b].x, im[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-va.x, vb[b].y, im[a][b], 0, 0, 0);
                    }
                }
            }
        }
    };

    // ---- K loop: double-buffered LDS, one barrier per stage
    if (nst > 0) {
        gload(0);
        lstore(0);
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            if (st + 1 < nst)
                gload(st + 1);
            compute(st & 1);
            if (st + 1 < nst)
                lstore((st + 1) & 1);
            __syncthreads();
        }
    }

    // ---- chunk sum of this tile -> partial[slot][tile][re|im][BM][BM] (FP64).
    // A chunk spans at most a few thousand samples, which bounds the FP32
    // accumulation error; later passes over a long T add into the same slot.
    // Accumulator layout of a 16x16 block: lane l, register r holds column
    // l % 16 of row 4 (l / 16) + r for the FP32-output MFMAs, and of row
    // l / 16 + 4 r for v_mfma_f64_16x16x4f64.
    double *out = d.partial + ((int64_t)slot * d.nupper + tile) * 2 * BM * BM;
    const int r0 = wm * (BM / 2) + (MODE == M_F64 ? (lane >> 4) : (lane >> 4) * 4);
    constexpr int RSTEP = (MODE == M_F64) ? 4 : 1;
    const int c0 = wn * (BM / 2) + (lane & 15);
    const bool acc_in = args.pass > 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = (r0 + a * 16 + r * RSTEP) * BM + c0 + b * 16;
                double vr = (double)re[a][b][r], vi = (double)im[a][b][r];
                if (acc_in) {
                    vr += out[e];
                    vi += out[BM * BM + e];
                }
                out[e] = vr;
                out[BM * BM + e] = vi;
            }
}

template <int MODE>
int occupancy_of()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, herk_kernel<MODE>, 256, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace

hipError_t launch_herk(int mode, const HerkArgs &a, int nwg, hipStream_t s)
{
    if (nwg <= 0)
        return hipSuccess;
    switch (mode) {
    case M_F64: herk_kernel<M_F64><<<nwg, 256, 0, s>>>(a); break;
    case M_F32: herk_kernel<M_F32><<<nwg, 256, 0, s>>>(a); break;
    case M_SPLIT: herk_kernel<M_SPLIT><<<nwg, 256, 0, s>>>(a); break;
    case M_BF16: herk_kernel<M_BF16><<<nwg, 256, 0, s>>>(a); break;
    case M_F16: herk_kernel<M_F16><<<nwg, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int herk_occupancy(int mode)
{
    switch (mode) {
    case M_F64: return occupancy_of<M_F64>();
    case M_F32: return occupancy_of<M_F32>();
    case M_SPLIT: return occupancy_of<M_SPLIT>();
    case M_BF16: return occupancy_of<M_BF16>();
    case M_F16: return occupancy_of<M_F16>();
    default: return 1;
    }
}

}  // namespace plv
