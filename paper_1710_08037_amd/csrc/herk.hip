// herk.hip -- the Gram contraction G = U U^H (Section II.A, Eqs. 5-7) on MFMA.
//
// One work-group computes one BM x BM tile (I, J), I <= J, of the upper
// triangle over one K-chunk of samples, and writes the tile's chunk sum
// (Re, Im as two BM x BM FP64 planes) to a slot of the partial buffer; the
// epilogue kernel adds the slots in a fixed order.  When T has more chunks
// than slots, the host launches several passes and pass p > 0 adds chunk
// p * nslot + s into slot s.  A problem whose T is a single chunk skips the
// partial buffer: the work-group divides by T and stores PLV, iPLV, ciPLV
// (and G) itself, with the same FP64 arithmetic as the epilogue.  Only the
// upper triangle is computed: G_ji = conj(G_ij).
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
// Tiling (all modes): 512 threads = 8 waves in two groups of four; within a
// group the waves sit 2 x 2, each one a (BM/2) x (BM/2) sub-tile made of
// 16 x 16 MFMA blocks, and the two groups take alternate K-units and add
// their sums at the end.  Each K-stage holds 64 bytes per row (16 / 8 / 4
// samples for 16-bit / f32 / f64) of the row panel I and the column panel J.
// They move global -> LDS directly (global_load_lds_dwordx4, no staging
// registers) into a ring of NS stages, with the 16-byte positions of each
// 64-byte LDS row XOR-swizzled by row.  A diagonal tile (I == J) loads one
// panel and uses it as both operands.  The groups ping-pong: in each barrier
// interval one group reads a unit's fragments from LDS into registers while
// the other runs the MFMAs of the unit it read in the interval before.
//
// Work-groups are handed out XCD-aware: the hardware deals work-group ids
// round-robin over the 8 XCDs, so ids are remapped to give each XCD a
// contiguous range of items (same chunk, neighbouring tiles), which keeps the
// shared row panels in that XCD's L2.
#include "metrics.h"

namespace plv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int RB = 64;  // bytes of one row staged per K-stage, per plane

// LDS ring depth per mode, in stages of planes x 2 panels x BM rows x 64 B.
// With units of SPI stages the ring holds NS / SPI units: while one is read,
// the loads of the next NS / SPI - 2 are in flight and one more is issued.
template <int MODE, int TBM>
struct Ring {
    static constexpr int BM = TBM;
    static constexpr int PL = planes_of(MODE);
    static constexpr int PANEL = BM * RB;          // one panel of one plane
    static constexpr int STAGE = PL * 2 * PANEL;   // A and B panels of every plane
    // split at the 64-wide tile: three stages (48 KB), so three work-groups
    // share a CU (short-K problems: the lookahead matters less than the
    // other work-groups' loads in flight)
    static constexpr int NS = (MODE == M_SPLIT) ? (TBM == 64 ? 3 : 4) : 8;
};

template <int MODE>
struct AccOf {
    typedef f32x4 type;
};
template <>
struct AccOf<M_F64> {
    typedef f64x4 type;
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

// LDS layout of one stage: each panel is a run of 1 KB blocks of 16 rows x
// 64 bytes, row-major, with the four 16-byte positions of each row
// XOR-swizzled by the row's index in its block.  The direct loads stay
// coalesced (four lanes fetch one row's 64 contiguous bytes) and the MFMA
// fragment reads (lane l: row l % 16, segment l / 16) spread over the banks.
// Measured on gfx950 this beats both plain 64-byte rows (FP32 fragments
// conflict) and a segment-major block (its loads coalesce poorly).
__device__ inline int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }
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

// s_waitcnt on the vector-memory counter only (gfx9 encoding: vmcnt in bits
// 3:0 and 15:14, expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ inline void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// s_waitcnt lgkmcnt(0) only (vmcnt and expcnt left at their maxima).
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4)); }

// Operand fragments of one unit of SPI K-stages, for one wave's
// (BM/2) x (BM/2) sub-tile: the row panel's blocks (a) and the column
// panel's blocks (b).  The 16-bit modes take two stages per unit so that a
// unit's MFMA work stays long next to the barrier that separates units.
template <int MODE, int BM>
struct Frags {
    static constexpr int NB = BM / 32;
    static constexpr int PL = planes_of(MODE);
    static constexpr int SPI = (MODE == M_BF16 || MODE == M_F16) ? 2 : 1;
    u32x4 a[SPI][PL][NB], b[SPI][PL][NB];
};
template <int BM>
struct Frags<M_F32, BM> {
    static constexpr int NB = BM / 32;
    static constexpr int SPI = 1;
    float2 a[2][NB], b[2][NB];  // two K-steps of 4 samples
};
template <int BM>
struct Frags<M_F64, BM> {
    static constexpr int NB = BM / 32;
    static constexpr int SPI = 1;
    double2 a[NB], b[NB];
};

// Work-group barrier without a memory fence.  __syncthreads() would make
// every wave drain all of its in-flight loads first (vmcnt(0)), which would
// collapse the ring to one stage; each wave instead waits for its own loads
// of the stage about to be read (wait_vm) and then meets the others here.
// The empty asm keeps the compiler from moving LDS accesses across it.
__device__ inline void stage_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void gvoid;

constexpr int WAVES = 8;   // two groups of four waves per work-group
constexpr int THREADS = 64 * WAVES;

template <int MODE, int TBM, bool DIAG>
__device__ inline void herk_tile(const GramDesc &d, const uint8_t *ua, const uint8_t *ub, int I, int J, int nst,
                                 typename AccOf<MODE>::type (&re)[TBM / 32][TBM / 32],
                                 typename AccOf<MODE>::type (&im)[TBM / 32][TBM / 32], uint8_t *smem)
{
    typedef Ring<MODE, TBM> R;
    constexpr int BM = R::BM, NB = BM / 32, PL = R::PL, PANEL = R::PANEL, STAGE = R::STAGE, NS = R::NS;
    constexpr int CB = cbytes_of(MODE);
    constexpr int BLKS = PANEL / 1024;            // 1 KB load blocks per panel and plane
    constexpr int SLOTS = PL * (DIAG ? 1 : 2) * BLKS;  // load blocks per stage
    // Who issues a unit's loads.  16-bit modes: only the group that reads in
    // the interval whose head issues them, so the computing group's MFMAs do
    // not queue behind a burst of loads (measured: 13-22% faster).  FP32 and
    // FP64, whose intervals are long, spread the loads over all waves.
    constexpr bool ONE_GROUP = (CB == 4);
    constexpr int IW = ONE_GROUP ? WAVES / 2 : WAVES;   // issuing waves
    static_assert(SLOTS % IW == 0 || SLOTS < IW, "load blocks per wave");
    constexpr int LPS = (SLOTS + IW - 1) / IW;          // loads per stage per issuing wave (last ones may idle)

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = wave >> 2, wq = wave & 3;
    const int wm = wq >> 1, wn = wq & 1;

    // ---- direct global -> LDS loads: lane L of a 1 KB block stages row L/4,
    // LDS position L%4, which holds the row's segment (L%4) ^ swz(L/4).
    // Stage-major planes: K-stage st of row r sits at st * rows * RB + r * RB,
    // so one load block (16 rows) is one contiguous kilobyte.
    const int64_t sa = (int64_t)d.npad * RB;                              // A: npad rows
    const int64_t sb = d.ub ? (int64_t)d.ntile_b * BM * RB : sa;         // B: its own row count
    const int lr = lane >> 2;
    const uint32_t voff = (uint32_t)(lr * RB) + (uint32_t)(((lane & 3) ^ swz(lr)) * 16);
    const uint8_t *gA = ua + (int64_t)I * BM * RB;
    const uint8_t *gB = ub + (int64_t)J * BM * RB;
    auto issue = [&](int st, int buf) {
        uint8_t *base = smem + buf * STAGE;
#pragma unroll
        for (int q = 0; q < LPS; ++q) {
            const int slot = (ONE_GROUP ? wq : wave) + IW * q;  // wave-uniform
            if (slot < SLOTS) {
                const int blk = slot % BLKS;
                const int pp = slot / BLKS;      // plane * (1 or 2) + panel
                const int p = DIAG ? pp : (pp >> 1);
                const int isb = DIAG ? 0 : (pp & 1);
                const uint8_t *g = (isb ? gB + st * sb : gA + st * sa) + p * d.plane_bytes + blk * 16 * RB;
                __builtin_amdgcn_global_load_lds((gvoid *)(g + voff),
                                                 (lds_void *)(base + p * 2 * PANEL + isb * PANEL + blk * 1024),
                                                 16, 0, 0);
            }
        }
    };

    // ---- fragment addressing (row within a 16-row block = lane & 15)
    const int fr = lane & 15;
    const int arow = (wm * (BM / 2) + fr) * RB;
    const int brow = (wn * (BM / 2) + fr) * RB + (DIAG ? 0 : PANEL);

    // One unit = SPI consecutive stages.  A wave reads all operand fragments
    // of a unit from LDS into registers (Frags), then runs that unit's MFMAs
    // from registers in the next interval.
    typedef Frags<MODE, BM> F;
    constexpr int SPI = F::SPI;
    constexpr int NU = NS / SPI;                  // units held by the ring
    constexpr int LPU = SPI * LPS;                // loads per unit per wave
    F fg;
    auto issue_unit = [&](int u) {
#pragma unroll
        for (int s = 0; s < SPI; ++s)
            issue(u * SPI + s, (u % NU) * SPI + s);
    };

    auto read_frags = [&](int u) {
#pragma unroll
        for (int s = 0; s < SPI; ++s) {
            const uint8_t *S = smem + ((u % NU) * SPI + s) * STAGE;
            if constexpr (CB == 4) {
                const int off = (((lane >> 4) ^ swz(fr)) * 16);
#pragma unroll
                for (int p = 0; p < PL; ++p)
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        fg.a[s][p][b] = *(const u32x4 *)(S + p * 2 * PANEL + arow + b * 16 * RB + off);
                        fg.b[s][p][b] = *(const u32x4 *)(S + p * 2 * PANEL + brow + b * 16 * RB + off);
                    }
            } else if constexpr (CB == 8) {
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int off = (((ks * 2 + (lane >> 5)) ^ swz(fr)) * 16) + ((lane >> 4) & 1) * 8;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        fg.a[ks][b] = *(const float2 *)(S + arow + b * 16 * RB + off);
                        fg.b[ks][b] = *(const float2 *)(S + brow + b * 16 * RB + off);
                    }
                }
            } else {
                const int off = (((lane >> 4) ^ swz(fr)) * 16);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    fg.a[b] = *(const double2 *)(S + arow + b * 16 * RB + off);
                    fg.b[b] = *(const double2 *)(S + brow + b * 16 * RB + off);
                }
            }
        }
    };

    auto mma = [&]() {
        if constexpr (CB == 4) {
            // 16 samples per stage = one K' = 32 step of v_mfma_*_16x16x32
#pragma unroll
            for (int s = 0; s < SPI; ++s)
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    u32x4 vq[PL];
#pragma unroll
                    for (int p = 0; p < PL; ++p)
                        vq[p] = swap_neg(fg.a[s][p][a]);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        re[a][b] = mfma16<MODE>(fg.a[s][0][a], fg.b[s][0][b], re[a][b]);
                        im[a][b] = mfma16<MODE>(vq[0], fg.b[s][0][b], im[a][b]);
                        if constexpr (PL == 2) {
                            re[a][b] = mfma16<MODE>(fg.a[s][0][a], fg.b[s][1][b], re[a][b]);
                            im[a][b] = mfma16<MODE>(vq[0], fg.b[s][1][b], im[a][b]);
                            re[a][b] = mfma16<MODE>(fg.a[s][1][a], fg.b[s][0][b], re[a][b]);
                            im[a][b] = mfma16<MODE>(vq[1], fg.b[s][0][b], im[a][b]);
                        }
                    }
                }
        } else if constexpr (CB == 8) {
            // FP32: 8 samples = 2 steps of 4; one sample (re, im) per lane
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    const float2 va = fg.a[ks][a];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float2 vb = fg.b[ks][b];
                        re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.x, vb.x, re[a][b], 0, 0, 0);
                        re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb.y, re[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb.x, im[a][b], 0, 0, 0);
                        im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-va.x, vb.y, im[a][b], 0, 0, 0);
                    }
                }
        } else {
            // FP64: 4 samples = 1 step of 4; one sample (re, im) per lane
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const double2 va = fg.a[a];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const double2 vb = fg.b[b];
                    re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.x, vb.x, re[a][b], 0, 0, 0);
                    re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.y, vb.y, re[a][b], 0, 0, 0);
                    im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va.y, vb.x, im[a][b], 0, 0, 0);
                    im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-va.x, vb.y, im[a][b], 0, 0, 0);
                }
            }
        }
    };

    // ---- K loop, ping-pong between the two wave groups (one wave of each
    // per SIMD).  In interval k group k % 2 reads unit k's fragments from LDS
    // while the other group runs the MFMAs of unit k - 1 from the fragments
    // it read in interval k - 1, so the matrix cores of a SIMD are fed by one
    // wave while the other waits on LDS.  Every interval opens with the same
    // head in every wave: wait for this wave's own loads of unit k, one
    // barrier (unit k landed for every wave; unit k - 1's fragments are in
    // registers, so its buffers are free), refill those buffers with unit
    // k + NU - 1.  Group 1 sits out interval 0; each loop trip is then one
    // read interval and one compute interval of the wave's own group.
    const int nu = nst / SPI;
    // Unit j is loaded at the head of interval j - NU + 1 (before the loop for
    // j < NU - 1): by every wave, or with ONE_GROUP by group (j + NU + 1) % 2,
    // the one reading in that interval.  Each wave issues exactly LPU loads
    // per unit it takes part in, or none.  After unit k a wave then has at
    // most W units outstanding, none of them beyond unit k + LAST.
    constexpr int W = ONE_GROUP ? (NU - 2) / 2 : NU - 2;
    constexpr int LAST = ONE_GROUP ? 2 * W : W;
    auto head = [&](int k) {
        if (k + LAST < nu)
            wait_vm<W * LPU>();
        else
            wait_vm<0>();
        stage_barrier();
        if (k + NU - 1 < nu && (!ONE_GROUP || (k & 1) == grp))
            issue_unit(k + NU - 1);
    };
#pragma unroll
    for (int v = 0; v < NU - 1; ++v)
        if (v < nu && (!ONE_GROUP || ((v + NU + 1) & 1) == grp))
            issue_unit(v);
    int k = grp;
    if (grp == 1)
        head(0);
    for (; k < nu; k += 2) {
        head(k);
        read_frags(k);
        wait_lgkm0();  // fragments in registers before the next barrier frees the buffers
        head(k + 1);
        mma();
    }
    if (k == nu + 1)
        return;  // the last trip ran the head of interval nu
    head(nu);    // k == nu: interval nu is still open (the other group's last compute)
}

// Folds group 1's accumulators into group 0's through LDS (after the K loop).
template <int MODE, int BM>
__device__ inline void fold_groups(typename AccOf<MODE>::type (&re)[BM / 32][BM / 32],
                                   typename AccOf<MODE>::type (&im)[BM / 32][BM / 32], uint8_t *smem)
{
    constexpr int NB = BM / 32;
    typedef typename AccOf<MODE>::type acc_t;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = wave >> 2, wq = wave & 3;
    acc_t *buf = (acc_t *)smem + (size_t)wq * NB * NB * 2 * 64;
    __syncthreads();  // every wave is done reading the ring
    if (grp == 1) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                buf[((a * NB + b) * 2 + 0) * 64 + lane] = re[a][b];
                buf[((a * NB + b) * 2 + 1) * 64 + lane] = im[a][b];
            }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                re[a][b] += buf[((a * NB + b) * 2 + 0) * 64 + lane];
                im[a][b] += buf[((a * NB + b) * 2 + 1) * 64 + lane];
            }
    }
}

// Fused store of a single-chunk tile (I, J): the measures (and G) of its
// upper-triangle entries at (i, j) and their mirror at (j, i), both written
// row by row.  Group 0's accumulators (after the fold) go to LDS as two
// BM x BM planes (Re, Im) of the accumulator type, the column of element
// (a, b) XOR-swizzled by a mod 64, so that reading a row (the block at rows
// of I) and reading a column (the mirrored block at rows of J) both spread
// over the banks.  Then all 8 waves store: consecutive threads take
// consecutive columns of one output row, every store a contiguous run.
template <int MODE, int BM>
__device__ inline void fused_store(const GramDesc &d, int I, int J,
                                   typename AccOf<MODE>::type (&re)[BM / 32][BM / 32],
                                   typename AccOf<MODE>::type (&im)[BM / 32][BM / 32], uint8_t *smem)
{
    constexpr int NB = BM / 32;
    typedef typename std::conditional<MODE == M_F64, double, float>::type acc_e;
    static_assert(2 * BM * BM * (int)sizeof(acc_e) <= Ring<MODE, BM>::NS * Ring<MODE, BM>::STAGE,
                  "the ring holds the tile");
    acc_e *tr = (acc_e *)smem, *ti = tr + BM * BM;
    auto at = [](int a, int b) { return a * BM + (b ^ (a & 63)); };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // the fold's reads of the ring are done
    if (wave < 4) {
        const int wm = wave >> 1, wn = wave & 1;
        const int r0 = wm * (BM / 2) + (MODE == M_F64 ? (lane >> 4) : (lane >> 4) * 4);
        constexpr int RSTEP = (MODE == M_F64) ? 4 : 1;
        const int c0 = wn * (BM / 2) + (lane & 15);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = at(r0 + a * 16 + r * RSTEP, c0 + b * 16);
                    tr[e] = re[a][b][r];
                    ti[e] = im[a][b][r];
                }
    }
    __syncthreads();
    const double inv_t = 1.0 / (double)d.t;
    const int64_t n = d.n;
    constexpr int LBM = BM == 128 ? 7 : 6;
    if constexpr (MODE != M_F64) {
        // Rows that start 16-byte aligned (n a multiple of 4, aligned
        // outputs): a thread takes four consecutive entries of a row, all
        // inside n or all outside, and stores them at once (store_four).  On
        // 148 signals x 40 trials x 4000 time points the Gram took 0.455 ms
        // with one 4-byte store per entry and takes 0.411 ms so (0.143 ms
        // with no store at all: writing the 1.05 GB of output is most of it).  A
        // diagonal tile is one pass over its square, the entries below its
        // diagonal taken from the conjugate of their mirror, so no group
        // straddles the diagonal; an off-diagonal tile writes block (I, J)
        // and then its mirror block (J, I).
        const uintptr_t al = (uintptr_t)d.plv | (uintptr_t)d.iplv | (uintptr_t)d.ciplv | (uintptr_t)d.g;
        if ((n & 3) == 0 && (al & 15) == 0) {
            const int nblk = I == J ? 1 : 2;
#pragma unroll 1
            for (int blk = 0; blk < nblk; ++blk) {
                const int64_t row0 = (int64_t)(blk ? J : I) * BM, col0 = (int64_t)(blk ? I : J) * BM;
                for (int e = threadIdx.x; e < BM * BM / 4; e += THREADS) {
                    const int a = e >> (LBM - 2), b = (e & (BM / 4 - 1)) * 4;
                    const int64_t gr = row0 + a, gc = col0 + b;
                    if (gr >= n || gc >= n)
                        continue;
                    vf4 vp, vi, vc, g01, g23;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool lower = blk != 0 || (I == J && b + q < a);
                        const int s = lower ? at(b + q, a) : at(a, b + q);
                        entry_of<MODE>(gr == gc + q, lower, (double)tr[s] * inv_t, (double)ti[s] * inv_t, q, vp, vi,
                                       vc, g01, g23);
                    }
                    store_four(d, gr * n + gc, vp, vi, vc, g01, g23);
                }
            }
            return;
        }
    }
    // block 0: rows of I, columns of J, entry (a, b) as accumulated;
    // block 1: rows of J, columns of I, entry (a, b) the conjugate of (b, a)
    // (one code path for both blocks: an entry and its mirror are computed
    // by the same instructions from the same values)
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
        const int64_t row0 = (int64_t)(blk ? J : I) * BM, col0 = (int64_t)(blk ? I : J) * BM;
        for (int e = threadIdx.x; e < BM * BM; e += THREADS) {
            const int a = e >> LBM, b = e & (BM - 1);
            const int64_t gr = row0 + a, gc = col0 + b;
            if (gr >= n || gc >= n || (blk ? gc >= gr : gr > gc))
                continue;
            const int s = blk ? at(b, a) : at(a, b);
            const double vr = (double)tr[s] * inv_t, vi = (double)ti[s] * inv_t;
            store_one<MODE>(d, gr * n + gc, gr == gc, blk != 0, vr, vi);
        }
    }
}

// Work-groups per CU the kernel is built for: the 64-wide tile of the 16-bit
// and FP32 modes takes half the LDS ring (split: three eighths) and a quarter
// of the accumulators, so two (split: three) work-groups share a CU.  The
// launch bounds take the matching waves per SIMD (8 waves per work-group over
// 4 SIMDs), which caps the registers so that they fit too.
template <int MODE, int BM>
constexpr int wg_per_cu() { return BM == 64 && MODE == M_SPLIT ? 3 : ((BM == 64 && MODE != M_F64) ? 2 : 1); }

template <int MODE, int BM>
__global__ __launch_bounds__(THREADS, (WAVES / 4 * wg_per_cu<MODE, BM>())) void herk_kernel(HerkArgs args)
{
    constexpr int NB = BM / 32;  // 16x16 blocks per wave side
    typedef typename AccOf<MODE>::type acc_t;
    typedef Ring<MODE, BM> R;
    static_assert(R::NS * R::STAGE >= 4 * NB * NB * 2 * 64 * (int)sizeof(acc_t),
                  "the ring must hold one group's accumulators for the fold");

    __shared__ __attribute__((aligned(1024))) uint8_t smem[R::NS * R::STAGE];

    // ---- which item
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    GramDesc d;
    int tile, slot;
    if (args.items) {
        const Item it = args.items[item];
        if (it.gram < 0)
            return;  // padding of an XCD's list
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
    if (d.ub) {  // general product: full grid, row-major over (I, J)
        I = tile / d.ntile_b;
        J = tile - I * d.ntile_b;
    } else if (args.blocked) {  // blocked launch order of a single problem
        // The position comes out of a VALU division: move it to a scalar
        // register first.  Decoded from a vector register, the decode's last
        // loop was compiled with a select on a stale SCC that never lowered
        // the position, so the work-group never left it.
        blocked_tile(__builtin_amdgcn_readfirstlane(tile), __builtin_amdgcn_readfirstlane(d.ntile), I, J);
    } else {
        tile_ij(tile, d.ntile, I, J);
    }
    const int k0 = chunk * d.chunk;
    const int k1 = min(k0 + d.chunk, d.tpad);
    const int nst = (k1 - k0) / (RB / cbytes_of(MODE));

    acc_t re[NB][NB], im[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            re[a][b] = acc_t{0, 0, 0, 0};
            im[a][b] = acc_t{0, 0, 0, 0};
        }
    // the chunk's block of the planes (one block, cstride 0, in product mode)
    const uint8_t *ua = d.u + (int64_t)chunk * d.cstride;
    const uint8_t *ub = (d.ub ? d.ub : d.u) + (int64_t)chunk * d.cstride;
    if (I == J && !d.ub)
        herk_tile<MODE, BM, true>(d, ua, ub, I, J, nst, re, im, smem);
    else
        herk_tile<MODE, BM, false>(d, ua, ub, I, J, nst, re, im, smem);
    fold_groups<MODE, BM>(re, im, smem);

    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (d.fused && !d.ub) {
        fused_store<MODE, BM>(d, I, J, re, im, smem);
        return;
    }
    if (wave >= 4)
        return;
    const int wm = wave >> 1, wn = wave & 1;
    if (d.ub) {
        // ---- general product: store the complex tile of C directly
        typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
        auto cp = gptr((cplx_t *)d.c);
        const int rr0 = wm * (BM / 2) + (MODE == M_F64 ? (lane >> 4) : (lane >> 4) * 4);
        constexpr int RS = (MODE == M_F64) ? 4 : 1;
        const int cc0 = wn * (BM / 2) + (lane & 15);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = (int64_t)I * BM + rr0 + a * 16 + r * RS;
                    const int64_t j = (int64_t)J * BM + cc0 + b * 16;
                    if (i < d.n && j < d.nb) {
                        cplx_t v;
                        v.x = re[a][b][r];
                        v.y = im[a][b][r];
                        cp[i * d.ldc + j] = v;
                    }
                }
        return;
    }
    // ---- chunk sum of this tile -> partial[slot][tile][re|im][BM][BM] (FP64).
    // A chunk spans at most a few thousand samples, which bounds the FP32
    // accumulation error; later passes over a long T add into the same slot.
    // Accumulator layout of a 16x16 block: lane l, register r holds column
    // l % 16 of row 4 (l / 16) + r for the FP32-output MFMAs, and of row
    // l / 16 + 4 r for v_mfma_f64_16x16x4f64.
    // Slots are indexed by the row-major upper-triangle index of (I, J),
    // which the epilogue decodes, whatever order the tiles were launched in.
    const int tile_rm = I * d.ntile - I * (I - 1) / 2 + (J - I);
    auto out = gptr(d.partial + ((int64_t)slot * d.nupper + tile_rm) * 2 * BM * BM);
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

template <int MODE, int BM>
int occupancy_of()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, herk_kernel<MODE, BM>, THREADS, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace

bool tile_supported(int mode, int bm)
{
    return mode == M_F64 ? bm == 64 : (bm == 64 || bm == 128);
}

hipError_t launch_herk(int mode, int bm, const HerkArgs &a, int nwg, hipStream_t s)
{
    if (nwg <= 0)
        return hipSuccess;
    if (!tile_supported(mode, bm))
        return hipErrorInvalidValue;
    if (bm == 64) {
        switch (mode) {
        case M_F64: herk_kernel<M_F64, 64><<<nwg, THREADS, 0, s>>>(a); break;
        case M_F32: herk_kernel<M_F32, 64><<<nwg, THREADS, 0, s>>>(a); break;
        case M_SPLIT: herk_kernel<M_SPLIT, 64><<<nwg, THREADS, 0, s>>>(a); break;
        case M_BF16: herk_kernel<M_BF16, 64><<<nwg, THREADS, 0, s>>>(a); break;
        case M_F16: herk_kernel<M_F16, 64><<<nwg, THREADS, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (mode) {
        case M_F32: herk_kernel<M_F32, 128><<<nwg, THREADS, 0, s>>>(a); break;
        case M_SPLIT: herk_kernel<M_SPLIT, 128><<<nwg, THREADS, 0, s>>>(a); break;
        case M_BF16: herk_kernel<M_BF16, 128><<<nwg, THREADS, 0, s>>>(a); break;
        case M_F16: herk_kernel<M_F16, 128><<<nwg, THREADS, 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

int herk_occupancy(int mode, int bm)
{
    if (!tile_supported(mode, bm))
        return 1;
    if (bm == 64) {
        switch (mode) {
        case M_F64: return occupancy_of<M_F64, 64>();
        case M_F32: return occupancy_of<M_F32, 64>();
        case M_SPLIT: return occupancy_of<M_SPLIT, 64>();
        case M_BF16: return occupancy_of<M_BF16, 64>();
        case M_F16: return occupancy_of<M_F16, 64>();
        default: return 1;
        }
    }
    switch (mode) {
    case M_F32: return occupancy_of<M_F32, 128>();
    case M_SPLIT: return occupancy_of<M_SPLIT, 128>();
    case M_BF16: return occupancy_of<M_BF16, 128>();
    case M_F16: return occupancy_of<M_F16, 128>();
    default: return 1;
    }
}

}  // namespace plv
