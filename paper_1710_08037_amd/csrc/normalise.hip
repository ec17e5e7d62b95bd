// normalise.hip -- analytic signal -> unit phasors (Section II.A, Eq. 4), and
// for coherency (Section II.B, Eq. 12) the rows scaled by a power of two.
//
// u = z / |z| replaces the angle() + exp() of the per-pair formulation.  For
// components of ordinary size 1/|z| is one hardware reciprocal square root;
// otherwise |z| is formed from components rescaled by an exact power of two,
// so FP32 neither underflows nor overflows for any finite z (phasor.h).  z = 0
// (either zero sign) maps to 1 + 0i, the phasor of angle(0) = 0.  The result is written in the Gram
// kernel's operand format: interleaved (re, im) per sample, as bf16 / f16 / f32
// / f64, or as two bf16 planes hi = rn(u), lo = rn(u - hi) for the split mode.
// Samples past the window are written as 0 + 0i up to the padded length.
//
// HBM-bound: each thread moves 4 consecutive samples (32 B in for c64, 16 to
// 64 B out).  A block covers 16 samples of 64 consecutive rows, so a wave
// reads whole 128-byte runs (c64) of 16 rows and writes, per plane stage,
// one contiguous run of 16 rows of the stage-major planes.
#include "phasor.h"

namespace plv {
namespace {

constexpr int VEC = 4;  // samples per thread

// A block covers SPB = 16 consecutive samples (one to four plane stages) of
// RPB = 64 consecutive rows: 4 threads per row, each 4 samples.
struct NormShape {
    static constexpr int SPB = 16;          // samples per block row
    static constexpr int QPS = SPB / VEC;   // threads per row
    static constexpr int RPB = 256 / QPS;   // rows per block
};

template <int MODE>
__global__ __launch_bounds__(256) void normalise_kernel(NormArgs a)
{
    typedef NormShape S;
    const int row = a.row0 + blockIdx.y * S::RPB + threadIdx.x / S::QPS;
    const int s0 = blockIdx.x * S::SPB + (threadIdx.x % S::QPS) * VEC;
    if (row >= a.n || s0 >= a.tpad)
        return;
    // 4 samples never straddle a stage or a chunk (both multiples of 4)
    uint8_t *dst = plane_at(a.u, a.cstride, a.chunk, a.rows, cbytes_of(MODE), row, s0);
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    auto src = gptr((const cplx_t *)a.in + (int64_t)row * a.ld + a.t0);
    real_t ur[VEC], ui[VEC];
    const real_t sc = a.scale ? (real_t)a.scale[row] : (real_t)1;  // a power of two: exact
    cplx_t zin[VEC];
    if constexpr (MODE != M_F64) {
        // the 4 samples on a 16-byte boundary (s0 is a multiple of 4, so the
        // row's first window sample must be): two 16-byte loads, half the
        // load instructions of per-sample loads
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0 && s0 + VEC <= a.tw) {
            auto q = (const PLV_GLOBAL vf4 *)(src + s0);
            const vf4 q0 = q[0], q1 = q[1];
            zin[0] = vf2{q0.x, q0.y};
            zin[1] = vf2{q0.z, q0.w};
            zin[2] = vf2{q1.x, q1.y};
            zin[3] = vf2{q1.z, q1.w};
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                zin[v] = s0 + v < a.tw ? src[s0 + v] : cplx_t{0, 0};
        }
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            zin[v] = s0 + v < a.tw ? src[s0 + v] : cplx_t{0, 0};
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int s = s0 + v;
        ur[v] = 0;
        ui[v] = 0;
        if (s < a.tw) {
            cplx_t z = zin[v];
            if (a.scale) {
                ur[v] = z.x * sc;
                ui[v] = z.y * sc;
            } else {
                unit_phasor(z.x, z.y, ur[v], ui[v]);
            }
        }
    }
    store4<MODE>(dst, a.plane_bytes, ur, ui);
}

// Across trials: a transpose through LDS.  A block covers TT consecutive
// time points x TR consecutive signals x 32 consecutive trials.  It reads
// z(k, i, t0 + tau) with consecutive threads on consecutive time points
// (512-byte runs when samples are contiguous in time: the reads, strided
// over signals and trials, set the kernel's time, and runs of 128 B over
// 8 signals were 6% slower), keeps the unit phasors in LDS, then writes each
// time point's planes with consecutive threads on 4-sample groups of one row
// and then on rows, so a wave stores runs of TR rows x 64 B of the
// stage-major planes.  Trials past ntr are written as 0 up to the padded
// length (a multiple of 4, not necessarily of 32: the last block's groups
// past it are not stored).
struct TrialShape {
    static constexpr int TR = 2;   // signals per block
    static constexpr int KB = 32;  // trials (plane samples) per block
};

template <int MODE>
__global__ __launch_bounds__(256) void trial_planes_kernel(TrialArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    constexpr int TR = TrialShape::TR, KB = TrialShape::KB;
    constexpr int TT = MODE == M_F64 ? 32 : 64;     // time points per block
    constexpr int NLD = TT * TR * KB / 256;         // loads per thread
    constexpr int NST = TT * TR * (KB / 4) / 256;   // 4-sample stores per thread
    // [tau][r][k], the 4-trial group of k swizzled by tau so that both the
    // tau-major writes and the k-major reads spread over the banks
    __shared__ cplx_t tile[TT * TR * KB];
    const int tau0 = blockIdx.x * TT;
    const int64_t i0 = (int64_t)a.row0 + (int64_t)blockIdx.y * TR;
    const int k0 = blockIdx.z * KB;
    const int t = threadIdx.x;

    cplx_t zin[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int item = q * 256 + t;
        const int tau = item % TT, p = item / TT;  // p = r * KB + k
        const int k = p % KB, r = p / KB;
        const int64_t i = i0 + r;
        zin[q] = cplx_t{0, 0};
        if (tau0 + tau < a.ntp && i < a.n && k0 + k < a.ntr)
            zin[q] = gptr((const cplx_t *)a.in)[i * a.ld + (a.t0 + tau0 + tau) * a.sstride + (int64_t)(k0 + k) * a.tstride];
    }
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
        const int item = q * 256 + t;
        const int tau = item % TT, p = item / TT;
        const int k = p % KB, r = p / KB;
        real_t ur = 0, ui = 0;
        if (k0 + k < a.ntr)
            unit_phasor(zin[q].x, zin[q].y, ur, ui);
        tile[(tau * TR + r) * KB + (((k >> 2) ^ (tau & 7)) << 2) + (k & 3)] = cplx_t{ur, ui};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NST; ++q) {
        const int item = q * 256 + t;
        const int kq = item % (KB / 4), r = (item / (KB / 4)) % TR, tau = item / (KB / 4 * TR);
        const int64_t i = i0 + r;
        if (tau0 + tau >= a.ntp || i >= a.n || k0 + kq * VEC >= a.tpad)
            continue;
        const cplx_t *src = tile + (tau * TR + r) * KB + ((kq ^ (tau & 7)) << 2);
        real_t ur[VEC], ui[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            ur[v] = src[v].x;
            ui[v] = src[v].y;
        }
        store4<MODE>(plane_at(a.u0 + (int64_t)(tau0 + tau) * a.gstride, a.cstride, a.chunk, a.rows, cbytes_of(MODE),
                              i, k0 + kq * VEC),
                     a.plane_bytes, ur, ui);
    }
}

// One work-group per row: the largest |Re z| or |Im z| over the window, and
// its exponent e (frexp convention, m = f 2^e with f in [0.5, 1)), give the
// scale 2^-e.  A zero row gets 1.  The exponent is clamped to [-126, 126] so
// the scale is a normal FP32 number too.
template <class R>
__global__ __launch_bounds__(256) void row_scale_kernel(ScaleArgs a)
{
    typedef typename std::conditional<sizeof(R) == 8, vd2, vf2>::type cplx_t;
    __shared__ R part[256];
    const int row = blockIdx.x;
    auto src = gptr((const cplx_t *)a.in + (int64_t)row * a.ld + a.t0);
    R m = 0;
#pragma unroll 8
    for (int s = threadIdx.x; s < a.tw; s += 256) {
        const cplx_t z = src[s];
        m = fmax(m, fmax(fabs(z.x), fabs(z.y)));
    }
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const R mx = part[0];
        int e = 0;
        if (mx > 0)
            (void)frexp(mx, &e);
        e = e < -126 ? -126 : (e > 126 ? 126 : e);
        a.scale[row] = ldexp(1.0, -e);
    }
}

}  // namespace

hipError_t launch_trial_planes(int mode, const TrialArgs &a, hipStream_t s)
{
    constexpr int TR = TrialShape::TR, KB = TrialShape::KB;
    if (a.tpad % VEC != 0)
        return hipErrorInvalidValue;
    const int tt = mode == M_F64 ? 32 : 64;
    for (int64_t r0 = 0; r0 < a.n; r0 += (int64_t)MAX_GRID_Y * TR) {
        TrialArgs b = a;
        b.row0 = (int32_t)r0;
        const int64_t nblk = (a.n - r0 + TR - 1) / TR;
        dim3 grid((a.ntp + tt - 1) / tt, (unsigned)std::min<int64_t>(MAX_GRID_Y, nblk), (a.tpad + KB - 1) / KB);
        switch (mode) {
        case M_F64: trial_planes_kernel<M_F64><<<grid, 256, 0, s>>>(b); break;
        case M_F32: trial_planes_kernel<M_F32><<<grid, 256, 0, s>>>(b); break;
        case M_SPLIT: trial_planes_kernel<M_SPLIT><<<grid, 256, 0, s>>>(b); break;
        case M_BF16: trial_planes_kernel<M_BF16><<<grid, 256, 0, s>>>(b); break;
        case M_F16: trial_planes_kernel<M_F16><<<grid, 256, 0, s>>>(b); break;
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_row_scale(bool f64, const ScaleArgs &a, hipStream_t s)
{
    if (a.n <= 0)
        return hipSuccess;
    if (f64)
        row_scale_kernel<double><<<a.n, 256, 0, s>>>(a);
    else
        row_scale_kernel<float><<<a.n, 256, 0, s>>>(a);
    return hipGetLastError();
}

namespace {

template <int MODE>
hipError_t normalise_rows(const NormArgs &a, hipStream_t s)
{
    typedef NormShape S;
    const int64_t span = (int64_t)MAX_GRID_Y * S::RPB;  // rows per launch
    for (int64_t r0 = 0; r0 < a.n; r0 += span) {
        NormArgs b = a;
        b.row0 = (int32_t)r0;
        const int64_t nr = std::min<int64_t>(span, a.n - r0);
        dim3 grid(a.tpad / S::SPB, (unsigned)((nr + S::RPB - 1) / S::RPB));
        normalise_kernel<MODE><<<grid, 256, 0, s>>>(b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_normalise(int mode, const NormArgs &a, hipStream_t s)
{
    if (a.tpad % 32 != 0)
        return hipErrorInvalidValue;  // tpad is a multiple of PLV_KGRAN, so of every stage width
    switch (mode) {
    case M_F64: return normalise_rows<M_F64>(a, s);
    case M_F32: return normalise_rows<M_F32>(a, s);
    case M_SPLIT: return normalise_rows<M_SPLIT>(a, s);
    case M_BF16: return normalise_rows<M_BF16>(a, s);
    case M_F16: return normalise_rows<M_F16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace plv
