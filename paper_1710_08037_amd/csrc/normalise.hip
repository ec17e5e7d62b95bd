// normalise.hip -- analytic signal -> unit phasors (Section II.A, Eq. 4), and
// for coherency (Section II.B, Eq. 12) the rows scaled by a power of two.
//
// u = z / |z| replaces the angle() + exp() of the per-pair formulation.  |z| is
// formed from components rescaled by an exact power of two, so FP32 neither
// underflows nor overflows for any finite z.  z = 0 (either zero sign) maps to
// 1 + 0i, the phasor of angle(0) = 0.  The result is written in the Gram
// kernel's operand format: interleaved (re, im) per sample, as bf16 / f16 / f32
// / f64, or as two bf16 planes hi = rn(u), lo = rn(u - hi) for the split mode.
// Samples past the window are written as 0 + 0i up to the padded length.
//
// HBM-bound: each thread moves 4 consecutive samples (32 B in for c64, 16 or
// 32 B out), rows map to blockIdx.y so every access is contiguous.
#include "phasor.h"

namespace plv {
namespace {

constexpr int VEC = 4;  // samples per thread

template <int MODE>
__global__ __launch_bounds__(256) void normalise_kernel(NormArgs a)
{
    const int row = a.row0 + blockIdx.y;
    const int s0 = (blockIdx.x * 256 + threadIdx.x) * VEC;
    if (s0 >= a.tpad)
        return;
    uint8_t *dst = plane_at(a.u, a.cstride, a.chunk, cbytes_of(MODE), row, s0);  // 4 samples never straddle chunks
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    auto src = gptr((const cplx_t *)a.in + (int64_t)row * a.ld + a.t0);
    real_t ur[VEC], ui[VEC];
    const real_t sc = a.scale ? (real_t)a.scale[row] : (real_t)1;  // a power of two: exact
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const int s = s0 + v;
        ur[v] = 0;
        ui[v] = 0;
        if (s < a.tw) {
            cplx_t z = src[s];
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

// Across trials: thread (time point tau, signal i, trials k0..k0+3) reads
// z(k, i, t0 + tau) -- consecutive threads take consecutive time points, so
// the reads coalesce when samples are contiguous in time -- and stores the
// four unit phasors at samples k0..k0+3 of row i of tau's planes (trials past
// ntr are written as 0).
template <int MODE>
__global__ __launch_bounds__(256) void trial_planes_kernel(TrialArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type real_t;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    const int tau = blockIdx.x * 256 + threadIdx.x;
    if (tau >= a.ntp)
        return;
    const int64_t i = a.row0 + blockIdx.y;
    const int k0 = blockIdx.z * VEC;
    auto src = gptr((const cplx_t *)a.in + i * a.ld + (a.t0 + tau) * a.sstride);
    real_t ur[VEC], ui[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        ur[v] = 0;
        ui[v] = 0;
        if (k0 + v < a.ntr) {
            const cplx_t z = src[(int64_t)(k0 + v) * a.tstride];
            unit_phasor(z.x, z.y, ur[v], ui[v]);
        }
    }
    store4<MODE>(plane_at(a.u0 + (int64_t)tau * a.gstride, a.cstride, a.chunk, cbytes_of(MODE), i, k0),
                 a.plane_bytes, ur, ui);
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
    for (int r0 = 0; r0 < a.n; r0 += MAX_GRID_Y) {
        TrialArgs b = a;
        b.row0 = r0;
        dim3 grid((a.ntp + 255) / 256, std::min(MAX_GRID_Y, a.n - r0), a.tpad / VEC);
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

hipError_t launch_normalise(int mode, const NormArgs &a, hipStream_t s)
{
    for (int r0 = 0; r0 < a.n; r0 += MAX_GRID_Y) {
        NormArgs b = a;
        b.row0 = r0;
        dim3 grid((a.tpad + 256 * VEC - 1) / (256 * VEC), std::min(MAX_GRID_Y, a.n - r0));
        switch (mode) {
        case M_F64: normalise_kernel<M_F64><<<grid, 256, 0, s>>>(b); break;
        case M_F32: normalise_kernel<M_F32><<<grid, 256, 0, s>>>(b); break;
        case M_SPLIT: normalise_kernel<M_SPLIT><<<grid, 256, 0, s>>>(b); break;
        case M_BF16: normalise_kernel<M_BF16><<<grid, 256, 0, s>>>(b); break;
        case M_F16: normalise_kernel<M_F16><<<grid, 256, 0, s>>>(b); break;
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace plv
