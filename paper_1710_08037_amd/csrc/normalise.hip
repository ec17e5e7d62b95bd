// normalise.hip -- analytic signal -> unit phasors (Section II.A, Eq. 4).
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
#include "plv_internal.h"

namespace plv {
namespace {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

__device__ inline void unit_phasor(float re, float im, float &ur, float &ui)
{
    if (re == 0.0f && im == 0.0f) {
        ur = 1.0f;
        ui = 0.0f;
        return;
    }
    float m = fmaxf(fabsf(re), fabsf(im));
    int e;
    (void)frexpf(m, &e);
    float a = ldexpf(re, -e), b = ldexpf(im, -e);  // exact rescale, max(|a|,|b|) in [0.5, 1)
    float inv = 1.0f / sqrtf(a * a + b * b);
    ur = a * inv;
    ui = b * inv;
}

__device__ inline void unit_phasor(double re, double im, double &ur, double &ui)
{
    if (re == 0.0 && im == 0.0) {
        ur = 1.0;
        ui = 0.0;
        return;
    }
    double m = fmax(fabs(re), fabs(im));
    int e;
    (void)frexp(m, &e);
    double a = ldexp(re, -e), b = ldexp(im, -e);
    double inv = 1.0 / sqrt(a * a + b * b);
    ur = a * inv;
    ui = b * inv;
}

__device__ inline uint32_t pack_bf16(float a, float b)
{
    bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ inline uint32_t pack_f16(float a, float b)
{
    f16x2 v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

constexpr int VEC = 4;  // samples per thread

template <int MODE>
__global__ __launch_bounds__(256) void normalise_kernel(NormArgs a)
{
    const int row = blockIdx.y;
    const int s0 = (blockIdx.x * 256 + threadIdx.x) * VEC;
    if (s0 >= a.tpad)
        return;
    auto dst = gptr(a.u + ((int64_t)row * a.ldu + s0) * cbytes_of(MODE));

    if constexpr (MODE == M_F64) {
        auto src = gptr((const vd2 *)a.in + (int64_t)row * a.ld + a.t0);
        vd2 out[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int s = s0 + v;
            double ur = 0.0, ui = 0.0;
            if (s < a.tw) {
                vd2 z = src[s];
                unit_phasor(z.x, z.y, ur, ui);
            }
            out[v] = vd2{ur, ui};
        }
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            ((PLV_GLOBAL vd2 *)dst)[v] = out[v];
    } else {
        auto src = gptr((const vf2 *)a.in + (int64_t)row * a.ld + a.t0);
        float ur[VEC], ui[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int s = s0 + v;
            ur[v] = 0.0f;
            ui[v] = 0.0f;
            if (s < a.tw) {
                vf2 z = src[s];
                unit_phasor(z.x, z.y, ur[v], ui[v]);
            }
        }
        if constexpr (MODE == M_F32) {
            auto d = (PLV_GLOBAL vf4 *)dst;
            d[0] = vf4{ur[0], ui[0], ur[1], ui[1]};
            d[1] = vf4{ur[2], ui[2], ur[3], ui[3]};
        } else if constexpr (MODE == M_BF16) {
            *(PLV_GLOBAL vu4 *)dst =
                vu4{pack_bf16(ur[0], ui[0]), pack_bf16(ur[1], ui[1]), pack_bf16(ur[2], ui[2]), pack_bf16(ur[3], ui[3])};
        } else if constexpr (MODE == M_F16) {
            *(PLV_GLOBAL vu4 *)dst =
                vu4{pack_f16(ur[0], ui[0]), pack_f16(ur[1], ui[1]), pack_f16(ur[2], ui[2]), pack_f16(ur[3], ui[3])};
        } else {  // M_SPLIT: hi = rn(u), lo = rn(u - hi); u - hi is exact in FP32
            uint32_t hw[VEC], lw[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                hw[v] = pack_bf16(ur[v], ui[v]);
                lw[v] = pack_bf16(ur[v] - bf16_lo(hw[v]), ui[v] - bf16_hi(hw[v]));
            }
            *(PLV_GLOBAL vu4 *)dst = vu4{hw[0], hw[1], hw[2], hw[3]};
            *(PLV_GLOBAL vu4 *)(dst + a.plane_bytes) = vu4{lw[0], lw[1], lw[2], lw[3]};
        }
    }
}

}  // namespace

hipError_t launch_normalise(int mode, const NormArgs &a, hipStream_t s)
{
    dim3 grid((a.tpad + 256 * VEC - 1) / (256 * VEC), a.n);
    switch (mode) {
    case M_F64: normalise_kernel<M_F64><<<grid, 256, 0, s>>>(a); break;
    case M_F32: normalise_kernel<M_F32><<<grid, 256, 0, s>>>(a); break;
    case M_SPLIT: normalise_kernel<M_SPLIT><<<grid, 256, 0, s>>>(a); break;
    case M_BF16: normalise_kernel<M_BF16><<<grid, 256, 0, s>>>(a); break;
    case M_F16: normalise_kernel<M_F16><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace plv
