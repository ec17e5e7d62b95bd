// phasor.h -- unit-phasor normalisation (Section II.A, Eq. 4) and the packing of
// phasors into the Gram kernel's operand formats.  Shared by the kernels that
// write phasor planes (normalise.hip, fft.hip).
#pragma once

#include "plv_internal.h"

namespace plv {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// u = z / |z|.  When the larger component lies in [2^-60, 2^60], re^2 + im^2
// is a normal FP32 number and one hardware reciprocal square root (about 1
// ulp) gives 1/|z|.  Otherwise |z| is formed from components rescaled by an
// exact power of two (no under/overflow for any finite z); z = 0 (either zero
// sign) -> 1 + 0i, the phasor of angle(0) = 0.  NaN/Inf propagate as NaN.
__device__ inline void unit_phasor(float re, float im, float &ur, float &ui)
{
    float m = fmaxf(fabsf(re), fabsf(im));
    if (m >= 0x1p-60f && m <= 0x1p60f) {
        const float inv = __builtin_amdgcn_rsqf(fmaf(re, re, im * im));
        ur = re * inv;
        ui = im * inv;
        return;
    }
    if (re == 0.0f && im == 0.0f) {
        ur = 1.0f;
        ui = 0.0f;
        return;
    }
    int e;
    (void)frexpf(m, &e);
    float a = ldexpf(re, -e), b = ldexpf(im, -e);  // exact rescale, max(|a|,|b|) in [0.5, 1)
    float inv = 1.0f / sqrtf(a * a + b * b);
    ur = a * inv;
    ui = b * inv;
}

// Four samples at once, with one branch: the hardware reciprocal square
// root for all four while every |z|^2 is a normal number well inside FP32's
// range (then no square underflows to a loss or overflows), else the full
// function for all four.
__device__ inline void unit_phasor4(const float (&re)[4], const float (&im)[4], float (&ur)[4], float (&ui)[4])
{
    bool all_ok = true;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float n2 = fmaf(re[v], re[v], im[v] * im[v]);
        // 2^-120 <= n2 <= 2^120 as one unsigned test on the bits (NaN and 0 fail)
        all_ok = all_ok && __float_as_uint(n2) - 0x03800000u <= 0x78000000u;
        const float inv = __builtin_amdgcn_rsqf(n2);
        ur[v] = re[v] * inv;
        ui[v] = im[v] * inv;
    }
    if (!all_ok) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            unit_phasor(re[v], im[v], ur[v], ui[v]);
    }
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

// Stores 4 consecutive phasors (ur[v], ui[v]) of one row at `dst` in the
// operand format of `MODE` (dst points at sample s0 of plane 0; the split
// mode's lo plane is plane_bytes further).
// One 16-byte store, streaming (non-temporal) when NT: the caller's planes
// are read back only by a later kernel, long after they have left the cache.
template <bool NT, class V>
__device__ inline void st16(uint8_t *dst, V v)
{
    auto p = (PLV_GLOBAL V *)gptr(dst);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int MODE, class R, bool NT = false>
__device__ inline void store4(uint8_t *dst, int64_t plane_bytes, const R (&ur)[4], const R (&ui)[4])
{
    if constexpr (MODE == M_F64) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            st16<NT>(dst + 16 * v, vd2{(double)ur[v], (double)ui[v]});
    } else if constexpr (MODE == M_F32) {
        st16<NT>(dst, vf4{(float)ur[0], (float)ui[0], (float)ur[1], (float)ui[1]});
        st16<NT>(dst + 16, vf4{(float)ur[2], (float)ui[2], (float)ur[3], (float)ui[3]});
    } else if constexpr (MODE == M_BF16) {
        st16<NT>(dst, vu4{pack_bf16(ur[0], ui[0]), pack_bf16(ur[1], ui[1]), pack_bf16(ur[2], ui[2]),
                          pack_bf16(ur[3], ui[3])});
    } else if constexpr (MODE == M_F16) {
        st16<NT>(dst, vu4{pack_f16(ur[0], ui[0]), pack_f16(ur[1], ui[1]), pack_f16(ur[2], ui[2]), pack_f16(ur[3], ui[3])});
    } else {  // M_SPLIT: hi = rn(u), lo = rn(u - hi); u - hi is exact in FP32
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            hw[v] = pack_bf16(ur[v], ui[v]);
            lw[v] = pack_bf16(ur[v] - bf16_lo(hw[v]), ui[v] - bf16_hi(hw[v]));
        }
        st16<NT>(dst, vu4{hw[0], hw[1], hw[2], hw[3]});
        st16<NT>(dst + plane_bytes, vu4{lw[0], lw[1], lw[2], lw[3]});
    }
}

}  // namespace plv
