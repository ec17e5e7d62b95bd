// backward.hip -- adjoint of the PLV path (not in the paper; derived from the
// forward map).  With G = U U^H / T, PLV = |G|, iPLV = |Im G| and
// ciPLV = |Im G| / sqrt(1 - Re^2) (Eqs. 2, 13, 14) and u = z / |z| (Eq. 4):
//
//   Gbar_ij (i < j) = dL/dRe G_ij + i dL/dIm G_ij from the metric derivatives,
//                     with the upstream gradients of (i, j) and (j, i) added;
//   H = (Gbar + Gbar^H) / T, so that dL/dU = H U  (computed on MFMA as
//                     H (conj U^T)^H by the Gram kernel's general mode);
//   zbar = i Im(conj(u) ubar) u / |z|  (0 at z = 0): the phase direction only.
//
// Kernels here: the transposed, conjugated phasor planes (the product's B
// operand), the metric adjoint that writes H in the operand format (its A
// operand), and the normalisation adjoint.
#include "phasor.h"

namespace plv {
namespace {

constexpr int TB = 64;  // transpose block: 64 signals x 64 samples

// W[s][k] = conj(u_k(s)) for s < tw, k < kpad (0 for k >= n): rows are
// samples, K runs over signals.  Reads z coalesced along samples, writes W
// in groups of 4 signals (one store4 each) along its plane stages, through
// an LDS tile.
template <int MODE>
__global__ __launch_bounds__(256) void planes_t_kernel(BwdPlanesArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type R;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    __shared__ R tre[TB][TB + 1], tim[TB][TB + 1];
    const int s0 = blockIdx.x * TB, k0 = blockIdx.y * TB;
    const int tid = threadIdx.x;
    // load: thread (kk = tid / 4 .. , ss strided) reads along samples
    for (int e = tid; e < TB * TB; e += 256) {
        const int kk = e / TB, ss = e % TB;
        const int k = k0 + kk, s = s0 + ss;
        R ur = 0, ui = 0;
        if (k < a.n && s < a.tw) {
            const cplx_t z = gptr((const cplx_t *)a.z)[(int64_t)k * a.ldz + s];
            unit_phasor(z.x, z.y, ur, ui);
            ui = -ui;  // conjugate
        }
        tre[kk][ss] = ur;
        tim[kk][ss] = ui;
    }
    __syncthreads();
    // store: 4 consecutive signals of one sample per thread; consecutive
    // threads fill one plane stage (SPS signals) of a row, then the next rows,
    // so a wave writes one contiguous run of the stage-major planes
    constexpr int SPS = 64 / cbytes_of(MODE);  // signals per plane stage
    constexpr int QS = SPS / 4;                // threads per row stage
    for (int e = tid; e < TB * TB / 4; e += 256) {
        const int ss = (e / QS) % TB, kq = (e / (QS * TB)) * SPS + (e % QS) * 4;
        const int s = s0 + ss;
        // kpad is a multiple of 32, not of the 64-wide block: stop at the row end
        if (s >= a.tw || k0 + kq >= a.kpad)
            continue;
        R ur[4], ui[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ur[v] = tre[kq + v][ss];
            ui[v] = tim[kq + v][ss];
        }
        store4<MODE>(a.w + plane_off(a.rows, cbytes_of(MODE), s, k0 + kq), a.plane_bytes, ur, ui);
    }
}

// H[i][j] for j < kpad (0 for j >= n and on the diagonal), in the operand
// format, from the forward G and the upstream gradients.  A thread owns a
// 4 x 4 block (rows i0.., columns j0..); a wave covers 32 x 32 as 8 x 8 such
// blocks, so every read below takes whole 128-byte runs of a row.  G comes
// from row i: the forward stores G_ji as the exact conjugate of G_ij, so
// G_{min(i,j), max(i,j)} is G_ij or its conjugate.  The upstream weight of
// pair {i, j} is dL/dy_ij + dL/dy_ji; the (j, i) entries are read along the
// rows j of the transposed block, and the 4 x 4 transpose is free in
// registers.
template <int MODE>
__global__ __launch_bounds__(256) void metric_adjoint_kernel(BwdMetricArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type R;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)a.row0 + (int64_t)blockIdx.y * 32 + (lane >> 3) * 4;
    const int64_t j0 = (int64_t)blockIdx.x * 128 + wave * 32 + (lane & 7) * 4;
    if (i0 >= a.n || j0 >= a.kpad)
        return;
    const int64_t n = a.n;
    auto G = gptr((const cplx_t *)a.g);
    R gx[4][4], gy[4][4];  // Re and Im of G_{min(i,j), max(i,j)}
    double gr[4][4], gm[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int64_t i = i0 + x, j = j0 + y;
            gx[x][y] = 0;
            gy[x][y] = 0;
            gr[x][y] = 0.0;
            gm[x][y] = 0.0;
            if (i < n && j < n) {
                const cplx_t g = G[i * n + j];
                gx[x][y] = g.x;
                gy[x][y] = i < j ? g.y : -g.y;
            }
        }
    // w[x][y] = u(i, j) + u(j, i) over the block (0 outside n)
    auto weights = [&](const void *up, double (&w)[4][4]) {
        auto u = gptr((const R *)up);
        R d[4][4], t[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                d[x][y] = 0;
                t[y][x] = 0;
                if (i0 + x < n && j0 + y < n) {
                    d[x][y] = u[(i0 + x) * n + j0 + y];
                    t[y][x] = u[(j0 + y) * n + i0 + x];
                }
            }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                w[x][y] = (double)d[x][y] + (double)t[y][x];
    };
    double w[4][4];
    if (a.dplv) {
        weights(a.dplv, w);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const double r = (double)gx[x][y], m = (double)gy[x][y];
                const double p = sqrt(r * r + m * m);
                if (p > 0.0) {
                    gr[x][y] += w[x][y] * r / p;
                    gm[x][y] += w[x][y] * m / p;
                }
            }
    }
    if (a.diplv) {
        weights(a.diplv, w);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const double m = (double)gy[x][y];
                const double sgn = m > 0.0 ? 1.0 : (m < 0.0 ? -1.0 : 0.0);
                gm[x][y] += w[x][y] * sgn;
            }
    }
    if (a.dciplv) {
        weights(a.dciplv, w);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const double r = (double)gx[x][y], m = (double)gy[x][y];
                const double sgn = m > 0.0 ? 1.0 : (m < 0.0 ? -1.0 : 0.0);
                const double dd = (1.0 - r) * (1.0 + r);
                if (dd > 0.0) {
                    const double sq = sqrt(dd);
                    gm[x][y] += w[x][y] * sgn / sq;
                    gr[x][y] += w[x][y] * fabs(m) * r / (sq * dd);
                }
            }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int64_t i = i0 + x;
        if (i >= n)
            break;
        R hr[4], hi[4];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int64_t j = j0 + y;
            // H_ij = Gbar_ij for i < j, conj(Gbar_ji) for i > j; scaled by 1/T
            const bool live = j < n && j != i;
            hr[y] = live ? (R)(gr[x][y] * a.inv_t) : (R)0;
            hi[y] = live ? (R)((i < j ? gm[x][y] : -gm[x][y]) * a.inv_t) : (R)0;
        }
        store4<MODE>(a.h + plane_off(a.rows, cbytes_of(MODE), i, j0), a.plane_bytes, hr, hi);
    }
}

// zbar = i Im(conj(u) ubar) u / |z| on the window; for the full-row form
// (analytic input) samples outside the window get 0.
template <class R>
__global__ __launch_bounds__(256) void normalise_adjoint_kernel(BwdNormArgs a)
{
    typedef typename std::conditional<sizeof(R) == 8, vd2, vf2>::type cplx_t;
    const int64_t row = a.row0 + blockIdx.y;
    const int q = blockIdx.x * 256 + threadIdx.x;  // position in the output row
    if (q >= a.len)
        return;
    const int s = q - a.off;  // sample in the window
    cplx_t out;
    out.x = 0;
    out.y = 0;
    if (s >= 0 && s < a.tw) {
        const cplx_t z = gptr((const cplx_t *)a.z)[row * a.ldz + s];
        const cplx_t ub = gptr((const cplx_t *)a.c)[row * a.ldc + s];
        if (!(z.x == 0 && z.y == 0)) {
            R ur, ui;
            unit_phasor(z.x, z.y, ur, ui);
            // |z| from the same exact rescaling as the phasor
            const R m = fmax(fabs(z.x), fabs(z.y));
            int e;
            (void)frexp(m, &e);
            const R az = ldexp(z.x, -e), bz = ldexp(z.y, -e);
            const R rinv = ldexp((R)1 / sqrt(az * az + bz * bz), -e);  // 1 / |z|
            const R w = ur * ub.y - ui * ub.x;  // Im(conj(u) ubar)
            out.x = -w * ui * rinv;
            out.y = w * ur * rinv;
        }
    }
    gptr((cplx_t *)a.dst)[row * a.ldd + q] = out;
}

}  // namespace

hipError_t launch_planes_t(int mode, const BwdPlanesArgs &a, hipStream_t s)
{
    dim3 grid((a.tw + TB - 1) / TB, (a.kpad + TB - 1) / TB);
    switch (mode) {
    case M_F64: planes_t_kernel<M_F64><<<grid, 256, 0, s>>>(a); break;
    case M_F32: planes_t_kernel<M_F32><<<grid, 256, 0, s>>>(a); break;
    case M_SPLIT: planes_t_kernel<M_SPLIT><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_metric_adjoint(int mode, const BwdMetricArgs &a, hipStream_t s)
{
    for (int64_t r0 = 0; r0 < a.n; r0 += (int64_t)MAX_GRID_Y * 32) {
        BwdMetricArgs b = a;
        b.row0 = (int32_t)r0;
        dim3 grid((a.kpad + 127) / 128, (unsigned)std::min<int64_t>(MAX_GRID_Y, (a.n - r0 + 31) / 32));
        switch (mode) {
        case M_F64: metric_adjoint_kernel<M_F64><<<grid, 256, 0, s>>>(b); break;
        case M_F32: metric_adjoint_kernel<M_F32><<<grid, 256, 0, s>>>(b); break;
        case M_SPLIT: metric_adjoint_kernel<M_SPLIT><<<grid, 256, 0, s>>>(b); break;
        default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_normalise_adjoint(bool f64, const BwdNormArgs &a, hipStream_t s)
{
    for (int r0 = 0; r0 < a.n; r0 += MAX_GRID_Y) {
        BwdNormArgs b = a;
        b.row0 = r0;
        dim3 grid((a.len + 255) / 256, std::min(MAX_GRID_Y, a.n - r0));
        if (f64)
            normalise_adjoint_kernel<double><<<grid, 256, 0, s>>>(b);
        else
            normalise_adjoint_kernel<float><<<grid, 256, 0, s>>>(b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace plv
