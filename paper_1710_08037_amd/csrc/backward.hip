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
// in groups of 4 signals (one store4 each), through an LDS tile.
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
    // store: 4 consecutive signals of one sample per thread
    for (int e = tid; e < TB * TB / 4; e += 256) {
        const int ss = e / (TB / 4), kq = (e % (TB / 4)) * 4;
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
// format, from the forward G and the upstream gradients.
template <int MODE>
__global__ __launch_bounds__(256) void metric_adjoint_kernel(BwdMetricArgs a)
{
    typedef typename std::conditional<MODE == M_F64, double, float>::type R;
    typedef typename std::conditional<MODE == M_F64, vd2, vf2>::type cplx_t;
    const int64_t i = a.row0 + blockIdx.y;
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * 4;
    if (j0 >= a.kpad)
        return;
    const int64_t n = a.n;
    auto G = gptr((const cplx_t *)a.g);
    auto up = gptr((const R *)a.dplv), ui_ = gptr((const R *)a.diplv), uc = gptr((const R *)a.dciplv);
    R hr[4], hi[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t j = j0 + v;
        hr[v] = 0;
        hi[v] = 0;
        if (j >= n || j == i)
            continue;
        const int64_t lo = i < j ? i : j, hiw = i < j ? j : i;
        const cplx_t g = G[lo * n + hiw];
        const double r = (double)g.x, m = (double)g.y;
        const double sgn = m > 0.0 ? 1.0 : (m < 0.0 ? -1.0 : 0.0);
        double gr = 0.0, gm = 0.0;
        if (a.dplv) {
            const double w = (double)up[lo * n + hiw] + (double)up[hiw * n + lo];
            const double p = sqrt(r * r + m * m);
            if (p > 0.0) {
                gr += w * r / p;
                gm += w * m / p;
            }
        }
        if (a.diplv)
            gm += ((double)ui_[lo * n + hiw] + (double)ui_[hiw * n + lo]) * sgn;
        if (a.dciplv) {
            const double w = (double)uc[lo * n + hiw] + (double)uc[hiw * n + lo];
            const double dd = (1.0 - r) * (1.0 + r);
            if (dd > 0.0) {
                const double sq = sqrt(dd);
                gm += w * sgn / sq;
                gr += w * fabs(m) * r / (sq * dd);
            }
        }
        // H_ij = Gbar_ij for i < j, conj(Gbar_ji) for i > j; scaled by 1/T
        hr[v] = (R)(gr * a.inv_t);
        hi[v] = (R)((i < j ? gm : -gm) * a.inv_t);
    }
    store4<MODE>(a.h + plane_off(a.rows, cbytes_of(MODE), i, j0), a.plane_bytes, hr, hi);
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
    for (int r0 = 0; r0 < a.n; r0 += MAX_GRID_Y) {
        BwdMetricArgs b = a;
        b.row0 = r0;
        dim3 grid((a.kpad / 4 + 255) / 256, std::min(MAX_GRID_Y, a.n - r0));
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
