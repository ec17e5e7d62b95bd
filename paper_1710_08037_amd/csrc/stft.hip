// stft.hip -- Fourier coefficients of windowed segments, the X_i(f, n) of the
// coherency (Section II.B, Eq. 12): for segment n of row i, starting at
// sample t0 + n * hop,
//   X_i(k, n) = sum_{m < L} w[m] x_i(t0 + n hop + m) exp(-2 pi i (k m mod L) / L)
// for the bins k = k_lo..k_hi of the segment length L (Section III.B computes
// coherence on Hamming-windowed segments).  The coefficients are written as
// complex rows, bin-major ([bin][row][segment]), which the coherency path
// then contracts over the segments.
//
// Bound by the multiply-adds of the direct sums (L per coefficient; a few
// bins per band make a transform of every segment more work).  One
// work-group per (row, run of spw segments, spw = 256 / bins): the twiddle
// table exp(-2 pi i j / L) and the window sit in LDS, the row's samples come
// through the cache; each thread sums one (bin, segment) pair, stepping its
// twiddle index by k mod L.
#include "plv_internal.h"

namespace plv {
namespace {

template <class R>
struct Cplx;
template <>
struct Cplx<float> {
    typedef vf2 type;
};
template <>
struct Cplx<double> {
    typedef vd2 type;
};

template <class R>
__global__ __launch_bounds__(256) void stft_tables_kernel(StftTables a)
{
    typedef typename Cplx<R>::type c_t;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.seg)
        return;
    double s, c;
    sincospi(-2.0 * (double)j / (double)a.seg, &s, &c);  // exp(-2 pi i j / L)
    c_t v;
    v.x = (R)c;
    v.y = (R)s;
    gptr((c_t *)a.tw)[j] = v;
    double w = 1.0;
    if (a.window != PLV_WINDOW_RECT && a.seg > 1) {
        const double cc = cospi(2.0 * (double)j / (double)(a.seg - 1));
        w = a.window == PLV_WINDOW_HAMMING ? 0.54 - 0.46 * cc : 0.5 - 0.5 * cc;
    }
    gptr((R *)a.win)[j] = (R)w;
}

template <class R>
__global__ __launch_bounds__(256) void stft_kernel(StftArgs a)
{
    typedef typename Cplx<R>::type c_t;
    __shared__ c_t tws[STFT_MAX_SEG];
    __shared__ R ws_[STFT_MAX_SEG];

    const int L = a.seg, H = a.hop;
    const int row = a.row0 + blockIdx.y;
    const int s_lo = blockIdx.x * a.spw;
    const int nsp = min(a.spw, a.nseg - s_lo);
    for (int j = threadIdx.x; j < L; j += 256) {
        tws[j] = gptr((const c_t *)a.tw)[j];
        ws_[j] = gptr((const R *)a.win)[j];
    }
    __syncthreads();

    const int nb = a.k_hi - a.k_lo + 1;
    auto x = gptr((const R *)a.x) + (int64_t)row * a.ld + a.t0 + (int64_t)s_lo * H;
    auto out = gptr((c_t *)a.coef);
    for (int p = threadIdx.x; p < nb * nsp; p += 256) {
        // bin-major: consecutive threads take consecutive segments, whose
        // samples (hop apart) stay in the cache across the next iterations
        const int b = p / nsp, s = p - b * nsp;
        const int k = a.k_lo + b;
        auto xr = x + (int64_t)s * H;
        R sr = 0, si = 0;
        int idx = 0;
        for (int m = 0; m < L; ++m) {
            const R v = xr[m] * ws_[m];
            const c_t t = tws[idx];
            sr = fma(v, t.x, sr);
            si = fma(v, t.y, si);
            idx += k;
            idx = idx >= L ? idx - L : idx;
        }
        c_t o;
        o.x = sr;
        o.y = si;
        out[((int64_t)b * a.n + row) * a.nseg + s_lo + s] = o;
    }
}

}  // namespace

hipError_t launch_stft_tables(bool f64, const StftTables &a, hipStream_t s)
{
    const int grid = (a.seg + 255) / 256;
    if (f64)
        stft_tables_kernel<double><<<grid, 256, 0, s>>>(a);
    else
        stft_tables_kernel<float><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_stft(bool f64, const StftArgs &args, hipStream_t s)
{
    StftArgs a = args;
    const int gx = (a.nseg + a.spw - 1) / a.spw;
    for (int r0 = 0; r0 < a.n; r0 += MAX_GRID_Y) {
        a.row0 = r0;
        dim3 grid(gx, std::min(MAX_GRID_Y, a.n - r0));
        if (f64)
            stft_kernel<double><<<grid, 256, 0, s>>>(a);
        else
            stft_kernel<float><<<grid, 256, 0, s>>>(a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace plv
