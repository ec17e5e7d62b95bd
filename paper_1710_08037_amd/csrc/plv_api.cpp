// plv_api.cpp -- the C ABI declared in include/plv.h.
//
// Host side only: argument checks, the workspace plan (where each problem's
// phasor planes, partial sums and the device-side work tables live), the
// K-chunk choice, and the kernel launches on the caller's stream.  Every step
// of the computation runs in the gfx950 kernels; nothing here touches data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plv_internal.h"
#include "plv_plan.h"

using namespace plv;

// Device scratch of plv_from_analytic_noalloc: one copy of this array per
// GPU the library runs on, held until the process ends.  Host code never
// uses its name as an address (that is a host-side stand-in); the device
// address of each GPU's copy is looked up once per device, in plv_create
// with that device current, and kept in scratch_ptr.
static __device__ __align__(256) uint8_t scratch[PLV_NOALLOC_MAX_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];          // device address of each device's copy, or nullptr
hipError_t scratch_err[MAX_DEVICES];     // the lookup's result when it failed
}  // namespace

struct TimingRec {
    int stage;
    int launches;
    hipEvent_t start, stop;
};

struct plv_ctx {
    int device = -1;
    int cus = 256;
    int occ[NOCC] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1};  // Gram work-groups per CU (occ_index)
    std::string err;
    void *staging = nullptr;  // pinned host buffer for the work tables
    size_t staging_bytes = 0;
    hipEvent_t staging_done = nullptr;
    bool staging_pending = false;
    bool timing = false;
    std::vector<TimingRec> recs;   // recorded, not yet read
    std::vector<hipEvent_t> pool;  // idle events
    plv::Tuning tune;              // measured K-chunk counts and tile edges (plv_autotune)
    void *scratch = nullptr;       // this device's copy of `scratch` (plv_from_analytic_noalloc)
    hipError_t scratch_err = hipSuccess;
};

namespace {

plv_status fail(plv_ctx *ctx, plv_status s, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return s;
}

plv_status hip_fail(plv_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, PLV_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Copy the work tables to the device through the context's pinned buffer.
plv_status upload(plv_ctx *ctx, const std::vector<uint8_t> &blob, void *dst, hipStream_t s)
{
    if (blob.empty())
        return PLV_OK;
    hipError_t e;
    if (ctx->staging_pending) {
        // the previous call's copy may still be reading the buffer
        if ((e = hipEventSynchronize(ctx->staging_done)) != hipSuccess)
            return hip_fail(ctx, e, "hipEventSynchronize");
        ctx->staging_pending = false;
    }
    if (blob.size() > ctx->staging_bytes) {
        if (ctx->staging)
            (void)hipHostFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        size_t want = std::max<size_t>(blob.size(), size_t(1) << 20);
        if ((e = hipHostMalloc(&ctx->staging, want, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(ctx, e, "hipHostMalloc");
        ctx->staging_bytes = want;
    }
    memcpy(ctx->staging, blob.data(), blob.size());
    if ((e = hipMemcpyAsync(dst, ctx->staging, blob.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync");
    if ((e = hipEventRecord(ctx->staging_done, s)) != hipSuccess)
        return hip_fail(ctx, e, "hipEventRecord");
    ctx->staging_pending = true;
    return PLV_OK;
}

hipEvent_t take_event(plv_ctx *ctx)
{
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Brackets one stage with an event pair when timing is on.
struct StageTimer {
    plv_ctx *ctx;
    hipStream_t s;
    TimingRec rec{};
    bool on = false;
    StageTimer(plv_ctx *c, int stage, hipStream_t st) : ctx(c), s(st)
    {
        if (!ctx->timing)
            return;
        rec.stage = stage;
        rec.start = take_event(ctx);
        rec.stop = take_event(ctx);
        on = rec.start && rec.stop && hipEventRecord(rec.start, s) == hipSuccess;
    }
    void launched(int k = 1) { rec.launches += k; }
    ~StageTimer()
    {
        if (on && hipEventRecord(rec.stop, s) == hipSuccess)
            ctx->recs.push_back(rec);
        else {
            if (rec.start)
                ctx->pool.push_back(rec.start);
            if (rec.stop)
                ctx->pool.push_back(rec.stop);
        }
    }
};

}  // namespace

// Times `runs` executions of run() between HIP events on stream s, after one
// untimed execution.  ms < 0 when a launch or event failed (st / e say which).
template <class F>
static float time_runs(F run, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int runs, plv_status &st, hipError_t &e)
{
    if ((st = run()) != PLV_OK)
        return -1.0f;
    if ((e = hipEventRecord(e0, s)) != hipSuccess)
        return -1.0f;
    for (int r = 0; r < runs && st == PLV_OK; ++r)
        st = run();
    if (st != PLV_OK)
        return -1.0f;
    float ms = 0.0f;
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
        (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        return -1.0f;
    return ms;
}

extern "C" {

plv_status plv_timing_enable(plv_ctx *ctx, int32_t on)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    ctx->timing = on != 0 && ctx->device >= 0;
    return PLV_OK;
}

plv_status plv_timing_read(plv_ctx *ctx, plv_timing *out, int32_t reset)
{
    if (!ctx || !out)
        return PLV_ERR_INVALID_ARG;
    memset(out, 0, sizeof *out);
    for (const TimingRec &r : ctx->recs) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess)
            return hip_fail(ctx, e, "reading stage timing events");
        out->ms[r.stage] += ms;
        out->calls[r.stage] += 1;
        out->launches[r.stage] += r.launches;
    }
    if (reset) {
        for (const TimingRec &r : ctx->recs) {
            ctx->pool.push_back(r.start);
            ctx->pool.push_back(r.stop);
        }
        ctx->recs.clear();
    }
    return PLV_OK;
}

plv_status plv_timing_list(plv_ctx *ctx, int32_t stage, double *ms, int32_t *launches, int64_t cap,
                           int64_t *count)
{
    if (!ctx || !count || stage < 0 || stage >= PLV_NSTAGES || cap < 0 || (cap > 0 && !ms))
        return PLV_ERR_INVALID_ARG;
    int64_t k = 0;
    for (const TimingRec &r : ctx->recs) {
        if (r.stage != stage)
            continue;
        if (k < cap) {
            float v = 0.0f;
            hipError_t e = hipEventSynchronize(r.stop);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&v, r.start, r.stop);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "reading stage timing events");
            ms[k] = v;
            if (launches)
                launches[k] = r.launches;
        }
        ++k;
    }
    *count = k;
    return PLV_OK;
}

int32_t plv_version(void) { return 10100; }

const char *plv_status_str(plv_status s)
{
    switch (s) {
    case PLV_OK: return "ok";
    case PLV_ERR_INVALID_ARG: return "invalid argument";
    case PLV_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case PLV_ERR_DEVICE: return "HIP runtime or launch failure";
    case PLV_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *plv_last_error(const plv_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

plv_status plv_create(plv_ctx **out, int device)
{
    if (!out)
        return PLV_ERR_INVALID_ARG;
    *out = nullptr;
    plv_ctx *ctx = new (std::nothrow) plv_ctx;
    if (!ctx)
        return PLV_ERR_DEVICE;
    if (device >= 0) {
        int cur = 0, ndev = 0;
        hipError_t e;
        if ((e = hipGetDeviceCount(&ndev)) != hipSuccess || device >= ndev) {
            delete ctx;
            return e != hipSuccess ? PLV_ERR_DEVICE : PLV_ERR_INVALID_ARG;
        }
        (void)hipGetDevice(&cur);
        if ((e = hipSetDevice(device)) != hipSuccess) {
            delete ctx;
            return PLV_ERR_DEVICE;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            ctx->cus = cus;
        for (int m = 0; m < 5; ++m)
            for (int bm : {64, 128})
                if (tile_supported(m, bm))
                    ctx->occ[occ_index(m, bm)] = herk_occupancy(m, bm);
        if (device < MAX_DEVICES) {
            // once per device, with the device current: its copy of the scratch array
            std::lock_guard<std::mutex> lk(scratch_mu);
            if (!scratch_ptr[device] && scratch_err[device] == hipSuccess) {
                void *p = nullptr;
                const hipError_t se = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
                if (se == hipSuccess && p)
                    scratch_ptr[device] = p;
                else
                    scratch_err[device] = se != hipSuccess ? se : hipErrorInvalidSymbol;
            }
            ctx->scratch = scratch_ptr[device];
            ctx->scratch_err = scratch_err[device];
        }
        e = hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming);
        (void)hipSetDevice(cur);
        if (e != hipSuccess) {
            delete ctx;
            return PLV_ERR_DEVICE;
        }
        ctx->device = device;
    }
    *out = ctx;
    return PLV_OK;
}

plv_status plv_destroy(plv_ctx *ctx)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    if (ctx->staging_pending)
        (void)hipEventSynchronize(ctx->staging_done);
    if (ctx->staging)
        (void)hipHostFree(ctx->staging);
    if (ctx->staging_done)
        (void)hipEventDestroy(ctx->staging_done);
    for (const TimingRec &r : ctx->recs) {
        (void)hipEventSynchronize(r.stop);
        ctx->pool.push_back(r.start);
        ctx->pool.push_back(r.stop);
    }
    for (hipEvent_t e : ctx->pool)
        (void)hipEventDestroy(e);
    delete ctx;
    return PLV_OK;
}

static plv_status workspace_size(const plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs,
                                 int64_t nprob, const plv_band *bands, int32_t nbands, size_t *bytes, bool unit_k)
{
    if (!bytes)
        return PLV_ERR_INVALID_ARG;
    *bytes = 0;
    Plan plan;
    std::string why;
    plv_status st = make_plan(ctx ? ctx->cus : 256, ctx ? ctx->occ : nullptr, op, prec, probs, nprob, bands, nbands,
                              plan, why, ctx ? &ctx->tune : nullptr, unit_k);
    if (st != PLV_OK) {
        if (ctx)
            const_cast<plv_ctx *>(ctx)->err = why;
        return st;
    }
    *bytes = plan.total;
    return PLV_OK;
}

plv_status plv_workspace_size(const plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs,
                              int64_t nprob, const plv_band *bands, int32_t nbands, size_t *bytes)
{
    return workspace_size(ctx, op, prec, probs, nprob, bands, nbands, bytes, false);
}

// Shared front half of the compute entry points: checks, plan, device.
// `unit_k` as in make_plan.
static plv_status begin(plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs, int64_t nprob,
                        const plv_band *bands, int32_t nbands, void *ws, size_t ws_bytes, Plan &plan,
                        bool unit_k = false)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    ctx->err.clear();
    if (ctx->device < 0)
        return fail(ctx, PLV_ERR_INVALID_ARG, "host-only context cannot compute");
    std::string why;
    plv_status st =
        make_plan(ctx->cus, ctx->occ, op, prec, probs, nprob, bands, nbands, plan, why, &ctx->tune, unit_k);
    if (st != PLV_OK)
        return fail(ctx, st, "%s", why.c_str());
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(ctx, PLV_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < plan.total)
        return fail(ctx, PLV_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, plan.total);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipSetDevice");
    return PLV_OK;
}

// Bins of the band [f_lo, f_hi] for a row of length t: the positive-frequency
// bins k (0 < k, 2k < t) with f_lo <= k*fs/t <= f_hi, compared in FP64.
// f_lo = f_hi = 0 selects the plain one-sided weights (klo = -1).
static BandBins band_bins(int t, double fs, const plv_band *band)
{
    if (!band || (band->f_lo == 0.0 && band->f_hi == 0.0))
        return BandBins{-1, -1};
    const int kmax = (t - 1) / 2;
    auto freq = [&](int k) { return (double)k * fs / (double)t; };
    int klo = std::max(1, (int)std::floor(band->f_lo * t / fs) - 2);
    while (klo <= kmax && freq(klo) < band->f_lo)
        ++klo;
    int khi = std::min(kmax, (int)std::ceil(band->f_hi * t / fs) + 2);
    while (khi >= 1 && freq(khi) > band->f_hi)
        --khi;
    if (klo > khi)
        return BandBins{1, 0};  // empty band: every weight 0
    return BandBins{klo, khi};
}

// Forward-backward FIR band-pass (the paper's pre-Hilbert filter, Section
// III, design not given there): taps c_m = ideal band-pass between f_lo and
// f_hi at n = m - L/2 times the Hamming window 0.54 - 0.46 cos(2 pi m / L),
// m = 0..L, scaled to unit gain at the band centre.  The taps are symmetric
// about L/2, so H(e^{i theta}) = e^{-i theta L/2} A(theta) with the real
// A(theta) = c_{L/2} + 2 sum_{j=1..L/2} c_{L/2+j} cos(j theta), and forward
// then backward filtering has the zero-phase gain A^2, which the weight-table
// kernel evaluates.  Returns c_{L/2}, ..., c_L (FP64).
static std::vector<double> fir_half_taps(const plv_band &band, double fs)
{
    const int L = band.fir_order, half = L / 2;
    const double pi = 3.141592653589793238462643383279502884;
    const double lo = band.f_lo / fs, hi = band.f_hi / fs, mid = 0.5 * (lo + hi);
    std::vector<double> c((size_t)half + 1);
    double gain = 0.0;
    for (int j = 0; j <= half; ++j) {
        const double n = (double)j;
        const double ideal = j == 0 ? 2.0 * (hi - lo) : (std::sin(2.0 * pi * hi * n) - std::sin(2.0 * pi * lo * n)) / (pi * n);
        c[j] = ideal * (0.54 - 0.46 * std::cos(2.0 * pi * (double)(half + j) / (double)L));
        gain += (j == 0 ? 1.0 : 2.0) * c[j] * std::cos(2.0 * pi * mid * n);
    }
    for (double &v : c)
        v /= gain;
    return c;
}

// Direct synthesis of a band costs about 4 K + 12 operations per output
// sample (K bins); the inverse transform about (2.5 log2 M + 6) M / t per
// sample, twice for a Bluestein length.  The cheaper one is taken.
static bool direct_band(const FftPlan &f, BandBins bb)
{
    if (bb.klo < 0 || bb.fir || !f.has_xbins)
        return false;  // plain analytic signal: every positive bin
    const int k = bb.khi >= bb.klo ? bb.khi - bb.klo + 1 : 0;
    if (k > DIRECT_KMAX)
        return false;  // more bins than a slot holds
    const double direct = 4.0 * k + 12.0;
    const double fft = (f.blue ? 2.0 : 1.0) * (double)(1 << f.logm) / (double)f.t * (2.5 * f.logm + 6.0);
    return direct < fft;
}

// Host tables of the FFT stage in the upload blob: problems, band bins, rows
// grouped by FFT size (class_start / class_count per size), per-length jobs.
// A problem whose bands are all synthesised from their bins, with at most
// DFT_MAX_BINS bins in all, takes them from the DFT-bins kernel (an MFMA
// product with the row) rather than a whole transform of the row (forward
// calls in the FP32 modes).  Its rows stay out of the transform launches.
static void fill_fft_tables(const Plan &plan, const plv_problem *probs, const plv_grad *grads,
                            const plv_band *bands, int nbands, double fs, uint8_t *ws, std::vector<uint8_t> &blob,
                            std::vector<int> &class_start, std::vector<int> &class_count, bool &any_direct,
                            int64_t &synth_jobs, int64_t &dft_jobs)
{
    any_direct = false;
    synth_jobs = 0;
    dft_jobs = 0;
    const bool backward = plan.op == PLV_OP_BACKWARD_REAL;
    int32_t *prefix = (int32_t *)(blob.data() + plan.synth_off);
    int32_t *dprefix = (int32_t *)(blob.data() + plan.dftp_off);
    std::vector<char> by_dft(plan.fft.size(), 0);
    const size_t nprob = plan.fft.size();
    HilbertProb *hp = (HilbertProb *)(blob.data() + plan.hp_off);
    BandBins *bins = (BandBins *)(blob.data() + plan.bin_off);
    RowRef *rows = (RowRef *)(blob.data() + plan.row_off);
    ChirpJob *jobs = (ChirpJob *)(blob.data() + plan.job_off);
    for (size_t q = 0; q < nprob; ++q) {
        const FftPlan &f = plan.fft[q];
        const LenPlan &l = plan.lens[f.len_index];
        const plv_problem &p = probs[q];
        HilbertProb h{};
        h.x = p.in;
        h.ld = p.ld;
        h.n = (int32_t)p.n;
        h.t = f.t;
        h.t0 = (int32_t)p.t0;
        h.tw = plan.grams[q * nbands].t;
        h.logm = f.logm;
        h.blue = f.blue ? 1 : 0;
        h.chirp = f.blue ? ws + l.chirp_off : nullptr;
        h.bhat = f.blue ? ws + l.bhat_off : nullptr;
        h.tw_tab = ws + plan.tw_off[f.tw_index];
        h.roots = ws + l.roots_off;
        h.gram0 = (int32_t)(q * nbands);
        h.nbands = nbands;
        h.bin0 = (int32_t)(q * nbands);
        h.xbar = grads ? grads[q].din : nullptr;
        h.xbins = f.has_xbins ? ws + f.xbin_off : nullptr;
        hp[q] = h;
        for (int b = 0; b < nbands; ++b) {
            BandBins bb{};
            if (bands && bands[b].fir_order > 0) {
                bb.fir = 1;  // every bin weighted: inverse transform
                bb.w = ws + plan.lens[f.len_index].firw_off[b];
            } else {
                bb = band_bins(f.t, fs, bands ? &bands[b] : nullptr);
            }
            // (the adjoint kernel takes every band through the transform)
            bb.direct = direct_band(f, bb) ? 1 : 0;
            any_direct = any_direct || bb.direct;
            bins[q * nbands + b] = bb;
        }
        int kt = 0;
        bool all_direct = !backward && plan.mode != M_F64;
        for (int b = 0; b < nbands; ++b) {
            const BandBins &bb = bins[q * nbands + b];
            all_direct = all_direct && bb.direct;
            kt += bb.khi >= bb.klo ? bb.khi - bb.klo + 1 : 0;
        }
        by_dft[q] = all_direct && kt <= DFT_MAX_BINS;
        dprefix[q] = (int32_t)std::min<int64_t>(dft_jobs, INT32_MAX);
        if (by_dft[q])
            dft_jobs += (p.n + DFT_ROWS_PER_WG - 1) / DFT_ROWS_PER_WG;
        // band synthesis work-groups of this problem (band_synth_kernel's decode)
        const GramPlan &g0 = plan.grams[q * nbands];
        const int64_t len = backward ? g0.t : g0.tpad;
        prefix[q] = (int32_t)synth_jobs;
        synth_jobs += (int64_t)nbands * ((len + SYNTH_S - 1) / SYNTH_S) * ((p.n + SYNTH_R - 1) / SYNTH_R);
    }
    prefix[nprob] = (int32_t)std::min<int64_t>(synth_jobs, INT32_MAX);
    dprefix[nprob] = (int32_t)std::min<int64_t>(dft_jobs, INT32_MAX);
    size_t r = 0;
    for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
        class_start.push_back((int)r);
        for (size_t q = 0; q < nprob; ++q)
            if (plan.fft[q].logm == plan.tw_logm[c] && !by_dft[q])
                for (int64_t i = 0; i < probs[q].n; ++i)
                    rows[r++] = RowRef{(int32_t)q, (int32_t)i};
        class_count.push_back((int)r - class_start.back());
    }
    // FIR bands: half of the (symmetric) taps, and a weight-table job per row length
    FirJob *fj = (FirJob *)(blob.data() + plan.firjob_off);
    int nj = 0;
    for (int b = 0; bands && b < nbands; ++b) {
        if (bands[b].fir_order <= 0)
            continue;
        const std::vector<double> c = fir_half_taps(bands[b], fs);
        memcpy(blob.data() + plan.fir_r_off[b], c.data(), c.size() * sizeof(double));
        for (const LenPlan &l : plan.lens)
            fj[nj++] = FirJob{l.t, bands[b].fir_order / 2, (const double *)(ws + plan.fir_r_off[b]),
                              ws + l.firw_off[b]};
    }
    // a length whose rows all take the DFT-bins kernel needs only its roots
    std::vector<char> len_fft(plan.lens.size(), 0);
    for (size_t q = 0; q < nprob; ++q)
        if (!by_dft[q])
            len_fft[plan.fft[q].len_index] = 1;
    for (size_t c = 0; c < plan.lens.size(); ++c) {
        const LenPlan &l = plan.lens[c];
        const size_t ti = std::find(plan.tw_logm.begin(), plan.tw_logm.end(), l.logm) - plan.tw_logm.begin();
        ChirpJob j{};
        j.t = l.t;
        j.logm = l.logm;
        j.blue = l.blue && len_fft[c] ? 1 : 0;
        j.chirp = l.blue ? ws + l.chirp_off : nullptr;
        j.bhat = l.blue ? ws + l.bhat_off : nullptr;
        j.roots = ws + l.roots_off;
        j.tw_tab = ws + plan.tw_off[ti];
        jobs[c] = j;
    }
}

// Twiddle tables per FFT size, then the per-length set-up jobs, one launch
// per size (the jobs are ordered by size).  With class_count, a size none of
// whose rows takes a transform gets no twiddle table (its lengths' jobs then
// write only their roots).
static hipError_t launch_fft_setup(const Plan &plan, uint8_t *ws, hipStream_t s, int &launches,
                                   const std::vector<int> *class_count = nullptr)
{
    const bool f64 = plan.mode == M_F64;
    hipError_t e;
    for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
        if (class_count && (*class_count)[c] == 0)
            continue;
        if ((e = launch_twiddles(f64, ws + plan.tw_off[c], plan.tw_logm[c], s)) != hipSuccess)
            return e;
        ++launches;
    }
    const ChirpJob *jobs = (const ChirpJob *)(ws + plan.job_off);
    for (size_t c = 0; c < plan.lens.size();) {
        size_t d = c;
        while (d < plan.lens.size() && plan.lens[d].logm == plan.lens[c].logm)
            ++d;
        if ((e = launch_chirps(f64, plan.lens[c].logm, jobs + c, (int)(d - c), s)) != hipSuccess)
            return e;
        ++launches;
        c = d;
    }
    if (plan.nfirjobs > 0) {
        if ((e = launch_fir_weights(f64, (const FirJob *)(ws + plan.firjob_off), plan.nfirjobs, plan.fir_max_t,
                                    s)) != hipSuccess)
            return e;
        ++launches;
    }
    return hipSuccess;
}

// The row-wise epilogue applies: FP32 outputs, and every problem's rows
// start 16-byte aligned (n a multiple of 4, aligned outputs).
static bool rows_ok(int mode, const GramDesc *gd, size_t ng)
{
    if (mode == M_F64)
        return false;
    for (size_t q = 0; q < ng; ++q) {
        const uintptr_t al = (uintptr_t)gd[q].plv | (uintptr_t)gd[q].iplv | (uintptr_t)gd[q].ciplv | (uintptr_t)gd[q].g;
        if (gd[q].n % 4 != 0 || al % 16 != 0)
            return false;
    }
    return true;
}

// Enqueues the whole forward path of a plan on stream s: one upload of the
// device tables, the front end (normalisation of analytic input, or the FFT
// analytic signal of real input), the Gram kernel and the epilogue.
static plv_status enqueue_forward(plv_ctx *ctx, const Plan &plan, const plv_problem *probs, const plv_band *bands,
                                  int nbands, double fs, uint8_t *ws, hipStream_t s, const plv_trials *tr = nullptr)
{
    const int mode = plan.mode;
    const bool real = plan.op == PLV_OP_FROM_REAL;
    std::vector<GramDesc> gd;
    fill_descs(plan, ws, gd);
    std::vector<Item> items;
    std::vector<TileRef> tiles;
    if (plan.grouped)
        build_tables(plan, gd, items, tiles);

    std::vector<int> class_start, class_count;  // FFT rows per size class
    bool any_direct = false;                    // some band synthesised from its bins
    int64_t synth_jobs = 0;                     // its work-groups
    int64_t dft_jobs = 0;                       // work-groups of the DFT-bins kernel
    if (plan.grouped || real) {
        std::vector<uint8_t> blob(plan.tables_bytes, 0);
        memcpy(blob.data() + plan.desc_off, gd.data(), gd.size() * sizeof(GramDesc));
        if (plan.grouped) {
            memcpy(blob.data() + plan.item_off, items.data(), items.size() * sizeof(Item));
            memcpy(blob.data() + plan.tile_off, tiles.data(), tiles.size() * sizeof(TileRef));
        }
        if (real)
            fill_fft_tables(plan, probs, nullptr, bands, nbands, fs, ws, blob, class_start, class_count, any_direct,
                            synth_jobs, dft_jobs);
        plv_status st = upload(ctx, blob, ws + plan.tables_off, s);
        if (st != PLV_OK)
            return st;
    }

    hipError_t e;
    if (real) {
        StageTimer tm(ctx, PLV_STAGE_HILBERT, s);
        int nl = 0;
        if ((e = launch_fft_setup(plan, ws, s, nl, &class_count)) != hipSuccess)
            return hip_fail(ctx, e, "FFT set-up kernel launch");
        tm.launched(nl);
        for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
            if (class_count[c] == 0)
                continue;  // every row of this size takes the DFT-bins kernel
            HilbertArgs ha{};
            ha.hp = (const HilbertProb *)(ws + plan.hp_off);
            ha.bins = (const BandBins *)(ws + plan.bin_off);
            ha.rows = (const RowRef *)(ws + plan.row_off) + class_start[c];
            ha.nrows = class_count[c];
            ha.logm = plan.tw_logm[c];
            ha.gd = (const GramDesc *)(ws + plan.desc_off);
            ha.nbands = nbands;
            ha.fir = plan.nfirjobs > 0 ? 1 : 0;
            ha.xs = plan.xs_slots[c] ? ws + plan.xs_off : nullptr;
            ha.xslots = plan.xs_slots[c];
            if ((e = launch_hilbert(mode, ha, ctx->cus, s)) != hipSuccess)
                return hip_fail(ctx, e, "analytic-signal kernel launch");
            tm.launched();
        }
        if (dft_jobs > 0) {
            if (dft_jobs >= INT32_MAX)
                return fail(ctx, PLV_ERR_UNSUPPORTED, "DFT bins need %lld work-groups", (long long)dft_jobs);
            HilbertArgs ha{};
            ha.hp = (const HilbertProb *)(ws + plan.hp_off);
            ha.bins = (const BandBins *)(ws + plan.bin_off);
            ha.nbands = nbands;
            ha.nprob = (int32_t)plan.fft.size();
            ha.dft_prefix = (const int32_t *)(ws + plan.dftp_off);
            if ((e = launch_dft_bins(ha, (int)dft_jobs, s)) != hipSuccess)
                return hip_fail(ctx, e, "DFT bins kernel launch");
            tm.launched();
        }
        if (any_direct) {
            if (synth_jobs > INT32_MAX)
                return fail(ctx, PLV_ERR_UNSUPPORTED, "band synthesis needs %lld work-groups", (long long)synth_jobs);
            HilbertArgs ha{};
            ha.hp = (const HilbertProb *)(ws + plan.hp_off);
            ha.bins = (const BandBins *)(ws + plan.bin_off);
            ha.gd = (const GramDesc *)(ws + plan.desc_off);
            ha.nbands = nbands;
            ha.fir = plan.nfirjobs > 0 ? 1 : 0;
            ha.nprob = (int32_t)plan.fft.size();
            ha.synth_prefix = (const int32_t *)(ws + plan.synth_off);
            if ((e = launch_band_synth(mode, ha, (int)synth_jobs, s)) != hipSuccess)
                return hip_fail(ctx, e, "band synthesis kernel launch");
            tm.launched();
        }
    } else {
        StageTimer tm(ctx, PLV_STAGE_NORMALISE, s);
        const bool coh = plan.op == PLV_OP_COHERENCE;
        if (tr) {
            // across trials: one gather launch fills every time point's planes
            const GramPlan &g0 = plan.grams[0];
            TrialArgs ta{};
            ta.in = tr->in;
            ta.ld = tr->ld;
            ta.tstride = tr->tstride;
            ta.sstride = tr->sstride;
            ta.t0 = tr->t0;
            ta.n = (int32_t)tr->n;
            ta.ntr = (int32_t)tr->ntr;
            ta.ntp = (int32_t)plan.grams.size();
            ta.u0 = ws + g0.u_off;
            ta.gstride = plan.grams.size() > 1 ? (int64_t)(plan.grams[1].u_off - g0.u_off) : 0;
            ta.plane_bytes = (int64_t)g0.plane_bytes;
            ta.cstride = (int64_t)g0.npad * g0.chunk * cbytes_of(mode);
            ta.chunk = g0.chunk;
            ta.rows = g0.npad;
            ta.tpad = g0.tpad;
            if ((e = launch_trial_planes(mode, ta, s)) != hipSuccess)
                return hip_fail(ctx, e, "trial planes kernel launch");
            tm.launched();
        }
        for (const GramPlan &gp : plan.grams) {
            if (tr)
                break;
            const plv_problem &p = probs[gp.prob];
            if (coh) {
                ScaleArgs sa{};
                sa.in = p.in;
                sa.ld = p.ld;
                sa.t0 = gp.t0;
                sa.tw = gp.t;
                sa.n = gp.n;
                sa.scale = (double *)(ws + gp.scale_off);
                if ((e = launch_row_scale(mode == M_F64, sa, s)) != hipSuccess)
                    return hip_fail(ctx, e, "row scale kernel launch");
                tm.launched();
            }
            NormArgs na{};
            na.scale = coh ? (const double *)(ws + gp.scale_off) : nullptr;
            na.in = p.in;
            na.ld = p.ld;
            na.t0 = gp.t0;
            na.tw = gp.t;
            na.n = gp.n;
            na.u = ws + gp.u_off;
            na.plane_bytes = (int64_t)gp.plane_bytes;
            na.cstride = (int64_t)gp.npad * gp.chunk * cbytes_of(mode);
            na.chunk = gp.chunk;
            na.rows = gp.npad;
            na.tpad = gp.tpad;
            if ((e = launch_normalise(mode, na, s)) != hipSuccess)
                return hip_fail(ctx, e, "normalise kernel launch");
            tm.launched();
        }
    }

    if (!plan.grouped) {
        const GramDesc &d = gd[0];
        const int passes = (d.nchunk + d.nslot - 1) / d.nslot;
        {
            StageTimer tm(ctx, PLV_STAGE_GRAM, s);
            for (int p = 0; p < passes; ++p) {
                HerkArgs ha{};
                ha.g = d;
                ha.pass = p;
                ha.blocked = plan.blocked ? 1 : 0;
                const int nch = std::min(d.nslot, d.nchunk - p * d.nslot);
                if ((e = launch_herk(mode, d.bm, ha, d.nupper * nch, s)) != hipSuccess)
                    return hip_fail(ctx, e, "gram kernel launch");
                tm.launched();
            }
        }
        if (d.fused)
            return PLV_OK;
        StageTimer tm(ctx, PLV_STAGE_EPILOGUE, s);
        EpiArgs ea{};
        ea.g = d;
        if (plan.op == PLV_OP_COHERENCE) {
            if ((e = launch_diag(mode, d, s)) != hipSuccess)
                return hip_fail(ctx, e, "diagonal kernel launch");
            tm.launched();
            ea.coherence = true;
        }
        if ((e = launch_epilogue(mode, ea, d.nupper, d.bm, rows_ok(mode, &d, 1), s)) != hipSuccess)
            return hip_fail(ctx, e, "epilogue kernel launch");
        tm.launched();
        return PLV_OK;
    }
    {
        // one launch per tile edge present (each an XCD-major item list)
        StageTimer tm(ctx, PLV_STAGE_GRAM, s);
        for (const Plan::ItemGroup &grp : plan.groups) {
            HerkArgs ha{};
            ha.gd = (const GramDesc *)(ws + plan.desc_off);
            ha.items = (const Item *)(ws + plan.item_off) + grp.off;
            ha.nitems = (int32_t)grp.count;
            if ((e = launch_herk(mode, grp.bm, ha, (int)grp.count, s)) != hipSuccess)
                return hip_fail(ctx, e, "gram kernel launch");
            tm.launched();
        }
    }
    if (tiles.empty())
        return PLV_OK;
    StageTimer tm(ctx, PLV_STAGE_EPILOGUE, s);
    EpiArgs ea{};
    ea.gd = (const GramDesc *)(ws + plan.desc_off);
    if (plan.op == PLV_OP_COHERENCE) {
        for (const GramDesc &d : gd)
            if ((e = launch_diag(mode, d, s)) != hipSuccess)
                return hip_fail(ctx, e, "diagonal kernel launch");
        tm.launched((int)gd.size());
        ea.coherence = true;
    }
    ea.tiles = (const TileRef *)(ws + plan.tile_off);
    if ((e = launch_epilogue(mode, ea, (int)tiles.size(), plan.bm_max, rows_ok(mode, gd.data(), gd.size()), s)) !=
        hipSuccess)
        return hip_fail(ctx, e, "epilogue kernel launch");
    tm.launched();
    return PLV_OK;
}

plv_status plv_from_analytic(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob, void *ws,
                             size_t ws_bytes, void *stream)
{
    Plan plan;
    plv_status st = begin(ctx, PLV_OP_FROM_ANALYTIC, prec, probs, nprob, nullptr, 1, ws, ws_bytes, plan);
    if (st != PLV_OK)
        return st;
    return enqueue_forward(ctx, plan, probs, nullptr, 1, 0.0, (uint8_t *)ws, (hipStream_t)stream);
}

plv_status plv_from_analytic_noalloc(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                                     void *stream)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    ctx->err.clear();
    if (ctx->device < 0)
        return fail(ctx, PLV_ERR_INVALID_ARG, "host-only context cannot compute");
    if (nprob != 1)
        return fail(ctx, PLV_ERR_UNSUPPORTED, "the allocation-free entry point takes exactly one problem (nprob = %lld)",
                    (long long)nprob);
    if (!ctx->scratch)
        return fail(ctx, PLV_ERR_DEVICE, "device scratch address not available: %s",
                    ctx->device >= MAX_DEVICES ? "device index beyond the library's table"
                                               : hipGetErrorString(ctx->scratch_err));
    Plan plan;
    std::string why;
    plv_status st = make_plan(ctx->cus, ctx->occ, PLV_OP_FROM_ANALYTIC, prec, probs, 1, nullptr, 1, plan, why,
                              &ctx->tune);
    if (st != PLV_OK)
        return fail(ctx, st, "%s", why.c_str());
    if (plan.total > (size_t)PLV_NOALLOC_MAX_BYTES)
        return fail(ctx, PLV_ERR_UNSUPPORTED,
                    "problem needs %zu bytes of scratch; the allocation-free entry point has %zu (use plv_from_analytic "
                    "with a workspace)",
                    plan.total, (size_t)PLV_NOALLOC_MAX_BYTES);
    if (plan.grouped)
        return fail(ctx, PLV_ERR_UNSUPPORTED, "internal: a single problem planned as a grouped launch");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipSetDevice");
    // a single analytic problem uploads no tables (its descriptor travels as
    // a kernel argument and its tile order is decoded on the device), so the
    // call below makes no allocation and no host-to-device copy
    return enqueue_forward(ctx, plan, probs, nullptr, 1, 0.0, (uint8_t *)ctx->scratch, (hipStream_t)stream);
}

// Across trials: one Gram problem per time point (rows = signals, samples =
// trials), described to the planner as problems whose input is never read by
// the per-problem normalisation (the gather kernel fills their planes).
static plv_status trials_problems(const plv_trials *p, plv_prec prec, std::vector<plv_problem> &probs,
                                  std::string &why)
{
    if (!p) {
        why = "trials descriptor is NULL";
        return PLV_ERR_INVALID_ARG;
    }
    const int64_t t1 = p->t1 == 0 ? p->t : p->t1;
    if (p->n < 1 || p->n > (1 << 20) || p->ntr < 1 || p->ntr > (1 << 17) || p->t < 1) {
        char b[160];
        snprintf(b, sizeof b, "need 1 <= n <= 2^20, 1 <= ntr <= 2^17, t >= 1 (n = %lld, ntr = %lld, t = %lld)",
                 (long long)p->n, (long long)p->ntr, (long long)p->t);
        why = b;
        return PLV_ERR_INVALID_ARG;
    }
    if (p->ld < 1 || p->tstride < 1 || p->sstride < 1) {
        why = "strides must be >= 1";
        return PLV_ERR_INVALID_ARG;
    }
    if (p->t0 < 0 || t1 <= p->t0 || t1 > p->t || t1 - p->t0 > (1 << 24)) {
        char b[160];
        snprintf(b, sizeof b, "need 0 <= t0 < t1 <= t and at most 2^24 time points (t0 = %lld, t1 = %lld)",
                 (long long)p->t0, (long long)t1);
        why = b;
        return PLV_ERR_INVALID_ARG;
    }
    const size_t esz = prec == PLV_PREC_F64 ? 8 : 4;
    const size_t nn = (size_t)p->n * (size_t)p->n;
    probs.assign((size_t)(t1 - p->t0), plv_problem{});
    for (size_t k = 0; k < probs.size(); ++k) {
        plv_problem &q = probs[k];
        q.n = p->n;
        q.t = p->ntr;
        q.ld = p->ntr;
        q.in = p->in;
        q.plv = p->plv ? (uint8_t *)p->plv + k * nn * esz : nullptr;
        q.iplv = p->iplv ? (uint8_t *)p->iplv + k * nn * esz : nullptr;
        q.ciplv = p->ciplv ? (uint8_t *)p->ciplv + k * nn * esz : nullptr;
        q.g = p->g ? (uint8_t *)p->g + k * nn * 2 * esz : nullptr;
    }
    return PLV_OK;
}

plv_status plv_trials_workspace_size(const plv_ctx *ctx, plv_prec prec, const plv_trials *p, size_t *bytes)
{
    if (!bytes)
        return PLV_ERR_INVALID_ARG;
    *bytes = 0;
    std::vector<plv_problem> probs;
    std::string why;
    plv_status st = trials_problems(p, prec, probs, why);
    if (st == PLV_OK)
        return workspace_size(ctx, PLV_OP_FROM_ANALYTIC, prec, probs.data(), (int64_t)probs.size(), nullptr, 1, bytes,
                              true);
    if (ctx)
        const_cast<plv_ctx *>(ctx)->err = why;
    return st;
}

plv_status plv_over_trials(plv_ctx *ctx, plv_prec prec, const plv_trials *p, void *ws, size_t ws_bytes,
                           void *stream)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    std::vector<plv_problem> probs;
    std::string why;
    plv_status st = trials_problems(p, prec, probs, why);
    if (st != PLV_OK)
        return fail(ctx, st, "%s", why.c_str());
    Plan plan;
    st = begin(ctx, PLV_OP_FROM_ANALYTIC, prec, probs.data(), (int64_t)probs.size(), nullptr, 1, ws, ws_bytes,
               plan, true);
    if (st != PLV_OK)
        return st;
    return enqueue_forward(ctx, plan, probs.data(), nullptr, 1, 0.0, (uint8_t *)ws, (hipStream_t)stream, p);
}

plv_status plv_coherence(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob, void *ws,
                         size_t ws_bytes, void *stream)
{
    Plan plan;
    plv_status st = begin(ctx, PLV_OP_COHERENCE, prec, probs, nprob, nullptr, 1, ws, ws_bytes, plan);
    if (st != PLV_OK)
        return st;
    return enqueue_forward(ctx, plan, probs, nullptr, 1, 0.0, (uint8_t *)ws, (hipStream_t)stream);
}

// Coherency over windowed segments: the segment spectra go into the front of
// the workspace, bin-major per problem, and every (problem, bin) becomes a
// coherency problem over those coefficient rows (rows = signals, samples =
// segments), planned behind them.
struct StftPlan {
    int nbins = 0;
    size_t tw_off = 0, win_off = 0;
    std::vector<int> nseg;          // per input problem
    std::vector<size_t> coef_off;   // per input problem
    std::vector<plv_problem> coh;   // per (problem, bin)
    size_t coh_off = 0;             // the coherency plan's part of the workspace
    Plan plan;
    size_t total = 0;
};

static size_t align256_(size_t x) { return (x + 255) & ~size_t(255); }

// base: the workspace (or any 256-byte aligned stand-in when only sizing)
static plv_status stft_plan(const plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                            const plv_stft *st, uint8_t *base, StftPlan &sp, std::string &why)
{
    char b[256];
    if ((int)prec < 0 || (int)prec > 4) {
        why = "unknown precision";
        return PLV_ERR_INVALID_ARG;
    }
    if (!st) {
        why = "stft descriptor is NULL";
        return PLV_ERR_INVALID_ARG;
    }
    if (st->seg < 2 || st->seg > STFT_MAX_SEG || st->hop < 1 || st->k_lo < 0 || st->k_hi < st->k_lo ||
        st->k_hi > st->seg / 2 || st->k_hi - st->k_lo + 1 > 512 || st->window < 0 || st->window > 2 ||
        st->reserved != 0) {
        snprintf(b, sizeof b,
                 "segmentation out of range: need 2 <= seg <= %d, hop >= 1, 0 <= k_lo <= k_hi <= seg/2, at most "
                 "512 bins, a known window, reserved 0 (seg %d, hop %d, bins %d..%d, window %d)",
                 STFT_MAX_SEG, st->seg, st->hop, st->k_lo, st->k_hi, st->window);
        why = b;
        return PLV_ERR_INVALID_ARG;
    }
    if (!probs || nprob < 1 || nprob > (1 << 20)) {
        why = "need 1 <= nprob <= 2^20 problems and a non-NULL array";
        return PLV_ERR_INVALID_ARG;
    }
    const bool f64 = prec == PLV_PREC_F64;
    const size_t rsz = f64 ? 8 : 4, csz = 2 * rsz;
    sp = StftPlan();
    sp.nbins = st->k_hi - st->k_lo + 1;
    size_t off = 0;
    sp.tw_off = off;
    off += align256_((size_t)st->seg * csz);
    sp.win_off = off;
    off += align256_((size_t)st->seg * rsz);
    for (int64_t q = 0; q < nprob; ++q) {
        const plv_problem &p = probs[q];
        const int64_t t1 = p.t1 == 0 ? p.t : p.t1;
        if (p.n < 1 || p.n > (1 << 20) || p.t < 1 || p.ld < p.t || p.t0 < 0 || t1 <= p.t0 || t1 > p.t || !p.in ||
            reinterpret_cast<uintptr_t>(p.in) % rsz) {
            snprintf(b, sizeof b,
                     "problem %lld: need 1 <= n <= 2^20, t >= 1, ld >= t, 0 <= t0 < t1 <= t and %d-byte aligned "
                     "input",
                     (long long)q, (int)rsz);
            why = b;
            return PLV_ERR_INVALID_ARG;
        }
        if (t1 - p.t0 < st->seg) {
            snprintf(b, sizeof b, "problem %lld: the window [t0, t1) holds %lld samples, less than one segment",
                     (long long)q, (long long)(t1 - p.t0));
            why = b;
            return PLV_ERR_INVALID_ARG;
        }
        const int64_t S = (t1 - p.t0 - st->seg) / st->hop + 1;
        if (S > (1 << 30)) {
            why = "too many segments";
            return PLV_ERR_INVALID_ARG;
        }
        sp.nseg.push_back((int)S);
        sp.coef_off.push_back(off);
        off += align256_((size_t)sp.nbins * p.n * S * csz);
    }
    const size_t esz = f64 ? 8 : 4;
    for (int64_t q = 0; q < nprob; ++q) {
        const plv_problem &p = probs[q];
        const int S = sp.nseg[q];
        const size_t nn = (size_t)p.n * (size_t)p.n;
        for (int k = 0; k < sp.nbins; ++k) {
            plv_problem d{};
            d.n = p.n;
            d.t = S;
            d.ld = S;
            d.in = base + sp.coef_off[q] + (size_t)k * p.n * S * csz;
            d.plv = p.plv ? (uint8_t *)p.plv + k * nn * esz : nullptr;
            d.iplv = p.iplv ? (uint8_t *)p.iplv + k * nn * esz : nullptr;
            d.ciplv = p.ciplv ? (uint8_t *)p.ciplv + k * nn * esz : nullptr;
            d.g = p.g ? (uint8_t *)p.g + 2 * k * nn * esz : nullptr;
            sp.coh.push_back(d);
        }
    }
    sp.coh_off = off;
    plv_status r = make_plan(ctx ? ctx->cus : 256, ctx ? ctx->occ : nullptr, PLV_OP_COHERENCE, prec, sp.coh.data(),
                             (int64_t)sp.coh.size(), nullptr, 1, sp.plan, why, ctx ? &ctx->tune : nullptr);
    if (r != PLV_OK)
        return r;
    sp.total = off + sp.plan.total;
    return PLV_OK;
}

plv_status plv_coherence_stft_workspace_size(const plv_ctx *ctx, plv_prec prec, const plv_problem *probs,
                                             int64_t nprob, const plv_stft *stft, size_t *bytes)
{
    if (!bytes)
        return PLV_ERR_INVALID_ARG;
    *bytes = 0;
    StftPlan sp;
    std::string why;
    const plv_status st = stft_plan(ctx, prec, probs, nprob, stft, (uint8_t *)(uintptr_t)256, sp, why);
    if (st != PLV_OK) {
        if (ctx)
            const_cast<plv_ctx *>(ctx)->err = why;
        return st;
    }
    *bytes = sp.total;
    return PLV_OK;
}

plv_status plv_coherence_stft(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                              const plv_stft *stft, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    ctx->err.clear();
    if (ctx->device < 0)
        return fail(ctx, PLV_ERR_INVALID_ARG, "host-only context cannot compute");
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(ctx, PLV_ERR_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    StftPlan sp;
    std::string why;
    plv_status st = stft_plan(ctx, prec, probs, nprob, stft, (uint8_t *)ws, sp, why);
    if (st != PLV_OK)
        return fail(ctx, st, "%s", why.c_str());
    if (ws_bytes < sp.total)
        return fail(ctx, PLV_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, sp.total);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "hipSetDevice");
    const hipStream_t s = (hipStream_t)stream;
    const bool f64 = prec == PLV_PREC_F64;
    uint8_t *w8 = (uint8_t *)ws;
    {
        StageTimer tm(ctx, PLV_STAGE_STFT, s);
        StftTables tt{};
        tt.seg = stft->seg;
        tt.window = stft->window;
        tt.tw = w8 + sp.tw_off;
        tt.win = w8 + sp.win_off;
        if ((e = launch_stft_tables(f64, tt, s)) != hipSuccess)
            return hip_fail(ctx, e, "segment table kernel launch");
        tm.launched();
        for (int64_t q = 0; q < nprob; ++q) {
            const plv_problem &p = probs[q];
            StftArgs a{};
            a.x = p.in;
            a.ld = p.ld;
            a.t0 = p.t0;
            a.n = (int32_t)p.n;
            a.seg = stft->seg;
            a.hop = stft->hop;
            a.nseg = sp.nseg[q];
            a.k_lo = stft->k_lo;
            a.k_hi = stft->k_hi;
            a.spw = std::max(1, std::min(a.nseg, 256 / sp.nbins));
            a.tw = tt.tw;
            a.win = tt.win;
            a.coef = w8 + sp.coef_off[q];
            if ((e = launch_stft(f64, a, s)) != hipSuccess)
                return hip_fail(ctx, e, "segment spectrum kernel launch");
            tm.launched();
        }
    }
    return enqueue_forward(ctx, sp.plan, sp.coh.data(), nullptr, 1, 0.0, w8 + sp.coh_off, s);
}

plv_status plv_from_real(plv_ctx *ctx, plv_prec prec, const plv_problem *probs, int64_t nprob,
                         const plv_band *bands, int32_t nbands, double fs, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    if (bands) {
        for (int32_t b = 0; b < nbands; ++b) {
            if ((bands[b].f_lo != 0.0 || bands[b].f_hi != 0.0) && !(fs > 0.0 && std::isfinite(fs)))
                return fail(ctx, PLV_ERR_INVALID_ARG, "a band-pass band needs a finite sampling rate fs > 0");
            if (bands[b].fir_order > 0 && !(bands[b].f_hi <= 0.5 * fs))
                return fail(ctx, PLV_ERR_INVALID_ARG, "band %d: an FIR band needs f_hi <= fs / 2", (int)b);
        }
    }
    Plan plan;
    plv_status st = begin(ctx, PLV_OP_FROM_REAL, prec, probs, nprob, bands, nbands, ws, ws_bytes, plan);
    if (st != PLV_OK)
        return st;
    return enqueue_forward(ctx, plan, probs, bands, bands ? nbands : 1, fs, (uint8_t *)ws, (hipStream_t)stream);
}

// Backward: recompute the phasors (and, for real input, the analytic signal),
// form H from the forward G and the upstream gradients, ubar = H U on MFMA,
// then the normalisation adjoint and, for real input, the analytic-signal
// adjoint.  Upstream gradients and G are [nbands][n][n] per problem.
static plv_status enqueue_backward(plv_ctx *ctx, const Plan &plan, const plv_problem *probs, const plv_grad *grads,
                                   const plv_band *bands, int nbands, double fs, uint8_t *ws, hipStream_t s)
{
    const int mode = plan.mode;
    const bool real = plan.op == PLV_OP_BACKWARD_REAL;
    const bool f64 = mode == M_F64;
    const size_t esz = f64 ? 8 : 4;  // output / gradient element
    std::vector<GramDesc> gd;
    fill_descs(plan, ws, gd);
    std::vector<Item> items;
    std::vector<TileRef> tiles;
    if (plan.grouped)
        build_tables(plan, gd, items, tiles);

    std::vector<int> class_start, class_count;
    bool any_direct = false;
    int64_t synth_jobs = 0;
    {
        std::vector<uint8_t> blob(plan.tables_bytes, 0);
        memcpy(blob.data() + plan.desc_off, gd.data(), gd.size() * sizeof(GramDesc));
        if (plan.grouped)
            memcpy(blob.data() + plan.item_off, items.data(), items.size() * sizeof(Item));
        int64_t dft_jobs = 0;  // (0: the backward takes every row through the transform)
        if (real)
            fill_fft_tables(plan, probs, grads, bands, nbands, fs, ws, blob, class_start, class_count, any_direct,
                            synth_jobs, dft_jobs);
        plv_status st = upload(ctx, blob, ws + plan.tables_off, s);
        if (st != PLV_OK)
            return st;
    }

    StageTimer tm(ctx, PLV_STAGE_BACKWARD, s);
    hipError_t e;
    HilbertArgs ha{};
    ha.hp = (const HilbertProb *)(ws + plan.hp_off);
    ha.bins = (const BandBins *)(ws + plan.bin_off);
    ha.gd = (const GramDesc *)(ws + plan.desc_off);
    ha.nbands = nbands;
    ha.fir = plan.nfirjobs > 0 ? 1 : 0;
    if (real) {
        // analytic signal of the window, kept unnormalised in zbuf
        int nl = 0;
        if ((e = launch_fft_setup(plan, ws, s, nl)) != hipSuccess)
            return hip_fail(ctx, e, "FFT set-up kernel launch");
        for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
            ha.rows = (const RowRef *)(ws + plan.row_off) + class_start[c];
            ha.nrows = class_count[c];
            ha.logm = plan.tw_logm[c];
            ha.xs = plan.xs_slots[c] ? ws + plan.xs_off : nullptr;
            ha.xslots = plan.xs_slots[c];
            if ((e = launch_hilbert(mode, ha, ctx->cus, s)) != hipSuccess)
                return hip_fail(ctx, e, "analytic-signal kernel launch");
            ++nl;
        }
        if (any_direct) {
            if (synth_jobs > INT32_MAX)
                return fail(ctx, PLV_ERR_UNSUPPORTED, "band synthesis needs %lld work-groups", (long long)synth_jobs);
            ha.nprob = (int32_t)plan.fft.size();
            ha.synth_prefix = (const int32_t *)(ws + plan.synth_off);
            if ((e = launch_band_synth(mode, ha, (int)synth_jobs, s)) != hipSuccess)
                return hip_fail(ctx, e, "band synthesis kernel launch");
            ++nl;
        }
        tm.launched(nl);
    }
    // operands of ubar = H (conj U^T)^H
    for (size_t q = 0; q < plan.grams.size(); ++q) {
        const GramPlan &g = plan.grams[q];
        const plv_problem &p = probs[g.prob];
        const plv_grad &gr = grads[g.prob];
        BwdPlanesArgs pa{};
        if (real) {
            pa.z = ws + g.z_off;
            pa.ldz = g.t;
        } else {
            pa.z = (const uint8_t *)p.in + (size_t)g.t0 * 2 * esz;
            pa.ldz = p.ld;
        }
        pa.n = g.n;
        pa.tw = g.t;
        pa.kpad = g.kpad;
        pa.rows = g.ntile_b * g.bm;
        pa.w = ws + g.w_off;
        pa.plane_bytes = (int64_t)g.plane_bytes;
        if ((e = launch_planes_t(mode, pa, s)) != hipSuccess)
            return hip_fail(ctx, e, "transposed phasor kernel launch");
        const size_t ob = (size_t)g.band * g.n * g.n * esz;
        BwdMetricArgs ma{};
        ma.g = (const uint8_t *)p.g + 2 * ob;
        ma.dplv = gr.dplv ? (const uint8_t *)gr.dplv + ob : nullptr;
        ma.diplv = gr.diplv ? (const uint8_t *)gr.diplv + ob : nullptr;
        ma.dciplv = gr.dciplv ? (const uint8_t *)gr.dciplv + ob : nullptr;
        ma.n = g.n;
        ma.kpad = g.kpad;
        ma.inv_t = 1.0 / (double)g.t;
        ma.rows = g.npad;
        ma.h = ws + g.u_off;
        ma.plane_bytes = (int64_t)g.plane_bytes;
        if ((e = launch_metric_adjoint(mode, ma, s)) != hipSuccess)
            return hip_fail(ctx, e, "metric adjoint kernel launch");
        tm.launched(2);
    }
    // ubar on MFMA
    if (!plan.grouped) {
        HerkArgs hk{};
        hk.g = gd[0];
        if ((e = launch_herk(mode, gd[0].bm, hk, gd[0].nupper, s)) != hipSuccess)
            return hip_fail(ctx, e, "product kernel launch");
    } else {
        for (const Plan::ItemGroup &grp : plan.groups) {
            HerkArgs hk{};
            hk.gd = (const GramDesc *)(ws + plan.desc_off);
            hk.items = (const Item *)(ws + plan.item_off) + grp.off;
            hk.nitems = (int32_t)grp.count;
            if ((e = launch_herk(mode, grp.bm, hk, (int)grp.count, s)) != hipSuccess)
                return hip_fail(ctx, e, "product kernel launch");
        }
    }
    tm.launched();
    // through the normalisation
    for (size_t q = 0; q < plan.grams.size(); ++q) {
        const GramPlan &g = plan.grams[q];
        const plv_problem &p = probs[g.prob];
        BwdNormArgs na{};
        na.c = ws + g.c_off;
        na.ldc = g.t;
        na.tw = g.t;
        na.n = g.n;
        if (real) {
            na.z = ws + g.z_off;  // zbar replaces z in place
            na.ldz = g.t;
            na.dst = ws + g.z_off;
            na.ldd = g.t;
            na.off = 0;
            na.len = g.t;
        } else {
            na.z = (const uint8_t *)p.in + (size_t)g.t0 * 2 * esz;
            na.ldz = p.ld;
            na.dst = grads[g.prob].din;
            na.ldd = p.ld;
            na.off = g.t0;
            na.len = (int32_t)p.t;
        }
        if ((e = launch_normalise_adjoint(f64, na, s)) != hipSuccess)
            return hip_fail(ctx, e, "normalisation adjoint kernel launch");
        tm.launched();
    }
    // through the analytic signal
    if (real) {
        for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
            ha.rows = (const RowRef *)(ws + plan.row_off) + class_start[c];
            ha.nrows = class_count[c];
            ha.logm = plan.tw_logm[c];
            ha.xs = plan.xs_slots[c] ? ws + plan.xs_off : nullptr;
            ha.xslots = plan.xs_slots[c];
            if ((e = launch_hilbert_adjoint(f64, ha, ctx->cus, s)) != hipSuccess)
                return hip_fail(ctx, e, "analytic-signal adjoint kernel launch");
            tm.launched();
        }
    }
    return PLV_OK;
}

plv_status plv_backward(plv_ctx *ctx, plv_prec prec, plv_input kind, const plv_problem *probs,
                        const plv_grad *grads, int64_t nprob, const plv_band *bands, int32_t nbands, double fs,
                        void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    if (kind != PLV_INPUT_ANALYTIC && kind != PLV_INPUT_REAL)
        return fail(ctx, PLV_ERR_INVALID_ARG, "unknown input kind");
    if (!grads)
        return fail(ctx, PLV_ERR_INVALID_ARG, "grads is NULL");
    const bool real = kind == PLV_INPUT_REAL;
    if (real && bands) {
        for (int32_t b = 0; b < nbands; ++b) {
            if ((bands[b].f_lo != 0.0 || bands[b].f_hi != 0.0) && !(fs > 0.0 && std::isfinite(fs)))
                return fail(ctx, PLV_ERR_INVALID_ARG, "a band-pass band needs a finite sampling rate fs > 0");
            if (bands[b].fir_order > 0 && !(bands[b].f_hi <= 0.5 * fs))
                return fail(ctx, PLV_ERR_INVALID_ARG, "band %d: an FIR band needs f_hi <= fs / 2", (int)b);
        }
    }
    Plan plan;
    const plv_op op = real ? PLV_OP_BACKWARD_REAL : PLV_OP_BACKWARD_ANALYTIC;
    plv_status st = begin(ctx, op, prec, probs, nprob, real ? bands : nullptr, real ? nbands : 1, ws, ws_bytes, plan);
    if (st != PLV_OK)
        return st;
    const size_t esz = plan.mode == M_F64 ? 8 : 4;
    for (int64_t q = 0; q < nprob; ++q) {
        if (!grads[q].din)
            return fail(ctx, PLV_ERR_INVALID_ARG, "problem %lld: din is NULL", (long long)q);
        const void *gp[3] = {grads[q].dplv, grads[q].diplv, grads[q].dciplv};
        for (int k = 0; k < 3; ++k)
            if (gp[k] && reinterpret_cast<uintptr_t>(gp[k]) % esz)
                return fail(ctx, PLV_ERR_INVALID_ARG, "problem %lld: upstream gradients misaligned", (long long)q);
        if (reinterpret_cast<uintptr_t>(grads[q].din) % (real ? esz : 2 * esz > 16 ? 16 : 2 * esz))
            return fail(ctx, PLV_ERR_INVALID_ARG, "problem %lld: din misaligned", (long long)q);
    }
    return enqueue_backward(ctx, plan, probs, grads, real ? bands : nullptr, real ? (bands ? nbands : 1) : 1, fs,
                            (uint8_t *)ws, (hipStream_t)stream);
}

// Measures the launch shape of a forward call and keeps the fastest in the
// context.  One problem (one band): the K-chunk count -- the planner's choice
// and up to two exact splits on either side.  Several problems or bands (a
// grouped launch): the tile edge of every distinct row count -- the call is
// run on the problems of that row count alone with each edge.  Each candidate
// runs once untimed and three times between HIP events on the caller's
// stream; a candidate replaces the best so far only when it is more than 1%
// faster.  The winners apply to every later plan on the context.
plv_status plv_autotune(plv_ctx *ctx, plv_op op, plv_prec prec, const plv_problem *probs, int64_t nprob,
                        const plv_band *bands, int32_t nbands, double fs, void *ws, size_t ws_bytes, void *stream,
                        int32_t *nchunk)
{
    if (!ctx)
        return PLV_ERR_INVALID_ARG;
    if (nchunk)
        *nchunk = 0;
    if (op != PLV_OP_FROM_ANALYTIC && op != PLV_OP_FROM_REAL && op != PLV_OP_COHERENCE)
        return fail(ctx, PLV_ERR_INVALID_ARG, "autotune takes a forward op");
    const bool real = op == PLV_OP_FROM_REAL;
    const plv_band *bb = real ? bands : nullptr;
    const int32_t nb = real ? nbands : 1;
    Plan plan;
    plv_status st = begin(ctx, op, prec, probs, nprob, bb, nb, ws, ws_bytes, plan);
    if (st != PLV_OK)
        return st;
    const hipStream_t s = (hipStream_t)stream;
    auto run_on = [&](const plv_problem *pp, int64_t np) -> plv_status {
        if (op == PLV_OP_FROM_ANALYTIC)
            return plv_from_analytic(ctx, prec, pp, np, ws, ws_bytes, stream);
        if (op == PLV_OP_COHERENCE)
            return plv_coherence(ctx, prec, pp, np, ws, ws_bytes, stream);
        return plv_from_real(ctx, prec, pp, np, bands, nbands, fs, ws, ws_bytes, stream);
    };
    // the call on these problems fits the caller's workspace
    auto fits = [&](const plv_problem *pp, int64_t np) {
        Plan trial;
        std::string why;
        return make_plan(ctx->cus, ctx->occ, op, prec, pp, np, bb, nb, trial, why, &ctx->tune) == PLV_OK &&
               trial.total <= ws_bytes;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return hip_fail(ctx, e, "hipEventCreate");
    }
    const bool timing = ctx->timing;
    ctx->timing = false;  // the trial runs stay out of the stage timings
    std::vector<int> counts;
    chunk_counts(plan, counts);
    if (!counts.empty()) {
        // ---- one problem: the K-chunk count
        const auto key = tune_key(plan);
        const int cur = plan.grams[0].nchunk;
        const size_t at = (size_t)(std::lower_bound(counts.begin(), counts.end(), cur) - counts.begin());
        std::vector<int> cand{cur};
        for (size_t d = 1; d <= 2; ++d) {
            if (at >= d)
                cand.push_back(counts[at - d]);
            if (at + d < counts.size())
                cand.push_back(counts[at + d]);
        }
        const auto old = ctx->tune.chunks.find(key);
        const bool had = old != ctx->tune.chunks.end();
        const int old_nc = had ? old->second : 0;
        int best = 0;
        float best_ms = 0.0f;
        for (int nc : cand) {
            ctx->tune.chunks[key] = nc;
            Plan trial;
            std::string why;
            if (make_plan(ctx->cus, ctx->occ, op, prec, probs, nprob, bb, nb, trial, why, &ctx->tune) != PLV_OK ||
                trial.total > ws_bytes || trial.grams[0].nchunk != nc)
                continue;  // needs more workspace than the caller gave
            const float ms = time_runs([&]() { return run_on(probs, nprob); }, s, e0, e1, 3, st, e);
            if (ms < 0.0f)
                break;
            if (best == 0 || ms < best_ms * 0.99f) {
                best = nc;
                best_ms = ms;
            }
        }
        if (st == PLV_OK && e == hipSuccess && best > 0)
            ctx->tune.chunks[key] = best;
        else if (had)
            ctx->tune.chunks[key] = old_nc;
        else
            ctx->tune.chunks.erase(key);
        if (nchunk && st == PLV_OK && e == hipSuccess)
            *nchunk = best;
    } else if (plan.mode != M_F64) {
        // ---- grouped launch: the tile edge of each distinct row count
        std::vector<int64_t> ns;
        for (int64_t q = 0; q < nprob; ++q)
            ns.push_back(probs[q].n);
        std::sort(ns.begin(), ns.end());
        ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
        for (int64_t n : ns) {
            std::vector<plv_problem> sub;
            for (int64_t q = 0; q < nprob; ++q)
                if (probs[q].n == n)
                    sub.push_back(probs[q]);
            const auto key = std::make_pair(plan.mode, n);
            const auto old = ctx->tune.tiles.find(key);
            const bool had = old != ctx->tune.tiles.end();
            const int old_bm = had ? old->second : 0;
            int best = 0;
            float best_ms = 0.0f;
            for (int bm : {128, 64}) {
                ctx->tune.tiles[key] = bm;
                if (!fits(sub.data(), (int64_t)sub.size()))
                    continue;
                const float ms =
                    time_runs([&]() { return run_on(sub.data(), (int64_t)sub.size()); }, s, e0, e1, 3, st, e);
                if (ms < 0.0f)
                    break;
                if (best == 0 || ms < best_ms * 0.99f) {
                    best = bm;
                    best_ms = ms;
                }
            }
            if (st == PLV_OK && e == hipSuccess && best > 0) {
                ctx->tune.tiles[key] = best;
            } else {
                if (had)
                    ctx->tune.tiles[key] = old_bm;
                else
                    ctx->tune.tiles.erase(key);
                break;
            }
        }
    }
    ctx->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PLV_OK)
        return st;
    if (e != hipSuccess)
        return hip_fail(ctx, e, "autotune timing");
    return PLV_OK;
}

plv_status plv_tile_edge(const plv_ctx *ctx, plv_prec prec, int64_t n, int32_t *bm)
{
    if (!bm || (int)prec < 0 || (int)prec > 4 || n < 1)
        return PLV_ERR_INVALID_ARG;
    *bm = tile_for((int)prec, n, ctx ? &ctx->tune : nullptr);
    return PLV_OK;
}

plv_status plv_set_tile_edge(plv_ctx *ctx, plv_prec prec, int64_t n, int32_t bm)
{
    if (!ctx || (int)prec < 0 || (int)prec > 4 || n < 1)
        return PLV_ERR_INVALID_ARG;
    if (bm == 0) {
        ctx->tune.tiles.erase(std::make_pair((int)prec, n));
        return PLV_OK;
    }
    if (!tile_supported((int)prec, bm))
        return fail(ctx, PLV_ERR_INVALID_ARG, "tile edge %d is not available in this precision", (int)bm);
    ctx->tune.tiles[std::make_pair((int)prec, n)] = bm;
    return PLV_OK;
}

}  // extern "C"
