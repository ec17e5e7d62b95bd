// plv_plan.cpp -- argument checks, workspace layout and K-chunk choice.
#include "plv_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace plv {
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

std::string msg(const char *fmt, long long a = 0, long long b = 0)
{
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b);
    return buf;
}

// A padded length off the PLV_KGRAN grid (make_plan's unit_k) is one chunk.
bool single_chunk_k(GramPlan &g)
{
    if (g.tpad % PLV_KGRAN == 0)
        return false;
    g.chunk = g.tpad;
    g.nchunk = 1;
    g.nslot = 1;
    return true;
}

// K-chunks of a problem computed alone.  Every (tile, chunk) item costs about
// the same, so a pass takes ceil(items / slots) rounds of work-groups; the
// chunk count is the one with the least estimated time (below), with no chunk
// longer than the mode's maximum and none shorter than MIN_CHUNK unless T
// itself is.  Partial slots are capped by PARTIAL_BUDGET; beyond it the chunks
// run in passes.
constexpr double ITEM_OVERHEAD = 512.0;  // fixed cost of a work item, in samples of K

// Chunk-count bounds of choose_chunks_single: no chunk longer than maxc, none
// shorter than MIN_CHUNK unless T itself is.
void chunk_bounds(const GramPlan &g, int maxc, int &lo, int &hi)
{
    const int kgr = g.tpad / PLV_KGRAN;
    lo = std::max(1, (g.tpad + maxc - 1) / maxc);
    hi = std::max(lo, std::min(kgr, std::max(1, g.tpad / MIN_CHUNK)));
}

// An exact split: nc chunks of ceil(kgr / nc) granules use all nc chunks.
bool exact_split(int kgr, int nc)
{
    const int per = (kgr + nc - 1) / nc;
    return (kgr + per - 1) / per == nc;
}

// `forced` > 0: a measured chunk count (plv_autotune), taken when it is an
// exact split within the bounds.
void choose_chunks_single(GramPlan &g, int slots, int bm, int maxc, int forced)
{
    if (single_chunk_k(g))
        return;
    // Estimated time of a chunk count: for each pass, the rounds of work-groups
    // the GPU runs (items / slots, rounded up) times the length of one item,
    // its chunk plus a fixed per-item cost (prologue, fold, partial store) in
    // samples.  Ties go to fewer chunks: fewer partial slots to write and sum.
    const int kgr = g.tpad / PLV_KGRAN;
    int lo, hi;
    chunk_bounds(g, maxc, lo, hi);
    const size_t slot_bytes = (size_t)g.nupper * 2 * bm * bm * sizeof(double);
    const int budget = (int)std::max<size_t>(1, std::min<size_t>(INT32_MAX, PARTIAL_BUDGET / slot_bytes));
    int best = lo;
    double best_cost = -1.0;
    for (int nc = lo; nc <= hi && nc <= lo + 4 * slots; ++nc) {
        const int per = (kgr + nc - 1) / nc;
        const int real_nc = (kgr + per - 1) / per;
        if (real_nc != nc)
            continue;
        const int nslot = std::min(nc, budget);
        double rounds = 0.0;
        for (int c0 = 0; c0 < nc; c0 += nslot)
            rounds += std::ceil((double)g.nupper * std::min(nslot, nc - c0) / slots);
        const double cost = rounds * ((double)per * PLV_KGRAN + ITEM_OVERHEAD);
        if (best_cost < 0.0 || cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = nc;
        }
    }
    if (forced >= lo && forced <= hi && exact_split(kgr, forced))
        best = forced;
    const int per = (kgr + best - 1) / best;  // granules per chunk
    g.chunk = per * PLV_KGRAN;
    g.nchunk = (kgr + per - 1) / per;
    g.nslot = std::min(g.nchunk, budget);
}

// Inside a grouped launch every chunk of a problem has its own slot (one pass).
void choose_chunks_grouped(GramPlan &g, int maxc)
{
    if (single_chunk_k(g))
        return;
    const int kgr = g.tpad / PLV_KGRAN;
    const int per = std::min(kgr, maxc / PLV_KGRAN);
    g.chunk = per * PLV_KGRAN;
    g.nchunk = (kgr + per - 1) / per;
    g.nslot = g.nchunk;
}

// Grouped launches: whole problems go to XCDs by longest-processing-time
// bin packing on their estimated cost, and each XCD's list keeps a problem's
// items together (its tiles share panels in that XCD's L2), most costly
// problems first.  The lists are padded with empty items (gram = -1) to one
// length and stored XCD after XCD, matching the kernel's remap of work-group
// ids (XCD x = id mod 8 runs entries x * len .. x * len + len - 1 in order).
// A plain longest-first order of items would hand XCD 0 all the longest ones.
constexpr int NXCD = 8;

// One XCD-major item list for the problems with tile edge bm, appended to
// plan.items as one launch group.
void schedule_group(Plan &plan, int bm)
{
    const size_t np = plan.grams.size();
    std::vector<std::pair<double, size_t>> cost;
    for (size_t q = 0; q < np; ++q) {
        const GramPlan &g = plan.grams[q];
        if (g.bm != bm)
            continue;
        double c = 0.0;
        for (int k = 0; k < g.nchunk; ++k)  // product mode (backward): K = kpad
            c += (g.kpad > 0 ? g.kpad : std::min(g.chunk, g.tpad - k * g.chunk)) + ITEM_OVERHEAD;
        // a 64-wide tile does a quarter of a 128-wide tile's MFMA work
        cost.push_back({c * g.nupper * (double)bm * bm / (128.0 * 128.0), q});
    }
    if (cost.empty())
        return;
    std::stable_sort(cost.begin(), cost.end(),
                     [](const std::pair<double, size_t> &a, const std::pair<double, size_t> &b) {
                         return a.first > b.first;
                     });
    double load[NXCD] = {};
    size_t count[NXCD] = {};
    std::vector<size_t> lists[NXCD];
    for (const auto &pc : cost) {
        int x = 0;
        for (int y = 1; y < NXCD; ++y)
            if (load[y] < load[x])
                x = y;
        load[x] += pc.first;
        const GramPlan &g = plan.grams[pc.second];
        count[x] += (size_t)g.nupper * g.nchunk;
        lists[x].push_back(pc.second);
    }
    size_t len = 0;
    for (int x = 0; x < NXCD; ++x)
        len = std::max(len, count[x]);
    const size_t base = plan.items.size();
    plan.items.resize(base + len * NXCD, Item{-1, 0, 0, 0});
    for (int x = 0; x < NXCD; ++x) {
        size_t k = base + (size_t)x * len;
        for (size_t q : lists[x]) {
            const GramPlan &g = plan.grams[q];
            for (int c = 0; c < g.nchunk; ++c)
                for (int t = 0; t < g.nupper; ++t)
                    plan.items[k++] = Item{(int32_t)q, t, c, 0};
        }
    }
    plan.groups.push_back(Plan::ItemGroup{bm, base, len * NXCD});
}

void schedule_items(Plan &plan)
{
    plan.items.clear();
    plan.groups.clear();
    schedule_group(plan, 128);
    schedule_group(plan, 64);
    plan.nitems = plan.items.size();
}

}  // namespace

int model_tile(int mode, int64_t n)
{
    if (mode == M_F64)
        return 64;
    auto work = [n](int bm) {
        const double nt = (double)((n + bm - 1) / bm);
        return nt * (nt + 1.0) / 2.0 * bm * bm;
    };
    return work(64) / 0.85 < work(128) ? 64 : 128;
}

int tile_for(int mode, int64_t n, const Tuning *tune)
{
    if (tune) {
        const auto it = tune->tiles.find(std::make_pair(mode, n));
        if (it != tune->tiles.end() && tile_supported(mode, it->second))
            return it->second;
    }
    return model_tile(mode, n);
}

plv_status make_plan(int cus, const int *occ, plv_op op, plv_prec prec, const plv_problem *probs, int64_t nprob,
                     const plv_band *bands, int32_t nbands, Plan &plan, std::string &why, const Tuning *tune,
                     bool unit_k)
{
    plan = Plan();
    if ((int)prec < 0 || (int)prec > 4) {
        why = "unknown precision";
        return PLV_ERR_INVALID_ARG;
    }
    if ((int)op < 0 || (int)op > 4) {
        why = "unknown op";
        return PLV_ERR_INVALID_ARG;
    }
    if (!probs || nprob < 1 || nprob > (1 << 24)) {
        why = msg("need 1 <= nprob <= 2^24 problems and a non-NULL array (nprob = %lld)", (long long)nprob);
        return PLV_ERR_INVALID_ARG;
    }
    const bool real = (op == PLV_OP_FROM_REAL || op == PLV_OP_BACKWARD_REAL);
    if (real) {
        if (nbands < 1 || nbands > 64) {
            why = msg("need 1 <= nbands <= 64 (nbands = %lld)", nbands);
            return PLV_ERR_INVALID_ARG;
        }
        if (bands) {
            for (int b = 0; b < nbands; ++b) {
                if (!(bands[b].f_lo >= 0.0) || !(bands[b].f_hi >= bands[b].f_lo)) {
                    why = msg("band %lld: need 0 <= f_lo <= f_hi", b);
                    return PLV_ERR_INVALID_ARG;
                }
                const int32_t L = bands[b].fir_order;
                if (bands[b].reserved != 0 || L < 0 || L > PLV_FIR_MAX_ORDER || (L & 1) ||
                    (L > 0 && !(bands[b].f_hi > bands[b].f_lo))) {
                    why = msg("band %lld: fir_order must be 0 or even in [2, %d] with f_lo < f_hi, reserved 0", b,
                              PLV_FIR_MAX_ORDER);
                    return PLV_ERR_INVALID_ARG;
                }
            }
        } else if (nbands != 1) {
            why = "bands == NULL requires nbands == 1";
            return PLV_ERR_INVALID_ARG;
        }
    } else {
        nbands = 1;
    }
    const int mode = (int)prec;
    plan.mode = mode;
    plan.op = op;
    const bool backward = (op == PLV_OP_BACKWARD_ANALYTIC || op == PLV_OP_BACKWARD_REAL);
    const int cb = cbytes_of(mode);
    const int pl = planes_of(mode);
    const size_t in_elem = (mode == M_F64 ? 8 : 4) * (real ? 1 : 2);
    const size_t out_elem = (mode == M_F64 ? 8 : 4);

    for (int64_t q = 0; q < nprob; ++q) {
        const plv_problem &p = probs[q];
        const int64_t t1 = p.t1 == 0 ? p.t : p.t1;
        if (p.n < 1 || p.n > (1 << 20)) {
            why = msg("problem %lld: need 1 <= n <= 2^20 (n = %lld)", q, p.n);
            return PLV_ERR_INVALID_ARG;
        }
        if (p.t < 1 || p.t > (int64_t(1) << 30)) {
            why = msg("problem %lld: need 1 <= t <= 2^30 (t = %lld)", q, p.t);
            return PLV_ERR_INVALID_ARG;
        }
        if (p.ld < p.t) {
            why = msg("problem %lld: need ld >= t (ld = %lld)", q, p.ld);
            return PLV_ERR_INVALID_ARG;
        }
        if (p.t0 < 0 || t1 <= p.t0 || t1 > p.t) {
            why = msg("problem %lld: need 0 <= t0 < t1 <= t (t0 = %lld)", q, p.t0);
            return PLV_ERR_INVALID_ARG;
        }
        if (!p.in) {
            why = msg("problem %lld: input is NULL", q);
            return PLV_ERR_INVALID_ARG;
        }
        const size_t in_align = std::min<size_t>(in_elem, 16);
        if (reinterpret_cast<uintptr_t>(p.in) % in_align) {
            why = msg("problem %lld: input must be %lld-byte aligned", q, (long long)in_align);
            return PLV_ERR_INVALID_ARG;
        }
        const void *outs[4] = {p.plv, p.iplv, p.ciplv, p.g};
        for (int k = 0; k < 4; ++k)
            if (outs[k] && reinterpret_cast<uintptr_t>(outs[k]) % out_elem) {
                why = msg("problem %lld: outputs must be %lld-byte aligned", q, (long long)out_elem);
                return PLV_ERR_INVALID_ARG;
            }
        if ((op == PLV_OP_BACKWARD_ANALYTIC || op == PLV_OP_BACKWARD_REAL) && !p.g) {
            why = msg("problem %lld: backward needs the forward's complex G in `g`", q);
            return PLV_ERR_INVALID_ARG;
        }
        // the backward's product runs on the largest tile; a forward problem
        // takes the measured or modelled edge for its row count
        const int bm = backward ? tile_of(mode) : tile_for(mode, p.n, tune);
        for (int b = 0; b < nbands; ++b) {
            GramPlan g;
            g.prob = q;
            g.band = b;
            g.bm = bm;
            g.n = (int)p.n;
            g.npad = (int)((p.n + bm - 1) / bm * bm);
            g.t0 = (int)p.t0;
            g.t = (int)(t1 - p.t0);
            g.tpad = (g.t + PLV_KGRAN - 1) / PLV_KGRAN * PLV_KGRAN;
            if (unit_k && !backward) {
                const int ku = k_unit(mode);
                const int tu = (g.t + ku - 1) / ku * ku;
                if (tu <= MAX_CHUNK)
                    g.tpad = tu;  // one chunk (single_chunk_k)
            }
            g.ntile = g.npad / bm;
            g.nupper = g.ntile * (g.ntile + 1) / 2;
            const size_t nn = (size_t)p.n * (size_t)p.n;
            const size_t ob = (size_t)b * nn * out_elem;
            g.plv = p.plv ? (uint8_t *)p.plv + ob : nullptr;
            g.iplv = p.iplv ? (uint8_t *)p.iplv + ob : nullptr;
            g.ciplv = p.ciplv ? (uint8_t *)p.ciplv + ob : nullptr;
            g.g = p.g ? (uint8_t *)p.g + 2 * ob : nullptr;
            plan.grams.push_back(g);
        }
    }

    if (backward && (mode == M_BF16 || mode == M_F16)) {
        // the backward operand H is unbounded: plain 16-bit phasors are not
        // accurate enough for it, so these modes run their adjoint in split form
        plan.mode = M_SPLIT;
    }
    for (const GramPlan &g : plan.grams)
        plan.bm_max = std::max(plan.bm_max, g.bm);
    const bool grouped = plan.grams.size() > 1;
    plan.grouped = grouped;
    // device tables: Gram problem descriptors always (the FFT stage reads them
    // too); items and tiles for a grouped launch; FFT tables for real input.
    size_t off = 0;
    plan.tables_off = 0;
    plan.desc_off = 0;
    off = align256(plan.grams.size() * sizeof(GramDesc));
    if (backward) {
        // general product tiles: rows of H x rows of W, one K-chunk (K = n)
        for (GramPlan &g : plan.grams) {
            g.kpad = (g.n + PLV_KGRAN - 1) / PLV_KGRAN * PLV_KGRAN;
            g.ntile_b = (g.t + g.bm - 1) / g.bm;
            g.nupper = g.ntile * g.ntile_b;
            g.chunk = g.kpad;
            g.nchunk = 1;
            g.nslot = 1;
        }
        if (grouped) {
            schedule_items(plan);
            if (plan.nitems > (size_t)INT32_MAX) {
                why = "too many work items";
                return PLV_ERR_INVALID_ARG;
            }
            plan.item_off = off;
            off += align256(plan.nitems * sizeof(Item));
        }
    } else if (grouped) {
        for (GramPlan &g : plan.grams) {
            choose_chunks_grouped(g, MAX_CHUNK);
            g.fused = g.nchunk == 1 && op != PLV_OP_COHERENCE;  // coherency needs every diagonal first
        }
        schedule_items(plan);
        for (const GramPlan &g : plan.grams)
            if (!g.fused)
                plan.ntiles += (size_t)g.nupper;
        if (plan.nitems > (size_t)INT32_MAX || plan.ntiles > (size_t)INT32_MAX) {
            why = "too many work items";
            return PLV_ERR_INVALID_ARG;
        }
        plan.item_off = off;
        off += align256(plan.nitems * sizeof(Item));
        plan.tile_off = off;
        off += align256(plan.ntiles * sizeof(TileRef));
    } else {
        int forced = 0;
        if (tune) {
            const auto it = tune->chunks.find(tune_key(plan));
            if (it != tune->chunks.end())
                forced = it->second;
        }
        const int bm = plan.grams[0].bm;
        const int slots = std::max(1, cus) * std::max(1, occ ? occ[occ_index(mode, bm)] : 1);
        choose_chunks_single(plan.grams[0], slots, bm, MAX_CHUNK, forced);
        plan.grams[0].fused = plan.grams[0].nchunk == 1 && op != PLV_OP_COHERENCE;
        plan.blocked = true;
    }
    if (real) {
        const int maxlog = mode == M_F64 ? FFT_MAXLOG_F64 : FFT_MAXLOG_F32;
        const size_t csz = mode == M_F64 ? 16 : 8;
        plan.fft.resize((size_t)nprob);
        for (int64_t q = 0; q < nprob; ++q) {
            FftPlan &f = plan.fft[q];
            f.t = (int)probs[q].t;
            const bool pow2 = f.t >= 2 && (f.t & (f.t - 1)) == 0;
            f.blue = !pow2;
            int need = pow2 ? f.t : std::max(2, 2 * f.t - 1);
            f.logm = 0;
            while ((1 << f.logm) < need)
                ++f.logm;
            if (f.logm > maxlog) {
                why = msg("problem %lld: row length %lld is beyond the FFT stage's LDS-resident sizes", q, f.t);
                return PLV_ERR_UNSUPPORTED;
            }
            auto it = std::find(plan.tw_logm.begin(), plan.tw_logm.end(), f.logm);
            f.tw_index = (int)(it - plan.tw_logm.begin());
            if (it == plan.tw_logm.end())
                plan.tw_logm.push_back(f.logm);
            bool seen = false;
            for (const LenPlan &l : plan.lens)
                seen = seen || l.t == f.t;
            if (!seen) {
                LenPlan l;
                l.t = f.t;
                l.logm = f.logm;
                l.blue = f.blue;
                plan.lens.push_back(l);
            }
            plan.nrows += (size_t)probs[q].n;
        }
        std::sort(plan.lens.begin(), plan.lens.end(),
                  [](const LenPlan &a, const LenPlan &b) { return a.logm != b.logm ? a.logm < b.logm : a.t < b.t; });
        for (FftPlan &f : plan.fft)
            for (size_t c = 0; c < plan.lens.size(); ++c)
                if (plan.lens[c].t == f.t)
                    f.len_index = (int)c;
        plan.hp_off = off;
        off += align256((size_t)nprob * sizeof(HilbertProb));
        plan.bin_off = off;
        off += align256((size_t)nprob * nbands * sizeof(BandBins));
        plan.row_off = off;
        off += align256(plan.nrows * sizeof(RowRef));
        plan.job_off = off;
        off += align256(plan.lens.size() * sizeof(ChirpJob));
        plan.synth_off = off;
        off += align256((size_t)(nprob + 1) * sizeof(int32_t));
        plan.dftp_off = off;
        off += align256((size_t)(nprob + 1) * sizeof(int32_t));
        // FIR bands: the taps' autocorrelation per band, and one weight-table
        // job per (row length, band); the tables themselves follow below
        std::vector<int> fir_bands;
        for (int b = 0; bands && b < nbands; ++b)
            if (bands[b].fir_order > 0)
                fir_bands.push_back(b);
        plan.fir_r_off.assign((size_t)nbands, 0);
        for (int b : fir_bands) {
            plan.fir_r_off[b] = off;
            off += align256((size_t)(bands[b].fir_order + 1) * sizeof(double));
        }
        plan.nfirjobs = (int)(plan.lens.size() * fir_bands.size());
        plan.firjob_off = off;
        off += align256((size_t)plan.nfirjobs * sizeof(FirJob));
        plan.tables_bytes = off;
        for (int lg : plan.tw_logm) {
            plan.tw_off.push_back(off);
            off += align256((size_t)(1 << lg) / 2 * csz);
        }
        for (LenPlan &l : plan.lens) {
            l.roots_off = off;
            off += align256((size_t)l.t * csz);
            if (l.blue) {
                l.chirp_off = off;
                off += align256((size_t)l.t * csz);
                l.bhat_off = off;
                off += align256((size_t)(1 << l.logm) * csz);
            }
            l.firw_off.assign((size_t)nbands, 0);
            for (int b : fir_bands) {
                l.firw_off[b] = off;
                off += align256((size_t)(l.t / 2 + 1) * (csz / 2));
            }
            if (!fir_bands.empty())
                plan.fir_max_t = std::max(plan.fir_max_t, l.t);
        }
        // several bands: one spectrum slot of M elements per resident
        // work-group of the transform launches (one region, reused by each
        // FFT size in turn)
        plan.xs_slots.assign(plan.tw_logm.size(), 0);
        if (nbands >= 2) {
            size_t most = 0;
            for (size_t c = 0; c < plan.tw_logm.size(); ++c) {
                const int lg = plan.tw_logm[c];
                plan.xs_slots[c] = std::max(1, cus) * fft_wg_per_cu(mode == M_F64, lg);
                most = std::max(most, (size_t)plan.xs_slots[c] * ((size_t)1 << lg) * csz);
            }
            plan.xs_off = off;
            off += align256(most);
        }
        // band-pass bands may be synthesised from their bins: a slot of
        // DIRECT_KMAX bins per row and band (fs, and so the bin counts, are
        // only known at the call)
        bool bandpass = false;
        for (int b = 0; bands && b < nbands; ++b)
            bandpass = bandpass || bands[b].f_lo != 0.0 || bands[b].f_hi != 0.0;
        if (bandpass) {
            for (int64_t q = 0; q < nprob; ++q) {
                FftPlan &f = plan.fft[q];
                f.has_xbins = true;
                f.xbin_off = off;
                off += align256((size_t)probs[q].n * nbands * DIRECT_KMAX * csz);
            }
        }
    } else {
        plan.tables_bytes = off;
    }
    if (backward) {
        const int bpl = planes_of(plan.mode), bcb = cbytes_of(plan.mode);
        const size_t csz = mode == M_F64 ? 16 : 8;
        for (GramPlan &g : plan.grams) {
            const size_t rows = (size_t)std::max(g.npad, g.ntile_b * g.bm);
            g.plane_bytes = align256(rows * g.kpad * bcb);
            g.u_off = off;
            off += g.plane_bytes * bpl;
            g.w_off = off;
            off += g.plane_bytes * bpl;
            g.c_off = off;
            off += align256((size_t)g.n * g.t * csz);
            if (real) {
                g.z_off = off;
                off += align256((size_t)g.n * g.t * csz);
            }
        }
        plan.total = off;
        return PLV_OK;
    }
    for (GramPlan &g : plan.grams) {
        // nchunk blocks of npad x chunk phasors (stage-major inside)
        g.plane_bytes = align256((size_t)g.nchunk * g.npad * g.chunk * cb);
        g.u_off = off;
        off += g.plane_bytes * pl;
    }
    for (GramPlan &g : plan.grams) {
        if (g.fused)
            continue;
        g.part_off = off;
        off += align256((size_t)g.nslot * g.nupper * 2 * g.bm * g.bm * sizeof(double));
    }
    if (op == PLV_OP_COHERENCE) {
        for (GramPlan &g : plan.grams) {
            g.scale_off = off;
            off += align256((size_t)g.n * sizeof(double));
            g.diag_off = off;
            off += align256((size_t)g.npad * sizeof(double));
        }
    }
    plan.total = off;
    return PLV_OK;
}

void fill_descs(const Plan &plan, uint8_t *ws, std::vector<GramDesc> &gd)
{
    gd.clear();
    for (const GramPlan &g : plan.grams) {
        GramDesc d{};
        d.u = ws + g.u_off;
        d.plane_bytes = (int64_t)g.plane_bytes;
        d.cstride = (int64_t)g.npad * g.chunk * cbytes_of(plan.mode);
        d.n = g.n;
        d.npad = g.npad;
        d.t = g.t;
        d.tpad = g.tpad;
        d.ntile = g.ntile;
        d.nupper = g.nupper;
        d.nchunk = g.nchunk;
        d.chunk = g.chunk;
        d.nslot = g.nslot;
        d.fused = g.fused ? 1 : 0;
        d.bm = g.bm;
        d.partial = g.fused ? nullptr : (double *)(ws + g.part_off);
        d.diag = plan.op == PLV_OP_COHERENCE ? (double *)(ws + g.diag_off) : nullptr;
        d.plv = g.plv;
        d.iplv = g.iplv;
        d.ciplv = g.ciplv;
        d.g = g.g;
        if (plan.op == PLV_OP_BACKWARD_ANALYTIC || plan.op == PLV_OP_BACKWARD_REAL) {
            d.cstride = 0;
            d.tpad = g.kpad;
            d.ub = ws + g.w_off;
            d.nb = g.t;
            d.ntile_b = g.ntile_b;
            d.c = ws + g.c_off;
            d.ldc = g.t;
            d.partial = nullptr;
            if (plan.op == PLV_OP_BACKWARD_REAL) {
                d.zbuf = ws + g.z_off;
                d.ldz = g.t;
            }
        }
        gd.push_back(d);
    }
}

void build_tables(const Plan &plan, const std::vector<GramDesc> &gd, std::vector<Item> &items,
                  std::vector<TileRef> &tiles)
{
    items = plan.items;
    tiles.clear();
    tiles.reserve(plan.ntiles);
    const bool backward = plan.op == PLV_OP_BACKWARD_ANALYTIC || plan.op == PLV_OP_BACKWARD_REAL;
    for (size_t q = 0; q < gd.size(); ++q) {
        const GramDesc &d = gd[q];
        if (!backward && !d.fused)
            for (int t = 0; t < d.nupper; ++t)
                tiles.push_back(TileRef{(int32_t)q, t});
    }
}

std::tuple<int, int64_t, int64_t> tune_key(const Plan &plan)
{
    const GramPlan &g = plan.grams[0];
    return std::make_tuple(plan.mode, (int64_t)g.n, (int64_t)g.tpad);
}

void chunk_counts(const Plan &plan, std::vector<int> &out)
{
    out.clear();
    if (plan.grams.size() != 1 || plan.grouped)
        return;
    const GramPlan &g = plan.grams[0];
    const int kgr = g.tpad / PLV_KGRAN;
    int lo, hi;
    chunk_bounds(g, MAX_CHUNK, lo, hi);
    for (int nc = lo; nc <= hi; ++nc)
        if (exact_split(kgr, nc))
            out.push_back(nc);
}

}  // namespace plv
