// plv_plan.h -- host-side planning: argument checks, workspace layout, K-chunks.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "plv_internal.h"

namespace plv {

constexpr int MAX_CHUNK = 16384;     // longest FP32 accumulation span of one work item (samples)
constexpr int MIN_CHUNK = 128;       // shortest K-chunk worth a work-group
constexpr size_t PARTIAL_BUDGET = size_t(2) << 30;  // partial-slot bytes before T is split into passes

struct GramPlan {
    int64_t prob = 0;
    int band = 0;
    int n = 0, npad = 0;
    int t = 0, t0 = 0, tpad = 0;       // window length, window start, padded length
    int bm = 0;                        // tile edge (64 or 128)
    int ntile = 0, nupper = 0;
    int nchunk = 0, chunk = 0, nslot = 0;
    bool fused = false;                // one chunk: the Gram kernel stores the measures
    size_t u_off = 0, plane_bytes = 0; // phasor planes (backward: the H operand)
    size_t part_off = 0;               // FP64 partial sums
    // backward only: C = H (conj U^T)^H over the full tile grid
    int kpad = 0, ntile_b = 0;
    size_t w_off = 0;                  // W = conj(U^T) planes (B operand)
    size_t c_off = 0;                  // ubar [n][t] complex
    size_t z_off = 0;                  // real input: z, then zbar, [n][t] complex
    size_t scale_off = 0, diag_off = 0; // coherency: row scales [n], row powers [npad] (FP64)
    void *plv = nullptr, *iplv = nullptr, *ciplv = nullptr, *g = nullptr;
};

// FFT stage of one real-input problem.
struct FftPlan {
    int t = 0, logm = 0;
    bool blue = false;
    int tw_index = 0;     // which twiddle table (by logm)
    int len_index = 0;    // which per-length set-up (by t)
    size_t xbin_off = 0;  // bins of directly synthesised bands (only with band-pass bands)
    bool has_xbins = false;
};

// Set-up tables of one distinct row length.
struct LenPlan {
    int t = 0, logm = 0;
    bool blue = false;
    size_t roots_off = 0, chirp_off = 0, bhat_off = 0;  // chirp/bhat: Bluestein only
    std::vector<size_t> firw_off;  // per band: FIR weight table of this length (0: not an FIR band)
};

struct Plan {
    int mode = 0;
    plv_op op = PLV_OP_FROM_ANALYTIC;
    std::vector<GramPlan> grams;
    size_t tables_off = 0, tables_bytes = 0;  // device tables, uploaded once per call
    size_t desc_off = 0, item_off = 0, tile_off = 0;
    bool blocked = false;                     // single Gram problem: blocked tile order (tile_order.h)
    size_t nitems = 0, ntiles = 0;
    std::vector<Item> items;                  // grouped launch: work items, XCD-major (see schedule_items)
    struct ItemGroup {
        int bm;                               // tile edge of every problem in the group
        size_t off, count;                    // its run of `items` (one launch)
    };
    std::vector<ItemGroup> groups;            // one per tile edge present, 128 first
    int bm_max = 0;                           // largest tile edge among the problems
    bool grouped = false;                     // Gram work from the item table
    // real input only
    std::vector<FftPlan> fft;                 // per problem
    std::vector<int> tw_logm;                 // distinct FFT sizes
    std::vector<size_t> tw_off;
    std::vector<LenPlan> lens;                // distinct row lengths, ordered by (logm, t)
    size_t hp_off = 0, bin_off = 0, row_off = 0, job_off = 0;
    size_t synth_off = 0;  // band synthesis: running work-group counts [nprob + 1]
    size_t dftp_off = 0;   // DFT-bins kernel: running work-group counts [nprob + 1]
    size_t xs_off = 0;     // calls with several bands: spectrum slots of the transform launches
    std::vector<int> xs_slots;  // per FFT size (as tw_logm): slots there (0: none reserved)
    std::vector<size_t> fir_r_off;  // per band: the FIR taps' autocorrelation (FP64, in the tables)
    size_t firjob_off = 0;          // FirJob per (row length, FIR band), in the tables
    int nfirjobs = 0, fir_max_t = 0;
    size_t nrows = 0;
    size_t total = 0;
};

// Measured choices that replace the planner's cost models (plv_autotune):
//   chunks: K-chunk counts of single-problem launches, keyed by (mode, rows,
//           padded length);
//   tiles:  the tile edge of a forward problem, keyed by (mode, rows).
typedef std::map<std::tuple<int, int64_t, int64_t>, int> TuneMap;
typedef std::map<std::pair<int, int64_t>, int> TileMap;
struct Tuning {
    TuneMap chunks;
    TileMap tiles;
};

// Work-groups per CU of the Gram kernel, per mode and tile edge:
// occ[2 * mode + (bm == 64)].
constexpr int NOCC = 10;
inline int occ_index(int mode, int bm) { return 2 * mode + (bm == 64 ? 1 : 0); }

// The planner's tile edge for a forward problem of n rows: the one with the
// smaller whole-tile MFMA work over the upper triangle, the 64-wide tile's
// work counted 1/0.85 times (its shorter MFMA runs per barrier).
int model_tile(int mode, int64_t n);
// The tile edge a forward problem of n rows gets: measured, else the model's.
int tile_for(int mode, int64_t n, const Tuning *tune);

// Checks the arguments and lays out the workspace.  `occ` (NOCC entries, see
// occ_index) may be NULL: then 1 is assumed.  `unit_k`: pad each problem's
// samples only to the Gram kernel's K-unit of its mode (k_unit) rather than
// to PLV_KGRAN, when that fits one K-chunk; such a problem runs as a single
// chunk.  Used for the problems across trials, whose K (the trial count) is
// a few dozen, where the granule would add up to 31 zero samples to each.
plv_status make_plan(int cus, const int *occ, plv_op op, plv_prec prec, const plv_problem *probs, int64_t nprob,
                     const plv_band *bands, int32_t nbands, Plan &plan, std::string &why,
                     const Tuning *tune = nullptr, bool unit_k = false);

// The K-chunk counts a single-problem plan can take (every chunk but the last
// the same whole number of granules), ascending; empty for a grouped plan.
void chunk_counts(const Plan &plan, std::vector<int> &out);
// Key of a single-problem plan in a TuneMap.
std::tuple<int, int64_t, int64_t> tune_key(const Plan &plan);

void fill_descs(const Plan &plan, uint8_t *ws, std::vector<GramDesc> &gd);
void build_tables(const Plan &plan, const std::vector<GramDesc> &gd, std::vector<Item> &items,
                  std::vector<TileRef> &tiles);

}  // namespace plv
