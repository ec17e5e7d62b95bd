// plv_internal.h -- descriptors shared by the host layer and the gfx950 kernels.
//
// Layout of the phasor planes U in the workspace (one "Gram problem" = one
// problem x band): chunk blocks, stage-major inside.  The window, rounded up
// to tpad (a multiple of PLV_KGRAN samples, or of k_unit for a problem that
// the planner keeps in one chunk; zero-filled beyond the window: padding adds
// nothing to G), is cut into K-chunks of `chunk` samples; chunk
// c of every row is stored together as one block of interleaved complex
// phasors u = z/|z| (Eq. 4), blocks cstride bytes apart.  Inside a block the
// samples go in 64-byte stages, all npad rows of one stage back to back
// (plane_off below), so each K-stage of a tile's row panel is one contiguous
// run.  Rows n..npad-1 are never written and only feed output entries that
// are discarded; the tail of the last block past tpad is never touched.
//   Element per complex sample: 2 x bf16/f16 (4 B), 2 x f32 (8 B), 2 x f64 (16 B).
//   PLV_PREC_SPLIT_BF16 has two such planes, hi then lo, plane_bytes apart.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plv.h"
#include "tile_order.h"

#define PLV_KGRAN 32  // sample granule of tpad and of every K-chunk

namespace plv {

// Global-address-space views of device pointers.  Memory accessed through
// them compiles to global_load / global_store (vector-memory counter only)
// rather than flat accesses, which also hold the LDS counter.
template <class T>
__device__ inline __attribute__((address_space(1))) T *gptr(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ inline const __attribute__((address_space(1))) T *gptr(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}

// Native clang vectors (usable through address-space-qualified pointers,
// unlike HIP's struct vector types).
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
typedef uint32_t vu4 __attribute__((ext_vector_type(4)));
#define PLV_GLOBAL __attribute__((address_space(1)))

enum Mode { M_F64 = 0, M_F32 = 1, M_SPLIT = 2, M_BF16 = 3, M_F16 = 4 };

// Phasor planes, stage-major.  K (samples; signals in the backward's product
// operands) is cut into blocks of `chunk`, block c starting c * cstride bytes
// in.  Inside a block, a 64-byte stage holds SPS = 64 / cb consecutive
// K-elements of one row, and the stages of all `rows` rows for the same K
// range lie back to back: element (row, k) of a block is at
// ((k / SPS) * rows + row) * 64 + (k % SPS) * cb.  A K-stage of 16 rows is
// then one contiguous kilobyte, the unit the Gram kernel moves into LDS.
__host__ __device__ inline int64_t plane_off(int64_t rows, int cb, int64_t row, int64_t k)
{
    const int lsps = cb == 4 ? 4 : (cb == 8 ? 3 : 2);  // log2(SPS)
    return (((k >> lsps) * rows + row) << 6) + (k & ((1 << lsps) - 1)) * cb;
}

// Address of sample s of `row` in the planes (plane 0).
__device__ inline uint8_t *plane_at(uint8_t *u, int64_t cstride, int chunk, int64_t rows, int cb, int64_t row, int s)
{
    const int c = s < chunk ? 0 : s / chunk;  // single-chunk problems skip the division
    return u + c * cstride + plane_off(rows, cb, row, s - c * chunk);
}

// Largest tile edge of the Gram kernel for each mode (output tiles are
// BM x BM).  The 16-bit and FP32 modes also have a 64-wide tile for small
// row counts; GramDesc::bm says which edge a problem uses.
__host__ __device__ constexpr int tile_of(int mode) { return mode == M_F64 ? 64 : 128; }
// Bytes per complex phasor element in one plane.
__host__ __device__ constexpr int cbytes_of(int mode) { return mode == M_F64 ? 16 : (mode == M_F32 ? 8 : 4); }
__host__ __device__ constexpr int planes_of(int mode) { return mode == M_SPLIT ? 2 : 1; }
// Samples of one K-unit of the Gram kernel: a 64-byte stage per plane row
// (16 / 8 / 4 samples), two stages for plain BF16 and FP16, whose unit is one
// 32-sample step of each of two MFMA chains.  A chunk's length is a multiple of it.
__host__ __device__ constexpr int k_unit(int mode)
{
    return (mode == M_BF16 || mode == M_F16) ? 32 : 64 / cbytes_of(mode);
}

// One Gram problem: G = U U^H / t over its own phasor planes.
struct GramDesc {
    const uint8_t *u;     // plane 0
    int64_t plane_bytes;  // plane 1 = u + plane_bytes (split only)
    int64_t cstride;      // bytes from one chunk block to the next (0: one block)
    int32_t n, npad;      // signals, rows rounded up to the tile (the planes' row count)
    int32_t t, tpad;      // true window length (the 1/T), padded length
    int32_t ntile;        // tiles per side = npad / bm
    int32_t nupper;       // tiles with I <= J = ntile (ntile + 1) / 2
    int32_t nchunk;       // K-chunks over tpad
    int32_t chunk;        // samples per chunk (multiple of PLV_KGRAN, or of k_unit when there is
                          // one chunk); last may be shorter
    int32_t nslot;        // partial slots (chunks per pass); passes = ceil(nchunk / nslot)
    int32_t fused;        // 1: one chunk, the Gram kernel stores the measures itself
    int32_t bm;           // tile edge BM of this problem (64 or 128; 64 in F64 mode)
    double *partial;      // [nslot][nupper][2][BM][BM] FP64 chunk sums (unused when fused)
    void *plv, *iplv, *ciplv, *g;  // outputs, [n][n] (g complex interleaved)
    // General product mode (used by the backward): C = A B^H over the full
    // tile grid, A = the planes at u (npad rows), B = the planes at ub
    // (ntile_b * BM rows), one block of K = tpad each; C stored directly as
    // complex (f32; f64 in F64 mode).
    const uint8_t *ub;    // B operand planes, nullptr in Gram mode
    int32_t nb, ntile_b;  // B rows, B tiles
    void *c;              // C [n][ldc] complex
    int64_t ldc;
    void *zbuf;           // FFT stage of the backward: complex z of the window
    int64_t ldz;          //   [n][ldz] written instead of phasor planes
    double *diag;         // coherency: [npad] row powers sum |z_i|^2 from the Gram's diagonal
};

// One unit of Gram work: a (problem, tile, chunk) triple.
struct Item {
    int32_t gram, tile, chunk, pad;
};

// One unit of epilogue work: a (problem, tile) pair.
struct TileRef {
    int32_t gram, tile;
};

struct HerkArgs {
    GramDesc g;             // the single problem when items == nullptr
    const GramDesc *gd;     // problem table (grouped launch)
    const Item *items;      // work items (grouped launch: `chunk` is the slot; gram < 0: none), or nullptr
    int32_t nitems;
    int32_t pass;           // chunk = pass * nslot + slot; pass > 0 adds into the slot
    int32_t blocked;        // single Gram problem: tiles in the blocked order (tile_order.h)
};

struct EpiArgs {
    GramDesc g;             // the single problem when tiles == nullptr
    const GramDesc *gd;
    const TileRef *tiles;   // grouped launch, or nullptr
    bool coherence;         // divide by sqrt(d_i d_j) (GramDesc::diag) instead of T
};

// Normalisation job: rows of one problem -> planes of one Gram problem.
struct NormArgs {
    const void *in;       // complex rows (c64 or c128)
    int64_t ld;           // row stride of `in`, complex elements
    int64_t t0;           // first sample of the window
    int32_t tw;           // window length
    int32_t n;            // rows
    uint8_t *u;           // plane 0
    int64_t plane_bytes;
    int64_t cstride;      // stage-major layout of the planes (see plane_off)
    int32_t chunk;
    int32_t rows;         // the planes' row count (npad)
    int32_t tpad;
    int32_t row0;         // first row of this launch (row blocks run on blockIdx.y)
    const double *scale;  // coherency: per-row power-of-two scale (no unit normalisation), else nullptr
};

// Across trials: one launch fills the phasor planes of every time point's
// Gram problem (rows = signals, samples = trials).
struct TrialArgs {
    const void *in;
    int64_t ld, tstride, sstride, t0;  // complex elements
    int32_t n, ntr, ntp;               // signals, trials, time points
    int32_t row0;                      // first signal of this launch (signals run on blockIdx.y)
    uint8_t *u0;                       // planes of time point 0
    int64_t gstride;                   // bytes from one time point's planes to the next
    int64_t plane_bytes, cstride;
    int32_t chunk, tpad;
    int32_t rows;                      // the planes' row count (npad)
};

// Coherency: per-row scale 2^-e with e the exponent of the row's largest
// component over the window, so scaled rows peak in [0.5, 1).
struct ScaleArgs {
    const void *in;       // complex rows (c64 or c128)
    int64_t ld, t0;
    int32_t tw, n;
    double *scale;        // [n]
};

// ------------------------------------------------- analytic signal (FFT) --
// One problem of real rows, transformed at its own length t through an FFT of
// size M = 2^logm (M = t for a power-of-two t; otherwise Bluestein, M >= 2t-1).
struct HilbertProb {
    const void *x;       // real rows [n][ld] (f32; f64 in F64 mode)
    int64_t ld;
    int32_t n, t;        // rows, DFT length
    int32_t t0, tw;      // window start and length (samples that enter the Gram)
    int32_t logm, blue;  // FFT size; 1 = Bluestein
    const void *chirp;   // [t] complex c_m = exp(i pi m^2 / t) (Bluestein)
    const void *bhat;    // [M] complex FFT_M of the circular chirp (Bluestein)
    const void *tw_tab;  // [M/2] complex exp(-2 pi i k / M)
    const void *roots;   // [t] complex exp(2 pi i m / t) (direct band synthesis)
    int32_t gram0;       // Gram problem of band 0 (band b -> gram0 + b)
    int32_t nbands;
    int32_t bin0;        // first entry of this problem in the band-bin table
    int32_t pad_;
    void *xbar;          // backward: dL/dx rows [n][ld] (same dtype as x)
    void *xbins;         // bins of the directly synthesised bands: row r, band b at
                         //   (r * nbands + b) * DIRECT_KMAX complex (nullptr: no band-pass bands)
};

// A band of at most DIRECT_KMAX bins may be synthesised directly from its
// bins (by the band synthesis kernel) instead of by an inverse transform.
constexpr int DIRECT_KMAX = 48;

// Positive-frequency bins [klo, khi] that get weight 2; klo < 0 selects the
// plain one-sided weights (1 at DC, 2 below Nyquist, 1 at Nyquist, 0 above).
// direct = 1: synthesise the band from its bins instead of an inverse FFT.
struct BandBins {
    int32_t klo, khi;
    int32_t direct;
    int32_t fir;          // 1: forward-backward FIR band: weights = one-sided x w[k]
    const void *w;        // FIR: |H|^2 at bins k = 0..t/2 of the row length (R precision)
};

// One FIR weight table: w[k] = |H(exp(2 pi i k / t))|^2 = A(theta)^2, k = 0..t/2,
// A(theta) = c[0] + 2 sum_{j=1..half} c[j] cos(j theta), c = the upper half of
// the filter's symmetric taps (FP64, c[0] the centre tap).
struct FirJob {
    int32_t t, half;
    const double *c;
    void *w;
};

struct RowRef {
    int32_t prob, row;
};

struct HilbertArgs {
    const HilbertProb *hp;
    const BandBins *bins;
    const RowRef *rows;   // rows of this launch (all share logm)
    int32_t nrows;
    int32_t logm;
    const GramDesc *gd;   // destinations of the phasor planes
    int32_t nbands;       // bands per problem (the same for every problem of a call)
    int32_t nprob;        // band synthesis: problems, and the running work-group counts
    const int32_t *synth_prefix;  //   [nprob + 1] of the problems (see band_synth_kernel)
    int32_t fir;          // some band of the call is an FIR band (selects the kernel variant)
    int32_t xslots;       // work-group slots at xs (the transform launches use at most this many)
    const int32_t *dft_prefix;    // DFT-bins kernel: [nprob + 1] running work-group counts
    void *xs;             // calls with several bands: [xslots][M] complex, a row's spectrum per
                          // work-group (forward) or its band sum (adjoint); nullptr otherwise
};

// Set-up for one distinct row length t: its root table, and for a Bluestein
// length the chirp and the transformed circular chirp.
struct ChirpJob {
    int32_t t, logm;
    int32_t blue, pad_;
    void *chirp;          // [t] complex (Bluestein)
    void *bhat;           // [M] complex (Bluestein)
    void *roots;          // [t] complex
    const void *tw_tab;   // [M/2] twiddles of this M
};

// ---------------------------------------------------------------- backward --
struct BwdPlanesArgs {      // W[s][k] = conj(u_k(s)): the product's B operand
    const void *z;           // complex rows of the window [n][ldz]
    int64_t ldz;
    int32_t n, tw, kpad;
    int32_t rows;            // row count of W's planes (>= tw, whole tiles)
    uint8_t *w;              // planes, rows x kpad (stage-major, one block)
    int64_t plane_bytes;
};

struct BwdMetricArgs {      // H = (Gbar + Gbar^H) / T: the product's A operand
    const void *g;           // forward complex G [n][n]
    const void *dplv, *diplv, *dciplv;  // upstream [n][n] (nullptr = 0)
    int32_t n, kpad;
    int32_t row0;            // first row of this launch (rows run on blockIdx.y)
    double inv_t;
    int32_t rows;            // row count of H's planes (npad)
    uint8_t *h;              // planes, npad x kpad (stage-major, one block)
    int64_t plane_bytes;
};

struct BwdNormArgs {        // zbar = i Im(conj(u) ubar) u / |z|
    const void *z;           // window rows [n][ldz]
    int64_t ldz;
    const void *c;           // ubar rows [n][ldc]
    int64_t ldc;
    void *dst;               // output rows [n][ldd]; sample s of the window at q = s + off
    int64_t ldd;
    int32_t off, len, tw, n; // q runs over [0, len); outside the window -> 0
    int32_t row0;            // first row of this launch (rows run on blockIdx.y)
};

// ------------------------------------------------------ segment spectra --
// Windowed-segment DFT bins for the coherency over segments (stft.hip).
constexpr int STFT_MAX_SEG = 4096;   // longest segment (LDS-resident twiddles and window)

struct StftTables {
    int32_t seg, window;  // L, plv_window
    void *tw;             // [L] complex exp(-2 pi i j / L) (R precision)
    void *win;            // [L] window w[m] (R precision)
};

struct StftArgs {
    const void *x;        // real rows [n][ld] (f32; f64 in F64 mode)
    int64_t ld, t0;       // row stride, first sample of segment 0
    int32_t n, seg, hop, nseg;
    int32_t k_lo, k_hi;
    int32_t spw;          // segments per work-group
    int32_t row0;         // first row of this launch (rows run on blockIdx.y)
    const void *tw, *win; // StftTables
    void *coef;           // [k_hi - k_lo + 1][n][nseg] complex (c64; c128 in F64 mode)
};

// -------------------------------------------------------------- launchers --
// Row-parallel launches put rows on gridDim.y, whose limit is 65535; the
// launchers cover larger n in blocks of rows.
constexpr int MAX_GRID_Y = 65535;
// Each returns hipSuccess or the launch error.
hipError_t launch_normalise(int mode, const NormArgs &a, hipStream_t s);
// Every problem a launch reaches must have GramDesc::bm == bm.
hipError_t launch_herk(int mode, int bm, const HerkArgs &a, int nwg, hipStream_t s);
// Tile edges the Gram kernel has for a mode.
bool tile_supported(int mode, int bm);
// bm_max: the largest tile edge among the tiles (the grid covers it).  rows:
// the row-wise kernel (FP32 outputs, every problem with n a multiple of 4
// and 16-byte aligned outputs; the caller checks).
hipError_t launch_epilogue(int mode, const EpiArgs &a, int ntiles, int bm_max, bool rows, hipStream_t s);
hipError_t launch_row_scale(bool f64, const ScaleArgs &a, hipStream_t s);
hipError_t launch_trial_planes(int mode, const TrialArgs &a, hipStream_t s);
// d[i] = fixed-order sum over slots of the diagonal entries of G's partials
hipError_t launch_diag(int mode, const GramDesc &g, hipStream_t s);
// Occupancy (work-groups per CU) of the Gram kernel of `mode` with tile edge bm.
int herk_occupancy(int mode, int bm);
// FFT stage (fft.hip).  f64 selects double precision tables and transforms.
constexpr int FFT_MAXLOG_F32 = 13;  // M <= 8192 complex FP32 transforms in LDS
constexpr int FFT_MAXLOG_F64 = 13;  // M <= 8192 complex FP64 (pass twiddles from global memory at 8192)
hipError_t launch_twiddles(bool f64, void *tab, int logm, hipStream_t s);
// jobs: device array of njobs set-ups that all have this logm
hipError_t launch_chirps(bool f64, int logm, const ChirpJob *jobs, int njobs, hipStream_t s);
// FIR weight tables; max_t = the longest row length among the jobs
hipError_t launch_fir_weights(bool f64, const FirJob *jobs, int njobs, int max_t, hipStream_t s);
// rows of a.rows all have FFT size a.logm; the grid is sized from cus and the
// kernel's occupancy
hipError_t launch_hilbert(int mode, const HilbertArgs &a, int cus, hipStream_t s);
hipError_t launch_hilbert_adjoint(bool f64, const HilbertArgs &a, int cus, hipStream_t s);
// Upper bound on the resident work-groups per CU of a transform kernel of
// size 2^logm (from its LDS), at most 16: the spectrum slots reserved per CU.
int fft_wg_per_cu(bool f64, int logm);
// after launch_hilbert: the bands with BandBins::direct of every problem, from
// their bins in HilbertProb::xbins; njobs = a.synth_prefix[a.nprob] work-groups
hipError_t launch_band_synth(int mode, const HilbertArgs &a, int njobs, hipStream_t s);
constexpr int SYNTH_S = 64, SYNTH_R = 256;  // samples and rows per band-synthesis work-group
// Problems whose bands are all narrow, with at most DFT_MAX_BINS bins in all,
// take their bins from the DFT-bins kernel (dft.hip, FP32 modes) instead of
// the transform kernel; njobs = a.dft_prefix[a.nprob] work-groups of 64 rows.
constexpr int DFT_MAX_BINS = 96;
constexpr int DFT_ROWS_PER_WG = 64;
hipError_t launch_dft_bins(const HilbertArgs &a, int njobs, hipStream_t s);
hipError_t launch_planes_t(int mode, const BwdPlanesArgs &a, hipStream_t s);
hipError_t launch_metric_adjoint(int mode, const BwdMetricArgs &a, hipStream_t s);
hipError_t launch_normalise_adjoint(bool f64, const BwdNormArgs &a, hipStream_t s);
hipError_t launch_stft_tables(bool f64, const StftTables &a, hipStream_t s);
hipError_t launch_stft(bool f64, const StftArgs &a, hipStream_t s);

}  // namespace plv
