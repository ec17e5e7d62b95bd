// plv_internal.h -- descriptors shared by the host layer and the gfx950 kernels.
//
// Layout of the phasor planes U in the workspace (one "Gram problem" = one
// problem x band):
//   rows [npad][ldu] of interleaved complex phasors u = z/|z| (Eq. 4), T-contiguous;
//   ldu = tpad = window length rounded up to PLV_KGRAN samples, zero-filled
//   beyond the window (padding adds nothing to G); rows n..npad-1 are never
//   written and only feed output entries that are discarded.
//   Element per complex sample: 2 x bf16/f16 (4 B), 2 x f32 (8 B), 2 x f64 (16 B).
//   PLV_PREC_SPLIT_BF16 has two such planes, hi then lo, plane_bytes apart.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plv.h"

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

// Tile edge of the Gram kernel for each mode (output tiles are BM x BM).
__host__ __device__ constexpr int tile_of(int mode) { return mode == M_F64 ? 64 : 128; }
// Bytes per complex phasor element in one plane.
__host__ __device__ constexpr int cbytes_of(int mode) { return mode == M_F64 ? 16 : (mode == M_F32 ? 8 : 4); }
__host__ __device__ constexpr int planes_of(int mode) { return mode == M_SPLIT ? 2 : 1; }

// One Gram problem: G = U U^H / t over its own phasor planes.
struct GramDesc {
    const uint8_t *u;     // plane 0
    int64_t plane_bytes;  // plane 1 = u + plane_bytes (split only)
    int64_t ldu;          // row pitch of U in complex elements (= tpad)
    int32_t n, npad;      // signals, rows rounded up to the tile
    int32_t t, tpad;      // true window length (the 1/T), padded length
    int32_t ntile;        // tiles per side = npad / BM
    int32_t nupper;       // tiles with I <= J = ntile (ntile + 1) / 2
    int32_t nchunk;       // K-chunks over tpad
    int32_t chunk;        // samples per chunk (multiple of PLV_KGRAN); last may be shorter
    int32_t nslot;        // partial slots (chunks per pass); passes = ceil(nchunk / nslot)
    int32_t pad_;
    double *partial;      // [nslot][nupper][2][BM][BM] FP64 chunk sums
    void *plv, *iplv, *ciplv, *g;  // outputs, [n][n] (g complex interleaved)
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
    const Item *items;      // work items (grouped launch: `chunk` is the slot), or nullptr
    int32_t nitems;
    int32_t pass;           // chunk = pass * nslot + slot; pass > 0 adds into the slot
};

struct EpiArgs {
    GramDesc g;             // the single problem when tiles == nullptr
    const GramDesc *gd;
    const TileRef *tiles;   // grouped launch, or nullptr
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
    int64_t ldu;          // = tpad
    int32_t tpad;
};

// -------------------------------------------------------------- launchers --
// Each returns hipSuccess or the launch error.
hipError_t launch_normalise(int mode, const NormArgs &a, hipStream_t s);
hipError_t launch_herk(int mode, const HerkArgs &a, int nwg, hipStream_t s);
hipError_t launch_epilogue(int mode, const EpiArgs &a, int ntiles, hipStream_t s);
// Occupancy (work-groups per CU) of the Gram kernel of `mode`.
int herk_occupancy(int mode);

}  // namespace plv
