// tile_order.h -- launch order of the upper-triangle tiles of one Gram problem.
//
// Tiles that run at the same time on one XCD (consecutive work-groups of a
// single problem) should form a compact block, so they share ORDER_BR row
// panels and ORDER_BC column panels in that XCD's L2 instead of one row
// panel and one column panel each.  The order is: blocks of ORDER_BR x
// ORDER_BC tiles, row-major over blocks, and inside a block row-major over
// the tiles (I, J) with I <= J < ntile.  blocked_tile() maps a position in
// that order to its tile by counting, so no table has to be built or copied
// to the device.  Plain C++ (no HIP types), so a host-only test can compile it.
#pragma once

#ifdef __HIPCC__
#define PLV_HD __host__ __device__
#else
#define PLV_HD
#endif

namespace plv {

constexpr int ORDER_BR = 4, ORDER_BC = 8;

PLV_HD inline int order_min(int a, int b) { return a < b ? a : b; }
PLV_HD inline int order_max(int a, int b) { return a > b ? a : b; }

// Tiles of block row / block (bi, bj) that lie in the upper triangle: row i
// of the block holds the columns [max(i, j0), j1).
PLV_HD inline int block_count(int i0, int i1, int j0, int j1)
{
    int c = 0;
    for (int i = i0; i < i1; ++i)
        c += order_max(0, j1 - order_max(i, j0));
    return c;
}

// Position p (0 <= p < ntile (ntile + 1) / 2) -> tile (I, J).
PLV_HD inline void blocked_tile(int p, int nt, int &I, int &J)
{
    int i0 = 0;
    for (;; i0 += ORDER_BR) {  // a block row's tiles: row i holds nt - i of them
        const int c = block_count(i0, order_min(nt, i0 + ORDER_BR), 0, nt);
        if (p < c)
            break;
        p -= c;
    }
    const int i1 = order_min(nt, i0 + ORDER_BR);
    int j0 = 0;
    for (;; j0 += ORDER_BC) {  // blocks wholly below the diagonal count 0
        const int c = block_count(i0, i1, j0, order_min(nt, j0 + ORDER_BC));
        if (p < c)
            break;
        p -= c;
    }
    const int j1 = order_min(nt, j0 + ORDER_BC);
    for (int i = i0;; ++i) {
        const int c = order_max(0, j1 - order_max(i, j0));
        if (p < c) {
            I = i;
            J = order_max(i, j0) + p;
            return;
        }
        p -= c;
    }
}

}  // namespace plv
