// Column-tile staging shared by the streaming kernels (Gram, TTM).
//
// A tile is J x KT columns of the block-column view Y[B][J][L] (TileMap).
// ColumnTile loads one tile into registers with a thread mapping that keeps
// every wave's global loads contiguous, widens to the compute type, and
// writes it to LDS as [i][kk] with a row pitch of KT + 1 elements (an odd
// pitch in 8-byte words spreads both the row-wise and the column-wise
// accesses across banks).
//   L == 1 : column kk is J contiguous elements -> thread t reads row
//            i = t % JB of column t / JB (+ column passes);
//   L  > 1 : rows are runs along kk -> thread t reads column kk = t % KT of
//            row t / KT (+ row passes); the column's offset inside the tile
//            is fixed per thread.
// Elements outside the tile (rows >= J, columns >= the tile's width) are 0.
#pragma once

#include "tk_common.hpp"

namespace tk {

// Offset (relative to a tile's base) of tile column kk: kk = bb * L + l maps
// to bb * J * L + l.  For strided tiles (L >= KT) this is kk itself.
__device__ __forceinline__ int64_t tile_col_offset(int kk, int64_t L, int J) {
    int64_t bb = kk / L;
    return bb * J * L + (kk - bb * L);
}

template <typename T, typename C, int JB, int KT, int THREADS>
struct ColumnTile {
    static_assert(JB * KT % THREADS == 0, "tile must split evenly over threads");
    static_assert(THREADS % JB == 0 && THREADS % KT == 0, "thread mappings need JB, KT | THREADS");
    static constexpr int kPer = JB * KT / THREADS;
    static constexpr int P = KT + 1;  // LDS row pitch (elements)
    C v[kPer];
    int64_t coff;  // L > 1: offset of this thread's column
    int kk0, i0;   // this thread's first (i, kk)
    bool unit;     // L == 1

    __device__ __forceinline__ void setup(const TileMap& tm, int tid) {
        unit = tm.L == 1;
        if (unit) {
            i0 = tid % JB;
            kk0 = tid / JB;
            coff = 0;
        } else {
            kk0 = tid % KT;
            i0 = tid / KT;
            coff = tile_col_offset(kk0, tm.L, tm.J);
        }
    }

    __device__ __forceinline__ void load(const T* __restrict__ y, const TileMap& tm,
                                         const Tile& t) {
        if (unit) {
            constexpr int colstep = THREADS / JB;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                int kk = kk0 + q * colstep;
                C val = C(0);
                if (i0 < tm.J && kk < t.ncols) val = (C)y[t.base + (int64_t)kk * tm.J + i0];
                v[q] = val;
            }
        } else {
            constexpr int rowstep = THREADS / KT;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                int i = i0 + q * rowstep;
                C val = C(0);
                if (i < tm.J && kk0 < t.ncols) val = (C)y[t.base + coff + (int64_t)i * tm.L];
                v[q] = val;
            }
        }
    }

    __device__ __forceinline__ void store(C* lds) const {
        if (unit) {
            constexpr int colstep = THREADS / JB;
#pragma unroll
            for (int q = 0; q < kPer; ++q) lds[i0 * P + kk0 + q * colstep] = v[q];
        } else {
            constexpr int rowstep = THREADS / KT;
#pragma unroll
            for (int q = 0; q < kPer; ++q) lds[(i0 + q * rowstep) * P + kk0] = v[q];
        }
    }
};

}  // namespace tk
