// The incremental sort's classification of the slots, as the kernels that
// place particles read it: one stayer bit and one mover bit per slot (a
// 64-bit word per 64 slots), the counts of both before each word inside its
// tile, before each tile inside its group, and before each group.  A
// stayer keeps its cell since the last sort; a mover does not (see
// k_sort.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffpic {

constexpr int kTileShift = 11;      // 2048 slots per tile
constexpr int kGroupShift = 10;     // 1024 tiles per group

struct ClassView {
    int nub;
    const uint64_t *smask, *mmask;   // stayer / mover bit per slot
    const uint32_t *wsm;             // stayers | movers << 16 before the word, in its tile
    const uint2 *ts;                 // stayers / movers before the tile, in its group
    const uint2 *gs;                 // stayers / movers before the group
    const uint32_t *tot;             // stayers, movers, slots before the sort
};

// stayers before slot x (0 <= x <= nub)
__device__ __forceinline__ uint32_t stayers_before(const ClassView &V, int x) {
    if (x >= V.nub) return V.tot[0];
    const int wd = x >> 6;
    const uint64_t below = (1ull << (x & 63)) - 1ull;
    return V.gs[x >> (kTileShift + kGroupShift)].x + V.ts[x >> kTileShift].x +
           (V.wsm[wd] & 0xffffu) + (uint32_t)__popcll(V.smask[wd] & below);
}

// movers before slot x (0 <= x < nub)
__device__ __forceinline__ uint32_t movers_before(const ClassView &V, int x) {
    const int wd = x >> 6;
    const uint64_t below = (1ull << (x & 63)) - 1ull;
    return V.gs[x >> (kTileShift + kGroupShift)].y + V.ts[x >> kTileShift].y + (V.wsm[wd] >> 16) +
           (uint32_t)__popcll(V.mmask[wd] & below);
}

// Where a push that also places its species' sort writes each particle
// (FP32): dest[q] is the place of the particle in slot q in the new order,
// -1 for a slot that holds none.
struct SortPlace {
    const int32_t *dest;
    int32_t *cell;                   // the state of the new order
    float *a, *b, *ur, *ut, *up;
};

}  // namespace ffpic
