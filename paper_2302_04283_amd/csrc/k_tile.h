// Tile geometry shared by the tiled kernels for spatially uniform geometry:
// a workgroup owns a kTX x kTY tile of cells in the (axis 0, axis 1) plane
// and marches along axis 2; the current plane is staged in LDS with a
// two-cell cross-shaped halo (the PLM stencil is five cells wide along each
// axis).  Each lane group of the workgroup owns one tile cell and stages
// kHPG of the halo cells.
#pragma once

#include <hip/hip_runtime.h>

#ifndef RT_TILE_Y
#define RT_TILE_Y 4
#endif

namespace rt {

constexpr int kTX = 4;                // tile extent along axis 0
constexpr int kTY = RT_TILE_Y;        // tile extent along axis 1
constexpr int kTC = kTX * kTY;        // interior cells per tile
constexpr int kHaloX = 4 * kTY;       // two columns left and right, kTY rows
constexpr int kHaloY = 4 * kTX;       // two rows below and above, kTX columns
constexpr int kHalo = kHaloX + kHaloY;
constexpr int kHPG = kHalo / kTC;     // halo cells staged per lane group
constexpr int kPlane = kTC + kHalo;
static_assert(kHalo % kTC == 0, "halo cells must split evenly over the tile cells");

// bits of the per-direction flag byte: motion along +/- each axis, masked
constexpr unsigned kXP = 1, kXN = 2, kYP = 4, kYN = 8, kZP = 16, kZN = 32, kMasked = 64;

// LDS slot of plane cell (x, y) relative to the tile origin: the tile cells,
// then the halo columns left/right of the tile, then the rows below/above it
__device__ __forceinline__ int plane_slot(int x, int y) {
    if (x >= 0 && x < kTX && y >= 0 && y < kTY) return y * kTX + x;
    if (y >= 0 && y < kTY) return kTC + y * 4 + (x < 0 ? x + 2 : x - kTX + 2);
    return kTC + kHaloX + (y < 0 ? y + 2 : y - kTY + 2) * kTX + x;
}

// Tile-relative position of halo slot h (plane_slot(x, y) == kTC + h).
__device__ __forceinline__ void halo_pos(int h, int &x, int &y) {
    if (h < kHaloX) {
        y = h / 4;
        const int hx = h % 4;
        x = hx < 2 ? hx - 2 : hx - 2 + kTX;
    } else {
        const int hh = h - kHaloX;
        const int hy = hh / kTX;
        x = hh % kTX;
        y = hy < 2 ? hy - 2 : hy - 2 + kTY;
    }
}

struct Seg {
    int tx0, ty0, z0, z1;
};

}  // namespace rt
