// Tile geometry shared by the tiled kernels for spatially uniform geometry:
// a workgroup owns a 4x4 tile of cells in the (axis 0, axis 1) plane and
// marches along axis 2; the current plane is staged in LDS with a two-cell
// cross-shaped halo (the PLM stencil is five cells wide along each axis).
#pragma once

namespace rt {

constexpr int kT = 4;            // tile edge
constexpr int kTC = kT * kT;     // interior cells per tile
constexpr int kHalo = 32;        // cross-shaped halo cells (2 deep)
constexpr int kPlane = kTC + kHalo;

// bits of the per-direction flag byte: motion along +/- each axis, masked
constexpr unsigned kXP = 1, kXN = 2, kYP = 4, kYN = 8, kZP = 16, kZN = 32, kMasked = 64;

// LDS slot of plane cell (x, y) relative to the tile origin: the 16 tile
// cells, then the halo rows left/right of the tile, then above/below it
__device__ __forceinline__ int plane_slot(int x, int y) {
    if (x >= 0 && x < kT && y >= 0 && y < kT) return y * kT + x;
    if (y >= 0 && y < kT) return kTC + y * 4 + (x < 0 ? x + 2 : x - 2);
    return kTC + 16 + (y < 0 ? y + 2 : y - 2) * 4 + x;
}

// Tile-relative position of halo slot h (inverse of plane_slot on the halo).
__device__ __forceinline__ void halo_pos(int h, int &x, int &y) {
    if (h < 16) {
        y = h / 4;
        const int hx = h % 4;
        x = hx < 2 ? hx - 2 : hx + 2;
    } else {
        const int hy = (h - 16) / 4;
        x = (h - 16) % 4;
        y = hy < 2 ? hy - 2 : hy + 2;
    }
}

struct Seg {
    int tx0, ty0, z0, z1;
};

}  // namespace rt
