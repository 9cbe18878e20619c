// Block/slab tiling shared by the per-level predict (compression) and
// reconstruct (decompression) kernels.
//
// Every level l is handled in its own grid coordinates (level coordinate =
// full-resolution coordinate / s_l), where a block of B^3 points is E^3 level
// points with E = B / s_l, the level-l points are those with an odd
// coordinate, and the previous level's grid is the all-even sub-grid. One
// work-group owns one block and walks it in z-slabs of H level planes: the
// coarse points the slab's stencils read (a halo of 3 level points, i.e. the
// even points from 2 below to 2 above) are staged in LDS, then every thread
// produces an adjacent (even x, odd x) pair of one row. Rows of the same
// (z, y) parity type go to the same wave, so the 2 classes a thread handles
// are the same across the wave and no lane diverges.
#pragma once

#include "stz_device.h"

namespace stz {
namespace dev {
namespace {

template <int E>
struct SlabShape {
  static constexpr int m = E / 2;                          // class sub-grid extent
  static constexpr int H = E >= 64 ? 2 : (E == 32 ? 8 : E);  // level planes per slab
  static constexpr int HZ = H / 2;                         // class rows (v_z) per slab
  static constexpr int T = m + 3;                          // coarse tile extent, x and y
  static constexpr int TZ = HZ + 3;                        // coarse tile planes
  static constexpr int TILE = TZ * T * T;
  static constexpr int P = m;                              // (even, odd) pairs per row
  static constexpr int RW = 64 / P < 1 ? 1 : 64 / P;       // rows per wave task
  static constexpr int G = (m + RW - 1) / RW;              // row groups per parity
  static constexpr int TASKS_PER_Z = 2 * G;                // wave tasks per level plane
};

// Work-group -> block. In full-domain launches blocks are handed out in
// contiguous raster ranges per XCD (work-group i runs on XCD i mod 8), so
// neighbouring blocks, which share coarse halos, share an L2.
__device__ inline int64_t wg_block(int64_t wg, int64_t nblocks, bool xcd_remap) {
  if (!xcd_remap || (nblocks & 7)) return wg;
  return (wg & 7) * (nblocks >> 3) + (wg >> 3);
}

// Load the coarse tile of a slab: level-(l-1) points (coarse coordinates
// cz0 + tz, cy0 + ty, cx0 + tx) inside the source grid box; others are zero
// and never read by a stencil whose flags allow them.
template <int E>
__device__ inline void load_tile(float* tile, const float* __restrict__ src, const int64_t sf[3],
                                 const int64_t sc[3], int64_t cz0, int64_t cy0, int64_t cx0) {
  using S = SlabShape<E>;
  for (int i = threadIdx.x; i < S::TILE; i += blockDim.x) {
    const int tx = i % S::T, r = i / S::T, ty = r % S::T, tz = r / S::T;
    const int64_t cz = cz0 + tz - sf[0], cy = cy0 + ty - sf[1], cx = cx0 + tx - sf[2];
    float v = 0.0f;
    if (cz >= 0 && cz < sc[0] && cy >= 0 && cy < sc[1] && cx >= 0 && cx < sc[2])
      v = src[(cz * sc[1] + cy) * sc[2] + cx];
    tile[i] = v;
  }
}

// Prediction of the level point at global level coordinates p, class parity
// o, from the slab's coarse tile whose origin (level coordinates, even) is
// (tz0, ty0, tx0). n = level grid extents.
template <int E>
__device__ inline float tile_predict(const float* tile, const int64_t p[3], const int64_t n[3],
                                     const int o[3], int64_t tz0, int64_t ty0, int64_t tx0) {
  using S = SlabShape<E>;
  return predict_point(p, 0, n, o, [&](int64_t z, int64_t y, int64_t x) {
    return tile[((((z - tz0) >> 1) * S::T) + ((y - ty0) >> 1)) * S::T + ((x - tx0) >> 1)];
  });
}

}  // namespace
}  // namespace dev
}  // namespace stz
