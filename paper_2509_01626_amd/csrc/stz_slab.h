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

// Default slab height (level planes) for block edge E.
constexpr int default_slab_h(int E) { return E >= 64 ? 2 : (E == 32 ? 8 : E); }

template <int E, int HH = default_slab_h(E)>
struct SlabShape {
  static constexpr int m = E / 2;                          // class sub-grid extent
  static constexpr int H = HH;                             // level planes per slab
  static constexpr int HZ = H / 2;                         // class rows (v_z) per slab
  static constexpr int T = m + 3;                          // coarse tile extent, x and y
  static constexpr int TZ = HZ + 3;                        // coarse tile planes
  static constexpr int TP = T;  // tile row pitch (values)
  static constexpr int TILE = TZ * T * TP;
  // Symbol staging: row pitch m+2 u16 (an odd number of 32-bit words for
  // m >= 4) and an 8-word skew between classes.
  static constexpr int SP = m + 2;
  static constexpr int SCP = HZ * m * SP + 16;
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

// The blocks of a level whose cubic stencils have full support on every axis
// (block_interior) form one box of block indices, [lo, hi) per axis (lo = hi
// on every axis when there is none). The predictor's plain launches for
// large blocks take the box and the shell of remaining blocks in two kernels,
// each compiled for its own kind of block only; these map a launch's i-th
// work item to its block (raster order inside the box, resp. over the shell).
struct BlockSplit {
  int64_t nb[3];         // blocks per axis
  int64_t lo[3], hi[3];  // the interior box
};

// The interior box of a level grid of extents n in blocks of E points:
// block b is interior when b*E >= 2 and b*E + E + 3 <= n on every axis.
__host__ __device__ inline BlockSplit block_split(const int64_t nb[3], int E, const int64_t n[3]) {
  BlockSplit b;
  bool empty = false;
  for (int d = 0; d < 3; ++d) {
    b.nb[d] = nb[d];
    b.lo[d] = (2 + E - 1) / E;
    const int64_t hi = n[d] - E - 3 >= 0 ? (n[d] - E - 3) / E + 1 : 0;
    b.hi[d] = hi < nb[d] ? hi : nb[d];
    empty = empty || b.hi[d] <= b.lo[d];
  }
  if (empty)
    for (int d = 0; d < 3; ++d) b.lo[d] = b.hi[d] = 0;
  return b;
}

__host__ __device__ inline int64_t box_count(const BlockSplit& b) {
  return (b.hi[0] - b.lo[0]) * (b.hi[1] - b.lo[1]) * (b.hi[2] - b.lo[2]);
}

__device__ inline int64_t box_block(const BlockSplit& b, int64_t i) {
  const int64_t w2 = b.hi[2] - b.lo[2], w1 = b.hi[1] - b.lo[1];
  const int64_t ix = i % w2, t = i / w2, iy = t % w1, iz = t / w1;
  return ((b.lo[0] + iz) * b.nb[1] + (b.lo[1] + iy)) * b.nb[2] + (b.lo[2] + ix);
}

__device__ inline int64_t shell_block(const BlockSplit& b, int64_t j) {
  const int64_t A = b.nb[1] * b.nb[2];
  const int64_t w1 = b.hi[1] - b.lo[1], w2 = b.hi[2] - b.lo[2];
  if (j < b.lo[0] * A) return j;  // whole planes before the box
  j -= b.lo[0] * A;
  const int64_t per = A - w1 * w2;  // shell blocks of a plane through the box
  if (j < (b.hi[0] - b.lo[0]) * per) {
    const int64_t pz = b.lo[0] + j / per;
    int64_t r = j % per;
    if (r < b.lo[1] * b.nb[2]) return pz * A + r;  // whole rows before the box
    r -= b.lo[1] * b.nb[2];
    const int64_t rowper = b.nb[2] - w2;  // shell blocks of a row through the box
    if (r < w1 * rowper) {
      const int64_t py = b.lo[1] + r / rowper, c = r % rowper;
      return pz * A + py * b.nb[2] + (c < b.lo[2] ? c : c + w2);
    }
    return pz * A + b.hi[1] * b.nb[2] + (r - w1 * rowper);  // rows after the box
  }
  return b.hi[0] * A + (j - (b.hi[0] - b.lo[0]) * per);  // planes after the box
}

// Load the coarse tile of a slab: level-(l-1) points (coarse coordinates
// cz0 + tz, cy0 + ty, cx0 + tx) inside the source grid box; others are zero
// and never read by a stencil whose flags allow them.
template <class S, class V>
__device__ inline void load_tile(V* tile, const V* __restrict__ src, const int64_t sf[3],
                                 const int64_t sc[3], int64_t cz0, int64_t cy0, int64_t cx0) {
  for (int i = threadIdx.x; i < S::TZ * S::T * S::T; i += blockDim.x) {
    const int tx = i % S::T, r = i / S::T, ty = r % S::T, tz = r / S::T;
    const int64_t cz = cz0 + tz - sf[0], cy = cy0 + ty - sf[1], cx = cx0 + tx - sf[2];
    V v = V(0);
    if (cz >= 0 && cz < sc[0] && cy >= 0 && cy < sc[1] && cx >= 0 && cx < sc[2])
      v = src[(cz * sc[1] + cy) * sc[2] + cx];
    tile[r * S::TP + tx] = v;
  }
}

// The same tile in two halves: fetch this thread's share of the tile into
// registers (NT threads), then store it, so that other work can run while
// the loads are in flight.
template <class S, class V, int NT = 256>
struct TileRegs {
  static constexpr int N = S::TZ * S::T * S::T;
  static constexpr int K = (N + NT - 1) / NT;
  V v[K];
};

template <class S, class V, int NT = 256>
__device__ inline void tile_fetch(TileRegs<S, V, NT>& r, const V* __restrict__ src,
                                  const int64_t sf[3], const int64_t sc[3], int64_t cz0,
                                  int64_t cy0, int64_t cx0) {
#pragma unroll
  for (int k = 0; k < TileRegs<S, V, NT>::K; ++k) {
    const int i = threadIdx.x + NT * k;
    V v = V(0);
    if (i < TileRegs<S, V, NT>::N) {
      const int tx = i % S::T, t = i / S::T, ty = t % S::T, tz = t / S::T;
      const int64_t cz = cz0 + tz - sf[0], cy = cy0 + ty - sf[1], cx = cx0 + tx - sf[2];
      if (cz >= 0 && cz < sc[0] && cy >= 0 && cy < sc[1] && cx >= 0 && cx < sc[2])
        v = src[(cz * sc[1] + cy) * sc[2] + cx];
    }
    r.v[k] = v;
  }
}

template <class S, class V, int NT = 256>
__device__ inline void tile_store(V* tile, const TileRegs<S, V, NT>& r) {
#pragma unroll
  for (int k = 0; k < TileRegs<S, V, NT>::K; ++k) {
    const int i = threadIdx.x + NT * k;
    if (i < TileRegs<S, V, NT>::N) tile[(i / S::T) * S::TP + i % S::T] = r.v[k];
  }
}

// Sliding coarse window: consecutive slabs of a block read overlapping coarse
// planes (TZ per slab, the last HZ of them new). Between two slabs the window
// moves down by HZ planes in LDS and the new planes are loaded into its top.
// NS threads (index st) do it, each owning the same (row, column) positions
// in every plane, so the moves need no barrier among them; nothing else may
// touch the window meanwhile. cz_new = coarse plane of the first new plane.
template <class S, class V, int NS>
__device__ inline void slide_window(V* tile, const V* __restrict__ src, const int64_t sf[3],
                                    const int64_t sc[3], int64_t cz_new, int64_t cy0,
                                    int64_t cx0, int st) {
  constexpr int PE = S::T * S::T, PL = S::T * S::TP, KE = (PE + NS - 1) / NS;
  V nv[KE][S::HZ];
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int e = st + NS * k;
    const int ty = e / S::T, tx = e % S::T;
    const int64_t cy = cy0 + ty - sf[1], cx = cx0 + tx - sf[2];
    const bool in_yx = e < PE && cy >= 0 && cy < sc[1] && cx >= 0 && cx < sc[2];
#pragma unroll
    for (int j = 0; j < S::HZ; ++j) {
      const int64_t cz = cz_new + j - sf[0];
      nv[k][j] = (in_yx && cz >= 0 && cz < sc[0]) ? src[(cz * sc[1] + cy) * sc[2] + cx] : V(0);
    }
  }
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int e = st + NS * k;
    if (e < PE) {
      const int off = (e / S::T) * S::TP + e % S::T;
#pragma unroll
      for (int q = 0; q + S::HZ < S::TZ; ++q) tile[q * PL + off] = tile[(q + S::HZ) * PL + off];
#pragma unroll
      for (int j = 0; j < S::HZ; ++j) tile[(S::TZ - S::HZ + j) * PL + off] = nv[k][j];
    }
  }
}

// True when every odd level coordinate of the block has full cubic support
// (offsets -3..+3 inside the level grid) on every axis: M3, P1 and P3 hold
// for all its points, so each class uses its Eq. 6 / 7 / 8 form.
__device__ inline bool block_interior(const int64_t o[3], int E, const int64_t n[3]) {
  bool in = true;
  for (int d = 0; d < 3; ++d) in = in && o[d] >= 2 && o[d] + E + 3 <= n[d];
  return in;
}

// One-axis rule of the nested fallback (format 2.2); f(i) is the value at
// offset index i along the axis: 0 = -3, 1 = -1, 2 = +1. V = value type.
template <class V, class F>
__device__ inline V nest_rule(bool p1, bool m3, F f) {
  if (p1) {
    const V lo = f(1);
    const V hi = f(2);
    return (lo + hi) * V(0.5);
  }
  if (m3) {
    const V lo = f(1);
    const V lo3 = f(0);
    return ((V(3) * lo) - lo3) * V(0.5);
  }
  return f(1);
}

// Prediction of a class-C point from the slab's coarse tile (format 2.2), with
// the class's odd axes fixed at compile time. w = tile-relative level
// coordinates (level coordinate - tile origin - 2): an even coordinate sits at
// tile index w/2 + 1; the neighbours of an odd one at offsets -3, -1, +1, +3
// (offset index 0..3) at tile indices k..k+3, k = (w-1)/2. p = global level
// coordinates and n = level grid extents give the availability flags; with
// FULL every flag is known to hold (interior blocks). V = value type: the
// same formulas and order in float32 or float64.
template <class V, int E, int C, bool FULL>
__device__ inline V tile_pred(const V* tile, int wz, int wy, int wx, const int64_t p[3],
                              const int64_t n[3]) {
  constexpr int T = SlabShape<E>::T, TP = SlabShape<E>::TP;
  constexpr bool OZ = (C >> 2) & 1, OY = (C >> 1) & 1, OX = C & 1;
  constexpr int ND = int(OZ) + int(OY) + int(OX);
  const int bz = OZ ? (wz - 1) >> 1 : (wz >> 1) + 1;
  const int by = OY ? (wy - 1) >> 1 : (wy >> 1) + 1;
  const int bx = OX ? (wx - 1) >> 1 : (wx >> 1) + 1;
  // v(i, j, k): offset indices along the odd axes in order z, y, x; the tap
  // offsets are compile-time constants relative to one base address.
  const V* tb = tile + (bz * T + by) * TP + bx;
  auto v = [&](int i, int j, int k) {
    int o[3] = {0, 0, 0};
    int q = 0;
    const int idx[3] = {i, j, k};
    if constexpr (OZ) o[0] = idx[q++];
    if constexpr (OY) o[1] = idx[q++];
    if constexpr (OX) o[2] = idx[q++];
    return tb[(o[0] * T + o[1]) * TP + o[2]];
  };
  // availability flags of the odd axes, in order
  bool P1[3] = {true, true, true}, M3[3] = {true, true, true}, P3[3] = {true, true, true};
  if constexpr (!FULL) {
    int q = 0;
    if constexpr (OZ) {
      P1[q] = p[0] + 1 <= n[0] - 1;
      M3[q] = p[0] >= 3;
      P3[q] = p[0] + 3 <= n[0] - 1;
      ++q;
    }
    if constexpr (OY) {
      P1[q] = p[1] + 1 <= n[1] - 1;
      M3[q] = p[1] >= 3;
      P3[q] = p[1] + 3 <= n[1] - 1;
      ++q;
    }
    if constexpr (OX) {
      P1[q] = p[2] + 1 <= n[2] - 1;
      M3[q] = p[2] >= 3;
      P3[q] = p[2] + 3 <= n[2] - 1;
      ++q;
    }
  }
  if constexpr (ND == 1) {
    if (P1[0]) {
      const V B = v(1, 0, 0), Cv = v(2, 0, 0);
      if (M3[0] && P3[0]) {
        const V A = v(0, 0, 0), D = v(3, 0, 0);
        return ((V(9) * (B + Cv)) - (A + D)) * V(0.0625);
      }
      if (P3[0]) {
        const V D = v(3, 0, 0);
        return ((V(3) * B + V(6) * Cv) - D) * V(0.125);
      }
      if (M3[0]) {
        const V A = v(0, 0, 0);
        return ((V(6) * B + V(3) * Cv) - A) * V(0.125);
      }
      return (B + Cv) * V(0.5);
    }
    const V B = v(1, 0, 0);
    if (M3[0]) {
      const V A = v(0, 0, 0);
      return ((V(3) * B) - A) * V(0.5);
    }
    return B;
  } else if constexpr (ND == 2) {
    if (FULL || (P1[0] && M3[0] && P3[0] && P1[1] && M3[1] && P3[1])) {
      const V i0 = v(1, 1, 0), i1 = v(1, 2, 0), i2 = v(2, 1, 0), i3 = v(2, 2, 0);
      const V o0 = v(0, 0, 0), o1 = v(0, 3, 0), o2 = v(3, 0, 0), o3 = v(3, 3, 0);
      V in = i0;
      in = in + i1;
      in = in + i2;
      in = in + i3;
      V out = o0;
      out = out + o1;
      out = out + o2;
      out = out + o3;
      return ((V(9) * in) - out) * V(0.03125);
    }
    return nest_rule<V>(P1[0], M3[0], [&](int i) {
      return nest_rule<V>(P1[1], M3[1], [&](int j) { return v(i, j, 0); });
    });
  } else {
    if (FULL || (P1[0] && M3[0] && P3[0] && P1[1] && M3[1] && P3[1] && P1[2] && M3[2] && P3[2])) {
      // all 16 taps read before the sums (independent LDS reads in flight)
      V t[16];
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = v(1 + (k >> 2), 1 + ((k >> 1) & 1), 1 + (k & 1));
#pragma unroll
      for (int k = 0; k < 8; ++k) t[8 + k] = v(3 * (k >> 2), 3 * ((k >> 1) & 1), 3 * (k & 1));
      V in = t[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) in = in + t[k];
      V out = t[8];
#pragma unroll
      for (int k = 9; k < 16; ++k) out = out + t[k];
      return ((V(9) * in) - out) * V(0.015625);
    }
    return nest_rule<V>(P1[0], M3[0], [&](int i) {
      return nest_rule<V>(P1[1], M3[1], [&](int j) {
        return nest_rule<V>(P1[2], M3[2], [&](int k) { return v(i, j, k); });
      });
    });
  }
}

}  // namespace
}  // namespace dev
}  // namespace stz

namespace stz {
namespace dev {
namespace {

// Rows of parity type (ZP, YP) in the slab [z0, z0 + hs) assigned to this
// wave (of NW): calls f(lz, ly, q, lyu) for the thread's (even, odd) x pair
// q of each row; lyu = the first row of the wave's task (ly - lyu depends on
// the lane only), so row addresses can be split into a scalar part and a
// per-lane offset. Every type has the same number of rows, so the waves stay
// balanced.
template <int E, int ZP, int YP, int NW, class F>
__device__ inline void for_type_rows(int z0, int hs, int Ey, int wave, int lane, F f) {
  using S = SlabShape<E>;
  const int nz = (hs - ZP + 1) >> 1;  // planes of parity ZP in the slab
  const int ntask = nz * S::G;
  const int r = lane / S::P, q = lane % S::P;
  if (r >= S::RW) return;
  for (int t = wave; t < ntask; t += NW) {
    const int iz = t / S::G, g = t - iz * S::G;
    const int lz = z0 + ZP + 2 * iz;
    const int lyu = YP + 2 * g * S::RW;  // the wave's first row: uniform
    const int ly = lyu + 2 * r;
    if (ly < Ey) f(lz, ly, q, lyu);
  }
}

// Tasks (rows) of one parity type a wave can get in a slab of H planes.
template <int E, int H, int NW>
constexpr int type_tasks_per_wave() {
  return (((H + 1) / 2) * SlabShape<E>::G + NW - 1) / NW;
}

// for_type_rows with the wave's task number k (0 .. type_tasks_per_wave - 1)
// unrolled at compile time, so per-task values can live in registers:
// calls f(k, lz, ly, q, lyu) in the same order.
template <int E, int H, int ZP, int YP, int NW, class F>
__device__ inline void for_type_rows_k(int z0, int hs, int Ey, int wave, int lane, F f) {
  using S = SlabShape<E>;
  constexpr int KT = type_tasks_per_wave<E, H, NW>();
  const int nz = (hs - ZP + 1) >> 1;
  const int ntask = nz * S::G;
  const int r = lane / S::P, q = lane % S::P;
  if (r >= S::RW) return;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int t = wave + k * NW;
    if (t < ntask) {
      const int iz = t / S::G, g = t - iz * S::G;
      const int lz = z0 + ZP + 2 * iz;
      const int lyu = YP + 2 * g * S::RW;
      const int ly = lyu + 2 * r;
      if (ly < Ey) f(k, lz, ly, q, lyu);
    }
  }
}

}  // namespace
}  // namespace dev
}  // namespace stz
