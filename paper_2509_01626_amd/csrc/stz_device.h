// Device-side helpers shared by the library's kernels: unit geometry, grid
// indexing, the prediction stencils (format section 2.2) and the quantizer
// (format section 2.3), wave-level reductions.
#pragma once

#include "stz_internal.h"

namespace stz {

void prof_begin(hipStream_t st, const char* name, int level);
void prof_end(hipStream_t st);

namespace dev {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Geometry helpers
// ---------------------------------------------------------------------------
struct UnitGeo {
  int64_t b[3];
  int o[3];
  int32_t M[3];
};

__device__ inline UnitGeo unit_geo(const Geo& g, int64_t u, int logs) {
  UnitGeo r;
  const int64_t blk = u / 7;
  const int c = int(u - blk * 7) + 1;
  r.b[2] = blk % g.nb[2];
  const int64_t t = blk / g.nb[2];
  r.b[1] = t % g.nb[1];
  r.b[0] = t / g.nb[1];
  r.o[0] = (c >> 2) & 1;
  r.o[1] = (c >> 1) & 1;
  r.o[2] = c & 1;
  const int64_t s = int64_t(1) << logs;
  for (int d = 0; d < 3; ++d) {
    const int64_t lo = r.b[d] << g.logB;
    const int64_t len = min(int64_t(g.B), g.n[d] - lo);
    const int32_t U = int32_t((len + s - 1) >> logs);
    r.M[d] = r.o[d] ? (U >> 1) : ((U + 1) >> 1);
  }
  return r;
}

__device__ inline int64_t gidx(const Grid& g, int64_t z, int64_t y, int64_t x) {
  return (((z - g.first[0]) >> g.logs) * g.cnt[1] + ((y - g.first[1]) >> g.logs)) * g.cnt[2] +
         ((x - g.first[2]) >> g.logs);
}

// ---------------------------------------------------------------------------
// Prediction (format 2.2). `at(z, y, x)` returns the reconstructed coarse
// value at an absolute coordinate.
// ---------------------------------------------------------------------------
template <class G>
__device__ inline float axis_rule(bool p1, bool m3, int64_t s, G f) {
  if (p1) {
    const float lo = f(-s);
    const float hi = f(s);
    return (lo + hi) * 0.5f;
  }
  if (m3) {
    const float lo = f(-s);
    const float lo3 = f(-3 * s);
    return ((3.0f * lo) - lo3) * 0.5f;
  }
  return f(-s);
}

template <class F>
__device__ inline float predict_point(const int64_t p[3], int logs, const int64_t n[3],
                                      const int o[3], F at) {
  const int64_t s = int64_t(1) << logs;
  int D[3] = {0, 0, 0};
  int nd = 0;
  for (int d = 0; d < 3; ++d)
    if (o[d]) D[nd++] = d;
  bool P1[3], M3[3], P3[3];
  bool full = true;
  for (int i = 0; i < nd; ++i) {
    const int d = D[i];
    P1[i] = p[d] + s <= n[d] - 1;
    M3[i] = p[d] >= 3 * s;
    P3[i] = p[d] + 3 * s <= n[d] - 1;
    full = full && P1[i] && M3[i] && P3[i];
  }
  auto off = [&](int64_t a, int64_t b, int64_t c) {
    int64_t q[3] = {p[0], p[1], p[2]};
    q[D[0]] += a;
    if (nd > 1) q[D[1]] += b;
    if (nd > 2) q[D[2]] += c;
    return at(q[0], q[1], q[2]);
  };
  if (nd == 1) {
    if (P1[0]) {
      const float Bv = off(-s, 0, 0);
      const float Cv = off(s, 0, 0);
      if (M3[0] && P3[0]) {
        const float A = off(-3 * s, 0, 0);
        const float Dv = off(3 * s, 0, 0);
        return ((9.0f * (Bv + Cv)) - (A + Dv)) * 0.0625f;
      }
      if (P3[0]) {
        const float Dv = off(3 * s, 0, 0);
        return ((3.0f * Bv + 6.0f * Cv) - Dv) * 0.125f;
      }
      if (M3[0]) {
        const float A = off(-3 * s, 0, 0);
        return ((6.0f * Bv + 3.0f * Cv) - A) * 0.125f;
      }
      return (Bv + Cv) * 0.5f;
    }
    const float Bv = off(-s, 0, 0);
    if (M3[0]) {
      const float A = off(-3 * s, 0, 0);
      return ((3.0f * Bv) - A) * 0.5f;
    }
    return Bv;
  }
  if (full) {
    float in = 0.0f, out = 0.0f;
    if (nd == 2) {
      in = off(-s, -s, 0);
      in = in + off(-s, s, 0);
      in = in + off(s, -s, 0);
      in = in + off(s, s, 0);
      out = off(-3 * s, -3 * s, 0);
      out = out + off(-3 * s, 3 * s, 0);
      out = out + off(3 * s, -3 * s, 0);
      out = out + off(3 * s, 3 * s, 0);
      return ((9.0f * in) - out) * 0.03125f;
    }
    bool first = true;
    for (int a = -1; a <= 1; a += 2)
      for (int b = -1; b <= 1; b += 2)
        for (int c = -1; c <= 1; c += 2) {
          const float vi = off(a * s, b * s, c * s);
          const float vo = off(3 * a * s, 3 * b * s, 3 * c * s);
          if (first) {
            in = vi;
            out = vo;
            first = false;
          } else {
            in = in + vi;
            out = out + vo;
          }
        }
    return ((9.0f * in) - out) * 0.015625f;
  }
  if (nd == 2) {
    return axis_rule(P1[0], M3[0], s, [&](int64_t a) {
      return axis_rule(P1[1], M3[1], s, [&](int64_t b) { return off(a, b, 0); });
    });
  }
  return axis_rule(P1[0], M3[0], s, [&](int64_t a) {
    return axis_rule(P1[1], M3[1], s, [&](int64_t b) {
      return axis_rule(P1[2], M3[2], s, [&](int64_t c) { return off(a, b, c); });
    });
  });
}

// Linear-scaling quantization (format 2.3). Returns the symbol (0 = outlier).
__device__ inline int quantize(float xv, float pred, float E2, float INV, double e, int R,
                               float* rec) {
  const float diff = xv - pred;
  const float t = rintf(diff * INV);
  if (fabsf(t) <= (float)(R - 1)) {
    const int q = (int)t;
    const float prod = (float)q * E2;
    const float xr = pred + prod;
    if (fabs((double)xv - (double)xr) <= e) {
      *rec = xr;
      return q + R;
    }
  }
  *rec = xv;
  return 0;
}

__device__ inline uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline uint32_t wave_excl_scan(uint32_t v, int lane) {
  uint32_t inc = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += t;
  }
  return inc - v;
}


inline int grid_for(uint64_t n, int per_block, int cap) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > uint64_t(cap)) b = cap;
  return int(b);
}

// Copy of a work-group-uniform argument block into scalar registers: each
// 32-bit word is loaded and broadcast from the first lane, so the compiler
// keeps the fields in SGPRs as it does for kernel arguments.
template <class T>
__device__ inline T uniform_load(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "argument blocks are whole words");
  T v;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(p);
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < int(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
  return v;
}

__host__ __device__ inline Grid full_grid(const Geo& g, int logs) {
  Grid r;
  for (int d = 0; d < 3; ++d) {
    r.first[d] = 0;
    r.cnt[d] = ((g.n[d] - 1) >> logs) + 1;
  }
  r.logs = logs;
  return r;
}

__host__ __device__ inline Grid box_grid(const Box& b, int logs) {
  Grid r;
  const int64_t s = int64_t(1) << logs;
  for (int d = 0; d < 3; ++d) {
    r.first[d] = (b.lo[d] + s - 1) >> logs << logs;
    r.cnt[d] = r.first[d] < b.hi[d] ? ((b.hi[d] - 1 - r.first[d]) >> logs) + 1 : 0;
  }
  r.logs = logs;
  return r;
}


// Copy the coarser grid's points (G_{l-1}) into level l's grid, inside box.
__global__ void k_upcopy(const float* __restrict__ src, Grid gs, float* __restrict__ dst, Grid gd) {
  // Points of the stride-2s grid inside gd's box.
  const int64_t s2 = int64_t(1) << gs.logs;
  int64_t f[3], c[3];
  for (int d = 0; d < 3; ++d) {
    const int64_t lo = gd.first[d];
    const int64_t hi = gd.first[d] + ((gd.cnt[d] - 1) << gd.logs) + 1;
    f[d] = (lo + s2 - 1) / s2 * s2;
    c[d] = f[d] < hi ? (hi - 1 - f[d]) / s2 + 1 : 0;
  }
  const int64_t n = c[0] * c[1] * c[2];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t ix = i % c[2], t = i / c[2], iy = t % c[1], iz = t / c[1];
    const int64_t z = f[0] + iz * s2, y = f[1] + iy * s2, x = f[2] + ix * s2;
    dst[gidx(gd, z, y, x)] = src[gidx(gs, z, y, x)];
  }
}

}  // namespace
}  // namespace dev
}  // namespace stz
