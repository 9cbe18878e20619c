// Device-side helpers shared by the library's kernels: unit geometry, grid
// indexing, the quantizer (format section 2.3), wave-level reductions.
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

// Linear-scaling quantization (format 2.3). Returns the symbol (0 = outlier).
// float32 values: the acceptance test |x - x'| <= e is evaluated exactly in
// double. float64 values: the test takes the rounded double difference
// against chk = e * (1 - 2^-50), which implies the exact |x - x'| <= e.
template <class T>
__device__ inline T rint_t(T v) {
  if constexpr (sizeof(T) == 4)
    return rintf(v);
  else
    return rint(v);
}
template <class T>
__device__ inline T fabs_t(T v) {
  if constexpr (sizeof(T) == 4)
    return fabsf(v);
  else
    return fabs(v);
}

// Every step is evaluated on every lane and the outcome selected, with no
// branches: the same operands and order as the per-case form, so the same
// symbols and reconstructions.
template <class T>
__device__ inline int quantize(T xv, T pred, T E2, T INV, double chk, int R, T* rec) {
  const T diff = xv - pred;
  const T t = rint_t(diff * INV);
  const bool inr = fabs_t(t) <= (T)(R - 1);
  const int q = inr ? (int)t : 0;
  const T prod = (T)q * E2;
  const T xr = pred + prod;
  bool ok;
  if constexpr (sizeof(T) == 4)
    ok = inr && fabs((double)xv - (double)xr) <= chk;
  else
    ok = inr && fabs(xv - xr) <= chk;
  *rec = ok ? xr : xv;
  return ok ? q + R : 0;
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


}  // namespace
}  // namespace dev
}  // namespace stz
