// Compression kernels (gfx950): range reduction and error-bound resolution,
// anchors, per-level predict+quantize (Sec. 3.1, Eqs. 3-8, Optimizations 3
// and 5) with the code histogram, per-lane code lengths, segmented scans for
// the stream layout, bit packing and outlier compaction.
#include <algorithm>
#include <cstring>

#include "stz_slab.h"

namespace stz {
using namespace dev;
namespace {

// ---------------------------------------------------------------------------
// Compression kernels
// ---------------------------------------------------------------------------
// Every kernel is a device body run by one work-group (`wg` of `ngrid` for
// grid-stride bodies) plus a plain launch; the batched launches run the same
// bodies over a work map of many jobs.
__device__ inline void init_body(DevParams* P) {
  if (threadIdx.x == 0) {
    P->flags = 0;
    P->total = 0;
  }
}

// Clear the partial histograms (n words), grid-stride.
__device__ inline void hzero_body(uint32_t* hpart, uint64_t n, uint64_t wg, uint64_t ngrid) {
  const uint64_t n4 = n >> 2;
  uint4* p4 = reinterpret_cast<uint4*>(hpart);
  for (uint64_t i = wg * blockDim.x + threadIdx.x; i < n4; i += ngrid * blockDim.x)
    p4[i] = make_uint4(0, 0, 0, 0);
  for (uint64_t i = (n4 << 2) + wg * blockDim.x + threadIdx.x; i < n; i += ngrid * blockDim.x)
    hpart[i] = 0;
}

// The call's device parameters initialized (work-group 0) and the partial
// histograms cleared.
__global__ void k_init_hzero(DevParams* P, uint32_t* hpart, uint64_t n) {
  if (blockIdx.x == 0) init_body(P);
  hzero_body(hpart, n, blockIdx.x, gridDim.x);
}

// hist[bin] = sum over the slots; work-group `wg` covers 256 bins.
__device__ inline void hred_body(const uint32_t* hpart, uint32_t nslots, int nsym,
                                 unsigned long long* hist, int wg) {
  const int bin = wg * 256 + int(threadIdx.x);
  if (bin >= nsym) return;
  // 32 independent loads in flight per round (the slots are few and the
  // loads latency-bound)
  unsigned long long v = 0;
  uint32_t s = 0;
  for (; s + 32 <= nslots; s += 32) {
    uint32_t w[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) w[k] = hpart[uint64_t(s + k) * nsym + bin];
#pragma unroll
    for (int k = 0; k < 32; ++k) v += w[k];
  }
  for (; s < nslots; ++s) v += hpart[uint64_t(s) * nsym + bin];
  hist[bin] = v;
}

__global__ __launch_bounds__(256) void k_hred(const uint32_t* hpart, uint32_t nslots, int nsym,
                                              unsigned long long* hist) {
  hred_body(hpart, nslots, nsym, hist, blockIdx.x);
}

template <class T>
__device__ inline T vmin(T a, T b) {
  if constexpr (sizeof(T) == 4)
    return fminf(a, b);
  else
    return fmin(a, b);
}
template <class T>
__device__ inline T vmax(T a, T b) {
  if constexpr (sizeof(T) == 4)
    return fmaxf(a, b);
  else
    return fmax(a, b);
}

// Min, max and finiteness of the field: 16-byte loads (4 floats or 2
// doubles) over the aligned part, scalar loads for the rest.
template <class T>
__device__ inline void minmax_body(const T* __restrict__ x, uint64_t N, MinMax<T>* part,
                                   DevParams* P, uint64_t wg, uint64_t ngrid) {
  T mn = T(INFINITY), mx = T(-INFINITY);
  bool bad = false;
  const uint64_t stride = ngrid * blockDim.x;
  const uint64_t t0 = wg * blockDim.x + threadIdx.x;
  uint64_t head = 0;  // elements handled by 16-byte loads
  if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    if constexpr (sizeof(T) == 4) {
      head = N & ~uint64_t(3);
      const float4* x4 = reinterpret_cast<const float4*>(x);
      for (uint64_t i = t0; i < (head >> 2); i += stride) {
        const float4 v = x4[i];
        bad |= !isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w);
        mn = fminf(fminf(mn, v.x), fminf(v.y, fminf(v.z, v.w)));
        mx = fmaxf(fmaxf(mx, v.x), fmaxf(v.y, fmaxf(v.z, v.w)));
      }
    } else {
      head = N & ~uint64_t(1);
      const double2* x2 = reinterpret_cast<const double2*>(x);
      for (uint64_t i = t0; i < (head >> 1); i += stride) {
        const double2 v = x2[i];
        bad |= !isfinite(v.x) || !isfinite(v.y);
        mn = fmin(mn, fmin(v.x, v.y));
        mx = fmax(mx, fmax(v.x, v.y));
      }
    }
  }
  for (uint64_t i = head + t0; i < N; i += stride) {
    const T v = x[i];
    bad |= !isfinite(v);
    mn = vmin(mn, v);
    mx = vmax(mx, v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = vmin(mn, __shfl_xor(mn, o, kWave));
    mx = vmax(mx, __shfl_xor(mx, o, kWave));
  }
  __shared__ T smn[4], smx[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smn[w] = mn;
    smx[w] = mx;
  }
  if (bad) atomicOr(&P->flags, kFlagNonfinite);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mn = vmin(mn, smn[i]);
      mx = vmax(mx, smx[i]);
    }
    part[wg].mn = mn;
    part[wg].mx = mx;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_minmax(const T* __restrict__ x, uint64_t N,
                                                MinMax<T>* part, DevParams* P) {
  minmax_body<T>(x, N, part, P, blockIdx.x, gridDim.x);
}

// Resolve the absolute bound and the per-level constants (format 2.3).
template <class T>
__device__ inline void resolve_body(DevParams* P, const MinMax<T>* part, uint32_t nparts, int mode,
                                    double eb, double ratio, int L) {
  // one wave of 64 threads: min and max of the partials (exact in any order)
  T mn = T(INFINITY), mx = T(-INFINITY);
  if (mode == 1)
    for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) {
      mn = vmin(mn, part[i].mn);
      mx = vmax(mx, part[i].mx);
    }
  for (int o = 32; o > 0; o >>= 1) {
    mn = vmin(mn, __shfl_xor(mn, o, kWave));
    mx = vmax(mx, __shfl_xor(mx, o, kWave));
  }
  if (threadIdx.x != 0) return;
  double eb_abs = eb;
  if (mode == 1) {
    P->mn = mn;
    P->mx = mx;
    const double range = (double)mx - (double)mn;
    if (range > 0.0)
      eb_abs = eb * range;
    else
      eb_abs = eb * (fabs((double)mn) > 0.0 ? fabs((double)mn) : 1.0);
  }
  if (!(eb_abs > 0.0) || !isfinite(eb_abs)) P->flags |= kFlagBadBound;
  P->eb_abs = eb_abs;
  for (int l = 1; l <= L; ++l) {
    double e;
    if (l == L)
      e = eb_abs;
    else if (l == L - 1)
      e = eb_abs / ratio;
    else
      e = (eb_abs / ratio) / ratio;
    P->e[l] = e;
    P->E2[l] = (float)(2.0 * e);
    P->INV[l] = (float)(1.0 / (2.0 * e));
    P->E2d[l] = 2.0 * e;
    P->INVd[l] = 1.0 / (2.0 * e);
    P->echk[l] = e * (1.0 - 0x1p-50);
  }
}

template <class T>
__global__ void k_resolve(DevParams* P, const MinMax<T>* part, uint32_t nparts, int mode,
                          double eb, double ratio, int L) {
  resolve_body<T>(P, part, nparts, mode, eb, ratio, L);
}

// Anchors: the stride-2^L grid, copied verbatim into the level-0 grid.
template <class T>
__device__ inline void anchor_body(const T* __restrict__ x, const Geo& g, T* rec0,
                                   DevParams* P, uint64_t wg, uint64_t ngrid) {
  const int logs = g.L;
  const int64_t c0 = ((g.n[0] - 1) >> logs) + 1, c1 = ((g.n[1] - 1) >> logs) + 1,
                c2 = ((g.n[2] - 1) >> logs) + 1;
  const int64_t na = c0 * c1 * c2;
  bool bad = false;
  for (int64_t i = int64_t(wg) * blockDim.x + threadIdx.x; i < na;
       i += int64_t(ngrid) * blockDim.x) {
    const int64_t ix = i % c2, t = i / c2, iy = t % c1, iz = t / c1;
    const T v = x[((iz << logs) * g.n[1] + (iy << logs)) * g.n[2] + (ix << logs)];
    bad |= !isfinite(v);
    rec0[i] = v;
  }
  if (bad) atomicOr(&P->flags, kFlagNonfinite);
}

template <class T>
__global__ void k_anchor(const T* __restrict__ x, Geo g, T* rec0, DevParams* P) {
  anchor_body<T>(x, g, rec0, P, blockIdx.x, gridDim.x);
}

struct PredSlabArgs {
  const void* x;     // field values (value type of the kernel)
  Geo g;
  int level, logs;
  int64_t n[3];      // level grid extents
  int64_t nc[3];     // previous level's grid extents
  const void* prev;  // level-(l-1) grid, complete
  void* cur;         // level-l grid; null at the finest level
  uint16_t* sym;
  DevParams* P;
  uint32_t* hpart;   // [nsym][nslots] partial histograms
  uint32_t nslots;
  int nsym;
};

// Per-slab state for predicting rows of one parity type (T = value type).
template <class T>
struct PredRows {
  const T* x;
  const T* tile;
  uint16_t* ssym;
  uint32_t* h;
  T* cur;
  int64_t oz, oy, ox;
  int z0, Ex, ls;
  int64_t n[3], fn[3];
  T E2, INV;
  double chk;  // acceptance bound of the quantizer
  int R;
};

// Magnitude bits of a value's top 32-bit word: infinities and NaNs have the
// largest, so the running maximum over a block tells whether any value was
// not finite (two vector instructions per point, no lane-mask bookkeeping).
__device__ inline uint32_t mag_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }
__device__ inline uint32_t mag_bits(double v) {
  return uint32_t(uint64_t(__double_as_longlong(v)) >> 32) & 0x7fffffffu;
}
template <class T>
constexpr uint32_t kMagNonfinite = sizeof(T) == 4 ? 0x7f800000u : 0x7ff00000u;

// Predict and quantize one point of class C (0 = coarse copy only).
template <class T, int E, int H, int C, bool INT>
__device__ inline void pred_point(const PredRows<T>& c, int lz, int ly, int lx, int srow,
                                  const T xv, T* grow, const int64_t p[3],
                                  uint32_t* n_center, uint32_t* mag) {
  using S = SlabShape<E, H>;
  if constexpr (C == 0) {
    if (grow) grow[lx] = c.tile[((((lz - c.z0) >> 1) + 1) * S::T + (ly >> 1) + 1) * S::TP + (lx >> 1) + 1];
  } else {
    *mag = max(*mag, mag_bits(xv));
    const T pred = tile_pred<T, E, C, INT>(c.tile, lz - c.z0, ly, lx, p, c.n);
    T rv;
    const int sy = quantize<T>(xv, pred, c.E2, c.INV, c.chk, c.R, &rv);
    c.ssym[(C - 1) * S::SCP + srow] = uint16_t(sy);
    if (grow) grow[lx] = rv;
    *n_center += sy == c.R ? 1u : 0u;
    if (sy != c.R) atomicAdd(&c.h[sy], 1u);
  }
}

// The field values of this wave's rows of parity type (ZP, YP) in the slab
// at z0: xs[k] = the (even x, odd x) pair of the wave's k-th row (the even
// one is not needed for type (0, 0), whose even-x points are coarse copies).
// Loaded for the next slab while the current one finishes.
template <class T, int E, int H, int NW, int ZP, int YP, int KT>
__device__ inline void pred_fetch_x(const PredRows<T>& c, int z0, int hs, int Ey, int wave,
                                    int lane, T (&xs)[KT][2]) {
  for_type_rows_k<E, H, ZP, YP, NW>(z0, hs, Ey, wave, lane, [&](int k, int lz, int ly, int q, int) {
    const T* xrow =
        c.x + ((((c.oz + lz) << c.ls) * c.fn[1]) + ((c.oy + ly) << c.ls)) * c.fn[2] + (c.ox << c.ls);
    const int l0 = 2 * q, l1 = 2 * q + 1;
    if constexpr (ZP != 0 || YP != 0) xs[k][0] = l0 < c.Ex ? xrow[l0 << c.ls] : T(0);
    xs[k][1] = l1 < c.Ex ? xrow[l1 << c.ls] : T(0);
  });
}

// This wave's rows of parity type (ZP, YP); classes fixed at compile time.
// PRE: xs = the rows' field values (pred_fetch_x); else they are loaded here.
// OUT: the level grid may be written (c.cur, when not null); without it (the
// finest level) no grid addresses are formed at all.
template <class T, int E, int H, int NW, int ZP, int YP, bool INT, bool PRE, bool OUT, int KT>
__device__ inline void pred_type(const PredRows<T>& c, int hs, int Ey, int wave, int lane,
                                 const T (&xs)[KT][2], uint32_t* n_center, uint32_t* mag) {
  using S = SlabShape<E, H>;
  constexpr int m = S::m;
  constexpr int C0 = 4 * ZP + 2 * YP;
  auto row = [&](int k, int lz, int ly, int q) {
    T* grow = nullptr;
    if constexpr (OUT)
      grow = c.cur ? c.cur + ((c.oz + lz) * c.n[1] + (c.oy + ly)) * c.n[2] + c.ox : nullptr;
    const int srow = (((lz - c.z0) >> 1) * m + (ly >> 1)) * S::SP + q;
    const int l0 = 2 * q, l1 = 2 * q + 1;
    const int64_t p0[3] = {c.oz + lz, c.oy + ly, c.ox + l0};
    const int64_t p1[3] = {c.oz + lz, c.oy + ly, c.ox + l1};
    T x0, x1;
    if constexpr (PRE) {
      x0 = xs[k][0];
      x1 = xs[k][1];
    } else {
      const T* xrow = c.x + ((((c.oz + lz) << c.ls) * c.fn[1]) + ((c.oy + ly) << c.ls)) * c.fn[2] +
                      (c.ox << c.ls);
      x0 = (C0 != 0 && l0 < c.Ex) ? xrow[l0 << c.ls] : T(0);
      x1 = l1 < c.Ex ? xrow[l1 << c.ls] : T(0);
    }
    if (l0 < c.Ex) pred_point<T, E, H, C0, INT>(c, lz, ly, l0, srow, x0, grow, p0, n_center, mag);
    if (l1 < c.Ex)
      pred_point<T, E, H, C0 + 1, INT>(c, lz, ly, l1, srow, x1, grow, p1, n_center, mag);
  };
  if constexpr (PRE)
    for_type_rows_k<E, H, ZP, YP, NW>(c.z0, hs, Ey, wave, lane,
                                      [&](int k, int lz, int ly, int q, int) { row(k, lz, ly, q); });
  else
    for_type_rows<E, ZP, YP, NW>(c.z0, hs, Ey, wave, lane,
                                 [&](int lz, int ly, int q, int) { row(0, lz, ly, q); });
}

// Predict and quantize every level-l point of one block (format 2.2, 2.3);
// also writes the block's part of the level-l grid (coarse points copied,
// level points reconstructed) for the next level's prediction.
// NT = threads of the work-group (256, or 64 for small blocks). OUT = false:
// the finest level, whose grid is not written (a.cur is null). KIND: 0 = any
// block (interior test at run time), 1 = interior blocks only, 2 = the other
// blocks only; a kernel built for one kind holds only that kind's code.
// `slot` = the partial histogram the block adds into.
template <class T, int E, int H, int NT = 256, bool OUT = true, int KIND = 0>
__device__ inline void pred_body(const PredSlabArgs& a, int64_t blk, uint64_t slot) {
  using S = SlabShape<E, H>;
  constexpr int m = S::m;
  constexpr int NW = NT / 64;
  __shared__ uint32_t h[kMaxAlphabet];
  __shared__ T tile[S::TILE];
  __shared__ uint16_t ssym[7 * S::SCP];  // slab symbols, [class][v_z][v_y][v_x] (padded)
  __shared__ uint64_t ubase[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Blocks of at most 4^3 level points (at most 56 symbols) add their symbol
  // counts straight into their partial histogram; larger ones count in LDS
  // and add the block's histogram once.
  constexpr bool kGH = E <= 4;
  const uint64_t hs0 = (slot % a.nslots) * uint64_t(a.nsym);
  if constexpr (!kGH)
    for (int i = tid; i < a.nsym; i += blockDim.x) h[i] = 0;
  const int64_t bx = blk % a.g.nb[2], by = (blk / a.g.nb[2]) % a.g.nb[1],
                bz = blk / (a.g.nb[2] * a.g.nb[1]);
  const int64_t oz = bz * E, oy = by * E, ox = bx * E;
  const int Ez = int(min<int64_t>(E, a.n[0] - oz)), Ey = int(min<int64_t>(E, a.n[1] - oy)),
            Ex = int(min<int64_t>(E, a.n[2] - ox));
  if (tid >= 1 && tid <= 7) ubase[tid] = uint64_t(unit_sym_off(a.g, a.logs, blk * 7 + tid - 1));
  T E2, INV;
  double chk;
  if constexpr (sizeof(T) == 4) {
    E2 = a.P->E2[a.level];
    INV = a.P->INV[a.level];
    chk = a.P->e[a.level];
  } else {
    E2 = a.P->E2d[a.level];
    INV = a.P->INVd[a.level];
    chk = a.P->echk[a.level];
  }
  const T* xv = static_cast<const T*>(a.x);
  const T* prev = static_cast<const T*>(a.prev);
  T* cur = static_cast<T*>(a.cur);
  const int R = a.g.R;
  const int64_t sf[3] = {0, 0, 0};
  const int ls = a.logs;
  const int64_t org[3] = {oz, oy, ox};
  const bool interior = KIND == 1 ? true : KIND == 2 ? false : block_interior(org, E, a.n);
  uint32_t n_center = 0;  // the zero-residual symbol is counted in a register
  uint32_t n_zero = 0, n_cover = 0;  // zero chunks found, centre symbols they cover
  uint32_t mag = 0;  // largest magnitude bits of the block's field values
  // Blocks walked in several slabs slide their window of coarse planes
  // between slabs (once the slab's predictions are done) instead of loading
  // every slab's whole tile: each slab adds HZ of its TZ planes.
  constexpr bool kSlide = S::H < E;
  const int64_t cz00 = (oz - 2) >> 1, cy0 = (oy - 2) >> 1, cx0 = (ox - 2) >> 1;
  if constexpr (kSlide) load_tile<S, T>(tile, prev, sf, a.nc, cz00, cy0, cx0);
  PredRows<T> ctx;
  ctx.x = xv;
  ctx.tile = tile;
  ctx.ssym = ssym;
  ctx.h = kGH ? a.hpart + hs0 : h;
  ctx.cur = cur;
  ctx.oz = oz;
  ctx.oy = oy;
  ctx.ox = ox;
  ctx.Ex = Ex;
  ctx.ls = ls;
  for (int d = 0; d < 3; ++d) {
    ctx.n[d] = a.n[d];
    ctx.fn[d] = a.g.n[d];
  }
  ctx.E2 = E2;
  ctx.INV = INV;
  ctx.chk = chk;
  ctx.R = R;
  // Field values of the thread's points, per parity type: for float fields
  // in 16^3 and 32^3 blocks loaded for the next slab while the current one
  // finishes (16 registers); other blocks load them where they are used.
  constexpr bool kPre = sizeof(T) == 4 && (E == 16 || E == 32);
  constexpr int KT = kPre ? type_tasks_per_wave<E, H, NW>() : 1;
  T x00[KT][2], x01[KT][2], x10[KT][2], x11[KT][2];
  auto fetch_x = [&](int zs) {
    if constexpr (kPre) {
      const int hn = min(S::H, Ez - zs);
      pred_fetch_x<T, E, H, NW, 0, 0>(ctx, zs, hn, Ey, wave, lane, x00);
      pred_fetch_x<T, E, H, NW, 0, 1>(ctx, zs, hn, Ey, wave, lane, x01);
      pred_fetch_x<T, E, H, NW, 1, 0>(ctx, zs, hn, Ey, wave, lane, x10);
      pred_fetch_x<T, E, H, NW, 1, 1>(ctx, zs, hn, Ey, wave, lane, x11);
    }
  };
  fetch_x(0);
  for (int z0 = 0; z0 < Ez; z0 += S::H) {
    if constexpr (!kSlide) load_tile<S, T>(tile, prev, sf, a.nc, cz00 + (z0 >> 1), cy0, cx0);
    __syncthreads();
    const int hs = min(S::H, Ez - z0);
    ctx.z0 = z0;
    if (interior) {
      pred_type<T, E, H, NW, 0, 0, true, kPre, OUT>(ctx, hs, Ey, wave, lane, x00, &n_center, &mag);
      pred_type<T, E, H, NW, 0, 1, true, kPre, OUT>(ctx, hs, Ey, wave, lane, x01, &n_center, &mag);
      pred_type<T, E, H, NW, 1, 0, true, kPre, OUT>(ctx, hs, Ey, wave, lane, x10, &n_center, &mag);
      pred_type<T, E, H, NW, 1, 1, true, kPre, OUT>(ctx, hs, Ey, wave, lane, x11, &n_center, &mag);
    } else {
      pred_type<T, E, H, NW, 0, 0, false, kPre, OUT>(ctx, hs, Ey, wave, lane, x00, &n_center, &mag);
      pred_type<T, E, H, NW, 0, 1, false, kPre, OUT>(ctx, hs, Ey, wave, lane, x01, &n_center, &mag);
      pred_type<T, E, H, NW, 1, 0, false, kPre, OUT>(ctx, hs, Ey, wave, lane, x10, &n_center, &mag);
      pred_type<T, E, H, NW, 1, 1, false, kPre, OUT>(ctx, hs, Ey, wave, lane, x11, &n_center, &mag);
    }
    if (z0 + S::H < Ez) fetch_x(z0 + S::H);
    __syncthreads();
    const int a0 = z0 >> 1;
    if constexpr (kSlide)
      if (z0 + S::H < Ez)
        slide_window<S, T, NT>(tile, prev, sf, a.nc, cz00 + a0 + S::TZ, cy0, cx0, tid);
    // Zero chunks (format 2.4): a chunk is the M_y symbols of one (class,
    // v_z, v_x); one whose symbols are all R becomes one token Z, so the
    // histogram counts Z once and those symbols not at all. Slabs hold whole
    // v_z rows, so every chunk lies in one slab.
    if (a.g.Z >= 0) {
      for (int i = tid; i < 7 * S::HZ * m; i += blockDim.x) {
        const int c = i / (S::HZ * m) + 1, rr = i - (c - 1) * (S::HZ * m);
        const int vzl = rr / m, j = rr - vzl * m;
        const int Mz = (c >> 2) & 1 ? Ez >> 1 : (Ez + 1) >> 1;
        const int My = (c >> 1) & 1 ? Ey >> 1 : (Ey + 1) >> 1;
        const int Mx = c & 1 ? Ex >> 1 : (Ex + 1) >> 1;
        if (a0 + vzl >= Mz || j >= Mx || My == 0) continue;
        const uint16_t* q = ssym + (c - 1) * S::SCP + (vzl * m) * S::SP + j;
        bool all = true;
#pragma unroll
        for (int vy = 0; vy < m; ++vy)
          if (vy < My) all &= q[vy * S::SP] == uint16_t(R);
        if (all) {
          ++n_zero;
          n_cover += uint32_t(My);
        }
      }
    }
    // The slab's rows of every unit, column-major inside the unit: column j of
    // a unit with M_z*M_y rows starts at unit base + j*M_z*M_y, so this slab's
    // part of each column is one contiguous run.
    for (int c = 1; c <= 7; ++c) {
      const int oz_ = (c >> 2) & 1, oy_ = (c >> 1) & 1, ox_ = c & 1;
      const int Mz = oz_ ? Ez >> 1 : (Ez + 1) >> 1, My = oy_ ? Ey >> 1 : (Ey + 1) >> 1,
                Mx = ox_ ? Ex >> 1 : (Ex + 1) >> 1;
      const int rz = min(a0 + S::HZ, Mz) - a0;
      if (rz <= 0) continue;
      const int run = rz * My;  // contiguous symbols per column in this slab
      const int cnt = run * Mx;
      uint16_t* dst = a.sym + ubase[c] + uint64_t(a0 * My);
      const uint64_t cstride = uint64_t(Mz * My);
      if (Ey == E && rz == S::HZ) {  // full extents: powers of two
        constexpr int LMY = __builtin_ctz(m), LRUN = __builtin_ctz(S::HZ * m);
        for (int i = tid; i < cnt; i += blockDim.x) {
          const int j = i >> LRUN, t = i & ((1 << LRUN) - 1);
          const int vz = t >> LMY, vy = t & (m - 1);
          dst[uint64_t(j) * cstride + t] = ssym[(c - 1) * S::SCP + (vz * m + vy) * S::SP + j];
        }
      } else {
        for (int i = tid; i < cnt; i += blockDim.x) {
          const int j = i / run, t = i - j * run;
          const int vz = t / My, vy = t - vz * My;
          dst[uint64_t(j) * cstride + t] = ssym[(c - 1) * S::SCP + (vz * m + vy) * S::SP + j];
        }
      }
    }
    __syncthreads();
  }
  if constexpr (kGH) {
    // the centre and zero-chunk counts summed over each wave's lanes
    const uint32_t dc = wave_sum(n_center - n_cover), dz = wave_sum(n_zero);  // mod 2^32
    if (lane == 0) {
      if (dc) atomicAdd(&a.hpart[hs0 + R], dc);
      if (dz) atomicAdd(&a.hpart[hs0 + a.g.Z], dz);
    }
    if (mag >= kMagNonfinite<T>) atomicOr(&a.P->flags, kFlagNonfinite);
  } else {
    if (n_center != n_cover) atomicAdd(&h[R], n_center - n_cover);  // mod 2^32, sums >= 0
    if (n_zero) atomicAdd(&h[a.g.Z], n_zero);
    __syncthreads();
    if (mag >= kMagNonfinite<T>) atomicOr(&a.P->flags, kFlagNonfinite);
    for (int i = tid; i < a.nsym; i += blockDim.x)
      if (h[i]) atomicAdd(&a.hpart[hs0 + i], h[i]);
  }
}

// Slab height of the plain predictor launches: 4 planes for 32^3-point blocks
// (24 KB of LDS, six work-groups per CU against four with 8 planes).
constexpr int pred_slab_h(int E) { return E == 32 ? 4 : default_slab_h(E); }

// Threads per work-group of the plain launches: blocks of at most 4^3 level
// points take one wave, so that four times as many fit on a CU (8^3 blocks
// are faster with four waves sharing the block's points).
constexpr int pred_threads(int E) { return E <= 4 ? 64 : 256; }

// Waves per SIMD the predictor is compiled for: the occupancy its LDS
// allows for float fields (6 work-groups per CU for 32^3-point blocks, 7 for
// 16^3), so the registers holding the next slab's field values do not cost
// resident blocks.
template <class T>
constexpr int pred_waves(int E) { return sizeof(T) != 4 ? 1 : (E == 32 ? 6 : (E == 16 ? 7 : 1)); }

// Plain launches: KIND 1 walks the interior box of blocks, KIND 2 the shell
// of the others, KIND 0 every block (with an empty box, the shell is all of
// them); work-groups take contiguous runs per XCD (wg_block).
template <class T, int E, bool OUT, int KIND>
__global__ __launch_bounds__(pred_threads(E)) __attribute__((amdgpu_waves_per_eu(pred_waves<T>(E))))
void k_pred_slab(PredSlabArgs a, BlockSplit bs) {
  const int64_t nI = box_count(bs);
  int64_t blk;
  if constexpr (KIND == 1) {
    blk = box_block(bs, wg_block(blockIdx.x, nI, true));
  } else {
    const int64_t nS = bs.nb[0] * bs.nb[1] * bs.nb[2] - nI;
    blk = shell_block(bs, wg_block(blockIdx.x, nS, true));
  }
  pred_body<T, E, pred_slab_h(E), pred_threads(E), OUT, KIND>(a, blk, blockIdx.x);
}

struct LaneLenArgs {
  Geo g;
  int logs;
  const uint16_t* sym;
  uint64_t nu;
  const uint8_t* lens;
  int nsym;
  uint16_t* lane_len;  // this level's lanes
  uint32_t* cnt_words;
  uint32_t* cnt_outl;
};

// Bit length of every lane stream and per-unit totals. One work-group per
// block: thread t < 7m owns column j = t mod m of the block's class t/m + 1.
// With zero chunks, a chunk (M_y consecutive rows of the column) whose
// symbols are all R costs the token Z's code instead.
// Full blocks of 32^3 level points, every unit's symbols 16-byte aligned:
// all threads read the units' symbols in coalesced 8-symbol groups
// (a lane's rows = TPL consecutive groups, a zero chunk of M_y = CT*8 rows =
// CT groups) and sum each lane's code lengths over its TPL threads.
template <int M>
__device__ inline void lanelen_full(const LaneLenArgs& a, const uint8_t* L, const int64_t* usym,
                                   const int64_t* ulane, uint32_t* ub, uint32_t* uo) {
  constexpr int rows = M * M, TPL = rows / 8, CT = M / 8, NG = rows * M / 8;
  static_assert(TPL <= 64 && (64 % TPL) == 0 && (CT == 1 || CT == 2) && NG % 256 == 0,
                "lane groups");
  const int tid = threadIdx.x;
  const bool zc = a.g.Z >= 0;
  const uint32_t R = uint32_t(a.g.R), LZ = zc ? L[a.g.Z] : 0u;
  for (int c = 1; c <= 7; ++c) {
    const uint4* g4 = reinterpret_cast<const uint4*>(a.sym + usym[c]);
    const int64_t lane0 = ulane[c];
    for (int s8 = tid; s8 < NG; s8 += 256) {  // whole waves take part
      uint32_t cb = 0, co = 0;
      bool all = true;
      {
        const uint4 w = g4[s8];
        const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t s0 = v[k] & 0xFFFFu, s1 = v[k] >> 16;
          cb += L[s0] + L[s1];
          co += (s0 == 0) + (s1 == 0);
          all = all && s0 == R && s1 == R;
        }
      }
      uint32_t bits = cb;
      if (zc) {
        if constexpr (CT == 1) {
          bits = all ? LZ : cb;
        } else {
          const bool pair = __shfl_xor(int(all), 1, kWave) != 0;  // every lane shuffles
          bits = (all && pair) ? ((s8 & 1) == 0 ? LZ : 0u) : cb;
        }
      }
#pragma unroll
      for (int o = 1; o < TPL; o <<= 1) {
        bits += __shfl_xor(bits, o, kWave);
        co += __shfl_xor(co, o, kWave);
      }
      if ((s8 % TPL) == 0) {
        a.lane_len[lane0 + s8 / TPL] = uint16_t(bits);
        atomicAdd(&ub[c], bits);
        atomicAdd(&uo[c], co);
      }
    }
  }
}

// Full blocks of 16^3 level points (units of 512 symbols, lanes of 64 rows,
// chunks of 8): the 7 units and their lanes are consecutive, so the block's
// 448 groups of 8 symbols are taken as one array, 8 groups per lane.
__device__ inline void lanelen_block16(const LaneLenArgs& a, const uint8_t* L, int64_t usym1,
                                       int64_t ulane1, uint32_t* ub, uint32_t* uo) {
  constexpr int TPL = 8, NG = 7 * 64;
  const int tid = threadIdx.x;
  const bool zc = a.g.Z >= 0;
  const uint32_t R = uint32_t(a.g.R), LZ = zc ? L[a.g.Z] : 0u;
  const uint4* g4 = reinterpret_cast<const uint4*>(a.sym + usym1);
  for (int s8 = tid; s8 < 512; s8 += 256) {  // whole waves take part
    uint32_t cb = 0, co = 0;
    bool all = true;
    if (s8 < NG) {
      const uint4 w = g4[s8];
      const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t s0 = v[k] & 0xFFFFu, s1 = v[k] >> 16;
        cb += L[s0] + L[s1];
        co += (s0 == 0) + (s1 == 0);
        all = all && s0 == R && s1 == R;
      }
    }
    uint32_t bits = (zc && all && s8 < NG) ? LZ : cb;
#pragma unroll
    for (int o = 1; o < TPL; o <<= 1) {
      bits += __shfl_xor(bits, o, kWave);
      co += __shfl_xor(co, o, kWave);
    }
    if (s8 < NG && (s8 % TPL) == 0) {
      a.lane_len[ulane1 + s8 / TPL] = uint16_t(bits);
      atomicAdd(&ub[s8 / 64 + 1], bits);
      atomicAdd(&uo[s8 / 64 + 1], co);
    }
  }
}

__device__ inline void lanelen_body(const LaneLenArgs& a, int64_t wg) {
  __shared__ uint8_t L[kMaxAlphabet];
  __shared__ uint32_t bits_s[256], out_s[256];
  __shared__ uint32_t ub[8], uo[8];
  __shared__ int64_t usym[8], ulane[8];
  __shared__ int s_fast;
  const int m = (a.g.B >> a.logs) >> 1;
  // Blocks of 16^3 level points and more copy the code lengths into LDS;
  // smaller ones (at most 16 symbols per lane) read them through the cache.
  if (m >= 8)
    for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) L[i] = a.lens[i];
  const uint8_t* Lt = m >= 8 ? static_cast<const uint8_t*>(L) : a.lens;
  const int tid = threadIdx.x, c = tid / m + 1, j = tid % m;
  if (m == 16 || m == 8) {
    // a full block (every class sub-grid m^3) with aligned unit symbols?
    if (tid == 0) s_fast = 1;
    if (tid < 8) ub[tid] = uo[tid] = 0;
    __syncthreads();
    if (tid < 7) {
      const UnitGeo ug = unit_geo(a.g, wg * 7 + tid, a.logs);
      usym[tid + 1] = unit_sym_off(a.g, a.logs, wg * 7 + tid);
      ulane[tid + 1] = unit_lane_off(a.g, a.logs, wg * 7 + tid);
      if (ug.M[0] != m || ug.M[1] != m || ug.M[2] != m || (usym[tid + 1] & 7) != 0 ||
          (reinterpret_cast<uintptr_t>(a.sym) & 15) != 0)
        s_fast = 0;
    }
    __syncthreads();
    if (s_fast) {
      if (m == 16)
        lanelen_full<16>(a, L, usym, ulane, ub, uo);
      else
        lanelen_block16(a, L, usym[1], ulane[1], ub, uo);
      __syncthreads();
      if (tid < 7) {
        a.cnt_words[wg * 7 + tid] = (ub[tid + 1] + 31) >> 5;
        a.cnt_outl[wg * 7 + tid] = uo[tid + 1];
      }
      return;
    }
  }
  const bool is_lane = tid < 7 * m;
  const int64_t u = wg * 7 + (c - 1);
  uint32_t bits = 0, no = 0;
  int Mx = 0;
  __syncthreads();
  if (is_lane) {
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    const uint32_t rows = uint32_t(ug.M[0]) * ug.M[1];
    Mx = ug.M[2];
    if (j < Mx && a.g.Z >= 0) {
      const uint16_t* col = a.sym + uint64_t(unit_sym_off(a.g, a.logs, u)) + uint64_t(j) * rows;
      const uint32_t My = uint32_t(ug.M[1]), R = uint32_t(a.g.R), LZ = Lt[a.g.Z];
      const bool vec = (reinterpret_cast<uintptr_t>(col) & 15) == 0 && (My & 7) == 0;
      for (uint32_t t0 = 0; t0 < rows; t0 += My) {
        uint32_t cb = 0, co = 0;
        bool all = true;
        if (vec) {
          const uint4* c4 = reinterpret_cast<const uint4*>(col + t0);
          for (uint32_t k8 = 0; k8 < (My >> 3); ++k8) {
            const uint4 w = c4[k8];
            const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const uint32_t s0 = v[k] & 0xFFFFu, s1 = v[k] >> 16;
              cb += Lt[s0] + Lt[s1];
              co += (s0 == 0) + (s1 == 0);
              all = all && s0 == R && s1 == R;
            }
          }
        } else {
          for (uint32_t t = t0; t < t0 + My; ++t) {
            const uint16_t s = col[t];
            cb += Lt[s];
            co += (s == 0);
            all = all && s == R;
          }
        }
        bits += all ? LZ : cb;
        no += co;
      }
      a.lane_len[unit_lane_off(a.g, a.logs, u) + j] = uint16_t(bits);
    } else if (j < Mx) {
      const uint16_t* col = a.sym + uint64_t(unit_sym_off(a.g, a.logs, u)) + uint64_t(j) * rows;
      uint32_t t = 0;
      if ((reinterpret_cast<uintptr_t>(col) & 15) == 0) {
        const uint4* c4 = reinterpret_cast<const uint4*>(col);
        for (; t + 8 <= rows; t += 8) {
          const uint4 w = c4[t >> 3];
          const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t s0 = v[k] & 0xFFFFu, s1 = v[k] >> 16;
            bits += Lt[s0] + Lt[s1];
            no += (s0 == 0) + (s1 == 0);
          }
        }
      }
      for (; t < rows; ++t) {
        const uint16_t s = col[t];
        bits += Lt[s];
        no += (s == 0);
      }
      a.lane_len[unit_lane_off(a.g, a.logs, u) + j] = uint16_t(bits);
    }
  }
  bits_s[tid] = bits;
  out_s[tid] = no;
  __syncthreads();
  if (is_lane && j == 0) {
    uint32_t tb = 0, to = 0;
    for (int k = 0; k < Mx; ++k) {
      tb += bits_s[tid + k];
      to += out_s[tid + k];
    }
    a.cnt_words[u] = (tb + 31) >> 5;
    a.cnt_outl[u] = to;
  }
}

__global__ __launch_bounds__(256) void k_lanelen(LaneLenArgs a) { lanelen_body(a, blockIdx.x); }

// ---------------------------------------------------------------------------
// Segmented exclusive scan: `nseg` segments of n u32 values, out[seg][n+1].
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256 * kScanItems;

__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
  __shared__ uint64_t ws[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t t = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += t;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  for (int i = 0; i < 4; ++i) {
    if (i < w) pre += ws[i];
    tot += ws[i];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__device__ inline void scan_a_body(const uint32_t* in, uint64_t n, uint64_t* part, int nblk,
                                   int seg, int bx) {
  const uint32_t* src = in + uint64_t(seg) * n;
  const uint64_t base = uint64_t(bx) * kScanBlock + uint64_t(threadIdx.x) * kScanItems;
  uint64_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += src[base + i];
  uint64_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[uint64_t(seg) * nblk + bx] = tot;
}

__global__ __launch_bounds__(256) void k_scan_a(const uint32_t* in, uint64_t n, uint64_t* part,
                                                int nblk) {
  scan_a_body(in, n, part, nblk, blockIdx.y, blockIdx.x);
}

__device__ inline void scan_b_body(uint64_t* part, int nblk, int seg) {
  uint64_t* p = part + uint64_t(seg) * nblk;
  uint64_t carry = 0;
  for (int b0 = 0; b0 < nblk; b0 += 256) {
    const int i = b0 + threadIdx.x;
    const uint64_t v = i < nblk ? p[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan(v, &tot);
    if (i < nblk) p[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(256) void k_scan_b(uint64_t* part, int nblk) {
  scan_b_body(part, nblk, blockIdx.x);
}

__device__ inline void scan_c_body(const uint32_t* in, uint64_t n, const uint64_t* part, int nblk,
                                   uint32_t* out, DevParams* P, int seg, int bx) {
  const uint32_t* src = in + uint64_t(seg) * n;
  uint32_t* dst = out + uint64_t(seg) * (n + 1);
  const uint64_t base = uint64_t(bx) * kScanBlock + uint64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? src[base + i] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = part[uint64_t(seg) * nblk + bx] + block_excl_scan(s, &tot);
  bool over = false;
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) {
      over |= run > 0xFFFFFFFFull;
      dst[base + i] = uint32_t(run);
    }
    run += v[i];
    if (base + i + 1 == n) {
      over |= run > 0xFFFFFFFFull;
      dst[n] = uint32_t(run);
    }
  }
  if (over) atomicOr(&P->flags, kFlagTooLarge);
}

__global__ __launch_bounds__(256) void k_scan_c(const uint32_t* in, uint64_t n, const uint64_t* part,
                                                int nblk, uint32_t* out, DevParams* P) {
  scan_c_body(in, n, part, nblk, out, P, blockIdx.y, blockIdx.x);
}

struct LayoutArgs {
  Geo g;
  int vb;        // bytes per stored value (anchors, outliers): 4 or 8
  int eb_mode;
  double eb, ratio;
  uint64_t out_cap;
  uint8_t* out;
  DevParams* P;
  const uint32_t* scan;   // [2L][nu+1]
  uint64_t nu;
  LevelConst lc[kMaxLevels + 1];
  uint64_t n_anchor;
};

__device__ inline void st32(uint8_t* p, uint32_t v) { *reinterpret_cast<uint32_t*>(p) = v; }
__device__ inline void st64(uint8_t* p, uint64_t v) {
  st32(p, uint32_t(v));
  st32(p + 4, uint32_t(v >> 32));
}

// Stream layout (format 2.5) from the scanned totals; writes the header.
__device__ inline void layout_body(const LayoutArgs& a) {
  if (threadIdx.x != 0) return;
  DevParams* P = a.P;
  const int L = a.g.L;
  const uint64_t anchor_off = kHeaderBytes + align16(uint64_t(alphabet(a.g)));
  const uint64_t vb = uint64_t(a.vb);
  uint64_t pos = anchor_off + align16(vb * a.n_anchor);
  for (int l = 1; l <= L; ++l) {
    const uint64_t W = a.scan[uint64_t(2 * (l - 1)) * (a.nu + 1) + a.nu];
    const uint64_t O = a.scan[uint64_t(2 * (l - 1) + 1) * (a.nu + 1) + a.nu];
    P->words[l] = W;
    P->outl[l] = O;
    P->sec[l] = pos;
    P->off_outl[l] = pos + align16(4 * (a.nu + 1));
    P->off_lane[l] = P->off_outl[l] + align16(4 * (a.nu + 1));
    P->off_pay[l] = P->off_lane[l] + align16(2 * a.lc[l].nl);
    P->off_out[l] = P->off_pay[l] + align16(4 * W);
    pos = P->off_out[l] + align16(vb * O);
  }
  P->total = pos;
  if (pos > a.out_cap) P->flags |= kFlagOverflow;
  if (P->flags) return;
  uint8_t* o = a.out;
  for (int i = 0; i < int(kHeaderBytes); i += 4) st32(o + i, 0);
  st32(o + 0, kMagic);
  st32(o + 4, kVersion);
  for (int d = 0; d < 3; ++d) st64(o + 8 + 8 * d, uint64_t(a.g.n[d]));
  st32(o + 32, uint32_t(a.g.B));
  st32(o + 36, uint32_t(L));
  st32(o + 40, uint32_t(a.g.R));
  st32(o + 44, uint32_t(kLmax));
  st32(o + 48, uint32_t(a.eb_mode));
  st32(o + 52, a.vb == 8 ? 1u : 0u);  // value type: 0 float32, 1 float64
  st64(o + 56, __double_as_longlong(a.eb));
  st64(o + 64, __double_as_longlong(P->eb_abs));
  st64(o + 72, __double_as_longlong(a.ratio));
  st64(o + 80, pos);
  st64(o + 88, kHeaderBytes);
  st64(o + 96, anchor_off);
  st64(o + 104, a.n_anchor);
  st32(o + 112, a.g.Z >= 0 ? 2u : 1u);  // coding: 1 Huffman only, 2 zero chunks
  for (int l = 1; l <= L; ++l) {
    uint8_t* e = o + kLevelTable + kLevelRec * uint64_t(l - 1);
    st64(e + 0, P->sec[l]);
    st64(e + 8, a.nu);
    st64(e + 16, a.lc[l].nl);
    st64(e + 24, a.lc[l].nsym);
    st64(e + 32, P->words[l]);
    st64(e + 40, P->outl[l]);
  }
}

__global__ void k_layout(LayoutArgs a) { layout_body(a); }

// Zero [from, total) of the stream (padding and the words packed with atomics),
// except the payload of level `skip` (-1: none), which the unit packer writes
// word by word in full (its last, partly padded 16 bytes are still cleared).
__device__ inline void zero_body(uint8_t* out, uint64_t from, const DevParams* P, uint64_t wg,
                                 uint64_t ngrid, int skip = -1) {
  if (P->flags) return;
  const uint64_t to = P->total;
  uint64_t s0 = 0, s1 = 0;  // skipped range, in 16-byte units
  if (skip >= 0) {
    s0 = P->off_pay[skip] / 16;
    s1 = (P->off_pay[skip] + 4 * P->words[skip]) / 16;
  }
  uint4* p = reinterpret_cast<uint4*>(out);
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (uint64_t i = from / 16 + wg * blockDim.x + threadIdx.x; i < to / 16;
       i += ngrid * blockDim.x)
    if (i < s0 || i >= s1) p[i] = z;
}

__global__ void k_zero(uint8_t* out, uint64_t from, const DevParams* P, int skip) {
  zero_body(out, from, P, blockIdx.x, gridDim.x, skip);
}

// Code lengths and anchors into the stream.
__device__ inline void fill_head_body(uint8_t* out, const uint8_t* lens, int nsym,
                                      const void* rec0, int vb, uint64_t na, const DevParams* P,
                                      uint64_t wg, uint64_t ngrid) {
  if (P->flags) return;
  const uint64_t anchor_off = kHeaderBytes + align16(uint64_t(nsym));
  for (uint64_t i = wg * blockDim.x + threadIdx.x; i < na + uint64_t(nsym);
       i += ngrid * blockDim.x) {
    if (i < uint64_t(nsym))
      out[kHeaderBytes + i] = lens[i];
    else if (vb == 8)
      reinterpret_cast<double*>(out + anchor_off)[i - nsym] =
          static_cast<const double*>(rec0)[i - nsym];
    else
      reinterpret_cast<float*>(out + anchor_off)[i - nsym] =
          static_cast<const float*>(rec0)[i - nsym];
  }
}

__global__ void k_fill_head(uint8_t* out, const uint8_t* lens, int nsym, const void* rec0,
                            int vb, uint64_t na, const DevParams* P) {
  fill_head_body(out, lens, nsym, rec0, vb, na, P, blockIdx.x, gridDim.x);
}

struct PackArgs {
  const void* x;  // field values, vb bytes each
  int vb;
  Geo g;
  int level, logs;
  const uint16_t* sym;
  uint64_t nu;
  const uint8_t* lens;
  const uint16_t* codes;
  int nsym;
  const uint16_t* lane_len;
  const uint32_t* scan_words;  // nu+1
  const uint32_t* scan_outl;   // nu+1
  uint8_t* out;
  const DevParams* P;
};

// Outlier k of a level: the input value at full-resolution index i, verbatim.
__device__ inline void put_outlier(uint8_t* outv, int vb, uint64_t k, const void* x, int64_t i) {
  if (vb == 8)
    reinterpret_cast<double*>(outv)[k] = static_cast<const double*>(x)[i];
  else
    reinterpret_cast<float*>(outv)[k] = static_cast<const float*>(x)[i];
}

__device__ inline void emit_word(uint32_t* pay, uint64_t wi, uint32_t w, uint64_t start,
                                 uint64_t end) {
  if (wi * 32 >= start && wi * 32 + 32 <= end)
    pay[wi] = w;
  else if (w)
    atomicOr(&pay[wi], w);
}

// Full blocks of 16^3 level points (units of 8^3 = 512 symbols, chunks of
// M_y = 8 rows) whose symbols are 16-byte aligned: the block's 7 units, one
// after the other in the level's symbol array, are encoded together. Thread
// t < 224 takes 16 consecutive symbols of unit t / 32 (two 16-byte loads);
// bit offsets come from a scan over the unit's 32 threads (half a wave) plus
// the unit's first word; codes go into an LDS buffer of the block's words,
// written out coalesced; outlier ranks (row-major) from per-row column masks.
// Returns false (nothing written) when the block does not qualify.
__device__ inline bool pack_block16(const PackArgs& a, int64_t wg, const uint8_t* Ls,
                                    const uint16_t* Cs, uint32_t* unit_word, uint32_t* unit_outl,
                                    uint16_t* lane_arr, uint32_t* pay, uint8_t* outv) {
  constexpr int kU = 512, kRows = 64, kTPU = 32, kWords = 7 * (kU * kLmax / 32) + 8;
  __shared__ uint32_t wb[kWords];
  __shared__ uint32_t rmask[7 * kRows];  // per unit row: columns holding an outlier
  __shared__ int64_t usym0;
  __shared__ int s_ok, s_out;
  const int tid = threadIdx.x;
  const int64_t u0 = wg * 7;
  if (tid == 0) {
    s_ok = (reinterpret_cast<uintptr_t>(a.sym) & 15) == 0;
    s_out = 0;
    usym0 = unit_sym_off(a.g, a.logs, u0);
    if (usym0 & 7) s_ok = 0;
  }
  if (tid < 7 * kRows) rmask[tid] = 0;
  for (int i = tid + 256; i < 7 * kRows; i += 256) rmask[i] = 0;
  __syncthreads();
  if (tid < 7) {
    const UnitGeo ug = unit_geo(a.g, u0 + tid, a.logs);
    if (ug.M[0] != 8 || ug.M[1] != 8 || ug.M[2] != 8) s_ok = 0;
  }
  __syncthreads();
  if (!s_ok) return false;
  // unit index entries and lane lengths
  if (tid < 56) {
    const int c = tid / 8, j = tid % 8;
    const int64_t u = u0 + c;
    const uint64_t li = uint64_t(unit_lane_off(a.g, a.logs, u)) + j;
    lane_arr[li] = a.lane_len[li];
    if (j == 0) {
      unit_word[u] = a.scan_words[u];
      unit_outl[u] = a.scan_outl[u];
      if (a.scan_outl[u + 1] != a.scan_outl[u]) s_out = 1;
      if (u == int64_t(a.nu) - 1) {
        unit_word[a.nu] = a.scan_words[a.nu];
        unit_outl[a.nu] = a.scan_outl[a.nu];
      }
    }
  }
  const uint32_t w0 = a.scan_words[u0];
  const uint32_t nw = a.scan_words[u0 + 7] - w0;
  for (uint32_t i = tid; i < nw; i += 256) wb[i] = 0;
  const int cu = tid / kTPU, r = tid % kTPU;  // unit, run within the unit
  const bool act = tid < 7 * kTPU;
  const bool zc = a.g.Z >= 0;
  const uint32_t R = uint32_t(a.g.R);
  const uint32_t lcz = zc ? (uint32_t(Cs[a.g.Z]) | (uint32_t(Ls[a.g.Z]) << 16)) : 0u;
  uint32_t lc[16];
  uint32_t mine = 0;
  if (act) {
    const uint4* g4 = reinterpret_cast<const uint4*>(a.sym + usym0 + cu * kU + r * 16);
    const uint4 q0 = g4[0], q1 = g4[1];
    const uint32_t v[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    uint32_t rm = 0;  // bit k: symbol k of the run is R
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t sy = (v[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      lc[k] = uint32_t(Cs[sy]) | (uint32_t(Ls[sy]) << 16);
      rm |= uint32_t(sy == R) << k;
      if (sy == 0) {  // outlier: symbol p of the unit is row p mod 64 of column p / 64
        const int p = r * 16 + k;
        atomicOr(&rmask[cu * kRows + (p & (kRows - 1))], 1u << (p / kRows));
      }
    }
    if (zc) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (((rm >> (8 * h)) & 0xFFu) == 0xFFu) {
#pragma unroll
          for (int k = 0; k < 8; ++k) lc[8 * h + k] = k == 0 ? lcz : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) mine += lc[k] >> 16;
  }
  // exclusive scan of the bit counts over the unit's 32 threads
  uint32_t inc = mine;
#pragma unroll
  for (int o = 1; o < kTPU; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, kTPU);
    if (r >= o) inc += t;
  }
  __syncthreads();  // buffer cleared, masks complete
  if (act) {
    const uint32_t pos = (a.scan_words[u0 + cu] - w0) * 32 + (inc - mine);
    uint32_t w = pos >> 5, fill = pos & 31;
    uint64_t acc = 0;
    bool first = true;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t len = lc[k] >> 16, code = lc[k] & 0xFFFFu;
      acc |= (uint64_t(code) << 20) << (44 - fill - len);  // code < 2^12: no overflow
      fill += len;
      if (fill >= 32) {
        const uint32_t word = uint32_t(acc >> 32);
        if (first)
          atomicOr(&wb[w], word);
        else
          wb[w] = word;
        first = false;
        acc <<= 32;
        fill -= 32;
        ++w;
      }
    }
    if (fill) atomicOr(&wb[w], uint32_t(acc >> 32));
  }
  __syncthreads();
  for (uint32_t i = tid; i < nw; i += 256) pay[w0 + i] = wb[i];
  // outliers in rank order per unit (row-major: row t, then column): wave 0,
  // one row per lane
  if (s_out && tid < kRows) {
    for (int c = 0; c < 7; ++c) {
      const int64_t u = u0 + c;
      const uint32_t uo = a.scan_outl[u], n_out = a.scan_outl[u + 1] - uo;
      if (n_out == 0) continue;
      uint32_t mk = rmask[c * kRows + tid];
      const uint32_t cnt = __popc(mk);
      uint32_t incl = cnt;
#pragma unroll
      for (int o = 1; o < kRows; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, kWave);
        if (tid >= o) incl += t;
      }
      uint32_t rank = incl - cnt;
      const UnitGeo ug = unit_geo(a.g, u, a.logs);
      const uint32_t vy = tid % 8, vz = tid / 8;
      const int64_t pz = (ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs);
      const int64_t py = (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs);
      while (mk) {
        const uint32_t jj = __ffs(mk) - 1;
        mk &= mk - 1;
        if (rank < n_out) {
          const int64_t px = (ug.b[2] << a.g.logB) + (int64_t(2 * jj + ug.o[2]) << a.logs);
          put_outlier(outv, a.vb, uo + rank, a.x, (pz * a.g.n[1] + py) * a.g.n[2] + px);
        }
        ++rank;
      }
    }
  }
  return true;
}

// Small units (block edge at this level below 32): one lane per column
// stream packs its codes directly (same block mapping as k_lanelen); a unit's
// lanes sit inside one wave, so the rank order of its outliers comes from a
// per-row ballot.
__device__ inline void pack_lanes_body(const PackArgs& a, int64_t wg) {
  const DevParams* P = a.P;
  if (P->flags) return;
  __shared__ uint8_t Ls[kMaxAlphabet];
  __shared__ uint16_t Cs[kMaxAlphabet];
  __shared__ uint32_t lb_s[256];
  const int m = (a.g.B >> a.logs) >> 1;
  // the code table in LDS for blocks of 16^3 level points; smaller ones (at
  // most 16 symbols per lane) read it through the cache
  if (m >= 8)
    for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) {
      Ls[i] = a.lens[i];
      Cs[i] = a.codes[i];
    }
  const uint8_t* Lt = m >= 8 ? static_cast<const uint8_t*>(Ls) : a.lens;
  const uint16_t* Ct = m >= 8 ? static_cast<const uint16_t*>(Cs) : a.codes;
  const int l = a.level;
  uint32_t* unit_word = reinterpret_cast<uint32_t*>(a.out + P->sec[l]);
  uint32_t* unit_outl = reinterpret_cast<uint32_t*>(a.out + P->off_outl[l]);
  uint16_t* lane_arr = reinterpret_cast<uint16_t*>(a.out + P->off_lane[l]);
  uint32_t* pay = reinterpret_cast<uint32_t*>(a.out + P->off_pay[l]);
  uint8_t* outv = a.out + P->off_out[l];
  const int tid = threadIdx.x, lane = tid & 63, c = tid / m + 1, j = tid % m;
  const bool is_lane = tid < 7 * m;
  const int64_t u = wg * 7 + (c - 1);
  UnitGeo ug;
  uint32_t lb = 0, rows = 0, M1 = 1;
  int Mx = 0;
  uint64_t lane0 = 0;
  if (is_lane) {
    ug = unit_geo(a.g, u, a.logs);
    M1 = ug.M[1];
    rows = uint32_t(ug.M[0]) * M1;
    Mx = ug.M[2];
    lane0 = uint64_t(unit_lane_off(a.g, a.logs, u));
    if (j < Mx) lb = a.lane_len[lane0 + j];
  }
  lb_s[tid] = lb;
  __syncthreads();
  if (!is_lane) return;
  uint32_t pre = 0;
  for (int k = 0; k < j; ++k) pre += lb_s[tid - j + k];
  const uint32_t uw = a.scan_words[u], uo = a.scan_outl[u];
  if (j == 0) {
    unit_word[u] = uw;
    unit_outl[u] = uo;
    if (u == int64_t(a.nu) - 1) {
      unit_word[a.nu] = a.scan_words[a.nu];
      unit_outl[a.nu] = a.scan_outl[a.nu];
    }
  }
  const bool act = j < Mx;
  if (act) lane_arr[lane0 + j] = uint16_t(lb);
  const uint64_t start = uint64_t(uw) * 32 + pre, end = start + lb;
  uint64_t pos = start;
  uint32_t cur = 0, run = 0;
  const uint64_t base = uint64_t(unit_sym_off(a.g, a.logs, u));
  const uint64_t segmask = (m >= 64 ? ~uint64_t(0) : ((uint64_t(1) << m) - 1)) << (lane - j);
  const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
  const uint16_t* col = a.sym + base + uint64_t(j) * rows;
  // zero chunks: at the first row of each chunk (M_y rows) the lane checks the
  // chunk; a chunk of all-R symbols emits Z there and nothing for its rows
  const bool zc = a.g.Z >= 0;
  const uint32_t Rs = uint32_t(a.g.R);
  uint32_t vyc = 0;     // row within the current chunk
  bool zrun = false;    // the current chunk is all R
  // zk: whether the chunk starting at this row is all R when the caller
  // knows it (-1: read the chunk's symbols here)
  auto step = [&](uint32_t s, uint32_t t, int zk) {
    uint32_t len = Lt[s], cw = Ct[s];
    if (zc) {
      if (vyc == 0) {
        bool all = act;
        if (zk >= 0)
          all = all && zk != 0;
        else
          for (uint32_t k = 0; k < M1 && all; ++k) all = col[t + k] == Rs;
        zrun = all;
      }
      if (zrun) {
        len = vyc == 0 ? Lt[a.g.Z] : 0u;
        cw = Ct[a.g.Z];
      }
      if (++vyc == M1) vyc = 0;
    }
    if (act && len) {
      const uint32_t o = uint32_t(pos & 31);
      if (o + len <= 32) {
        cur |= cw << (32 - o - len);
        pos += len;
        if ((pos & 31) == 0) {
          emit_word(pay, (pos >> 5) - 1, cur, start, end);
          cur = 0;
        }
      } else {
        const uint32_t hi = len - (32 - o);
        cur |= cw >> hi;
        emit_word(pay, pos >> 5, cur, start, end);
        cur = cw << (32 - hi);
        pos += len;
      }
    }
    const bool is_out = act && s == 0;
    const uint64_t mk = __ballot(is_out) & segmask;
    if (is_out) {
      const uint32_t vy = t % M1, vz = t / M1;
      const int64_t pz = (ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs);
      const int64_t py = (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs);
      const int64_t px = (ug.b[2] << a.g.logB) + (int64_t(2 * j + ug.o[2]) << a.logs);
      put_outlier(outv, a.vb, uo + run + __popcll(mk & lt_mask), a.x,
                  (pz * a.g.n[1] + py) * a.g.n[2] + px);
    }
    run += __popcll(mk);
  };
  // Rows in lockstep across the unit's lanes (the outlier ballot needs it);
  // 8 symbols per 16-byte load when the column is aligned, which holds for
  // every lane of a unit or for none.
  uint32_t t = 0;
  if ((reinterpret_cast<uintptr_t>(a.sym + base + uint64_t(0) * rows) & 15) == 0 && (rows & 7) == 0) {
    const uint4* c4 = reinterpret_cast<const uint4*>(col);
    for (; t < rows; t += 8) {
      const uint4 w = act ? c4[t >> 3] : make_uint4(0x00010001u, 0x00010001u, 0x00010001u,
                                                    0x00010001u);
      const uint32_t v[4] = {w.x, w.y, w.z, w.w};
      // chunks of M_y rows dividing the 8 loaded rows: their all-R flags
      // come from these symbols (bit i: row t + i is R)
      uint32_t r8 = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        r8 |= (uint32_t((v[k] & 0xFFFFu) == Rs) << (2 * k)) | (uint32_t((v[k] >> 16) == Rs) << (2 * k + 1));
      const bool known = (8 % M1) == 0;
      const uint32_t cm = (1u << M1) - 1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i0 = 2 * k, i1 = 2 * k + 1;
        step(v[k] & 0xFFFFu, t + i0, known ? int(((r8 >> i0) & cm) == cm) : -1);
        step(v[k] >> 16, t + i1, known ? int(((r8 >> i1) & cm) == cm) : -1);
      }
    }
  }
  for (; t < rows; ++t) step(act ? col[t] : uint16_t(1), t, -1);
  if (act && (pos & 31)) emit_word(pay, pos >> 5, cur, start, end);
}

// Bit-pack the block's 7 units, write the unit index, the lane lengths and
// the outliers. A unit's stream is the concatenation of its lanes, i.e. the
// Huffman codes of the unit's symbols in their memory order (columns one after
// the other), and starts on a word boundary; so a work-group encodes each unit
// in chunks: coalesced symbol loads into LDS, a block scan of code lengths for
// bit offsets, codes OR-ed into an LDS word buffer, complete words written out
// with coalesced stores (the last partial word carries into the next chunk).
constexpr int kPackChunk = 4096;                     // symbols per chunk
constexpr int kPackPer = kPackChunk / 256;           // per thread
static_assert(kPackPer % 8 == 0, "a run is whole 16-byte groups");
constexpr int kPackWords = kPackChunk * kLmax / 32 + 2;
constexpr int kPackRows = 32 * 32;  // rows (M_z * M_y) of a unit, E <= 64

// 32-bit exclusive scan over the work-group (256 threads).
__device__ inline uint32_t block_excl_scan32(uint32_t v, uint32_t* total) {
  __shared__ uint32_t ws[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += t;
  }
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int i = 0; i < 4; ++i) {
    if (i < w) pre += ws[i];
    tot += ws[i];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__device__ inline void pack_units_body(const PackArgs& a, int64_t wg) {
  const DevParams* P = a.P;
  if (P->flags) return;
  __shared__ uint32_t LC[kMaxAlphabet];  // code | length << 16
  __shared__ __align__(16) uint16_t us[kPackChunk];
  __shared__ uint32_t zf[kPackChunk / 32];  // zero-chunk flags of the buffer (bits)
  __shared__ uint32_t wb[kPackWords];
  __shared__ uint32_t rmask[kPackRows];  // per unit row: columns holding an outlier
  __shared__ uint32_t u_rows[8], u_mx[8], u_my[8];
  __shared__ uint64_t u_src[8];
  const int tid = threadIdx.x;
  for (int i = tid; i < a.nsym; i += blockDim.x)
    LC[i] = uint32_t(a.codes[i]) | (uint32_t(a.lens[i]) << 16);
  const int l = a.level;
  uint32_t* unit_word = reinterpret_cast<uint32_t*>(a.out + P->sec[l]);
  uint32_t* unit_outl = reinterpret_cast<uint32_t*>(a.out + P->off_outl[l]);
  uint16_t* lane_arr = reinterpret_cast<uint16_t*>(a.out + P->off_lane[l]);
  uint32_t* pay = reinterpret_cast<uint32_t*>(a.out + P->off_pay[l]);
  uint8_t* outv = a.out + P->off_out[l];
  const int m = (a.g.B >> a.logs) >> 1;
  // per-unit geometry once per block (threads 0..6), unit index entries
  if (tid < 7) {
    const int64_t u = wg * 7 + tid;
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    u_rows[tid + 1] = uint32_t(ug.M[0]) * ug.M[1];
    u_my[tid + 1] = uint32_t(ug.M[1]);
    u_mx[tid + 1] = uint32_t(ug.M[2]);
    u_src[tid + 1] = uint64_t(unit_sym_off(a.g, a.logs, u));
    unit_word[u] = a.scan_words[u];
    unit_outl[u] = a.scan_outl[u];
    if (u == int64_t(a.nu) - 1) {
      unit_word[a.nu] = a.scan_words[a.nu];
      unit_outl[a.nu] = a.scan_outl[a.nu];
    }
  }
  __syncthreads();
  if (tid < 7 * m) {  // lane lengths of the block's units
    const int c = tid / m + 1, j = tid % m;
    if (uint32_t(j) < u_mx[c]) {
      const uint64_t li = uint64_t(unit_lane_off(a.g, a.logs, wg * 7 + c - 1)) + j;
      lane_arr[li] = a.lane_len[li];
    }
  }
  for (int c = 1; c <= 7; ++c) {
    const int64_t u = wg * 7 + (c - 1);
    const uint32_t rows = u_rows[c];
    const uint32_t n_u = rows * u_mx[c];
    if (n_u == 0) continue;
    const uint16_t* src = a.sym + u_src[c];
    uint32_t* dst = pay + a.scan_words[u];
    uint32_t wdone = 0;  // whole words of the unit written so far
    uint32_t sk = 0;     // bits carried in the partial word
    uint32_t carry = 0;
    // Zero chunks: chunk k of the unit = symbols [k*M_y, (k+1)*M_y) (one v_z of
    // one column). Buffers hold whole chunks, so each buffer flags its own.
    const uint32_t My = u_my[c];
    const bool zc = a.g.Z >= 0 && My > 0;
    const uint32_t bstep = zc ? (kPackChunk / My) * My : kPackChunk;
    const uint32_t lcz = zc ? LC[a.g.Z] : 0u;
    // How a thread finds its zero chunks: 1 = M_y divides its run of kPackPer
    // symbols (chunks inside the run), 2 = M_y is two runs (the chunk is this
    // run and its pair's), 3 = other M_y (edge blocks): flags in LDS.
    const int zmode = !zc ? 0
                      : ((kPackPer % My) == 0 ? 1 : (My == 2 * kPackPer ? 2 : 3));
    // Outliers: while the symbols pass through LDS, each outlier sets its
    // column's bit in its row's mask; ranks (row-major) come from the masks.
    const uint32_t uo = a.scan_outl[u], n_out = a.scan_outl[u + 1] - uo;
    const uint32_t Mx = u_mx[c];
    if (n_out)
      for (uint32_t i = tid; i < rows; i += 256) rmask[i] = 0;
    for (uint32_t c0 = 0; c0 < n_u; c0 += bstep) {
      const int n = int(min<uint32_t>(bstep, n_u - c0));
      if (((reinterpret_cast<uintptr_t>(src + c0) | uint32_t(n)) & 15) == 0) {
        // whole 16-byte groups of 8 symbols
        const uint4* s4 = reinterpret_cast<const uint4*>(src + c0);
        uint4* d4 = reinterpret_cast<uint4*>(us);
        for (int i = tid; i < n / 8; i += 256) d4[i] = s4[i];
      } else {
        for (int i = tid; i < n; i += 256) us[i] = src[c0 + i];
      }
      __syncthreads();
      if (zmode == 3) {
        const int nch = n / int(My);
        for (int k = tid; k < (nch + 31) / 32; k += 256) zf[k] = 0;
        __syncthreads();
        for (int k = tid; k < nch; k += 256) {
          bool all = true;
#pragma unroll 8
          for (uint32_t v = 0; v < My; ++v) all &= us[k * My + v] == uint16_t(a.g.R);
          if (all) atomicOr(&zf[k >> 5], 1u << (k & 31));
        }
        __syncthreads();
      }
      // this thread's run of kPackPer symbols: (code, length) in registers; a
      // zero chunk's first symbol carries Z's code, its others nothing
      const int i0 = tid * kPackPer;
      uint32_t lc[kPackPer];
      uint32_t rm = 0;  // bit k: symbol k of the run is R
      // the run's symbols as 16-byte LDS reads of 8 symbols each
#pragma unroll
      for (int g = 0; g < kPackPer / 8; ++g) {
        const uint4 q = reinterpret_cast<const uint4*>(us + i0)[g];
        const uint32_t sw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int k = 8 * g + h;
          const bool ok = i0 + k < n;
          const uint32_t sy = ok ? (sw[h >> 1] >> (16 * (h & 1))) & 0xFFFFu : 0u;
          lc[k] = ok ? LC[sy] : 0u;
          rm |= uint32_t(ok && sy == uint32_t(a.g.R)) << k;
        }
      }
      if (n_out)  // symbol p of the unit: column p / rows, row p % rows
        for (int i = tid; i < n; i += 256)
          if (us[i] == 0) {
            const uint32_t p = c0 + uint32_t(i), jj = p / rows;
            atomicOr(&rmask[p - jj * rows], 1u << jj);
          }
      if (zmode == 1) {
        // bit k of f: symbols k..k+M_y-1 all R (M_y a power of two)
        uint32_t f = rm;
        for (uint32_t sft = 1; sft < My; sft <<= 1) f &= f >> sft;
#pragma unroll
        for (int k = 0; k < kPackPer; ++k) {
          const uint32_t base = uint32_t(k) & ~(My - 1);
          if ((f >> base) & 1u) lc[k] = uint32_t(k) == base ? lcz : 0u;
        }
      } else if (zmode == 2) {
        const bool mine_all = rm == (1u << kPackPer) - 1;
        // every lane takes part in the shuffle (no short circuit around it)
        const int pair_all = __shfl_xor(int(mine_all), 1, kWave);
        const bool all = mine_all && pair_all != 0;
        if (all) {
#pragma unroll
          for (int k = 0; k < kPackPer; ++k) lc[k] = (k == 0 && (tid & 1) == 0) ? lcz : 0u;
        }
      } else if (zmode == 3) {
        uint32_t q = uint32_t(i0) / My, r = uint32_t(i0) - q * My;
#pragma unroll
        for (int k = 0; k < kPackPer; ++k) {
          if (i0 + k < n) {
            if ((zf[q >> 5] >> (q & 31)) & 1u) lc[k] = r == 0 ? lcz : 0u;
            if (++r == My) {
              r = 0;
              ++q;
            }
          }
        }
      }
      uint32_t mine = 0;
#pragma unroll
      for (int k = 0; k < kPackPer; ++k) mine += lc[k] >> 16;
      uint32_t total;
      const uint32_t off = block_excl_scan32(mine, &total);
      const uint32_t nw = (sk + total + 31) >> 5;
      for (uint32_t i = tid; i < nw; i += 256) wb[i] = i == 0 ? carry : 0u;
      if (nw == 0 && tid == 0) wb[0] = carry;
      __syncthreads();
      // codes of the run into the word buffer (chunk-relative bit positions):
      // a 64-bit accumulator holds the word being filled (high half) and the
      // next; words wholly inside the run are stored, its first and last
      // words (shared with the neighbouring runs) OR-ed in
      {
        uint32_t w = (sk + off) >> 5, fill = (sk + off) & 31;
        uint64_t acc = 0;
        bool first = true;
#pragma unroll
        for (int k = 0; k < kPackPer; ++k) {
          const uint32_t len = lc[k] >> 16, code = lc[k] & 0xFFFFu;
          acc |= (uint64_t(code) << 20) << (44 - fill - len);  // code < 2^12: no overflow
          fill += len;
          if (fill >= 32) {
            const uint32_t word = uint32_t(acc >> 32);
            if (first)
              atomicOr(&wb[w], word);
            else
              wb[w] = word;
            first = false;
            acc <<= 32;
            fill -= 32;
            ++w;
          }
        }
        if (fill) atomicOr(&wb[w], uint32_t(acc >> 32));
      }
      __syncthreads();
      // complete words out; the partial last word carries over
      const uint32_t end = sk + total;
      const uint32_t full = end >> 5;
      for (uint32_t i = tid; i < full; i += 256) dst[wdone + i] = wb[i];
      carry = (end & 31) ? wb[full] : 0u;
      wdone += full;
      sk = end & 31;
      __syncthreads();
    }
    if (sk && tid == 0) dst[wdone] = carry;
    // outliers in rank order (row-major: row t, then column j): thread tid
    // owns rows [tid*rpt, (tid+1)*rpt); a block scan of its outlier count
    // gives the rank of its first one
    if (n_out) {
      const UnitGeo ug = unit_geo(a.g, u, a.logs);
      const uint32_t M1 = u_my[c];
      const uint32_t rpt = (rows + 255) / 256, t0 = tid * rpt;
      uint32_t cnt = 0;
      for (uint32_t t = t0; t < t0 + rpt && t < rows; ++t) cnt += __popc(rmask[t]);
      uint32_t tot;
      uint32_t rank = block_excl_scan32(cnt, &tot);
      for (uint32_t t = t0; t < t0 + rpt && t < rows; ++t) {
        uint32_t mk = rmask[t];
        while (mk) {
          const uint32_t jj = __ffs(mk) - 1;
          mk &= mk - 1;
          if (rank < n_out && jj < Mx) {
            const uint32_t vy = t % M1, vz = t / M1;
            const int64_t pz = (ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs);
            const int64_t py = (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs);
            const int64_t px = (ug.b[2] << a.g.logB) + (int64_t(2 * jj + ug.o[2]) << a.logs);
            put_outlier(outv, a.vb, uo + rank, a.x, (pz * a.g.n[1] + py) * a.g.n[2] + px);
          }
          ++rank;
        }
      }
      __syncthreads();  // the masks are cleared for the next unit
    }
  }
}


// Plain launches take the packer of their block edge: separate kernels keep
// each one's LDS to its own buffers.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_pack_units(
    PackArgs a) {
  pack_units_body(a, blockIdx.x);
}
__global__ __launch_bounds__(256) void k_pack_lanes(PackArgs a) { pack_lanes_body(a, blockIdx.x); }

// Levels with 16^3-point blocks: the whole-block encoder, the lane packer
// for blocks it does not take (domain edges).
__global__ __launch_bounds__(256) void k_pack_blocks16(PackArgs a) {
  const DevParams* P = a.P;
  if (P->flags) return;
  __shared__ uint8_t Ls[kMaxAlphabet];
  __shared__ uint16_t Cs[kMaxAlphabet];
  for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) {
    Ls[i] = a.lens[i];
    Cs[i] = a.codes[i];
  }
  __syncthreads();
  const int l = a.level;
  if (pack_block16(a, blockIdx.x, Ls, Cs, reinterpret_cast<uint32_t*>(a.out + P->sec[l]),
                   reinterpret_cast<uint32_t*>(a.out + P->off_outl[l]),
                   reinterpret_cast<uint16_t*>(a.out + P->off_lane[l]),
                   reinterpret_cast<uint32_t*>(a.out + P->off_pay[l]), a.out + P->off_out[l]))
    return;
  pack_lanes_body(a, blockIdx.x);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch sequences
// ---------------------------------------------------------------------------
namespace {

// Per-level argument blocks of one job, built the same way on the host (plain
// launches) and on the device (batched launches, from the job table).
__host__ __device__ inline PredSlabArgs pred_args(const CompressArgs& a, int l) {
  const Geo& g = a.geo;
  const int logs = g.L - l;
  PredSlabArgs p;
  p.x = a.x;
  p.g = g;
  p.level = l;
  p.logs = logs;
  for (int q = 0; q < 3; ++q) {
    p.n[q] = ((g.n[q] - 1) >> logs) + 1;
    p.nc[q] = ((g.n[q] - 1) >> (logs + 1)) + 1;
  }
  p.prev = a.rec[l - 1];
  p.cur = l < g.L ? a.rec[l] : nullptr;
  p.sym = a.sym[l];
  p.P = a.params;
  p.hpart = a.hpart;
  p.nslots = a.nslots;
  p.nsym = alphabet(g);
  return p;
}

__host__ __device__ inline LaneLenArgs lanelen_args(const CompressArgs& a, int l) {
  const uint64_t nu = a.lc[1].nu;
  LaneLenArgs q;
  q.g = a.geo;
  q.logs = a.geo.L - l;
  q.sym = a.sym[l];
  q.nu = nu;
  q.lens = a.lens;
  q.nsym = alphabet(a.geo);
  q.lane_len = a.lane_len + a.lane_base[l];
  q.cnt_words = a.cnt + uint64_t(2 * (l - 1)) * nu;
  q.cnt_outl = a.cnt + uint64_t(2 * (l - 1) + 1) * nu;
  return q;
}

__host__ __device__ inline LayoutArgs layout_args(const CompressArgs& a) {
  LayoutArgs la;
  la.g = a.geo;
  la.vb = a.vb;
  la.eb_mode = a.eb_mode;
  la.eb = a.eb;
  la.ratio = a.ratio;
  la.out_cap = a.out_cap;
  la.out = a.out;
  la.P = a.params;
  la.scan = a.scan;
  la.nu = a.lc[1].nu;
  for (int l = 0; l <= kMaxLevels; ++l) la.lc[l] = a.lc[l];
  la.n_anchor = a.n_anchor;
  return la;
}

__host__ __device__ inline PackArgs pack_args(const CompressArgs& a, int l) {
  const uint64_t nu = a.lc[1].nu;
  PackArgs p;
  p.x = a.x;
  p.vb = a.vb;
  p.g = a.geo;
  p.level = l;
  p.logs = a.geo.L - l;
  p.sym = a.sym[l];
  p.nu = nu;
  p.lens = a.lens;
  p.codes = a.codes;
  p.nsym = alphabet(a.geo);
  p.lane_len = a.lane_len + a.lane_base[l];
  p.scan_words = a.scan + uint64_t(2 * (l - 1)) * (nu + 1);
  p.scan_outl = a.scan + uint64_t(2 * (l - 1) + 1) * (nu + 1);
  p.out = a.out;
  p.P = a.params;
  return p;
}

__host__ __device__ inline int scan_blocks(const CompressArgs& a) {
  return int((a.lc[1].nu + kScanBlock - 1) / kScanBlock);
}

// ---------------------------------------------------------------------------
// Batched launches: a work map gives each job [first[i], first[i+1]) of the
// launch's items (job[i] = index into the job table); persistent work-groups
// walk the items with a grid stride, so any grid size covers any batch.
// ---------------------------------------------------------------------------
// The item is the same for the whole work-group, so the results are moved to
// scalar registers (readfirstlane): argument blocks indexed by them then come
// through scalar loads.
__device__ inline int map_find(const ItemMap& m, uint32_t item, uint32_t* loc, uint32_t* cnt) {
  int lo = 0, hi = int(m.n);  // first[lo] <= item < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m.first[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  *loc = __builtin_amdgcn_readfirstlane(item - m.first[lo]);
  *cnt = __builtin_amdgcn_readfirstlane(m.first[lo + 1] - m.first[lo]);
  return __builtin_amdgcn_readfirstlane(int(m.job[lo]));
}

#define STZ_FOR_ITEMS(m)                                                    \
  for (uint32_t it_ = blockIdx.x, tot_ = (m).first[(m).n]; it_ < tot_;      \
       it_ += gridDim.x, __syncthreads())

__global__ void kb_init(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    init_body(a.params);
  }
}

__global__ __launch_bounds__(256) void kb_hzero(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    hzero_body(a.hpart, uint64_t(alphabet(a.geo)) * a.nslots, loc, cnt);
  }
}

__global__ __launch_bounds__(256) void kb_hred(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    hred_body(a.hpart, a.nslots, alphabet(a.geo), a.hist, int(loc));
  }
}

__global__ __launch_bounds__(256) void kb_minmax(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    const uint64_t N = uint64_t(a.geo.n[0]) * a.geo.n[1] * a.geo.n[2];
    minmax_body<float>(static_cast<const float*>(a.x), N, static_cast<MinMax<float>*>(a.part),
                       a.params, loc, cnt);
  }
}

__global__ void kb_resolve(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    resolve_body<float>(a.params, static_cast<const MinMax<float>*>(a.part), a.nparts, a.eb_mode,
                        a.eb, a.ratio, a.geo.L);
  }
}

__global__ void kb_anchor(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    anchor_body<float>(static_cast<const float*>(a.x), a.geo, static_cast<float*>(a.rec[0]),
                       a.params, loc, cnt);
  }
}

// Per-level argument blocks of a batch are built on the host (the same
// builders as the plain launches) and read here through restrict pointers.
template <int E, int H>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(H == pred_slab_h(E) ? pred_waves<float>(E) : 1)))
void kb_pred(const PredSlabArgs* __restrict__ P, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const PredSlabArgs& a = P[map_find(m, it_, &loc, &cnt)];
    const uint32_t nblk = uint32_t(a.g.nb[0] * a.g.nb[1] * a.g.nb[2]);
    // padded range (multiple of 8): contiguous blocks per XCD, padding skipped
    const uint32_t blk = uint32_t(wg_block(loc, cnt, true));
    if (blk < nblk) pred_body<float, E, H>(a, blk, blk);
  }
}

__global__ __launch_bounds__(256) void kb_lanelen(const LaneLenArgs* __restrict__ Q, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    lanelen_body(Q[map_find(m, it_, &loc, &cnt)], loc);
  }
}

__global__ __launch_bounds__(256) void kb_scan_a(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    const int nb = scan_blocks(a);
    scan_a_body(a.cnt, a.lc[1].nu, a.scan_part, nb, int(loc) / nb, int(loc) % nb);
  }
}

__global__ __launch_bounds__(256) void kb_scan_b(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    scan_b_body(a.scan_part, scan_blocks(a), int(loc));
  }
}

__global__ __launch_bounds__(256) void kb_scan_c(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    const int nb = scan_blocks(a);
    scan_c_body(a.cnt, a.lc[1].nu, a.scan_part, nb, a.scan, a.params, int(loc) / nb,
                int(loc) % nb);
  }
}

__global__ void kb_layout(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    layout_body(layout_args(a));
  }
}

__global__ void kb_zero(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    zero_body(a.out, kHeaderBytes, a.params, loc, cnt);
  }
}

__global__ void kb_fill_head(const CompressArgs* J, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const CompressArgs& a = J[map_find(m, it_, &loc, &cnt)];
    fill_head_body(a.out, a.lens, alphabet(a.geo), a.rec[0], a.vb, a.n_anchor, a.params, loc,
                   cnt);
  }
}

// Batched packers, one per packer kind (separate kernels keep each one's LDS
// and registers to its own): the work maps hold jobs whose level edge is
// >= 32 (units) or < 32 (lanes).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void kb_pack_units(
    const PackArgs* __restrict__ Q, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    pack_units_body(Q[map_find(m, it_, &loc, &cnt)], loc);
  }
}

__global__ __launch_bounds__(256) void kb_pack_lanes(const PackArgs* __restrict__ Q, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    pack_lanes_body(Q[map_find(m, it_, &loc, &cnt)], loc);
  }
}

template <class T, int E>
void launch_pred(const PredSlabArgs& p, int64_t nblk, hipStream_t st) {
  // Blocks of 32^3 points and more: the interior box and the shell run as two
  // kernels, each holding only its kind's code (fewer registers and scalar
  // spills for the interior one), the shell's on an auxiliary stream so the
  // two overlap. Smaller blocks: one kernel for all (the launches are short;
  // split, 16^3 blocks measured 3 % slower).
  BlockSplit bs = block_split(p.g.nb, E, p.n);
  const dim3 blk(pred_threads(E));
  if constexpr (E < 32) {
    for (int d = 0; d < 3; ++d) bs.lo[d] = bs.hi[d] = 0;  // every block in the "shell"
    if (p.cur)
      hipLaunchKernelGGL((k_pred_slab<T, E, true, 0>), dim3(unsigned(nblk)), blk, 0, st, p, bs);
    else
      hipLaunchKernelGGL((k_pred_slab<T, E, false, 0>), dim3(unsigned(nblk)), blk, 0, st, p, bs);
  } else {
    const int64_t nI = box_count(bs), nS = nblk - nI;
    // (under graph capture the two kernels go in stream order)
    const AuxStream* aux = (nI && nS && !capturing(st)) ? aux_stream(st) : nullptr;
    hipStream_t ss = st;  // the shell's stream
    if (aux && hipEventRecord(aux->fork, st) == hipSuccess &&
        hipStreamWaitEvent(aux->s, aux->fork, 0) == hipSuccess)
      ss = aux->s;
    if (p.cur) {
      if (nS)
        hipLaunchKernelGGL((k_pred_slab<T, E, true, 2>), dim3(unsigned(nS)), blk, 0, ss, p, bs);
      if (nI)
        hipLaunchKernelGGL((k_pred_slab<T, E, true, 1>), dim3(unsigned(nI)), blk, 0, st, p, bs);
    } else {
      if (nS)
        hipLaunchKernelGGL((k_pred_slab<T, E, false, 2>), dim3(unsigned(nS)), blk, 0, ss, p, bs);
      if (nI)
        hipLaunchKernelGGL((k_pred_slab<T, E, false, 1>), dim3(unsigned(nI)), blk, 0, st, p, bs);
    }
    if (ss != st) {
      // the join: st goes on only after the shell's kernel
      if (hipEventRecord(aux->join, ss) != hipSuccess ||
          hipStreamWaitEvent(st, aux->join, 0) != hipSuccess)
        (void)hipStreamSynchronize(ss);
    }
  }
}

template <int E, int H>
void launch_pred_b(const PredSlabArgs* P, const ItemMap& m, unsigned grid, hipStream_t st) {
  hipLaunchKernelGGL((kb_pred<E, H>), dim3(grid), dim3(256), 0, st, P, m);
}

// Slab heights the batched predictor is built for, per level block edge.
template <int E>
void launch_pred_bh(int h, const PredSlabArgs* P, const ItemMap& m, unsigned grid,
                    hipStream_t st) {
  if constexpr (E == 8) {
    if (h == 4) return launch_pred_b<8, 4>(P, m, grid, st);
  } else if constexpr (E == 16) {
    if (h == 4) return launch_pred_b<16, 4>(P, m, grid, st);
    if (h == 8) return launch_pred_b<16, 8>(P, m, grid, st);
  } else if constexpr (E == 32) {
    if (h == 2) return launch_pred_b<32, 2>(P, m, grid, st);
    if (h == 4) return launch_pred_b<32, 4>(P, m, grid, st);
  } else if constexpr (E == 64) {
    if (h == 4) return launch_pred_b<64, 4>(P, m, grid, st);
  }
  launch_pred_b<E, default_slab_h(E)>(P, m, grid, st);
}

}  // namespace

// Per-level argument blocks of a batch: [level 1..max_levels][job] for the
// predictor, the lane lengths and the packer, each array 256-byte aligned.
namespace {
struct BatchArgLayout {
  uint64_t pred, lane, pack, total;
  BatchArgLayout(uint32_t n, int levels) {
    auto al = [](uint64_t v) { return (v + 255) & ~uint64_t(255); };
    const uint64_t k = uint64_t(n) * uint64_t(levels);
    pred = 0;
    lane = al(pred + k * sizeof(PredSlabArgs));
    pack = al(lane + k * sizeof(LaneLenArgs));
    total = al(pack + k * sizeof(PackArgs));
  }
};
}  // namespace

uint64_t compress_batch_args_bytes(uint32_t n, int max_levels) {
  return BatchArgLayout(n, max_levels).total;
}

void build_compress_batch_args(const CompressArgs* jobs, uint32_t n, int max_levels,
                               uint8_t* dst) {
  const BatchArgLayout lay(n, max_levels);
  auto* P = reinterpret_cast<PredSlabArgs*>(dst + lay.pred);
  auto* Q = reinterpret_cast<LaneLenArgs*>(dst + lay.lane);
  auto* K = reinterpret_cast<PackArgs*>(dst + lay.pack);
  std::memset(dst, 0, lay.total);
  for (int l = 1; l <= max_levels; ++l)
    for (uint32_t j = 0; j < n; ++j) {
      if (jobs[j].geo.L < l) continue;
      const uint64_t i = uint64_t(l - 1) * n + j;
      P[i] = pred_args(jobs[j], l);
      Q[i] = lanelen_args(jobs[j], l);
      K[i] = pack_args(jobs[j], l);
    }
}

namespace {

template <class T>
hipError_t launch_compress_t(const CompressArgs& a, hipStream_t st) {
  const Geo& g = a.geo;
  const int L = g.L;
  const int nsym = alphabet(g);
  const uint64_t N = uint64_t(g.n[0]) * g.n[1] * g.n[2];
  const uint64_t nu = a.lc[1].nu;
  prof_begin(st, "init", -1);
  const uint64_t nh = uint64_t(nsym) * a.nslots;
  hipLaunchKernelGGL(k_init_hzero, dim3(grid_for(nh, 256 * 16, 1024)), dim3(256), 0, st,
                     a.params, a.hpart, nh);
  prof_end(st);
  if (a.eb_mode == 1) {
    prof_begin(st, "minmax", -1);
    hipLaunchKernelGGL(k_minmax<T>, dim3(a.nparts), dim3(256), 0, st, static_cast<const T*>(a.x),
                       N, static_cast<MinMax<T>*>(a.part), a.params);
    prof_end(st);
  }
  prof_begin(st, "resolve", -1);
  hipLaunchKernelGGL(k_resolve<T>, dim3(1), dim3(64), 0, st, a.params,
                     static_cast<const MinMax<T>*>(a.part), a.nparts, a.eb_mode, a.eb, a.ratio, L);
  prof_end(st);
  prof_begin(st, "anchor", -1);
  hipLaunchKernelGGL(k_anchor<T>, dim3(grid_for(a.n_anchor, 256, 4096)), dim3(256), 0, st,
                     static_cast<const T*>(a.x), g, static_cast<T*>(a.rec[0]), a.params);
  prof_end(st);
  for (int l = 1; l <= L; ++l) {
    const PredSlabArgs p = pred_args(a, l);
    const int64_t nblk = g.nb[0] * g.nb[1] * g.nb[2];
    const int E = g.B >> (L - l);
    prof_begin(st, "predict", l);
    switch (E) {
      case 2: launch_pred<T, 2>(p, nblk, st); break;
      case 4: launch_pred<T, 4>(p, nblk, st); break;
      case 8: launch_pred<T, 8>(p, nblk, st); break;
      case 16: launch_pred<T, 16>(p, nblk, st); break;
      case 32: launch_pred<T, 32>(p, nblk, st); break;
      default: launch_pred<T, 64>(p, nblk, st); break;
    }
    prof_end(st);
  }
  prof_begin(st, "hist", -1);
  hipLaunchKernelGGL(k_hred, dim3((nsym + 255) / 256), dim3(256), 0, st, a.hpart, a.nslots, nsym,
                     a.hist);
  prof_end(st);
  launch_codebook(a.hist, nsym, a.lens, a.codes, a.cb_scratch, st);
  for (int l = 1; l <= L; ++l) {
    prof_begin(st, "lanelen", l);
    // blocks of at most 8^3 level points (at most 28 lanes): one-wave
    // work-groups, four times as many per CU
    const unsigned nt = (g.B >> (L - l)) <= 8 ? 64u : 256u;
    hipLaunchKernelGGL(k_lanelen, dim3(unsigned(nu / 7)), dim3(nt), 0, st, lanelen_args(a, l));
    prof_end(st);
  }
  const int nblk = scan_blocks(a);
  prof_begin(st, "scan_a", -1);
  hipLaunchKernelGGL(k_scan_a, dim3(nblk, 2 * L), dim3(256), 0, st, a.cnt, nu, a.scan_part, nblk);
  prof_end(st);
  prof_begin(st, "scan_b", -1);
  hipLaunchKernelGGL(k_scan_b, dim3(2 * L), dim3(256), 0, st, a.scan_part, nblk);
  prof_end(st);
  prof_begin(st, "scan_c", -1);
  hipLaunchKernelGGL(k_scan_c, dim3(nblk, 2 * L), dim3(256), 0, st, a.cnt, nu, a.scan_part, nblk,
                     a.scan, a.params);
  prof_end(st);
  prof_begin(st, "layout", -1);
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(64), 0, st, layout_args(a));
  prof_end(st);
  prof_begin(st, "zero", -1);
  // the finest level's payload, when the unit packer writes it, needs no clearing
  hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, st, a.out, kHeaderBytes, a.params,
                     g.B >= 32 ? L : -1);
  prof_end(st);
  prof_begin(st, "fill_head", -1);
  hipLaunchKernelGGL(k_fill_head, dim3(grid_for(a.n_anchor + nsym, 256, 4096)), dim3(256), 0, st,
                     a.out, a.lens, nsym, a.rec[0], a.vb, a.n_anchor, a.params);
  prof_end(st);
  for (int l = 1; l <= L; ++l) {
    prof_begin(st, "pack", l);
    if ((g.B >> (L - l)) >= 32)
      hipLaunchKernelGGL(k_pack_units, dim3(unsigned(nu / 7)), dim3(256), 0, st, pack_args(a, l));
    else if ((g.B >> (L - l)) == 16)
      hipLaunchKernelGGL(k_pack_blocks16, dim3(unsigned(nu / 7)), dim3(256), 0, st,
                         pack_args(a, l));
    else  // at most 28 lanes: one-wave work-groups
      hipLaunchKernelGGL(k_pack_lanes, dim3(unsigned(nu / 7)), dim3(64), 0, st, pack_args(a, l));
    prof_end(st);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_compress(const CompressArgs& a, hipStream_t st) {
  return a.vb == 8 ? launch_compress_t<double>(a, st) : launch_compress_t<float>(a, st);
}

namespace {

// Order-independent digest of a byte range (whole 32-bit words; a partial
// last word is zero-padded): the sum over words of a mix of (value, index).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_hash(const uint8_t* p, uint64_t bytes, unsigned long long* out) {
  uint64_t acc = 0;
  const uint64_t nw = (bytes + 3) / 4;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nw;
       i += uint64_t(gridDim.x) * blockDim.x) {
    uint32_t w = 0;
    for (int k = 0; k < 4; ++k)
      if (4 * i + k < bytes) w |= uint32_t(p[4 * i + k]) << (8 * k);
    acc += mix64((uint64_t(w) << 32) ^ (i * 0x9e3779b97f4a7c15ull));
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}

__global__ void k_clear64(unsigned long long* p, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

}  // namespace

hipError_t launch_hash(const void* const* ptrs, const uint64_t* bytes, uint64_t n,
                       unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_clear64, dim3(grid_for(n, 256, 256)), dim3(256), 0, st, out, n);
  for (uint64_t i = 0; i < n; ++i)
    if (bytes[i])
      hipLaunchKernelGGL(k_hash, dim3(grid_for((bytes[i] + 3) / 4, 256, 1024)), dim3(256), 0, st,
                         static_cast<const uint8_t*>(ptrs[i]), bytes[i], out + i);
  return hipGetLastError();
}

hipError_t launch_compress_batch(const CompressBatch& b, hipStream_t st) {
  // jobs that fill the GPU by themselves: their plain launch sequence
  for (uint32_t i = 0; i < b.n_whole; ++i) {
    const hipError_t e = launch_compress(b.host_J[b.whole[i]], st);
    if (e != hipSuccess) return e;
  }
  const BatchArgLayout lay(b.njobs, b.max_levels);
  const unsigned G = b.grid;
  auto grid = [&](const ItemMap& m, uint32_t total) {
    return dim3(std::max(1u, std::min<unsigned>(G, total)));
  };
  prof_begin(st, "b_init", -1);
  hipLaunchKernelGGL(kb_init, grid(b.jobs1, b.n_jobs1), dim3(256), 0, st, b.J, b.jobs1);
  hipLaunchKernelGGL(kb_hzero, grid(b.hzero, b.n_hzero), dim3(256), 0, st, b.J, b.hzero);
  prof_end(st);
  if (b.n_minmax) {
    prof_begin(st, "b_minmax", -1);
    hipLaunchKernelGGL(kb_minmax, grid(b.minmax, b.n_minmax), dim3(256), 0, st, b.J, b.minmax);
    prof_end(st);
  }
  prof_begin(st, "b_resolve", -1);
  hipLaunchKernelGGL(kb_resolve, grid(b.jobs1, b.n_jobs1), dim3(64), 0, st, b.J, b.jobs1);
  prof_end(st);
  prof_begin(st, "b_anchor", -1);
  hipLaunchKernelGGL(kb_anchor, grid(b.anchor, b.n_anchor), dim3(256), 0, st, b.J, b.anchor);
  prof_end(st);
  for (int l = 1; l <= b.max_levels; ++l) {
    // jobs with many large blocks at this level: the plain launch
    for (uint32_t i = 0; i < b.n_pdirect; ++i) {
      if (b.pdirect[i].level != l) continue;
      const CompressArgs& a = b.host_J[b.pdirect[i].job];
      const PredSlabArgs p = pred_args(a, l);
      const int64_t nblk = a.geo.nb[0] * a.geo.nb[1] * a.geo.nb[2];
      prof_begin(st, "b_predict_direct", l);
      if ((a.geo.B >> (a.geo.L - l)) == 32)
        launch_pred<float, 32>(p, nblk, st);
      else
        launch_pred<float, 64>(p, nblk, st);
      prof_end(st);
    }
    for (int e = 0; e < kBatchEdges; ++e) {
      const ItemMap& m = b.pred[l][e];
      if (!b.n_pred[l][e]) continue;
      const unsigned gp = std::max(1u, std::min<unsigned>(b.grid_pred[e], b.n_pred[l][e]));
      prof_begin(st, "b_predict", l);
      const int h = b.pred_h[e];
      const PredSlabArgs* P = reinterpret_cast<const PredSlabArgs*>(b.args + lay.pred) +
                              uint64_t(l - 1) * b.njobs;
      switch (e) {
        case 1: launch_pred_bh<2>(h, P, m, gp, st); break;
        case 2: launch_pred_bh<4>(h, P, m, gp, st); break;
        case 3: launch_pred_bh<8>(h, P, m, gp, st); break;
        case 4: launch_pred_bh<16>(h, P, m, gp, st); break;
        case 5: launch_pred_bh<32>(h, P, m, gp, st); break;
        default: launch_pred_bh<64>(h, P, m, gp, st); break;
      }
      prof_end(st);
    }
  }
  prof_begin(st, "b_hist", -1);
  hipLaunchKernelGGL(kb_hred, grid(b.hred, b.n_hred), dim3(256), 0, st, b.J, b.hred);
  prof_end(st);
  launch_codebook_batch(b.J, b.njobs, st);
  for (int l = 1; l <= b.max_levels; ++l) {
    prof_begin(st, "b_lanelen", l);
    hipLaunchKernelGGL(kb_lanelen, grid(b.level[l], b.n_level[l]), dim3(256), 0, st,
                       reinterpret_cast<const LaneLenArgs*>(b.args + lay.lane) +
                           uint64_t(l - 1) * b.njobs,
                       b.level[l]);
    prof_end(st);
  }
  prof_begin(st, "b_scan", -1);
  hipLaunchKernelGGL(kb_scan_a, grid(b.scan_ac, b.n_scan_ac), dim3(256), 0, st, b.J, b.scan_ac);
  hipLaunchKernelGGL(kb_scan_b, grid(b.scan_b, b.n_scan_b), dim3(256), 0, st, b.J, b.scan_b);
  hipLaunchKernelGGL(kb_scan_c, grid(b.scan_ac, b.n_scan_ac), dim3(256), 0, st, b.J, b.scan_ac);
  prof_end(st);
  prof_begin(st, "b_layout", -1);
  hipLaunchKernelGGL(kb_layout, grid(b.jobs1, b.n_jobs1), dim3(64), 0, st, b.J, b.jobs1);
  hipLaunchKernelGGL(kb_zero, grid(b.zero, b.n_zero), dim3(256), 0, st, b.J, b.zero);
  hipLaunchKernelGGL(kb_fill_head, grid(b.head, b.n_head), dim3(256), 0, st, b.J, b.head);
  prof_end(st);
  for (int l = 1; l <= b.max_levels; ++l) {
    prof_begin(st, "b_pack", l);
    const PackArgs* K = reinterpret_cast<const PackArgs*>(b.args + lay.pack) +
                        uint64_t(l - 1) * b.njobs;
    if (b.n_pack_u[l])
      hipLaunchKernelGGL(kb_pack_units, grid(b.pack_u[l], b.n_pack_u[l]), dim3(256), 0, st, K,
                         b.pack_u[l]);
    if (b.n_pack_l[l])
      hipLaunchKernelGGL(kb_pack_lanes, grid(b.pack_l[l], b.n_pack_l[l]), dim3(256), 0, st, K,
                         b.pack_l[l]);
    prof_end(st);
  }
  return hipGetLastError();
}

}  // namespace stz
