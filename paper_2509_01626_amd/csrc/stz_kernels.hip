// HIP kernels of the STZ hot path for gfx950 (wave64).
//
// Compression: range reduction and bound resolution, anchors, per-level
// predict+quantize (Sec. 3.1 Eqs. 3-8, Optimizations 3 and 5), histogram,
// on-device canonical Huffman code book, per-lane code lengths, segmented
// scans for the stream layout, bit packing and outlier compaction.
// Decompression: per-level decode+reconstruct over the dependency cone of a
// box (Sec. 3.3), which covers full, progressive and region decoding.
//
// Float32 arithmetic follows the format's evaluation order exactly; the file
// is compiled with -ffp-contract=off and without fast-math or denormal
// flushing, so the results are bit-identical to any other IEEE implementation
// of the same sequence.

#include "stz_internal.h"

namespace stz {

void prof_begin(hipStream_t st, const char* name, int level);
void prof_end(hipStream_t st);

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

// ---------------------------------------------------------------------------
// Compression kernels
// ---------------------------------------------------------------------------
__global__ void k_init(DevParams* P, unsigned long long* hist, int nsym) {
  const int t = threadIdx.x;
  if (t == 0) {
    P->flags = 0;
    P->total = 0;
  }
  for (int i = t; i < nsym; i += blockDim.x) hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ x, uint64_t N,
                                                float2* part, DevParams* P) {
  float mn = INFINITY, mx = -INFINITY;
  bool bad = false;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
    const float v = x[i];
    bad |= !isfinite(v);
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o, kWave));
    mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
  }
  __shared__ float smn[4], smx[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smn[w] = mn;
    smx[w] = mx;
  }
  if (bad) atomicOr(&P->flags, kFlagNonfinite);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mn = fminf(mn, smn[i]);
      mx = fmaxf(mx, smx[i]);
    }
    part[blockIdx.x] = make_float2(mn, mx);
  }
}

// Resolve the absolute bound and the per-level constants (format 2.3).
__global__ void k_resolve(DevParams* P, const float2* part, uint32_t nparts, int mode, double eb,
                          double ratio, int L) {
  if (threadIdx.x != 0) return;
  double eb_abs = eb;
  if (mode == 1) {
    float mn = part[0].x, mx = part[0].y;
    for (uint32_t i = 1; i < nparts; ++i) {
      mn = fminf(mn, part[i].x);
      mx = fmaxf(mx, part[i].y);
    }
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
  }
}

// Anchors: the stride-2^L grid, copied verbatim into the level-0 grid.
__global__ void k_anchor(const float* __restrict__ x, Geo g, float* rec0, DevParams* P) {
  const int logs = g.L;
  const int64_t c0 = ((g.n[0] - 1) >> logs) + 1, c1 = ((g.n[1] - 1) >> logs) + 1,
                c2 = ((g.n[2] - 1) >> logs) + 1;
  const int64_t na = c0 * c1 * c2;
  bool bad = false;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < na;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t ix = i % c2, t = i / c2, iy = t % c1, iz = t / c1;
    const float v = x[((iz << logs) * g.n[1] + (iy << logs)) * g.n[2] + (ix << logs)];
    bad |= !isfinite(v);
    rec0[i] = v;
  }
  if (bad) atomicOr(&P->flags, kFlagNonfinite);
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

struct PredictArgs {
  const float* x;
  Geo g;
  int level, logs;
  const float* prev;
  Grid gprev;
  float* cur;  // null at the finest level
  Grid gcur;
  uint16_t* sym;
  uint64_t nu;
  const DevParams* P;
  DevParams* Pw;
  unsigned long long* hist;
  int nsym;
};

// Predict and quantize every level-l point (one wave per unit).
__global__ __launch_bounds__(256) void k_predict(PredictArgs a) {
  __shared__ uint32_t h[2 * kMaxRadius];
  for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / kWave);
  const float E2 = a.P->E2[a.level], INV = a.P->INV[a.level];
  const double e = a.P->e[a.level];
  const int R = a.g.R;
  bool bad = false;
  for (int64_t u = int64_t(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); u < int64_t(a.nu);
       u += nwaves) {
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    const uint32_t M1 = ug.M[1], M2 = ug.M[2];
    const uint32_t nsu = uint32_t(ug.M[0]) * M1 * M2;
    const uint64_t base = unit_sym_off(a.g, a.logs, u);
    for (uint32_t r = lane; r < nsu; r += kWave) {
      const uint32_t vx = r % M2, t = r / M2, vy = t % M1, vz = t / M1;
      const int64_t p[3] = {(ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs),
                            (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs),
                            (ug.b[2] << a.g.logB) + (int64_t(2 * vx + ug.o[2]) << a.logs)};
      const float xv = a.x[(p[0] * a.g.n[1] + p[1]) * a.g.n[2] + p[2]];
      bad |= !isfinite(xv);
      const float pred = predict_point(p, a.logs, a.g.n, ug.o, [&](int64_t z, int64_t y, int64_t x) {
        return a.prev[gidx(a.gprev, z, y, x)];
      });
      float rv;
      const int sy = quantize(xv, pred, E2, INV, e, R, &rv);
      a.sym[base + r] = (uint16_t)sy;
      if (a.cur) a.cur[gidx(a.gcur, p[0], p[1], p[2])] = rv;
      atomicAdd(&h[sy], 1u);
    }
  }
  if (bad) atomicOr(&a.Pw->flags, kFlagNonfinite);
  __syncthreads();
  for (int i = threadIdx.x; i < a.nsym; i += blockDim.x)
    if (h[i]) atomicAdd(&a.hist[i], (unsigned long long)h[i]);
}

// ---------------------------------------------------------------------------
// Code book (format 2.4), one work-group of 1024 threads.
// ---------------------------------------------------------------------------
constexpr int kCbThreads = 1024;
constexpr int kCbMax = 2 * kMaxRadius;  // alphabet

// Ascending bitonic sort of n (power of two) 64-bit keys in LDS.
__device__ void bitonic_sort(uint64_t* k, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == up) {
          k[lo] = b;
          k[hi] = a;
        }
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kCbThreads) void k_codebook(const unsigned long long* hist, int nsym,
                                                         uint8_t* lens_out, uint16_t* codes_out) {
  __shared__ uint64_t buf[2 * kCbMax];         // sort keys, then node weights
  __shared__ uint16_t leaf_sym[kCbMax];
  __shared__ uint16_t par[2 * kCbMax];
  __shared__ uint16_t dep[2 * kCbMax];
  __shared__ uint8_t lens[kCbMax];
  __shared__ uint64_t cnt[kCbMax];
  __shared__ int s_m, s_maxlen;
  __shared__ uint32_t bl[kLmax + 2];
  const int t = threadIdx.x;
  int np2 = 1;
  while (np2 < nsym) np2 <<= 1;
  for (int i = t; i < nsym; i += blockDim.x) cnt[i] = hist[i];
  __syncthreads();
  for (;;) {
    // Sort used symbols by (count, symbol); unused ones go last.
    for (int i = t; i < np2; i += blockDim.x)
      buf[i] = (i < nsym && cnt[i]) ? ((cnt[i] << 11) | uint64_t(i)) : ~uint64_t(0);
    for (int i = t; i < nsym; i += blockDim.x) lens[i] = 0;
    if (t == 0) s_m = 0;
    __syncthreads();
    for (int i = t; i < nsym; i += blockDim.x)
      if (cnt[i]) atomicAdd(&s_m, 1);
    bitonic_sort(buf, np2);
    const int m = s_m;
    if (m <= 1) {
      if (m == 1 && t == 0) lens[buf[0] & 2047] = 1;
      __syncthreads();
      break;
    }
    for (int i = t; i < m; i += blockDim.x) {
      leaf_sym[i] = uint16_t(buf[i] & 2047);
      buf[i] = buf[i] >> 11;
    }
    __syncthreads();
    // Two-queue merge (serial).
    if (t == 0) {
      int li = 0, ii = m, next = m;
      uint64_t lw = buf[0];
      uint64_t iw = 0;
      for (int k = 0; k < m - 1; ++k) {
        int a, b;
        uint64_t aw, bw;
        if (li < m && (ii == next || lw <= iw)) {
          a = li;
          aw = lw;
          ++li;
          lw = li < m ? buf[li] : 0;
        } else {
          a = ii;
          aw = iw;
          ++ii;
          iw = ii < next ? buf[ii] : 0;
        }
        if (li < m && (ii == next || lw <= iw)) {
          b = li;
          bw = lw;
          ++li;
          lw = li < m ? buf[li] : 0;
        } else {
          b = ii;
          bw = iw;
          ++ii;
          iw = ii < next ? buf[ii] : 0;
        }
        const uint64_t nw = aw + bw;
        buf[next] = nw;
        par[a] = uint16_t(next);
        par[b] = uint16_t(next);
        if (ii == next) iw = nw;
        ++next;
      }
      par[2 * m - 2] = uint16_t(2 * m - 2);
    }
    __syncthreads();
    // Depths by pointer jumping.
    const int nn = 2 * m - 1;
    for (int i = t; i < nn; i += blockDim.x) dep[i] = (i == nn - 1) ? 0 : 1;
    __syncthreads();
    for (int round = 0; (1 << round) < nn; ++round) {
      uint16_t nd[2 * kCbMax / kCbThreads], npr[2 * kCbMax / kCbThreads];
      int j = 0;
      for (int i = t; i < nn; i += blockDim.x, ++j) {
        const int p = par[i];
        nd[j] = dep[i] + dep[p];
        npr[j] = par[p];
      }
      __syncthreads();
      j = 0;
      for (int i = t; i < nn; i += blockDim.x, ++j) {
        dep[i] = nd[j];
        par[i] = npr[j];
      }
      __syncthreads();
    }
    if (t == 0) s_maxlen = 0;
    __syncthreads();
    for (int i = t; i < m; i += blockDim.x) atomicMax(&s_maxlen, int(dep[i]));
    __syncthreads();
    if (s_maxlen <= kLmax) {
      for (int i = t; i < m; i += blockDim.x) lens[leaf_sym[i]] = uint8_t(dep[i]);
      __syncthreads();
      break;
    }
    for (int i = t; i < nsym; i += blockDim.x)
      if (cnt[i]) cnt[i] = (cnt[i] + 1) >> 1;
    __syncthreads();
  }
  // Canonical codes: rank of (length, symbol) among used symbols.
  if (t < kLmax + 2) bl[t] = 0;
  __syncthreads();
  for (int i = t; i < nsym; i += blockDim.x)
    if (lens[i]) atomicAdd(&bl[lens[i]], 1u);
  for (int i = t; i < np2; i += blockDim.x)
    buf[i] = (i < nsym && lens[i]) ? ((uint64_t(lens[i]) << 11) | uint64_t(i)) : ~uint64_t(0);
  bitonic_sort(buf, np2);
  __shared__ uint32_t first[kLmax + 1], start[kLmax + 1];
  if (t == 0) {
    uint32_t code = 0, st = 0;
    for (int l = 1; l <= kLmax; ++l) {
      code = (code + bl[l - 1]) << 1;
      first[l] = code;
      start[l] = st;
      st += bl[l];
    }
  }
  __syncthreads();
  for (int i = t; i < nsym; i += blockDim.x) {
    lens_out[i] = lens[i];
    codes_out[i] = 0;
  }
  __syncthreads();
  for (int i = t; i < np2; i += blockDim.x) {
    const uint64_t k = buf[i];
    if (k == ~uint64_t(0)) continue;
    const int l = int(k >> 11), sy = int(k & 2047);
    codes_out[sy] = uint16_t(first[l] + (uint32_t(i) - start[l]));
  }
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

// Bit length of every lane stream and per-unit totals.
__global__ __launch_bounds__(256) void k_lanelen(LaneLenArgs a) {
  __shared__ uint8_t L[2 * kMaxRadius];
  for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) L[i] = a.lens[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / kWave);
  for (int64_t u = int64_t(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); u < int64_t(a.nu);
       u += nwaves) {
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    const uint32_t rows = uint32_t(ug.M[0]) * ug.M[1], Mx = ug.M[2];
    const uint64_t base = unit_sym_off(a.g, a.logs, u);
    uint32_t bits = 0, no = 0;
    if (lane < int(Mx)) {
      for (uint32_t t = 0; t < rows; ++t) {
        const uint16_t s = a.sym[base + uint64_t(t) * Mx + lane];
        bits += L[s];
        no += (s == 0);
      }
      a.lane_len[unit_lane_off(a.g, a.logs, u) + lane] = uint16_t(bits);
    }
    const uint32_t tb = wave_sum(bits), to = wave_sum(no);
    if (lane == 0) {
      a.cnt_words[u] = (tb + 31) >> 5;
      a.cnt_outl[u] = to;
    }
  }
}

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

__global__ __launch_bounds__(256) void k_scan_a(const uint32_t* in, uint64_t n, uint64_t* part,
                                                int nblk) {
  const int seg = blockIdx.y;
  const uint32_t* src = in + uint64_t(seg) * n;
  const uint64_t base = uint64_t(blockIdx.x) * kScanBlock + uint64_t(threadIdx.x) * kScanItems;
  uint64_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += src[base + i];
  uint64_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[uint64_t(seg) * nblk + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_b(uint64_t* part, int nblk) {
  uint64_t* p = part + uint64_t(blockIdx.x) * nblk;
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

__global__ __launch_bounds__(256) void k_scan_c(const uint32_t* in, uint64_t n, const uint64_t* part,
                                                int nblk, uint32_t* out, DevParams* P) {
  const int seg = blockIdx.y;
  const uint32_t* src = in + uint64_t(seg) * n;
  uint32_t* dst = out + uint64_t(seg) * (n + 1);
  const uint64_t base = uint64_t(blockIdx.x) * kScanBlock + uint64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? src[base + i] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = part[uint64_t(seg) * nblk + blockIdx.x] + block_excl_scan(s, &tot);
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

struct LayoutArgs {
  Geo g;
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
__global__ void k_layout(LayoutArgs a) {
  if (threadIdx.x != 0) return;
  DevParams* P = a.P;
  const int L = a.g.L;
  const uint64_t anchor_off = kHeaderBytes + align16(uint64_t(2 * a.g.R));
  uint64_t pos = anchor_off + align16(4 * a.n_anchor);
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
    pos = P->off_out[l] + align16(4 * O);
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
  st64(o + 56, __double_as_longlong(a.eb));
  st64(o + 64, __double_as_longlong(P->eb_abs));
  st64(o + 72, __double_as_longlong(a.ratio));
  st64(o + 80, pos);
  st64(o + 88, kHeaderBytes);
  st64(o + 96, anchor_off);
  st64(o + 104, a.n_anchor);
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

// Zero [from, total) of the stream (padding and the words packed with atomics).
__global__ void k_zero(uint8_t* out, uint64_t from, const DevParams* P) {
  if (P->flags) return;
  const uint64_t to = P->total;
  uint4* p = reinterpret_cast<uint4*>(out);
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (uint64_t i = from / 16 + uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < to / 16;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = z;
}

// Code lengths and anchors into the stream.
__global__ void k_fill_head(uint8_t* out, const uint8_t* lens, int nsym, const float* rec0,
                            uint64_t na, const DevParams* P) {
  if (P->flags) return;
  const uint64_t anchor_off = kHeaderBytes + align16(uint64_t(nsym));
  float* an = reinterpret_cast<float*>(out + anchor_off);
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < na + uint64_t(nsym);
       i += uint64_t(gridDim.x) * blockDim.x) {
    if (i < uint64_t(nsym))
      out[kHeaderBytes + i] = lens[i];
    else
      an[i - nsym] = rec0[i - nsym];
  }
}

struct PackArgs {
  const float* x;
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

__device__ inline void emit_word(uint32_t* pay, uint64_t wi, uint32_t w, uint64_t start,
                                 uint64_t end) {
  if (wi * 32 >= start && wi * 32 + 32 <= end)
    pay[wi] = w;
  else if (w)
    atomicOr(&pay[wi], w);
}

// Bit-pack every lane stream, write the unit index and the outliers.
__global__ __launch_bounds__(256) void k_pack(PackArgs a) {
  const DevParams* P = a.P;
  if (P->flags) return;
  __shared__ uint8_t Ls[2 * kMaxRadius];
  __shared__ uint16_t Cs[2 * kMaxRadius];
  for (int i = threadIdx.x; i < a.nsym; i += blockDim.x) {
    Ls[i] = a.lens[i];
    Cs[i] = a.codes[i];
  }
  __syncthreads();
  const int l = a.level;
  uint32_t* unit_word = reinterpret_cast<uint32_t*>(a.out + P->sec[l]);
  uint32_t* unit_outl = reinterpret_cast<uint32_t*>(a.out + P->off_outl[l]);
  uint16_t* lane_arr = reinterpret_cast<uint16_t*>(a.out + P->off_lane[l]);
  uint32_t* pay = reinterpret_cast<uint32_t*>(a.out + P->off_pay[l]);
  float* outv = reinterpret_cast<float*>(a.out + P->off_out[l]);
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / kWave);
  for (int64_t u = int64_t(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); u < int64_t(a.nu);
       u += nwaves) {
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    const uint32_t M1 = ug.M[1], Mx = ug.M[2], rows = uint32_t(ug.M[0]) * M1;
    const bool act = lane < int(Mx);
    const uint64_t lane0 = unit_lane_off(a.g, a.logs, u);
    const uint32_t lb = act ? a.lane_len[lane0 + lane] : 0;
    const uint32_t pre = wave_excl_scan(lb, lane);
    const uint32_t uw = a.scan_words[u], uo = a.scan_outl[u];
    if (lane == 0) {
      unit_word[u] = uw;
      unit_outl[u] = uo;
      if (u == int64_t(a.nu) - 1) {
        unit_word[a.nu] = a.scan_words[a.nu];
        unit_outl[a.nu] = a.scan_outl[a.nu];
      }
    }
    if (act) lane_arr[lane0 + lane] = uint16_t(lb);
    const uint64_t start = uint64_t(uw) * 32 + pre, end = start + lb;
    uint64_t pos = start;
    uint32_t cur = 0;
    uint32_t run = 0;
    const uint64_t base = unit_sym_off(a.g, a.logs, u);
    for (uint32_t t = 0; t < rows; ++t) {
      const uint16_t s = act ? a.sym[base + uint64_t(t) * Mx + lane] : uint16_t(1);
      if (act) {
        const uint32_t len = Ls[s], c = Cs[s];
        const uint32_t o = uint32_t(pos & 31);
        if (o + len <= 32) {
          cur |= c << (32 - o - len);
          pos += len;
          if ((pos & 31) == 0) {
            emit_word(pay, (pos >> 5) - 1, cur, start, end);
            cur = 0;
          }
        } else {
          const uint32_t hi = len - (32 - o);
          cur |= c >> hi;
          emit_word(pay, pos >> 5, cur, start, end);
          cur = c << (32 - hi);
          pos += len;
        }
      }
      const bool is_out = act && s == 0;
      const uint64_t m = __ballot(is_out);
      if (is_out) {
        const uint32_t vy = t % M1, vz = t / M1;
        const int64_t pz = (ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs);
        const int64_t py = (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs);
        const int64_t px = (ug.b[2] << a.g.logB) + (int64_t(2 * lane + ug.o[2]) << a.logs);
        outv[uo + run + __popcll(m & lt_mask)] = a.x[(pz * a.g.n[1] + py) * a.g.n[2] + px];
      }
      run += __popcll(m);
    }
    if (act && (pos & 31)) emit_word(pay, pos >> 5, cur, start, end);
  }
}

// ---------------------------------------------------------------------------
// Decoding
// ---------------------------------------------------------------------------
struct DecLevelArgs {
  const uint8_t* comp;
  Geo g;
  int level, logs;
  Box box;                  // R_k
  int64_t bb_lo[3], bb_n[3];  // blocks intersecting the box
  const float* prev;
  Grid gprev;
  float* cur;
  Grid gcur;
  const uint32_t* unit_word;
  const uint32_t* unit_outl;
  const uint16_t* lane_len;
  const uint32_t* pay;
  const float* outv;
  uint64_t words, noutl, nlanes;
  uint64_t nu;
  float E2;
  const uint16_t* lut;
  uint32_t* flags;
};

// Range of class-grid indices v with b*B + s*(2v+o) in [lo, hi).
__device__ inline void vrange(int64_t base, int o, int logs, int64_t lo, int64_t hi, int32_t M,
                              int32_t* v0, int32_t* v1) {
  // p = base + s*(2v+o) >= lo  <=>  v >= ceil((lo - base - s*o) / 2s)
  const int64_t s = int64_t(1) << logs;
  const int64_t a = lo - base - s * o;
  int64_t lo_v = a <= 0 ? 0 : (a + 2 * s - 1) >> (logs + 1);
  const int64_t b = hi - 1 - base - s * o;  // p <= hi-1
  int64_t hi_v = b < 0 ? -1 : (b >> (logs + 1));
  if (hi_v > M - 1) hi_v = M - 1;
  *v0 = int32_t(lo_v);
  *v1 = int32_t(hi_v + 1);
}

__global__ __launch_bounds__(256) void k_decode(DecLevelArgs a) {
  __shared__ uint16_t lut[1 << kLutBits];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += blockDim.x) lut[i] = a.lut[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
  const int64_t nwork = a.bb_n[0] * a.bb_n[1] * a.bb_n[2] * 7;
  const int64_t nwaves = int64_t(gridDim.x) * (blockDim.x / kWave);
  const int R = a.g.R;
  bool corrupt = false;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    corrupt = a.unit_word[0] != 0 || a.unit_outl[0] != 0 || a.unit_word[a.nu] != a.words ||
              a.unit_outl[a.nu] != a.noutl;
  for (int64_t w = int64_t(blockIdx.x) * (blockDim.x / kWave) + (threadIdx.x >> 6); w < nwork;
       w += nwaves) {
    const int64_t blk = w / 7;
    const int c = int(w - blk * 7);
    const int64_t bx = a.bb_lo[2] + blk % a.bb_n[2];
    const int64_t t1 = blk / a.bb_n[2];
    const int64_t by = a.bb_lo[1] + t1 % a.bb_n[1];
    const int64_t bz = a.bb_lo[0] + t1 / a.bb_n[1];
    const int64_t u = ((bz * a.g.nb[1] + by) * a.g.nb[2] + bx) * 7 + c;
    const UnitGeo ug = unit_geo(a.g, u, a.logs);
    const uint32_t M1 = ug.M[1], Mx = ug.M[2], rows = uint32_t(ug.M[0]) * M1;
    if (rows * Mx == 0) continue;
    int32_t vlo[3], vhi[3];
    bool any = true;
    for (int d = 0; d < 3; ++d) {
      vrange(ug.b[d] << a.g.logB, ug.o[d], a.logs, a.box.lo[d], a.box.hi[d], ug.M[d], &vlo[d],
             &vhi[d]);
      any = any && vlo[d] < vhi[d];
    }
    if (!any) continue;
    const uint32_t w0 = a.unit_word[u], w1 = a.unit_word[u + 1];
    const uint32_t o0 = a.unit_outl[u], o1 = a.unit_outl[u + 1];
    const uint64_t lane0 = unit_lane_off(a.g, a.logs, u);
    bool ok = w0 <= w1 && w1 <= a.words && o0 <= o1 && o1 <= a.noutl && lane0 + Mx <= a.nlanes;
    const bool act = lane < int(Mx);
    const uint32_t lb = (act && ok) ? a.lane_len[lane0 + lane] : 0;
    const uint32_t pre = wave_excl_scan(lb, lane);
    const uint32_t tot = wave_sum(lb);
    ok = ok && uint64_t(tot) <= uint64_t(w1 - w0) * 32 && (uint64_t(tot) + 31) / 32 == (w1 - w0);
    if (!ok) {
      corrupt = true;
      continue;
    }
    const uint64_t start = uint64_t(w0) * 32 + pre;
    // Bit window: `buf` holds `nb` valid bits, left aligned.
    uint64_t wi = start >> 5;
    uint64_t buf = 0;
    int nb = 0;
    if (act) {
      const uint32_t w = wi < a.words ? a.pay[wi] : 0;
      ++wi;
      const int sk = int(start & 31);
      buf = (uint64_t(w) << 32) << sk;
      nb = 32 - sk;
    }
    uint64_t used = 0;
    bool alive = act;
    uint32_t run = 0;
    const int64_t px = (ug.b[2] << a.g.logB) + (int64_t(2 * lane + ug.o[2]) << a.logs);
    const bool in_x = lane >= vlo[2] && lane < vhi[2];
    for (uint32_t t = 0; t < rows; ++t) {
      int sy = 1;
      if (alive) {
        if (nb < kLmax) {
          const uint32_t w = wi < a.words ? a.pay[wi] : 0;
          ++wi;
          buf |= uint64_t(w) << (32 - nb);
          nb += 32;
        }
        const uint16_t e = lut[buf >> (64 - kLutBits)];
        const int len = e >> 12;
        if (len == 0 || used + len > lb) {
          alive = false;
          corrupt = true;
        } else {
          sy = e & 4095;
          buf <<= len;
          nb -= len;
          used += len;
        }
      }
      const bool is_out = alive && sy == 0;
      const uint64_t m = __ballot(is_out);
      const uint32_t vy = t % M1, vz = t / M1;
      const bool inside = alive && in_x && int32_t(vy) >= vlo[1] && int32_t(vy) < vhi[1] &&
                          int32_t(vz) >= vlo[0] && int32_t(vz) < vhi[0];
      if (inside) {
        const int64_t p[3] = {(ug.b[0] << a.g.logB) + (int64_t(2 * vz + ug.o[0]) << a.logs),
                              (ug.b[1] << a.g.logB) + (int64_t(2 * vy + ug.o[1]) << a.logs), px};
        float val;
        if (is_out) {
          const uint64_t oi = uint64_t(o0) + run + __popcll(m & lt_mask);
          if (oi < o1) {
            val = a.outv[oi];
          } else {
            val = 0.0f;
            corrupt = true;
          }
        } else {
          const float pred = predict_point(p, a.logs, a.g.n, ug.o,
                                           [&](int64_t z, int64_t y, int64_t x) {
                                             return a.prev[gidx(a.gprev, z, y, x)];
                                           });
          const float prod = (float)(sy - R) * a.E2;
          val = pred + prod;
        }
        a.cur[gidx(a.gcur, p[0], p[1], p[2])] = val;
      }
      run += __popcll(m);
    }
    if (act && alive && used != lb) corrupt = true;
    if (uint64_t(run) != uint64_t(o1 - o0)) corrupt = true;
  }
  if (corrupt) atomicOr(a.flags, kFlagCorrupt);
}

// Anchors of the box R_0 from the stream into the level-0 box grid.
__global__ void k_dec_anchor(const uint8_t* comp, uint64_t anchor_off, Geo g, float* rec0,
                             Grid g0) {
  const int logs = g.L;
  const int64_t c1 = ((g.n[1] - 1) >> logs) + 1, c2 = ((g.n[2] - 1) >> logs) + 1;
  const float* an = reinterpret_cast<const float*>(comp + anchor_off);
  const int64_t n = g0.cnt[0] * g0.cnt[1] * g0.cnt[2];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t ix = i % g0.cnt[2], t = i / g0.cnt[2], iy = t % g0.cnt[1], iz = t / g0.cnt[1];
    const int64_t z = g0.first[0] + (iz << logs), y = g0.first[1] + (iy << logs),
                  x = g0.first[2] + (ix << logs);
    rec0[i] = an[((z >> logs) * c1 + (y >> logs)) * c2 + (x >> logs)];
  }
}

inline int grid_for(uint64_t n, int per_block, int cap) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > uint64_t(cap)) b = cap;
  return int(b);
}

Grid full_grid(const Geo& g, int logs) {
  Grid r;
  for (int d = 0; d < 3; ++d) {
    r.first[d] = 0;
    r.cnt[d] = ((g.n[d] - 1) >> logs) + 1;
  }
  r.logs = logs;
  return r;
}

Grid box_grid(const Box& b, int logs) {
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

// ---------------------------------------------------------------------------
// Launch sequences
// ---------------------------------------------------------------------------
hipError_t launch_compress(const CompressArgs& a, hipStream_t st) {
  const Geo& g = a.geo;
  const int L = g.L;
  const int nsym = 2 * g.R;
  const uint64_t N = uint64_t(g.n[0]) * g.n[1] * g.n[2];
  const uint64_t nu = a.lc[1].nu;
  prof_begin(st, "init", -1);
  hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, st, a.params, a.hist, nsym);
  prof_end(st);
  if (a.eb_mode == 1) {
    prof_begin(st, "minmax", -1);
    hipLaunchKernelGGL(k_minmax, dim3(a.nparts), dim3(256), 0, st, a.x, N, a.part, a.params);
    prof_end(st);
  }
  prof_begin(st, "resolve", -1);
  hipLaunchKernelGGL(k_resolve, dim3(1), dim3(64), 0, st, a.params, a.part, a.nparts, a.eb_mode,
                     a.eb, a.ratio, L);
  prof_end(st);
  prof_begin(st, "anchor", -1);
  hipLaunchKernelGGL(k_anchor, dim3(grid_for(a.n_anchor, 256, 4096)), dim3(256), 0, st, a.x, g,
                     a.rec[0], a.params);
  prof_end(st);
  for (int l = 1; l <= L; ++l) {
    const int logs = L - l;
    if (l >= 2) {
      const Grid gs = full_grid(g, logs + 2), gd = full_grid(g, logs + 1);
      const uint64_t n = uint64_t(gs.cnt[0]) * gs.cnt[1] * gs.cnt[2];
      prof_begin(st, "upcopy", l);
      hipLaunchKernelGGL(k_upcopy, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, a.rec[l - 2], gs,
                         a.rec[l - 1], gd);
      prof_end(st);
    }
    PredictArgs p;
    p.x = a.x;
    p.g = g;
    p.level = l;
    p.logs = logs;
    p.prev = a.rec[l - 1];
    p.gprev = full_grid(g, logs + 1);
    p.cur = l < L ? a.rec[l] : nullptr;
    p.gcur = full_grid(g, logs);
    p.sym = a.sym[l];
    p.nu = nu;
    p.P = a.params;
    p.Pw = a.params;
    p.hist = a.hist;
    p.nsym = nsym;
    prof_begin(st, "predict", l);
    hipLaunchKernelGGL(k_predict, dim3(grid_for(nu, 4, 2048)), dim3(256), 0, st, p);
    prof_end(st);
  }
  prof_begin(st, "codebook", -1);
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kCbThreads), 0, st, a.hist, nsym, a.lens, a.codes);
  prof_end(st);
  for (int l = 1; l <= L; ++l) {
    LaneLenArgs q;
    q.g = g;
    q.logs = L - l;
    q.sym = a.sym[l];
    q.nu = nu;
    q.lens = a.lens;
    q.nsym = nsym;
    q.lane_len = a.lane_len + a.lane_base[l];
    q.cnt_words = a.cnt + uint64_t(2 * (l - 1)) * nu;
    q.cnt_outl = a.cnt + uint64_t(2 * (l - 1) + 1) * nu;
    prof_begin(st, "lanelen", l);
    hipLaunchKernelGGL(k_lanelen, dim3(grid_for(nu, 4, 2048)), dim3(256), 0, st, q);
    prof_end(st);
  }
  const int nblk = int((nu + kScanBlock - 1) / kScanBlock);
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
  LayoutArgs la;
  la.g = g;
  la.eb_mode = a.eb_mode;
  la.eb = a.eb;
  la.ratio = a.ratio;
  la.out_cap = a.out_cap;
  la.out = a.out;
  la.P = a.params;
  la.scan = a.scan;
  la.nu = nu;
  for (int l = 0; l <= kMaxLevels; ++l) la.lc[l] = a.lc[l];
  la.n_anchor = a.n_anchor;
  prof_begin(st, "layout", -1);
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(64), 0, st, la);
  prof_end(st);
  prof_begin(st, "zero", -1);
  hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, st, a.out, kHeaderBytes, a.params);
  prof_end(st);
  prof_begin(st, "fill_head", -1);
  hipLaunchKernelGGL(k_fill_head, dim3(grid_for(a.n_anchor + nsym, 256, 4096)), dim3(256), 0, st,
                     a.out, a.lens, nsym, a.rec[0], a.n_anchor, a.params);
  prof_end(st);
  for (int l = 1; l <= L; ++l) {
    PackArgs p;
    p.x = a.x;
    p.g = g;
    p.level = l;
    p.logs = L - l;
    p.sym = a.sym[l];
    p.nu = nu;
    p.lens = a.lens;
    p.codes = a.codes;
    p.nsym = nsym;
    p.lane_len = a.lane_len + a.lane_base[l];
    p.scan_words = a.scan + uint64_t(2 * (l - 1)) * (nu + 1);
    p.scan_outl = a.scan + uint64_t(2 * (l - 1) + 1) * (nu + 1);
    p.out = a.out;
    p.P = a.params;
    prof_begin(st, "pack", l);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nu, 4, 4096)), dim3(256), 0, st, p);
    prof_end(st);
  }
  return hipGetLastError();
}

hipError_t launch_decode(const DecodeArgs& a, hipStream_t st) {
  const Geo& g = a.geo;
  const int L = g.L;
  const int lo = a.level_out;
  const Grid g0 = box_grid(a.box[0], L);
  const uint64_t n0 = uint64_t(g0.cnt[0]) * g0.cnt[1] * g0.cnt[2];
  prof_begin(st, "dec_anchor", -1);
  hipLaunchKernelGGL(k_dec_anchor, dim3(grid_for(n0, 256, 4096)), dim3(256), 0, st, a.comp,
                     a.anchor_off, g, a.rec[0], g0);
  prof_end(st);
  for (int k = 1; k <= lo; ++k) {
    const int logs = L - k;
    const Grid gp = box_grid(a.box[k - 1], logs + 1);
    const Grid gc = box_grid(a.box[k], logs);
    const uint64_t ncopy = uint64_t(gc.cnt[0]) * gc.cnt[1] * gc.cnt[2];
    prof_begin(st, "upcopy", k);
    hipLaunchKernelGGL(k_upcopy, dim3(grid_for(ncopy / 8 + 1, 256, 8192)), dim3(256), 0, st,
                       a.rec[k - 1], gp, a.rec[k], gc);
    prof_end(st);
    DecLevelArgs d;
    d.comp = a.comp;
    d.g = g;
    d.level = k;
    d.logs = logs;
    d.box = a.box[k];
    for (int q = 0; q < 3; ++q) {
      d.bb_lo[q] = a.box[k].lo[q] >> g.logB;
      d.bb_n[q] = ((a.box[k].hi[q] - 1) >> g.logB) - d.bb_lo[q] + 1;
    }
    d.prev = a.rec[k - 1];
    d.gprev = gp;
    d.cur = a.rec[k];
    d.gcur = gc;
    d.unit_word = reinterpret_cast<const uint32_t*>(a.comp + a.sec[k]);
    d.unit_outl = reinterpret_cast<const uint32_t*>(a.comp + a.off_outl[k]);
    d.lane_len = reinterpret_cast<const uint16_t*>(a.comp + a.off_lane[k]);
    d.pay = reinterpret_cast<const uint32_t*>(a.comp + a.off_pay[k]);
    d.outv = reinterpret_cast<const float*>(a.comp + a.off_out[k]);
    d.words = a.words[k];
    d.noutl = a.outl[k];
    d.nlanes = a.lc[k].nl;
    d.nu = a.lc[k].nu;
    d.E2 = a.E2[k];
    d.lut = a.lut;
    d.flags = a.flags;
    const uint64_t nwork = uint64_t(d.bb_n[0]) * d.bb_n[1] * d.bb_n[2] * 7;
    prof_begin(st, "decode", k);
    hipLaunchKernelGGL(k_decode, dim3(grid_for(nwork, 4, 4096)), dim3(256), 0, st, d);
    prof_end(st);
  }
  return hipGetLastError();
}

}  // namespace stz
