// STZ reference oracle: a plain, slow, single-threaded CPU implementation of
// the streaming compressor's hot path.
//
// THIS FILE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it. The GPU library never
// links, includes or calls it, and it shares no code with the GPU library:
// every constant and layout rule below is written out again from the format
// specification, not taken from the GPU sources.
//
// What it computes (paper: "STZ: A High Quality and High Speed Streaming Lossy
// Compression Framework for Scientific Data", SC'25):
//   * hierarchical partition by stride-2 sampling, applied recursively, so the
//     field splits into levels (Sec. 3.1 "Hierarchical partition", Sec. 3.2);
//   * each finer point predicted only from already-reconstructed coarser points
//     by multi-dimensional interpolation: linear/bilinear/trilinear (Eqs. 3-5)
//     and the cubic forms (Eq. 6 one axis, Eq. 7 two axes, Eq. 8 three axes);
//   * the prediction difference quantized directly (Sec. 3.1, Optimization 3)
//     under a per-level error bound that is looser by a fixed ratio at the finer
//     level (Sec. 3.1, Optimization 5);
//   * Huffman coding of the quantization codes, one coding unit per sub-block
//     (Sec. 2.3 and Sec. 3.3), decodable per level (progressive, Sec. 3.3) and
//     per block (random access, Sec. 3.3);
//   * optionally (the default) a lossless zero-chunk stage ahead of the
//     Huffman coder: a run of centre codes (zero residual) covering one
//     chunk of a lane stream is coded as one extra token. The paper's
//     ratios need a stage beyond Huffman coding; this is the format's own.
// Readings where the paper is silent (boundary stencils, float evaluation order,
// quantizer parameters, the coarsest level, Huffman tie-breaks, byte layout) are
// the format's, listed with the design notes of this repository.
//
// Arithmetic: IEEE float32 in the stated evaluation order, no contraction into
// fused multiply-add (build with -ffp-contract=off), no fast-math; float64 only
// for the error-bound resolution and the final |x - x'| <= e check.
//
// Parity: pinned by the CPU test suite (stencil impulse responses against the
// printed coefficients of Eqs. 6-8, polynomial exactness, a recursive per-point
// brute force, Huffman optimality against an independent merge, round-trip,
// progressive and region invariants).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

// ----------------------------------------------------------------------------
// Format constants (written out from the format specification).
// ----------------------------------------------------------------------------
constexpr uint32_t kMagic = 0x315A5453u;  // bytes 'S','T','Z','1'
constexpr uint32_t kVersion = 1;
constexpr size_t kHeaderBytes = 512;
constexpr int kLmax = 12;          // longest Huffman code, in bits
constexpr int kMaxLevels = 8;      // level table entries in the header
constexpr size_t kLevelRec = 48;   // bytes per level-table entry
constexpr size_t kLevelTable = 128;

enum Status {
  OK = 0,
  ERR_ARG = -1,
  ERR_NONFINITE = -2,
  ERR_BUFFER = -3,
  ERR_CORRUPT = -4,
};

size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// ----------------------------------------------------------------------------
// Geometry: level grids, blocks and classes (Sec. 3.1 partition, Sec. 3.2).
// Level l in 0..L has stride s_l = 2^(L-l). Level 0 points (stride 2^L) are the
// anchors, stored verbatim. A point belongs to level l when it lies on the
// stride-s_l grid but not on the stride-2*s_l grid. Inside a block, the level-l
// points split into 7 classes by the parity of their coordinates on the
// stride-s_l grid: these are the sub-blocks b..h of Sec. 3.1 (one odd axis:
// 1,2,4; two: 3,5,6; three: 7).
// ----------------------------------------------------------------------------
struct Geo {
  size_t n[3];   // nz, ny, nx
  int B;         // block edge, power of two
  int L;         // number of levels above the anchors
  int R;         // quantization radius; alphabet has 2R symbols
  size_t nb[3];  // blocks per axis
  size_t nblocks;
  size_t N;

  size_t stride(int l) const { return size_t(1) << (L - l); }
  size_t idx(size_t z, size_t y, size_t x) const { return (z * n[1] + y) * n[2] + x; }
  // Number of multiples of s in [0, n_d).
  size_t grid_n(int d, size_t s) const { return (n[d] - 1) / s + 1; }
};

struct Unit {       // one coding unit: (level, block, class)
  size_t b[3];      // block coordinates
  int o[3];         // class parity per axis (z, y, x)
  size_t M[3];      // class sub-grid extent per axis
  size_t nsym() const { return M[0] * M[1] * M[2]; }
};

// Units of level l in stream order: blocks in raster order, classes 1..7.
std::vector<Unit> level_units(const Geo& g, int l) {
  std::vector<Unit> us;
  const size_t s = g.stride(l);
  for (size_t bz = 0; bz < g.nb[0]; ++bz)
    for (size_t by = 0; by < g.nb[1]; ++by)
      for (size_t bx = 0; bx < g.nb[2]; ++bx) {
        const size_t bb[3] = {bz, by, bx};
        size_t U[3];
        for (int d = 0; d < 3; ++d) {
          size_t lo = bb[d] * size_t(g.B);
          size_t len = std::min(size_t(g.B), g.n[d] - lo);
          U[d] = (len + s - 1) / s;  // grid points of stride s inside the block
        }
        for (int c = 1; c <= 7; ++c) {
          Unit u;
          u.o[0] = (c >> 2) & 1;
          u.o[1] = (c >> 1) & 1;
          u.o[2] = c & 1;
          for (int d = 0; d < 3; ++d) {
            u.b[d] = bb[d];
            u.M[d] = u.o[d] ? U[d] / 2 : (U[d] + 1) / 2;
          }
          us.push_back(u);
        }
      }
  return us;
}

// Full-resolution coordinate of sub-grid position v of unit u at stride s.
void unit_point(const Geo& g, const Unit& u, size_t s, size_t vz, size_t vy, size_t vx,
                size_t p[3]) {
  const size_t v[3] = {vz, vy, vx};
  for (int d = 0; d < 3; ++d) p[d] = u.b[d] * size_t(g.B) + s * (2 * v[d] + size_t(u.o[d]));
}

// ----------------------------------------------------------------------------
// Prediction from the coarser level (Sec. 3.1, Optimizations 2 and 4).
// `rec` is a full-resolution array; only stride-2s points are read.
// ----------------------------------------------------------------------------
// Values are float32 (the default) or float64 (dtype 1): the same formulas in
// the same evaluation order, with T-typed constants.
template <class T>
struct Reader {
  const T* rec;
  const Geo* g;
  bool check;     // region decode: every value read must have been reconstructed
  bool* bad;
  T at(long long z, long long y, long long x) const {
    T v = rec[g->idx(size_t(z), size_t(y), size_t(x))];
    if (check && std::isnan(v)) *bad = true;
    return v;
  }
};

// Availability flags along an odd axis d at coordinate pd (pd/s odd, so pd-s>=0).
struct AxisFlags {
  bool P1, M3, P3;
};

AxisFlags axis_flags(const Geo& g, int d, size_t pd, size_t s) {
  AxisFlags f;
  f.P1 = pd + s <= g.n[d] - 1;
  f.M3 = pd >= 3 * s;
  f.P3 = pd + 3 * s <= g.n[d] - 1;
  return f;
}

// One-axis rule used inside the nested multi-dimensional fallback: linear
// midpoint when both neighbours exist (Eq. 3), else linear extrapolation from
// the two lower neighbours, else copy of the lower neighbour (Sec. 3.1 lets
// boundary points fall back to whichever coarse neighbours exist).
template <class T, class F>
T nested_rule(const AxisFlags& f, size_t s, F val) {
  const long long ss = (long long)s;
  if (f.P1) {
    T lo = val(-ss);
    T hi = val(ss);
    return (lo + hi) * T(0.5);
  }
  if (f.M3) {
    T lo = val(-ss);
    T lo3 = val(-3 * ss);
    return ((T(3) * lo) - lo3) * T(0.5);
  }
  return val(-ss);
}

template <class T>
T predict(const Reader<T>& r, const Geo& g, const size_t p[3], size_t s) {
  int D[3];
  int nd = 0;
  for (int d = 0; d < 3; ++d)
    if ((p[d] / s) & 1) D[nd++] = d;  // odd axes in order z, y, x
  const long long pz = (long long)p[0], py = (long long)p[1], px = (long long)p[2];
  const long long ss = (long long)s;

  AxisFlags f[3];
  bool full = true;
  for (int i = 0; i < nd; ++i) {
    f[i] = axis_flags(g, D[i], p[D[i]], s);
    full = full && f[i].M3 && f[i].P1 && f[i].P3;
  }

  // Value at offset (a, b, c) along the odd axes D[0], D[1], D[2].
  auto at_off = [&](long long a, long long b, long long c) {
    long long q[3] = {pz, py, px};
    const long long off[3] = {a, b, c};
    for (int i = 0; i < nd; ++i) q[D[i]] += off[i];
    return r.at(q[0], q[1], q[2]);
  };

  if (nd == 1) {
    const AxisFlags& a = f[0];
    if (a.P1) {
      T Bv = at_off(-ss, 0, 0);
      T Cv = at_off(ss, 0, 0);
      if (a.M3 && a.P3) {
        // Eq. 6: (-1, 9, 9, -1) / 16.
        T A = at_off(-3 * ss, 0, 0);
        T Dv = at_off(3 * ss, 0, 0);
        return ((T(9) * (Bv + Cv)) - (A + Dv)) * T(0.0625);
      }
      if (!a.M3 && a.P3) {
        // Quadratic through offsets -1, +1, +3: weights 3/8, 6/8, -1/8.
        T Dv = at_off(3 * ss, 0, 0);
        return ((T(3) * Bv + T(6) * Cv) - Dv) * T(0.125);
      }
      if (a.M3 && !a.P3) {
        // Quadratic through offsets -3, -1, +1: weights -1/8, 6/8, 3/8.
        T A = at_off(-3 * ss, 0, 0);
        return ((T(6) * Bv + T(3) * Cv) - A) * T(0.125);
      }
      return (Bv + Cv) * T(0.5);  // Eq. 3
    }
    T Bv = at_off(-ss, 0, 0);
    if (a.M3) {
      T A = at_off(-3 * ss, 0, 0);
      return ((T(3) * Bv) - A) * T(0.5);
    }
    return Bv;
  }

  if (full && nd == 2) {
    // Eq. 7: mean of the two diagonal cubics: 9/32 * inner corners - 1/32 * outer.
    T in = T(0), out = T(0);
    bool first = true;
    for (int s0 = -1; s0 <= 1; s0 += 2)
      for (int s1 = -1; s1 <= 1; s1 += 2) {
        T vi = at_off(s0 * ss, s1 * ss, 0);
        T vo = at_off(3 * s0 * ss, 3 * s1 * ss, 0);
        if (first) {
          in = vi;
          out = vo;
          first = false;
        } else {
          in = in + vi;
          out = out + vo;
        }
      }
    return ((T(9) * in) - out) * T(0.03125);
  }
  if (full && nd == 3) {
    // Eq. 8: mean of the four body-diagonal cubics: 9/64 inner - 1/64 outer.
    T in = T(0), out = T(0);
    bool first = true;
    for (int s0 = -1; s0 <= 1; s0 += 2)
      for (int s1 = -1; s1 <= 1; s1 += 2)
        for (int s2 = -1; s2 <= 1; s2 += 2) {
          T vi = at_off(s0 * ss, s1 * ss, s2 * ss);
          T vo = at_off(3 * s0 * ss, 3 * s1 * ss, 3 * s2 * ss);
          if (first) {
            in = vi;
            out = vo;
            first = false;
          } else {
            in = in + vi;
            out = out + vo;
          }
        }
    return ((T(9) * in) - out) * T(0.015625);
  }

  // Multi-dimensional fallback (two or three odd axes, some cubic support
  // missing): the one-axis rule nested over the odd axes, outermost first. With
  // both neighbours present on every axis this is Eq. 4 (two axes) or Eq. 5
  // (three axes) in real arithmetic.
  if (nd == 2) {
    return nested_rule<T>(f[0], s, [&](long long a) {
      return nested_rule<T>(f[1], s, [&](long long b) { return at_off(a, b, 0); });
    });
  }
  return nested_rule<T>(f[0], s, [&](long long a) {
    return nested_rule<T>(f[1], s, [&](long long b) {
      return nested_rule<T>(f[2], s, [&](long long c) { return at_off(a, b, c); });
    });
  });
}

// ----------------------------------------------------------------------------
// Error bounds per level (Sec. 3.1, Optimization 5; Sec. 3.2). The finest level
// takes the user bound, the next coarser one the bound divided by the ratio,
// and every coarser level (the paper's coarsest level 1) that bound divided by
// the ratio once more.
// ----------------------------------------------------------------------------
struct Bounds {
  double eb_abs;
  double e[kMaxLevels + 1];
  float E2[kMaxLevels + 1];
  float INV[kMaxLevels + 1];
  double E2d[kMaxLevels + 1];    // float64 data: 2e and 1/(2e) in double
  double INVd[kMaxLevels + 1];
  double echk[kMaxLevels + 1];   // float64 data: acceptance bound e*(1 - 2^-50)
};

void level_bounds(double eb_abs, double ratio, int L, Bounds* b) {
  b->eb_abs = eb_abs;
  for (int l = 1; l <= L; ++l) {
    double e;
    if (l == L)
      e = eb_abs;
    else if (l == L - 1)
      e = eb_abs / ratio;
    else
      e = (eb_abs / ratio) / ratio;
    b->e[l] = e;
    b->E2[l] = (float)(2.0 * e);
    b->INV[l] = (float)(1.0 / (2.0 * e));
    b->E2d[l] = 2.0 * e;
    b->INVd[l] = 1.0 / (2.0 * e);
    b->echk[l] = e * (1.0 - 0x1p-50);
  }
}

// Linear-scaling quantization of the prediction difference (Sec. 2.1 step 2,
// Sec. 3.1 Optimization 3). Returns the symbol; 0 marks an outlier whose value
// is stored verbatim.
//
// float32 data: E2, INV are the float constants, the bound check |x - xr| <= e
// is exact in double. float64 data: E2, INV in double; the check is evaluated
// in double against e*(1 - 2^-50), which keeps the exact |x - xr| <= e despite
// the rounding of the difference.
template <class T>
int quantize(T xv, T pred, const Bounds& bd, int l, int R, T* rec) {
  T E2, INV;
  if constexpr (sizeof(T) == 4) {
    E2 = bd.E2[l];
    INV = bd.INV[l];
  } else {
    E2 = bd.E2d[l];
    INV = bd.INVd[l];
  }
  T diff = xv - pred;
  T t = std::rint(diff * INV);
  if (std::fabs(t) <= (T)(R - 1)) {
    int q = (int)t;
    T prod = (T)q * E2;
    T xr = pred + prod;
    bool ok;
    if constexpr (sizeof(T) == 4)
      ok = std::fabs((double)xv - (double)xr) <= bd.e[l];
    else
      ok = std::fabs(xv - xr) <= bd.echk[l];
    if (ok) {
      *rec = xr;
      return q + R;
    }
  }
  *rec = xv;
  return 0;
}

// ----------------------------------------------------------------------------
// Huffman code lengths: two-queue construction over the used symbols sorted by
// (count, symbol); ties between the queues go to the leaf queue; internal
// nodes are taken in creation order. If the longest code exceeds kLmax, every
// nonzero count c becomes (c+1)/2 and the tree is rebuilt.
// ----------------------------------------------------------------------------
void huffman_lengths(const uint64_t* counts, int nsym, int lmax, uint8_t* lens) {
  std::vector<uint64_t> w(counts, counts + nsym);
  for (;;) {
    std::vector<int> used;
    for (int i = 0; i < nsym; ++i)
      if (w[i]) used.push_back(i);
    std::fill(lens, lens + nsym, 0);
    const int m = (int)used.size();
    if (m == 0) return;
    if (m == 1) {
      lens[used[0]] = 1;
      return;
    }
    std::sort(used.begin(), used.end(), [&](int a, int b) {
      return w[a] != w[b] ? w[a] < w[b] : a < b;
    });
    const int nn = 2 * m - 1;
    std::vector<uint64_t> wt(nn);
    std::vector<int> parent(nn, -1);
    for (int i = 0; i < m; ++i) wt[i] = w[used[i]];
    int li = 0, ii = m, next = m;
    auto pop = [&]() {
      if (li < m && (ii == next || wt[li] <= wt[ii])) return li++;
      return ii++;
    };
    for (int k = 0; k < m - 1; ++k) {
      int a = pop();
      int b = pop();
      wt[next] = wt[a] + wt[b];
      parent[a] = next;
      parent[b] = next;
      ++next;
    }
    std::vector<int> depth(nn, 0);
    for (int i = nn - 2; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
    int maxlen = 0;
    for (int i = 0; i < m; ++i) maxlen = std::max(maxlen, depth[i]);
    if (maxlen <= lmax) {
      for (int i = 0; i < m; ++i) lens[used[i]] = (uint8_t)depth[i];
      return;
    }
    for (int i = 0; i < nsym; ++i)
      if (w[i]) w[i] = (w[i] + 1) >> 1;
  }
}

// Canonical codes: ascending length, then ascending symbol.
void canonical_codes(const uint8_t* lens, int nsym, uint32_t* codes) {
  uint32_t bl_count[33] = {0};
  for (int i = 0; i < nsym; ++i)
    if (lens[i]) bl_count[lens[i]]++;
  uint32_t next_code[33] = {0};
  uint32_t code = 0;
  for (int len = 1; len <= 32; ++len) {
    code = (code + bl_count[len - 1]) << 1;
    next_code[len] = code;
  }
  for (int i = 0; i < nsym; ++i) {
    codes[i] = 0;
    if (lens[i]) codes[i] = next_code[lens[i]]++;
  }
}

// MSB-first bit string: stream bit k sits in 32-bit word k/32 at bit 31-(k%32).
struct BitWriter {
  std::vector<uint32_t>* words;
  uint64_t pos;  // bit position
  void put(uint32_t code, int len) {
    for (int i = len - 1; i >= 0; --i) {
      uint64_t w = pos >> 5;
      if (w >= words->size()) words->push_back(0);
      if ((code >> i) & 1u) (*words)[w] |= 1u << (31 - (pos & 31));
      ++pos;
    }
  }
};

// Canonical decoder walking one bit at a time: codes of length l are the
// consecutive integers first[l] .. first[l]+count[l]-1, assigned to the symbols
// of that length in ascending order.
struct Decoder {
  uint32_t first[kLmax + 1];
  uint32_t count[kLmax + 1];
  std::vector<int> by_len[kLmax + 1];
  bool build(const uint8_t* lens, int nsym) {
    std::vector<uint32_t> codes(nsym);
    for (int i = 0; i < nsym; ++i)
      if (lens[i] > kLmax) return false;
    canonical_codes(lens, nsym, codes.data());
    for (int l = 0; l <= kLmax; ++l) {
      count[l] = 0;
      first[l] = 0;
      by_len[l].clear();
    }
    for (int i = 0; i < nsym; ++i)
      if (lens[i]) {
        if (by_len[lens[i]].empty()) first[lens[i]] = codes[i];
        by_len[lens[i]].push_back(i);
        count[lens[i]]++;
      }
    return true;
  }
};

// Read one bit from a word array (MSB-first); returns -1 past the end.
inline int get_bit(const uint32_t* words, uint64_t nwords, uint64_t pos) {
  uint64_t w = pos >> 5;
  if (w >= nwords) return -1;
  return (words[w] >> (31 - (pos & 31))) & 1u;
}

// ----------------------------------------------------------------------------
// Little-endian byte helpers.
// ----------------------------------------------------------------------------
void put32(uint8_t* p, uint32_t v) { std::memcpy(p, &v, 4); }
void put64(uint8_t* p, uint64_t v) { std::memcpy(p, &v, 8); }
void putf64(uint8_t* p, double v) { std::memcpy(p, &v, 8); }
uint32_t get32(const uint8_t* p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
uint64_t get64(const uint8_t* p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}
double getf64(const uint8_t* p) {
  double v;
  std::memcpy(&v, p, 8);
  return v;
}

}  // namespace

// ============================================================================
// C interface (mirrors the library's boundary on host pointers).
// ============================================================================
extern "C" {

struct stz_ref_config {
  uint32_t block;   // B: power of two in [2, 64]; 0 selects 32
  uint32_t levels;  // L: 1..log2(B); 0 selects log2(B)
  uint32_t radius;  // R: 1..1024; 0 selects 512
  uint32_t coding;  // 1 = Huffman only, 2 = zero chunks + Huffman; 0 selects 2
  double eb_ratio;  // >= 1; 0 selects 2.5
};

struct stz_ref_info {
  uint64_t dims[3];
  uint32_t block, levels, radius, lmax, eb_mode, dtype;  // dtype: 0 float32, 1 float64
  double eb, eb_abs, eb_ratio;
  uint64_t total_bytes;
  uint32_t coding, reserved;  // coding: 1 Huffman only, 2 zero chunks
};

}  // extern "C"

namespace {

struct Cfg {
  int B, L, R;
  int coding;  // 1 Huffman only, 2 zero chunks + Huffman
  double ratio;
};

// Code alphabet: the 2R quantization symbols, plus the zero-chunk token 2R
// when that stage is on.
int alphabet(const Cfg& c) { return 2 * c.R + (c.coding == 2 ? 1 : 0); }

int resolve_cfg(const stz_ref_config* c, Cfg* out) {
  stz_ref_config d = {0, 0, 0, 0, 0.0};
  if (c) d = *c;
  int B = d.block ? (int)d.block : 32;
  if (B < 2 || B > 64 || (B & (B - 1))) return ERR_ARG;
  int k = 0;
  while ((1 << k) < B) ++k;
  int L = d.levels ? (int)d.levels : k;
  if (L < 1 || L > k) return ERR_ARG;
  int R = d.radius ? (int)d.radius : 512;
  if (R < 1 || R > 1024) return ERR_ARG;
  double ratio = d.eb_ratio != 0.0 ? d.eb_ratio : 2.5;
  if (!(ratio >= 1.0) || !std::isfinite(ratio)) return ERR_ARG;
  if (d.coding > 2) return ERR_ARG;
  out->coding = d.coding ? (int)d.coding : 2;
  out->B = B;
  out->L = L;
  out->R = R;
  out->ratio = ratio;
  return OK;
}

bool make_geo(const uint64_t dims[3], const Cfg& c, Geo* g) {
  g->N = 1;
  for (int d = 0; d < 3; ++d) {
    if (dims[d] < 1 || dims[d] > (uint64_t(1) << 32)) return false;
    g->n[d] = dims[d];
    g->N *= dims[d];
    if (g->N > (uint64_t(1) << 40)) return false;
  }
  g->B = c.B;
  g->L = c.L;
  g->R = c.R;
  g->nblocks = 1;
  for (int d = 0; d < 3; ++d) {
    g->nb[d] = (g->n[d] + c.B - 1) / c.B;
    g->nblocks *= g->nb[d];
  }
  return true;
}

size_t n_anchor(const Geo& g) {
  const size_t s = g.stride(0);
  return g.grid_n(0, s) * g.grid_n(1, s) * g.grid_n(2, s);
}

struct LevelLayout {
  size_t nu, nl, nsym;
  size_t words, outl;
  size_t vbytes = 4;  // bytes per stored value (outliers): 4 or 8
  size_t off_unit_word, off_unit_outl, off_lane, off_payload, off_outl, size;
};

void layout_level(LevelLayout* ll) {
  ll->off_unit_word = 0;
  ll->off_unit_outl = align16(4 * (ll->nu + 1));
  ll->off_lane = ll->off_unit_outl + align16(4 * (ll->nu + 1));
  ll->off_payload = ll->off_lane + align16(2 * ll->nl);
  ll->off_outl = ll->off_payload + align16(4 * ll->words);
  ll->size = ll->off_outl + align16(ll->vbytes * ll->outl);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

uint64_t compress_bound_impl(const uint64_t dims[3], const stz_ref_config* cfg, size_t vb) {
  Cfg c;
  Geo g;
  if (resolve_cfg(cfg, &c) != OK || !make_geo(dims, c, &g)) return 0;
  size_t total = kHeaderBytes + align16(size_t(alphabet(c)));
  total += align16(vb * n_anchor(g));
  for (int l = 1; l <= c.L; ++l) {
    std::vector<Unit> us = level_units(g, l);
    LevelLayout ll;
    ll.nu = us.size();
    ll.nl = 0;
    ll.nsym = 0;
    ll.words = 0;
    for (const Unit& u : us) {
      ll.nl += u.M[2];
      ll.nsym += u.nsym();
      ll.words += (u.nsym() * kLmax + 31) / 32;
    }
    ll.outl = ll.nsym;
    ll.vbytes = vb;
    layout_level(&ll);
    total += ll.size;
  }
  return total;
}

// Compression (Sec. 3.1-3.2 prediction and quantization, Huffman coding per
// sub-block). Writes the stream to `out` (host memory). T = float (value type
// 0) or double (value type 1).
template <class T>
int compress_impl(const T* x, const uint64_t dims[3], int eb_mode, double eb,
                  const stz_ref_config* cfg, void* out, uint64_t out_cap, uint64_t* out_size) {
  constexpr size_t VB = sizeof(T);
  Cfg c;
  Geo g;
  if (!x || !dims || !out_size) return ERR_ARG;
  if (resolve_cfg(cfg, &c) != OK || !make_geo(dims, c, &g)) return ERR_ARG;
  if (eb_mode != 0 && eb_mode != 1) return ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb)) return ERR_ARG;
  for (size_t i = 0; i < g.N; ++i)
    if (!std::isfinite(x[i])) return ERR_NONFINITE;

  // Resolve the absolute bound: a value-range-relative bound scales by max-min.
  double eb_abs = eb;
  if (eb_mode == 1) {
    T mn = x[0], mx = x[0];
    for (size_t i = 1; i < g.N; ++i) {
      mn = std::min(mn, x[i]);
      mx = std::max(mx, x[i]);
    }
    double range = (double)mx - (double)mn;
    if (range > 0.0)
      eb_abs = eb * range;
    else
      eb_abs = eb * (std::fabs((double)mn) > 0.0 ? std::fabs((double)mn) : 1.0);
  }
  if (!(eb_abs > 0.0) || !std::isfinite(eb_abs)) return ERR_ARG;
  Bounds bd;
  level_bounds(eb_abs, c.ratio, c.L, &bd);

  // Anchors: the stride-2^L grid, stored verbatim (replaces the paper's
  // separately coded coarsest level).
  std::vector<T> rec(g.N, T(0));
  const size_t s0 = g.stride(0);
  std::vector<T> anchors;
  for (size_t z = 0; z < g.n[0]; z += s0)
    for (size_t y = 0; y < g.n[1]; y += s0)
      for (size_t xx = 0; xx < g.n[2]; xx += s0) {
        size_t i = g.idx(z, y, xx);
        rec[i] = x[i];
        anchors.push_back(x[i]);
      }

  // Predict and quantize level by level, coarse to fine (Sec. 3.2).
  const int nsym = alphabet(c);
  const int Z = 2 * c.R;  // zero-chunk token (when coding == 2)
  std::vector<uint64_t> hist(nsym, 0);
  std::vector<std::vector<uint16_t>> syms(c.L + 1);
  std::vector<std::vector<T>> outl(c.L + 1);
  std::vector<std::vector<Unit>> units(c.L + 1);
  Reader<T> rd{rec.data(), &g, false, nullptr};
  for (int l = 1; l <= c.L; ++l) {
    const size_t s = g.stride(l);
    units[l] = level_units(g, l);
    for (const Unit& u : units[l])
      for (size_t vz = 0; vz < u.M[0]; ++vz)
        for (size_t vy = 0; vy < u.M[1]; ++vy)
          for (size_t vx = 0; vx < u.M[2]; ++vx) {
            size_t p[3];
            unit_point(g, u, s, vz, vy, vx, p);
            size_t i = g.idx(p[0], p[1], p[2]);
            T pred = predict(rd, g, p, s);
            T r;
            int sym = quantize(x[i], pred, bd, l, c.R, &r);
            rec[i] = r;
            if (sym == 0) outl[l].push_back(x[i]);
            syms[l].push_back((uint16_t)sym);
          }
  }

  // Tokens: lane j of a unit lists its symbols in (v_z, v_y) order; a chunk
  // is the M_y symbols of one v_z. With zero chunks on, a nonempty chunk whose
  // symbols are all the centre symbol R is one token Z; every other symbol is
  // its own token. The histogram counts tokens.
  auto chunk_is_zero = [&](int l, size_t base, const Unit& u, size_t j, size_t vz) {
    if (c.coding != 2 || u.M[1] == 0) return false;  // empty chunks have no token
    for (size_t vy = 0; vy < u.M[1]; ++vy)
      if (syms[l][base + (vz * u.M[1] + vy) * u.M[2] + j] != (uint16_t)c.R) return false;
    return true;
  };
  for (int l = 1; l <= c.L; ++l) {
    size_t base = 0;
    for (const Unit& u : units[l]) {
      for (size_t j = 0; j < u.M[2]; ++j)
        for (size_t vz = 0; vz < u.M[0]; ++vz) {
          if (chunk_is_zero(l, base, u, j, vz)) {
            hist[Z]++;
          } else {
            for (size_t vy = 0; vy < u.M[1]; ++vy)
              hist[syms[l][base + (vz * u.M[1] + vy) * u.M[2] + j]]++;
          }
        }
      base += u.nsym();
    }
  }

  // Huffman codebook over all tokens of all levels.
  std::vector<uint8_t> lens(nsym);
  std::vector<uint32_t> codes(nsym);
  huffman_lengths(hist.data(), nsym, kLmax, lens.data());
  canonical_codes(lens.data(), nsym, codes.data());

  // Encode each unit: one lane stream per x-column of the class sub-grid,
  // lanes back to back, unit padded to a 32-bit word.
  struct LevelOut {
    LevelLayout ll;
    std::vector<uint32_t> unit_word, unit_outl;
    std::vector<uint16_t> lane_len;
    std::vector<uint32_t> payload;
  };
  std::vector<LevelOut> lv(c.L + 1);
  for (int l = 1; l <= c.L; ++l) {
    LevelOut& o = lv[l];
    size_t sym_base = 0, outl_base = 0;
    for (const Unit& u : units[l]) {
      o.unit_word.push_back((uint32_t)o.payload.size());
      o.unit_outl.push_back((uint32_t)outl_base);
      std::vector<uint32_t> words;
      BitWriter bw{&words, 0};
      for (size_t j = 0; j < u.M[2]; ++j) {
        uint64_t start = bw.pos;
        for (size_t vz = 0; vz < u.M[0]; ++vz) {
          if (chunk_is_zero(l, sym_base, u, j, vz)) {
            bw.put(codes[Z], lens[Z]);
            continue;
          }
          for (size_t vy = 0; vy < u.M[1]; ++vy) {
            uint16_t sy = syms[l][sym_base + (vz * u.M[1] + vy) * u.M[2] + j];
            bw.put(codes[sy], lens[sy]);
          }
        }
        uint64_t bits = bw.pos - start;
        if (bits > 0xFFFFu) return ERR_ARG;  // cannot happen for B <= 64
        o.lane_len.push_back((uint16_t)bits);
      }
      for (size_t t = 0; t < u.nsym(); ++t)
        if (syms[l][sym_base + t] == 0) ++outl_base;
      o.payload.insert(o.payload.end(), words.begin(), words.end());
      if (o.payload.size() > 0xFFFFFFFFull) return ERR_ARG;
      sym_base += u.nsym();
    }
    o.unit_word.push_back((uint32_t)o.payload.size());
    o.unit_outl.push_back((uint32_t)outl_base);
    o.ll.nu = units[l].size();
    o.ll.nl = o.lane_len.size();
    o.ll.nsym = syms[l].size();
    o.ll.words = o.payload.size();
    o.ll.outl = outl[l].size();
    o.ll.vbytes = VB;
    layout_level(&o.ll);
  }

  // Assemble the stream.
  const size_t codelen_off = kHeaderBytes;
  const size_t anchor_off = codelen_off + align16(size_t(nsym));
  size_t pos = anchor_off + align16(VB * anchors.size());
  std::vector<size_t> sec(c.L + 1, 0);
  for (int l = 1; l <= c.L; ++l) {
    sec[l] = pos;
    pos += lv[l].ll.size;
  }
  const size_t total = pos;
  *out_size = total;
  if (!out || total > out_cap) return ERR_BUFFER;
  uint8_t* o = static_cast<uint8_t*>(out);
  std::memset(o, 0, total);
  put32(o + 0, kMagic);
  put32(o + 4, kVersion);
  for (int d = 0; d < 3; ++d) put64(o + 8 + 8 * d, g.n[d]);
  put32(o + 32, (uint32_t)c.B);
  put32(o + 36, (uint32_t)c.L);
  put32(o + 40, (uint32_t)c.R);
  put32(o + 44, (uint32_t)kLmax);
  put32(o + 48, (uint32_t)eb_mode);
  put32(o + 52, VB == 8 ? 1u : 0u);  // value type: 0 float32, 1 float64
  putf64(o + 56, eb);
  putf64(o + 64, eb_abs);
  putf64(o + 72, c.ratio);
  put64(o + 80, total);
  put64(o + 88, codelen_off);
  put64(o + 96, anchor_off);
  put64(o + 104, anchors.size());
  put32(o + 112, (uint32_t)c.coding);
  for (int l = 1; l <= c.L; ++l) {
    uint8_t* e = o + kLevelTable + kLevelRec * size_t(l - 1);
    put64(e + 0, sec[l]);
    put64(e + 8, lv[l].ll.nu);
    put64(e + 16, lv[l].ll.nl);
    put64(e + 24, lv[l].ll.nsym);
    put64(e + 32, lv[l].ll.words);
    put64(e + 40, lv[l].ll.outl);
  }
  std::memcpy(o + codelen_off, lens.data(), size_t(nsym));
  std::memcpy(o + anchor_off, anchors.data(), VB * anchors.size());
  for (int l = 1; l <= c.L; ++l) {
    const LevelOut& L_ = lv[l];
    uint8_t* base = o + sec[l];
    // (an empty vector may hold no storage: copy only nonempty arrays)
    auto put = [](uint8_t* dst, const void* src, size_t bytes) {
      if (bytes) std::memcpy(dst, src, bytes);
    };
    put(base + L_.ll.off_unit_word, L_.unit_word.data(), 4 * L_.unit_word.size());
    put(base + L_.ll.off_unit_outl, L_.unit_outl.data(), 4 * L_.unit_outl.size());
    put(base + L_.ll.off_lane, L_.lane_len.data(), 2 * L_.lane_len.size());
    put(base + L_.ll.off_payload, L_.payload.data(), 4 * L_.payload.size());
    put(base + L_.ll.off_outl, outl[l].data(), VB * outl[l].size());
  }
  return OK;
}

}  // namespace

extern "C" {

uint64_t stz_ref_compress_bound(const uint64_t dims[3], const stz_ref_config* cfg) {
  return compress_bound_impl(dims, cfg, 4);
}

uint64_t stz_ref_compress_bound_f64(const uint64_t dims[3], const stz_ref_config* cfg) {
  return compress_bound_impl(dims, cfg, 8);
}

int stz_ref_compress(const float* x, const uint64_t dims[3], int eb_mode, double eb,
                     const stz_ref_config* cfg, void* out, uint64_t out_cap,
                     uint64_t* out_size) {
  return compress_impl<float>(x, dims, eb_mode, eb, cfg, out, out_cap, out_size);
}

int stz_ref_compress_f64(const double* x, const uint64_t dims[3], int eb_mode, double eb,
                         const stz_ref_config* cfg, void* out, uint64_t out_cap,
                         uint64_t* out_size) {
  return compress_impl<double>(x, dims, eb_mode, eb, cfg, out, out_cap, out_size);
}

}  // extern "C"

// ============================================================================
// Decoding (Sec. 3.3): full, progressive (stop at a level) and region.
// ============================================================================
namespace {

struct Parsed {
  Geo g;
  Cfg c;
  int dtype;      // 0 float32, 1 float64
  size_t vb;      // bytes per stored value
  int eb_mode;
  double eb, eb_abs;
  uint64_t total;
  uint64_t codelen_off, anchor_off, n_anch;
  struct Lv {
    uint64_t off, nu, nl, nsym, words, outl;
    LevelLayout ll;
  } lv[kMaxLevels + 1];
};

int parse(const void* comp, uint64_t size, Parsed* P) {
  if (!comp || size < kHeaderBytes) return ERR_CORRUPT;
  const uint8_t* b = static_cast<const uint8_t*>(comp);
  if (get32(b) != kMagic || get32(b + 4) != kVersion) return ERR_CORRUPT;
  uint64_t dims[3] = {get64(b + 8), get64(b + 16), get64(b + 24)};
  stz_ref_config cf;
  cf.block = get32(b + 32);
  cf.levels = get32(b + 36);
  cf.radius = get32(b + 40);
  cf.coding = get32(b + 112);
  cf.eb_ratio = getf64(b + 72);
  if (cf.block == 0 || cf.levels == 0 || cf.radius == 0) return ERR_CORRUPT;
  if (cf.coding != 1 && cf.coding != 2) return ERR_CORRUPT;
  if (get32(b + 44) != (uint32_t)kLmax) return ERR_CORRUPT;
  if (resolve_cfg(&cf, &P->c) != OK || !make_geo(dims, P->c, &P->g)) return ERR_CORRUPT;
  P->eb_mode = (int)get32(b + 48);
  const uint32_t dt = get32(b + 52);
  if (dt > 1) return ERR_CORRUPT;
  P->dtype = (int)dt;
  P->vb = dt ? 8 : 4;
  P->eb = getf64(b + 56);
  P->eb_abs = getf64(b + 64);
  if (!(P->eb_abs > 0.0) || !std::isfinite(P->eb_abs)) return ERR_CORRUPT;
  P->total = get64(b + 80);
  if (P->total > size) return ERR_CORRUPT;
  P->codelen_off = get64(b + 88);
  P->anchor_off = get64(b + 96);
  P->n_anch = get64(b + 104);
  if (P->codelen_off != kHeaderBytes) return ERR_CORRUPT;
  if (P->anchor_off != kHeaderBytes + align16(size_t(alphabet(P->c)))) return ERR_CORRUPT;
  if (P->n_anch != n_anchor(P->g)) return ERR_CORRUPT;
  uint64_t pos = P->anchor_off + align16(P->vb * P->n_anch);
  for (int l = 1; l <= P->c.L; ++l) {
    const uint8_t* e = b + kLevelTable + kLevelRec * size_t(l - 1);
    Parsed::Lv& v = P->lv[l];
    v.off = get64(e);
    v.nu = get64(e + 8);
    v.nl = get64(e + 16);
    v.nsym = get64(e + 24);
    v.words = get64(e + 32);
    v.outl = get64(e + 40);
    std::vector<Unit> us = level_units(P->g, l);
    size_t nl = 0, ns = 0;
    for (const Unit& u : us) {
      nl += u.M[2];
      ns += u.nsym();
    }
    if (v.off != pos || v.nu != us.size() || v.nl != nl || v.nsym != ns) return ERR_CORRUPT;
    if (v.words > (uint64_t(1) << 32) || v.outl > v.nsym) return ERR_CORRUPT;
    v.ll.nu = v.nu;
    v.ll.nl = v.nl;
    v.ll.nsym = v.nsym;
    v.ll.words = v.words;
    v.ll.outl = v.outl;
    v.ll.vbytes = P->vb;
    layout_level(&v.ll);
    pos += v.ll.size;
    if (pos > P->total) return ERR_CORRUPT;
  }
  if (pos != P->total) return ERR_CORRUPT;
  return OK;
}

// Decode every lane of one unit into `sy` (rank order). Returns false on any
// inconsistency (code not in the book, lane length or unit size mismatch).
// Z = zero-chunk token (-1 when that stage is off), R = centre symbol.
bool decode_unit(const Decoder& dec, const uint32_t* payload, uint64_t nwords, uint64_t w0,
                 uint64_t w1, const uint16_t* lane_len, const Unit& u, int Z, int R,
                 std::vector<int>* sy) {
  sy->assign(u.nsym(), 0);
  uint64_t pos = w0 * 32;
  const uint64_t end = w1 * 32;
  if (w1 < w0 || w1 > nwords) return false;
  for (size_t j = 0; j < u.M[2]; ++j) {
    const uint64_t lane_end = pos + lane_len[j];
    if (lane_end > end) return false;
    for (size_t vz = 0; vz < u.M[0]; ++vz)
      for (size_t vy = 0; vy < u.M[1]; ++vy) {
        uint32_t code = 0;
        int sym = -1;
        for (int l = 1; l <= kLmax; ++l) {
          if (pos >= lane_end) return false;
          int bit = get_bit(payload, nwords, pos++);
          if (bit < 0) return false;
          code = (code << 1) | uint32_t(bit);
          if (dec.count[l] && code >= dec.first[l] && code - dec.first[l] < dec.count[l]) {
            sym = dec.by_len[l][code - dec.first[l]];
            break;
          }
        }
        if (sym < 0) return false;
        if (sym == Z) {
          // a zero-chunk token starts a chunk and stands for all of it
          if (vy != 0) return false;
          for (size_t k = 0; k < u.M[1]; ++k) (*sy)[(vz * u.M[1] + k) * u.M[2] + j] = R;
          break;
        }
        (*sy)[(vz * u.M[1] + vy) * u.M[2] + j] = sym;
      }
    if (pos != lane_end) return false;
  }
  // The unit occupies whole words: at most 31 padding bits.
  if ((pos + 31) / 32 != w1) return false;
  return true;
}

// Units decoded by the last decode call, per level and class (a test hook for
// the random-access claims of Sec. 3.3).
uint64_t g_units_decoded[kMaxLevels + 1][8];

// Decode levels 1..level inside the boxes box[k] (half-open, per level k), or
// the whole domain when region == false. `rec` is full resolution, NaN where
// nothing was reconstructed.
template <class T>
int decode_levels(const void* comp, const Parsed& P, int level, bool region,
                  const uint64_t (*box)[6], std::vector<T>* recp) {
  const Geo& g = P.g;
  const uint8_t* b = static_cast<const uint8_t*>(comp);
  std::vector<T>& rec = *recp;
  if (P.vb != sizeof(T)) return ERR_ARG;
  rec.assign(g.N, std::numeric_limits<T>::quiet_NaN());
  const int nsym = alphabet(P.c);
  const int Z = P.c.coding == 2 ? 2 * P.c.R : -1;
  const uint8_t* lens = b + P.codelen_off;
  Decoder dec;
  if (!dec.build(lens, nsym)) return ERR_CORRUPT;
  // Kraft check: the code book must be a valid prefix code.
  {
    int used = 0;
    double kraft = 0.0;
    for (int i = 0; i < nsym; ++i)
      if (lens[i]) {
        ++used;
        kraft += std::ldexp(1.0, -int(lens[i]));
      }
    if (kraft > 1.0) return ERR_CORRUPT;
    (void)used;
  }
  Bounds bd;
  level_bounds(P.eb_abs, P.c.ratio, P.c.L, &bd);

  auto inside = [&](int k, const size_t p[3]) {
    if (!region) return true;
    for (int d = 0; d < 3; ++d)
      if (p[d] < box[k][2 * d] || p[d] >= box[k][2 * d + 1]) return false;
    return true;
  };

  // Anchors.
  const size_t s0 = g.stride(0);
  const uint8_t* anch = b + P.anchor_off;
  size_t ai = 0;
  for (size_t z = 0; z < g.n[0]; z += s0)
    for (size_t y = 0; y < g.n[1]; y += s0)
      for (size_t xx = 0; xx < g.n[2]; xx += s0, ++ai) {
        size_t p[3] = {z, y, xx};
        if (inside(0, p)) {
          T v;
          std::memcpy(&v, anch + sizeof(T) * ai, sizeof(T));
          rec[g.idx(z, y, xx)] = v;
        }
      }

  bool bad = false;
  Reader<T> rd{rec.data(), &g, region, &bad};
  std::vector<int> sy;
  std::memset(g_units_decoded, 0, sizeof(g_units_decoded));
  for (int l = 1; l <= level; ++l) {
    const Parsed::Lv& v = P.lv[l];
    const uint8_t* base = b + v.off;
    const uint32_t* unit_word = reinterpret_cast<const uint32_t*>(base + v.ll.off_unit_word);
    const uint32_t* unit_outl = reinterpret_cast<const uint32_t*>(base + v.ll.off_unit_outl);
    const uint16_t* lane_len = reinterpret_cast<const uint16_t*>(base + v.ll.off_lane);
    const uint32_t* payload = reinterpret_cast<const uint32_t*>(base + v.ll.off_payload);
    const uint8_t* outl = base + v.ll.off_outl;
    if (unit_word[0] != 0 || unit_word[v.nu] != v.words) return ERR_CORRUPT;
    if (unit_outl[0] != 0 || unit_outl[v.nu] != v.outl) return ERR_CORRUPT;
    const size_t s = g.stride(l);
    std::vector<Unit> us = level_units(g, l);
    size_t lane_base = 0;
    for (size_t ui = 0; ui < us.size(); ++ui) {
      const Unit& u = us[ui];
      const size_t lb = lane_base;
      lane_base += u.M[2];
      if (u.nsym() == 0) continue;
      // Skip units with no point inside the level's box.
      if (region) {
        bool any = false;
        for (size_t vz = 0; vz < u.M[0] && !any; ++vz)
          for (size_t vy = 0; vy < u.M[1] && !any; ++vy)
            for (size_t vx = 0; vx < u.M[2] && !any; ++vx) {
              size_t p[3];
              unit_point(g, u, s, vz, vy, vx, p);
              any = inside(l, p);
            }
        if (!any) continue;
      }
      if (!decode_unit(dec, payload, v.words, unit_word[ui], unit_word[ui + 1], lane_len + lb, u,
                       Z, P.c.R, &sy))
        return ERR_CORRUPT;
      g_units_decoded[l][4 * u.o[0] + 2 * u.o[1] + u.o[2]]++;
      uint32_t oi = unit_outl[ui];
      const uint32_t oe = unit_outl[ui + 1];
      if (oe < oi || oe > v.outl) return ERR_CORRUPT;
      size_t t = 0;
      for (size_t vz = 0; vz < u.M[0]; ++vz)
        for (size_t vy = 0; vy < u.M[1]; ++vy)
          for (size_t vx = 0; vx < u.M[2]; ++vx, ++t) {
            size_t p[3];
            unit_point(g, u, s, vz, vy, vx, p);
            const int sym = sy[t];
            T val = T(0);
            if (sym == 0) {
              if (oi >= oe) return ERR_CORRUPT;
              std::memcpy(&val, outl + sizeof(T) * oi, sizeof(T));
              ++oi;
            }
            if (!inside(l, p)) continue;
            if (sym != 0) {
              // The quantizer's reconstruction, same operands and order.
              T pred = predict(rd, g, p, s);
              T E2;
              if constexpr (sizeof(T) == 4)
                E2 = bd.E2[l];
              else
                E2 = bd.E2d[l];
              T prod = (T)(sym - P.c.R) * E2;
              val = pred + prod;
            }
            rec[g.idx(p[0], p[1], p[2])] = val;
          }
      if (oi != oe) return ERR_CORRUPT;
    }
    if (bad) return ERR_CORRUPT;  // cannot happen unless the cone is wrong
  }
  return OK;
}

}  // namespace

extern "C" {

int stz_ref_info(const void* comp, uint64_t size, stz_ref_info* info) {
  Parsed P;
  int st = parse(comp, size, &P);
  if (st != OK) return st;
  if (info) {
    for (int d = 0; d < 3; ++d) info->dims[d] = P.g.n[d];
    info->block = (uint32_t)P.c.B;
    info->levels = (uint32_t)P.c.L;
    info->radius = (uint32_t)P.c.R;
    info->lmax = (uint32_t)kLmax;
    info->eb_mode = (uint32_t)P.eb_mode;
    info->dtype = (uint32_t)P.dtype;
    info->eb = P.eb;
    info->eb_abs = P.eb_abs;
    info->eb_ratio = P.c.ratio;
    info->total_bytes = P.total;
    info->coding = (uint32_t)P.c.coding;
    info->reserved = 0;
  }
  return OK;
}

}  // extern "C"

namespace {

// Progressive decompression: reconstruct levels 0..level and emit the stride
// 2^(L-level) grid (Sec. 3.3, progressive decompression). level == L gives the
// full field. A stream of the other value type is rejected with ERR_ARG.
template <class T>
int decompress_level_impl(const void* comp, uint64_t size, uint32_t level, T* out,
                          uint64_t out_cap, uint64_t out_dims[3]) {
  Parsed P;
  int st = parse(comp, size, &P);
  if (st != OK) return st;
  if (P.vb != sizeof(T)) return ERR_ARG;
  if ((int)level > P.c.L) return ERR_ARG;
  const Geo& g = P.g;
  const size_t s = g.stride((int)level);
  size_t od[3];
  for (int d = 0; d < 3; ++d) od[d] = g.grid_n(d, s);
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = od[d];
  if (!out || od[0] * od[1] * od[2] > out_cap) return ERR_BUFFER;
  std::vector<T> rec;
  st = decode_levels<T>(comp, P, (int)level, false, nullptr, &rec);
  if (st != OK) return st;
  size_t o = 0;
  for (size_t z = 0; z < g.n[0]; z += s)
    for (size_t y = 0; y < g.n[1]; y += s)
      for (size_t x = 0; x < g.n[2]; x += s) out[o++] = rec[g.idx(z, y, x)];
  return OK;
}

template <class T>
int decompress_impl(const void* comp, uint64_t size, T* out, uint64_t out_cap) {
  Parsed P;
  int st = parse(comp, size, &P);
  if (st != OK) return st;
  uint64_t od[3];
  return decompress_level_impl<T>(comp, size, (uint32_t)P.c.L, out, out_cap, od);
}

// Random-access decompression of the box [lo, hi) at a level (Sec. 3.3): the
// box at the output level needs, at every coarser level k-1, the box widened by
// the stencil reach 3*s_k; only units with a point inside their level's box are
// decoded, and only points inside are predicted.
template <class T>
int decompress_region_impl(const void* comp, uint64_t size, const uint64_t lo[3],
                           const uint64_t hi[3], uint32_t level, T* out, uint64_t out_cap,
                           uint64_t out_dims[3]) {
  Parsed P;
  int st = parse(comp, size, &P);
  if (st != OK) return st;
  if (P.vb != sizeof(T)) return ERR_ARG;
  const Geo& g = P.g;
  if ((int)level > P.c.L || !lo || !hi) return ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (!(lo[d] < hi[d]) || hi[d] > g.n[d]) return ERR_ARG;
  uint64_t box[kMaxLevels + 1][6];
  for (int d = 0; d < 3; ++d) {
    box[level][2 * d] = lo[d];
    box[level][2 * d + 1] = hi[d];
  }
  for (int k = (int)level; k >= 1; --k) {
    const uint64_t r = 3 * g.stride(k);
    for (int d = 0; d < 3; ++d) {
      uint64_t a = box[k][2 * d], e = box[k][2 * d + 1];
      box[k - 1][2 * d] = a > r ? a - r : 0;
      box[k - 1][2 * d + 1] = std::min<uint64_t>(g.n[d], e + r);
    }
  }
  const size_t s = g.stride((int)level);
  size_t od[3], first[3];
  for (int d = 0; d < 3; ++d) {
    first[d] = (lo[d] + s - 1) / s * s;
    od[d] = first[d] < hi[d] ? (hi[d] - 1 - first[d]) / s + 1 : 0;
  }
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = od[d];
  const size_t cnt = od[0] * od[1] * od[2];
  if (cnt == 0) return OK;
  if (!out || cnt > out_cap) return ERR_BUFFER;
  std::vector<T> rec;
  st = decode_levels<T>(comp, P, (int)level, true, box, &rec);
  if (st != OK) return st;
  size_t o = 0;
  for (size_t z = first[0]; z < hi[0]; z += s)
    for (size_t y = first[1]; y < hi[1]; y += s)
      for (size_t x = first[2]; x < hi[2]; x += s) {
        T v = rec[g.idx(z, y, x)];
        if (std::isnan(v)) return ERR_CORRUPT;
        out[o++] = v;
      }
  return OK;
}

}  // namespace

extern "C" {

int stz_ref_decompress_level(const void* comp, uint64_t size, uint32_t level, float* out,
                             uint64_t out_cap, uint64_t out_dims[3]) {
  return decompress_level_impl<float>(comp, size, level, out, out_cap, out_dims);
}

int stz_ref_decompress_level_f64(const void* comp, uint64_t size, uint32_t level, double* out,
                                 uint64_t out_cap, uint64_t out_dims[3]) {
  return decompress_level_impl<double>(comp, size, level, out, out_cap, out_dims);
}

int stz_ref_decompress(const void* comp, uint64_t size, float* out, uint64_t out_cap) {
  return decompress_impl<float>(comp, size, out, out_cap);
}

int stz_ref_decompress_f64(const void* comp, uint64_t size, double* out, uint64_t out_cap) {
  return decompress_impl<double>(comp, size, out, out_cap);
}

int stz_ref_decompress_region(const void* comp, uint64_t size, const uint64_t lo[3],
                              const uint64_t hi[3], uint32_t level, float* out,
                              uint64_t out_cap, uint64_t out_dims[3]) {
  return decompress_region_impl<float>(comp, size, lo, hi, level, out, out_cap, out_dims);
}

int stz_ref_decompress_region_f64(const void* comp, uint64_t size, const uint64_t lo[3],
                                  const uint64_t hi[3], uint32_t level, double* out,
                                  uint64_t out_cap, uint64_t out_dims[3]) {
  return decompress_region_impl<double>(comp, size, lo, hi, level, out, out_cap, out_dims);
}

// ---------------------------------------------------------------------------
// Test hooks (intermediate results, for the pins).
// ---------------------------------------------------------------------------

// Per-point symbols and reconstruction of the compressor, in full-resolution
// order: sym[i] = -1 for anchors, else the symbol of point i; rec[i] = the value
// the decoder reproduces. Also returns the level of each point.
}  // extern "C"

namespace {

template <class T>
int symbols_impl(const T* x, const uint64_t dims[3], int eb_mode, double eb,
                 const stz_ref_config* cfg, int32_t* sym, T* rec_out, int32_t* level_of) {
  Cfg c;
  Geo g;
  if (resolve_cfg(cfg, &c) != OK || !make_geo(dims, c, &g)) return ERR_ARG;
  if (!(eb > 0.0)) return ERR_ARG;
  for (size_t i = 0; i < g.N; ++i)
    if (!std::isfinite(x[i])) return ERR_NONFINITE;
  double eb_abs = eb;
  if (eb_mode == 1) {
    T mn = x[0], mx = x[0];
    for (size_t i = 1; i < g.N; ++i) {
      mn = std::min(mn, x[i]);
      mx = std::max(mx, x[i]);
    }
    double range = (double)mx - (double)mn;
    eb_abs = range > 0.0 ? eb * range
                         : eb * (std::fabs((double)mn) > 0.0 ? std::fabs((double)mn) : 1.0);
  }
  Bounds bd;
  level_bounds(eb_abs, c.ratio, c.L, &bd);
  std::vector<T> rec(g.N, T(0));
  const size_t s0 = g.stride(0);
  for (size_t i = 0; i < g.N; ++i) {
    sym[i] = -2;
    level_of[i] = -1;
  }
  for (size_t z = 0; z < g.n[0]; z += s0)
    for (size_t y = 0; y < g.n[1]; y += s0)
      for (size_t xx = 0; xx < g.n[2]; xx += s0) {
        size_t i = g.idx(z, y, xx);
        rec[i] = x[i];
        sym[i] = -1;
        level_of[i] = 0;
      }
  Reader<T> rd{rec.data(), &g, false, nullptr};
  for (int l = 1; l <= c.L; ++l) {
    const size_t s = g.stride(l);
    for (const Unit& u : level_units(g, l))
      for (size_t vz = 0; vz < u.M[0]; ++vz)
        for (size_t vy = 0; vy < u.M[1]; ++vy)
          for (size_t vx = 0; vx < u.M[2]; ++vx) {
            size_t p[3];
            unit_point(g, u, s, vz, vy, vx, p);
            size_t i = g.idx(p[0], p[1], p[2]);
            T pred = predict(rd, g, p, s);
            T r;
            sym[i] = quantize<T>(x[i], pred, bd, l, c.R, &r);
            rec[i] = r;
            level_of[i] = l;
          }
  }
  std::memcpy(rec_out, rec.data(), sizeof(T) * g.N);
  return OK;
}

}  // namespace

extern "C" {

int stz_ref_symbols(const float* x, const uint64_t dims[3], int eb_mode, double eb,
                    const stz_ref_config* cfg, int32_t* sym, float* rec_out, int32_t* level_of) {
  return symbols_impl<float>(x, dims, eb_mode, eb, cfg, sym, rec_out, level_of);
}

int stz_ref_symbols_f64(const double* x, const uint64_t dims[3], int eb_mode, double eb,
                        const stz_ref_config* cfg, int32_t* sym, double* rec_out,
                        int32_t* level_of) {
  return symbols_impl<double>(x, dims, eb_mode, eb, cfg, sym, rec_out, level_of);
}

// The prediction of point p at stride s from a full-resolution array `rec`.
float stz_ref_predict(const float* rec, const uint64_t dims[3], const uint64_t p[3],
                      uint64_t s) {
  Geo g;
  for (int d = 0; d < 3; ++d) g.n[d] = dims[d];
  g.N = dims[0] * dims[1] * dims[2];
  Reader<float> rd{rec, &g, false, nullptr};
  size_t pp[3] = {p[0], p[1], p[2]};
  return predict(rd, g, pp, s);
}

double stz_ref_predict_f64(const double* rec, const uint64_t dims[3], const uint64_t p[3],
                           uint64_t s) {
  Geo g;
  for (int d = 0; d < 3; ++d) g.n[d] = dims[d];
  g.N = dims[0] * dims[1] * dims[2];
  Reader<double> rd{rec, &g, false, nullptr};
  size_t pp[3] = {p[0], p[1], p[2]};
  return predict(rd, g, pp, s);
}

// Units decoded by the last decode call: out[8*level + class].
void stz_ref_units_decoded(uint64_t* out) {
  for (int l = 0; l <= kMaxLevels; ++l)
    for (int c = 0; c < 8; ++c) out[8 * l + c] = g_units_decoded[l][c];
}

void stz_ref_huffman_lengths(const uint64_t* counts, int nsym, int lmax, uint8_t* lens) {
  huffman_lengths(counts, nsym, lmax, lens);
}

void stz_ref_canonical_codes(const uint8_t* lens, int nsym, uint32_t* codes) {
  canonical_codes(lens, nsym, codes);
}

}  // extern "C"

namespace {

// Per-unit statistic of the ROI selection below over the decoded level grid.
template <class T>
int roi_stats(const void* comp, const Parsed& P, uint32_t level, uint32_t unit, uint32_t stat,
              std::vector<double>* out) {
  const Geo& g = P.g;
  const size_t s = g.stride((int)level);
  std::vector<T> rec;
  int st = decode_levels<T>(comp, P, (int)level, false, nullptr, &rec);
  if (st != OK) return st;
  const size_t nb[3] = {(g.n[0] + g.B - 1) / g.B, (g.n[1] + g.B - 1) / g.B,
                        (g.n[2] + g.B - 1) / g.B};
  size_t nunits;
  if (unit == 0)
    nunits = nb[0] * nb[1] * nb[2];
  else
    nunits = g.grid_n(int(unit - 1), s);
  std::vector<T> mx(nunits, -std::numeric_limits<T>::infinity());
  std::vector<T> mn(nunits, std::numeric_limits<T>::infinity());
  for (size_t z = 0; z < g.n[0]; z += s)
    for (size_t y = 0; y < g.n[1]; y += s)
      for (size_t x = 0; x < g.n[2]; x += s) {
        size_t u;
        if (unit == 0)
          u = ((z / g.B) * nb[1] + y / g.B) * nb[2] + x / g.B;
        else
          u = (unit == 1 ? z : unit == 2 ? y : x) / s;
        const T v = rec[g.idx(z, y, x)];
        if (v > mx[u]) mx[u] = v;
        if (v < mn[u]) mn[u] = v;
      }
  out->assign(nunits, 0.0);
  for (size_t u = 0; u < nunits; ++u)
    (*out)[u] = stat == 0 ? (double)mx[u] : (double)mx[u] - (double)mn[u];
  return OK;
}

}  // namespace

extern "C" {

// ROI selection (Sec. 3.3, "flexible scientific workflow"): the value range
// or the maximum of every 3-D block or every 2-D slice of the field, taken over
// the points of a progressive level's grid, then a threshold or the top
// fraction. unit: 0 = blocks of B^3 full-resolution points (raster order),
// 1/2/3 = planes of the level grid across axis z/y/x (index = plane number).
// stat: 0 = max, 1 = range (max - min, in double). rule: 0 = stat > value,
// 1 = the ceil(value * units) units with the largest stat (ties: smaller index
// first). Selected indices ascending into blocks[], their number in *count;
// stats[] (units entries) receives every unit's statistic when not null.
// Either value type.
int stz_ref_roi_select(const void* comp, uint64_t size, uint32_t level, uint32_t unit,
                       uint32_t stat, uint32_t rule, double value, uint32_t* sel, uint64_t cap,
                       uint64_t* count, double* stats) {
  Parsed P;
  int st = parse(comp, size, &P);
  if (st != OK) return st;
  if ((int)level > P.c.L || unit > 3 || stat > 1 || rule > 1) return ERR_ARG;
  if (rule == 1 && !(value > 0.0 && value <= 1.0)) return ERR_ARG;
  std::vector<double> st_all;
  st = P.dtype == 0 ? roi_stats<float>(comp, P, level, unit, stat, &st_all)
                    : roi_stats<double>(comp, P, level, unit, stat, &st_all);
  if (st != OK) return st;
  const size_t nunits = st_all.size();
  if (stats)
    for (size_t u = 0; u < nunits; ++u) stats[u] = st_all[u];
  std::vector<uint32_t> pick;
  if (rule == 0) {
    for (size_t u = 0; u < nunits; ++u)
      if (st_all[u] > value) pick.push_back(uint32_t(u));
  } else {
    const size_t k = std::min(nunits, (size_t)std::ceil(value * (double)nunits));
    std::vector<uint32_t> order(nunits);
    for (size_t u = 0; u < nunits; ++u) order[u] = uint32_t(u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
      return st_all[a] > st_all[b] || (st_all[a] == st_all[b] && a < b);
    });
    pick.assign(order.begin(), order.begin() + k);
    std::sort(pick.begin(), pick.end());
  }
  if (count) *count = pick.size();
  if (pick.size() > cap) return ERR_BUFFER;
  for (size_t i = 0; i < pick.size(); ++i) sel[i] = pick[i];
  return OK;
}

// Per-level error bound constants: e (double), 2e and 1/(2e) as float.
void stz_ref_level_bounds(double eb_abs, double ratio, int L, double* e, float* E2, float* INV) {
  Bounds bd;
  level_bounds(eb_abs, ratio, L, &bd);
  for (int l = 1; l <= L; ++l) {
    e[l] = bd.e[l];
    E2[l] = bd.E2[l];
    INV[l] = bd.INV[l];
  }
}

}  // extern "C"
