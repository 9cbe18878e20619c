// Decoding kernels (gfx950): per-level decode + reconstruct over the
// dependency cone of a box (Sec. 3.3), which covers full, progressive and
// region decoding.
//
// One work-group per block of the level. Its 7 sub-block units are decoded by
// one lane per x-column stream (units never straddle a wave), a z-slab of rows
// at a time into LDS; outliers get their rank-order index from a per-row
// ballot over the unit's lanes. The slab's coarse halo is staged in LDS, and
// the whole slab of the level grid (coarse points copied, level points
// predicted and dequantized) is written with coalesced rows.
#include <algorithm>
#include <cstring>

#include "stz_slab.h"

namespace stz {
using namespace dev;
namespace {

struct DecSlabArgs {
  Geo g;
  int level;
  int logs;                     // L - level
  int64_t n[3];                 // level grid extents
  int64_t bb_lo[3], bb_n[3];    // blocks to process
  bool xcd_remap;
  const void* prev;             // level-(l-1) box grid (value type of the kernel)
  int64_t in_first[3], in_cnt[3];  // (coarse coordinates)
  void* cur;                    // level-l box grid (output)
  int64_t out_first[3], out_cnt[3];
  const uint32_t* unit_word;
  const uint32_t* unit_outl;
  const uint16_t* lane_len;
  const uint32_t* pay;
  const void* outv;             // outlier values
  uint64_t words, noutl, nlanes, nu;
  float E2;                     // 2e for float32 fields
  double E2d;                   // 2e for float64 fields
  const uint16_t* lut;
  uint32_t* flags;
};

// Per-slab state for reconstructing rows of one parity type (T = value type).
template <class T>
struct DecRows {
  const T* tile;
  const uint16_t* symb;
  const uint32_t* uo0;
  const uint32_t* uo1;
  const T* outv;
  uint32_t* flags;
  T* cur;
  int64_t oz, oy, ox;
  int z0, a0, Ex, rz0, rz1, ry0, ry1, rx0, rx1;
  int tz0;  // level plane of the coarse tile's origin (relative to the block)
  int64_t of[3], oc[3], n[3];
  T E2;
  int R;
  bool pair;  // output rows start on even elements of a grid aligned to two values
};

// Output stores. NTS: non-temporal, for the call's final output grid, which
// nothing in the call reads back: it streams to memory instead of displacing
// the stream words and coarse planes other blocks still read from the caches.
template <bool NTS, class T>
__device__ inline void st_out(T* p, T v) {
  if constexpr (NTS)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <bool NTS, class T>
__device__ inline void st_pair(T* p, T v0, T v1) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 w;
  w.x = v0;
  w.y = v1;
  if constexpr (NTS)
    __builtin_nontemporal_store(w, reinterpret_cast<V2*>(p));
  else
    *reinterpret_cast<V2*>(p) = w;
}

// Slab height of the decoder: for 32^3-point blocks, 2 planes keep the LDS
// footprint (code table, slab symbols, coarse tile, stream ring) at 26 KB, for
// six work-groups per CU; 16^3-point blocks take 4 planes (17 KB, 72 VGPRs,
// seven per CU). The per-symbol decode chains
// (one per lane stream) are latency-bound, so more blocks in flight win over
// the extra slab passes.
constexpr int dec_slab_h(int E) { return E == 32 ? 2 : (E == 16 ? 4 : default_slab_h(E)); }

constexpr int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Sentinel entries of a level's unit index (first offsets 0, last = totals).
__device__ inline void dec_check_body(const DecSlabArgs& d) {
  if (threadIdx.x == 0 && (d.unit_word[0] != 0 || d.unit_outl[0] != 0 ||
                           d.unit_word[d.nu] != d.words || d.unit_outl[d.nu] != d.noutl))
    atomicOr(d.flags, kFlagCorrupt);
}

// Value of one point of class C (0 = copy of a coarse point).
template <class T, int E, int H, int C, bool INT>
__device__ inline T dec_point(const DecRows<T>& x, int lz, int ly, int lx, int srow,
                              const int64_t p[3]) {
  using S = SlabShape<E, H>;
  if constexpr (C == 0) {
    return x.tile[((((lz - x.tz0) >> 1) + 1) * S::T + (ly >> 1) + 1) * S::TP + (lx >> 1) + 1];
  } else {
    const uint16_t e = x.symb[(C - 1) * S::SCP + srow];
    if (e & 0x8000u) {
      const uint64_t oi = uint64_t(x.uo0[C]) + (e & 0x7FFFu);
      if (oi < x.uo1[C]) return x.outv[oi];
      atomicOr(x.flags, kFlagCorrupt);
      return T(0);
    }
    // the quantizer's reconstruction: same operands, same order
    const T pred = tile_pred<T, E, C, INT>(x.tile, lz - x.tz0, ly, lx, p, x.n);
    const T prod = (T)(int(e) - x.R) * x.E2;
    return pred + prod;
  }
}

// Reconstruct this wave's rows of parity type (ZP, YP): classes 4ZP+2YP (even
// x) and 4ZP+2YP+1 (odd x), both fixed at compile time.
template <class T, int E, int H, int NW, int ZP, int YP, bool INT, bool NTS>
__device__ inline void dec_type(const DecRows<T>& x, int hs, int Ey, int wave, int lane) {
  using S = SlabShape<E, H>;
  constexpr int m = S::m;
  constexpr int C0 = 4 * ZP + 2 * YP;
  // the lane's row offset from its wave's first row (lanes of one row group
  // are 2*(lane / P) rows apart)
  const int64_t lane_row = int64_t(2 * (lane / S::P)) * x.oc[2];
  for_type_rows<E, ZP, YP, NW>(x.z0, hs, Ey, wave, lane, [&](int lz, int ly, int q, int lyu) {
    if (lz < x.rz0 || lz >= x.rz1 || ly < x.ry0 || ly >= x.ry1) return;
    T* orow = x.cur + ((x.oz + lz - x.of[0]) * x.oc[1] + (x.oy + lyu - x.of[1])) * x.oc[2] +
                  (x.ox - x.of[2]) + lane_row;
    const int srow = (((lz >> 1) - x.a0) * m + (ly >> 1)) * S::SP + q;
    const int l0 = 2 * q, l1 = 2 * q + 1;
    const int64_t p0[3] = {x.oz + lz, x.oy + ly, x.ox + l0};
    const int64_t p1[3] = {x.oz + lz, x.oy + ly, x.ox + l1};
    const bool in0 = l0 < x.Ex && l0 >= x.rx0 && l0 < x.rx1;
    const bool in1 = l1 < x.Ex && l1 >= x.rx0 && l1 < x.rx1;
    if (x.pair && in0 && in1) {
      const T v0 = dec_point<T, E, H, C0, INT>(x, lz, ly, l0, srow, p0);
      const T v1 = dec_point<T, E, H, C0 + 1, INT>(x, lz, ly, l1, srow, p1);
      st_pair<NTS>(orow + l0, v0, v1);
    } else {
      if (in0) st_out<NTS>(orow + l0, dec_point<T, E, H, C0, INT>(x, lz, ly, l0, srow, p0));
      if (in1) st_out<NTS>(orow + l1, dec_point<T, E, H, C0 + 1, INT>(x, lz, ly, l1, srow, p1));
    }
  });
}

// NT = threads of the work-group (256, or 64 for small blocks); NTS =
// non-temporal output stores.
template <class T, int E, int H, int NT = 256, bool NTS = false>
__device__ inline void dec_body(const DecSlabArgs& a, int64_t wg) {
  using S = SlabShape<E, H>;
  constexpr int m = S::m;
  constexpr int NW = NT / 64;
  constexpr int NL = 7 * m;  // decoding lanes: one per (class, x column)
  static_assert(NL <= NT, "a work-group holds every decoding lane");
  // Stream words a lane can touch while decoding one slab: at most HZ*m codes
  // of <= kLmax bits, plus the bit window's lookahead (< 2 words).
  constexpr int WPL = (S::HZ * m * kLmax + 31) / 32 + 2;
  // Wide work-groups (one per CU, latency-bound launches of few blocks) of
  // 16^3 and 32^3 level points load each lane's whole stream into its ring
  // and the block's whole coarse tile up front, so the slabs wait on no
  // global loads: WLW = the most words a lane stream of the block can span.
  constexpr bool kWhole = NW >= 16 && (E == 16 || E == 32);
  constexpr int WLW = (m * m * kLmax + 31) / 32 + 2;
  // Per-lane ring of RB stream words (a power of two), [slot][lane]: the
  // words of the current slab plus the prefetched words of the next one
  // (RB >= 2*WPL), or the whole stream (kWhole: RB > WLW).
  constexpr int RB = kWhole ? pow2_ceil(WLW + 1) : pow2_ceil(2 * WPL);
  constexpr int WF = kWhole ? WLW : WPL;  // words loaded before the first slab, less one
  // Blocks of 16^3 level points and more copy the code table into LDS; for
  // smaller ones (a few symbols per lane) the copy would cost more than it
  // saves, and the table is read through the cache.
  constexpr bool kLdsLut = E >= 16;
  __shared__ __align__(16) uint16_t lut_s[kLdsLut ? (1 << kLutBits) : 1];
  const uint16_t* lut = kLdsLut ? lut_s : a.lut;
  __shared__ uint16_t symb[7 * S::SCP];
  // Blocks of 16^3 and 32^3 level points decoded in several slabs slide a
  // window of coarse planes: the waves that hold no decoding lane move it and
  // load the slab's HZ new planes while the other waves decode. Other blocks
  // load each slab's whole coarse tile.
  constexpr int NLW = (NL + 63) / 64;  // waves holding decoding lanes
  constexpr bool kSlide = !kWhole && (E == 16 || E == 32) && S::H < E && NLW * 64 < NT;
  using SW = SlabShape<E, E>;  // the whole block as one slab (coarse tile of m+3 planes)
  __shared__ T tile[kWhole ? SW::TILE : S::TILE];
  __shared__ uint32_t ring[RB * NL];
  __shared__ uint32_t lanelen_s[NL];
  __shared__ uint32_t uo0[8], uo1[8];
  __shared__ int uok[8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar)
  if constexpr (kLdsLut) {
    // 16-byte copies when the table is aligned (8 entries per thread and pass)
    if ((reinterpret_cast<uintptr_t>(a.lut) & 15) == 0) {
      const uint4* src = reinterpret_cast<const uint4*>(a.lut);
      uint4* dst = reinterpret_cast<uint4*>(lut_s);
      for (int i = tid; i < (1 << kLutBits) / 8; i += blockDim.x) dst[i] = src[i];
    } else {
      for (int i = tid; i < (1 << kLutBits); i += blockDim.x) lut_s[i] = a.lut[i];
    }
  }
  if (wg == 0 && tid == 0) dec_check_body(a);  // the level's unit-index sentinels

  const int64_t nblk = a.bb_n[0] * a.bb_n[1] * a.bb_n[2];
  const int64_t bl = wg_block(wg, nblk, a.xcd_remap);
  const int64_t bx = a.bb_lo[2] + bl % a.bb_n[2];
  const int64_t by = a.bb_lo[1] + (bl / a.bb_n[2]) % a.bb_n[1];
  const int64_t bz = a.bb_lo[0] + bl / (a.bb_n[2] * a.bb_n[1]);
  const int64_t blk = (bz * a.g.nb[1] + by) * a.g.nb[2] + bx;
  const int64_t oz = bz * E, oy = by * E, ox = bx * E;  // block origin, level coordinates
  const int Ez = int(min<int64_t>(E, a.n[0] - oz)), Ey = int(min<int64_t>(E, a.n[1] - oy)),
            Ex = int(min<int64_t>(E, a.n[2] - ox));
  // Output box (level coordinates) clipped to the block, block-local.
  const int rz0 = int(max<int64_t>(0, a.out_first[0] - oz));
  const int rz1 = int(min<int64_t>(Ez, a.out_first[0] + a.out_cnt[0] - oz));
  const int ry0 = int(max<int64_t>(0, a.out_first[1] - oy));
  const int ry1 = int(min<int64_t>(Ey, a.out_first[1] + a.out_cnt[1] - oy));
  const int rx0 = int(max<int64_t>(0, a.out_first[2] - ox));
  const int rx1 = int(min<int64_t>(Ex, a.out_first[2] + a.out_cnt[2] - ox));

  // ---- decode setup: lane t < 7m handles class c = t/m + 1, column j ------
  const int c = tid / m + 1, j = tid % m;
  const bool is_lane = tid < NL;
  const int ocz = (c >> 2) & 1, ocy = (c >> 1) & 1, ocx = c & 1;
  const int Mz = ocz ? Ez >> 1 : (Ez + 1) >> 1;
  const int My = ocy ? Ey >> 1 : (Ey + 1) >> 1;
  const int Mx = ocx ? Ex >> 1 : (Ex + 1) >> 1;
  // Does the unit have a point inside the output box? (v range per axis)
  bool needed = Mz > 0 && My > 0 && Mx > 0;
  {
    const int lo[3] = {rz0, ry0, rx0}, hi[3] = {rz1, ry1, rx1}, oo[3] = {ocz, ocy, ocx};
    for (int d = 0; d < 3; ++d) {
      // v with 2v+o in [lo, hi)
      const int v0 = lo[d] - oo[d] <= 0 ? 0 : (lo[d] - oo[d] + 1) >> 1;
      const int v1 = hi[d] - oo[d] <= 0 ? 0 : ((hi[d] - 1 - oo[d]) >> 1) + 1;
      needed = needed && v0 < v1;
    }
  }
  const bool lane_active = is_lane && needed && j < Mx;
  const int64_t u = blk * 7 + (c - 1);
  uint32_t lb = 0, w0 = 0, w1 = 0, o0 = 0, o1 = 0;
  uint64_t pos = 0;
  if (lane_active) {
    // the unit's index entries load alongside the lane length
    w0 = a.unit_word[u];
    w1 = a.unit_word[u + 1];
    o0 = a.unit_outl[u];
    o1 = a.unit_outl[u + 1];
    const uint64_t lane0 = uint64_t(unit_lane_off(a.g, a.logs, u));
    lb = lane0 + j < a.nlanes ? a.lane_len[lane0 + j] : 0;
  }
  if (is_lane) lanelen_s[tid] = lb;
  if (tid < 8) uok[tid] = 1;
  __syncthreads();
  bool alive = false;
  if (lane_active) {
    uint32_t pre = 0, tot = 0;
    for (int k = 0; k < Mx; ++k) {
      const uint32_t v = lanelen_s[(c - 1) * m + k];
      if (k < j) pre += v;
      tot += v;
    }
    const bool ok = w0 <= w1 && w1 <= a.words && o0 <= o1 && o1 <= a.noutl &&
                    (uint64_t(tot) + 31) / 32 == uint64_t(w1 - w0);
    if (j == 0) {
      // An inconsistent unit gets an empty outlier range, so no outlier
      // index can leave the level's list.
      uo0[c] = ok ? o0 : 0;
      uo1[c] = ok ? o1 : 0;
      uok[c] = ok;
    }
    if (!ok) atomicOr(a.flags, kFlagCorrupt);
    alive = ok;
    pos = uint64_t(w0) * 32 + pre;
  }
  // Bit window: `buf` holds `nb` valid bits, left aligned; `wi` = next stream
  // word, found in ring slot `rk`. Slot of word w = (w - first word) mod RB.
  // Before each slab the ring holds the WPL words from `wi` on (kWhole: the
  // whole stream). Bits consumed so far = 32*wi - pos - nb.
  uint64_t wi = pos >> 5, buf = 0;
  int nb = 0, rk = 0;
  if constexpr (kWhole) {
    // every thread loads (lane, word) pairs of the lanes' whole streams: the
    // lanes' first words pass through LDS (~0u: a lane that decodes nothing)
    __shared__ uint32_t wfirst[NL];
    if (is_lane) wfirst[tid] = lane_active && alive ? uint32_t(wi) : ~0u;
    __syncthreads();
    for (int i = tid; i < NL * (WF + 1); i += NT) {
      const int l = i % NL, k = i / NL;
      const uint32_t w0l = wfirst[l];
      const uint64_t idx = uint64_t(w0l) + uint64_t(k);
      ring[k * NL + l] = (w0l != ~0u && idx < a.words) ? a.pay[idx] : 0u;
    }
    __syncthreads();
  }
  if (lane_active) {
    if constexpr (!kWhole) {
#pragma unroll
      for (int k = 0; k <= WF; ++k) {
        const uint64_t idx = wi + k;
        ring[k * NL + tid] = (alive && idx < a.words) ? a.pay[idx] : 0u;
      }
    }
    const int sk = int(pos & 31);
    buf = (uint64_t(ring[tid]) << 32) << sk;
    nb = 32 - sk;
    ++wi;
    rk = 1;
  }
  uint32_t run = 0;
  bool bad = false;
  // Lanes of this unit inside the wave (units never straddle a wave).
  const int seg = lane - j;
  const uint64_t segmask = (m >= 64 ? ~uint64_t(0) : ((uint64_t(1) << m) - 1)) << seg;
  const uint64_t ltmask = (uint64_t(1) << lane) - 1;

  const int64_t org[3] = {oz, oy, ox};
  const bool interior = block_interior(org, E, a.n);
  constexpr bool kFullPath = m >= 8;
  const bool full_rows = Ez == E && Ey == E;
  const int zlast = min(Ez, rz1);  // no output needed beyond this level plane
  bool complete = true;
  // block origin of the coarse window (level coordinates, even)
  const int64_t cz00 = (oz - 2) >> 1, cy0 = (oy - 2) >> 1, cx0 = (ox - 2) >> 1;
  if constexpr (kSlide) {
    // the first slab's TZ planes; later slabs slide the window by HZ
    TileRegs<S, T, NT> r0;
    tile_fetch<S, T, NT>(r0, static_cast<const T*>(a.prev), a.in_first, a.in_cnt, cz00, cy0, cx0);
    tile_store<S, T, NT>(tile, r0);
  }
  if constexpr (kWhole) {
    TileRegs<SW, T, NT> r0;
    tile_fetch<SW, T, NT>(r0, static_cast<const T*>(a.prev), a.in_first, a.in_cnt, cz00, cy0,
                          cx0);
    tile_store<SW, T, NT>(tile, r0);
  }
  for (int z0 = 0; z0 < Ez; z0 += S::H) {
    if (z0 >= zlast) {
      complete = false;
      break;
    }
    const int a0 = z0 >> 1;
    // ---- coarse planes of the slab (global loads in flight during decoding) ----
    TileRegs<S, T, NT> tr;
    if constexpr (!kSlide && !kWhole)
      tile_fetch<S, T, NT>(tr, static_cast<const T*>(a.prev), a.in_first, a.in_cnt, cz00 + a0, cy0,
                           cx0);
    if constexpr (kSlide) {
      if (z0 > 0 && wave >= NLW)
        slide_window<S, T, NT - NLW * 64>(tile, static_cast<const T*>(a.prev), a.in_first,
                                          a.in_cnt, cz00 + a0 + S::TZ - S::HZ, cy0, cx0,
                                          tid - NLW * 64);
    }
    // ---- decode this slab's rows into LDS -----------------------------------
    if (lane_active) {
      // Prefetch the WPL words after this slab's window into registers; they
      // land in the ring once the slab is decoded.
      const uint64_t wb = wi;
      const int rb = rk;
      uint32_t pf[kWhole ? 1 : WPL];
      if constexpr (!kWhole) {
#pragma unroll
        for (int k = 0; k < WPL; ++k) {
          const uint64_t idx = wb + WPL + k;
          pf[k] = (alive && idx < a.words) ? a.pay[idx] : 0u;
        }
      }
      const int r0 = a0 * My, r1 = min(a0 + S::HZ, Mz) * My;
      const int Zt = a.g.Z, Rc = a.g.R;  // zero-chunk token (-1: off), centre symbol
      const uint32_t eR = uint32_t(Rc);  // table entry of a zero-chunk row: R, no bits
      uint32_t nw = ring[rk * NL + tid];  // next stream word (word wi)
      if (kFullPath && full_rows) {
        // Full blocks: every unit has M_y = m rows per chunk and HZ chunks in
        // the slab, so the row loop unrolls completely. The bit window is
        // topped up to at least 32 bits before every two codes (of at most
        // kLmax bits each); a chunk's first token decides whether it is a zero
        // chunk; codes that are not in the book give symbol 0 with no bits and
        // are caught in the (rare) outlier branch.
        bool zmid = false;  // a Z token after a chunk's first row
#pragma unroll
        for (int hz = 0; hz < S::HZ; ++hz) {
          bool inz = false;
#pragma unroll
          for (int vy = 0; vy < m; vy += 2) {
            const bool rf = nb < 32;
            const int sh = rf ? 32 - nb : 0;
            buf |= uint64_t(rf ? nw : 0u) << sh;
            nb += rf ? 32 : 0;
            rk = (rk + (rf ? 1 : 0)) & (RB - 1);
            nw = ring[rk * NL + tid];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const uint32_t ei = lut[uint32_t(buf >> 32) >> (32 - kLutBits)];
              const uint32_t e = inz ? eR : ei;
              const int len = int(e >> 12);
              int sy = int(e & 4095);
              buf <<= len;
              nb -= len;
              if (vy + u == 0) {
                inz = sy == Zt;
                sy = inz ? Rc : sy;
              } else {
                zmid |= sy == Zt;
              }
              uint16_t st = uint16_t(sy);
              if (__ballot(sy == 0) != 0) {  // wave-uniform: outliers are rare
                const bool is_out = sy == 0 && len != 0;
                bad |= sy == 0 && len == 0;  // not a code of the book
                const uint64_t mk = __ballot(is_out) & segmask;
                if (is_out) st = uint16_t(0x8000u | ((run + __popcll(mk & ltmask)) & 0x7FFFu));
                run += __popcll(mk);
              }
              symb[(c - 1) * S::SCP + (hz * m + vy + u) * S::SP + j] = st;
            }
          }
        }
        bad |= zmid;
      } else {
        int zr = 0;                        // rows left in the current zero chunk
        int vy = 0;                        // row r = vz*My + vy, advanced incrementally
        int so = (c - 1) * S::SCP + j;     // LDS slot of the row's symbol
        for (int r = r0; r < r1; ++r) {
          // Branch-free refill: merge the next word when fewer than kLmax
          // bits are left, then read the following one from the ring.
          const bool rf = nb < kLmax;
          const int sh = rf ? 32 - nb : 0;
          buf |= uint64_t(rf ? nw : 0u) << sh;
          nb += rf ? 32 : 0;
          rk = (rk + (rf ? 1 : 0)) & (RB - 1);
          nw = ring[rk * NL + tid];
          // Inside a zero chunk a row takes R and no bits; a Z token starts one
          // (valid only at a chunk's first row: checked when the chunk ends).
          const bool inz = zr != 0;
          const uint32_t ei = lut[uint32_t(buf >> 32) >> (32 - kLutBits)];
          const uint32_t e = inz ? eR : ei;
          const int len = int(e >> 12);
          const int se = int(e & 4095);
          bad |= e == 0;  // not a code of the book; lane totals are checked at the end
          const bool isz = se == Zt;
          const int sy = isz ? Rc : se;
          zr = isz ? My - 1 : zr - (inz ? 1 : 0);
          buf <<= len;
          nb -= len;
          const bool is_out = sy == 0 && len != 0;
          const uint64_t wm = __ballot(is_out);
          uint16_t st = uint16_t(sy);
          if (wm != 0) {  // wave-uniform: outliers are rare
            const uint64_t mk = wm & segmask;
            if (is_out) st = uint16_t(0x8000u | ((run + __popcll(mk & ltmask)) & 0x7FFFu));
            run += __popcll(mk);
          }
          symb[so] = st;
          so += S::SP;
          if (++vy == My) {
            vy = 0;
            so += (m - My) * S::SP;
            bad |= zr != 0;  // a token after a chunk's first row runs past its end
          }
        }
      }
      wi = wb + uint64_t((rk - rb) & (RB - 1));  // words merged: fewer than RB per slab
      if constexpr (!kWhole) {
#pragma unroll
        for (int k = 0; k < WPL; ++k) ring[((rb + WPL + k) & (RB - 1)) * NL + tid] = pf[k];
      }
    }
    if constexpr (!kSlide && !kWhole) tile_store<S, T, NT>(tile, tr);
    __syncthreads();
    // ---- reconstruct the slab ------------------------------------------------------
    const int hs = min(S::H, Ez - z0);
    DecRows<T> ctx;
    ctx.tile = tile;
    ctx.symb = symb;
    ctx.uo0 = uo0;
    ctx.uo1 = uo1;
    ctx.outv = static_cast<const T*>(a.outv);
    ctx.flags = a.flags;
    ctx.cur = static_cast<T*>(a.cur);
    ctx.oz = oz;
    ctx.oy = oy;
    ctx.ox = ox;
    ctx.z0 = z0;
    ctx.tz0 = kWhole ? 0 : z0;
    ctx.a0 = a0;
    ctx.Ex = Ex;
    ctx.rz0 = rz0;
    ctx.rz1 = rz1;
    ctx.ry0 = ry0;
    ctx.ry1 = ry1;
    ctx.rx0 = rx0;
    ctx.rx1 = rx1;
    for (int d = 0; d < 3; ++d) {
      ctx.of[d] = a.out_first[d];
      ctx.oc[d] = a.out_cnt[d];
      ctx.n[d] = a.n[d];
    }
    if constexpr (sizeof(T) == 4)
      ctx.E2 = a.E2;
    else
      ctx.E2 = a.E2d;
    ctx.R = a.g.R;
    ctx.pair = (a.out_cnt[2] & 1) == 0 && ((ox - a.out_first[2]) & 1) == 0 &&
               (reinterpret_cast<uintptr_t>(a.cur) & (2 * sizeof(T) - 1)) == 0;
    if constexpr (NW >= 16) {
      // Wide work-groups (launches of few blocks, latency-bound): each group
      // of NW/4 waves reconstructs one parity type, the four at once.
      constexpr int GW = NW / 4;
      const int g = wave / GW, wg_ = wave % GW;
      if (interior) {
        if (g == 0) dec_type<T, E, H, GW, 0, 0, true, NTS>(ctx, hs, Ey, wg_, lane);
        else if (g == 1) dec_type<T, E, H, GW, 0, 1, true, NTS>(ctx, hs, Ey, wg_, lane);
        else if (g == 2) dec_type<T, E, H, GW, 1, 0, true, NTS>(ctx, hs, Ey, wg_, lane);
        else dec_type<T, E, H, GW, 1, 1, true, NTS>(ctx, hs, Ey, wg_, lane);
      } else {
        if (g == 0) dec_type<T, E, H, GW, 0, 0, false, NTS>(ctx, hs, Ey, wg_, lane);
        else if (g == 1) dec_type<T, E, H, GW, 0, 1, false, NTS>(ctx, hs, Ey, wg_, lane);
        else if (g == 2) dec_type<T, E, H, GW, 1, 0, false, NTS>(ctx, hs, Ey, wg_, lane);
        else dec_type<T, E, H, GW, 1, 1, false, NTS>(ctx, hs, Ey, wg_, lane);
      }
    } else if (interior) {
      dec_type<T, E, H, NW, 0, 0, true, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 0, 1, true, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 1, 0, true, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 1, 1, true, NTS>(ctx, hs, Ey, wave, lane);
    } else {
      dec_type<T, E, H, NW, 0, 0, false, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 0, 1, false, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 1, 0, false, NTS>(ctx, hs, Ey, wave, lane);
      dec_type<T, E, H, NW, 1, 1, false, NTS>(ctx, hs, Ey, wave, lane);
    }
    __syncthreads();
  }
  if (lane_active && alive && complete) {
    if (32 * wi - pos - uint64_t(nb) != uint64_t(lb)) bad = true;
    if (j == 0 && uok[c] && run != uo1[c] - uo0[c]) bad = true;
  }
  if (bad && lane_active && alive) atomicOr(a.flags, kFlagCorrupt);
}

// Waves per SIMD the decoder is compiled for: 6 for float fields in 32^3-point
// blocks (at most 80 VGPRs, no spills), so six work-groups of 26 KB LDS share
// a CU (the decode chains are latency-bound, so occupancy pays); 5 for double
// fields, whose wider values need more registers.
template <class T>
constexpr int dec_waves(int E) { return E == 32 ? (sizeof(T) == 4 ? 6 : 5) : 1; }
// Threads per work-group of the plain launches: blocks of at most 8^3 level
// points (at most 28 decoding lanes, a few hundred points) take one wave, so
// four times as many blocks fit on a CU; their latency chains overlap.
constexpr int slab_threads(int E) { return E <= 8 ? 64 : 256; }

template <class T, int E, bool NTS>
__global__ __launch_bounds__(slab_threads(E)) __attribute__((amdgpu_waves_per_eu(dec_waves<T>(E))))
void k_dec_slab(DecSlabArgs a) {
  dec_body<T, E, dec_slab_h(E), slab_threads(E), NTS>(a, blockIdx.x);
}

// Anchors of the box R_0 from the stream into the level-0 box grid.
template <class T>
__device__ inline void dec_anchor_body(const uint8_t* comp, uint64_t anchor_off, const Geo& g,
                                       T* rec0, const Grid& g0, uint64_t wg, uint64_t ngrid) {
  const int logs = g.L;
  const int64_t c1 = ((g.n[1] - 1) >> logs) + 1, c2 = ((g.n[2] - 1) >> logs) + 1;
  const T* an = reinterpret_cast<const T*>(comp + anchor_off);
  const int64_t n = g0.cnt[0] * g0.cnt[1] * g0.cnt[2];
  for (int64_t i = int64_t(wg) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(ngrid) * blockDim.x) {
    const int64_t ix = i % g0.cnt[2], t = i / g0.cnt[2], iy = t % g0.cnt[1], iz = t / g0.cnt[1];
    const int64_t z = g0.first[0] + (iz << logs), y = g0.first[1] + (iy << logs),
                  x = g0.first[2] + (ix << logs);
    rec0[i] = an[((z >> logs) * c1 + (y >> logs)) * c2 + (x >> logs)];
  }
}

template <class T>
__global__ void k_dec_anchor(const uint8_t* comp, uint64_t anchor_off, Geo g, T* rec0, Grid g0,
                             uint32_t* flags, const HdrRef ref) {
  // the call's corruption flag starts at zero (the level kernels follow in
  // stream order)
  if (blockIdx.x == 0 && threadIdx.x == 0) *flags = 0;
  if (ref.n && blockIdx.x == 0) {
    // a kept header: flags[1] = whether the stream's header bytes differ
    bool d = false;
    for (uint32_t i = threadIdx.x; i < ref.n; i += blockDim.x) d |= comp[i] != ref.b[i];
    const int any = __syncthreads_or(d ? 1 : 0);
    if (threadIdx.x == 0) flags[1] = any ? 1u : 0u;
  }
  dec_anchor_body<T>(comp, anchor_off, g, rec0, g0, blockIdx.x, gridDim.x);
}

// Level-k argument block of a decode, built the same way on the host (plain
// launches) and on the device (batched launches, from the request table).
__host__ __device__ inline DecSlabArgs dec_args(const DecodeArgs& a, int k) {
  const Geo& g = a.geo;
  const int logs = g.L - k;
  const Grid gp = box_grid(a.box[k - 1], logs + 1);
  const Grid gc = box_grid(a.box[k], logs);
  DecSlabArgs d;
  d.g = g;
  d.level = k;
  d.logs = logs;
  bool full = true;
  for (int q = 0; q < 3; ++q) {
    d.n[q] = ((g.n[q] - 1) >> logs) + 1;
    // grids in level coordinates: level-k coordinate = full / 2^logs
    d.in_first[q] = gp.first[q] >> (logs + 1);
    d.in_cnt[q] = gp.cnt[q];
    d.out_first[q] = gc.first[q] >> logs;
    d.out_cnt[q] = gc.cnt[q];
    d.bb_lo[q] = a.box[k].lo[q] >> g.logB;
    d.bb_n[q] = ((a.box[k].hi[q] - 1) >> g.logB) - d.bb_lo[q] + 1;
    full = full && a.box[k].lo[q] == 0 && a.box[k].hi[q] == g.n[q];
  }
  d.xcd_remap = full;
  d.prev = a.rec[k - 1];
  d.cur = a.rec[k];
  d.unit_word = reinterpret_cast<const uint32_t*>(a.comp + a.sec[k]);
  d.unit_outl = reinterpret_cast<const uint32_t*>(a.comp + a.off_outl[k]);
  d.lane_len = reinterpret_cast<const uint16_t*>(a.comp + a.off_lane[k]);
  d.pay = reinterpret_cast<const uint32_t*>(a.comp + a.off_pay[k]);
  d.outv = a.comp + a.off_out[k];
  d.words = a.words[k];
  d.noutl = a.outl[k];
  d.nlanes = a.lc[k].nl;
  d.nu = a.lc[k].nu;
  d.E2 = a.E2[k];
  d.E2d = a.E2d[k];
  d.lut = a.lut;
  d.flags = a.flags;
  return d;
}


// Launches of fewer blocks than CUs, each block alone on its CU, are bound by
// one block's latency: 1024-thread work-groups reconstruct the four parity
// types of a slab at once (blocks of 16^3 points and more).
template <class T, int E, bool NTS>
__global__ __launch_bounds__(1024) void k_dec_slab_wide(DecSlabArgs a) {
  dec_body<T, E, dec_slab_h(E), 1024, NTS>(a, blockIdx.x);
}
constexpr int64_t kWideBlocks = 256;

template <class T, int E>
void launch_slab(const DecSlabArgs& d, int64_t nblk, bool nts, hipStream_t st) {
  if constexpr (E >= 16) {
    if (nblk < kWideBlocks) {
      if (nts)
        hipLaunchKernelGGL((k_dec_slab_wide<T, E, true>), dim3(unsigned(nblk)), dim3(1024), 0, st,
                           d);
      else
        hipLaunchKernelGGL((k_dec_slab_wide<T, E, false>), dim3(unsigned(nblk)), dim3(1024), 0,
                           st, d);
      return;
    }
  }
  if (nts)
    hipLaunchKernelGGL((k_dec_slab<T, E, true>), dim3(unsigned(nblk)), dim3(slab_threads(E)), 0,
                       st, d);
  else
    hipLaunchKernelGGL((k_dec_slab<T, E, false>), dim3(unsigned(nblk)), dim3(slab_threads(E)), 0,
                       st, d);
}

// Plain launch of one level of a decode, by level block edge; nts = the level
// writes the call's final output (non-temporal stores).
template <class T>
void launch_slab_e(int E, const DecSlabArgs& d, int64_t nblk, bool nts, hipStream_t st) {
  switch (E) {
    case 2: launch_slab<T, 2>(d, nblk, nts, st); break;
    case 4: launch_slab<T, 4>(d, nblk, nts, st); break;
    case 8: launch_slab<T, 8>(d, nblk, nts, st); break;
    case 16: launch_slab<T, 16>(d, nblk, nts, st); break;
    case 32: launch_slab<T, 32>(d, nblk, nts, st); break;
    default: launch_slab<T, 64>(d, nblk, nts, st); break;
  }
}

// ---- batched decoding over a request table ----------------------------------
__device__ inline int map_find_d(const ItemMap& m, uint32_t item, uint32_t* loc, uint32_t* cnt) {
  int lo = 0, hi = int(m.n);  // first[lo] <= item < first[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m.first[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: scalar registers
  *loc = __builtin_amdgcn_readfirstlane(item - m.first[lo]);
  *cnt = __builtin_amdgcn_readfirstlane(m.first[lo + 1] - m.first[lo]);
  return __builtin_amdgcn_readfirstlane(int(m.job[lo]));
}

#define STZ_FOR_ITEMS(m)                                                    \
  for (uint32_t it_ = blockIdx.x, tot_ = (m).first[(m).n]; it_ < tot_;      \
       it_ += gridDim.x, __syncthreads())

__global__ void kb_dec_anchor(const DecodeArgs* R, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const DecodeArgs& a = R[map_find_d(m, it_, &loc, &cnt)];
    dec_anchor_body<float>(a.comp, a.anchor_off, a.geo, static_cast<float*>(a.rec[0]),
                           box_grid(a.box[0], a.geo.L), loc, cnt);
  }
}

// Per-level argument blocks of a batch are built on the host (the same
// builder as the plain launches) and read here through restrict pointers.
template <int E, int H>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(H == dec_slab_h(E) ? dec_waves<float>(E) : 1)))
void kb_dec(const DecSlabArgs* __restrict__ D, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const DecSlabArgs d = uniform_load(D + map_find_d(m, it_, &loc, &cnt));
    // padded range (multiple of 8): contiguous blocks per XCD, padding skipped
    const int64_t blk = wg_block(loc, cnt, true);
    if (blk < d.bb_n[0] * d.bb_n[1] * d.bb_n[2]) dec_body<float, E, H>(d, blk);
  }
}

// Batched levels with fewer blocks than CUs (a few small requests): one
// 1024-thread work-group per block, as the plain path's wide launches.
template <int E>
__global__ __launch_bounds__(1024) void kb_dec_wide(const DecSlabArgs* __restrict__ D, ItemMap m) {
  STZ_FOR_ITEMS(m) {
    uint32_t loc, cnt;
    const DecSlabArgs d = uniform_load(D + map_find_d(m, it_, &loc, &cnt));
    const int64_t blk = wg_block(loc, cnt, true);
    if (blk < d.bb_n[0] * d.bb_n[1] * d.bb_n[2]) dec_body<float, E, dec_slab_h(E), 1024>(d, blk);
  }
}

template <int E, int H>
void launch_dec_b(const DecSlabArgs* D, const ItemMap& m, unsigned grid, hipStream_t st) {
  hipLaunchKernelGGL((kb_dec<E, H>), dim3(grid), dim3(256), 0, st, D, m);
}

// Slab heights the batched decoder is built for, per level block edge.
template <int E>
void launch_dec_bh(int h, const DecSlabArgs* D, const ItemMap& m, unsigned grid,
                   hipStream_t st) {
  if constexpr (E == 16) {
    if (h == 4) return launch_dec_b<16, 4>(D, m, grid, st);
    if (h == 8) return launch_dec_b<16, 8>(D, m, grid, st);
  } else if constexpr (E == 32) {
    if (h == 2) return launch_dec_b<32, 2>(D, m, grid, st);
    if (h == 8) return launch_dec_b<32, 8>(D, m, grid, st);
  }
  launch_dec_b<E, dec_slab_h(E)>(D, m, grid, st);
}

}  // namespace

// ROI statistics (Sec. 3.3): maximum and minimum of one unit of a level grid
// (dims gn, stride s), unit = a block of B^3 full-resolution points (E = B/s
// grid points per axis) or one plane across an axis; stat 0 = max, 1 = range.
template <class T>
__global__ __launch_bounds__(256) void k_roi_stats(const T* __restrict__ grid, int64_t gn0,
                                                   int64_t gn1, int64_t gn2, int64_t E, int unit,
                                                   int stat, int64_t nb1, int64_t nb2,
                                                   double* out) {
  const int64_t u = blockIdx.x;
  int64_t lo[3] = {0, 0, 0}, hi[3] = {gn0, gn1, gn2};
  if (unit == 0) {
    const int64_t b[3] = {u / (nb1 * nb2), (u / nb2) % nb1, u % nb2};
    for (int d = 0; d < 3; ++d) {
      lo[d] = b[d] * E;
      hi[d] = min(hi[d], lo[d] + E);
    }
  } else {
    lo[unit - 1] = u;
    hi[unit - 1] = u + 1;
  }
  const int64_t e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
  const int64_t cnt = (hi[0] - lo[0]) * e1 * e2;
  // max/min are exact in any order, in either value type
  T mx = T(-INFINITY), mn = T(INFINITY);
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int64_t x = i % e2, t = i / e2, y = t % e1, z = t / e1;
    const T v = grid[((lo[0] + z) * gn1 + lo[1] + y) * gn2 + lo[2] + x];
    mx = v > mx ? v : mx;
    mn = v < mn ? v : mn;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const T a = __shfl_xor(mx, o, kWave), b = __shfl_xor(mn, o, kWave);
    mx = a > mx ? a : mx;
    mn = b < mn ? b : mn;
  }
  __shared__ T smx[4], smn[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smx[w] = mx;
    smn[w] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mx = smx[i] > mx ? smx[i] : mx;
      mn = smn[i] < mn ? smn[i] : mn;
    }
    out[u] = stat == 0 ? (double)mx : (double)mx - (double)mn;
  }
}

hipError_t launch_roi_stats(const void* grid, int vb, const int64_t gn[3], int64_t E, int unit,
                            int stat, const int64_t nb[3], uint64_t nunits, double* out,
                            hipStream_t st) {
  if (nunits == 0) return hipSuccess;
  prof_begin(st, "roi_stats", -1);
  if (vb == 8)
    hipLaunchKernelGGL(k_roi_stats<double>, dim3(unsigned(nunits)), dim3(256), 0, st,
                       static_cast<const double*>(grid), gn[0], gn[1], gn[2], E, unit, stat,
                       nb[1], nb[2], out);
  else
    hipLaunchKernelGGL(k_roi_stats<float>, dim3(unsigned(nunits)), dim3(256), 0, st,
                       static_cast<const float*>(grid), gn[0], gn[1], gn[2], E, unit, stat,
                       nb[1], nb[2], out);
  prof_end(st);
  return hipGetLastError();
}

namespace {

// Device-side ROI selection (Sec. 3.3, ROI workflow) over per-unit statistics.
// rule 0 keeps the units whose statistic exceeds a threshold; rule 1 keeps the
// k largest, ties to the smaller index. Rule 1 finds the k-th largest
// statistic by radix selection on an order-preserving 64-bit key (eight 8-bit
// digit passes, most significant first), so a unit is taken when its key is
// above that key, or equal to it and among the first `need` equal ones in
// index order. The compaction then writes the taken indices in ascending
// order; with one chunk it runs in one work-group, else chunk counts are
// scanned first.
struct RoiState {
  uint64_t prefix;  // digits of the k-th largest key fixed so far
  uint64_t mask;    // which digits are fixed
  uint64_t kr;      // its rank among the keys that match prefix (1-based);
                    // after the last pass, how many keys equal to it are taken
  uint64_t pad;
  uint32_t hist[256];
};
static_assert(sizeof(RoiState) <= kRoiStateBytes, "ROI state size");
constexpr int kRoiOneMax = 16384;  // units handled by the one-work-group path
constexpr int kRoiChunks = 1024;   // chunks of the multi-work-group path

// Order-preserving key: a > b as doubles iff key(a) > key(b); -0 and +0 equal.
__device__ __forceinline__ uint64_t roi_key(double v) {
  const uint64_t b = v == 0.0 ? 0ull : uint64_t(__double_as_longlong(v));
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

// Fix the next digit from a histogram of the keys matching the prefix.
__device__ void roi_pick(const uint32_t* hist, uint64_t& prefix, uint64_t& mask, uint64_t& kr,
                         int shift) {
  uint64_t acc = 0;
  int d = 255;
  for (; d > 0; --d) {
    if (acc + hist[d] >= kr) break;
    acc += hist[d];
  }
  kr -= acc;
  prefix |= uint64_t(d) << shift;
  mask |= 0xffull << shift;
}

// Rule 1 threshold for n <= kRoiOneMax: one work-group, keys kept in registers.
__global__ __launch_bounds__(1024) void k_roi_radix_one(const double* __restrict__ st,
                                                        uint64_t n, uint64_t k,
                                                        RoiState* __restrict__ out) {
  constexpr int kPer = kRoiOneMax / 1024;
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix, s_mask, s_kr;
  const int tid = threadIdx.x;
  uint64_t key[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const uint64_t i = uint64_t(j) * 1024 + tid;
    key[j] = i < n ? roi_key(st[i]) : 0;
  }
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_kr = k;
  }
  for (int shift = 56; shift >= 0; shift -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    const uint64_t p = s_prefix, m = s_mask;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const uint64_t i = uint64_t(j) * 1024 + tid;
      if (i < n && (key[j] & m) == p) atomicAdd(&hist[(key[j] >> shift) & 255], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t pr = s_prefix, ms = s_mask, kr = s_kr;
      roi_pick(hist, pr, ms, kr, shift);
      s_prefix = pr;
      s_mask = ms;
      s_kr = kr;
    }
    __syncthreads();
  }
  if (tid == 0) {
    out->prefix = s_prefix;
    out->mask = s_mask;
    out->kr = s_kr;
  }
}

// Rule 1 threshold for large n: a grid-wide histogram and a one-group pick per digit.
__global__ __launch_bounds__(256) void k_roi_init(RoiState* __restrict__ s, uint64_t k) {
  s->hist[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    s->prefix = 0;
    s->mask = 0;
    s->kr = k;
  }
}

__global__ __launch_bounds__(256) void k_roi_hist(const double* __restrict__ st, uint64_t n,
                                                  RoiState* __restrict__ s, int shift) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint64_t p = s->prefix, m = s->mask;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + tid; i < n; i += uint64_t(gridDim.x) * 256) {
    const uint64_t key = roi_key(st[i]);
    if ((key & m) == p) atomicAdd(&h[(key >> shift) & 255], 1u);
  }
  __syncthreads();
  if (h[tid]) atomicAdd(&s->hist[tid], h[tid]);
}

__global__ __launch_bounds__(256) void k_roi_pick(RoiState* __restrict__ s, int shift) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = s->hist[tid];
  s->hist[tid] = 0;
  __syncthreads();
  if (tid == 0) {
    uint64_t pr = s->prefix, ms = s->mask, kr = s->kr;
    roi_pick(h, pr, ms, kr, shift);
    s->prefix = pr;
    s->mask = ms;
    s->kr = kr;
  }
}

__device__ __forceinline__ void roi_class(double v, int rule, double value, uint64_t T,
                                          bool& gt, bool& eq) {
  if (rule == 0) {
    gt = v > value;
    eq = false;
  } else {
    const uint64_t key = roi_key(v);
    gt = key > T;
    eq = key == T;
  }
}

// Per-chunk counts of units above the threshold and equal to it.
__global__ __launch_bounds__(1024) void k_roi_count(const double* __restrict__ st, uint64_t n,
                                                    int rule, double value,
                                                    const RoiState* __restrict__ s,
                                                    uint64_t chunk, uint64_t* __restrict__ cnt) {
  __shared__ uint32_t c_gt, c_eq;
  const int tid = threadIdx.x;
  if (tid == 0) c_gt = c_eq = 0;
  __syncthreads();
  const uint64_t T = rule == 1 ? s->prefix : 0;
  const uint64_t lo = uint64_t(blockIdx.x) * chunk, hi = lo + chunk < n ? lo + chunk : n;
  uint32_t ngt = 0, neq = 0;
  for (uint64_t u = lo + tid; u < hi; u += 1024) {
    bool gt, eq;
    roi_class(st[u], rule, value, T, gt, eq);
    ngt += gt;
    neq += eq;
  }
  if (ngt) atomicAdd(&c_gt, ngt);
  if (neq) atomicAdd(&c_eq, neq);
  __syncthreads();
  if (tid == 0) {
    cnt[2 * blockIdx.x] = c_gt;
    cnt[2 * blockIdx.x + 1] = c_eq;
  }
}

// Inclusive scan of one value per thread over a 1024-thread group.
__device__ uint64_t roi_scan1024(uint64_t v, uint64_t* buf) {
  const int tid = threadIdx.x;
  buf[tid] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t add = tid >= d ? buf[tid - d] : 0;
    __syncthreads();
    buf[tid] += add;
    __syncthreads();
  }
  return buf[tid];
}

// Chunk offsets: where each chunk's first taken index goes, and how many
// equal keys come before it; the total taken goes to *count.
__global__ __launch_bounds__(1024) void k_roi_scan(const uint64_t* __restrict__ cnt, int C,
                                                   int rule, const RoiState* __restrict__ s,
                                                   uint64_t* __restrict__ offs,
                                                   uint64_t* __restrict__ count) {
  __shared__ uint64_t buf[1024];
  const int tid = threadIdx.x;
  const uint64_t gt = tid < C ? cnt[2 * tid] : 0, eq = tid < C ? cnt[2 * tid + 1] : 0;
  const uint64_t need = rule == 1 ? s->kr : 0;
  const uint64_t eq_before = roi_scan1024(eq, buf) - eq;
  const uint64_t left = need > eq_before ? need - eq_before : 0;
  const uint64_t take = gt + (left < eq ? left : eq);
  const uint64_t sel_incl = roi_scan1024(take, buf);
  if (tid < C) {
    offs[2 * tid] = sel_incl - take;
    offs[2 * tid + 1] = eq_before;
  }
  if (tid == 1023) *count = sel_incl;
}

// Ascending indices of the taken units of each chunk. Without offsets there is
// one chunk (the whole range), and the total goes to *count.
__global__ __launch_bounds__(1024) void k_roi_write(const double* __restrict__ st, uint64_t n,
                                                    int rule, double value,
                                                    const RoiState* __restrict__ s,
                                                    uint64_t chunk,
                                                    const uint64_t* __restrict__ offs,
                                                    uint32_t* __restrict__ sel, uint64_t cap,
                                                    uint64_t* __restrict__ count) {
  __shared__ uint32_t w_eq[16], w_tk[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t lanemask = (1ull << lane) - 1;
  const uint64_t T = rule == 1 ? s->prefix : 0;
  const uint64_t need = rule == 1 ? s->kr : 0;
  uint64_t sel_base = offs ? offs[2 * blockIdx.x] : 0;
  uint64_t eq_base = offs ? offs[2 * blockIdx.x + 1] : 0;
  const uint64_t lo = uint64_t(blockIdx.x) * chunk, hi = lo + chunk < n ? lo + chunk : n;
  for (uint64_t c0 = lo; c0 < hi; c0 += 1024) {
    const uint64_t u = c0 + tid;
    bool gt = false, eq = false;
    if (u < hi) roi_class(st[u], rule, value, T, gt, eq);
    const uint64_t beq = __ballot(eq);
    if (lane == 0) w_eq[w] = uint32_t(__popcll(beq));
    __syncthreads();
    uint64_t eq_w = 0, eq_all = 0;
    for (int i = 0; i < 16; ++i) {
      eq_w += i < w ? w_eq[i] : 0u;
      eq_all += w_eq[i];
    }
    const uint64_t eqrank = eq_base + eq_w + __popcll(beq & lanemask);
    const bool take = gt || (eq && eqrank < need);
    const uint64_t btk = __ballot(take);
    if (lane == 0) w_tk[w] = uint32_t(__popcll(btk));
    __syncthreads();
    uint64_t tk_w = 0, tk_all = 0;
    for (int i = 0; i < 16; ++i) {
      tk_w += i < w ? w_tk[i] : 0u;
      tk_all += w_tk[i];
    }
    const uint64_t pos = sel_base + tk_w + __popcll(btk & lanemask);
    if (take && pos < cap) sel[pos] = uint32_t(u);
    sel_base += tk_all;
    eq_base += eq_all;
    __syncthreads();
  }
  if (!offs && tid == 0) *count = sel_base;
}

}  // namespace

hipError_t launch_roi_select(const double* stats, uint64_t n, int rule, double value, uint64_t k,
                             void* scratch, uint32_t* sel, uint64_t cap, uint64_t* count,
                             hipStream_t st) {
  if (n > 0xffffffffull) return hipErrorInvalidValue;
  auto* s = static_cast<RoiState*>(scratch);
  auto* offs = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(scratch) + kRoiStateBytes);
  prof_begin(st, "roi_select", -1);
  if (n <= uint64_t(kRoiOneMax)) {
    if (rule == 1)
      hipLaunchKernelGGL(k_roi_radix_one, dim3(1), dim3(1024), 0, st, stats, n, k, s);
    hipLaunchKernelGGL(k_roi_write, dim3(1), dim3(1024), 0, st, stats, n, rule, value, s, n,
                       static_cast<const uint64_t*>(nullptr), sel, cap, count);
  } else {
    if (rule == 1) {
      const unsigned G = unsigned(std::min<uint64_t>(1024, (n + 4095) / 4096));
      hipLaunchKernelGGL(k_roi_init, dim3(1), dim3(256), 0, st, s, k);
      for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_roi_hist, dim3(G), dim3(256), 0, st, stats, n, s, shift);
        hipLaunchKernelGGL(k_roi_pick, dim3(1), dim3(256), 0, st, s, shift);
      }
    }
    const uint64_t C0 = std::min<uint64_t>(kRoiChunks, (n + 8191) / 8192);
    const uint64_t chunk = (n + C0 - 1) / C0;
    const int C = int((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_roi_count, dim3(C), dim3(1024), 0, st, stats, n, rule, value, s, chunk,
                       offs + 2 * kRoiChunks);
    hipLaunchKernelGGL(k_roi_scan, dim3(1), dim3(1024), 0, st, offs + 2 * kRoiChunks, C, rule, s,
                       offs, count);
    hipLaunchKernelGGL(k_roi_write, dim3(C), dim3(1024), 0, st, stats, n, rule, value, s, chunk,
                       static_cast<const uint64_t*>(offs), sel, cap, count);
  }
  prof_end(st);
  return hipGetLastError();
}

namespace {

template <class T>
hipError_t launch_decode_t(const DecodeArgs& a, hipStream_t st, const HdrRef* ref) {
  const Geo& g = a.geo;
  const int L = g.L;
  const Grid g0 = box_grid(a.box[0], L);
  const uint64_t n0 = uint64_t(g0.cnt[0]) * g0.cnt[1] * g0.cnt[2];
  prof_begin(st, "dec_anchor", -1);
  hipLaunchKernelGGL(k_dec_anchor<T>, dim3(grid_for(n0, 256, 4096)), dim3(256), 0, st, a.comp,
                     a.anchor_off, g, static_cast<T*>(a.rec[0]), g0, a.flags, *ref);
  prof_end(st);
  for (int k = 1; k <= a.level_out; ++k) {
    const DecSlabArgs d = dec_args(a, k);
    const int64_t nblk = d.bb_n[0] * d.bb_n[1] * d.bb_n[2];
    const int E = g.B >> (L - k);
    prof_begin(st, d.xcd_remap ? "decode" : "rdecode", k);
    launch_slab_e<T>(E, d, nblk, k == a.level_out, st);
    prof_end(st);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_decode(const DecodeArgs& a, hipStream_t st, const HdrRef* ref) {
  static const HdrRef kNoRef = {};  // n = 0: no check
  if (!ref) ref = &kNoRef;
  return a.vb == 8 ? launch_decode_t<double>(a, st, ref) : launch_decode_t<float>(a, st, ref);
}

uint64_t decode_batch_args_bytes(uint32_t n, int max_level) {
  return uint64_t(n) * uint64_t(max_level) * sizeof(DecSlabArgs);
}

void build_decode_batch_args(const DecodeArgs* reqs, uint32_t n, int max_level, uint8_t* dst) {
  auto* D = reinterpret_cast<DecSlabArgs*>(dst);
  std::memset(dst, 0, decode_batch_args_bytes(n, max_level));
  for (int k = 1; k <= max_level; ++k)
    for (uint32_t r = 0; r < n; ++r) {
      if (reqs[r].level_out < k) continue;
      DecSlabArgs d = dec_args(reqs[r], k);
      d.xcd_remap = false;
      D[uint64_t(k - 1) * n + r] = d;
    }
}

hipError_t launch_decode_batch(const DecodeBatch& b, hipStream_t st) {
  auto grid = [](unsigned cap, uint32_t total) {
    return std::max(1u, std::min<unsigned>(cap, total));
  };
  prof_begin(st, "b_dec_anchor", -1);
  hipLaunchKernelGGL(kb_dec_anchor, dim3(grid(b.grid, b.n_anchor)), dim3(256), 0, st, b.R,
                     b.anchor);
  prof_end(st);
  for (int k = 1; k <= b.max_level; ++k) {
    // Requests with many blocks at this level fill the device on their own:
    // they get the plain launch (arguments by value, in scalar registers).
    for (uint32_t i = 0; i < b.n_direct; ++i) {
      if (b.direct[i].level != k) continue;
      const DecSlabArgs d = dec_args(b.host_R[b.direct[i].req], k);
      const int64_t nblk = d.bb_n[0] * d.bb_n[1] * d.bb_n[2];
      prof_begin(st, "b_decode_direct", k);
      launch_slab_e<float>(d.g.B >> (d.g.L - k), d, nblk,
                           k == b.host_R[b.direct[i].req].level_out, st);
      prof_end(st);
    }
    if (!b.n_check[k]) continue;
    const DecSlabArgs* D = reinterpret_cast<const DecSlabArgs*>(b.args) + uint64_t(k - 1) * b.nreq;
    for (int e = 1; e < kBatchEdges; ++e) {
      if (!b.n_dec[k][e]) continue;
      const unsigned gd = grid(b.grid_dec[e], b.n_dec[k][e]);
      const int h = b.dec_h[e];
      prof_begin(st, "b_decode", k);
      if (e >= 4 && b.n_dec[k][e] < kWideBlocks) {
        const dim3 gw(b.n_dec[k][e]), tw(1024);
        if (e == 4)
          hipLaunchKernelGGL(kb_dec_wide<16>, gw, tw, 0, st, D, b.dec[k][e]);
        else if (e == 5)
          hipLaunchKernelGGL(kb_dec_wide<32>, gw, tw, 0, st, D, b.dec[k][e]);
        else
          hipLaunchKernelGGL(kb_dec_wide<64>, gw, tw, 0, st, D, b.dec[k][e]);
        prof_end(st);
        continue;
      }
      switch (e) {
        case 1: launch_dec_bh<2>(h, D, b.dec[k][e], gd, st); break;
        case 2: launch_dec_bh<4>(h, D, b.dec[k][e], gd, st); break;
        case 3: launch_dec_bh<8>(h, D, b.dec[k][e], gd, st); break;
        case 4: launch_dec_bh<16>(h, D, b.dec[k][e], gd, st); break;
        case 5: launch_dec_bh<32>(h, D, b.dec[k][e], gd, st); break;
        default: launch_dec_bh<64>(h, D, b.dec[k][e], gd, st); break;
      }
      prof_end(st);
    }
  }
  return hipGetLastError();
}

}  // namespace stz
