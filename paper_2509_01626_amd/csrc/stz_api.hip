// Host side of the C ABI declared in include/stz.h: argument validation,
// stream-header parsing, workspace management and kernel launch sequences.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "stz.h"
#include "stz_internal.h"

namespace stz {

void prof_flush();

namespace {

struct Cfg {
  int B, logB, L, R;
  double ratio;
};

stz_status resolve_cfg(const stz_config* c, Cfg* o) {
  stz_config d = {0, 0, 0, 0, 0.0};
  if (c) d = *c;
  if (d.reserved != 0) return STZ_ERR_ARG;
  const int B = d.block ? int(d.block) : 32;
  if (B < 2 || B > 64 || (B & (B - 1))) return STZ_ERR_ARG;
  int k = 0;
  while ((1 << k) < B) ++k;
  const int L = d.levels ? int(d.levels) : k;
  if (L < 1 || L > k) return STZ_ERR_ARG;
  const int R = d.radius ? int(d.radius) : 512;
  if (R < 1 || R > kMaxRadius) return STZ_ERR_ARG;
  const double ratio = d.eb_ratio != 0.0 ? d.eb_ratio : 2.5;
  if (!(ratio >= 1.0) || !std::isfinite(ratio)) return STZ_ERR_ARG;
  o->B = B;
  o->logB = k;
  o->L = L;
  o->R = R;
  o->ratio = ratio;
  return STZ_OK;
}

bool make_geo(const uint64_t dims[3], const Cfg& c, Geo* g) {
  uint64_t N = 1;
  for (int d = 0; d < 3; ++d) {
    if (dims[d] < 1 || dims[d] > (uint64_t(1) << 32)) return false;
    N *= dims[d];
    if (N > (uint64_t(1) << 40)) return false;
    g->n[d] = int64_t(dims[d]);
    g->nb[d] = (int64_t(dims[d]) + c.B - 1) / c.B;
  }
  g->B = c.B;
  g->logB = c.logB;
  g->L = c.L;
  g->R = c.R;
  return true;
}

uint64_t grid_count(const Geo& g, int logs) {
  uint64_t n = 1;
  for (int d = 0; d < 3; ++d) n *= uint64_t(((g.n[d] - 1) >> logs) + 1);
  return n;
}

uint64_t n_units(const Geo& g) { return uint64_t(g.nb[0] * g.nb[1] * g.nb[2]) * 7; }

void level_consts(const Geo& g, LevelConst* lc) {
  for (int l = 1; l <= g.L; ++l) {
    lc[l].nu = n_units(g);
    lc[l].nl = uint64_t(level_nlanes(g, g.L - l));
    lc[l].nsym = uint64_t(level_nsym(g, g.L - l));
  }
}

// Keep freed stream-ordered allocations cached in the device pool.
void pool_setup() {
  static std::mutex mu;
  static bool done[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(mu);
  if (done[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = ~uint64_t(0);
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[dev] = true;
}

// Device scratch cached per (device, stream): every call on a stream reuses
// that stream's buffer, growing it when a call needs more. Calls on one stream
// run in stream order, so they never use the buffer at the same time; the
// allocation and release calls of the runtime (slow on the host) are paid
// only when a buffer grows. stz_trim() returns the buffers.
struct WsCache {
  std::mutex mu;
  std::unordered_map<uint64_t, std::pair<char*, uint64_t>> m;  // key -> (buffer, size)
};

WsCache& ws_cache() {
  static WsCache* c = new WsCache;  // never destroyed: may be used during exit
  return *c;
}

uint64_t ws_key(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  return (reinterpret_cast<uint64_t>(st) << 8) ^ uint64_t(dev & 255);
}

// Sub-buffers are laid out first (take), then the stream's cached buffer
// backs all of them (commit).
struct Workspace {
  hipStream_t st;
  char* base = nullptr;
  uint64_t size = 0;
  explicit Workspace(hipStream_t s) : st(s) { pool_setup(); }
  template <class T>
  uint64_t take(uint64_t n) {
    const uint64_t off = size;
    size += (std::max<uint64_t>(n, 1) * sizeof(T) + 255) & ~uint64_t(255);
    return off;
  }
  bool commit() {
    WsCache& c = ws_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto& e = c.m[ws_key(st)];
    if (e.second < size) {
      if (e.first) (void)hipFreeAsync(e.first, st);
      e.first = nullptr;
      e.second = 0;
      const uint64_t want = std::max<uint64_t>(size + size / 4, 1 << 20);
      void* p = nullptr;
      if (hipMallocAsync(&p, want, st) != hipSuccess) return false;
      e.first = static_cast<char*>(p);
      e.second = want;
    }
    base = e.first;
    return true;
  }
  template <class T>
  T* at(uint64_t off) const {
    return reinterpret_cast<T*>(base + off);
  }
};

// Per-thread pinned host staging for every small copy of a call: the decoder
// table with the flag reset behind it (host to device), the stream header and
// the status words (device to host). Pinned memory keeps these copies
// asynchronous DMA transfers; each call ends with a stream synchronization,
// after which the area may be reused.
struct Staging {
  static constexpr uint64_t kLutBytes = (uint64_t(1) << kLutBits) * 2 + 16;
  static constexpr uint64_t kHdrBytes = kHeaderBytes + 2 * kMaxRadius;
  uint8_t* base = nullptr;
  uint16_t* lut = nullptr;    // 2^kLutBits entries, then 16 zero bytes
  uint8_t* hdr = nullptr;     // stream header and code lengths
  DevParams* params = nullptr;
  uint32_t* flags = nullptr;
  Staging() {
    const uint64_t o_hdr = (kLutBytes + 255) & ~uint64_t(255);
    const uint64_t o_par = (o_hdr + kHdrBytes + 255) & ~uint64_t(255);
    const uint64_t o_flg = (o_par + sizeof(DevParams) + 255) & ~uint64_t(255);
    if (hipHostMalloc(reinterpret_cast<void**>(&base), o_flg + 256) != hipSuccess) {
      base = nullptr;
      return;
    }
    lut = reinterpret_cast<uint16_t*>(base);
    hdr = base + o_hdr;
    params = reinterpret_cast<DevParams*>(base + o_par);
    flags = reinterpret_cast<uint32_t*>(base + o_flg);
  }
  ~Staging() {
    if (base) (void)hipHostFree(base);
  }
};

Staging* staging() {
  thread_local Staging stage;
  return stage.base ? &stage : nullptr;
}

// Parsed stream header (format 2.5), validated against the geometry.
struct Header {
  Geo g;
  Cfg c;
  int eb_mode;
  double eb, eb_abs;
  uint64_t total, anchor_off, n_anchor;
  uint64_t sec[kMaxLevels + 1], words[kMaxLevels + 1], outl[kMaxLevels + 1];
  uint64_t off_outl[kMaxLevels + 1], off_lane[kMaxLevels + 1], off_pay[kMaxLevels + 1],
      off_out[kMaxLevels + 1];
  LevelConst lc[kMaxLevels + 1];
  std::vector<uint8_t> lens;
};

template <class T>
T rd(const uint8_t* p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}

stz_status read_header(const void* comp, uint64_t size, hipStream_t st, Header* h) {
  if (!comp || size < kHeaderBytes) return STZ_ERR_CORRUPT;
  const uint64_t want = std::min<uint64_t>(size, Staging::kHdrBytes);
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  if (hipMemcpyAsync(stage->hdr, comp, want, hipMemcpyDeviceToHost, st) != hipSuccess)
    return STZ_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return STZ_ERR_DEVICE;
  const uint8_t* p = stage->hdr;
  if (rd<uint32_t>(p) != kMagic || rd<uint32_t>(p + 4) != kVersion) return STZ_ERR_CORRUPT;
  uint64_t dims[3] = {rd<uint64_t>(p + 8), rd<uint64_t>(p + 16), rd<uint64_t>(p + 24)};
  stz_config cf;
  cf.block = rd<uint32_t>(p + 32);
  cf.levels = rd<uint32_t>(p + 36);
  cf.radius = rd<uint32_t>(p + 40);
  cf.reserved = 0;
  cf.eb_ratio = rd<double>(p + 72);
  if (!cf.block || !cf.levels || !cf.radius) return STZ_ERR_CORRUPT;
  if (rd<uint32_t>(p + 44) != uint32_t(kLmax)) return STZ_ERR_CORRUPT;
  if (resolve_cfg(&cf, &h->c) != STZ_OK || !make_geo(dims, h->c, &h->g)) return STZ_ERR_CORRUPT;
  h->eb_mode = int(rd<uint32_t>(p + 48));
  h->eb = rd<double>(p + 56);
  h->eb_abs = rd<double>(p + 64);
  if (!(h->eb_abs > 0.0) || !std::isfinite(h->eb_abs)) return STZ_ERR_CORRUPT;
  h->total = rd<uint64_t>(p + 80);
  if (h->total > size) return STZ_ERR_CORRUPT;
  const uint64_t nsym = 2 * uint64_t(h->c.R);
  if (rd<uint64_t>(p + 88) != kHeaderBytes) return STZ_ERR_CORRUPT;
  h->anchor_off = rd<uint64_t>(p + 96);
  h->n_anchor = rd<uint64_t>(p + 104);
  if (h->anchor_off != kHeaderBytes + align16(nsym)) return STZ_ERR_CORRUPT;
  if (h->n_anchor != grid_count(h->g, h->g.L)) return STZ_ERR_CORRUPT;
  if (kHeaderBytes + nsym > want) return STZ_ERR_CORRUPT;
  h->lens.assign(p + kHeaderBytes, p + kHeaderBytes + nsym);
  level_consts(h->g, h->lc);
  uint64_t pos = h->anchor_off + align16(4 * h->n_anchor);
  for (int l = 1; l <= h->g.L; ++l) {
    const uint8_t* e = p + kLevelTable + kLevelRec * uint64_t(l - 1);
    const uint64_t sec = rd<uint64_t>(e), nu = rd<uint64_t>(e + 8), nl = rd<uint64_t>(e + 16),
                   ns = rd<uint64_t>(e + 24), W = rd<uint64_t>(e + 32), O = rd<uint64_t>(e + 40);
    if (sec != pos || nu != h->lc[l].nu || nl != h->lc[l].nl || ns != h->lc[l].nsym)
      return STZ_ERR_CORRUPT;
    if (W > 0xFFFFFFFFull || O > ns) return STZ_ERR_CORRUPT;
    h->sec[l] = sec;
    h->words[l] = W;
    h->outl[l] = O;
    h->off_outl[l] = sec + align16(4 * (nu + 1));
    h->off_lane[l] = h->off_outl[l] + align16(4 * (nu + 1));
    h->off_pay[l] = h->off_lane[l] + align16(2 * nl);
    h->off_out[l] = h->off_pay[l] + align16(4 * W);
    pos = h->off_out[l] + align16(4 * O);
    if (pos > h->total) return STZ_ERR_CORRUPT;
  }
  if (pos != h->total) return STZ_ERR_CORRUPT;
  return STZ_OK;
}

// Decoder table: entry for every 12-bit window = symbol | length << 12, or 0
// when no code is a prefix of the window. Fails when the lengths do not form a
// prefix code.
bool build_lut(const std::vector<uint8_t>& lens, std::vector<uint16_t>* lut) {
  const int nsym = int(lens.size());
  uint32_t bl[kLmax + 1] = {0};
  uint64_t kraft = 0;  // in units of 2^-kLmax
  for (int i = 0; i < nsym; ++i) {
    if (lens[i] > kLmax) return false;
    if (lens[i]) {
      bl[lens[i]]++;
      kraft += uint64_t(1) << (kLmax - lens[i]);
    }
  }
  if (kraft > (uint64_t(1) << kLmax)) return false;
  uint32_t next[kLmax + 1] = {0};
  uint32_t code = 0;
  for (int l = 1; l <= kLmax; ++l) {
    code = (code + bl[l - 1]) << 1;
    next[l] = code;
  }
  lut->assign(size_t(1) << kLutBits, 0);
  for (int i = 0; i < nsym; ++i) {
    const int l = lens[i];
    if (!l) continue;
    const uint32_t c = next[l]++;
    const uint32_t lo = c << (kLutBits - l), n = 1u << (kLutBits - l);
    for (uint32_t k = 0; k < n; ++k) (*lut)[lo + k] = uint16_t(i | (l << 12));
  }
  return true;
}

Box dilate(const Box& b, int64_t r, const Geo& g) {
  Box o;
  for (int d = 0; d < 3; ++d) {
    o.lo[d] = b.lo[d] > r ? b.lo[d] - r : 0;
    o.hi[d] = std::min<int64_t>(g.n[d], b.hi[d] + r);
  }
  return o;
}

uint64_t box_points(const Box& b, int logs) {
  uint64_t n = 1;
  const int64_t s = int64_t(1) << logs;
  for (int d = 0; d < 3; ++d) {
    const int64_t f = (b.lo[d] + s - 1) >> logs << logs;
    n *= f < b.hi[d] ? uint64_t(((b.hi[d] - 1 - f) >> logs) + 1) : 0;
  }
  return n;
}

// Decode the box (null = the whole domain) at `level` (negative = finest).
stz_status decode_box(const void* comp, uint64_t size, const Box* boxp, int level, float* out,
                      uint64_t out_cap, uint64_t out_dims[3], hipStream_t st) {
  Header h;
  stz_status s = read_header(comp, size, st, &h);
  if (s != STZ_OK) return s;
  const Geo& g = h.g;
  if (level < 0) level = g.L;
  if (level > g.L) return STZ_ERR_ARG;
  Box box;
  if (boxp) {
    box = *boxp;
  } else {
    for (int d = 0; d < 3; ++d) {
      box.lo[d] = 0;
      box.hi[d] = g.n[d];
    }
  }
  for (int d = 0; d < 3; ++d)
    if (!(box.lo[d] < box.hi[d]) || box.hi[d] > g.n[d] || box.lo[d] < 0) return STZ_ERR_ARG;
  const int logs_out = g.L - level;
  const int64_t so = int64_t(1) << logs_out;
  uint64_t od[3];
  for (int d = 0; d < 3; ++d) {
    const int64_t f = (box.lo[d] + so - 1) >> logs_out << logs_out;
    od[d] = f < box.hi[d] ? uint64_t(((box.hi[d] - 1 - f) >> logs_out) + 1) : 0;
  }
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = od[d];
  const uint64_t cnt = od[0] * od[1] * od[2];
  if (cnt == 0) return STZ_OK;
  if (!out || cnt > out_cap) return STZ_ERR_BUFFER;
  std::vector<uint16_t> lut;
  if (!build_lut(h.lens, &lut)) return STZ_ERR_CORRUPT;

  DecodeArgs a;
  std::memset(&a, 0, sizeof(a));
  a.comp = static_cast<const uint8_t*>(comp);
  a.size = size;
  a.geo = g;
  a.level_out = level;
  a.box[level] = box;
  for (int k = level; k >= 1; --k) a.box[k - 1] = dilate(a.box[k], 3 * (int64_t(1) << (g.L - k)), g);
  Workspace ws(st);
  uint64_t o_rec[kMaxLevels + 1];
  for (int k = 0; k < level; ++k) o_rec[k] = ws.take<float>(box_points(a.box[k], g.L - k));
  const uint64_t o_lut = ws.take<uint8_t>(lut.size() * 2 + 16);
  if (!ws.commit()) return STZ_ERR_NOMEM;
  for (int k = 0; k < level; ++k) a.rec[k] = ws.at<float>(o_rec[k]);
  a.rec[level] = out;
  uint16_t* dlut = ws.at<uint16_t>(o_lut);
  uint32_t* dflags = reinterpret_cast<uint32_t*>(dlut + lut.size());
  for (int l = 1; l <= g.L; ++l) {
    a.sec[l] = h.sec[l];
    a.off_outl[l] = h.off_outl[l];
    a.off_lane[l] = h.off_lane[l];
    a.off_pay[l] = h.off_pay[l];
    a.off_out[l] = h.off_out[l];
    a.words[l] = h.words[l];
    a.outl[l] = h.outl[l];
    a.lc[l] = h.lc[l];
  }
  a.anchor_off = h.anchor_off;
  for (int l = 1; l <= g.L; ++l) {
    double e;
    if (l == g.L)
      e = h.eb_abs;
    else if (l == g.L - 1)
      e = h.eb_abs / h.c.ratio;
    else
      e = (h.eb_abs / h.c.ratio) / h.c.ratio;
    a.E2[l] = float(2.0 * e);
  }
  a.lut = dlut;
  a.flags = dflags;
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  std::memcpy(stage->lut, lut.data(), lut.size() * 2);
  std::memset(stage->lut + lut.size(), 0, 16);
  if (hipMemcpyAsync(dlut, stage->lut, lut.size() * 2 + 16, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return STZ_ERR_DEVICE;
  if (launch_decode(a, st) != hipSuccess) return STZ_ERR_DEVICE;
  if (hipMemcpyAsync(stage->flags, dflags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  prof_flush();
  return *stage->flags ? STZ_ERR_CORRUPT : STZ_OK;
}

}  // namespace
}  // namespace stz

using namespace stz;

extern "C" {

stz_status stz_trim(void) {
  WsCache& c = ws_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (hipDeviceSynchronize() != hipSuccess) return STZ_ERR_DEVICE;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return STZ_ERR_DEVICE;
  for (auto it = c.m.begin(); it != c.m.end();) {
    if (int(it->first & 255) == (cur & 255)) {
      if (it->second.first) (void)hipFreeAsync(it->second.first, nullptr);
      it = c.m.erase(it);
    } else {
      ++it;
    }
  }
  return hipDeviceSynchronize() == hipSuccess ? STZ_OK : STZ_ERR_DEVICE;
}

uint64_t stz_compress_bound(const uint64_t dims[3], const stz_config* cfg) {
  Cfg c;
  Geo g;
  if (!dims || resolve_cfg(cfg, &c) != STZ_OK || !make_geo(dims, c, &g)) return 0;
  LevelConst lc[kMaxLevels + 1];
  level_consts(g, lc);
  uint64_t total = kHeaderBytes + align16(2 * uint64_t(c.R)) + align16(4 * grid_count(g, g.L));
  for (int l = 1; l <= g.L; ++l) {
    const uint64_t nu = lc[l].nu;
    // every unit: at most kLmax bits per symbol plus one padding word
    const uint64_t words = (lc[l].nsym * kLmax + 31) / 32 + nu;
    total += 2 * align16(4 * (nu + 1)) + align16(2 * lc[l].nl) + align16(4 * words) +
             align16(4 * lc[l].nsym);
  }
  return total;
}

stz_status stz_compress(const float* x, const uint64_t dims[3], int eb_mode, double eb,
                        const stz_config* cfg, void* out, uint64_t out_cap, uint64_t* out_size,
                        void* stream) {
  Cfg c;
  Geo g;
  if (!x || !dims || !out_size) return STZ_ERR_ARG;
  if (resolve_cfg(cfg, &c) != STZ_OK || !make_geo(dims, c, &g)) return STZ_ERR_ARG;
  if (eb_mode != STZ_EB_ABS && eb_mode != STZ_EB_REL) return STZ_ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb)) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint64_t N = uint64_t(g.n[0]) * g.n[1] * g.n[2];
  const int L = g.L, nsym = 2 * g.R;

  CompressArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.geo = g;
  a.eb_mode = eb_mode;
  a.eb = eb;
  a.ratio = c.ratio;
  a.out = static_cast<uint8_t*>(out);
  a.out_cap = out ? out_cap : 0;
  level_consts(g, a.lc);
  a.n_anchor = grid_count(g, L);
  const uint64_t nu = a.lc[1].nu;
  if (nu > 0xFFFFFFF0ull) return STZ_ERR_ARG;

  Workspace ws(st);
  const uint64_t o_params = ws.take<DevParams>(1);
  a.nparts = uint32_t(std::min<uint64_t>(1024, (N + 4095) / 4096));
  const uint64_t o_part = ws.take<float2>(a.nparts);
  uint64_t o_rec[kMaxLevels], o_sym[kMaxLevels + 1];
  for (int l = 0; l < L; ++l) o_rec[l] = ws.take<float>(grid_count(g, L - l));
  uint64_t lanes = 0;
  for (int l = 1; l <= L; ++l) {
    o_sym[l] = ws.take<uint16_t>(a.lc[l].nsym);
    a.lane_base[l] = lanes;
    lanes += a.lc[l].nl;
  }
  const uint64_t o_lane = ws.take<uint16_t>(lanes);
  const uint64_t o_hist = ws.take<unsigned long long>(nsym);
  const uint64_t o_lens = ws.take<uint8_t>(nsym);
  const uint64_t o_codes = ws.take<uint16_t>(nsym);
  const uint64_t o_cb = ws.take<uint8_t>(codebook_scratch_bytes(nsym));
  const uint64_t o_cnt = ws.take<uint32_t>(2 * L * nu);
  const uint64_t o_scan = ws.take<uint32_t>(2 * L * (nu + 1));
  const uint64_t nblk = (nu + 2047) / 2048;
  const uint64_t o_spart = ws.take<uint64_t>(2 * L * nblk);
  if (!ws.commit()) return STZ_ERR_NOMEM;
  a.params = ws.at<DevParams>(o_params);
  a.part = ws.at<float2>(o_part);
  for (int l = 0; l < L; ++l) a.rec[l] = ws.at<float>(o_rec[l]);
  for (int l = 1; l <= L; ++l) a.sym[l] = ws.at<uint16_t>(o_sym[l]);
  a.lane_len = ws.at<uint16_t>(o_lane);
  a.hist = ws.at<unsigned long long>(o_hist);
  a.lens = ws.at<uint8_t>(o_lens);
  a.codes = ws.at<uint16_t>(o_codes);
  a.cb_scratch = ws.at<uint8_t>(o_cb);
  a.cnt = ws.at<uint32_t>(o_cnt);
  a.scan = ws.at<uint32_t>(o_scan);
  a.scan_part = ws.at<uint64_t>(o_spart);
  if (launch_compress(a, st) != hipSuccess) return STZ_ERR_DEVICE;
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  if (hipMemcpyAsync(stage->params, a.params, sizeof(DevParams), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  const DevParams& P = *stage->params;
  prof_flush();
  *out_size = P.total;
  if (P.flags & kFlagNonfinite) return STZ_ERR_NONFINITE;
  if (P.flags & (kFlagBadBound | kFlagTooLarge)) return STZ_ERR_ARG;
  if (P.flags & kFlagOverflow) return STZ_ERR_BUFFER;
  return STZ_OK;
}

stz_status stz_info(const void* comp, uint64_t size, stz_info_t* info, void* stream) {
  Header h;
  const stz_status s = read_header(comp, size, static_cast<hipStream_t>(stream), &h);
  if (s != STZ_OK) return s;
  if (info) {
    for (int d = 0; d < 3; ++d) info->dims[d] = uint64_t(h.g.n[d]);
    info->block = uint32_t(h.c.B);
    info->levels = uint32_t(h.c.L);
    info->radius = uint32_t(h.c.R);
    info->lmax = uint32_t(kLmax);
    info->eb_mode = uint32_t(h.eb_mode);
    info->reserved = 0;
    info->eb = h.eb;
    info->eb_abs = h.eb_abs;
    info->eb_ratio = h.c.ratio;
    info->total_bytes = h.total;
  }
  return STZ_OK;
}

stz_status stz_decompress_region(const void* comp, uint64_t size, const uint64_t lo[3],
                                 const uint64_t hi[3], uint32_t level, float* out,
                                 uint64_t out_cap_elems, uint64_t out_dims[3], void* stream) {
  if (!lo || !hi) return STZ_ERR_ARG;
  Box b;
  for (int d = 0; d < 3; ++d) {
    if (lo[d] > (uint64_t(1) << 32) || hi[d] > (uint64_t(1) << 32)) return STZ_ERR_ARG;
    b.lo[d] = int64_t(lo[d]);
    b.hi[d] = int64_t(hi[d]);
  }
  if (level > uint32_t(kMaxLevels)) return STZ_ERR_ARG;
  return decode_box(comp, size, &b, int(level), out, out_cap_elems, out_dims,
                    static_cast<hipStream_t>(stream));
}

stz_status stz_decompress_level(const void* comp, uint64_t size, uint32_t level, float* out,
                                uint64_t out_cap_elems, uint64_t out_dims[3], void* stream) {
  if (level > uint32_t(kMaxLevels)) return STZ_ERR_ARG;
  return decode_box(comp, size, nullptr, int(level), out, out_cap_elems, out_dims,
                    static_cast<hipStream_t>(stream));
}

stz_status stz_decompress(const void* comp, uint64_t size, float* out, uint64_t out_cap_elems,
                          void* stream) {
  uint64_t od[3];
  return decode_box(comp, size, nullptr, -1, out, out_cap_elems, od,
                    static_cast<hipStream_t>(stream));
}

const char* stz_status_string(stz_status st) {
  switch (st) {
    case STZ_OK: return "ok";
    case STZ_ERR_ARG: return "invalid argument";
    case STZ_ERR_NONFINITE: return "input holds NaN or Inf";
    case STZ_ERR_BUFFER: return "output buffer too small";
    case STZ_ERR_CORRUPT: return "corrupt stream";
    case STZ_ERR_DEVICE: return "HIP runtime error";
    case STZ_ERR_NOMEM: return "out of device memory";
  }
  return "unknown status";
}

}  // extern "C"
