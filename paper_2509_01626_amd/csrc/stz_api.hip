// Host side of the C ABI declared in include/stz.h: argument validation,
// stream-header parsing, workspace management and kernel launch sequences.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "stz.h"
#include "stz_internal.h"

namespace stz {

void prof_flush();

namespace {

struct Cfg {
  int B, logB, L, R;
  int coding;  // STZ_CODING_HUFFMAN or STZ_CODING_ZERO_CHUNKS
  double ratio;
};

stz_status resolve_cfg(const stz_config* c, Cfg* o) {
  stz_config d = {0, 0, 0, 0, 0.0};
  if (c) d = *c;
  if (d.coding > STZ_CODING_ZERO_CHUNKS) return STZ_ERR_ARG;
  o->coding = d.coding == STZ_CODING_DEFAULT ? int(STZ_CODING_ZERO_CHUNKS) : int(d.coding);
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
  g->Z = c.coding == STZ_CODING_ZERO_CHUNKS ? 2 * c.R : -1;
  g->pad = 0;
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

}  // namespace

BatchTuning& batch_tuning() {
  static BatchTuning t = [] {
    BatchTuning d;
    d.grid = 2048;
    for (int e = 0; e < kBatchEdges; ++e) {
      d.grid_pred[e] = 1u << 20;
      d.grid_dec[e] = 1u << 20;
      d.pred_h[e] = 0;  // 0 = the plain launch's slab height
      d.dec_h[e] = 0;
    }
    return d;
  }();
  return t;
}

namespace {

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

// Auxiliary streams: one per (device, caller stream), created on first use
// with default priority, for launches that run beside the caller's stream
// between a fork and a join event (see launch_pred).
struct AuxCache {
  std::mutex mu;
  std::unordered_map<uint64_t, AuxStream> m;
};

AuxCache& aux_cache() {
  static AuxCache* c = new AuxCache;  // never destroyed: may be used during exit
  return *c;
}

}  // namespace

const AuxStream* aux_stream(hipStream_t st) {
  AuxCache& c = aux_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  const uint64_t key = ws_key(st);
  auto it = c.m.find(key);
  if (it != c.m.end()) return &it->second;
  AuxStream a{};
  if (hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a.join, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(a.s);
    return nullptr;
  }
  return &c.m.emplace(key, a).first->second;
}

namespace {

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
  static constexpr uint64_t kHdrBytes = kHeaderBytes + kMaxAlphabet;
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
  int vb;  // bytes per stored value: 4 (value type 0, float32) or 8 (1, float64)
  int eb_mode;
  double eb, eb_abs;
  uint64_t total, anchor_off, n_anchor;
  uint64_t sec[kMaxLevels + 1], words[kMaxLevels + 1], outl[kMaxLevels + 1];
  uint64_t off_outl[kMaxLevels + 1], off_lane[kMaxLevels + 1], off_pay[kMaxLevels + 1],
      off_out[kMaxLevels + 1];
  LevelConst lc[kMaxLevels + 1];
  uint8_t lens[kMaxAlphabet];  // code lengths of the alphabet (nsym entries)
  int nsym = 0;
};

template <class T>
T rd(const uint8_t* p) {
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}

// Parse the first `want` = min(size, kHdrBytes) bytes of a stream of `size`
// bytes, already copied to host memory at p.
stz_status parse_header(const uint8_t* p, uint64_t want, uint64_t size, Header* h) {
  if (rd<uint32_t>(p) != kMagic || rd<uint32_t>(p + 4) != kVersion) return STZ_ERR_CORRUPT;
  uint64_t dims[3] = {rd<uint64_t>(p + 8), rd<uint64_t>(p + 16), rd<uint64_t>(p + 24)};
  stz_config cf;
  cf.block = rd<uint32_t>(p + 32);
  cf.levels = rd<uint32_t>(p + 36);
  cf.radius = rd<uint32_t>(p + 40);
  cf.coding = rd<uint32_t>(p + 112);
  cf.eb_ratio = rd<double>(p + 72);
  if (!cf.block || !cf.levels || !cf.radius) return STZ_ERR_CORRUPT;
  if (cf.coding != STZ_CODING_HUFFMAN && cf.coding != STZ_CODING_ZERO_CHUNKS)
    return STZ_ERR_CORRUPT;
  if (rd<uint32_t>(p + 44) != uint32_t(kLmax)) return STZ_ERR_CORRUPT;
  if (resolve_cfg(&cf, &h->c) != STZ_OK || !make_geo(dims, h->c, &h->g)) return STZ_ERR_CORRUPT;
  h->eb_mode = int(rd<uint32_t>(p + 48));
  const uint32_t vt = rd<uint32_t>(p + 52);
  if (vt > 1) return STZ_ERR_CORRUPT;
  h->vb = vt ? 8 : 4;
  h->eb = rd<double>(p + 56);
  h->eb_abs = rd<double>(p + 64);
  if (!(h->eb_abs > 0.0) || !std::isfinite(h->eb_abs)) return STZ_ERR_CORRUPT;
  h->total = rd<uint64_t>(p + 80);
  if (h->total > size) return STZ_ERR_CORRUPT;
  const uint64_t nsym = uint64_t(alphabet(h->g));
  if (rd<uint64_t>(p + 88) != kHeaderBytes) return STZ_ERR_CORRUPT;
  h->anchor_off = rd<uint64_t>(p + 96);
  h->n_anchor = rd<uint64_t>(p + 104);
  if (h->anchor_off != kHeaderBytes + align16(nsym)) return STZ_ERR_CORRUPT;
  if (h->n_anchor != grid_count(h->g, h->g.L)) return STZ_ERR_CORRUPT;
  if (kHeaderBytes + nsym > want || nsym > uint64_t(kMaxAlphabet)) return STZ_ERR_CORRUPT;
  std::memcpy(h->lens, p + kHeaderBytes, nsym);
  h->nsym = int(nsym);
  level_consts(h->g, h->lc);
  const uint64_t vb = uint64_t(h->vb);
  uint64_t pos = h->anchor_off + align16(vb * h->n_anchor);
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
    pos = h->off_out[l] + align16(vb * O);
    if (pos > h->total) return STZ_ERR_CORRUPT;
  }
  if (pos != h->total) return STZ_ERR_CORRUPT;
  return STZ_OK;
}

// Copy the header of a device stream to the calling thread's pinned staging
// (one synchronization) and parse it.
stz_status read_header(const void* comp, uint64_t size, hipStream_t st, Header* h) {
  if (!comp || size < kHeaderBytes) return STZ_ERR_CORRUPT;
  const uint64_t want = std::min<uint64_t>(size, Staging::kHdrBytes);
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  if (hipMemcpyAsync(stage->hdr, comp, want, hipMemcpyDeviceToHost, st) != hipSuccess)
    return STZ_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return STZ_ERR_DEVICE;
  return parse_header(stage->hdr, want, size, h);
}

// Decoder table: entry for every 12-bit window = symbol | length << 12, or 0
// when no code is a prefix of the window. Fails when the lengths do not form a
// prefix code.
bool build_lut(const uint8_t* lens, int nsym, uint16_t* lut) {
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
  std::memset(lut, 0, sizeof(uint16_t) << kLutBits);
  for (int i = 0; i < nsym; ++i) {
    const int l = lens[i];
    if (!l) continue;
    const uint32_t c = next[l]++;
    const uint32_t lo = c << (kLutBits - l), n = 1u << (kLutBits - l);
    for (uint32_t k = 0; k < n; ++k) lut[lo + k] = uint16_t(i | (l << 12));
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

// Validated arguments and scratch layout of one box decode (null box = the
// whole domain, negative level = finest) against a parsed header; the same
// plan serves a plain call and a request of a batch. A plan whose output is
// empty (an axis without grid points) has cnt == 0 and launches nothing.
struct DecodePlan {
  DecodeArgs a;
  uint64_t od[3] = {0, 0, 0}, cnt = 0;
  uint64_t o_rec[kMaxLevels + 1] = {};

  stz_status init(const Header& h, const void* comp, uint64_t size, const Box* boxp, int level,
                  void* out, uint64_t out_cap) {
    const Geo& g = h.g;
    std::memset(&a, 0, sizeof(a));
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
    for (int d = 0; d < 3; ++d) {
      const int64_t f = (box.lo[d] + so - 1) >> logs_out << logs_out;
      od[d] = f < box.hi[d] ? uint64_t(((box.hi[d] - 1 - f) >> logs_out) + 1) : 0;
    }
    cnt = od[0] * od[1] * od[2];
    if (cnt == 0) return STZ_OK;
    if (!out || cnt > out_cap) return STZ_ERR_BUFFER;
    a.comp = static_cast<const uint8_t*>(comp);
    a.size = size;
    a.geo = g;
    a.vb = h.vb;
    a.level_out = level;
    a.box[level] = box;
    for (int k = level; k >= 1; --k)
      a.box[k - 1] = dilate(a.box[k], 3 * (int64_t(1) << (g.L - k)), g);
    a.rec[level] = out;
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
      a.E2d[l] = 2.0 * e;
    }
    return STZ_OK;
  }

  void take(Workspace& ws) {
    for (int k = 0; k < a.level_out; ++k)
      o_rec[k] = ws.take<uint8_t>(uint64_t(a.vb) * box_points(a.box[k], a.geo.L - k));
  }

  void bind(const Workspace& ws, const uint16_t* lut, uint32_t* flags) {
    for (int k = 0; k < a.level_out; ++k) a.rec[k] = ws.at<uint8_t>(o_rec[k]);
    a.lut = lut;
    a.flags = flags;
  }
};

// Decoder tables of plain decodes, kept in device memory per device and code
// (the code lengths, compared in full): repeated decodes of one stream, or of
// streams with the same code, build and upload no table. An entry is written
// once, by the call that creates it, and used by other calls only after that
// call has synchronized (ready). At most kLutCacheMax entries per process;
// beyond them calls upload their table into their own scratch as before.
// stz_trim frees a device's entries.
struct LutEntry {
  int device;
  int nsym;
  uint64_t hash;
  std::vector<uint8_t> lens;
  uint16_t* dev;
  bool ready;
};
struct LutCache {
  std::mutex mu;
  std::deque<LutEntry> e;  // appending keeps references to the other entries
};
constexpr size_t kLutCacheMax = 64;

LutCache& lut_cache() {
  static LutCache* c = new LutCache;  // never destroyed: may be used during exit
  return *c;
}

uint64_t lens_hash(const uint8_t* lens, int nsym) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  for (int i = 0; i < nsym; ++i) h = (h ^ lens[i]) * 1099511628211ull;
  return h ^ uint64_t(nsym);
}

// The ready table for this code on the current device, or null. With mine
// (a table this call has built and checked), a miss reserves a new entry for
// the call to fill: *mine, null when the cache is full or the entry exists
// but is not ready yet.
const uint16_t* lut_lookup(const uint8_t* lens, int nsym, LutEntry** mine) {
  if (mine) *mine = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const uint64_t hh = lens_hash(lens, nsym);
  LutCache& c = lut_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto& e : c.e)
    if (e.device == dev && e.nsym == nsym && e.hash == hh &&
        std::memcmp(e.lens.data(), lens, size_t(nsym)) == 0)
      return e.ready ? e.dev : nullptr;
  if (!mine || c.e.size() >= kLutCacheMax) return nullptr;
  uint16_t* d = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d), (size_t(1) << kLutBits) * 2 + 16) != hipSuccess)
    return nullptr;
  c.e.push_back({dev, nsym, hh, std::vector<uint8_t>(lens, lens + nsym), d, false});
  *mine = &c.e.back();
  return nullptr;
}

void lut_mark_ready(LutEntry* e) {
  LutCache& c = lut_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  e->ready = true;
}

// Parsed headers of the streams plain decodes were last given, per device,
// stream address and size, with the header bytes they were parsed from (the
// bytes parse_header reads: the fixed part and the code lengths). A call whose
// stream is kept launches at once: the kept bytes travel as an argument of
// the decode's first kernel (the anchors), which compares them with the
// stream's header before any level is decoded. When they differ the call
// reads and parses the header again and decodes again, so results and
// statuses are those of a call that reads the header first. Kept headers only ever steer launches
// whose reads the header's own checks bound to the stream's size. At most
// kHdrCacheMax entries (oldest out first); stz_trim drops a device's entries.
struct HdrEntry {
  int device;
  const void* comp;
  uint64_t size;
  std::vector<uint8_t> bytes;
  Header h;
};
struct HdrCache {
  std::mutex mu;
  std::deque<HdrEntry> e;
};
constexpr size_t kHdrCacheMax = 16;

HdrCache& hdr_cache() {
  static HdrCache* c = new HdrCache;  // never destroyed: may be used during exit
  return *c;
}

// On a hit: the kept header in *h and the bytes it was parsed from in *ref.
bool hdr_lookup(const void* comp, uint64_t size, Header* h, HdrRef* ref) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  HdrCache& c = hdr_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (const auto& e : c.e)
    if (e.device == dev && e.comp == comp && e.size == size) {
      *h = e.h;
      std::memcpy(ref->b, e.bytes.data(), e.bytes.size());
      ref->n = uint32_t(e.bytes.size());
      return true;
    }
  return false;
}

// Keep (or replace) the header just parsed from `bytes`.
void hdr_keep(const void* comp, uint64_t size, const Header& h, const uint8_t* bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  const uint64_t nb = kHeaderBytes + uint64_t(h.nsym);
  HdrCache& c = hdr_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto it = c.e.begin(); it != c.e.end(); ++it)
    if (it->device == dev && it->comp == comp && it->size == size) {
      c.e.erase(it);
      break;
    }
  if (c.e.size() >= kHdrCacheMax) c.e.pop_front();
  c.e.push_back({dev, comp, size, std::vector<uint8_t>(bytes, bytes + nb), h});
}

// vb = the caller's value type; a stream of the other type is rejected.
// use_kept = false: read the header even when it is kept.
stz_status decode_box(const void* comp, uint64_t size, const Box* boxp, int level, void* out,
                      uint64_t out_cap, uint64_t out_dims[3], int vb, hipStream_t st,
                      bool use_kept = true) {
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  Header h;
  HdrRef ref;  // kept header bytes to check the stream against (n = 0: read here)
  ref.n = 0;
  stz_status s = STZ_OK;
  if (!use_kept || !comp || !hdr_lookup(comp, size, &h, &ref)) {
    ref.n = 0;
    s = read_header(comp, size, st, &h);
    if (s != STZ_OK) return s;
    hdr_keep(comp, size, h, stage->hdr);
  }
  const uint32_t nref = ref.n;
  // A call steered by a kept header takes any outcome other than a decode
  // from a fresh read.
  auto reread = [&]() {
    return decode_box(comp, size, boxp, level, out, out_cap, out_dims, vb, st, false);
  };
  if (h.vb != vb) return nref ? reread() : STZ_ERR_ARG;
  DecodePlan pl;
  s = pl.init(h, comp, size, boxp, level, out, out_cap);
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = pl.od[d];
  if (s != STZ_OK || pl.cnt == 0) return nref ? reread() : s;
  constexpr uint64_t nlut = uint64_t(1) << kLutBits;
  LutEntry* mine = nullptr;
  const uint16_t* cached = lut_lookup(h.lens, h.nsym, nullptr);
  if (!cached) {
    if (!build_lut(h.lens, h.nsym, stage->lut))  // not a prefix code
      return nref ? reread() : STZ_ERR_CORRUPT;
    cached = lut_lookup(h.lens, h.nsym, &mine);  // ready meanwhile, or reserve an entry
  }
  Workspace ws(st);
  pl.take(ws);
  const uint64_t o_lut = ws.take<uint8_t>(cached || mine ? 1 : nlut * 2 + 16);
  const uint64_t o_flags = ws.take<uint32_t>(2);
  if (!ws.commit()) return STZ_ERR_NOMEM;
  uint16_t* dlut = cached ? const_cast<uint16_t*>(cached)
                          : (mine ? mine->dev : ws.at<uint16_t>(o_lut));
  // [0] decode flags, zeroed by the anchor kernel; [1] header check result
  uint32_t* dflags = ws.at<uint32_t>(o_flags);
  pl.bind(ws, dlut, dflags);
  if (!cached) {
    std::memset(stage->lut + nlut, 0, 16);
    if (hipMemcpyAsync(dlut, stage->lut, nlut * 2 + 16, hipMemcpyHostToDevice, st) != hipSuccess)
      return STZ_ERR_DEVICE;
  }
  if (launch_decode(pl.a, st, nref ? &ref : nullptr) != hipSuccess) return STZ_ERR_DEVICE;
  if (hipMemcpyAsync(stage->flags, dflags, nref ? 8 : 4, hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  if (mine) lut_mark_ready(mine);  // the table's copy has completed
  prof_flush();
  if (nref && stage->flags[1]) return reread();  // the stream's header is not the kept one
  return stage->flags[0] ? STZ_ERR_CORRUPT : STZ_OK;
}

// ---- decoding without allocation --------------------------------------------
// Device address of the file-scope scratch array on the current device
// (set up once per device with that device current), or null.
void* noalloc_scratch();

// A box decode like decode_box (float32 streams) whose scratch (level grids,
// decoder table, corruption flag) lives in the fixed scratch array: no device
// or pinned allocation, the header and table pass through stack buffers.
stz_status decode_box_noalloc(const void* comp, uint64_t size, const Box* boxp, int level,
                              float* out, uint64_t out_cap, uint64_t out_dims[3], hipStream_t st) {
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = 0;
  uint8_t* base = static_cast<uint8_t*>(noalloc_scratch());
  if (!base) return STZ_ERR_DEVICE;
  if (!comp || size < kHeaderBytes) return STZ_ERR_CORRUPT;
  uint8_t hb[kHeaderBytes + kMaxAlphabet];
  const uint64_t want = std::min<uint64_t>(size, sizeof(hb));
  if (hipMemcpyAsync(hb, comp, want, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  Header h;
  stz_status s = parse_header(hb, want, size, &h);
  if (s != STZ_OK) return s;
  if (h.vb != 4) return STZ_ERR_ARG;
  DecodePlan pl;
  s = pl.init(h, comp, size, boxp, level, out, out_cap);
  if (out_dims)
    for (int d = 0; d < 3; ++d) out_dims[d] = pl.od[d];
  if (s != STZ_OK || pl.cnt == 0) return s;
  // layout: the cone's level grids, then the table with the flag word behind it
  constexpr uint64_t nlut = uint64_t(1) << kLutBits;
  uint64_t used = 0;
  for (int k = 0; k < pl.a.level_out; ++k) {
    pl.a.rec[k] = base + used;
    used += (uint64_t(h.vb) * std::max<uint64_t>(box_points(pl.a.box[k], h.g.L - k), 1) + 255) &
            ~uint64_t(255);
  }
  const uint64_t o_lut = used;
  used += nlut * 2 + 16;
  if (used > uint64_t(STZ_NOALLOC_SCRATCH_BYTES)) return STZ_ERR_NOMEM;
  uint16_t lut[nlut + 8];
  if (!build_lut(h.lens, h.nsym, lut)) return STZ_ERR_CORRUPT;
  std::memset(lut + nlut, 0, 16);  // clears the flag word
  pl.a.lut = reinterpret_cast<const uint16_t*>(base + o_lut);
  pl.a.flags = reinterpret_cast<uint32_t*>(base + o_lut + nlut * 2);
  if (hipMemcpyAsync(base + o_lut, lut, sizeof(lut), hipMemcpyHostToDevice, st) != hipSuccess)
    return STZ_ERR_DEVICE;
  if (launch_decode(pl.a, st) != hipSuccess) return STZ_ERR_DEVICE;
  uint32_t flag = 0;
  if (hipMemcpyAsync(&flag, pl.a.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  return flag ? STZ_ERR_CORRUPT : STZ_OK;
}

// ---- compression plan of one field ----------------------------------------
stz_status params_status(const DevParams& P) {
  if (P.flags & kFlagNonfinite) return STZ_ERR_NONFINITE;
  if (P.flags & (kFlagBadBound | kFlagTooLarge)) return STZ_ERR_ARG;
  if (P.flags & kFlagOverflow) return STZ_ERR_BUFFER;
  return STZ_OK;
}

// Validated arguments, kernel argument block and scratch layout of one
// compression; the same plan serves a plain call and a job of a batch.
struct CompressPlan {
  CompressArgs a;
  uint64_t o_part = 0, o_rec[kMaxLevels] = {}, o_sym[kMaxLevels + 1] = {}, o_lane = 0,
           o_hist = 0, o_hpart = 0, o_lens = 0, o_codes = 0, o_cb = 0, o_cnt = 0, o_scan = 0,
           o_spart = 0;

  stz_status init(const void* x, int vb, const uint64_t dims[3], int eb_mode, double eb,
                  const stz_config* cfg, void* out, uint64_t out_cap) {
    Cfg c;
    Geo g;
    std::memset(&a, 0, sizeof(a));
    if (!x || !dims) return STZ_ERR_ARG;
    if (resolve_cfg(cfg, &c) != STZ_OK || !make_geo(dims, c, &g)) return STZ_ERR_ARG;
    if (eb_mode != STZ_EB_ABS && eb_mode != STZ_EB_REL) return STZ_ERR_ARG;
    if (!(eb > 0.0) || !std::isfinite(eb)) return STZ_ERR_ARG;
    const uint64_t N = uint64_t(g.n[0]) * g.n[1] * g.n[2];
    a.x = x;
    a.vb = vb;
    a.geo = g;
    a.eb_mode = eb_mode;
    a.eb = eb;
    a.ratio = c.ratio;
    a.out = static_cast<uint8_t*>(out);
    a.out_cap = out ? out_cap : 0;
    level_consts(g, a.lc);
    a.n_anchor = grid_count(g, g.L);
    if (a.lc[1].nu > 0xFFFFFFF0ull) return STZ_ERR_ARG;
    // 2048 min/max partials (eight work-groups per CU): the pass reads at
    // 5.9 TB/s, against 5.3 TB/s with 1024
    a.nparts = uint32_t(std::min<uint64_t>(2048, (N + 4095) / 4096));
    return STZ_OK;
  }

  void take(Workspace& ws) {
    const Geo& g = a.geo;
    const int L = g.L, nsym = alphabet(g);
    const uint64_t nu = a.lc[1].nu;
    o_part = ws.take<uint8_t>(2 * uint64_t(a.vb) * a.nparts);
    for (int l = 0; l < L; ++l) o_rec[l] = ws.take<uint8_t>(uint64_t(a.vb) * grid_count(g, L - l));
    uint64_t lanes = 0;
    for (int l = 1; l <= L; ++l) {
      o_sym[l] = ws.take<uint16_t>(a.lc[l].nsym);
      a.lane_base[l] = lanes;
      lanes += a.lc[l].nl;
    }
    o_lane = ws.take<uint16_t>(lanes);
    o_hist = ws.take<unsigned long long>(nsym);
    a.nslots = uint32_t(std::min<uint64_t>(kHistSlots, uint64_t(g.nb[0] * g.nb[1] * g.nb[2])));
    o_hpart = ws.take<uint32_t>(uint64_t(nsym) * a.nslots);
    o_lens = ws.take<uint8_t>(nsym);
    o_codes = ws.take<uint16_t>(nsym);
    o_cb = ws.take<uint8_t>(codebook_scratch_bytes(nsym));
    o_cnt = ws.take<uint32_t>(2 * L * nu);
    o_scan = ws.take<uint32_t>(2 * L * (nu + 1));
    o_spart = ws.take<uint64_t>(2 * L * scan_blocks());
  }

  uint64_t scan_blocks() const { return (a.lc[1].nu + 2047) / 2048; }

  void bind(const Workspace& ws, DevParams* params) {
    const int L = a.geo.L;
    a.params = params;
    a.part = ws.at<uint8_t>(o_part);
    for (int l = 0; l < L; ++l) a.rec[l] = ws.at<uint8_t>(o_rec[l]);
    for (int l = 1; l <= L; ++l) a.sym[l] = ws.at<uint16_t>(o_sym[l]);
    a.lane_len = ws.at<uint16_t>(o_lane);
    a.hist = ws.at<unsigned long long>(o_hist);
    a.hpart = ws.at<uint32_t>(o_hpart);
    a.lens = ws.at<uint8_t>(o_lens);
    a.codes = ws.at<uint16_t>(o_codes);
    a.cb_scratch = ws.at<uint8_t>(o_cb);
    a.cnt = ws.at<uint32_t>(o_cnt);
    a.scan = ws.at<uint32_t>(o_scan);
    a.scan_part = ws.at<uint64_t>(o_spart);
  }
};

// Per-thread pinned host buffer for job tables and work maps (host to
// device) and the per-job status blocks (device to host); grows on demand.
// Every batch call ends with a stream synchronization.
struct HostBuf {
  uint8_t* p = nullptr;
  uint64_t cap = 0;
  hipEvent_t done = nullptr;  // recorded after the last copy out of the buffer
  bool pending = false;
  // Wait until the copies of an asynchronous call that read the buffer ran.
  bool settle() {
    if (pending && done && hipEventSynchronize(done) != hipSuccess) return false;
    pending = false;
    return true;
  }
  bool mark(hipStream_t st) {
    if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
      done = nullptr;
      return false;
    }
    pending = hipEventRecord(done, st) == hipSuccess;
    return pending;
  }
  bool reserve(uint64_t n) {
    if (!settle()) return false;
    if (n <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const uint64_t want = std::max<uint64_t>(n + n / 2, 1 << 16);
    if (hipHostMalloc(reinterpret_cast<void**>(&p), want) != hipSuccess) return false;
    cap = want;
    return true;
  }
  ~HostBuf() {
    settle();
    if (p) (void)hipHostFree(p);
    if (done) (void)hipEventDestroy(done);
  }
};

// One buffer per (thread, stream): a call waits only for the copies of the
// previous call on the same stream.
HostBuf& host_buf(hipStream_t st) {
  thread_local std::unordered_map<uint64_t, HostBuf> m;
  return m[ws_key(st)];
}

// Work maps of a batch, built on the host into one array of u32: every map is
// first[n+1] followed by job[n]; bind() turns offsets into device pointers.
struct BatchMaps {
  std::vector<uint32_t> buf;
  std::vector<std::pair<ItemMap*, uint64_t>> fix;  // map, offset of its first[]

  // counts[k] items for table entry k; entries with no items are left out.
  // With pad8 every entry's range is rounded up to a multiple of 8 items, so
  // that in a launch whose grid is a multiple of 8 the item's position within
  // its job mod 8 is the XCD its work-group runs on (kernels skip the padding).
  uint32_t add(ItemMap* m, const std::vector<uint32_t>& counts, bool pad8 = false) {
    std::vector<uint32_t> first, job;
    uint32_t run = 0;
    for (uint32_t k = 0; k < counts.size(); ++k) {
      if (!counts[k]) continue;
      first.push_back(run);
      job.push_back(k);
      run += pad8 ? (counts[k] + 7) & ~7u : counts[k];
    }
    first.push_back(run);
    m->n = uint32_t(job.size());
    const uint64_t off = buf.size();
    buf.insert(buf.end(), first.begin(), first.end());
    buf.insert(buf.end(), job.begin(), job.end());
    if (job.empty()) buf.push_back(0);
    fix.push_back({m, off});
    return run;
  }

  void bind(const uint32_t* dev) {
    for (auto& f : fix) {
      f.first->first = dev + f.second;
      f.first->job = dev + f.second + f.first->n + 1;
    }
  }
};

uint32_t cap_items(uint64_t n, uint64_t per, uint64_t cap) {
  return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(cap, (n + per - 1) / per)));
}

int ilog2(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

// Work maps of a batched compression over the live jobs (table order). Jobs
// with at least kDirectBlocks blocks of 32^3 points or more at a level are
// left out of that level's predictor map and listed in *pdirect: they take
// the plain launch (interior and shell kernels), which fills the device alone.
void build_compress_maps(const std::vector<CompressPlan>& pl, const std::vector<uint32_t>& live,
                         BatchMaps* maps, CompressBatch* b, std::vector<PredDirect>* pdirect,
                         std::vector<uint32_t>* whole) {
  std::memset(b, 0, sizeof(*b));
  const uint32_t n = uint32_t(live.size());
  b->njobs = n;
  const BatchTuning& tu = batch_tuning();
  b->grid = tu.grid;
  for (int e = 0; e < kBatchEdges; ++e) {
    b->grid_pred[e] = tu.grid_pred[e];
    b->pred_h[e] = tu.pred_h[e];
  }
  // jobs that fill the GPU by themselves run their plain launch sequence
  std::vector<char> is_whole(n, 0);
  for (uint32_t k = 0; k < n; ++k) {
    const Geo& g = pl[live[k]].a.geo;
    if (uint64_t(g.n[0]) * uint64_t(g.n[1]) * uint64_t(g.n[2]) >= kWholeJobPoints) {
      is_whole[k] = 1;
      whole->push_back(k);
    }
  }
  std::vector<uint32_t> c(n);
  auto per_job = [&](auto f) {
    for (uint32_t k = 0; k < n; ++k) c[k] = is_whole[k] ? 0u : f(pl[live[k]].a);
    return c;
  };
  b->n_jobs1 = maps->add(&b->jobs1, per_job([](const CompressArgs&) { return 1u; }));
  b->n_minmax = maps->add(&b->minmax, per_job([](const CompressArgs& a) {
    return a.eb_mode == STZ_EB_REL ? a.nparts : 0u;
  }));
  b->n_anchor = maps->add(&b->anchor, per_job([](const CompressArgs& a) {
    return cap_items(a.n_anchor, 256, 4096);
  }));
  b->n_hzero = maps->add(&b->hzero, per_job([](const CompressArgs& a) {
    return cap_items(uint64_t(alphabet(a.geo)) * a.nslots, 256 * 16, 1024);
  }));
  b->n_hred = maps->add(&b->hred, per_job([](const CompressArgs& a) {
    return uint32_t((alphabet(a.geo) + 255) / 256);
  }));
  int maxL = 0;
  for (uint32_t k = 0; k < n; ++k) maxL = std::max(maxL, pl[live[k]].a.geo.L);
  b->max_levels = maxL;
  for (int l = 1; l <= maxL; ++l) {
    for (int e = 1; e < kBatchEdges; ++e) {
      for (uint32_t k = 0; k < n; ++k) {
        const Geo& g = pl[live[k]].a.geo;
        c[k] = 0;
        if (is_whole[k] || g.L < l || ilog2(g.B >> (g.L - l)) != e) continue;
        const uint64_t nbk = uint64_t(g.nb[0] * g.nb[1] * g.nb[2]);
        if ((g.B >> (g.L - l)) >= 32 && nbk >= kDirectBlocks) {
          pdirect->push_back({k, l});
          continue;
        }
        c[k] = uint32_t(nbk);
      }
      b->n_pred[l][e] = maps->add(&b->pred[l][e], c, true);
    }
    b->n_level[l] = maps->add(&b->level[l], per_job([&](const CompressArgs& a) {
      const Geo& g = a.geo;
      return g.L < l ? 0u : uint32_t(g.nb[0] * g.nb[1] * g.nb[2]);
    }));
    for (int units = 0; units < 2; ++units) {
      ItemMap* m = units ? &b->pack_u[l] : &b->pack_l[l];
      uint32_t* n = units ? &b->n_pack_u[l] : &b->n_pack_l[l];
      *n = maps->add(m, per_job([&](const CompressArgs& a) {
        const Geo& g = a.geo;
        if (g.L < l || ((g.B >> (g.L - l)) >= 32) != (units == 1)) return 0u;
        return uint32_t(g.nb[0] * g.nb[1] * g.nb[2]);
      }));
    }
  }
  b->n_scan_ac = maps->add(&b->scan_ac, per_job([](const CompressArgs& a) {
    return uint32_t((a.lc[1].nu + 2047) / 2048) * uint32_t(2 * a.geo.L);
  }));
  b->n_scan_b = maps->add(&b->scan_b, per_job([](const CompressArgs& a) {
    return uint32_t(2 * a.geo.L);
  }));
  b->n_zero = maps->add(&b->zero, per_job([](const CompressArgs& a) {
    return cap_items(a.out_cap, 16 * 256 * 8, 2048);
  }));
  b->n_head = maps->add(&b->head, per_job([](const CompressArgs& a) {
    return cap_items(a.n_anchor + uint64_t(alphabet(a.geo)), 256, 4096);
  }));
}

// Work maps of a batched decode over the live requests (table order).
void build_decode_maps(const std::vector<DecodePlan>& pl, const std::vector<uint32_t>& live,
                       BatchMaps* maps, DecodeBatch* b, std::vector<DirectItem>* direct) {
  std::memset(b, 0, sizeof(*b));
  const uint32_t n = uint32_t(live.size());
  b->nreq = n;
  const BatchTuning& tu = batch_tuning();
  b->grid = tu.grid;
  for (int e = 0; e < kBatchEdges; ++e) {
    b->grid_dec[e] = tu.grid_dec[e];
    b->dec_h[e] = tu.dec_h[e];
  }
  std::vector<uint32_t> c(n);
  auto per_req = [&](auto f) {
    for (uint32_t k = 0; k < n; ++k) c[k] = f(pl[live[k]].a);
    return c;
  };
  b->n_anchor = maps->add(&b->anchor, per_req([](const DecodeArgs& a) {
    return cap_items(box_points(a.box[0], a.geo.L), 256, 4096);
  }));
  int maxk = 0;
  for (uint32_t k = 0; k < n; ++k) maxk = std::max(maxk, pl[live[k]].a.level_out);
  b->max_level = maxk;
  for (int k = 1; k <= maxk; ++k) {
    b->n_check[k] = 0;
    for (uint32_t r = 0; r < n; ++r) b->n_check[k] += pl[live[r]].a.level_out >= k ? 1u : 0u;
    for (uint32_t r = 0; r < n; ++r) {
      const DecodeArgs& a = pl[live[r]].a;
      if (a.level_out < k) continue;
      uint64_t nb = 1;
      for (int q = 0; q < 3; ++q)
        nb *= uint64_t(((a.box[k].hi[q] - 1) >> a.geo.logB) - (a.box[k].lo[q] >> a.geo.logB) + 1);
      if (nb >= kDirectBlocks) direct->push_back({r, k});
    }
    for (int e = 1; e < kBatchEdges; ++e) {
      b->n_dec[k][e] = maps->add(&b->dec[k][e], per_req([&](const DecodeArgs& a) {
        const Geo& g = a.geo;
        if (a.level_out < k || ilog2(g.B >> (g.L - k)) != e) return 0u;
        uint64_t nb = 1;
        for (int q = 0; q < 3; ++q)
          nb *= uint64_t(((a.box[k].hi[q] - 1) >> g.logB) - (a.box[k].lo[q] >> g.logB) + 1);
        return nb >= kDirectBlocks ? 0u : uint32_t(nb);
      }), true);
    }
  }
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
  {
    HdrCache& hc = hdr_cache();
    std::lock_guard<std::mutex> lk4(hc.mu);
    for (auto it = hc.e.begin(); it != hc.e.end();) {
      if (it->device == cur)
        it = hc.e.erase(it);
      else
        ++it;
    }
  }
  {
    LutCache& lc = lut_cache();
    std::lock_guard<std::mutex> lk3(lc.mu);
    for (auto it = lc.e.begin(); it != lc.e.end();) {
      if (it->device == cur) {
        (void)hipFree(it->dev);
        it = lc.e.erase(it);
      } else {
        ++it;
      }
    }
  }
  {
    AuxCache& ac = aux_cache();
    std::lock_guard<std::mutex> lk2(ac.mu);
    for (auto it = ac.m.begin(); it != ac.m.end();) {
      if (int(it->first & 255) == (cur & 255)) {
        (void)hipEventDestroy(it->second.fork);
        (void)hipEventDestroy(it->second.join);
        (void)hipStreamDestroy(it->second.s);
        it = ac.m.erase(it);
      } else {
        ++it;
      }
    }
  }
  return hipDeviceSynchronize() == hipSuccess ? STZ_OK : STZ_ERR_DEVICE;
}

}  // extern "C"

namespace stz {
namespace {

uint64_t compress_bound(const uint64_t dims[3], const stz_config* cfg, uint64_t vb) {
  Cfg c;
  Geo g;
  if (!dims || resolve_cfg(cfg, &c) != STZ_OK || !make_geo(dims, c, &g)) return 0;
  LevelConst lc[kMaxLevels + 1];
  level_consts(g, lc);
  uint64_t total =
      kHeaderBytes + align16(uint64_t(alphabet(g))) + align16(vb * grid_count(g, g.L));
  for (int l = 1; l <= g.L; ++l) {
    const uint64_t nu = lc[l].nu;
    // every unit: at most kLmax bits per symbol plus one padding word
    const uint64_t words = (lc[l].nsym * kLmax + 31) / 32 + nu;
    total += 2 * align16(4 * (nu + 1)) + align16(2 * lc[l].nl) + align16(4 * words) +
             align16(vb * lc[l].nsym);
  }
  return total;
}

stz_status compress_one(const void* x, int vb, const uint64_t dims[3], int eb_mode, double eb,
                        const stz_config* cfg, void* out, uint64_t out_cap, uint64_t* out_size,
                        void* stream) {
  if (!out_size) return STZ_ERR_ARG;
  CompressPlan pl;
  const stz_status s0 = pl.init(x, vb, dims, eb_mode, eb, cfg, out, out_cap);
  if (s0 != STZ_OK) return s0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace ws(st);
  const uint64_t o_params = ws.take<DevParams>(1);
  pl.take(ws);
  if (!ws.commit()) return STZ_ERR_NOMEM;
  pl.bind(ws, ws.at<DevParams>(o_params));
  if (launch_compress(pl.a, st) != hipSuccess) return STZ_ERR_DEVICE;
  Staging* stage = staging();
  if (!stage) return STZ_ERR_NOMEM;
  if (hipMemcpyAsync(stage->params, pl.a.params, sizeof(DevParams), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  prof_flush();
  *out_size = stage->params->total;
  return params_status(*stage->params);
}

}  // namespace
}  // namespace stz

extern "C" {

uint64_t stz_compress_bound(const uint64_t dims[3], const stz_config* cfg) {
  return compress_bound(dims, cfg, 4);
}

uint64_t stz_compress_bound_f64(const uint64_t dims[3], const stz_config* cfg) {
  return compress_bound(dims, cfg, 8);
}

stz_status stz_compress(const float* x, const uint64_t dims[3], int eb_mode, double eb,
                        const stz_config* cfg, void* out, uint64_t out_cap, uint64_t* out_size,
                        void* stream) {
  return compress_one(x, 4, dims, eb_mode, eb, cfg, out, out_cap, out_size, stream);
}

stz_status stz_compress_f64(const double* x, const uint64_t dims[3], int eb_mode, double eb,
                            const stz_config* cfg, void* out, uint64_t out_cap,
                            uint64_t* out_size, void* stream) {
  return compress_one(x, 8, dims, eb_mode, eb, cfg, out, out_cap, out_size, stream);
}

stz_status stz_compress_batch(stz_job* jobs, uint64_t njobs, void* stream) {
  if (!jobs && njobs) return STZ_ERR_ARG;
  if (njobs == 0) return STZ_OK;
  if (njobs > STZ_MAX_BATCH) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<CompressPlan> pl(njobs);
  std::vector<uint32_t> live;  // jobs that passed validation
  for (uint64_t i = 0; i < njobs; ++i) {
    jobs[i].out_size = 0;
    jobs[i].status = jobs[i].reserved ? STZ_ERR_ARG
                                      : pl[i].init(jobs[i].x, 4, jobs[i].dims, jobs[i].eb_mode,
                                                   jobs[i].eb, &jobs[i].cfg, jobs[i].out,
                                                   jobs[i].out_cap);
    if (jobs[i].status == STZ_OK) live.push_back(uint32_t(i));
  }
  const uint32_t nl = uint32_t(live.size());
  if (nl) {
    Workspace ws(st);
    const uint64_t o_params = ws.take<DevParams>(nl);
    for (uint32_t k = 0; k < nl; ++k) pl[live[k]].take(ws);
    BatchMaps maps;
    CompressBatch b;
    std::vector<PredDirect> pdirect;
    std::vector<uint32_t> whole;
    build_compress_maps(pl, live, &maps, &b, &pdirect, &whole);
    // one staging blob, laid out as on the device and sent with one copy:
    // job table | work maps | per-level argument blocks (256-aligned)
    const uint64_t jb = (uint64_t(nl) * sizeof(CompressArgs) + 15) & ~uint64_t(15);
    const uint64_t mb = maps.buf.size() * sizeof(uint32_t);
    const uint64_t ao = (jb + mb + 255) & ~uint64_t(255);
    const uint64_t ab = compress_batch_args_bytes(nl, b.max_levels);
    const uint64_t o_blob = ws.take<uint8_t>(ao + ab);
    if (!ws.commit()) return STZ_ERR_NOMEM;
    DevParams* dpar = ws.at<DevParams>(o_params);
    for (uint32_t k = 0; k < nl; ++k) pl[live[k]].bind(ws, dpar + k);
    HostBuf& hb = host_buf(st);
    const uint64_t pb = uint64_t(nl) * sizeof(DevParams);
    if (!hb.reserve(std::max(ao + ab, pb))) return STZ_ERR_NOMEM;
    for (uint32_t k = 0; k < nl; ++k)
      std::memcpy(hb.p + uint64_t(k) * sizeof(CompressArgs), &pl[live[k]].a, sizeof(CompressArgs));
    std::memcpy(hb.p + jb, maps.buf.data(), mb);
    build_compress_batch_args(reinterpret_cast<const CompressArgs*>(hb.p), nl, b.max_levels,
                              hb.p + ao);
    uint8_t* blob = ws.at<uint8_t>(o_blob);
    CompressArgs* dj = reinterpret_cast<CompressArgs*>(blob);
    uint32_t* dm = reinterpret_cast<uint32_t*>(blob + jb);
    uint8_t* da = blob + ao;
    if (hipMemcpyAsync(blob, hb.p, ao + ab, hipMemcpyHostToDevice, st) != hipSuccess)
      return STZ_ERR_DEVICE;
    b.J = dj;
    b.args = da;
    b.host_J = reinterpret_cast<const CompressArgs*>(hb.p);
    b.pdirect = pdirect.data();
    b.n_pdirect = uint32_t(pdirect.size());
    b.whole = whole.data();
    b.n_whole = uint32_t(whole.size());
    maps.bind(dm);
    if (launch_compress_batch(b, st) != hipSuccess) return STZ_ERR_DEVICE;
    if (hipMemcpyAsync(hb.p, dpar, pb, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return STZ_ERR_DEVICE;
    prof_flush();
    const DevParams* hp = reinterpret_cast<const DevParams*>(hb.p);
    for (uint32_t k = 0; k < nl; ++k) {
      jobs[live[k]].out_size = hp[k].total;
      jobs[live[k]].status = params_status(hp[k]);
    }
  }
  for (uint64_t i = 0; i < njobs; ++i)
    if (jobs[i].status != STZ_OK) return static_cast<stz_status>(jobs[i].status);
  return STZ_OK;
}

}  // extern "C"

struct stz_field_s {
  stz::Header h;
  const uint8_t* comp = nullptr;
  uint64_t size = 0;
  uint16_t* lut = nullptr;  // device decoder table
  uint64_t lut_entries = 0;
  int device = 0;
  // per-unit ROI statistics already computed, by (level, unit kind, statistic)
  struct RoiStats {
    uint32_t key;
    double* dev;
    uint64_t n;
  };
  std::vector<RoiStats> roi;
};

extern "C" {

stz_status stz_open(const void* comp, uint64_t size, stz_field* field, void* stream) {
  if (!field) return STZ_ERR_ARG;
  *field = nullptr;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* f = new (std::nothrow) stz_field_s;
  if (!f) return STZ_ERR_NOMEM;
  stz_status s = read_header(comp, size, st, &f->h);
  Staging* stage = staging();
  if (s == STZ_OK && !stage) s = STZ_ERR_NOMEM;
  if (s == STZ_OK && !build_lut(f->h.lens, f->h.nsym, stage->lut)) s = STZ_ERR_CORRUPT;
  if (s != STZ_OK) {
    delete f;
    return s;
  }
  f->comp = static_cast<const uint8_t*>(comp);
  f->size = size;
  f->lut_entries = uint64_t(1) << kLutBits;
  if (hipGetDevice(&f->device) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&f->lut), f->lut_entries * 2) != hipSuccess) {
    delete f;
    return STZ_ERR_NOMEM;
  }
  if (hipMemcpyAsync(f->lut, stage->lut, f->lut_entries * 2, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipFree(f->lut);
    delete f;
    return STZ_ERR_DEVICE;
  }
  *field = f;
  return STZ_OK;
}

stz_status stz_field_info(stz_field f, stz_info_t* info) {
  if (!f || !info) return STZ_ERR_ARG;
  const Header& h = f->h;
  for (int d = 0; d < 3; ++d) info->dims[d] = uint64_t(h.g.n[d]);
  info->block = uint32_t(h.c.B);
  info->levels = uint32_t(h.c.L);
  info->radius = uint32_t(h.c.R);
  info->lmax = uint32_t(kLmax);
  info->eb_mode = uint32_t(h.eb_mode);
  info->dtype = h.vb == 8 ? 1u : 0u;
  info->eb = h.eb;
  info->eb_abs = h.eb_abs;
  info->eb_ratio = h.c.ratio;
  info->total_bytes = h.total;
  info->coding = uint32_t(h.c.coding);
  info->reserved = 0;
  return STZ_OK;
}

void stz_close(stz_field f) {
  if (!f) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != f->device) (void)hipSetDevice(f->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(f->lut);
  for (auto& r : f->roi) (void)hipFree(r.dev);
  if (cur != f->device) (void)hipSetDevice(cur);
  delete f;
}

stz_status stz_decompress_batch(stz_request* reqs, uint64_t n, uint32_t* dev_flags,
                                void* stream) {
  if (!reqs && n) return STZ_ERR_ARG;
  if (n == 0) return STZ_OK;
  if (n > STZ_MAX_BATCH) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<DecodePlan> pl(n);
  std::vector<uint32_t> live;
  for (uint64_t i = 0; i < n; ++i) {
    stz_request& r = reqs[i];
    for (int d = 0; d < 3; ++d) r.out_dims[d] = 0;
    if (!r.field || r.reserved) {
      r.status = STZ_ERR_ARG;
      continue;
    }
    Box box;
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      ok = ok && r.lo[d] < (uint64_t(1) << 40) && r.hi[d] < (uint64_t(1) << 40);
      box.lo[d] = int64_t(r.lo[d]);
      box.hi[d] = int64_t(r.hi[d]);
    }
    if (!ok || r.level > 64 || r.field->h.vb != 4) {  // batches decode float32 fields
      r.status = STZ_ERR_ARG;
      continue;
    }
    r.status = pl[i].init(r.field->h, r.field->comp, r.field->size, &box, int(r.level), r.out,
                          r.out_cap_elems);
    for (int d = 0; d < 3; ++d) r.out_dims[d] = pl[i].od[d];
    if (r.status == STZ_OK && pl[i].cnt) live.push_back(uint32_t(i));
  }
  const uint32_t nl = uint32_t(live.size());
  HostBuf& hb = host_buf(st);
  Workspace ws(st);
  BatchMaps maps;
  DecodeBatch b;
  std::vector<DirectItem> direct;
  if (nl) build_decode_maps(pl, live, &maps, &b, &direct);
  // One staging blob, laid out as on the device and sent with one copy:
  // request table | work maps | zero flags | per-level argument blocks
  // (256-aligned); the caller's zero flags follow it in host memory.
  const uint64_t rb = (uint64_t(nl) * sizeof(DecodeArgs) + 15) & ~uint64_t(15);
  const uint64_t mb = maps.buf.size() * sizeof(uint32_t);
  const uint64_t fb = uint64_t(nl) * 4;
  const uint64_t ao = (rb + mb + fb + 255) & ~uint64_t(255);
  const uint64_t ab = nl ? decode_batch_args_bytes(nl, b.max_level) : 0;
  const uint64_t cb = dev_flags ? n * 4 : 0;
  uint64_t o_blob = 0;
  if (nl) {
    for (uint32_t k = 0; k < nl; ++k) pl[live[k]].take(ws);
    o_blob = ws.take<uint8_t>(ao + ab);
    if (!ws.commit()) return STZ_ERR_NOMEM;
  }
  if (!hb.reserve(ao + ab + cb)) return STZ_ERR_NOMEM;
  std::memset(hb.p + rb + mb, 0, fb);
  std::memset(hb.p + ao + ab, 0, cb);
  if (dev_flags &&
      hipMemcpyAsync(dev_flags, hb.p + ao + ab, cb, hipMemcpyHostToDevice, st) != hipSuccess)
    return STZ_ERR_DEVICE;
  if (nl) {
    uint8_t* blob = ws.at<uint8_t>(o_blob);
    uint32_t* wflags = reinterpret_cast<uint32_t*>(blob + rb + mb);
    for (uint32_t k = 0; k < nl; ++k) {
      const stz_request& r = reqs[live[k]];
      pl[live[k]].bind(ws, r.field->lut, dev_flags ? dev_flags + live[k] : wflags + k);
    }
    for (uint32_t k = 0; k < nl; ++k)
      std::memcpy(hb.p + uint64_t(k) * sizeof(DecodeArgs), &pl[live[k]].a, sizeof(DecodeArgs));
    std::memcpy(hb.p + rb, maps.buf.data(), mb);
    build_decode_batch_args(reinterpret_cast<const DecodeArgs*>(hb.p), nl, b.max_level,
                            hb.p + ao);
    DecodeArgs* dr = reinterpret_cast<DecodeArgs*>(blob);
    uint32_t* dm = reinterpret_cast<uint32_t*>(blob + rb);
    uint8_t* da = blob + ao;
    if (hipMemcpyAsync(blob, hb.p, ao + ab, hipMemcpyHostToDevice, st) != hipSuccess)
      return STZ_ERR_DEVICE;
    if (!hb.mark(st)) return STZ_ERR_DEVICE;
    b.R = dr;
    b.args = da;
    b.host_R = reinterpret_cast<const DecodeArgs*>(hb.p);
    b.direct = direct.data();
    b.n_direct = uint32_t(direct.size());
    maps.bind(dm);
    if (launch_decode_batch(b, st) != hipSuccess) return STZ_ERR_DEVICE;
    if (!dev_flags) {
      // the flag words come back into the staging of the zero flags, which
      // the stream has consumed before the kernels ran
      if (hipMemcpyAsync(hb.p + rb + mb, wflags, fb, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return STZ_ERR_DEVICE;
      hb.pending = false;
      prof_flush();
      const uint32_t* hf = reinterpret_cast<const uint32_t*>(hb.p + rb + mb);
      for (uint32_t k = 0; k < nl; ++k)
        if (hf[k]) reqs[live[k]].status = STZ_ERR_CORRUPT;
    }
  } else if (dev_flags && !hb.mark(st)) {
    return STZ_ERR_DEVICE;
  }
  for (uint64_t i = 0; i < n; ++i)
    if (reqs[i].status != STZ_OK) return static_cast<stz_status>(reqs[i].status);
  return STZ_OK;
}

}  // extern "C"

// ---- captured batches (HIP graphs) -------------------------------------------
namespace stz {
namespace {

// Fills n words with v: the only way a captured graph clears memory (no
// memset nodes).
__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}

// Scratch owned by a plan: laid out by a Workspace, allocated once.
bool own_workspace(Workspace& ws, char** owned) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<uint64_t>(ws.size, 256)) != hipSuccess) return false;
  *owned = static_cast<char*>(p);
  ws.base = *owned;
  return true;
}

// Capture whatever `launch` enqueues into an executable graph, on a private
// stream (the caller's may be the legacy stream, which cannot capture).
template <class F>
stz_status capture_graph(F launch, hipGraph_t* g, hipGraphExec_t* x) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return STZ_ERR_DEVICE;
  stz_status s = STZ_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    s = STZ_ERR_DEVICE;
  } else {
    const bool ok = launch(cs);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(cs, &graph) != hipSuccess || !ok || !graph) {
      s = STZ_ERR_DEVICE;
      if (graph) (void)hipGraphDestroy(graph);
    } else if (hipGraphInstantiate(x, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      s = STZ_ERR_DEVICE;
    } else {
      *g = graph;
    }
  }
  (void)hipStreamDestroy(cs);
  return s;
}

}  // namespace
}  // namespace stz

struct stz_batch_s {
  int kind = 0;  // 0 compression, 1 decoding
  int device = 0;
  uint64_t n = 0;                  // jobs or requests
  std::vector<int32_t> status;     // validation status per entry
  std::vector<uint32_t> live;      // entries in the graph
  char* scratch = nullptr;         // plan-owned device memory
  stz::DevParams* dpar = nullptr;  // compression: per-live-job parameters
  uint32_t* flags = nullptr;       // decoding: per-live-request corruption flag
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace stz {
namespace {

void destroy_plan(stz_batch_s* b) {
  if (!b) return;
  int cur = 0;
  const bool sw = hipGetDevice(&cur) == hipSuccess && cur != b->device;
  if (sw) (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->scratch) (void)hipFree(b->scratch);
  if (sw) (void)hipSetDevice(cur);
  delete b;
}

}  // namespace
}  // namespace stz

extern "C" {

stz_status stz_compress_batch_plan(const stz_job* jobs, uint64_t njobs, stz_batch* plan,
                                   void* stream) {
  if (!plan) return STZ_ERR_ARG;
  *plan = nullptr;
  if ((!jobs && njobs) || njobs > STZ_MAX_BATCH) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* B = new (std::nothrow) stz_batch_s;
  if (!B) return STZ_ERR_NOMEM;
  B->kind = 0;
  B->n = njobs;
  B->status.assign(njobs, STZ_OK);
  if (hipGetDevice(&B->device) != hipSuccess) {
    delete B;
    return STZ_ERR_DEVICE;
  }
  std::vector<CompressPlan> pl(njobs);
  for (uint64_t i = 0; i < njobs; ++i) {
    B->status[i] = jobs[i].reserved ? STZ_ERR_ARG
                                    : pl[i].init(jobs[i].x, 4, jobs[i].dims, jobs[i].eb_mode,
                                                 jobs[i].eb, &jobs[i].cfg, jobs[i].out,
                                                 jobs[i].out_cap);
    if (B->status[i] == STZ_OK) B->live.push_back(uint32_t(i));
  }
  const uint32_t nl = uint32_t(B->live.size());
  if (nl == 0) {
    *plan = B;
    return STZ_OK;
  }
  Workspace ws(st);
  const uint64_t o_params = ws.take<DevParams>(nl);
  for (uint32_t k = 0; k < nl; ++k) pl[B->live[k]].take(ws);
  const uint64_t o_jobs = ws.take<CompressArgs>(nl);
  BatchMaps maps;
  CompressBatch b;
  std::vector<PredDirect> pdirect;
  std::vector<uint32_t> whole;
  build_compress_maps(pl, B->live, &maps, &b, &pdirect, &whole);
  const uint64_t o_maps = ws.take<uint32_t>(maps.buf.size());
  const uint64_t ab = compress_batch_args_bytes(nl, b.max_levels);
  const uint64_t o_args = ws.take<uint8_t>(ab);
  if (!own_workspace(ws, &B->scratch)) {
    destroy_plan(B);
    return STZ_ERR_NOMEM;
  }
  B->dpar = ws.at<DevParams>(o_params);
  for (uint32_t k = 0; k < nl; ++k) pl[B->live[k]].bind(ws, B->dpar + k);
  std::vector<CompressArgs> hj(nl);
  for (uint32_t k = 0; k < nl; ++k) hj[k] = pl[B->live[k]].a;
  std::vector<uint8_t> ha(ab);
  build_compress_batch_args(hj.data(), nl, b.max_levels, ha.data());
  CompressArgs* dj = ws.at<CompressArgs>(o_jobs);
  uint32_t* dm = ws.at<uint32_t>(o_maps);
  uint8_t* da = ws.at<uint8_t>(o_args);
  if (hipMemcpy(dj, hj.data(), nl * sizeof(CompressArgs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dm, maps.buf.data(), maps.buf.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(da, ha.data(), ab, hipMemcpyHostToDevice) != hipSuccess) {
    destroy_plan(B);
    return STZ_ERR_DEVICE;
  }
  b.J = dj;
  b.args = da;
  b.host_J = hj.data();
  b.pdirect = pdirect.data();
  b.n_pdirect = uint32_t(pdirect.size());
  b.whole = whole.data();
  b.n_whole = uint32_t(whole.size());
  maps.bind(dm);
  const stz_status s = capture_graph(
      [&](hipStream_t cs) { return launch_compress_batch(b, cs) == hipSuccess; }, &B->graph,
      &B->exec);
  if (s != STZ_OK) {
    destroy_plan(B);
    return s;
  }
  *plan = B;
  return STZ_OK;
}

stz_status stz_decompress_batch_plan(const stz_request* reqs, uint64_t n, stz_batch* plan,
                                     void* stream) {
  if (!plan) return STZ_ERR_ARG;
  *plan = nullptr;
  if ((!reqs && n) || n > STZ_MAX_BATCH) return STZ_ERR_ARG;
  (void)stream;
  auto* B = new (std::nothrow) stz_batch_s;
  if (!B) return STZ_ERR_NOMEM;
  B->kind = 1;
  B->n = n;
  B->status.assign(n, STZ_OK);
  if (hipGetDevice(&B->device) != hipSuccess) {
    delete B;
    return STZ_ERR_DEVICE;
  }
  std::vector<DecodePlan> pl(n);
  for (uint64_t i = 0; i < n; ++i) {
    const stz_request& r = reqs[i];
    if (!r.field || r.reserved) {
      B->status[i] = STZ_ERR_ARG;
      continue;
    }
    Box box;
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      ok = ok && r.lo[d] < (uint64_t(1) << 40) && r.hi[d] < (uint64_t(1) << 40);
      box.lo[d] = int64_t(r.lo[d]);
      box.hi[d] = int64_t(r.hi[d]);
    }
    if (!ok || r.level > 64 || r.field->h.vb != 4) {
      B->status[i] = STZ_ERR_ARG;
      continue;
    }
    B->status[i] = pl[i].init(r.field->h, r.field->comp, r.field->size, &box, int(r.level),
                              r.out, r.out_cap_elems);
    if (B->status[i] == STZ_OK && pl[i].cnt) B->live.push_back(uint32_t(i));
  }
  const uint32_t nl = uint32_t(B->live.size());
  if (nl == 0) {
    *plan = B;
    return STZ_OK;
  }
  Workspace ws(nullptr);
  for (uint32_t k = 0; k < nl; ++k) pl[B->live[k]].take(ws);
  const uint64_t o_req = ws.take<DecodeArgs>(nl);
  const uint64_t o_flags = ws.take<uint32_t>(nl);
  BatchMaps maps;
  DecodeBatch b;
  std::vector<DirectItem> direct;
  build_decode_maps(pl, B->live, &maps, &b, &direct);
  const uint64_t o_maps = ws.take<uint32_t>(maps.buf.size());
  const uint64_t ab = decode_batch_args_bytes(nl, b.max_level);
  const uint64_t o_args = ws.take<uint8_t>(ab);
  if (!own_workspace(ws, &B->scratch)) {
    destroy_plan(B);
    return STZ_ERR_NOMEM;
  }
  B->flags = ws.at<uint32_t>(o_flags);
  std::vector<DecodeArgs> hr(nl);
  for (uint32_t k = 0; k < nl; ++k) {
    pl[B->live[k]].bind(ws, reqs[B->live[k]].field->lut, B->flags + k);
    hr[k] = pl[B->live[k]].a;
  }
  std::vector<uint8_t> ha(ab);
  build_decode_batch_args(hr.data(), nl, b.max_level, ha.data());
  DecodeArgs* dr = ws.at<DecodeArgs>(o_req);
  uint32_t* dm = ws.at<uint32_t>(o_maps);
  uint8_t* da = ws.at<uint8_t>(o_args);
  if (hipMemcpy(dr, hr.data(), nl * sizeof(DecodeArgs), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dm, maps.buf.data(), maps.buf.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(da, ha.data(), ab, hipMemcpyHostToDevice) != hipSuccess) {
    destroy_plan(B);
    return STZ_ERR_DEVICE;
  }
  b.R = dr;
  b.args = da;
  b.host_R = hr.data();
  b.direct = direct.data();
  b.n_direct = uint32_t(direct.size());
  maps.bind(dm);
  uint32_t* flags = B->flags;
  const stz_status s = capture_graph(
      [&](hipStream_t cs) {
        hipLaunchKernelGGL(k_fill_u32, dim3(std::min<uint32_t>((nl + 255) / 256, 1024)),
                           dim3(256), 0, cs, flags, nl, 0u);
        return launch_decode_batch(b, cs) == hipSuccess;
      },
      &B->graph, &B->exec);
  if (s != STZ_OK) {
    destroy_plan(B);
    return s;
  }
  *plan = B;
  return STZ_OK;
}

stz_status stz_batch_run(stz_batch plan, void* stream) {
  if (!plan) return STZ_ERR_ARG;
  if (!plan->exec) return STZ_OK;
  return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess
             ? STZ_OK
             : STZ_ERR_DEVICE;
}

stz_status stz_batch_status(stz_batch plan, stz_job* jobs, stz_request* reqs, uint64_t n,
                            void* stream) {
  if (!plan || n != plan->n) return STZ_ERR_ARG;
  if (plan->kind == 0 ? !jobs && n : !reqs && n) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t nl = uint32_t(plan->live.size());
  std::vector<DevParams> hp(plan->kind == 0 ? nl : 0);
  std::vector<uint32_t> hf(plan->kind == 1 ? nl : 0);
  if (nl) {
    const hipError_t e =
        plan->kind == 0
            ? hipMemcpyAsync(hp.data(), plan->dpar, nl * sizeof(DevParams), hipMemcpyDeviceToHost,
                             st)
            : hipMemcpyAsync(hf.data(), plan->flags, nl * 4, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return STZ_ERR_DEVICE;
  }
  for (uint64_t i = 0; i < n; ++i) {
    if (plan->kind == 0) {
      jobs[i].status = plan->status[i];
      jobs[i].out_size = 0;
    } else {
      reqs[i].status = plan->status[i];
    }
  }
  for (uint32_t k = 0; k < nl; ++k) {
    const uint32_t i = plan->live[k];
    if (plan->kind == 0) {
      jobs[i].out_size = hp[k].total;
      jobs[i].status = params_status(hp[k]);
    } else if (hf[k]) {
      reqs[i].status = STZ_ERR_CORRUPT;
    }
  }
  for (uint64_t i = 0; i < n; ++i) {
    const int32_t v = plan->kind == 0 ? jobs[i].status : reqs[i].status;
    if (v != STZ_OK) return static_cast<stz_status>(v);
  }
  return STZ_OK;
}

void stz_batch_destroy(stz_batch plan) { stz::destroy_plan(plan); }

}  // extern "C"

namespace stz {
namespace {

// Candidate slab heights of the batched kernels per level block edge 2^e
// (the heights the kernels are instantiated for).
std::vector<int> pred_heights(int e) {
  switch (e) {
    case 3: return {8, 4};
    case 4: return {16, 8, 4};
    case 5: return {8, 4, 2};
    case 6: return {2, 4};
    default: return {0};
  }
}
std::vector<int> dec_heights(int e) {
  switch (e) {
    case 4: return {16, 8, 4};
    case 5: return {4, 8, 2};
    default: return {0};
  }
}

BatchTuning default_tuning() {
  BatchTuning d;
  d.grid = 2048;
  for (int e = 0; e < kBatchEdges; ++e) {
    d.grid_pred[e] = 1u << 20;
    d.grid_dec[e] = 1u << 20;
    d.pred_h[e] = 0;
    d.dec_h[e] = 0;
  }
  return d;
}

struct Tuner {
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  unsigned long long* dh = nullptr;  // digests (device)
  std::vector<unsigned long long> hh;
  std::string rep;

  bool setup(uint64_t n) {
    hh.resize(n);
    return hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&dh), std::max<uint64_t>(n, 1) * 8) == hipSuccess;
  }
  ~Tuner() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dh) (void)hipFree(dh);
  }
  // Digests of n device ranges; false on a runtime error.
  bool digest(const std::vector<const void*>& p, const std::vector<uint64_t>& b) {
    if (launch_hash(p.data(), b.data(), p.size(), dh, st) != hipSuccess ||
        hipMemcpy(hh.data(), dh, p.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return false;
    return true;
  }
  // Mean milliseconds of `reps` runs of f (after one untimed run), or -1.
  template <class F>
  double time(F f, int reps) {
    if (!f()) return -1.0;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.0;
    for (int r = 0; r < reps; ++r)
      if (!f()) return -1.0;
    float ms = 0.0f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1.0;
    return double(ms) / reps;
  }
  void note(const char* fmt, ...) {
    char line[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(line, sizeof(line), fmt, ap);
    va_end(ap);
    rep += line;
    rep += "\n";
  }
};

}  // namespace
}  // namespace stz

extern "C" {

stz_status stz_autotune_batch(stz_job* jobs, uint64_t njobs, char* report, uint64_t report_cap,
                              void* stream) {
  if (!jobs || njobs == 0 || njobs > STZ_MAX_BATCH) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  BatchTuning& tu = batch_tuning();
  tu = default_tuning();
  Tuner t;
  t.st = st;
  if (!t.setup(njobs)) return STZ_ERR_NOMEM;
  const int reps = 3;
  // Reference outputs with the default shapes.
  stz_status s = stz_compress_batch(jobs, njobs, stream);
  if (s != STZ_OK) return s;
  std::vector<const void*> ptr(njobs);
  std::vector<uint64_t> len(njobs);
  for (uint64_t i = 0; i < njobs; ++i) {
    ptr[i] = jobs[i].out;
    len[i] = jobs[i].out_size;
  }
  if (!t.digest(ptr, len)) return STZ_ERR_DEVICE;
  const std::vector<unsigned long long> ref = t.hh;
  // Level block edges present in the batch, with their total block counts.
  uint64_t edge_blocks[kBatchEdges] = {};
  for (uint64_t i = 0; i < njobs; ++i) {
    Cfg c;
    Geo g;
    if (resolve_cfg(&jobs[i].cfg, &c) != STZ_OK || !make_geo(jobs[i].dims, c, &g)) continue;
    for (int l = 1; l <= g.L; ++l)
      edge_blocks[ilog2(g.B >> (g.L - l))] += uint64_t(g.nb[0] * g.nb[1] * g.nb[2]);
  }
  bool mismatch = false;
  auto run_c = [&]() { return stz_compress_batch(jobs, njobs, stream) == STZ_OK; };
  auto check_c = [&]() {
    if (!t.digest(ptr, len)) return false;
    const bool same = t.hh == ref;
    mismatch = mismatch || !same;
    return same;
  };
  double best = t.time(run_c, reps);
  if (best < 0) return STZ_ERR_DEVICE;
  t.note("compress default: %.3f ms", best);
  const unsigned grids[] = {256, 512, 1024, 2048, 4096, 1u << 20};
  // Coordinate descent, the edges with most blocks first.
  std::vector<int> order;
  for (int e = 1; e < kBatchEdges; ++e)
    if (edge_blocks[e]) order.push_back(e);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return edge_blocks[x] > edge_blocks[y]; });
  for (int e : order) {
    for (int h : pred_heights(e)) {
      const int keep = tu.pred_h[e];
      tu.pred_h[e] = h;
      const double ms = t.time(run_c, reps);
      if (ms >= 0 && check_c() && ms < best) {
        best = ms;
        t.note("  edge %d predict slab height %d: %.3f ms", 1 << e, h, ms);
      } else {
        tu.pred_h[e] = keep;
      }
    }
    for (unsigned gsz : grids) {
      const unsigned keep = tu.grid_pred[e];
      tu.grid_pred[e] = gsz;
      const double ms = t.time(run_c, reps);
      if (ms >= 0 && check_c() && ms < best) {
        best = ms;
        t.note("  edge %d predict grid %u: %.3f ms", 1 << e, gsz, ms);
      } else {
        tu.grid_pred[e] = keep;
      }
    }
  }
  for (unsigned gsz : grids) {
    const unsigned keep = tu.grid;
    tu.grid = gsz;
    const double ms = t.time(run_c, reps);
    if (ms >= 0 && check_c() && ms < best) {
      best = ms;
      t.note("  grid %u: %.3f ms", gsz, ms);
    } else {
      tu.grid = keep;
    }
  }
  t.note("compress tuned: %.3f ms", best);
  if (!run_c()) return STZ_ERR_DEVICE;  // leave the jobs' outputs as produced

  // Decoder shapes: full decodes of every job's stream.
  std::vector<stz_field> fields(njobs, nullptr);
  float* dout = nullptr;
  uint64_t total = 0;
  std::vector<uint64_t> off(njobs);
  for (uint64_t i = 0; i < njobs; ++i) {
    off[i] = total;
    total += jobs[i].dims[0] * jobs[i].dims[1] * jobs[i].dims[2];
  }
  stz_status ds = STZ_OK;
  if (hipMalloc(reinterpret_cast<void**>(&dout), std::max<uint64_t>(total, 1) * 4) != hipSuccess)
    ds = STZ_ERR_NOMEM;
  for (uint64_t i = 0; i < njobs && ds == STZ_OK; ++i)
    ds = stz_open(jobs[i].out, jobs[i].out_size, &fields[i], stream);
  std::vector<stz_request> rq(njobs);
  std::vector<const void*> dptr(njobs);
  std::vector<uint64_t> dlen(njobs);
  if (ds == STZ_OK) {
    for (uint64_t i = 0; i < njobs; ++i) {
      stz_request& r = rq[i];
      std::memset(&r, 0, sizeof(r));
      r.field = fields[i];
      for (int d = 0; d < 3; ++d) r.hi[d] = jobs[i].dims[d];
      r.level = fields[i]->h.c.L;
      r.out = dout + off[i];
      r.out_cap_elems = total - off[i];
      dptr[i] = r.out;
      dlen[i] = 4 * jobs[i].dims[0] * jobs[i].dims[1] * jobs[i].dims[2];
    }
    auto run_d = [&]() { return stz_decompress_batch(rq.data(), njobs, nullptr, stream) == STZ_OK; };
    std::vector<unsigned long long> dref;
    if (!run_d() || !t.digest(dptr, dlen)) ds = STZ_ERR_DEVICE;
    dref = t.hh;
    auto check_d = [&]() {
      if (!t.digest(dptr, dlen)) return false;
      const bool same = t.hh == dref;
      mismatch = mismatch || !same;
      return same;
    };
    double dbest = ds == STZ_OK ? t.time(run_d, reps) : -1.0;
    if (dbest < 0) ds = STZ_ERR_DEVICE;
    if (ds == STZ_OK) {
      t.note("decode default: %.3f ms", dbest);
      for (int e : order) {
        for (int h : dec_heights(e)) {
          const int keep = tu.dec_h[e];
          tu.dec_h[e] = h;
          const double ms = t.time(run_d, reps);
          if (ms >= 0 && check_d() && ms < dbest) {
            dbest = ms;
            t.note("  edge %d decode slab height %d: %.3f ms", 1 << e, h, ms);
          } else {
            tu.dec_h[e] = keep;
          }
        }
        for (unsigned gsz : grids) {
          const unsigned keep = tu.grid_dec[e];
          tu.grid_dec[e] = gsz;
          const double ms = t.time(run_d, reps);
          if (ms >= 0 && check_d() && ms < dbest) {
            dbest = ms;
            t.note("  edge %d decode grid %u: %.3f ms", 1 << e, gsz, ms);
          } else {
            tu.grid_dec[e] = keep;
          }
        }
      }
      t.note("decode tuned: %.3f ms", dbest);
    }
  }
  for (stz_field f : fields) stz_close(f);
  if (dout) (void)hipFree(dout);
  if (mismatch) t.note("some candidates changed the output and were rejected");
  if (report && report_cap) {
    const uint64_t k = std::min<uint64_t>(report_cap - 1, t.rep.size());
    std::memcpy(report, t.rep.data(), k);
    report[k] = 0;
  }
  return ds;
}

stz_status stz_roi_select(stz_field f, uint32_t level, uint32_t unit, uint32_t stat,
                          uint32_t rule, double value, uint32_t* sel, uint64_t cap,
                          uint64_t* count, double* stats, void* stream) {
  if (!f || !count || unit > 3 || stat > 1 || rule > 1) return STZ_ERR_ARG;
  if (rule == 1 && !(value > 0.0 && value <= 1.0)) return STZ_ERR_ARG;
  if (rule == 0 && std::isnan(value)) return STZ_ERR_ARG;
  const Header& h = f->h;
  const Geo& g = h.g;
  if (int64_t(level) > g.L) return STZ_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int logs = g.L - int(level);
  int64_t gn[3];
  for (int d = 0; d < 3; ++d) gn[d] = ((g.n[d] - 1) >> logs) + 1;
  const uint64_t ngrid = uint64_t(gn[0]) * gn[1] * gn[2];
  const uint64_t nunits =
      unit == 0 ? uint64_t(g.nb[0] * g.nb[1] * g.nb[2]) : uint64_t(gn[unit - 1]);
  const uint32_t key = (level << 8) | (unit << 4) | stat;
  double* dstats = nullptr;
  for (auto& r : f->roi)
    if (r.key == key) dstats = r.dev;
  HostBuf& hb = host_buf(st);
  if (!dstats) {
    // First selection of this kind: decode the whole domain at `level` into
    // scratch and compute the per-unit statistics into device memory the field
    // keeps, so later selections need no decode. The plan is made against a
    // placeholder output and pointed at the scratch grid.
    if (hipMalloc(reinterpret_cast<void**>(&dstats), std::max<uint64_t>(nunits, 1) * 8) !=
        hipSuccess)
      return STZ_ERR_NOMEM;
    DecodePlan pl;
    stz_status s = pl.init(h, f->comp, f->size, nullptr, int(level),
                           reinterpret_cast<void*>(uintptr_t(256)), ngrid);
    Workspace ws(st);
    uint64_t o_grid = 0, o_flags = 0;
    if (s == STZ_OK) {
      pl.take(ws);
      o_grid = ws.take<uint8_t>(uint64_t(h.vb) * ngrid);
      o_flags = ws.take<uint32_t>(1);
      if (!ws.commit()) s = STZ_ERR_NOMEM;
    }
    Staging* stage = staging();
    if (s == STZ_OK && !stage) s = STZ_ERR_NOMEM;
    if (s != STZ_OK) {
      (void)hipFree(dstats);
      return s;
    }
    void* grid = ws.at<uint8_t>(o_grid);
    uint32_t* dflags = ws.at<uint32_t>(o_flags);
    pl.a.rec[pl.a.level_out] = grid;
    pl.bind(ws, f->lut, dflags);
    *stage->flags = 0;
    const int64_t E = int64_t(g.B) >> logs;
    const int64_t nb[3] = {g.nb[0], g.nb[1], g.nb[2]};
    if (hipMemcpyAsync(dflags, stage->flags, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_decode(pl.a, st) != hipSuccess ||
        launch_roi_stats(grid, h.vb, gn, E, int(unit), int(stat), nb, nunits, dstats, st) !=
            hipSuccess ||
        hipMemcpyAsync(stage->flags, dflags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      (void)hipFree(dstats);
      return STZ_ERR_DEVICE;
    }
    prof_flush();
    if (*stage->flags) {
      (void)hipFree(dstats);
      return STZ_ERR_CORRUPT;
    }
    f->roi.push_back({key, dstats, nunits});
  }
  // selection on the device: flags, then the ascending selected indices
  const uint64_t k =
      rule == 1 ? std::min<uint64_t>(nunits, uint64_t(std::ceil(value * double(nunits)))) : 0;
  Workspace ws(st);
  const uint64_t o_scr = ws.take<uint8_t>(kRoiScratchBytes);
  const uint64_t o_sel = ws.take<uint32_t>(nunits);
  const uint64_t o_cnt = ws.take<uint64_t>(1);
  if (!ws.commit()) return STZ_ERR_NOMEM;
  uint32_t* dsel = ws.at<uint32_t>(o_sel);
  uint64_t* dcnt = ws.at<uint64_t>(o_cnt);
  const uint64_t hs = 8 + nunits * 4 + (stats ? nunits * 8 : 0);
  if (!hb.reserve(hs)) return STZ_ERR_NOMEM;
  if (launch_roi_select(dstats, nunits, int(rule), value, k, ws.at<uint8_t>(o_scr), dsel,
                        nunits, dcnt, st) != hipSuccess ||
      hipMemcpyAsync(hb.p, dcnt, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hb.p + 8, dsel, nunits * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      (stats && hipMemcpyAsync(hb.p + 8 + nunits * 4, dstats, nunits * 8, hipMemcpyDeviceToHost,
                               st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return STZ_ERR_DEVICE;
  prof_flush();
  uint64_t n_sel = 0;
  std::memcpy(&n_sel, hb.p, 8);
  if (stats) std::memcpy(stats, hb.p + 8 + nunits * 4, nunits * 8);
  *count = n_sel;
  if (n_sel > cap || (!sel && n_sel)) return STZ_ERR_BUFFER;
  if (n_sel) std::memcpy(sel, hb.p + 8, n_sel * 4);
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
    info->dtype = h.vb == 8 ? 1u : 0u;
    info->eb = h.eb;
    info->eb_abs = h.eb_abs;
    info->eb_ratio = h.c.ratio;
    info->total_bytes = h.total;
    info->coding = uint32_t(h.c.coding);
    info->reserved = 0;
  }
  return STZ_OK;
}

}  // extern "C"

namespace stz {
namespace {

stz_status region_one(const void* comp, uint64_t size, const uint64_t lo[3], const uint64_t hi[3],
                      uint32_t level, void* out, uint64_t out_cap_elems, uint64_t out_dims[3],
                      int vb, void* stream) {
  if (!lo || !hi) return STZ_ERR_ARG;
  Box b;
  for (int d = 0; d < 3; ++d) {
    if (lo[d] > (uint64_t(1) << 32) || hi[d] > (uint64_t(1) << 32)) return STZ_ERR_ARG;
    b.lo[d] = int64_t(lo[d]);
    b.hi[d] = int64_t(hi[d]);
  }
  if (level > uint32_t(kMaxLevels)) return STZ_ERR_ARG;
  return decode_box(comp, size, &b, int(level), out, out_cap_elems, out_dims, vb,
                    static_cast<hipStream_t>(stream));
}

stz_status level_one(const void* comp, uint64_t size, uint32_t level, void* out,
                     uint64_t out_cap_elems, uint64_t out_dims[3], int vb, void* stream) {
  if (level > uint32_t(kMaxLevels)) return STZ_ERR_ARG;
  return decode_box(comp, size, nullptr, int(level), out, out_cap_elems, out_dims, vb,
                    static_cast<hipStream_t>(stream));
}

}  // namespace

// Scratch of stz_decompress_region_noalloc. Each GPU holds its own copy from
// module load until the process ends. In host code the name is only a
// stand-in: every use goes through the address from hipGetSymbolAddress.
__device__ __align__(256) uint8_t scratch[STZ_NOALLOC_SCRATCH_BYTES];

namespace {

void* noalloc_scratch() {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace
}  // namespace stz

extern "C" {

stz_status stz_decompress_region_noalloc(const void* comp, uint64_t size, const uint64_t lo[3],
                                         const uint64_t hi[3], uint32_t level, float* out,
                                         uint64_t out_cap_elems, uint64_t out_dims[3],
                                         void* stream) {
  if (!lo || !hi) return STZ_ERR_ARG;
  Box b;
  for (int d = 0; d < 3; ++d) {
    if (lo[d] > (uint64_t(1) << 32) || hi[d] > (uint64_t(1) << 32)) return STZ_ERR_ARG;
    b.lo[d] = int64_t(lo[d]);
    b.hi[d] = int64_t(hi[d]);
  }
  if (level > uint32_t(kMaxLevels)) return STZ_ERR_ARG;
  return decode_box_noalloc(comp, size, &b, int(level), out, out_cap_elems, out_dims,
                            static_cast<hipStream_t>(stream));
}

stz_status stz_decompress_region(const void* comp, uint64_t size, const uint64_t lo[3],
                                 const uint64_t hi[3], uint32_t level, float* out,
                                 uint64_t out_cap_elems, uint64_t out_dims[3], void* stream) {
  return region_one(comp, size, lo, hi, level, out, out_cap_elems, out_dims, 4, stream);
}

stz_status stz_decompress_region_f64(const void* comp, uint64_t size, const uint64_t lo[3],
                                     const uint64_t hi[3], uint32_t level, double* out,
                                     uint64_t out_cap_elems, uint64_t out_dims[3],
                                     void* stream) {
  return region_one(comp, size, lo, hi, level, out, out_cap_elems, out_dims, 8, stream);
}

stz_status stz_decompress_level(const void* comp, uint64_t size, uint32_t level, float* out,
                                uint64_t out_cap_elems, uint64_t out_dims[3], void* stream) {
  return level_one(comp, size, level, out, out_cap_elems, out_dims, 4, stream);
}

stz_status stz_decompress_level_f64(const void* comp, uint64_t size, uint32_t level, double* out,
                                    uint64_t out_cap_elems, uint64_t out_dims[3], void* stream) {
  return level_one(comp, size, level, out, out_cap_elems, out_dims, 8, stream);
}

stz_status stz_decompress(const void* comp, uint64_t size, float* out, uint64_t out_cap_elems,
                          void* stream) {
  uint64_t od[3];
  return decode_box(comp, size, nullptr, -1, out, out_cap_elems, od, 4,
                    static_cast<hipStream_t>(stream));
}

stz_status stz_decompress_f64(const void* comp, uint64_t size, double* out,
                              uint64_t out_cap_elems, void* stream) {
  uint64_t od[3];
  return decode_box(comp, size, nullptr, -1, out, out_cap_elems, od, 8,
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
