// Internal definitions of the HIP library: format constants, geometry
// descriptors passed to kernels, the device parameter block and the kernel
// launchers. Host code and kernels include this file; nothing outside the
// library does.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stz {

// ---- format constants (compressed-stream specification) --------------------
constexpr uint32_t kMagic = 0x315A5453u;  // 'S','T','Z','1'
constexpr uint32_t kVersion = 1;
constexpr uint64_t kHeaderBytes = 512;
constexpr int kLmax = 12;             // longest Huffman code
constexpr int kLutBits = kLmax;       // decoder table indexed by the next 12 bits
constexpr int kMaxLevels = 6;         // B <= 64
constexpr int kMaxRadius = 1024;      // quantization symbols 2R <= 2048
constexpr int kMaxAlphabet = 2 * kMaxRadius + 1;  // plus the zero-chunk token
constexpr uint64_t kLevelTable = 128;
constexpr uint64_t kLevelRec = 48;

// Device-side error flags.
constexpr uint32_t kFlagNonfinite = 1u;
constexpr uint32_t kFlagOverflow = 2u;   // output capacity exceeded
constexpr uint32_t kFlagCorrupt = 4u;
constexpr uint32_t kFlagBadBound = 8u;   // resolved bound not positive and finite
constexpr uint32_t kFlagTooLarge = 16u;  // a per-level count exceeds 32 bits

__host__ __device__ inline uint64_t align16(uint64_t v) { return (v + 15) & ~uint64_t(15); }

// ---- geometry --------------------------------------------------------------
struct Geo {
  int64_t n[3];    // nz, ny, nx
  int64_t nb[3];   // blocks per axis
  int32_t B, logB, L, R;
  int32_t Z;       // zero-chunk token (2R), or -1 when that stage is off
  int32_t pad;
};

// Code alphabet: the 2R quantization symbols, plus the zero-chunk token.
__host__ __device__ inline int alphabet(const Geo& g) { return 2 * g.R + (g.Z >= 0 ? 1 : 0); }

// Class sub-grid extent along axis d of block b, class parity o, stride 2^logs.
__host__ __device__ inline int64_t axis_M(const Geo& g, int d, int64_t b, int o, int logs) {
  const int64_t lo = b << g.logB;
  const int64_t rest = g.n[d] - lo;
  const int64_t len = rest < int64_t(g.B) ? rest : int64_t(g.B);
  const int64_t U = (len + (int64_t(1) << logs) - 1) >> logs;
  return o ? (U >> 1) : ((U + 1) >> 1);
}
// Sum of axis_M over blocks b' < b (all of them full blocks).
__host__ __device__ inline int64_t axis_P(const Geo& g, int64_t b, int logs) {
  return b * (int64_t(g.B) >> (logs + 1));
}
// Sum of axis_M over all blocks along axis d.
__host__ __device__ inline int64_t axis_T(const Geo& g, int d, int o, int logs) {
  return axis_P(g, g.nb[d] - 1, logs) + axis_M(g, d, g.nb[d] - 1, o, logs);
}

// Symbols of level 2^logs that precede unit u in stream order (blocks raster,
// classes 1..7, rank order inside a unit), in closed form.
__host__ __device__ inline int64_t unit_sym_off(const Geo& g, int logs, int64_t u) {
  const int64_t blk = u / 7;
  const int c = int(u - blk * 7) + 1;
  const int64_t bx = blk % g.nb[2], t = blk / g.nb[2], by = t % g.nb[1], bz = t / g.nb[1];
  int64_t sum = 0;
  for (int k = 1; k <= 7; ++k) {
    const int oz = (k >> 2) & 1, oy = (k >> 1) & 1, ox = k & 1;
    const int64_t Mz = axis_M(g, 0, bz, oz, logs), My = axis_M(g, 1, by, oy, logs),
                  Mx = axis_M(g, 2, bx, ox, logs);
    const int64_t Ty = axis_T(g, 1, oy, logs), Tx = axis_T(g, 2, ox, logs);
    sum += axis_P(g, bz, logs) * Ty * Tx + Mz * axis_P(g, by, logs) * Tx +
           Mz * My * axis_P(g, bx, logs);
    if (k < c) sum += Mz * My * Mx;
  }
  return sum;
}

// Lane streams (one per x-column of a unit) that precede unit u.
__host__ __device__ inline int64_t unit_lane_off(const Geo& g, int logs, int64_t u) {
  const int64_t blk = u / 7;
  const int c = int(u - blk * 7) + 1;
  const int64_t bx = blk % g.nb[2], t = blk / g.nb[2], by = t % g.nb[1], bz = t / g.nb[1];
  int64_t sum = 0;
  for (int k = 1; k <= 7; ++k) {
    const int ox = k & 1;
    sum += (bz * g.nb[1] + by) * axis_T(g, 2, ox, logs) + axis_P(g, bx, logs);
    if (k < c) sum += axis_M(g, 2, bx, ox, logs);
  }
  return sum;
}

// Level totals: symbols and lanes.
__host__ __device__ inline int64_t level_nsym(const Geo& g, int logs) {
  int64_t sum = 0;
  for (int k = 1; k <= 7; ++k)
    sum += axis_T(g, 0, (k >> 2) & 1, logs) * axis_T(g, 1, (k >> 1) & 1, logs) *
           axis_T(g, 2, k & 1, logs);
  return sum;
}
__host__ __device__ inline int64_t level_nlanes(const Geo& g, int logs) {
  int64_t sum = 0;
  for (int k = 1; k <= 7; ++k) sum += g.nb[0] * g.nb[1] * axis_T(g, 2, k & 1, logs);
  return sum;
}

// Points of one level's grid inside a box: coordinates first[d] + i*s,
// i < cnt[d]. The full domain is first = 0, cnt = (n-1)/s + 1.
struct Grid {
  int64_t first[3];
  int64_t cnt[3];
  int32_t logs;
};

// Half-open box in full-resolution coordinates.
struct Box {
  int64_t lo[3];
  int64_t hi[3];
};

// Parameters resolved on the device (error bounds) and the stream layout.
// Quantizer constants for both value types: float32 fields use E2/INV and the
// exact bound e; float64 fields use E2d/INVd and the acceptance bound echk.
struct DevParams {
  double eb_abs;
  double e[kMaxLevels + 1];
  float E2[kMaxLevels + 1];
  float INV[kMaxLevels + 1];
  double E2d[kMaxLevels + 1];
  double INVd[kMaxLevels + 1];
  double echk[kMaxLevels + 1];
  double mn, mx;
  uint32_t flags;
  uint32_t pad;
  uint64_t total;                          // stream bytes
  uint64_t sec[kMaxLevels + 1];            // level section offset
  uint64_t off_outl[kMaxLevels + 1];       // unit_outl array offset (absolute)
  uint64_t off_lane[kMaxLevels + 1];       // lane_len array offset (absolute)
  uint64_t off_pay[kMaxLevels + 1];        // payload offset (absolute)
  uint64_t off_out[kMaxLevels + 1];        // outlier values offset (absolute)
  uint64_t words[kMaxLevels + 1];          // payload words per level
  uint64_t outl[kMaxLevels + 1];           // outliers per level
};

// Per-level constants known on the host (geometry only).
struct LevelConst {
  uint64_t nu;     // units
  uint64_t nl;     // lanes
  uint64_t nsym;   // symbols
};

// Value type of a field: 4 = float32 (stream value type 0), 8 = float64 (1).
// Min/max partials of the range reduction, in the field's value type.
template <class T>
struct MinMax {
  T mn, mx;
};

// ---- launchers (defined with the kernels) ----------------------------------
struct CompressArgs {
  const void* x;           // field values (float or double, see vb)
  int vb;                  // bytes per value: 4 or 8
  Geo geo;
  int eb_mode;
  double eb, ratio;
  uint8_t* out;
  uint64_t out_cap;
  DevParams* params;
  // scratch
  void* part;              // MinMax<value type> partials
  uint32_t nparts;
  void* rec[kMaxLevels];   // compact grids of levels 0..L-1 (value type)
  uint16_t* sym[kMaxLevels + 1];
  LevelConst lc[kMaxLevels + 1];
  unsigned long long* hist;   // token counts (alphabet entries)
  uint32_t* hpart;            // [nslots][alphabet] partial counts of the predictor
  uint32_t nslots;            // histogram slots: min(blocks, kHistSlots)
  uint8_t* lens;              // 2R
  uint16_t* codes;            // 2R
  void* cb_scratch;           // codebook_scratch_bytes(2R)
  uint16_t* lane_len;         // per level, at lane_base[l]
  uint64_t lane_base[kMaxLevels + 1];
  uint32_t* cnt;              // [2L segments][nu]: unit words, unit outliers
  uint32_t* scan;             // [2L segments][nu+1]
  uint64_t* scan_part;        // block partials for the segmented scan
  uint64_t n_anchor;
};

hipError_t launch_compress(const CompressArgs& a, hipStream_t st);

// ---- batched launches -------------------------------------------------------
// Work map of a batched launch: entry i covers items [first[i], first[i+1])
// of job job[i]; first has n+1 entries. Device pointers.
struct ItemMap {
  const uint32_t* first;
  const uint32_t* job;
  uint32_t n;
};

constexpr int kBatchEdges = 7;  // level block edge E = 2^e, e = 1..6

// The predictor's work-groups add their block histograms into one of
// kHistSlots partial histograms (chosen by work-group index, so concurrent
// work-groups rarely meet on an address; a slot's bins are contiguous); a
// reduction sums the slots. A slot holds at most 2^40 / 128 counts, within
// 32 bits.
constexpr uint32_t kHistSlots = 128;

// One batched compression: the job table (device) and the work map of every
// launch; n_* are the item totals (host copies of first[n]).
// A (job, level) pair whose predictor runs as a plain launch of its own
// inside a batched compression (many blocks of 32^3 points or more).
struct PredDirect {
  uint32_t job;
  int level;
};
constexpr uint64_t kWholeJobPoints = uint64_t(1) << 27;  // 512^3

struct CompressBatch {
  const CompressArgs* J;
  const uint8_t* args;                         // per-level argument blocks (device)
  const CompressArgs* host_J;                  // host copy of the job table
  const PredDirect* pdirect;                   // host array
  uint32_t n_pdirect;
  // Jobs of at least kWholeJobPoints values (each fills the GPU by itself):
  // the plain launch sequence of their own, no work items in the maps.
  const uint32_t* whole;                       // host array of job-table indices
  uint32_t n_whole;
  uint32_t njobs;
  unsigned grid;                               // persistent work-groups per launch
  unsigned grid_pred[kBatchEdges];             // per level block edge
  int max_levels;
  ItemMap jobs1, minmax, anchor, scan_ac, scan_b, zero, head, hzero, hred;
  uint32_t n_jobs1, n_minmax, n_anchor, n_scan_ac, n_scan_b, n_zero, n_head, n_hzero, n_hred;
  ItemMap pred[kMaxLevels + 1][kBatchEdges];   // blocks of level l with edge 2^e
  uint32_t n_pred[kMaxLevels + 1][kBatchEdges];
  ItemMap level[kMaxLevels + 1];               // blocks of every job with L >= l
  uint32_t n_level[kMaxLevels + 1];
  ItemMap pack_u[kMaxLevels + 1], pack_l[kMaxLevels + 1];  // the same, by packer:
  uint32_t n_pack_u[kMaxLevels + 1], n_pack_l[kMaxLevels + 1];  // level edge >= 32 / < 32
  int pred_h[kBatchEdges];                     // predictor slab height per edge
};

// Launch shapes of the batched kernels (output-invariant), set by the
// autotuner: persistent work-groups per launch and, per level block edge
// 2^e, the predictor's and decoder's grids and slab heights.
struct BatchTuning {
  unsigned grid;
  unsigned grid_pred[kBatchEdges];
  int pred_h[kBatchEdges];
  unsigned grid_dec[kBatchEdges];
  int dec_h[kBatchEdges];
};
BatchTuning& batch_tuning();

hipError_t launch_compress_batch(const CompressBatch& b, hipStream_t st);
// Per-level argument blocks of a batched compression, built on the host from
// the bound job table (device pointers filled in) and uploaded with it.
uint64_t compress_batch_args_bytes(uint32_t n, int max_levels);
void build_compress_batch_args(const CompressArgs* jobs, uint32_t n, int max_levels,
                               uint8_t* dst);
void launch_codebook_batch(const CompressArgs* J, uint32_t njobs, hipStream_t st);

// Code book from the histogram (lengths and canonical codes, 2R entries).
size_t codebook_scratch_bytes(int nsym);
void launch_codebook(const unsigned long long* hist, int nsym, uint8_t* lens, uint16_t* codes,
                     void* scratch, hipStream_t st);

struct DecodeArgs {
  const uint8_t* comp;
  uint64_t size;
  Geo geo;
  int vb;                     // bytes per value: 4 or 8
  int level_out;
  Box box[kMaxLevels + 1];    // R_k per level
  void* rec[kMaxLevels + 1];  // box grids of levels 0..level_out (last = output)
  uint64_t sec[kMaxLevels + 1];
  uint64_t off_outl[kMaxLevels + 1], off_lane[kMaxLevels + 1], off_pay[kMaxLevels + 1],
      off_out[kMaxLevels + 1];
  uint64_t words[kMaxLevels + 1], outl[kMaxLevels + 1];
  LevelConst lc[kMaxLevels + 1];
  uint64_t anchor_off;
  float E2[kMaxLevels + 1];
  double E2d[kMaxLevels + 1];
  const uint16_t* lut;   // 2^kLutBits entries: symbol | length << 12
  uint32_t* flags;       // device word
};

// The header bytes a plain decode launched on a kept header was parsed from,
// passed by value to the decode's anchor kernel, which sets flags[1] to 1 when
// the stream's first n bytes differ from them, else 0.
struct HdrRef {
  uint32_t n;
  uint8_t b[kHeaderBytes + kMaxAlphabet];
};

// ref: null, or the kept header bytes to check the stream against.
hipError_t launch_decode(const DecodeArgs& a, hipStream_t st, const HdrRef* ref = nullptr);
// Per-unit ROI statistics of a level grid (see stz_roi_select).
hipError_t launch_roi_stats(const void* grid, int vb, const int64_t gn[3], int64_t E, int unit,
                            int stat, const int64_t nb[3], uint64_t nunits, double* out,
                            hipStream_t st);
// A second stream beside the caller's stream `st` (same device, default
// priority, created on first use and kept until stz_trim), with a fork and a
// join event: work enqueued on it after it waits for `fork` (recorded on st)
// runs concurrently with st's, and st waits for `join` before going on.
// nullptr when it cannot be created (run the work on st instead).
struct AuxStream {
  hipStream_t s;
  hipEvent_t fork, join;
};
const AuxStream* aux_stream(hipStream_t st);
// Whether `st` is being captured into a graph.
bool capturing(hipStream_t st);

// Device ROI selection over n per-unit statistics (n < 2^32): rule 0 keeps
// statistics above `value`, rule 1 the k largest (ties to the smaller index).
// The ascending selected indices go to sel (at most cap written) and their
// number to *count (device). `scratch` holds kRoiScratchBytes.
constexpr uint64_t kRoiStateBytes = 2048;
constexpr uint64_t kRoiScratchBytes = kRoiStateBytes + 4 * 1024 * 8;
hipError_t launch_roi_select(const double* stats, uint64_t n, int rule, double value, uint64_t k,
                             void* scratch, uint32_t* sel, uint64_t cap, uint64_t* count,
                             hipStream_t st);

// One batched decode: the request table (device) and the work maps of every
// launch. Level k of request r has edge E = B_r >> (L_r - k).
// A (request, level) pair decoded by a plain launch of its own.
struct DirectItem {
  uint32_t req;
  int level;
};
constexpr uint64_t kDirectBlocks = 1024;  // blocks at one level that fill the device

struct DecodeBatch {
  const DecodeArgs* R;
  const uint8_t* args;                        // per-level argument blocks (device)
  const DecodeArgs* host_R;                   // host copy of the request table
  const DirectItem* direct;                   // host array
  uint32_t n_direct;
  uint32_t nreq;
  unsigned grid;
  unsigned grid_dec[kBatchEdges];
  int dec_h[kBatchEdges];
  int max_level;
  ItemMap anchor;
  uint32_t n_anchor;
  uint32_t n_check[kMaxLevels + 1];           // requests that decode level k
  ItemMap dec[kMaxLevels + 1][kBatchEdges];   // blocks of each request's box at level k
  uint32_t n_dec[kMaxLevels + 1][kBatchEdges];
};

hipError_t launch_decode_batch(const DecodeBatch& b, hipStream_t st);
// Per-level argument blocks of a batched decode, [level 1..max_level][request],
// built on the host from the bound request table.
uint64_t decode_batch_args_bytes(uint32_t n, int max_level);
void build_decode_batch_args(const DecodeArgs* reqs, uint32_t n, int max_level, uint8_t* dst);

// Digest of each of n device byte ranges into out[i] (device), for checking
// that two launch shapes give identical outputs.
hipError_t launch_hash(const void* const* ptrs, const uint64_t* bytes, uint64_t n,
                       unsigned long long* out, hipStream_t st);

}  // namespace stz
