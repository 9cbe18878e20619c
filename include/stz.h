/*
 * stz.h - C ABI of the MI355X (gfx950) STZ streaming-compressor hot path.
 *
 * Method (paper: "STZ: A High Quality and High Speed Streaming Lossy
 * Compression Framework for Scientific Data", SC'25):
 *   - hierarchical partition of a 3-D field into levels by stride-2 sampling,
 *     recursively (Sec. 3.1 "Hierarchical partition", Sec. 3.2);
 *   - prediction of each finer point from already reconstructed coarser points
 *     by multi-dimensional linear and cubic interpolation (Sec. 3.1,
 *     Eqs. 3-8), quantization of the prediction difference directly
 *     (Optimization 3) under per-level error bounds (Optimization 5);
 *   - Huffman coding of the quantization codes with per-(level, block,
 *     sub-block) offsets, so levels and blocks decode independently;
 *   - full, progressive (stop at a level) and random-access (box) decoding
 *     (Sec. 3.3).
 *
 * Conventions for every call:
 *   - Pointers marked "device" are HIP device pointers on the current device;
 *     "host" pointers are ordinary host memory. The caller owns every buffer;
 *     the library keeps no pointer after a call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream).
 *     Host out-parameters are valid when the call returns; device outputs are
 *     valid once the stream reaches the end of the call's work. A call may run
 *     part of its work on an internal stream of the library (one per caller
 *     stream and device, default priority); that work starts after the
 *     caller's earlier work on `stream` and `stream` waits for it before any
 *     later work (events), so stream order is what the caller sees. Calls that
 *     return a host value (sizes, status of device-side checks) synchronize
 *     the stream once at their end.
 *   - Dims are {nz, ny, nx}, C order, x fastest.
 *   - Internal scratch memory is a per-(device, stream) buffer that the
 *     library grows on demand (see stz_trim); a call returns STZ_ERR_NOMEM
 *     when it cannot be obtained.
 *   - Errors: STZ_ERR_ARG for invalid arguments, STZ_ERR_NONFINITE when the
 *     input holds NaN or Inf, STZ_ERR_BUFFER when an output capacity is too
 *     small (nothing meaningful is written), STZ_ERR_CORRUPT when a stream
 *     fails validation (decoders never read or write out of bounds on corrupt
 *     input), STZ_ERR_DEVICE on a HIP runtime failure.
 */
#ifndef STZ_H
#define STZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STZ_OK = 0,
  STZ_ERR_ARG = -1,
  STZ_ERR_NONFINITE = -2,
  STZ_ERR_BUFFER = -3,
  STZ_ERR_CORRUPT = -4,
  STZ_ERR_DEVICE = -5,
  STZ_ERR_NOMEM = -6
} stz_status;

/* Error-bound mode: absolute, or relative to the field's value range
 * (max - min), as in the paper's problem statement (Sec. 2.1). */
typedef enum { STZ_EB_ABS = 0, STZ_EB_REL = 1 } stz_eb_mode;

/* Entropy-coding stage. Huffman only codes every quantization symbol; the
 * zero-chunk stage first replaces each chunk of a lane stream (the symbols of
 * one sub-block row along y inside a block) whose symbols all have zero
 * residual by one extra token, then Huffman-codes the tokens. It is lossless:
 * both modes reconstruct the same values. */
typedef enum {
  STZ_CODING_DEFAULT = 0,     /* zero chunks + Huffman                         */
  STZ_CODING_HUFFMAN = 1,
  STZ_CODING_ZERO_CHUNKS = 2
} stz_coding;

/* Block and level configuration. Zero fields select the defaults. */
typedef struct {
  uint32_t block;    /* B: block edge, power of two in [2, 64]; 0 -> 32      */
  uint32_t levels;   /* L: levels above the anchors, 1..log2(B); 0 -> log2 B */
  uint32_t radius;   /* R: quantization radius, 1..1024, alphabet 2R; 0->512 */
  uint32_t coding;   /* stz_coding                                           */
  double eb_ratio;   /* bound ratio between adjacent paper levels (Sec. 3.1,
                        Optimization 5), >= 1; 0 -> 2.5                      */
} stz_config;

/* Stream description (parsed header). dtype is the value type of the field
 * (header byte offset 52): 0 = float32, 1 = float64. coding is the resolved
 * stz_coding (1 or 2). */
typedef struct {
  uint64_t dims[3];
  uint32_t block, levels, radius, lmax, eb_mode, dtype;
  double eb, eb_abs, eb_ratio;
  uint64_t total_bytes;
  uint32_t coding, reserved;
} stz_info_t;

/* Upper bound of the compressed size in bytes for `dims` and `cfg` (host
 * only; no device work). Returns 0 for invalid arguments. */
uint64_t stz_compress_bound(const uint64_t dims[3], const stz_config* cfg);

/* Compress the float32 field `x` (device, dims[0]*dims[1]*dims[2] values)
 * under error bound `eb` (> 0) in mode `eb_mode` into `out` (device,
 * `out_cap` bytes). `*out_size` (host) receives the stream size; on
 * STZ_ERR_BUFFER it holds the size that would have been needed. Every
 * reconstructed value differs from the input by at most the resolved absolute
 * bound (Sec. 2.1). The steps, in order: bound resolution (Sec. 2.1), anchors
 * on the stride-B grid, then per level from coarse to fine the prediction of
 * each point from reconstructed coarser points (Sec. 3.1, Eqs. 3-8) and its
 * linear quantization under the level's bound (Sec. 3.1, Optimizations 3 and
 * 5), and the Huffman coding of the symbols with per-level, per-block
 * offsets (Sec. 3.2, 3.3), so that every level and block decodes alone.
 * Synchronizes `stream` once (the stream size). */
stz_status stz_compress(const float* x, const uint64_t dims[3], int eb_mode, double eb,
                        const stz_config* cfg, void* out, uint64_t out_cap,
                        uint64_t* out_size, void* stream);

/* Parse the header of the stream `comp` (device, `size` bytes) into `info`
 * (host). Copies 512 bytes to the host and synchronizes `stream`. */
stz_status stz_info(const void* comp, uint64_t size, stz_info_t* info, void* stream);

/* Full decompression (Sec. 3.3, the finest level of progressive decoding)
 * into `out` (device, at least dims product floats, raster order): anchors,
 * then level by level the Huffman decode of the symbols and the same
 * prediction as the compressor (Sec. 3.1, Eqs. 3-8) plus dequantization, so
 * every value equals the compressor's reconstruction bit for bit. The call
 * synchronizes `stream` twice: for the stream header (the launch shapes and
 * the decoder table come from it) and for the corruption flag; a stream
 * opened with stz_open and decoded through stz_decompress_batch or a captured
 * decode plan needs neither round trip. The parsed headers of the last 16
 * (device, comp, size) triples decoded are kept on the host: a call on a
 * kept one skips the header round trip, and the decode's first kernel
 * compares the stream's header bytes with the kept ones; when they
 * differ (new contents at the same address and size) the call reads the
 * header and decodes again, so its result and status are those of a fresh
 * read. Decoder tables are kept in device memory per code (up to 64 codes per
 * process, freed by stz_trim), so repeated decodes of a stream upload none.
 * The same holds for stz_decompress_level, stz_decompress_region and the
 * float64 variants. */
stz_status stz_decompress(const void* comp, uint64_t size, float* out, uint64_t out_cap_elems,
                          void* stream);

/* Progressive decompression (Sec. 3.3, progressive decoding; the level
 * hierarchy of Sec. 3.1-3.2): reconstruct levels 0..level and write
 * the stride-2^(L-level) grid, dims floor((n-1)/s)+1 per axis, into `out`
 * (device). `out_dims` (host) receives its shape. level == L is the full
 * field; level 0 returns the anchors. */
stz_status stz_decompress_level(const void* comp, uint64_t size, uint32_t level, float* out,
                                uint64_t out_cap_elems, uint64_t out_dims[3], void* stream);

/* Random-access decompression (Sec. 3.3) of the half-open box [lo, hi)
 * (full-resolution coordinates, lo < hi <= dims) at progressive level `level`:
 * writes the points of the stride-2^(L-level) grid inside the box, raster
 * order, into `out` (device); `out_dims` (host) receives the shape (an axis
 * with no grid point gives 0 and nothing is written). Only the sub-blocks in
 * the box's dependency cone are decoded and predicted. */
stz_status stz_decompress_region(const void* comp, uint64_t size, const uint64_t lo[3],
                                 const uint64_t hi[3], uint32_t level, float* out,
                                 uint64_t out_cap_elems, uint64_t out_dims[3], void* stream);

/* Size in bytes of the fixed device scratch of stz_decompress_region_noalloc. */
#define STZ_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* stz_decompress_region for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, layouts, results and errors, but the call allocates nothing.
 * Its scratch (the dependency cone's coarse level grids, the decoder table and
 * a flag word) is a fixed device array of STZ_NOALLOC_SCRATCH_BYTES that each
 * GPU holds from the library's load until the process ends; the stream header
 * and the table pass through host stack buffers (pageable copies). A decode
 * whose scratch would exceed that size returns STZ_ERR_NOMEM and does nothing
 * (for float32 fields, about sum over levels k < level of 4 * (cone points at
 * level k): a 256^3 box at the finest level of a 512^3 field needs ~12 MB, a
 * full 512^3 decode ~77 MB, too much). float32 streams only (STZ_ERR_ARG for
 * others). Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (different streams or host threads) race; calls on one
 * stream from one thread are safe. The call synchronizes `stream` twice (the
 * header, then the status). With the stage profiler on it still creates
 * timing events. */
stz_status stz_decompress_region_noalloc(const void* comp, uint64_t size, const uint64_t lo[3],
                                         const uint64_t hi[3], uint32_t level, float* out,
                                         uint64_t out_cap_elems, uint64_t out_dims[3],
                                         void* stream);

/* ---- float64 fields -------------------------------------------------------
 * Double-precision fields (the paper's WarpX data are float64, Sec. 4.1,
 * Table 2) use the same format with value type 1 in the header: prediction
 * (Eqs. 3-8) and quantization evaluated in double in the same order, and the
 * anchors and outliers stored as 8-byte values. The acceptance test of a
 * quantized value is |x - x'| <= e*(1 - 2^-50) on the rounded double
 * difference, which guarantees the exact |x - x'| <= e. Arguments, layouts
 * and errors are those of the float32 calls above, with double in place of
 * float; each decoder accepts only streams of its own value type and returns
 * STZ_ERR_ARG for the other. The batched calls, fields opened for batches and
 * ROI selection: see their own comments. */
uint64_t stz_compress_bound_f64(const uint64_t dims[3], const stz_config* cfg);
stz_status stz_compress_f64(const double* x, const uint64_t dims[3], int eb_mode, double eb,
                            const stz_config* cfg, void* out, uint64_t out_cap,
                            uint64_t* out_size, void* stream);
stz_status stz_decompress_f64(const void* comp, uint64_t size, double* out,
                              uint64_t out_cap_elems, void* stream);
stz_status stz_decompress_level_f64(const void* comp, uint64_t size, uint32_t level, double* out,
                                    uint64_t out_cap_elems, uint64_t out_dims[3], void* stream);
stz_status stz_decompress_region_f64(const void* comp, uint64_t size, const uint64_t lo[3],
                                     const uint64_t hi[3], uint32_t level, double* out,
                                     uint64_t out_cap_elems, uint64_t out_dims[3],
                                     void* stream);

/* ---- Batched compression ------------------------------------------------
 * Many independent fields of any sizes, each with its own bound and
 * configuration, compressed by one sequence of persistent launches (every
 * launch walks the blocks of all fields). Each job's stream is byte-identical
 * to what stz_compress produces for the same arguments. Launch shapes
 * (persistent grid sizes, slab heights) come from the batch tuning table,
 * which stz_autotune_batch fills; they never change the output. */
typedef struct {
  const float* x;      /* device, dims[0]*dims[1]*dims[2] values              */
  uint64_t dims[3];
  int32_t eb_mode;     /* stz_eb_mode                                          */
  uint32_t reserved;   /* must be 0                                            */
  double eb;
  stz_config cfg;
  void* out;           /* device, out_cap bytes                                */
  uint64_t out_cap;
  uint64_t out_size;   /* written: stream size (or the size needed)            */
  int32_t status;      /* written: the stz_status stz_compress would return    */
  uint32_t reserved2;
} stz_job;

#define STZ_MAX_BATCH 65536

/* Compress `njobs` (<= STZ_MAX_BATCH) float32 fields described by `jobs`
 * (host array). Invalid jobs get their status and are left out; the others run.
 * Returns STZ_OK when every job succeeded, else the first failing job's
 * status. Synchronizes `stream` once. */
stz_status stz_compress_batch(stz_job* jobs, uint64_t njobs, void* stream);

/* ---- Resident fields and batched decoding (serving) ---------------------
 * stz_open validates the header of a compressed stream that stays in device
 * memory (`comp`, `size` bytes, owned by the caller and kept alive and
 * unchanged until stz_close) and uploads its decoder table once; later
 * decodes need no host round trip. */
typedef struct stz_field_s* stz_field;

stz_status stz_open(const void* comp, uint64_t size, stz_field* field, void* stream);
stz_status stz_field_info(stz_field field, stz_info_t* info);
/* Synchronizes the device before releasing the field's table. */
void stz_close(stz_field field);

/* One decode request: the box [lo, hi) (full-resolution coordinates) of a
 * resident field at progressive level `level` (levels of the field: the whole
 * domain at level L is a full decompression), written in raster order into
 * `out` (device, out_cap_elems floats), exactly as stz_decompress_region
 * would write it. */
typedef struct {
  stz_field field;
  uint64_t lo[3], hi[3];
  uint32_t level;
  uint32_t reserved;      /* must be 0                                          */
  float* out;
  uint64_t out_cap_elems;
  uint64_t out_dims[3];   /* written: output shape                              */
  int32_t status;         /* written: argument status; corruption found on the
                             device is reported through the flags word          */
  uint32_t reserved2;
} stz_request;

/* Decode `n` requests (host array) with one launch sequence: per level, one
 * persistent launch per level block edge walks the blocks of every request's
 * dependency cone. Requests take float32 fields; a request on a float64 field
 * gets STZ_ERR_ARG (decode those with stz_decompress_region_f64).
 * Asynchronous: when `dev_flags` (device, n words) is not
 * NULL, the call does not synchronize; word i becomes nonzero when request i
 * met a corrupt stream, and host-side argument errors are in status. With
 * dev_flags NULL the call synchronizes and sets status to STZ_ERR_CORRUPT
 * where needed. Returns STZ_OK when every request was accepted (and, when
 * synchronous, decoded), else the first failing request's status. The
 * library's host staging for a stream is reused by the next call on that
 * stream only after the previous call's copies have run. */
stz_status stz_decompress_batch(stz_request* reqs, uint64_t n, uint32_t* dev_flags,
                                void* stream);

/* ---- Captured batches (HIP graphs) ----------------------------------------
 * The batching pattern with persistent kernels captured once (Sec. 3.3's
 * many-field workflows: in-situ compression of successive time steps, repeated
 * region decodes). A plan fixes a job array (or request array): pointers,
 * extents, bounds, configurations and output buffers. Planning validates it,
 * lays out and allocates the plan's own scratch once, uploads the job tables
 * once and captures the whole launch sequence of stz_compress_batch
 * (stz_decompress_batch) into a HIP graph. Every device-side clear inside the
 * graph is a kernel. stz_batch_run replays the graph on `stream` with no host
 * work, no allocation and no synchronization; the contents of the inputs may
 * change between runs (the outputs are then exactly those of the eager call
 * on the new data). Statuses and compressed sizes stay on the device until
 * stz_batch_status reads them. Runs of one plan must not overlap (they share
 * its scratch); resident fields of a decode plan must stay open. Invalid
 * entries are left out of the graph and keep their validation status. */
typedef struct stz_batch_s* stz_batch;

/* Plan and capture a compression batch; `jobs` (host, njobs <= STZ_MAX_BATCH)
 * is read during the call only. */
stz_status stz_compress_batch_plan(const stz_job* jobs, uint64_t njobs, stz_batch* plan,
                                   void* stream);
/* Plan and capture a decode batch of `n` requests (host array, read during
 * the call only; out_dims and status are not written here). */
stz_status stz_decompress_batch_plan(const stz_request* reqs, uint64_t n, stz_batch* plan,
                                     void* stream);
/* Enqueue one replay of the plan's graph on `stream` (asynchronous). */
stz_status stz_batch_run(stz_batch plan, void* stream);
/* Synchronize `stream` and report the last run: for a compression plan
 * jobs[i].status and out_size, for a decode plan reqs[i].status (corruption
 * found on the device gives STZ_ERR_CORRUPT); n must equal the planned count
 * and the other array pointer may be NULL. Returns the first failing status. */
stz_status stz_batch_status(stz_batch plan, stz_job* jobs, stz_request* reqs, uint64_t n,
                            void* stream);
/* Synchronizes the plan's device, then frees the graph and its scratch. */
void stz_batch_destroy(stz_batch plan);


/* ---- ROI selection (Sec. 3.3, flexible scientific workflow) ---------------
 * Decodes the resident field at progressive level `level` (cheap at coarse
 * levels), computes for every unit the maximum (stat 0) or the value range
 * max - min (stat 1, in double) over the level's grid points, and selects:
 * rule 0 = units whose statistic exceeds `value`; rule 1 = the
 * ceil(value * units) units with the largest statistic (0 < value <= 1; ties
 * go to the smaller index). unit 0 = the blocks of B^3 full-resolution points
 * (raster index; block b spans [b*B, (b+1)*B) per axis, so a selected block is
 * a box for stz_decompress_region / stz_decompress_batch); unit 1/2/3 = the
 * level grid's planes across axis z/y/x (index = plane number, full-resolution
 * coordinate index * 2^(L-level)). Selected indices go to `sel` (host, cap
 * entries, ascending), their number to *count (host; on STZ_ERR_BUFFER the
 * number needed); `stats` (host, may be NULL) receives every unit's statistic.
 * The statistics are computed on the device and kept with the field: only
 * the first selection for a (level, unit, statistic) decodes the level; later
 * ones reuse the statistics. The selection itself (threshold, or the k largest
 * by rank over all pairs) and the compaction of the selected indices run on
 * the device too. The kept statistics are freed by stz_close; calls on one
 * field from several host threads must not overlap. Fields of either value
 * type. Synchronizes `stream`. */
stz_status stz_roi_select(stz_field field, uint32_t level, uint32_t unit, uint32_t stat,
                          uint32_t rule, double value, uint32_t* sel, uint64_t cap,
                          uint64_t* count, double* stats, void* stream);

/* ---- Autotuner -------------------------------------------------------------
 * Times candidate launch shapes of the batched kernels (persistent grid sizes
 * and slab heights, per level block edge) on the given jobs, keeps the
 * fastest that reproduces the reference outputs exactly, and stores them in
 * the process-wide batch tuning table. `jobs` are run several times (their
 * outputs are overwritten); `report` (host, may be NULL) receives a text
 * summary of at most report_cap bytes. Synchronizes `stream`. */
stz_status stz_autotune_batch(stz_job* jobs, uint64_t njobs, char* report, uint64_t report_cap,
                              void* stream);

/* Device scratch (auxiliary): every call takes its scratch from a buffer the
 * library keeps per (device, stream) and grows on demand, so repeated calls
 * allocate nothing. Calls on one stream run in stream order and share that
 * stream's buffer; calls on different streams use different buffers.
 * stz_trim synchronizes the current device and releases its buffers, its kept
 * decoder tables and headers and the library's internal streams (for a process that is done with the library, or
 * before a stream is destroyed and its handle value reused by another stream
 * would keep a large buffer alive). */
stz_status stz_trim(void);

/* Stage profiler (auxiliary; off by default, or on with STZ_PROFILE=1):
 * records HIP events on the call's stream around every kernel and
 * accumulates the elapsed time per kernel name and level ("predict@5") when
 * the call synchronizes. stz_profile_entry copies entry i's name (at most
 * name_cap bytes, NUL-terminated) and totals; returns -1 when i is out of
 * range. Intended for single-threaded measurement runs. */
void stz_profile_enable(int enable);
void stz_profile_reset(void);
int stz_profile_count(void);
int stz_profile_entry(int i, char* name, int name_cap, uint64_t* launches, double* total_ms);

/* Static description of a status code. */
const char* stz_status_string(stz_status st);

#ifdef __cplusplus
}
#endif

#endif /* STZ_H */
