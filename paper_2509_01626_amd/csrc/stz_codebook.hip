// Canonical Huffman code book on the device (format section 2.4).
//
// The format limits code lengths to kLmax by repeatedly replacing every
// nonzero count c with (c+1)>>1 and rebuilding. Applying that k times gives
// ceil(c / 2^k), so the rule is: the smallest k >= 0 whose Huffman code for
// the counts ceil(c / 2^k) has no code longer than kLmax. Counts never exceed
// 2^40, so k <= 40 always succeeds (all counts 1, at most 2049 tokens). The
// device builds the trees for every k in parallel, one work-group per k, and a
// second kernel picks the first k that fits: the latency of one build instead
// of one build per halving.
#include "stz_device.h"

namespace stz {
using namespace dev;
namespace {

constexpr int kCbThreads = 1024;
constexpr int kCbMax = 4096;            // power of two >= the largest alphabet
constexpr int kCbNodes = 2 * kMaxAlphabet;  // >= max(kCbMax, 2 * alphabet - 1)
constexpr int kCbPer = (kCbNodes + kCbThreads - 1) / kCbThreads;
constexpr int kSymBits = 12;            // symbol field of the sort keys
constexpr uint64_t kSymMask = (uint64_t(1) << kSymBits) - 1;
static_assert(kMaxAlphabet <= kCbMax && kCbMax <= (1 << kSymBits), "alphabet too large");
static_assert(kCbNodes >= kCbMax && kCbNodes >= 2 * kMaxAlphabet - 1, "node arrays too small");
constexpr int kCbScales = 42;           // k = 0..41
constexpr uint64_t kInf = ~uint64_t(0);

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor(uint32_t(v), m, 64);
  const uint32_t hi = __shfl_xor(uint32_t(v >> 32), m, 64);
  return (uint64_t(hi) << 32) | lo;
}

// Number of entries of the ascending a[0, len) below t (AT_MOST: at most t),
// by binary search.
template <bool AT_MOST>
__device__ inline int rank_below(const uint64_t* a, int len, uint64_t t) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (AT_MOST ? a[mid] <= t : a[mid] < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Ascending sort of n 64-bit keys in LDS (n a power of two, 64 <= n <=
// kCbMax): runs of 64 sorted in registers by one wave each (a bitonic network
// over the lanes, no barriers), then merged pairwise: a key's place in the
// merged pair is its index in its run plus the number of keys of the other
// run below it (first run) or at most it (second run), so equal keys (the
// padding) land on distinct places. Uses tmp (n keys); the result is in key.
__device__ void block_sort_u64(uint64_t* key, uint64_t* tmp, int n) {
  const int t = threadIdx.x, lane = t & 63, nw = blockDim.x >> 6;
  for (int r = t >> 6; r < n / 64; r += nw) {
    uint64_t v = key[r * 64 + lane];
    for (int k = 2; k <= 64; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        const uint64_t o = shfl_xor64(v, j);
        const bool keep_min = ((lane & k) == 0) == ((lane & j) == 0);
        v = keep_min ? (o < v ? o : v) : (o < v ? v : o);
      }
    key[r * 64 + lane] = v;
  }
  __syncthreads();
  uint64_t* src = key;
  uint64_t* dst = tmp;
  for (int len = 64; len < n; len <<= 1) {
    for (int i = t; i < n; i += blockDim.x) {
      const int base = i & ~(2 * len - 1), off = i - base;
      const bool in_a = off < len;
      const uint64_t v = src[i];
      const int other = in_a ? base + len : base;
      const int pos = in_a ? off + rank_below<false>(src + other, len, v)
                           : off - len + rank_below<true>(src + other, len, v);
      dst[base + pos] = v;
    }
    __syncthreads();
    uint64_t* sw = src;
    src = dst;
    dst = sw;
  }
  if (src != key) {
    for (int i = t; i < n; i += blockDim.x) key[i] = src[i];
    __syncthreads();
  }
}

// Two-queue merge (leaves W[0..m) ascending; merged nodes appended from W[m]
// in creation order; ties go to the leaf queue): parent of every node into
// par, node ids = positions. Run by one thread. 64-bit weights, with a
// two-deep register lookahead on both queues.
__device__ inline void merge64(uint64_t* W, int m, uint16_t* par) {
  // leaves are W[li..m), merged nodes W[ii..next)
  int li = 0, ii = m, next = m;
  uint64_t l0 = W[0], l1 = W[1], i0 = kInf, i1 = kInf;
  for (int it = 0; it < m - 1; ++it) {
    int a, b;
    uint64_t wa, wb;
    if (li < m && (ii == next || l0 <= i0)) {
      a = li;
      wa = l0;
      ++li;
      l0 = l1;
      l1 = li + 1 < m ? W[li + 1] : kInf;
    } else {
      a = ii;
      wa = i0;
      ++ii;
      i0 = i1;
      i1 = ii + 1 < next ? W[ii + 1] : kInf;
    }
    if (li < m && (ii == next || l0 <= i0)) {
      b = li;
      wb = l0;
      ++li;
      l0 = l1;
      l1 = li + 1 < m ? W[li + 1] : kInf;
    } else {
      b = ii;
      wb = i0;
      ++ii;
      i0 = i1;
      i1 = ii + 1 < next ? W[ii + 1] : kInf;
    }
    const uint64_t nw = wa + wb;
    W[next] = nw;
    par[a] = uint16_t(next);
    par[b] = uint16_t(next);
    if (ii == next)
      i0 = nw;
    else if (ii + 1 == next)
      i1 = nw;
    ++next;
  }
  par[2 * m - 2] = uint16_t(2 * m - 2);
  }

// Orders LDS accesses of one wave: what a lane wrote before the call is seen
// by every lane of the same wave after it.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// First index in [lo, hi) of the ascending array A whose value exceeds t (hi
// if none), found by one wave in 64-way steps; every lane returns it.
__device__ inline int wave_upper_bound(const uint32_t* A, int lo, int hi, uint32_t t) {
  const int lane = threadIdx.x & 63;
  while (hi - lo > 64) {
    const int step = (hi - lo + 63) >> 6;
    const int idx = lo + lane * step;
    const int c = __popcll(__ballot(idx < hi && A[idx] <= t));
    if (c == 0) return lo;
    lo += (c - 1) * step;
    hi = min(hi, lo + step);
  }
  const int idx = lo + lane;
  return lo + __popcll(__ballot(idx < hi && A[idx] <= t));
}

// Number of entries of the ascending A[lo, hi) below t (strict) or at most t,
// by binary search in one lane.
template <bool STRICT>
__device__ inline int count_before(const uint32_t* A, int lo, int hi, uint32_t t) {
  const int base = lo;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool go = STRICT ? A[mid] < t : A[mid] <= t;
    lo = go ? mid + 1 : lo;
    hi = go ? hi : mid;
  }
  return lo - base;
}

// The two-queue merge with 32-bit weights (total below 2^32 - 1), by one wave,
// in phases that reproduce the serial merge exactly. The serial merge removes
// nodes in the order S = the merge of the leaf queue and the merged-node queue
// (a leaf first on equal weights, merged nodes in creation order), and merged
// node k is S[2k] + S[2k+1]. Let t be the weight of the next merged node to be
// created. Every remaining node of weight <= t precedes it (and every later
// one) in S, so a phase appends all of them to S at once, placed by the merge
// rule, and then creates every merged node whose two children are in S. The
// threshold at least doubles every two phases, so there are at most about
// 2*log2(total) phases (about 26 on these histograms).
// LDS layout: LW = leaves [0, m) plus two ~0 pads; IW = merged nodes
// [0, m - 1); SW = weights of S [0, 2m - 2); Sid = node ids of S (leaf i = i,
// merged node k = m + k); par = parent of each node id.
__device__ inline void merge_phased(const uint32_t* LW, uint32_t* IW, uint32_t* SW, uint16_t* Sid,
                                    int m, uint16_t* par) {
  const int lane = threadIdx.x & 63;
  int li = 0, ki = 0, q = 0, p = 0;  // next leaf, next merged node, merged count, |S|
  while (q < m - 1) {
    const uint32_t a0 = LW[li], a1 = LW[li + 1];
    const uint32_t b0 = ki < q ? IW[ki] : ~0u, b1 = ki + 1 < q ? IW[ki + 1] : ~0u;
    uint32_t t;
    if (p & 1) {
      t = SW[p - 1] + min(a0, b0);
    } else {
      const uint32_t s1 = min(a0, b0);
      const uint32_t s2 = a0 <= b0 ? min(a1, b0) : min(a0, b1);
      t = s1 + s2;
    }
    const int cl = wave_upper_bound(LW, li, m, t) - li;
    const int ci = wave_upper_bound(IW, ki, q, t) - ki;
    for (int e = lane; e < cl + ci; e += 64) {
      if (e < cl) {
        const uint32_t w = LW[li + e];
        const int pos = e + count_before<true>(IW, ki, ki + ci, w);
        SW[p + pos] = w;
        Sid[p + pos] = uint16_t(li + e);
      } else {
        const int b = e - cl;
        const uint32_t w = IW[ki + b];
        const int pos = b + count_before<false>(LW, li, li + cl, w);
        SW[p + pos] = w;
        Sid[p + pos] = uint16_t(m + ki + b);
      }
    }
    wave_sync();
    p += cl + ci;
    const int q1 = p >> 1;
    for (int k = q + lane; k < q1; k += 64) {
      IW[k] = SW[2 * k] + SW[2 * k + 1];
      par[Sid[2 * k]] = uint16_t(m + k);
      par[Sid[2 * k + 1]] = uint16_t(m + k);
    }
    wave_sync();
    li += cl;
    ki += ci;
    q = q1;
  }
  if (lane == 0) par[2 * m - 2] = uint16_t(2 * m - 2);
}

// Code lengths for counts ceil(hist / 2^k), k = blockIdx.x: two queues over the
// leaves sorted by (count, symbol), ties to the leaf queue, merged nodes in
// creation order; depths by pointer jumping.
__device__ inline void cb_build_body(const unsigned long long* hist, int nsym, uint8_t* lens_k,
                                     int* maxlen_k, int k) {
  // nodes: the sorted leaves (padded to a power of two while sorting) and then
  // the m - 1 merged nodes: at most kCbNodes entries
  __shared__ uint64_t W[kCbNodes + 2];
  __shared__ uint64_t sort_tmp[kCbMax];
  __shared__ uint16_t par[2][kCbNodes];  // ping-pong buffers of the depth pass
  __shared__ uint16_t dep[2][kCbNodes];
  __shared__ uint16_t leaf[kCbMax];
  __shared__ int s_max;
  __shared__ int wcnt[kCbMax / 64];
  __shared__ unsigned long long s_tot;
  const int t = threadIdx.x, lane = t & 63;
  uint8_t* lens = lens_k + size_t(k) * nsym;
  if (t == 0) s_max = 0;
  // the used symbols' keys, compacted in symbol order (any order would do:
  // the sort orders them) with per-wave ballots
  const uint64_t add = (uint64_t(1) << k) - 1;
  constexpr int kPassC = kCbMax / kCbThreads;
  uint64_t cs[kPassC];
  uint64_t bal[kPassC];
#pragma unroll
  for (int q = 0; q < kPassC; ++q) {
    const int i = q * kCbThreads + t;
    cs[q] = i < nsym ? uint64_t(hist[i]) : 0;
    bal[q] = __ballot(cs[q] != 0);
    if (lane == 0) wcnt[i >> 6] = __popcll(bal[q]);
    if (i < nsym) lens[i] = 0;
  }
  __syncthreads();
  int m = 0;
#pragma unroll
  for (int q = 0; q < kPassC; ++q) {
    const int i = q * kCbThreads + t;
    int before = 0;
    for (int w = 0; w < kCbMax / 64; ++w) {
      before += w < (i >> 6) ? wcnt[w] : 0;
      m += q == 0 ? wcnt[w] : 0;
    }
    if (cs[q])
      W[before + __popcll(bal[q] & ((uint64_t(1) << lane) - 1))] =
          (((cs[q] + add) >> k) << kSymBits) | uint64_t(i);
  }
  int np2 = 64;
  while (np2 < m) np2 <<= 1;
  for (int i = m + t; i < np2; i += blockDim.x) W[i] = kInf;
  __syncthreads();
  block_sort_u64(W, sort_tmp, np2);
  if (m <= 1) {
    if (m == 1 && t == 0) lens[W[0] & kSymMask] = 1;
    if (t == 0) maxlen_k[k] = m;
    return;
  }
  unsigned long long tot = 0;  // total weight (the root's)
  for (int i = t; i < m; i += blockDim.x) {
    leaf[i] = uint16_t(W[i] & kSymMask);
    W[i] = W[i] >> kSymBits;
    tot += W[i];
  }
  if (t == 0) s_tot = 0;
  __syncthreads();
  if (tot) atomicAdd(&s_tot, tot);
  __syncthreads();
  if (s_tot < 0xFFFFFFFFull) {
    // 32-bit weights: repack the leaves in place as u32 (LW), then merged
    // nodes (IW) and the removal order (SW) behind them, within W's storage
    // (4m + 3 words); the removal order's node ids go to dep until the depths
    // are computed
    uint32_t wv[kCbPer];
    int j = 0;
    for (int i = t; i < m; i += blockDim.x, ++j) wv[j] = uint32_t(W[i]);
    __syncthreads();
    uint32_t* LW = reinterpret_cast<uint32_t*>(W);
    j = 0;
    for (int i = t; i < m; i += blockDim.x, ++j) LW[i] = wv[j];
    if (t < 2) LW[m + t] = ~0u;
    __syncthreads();
    if (t < 64) merge_phased(LW, LW + m + 2, LW + 2 * m + 1, dep[0], m, par[0]);
  } else if (t == 0) {
    merge64(W, m, par[0]);
  }
  __syncthreads();
  // depths by pointer jumping: each round reads one buffer and writes the
  // other, so one barrier per round
  const int nn = 2 * m - 1;
  for (int i = t; i < nn; i += blockDim.x) dep[0][i] = (i == nn - 1) ? 0 : 1;
  __syncthreads();
  int cur = 0;
  for (int round = 0; (1 << round) < nn; ++round) {
    const uint16_t* pd = dep[cur];
    const uint16_t* pp = par[cur];
    uint16_t* nd = dep[cur ^ 1];
    uint16_t* np = par[cur ^ 1];
    for (int i = t; i < nn; i += blockDim.x) {
      const int p = pp[i];
      nd[i] = pd[i] + pd[p];
      np[i] = pp[p];
    }
    cur ^= 1;
    __syncthreads();
  }
  int mx = 0;
  for (int i = t; i < m; i += blockDim.x) {
    const int d = dep[cur][i];
    lens[leaf[i]] = uint8_t(d > 255 ? 255 : d);
    mx = max(mx, d);
  }
  atomicMax(&s_max, mx);
  __syncthreads();
  if (t == 0) maxlen_k[k] = s_max;
}

__global__ __launch_bounds__(kCbThreads) void k_cb_build(const unsigned long long* hist, int nsym,
                                                         uint8_t* lens_k, int* maxlen_k) {
  cb_build_body(hist, nsym, lens_k, maxlen_k, blockIdx.x);
}

// Pick the first scale whose code fits in kLmax bits; canonical codes (by
// length, then symbol): a symbol's code = the first code of its length + the
// number of smaller symbols with the same length, counted with per-wave
// ballots and per-wave totals (no sort).
__device__ inline void cb_final_body(const uint8_t* lens_k, const int* maxlen_k, int nsym,
                                     uint8_t* lens_out, uint16_t* codes_out) {
  constexpr int kW = kCbThreads / 64;     // waves
  constexpr int kPass = kCbMax / kCbThreads;  // symbols per thread, one per pass
  __shared__ uint32_t wcnt[kPass][kW][kLmax + 1];  // per pass and wave: symbols per length
  __shared__ uint32_t bl[kLmax + 2], first[kLmax + 1];
  __shared__ int s_k;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) {
    int kk = kCbScales - 1;
    for (int k = 0; k < kCbScales; ++k)
      if (maxlen_k[k] <= kLmax) {
        kk = k;
        break;
      }
    s_k = kk;
  }
  __syncthreads();
  const uint8_t* lens = lens_k + size_t(s_k) * nsym;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  int len[kPass];
  uint32_t rank[kPass];
#pragma unroll
  for (int p = 0; p < kPass; ++p) {
    const int i = p * kCbThreads + t;
    len[p] = i < nsym ? int(lens[i]) : 0;
    rank[p] = 0;
    for (int l = 1; l <= kLmax; ++l) {
      const uint64_t m = __ballot(len[p] == l);
      if (len[p] == l) rank[p] = __popcll(m & below);
      if (lane == 0) wcnt[p][w][l] = __popcll(m);
    }
  }
  __syncthreads();
  if (t <= kLmax) {  // symbols per length, then the first code of each length
    uint32_t n = 0;
    for (int p = 0; p < kPass; ++p)
      for (int ww = 0; ww < kW; ++ww) n += t == 0 ? 0u : wcnt[p][ww][t];
    bl[t] = n;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t code = 0;
    bl[kLmax + 1] = 0;
    for (int l = 1; l <= kLmax; ++l) {
      code = (code + bl[l - 1]) << 1;
      first[l] = code;
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kPass; ++p) {
    const int i = p * kCbThreads + t;
    if (i >= nsym) continue;
    const int l = len[p];
    uint32_t code = 0;
    if (l) {
      uint32_t r = rank[p];
      for (int q = 0; q < p; ++q)
        for (int ww = 0; ww < kW; ++ww) r += wcnt[q][ww][l];
      for (int ww = 0; ww < w; ++ww) r += wcnt[p][ww][l];
      code = first[l] + r;
    }
    lens_out[i] = uint8_t(l);
    codes_out[i] = uint16_t(code);
  }
}

__global__ __launch_bounds__(kCbThreads) void k_cb_final(const uint8_t* lens_k, const int* maxlen_k,
                                                         int nsym, uint8_t* lens_out,
                                                         uint16_t* codes_out) {
  cb_final_body(lens_k, maxlen_k, nsym, lens_out, codes_out);
}

// Scratch split: per-scale lengths, then per-scale longest code.
__host__ __device__ inline uint8_t* cb_lens_k(void* scratch) {
  return static_cast<uint8_t*>(scratch);
}
__host__ __device__ inline int* cb_maxlen_k(void* scratch, int nsym) {
  return reinterpret_cast<int*>(static_cast<uint8_t*>(scratch) +
                                ((size_t(kCbScales) * nsym + 15) & ~size_t(15)));
}

// Batched code books, one job per blockIdx.y, scale k0 + blockIdx.x. The
// scales run in launches of growing k: 0, then 1..7, then groups of eight;
// a launch skips a job when one of its scales below k0 already fits. A field
// pays for one tree unless it needs the length limit, and then for the
// groups up to the first scale that fits. (Scales a launch skips keep stale
// longest-code entries; the final pick never reaches them, as it stops at the
// first scale that fits, and every scale before that one was built.)
constexpr int kCbGroup = 8;
__global__ __launch_bounds__(kCbThreads) void kb_cb_build(const CompressArgs* J, int k0) {
  const CompressArgs& a = J[blockIdx.y];
  const int nsym = alphabet(a.geo);
  int* mk = cb_maxlen_k(a.cb_scratch, nsym);
  bool fits = false;
  for (int k = 0; k < k0; ++k) fits = fits || mk[k] <= kLmax;
  if (fits) return;
  cb_build_body(a.hist, nsym, cb_lens_k(a.cb_scratch), mk, k0 + int(blockIdx.x));
}

__global__ __launch_bounds__(kCbThreads) void kb_cb_final(const CompressArgs* J) {
  const CompressArgs& a = J[blockIdx.x];
  const int nsym = alphabet(a.geo);
  cb_final_body(cb_lens_k(a.cb_scratch), cb_maxlen_k(a.cb_scratch, nsym), nsym, a.lens, a.codes);
}

}  // namespace

size_t codebook_scratch_bytes(int nsym) { return size_t(kCbScales) * (size_t(nsym) + 4) + 64; }

void launch_codebook(const unsigned long long* hist, int nsym, uint8_t* lens, uint16_t* codes,
                     void* scratch, hipStream_t st) {
  uint8_t* lens_k = cb_lens_k(scratch);
  int* maxlen_k = cb_maxlen_k(scratch, nsym);
  prof_begin(st, "cb_build", -1);
  hipLaunchKernelGGL(k_cb_build, dim3(kCbScales), dim3(kCbThreads), 0, st, hist, nsym, lens_k,
                     maxlen_k);
  prof_end(st);
  prof_begin(st, "cb_final", -1);
  hipLaunchKernelGGL(k_cb_final, dim3(1), dim3(kCbThreads), 0, st, lens_k, maxlen_k, nsym, lens,
                     codes);
  prof_end(st);
}

void launch_codebook_batch(const CompressArgs* J, uint32_t njobs, hipStream_t st) {
  prof_begin(st, "b_cb_build", -1);
  for (int k0 = 0; k0 < kCbScales;) {
    const int n = k0 == 0 ? 1 : k0 == 1 ? kCbGroup - 1 : std::min(kCbGroup, kCbScales - k0);
    hipLaunchKernelGGL(kb_cb_build, dim3(n, njobs), dim3(kCbThreads), 0, st, J, k0);
    k0 += n;
  }
  prof_end(st);
  prof_begin(st, "b_cb_final", -1);
  hipLaunchKernelGGL(kb_cb_final, dim3(njobs), dim3(kCbThreads), 0, st, J);
  prof_end(st);
}

}  // namespace stz
