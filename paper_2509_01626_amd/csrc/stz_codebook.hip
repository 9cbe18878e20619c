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

// Ascending bitonic sort of n (power of two) 64-bit keys in LDS.
__device__ void bitonic_sort(uint64_t* key, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t a = key[lo], b = key[hi];
        if ((a > b) == up) {
          key[lo] = b;
          key[hi] = a;
        }
      }
    }
  }
  __syncthreads();
}

// Code lengths for counts ceil(hist / 2^k), k = blockIdx.x: two queues over the
// leaves sorted by (count, symbol), ties to the leaf queue, merged nodes in
// creation order; depths by pointer jumping.
__device__ inline void cb_build_body(const unsigned long long* hist, int nsym, uint8_t* lens_k,
                                     int* maxlen_k, int k) {
  // nodes: the sorted leaves (padded to a power of two while sorting) and then
  // the m - 1 merged nodes: at most kCbNodes entries
  __shared__ uint64_t W[kCbNodes];
  __shared__ uint16_t par[kCbNodes];
  __shared__ uint16_t dep[kCbNodes];
  __shared__ uint16_t leaf[kCbMax];
  __shared__ int s_m, s_max;
  const int t = threadIdx.x;
  uint8_t* lens = lens_k + size_t(k) * nsym;
  if (t == 0) {
    s_m = 0;
    s_max = 0;
  }
  __syncthreads();
  // the used symbols' keys, compacted (any order: the sort orders them)
  const uint64_t add = (uint64_t(1) << k) - 1;
  for (int i = t; i < nsym; i += blockDim.x) {
    const uint64_t c = uint64_t(hist[i]);
    if (c) W[atomicAdd(&s_m, 1)] = (((c + add) >> k) << kSymBits) | uint64_t(i);
    lens[i] = 0;
  }
  __syncthreads();
  const int m = s_m;
  int np2 = 1;
  while (np2 < m) np2 <<= 1;
  for (int i = m + t; i < np2; i += blockDim.x) W[i] = kInf;
  bitonic_sort(W, np2);
  if (m <= 1) {
    if (m == 1 && t == 0) lens[W[0] & kSymMask] = 1;
    if (t == 0) maxlen_k[k] = m;
    return;
  }
  for (int i = t; i < m; i += blockDim.x) {
    leaf[i] = uint16_t(W[i] & kSymMask);
    W[i] = W[i] >> kSymBits;
  }
  __syncthreads();
  if (t == 0) {
    // Two-queue merge with a two-deep register lookahead on both queues:
    // leaves are W[li..m), merged nodes W[ii..next).
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
  __syncthreads();
  const int nn = 2 * m - 1;
  for (int i = t; i < nn; i += blockDim.x) dep[i] = (i == nn - 1) ? 0 : 1;
  __syncthreads();
  for (int round = 0; (1 << round) < nn; ++round) {
    uint16_t nd[kCbPer], np[kCbPer];
    int j = 0;
    for (int i = t; i < nn; i += blockDim.x, ++j) {
      const int p = par[i];
      nd[j] = dep[i] + dep[p];
      np[j] = par[p];
    }
    __syncthreads();
    j = 0;
    for (int i = t; i < nn; i += blockDim.x, ++j) {
      dep[i] = nd[j];
      par[i] = np[j];
    }
    __syncthreads();
  }
  int mx = 0;
  for (int i = t; i < m; i += blockDim.x) {
    lens[leaf[i]] = uint8_t(dep[i] > 255 ? 255 : dep[i]);
    mx = max(mx, int(dep[i]));
  }
  atomicMax(&s_max, mx);
  __syncthreads();
  if (t == 0) maxlen_k[k] = s_max;
}

__global__ __launch_bounds__(kCbThreads) void k_cb_build(const unsigned long long* hist, int nsym,
                                                         uint8_t* lens_k, int* maxlen_k) {
  cb_build_body(hist, nsym, lens_k, maxlen_k, blockIdx.x);
}

// Pick the first scale whose code fits in kLmax bits; canonical codes.
__device__ inline void cb_final_body(const uint8_t* lens_k, const int* maxlen_k, int nsym,
                                     uint8_t* lens_out, uint16_t* codes_out) {
  __shared__ uint64_t key[kCbMax];
  __shared__ uint32_t bl[kLmax + 2], first[kLmax + 1], start[kLmax + 1];
  __shared__ int s_k, s_n;
  const int t = threadIdx.x;
  if (t == 0) {
    int kk = kCbScales - 1;
    for (int k = 0; k < kCbScales; ++k)
      if (maxlen_k[k] <= kLmax) {
        kk = k;
        break;
      }
    s_k = kk;
  }
  if (t < kLmax + 2) bl[t] = 0;
  if (t == 0) s_n = 0;
  __syncthreads();
  const uint8_t* lens = lens_k + size_t(s_k) * nsym;
  for (int i = t; i < nsym; i += blockDim.x) {
    const int l = lens[i];
    if (l) {
      key[atomicAdd(&s_n, 1)] = (uint64_t(l) << kSymBits) | uint64_t(i);
      atomicAdd(&bl[l], 1u);
    }
    lens_out[i] = uint8_t(l);
    codes_out[i] = 0;
  }
  __syncthreads();
  const int nk = s_n;
  int np2 = 1;
  while (np2 < nk) np2 <<= 1;
  for (int i = nk + t; i < np2; i += blockDim.x) key[i] = kInf;
  bitonic_sort(key, np2);
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
  for (int i = t; i < np2; i += blockDim.x) {
    const uint64_t k = key[i];
    if (k == kInf) continue;
    const int l = int(k >> kSymBits), sy = int(k & kSymMask);
    codes_out[sy] = uint16_t(first[l] + (uint32_t(i) - start[l]));
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
// scales run in three launches: 0; 1..7 unless 0 fits; 8..41 unless one of
// 0..7 fits. A field pays for one tree unless it needs the length limit,
// and then rarely for more than eight. (Scales a launch skips keep stale
// longest-code entries, which the final pick never reaches: it stops at the
// first scale that fits.)
constexpr int kCbFirst = 8;
__global__ __launch_bounds__(kCbThreads) void kb_cb_build(const CompressArgs* J, int k0) {
  const CompressArgs& a = J[blockIdx.y];
  const int nsym = alphabet(a.geo);
  int* mk = cb_maxlen_k(a.cb_scratch, nsym);
  if (k0 > 0) {
    bool fits = mk[0] <= kLmax;
    if (k0 >= kCbFirst)
      for (int k = 1; k < kCbFirst; ++k) fits = fits || mk[k] <= kLmax;
    if (fits) return;
  }
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
  hipLaunchKernelGGL(kb_cb_build, dim3(1, njobs), dim3(kCbThreads), 0, st, J, 0);
  hipLaunchKernelGGL(kb_cb_build, dim3(kCbFirst - 1, njobs), dim3(kCbThreads), 0, st, J, 1);
  hipLaunchKernelGGL(kb_cb_build, dim3(kCbScales - kCbFirst, njobs), dim3(kCbThreads), 0, st, J,
                     kCbFirst);
  prof_end(st);
  prof_begin(st, "b_cb_final", -1);
  hipLaunchKernelGGL(kb_cb_final, dim3(njobs), dim3(kCbThreads), 0, st, J);
  prof_end(st);
}

}  // namespace stz
