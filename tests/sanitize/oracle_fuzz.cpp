// Sanitizer and byte-flip fuzz driver for the CPU oracle (test infrastructure).
//
// Built by tests/test_oracle_sanitize.py with AddressSanitizer and
// UndefinedBehaviorSanitizer (any finding aborts). It compresses small
// seeded fields of both value types over many shapes, block sizes, levels,
// radii and both codings; decodes each stream fully, at every level and over
// random boxes (checking the error bound); then decodes many corrupted copies
// (single-bit flips, byte overwrites, truncations) through every decoder,
// which must each return OK or a corrupt-stream status and never touch memory
// outside the buffers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/stz_oracle.cpp"

namespace {

uint64_t g_rng = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_rng += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double uniform() { return double(next_u64() >> 11) * (1.0 / 9007199254740992.0); }
uint64_t below(uint64_t n) { return n ? next_u64() % n : 0; }

int failures = 0;
void fail(const char* what, int a, int b) {
  std::fprintf(stderr, "FAIL %s (%d, %d)\n", what, a, b);
  ++failures;
}

template <class T>
std::vector<T> make_field(const uint64_t d[3], double rough) {
  std::vector<T> x(d[0] * d[1] * d[2]);
  const double fz = 0.3 + uniform(), fy = 0.2 + uniform(), fx = 0.1 + uniform();
  for (uint64_t z = 0; z < d[0]; ++z)
    for (uint64_t y = 0; y < d[1]; ++y)
      for (uint64_t i = 0; i < d[2]; ++i)
        x[(z * d[1] + y) * d[2] + i] =
            T(std::sin(fz * z) * std::cos(fy * y) + 0.5 * std::sin(fx * i + 0.7 * z) +
              rough * (uniform() - 0.5));
  return x;
}

template <class T>
int ref_decompress(const void* c, uint64_t n, T* out, uint64_t cap);
template <>
int ref_decompress<float>(const void* c, uint64_t n, float* out, uint64_t cap) {
  return stz_ref_decompress(c, n, out, cap);
}
template <>
int ref_decompress<double>(const void* c, uint64_t n, double* out, uint64_t cap) {
  return stz_ref_decompress_f64(c, n, out, cap);
}
template <class T>
int ref_level(const void* c, uint64_t n, uint32_t l, T* out, uint64_t cap, uint64_t od[3]);
template <>
int ref_level<float>(const void* c, uint64_t n, uint32_t l, float* out, uint64_t cap,
                     uint64_t od[3]) {
  return stz_ref_decompress_level(c, n, l, out, cap, od);
}
template <>
int ref_level<double>(const void* c, uint64_t n, uint32_t l, double* out, uint64_t cap,
                      uint64_t od[3]) {
  return stz_ref_decompress_level_f64(c, n, l, out, cap, od);
}
template <class T>
int ref_region(const void* c, uint64_t n, const uint64_t lo[3], const uint64_t hi[3], uint32_t l,
               T* out, uint64_t cap, uint64_t od[3]);
template <>
int ref_region<float>(const void* c, uint64_t n, const uint64_t lo[3], const uint64_t hi[3],
                      uint32_t l, float* out, uint64_t cap, uint64_t od[3]) {
  return stz_ref_decompress_region(c, n, lo, hi, l, out, cap, od);
}
template <>
int ref_region<double>(const void* c, uint64_t n, const uint64_t lo[3], const uint64_t hi[3],
                       uint32_t l, double* out, uint64_t cap, uint64_t od[3]) {
  return stz_ref_decompress_region_f64(c, n, lo, hi, l, out, cap, od);
}

// Every decoder on one (possibly corrupt) stream; returns the full-decode status.
template <class T>
int decode_all(const std::vector<uint8_t>& s, uint64_t size, const uint64_t d[3], uint32_t L,
               std::vector<T>* full) {
  const uint64_t N = d[0] * d[1] * d[2];
  // exact-size heap buffers: an overrun is an ASan report
  full->assign(N, T(0));
  const int st = ref_decompress<T>(s.data(), size, full->data(), N);
  uint64_t od[3];
  for (uint32_t l = 0; l <= L + 1; ++l) {
    std::vector<T> g(N);
    const int r = ref_level<T>(s.data(), size, l, g.data(), N, od);
    if (r != 0 && r != -4 && r != -1) fail("level status", r, int(l));
  }
  for (int k = 0; k < 3; ++k) {
    uint64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = below(d[a]);
      hi[a] = lo[a] + 1 + below(d[a] - lo[a]);
    }
    const uint32_t l = uint32_t(below(L + 1));
    const uint64_t cap = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    std::vector<T> r(cap);
    const int q = ref_region<T>(s.data(), size, lo, hi, l, r.data(), cap, od);
    if (q != 0 && q != -4) fail("region status", q, int(l));
  }
  return st;
}

template <class T>
int compress_one(const T* x, const uint64_t d[3], double eb, const stz_ref_config* cfg, void* out,
                 uint64_t cap, uint64_t* size);
template <>
int compress_one<float>(const float* x, const uint64_t d[3], double eb, const stz_ref_config* cfg,
                        void* out, uint64_t cap, uint64_t* size) {
  return stz_ref_compress(x, d, 1, eb, cfg, out, cap, size);
}
template <>
int compress_one<double>(const double* x, const uint64_t d[3], double eb,
                         const stz_ref_config* cfg, void* out, uint64_t cap, uint64_t* size) {
  return stz_ref_compress_f64(x, d, 1, eb, cfg, out, cap, size);
}

template <class T>
void run_case(const uint64_t d[3], uint32_t B, uint32_t L, uint32_t R, uint32_t coding, double eb,
              int flips) {
  stz_ref_config cfg = {B, L, R, coding, 0.0};
  const std::vector<T> x = make_field<T>(d, 0.05);
  const uint64_t cap = sizeof(T) == 4 ? stz_ref_compress_bound(d, &cfg)
                                      : stz_ref_compress_bound_f64(d, &cfg);
  std::vector<uint8_t> s(cap);
  uint64_t size = 0;
  int st = compress_one<T>(x.data(), d, eb, &cfg, s.data(), cap, &size);
  if (st != 0) return fail("compress", st, int(B));
  s.resize(size);
  struct stz_ref_info info;
  if (stz_ref_info(s.data(), size, &info) != 0) return fail("info", 0, int(B));
  std::vector<T> full;
  st = decode_all<T>(s, size, d, info.levels, &full);
  if (st != 0) return fail("decode", st, int(B));
  for (uint64_t i = 0; i < x.size(); ++i)
    if (std::fabs(double(full[i]) - double(x[i])) > info.eb_abs) return fail("bound", int(i), 0);
  // corrupted copies: bit flips, byte overwrites, truncations
  for (int k = 0; k < flips; ++k) {
    std::vector<uint8_t> c = s;
    uint64_t n = size;
    const int kind = int(below(3));
    if (kind == 0) {
      c[below(size)] ^= uint8_t(1u << below(8));
    } else if (kind == 1) {
      const uint64_t p = below(size);
      for (uint64_t q = p; q < std::min<uint64_t>(size, p + 1 + below(8)); ++q)
        c[q] = uint8_t(next_u64());
    } else {
      n = below(size);
      c.resize(n);
    }
    std::vector<T> o;
    const int r = decode_all<T>(c, n, d, info.levels, &o);
    if (r != 0 && r != -4) fail("corrupt status", r, k);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int flips = argc > 1 ? std::atoi(argv[1]) : 40;
  struct Case {
    uint64_t d[3];
    uint32_t B, L, R;
  };
  const Case cases[] = {
      {{1, 1, 100}, 8, 0, 0},   {{5, 70, 1}, 4, 2, 0},   {{33, 17, 29}, 8, 0, 0},
      {{17, 18, 19}, 2, 1, 0},  {{30, 30, 30}, 8, 3, 8}, {{23, 31, 47}, 32, 0, 0},
      {{40, 40, 40}, 16, 3, 2}, {{1, 37, 41}, 16, 0, 0}, {{9, 17, 70}, 64, 0, 0},
  };
  int n = 0;
  for (const Case& c : cases)
    for (uint32_t coding = 1; coding <= 2; ++coding) {
      run_case<float>(c.d, c.B, c.L, c.R, coding, 1e-3, flips);
      run_case<double>(c.d, c.B, c.L, c.R, coding, 1e-4, flips / 2);
      ++n;
    }
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("ok: %d cases, %d corrupted streams each\n", n, flips);
  return 0;
}
