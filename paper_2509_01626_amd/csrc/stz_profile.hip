// Opt-in stage timer: HIP events recorded on the launch stream around every
// kernel of the library, accumulated per (kernel, level) when the calling
// API function has synchronized its stream. Disabled by default; enabled with
// stz_profile_enable(1) or the environment variable STZ_PROFILE=1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "stz.h"
#include "stz_internal.h"

namespace stz {
namespace {

struct Pending {
  std::string key;
  hipEvent_t e0, e1;
};

struct Acc {
  uint64_t launches = 0;
  double ms = 0.0;
};

struct Prof {
  std::mutex mu;
  bool enabled = false;
  bool env_checked = false;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::map<std::string, Acc> acc;
};

Prof& prof() {
  static Prof p;
  return p;
}

hipEvent_t take_event(Prof& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

bool on(Prof& p) {
  if (!p.env_checked) {
    const char* v = std::getenv("STZ_PROFILE");
    if (v && v[0] == '1') p.enabled = true;
    p.env_checked = true;
  }
  return p.enabled;
}

}  // namespace

// Streams being captured into a graph get no timing events.
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void prof_begin(hipStream_t st, const char* name, int level) {
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!on(p) || capturing(st)) return;
  Pending q;
  char buf[64];
  std::snprintf(buf, sizeof(buf), level >= 0 ? "%s@%d" : "%s", name, level);
  q.key = buf;
  q.e0 = take_event(p);
  q.e1 = take_event(p);
  if (!q.e0 || !q.e1) return;
  (void)hipEventRecord(q.e0, st);
  p.pending.push_back(q);
}

void prof_end(hipStream_t st) {
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.enabled || p.pending.empty() || capturing(st)) return;
  (void)hipEventRecord(p.pending.back().e1, st);
}

void prof_flush() {
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  for (Pending& q : p.pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(q.e1) == hipSuccess && hipEventElapsedTime(&ms, q.e0, q.e1) == hipSuccess) {
      Acc& a = p.acc[q.key];
      a.launches++;
      a.ms += ms;
    }
    p.pool.push_back(q.e0);
    p.pool.push_back(q.e1);
  }
  p.pending.clear();
}

}  // namespace stz

extern "C" {

void stz_profile_enable(int enable) {
  stz::Prof& p = stz::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.env_checked = true;
  p.enabled = enable != 0;
}

void stz_profile_reset(void) {
  stz::Prof& p = stz::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.acc.clear();
}

int stz_profile_count(void) {
  stz::Prof& p = stz::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  return int(p.acc.size());
}

int stz_profile_entry(int i, char* name, int name_cap, uint64_t* launches, double* total_ms) {
  stz::Prof& p = stz::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (i < 0 || i >= int(p.acc.size())) return -1;
  auto it = p.acc.begin();
  std::advance(it, i);
  if (name && name_cap > 0) {
    std::strncpy(name, it->first.c_str(), size_t(name_cap - 1));
    name[name_cap - 1] = 0;
  }
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  return 0;
}

}  // extern "C"
