// The library's autotuner (gfx950): launch choices that depend on the part and the shape are
// timed with HIP events the first time a shape is seen on a device, on the caller's own
// workspace, and kept in a process-wide cache per device, so that later plans and batches of
// the same shape reuse the choice without timing again.  The choices themselves (the fused
// kernel's column-tile width of a plan and of every class of a batch, the intermediates of a
// float32 plan's physical-basis P^{-1}) are made where they are used; this file holds the
// cache and the timing loop they share.
#include "smr_internal.h"

#include <map>
#include <mutex>
#include <vector>

namespace smr {

namespace {

struct TuneCache {
  std::mutex mu;
  std::map<std::vector<long>, int> v;
  long hits = 0, misses = 0;
};

TuneCache &tune_cache() {
  static TuneCache c;
  return c;
}

std::vector<long> with_device(const std::vector<long> &key) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<long> k;
  k.reserve(key.size() + 1);
  k.push_back(dev);
  k.insert(k.end(), key.begin(), key.end());
  return k;
}

}  // namespace

bool tune_get(const std::vector<long> &key, int *choice) {
  const std::vector<long> k = with_device(key);
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  const auto it = c.v.find(k);
  if (it == c.v.end()) {
    ++c.misses;
    return false;
  }
  ++c.hits;
  *choice = it->second;
  return true;
}

void tune_put(const std::vector<long> &key, int choice) {
  const std::vector<long> k = with_device(key);
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.v[k] = choice;
}

void tune_stats(long *entries, long *hits, long *misses) {
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  *entries = (long)c.v.size();
  *hits = c.hits;
  *misses = c.misses;
}

void tune_clear() {
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.v.clear();
  c.hits = c.misses = 0;
}

hipError_t tune_time(hipStream_t st, int reps, const std::function<hipError_t()> &run, float *ms_per_call) {
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = run();   // warm: first-launch costs stay out of the timing
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (hipEvent_t v : ev)
    if (v) hipEventDestroy(v);
  if (e == hipSuccess) *ms_per_call = ms / (float)(reps > 0 ? reps : 1);
  return e;
}

}  // namespace smr
