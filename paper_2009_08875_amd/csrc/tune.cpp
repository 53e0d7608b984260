// Launch-shape autotuner (see tune.h).
#include "tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace stp {

namespace {

std::mutex g_mu;
std::map<uint64_t, int> g_choice;
thread_local bool t_no_tuning = false;

bool env_flag(const char* name, bool dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::strcmp(v, "0") != 0;
}

}  // namespace

int tuned(uint64_t key, int candidates, int fallback, hipStream_t stream,
          const std::function<hipError_t(int)>& launch) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_choice.find(key);
    if (it != g_choice.end()) return it->second;
  }
  if (t_no_tuning) return fallback;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return fallback;
  static const bool enabled = env_flag("STP_TUNE", true);
  static const bool log = env_flag("STP_TUNE_LOG", false);
  int best = fallback;
  if (enabled && candidates > 1) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      // Each candidate is timed in kRounds rounds over all candidates, the
      // direction alternating, and keeps its fastest round: a single pass
      // in a fixed order let the GPU's warm-up (clocks, caches) make the
      // later candidates look faster, and a process that tuned on a cold GPU
      // kept launch shapes up to 12 % slower than its best.
      constexpr int kRounds = 3;
      std::vector<float> ms(candidates, -1.0f);
      std::vector<bool> ok(candidates, true);
      for (int r = 0; r < kRounds; ++r) {
        for (int i = 0; i < candidates; ++i) {
          const int c = r % 2 == 0 ? i : candidates - 1 - i;
          if (!ok[c]) continue;
          float t = 0.0f;
          if ((r == 0 && launch(c) != hipSuccess) ||  // warm-up run
              hipEventRecord(e0, stream) != hipSuccess || launch(c) != hipSuccess ||
              launch(c) != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
              hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            ok[c] = false;
            ms[c] = -1.0f;
            continue;
          }
          if (ms[c] < 0.0f || t < ms[c]) ms[c] = t;
        }
      }
      float best_ms = 0.0f;
      for (int c = 0; c < candidates; ++c) {
        if (!ok[c] || ms[c] < 0.0f) continue;
        if (best_ms == 0.0f || ms[c] < best_ms) {
          best_ms = ms[c];
          best = c;
        }
      }
      if (log) {
        std::fprintf(stderr, "[stp tune] key %016llx:", (unsigned long long)key);
        for (int c = 0; c < candidates; ++c) std::fprintf(stderr, " %d:%.3fms", c, ms[c] / 2);
        std::fprintf(stderr, " -> %d\n", best);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGetLastError();
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_choice[key] = best;
  return best;
}

NoTuning::NoTuning() : prev_(t_no_tuning) { t_no_tuning = true; }
NoTuning::~NoTuning() { t_no_tuning = prev_; }

int tuned_choice(uint64_t key, int fallback) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_choice.find(key);
  return it == g_choice.end() ? fallback : it->second;
}

}  // namespace stp
