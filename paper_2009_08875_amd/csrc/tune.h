// Launch-shape autotuner.
//
// Some kernels can be launched in several shapes that compute bitwise the
// same result (how waves are grouped over the rows of a multigrid level, how
// many time rows a stencil workgroup walks).  The first time a launch site
// meets a problem shape, tuned() runs every candidate on the launch's real
// arguments (the kernels are pure: they read their inputs and overwrite their
// outputs, so repeating them is harmless), times each with HIP events on the
// launch stream in three rounds over all candidates (alternating direction;
// a candidate's time is its fastest round), and remembers the fastest for that
// shape for the rest of the process.  While the stream is being captured into a graph nothing can be
// timed: an unknown shape then gets the fallback candidate, not remembered.
// STP_TUNE=0 in the environment disables tuning (always the fallback);
// STP_TUNE_LOG=1 prints each decision to stderr.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

namespace stp {

int tuned(uint64_t key, int candidates, int fallback, hipStream_t stream,
          const std::function<hipError_t(int)>& launch);

// The choice remembered for key, or fallback; never runs anything (for
// launches that update their output in place and so cannot be repeated).
int tuned_choice(uint64_t key, int fallback);

// While an object of this type lives on a thread, tuned() on that thread
// behaves like tuned_choice(): no trial launches, events or waits (for entry
// points that must only enqueue work).
struct NoTuning {
  NoTuning();
  ~NoTuning();
  NoTuning(const NoTuning&) = delete;
  NoTuning& operator=(const NoTuning&) = delete;

 private:
  bool prev_;
};

inline uint64_t tune_key(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  return (a << 56) ^ (b << 40) ^ (c << 24) ^ d;
}

}  // namespace stp
