// Internal solver context shared by the C-ABI (api.cpp) and the server (server.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stp.h"
#include "kernels.h"

namespace stp {

void set_error(const std::string& msg);

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      stp::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                    \
      return STP_E_DEVICE;                                                                  \
    }                                                                                       \
  } while (0)

#define STP_TRY(expr)                       \
  do {                                      \
    stp_status s_ = (expr);                 \
    if (s_ < 0) return s_;                  \
  } while (0)

// Multigrid work space for up to `chunk_rows` rows of level K.
template <typename T>
struct MgScratch {
  int K = 0;
  int64_t chunk_rows = 0;
  T* xb[kMaxK + 1] = {};   // level l (1..K): smoothed iterate before the coarse correction
  T* xa[kMaxK + 1] = {};   // level l < K: corrected iterate (the coarse correction of level l+1)
  T* b[kMaxK + 1] = {};    // level l < K: restricted residual
};

// Buffers of the operators in type T (one set per precision in use).
template <typename T>
struct Ops {
  bool ready = false;
  T* X = nullptr;      // nodal W p                                  (vec)
  T* y = nullptr;      // y1 | y2                                    (2 vec)
  T* z = nullptr;      // K_x y1 | K_x y2                            (2 vec)
  MgScratch<T> mg;     // two space dimensions
  Mg3Work<T> mg3;      // three space dimensions (mg.chunk_rows rows per level)
};

template <typename T>
struct PcgVecs {
  bool ready = false;
  T *w = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *rhs = nullptr;
};

}  // namespace stp

struct stp_ctx {
  int J = 0, K = 0, nrhs = 1, prec = STP_FP64;
  int dim = 2;             // space dimensions: 2 (unit square) or 3 (unit cube)
  int64_t nx = 0;          // interior nodes per time row, (2^K - 1)^dim
  stp_options opt{};
  stp::SpaceOp op;          // A_x = A_D + c M_x (Section 4); the heat equation by default
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t slab = 0;        // elements per time row
  int64_t rows_per = 0;    // 2^J + 1
  int64_t rows = 0;        // nrhs * rows_per
  int64_t vec = 0;         // rows * slab (one right-hand side set)
  int64_t per_rhs = 0;     // rows_per * slab
  std::vector<void*> allocations;
  size_t bytes = 0;

  // FP64 data and results
  double* g = nullptr;      // forcing, nodal (vec)
  double* u0 = nullptr;     // nrhs slabs
  double* fhat = nullptr;   // W^T f (vec)
  double* u = nullptr;      // W w of the last solve (vec)
  double* w64 = nullptr;    // mixed: FP64 iterate; FP64 mode: alias of pcg64.w
  double* r64 = nullptr;    // mixed: FP64 outer residual
  std::vector<int> has_g;
  bool solved = false;
  std::vector<int> iters;
  std::vector<stp_stats> stats;

  double* sigma = nullptr;  // 2^level per time row (K_X)
  double* rhoref = nullptr; // f-hat^T K_X f-hat per right-hand side (PCG from an initial guess)
  int* syn_order = nullptr;  // synthesis_read_order(J) on the device
  std::vector<stp_ctx*> nest;  // nested iteration: meshes (J - d, K - d), d = 1..nest.size()
  double* partials = nullptr;
  stp::PcgScalars sc{};
  stp::MixedState ms{};      // STP_MIXED only
  double* tolv = nullptr;    // relative tolerance per right-hand side (device)

  // pinned host memory read between units of a solve
  double* h_flags = nullptr;  // pinned copy of dflags
  double* dflags = nullptr;   // per right-hand side: active, its, rho, rho0, target
  double* h_stats = nullptr;  // 2 * nrhs doubles, then 4 * nrhs ints
  double* h_tol = nullptr;    // nrhs
  hipEvent_t ev_flags = nullptr;

  // solve driver state (see drive_begin / drive_next)
  enum Phase { kIdle = 0, kIter, kFinish, kDone };
  struct Drive {
    int phase = kIdle;
    int outer_k = 0;
    bool adjusted = false;  // the last unit ended with an inner PCG start
  } drv;

  // captured PCG iteration per precision
  struct Graph {
    bool warm = false;
    hipGraphExec_t exec = nullptr;
  };
  bool use_graph = false;
  Graph graph64, graph32;

  // stp_apply staging (allocated on first use): compact in/out and slab in/out
  double* apply_buf = nullptr;  // 4 * per_rhs doubles

  stp::Ops<double> ops64;
  stp::Ops<float> ops32;
  stp::PcgVecs<double> pcg64;
  stp::PcgVecs<float> pcg32;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  // kernel timing (stp_profile)
  struct Timed {
    hipEvent_t a, b;
    int kernel;
    double bytes;
  };
  bool profiling = false;
  std::vector<Timed> timed;          // recorded, not yet accumulated
  std::vector<hipEvent_t> ev_pool;   // reusable events
  stp_kernel_stat kstat[STP_KERNEL_COUNT] = {};
};

namespace stp {
// Solve driver (api.cpp): a solve is a chain of device-side units; the host
// picks the next unit from pinned per-right-hand-side flags once the last one
// has completed.  drive_begin enqueues the first unit (tol: nrhs relative
// tolerances in host memory); drive_ready polls without blocking; drive_next
// enqueues the next unit, and sets drv.phase = kDone (statistics in
// ctx->stats, solution in ctx->u) after the last one.
// coarse (may be NULL): a context of mesh (J - 1, K - 1) whose last solve's
// w, carried to this mesh, is the initial guess.
stp_status drive_begin(stp_ctx* c, const double* tol, const stp_ctx* coarse = nullptr);
bool drive_ready(stp_ctx* c);
stp_status drive_wait(stp_ctx* c);
stp_status drive_next(stp_ctx* c);

// K_x (`vcycles` V-cycles from zero for A_x, Section 3.1) on `rows` slabs of
// level K held in b, result in x, using the multigrid work space in mg
// (mg.K == K; mg.chunk_rows >= 1; rows are processed mg.chunk_rows at a time).
// Allocates nothing.
stp_status kspace_apply_slabs(hipStream_t s, MgScratch<double>& mg, const double* b, double* x,
                              int K, int rows, int vcycles);
}  // namespace stp
