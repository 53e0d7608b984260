// C-ABI of the solver and its host-side driver: memory planning, the
// multigrid cycle schedule, the operators S, S-hat, K_X and f as launch
// sequences, and PCG (FP64, and FP32-inner / FP64-outer refinement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "solver.h"

using namespace stp;

namespace stp {

namespace {
thread_local std::string g_last_error;
constexpr double kDefaultAlpha = 0.3;   // Section 5.1
constexpr int kMaxGridY = 65535;
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace stp

namespace {

// Default relative reduction of an FP32 inner solve.  The rounding of the FP32
// K_X grows with the mesh (A's cancellation amplifies it: about 20x at h = 2^-6,
// 130x at h = 2^-9), so on fine meshes an inner solve stops earlier and the
// FP64 refinement does the rest; on coarser meshes a deeper inner solve saves
// refinement steps.  Measured optima: 1e-4 at K = 7, 3e-3 at K = 9.
double default_inner_tol(int K) { return K <= 7 ? 1e-4 : (K == 8 ? 1e-3 : 3e-3); }

stp_options resolve(const stp_options* o) {
  stp_options r{};
  if (o) r = *o;
  if (r.alpha <= 0.0) r.alpha = kDefaultAlpha;
  if (r.vcycles <= 0) r.vcycles = 2;
  if (r.sweeps <= 0) r.sweeps = 3;
  if (r.maxit <= 0) r.maxit = 200;
  // inner_tol <= 0: chosen from the mesh in stp_create (default_inner_tol)
  if (r.max_outer <= 0) r.max_outer = 20;
  if (r.graph > 0) r.graph = 1;
  if (r.nested < 0) r.nested = 0;
  r.lookahead = r.lookahead < 0 ? -1 : 0;
  if (r.diffusion[0] == 0.0 && r.diffusion[1] == 0.0 && r.diffusion[2] == 0.0) {
    r.diffusion[0] = 1.0;
    r.diffusion[1] = 1.0;
  }
  return r;
}

// ------------------------------------------------------------ memory plan
//
// Every device allocation of a context goes through Arena so that the same
// code computes the footprint (dry run) and allocates.  New memory is zeroed
// on the context's stream: a plain hipMemset runs on the null stream, which
// a non-blocking stream does not wait for, so the context's first kernels
// could otherwise run before the zeroing.
struct Arena {
  bool dry = true;
  size_t bytes = 0;
  std::vector<void*>* list = nullptr;
  hipStream_t stream = nullptr;
  template <typename T>
  stp_status get(T** p, int64_t count) {
    size_t b = ((size_t)count * sizeof(T) + 511) & ~(size_t)511;
    bytes += b;
    if (dry) {
      *p = nullptr;
      return STP_OK;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
      return STP_E_OUT_OF_MEMORY;
    }
    list->push_back(q);
    e = hipMemsetAsync(q, 0, b, stream);
    if (e != hipSuccess) {
      set_error(std::string("hipMemsetAsync: ") + hipGetErrorString(e));
      return STP_E_DEVICE;
    }
    *p = (T*)q;
    return STP_OK;
  }
};

template <typename T>
stp_status plan_mg3(Arena& ar, MgScratch<T>& mg, Mg3Work<T>& w, int K, int64_t chunk_rows) {
  mg.K = K;
  mg.chunk_rows = chunk_rows;
  STP_TRY(ar.get(&w.x[K], chunk_rows * slab3_elems(K)));
  for (int l = 2; l <= K; ++l) STP_TRY(ar.get(&w.r[l], chunk_rows * slab3_elems(l)));
  for (int l = 1; l < K; ++l) {
    STP_TRY(ar.get(&w.x[l], chunk_rows * slab3_elems(l)));
    STP_TRY(ar.get(&w.b[l], chunk_rows * slab3_elems(l)));
  }
  return STP_OK;
}

template <typename T>
stp_status plan_mg(Arena& ar, MgScratch<T>& mg, int K, int64_t chunk_rows) {
  mg.K = K;
  mg.chunk_rows = chunk_rows;
  STP_TRY(ar.get(&mg.xb[K], chunk_rows * slab_elems(K)));
  for (int l = 1; l < K; ++l) {
    STP_TRY(ar.get(&mg.xa[l], chunk_rows * slab_elems(l)));
    STP_TRY(ar.get(&mg.xb[l], chunk_rows * slab_elems(l)));
    STP_TRY(ar.get(&mg.b[l], chunk_rows * slab_elems(l)));
  }
  return STP_OK;
}

template <typename T>
stp_status plan_ops(Arena& ar, Ops<T>& o, int K, int64_t rows, int64_t vec, int dim) {
  STP_TRY(ar.get(&o.X, vec));
  STP_TRY(ar.get(&o.y, 2 * vec));
  STP_TRY(ar.get(&o.z, 2 * vec));
  // S and f apply K_x to two arrays at once (2 * rows rows in one launch)
  if (dim == 3)
    STP_TRY(plan_mg3(ar, o.mg, o.mg3, K, std::min<int64_t>(2 * rows, kMaxGridY)));
  else
    STP_TRY(plan_mg(ar, o.mg, K, std::min<int64_t>(2 * rows, kMaxGridY)));
  o.ready = !ar.dry;
  return STP_OK;
}

template <typename T>
stp_status plan_pcg(Arena& ar, PcgVecs<T>& v, int64_t vec, bool with_rhs) {
  STP_TRY(ar.get(&v.w, vec));
  STP_TRY(ar.get(&v.r, vec));
  STP_TRY(ar.get(&v.z, vec));
  STP_TRY(ar.get(&v.p, vec));
  STP_TRY(ar.get(&v.q, vec));
  if (with_rhs) STP_TRY(ar.get(&v.rhs, vec));
  v.ready = !ar.dry;
  return STP_OK;
}

stp_status plan_context(Arena& ar, stp_ctx* c) {
  const int64_t vec = c->vec;
  STP_TRY(ar.get(&c->g, vec));
  STP_TRY(ar.get(&c->u0, (int64_t)c->nrhs * c->slab));
  STP_TRY(ar.get(&c->fhat, vec));
  STP_TRY(ar.get(&c->u, vec));
  STP_TRY(ar.get(&c->sigma, c->rows));
  STP_TRY(ar.get(&c->rhoref, c->nrhs));
  STP_TRY(ar.get(&c->syn_order, (int64_t)c->rows_per));
  STP_TRY(ar.get(&c->partials, (int64_t)c->nrhs * std::max(1024, analysis_dot_blocks(c->slab))));
  STP_TRY(ar.get(&c->tolv, c->nrhs));
  STP_TRY(ar.get(&c->sc.rho, c->nrhs));
  STP_TRY(ar.get(&c->sc.rho0, c->nrhs));
  STP_TRY(ar.get(&c->sc.pq, c->nrhs));
  STP_TRY(ar.get(&c->sc.rhonew, c->nrhs));
  STP_TRY(ar.get(&c->sc.gamma, c->nrhs));
  STP_TRY(ar.get(&c->sc.beta, c->nrhs));
  STP_TRY(ar.get(&c->sc.target, c->nrhs));
  STP_TRY(ar.get(&c->sc.active, c->nrhs));
  STP_TRY(ar.get(&c->sc.its, c->nrhs));
  STP_TRY(ar.get(&c->sc.status, c->nrhs));
  STP_TRY(ar.get(&c->dflags, 5 * (int64_t)c->nrhs));
  STP_TRY(plan_ops(ar, c->ops64, c->K, c->rows, vec, c->dim));
  if (c->prec == STP_FP64) {
    STP_TRY(plan_pcg(ar, c->pcg64, vec, false));
  } else {
    STP_TRY(ar.get(&c->ms.rho0_first, c->nrhs));
    STP_TRY(ar.get(&c->ms.rel, c->nrhs));
    STP_TRY(ar.get(&c->ms.done, c->nrhs));
    STP_TRY(ar.get(&c->ms.status, c->nrhs));
    STP_TRY(ar.get(&c->ms.outer, c->nrhs));
    STP_TRY(ar.get(&c->ms.inner_its, c->nrhs));
    STP_TRY(ar.get(&c->w64, vec));
    STP_TRY(ar.get(&c->r64, vec));
    STP_TRY(plan_ops(ar, c->ops32, c->K, c->rows, vec, c->dim));
    STP_TRY(plan_pcg(ar, c->pcg32, vec, true));
  }
  return STP_OK;
}

void free_all(stp_ctx* c) {
  for (stp_ctx* n : c->nest) stp_destroy(n);
  c->nest.clear();
  for (auto& t : c->timed) {
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timed.clear();
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  for (void* p : c->allocations) (void)hipFree(p);
  c->allocations.clear();
  if (c->graph64.exec) (void)hipGraphExecDestroy(c->graph64.exec);
  if (c->graph32.exec) (void)hipGraphExecDestroy(c->graph32.exec);
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  if (c->h_stats) (void)hipHostFree(c->h_stats);
  if (c->h_tol) (void)hipHostFree(c->h_tol);
  if (c->ev_flags) (void)hipEventDestroy(c->ev_flags);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// ------------------------------------------------------------ operators

template <typename T>
Ops<T>& ops_of(stp_ctx* c);
template <>
Ops<double>& ops_of<double>(stp_ctx* c) { return c->ops64; }
template <>
Ops<float>& ops_of<float>(stp_ctx* c) { return c->ops32; }

// Compact FP64 rows of nx values <-> slabs, in the context's dimension.
template <typename T>
hipError_t pack_rows(const stp_ctx* c, const double* src, T* dst, int rows) {
  return c->dim == 3 ? pack3<T>(c->stream, src, dst, c->K, rows)
                     : pack<T>(c->stream, src, dst, c->K, rows);
}
template <typename T>
hipError_t unpack_rows(const stp_ctx* c, const T* src, double* dst, int rows) {
  return c->dim == 3 ? unpack3<T>(c->stream, src, dst, c->K, rows)
                     : unpack<T>(c->stream, src, dst, c->K, rows);
}

// ------------------------------------------------------------ kernel timing

stp_status take_event(stp_ctx* c, hipEvent_t* e) {
  if (!c->ev_pool.empty()) {
    *e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return STP_OK;
  }
  HIP_TRY(hipEventCreate(e));
  return STP_OK;
}

stp_status flush_timing(stp_ctx* c) {
  for (auto& t : c->timed) {
    HIP_TRY(hipEventSynchronize(t.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    stp_kernel_stat& k = c->kstat[t.kernel];
    k.launches += 1;
    k.total_ms += ms;
    k.alg_bytes += t.bytes;
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timed.clear();
  return STP_OK;
}

// Launch `f` (returning hipError_t); when profiling, bracket it with events.
template <typename F>
stp_status timed_launch(stp_ctx* c, int kernel, double bytes, F f) {
  if (!c->profiling) {
    HIP_TRY(f());
    return STP_OK;
  }
  if (c->timed.size() >= 4096) STP_TRY(flush_timing(c));
  stp_ctx::Timed t{};
  STP_TRY(take_event(c, &t.a));
  STP_TRY(take_event(c, &t.b));
  t.kernel = kernel;
  t.bytes = bytes;
  HIP_TRY(hipEventRecord(t.a, c->stream));
  HIP_TRY(f());
  HIP_TRY(hipEventRecord(t.b, c->stream));
  c->timed.push_back(t);
  return STP_OK;
}

// x = K[a, sigma] b: `vcycles` V-cycles from zero on `rows` slabs of level K;
// with write_Ax, x receives A_x K[a, sigma] b instead.
template <typename T>
stp_status mg_apply(stp_ctx* c, MgScratch<T>& mg, const T* b, T* x, int64_t rows, double a,
                    const double* sigma, bool write_Ax = false) {
  const int K = c->K;
  if (c->dim == 3) {
    // three dimensions (space3d.hip): the chunk's rows through mg3_apply
    const Ops<T>& o = ops_of<T>(c);
    for (int64_t r0 = 0; r0 < rows; r0 += mg.chunk_rows) {
      const int nr = (int)std::min<int64_t>(mg.chunk_rows, rows - r0);
      HIP_TRY(mg3_apply<T>(c->stream, o.mg3, b + r0 * c->slab, x + r0 * c->slab, K, nr, a,
                           sigma ? sigma + r0 : nullptr, c->opt.vcycles, write_Ax));
    }
    return STP_OK;
  }
  const int64_t slab = slab_elems(K);
  for (int64_t r0 = 0; r0 < rows; r0 += mg.chunk_rows) {
    const int nr = (int)std::min<int64_t>(mg.chunk_rows, rows - r0);
    const T* bb = b + r0 * slab;
    T* xx = x + r0 * slab;
    const double* sg = sigma ? sigma + r0 : nullptr;
    constexpr int CL = coarse_levels<T>();
    if (K <= CL) {
      // every cycle in one workgroup per row (all levels in LDS): b read
      // once, x written once
      HIP_TRY(mg_coarse_cycle<T>(c->stream, nullptr, bb, xx, K, nr, a, sg, write_Ax, c->op,
                                 c->opt.vcycles));
      continue;
    }
    // algorithmic bytes of the fine-level kernels: every input element read
    // once, every output element written once (interior nodes only)
    const double nodes = (double)nr * grid_n(K) * grid_n(K);
    const double cnodes = (double)nr * grid_n(K - 1) * grid_n(K - 1);
    for (int cyc = 0; cyc < c->opt.vcycles; ++cyc) {
      const bool last = cyc == c->opt.vcycles - 1;
      // a fused A x output replaces x, so the next cycle could not start from it
      const T* xin = cyc == 0 ? nullptr : xx;
      const double pre_bytes = sizeof(T) * ((xin ? 3.0 : 2.0) * nodes + cnodes);
      STP_TRY(timed_launch(c, STP_KERNEL_MG_PRE, pre_bytes, [&] {
        return mg_pre_stream<T>(c->stream, xin, bb, mg.xb[K], mg.b[K - 1], K, nr, a, sg, c->op);
      }));
      for (int l = K - 1; l > CL; --l)
        HIP_TRY(mg_pre_stream<T>(c->stream, nullptr, mg.b[l], mg.xb[l], mg.b[l - 1], l, nr, a, sg,
                                 c->op));
      // levels CL .. 1 in one launch, from zero
      HIP_TRY(mg_coarse_cycle<T>(c->stream, nullptr, mg.b[CL], mg.xa[CL], CL, nr, a, sg, false,
                                 c->op));
      for (int l = CL + 1; l <= K - 1; ++l)
        HIP_TRY(mg_post_stream<T>(c->stream, mg.xb[l], mg.b[l], mg.xa[l - 1], mg.xa[l], l, nr, a, sg,
                                  false, c->op));
      const double post_bytes = sizeof(T) * (3.0 * nodes + cnodes);
      STP_TRY(timed_launch(c, STP_KERNEL_MG_POST, post_bytes, [&] {
        return mg_post_stream<T>(c->stream, mg.xb[K], bb, mg.xa[K - 1], xx, K, nr, a, sg,
                                 write_Ax && last, c->op);
      }));
    }
  }
  return STP_OK;
}

// Algorithmic bytes of a pass that moves `words` values of type T per
// interior node of `rows` time rows.
template <typename T>
double row_bytes(const stp_ctx* c, int64_t rows, double words) {
  return words * sizeof(T) * (double)rows * (double)c->nx;
}

// out = S X (Lemma 4.2) for `nrhs` right-hand sides starting at X.
template <typename T>
stp_status S_apply(stp_ctx* c, Ops<T>& o, const T* X, T* out, int nrhs) {
  const int64_t v = (int64_t)nrhs * c->per_rhs;
  const int64_t rows = (int64_t)nrhs * c->rows_per;
  T* y1 = o.y;
  T* y2 = o.y + v;
  T* z1 = o.z;
  T* z2 = o.z + v;
  // X in; y1, y2 out
  STP_TRY(timed_launch(c, STP_KERNEL_TIME_STENCIL, row_bytes<T>(c, rows, 3.0), [&] {
    if (c->dim == 3) return time_stencil_pair3<T>(c->stream, X, y1, y2, c->J, c->K, nrhs);
    return time_stencil_pair<T>(c->stream, X, y1, y2, c->J, c->K, nrhs, c->op);
  }));
  // y1 | y2 and z1 | z2 are contiguous: one K_x application over both
  STP_TRY(mg_apply<T>(c, o.mg, y1, z1, 2 * rows, 1.0, nullptr));
  // z1, z2 in; S X out (row 0's M X_0 term is one row in 2^J + 1)
  STP_TRY(timed_launch(c, STP_KERNEL_COMBINE, row_bytes<T>(c, rows, 3.0), [&] {
    if (c->dim == 3) return combine3<T>(c->stream, z1, z2, X, c->per_rhs, out, c->J, c->K, nrhs);
    return combine<T>(c->stream, z1, z2, X, c->per_rhs, out, c->J, c->K, nrhs, c->op);
  }));
  return STP_OK;
}

// out = S-hat p = W^T S W p (eq. (11)).
template <typename T>
stp_status Shat_apply(stp_ctx* c, Ops<T>& o, const T* p, T* out, int nrhs) {
  HIP_TRY(synthesis<T>(c->stream, p, o.X, c->J, c->slab, nrhs, c->syn_order));
  STP_TRY(S_apply<T>(c, o, o.X, out, nrhs));
  HIP_TRY(wavelet<T>(c->stream, out, c->J, c->slab, nrhs, false, c->syn_order));
  return STP_OK;
}

// The S-hat product of a PCG iteration: p = z + beta p (the direction update
// of the previous iteration, fused into the synthesis), q = S-hat p, and
// pq = p^T q (fused into the analysis).
template <typename T>
stp_status Shat_iteration(stp_ctx* c, Ops<T>& o, PcgVecs<T>& v) {
  // z, p in; p, X out
  STP_TRY(timed_launch(c, STP_KERNEL_SYN_UPDATE, row_bytes<T>(c, c->rows, 4.0), [&] {
    return synthesis_update<T>(c->stream, v.p, v.z, c->sc.beta, o.X, c->J, c->slab, c->nrhs,
                               c->syn_order);
  }));
  STP_TRY(S_apply<T>(c, o, o.X, v.q, c->nrhs));
  // q (= S X), X in; q = W^T S X out, p^T q = X^T S X (X = W p)
  STP_TRY(timed_launch(c, STP_KERNEL_ANA_DOT, row_bytes<T>(c, c->rows, 3.0), [&] {
    return analysis_dot<T>(c->stream, v.q, o.X, c->partials, c->sc.pq, c->J, c->slab, c->nrhs);
  }));
  return STP_OK;
}

// z = K_X r: row i gets K_l A K_l r_i, K_l = MG for (alpha A + 2^l M) (Theorem 3.1).
// The first application writes A K_l r directly (fused into its last smoothing).
template <typename T>
stp_status KX_apply(stp_ctx* c, Ops<T>& o, const T* r, T* z, int nrhs) {
  const int64_t rows = (int64_t)nrhs * c->rows_per;
  T* t = o.y;
  STP_TRY(mg_apply<T>(c, o.mg, r, t, rows, c->opt.alpha, c->sigma, true));
  STP_TRY(mg_apply<T>(c, o.mg, t, z, rows, c->opt.alpha, c->sigma));
  return STP_OK;
}

// f of Lemma 4.1 (FP64): f_i = M K_x G1_i + A K_x G0_i + [i = 0] M u0.
stp_status rhs_apply(stp_ctx* c, double* f) {
  Ops<double>& o = c->ops64;
  const int64_t v = c->vec;
  bool any_g = false;
  for (int b = 0; b < c->nrhs; ++b) any_g = any_g || c->has_g[b];
  double* z1 = o.z;
  double* z2 = o.z + v;
  if (any_g) {
    double* G1 = o.y;
    double* G0 = o.y + v;
    if (c->dim == 3)
      HIP_TRY(rhs_stencil_pair3<double>(c->stream, c->g, G1, G0, c->J, c->K, c->nrhs));
    else
      HIP_TRY(rhs_stencil_pair<double>(c->stream, c->g, G1, G0, c->J, c->K, c->nrhs));
    STP_TRY(mg_apply<double>(c, o.mg, G1, z1, 2 * c->rows, 1.0, nullptr));  // G1 | G0 -> z1 | z2
  } else {
    HIP_TRY(hipMemsetAsync(z1, 0, sizeof(double) * 2 * v, c->stream));
  }
  if (c->dim == 3)
    HIP_TRY(combine3<double>(c->stream, z1, z2, c->u0, c->slab, f, c->J, c->K, c->nrhs));
  else
    HIP_TRY(combine<double>(c->stream, z1, z2, c->u0, c->slab, f, c->J, c->K, c->nrhs, c->op));
  return STP_OK;
}

// ------------------------------------------------------------ PCG
//
// A solve is a sequence of units of device work.  After each unit the host
// reads the per-right-hand-side flags (active, done) through pinned memory
// and picks the next unit; every decision that needs a PCG scalar is taken on
// the device (pcg_start, pcg_gamma, pcg_beta, mixed_adjust), so a unit never
// waits for the host.  stp_solve runs the units back to back; the server
// interleaves the units of many contexts.

// PCG start on S-hat w = rhs, w_0 = 0 (Section 3.4): r = rhs, z = K_X r,
// rho0 = r^T z, p = z.
template <typename T>
stp_status pcg_init(stp_ctx* c, PcgVecs<T>& v, const T* rhs, const double* tol) {
  Ops<T>& o = ops_of<T>(c);
  HIP_TRY(hipMemsetAsync(v.w, 0, sizeof(T) * c->vec, c->stream));
  HIP_TRY(copy<T>(c->stream, rhs, v.r, c->vec));
  STP_TRY(KX_apply<T>(c, o, v.r, v.z, c->nrhs));
  HIP_TRY(dot<T>(c->stream, v.r, v.z, c->per_rhs, c->nrhs, c->partials, c->sc.rhonew));
  HIP_TRY(pcg_start(c->stream, c->sc, c->nrhs, tol));
  HIP_TRY(copy<T>(c->stream, v.z, v.p, c->vec));
  return STP_OK;
}

// PCG start from the initial guess w = the coarse context's solution carried
// to this mesh (nested iteration, Section 4.2): r = f-hat - S-hat w,
// z = K_X r, rho = r^T z, p = z; the stopping test and rho0 refer to
// f-hat^T K_X f-hat, the first residual's quantity from w = 0.  FP64.
stp_status pcg_init_from(stp_ctx* c, const stp_ctx* coarse, const double* tol) {
  PcgVecs<double>& v = c->pcg64;
  Ops<double>& o = c->ops64;
  HIP_TRY(prolong_w(c->stream, coarse->pcg64.w, v.w, c->J, c->K, c->nrhs));
  STP_TRY(KX_apply<double>(c, o, c->fhat, v.z, c->nrhs));
  HIP_TRY(dot<double>(c->stream, c->fhat, v.z, c->per_rhs, c->nrhs, c->partials, c->rhoref));
  STP_TRY(Shat_apply<double>(c, o, v.w, v.q, c->nrhs));
  HIP_TRY(residual64(c->stream, c->fhat, v.q, v.r, c->vec));
  STP_TRY(KX_apply<double>(c, o, v.r, v.z, c->nrhs));
  HIP_TRY(dot<double>(c->stream, v.r, v.z, c->per_rhs, c->nrhs, c->partials, c->sc.rhonew));
  HIP_TRY(pcg_start(c->stream, c->sc, c->nrhs, tol, c->rhoref));
  HIP_TRY(copy<double>(c->stream, v.z, v.p, c->vec));
  return STP_OK;
}

// One PCG iteration for every right-hand side; inactive ones get gamma = 0
// and keep w and r.  The direction update p = z + beta p of the previous
// iteration happens at the start of this one (beta = 0 after the start, where
// p = z already).  No host synchronisation, no memset: graph-capturable.
template <typename T>
stp_status pcg_iteration(stp_ctx* c, PcgVecs<T>& v) {
  Ops<T>& o = ops_of<T>(c);
  const int nrhs = c->nrhs;
  const int64_t n = c->per_rhs;
  STP_TRY(Shat_iteration<T>(c, o, v));
  HIP_TRY(pcg_gamma(c->stream, c->sc, nrhs));
  // w, r, p, q in; w, r out
  STP_TRY(timed_launch(c, STP_KERNEL_UPDATE_WR, row_bytes<T>(c, c->rows, 6.0), [&] {
    return update_wr<T>(c->stream, v.w, v.r, v.p, v.q, c->sc.gamma, n, nrhs);
  }));
  STP_TRY(KX_apply<T>(c, o, v.r, v.z, nrhs));
  // r, z in
  STP_TRY(timed_launch(c, STP_KERNEL_DOT, row_bytes<T>(c, c->rows, 2.0), [&] {
    return dot<T>(c->stream, v.r, v.z, n, nrhs, c->partials, c->sc.rhonew);
  }));
  HIP_TRY(pcg_beta(c->stream, c->sc, nrhs, c->opt.maxit));
  return STP_OK;
}

template <typename T>
stp_ctx::Graph& graph_of(stp_ctx* c);
template <>
stp_ctx::Graph& graph_of<double>(stp_ctx* c) { return c->graph64; }
template <>
stp_ctx::Graph& graph_of<float>(stp_ctx* c) { return c->graph32; }

// One iteration, replayed from a captured HIP graph once one exists.  The
// first iteration of a context runs eagerly (it also initialises the
// kernels' launch-shape caches); the second is captured.  Profiling needs
// per-launch events and always runs eagerly.
template <typename T>
stp_status iterate(stp_ctx* c, PcgVecs<T>& v) {
  stp_ctx::Graph& g = graph_of<T>(c);
  if (!c->use_graph || c->profiling || c->stream == nullptr) return pcg_iteration<T>(c, v);
  if (!g.exec) {
    if (!g.warm) {
      g.warm = true;
      return pcg_iteration<T>(c, v);
    }
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const stp_status st = pcg_iteration<T>(c, v);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (st < 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    HIP_TRY(e);
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(ei);
  }
  HIP_TRY(hipGraphLaunch(g.exec, c->stream));
  return STP_OK;
}

// Copy the convergence state to pinned host memory and mark the end of the
// unit.
stp_status post_flags(stp_ctx* c) {
  const int nr = c->nrhs;
  HIP_TRY(pack_flags(c->stream, c->sc, nr, c->dflags));
  HIP_TRY(hipMemcpyAsync(c->h_flags, c->dflags, sizeof(double) * 5 * nr, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipEventRecord(c->ev_flags, c->stream));
  return STP_OK;
}

bool any_active(const stp_ctx* c) {
  for (int b = 0; b < c->nrhs; ++b)
    if (c->h_flags[5 * b] != 0.0) return true;
  return false;
}

// How many PCG iterations to enqueue before the host reads the flags again.
// Per active right-hand side: with target 0 (run to the limit) all that are
// left; else half of log(sqrt(rho) / target) / -log(q) with q the mean
// reduction of sqrt(rho) per iteration so far, and 1 before the first
// iteration.  The batch is the largest over the active right-hand sides: an
// iteration enqueued after every one has stopped is wasted time, never a
// change of results (inactive right-hand sides get gamma = 0).
int iteration_batch(const stp_ctx* c) {
  if (c->opt.lookahead < 0) return 1;
  const double* h = c->h_flags;
  const int maxit = c->opt.maxit;
  int batch = 1;
  for (int b = 0; b < c->nrhs; ++b) {
    if (h[5 * b] == 0.0) continue;
    const int its = (int)h[5 * b + 1];
    const double rho = h[5 * b + 2], rho0 = h[5 * b + 3], target = h[5 * b + 4];
    const int left = maxit - its;
    int m = 1;
    if (target <= 0.0) {
      m = left;
    } else if (its > 0 && rho > 0.0 && rho0 > 0.0) {
      const double d = std::sqrt(rho) / target;
      const double q = std::pow(rho / rho0, 0.5 / its);
      if (q > 0.0 && q < 1.0 && d > 1.0) {
        const double est = 0.5 * std::log(d) / -std::log(q);
        m = est >= (double)left ? left : std::max(1, (int)est);
      }
    }
    batch = std::max(batch, std::min(m, left));
  }
  return std::max(batch, 1);
}

// Last unit: u = W w (out of place), and the statistics to pinned host memory.
stp_status finish_unit(stp_ctx* c) {
  const int nr = c->nrhs;
  double* hs = c->h_stats;
  int* hi = (int*)(c->h_stats + 2 * nr);
  if (c->prec == STP_FP64) {
    HIP_TRY(synthesis<double>(c->stream, c->pcg64.w, c->u, c->J, c->slab, nr, c->syn_order));
    HIP_TRY(hipMemcpyAsync(hs, c->sc.rho, sizeof(double) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hs + nr, c->sc.rho0, sizeof(double) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi, c->sc.its, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi + nr, c->sc.status, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
  } else {
    HIP_TRY(synthesis<double>(c->stream, c->w64, c->u, c->J, c->slab, nr, c->syn_order));
    HIP_TRY(hipMemcpyAsync(hs, c->ms.rel, sizeof(double) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi, c->ms.inner_its, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi + nr, c->ms.status, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi + 2 * nr, c->ms.outer, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hi + 3 * nr, c->ms.done, sizeof(int) * nr, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  HIP_TRY(hipEventRecord(c->ev_flags, c->stream));
  c->drv.phase = stp_ctx::kFinish;
  return STP_OK;
}

// Statistics of a finished solve from the pinned copies.
void collect_stats(stp_ctx* c) {
  const int nr = c->nrhs;
  const double* hs = c->h_stats;
  const int* hi = (const int*)(c->h_stats + 2 * nr);
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) ms = 0.0f;
  for (int b = 0; b < nr; ++b) {
    stp_stats& s = c->stats[b];
    const double tol = c->h_tol[b];
    if (c->prec == STP_FP64) {
      const double rho = hs[b], rho0 = hs[nr + b];
      const int st = hi[nr + b];
      s.iterations = hi[b];
      s.outer_iterations = 0;
      s.rel_residual = rho0 > 0 ? std::sqrt(std::max(rho, 0.0) / rho0) : 0.0;
      if (st == -3)
        s.status = STP_E_BREAKDOWN;
      else if (st == 1 || (tol > 0 && s.rel_residual <= tol) || rho0 == 0.0 || tol == 0.0)
        s.status = STP_OK;
      else
        s.status = STP_NOT_CONVERGED;
    } else {
      s.iterations = hi[b];
      s.rel_residual = hs[b];
      s.outer_iterations = hi[2 * nr + b] + 1;
      const int st = hi[nr + b], done = hi[3 * nr + b];
      s.status = !done ? STP_NOT_CONVERGED : st == -3 ? STP_E_BREAKDOWN : STP_OK;
    }
    s.seconds = ms * 1e-3;
    c->iters[b] = s.iterations;
  }
  c->drv.phase = stp_ctx::kDone;
}

// Mixed form: outer step k > 0 starts from the FP64 residual f-hat - S-hat w.
// The stopping quantity r^T K_X r is taken with the FP32 K_X on the residual
// rounded to FP32 (the inner PCG start computes it anyway); relative to the
// same quantity of the first step its rounding largely cancels.  `last`: the
// refinement-step limit is reached, so this evaluation only reports.
stp_status mixed_outer_start(stp_ctx* c, int k, bool last) {
  PcgVecs<float>& v = c->pcg32;
  if (k > 0) {
    STP_TRY(Shat_apply<double>(c, c->ops64, c->w64, c->r64, c->nrhs));
    HIP_TRY(residual64(c->stream, c->fhat, c->r64, c->r64, c->vec));
  }
  HIP_TRY((cast<double, float>(c->stream, c->r64, v.rhs, c->vec)));
  STP_TRY(pcg_init<float>(c, v, v.rhs, nullptr));
  HIP_TRY(mixed_adjust(c->stream, c->sc, c->ms, c->nrhs, c->tolv, c->opt.inner_tol, k, last));
  return STP_OK;
}

}  // namespace

namespace stp {

// First unit of a solve: f (Lemma 4.1), f-hat = W^T f, the PCG start.
// `tol` holds one relative tolerance per right-hand side (host memory).
stp_status drive_begin(stp_ctx* c, const double* tol, const stp_ctx* coarse) {
  const int nr = c->nrhs;
  for (int b = 0; b < nr; ++b) c->h_tol[b] = tol[b];
  c->solved = false;
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  HIP_TRY(hipMemcpyAsync(c->tolv, c->h_tol, sizeof(double) * nr, hipMemcpyHostToDevice, c->stream));
  STP_TRY(rhs_apply(c, c->fhat));
  HIP_TRY(wavelet<double>(c->stream, c->fhat, c->J, c->slab, nr, false, c->syn_order));
  if (c->prec == STP_FP64) {
    if (coarse)
      STP_TRY(pcg_init_from(c, coarse, c->tolv));
    else
      STP_TRY(pcg_init<double>(c, c->pcg64, c->fhat, c->tolv));
  } else {
    HIP_TRY(mixed_reset(c->stream, c->ms, nr));
    HIP_TRY(hipMemsetAsync(c->w64, 0, sizeof(double) * c->vec, c->stream));
    HIP_TRY(copy<double>(c->stream, c->fhat, c->r64, c->vec));
    STP_TRY(mixed_outer_start(c, 0, false));
  }
  c->drv.phase = stp_ctx::kIter;
  c->drv.outer_k = 0;
  c->drv.adjusted = true;
  STP_TRY(post_flags(c));
  return STP_OK;
}

// K_x (vcycles V-cycles from zero for A_x) on `rows` slabs of level K, with
// the multigrid work space the caller provides (no allocation).
stp_status kspace_apply_slabs(hipStream_t s, MgScratch<double>& mg, const double* b, double* x,
                              int K, int rows, int vcycles) {
  stp_ctx c;
  c.K = K;
  c.stream = s;
  c.opt.vcycles = vcycles;
  return mg_apply<double>(&c, mg, b, x, rows, 1.0, nullptr);
}

// Whether the last unit has completed (never blocks).
bool drive_ready(stp_ctx* c) { return hipEventQuery(c->ev_flags) == hipSuccess; }

stp_status drive_wait(stp_ctx* c) {
  HIP_TRY(hipEventSynchronize(c->ev_flags));
  return STP_OK;
}

// Enqueue the unit that follows the completed one; phase becomes kDone when
// the solve has finished and its statistics are in c->stats.
stp_status drive_next(stp_ctx* c) {
  stp_ctx::Drive& d = c->drv;
  if (d.phase == stp_ctx::kFinish) {
    collect_stats(c);
    c->solved = true;
    return STP_OK;
  }
  if (d.phase != stp_ctx::kIter) {
    set_error("no solve in progress");
    return STP_E_INVALID_ARG;
  }
  if (any_active(c)) {
    const int m = iteration_batch(c);
    for (int i = 0; i < m; ++i) {
      if (c->prec == STP_FP64)
        STP_TRY(iterate<double>(c, c->pcg64));
      else
        STP_TRY(iterate<float>(c, c->pcg32));
    }
    d.adjusted = false;
    return post_flags(c);
  }
  if (c->prec == STP_FP64 || d.adjusted) return finish_unit(c);
  // mixed: the inner solve has ended; refine w and start the next outer step.
  // At the step limit the residual of the refined w is still evaluated, so
  // that the reported residual belongs to the returned solution.
  HIP_TRY(mixed_inner_done(c->stream, c->sc, c->ms, c->nrhs));
  HIP_TRY(add_correction(c->stream, c->w64, c->pcg32.w, c->per_rhs, c->nrhs, c->ms.status));
  d.outer_k += 1;
  const bool last = d.outer_k >= c->opt.max_outer;
  STP_TRY(mixed_outer_start(c, d.outer_k, last));
  d.adjusted = true;
  if (last) return finish_unit(c);
  return post_flags(c);
}

}  // namespace stp

namespace {

template <typename T>
stp_status ensure_ops(stp_ctx* c, Ops<T>& o) {
  if (o.ready) return STP_OK;
  Arena ar;
  ar.dry = false;
  ar.list = &c->allocations;
  ar.stream = c->stream;
  STP_TRY(plan_ops(ar, o, c->K, c->rows, c->vec, c->dim));
  c->bytes += ar.bytes;
  return STP_OK;
}

stp_status check_ctx(const stp_ctx* c) {
  if (!c) {
    set_error("NULL context");
    return STP_E_INVALID_ARG;
  }
  return STP_OK;
}

stp_status check_rhs(const stp_ctx* c, int rhs) {
  STP_TRY(check_ctx(c));
  if (rhs < 0 || rhs >= c->nrhs) {
    set_error("rhs index " + std::to_string(rhs) + " out of range [0, " + std::to_string(c->nrhs) + ")");
    return STP_E_INVALID_ARG;
  }
  return STP_OK;
}

stp_status check_sizes(int J, int K, int nrhs, int precision) {
  if (J < 0 || J > kMaxJ || K < 1 || K > kMaxK || nrhs < 1 || nrhs > 4096 ||
      (precision != STP_FP64 && precision != STP_MIXED)) {
    set_error("need 0 <= J <= 14, 1 <= K <= 10, 1 <= nrhs <= 4096 and a valid precision");
    return STP_E_INVALID_ARG;
  }
  return STP_OK;
}

void init_dims(stp_ctx* c, int J, int K, int nrhs, int precision, int dim = 2) {
  c->J = J;
  c->K = K;
  c->nrhs = nrhs;
  c->prec = precision;
  c->dim = dim;
  const int64_t n = grid_n(K);
  c->nx = dim == 3 ? n * n * n : n * n;
  c->slab = dim == 3 ? slab3_elems(K) : slab_elems(K);
  c->rows_per = (1 << J) + 1;
  c->rows = (int64_t)nrhs * c->rows_per;
  c->per_rhs = c->rows_per * c->slab;
  c->vec = c->rows * c->slab;
}

// copy `count` FP64 values (host or device) into a device scratch buffer
stp_status stage_in(stp_ctx* c, const double* src, int on_device, int64_t count, double* dst) {
  HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * count,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(c->stream));
  return STP_OK;
}

}  // namespace

// ================================================================== C-ABI

extern "C" {

const char* stp_status_string(stp_status s) {
  switch (s) {
    case STP_OK: return "ok";
    case STP_NOT_CONVERGED: return "not converged (maxit reached)";
    case STP_E_INVALID_ARG: return "invalid argument";
    case STP_E_OUT_OF_MEMORY: return "out of device memory";
    case STP_E_BREAKDOWN: return "PCG breakdown";
    case STP_E_DEVICE: return "HIP device error";
    case STP_E_UNSUPPORTED: return "unsupported";
    case STP_E_BUSY: return "not ready";
    default: return "unknown status";
  }
}

const char* stp_last_error(void) { return g_last_error.c_str(); }

stp_status stp_footprint(int J, int K, int nrhs, int precision, size_t* bytes) {
  STP_TRY(check_sizes(J, K, nrhs, precision));
  if (!bytes) {
    set_error("NULL output");
    return STP_E_INVALID_ARG;
  }
  stp_ctx c;
  init_dims(&c, J, K, nrhs, precision);
  Arena ar;
  ar.dry = true;
  STP_TRY(plan_context(ar, &c));
  *bytes = ar.bytes;
  return STP_OK;
}

stp_status stp_create(int J, int K, int nrhs, int precision, const stp_options* opt,
                      void* hip_stream, stp_ctx** out) {
  if (!out) {
    set_error("NULL output");
    return STP_E_INVALID_ARG;
  }
  *out = nullptr;
  STP_TRY(check_sizes(J, K, nrhs, precision));
  stp_options o = resolve(opt);
  if (o.sweeps != 3) {
    set_error("the GPU kernels implement 3 Gauss-Seidel steps per grid (sweeps = 3)");
    return STP_E_UNSUPPORTED;
  }
  if (!(o.diffusion[0] > 0.0 && o.diffusion[1] > 0.0 &&
        o.diffusion[0] * o.diffusion[1] > o.diffusion[2] * o.diffusion[2]) ||
      !(o.reaction >= 0.0) || !std::isfinite(o.reaction)) {
    set_error("the diffusion tensor must be symmetric positive definite and the reaction >= 0");
    return STP_E_INVALID_ARG;
  }
  const int dim = o.dim == 3 ? 3 : 2;
  if (o.dim != 0 && o.dim != 2 && o.dim != 3) {
    set_error("dim must be 0, 2 or 3");
    return STP_E_INVALID_ARG;
  }
  if (dim == 3 && (K > kMaxK3 || o.nested > 0 || o.diffusion[2] != 0.0 ||
                   o.diffusion[0] != 1.0 || o.diffusion[1] != 1.0 || o.reaction != 0.0)) {
    set_error("the 3D problem is the heat equation with K <= 8, without nested iteration");
    return dim == 3 && K > kMaxK3 ? STP_E_INVALID_ARG : STP_E_UNSUPPORTED;
  }
  if (o.nested > 0 && precision != STP_FP64) {
    set_error("nested iteration is implemented for STP_FP64");
    return STP_E_UNSUPPORTED;
  }
  const int depth = std::min(o.nested, std::min(J, K - 1));
  stp_ctx* c = new (std::nothrow) stp_ctx();
  if (!c) {
    set_error("host allocation failed");
    return STP_E_OUT_OF_MEMORY;
  }
  init_dims(c, J, K, nrhs, precision, dim);
  c->opt = o;
  c->op.dxx = o.diffusion[0];
  c->op.dyy = o.diffusion[1];
  c->op.dxy = o.diffusion[2];
  c->op.c = o.reaction;
  if (c->opt.inner_tol <= 0.0) c->opt.inner_tol = default_inner_tol(K);
  c->use_graph = o.graph >= 0;
  c->has_g.assign(nrhs, 0);
  c->iters.assign(nrhs, 0);
  c->stats.assign(nrhs, stp_stats{});
  auto fail = [&](stp_status s) {
    free_all(c);
    delete c;
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    set_error("no HIP device");
    return fail(STP_E_DEVICE);
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      set_error("hipStreamCreate failed");
      return fail(STP_E_DEVICE);
    }
    c->own_stream = true;
  }
  {
    // refuse early when the context cannot fit in what the device has free
    Arena dry;
    stp_ctx probe;
    init_dims(&probe, J, K, nrhs, precision, dim);
    size_t free_b = 0, total_b = 0;
    bool ok = plan_context(dry, &probe) == STP_OK;
    for (int d = 1; ok && d <= depth; ++d) {
      stp_ctx coarse;
      init_dims(&coarse, J - d, K - d, nrhs, precision);
      ok = plan_context(dry, &coarse) == STP_OK;
    }
    if (ok && hipMemGetInfo(&free_b, &total_b) == hipSuccess && dry.bytes > free_b) {
      set_error("context needs " + std::to_string(dry.bytes) + " bytes of device memory, " +
                std::to_string(free_b) + " are free");
      return fail(STP_E_OUT_OF_MEMORY);
    }
  }
  Arena ar;
  ar.dry = false;
  ar.list = &c->allocations;
  ar.stream = c->stream;
  stp_status st = plan_context(ar, c);
  if (st < 0) return fail(st);
  c->bytes = ar.bytes;
  if (hipHostMalloc((void**)&c->h_flags, sizeof(double) * 5 * nrhs) != hipSuccess ||
      hipHostMalloc((void**)&c->h_stats, sizeof(double) * 4 * nrhs) != hipSuccess ||
      hipHostMalloc((void**)&c->h_tol, sizeof(double) * nrhs) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_flags, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    set_error("pinned host allocation or event creation failed");
    return fail(STP_E_DEVICE);
  }
  // the read order of the one-pass synthesis (the host copy lives until the
  // synchronisation below)
  const std::vector<int> order = synthesis_read_order(J);
  if (fill_level_sigma(c->stream, c->sigma, J, nrhs) != hipSuccess ||
      hipMemcpyAsync(c->syn_order, order.data(), sizeof(int) * order.size(),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    set_error("initialisation kernels failed");
    return fail(STP_E_DEVICE);
  }
  // nested iteration: one context per coarser mesh, on this context's stream
  for (int d = 1; d <= depth; ++d) {
    stp_options oc = o;
    oc.nested = 0;
    stp_ctx* n = nullptr;
    st = stp_create(J - d, K - d, nrhs, precision, &oc, c->stream, &n);
    if (st < 0) return fail(st);
    c->nest.push_back(n);
  }
  *out = c;
  return STP_OK;
}

void stp_destroy(stp_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

stp_status stp_set_u0(stp_ctx* c, int rhs, const double* u0, int on_device) {
  STP_TRY(check_rhs(c, rhs));
  double* dst = c->u0 + (int64_t)rhs * c->slab;
  if (!u0) {
    HIP_TRY(hipMemsetAsync(dst, 0, sizeof(double) * c->slab, c->stream));
    return STP_OK;
  }
  double* tmp = c->ops64.z;  // compact staging area (large enough: >= vec elements)
  STP_TRY(stage_in(c, u0, on_device, c->nx, tmp));
  HIP_TRY(pack_rows<double>(c, tmp, dst, 1));
  return STP_OK;
}

stp_status stp_set_g(stp_ctx* c, int rhs, const double* g, int on_device) {
  STP_TRY(check_rhs(c, rhs));
  double* dst = c->g + (int64_t)rhs * c->per_rhs;
  if (!g) {
    HIP_TRY(hipMemsetAsync(dst, 0, sizeof(double) * c->per_rhs, c->stream));
    c->has_g[rhs] = 0;
    return STP_OK;
  }
  double* tmp = c->ops64.z;
  STP_TRY(stage_in(c, g, on_device, c->nx * c->rows_per, tmp));
  HIP_TRY(pack_rows<double>(c, tmp, dst, (int)c->rows_per));
  c->has_g[rhs] = 1;
  return STP_OK;
}

stp_status stp_solve(stp_ctx* c, double rel_tol, stp_stats* per_rhs) {
  STP_TRY(check_ctx(c));
  if (!(rel_tol >= 0.0) || rel_tol >= 1.0) {
    set_error("rel_tol must be in [0, 1)");
    return STP_E_INVALID_ARG;
  }
  if (c->drv.phase == stp_ctx::kIter || c->drv.phase == stp_ctx::kFinish) {
    set_error("a solve is already in progress on this context");
    return STP_E_INVALID_ARG;
  }
  auto run = [](stp_ctx* x, double t, const stp_ctx* coarse) -> stp_status {
    std::vector<double> tol(x->nrhs, t);
    STP_TRY(drive_begin(x, tol.data(), coarse));
    while (x->drv.phase != stp_ctx::kDone) {
      STP_TRY(drive_wait(x));
      STP_TRY(drive_next(x));
    }
    return STP_OK;
  };
  // nested iteration (Section 4.2): the coarsest mesh from zero, every finer
  // mesh from the coarser solution, each to a tolerance that halves with
  // the mesh width like the X-norm discretisation error
  std::vector<int> coarse_its(c->nrhs, 0);
  double coarse_seconds = 0.0;
  stp_status st = STP_OK;
  const int depth = (int)c->nest.size();
  for (int d = depth; d >= 1 && st >= 0; --d) {
    stp_ctx* n = c->nest[d - 1];
    n->has_g = c->has_g;
    if (hipSuccess != inject(c->stream, c->g, n->g, c->K, d, (int)c->rows_per, (int)n->rows_per,
                             1 << d, c->nrhs) ||
        hipSuccess != inject(c->stream, c->u0, n->u0, c->K, d, 1, 1, 1, c->nrhs)) {
      set_error("nested iteration: injection of the data failed");
      st = STP_E_DEVICE;
      break;
    }
    st = run(n, rel_tol * std::ldexp(1.0, d), d < depth ? c->nest[d] : nullptr);
    if (st < 0) {
      n->drv.phase = stp_ctx::kIdle;
      break;
    }
    for (int b = 0; b < c->nrhs; ++b) coarse_its[b] += n->stats[b].iterations;
    coarse_seconds += n->stats[0].seconds;
  }
  if (st >= 0) st = run(c, rel_tol, depth > 0 ? c->nest[0] : nullptr);
  if (st < 0) {
    c->drv.phase = stp_ctx::kIdle;
    return st;
  }
  for (int b = 0; b < c->nrhs; ++b) {
    c->stats[b].coarse_iterations = coarse_its[b];
    c->stats[b].seconds += coarse_seconds;
  }
  stp_status worst = STP_OK;
  for (int b = 0; b < c->nrhs; ++b) {
    if (c->stats[b].status == STP_E_BREAKDOWN) worst = STP_E_BREAKDOWN;
    else if (c->stats[b].status == STP_NOT_CONVERGED && worst == STP_OK) worst = STP_NOT_CONVERGED;
    if (per_rhs) per_rhs[b] = c->stats[b];
  }
  if (worst == STP_E_BREAKDOWN) set_error("PCG breakdown (p^T S-hat p <= 0 or non-finite)");
  return worst;
}

stp_status stp_get_solution(stp_ctx* c, int rhs, double* u, int on_device) {
  STP_TRY(check_rhs(c, rhs));
  if (!u) {
    set_error("NULL output");
    return STP_E_INVALID_ARG;
  }
  if (!c->solved) {
    set_error("no solve has run on this context");
    return STP_E_INVALID_ARG;
  }
  const int64_t count = c->nx * c->rows_per;
  double* src = c->u + (int64_t)rhs * c->per_rhs;
  if (on_device) {
    HIP_TRY(unpack_rows<double>(c, src, u, (int)c->rows_per));
  } else {
    double* tmp = c->ops64.z;
    HIP_TRY(unpack_rows<double>(c, src, tmp, (int)c->rows_per));
    HIP_TRY(hipMemcpyAsync(u, tmp, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return STP_OK;
}

stp_status stp_profile(stp_ctx* c, int enable) {
  STP_TRY(check_ctx(c));
  STP_TRY(flush_timing(c));
  c->profiling = enable != 0;
  if (enable)
    for (auto& k : c->kstat) k = stp_kernel_stat{};
  return STP_OK;
}

stp_status stp_profile_read(stp_ctx* c, int kernel, stp_kernel_stat* out) {
  STP_TRY(check_ctx(c));
  if (kernel < 0 || kernel >= STP_KERNEL_COUNT || !out) {
    set_error("stp_profile_read: bad kernel id or NULL output");
    return STP_E_INVALID_ARG;
  }
  STP_TRY(flush_timing(c));
  *out = c->kstat[kernel];
  return STP_OK;
}

stp_status stp_get_iterations(const stp_ctx* c, int rhs, int* iterations) {
  STP_TRY(check_rhs(c, rhs));
  if (!iterations) {
    set_error("NULL output");
    return STP_E_INVALID_ARG;
  }
  *iterations = c->iters[rhs];
  return STP_OK;
}

}  // extern "C"

namespace {

template <typename T>
stp_status apply_op_t(stp_ctx* c, int op, const double* in_dev, double* out_dev) {
  Ops<T>& o = ops_of<T>(c);
  STP_TRY(ensure_ops<T>(c, o));
  const int K = c->K, J = c->J;
  const int rows = (int)c->rows_per;
  T* in_t = (T*)(c->apply_buf + 2 * c->per_rhs);
  T* out_t = (T*)(c->apply_buf + 3 * c->per_rhs);
  HIP_TRY(pack_rows<T>(c, in_dev, in_t, rows));
  switch (op) {
    case STP_OP_W:
      HIP_TRY(copy<T>(c->stream, in_t, out_t, c->per_rhs));
      HIP_TRY(wavelet<T>(c->stream, out_t, J, c->slab, 1, true, c->syn_order));
      break;
    case STP_OP_WT:
      HIP_TRY(copy<T>(c->stream, in_t, out_t, c->per_rhs));
      HIP_TRY(wavelet<T>(c->stream, out_t, J, c->slab, 1, false, c->syn_order));
      break;
    case STP_OP_S:
      STP_TRY(S_apply<T>(c, o, in_t, out_t, 1));
      break;
    case STP_OP_SHAT:
      STP_TRY(Shat_apply<T>(c, o, in_t, out_t, 1));
      break;
    case STP_OP_KX:
      STP_TRY(KX_apply<T>(c, o, in_t, out_t, 1));
      break;
    case STP_OP_KSPACE:
      STP_TRY(mg_apply<T>(c, o.mg, in_t, out_t, rows, 1.0, nullptr));
      break;
    case STP_OP_A:
      if (c->dim == 3)
        HIP_TRY(apply_A3<T>(c->stream, in_t, out_t, K, rows));
      else
        HIP_TRY(apply_A<T>(c->stream, in_t, out_t, K, rows, c->op));
      break;
    case STP_OP_M:
      if (c->dim == 3)
        HIP_TRY(apply_M3<T>(c->stream, in_t, out_t, K, rows));
      else
        HIP_TRY(apply_M<T>(c->stream, in_t, out_t, K, rows));
      break;
    default:
      set_error("unknown operator");
      return STP_E_INVALID_ARG;
  }
  HIP_TRY(unpack_rows<T>(c, out_t, out_dev, rows));
  return STP_OK;
}

}  // namespace

extern "C" stp_status stp_apply(stp_ctx* c, int op, int precision, int rhs, const double* in,
                                double* out, int on_device) {
  STP_TRY(check_rhs(c, rhs));
  if (!out || (!in && op != STP_OP_RHS) || (precision != STP_FP64 && precision != STP_MIXED)) {
    set_error("stp_apply: NULL buffer or bad precision");
    return STP_E_INVALID_ARG;
  }
  if (c->nrhs != 1) {
    set_error("stp_apply needs a context with nrhs = 1");
    return STP_E_UNSUPPORTED;
  }
  if (op < STP_OP_W || op > STP_OP_M) {
    set_error("unknown operator");
    return STP_E_INVALID_ARG;
  }
  const int64_t count = c->nx * c->rows_per;
  if (!c->apply_buf) {
    Arena ar;
    ar.dry = false;
    ar.list = &c->allocations;
    ar.stream = c->stream;
    STP_TRY(ar.get(&c->apply_buf, 4 * c->per_rhs));
    c->bytes += ar.bytes;
  }
  double* in_dev = on_device ? (double*)in : c->apply_buf;
  double* out_dev = on_device ? out : c->apply_buf + c->per_rhs;
  if (op == STP_OP_RHS) {
    double* f = (double*)(c->apply_buf + 3 * c->per_rhs);
    STP_TRY(rhs_apply(c, f));
    HIP_TRY(unpack_rows<double>(c, f, out_dev, (int)c->rows_per));
  } else {
    if (!on_device)
      HIP_TRY(hipMemcpyAsync(in_dev, in, sizeof(double) * count, hipMemcpyHostToDevice, c->stream));
    if (precision == STP_FP64)
      STP_TRY(apply_op_t<double>(c, op, in_dev, out_dev));
    else
      STP_TRY(apply_op_t<float>(c, op, in_dev, out_dev));
  }
  if (!on_device)
    HIP_TRY(hipMemcpyAsync(out, out_dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return STP_OK;
}
