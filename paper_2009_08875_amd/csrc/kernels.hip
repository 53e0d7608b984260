// HIP kernels of the space-time solver for gfx950 (MI355X).
//
// All operators are constant-coefficient stencils on uniform grids, so no
// matrix is stored: every kernel reads its input once per needed element and
// recomputes coefficients from the mesh width.  The hot kernels (multigrid smoothing and
// the space-time stencils) live in mg_stream.hip and stencil.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace stp {

namespace {

constexpr int kBlock = 256;

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

inline unsigned blocks_for(int64_t count, int per_block = kBlock) {
  return (unsigned)((count + per_block - 1) / per_block);
}

// ------------------------------------------------------------ row stencils

__device__ inline bool node_of(int64_t idx, int K, int& gx, int& gy) {
  const int pitch = line_pitch(K);
  const int n = grid_n(K);
  gy = (int)(idx / pitch) + 1;
  gx = (int)(idx - (int64_t)(gy - 1) * pitch) + 1;
  return gx <= n && gy <= n;
}

// value of a slab at node (gx + dx, gy + dy), zero outside the grid
template <typename T>
__device__ inline T at(const T* s, int gx, int gy, int dx, int dy, int n, int pitch) {
  const int x = gx + dx, y = gy + dy;
  return (x >= 1 && x <= n && y >= 1 && y <= n) ? s[(int64_t)(y - 1) * pitch + (x - 1)] : T(0);
}

template <typename T>
__device__ inline T A_at(const T* s, int gx, int gy, int n, int pitch) {
  const T c = at(s, gx, gy, 0, 0, n, pitch);
  return T(4) * c - at(s, gx, gy, 1, 0, n, pitch) - at(s, gx, gy, -1, 0, n, pitch) -
         at(s, gx, gy, 0, 1, n, pitch) - at(s, gx, gy, 0, -1, n, pitch);
}

template <typename T>
__device__ inline T M_at(const T* s, int gx, int gy, int n, int pitch, T m12) {
  const T c = at(s, gx, gy, 0, 0, n, pitch);
  return m12 * (T(6) * c + at(s, gx, gy, 1, 0, n, pitch) + at(s, gx, gy, -1, 0, n, pitch) +
                at(s, gx, gy, 0, 1, n, pitch) + at(s, gx, gy, 0, -1, n, pitch) +
                at(s, gx, gy, 1, 1, n, pitch) + at(s, gx, gy, -1, -1, n, pitch));
}

// A_x = A_D + c M_x (Section 4) at node (gx, gy), with the stencil of
// stencil_of(op, 1, 0, K).
template <typename T>
__device__ inline T Aop_at(const T* s, int gx, int gy, int n, int pitch, const Stencil& st) {
  return ((T(st.c0) * at(s, gx, gy, 0, 0, n, pitch) +
           T(st.cx) * (at(s, gx, gy, 1, 0, n, pitch) + at(s, gx, gy, -1, 0, n, pitch))) +
          T(st.cy) * (at(s, gx, gy, 0, 1, n, pitch) + at(s, gx, gy, 0, -1, n, pitch))) +
         T(st.cd) * (at(s, gx, gy, 1, 1, n, pitch) + at(s, gx, gy, -1, -1, n, pitch));
}

template <typename T, bool IS_A>
__global__ __launch_bounds__(kBlock) void apply_AM_kernel(const T* __restrict__ x,
                                                          T* __restrict__ y, int K, SpaceOp op) {
  const int64_t slab = slab_elems(K);
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= slab) return;
  const int64_t row = blockIdx.y;
  int gx, gy;
  if (!node_of(idx, K, gx, gy)) {
    y[row * slab + idx] = T(0);
    return;
  }
  const int n = grid_n(K), pitch = line_pitch(K);
  const double h = 1.0 / (double)(1 << K);
  const T m12 = T(h * h / 12.0);
  if constexpr (IS_A) {
    y[row * slab + idx] = op.heat() ? A_at(x + row * slab, gx, gy, n, pitch)
                                    : Aop_at(x + row * slab, gx, gy, n, pitch, stencil_of(op, 1.0, 0.0, K));
  } else {
    y[row * slab + idx] = M_at(x + row * slab, gx, gy, n, pitch, m12);
  }
}

// ------------------------------------------------------------ reductions

__device__ double block_sum(double v) {
  __shared__ double part[kBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < kBlock / 64; ++k) t += part[k];
  }
  __syncthreads();
  return t;
}

// 16 bytes of T: the widest load a lane issues (four floats or two doubles).
template <typename T>
struct alignas(16) Vec16 {
  static constexpr int W = 16 / (int)sizeof(T);
  T e[W];
};

// Partial sums of a . b over 16-byte vectors, two independent loads per
// thread and step to keep more bytes in flight; n is a multiple of the
// vector width and the segments are 16-byte aligned (checked by the launcher).
template <typename T>
__global__ __launch_bounds__(kBlock) void dot_partial_vec_kernel(const T* __restrict__ a,
                                                                 const T* __restrict__ b,
                                                                 int64_t n,
                                                                 double* __restrict__ partials) {
  using V = Vec16<T>;
  const int nblk = gridDim.x;
  const int64_t seg = (int64_t)blockIdx.y * n;
  const V* av = reinterpret_cast<const V*>(a + seg);
  const V* bv = reinterpret_cast<const V*>(b + seg);
  const int64_t nv = n / V::W;
  const int64_t stride = (int64_t)nblk * kBlock;
  double acc0 = 0.0, acc1 = 0.0;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + stride < nv; i += 2 * stride) {
    const V x0 = av[i], y0 = bv[i], x1 = av[i + stride], y1 = bv[i + stride];
#pragma unroll
    for (int w = 0; w < V::W; ++w) {
      acc0 += (double)x0.e[w] * (double)y0.e[w];
      acc1 += (double)x1.e[w] * (double)y1.e[w];
    }
  }
  if (i < nv) {
    const V x0 = av[i], y0 = bv[i];
#pragma unroll
    for (int w = 0; w < V::W; ++w) acc0 += (double)x0.e[w] * (double)y0.e[w];
  }
  const double acc = block_sum(acc0 + acc1);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * nblk + blockIdx.x] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dot_partial_kernel(const T* __restrict__ a,
                                                             const T* __restrict__ b, int64_t n,
                                                             double* __restrict__ partials) {
  const int nblk = gridDim.x;
  const int64_t seg = (int64_t)blockIdx.y * n;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)nblk * kBlock)
    acc += (double)a[seg + i] * (double)b[seg + i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * nblk + blockIdx.x] = acc;
}

__global__ __launch_bounds__(kBlock) void dot_final_kernel(const double* __restrict__ partials,
                                                           int nblk, double* __restrict__ out) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kBlock) acc += partials[(int64_t)blockIdx.x * nblk + k];
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// ------------------------------------------------------------ vector updates

template <typename T>
__global__ __launch_bounds__(kBlock) void copy_vec_kernel(const Vec16<T>* __restrict__ s,
                                                          Vec16<T>* __restrict__ d, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < nv) d[i] = s[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void copy_kernel(const T* __restrict__ s, T* __restrict__ d,
                                                      int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) d[i] = s[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void update_wr_kernel(T* __restrict__ w, T* __restrict__ r,
                                                           const T* __restrict__ p,
                                                           const T* __restrict__ q,
                                                           const double* __restrict__ gamma,
                                                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double g = gamma[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.y * n + i;
  w[k] = (T)((double)w[k] + g * (double)p[k]);
  r[k] = (T)((double)r[k] - g * (double)q[k]);
}

// Vector forms of the two updates: 16 bytes per lane and array; n is a
// multiple of the vector width and every array is 16-byte aligned.
template <typename T>
__global__ __launch_bounds__(kBlock) void update_wr_vec_kernel(Vec16<T>* __restrict__ w,
                                                               Vec16<T>* __restrict__ r,
                                                               const Vec16<T>* __restrict__ p,
                                                               const Vec16<T>* __restrict__ q,
                                                               const double* __restrict__ gamma,
                                                               int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nv) return;
  const double g = gamma[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.y * nv + i;
  Vec16<T> wv = w[k], rv = r[k];
  const Vec16<T> pv = p[k], qv = q[k];
#pragma unroll
  for (int e = 0; e < Vec16<T>::W; ++e) {
    wv.e[e] = (T)((double)wv.e[e] + g * (double)pv.e[e]);
    rv.e[e] = (T)((double)rv.e[e] - g * (double)qv.e[e]);
  }
  w[k] = wv;
  r[k] = rv;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void update_p_vec_kernel(Vec16<T>* __restrict__ p,
                                                              const Vec16<T>* __restrict__ z,
                                                              const double* __restrict__ beta,
                                                              int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nv) return;
  const double bt = beta[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.y * nv + i;
  Vec16<T> pv = p[k];
  const Vec16<T> zv = z[k];
#pragma unroll
  for (int e = 0; e < Vec16<T>::W; ++e) pv.e[e] = (T)((double)zv.e[e] + bt * (double)pv.e[e]);
  p[k] = pv;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void update_p_kernel(T* __restrict__ p,
                                                          const T* __restrict__ z,
                                                          const double* __restrict__ beta,
                                                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double bt = beta[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.y * n + i;
  p[k] = (T)((double)z[k] + bt * (double)p[k]);
}

__global__ void pcg_start_kernel(PcgScalars sc, int nrhs, const double* __restrict__ tol,
                                 const double* __restrict__ ref) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  const double rho = sc.rhonew[b];
  const double t = tol ? tol[b] : 0.0;
  // the stopping test is relative to f-hat^T K_X f-hat: the first residual's
  // quantity from w = 0, computed separately (ref) from an initial guess
  const double r0 = ref ? ref[b] : rho;
  sc.rho[b] = rho;
  sc.rho0[b] = r0;
  sc.its[b] = 0;
  sc.gamma[b] = 0.0;
  sc.beta[b] = 0.0;
  sc.target[b] = t > 0.0 ? t * sqrt(fmax(r0, 0.0)) : 0.0;
  if (!isfinite(rho) || rho < 0.0) {
    sc.active[b] = 0;
    sc.status[b] = -3;
  } else if (rho == 0.0) {
    sc.active[b] = 0;  // zero right-hand side: w = 0 is exact
    sc.status[b] = 1;
  } else {
    sc.active[b] = 1;
    sc.status[b] = 0;
  }
}

__global__ void pack_flags_kernel(PcgScalars sc, int nrhs, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  out[5 * b] = (double)sc.active[b];
  out[5 * b + 1] = (double)sc.its[b];
  out[5 * b + 2] = sc.rho[b];
  out[5 * b + 3] = sc.rho0[b];
  out[5 * b + 4] = sc.target[b];
}

__global__ void pcg_gamma_kernel(PcgScalars sc, int nrhs) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  if (!sc.active[b]) {
    sc.gamma[b] = 0.0;
    return;
  }
  const double pq = sc.pq[b];
  if (!(pq > 0.0) || !isfinite(pq)) {
    sc.gamma[b] = 0.0;
    sc.active[b] = 0;
    sc.status[b] = -3;
    return;
  }
  sc.gamma[b] = sc.rho[b] / pq;
}

__global__ void pcg_beta_kernel(PcgScalars sc, int nrhs, int maxit) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  if (!sc.active[b]) {
    sc.beta[b] = 0.0;
    return;
  }
  const double rn = sc.rhonew[b];
  sc.its[b] += 1;
  if (!isfinite(rn) || rn < 0.0) {
    sc.beta[b] = 0.0;
    sc.active[b] = 0;
    sc.status[b] = -3;
    return;
  }
  sc.beta[b] = rn / sc.rho[b];
  sc.rho[b] = rn;
  if (rn == 0.0 || sqrt(rn) <= sc.target[b]) {
    sc.active[b] = 0;
    sc.status[b] = 1;
  } else if (sc.its[b] >= maxit) {
    sc.active[b] = 0;  // iteration limit: status stays 0 (not converged)
  }
}

// Mixed form, start of outer step k (after the inner PCG start): decide per
// right-hand side whether the FP64 residual already meets the tolerance, and
// set the inner stopping target.
__global__ void mixed_adjust_kernel(PcgScalars sc, MixedState ms, int nrhs,
                                    const double* __restrict__ tol, double inner_tol, int k,
                                    int last) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  if (ms.done[b]) {
    sc.active[b] = 0;
    sc.target[b] = 0.0;
    return;
  }
  const double t = tol[b];
  const double rho0 = sc.rho0[b];
  ms.outer[b] = k;
  if (k == 0) ms.rho0_first[b] = rho0;
  const double first = ms.rho0_first[b];
  const double rel = first > 0.0 ? sqrt(fmax(rho0, 0.0) / first) : 0.0;
  ms.rel[b] = rel;
  if (sc.status[b] == -3) {
    ms.done[b] = 1;
    ms.status[b] = -3;
    sc.active[b] = 0;
  } else if (first <= 0.0 || (t > 0.0 && rel <= t) || rho0 == 0.0) {
    ms.done[b] = 1;
    ms.status[b] = 0;
    sc.active[b] = 0;
  } else {
    // at the refinement-step limit the solve ends unconverged (done stays 0)
    sc.active[b] = last ? 0 : 1;
  }
  // stop the inner solve at a relative reduction of inner_tol, but not below
  // what the outer tolerance still needs
  sc.target[b] = fmax(inner_tol * sqrt(fmax(rho0, 0.0)), 0.5 * t * sqrt(fmax(first, 0.0)));
}

// Mixed form, end of an inner solve: count its iterations, record breakdown.
__global__ void mixed_inner_done_kernel(PcgScalars sc, MixedState ms, int nrhs) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs || ms.done[b]) return;
  ms.inner_its[b] += sc.its[b];
  if (sc.status[b] == -3) {
    ms.done[b] = 1;
    ms.status[b] = -3;
  }
}

__global__ void mixed_reset_kernel(MixedState ms, int nrhs) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  ms.rho0_first[b] = -1.0;
  ms.rel[b] = 1.0;
  ms.done[b] = 0;
  ms.status[b] = 1;
  ms.outer[b] = 0;
  ms.inner_its[b] = 0;
}

// ------------------------------------------------------------ layout / casts

template <typename T>
__global__ __launch_bounds__(kBlock) void pack_kernel(const double* __restrict__ src,
                                                      T* __restrict__ dst, int K) {
  const int64_t slab = slab_elems(K);
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= slab) return;
  const int64_t row = blockIdx.y;
  int gx, gy;
  const int n = grid_n(K);
  T v = T(0);
  if (node_of(idx, K, gx, gy)) v = (T)src[row * n * n + (int64_t)(gy - 1) * n + (gx - 1)];
  dst[row * slab + idx] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void unpack_kernel(const T* __restrict__ src,
                                                        double* __restrict__ dst, int K) {
  const int n = grid_n(K);
  const int64_t nn = (int64_t)n * n;
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= nn) return;
  const int64_t row = blockIdx.y;
  const int gy = (int)(idx / n), gx = (int)(idx % n);
  dst[row * nn + idx] = (double)src[row * slab_elems(K) + (int64_t)gy * line_pitch(K) + gx];
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void cast_kernel(const Tin* __restrict__ in,
                                                      Tout* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) out[i] = (Tout)in[i];
}

__global__ __launch_bounds__(kBlock) void residual64_kernel(const double* __restrict__ f,
                                                            const double* __restrict__ q,
                                                            double* __restrict__ r,
                                                            int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) r[i] = f[i] - q[i];
}

// w += (double) d per right-hand side segment, except where status is -3
// (the inner solve broke down: its correction is not finite).
__global__ __launch_bounds__(kBlock) void add_correction_kernel(double* __restrict__ w,
                                                                const float* __restrict__ d,
                                                                int64_t n,
                                                                const int* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || status[blockIdx.y] == -3) return;
  const int64_t k = (int64_t)blockIdx.y * n + i;
  w[k] += (double)d[k];
}

// Nested iteration: the data of a coarser mesh (level Kc = Kf - d in space)
// are the values at its nodes, which are nodes of the fine mesh too: coarse
// row i of right-hand side b is fine row i * tstride, coarse node (a, b) is
// fine node (2^d a, 2^d b).  Pads are written zero.
__global__ __launch_bounds__(kBlock) void inject_kernel(const double* __restrict__ src,
                                                        double* __restrict__ dst, int Kf, int d,
                                                        int rows_f, int rows_c, int tstride) {
  const int Kc = Kf - d;
  const int64_t slab_c = slab_elems(Kc);
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= slab_c) return;
  const int row = blockIdx.y;  // coarse row within the right-hand side
  const int b = blockIdx.z;
  int gx, gy;
  double v = 0.0;
  if (node_of(idx, Kc, gx, gy)) {
    const int64_t fr = (int64_t)b * rows_f + (int64_t)row * tstride;
    v = src[fr * slab_elems(Kf) + (int64_t)((gy << d) - 1) * line_pitch(Kf) + ((gx << d) - 1)];
  }
  dst[((int64_t)b * rows_c + row) * slab_c + idx] = v;
}

// Nested iteration: wavelet-in-time, nodal-in-space coefficients of mesh
// (J - 1, K - 1) carried to mesh (J, K).  The wavelets of the coarse mesh are
// wavelets of the fine one: coarse row i moves to fine row 2 i and the odd
// fine rows (the new finest level) are zero; in space the coarse P1 function
// is interpolated at the fine nodes on the "/" mesh (Section 4, Section 4.2).
__global__ __launch_bounds__(kBlock) void prolong_w_kernel(const double* __restrict__ wc,
                                                           double* __restrict__ wf, int J,
                                                           int K) {
  const int64_t slab_f = slab_elems(K);
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= slab_f) return;
  const int row = blockIdx.y;  // fine row within the right-hand side
  const int b = blockIdx.z;
  const int Nf = 1 << J;
  double v = 0.0;
  int gx, gy;
  if ((row & 1) == 0 && node_of(idx, K, gx, gy)) {
    const int nc = grid_n(K - 1), pc = line_pitch(K - 1);
    const double* c =
        wc + ((int64_t)b * ((Nf >> 1) + 1) + (row >> 1)) * slab_elems(K - 1);
    // coarse value at coarse node (I, Jn), zero on the boundary
    auto at = [&](int I, int Jn) {
      return (I >= 1 && I <= nc && Jn >= 1 && Jn <= nc) ? c[(int64_t)(Jn - 1) * pc + (I - 1)] : 0.0;
    };
    const int I = gx >> 1, Jn = gy >> 1;
    if (!(gx & 1) && !(gy & 1))
      v = at(I, Jn);
    else if ((gx & 1) && !(gy & 1))
      v = 0.5 * (at(I, Jn) + at(I + 1, Jn));
    else if (!(gx & 1) && (gy & 1))
      v = 0.5 * (at(I, Jn) + at(I, Jn + 1));
    else
      v = 0.5 * (at(I, Jn) + at(I + 1, Jn + 1));
  }
  wf[((int64_t)b * (Nf + 1) + row) * slab_f + idx] = v;
}

__global__ void fill_level_sigma_kernel(double* sigma, int J, int nrhs) {
  const int N = 1 << J;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)nrhs * (N + 1)) return;
  const int i = (int)(k % (N + 1));
  sigma[k] = exp2((double)row_level(i, J));
}

}  // namespace

// ================================================================ launchers

template <typename T>
hipError_t apply_A(hipStream_t s, const T* x, T* y, int K, int rows, const SpaceOp& op) {
  apply_AM_kernel<T, true><<<dim3(blocks_for(slab_elems(K)), rows), kBlock, 0, s>>>(x, y, K, op);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_M(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply_AM_kernel<T, false><<<dim3(blocks_for(slab_elems(K)), rows), kBlock, 0, s>>>(x, y, K,
                                                                                     SpaceOp{});
  return hipGetLastError();
}

// The wavelet launches (the one-pass kernels of wavelet_stream.hip).
template <typename T, bool DOT>
hipError_t launch_ana(hipStream_t s, T* X, const T* p, double* partials, int J, int64_t slab, int nrhs,
                      int* nblk) {
  return wavelet_ana_stream<T, DOT>(s, X, p, partials, J, slab, nrhs, nblk);
}

template <typename T>
hipError_t wavelet(hipStream_t s, T* X, int J, int64_t slab, int nrhs, bool synthesis,
                   const int* order) {
  if (J == 0) return hipSuccess;
  if (synthesis)
    return wavelet_syn_stream<T, false>(s, X, X, nullptr, nullptr, nullptr, order, J, slab, nrhs);
  int nblk = 0;
  return launch_ana<T, false>(s, X, nullptr, nullptr, J, slab, nrhs, &nblk);
}

template <typename T>
hipError_t synthesis(hipStream_t s, const T* src, T* dst, int J, int64_t slab, int nrhs,
                     const int* order) {
  return wavelet_syn_stream<T, false>(s, src, dst, nullptr, nullptr, nullptr, order, J, slab, nrhs);
}

template <typename T>
hipError_t synthesis_update(hipStream_t s, T* p, const T* z, const double* beta, T* X, int J,
                            int64_t slab, int nrhs, const int* order) {
  return wavelet_syn_stream<T, true>(s, p, X, p, z, beta, order, J, slab, nrhs);
}

int analysis_dot_blocks(int64_t slab) { return wavelet_stream_blocks(slab); }

template <typename T>
hipError_t analysis_dot(hipStream_t s, T* X, const T* p, double* partials, double* out, int J,
                        int64_t slab, int nrhs) {
  int nblk = 0;
  const hipError_t e = launch_ana<T, true>(s, X, p, partials, J, slab, nrhs, &nblk);
  if (e != hipSuccess) return e;
  dot_final_kernel<<<nrhs, kBlock, 0, s>>>(partials, nblk, out);
  return hipGetLastError();
}

int dot_blocks(int64_t n) {
  int64_t b = (n + kBlock * 8 - 1) / (kBlock * 8);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
hipError_t dot(hipStream_t s, const T* a, const T* b, int64_t n, int nrhs, double* partials,
               double* out) {
  const int nblk = dot_blocks(n);
  // the vector form helps FP32 (16-byte loads); FP64 streams as fast with 8-byte ones
  if (sizeof(T) == 4 && n % Vec16<T>::W == 0 && aligned16(a) && aligned16(b))
    dot_partial_vec_kernel<T><<<dim3(nblk, nrhs), kBlock, 0, s>>>(a, b, n, partials);
  else
    dot_partial_kernel<T><<<dim3(nblk, nrhs), kBlock, 0, s>>>(a, b, n, partials);
  dot_final_kernel<<<nrhs, kBlock, 0, s>>>(partials, nblk, out);
  return hipGetLastError();
}

template <typename T>
hipError_t copy(hipStream_t s, const T* src, T* dst, int64_t count) {
  constexpr int W = Vec16<T>::W;
  if (count % W == 0 && aligned16(src) && aligned16(dst)) {
    const int64_t nv = count / W;
    copy_vec_kernel<T><<<blocks_for(nv), kBlock, 0, s>>>(
        reinterpret_cast<const Vec16<T>*>(src), reinterpret_cast<Vec16<T>*>(dst), nv);
    return hipGetLastError();
  }
  copy_kernel<T><<<blocks_for(count), kBlock, 0, s>>>(src, dst, count);
  return hipGetLastError();
}

template <typename T>
hipError_t update_wr(hipStream_t s, T* w, T* r, const T* p, const T* q, const double* gamma,
                     int64_t n, int nrhs) {
  if (sizeof(T) == 4 && n % Vec16<T>::W == 0 && aligned16(w) && aligned16(r) && aligned16(p) &&
      aligned16(q)) {
    const int64_t nv = n / Vec16<T>::W;
    update_wr_vec_kernel<T><<<dim3(blocks_for(nv), nrhs), kBlock, 0, s>>>(
        reinterpret_cast<Vec16<T>*>(w), reinterpret_cast<Vec16<T>*>(r),
        reinterpret_cast<const Vec16<T>*>(p), reinterpret_cast<const Vec16<T>*>(q), gamma, nv);
    return hipGetLastError();
  }
  update_wr_kernel<T><<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(w, r, p, q, gamma, n);
  return hipGetLastError();
}

template <typename T>
hipError_t update_p(hipStream_t s, T* p, const T* z, const double* beta, int64_t n, int nrhs) {
  if (sizeof(T) == 4 && n % Vec16<T>::W == 0 && aligned16(p) && aligned16(z)) {
    const int64_t nv = n / Vec16<T>::W;
    update_p_vec_kernel<T><<<dim3(blocks_for(nv), nrhs), kBlock, 0, s>>>(
        reinterpret_cast<Vec16<T>*>(p), reinterpret_cast<const Vec16<T>*>(z), beta, nv);
    return hipGetLastError();
  }
  update_p_kernel<T><<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(p, z, beta, n);
  return hipGetLastError();
}

hipError_t pcg_start(hipStream_t s, PcgScalars sc, int nrhs, const double* tol, const double* ref) {
  pcg_start_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs, tol, ref);
  return hipGetLastError();
}
hipError_t pack_flags(hipStream_t s, PcgScalars sc, int nrhs, double* out) {
  pack_flags_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs, out);
  return hipGetLastError();
}
hipError_t pcg_gamma(hipStream_t s, PcgScalars sc, int nrhs) {
  pcg_gamma_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs);
  return hipGetLastError();
}
hipError_t pcg_beta(hipStream_t s, PcgScalars sc, int nrhs, int maxit) {
  pcg_beta_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs, maxit);
  return hipGetLastError();
}

template <typename T>
hipError_t pack(hipStream_t s, const double* src, T* dst, int K, int rows) {
  pack_kernel<T><<<dim3(blocks_for(slab_elems(K)), rows), kBlock, 0, s>>>(src, dst, K);
  return hipGetLastError();
}

template <typename T>
hipError_t unpack(hipStream_t s, const T* src, double* dst, int K, int rows) {
  const int64_t nn = (int64_t)grid_n(K) * grid_n(K);
  unpack_kernel<T><<<dim3(blocks_for(nn), rows), kBlock, 0, s>>>(src, dst, K);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t cast(hipStream_t s, const Tin* in, Tout* out, int64_t count) {
  cast_kernel<Tin, Tout><<<blocks_for(count), kBlock, 0, s>>>(in, out, count);
  return hipGetLastError();
}

hipError_t residual64(hipStream_t s, const double* f, const double* q, double* r, int64_t count) {
  residual64_kernel<<<blocks_for(count), kBlock, 0, s>>>(f, q, r, count);
  return hipGetLastError();
}

hipError_t add_correction(hipStream_t s, double* w, const float* d, int64_t n, int nrhs,
                          const int* status) {
  add_correction_kernel<<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(w, d, n, status);
  return hipGetLastError();
}

hipError_t mixed_reset(hipStream_t s, MixedState ms, int nrhs) {
  mixed_reset_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(ms, nrhs);
  return hipGetLastError();
}
hipError_t mixed_adjust(hipStream_t s, PcgScalars sc, MixedState ms, int nrhs, const double* tol,
                        double inner_tol, int k, bool last) {
  mixed_adjust_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, ms, nrhs, tol, inner_tol, k,
                                                          last ? 1 : 0);
  return hipGetLastError();
}
hipError_t mixed_inner_done(hipStream_t s, PcgScalars sc, MixedState ms, int nrhs) {
  mixed_inner_done_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, ms, nrhs);
  return hipGetLastError();
}

hipError_t inject(hipStream_t s, const double* src, double* dst, int Kf, int d, int rows_f,
                  int rows_c, int tstride, int nrhs) {
  const dim3 grid(blocks_for(slab_elems(Kf - d)), rows_c, nrhs);
  inject_kernel<<<grid, kBlock, 0, s>>>(src, dst, Kf, d, rows_f, rows_c, tstride);
  return hipGetLastError();
}

hipError_t prolong_w(hipStream_t s, const double* wc, double* wf, int J, int K, int nrhs) {
  const dim3 grid(blocks_for(slab_elems(K)), (1 << J) + 1, nrhs);
  prolong_w_kernel<<<grid, kBlock, 0, s>>>(wc, wf, J, K);
  return hipGetLastError();
}

hipError_t fill_level_sigma(hipStream_t s, double* sigma, int J, int nrhs) {
  const int64_t count = (int64_t)nrhs * ((1 << J) + 1);
  fill_level_sigma_kernel<<<blocks_for(count), kBlock, 0, s>>>(sigma, J, nrhs);
  return hipGetLastError();
}

// ---------------------------------------------------------- instantiations
#define STP_INSTANTIATE(T)                                                                        \
  template hipError_t apply_A<T>(hipStream_t, const T*, T*, int, int, const SpaceOp&);            \
  template hipError_t apply_M<T>(hipStream_t, const T*, T*, int, int);                            \
  template hipError_t wavelet<T>(hipStream_t, T*, int, int64_t, int, bool, const int*);           \
  template hipError_t synthesis<T>(hipStream_t, const T*, T*, int, int64_t, int, const int*);     \
  template hipError_t synthesis_update<T>(hipStream_t, T*, const T*, const double*, T*, int,      \
                                          int64_t, int, const int*);                              \
  template hipError_t analysis_dot<T>(hipStream_t, T*, const T*, double*, double*, int, int64_t, \
                                      int);                                                       \
  template hipError_t dot<T>(hipStream_t, const T*, const T*, int64_t, int, double*, double*);    \
  template hipError_t copy<T>(hipStream_t, const T*, T*, int64_t);                                \
  template hipError_t update_wr<T>(hipStream_t, T*, T*, const T*, const T*, const double*,        \
                                   int64_t, int);                                                \
  template hipError_t update_p<T>(hipStream_t, T*, const T*, const double*, int64_t, int);        \
  template hipError_t pack<T>(hipStream_t, const double*, T*, int, int);                          \
  template hipError_t unpack<T>(hipStream_t, const T*, double*, int, int);

STP_INSTANTIATE(double)
STP_INSTANTIATE(float)
template hipError_t cast<double, float>(hipStream_t, const double*, float*, int64_t);
template hipError_t cast<float, double>(hipStream_t, const float*, double*, int64_t);

}  // namespace stp
