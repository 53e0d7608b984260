// HIP kernels of the space-time solver for gfx950 (MI355X).
//
// All operators are constant-coefficient stencils on uniform grids, so no
// matrix is stored: every kernel reads its input once per needed element and
// recomputes coefficients from the mesh width.  The hot kernels are the fused
// multigrid smoothing kernels; see mg_pre_kernel for their tiling scheme.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace stp {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t count, int per_block = kBlock) {
  return (unsigned)((count + per_block - 1) / per_block);
}

// Stencil coefficients of C = a A_x + sigma M_x on mesh width h = 2^-l:
// centre 4a + sigma h^2/2, axis neighbours -a + sigma h^2/12, and the two
// neighbours across the "/" diagonal sigma h^2/12.
struct Coef {
  double c0, c1, c2;
};
__device__ inline Coef coefficients(double a, double sigma, int l) {
  double h = 1.0 / (double)(1 << l);
  double m = h * h / 12.0;
  return {4.0 * a + 6.0 * m * sigma, -a + m * sigma, m * sigma};
}

// ---------------------------------------------------------------- multigrid
//
// A workgroup owns a TW x TH tile of one slab and stages it in LDS together
// with a halo of H nodes.  The three-colour Gauss-Seidel phases run in LDS;
// phase p (0-based) updates only the region whose distance to the LDS border
// is at least p + 1, so after 3 steps x 3 colours the values are exact (equal
// to a global sweep) at distance >= 9 from the border.  The pre-smoothing
// kernel additionally needs the residual one node further out and the
// restriction one more, hence H = 11 there and H = 9 in the post-smoothing
// kernel.  Overlapping halos are recomputed redundantly by neighbouring tiles;
// every tile computes the same value for a node (same operands, same order),
// so the result does not depend on the tiling.

constexpr int kSweeps = 3;
constexpr int kHpre = 3 * kSweeps + 2;
constexpr int kHpost = 3 * kSweeps;

template <typename T, int W, int HH>
__device__ inline void relax_colour(T (*xs)[W], const T (*bs)[W], int c, int lo, int hix, int hiy,
                                    int gx0, int gy0, int n, T c0inv, T c1, T c2) {
  const int r = threadIdx.x & 31;
  const int q = threadIdx.x >> 5;
  for (int ly = lo + q; ly <= hiy; ly += kBlock / 32) {
    const int gy = gy0 + ly;
    if (gy < 1 || gy > n) continue;
    const int first = lo + (((c - gy - gx0 - lo) % 3) + 3) % 3;
    for (int lx = first + 3 * r; lx <= hix; lx += 96) {
      const int gx = gx0 + lx;
      if (gx < 1 || gx > n) continue;
      T off = c1 * (((xs[ly][lx + 1] + xs[ly][lx - 1]) + xs[ly + 1][lx]) + xs[ly - 1][lx]) +
              c2 * (xs[ly + 1][lx + 1] + xs[ly - 1][lx - 1]);
      xs[ly][lx] = (bs[ly][lx] - off) * c0inv;
    }
  }
}

template <typename T, int TW, int TH>
__global__ __launch_bounds__(kBlock) void mg_pre_kernel(const T* __restrict__ xin,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ xout, T* __restrict__ bc,
                                                        int l, int tiles_x, double a,
                                                        const double* __restrict__ sigma) {
  constexpr int H = kHpre;
  constexpr int W = TW + 2 * H;
  constexpr int HH = TH + 2 * H;
  __shared__ T xs[HH][W];
  __shared__ T bs[HH][W];

  const int row = blockIdx.y;
  const int tx = blockIdx.x % tiles_x;
  const int ty = blockIdx.x / tiles_x;
  const int n = grid_n(l);
  const int pitch = line_pitch(l);
  const int64_t slab = slab_elems(l);
  const int nc = grid_n(l - 1);
  const int pitch_c = line_pitch(l - 1);
  const int64_t slab_c = slab_elems(l - 1);
  const int gx0 = 1 + tx * TW - H;  // node coordinates of LDS cell (0, 0)
  const int gy0 = 1 + ty * TH - H;

  const T* xr = xin ? xin + (int64_t)row * slab : nullptr;
  const T* br = b + (int64_t)row * slab;
  for (int idx = threadIdx.x; idx < W * HH; idx += kBlock) {
    const int ly = idx / W, lx = idx - (idx / W) * W;
    const int gx = gx0 + lx, gy = gy0 + ly;
    const bool in = gx >= 1 && gx <= n && gy >= 1 && gy <= n;
    const int64_t off = (int64_t)(gy - 1) * pitch + (gx - 1);
    xs[ly][lx] = (in && xr) ? xr[off] : T(0);
    bs[ly][lx] = in ? br[off] : T(0);
  }
  __syncthreads();

  const Coef cf = coefficients(a, sigma ? sigma[row] : 0.0, l);
  const T c0 = (T)cf.c0, c0inv = (T)(1.0 / cf.c0), c1 = (T)cf.c1, c2 = (T)cf.c2;

  for (int sw = 0; sw < kSweeps; ++sw) {
    for (int c = 0; c < 3; ++c) {
      const int p = sw * 3 + c;
      relax_colour<T, W, HH>(xs, bs, c, p + 1, W - 2 - p, HH - 2 - p, gx0, gy0, n, c0inv, c1, c2);
      __syncthreads();
    }
  }

  // residual r = b - C x, in place of b, on the nodes the restriction reads
  for (int idx = threadIdx.x; idx < (TW + 2) * (TH + 2); idx += kBlock) {
    const int ly = H - 1 + idx / (TW + 2);
    const int lx = H - 1 + idx % (TW + 2);
    const int gx = gx0 + lx, gy = gy0 + ly;
    T r = T(0);
    if (gx >= 1 && gx <= n && gy >= 1 && gy <= n) {
      T off = c1 * (((xs[ly][lx + 1] + xs[ly][lx - 1]) + xs[ly + 1][lx]) + xs[ly - 1][lx]) +
              c2 * (xs[ly + 1][lx + 1] + xs[ly - 1][lx - 1]);
      r = bs[ly][lx] - (c0 * xs[ly][lx] + off);
    }
    bs[ly][lx] = r;
  }

  // smoothed x of the tile interior
  T* xo = xout + (int64_t)row * slab;
  for (int idx = threadIdx.x; idx < TW * TH; idx += kBlock) {
    const int ly = H + idx / TW, lx = H + idx % TW;
    const int gx = gx0 + lx, gy = gy0 + ly;
    if (gx <= n && gy <= n) xo[(int64_t)(gy - 1) * pitch + (gx - 1)] = xs[ly][lx];
  }
  __syncthreads();

  // restriction: coarse node (I, J) sits at fine node (2I, 2J) and collects its
  // residual plus half of each of the six neighbours' residuals
  T* bco = bc + (int64_t)row * slab_c;
  for (int idx = threadIdx.x; idx < (TW / 2) * (TH / 2); idx += kBlock) {
    const int I = 1 + tx * (TW / 2) + idx % (TW / 2);
    const int J = 1 + ty * (TH / 2) + idx / (TW / 2);
    if (I > nc || J > nc) continue;
    const int lx = 2 * I - gx0, ly = 2 * J - gy0;
    T half = ((((bs[ly][lx + 1] + bs[ly][lx - 1]) + bs[ly + 1][lx]) + bs[ly - 1][lx]) +
              bs[ly + 1][lx + 1]) +
             bs[ly - 1][lx - 1];
    bco[(int64_t)(J - 1) * pitch_c + (I - 1)] = bs[ly][lx] + T(0.5) * half;
  }
}

template <typename T>
__device__ inline T coarse_at(const T* ec, int I, int J, int nc, int pitch_c) {
  return (I >= 1 && I <= nc && J >= 1 && J <= nc) ? ec[(int64_t)(J - 1) * pitch_c + (I - 1)] : T(0);
}

template <typename T, int TW, int TH>
__global__ __launch_bounds__(kBlock) void mg_post_kernel(const T* __restrict__ xin,
                                                         const T* __restrict__ b,
                                                         const T* __restrict__ ec,
                                                         T* __restrict__ xout, int l, int tiles_x,
                                                         double a,
                                                         const double* __restrict__ sigma) {
  constexpr int H = kHpost;
  constexpr int W = TW + 2 * H;
  constexpr int HH = TH + 2 * H;
  __shared__ T xs[HH][W];
  __shared__ T bs[HH][W];

  const int row = blockIdx.y;
  const int tx = blockIdx.x % tiles_x;
  const int ty = blockIdx.x / tiles_x;
  const int n = grid_n(l);
  const int pitch = line_pitch(l);
  const int64_t slab = slab_elems(l);
  const int nc = grid_n(l - 1);
  const int pitch_c = line_pitch(l - 1);
  const int64_t slab_c = slab_elems(l - 1);
  const int gx0 = 1 + tx * TW - H;
  const int gy0 = 1 + ty * TH - H;

  const T* xr = xin + (int64_t)row * slab;
  const T* br = b + (int64_t)row * slab;
  const T* er = ec + (int64_t)row * slab_c;
  for (int idx = threadIdx.x; idx < W * HH; idx += kBlock) {
    const int ly = idx / W, lx = idx - (idx / W) * W;
    const int gx = gx0 + lx, gy = gy0 + ly;
    T xv = T(0), bv = T(0);
    if (gx >= 1 && gx <= n && gy >= 1 && gy <= n) {
      const int64_t off = (int64_t)(gy - 1) * pitch + (gx - 1);
      bv = br[off];
      // x + P e: P1 interpolation of the coarse correction on the "/" mesh
      const int I = gx >> 1, J = gy >> 1;
      T e;
      if (!(gx & 1) && !(gy & 1)) {
        e = coarse_at(er, I, J, nc, pitch_c);
      } else if ((gx & 1) && !(gy & 1)) {
        e = T(0.5) * (coarse_at(er, I, J, nc, pitch_c) + coarse_at(er, I + 1, J, nc, pitch_c));
      } else if (!(gx & 1) && (gy & 1)) {
        e = T(0.5) * (coarse_at(er, I, J, nc, pitch_c) + coarse_at(er, I, J + 1, nc, pitch_c));
      } else {
        e = T(0.5) * (coarse_at(er, I, J, nc, pitch_c) + coarse_at(er, I + 1, J + 1, nc, pitch_c));
      }
      xv = xr[off] + e;
    }
    xs[ly][lx] = xv;
    bs[ly][lx] = bv;
  }
  __syncthreads();

  const Coef cf = coefficients(a, sigma ? sigma[row] : 0.0, l);
  const T c0inv = (T)(1.0 / cf.c0), c1 = (T)cf.c1, c2 = (T)cf.c2;
  for (int sw = 0; sw < kSweeps; ++sw) {
    for (int cc = 0; cc < 3; ++cc) {
      const int p = sw * 3 + cc;
      relax_colour<T, W, HH>(xs, bs, 2 - cc, p + 1, W - 2 - p, HH - 2 - p, gx0, gy0, n, c0inv, c1,
                             c2);
      __syncthreads();
    }
  }

  T* xo = xout + (int64_t)row * slab;
  for (int idx = threadIdx.x; idx < TW * TH; idx += kBlock) {
    const int ly = H + idx / TW, lx = H + idx % TW;
    const int gx = gx0 + lx, gy = gy0 + ly;
    if (gx <= n && gy <= n) xo[(int64_t)(gy - 1) * pitch + (gx - 1)] = xs[ly][lx];
  }
}

template <typename T>
__global__ void mg_coarsest_kernel(const T* __restrict__ b, T* __restrict__ x, int rows, double a,
                                   const double* __restrict__ sigma) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const double sg = sigma ? sigma[row] : 0.0;
  const double c0 = 4.0 * a + sg / 8.0;  // h = 1/2: sigma h^2 / 2 = sigma / 8
  const int64_t slab = slab_elems(1);
  x[(int64_t)row * slab] = (T)((double)b[(int64_t)row * slab] / c0);
}

template <typename T>
struct TileShape;
template <>
struct TileShape<double> {
  static constexpr int TW = 32, TH = 32;
};
template <>
struct TileShape<float> {
  static constexpr int TW = 32, TH = 32;
};

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

template <typename T, bool IS_A>
__global__ __launch_bounds__(kBlock) void apply_AM_kernel(const T* __restrict__ x,
                                                          T* __restrict__ y, int K) {
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
  y[row * slab + idx] = IS_A ? A_at(x + row * slab, gx, gy, n, pitch)
                             : M_at(x + row * slab, gx, gy, n, pitch, m12);
}

// ------------------------------------------------------------------ wavelet
//
// One thread per slab element (a column along time); the column is processed
// level by level in place, each level as a single left-to-right pass that
// keeps the old value of the current even node in registers.
__device__ inline double boundary_weight(int e, int N) { return (e == 0 || e == N) ? 1.0 : 0.5; }

template <typename T>
__global__ __launch_bounds__(kBlock) void wavelet_kernel(T* __restrict__ X, int J, int K,
                                                         bool synthesis) {
  const int64_t slab = slab_elems(K);
  const int64_t col = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (col >= slab) return;
  const int N = 1 << J;
  T* base = X + (int64_t)blockIdx.y * (N + 1) * slab + col;
  if (synthesis) {
    for (int l = 1; l <= J; ++l) {
      const int s = N >> l;
      const T c = (T)exp2(0.5 * (double)l);
      T e_old = base[0];
      T e_acc = e_old;
      for (int m = s; m < N; m += 2 * s) {
        const T d = base[(int64_t)m * slab];
        const T r_old = base[(int64_t)(m + s) * slab];
        base[(int64_t)m * slab] = T(0.5) * (e_old + r_old) + c * d;
        e_acc -= c * T(boundary_weight(m - s, N)) * d;
        base[(int64_t)(m - s) * slab] = e_acc;
        e_old = r_old;
        e_acc = r_old - c * T(boundary_weight(m + s, N)) * d;
      }
      base[(int64_t)N * slab] = e_acc;
    }
  } else {
    for (int l = J; l >= 1; --l) {
      const int s = N >> l;
      const T c = (T)exp2(0.5 * (double)l);
      T e_old = base[0];
      T e_acc = e_old;
      for (int m = s; m < N; m += 2 * s) {
        const T yo = base[(int64_t)m * slab];
        const T r_old = base[(int64_t)(m + s) * slab];
        base[(int64_t)m * slab] =
            c * ((yo - T(boundary_weight(m - s, N)) * e_old) - T(boundary_weight(m + s, N)) * r_old);
        e_acc += T(0.5) * yo;
        base[(int64_t)(m - s) * slab] = e_acc;
        e_old = r_old;
        e_acc = r_old + T(0.5) * yo;
      }
      base[(int64_t)N * slab] = e_acc;
    }
  }
}

// ------------------------------------------------------------ reductions

__device__ inline double block_sum(double v) {
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

__global__ void pcg_start_kernel(PcgScalars sc, int nrhs, double tol) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrhs) return;
  const double rho = sc.rhonew[b];
  sc.rho[b] = rho;
  sc.rho0[b] = rho;
  sc.its[b] = 0;
  sc.gamma[b] = 0.0;
  sc.beta[b] = 0.0;
  sc.target[b] = tol > 0.0 ? tol * sqrt(rho) : 0.0;
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

__global__ void pcg_beta_kernel(PcgScalars sc, int nrhs) {
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
  }
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

__global__ __launch_bounds__(kBlock) void add_correction_kernel(double* __restrict__ w,
                                                                const float* __restrict__ d,
                                                                int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) w[i] += (double)d[i];
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
hipError_t mg_pre(hipStream_t s, const T* xin, const T* b, T* xout, T* bc, int l, int rows,
                  double a, const double* sigma) {
  constexpr int TW = TileShape<T>::TW, TH = TileShape<T>::TH;
  const int n = grid_n(l);
  const int tiles_x = (n + TW - 1) / TW, tiles_y = (n + TH - 1) / TH;
  mg_pre_kernel<T, TW, TH><<<dim3(tiles_x * tiles_y, rows), kBlock, 0, s>>>(xin, b, xout, bc, l,
                                                                            tiles_x, a, sigma);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_post(hipStream_t s, const T* xin, const T* b, const T* ec, T* xout, int l, int rows,
                   double a, const double* sigma) {
  constexpr int TW = TileShape<T>::TW, TH = TileShape<T>::TH;
  const int n = grid_n(l);
  const int tiles_x = (n + TW - 1) / TW, tiles_y = (n + TH - 1) / TH;
  mg_post_kernel<T, TW, TH><<<dim3(tiles_x * tiles_y, rows), kBlock, 0, s>>>(xin, b, ec, xout, l,
                                                                             tiles_x, a, sigma);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_coarsest(hipStream_t s, const T* b, T* x, int rows, double a, const double* sigma) {
  mg_coarsest_kernel<T><<<blocks_for(rows), kBlock, 0, s>>>(b, x, rows, a, sigma);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_A(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply_AM_kernel<T, true><<<dim3(blocks_for(slab_elems(K)), rows), kBlock, 0, s>>>(x, y, K);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_M(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply_AM_kernel<T, false><<<dim3(blocks_for(slab_elems(K)), rows), kBlock, 0, s>>>(x, y, K);
  return hipGetLastError();
}

template <typename T>
hipError_t wavelet(hipStream_t s, T* X, int J, int K, int nrhs, bool synthesis) {
  if (J == 0) return hipSuccess;
  wavelet_kernel<T><<<dim3(blocks_for(slab_elems(K)), nrhs), kBlock, 0, s>>>(X, J, K, synthesis);
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
  dot_partial_kernel<T><<<dim3(nblk, nrhs), kBlock, 0, s>>>(a, b, n, partials);
  dot_final_kernel<<<nrhs, kBlock, 0, s>>>(partials, nblk, out);
  return hipGetLastError();
}

template <typename T>
hipError_t copy(hipStream_t s, const T* src, T* dst, int64_t count) {
  copy_kernel<T><<<blocks_for(count), kBlock, 0, s>>>(src, dst, count);
  return hipGetLastError();
}

template <typename T>
hipError_t update_wr(hipStream_t s, T* w, T* r, const T* p, const T* q, const double* gamma,
                     int64_t n, int nrhs) {
  update_wr_kernel<T><<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(w, r, p, q, gamma, n);
  return hipGetLastError();
}

template <typename T>
hipError_t update_p(hipStream_t s, T* p, const T* z, const double* beta, int64_t n, int nrhs) {
  update_p_kernel<T><<<dim3(blocks_for(n), nrhs), kBlock, 0, s>>>(p, z, beta, n);
  return hipGetLastError();
}

hipError_t pcg_start(hipStream_t s, PcgScalars sc, int nrhs, double tol) {
  pcg_start_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs, tol);
  return hipGetLastError();
}
hipError_t pcg_gamma(hipStream_t s, PcgScalars sc, int nrhs) {
  pcg_gamma_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs);
  return hipGetLastError();
}
hipError_t pcg_beta(hipStream_t s, PcgScalars sc, int nrhs) {
  pcg_beta_kernel<<<blocks_for(nrhs, 64), 64, 0, s>>>(sc, nrhs);
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

hipError_t add_correction(hipStream_t s, double* w, const float* d, int64_t count) {
  add_correction_kernel<<<blocks_for(count), kBlock, 0, s>>>(w, d, count);
  return hipGetLastError();
}

hipError_t fill_level_sigma(hipStream_t s, double* sigma, int J, int nrhs) {
  const int64_t count = (int64_t)nrhs * ((1 << J) + 1);
  fill_level_sigma_kernel<<<blocks_for(count), kBlock, 0, s>>>(sigma, J, nrhs);
  return hipGetLastError();
}

// ---------------------------------------------------------- instantiations
#define STP_INSTANTIATE(T)                                                                        \
  template hipError_t mg_pre<T>(hipStream_t, const T*, const T*, T*, T*, int, int, double,       \
                                const double*);                                                  \
  template hipError_t mg_post<T>(hipStream_t, const T*, const T*, const T*, T*, int, int, double, \
                                 const double*);                                                 \
  template hipError_t mg_coarsest<T>(hipStream_t, const T*, T*, int, double, const double*);      \
  template hipError_t apply_A<T>(hipStream_t, const T*, T*, int, int);                            \
  template hipError_t apply_M<T>(hipStream_t, const T*, T*, int, int);                            \
  template hipError_t wavelet<T>(hipStream_t, T*, int, int, int, bool);                           \
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
