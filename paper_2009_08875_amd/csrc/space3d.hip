// The three-dimensional problem of Section 5.2 (gfx950): P1 on the Kuhn
// tetrahedral mesh of the unit cube (each of the 2^(3l) cubes of a level cut
// into 6 tetrahedra around its (1, 1, 1) diagonal).  On this mesh the
// stiffness is h times the 7-point Laplacian (6 at the node, -1 at the six
// axis neighbours) and the mass h^3 times the 15-point stencil
// (0.4 at the node, 1/20 at the six axis and the two (1, 1, 1)-diagonal
// neighbours, 1/30 at the six neighbours across the face diagonals (1, 1, 0),
// (1, 0, 1), (0, 1, 1)), the sums of the element matrices of the 24
// tetrahedra around a node.
//
// Kernels run one thread per slab element and time row (a grid-stride loop
// over the rows).  Neighbour values come straight from global memory, which
// the L2 caches; these kernels are written for correctness and a clear
// structure, not tiled like the two-dimensional ones.
//
// Multigrid (K_x and the K_l of Theorem 3.1, Section 5.1's two V-cycles with
// three Gauss-Seidel steps per grid): the colours (i + j + k) mod 4 -- the
// seven edge directions change i + j + k by 1, 2 or 3, so no two nodes of one
// colour are coupled and a colour is relaxed in one launch -- forward
// 0, 1, 2, 3 before the coarse grid and backward 3, 2, 1, 0 after it;
// residual, P^T, the coarse cycle from zero, P1 interpolation; the one-node
// grid solved exactly.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace stp {

namespace {

constexpr int kBlock3 = 256;
constexpr int kMaxGridRows = 65535;

// the 15 mass offsets: the node, +- the seven edge directions
__constant__ int kOff[15][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, 0, 1},
                               {-1, 0, -1}, {0, 1, 1},   {0, -1, -1}, {1, 1, 1},  {-1, -1, -1}};

struct Node3 {
  int i, j, k;  // 1-based
};

__device__ __forceinline__ bool node3_of(int64_t idx, int l, Node3& p) {
  const int n = grid_n(l), pitch = line_pitch(l);
  const int64_t line = idx / pitch;
  p.i = (int)(idx - line * pitch) + 1;
  p.j = (int)(line % n) + 1;
  p.k = (int)(line / n) + 1;
  return p.i <= n && p.k <= n;
}

template <typename T>
__device__ __forceinline__ T at3(const T* s, int l, int i, int j, int k) {
  const int n = grid_n(l);
  if (i < 1 || i > n || j < 1 || j > n || k < 1 || k > n) return T(0);
  return s[((int64_t)(k - 1) * n + (j - 1)) * line_pitch(l) + (i - 1)];
}

// Stencil weights of C = a A_x + sigma M_x on level l, by offset index of kOff.
struct C3 {
  double w[15];
};
__device__ __forceinline__ C3 coef3(double a, double sigma, int l) {
  const double h = 1.0 / (double)(1 << l);
  const double m = sigma * h * h * h;
  C3 c;
  c.w[0] = a * 6.0 * h + 0.4 * m;
  for (int q = 1; q <= 6; ++q) c.w[q] = -a * h + m / 20.0;
  for (int q = 7; q <= 12; ++q) c.w[q] = m / 30.0;
  c.w[13] = c.w[14] = m / 20.0;
  return c;
}

// sum_q w_q x(p + off_q) over the offsets [q0, q1)
template <typename T>
__device__ __forceinline__ T stencil3(const T* s, int l, const Node3& p, const C3& c, int q0,
                                      int q1) {
  T acc = T(0);
  for (int q = q0; q < q1; ++q)
    acc += T(c.w[q]) * at3(s, l, p.i + kOff[q][0], p.j + kOff[q][1], p.k + kOff[q][2]);
  return acc;
}

// thread -> (slab element, row) over a 2D grid, rows in a grid-stride loop
#define FOR_ELEMS_3D(l, rows)                                                     \
  const int64_t idx = (int64_t)blockIdx.x * kBlock3 + threadIdx.x;               \
  if (idx >= slab3_elems(l)) return;                                               \
  for (int row = blockIdx.y; row < (rows); row += gridDim.y)

inline dim3 grid3(int l, int rows) {
  return dim3((unsigned)((slab3_elems(l) + kBlock3 - 1) / kBlock3),
              (unsigned)std::min(rows, kMaxGridRows));
}

template <typename T>
__global__ __launch_bounds__(kBlock3) void pack3_kernel(const double* __restrict__ src,
                                                        T* __restrict__ dst, int K, int rows) {
  const int64_t nx = (int64_t)grid_n(K) * grid_n(K) * grid_n(K);
  FOR_ELEMS_3D(K, rows) {
    Node3 p;
    T v = T(0);
    if (node3_of(idx, K, p))
      v = (T)src[row * nx + ((int64_t)(p.k - 1) * grid_n(K) + (p.j - 1)) * grid_n(K) + (p.i - 1)];
    dst[row * slab3_elems(K) + idx] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock3) void unpack3_kernel(const T* __restrict__ src,
                                                          double* __restrict__ dst, int K,
                                                          int rows) {
  const int64_t nx = (int64_t)grid_n(K) * grid_n(K) * grid_n(K);
  FOR_ELEMS_3D(K, rows) {
    Node3 p;
    if (!node3_of(idx, K, p)) continue;
    dst[row * nx + ((int64_t)(p.k - 1) * grid_n(K) + (p.j - 1)) * grid_n(K) + (p.i - 1)] =
        (double)src[row * slab3_elems(K) + idx];
  }
}

// y = (a A + sigma M) x per row (A: a = 1, sigma = 0; M: a = 0, sigma = 1)
template <typename T>
__global__ __launch_bounds__(kBlock3) void apply3_kernel(const T* __restrict__ x,
                                                         T* __restrict__ y, int K, int rows,
                                                         double a, double sigma) {
  const C3 c = coef3(a, sigma, K);
  FOR_ELEMS_3D(K, rows) {
    Node3 p;
    T v = T(0);
    if (node3_of(idx, K, p)) v = stencil3(x + row * slab3_elems(K), K, p, c, 0, 15);
    y[row * slab3_elems(K) + idx] = v;
  }
}

// The four time combinations of Lemma 4.2 at a node of row i (exact hat
// integrals, one-sided at t = 0 and t = 1).
template <typename T>
struct TC3 {
  T At, Mt, L, LT;
};
template <typename T>
__device__ __forceinline__ TC3<T> tc3(const T* X, int64_t base, int64_t slab, int i, int N, int K,
                                      int a, int b, int c) {
  const T x0 = at3(X + base + (int64_t)i * slab, K, a, b, c);
  const T xm = i > 0 ? at3(X + base + (int64_t)(i - 1) * slab, K, a, b, c) : T(0);
  const T xp = i < N ? at3(X + base + (int64_t)(i + 1) * slab, K, a, b, c) : T(0);
  const T inv_tau = T((double)N), tau6 = T(1.0 / (6.0 * (double)N));
  TC3<T> r;
  if (i == 0) {
    r.At = (x0 - xp) * inv_tau;
    r.Mt = tau6 * (T(2) * x0 + xp);
    r.L = (xp - x0) / T(2);
    r.LT = -(x0 + xp) / T(2);
  } else if (i == N) {
    r.At = (x0 - xm) * inv_tau;
    r.Mt = tau6 * (xm + T(2) * x0);
    r.L = (x0 - xm) / T(2);
    r.LT = (xm + x0) / T(2);
  } else {
    r.At = (T(2) * x0 - xm - xp) * inv_tau;
    r.Mt = tau6 * ((xm + T(4) * x0) + xp);
    r.L = (xp - xm) / T(2);
    r.LT = (xm - xp) / T(2);
  }
  return r;
}

// MODE 0: y1 = M (A_t X) + A (L^T X), y2 = A (M_t X) + M (L X)
// MODE 1: G1 = M (L^T g), G0 = M (M_t g)
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock3) void time_pair3_kernel(const T* __restrict__ X,
                                                             T* __restrict__ y1,
                                                             T* __restrict__ y2, int J, int K,
                                                             int rows) {
  const int N = 1 << J;
  const int64_t slab = slab3_elems(K);
  const C3 ca = coef3(1.0, 0.0, K), cm = coef3(0.0, 1.0, K);
  FOR_ELEMS_3D(K, rows) {
    Node3 p;
    T o1 = T(0), o2 = T(0);
    if (node3_of(idx, K, p)) {
      const int rhs = row / (N + 1), i = row - rhs * (N + 1);
      const int64_t base = (int64_t)rhs * (N + 1) * slab;
      for (int q = 0; q < 15; ++q) {
        const TC3<T> t =
            tc3(X, base, slab, i, N, K, p.i + kOff[q][0], p.j + kOff[q][1], p.k + kOff[q][2]);
        const T wm = T(cm.w[q]), wa = T(ca.w[q]);
        if constexpr (MODE == 0) {
          o1 += wm * t.At + wa * t.LT;
          o2 += wa * t.Mt + wm * t.L;
        } else {
          o1 += wm * t.LT;
          o2 += wm * t.Mt;
        }
      }
    }
    y1[row * slab + idx] = o1;
    y2[row * slab + idx] = o2;
  }
}

// out = M z1 + A z2, plus M e_b in row 0 of right-hand side b
template <typename T>
__global__ __launch_bounds__(kBlock3) void combine3_kernel(const T* __restrict__ z1,
                                                          const T* __restrict__ z2,
                                                          const T* __restrict__ extra,
                                                          int64_t extra_stride, T* __restrict__ out,
                                                          int J, int K, int rows) {
  const int N = 1 << J;
  const int64_t slab = slab3_elems(K);
  const C3 ca = coef3(1.0, 0.0, K), cm = coef3(0.0, 1.0, K);
  FOR_ELEMS_3D(K, rows) {
    Node3 p;
    T v = T(0);
    if (node3_of(idx, K, p)) {
      v = stencil3(z1 + row * slab, K, p, cm, 0, 15) + stencil3(z2 + row * slab, K, p, ca, 0, 7);
      const int rhs = row / (N + 1), i = row - rhs * (N + 1);
      if (i == 0 && extra) v += stencil3(extra + (int64_t)rhs * extra_stride, K, p, cm, 0, 15);
    }
    out[row * slab + idx] = v;
  }
}

// One colour of Gauss-Seidel on level l for C = a A + sigma_row M.
template <typename T>
__global__ __launch_bounds__(kBlock3) void relax3_kernel(T* __restrict__ x,
                                                         const T* __restrict__ b, int l, int rows,
                                                         double a,
                                                         const double* __restrict__ sigma,
                                                         int colour) {
  FOR_ELEMS_3D(l, rows) {
    Node3 p;
    if (!node3_of(idx, l, p) || ((p.i + p.j + p.k) & 3) != colour) continue;
    const C3 c = coef3(a, sigma ? sigma[row] : 0.0, l);
    T* xr = x + row * slab3_elems(l);
    const T off = stencil3(xr, l, p, c, 1, sigma ? 15 : 7);
    xr[idx] = (b[row * slab3_elems(l) + idx] - off) / T(c.w[0]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock3) void residual3_kernel(const T* __restrict__ x,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ r, int l, int rows,
                                                            double a,
                                                            const double* __restrict__ sigma) {
  FOR_ELEMS_3D(l, rows) {
    Node3 p;
    T v = T(0);
    if (node3_of(idx, l, p)) {
      const C3 c = coef3(a, sigma ? sigma[row] : 0.0, l);
      v = b[row * slab3_elems(l) + idx] -
          stencil3(x + row * slab3_elems(l), l, p, c, 0, sigma ? 15 : 7);
    }
    r[row * slab3_elems(l) + idx] = v;
  }
}

// bc (level l - 1) = P^T r (level l): the coarse node's own fine value plus
// half of each of its 14 fine neighbours along the edge directions.
template <typename T>
__global__ __launch_bounds__(kBlock3) void restrict3_kernel(const T* __restrict__ r,
                                                            T* __restrict__ bc, int l, int rows) {
  const int lc = l - 1;
  FOR_ELEMS_3D(lc, rows) {
    Node3 p;
    T v = T(0);
    if (node3_of(idx, lc, p)) {
      const T* rr = r + row * slab3_elems(l);
      const int i = 2 * p.i, j = 2 * p.j, k = 2 * p.k;
      T half = T(0);
      for (int q = 1; q < 15; ++q) half += at3(rr, l, i + kOff[q][0], j + kOff[q][1], k + kOff[q][2]);
      v = at3(rr, l, i, j, k) + T(0.5) * half;
    }
    bc[row * slab3_elems(lc) + idx] = v;
  }
}

// x (level l) += P e (e on level l - 1): fine node (2I + a, 2J + b, 2K + c)
// takes the mean of the coarse ends of the edge it bisects.
template <typename T>
__global__ __launch_bounds__(kBlock3) void prolong_add3_kernel(const T* __restrict__ e,
                                                               T* __restrict__ x, int l, int rows) {
  FOR_ELEMS_3D(l, rows) {
    Node3 p;
    if (!node3_of(idx, l, p)) continue;
    const T* ee = e + row * slab3_elems(l - 1);
    const int a = p.i & 1, b = p.j & 1, c = p.k & 1;
    const int I = p.i >> 1, J = p.j >> 1, Kc = p.k >> 1;
    T v = at3(ee, l - 1, I, J, Kc);
    if (a | b | c) v = T(0.5) * (v + at3(ee, l - 1, I + a, J + b, Kc + c));
    x[row * slab3_elems(l) + idx] += v;
  }
}

// the one-node grid (level 1): x = b / c_0
template <typename T>
__global__ void coarsest3_kernel(const T* __restrict__ b, T* __restrict__ x, int rows, double a,
                                 const double* __restrict__ sigma) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const C3 c = coef3(a, sigma ? sigma[row] : 0.0, 1);
  const int64_t s = slab3_elems(1);
  x[row * s] = b[row * s] / T(c.w[0]);
}

template <typename T>
__global__ __launch_bounds__(kBlock3) void zero3_kernel(T* __restrict__ x, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock3 + threadIdx.x;
  if (i < count) x[i] = T(0);
}

}  // namespace

template <typename T>
hipError_t pack3(hipStream_t s, const double* src, T* dst, int K, int rows) {
  pack3_kernel<T><<<grid3(K, rows), kBlock3, 0, s>>>(src, dst, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t unpack3(hipStream_t s, const T* src, double* dst, int K, int rows) {
  unpack3_kernel<T><<<grid3(K, rows), kBlock3, 0, s>>>(src, dst, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t apply_A3(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply3_kernel<T><<<grid3(K, rows), kBlock3, 0, s>>>(x, y, K, rows, 1.0, 0.0);
  return hipGetLastError();
}
template <typename T>
hipError_t apply_M3(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply3_kernel<T><<<grid3(K, rows), kBlock3, 0, s>>>(x, y, K, rows, 0.0, 1.0);
  return hipGetLastError();
}
template <typename T>
hipError_t time_stencil_pair3(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  time_pair3_kernel<T, 0><<<grid3(K, rows), kBlock3, 0, s>>>(X, y1, y2, J, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t rhs_stencil_pair3(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  time_pair3_kernel<T, 1><<<grid3(K, rows), kBlock3, 0, s>>>(g, G1, G0, J, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t combine3(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                    T* out, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  combine3_kernel<T><<<grid3(K, rows), kBlock3, 0, s>>>(z1, z2, extra, extra_stride, out, J, K,
                                                        rows);
  return hipGetLastError();
}

// V-cycle on level l for x (in place), b; w: level-l residual buffer.
template <typename T>
hipError_t vcycle3(hipStream_t s, const Mg3Work<T>& w, T* x, const T* b, int l, int rows,
                   double a, const double* sigma) {
  const dim3 g = grid3(l, rows);
  for (int sw = 0; sw < 3; ++sw)
    for (int c = 0; c < 4; ++c) relax3_kernel<T><<<g, kBlock3, 0, s>>>(x, b, l, rows, a, sigma, c);
  residual3_kernel<T><<<g, kBlock3, 0, s>>>(x, b, w.r[l], l, rows, a, sigma);
  restrict3_kernel<T><<<grid3(l - 1, rows), kBlock3, 0, s>>>(w.r[l], w.b[l - 1], l, rows);
  if (l - 1 == 1) {
    coarsest3_kernel<T><<<(rows + 63) / 64, 64, 0, s>>>(w.b[1], w.x[1], rows, a, sigma);
  } else {
    const int64_t cnt = (int64_t)rows * slab3_elems(l - 1);
    zero3_kernel<T><<<(unsigned)((cnt + kBlock3 - 1) / kBlock3), kBlock3, 0, s>>>(w.x[l - 1], cnt);
    const hipError_t e = vcycle3<T>(s, w, w.x[l - 1], w.b[l - 1], l - 1, rows, a, sigma);
    if (e != hipSuccess) return e;
  }
  prolong_add3_kernel<T><<<g, kBlock3, 0, s>>>(w.x[l - 1], x, l, rows);
  for (int sw = 0; sw < 3; ++sw)
    for (int c = 3; c >= 0; --c) relax3_kernel<T><<<g, kBlock3, 0, s>>>(x, b, l, rows, a, sigma, c);
  return hipGetLastError();
}

template <typename T>
hipError_t mg3_apply(hipStream_t s, const Mg3Work<T>& w, const T* b, T* x, int K, int rows,
                     double a, const double* sigma, int vcycles, bool write_Ax) {
  T* xk = write_Ax ? w.x[K] : x;
  const int64_t cnt = (int64_t)rows * slab3_elems(K);
  zero3_kernel<T><<<(unsigned)((cnt + kBlock3 - 1) / kBlock3), kBlock3, 0, s>>>(xk, cnt);
  if (K == 1) {
    coarsest3_kernel<T><<<(rows + 63) / 64, 64, 0, s>>>(b, xk, rows, a, sigma);
  } else {
    for (int c = 0; c < vcycles; ++c) {
      const hipError_t e = vcycle3<T>(s, w, xk, b, K, rows, a, sigma);
      if (e != hipSuccess) return e;
    }
  }
  if (write_Ax) return apply_A3<T>(s, xk, x, K, rows);
  return hipGetLastError();
}

#define STP_INSTANTIATE_3D(T)                                                                      \
  template hipError_t pack3<T>(hipStream_t, const double*, T*, int, int);                          \
  template hipError_t unpack3<T>(hipStream_t, const T*, double*, int, int);                        \
  template hipError_t apply_A3<T>(hipStream_t, const T*, T*, int, int);                            \
  template hipError_t apply_M3<T>(hipStream_t, const T*, T*, int, int);                            \
  template hipError_t time_stencil_pair3<T>(hipStream_t, const T*, T*, T*, int, int, int);         \
  template hipError_t rhs_stencil_pair3<T>(hipStream_t, const T*, T*, T*, int, int, int);          \
  template hipError_t combine3<T>(hipStream_t, const T*, const T*, const T*, int64_t, T*, int, int, \
                                  int);                                                           \
  template hipError_t mg3_apply<T>(hipStream_t, const Mg3Work<T>&, const T*, T*, int, int, double, \
                                   const double*, int, bool);
STP_INSTANTIATE_3D(double)
STP_INSTANTIATE_3D(float)

}  // namespace stp
