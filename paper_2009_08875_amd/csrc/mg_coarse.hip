// Whole V-cycles on the coarse grids, one workgroup per time row, in LDS.
//
// The streaming kernels (mg_stream.hip) need a grid wide enough to keep a
// wavefront busy; on grids of at most 31 x 31 nodes their launches are short
// and the cycle becomes a chain of ~20 launch latencies.  This kernel runs
// the part of a V-cycle on levels L..1 (L <= kCoarseLevels) of one time row
// in a single workgroup: the right-hand side is read from HBM once, every
// level's iterate and right-hand side live in LDS, and the result (or A_x
// applied to it) is written once.  The schedule is the one the streaming
// kernels follow (Section 3.1, Section 5.1: three Gauss-Seidel steps in the
// colours (i + j) mod 3 -- forward 0, 1, 2 before the coarse grid, backward
// 2, 1, 0 after it -- the residual restricted by P^T, the coarse correction
// prolongated by P1 interpolation on the "/" mesh, the one-node grid solved
// exactly), so the operator is the same.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tune.h"

namespace stp {

namespace {


struct LevelCoef {
  double c0, cx, cy, c2;  // centre, x- and y-neighbours, the two "/" diagonal neighbours
  double inv_c0;
  bool iso;               // cx == cy: the four axis neighbours share one coefficient
};

__device__ __forceinline__ LevelCoef level_coef(double a, double sigma, int l, const SpaceOp& op) {
  const Stencil st = stencil_of(op, a, sigma, l);
  return {st.c0, st.cx, st.cy, st.cd, 1.0 / st.c0, st.cx == st.cy};
}



// Compact n x n arrays in LDS; node (i, j), 1-based, at (j - 1) n + (i - 1).
template <typename T>
__device__ __forceinline__ T at(const T* v, int n, int i, int j) {
  return (i >= 1 && i <= n && j >= 1 && j <= n) ? v[(j - 1) * n + (i - 1)] : T(0);
}

// sum_nb C_nb x_nb at node (i, j) (the off-centre part of the stencil)
template <typename T>
__device__ __forceinline__ T off_centre(const T* x, int n, int i, int j, const LevelCoef& cf) {
  const T diag = T(cf.c2) * (at(x, n, i + 1, j + 1) + at(x, n, i - 1, j - 1));
  if (cf.iso)
    return T(cf.cx) * (((at(x, n, i + 1, j) + at(x, n, i - 1, j)) + at(x, n, i, j + 1)) +
                       at(x, n, i, j - 1)) +
           diag;
  return (T(cf.cx) * (at(x, n, i + 1, j) + at(x, n, i - 1, j)) +
          T(cf.cy) * (at(x, n, i, j + 1) + at(x, n, i, j - 1))) +
         diag;
}

// One colour of Gauss-Seidel: every node (i, j) with (i + j) mod 3 == colour
// gets (b - sum_nb C_nb x_nb) / C_centre from the current neighbours (no two
// nodes of one colour are coupled, so the update is in place).
template <int NT, typename T>
__device__ void relax(T* x, const T* b, int n, int colour, const LevelCoef& cf) {
  const int m = (n + 2) / 3;  // nodes of one colour per grid line, at most
  for (int k = threadIdx.x; k < n * m; k += NT) {
    const int j = k / m + 1;
    int i = ((colour - j) % 3 + 3) % 3;
    if (i == 0) i = 3;
    i += 3 * (k % m);
    if (i > n) continue;
    const T off = off_centre(x, n, i, j, cf);
    x[(j - 1) * n + (i - 1)] = (b[(j - 1) * n + (i - 1)] - off) * T(cf.inv_c0);
  }
}

template <int NT, typename T>
__device__ void sweeps(T* x, const T* b, int n, const LevelCoef& cf, bool forward) {
  for (int s = 0; s < 3; ++s) {
    for (int c = 0; c < 3; ++c) {
      relax<NT>(x, b, n, forward ? c : 2 - c, cf);
      __syncthreads();
    }
  }
}

// NT threads per workgroup (one time row each); the result does not depend on NT.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void mg_coarse_kernel(const T* xin, const T* b, T* xout,
                                                             int L, double a,
                                                             const double* __restrict__ sigma,
                                                             int write_Ax, SpaceOp op) {
  extern __shared__ unsigned char smem[];
  T* sh = reinterpret_cast<T*>(smem);
  // LDS: x_l and b_l for l = L..1, then a residual array of level L
  auto nl = [](int l) { return (1 << l) - 1; };
  auto off_x = [&](int l) {
    int o = 0;
    for (int k = L; k > l; --k) o += 2 * nl(k) * nl(k);
    return o;
  };
  auto off_b = [&](int l) { return off_x(l) + nl(l) * nl(l); };
  T* r = sh + off_x(0);
  const int row = blockIdx.x;
  const double sg = sigma ? sigma[row] : 0.0;
  const int n = nl(L), pitch = line_pitch(L);
  const int64_t base = (int64_t)row * slab_elems(L);
  for (int k = threadIdx.x; k < n * n; k += NT) {
    const int64_t g = base + (int64_t)(k / n) * pitch + (k % n);
    sh[off_b(L) + k] = b[g];
    sh[off_x(L) + k] = xin ? xin[g] : T(0);
  }
  __syncthreads();
  // down: smooth, residual, restrict
  for (int l = L; l >= 2; --l) {
    const LevelCoef cf = level_coef(a, sg, l, op);
    T* x = sh + off_x(l);
    const T* bl = sh + off_b(l);
    const int nn = nl(l);
    if (l < L) {
      for (int k = threadIdx.x; k < nn * nn; k += NT) x[k] = T(0);
      __syncthreads();
    }
    sweeps<NT>(x, bl, nn, cf, true);
    for (int k = threadIdx.x; k < nn * nn; k += NT) {
      const int i = k % nn + 1, j = k / nn + 1;
      const T cx = T(cf.c0) * x[k] + off_centre(x, nn, i, j, cf);
      r[k] = bl[k] - cx;
    }
    __syncthreads();
    T* bc = sh + off_b(l - 1);
    const int mc = nl(l - 1);
    for (int k = threadIdx.x; k < mc * mc; k += NT) {
      const int I = k % mc + 1, J = k / mc + 1;
      const int i = 2 * I, j = 2 * J;
      const T half = ((((at(r, nn, i + 1, j) + at(r, nn, i - 1, j)) + at(r, nn, i, j + 1)) +
                       at(r, nn, i, j - 1)) +
                      at(r, nn, i + 1, j + 1)) +
                     at(r, nn, i - 1, j - 1);
      bc[k] = at(r, nn, i, j) + T(0.5) * half;
    }
    __syncthreads();
  }
  // the one-node grid (h = 1/2)
  if (threadIdx.x == 0) sh[off_x(1)] = sh[off_b(1)] * T(level_coef(a, sg, 1, op).inv_c0);
  __syncthreads();
  // up: prolongate the correction, smooth backwards
  for (int l = 2; l <= L; ++l) {
    const LevelCoef cf = level_coef(a, sg, l, op);
    T* x = sh + off_x(l);
    const T* e = sh + off_x(l - 1);
    const int nn = nl(l), mc = nl(l - 1);
    for (int k = threadIdx.x; k < nn * nn; k += NT) {
      const int i = k % nn + 1, j = k / nn + 1;
      T p;
      if (!(i & 1) && !(j & 1)) {
        p = at(e, mc, i / 2, j / 2);
      } else if ((i & 1) && !(j & 1)) {
        p = T(0.5) * (at(e, mc, (i - 1) / 2, j / 2) + at(e, mc, (i + 1) / 2, j / 2));
      } else if (!(i & 1) && (j & 1)) {
        p = T(0.5) * (at(e, mc, i / 2, (j - 1) / 2) + at(e, mc, i / 2, (j + 1) / 2));
      } else {
        p = T(0.5) * (at(e, mc, (i - 1) / 2, (j - 1) / 2) + at(e, mc, (i + 1) / 2, (j + 1) / 2));
      }
      x[k] += p;
    }
    __syncthreads();
    sweeps<NT>(x, sh + off_b(l), nn, cf, false);
  }
  const T* x = sh + off_x(L);
  const bool heat = op.heat();
  const LevelCoef ac = level_coef(1.0, 0.0, L, op);  // A_x itself (Section 4)
  for (int k = threadIdx.x; k < n * n; k += NT) {
    const int i = k % n + 1, j = k / n + 1;
    T v = x[k];
    if (write_Ax) {
      if (heat)
        v = (((T(4) * v - at(x, n, i + 1, j)) - at(x, n, i - 1, j)) - at(x, n, i, j + 1)) -
            at(x, n, i, j - 1);
      else
        v = T(ac.c0) * v + off_centre(x, n, i, j, ac);
    }
    xout[base + (int64_t)(j - 1) * pitch + (i - 1)] = v;
  }
}

size_t mg_coarse_lds_bytes(int L, size_t elem) {
  size_t nodes = 0;
  for (int l = L; l >= 1; --l) nodes += 2 * (size_t)((1 << l) - 1) * ((1 << l) - 1);
  nodes += (size_t)((1 << L) - 1) * ((1 << L) - 1);
  return nodes * elem;
}

}  // namespace

template <typename T>
hipError_t mg_coarse_cycle(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows,
                           double a, const double* sigma, bool write_Ax, const SpaceOp& op) {
  if (L < 1 || L > kCoarseLevels) return hipErrorInvalidValue;
  const size_t lds = mg_coarse_lds_bytes(L, sizeof(T));
  // workgroups of 2, 4 or 8 waves per time row (tuned per level and row count)
  auto go = [&](int c) -> hipError_t {
    const int wa = write_Ax ? 1 : 0;
    if (c == 0)
      mg_coarse_kernel<T, 256><<<rows, 256, lds, s>>>(xin, b, xout, L, a, sigma, wa, op);
    else if (c == 1)
      mg_coarse_kernel<T, 128><<<rows, 128, lds, s>>>(xin, b, xout, L, a, sigma, wa, op);
    else
      mg_coarse_kernel<T, 512><<<rows, 512, lds, s>>>(xin, b, xout, L, a, sigma, wa, op);
    return hipGetLastError();
  };
  const uint64_t key = tune_key(3, sizeof(T), (uint64_t)L, (uint64_t)rows);
  // a cycle that starts from its own output cannot be repeated for timing:
  // it takes the choice made for the same shape from zero
  if (xin != nullptr && xin == xout) return go(tuned_choice(key, 0));
  return go(tuned(key, 3, 0, s, go));
}

template hipError_t mg_coarse_cycle<double>(hipStream_t, const double*, const double*, double*,
                                            int, int, double, const double*, bool,
                                            const SpaceOp&);
template hipError_t mg_coarse_cycle<float>(hipStream_t, const float*, const float*, float*, int,
                                           int, double, const double*, bool, const SpaceOp&);

}  // namespace stp
