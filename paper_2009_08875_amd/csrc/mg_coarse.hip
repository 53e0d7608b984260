// Whole V-cycles on small grids, one workgroup per time row, in LDS.
//
// The streaming kernels (mg_stream.hip) need a grid wide enough to keep a
// wavefront busy; on small grids their launches are short and the cycle
// becomes a chain of launch latencies.  This kernel runs V-cycles on levels
// L..1 of one time row in a single workgroup: the right-hand side is read
// from HBM once, every level's iterate and right-hand side live in LDS, and
// the result (or A_x applied to it) is written once, after all the cycles
// asked for.  The schedule is the one the streaming kernels follow (Section
// 3.1, Section 5.1: three Gauss-Seidel steps in the colours (i + j) mod 3 --
// forward 0, 1, 2 before the coarse grid, backward 2, 1, 0 after it -- the
// residual restricted by P^T, the coarse correction prolongated by P1
// interpolation on the "/" mesh, the one-node grid solved exactly), so the
// operator is the same.
//
// Every level is a template parameter: grid sizes, line pitches and the
// divisions that map a thread's work item to a node are compile-time
// constants.  Each level's arrays are stored with a one-node zero border
// ((n + 2) x (n + 2)), so a stencil reads its neighbours without bounds
// checks; the border is never written.  A border read returns the zero that
// a bounds check would, so the arithmetic is the same value for value.
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

// Level l: n x n interior nodes in an (n + 2) x (n + 2) array; node (i, j),
// 1-based, at j (n + 2) + i.
template <int l>
struct Lv {
  static constexpr int n = (1 << l) - 1;
  static constexpr int p = n + 2;
  static constexpr int size = p * p;
  static constexpr int m = (n + 2) / 3;  // nodes of one colour per grid line, at most
};

// LDS layout for top level L: x_l then b_l for l = L..1, then the residual
// array of level L.
template <int L>
struct Layout {
  static constexpr int x(int l) {
    int o = 0;
    for (int k = L; k > l; --k) o += 2 * (((1 << k) + 1) * ((1 << k) + 1));
    return o;
  }
  static constexpr int b(int l) { return x(l) + ((1 << l) + 1) * ((1 << l) + 1); }
  static constexpr int r = x(0);
  static constexpr int total = r + ((1 << L) + 1) * ((1 << L) + 1);
};

// sum_nb C_nb x_nb at the node at offset q (the off-centre part of the stencil)
template <int l, typename T>
__device__ __forceinline__ T off_centre(const T* x, int q, const LevelCoef& cf) {
  constexpr int p = Lv<l>::p;
  const T diag = T(cf.c2) * (x[q + p + 1] + x[q - p - 1]);
  if (cf.iso) return T(cf.cx) * (((x[q + 1] + x[q - 1]) + x[q + p]) + x[q - p]) + diag;
  return (T(cf.cx) * (x[q + 1] + x[q - 1]) + T(cf.cy) * (x[q + p] + x[q - p])) + diag;
}

// One colour of Gauss-Seidel: every node (i, j) with (i + j) mod 3 == colour
// gets (b - sum_nb C_nb x_nb) / C_centre from the current neighbours (no two
// nodes of one colour are coupled, so the update is in place).
template <int l, int NT, typename T>
__device__ __forceinline__ void relax(T* x, const T* b, int colour, const LevelCoef& cf) {
  constexpr int n = Lv<l>::n, m = Lv<l>::m, p = Lv<l>::p;
  for (int k = threadIdx.x; k < n * m; k += NT) {
    const int j = k / m + 1;
    int i = (colour + 3 * n - j) % 3;
    if (i == 0) i = 3;
    i += 3 * (k % m);
    if (i > n) continue;
    const int q = j * p + i;
    x[q] = (b[q] - off_centre<l>(x, q, cf)) * T(cf.inv_c0);
  }
}

template <int l, int NT, typename T>
__device__ void sweeps(T* x, const T* b, const LevelCoef& cf, bool forward) {
  for (int s = 0; s < 3; ++s) {
    for (int c = 0; c < 3; ++c) {
      relax<l, NT>(x, b, forward ? c : 2 - c, cf);
      __syncthreads();
    }
  }
}

// Down the V-cycle from level l: smooth, residual, P^T into level l - 1,
// the cycle below, then P1 interpolation of its correction and backward
// smoothing.  x_l holds the start iterate (zero below the top level).
template <int L, int l, int NT, typename T>
__device__ void vcycle(T* sh, double a, double sg, const SpaceOp& op) {
  T* x = sh + Layout<L>::x(l);
  T* bl = sh + Layout<L>::b(l);
  if constexpr (l == 1) {
    if (threadIdx.x == 0) x[Lv<1>::p + 1] = bl[Lv<1>::p + 1] * T(level_coef(a, sg, 1, op).inv_c0);
    __syncthreads();
  } else {
    constexpr int n = Lv<l>::n, p = Lv<l>::p;
    constexpr int nc = Lv<l - 1>::n, pc = Lv<l - 1>::p;
    {
      // the level's coefficients are formed again after the coarse cycle
      // rather than held in registers across it
      const LevelCoef cf = level_coef(a, sg, l, op);
      sweeps<l, NT>(x, bl, cf, true);
      T* r = sh + Layout<L>::r;
      for (int k = threadIdx.x; k < n * n; k += NT) {
        const int q = (k / n + 1) * p + k % n + 1;
        r[q] = bl[q] - (T(cf.c0) * x[q] + off_centre<l>(x, q, cf));
      }
    }
    __syncthreads();
    const T* r = sh + Layout<L>::r;
    T* bc = sh + Layout<L>::b(l - 1);
    T* xc = sh + Layout<L>::x(l - 1);
    for (int k = threadIdx.x; k < nc * nc; k += NT) {
      const int I = k % nc + 1, J = k / nc + 1;
      const int q = 2 * J * p + 2 * I;
      const T half = ((((r[q + 1] + r[q - 1]) + r[q + p]) + r[q - p]) + r[q + p + 1]) + r[q - p - 1];
      bc[J * pc + I] = r[q] + T(0.5) * half;
      xc[J * pc + I] = T(0);
    }
    __syncthreads();
    vcycle<L, l - 1, NT>(sh, a, sg, op);
    const T* e = xc;
    for (int k = threadIdx.x; k < n * n; k += NT) {
      const int i = k % n + 1, j = k / n + 1;
      const int qc = (j >> 1) * pc + (i >> 1);  // coarse node (i/2, j/2), rounded down
      T v;
      if (!(i & 1) && !(j & 1))
        v = e[qc];
      else if ((i & 1) && !(j & 1))
        v = T(0.5) * (e[qc] + e[qc + 1]);
      else if (!(i & 1) && (j & 1))
        v = T(0.5) * (e[qc] + e[qc + pc]);
      else
        v = T(0.5) * (e[qc] + e[qc + pc + 1]);
      x[j * p + i] += v;
    }
    __syncthreads();
    sweeps<l, NT>(x, bl, level_coef(a, sg, l, op), false);
  }
}

// `cycles` V-cycles on levels L..1 of one time row per workgroup: from xin
// (NULL: zero), the result or A_x applied to it to xout.
template <typename T, int NT, int L>
__global__ __launch_bounds__(NT) void mg_coarse_kernel(const T* xin, const T* b, T* xout,
                                                       double a, const double* __restrict__ sigma,
                                                       int write_Ax, SpaceOp op, int cycles) {
  __shared__ T sh[Layout<L>::total];
  constexpr int n = Lv<L>::n, p = Lv<L>::p, pitch = 1 << L;
  for (int k = threadIdx.x; k < Layout<L>::total; k += NT) sh[k] = T(0);
  __syncthreads();
  const int row = blockIdx.x;
  const double sg = sigma ? sigma[row] : 0.0;
  const int64_t base = (int64_t)row * slab_elems(L);
  T* x = sh + Layout<L>::x(L);
  T* bl = sh + Layout<L>::b(L);
  for (int k = threadIdx.x; k < n * n; k += NT) {
    const int64_t g = base + (int64_t)(k / n) * pitch + (k % n);
    const int q = (k / n + 1) * p + k % n + 1;
    bl[q] = b[g];
    if (xin) x[q] = xin[g];
  }
  __syncthreads();
  for (int c = 0; c < cycles; ++c) vcycle<L, L, NT>(sh, a, sg, op);
  const bool heat = op.heat();
  const LevelCoef ac = level_coef(1.0, 0.0, L, op);  // A_x itself (Section 4)
  for (int k = threadIdx.x; k < n * n; k += NT) {
    const int q = (k / n + 1) * p + k % n + 1;
    T v = x[q];
    if (write_Ax) {
      if (heat)
        v = (((T(4) * v - x[q + 1]) - x[q - 1]) - x[q + p]) - x[q - p];
      else
        v = T(ac.c0) * v + off_centre<L>(x, q, ac);
    }
    xout[base + (int64_t)(k / n) * pitch + (k % n)] = v;
  }
}

template <typename T, int NT>
hipError_t launch_coarse(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows,
                         double a, const double* sigma, int wa, const SpaceOp& op, int cycles) {
  switch (L) {
    case 1: mg_coarse_kernel<T, NT, 1><<<rows, NT, 0, s>>>(xin, b, xout, a, sigma, wa, op, cycles); break;
    case 2: mg_coarse_kernel<T, NT, 2><<<rows, NT, 0, s>>>(xin, b, xout, a, sigma, wa, op, cycles); break;
    case 3: mg_coarse_kernel<T, NT, 3><<<rows, NT, 0, s>>>(xin, b, xout, a, sigma, wa, op, cycles); break;
    case 4: mg_coarse_kernel<T, NT, 4><<<rows, NT, 0, s>>>(xin, b, xout, a, sigma, wa, op, cycles); break;
    case 5: mg_coarse_kernel<T, NT, 5><<<rows, NT, 0, s>>>(xin, b, xout, a, sigma, wa, op, cycles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t mg_coarse_cycle(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows,
                           double a, const double* sigma, bool write_Ax, const SpaceOp& op,
                           int cycles) {
  if (L < 1 || L > coarse_levels<T>() || cycles < 1) return hipErrorInvalidValue;
  const int wa = write_Ax ? 1 : 0;
  // workgroups of 2, 4 or 8 waves per time row, tuned per level and row count
  auto go = [&](int c) -> hipError_t {
    if (c == 0) return launch_coarse<T, 256>(s, xin, b, xout, L, rows, a, sigma, wa, op, cycles);
    if (c == 1) return launch_coarse<T, 128>(s, xin, b, xout, L, rows, a, sigma, wa, op, cycles);
    return launch_coarse<T, 512>(s, xin, b, xout, L, rows, a, sigma, wa, op, cycles);
  };
  const uint64_t key = tune_key(3, sizeof(T), (uint64_t)L | ((uint64_t)cycles << 8), (uint64_t)rows);
  // a cycle that starts from its own output cannot be repeated for timing:
  // it takes the choice made for the same shape from zero
  if (xin != nullptr && xin == xout) return go(tuned_choice(key, 0));
  return go(tuned(key, 3, 0, s, go));
}

template hipError_t mg_coarse_cycle<double>(hipStream_t, const double*, const double*, double*,
                                            int, int, double, const double*, bool,
                                            const SpaceOp&, int);
template hipError_t mg_coarse_cycle<float>(hipStream_t, const float*, const float*, float*, int,
                                           int, double, const double*, bool, const SpaceOp&, int);

}  // namespace stp
