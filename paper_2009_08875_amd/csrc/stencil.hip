// LDS-tiled space-time stencils (gfx950): the Kronecker products of Lemma 4.2
// and Lemma 4.1 applied row by row (the matrix-free identity of Section 5.2).
//
// A workgroup owns a 64 x 16 tile of the spatial grid and walks a chunk of
// consecutive time rows.  For each time row it holds the tile plus a one-node
// halo: the time combinations (A_t X, M_t X, L X, L^T X, built from rows
// i - 1, i, i + 1 kept in registers) go to LDS, and the spatial stencils
// (A_x: 5 points for the heat equation, 7 with a diffusion tensor or a
// reaction term; M_x: 7 points on the "/" mesh) read them back.  Every input
// element is read from HBM once per tile (plus the halo and one time row at
// each end of a chunk).  Workgroups are numbered so that neighbouring tiles
// run on the same XCD and share its L2 for the halos.  The chunk length (8 to
// 64 time rows) is picked per problem shape by the launch autotuner.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tune.h"

namespace stp {

namespace {

constexpr int kTX = 64, kTY = 16;               // tile
constexpr int kHX = kTX + 2, kHY = kTY + 2;     // tile with halo
constexpr int kHalo = kHX * kHY;                // 1188 nodes
constexpr int kThreads = 256;
constexpr int kRowsPerThread = kTY * kTX / kThreads;  // consecutive tile rows per thread (4)
constexpr int kPer = (kHalo + kThreads - 1) / kThreads;  // halo nodes per thread (5)
constexpr int kChunks[] = {8, 16, 32, 64};      // candidate time rows per workgroup

enum Mode { kTimePair = 0, kRhsPair = 1, kCombine = 2 };

// Workgroup number -> logical tile index such that consecutive logical tiles
// are dispatched to the same XCD (workgroups go round-robin over 8 XCDs).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int per = nblocks / 8;
  if (per * 8 != nblocks) return b;
  return (b % 8) * per + b / 8;
}

template <typename T>
struct TC {
  T At, Mt, L, LT;
};

// exact hat integrals (Lemma 4.2): one-sided at t = 0 and t = 1
template <typename T>
__device__ __forceinline__ TC<T> time_combo(T xm, T x0, T xp, int i, int N, T inv_tau, T tau6) {
  TC<T> c;
  if (i == 0) {
    c.At = (x0 - xp) * inv_tau;
    c.Mt = tau6 * (T(2) * x0 + xp);
    c.L = (xp - x0) / T(2);
    c.LT = -(x0 + xp) / T(2);
  } else if (i == N) {
    c.At = (x0 - xm) * inv_tau;
    c.Mt = tau6 * (xm + T(2) * x0);
    c.L = (x0 - xm) / T(2);
    c.LT = (xm + x0) / T(2);
  } else {
    c.At = (T(2) * x0 - xm - xp) * inv_tau;
    c.Mt = tau6 * ((xm + T(4) * x0) + xp);
    c.L = (xp - xm) / T(2);
    c.LT = (xm - xp) / T(2);
  }
  return c;
}

// Spatial stencils on a 3 x 3 register window w[row][column] (row 0 below,
// column 0 left): M on the "/" mesh (centre 6, the four axis neighbours and
// the two across the diagonal, times h^2 / 12) and the 5-point A.
template <typename T>
__device__ __forceinline__ T Mw(const T (&w)[3][3], T m12) {
  return m12 * ((((((T(6) * w[1][1] + w[1][2]) + w[1][0]) + w[2][1]) + w[0][1]) + w[2][2]) +
                w[0][0]);
}
template <typename T>
__device__ __forceinline__ T Aw(const T (&w)[3][3]) {
  return (((T(4) * w[1][1] - w[1][2]) - w[1][0]) - w[2][1]) - w[0][1];
}
// A_x = A_D + c M_x of Section 4 on the window, stencil st = stencil_of(op, 1, 0, K)
template <typename T>
__device__ __forceinline__ T Aw_op(const T (&w)[3][3], const T (&st)[4]) {
  return ((st[0] * w[1][1] + st[1] * (w[1][2] + w[1][0])) + st[2] * (w[2][1] + w[0][1])) +
         st[3] * (w[2][2] + w[0][0]);
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void row_stencil_kernel(
    const T* __restrict__ in0, const T* __restrict__ in1, const T* __restrict__ extra,
    int64_t extra_stride, T* __restrict__ out0, T* __restrict__ out1, int J, int K, int tiles_x,
    int tiles, int chunks, int chunk_rows, SpaceOp op) {
  __shared__ T s0[kHalo], s1[kHalo], s2[kHalo], s3[kHalo];
  const int nb = tiles * chunks;
  const int lb = xcd_remap(blockIdx.x, nb);
  const int rhs = blockIdx.y;
  const int tile = lb % tiles;
  const int chunk = lb / tiles;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int n = grid_n(K), pitch = line_pitch(K);
  const int64_t slab = slab_elems(K);
  const int N = 1 << J;
  const int64_t base = (int64_t)rhs * (N + 1) * slab;
  const int gx0 = tx * kTX, gy0 = ty * kTY;  // node (gx0 + lx, gy0 + ly), lx, ly in [0, kHX)
  const T inv_tau = T((double)N);
  const T tau6 = T(1.0 / (6.0 * (double)N));
  const double h = 1.0 / (double)(1 << K);
  const T m12 = T(h * h / 12.0);
  const bool heat = op.heat();
  T ast[4];
  {
    const Stencil a = stencil_of(op, 1.0, 0.0, K);
    ast[0] = T(a.c0);
    ast[1] = T(a.cx);
    ast[2] = T(a.cy);
    ast[3] = T(a.cd);
  }

  // this thread's halo nodes: offsets into a slab (-1 outside the grid)
  int64_t goff[kPer];
  int hk[kPer];
#pragma unroll
  for (int p = 0; p < kPer; ++p) {
    const int k = threadIdx.x + p * kThreads;
    hk[p] = k;
    goff[p] = -1;
    if (k < kHalo) {
      const int gx = gx0 + k % kHX, gy = gy0 + k / kHX;  // 1-based node coordinates
      if (gx >= 1 && gx <= n && gy >= 1 && gy <= n) goff[p] = (int64_t)(gy - 1) * pitch + (gx - 1);
    }
  }
  auto ld = [&](const T* a, int row, int p) -> T {
    return goff[p] >= 0 ? a[base + (int64_t)row * slab + goff[p]] : T(0);
  };

  const int i0 = chunk * chunk_rows;
  const int i1 = min(i0 + chunk_rows, N + 1);
  // time window X_{i-1}, X_i, X_{i+1} of this thread's halo nodes, and the
  // next row's values loaded one step ahead (combine: z1, z2 of the next row)
  T xm[kPer], x0[kPer], xp[kPer], nx0[kPer], nx1[kPer];
#pragma unroll
  for (int p = 0; p < kPer; ++p) {
    if constexpr (MODE != kCombine) {
      xm[p] = i0 > 0 ? ld(in0, i0 - 1, p) : T(0);
      x0[p] = ld(in0, i0, p);
      nx0[p] = i0 < N ? ld(in0, i0 + 1, p) : T(0);
    } else {
      nx0[p] = ld(in0, i0, p);
      nx1[p] = ld(in1, i0, p);
    }
  }
  // interior nodes: thread t takes column 1 + t % 64 and the consecutive
  // rows 1 + 4 (t / 64) .. + 3 of the tile
  const int lx = 1 + (threadIdx.x & (kTX - 1));
  const int ly0 = 1 + (threadIdx.x / kTX) * kRowsPerThread;
  const int gx = gx0 + lx;
  for (int i = i0; i < i1; ++i) {
    if constexpr (MODE != kCombine) {
#pragma unroll
      for (int p = 0; p < kPer; ++p) {
        xp[p] = nx0[p];
        nx0[p] = i + 1 < N ? ld(in0, i + 2, p) : T(0);  // in flight during this row
        if (hk[p] < kHalo) {
          const TC<T> c = time_combo(xm[p], x0[p], xp[p], i, N, inv_tau, tau6);
          if constexpr (MODE == kTimePair) {
            s0[hk[p]] = c.At;
            s1[hk[p]] = c.LT;
            s2[hk[p]] = c.Mt;
            s3[hk[p]] = c.L;
          } else {
            s0[hk[p]] = c.LT;
            s1[hk[p]] = c.Mt;
          }
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < kPer; ++p) {
        if (hk[p] < kHalo) {
          s0[hk[p]] = nx0[p];
          s1[hk[p]] = nx1[p];
          s2[hk[p]] = (i == 0 && extra && goff[p] >= 0)
                          ? extra[(int64_t)rhs * extra_stride + goff[p]]
                          : T(0);
        }
        nx0[p] = i + 1 < i1 ? ld(in0, i + 1, p) : T(0);
        nx1[p] = i + 1 < i1 ? ld(in1, i + 1, p) : T(0);
      }
    }
    __syncthreads();
    // spatial stencils, one LDS array at a time: a three-row window of the
    // array in registers walks up the thread's rows (three new LDS values
    // per row) and each result is added into the outputs in a fixed order
    T acc0[kRowsPerThread], acc1[kRowsPerThread];
    auto pass = [&](const T* arr, bool is_m, T* acc, bool add) {
      T w[3][3];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[r + 1][c] = arr[(ly0 - 1 + r) * kHX + lx - 1 + c];
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w[0][c] = w[1][c];
          w[1][c] = w[2][c];
          w[2][c] = arr[(ly0 + k + 1) * kHX + lx - 1 + c];
        }
        const T v = is_m ? Mw(w, m12) : (heat ? Aw(w) : Aw_op(w, ast));
        acc[k] = add ? acc[k] + v : v;
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each pass's window live alone
    };
    if constexpr (MODE == kTimePair) {
      // y1 = M (A_t X) + A (L^T X),  y2 = A (M_t X) + M (L X)
      pass(s0, true, acc0, false);
      pass(s1, false, acc0, true);
      pass(s2, false, acc1, false);
      pass(s3, true, acc1, true);
    } else if constexpr (MODE == kRhsPair) {
      // G1 = M (L^T g),  G0 = M (M_t g)
      pass(s0, true, acc0, false);
      pass(s1, true, acc1, false);
    } else {
      // M z1 + A z2 (+ M e in row 0)
      pass(s0, true, acc0, false);
      pass(s1, false, acc0, true);
      if (i == 0 && extra) pass(s2, true, acc0, true);
    }
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const int gy = gy0 + ly0 + k;
      if (gx > n || gy > n) continue;
      const int64_t o = base + (int64_t)i * slab + (int64_t)(gy - 1) * pitch + (gx - 1);
      out0[o] = acc0[k];
      if constexpr (MODE != kCombine) out1[o] = acc1[k];
    }
    __syncthreads();
    if constexpr (MODE != kCombine) {
#pragma unroll
      for (int p = 0; p < kPer; ++p) {
        xm[p] = x0[p];
        x0[p] = xp[p];
      }
    }
  }
}

template <typename T, int MODE>
hipError_t launch_rows(hipStream_t s, const T* in0, const T* in1, const T* extra,
                       int64_t extra_stride, T* out0, T* out1, int J, int K, int nrhs,
                       const SpaceOp& op) {
  const int n = grid_n(K);
  const int tiles_x = (n + kTX - 1) / kTX, tiles_y = (n + kTY - 1) / kTY;
  const int tiles = tiles_x * tiles_y;
  auto go = [&](int c) -> hipError_t {
    const int cr = kChunks[c];
    const int chunks = ((1 << J) + 1 + cr - 1) / cr;
    row_stencil_kernel<T, MODE><<<dim3(tiles * chunks, nrhs), kThreads, 0, s>>>(
        in0, in1, extra, extra_stride, out0, out1, J, K, tiles_x, tiles, chunks, cr, op);
    return hipGetLastError();
  };
  const uint64_t variant = (sizeof(T) == 8 ? 4 : 0) | (uint64_t)MODE;
  const int c = tuned(tune_key(2, variant, (uint64_t)(J * 16 + K), (uint64_t)nrhs),
                      (int)(sizeof(kChunks) / sizeof(kChunks[0])), 2, s, go);
  return go(c);
}

}  // namespace

template <typename T>
hipError_t time_stencil_pair(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs,
                             const SpaceOp& op) {
  return launch_rows<T, kTimePair>(s, X, nullptr, nullptr, 0, y1, y2, J, K, nrhs, op);
}

template <typename T>
hipError_t rhs_stencil_pair(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs) {
  return launch_rows<T, kRhsPair>(s, g, nullptr, nullptr, 0, G1, G0, J, K, nrhs, SpaceOp{});
}

template <typename T>
hipError_t combine(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                   T* out, int J, int K, int nrhs, const SpaceOp& op) {
  return launch_rows<T, kCombine>(s, z1, z2, extra, extra_stride, out, nullptr, J, K, nrhs, op);
}

#define STP_INSTANTIATE_ROWS(T)                                                                   \
  template hipError_t time_stencil_pair<T>(hipStream_t, const T*, T*, T*, int, int, int,          \
                                           const SpaceOp&);                                       \
  template hipError_t rhs_stencil_pair<T>(hipStream_t, const T*, T*, T*, int, int, int);          \
  template hipError_t combine<T>(hipStream_t, const T*, const T*, const T*, int64_t, T*, int, int, \
                                 int, const SpaceOp&);
STP_INSTANTIATE_ROWS(double)
STP_INSTANTIATE_ROWS(float)

}  // namespace stp
