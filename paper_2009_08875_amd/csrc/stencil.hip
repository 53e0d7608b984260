// LDS-tiled space-time stencils (gfx950): the Kronecker products of Lemma 4.2
// and Lemma 4.1 applied row by row (the matrix-free identity of Section 5.2).
//
// A workgroup owns a 64 x 16 tile of the spatial grid and walks a chunk of
// consecutive time rows.  For each time row it holds the tile plus a one-node
// halo: the time combinations (A_t X, M_t X, L X, L^T X, built from rows
// i - 1, i, i + 1 kept in registers) go to LDS, and the spatial stencils
// (A_x: 5 points, M_x: 7 points on the "/" mesh) read them back.  Every input
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

template <typename T>
__device__ __forceinline__ T Mst(const T* a, int k, T m12) {
  // k: index of the node in the halo tile; neighbours at +-1 (x), +-kHX (y)
  return m12 * ((((((T(6) * a[k] + a[k + 1]) + a[k - 1]) + a[k + kHX]) + a[k - kHX]) +
                 a[k + kHX + 1]) + a[k - kHX - 1]);
}
template <typename T>
__device__ __forceinline__ T Ast(const T* a, int k) {
  return (((T(4) * a[k] - a[k + 1]) - a[k - 1]) - a[k + kHX]) - a[k - kHX];
}

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void row_stencil_kernel(
    const T* __restrict__ in0, const T* __restrict__ in1, const T* __restrict__ extra,
    int64_t extra_stride, T* __restrict__ out0, T* __restrict__ out1, int J, int K, int tiles_x,
    int tiles, int chunks, int chunk_rows) {
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
  T xm[kPer], x0[kPer], xp[kPer];
  if constexpr (MODE != kCombine) {
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
      xm[p] = i0 > 0 ? ld(in0, i0 - 1, p) : T(0);
      x0[p] = ld(in0, i0, p);
    }
  }
  for (int i = i0; i < i1; ++i) {
    if constexpr (MODE != kCombine) {
#pragma unroll
      for (int p = 0; p < kPer; ++p) {
        xp[p] = i < N ? ld(in0, i + 1, p) : T(0);
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
          s0[hk[p]] = ld(in0, i, p);
          s1[hk[p]] = ld(in1, i, p);
          s2[hk[p]] = (i == 0 && extra && goff[p] >= 0)
                          ? extra[(int64_t)rhs * extra_stride + goff[p]]
                          : T(0);
        }
      }
    }
    __syncthreads();
    // interior nodes of the tile
    for (int q = threadIdx.x; q < kTX * kTY; q += kThreads) {
      const int lx = 1 + q % kTX, ly = 1 + q / kTX;
      const int gx = gx0 + lx, gy = gy0 + ly;
      if (gx > n || gy > n) continue;
      const int k = ly * kHX + lx;
      const int64_t o = base + (int64_t)i * slab + (int64_t)(gy - 1) * pitch + (gx - 1);
      if constexpr (MODE == kTimePair) {
        // y1 = M (A_t X) + A (L^T X),  y2 = A (M_t X) + M (L X)
        out0[o] = Mst(s0, k, m12) + Ast(s1, k);
        out1[o] = Ast(s2, k) + Mst(s3, k, m12);
      } else if constexpr (MODE == kRhsPair) {
        // G1 = M (L^T g),  G0 = M (M_t g)
        out0[o] = Mst(s0, k, m12);
        out1[o] = Mst(s1, k, m12);
      } else {
        // M z1 + A z2 (+ M e in row 0)
        T v = Mst(s0, k, m12) + Ast(s1, k);
        if (i == 0 && extra) v += Mst(s2, k, m12);
        out0[o] = v;
      }
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
                       int64_t extra_stride, T* out0, T* out1, int J, int K, int nrhs) {
  const int n = grid_n(K);
  const int tiles_x = (n + kTX - 1) / kTX, tiles_y = (n + kTY - 1) / kTY;
  const int tiles = tiles_x * tiles_y;
  auto go = [&](int c) -> hipError_t {
    const int cr = kChunks[c];
    const int chunks = ((1 << J) + 1 + cr - 1) / cr;
    row_stencil_kernel<T, MODE><<<dim3(tiles * chunks, nrhs), kThreads, 0, s>>>(
        in0, in1, extra, extra_stride, out0, out1, J, K, tiles_x, tiles, chunks, cr);
    return hipGetLastError();
  };
  const uint64_t variant = (sizeof(T) == 8 ? 4 : 0) | (uint64_t)MODE;
  const int c = tuned(tune_key(2, variant, (uint64_t)(J * 16 + K), (uint64_t)nrhs),
                      (int)(sizeof(kChunks) / sizeof(kChunks[0])), 2, s, go);
  return go(c);
}

}  // namespace

template <typename T>
hipError_t time_stencil_pair(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs) {
  return launch_rows<T, kTimePair>(s, X, nullptr, nullptr, 0, y1, y2, J, K, nrhs);
}

template <typename T>
hipError_t rhs_stencil_pair(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs) {
  return launch_rows<T, kRhsPair>(s, g, nullptr, nullptr, 0, G1, G0, J, K, nrhs);
}

template <typename T>
hipError_t combine(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                   T* out, int J, int K, int nrhs) {
  return launch_rows<T, kCombine>(s, z1, z2, extra, extra_stride, out, nullptr, J, K, nrhs);
}

#define STP_INSTANTIATE_ROWS(T)                                                                   \
  template hipError_t time_stencil_pair<T>(hipStream_t, const T*, T*, T*, int, int, int);         \
  template hipError_t rhs_stencil_pair<T>(hipStream_t, const T*, T*, T*, int, int, int);          \
  template hipError_t combine<T>(hipStream_t, const T*, const T*, const T*, int64_t, T*, int, int, \
                                 int);
STP_INSTANTIATE_ROWS(double)
STP_INSTANTIATE_ROWS(float)

}  // namespace stp
