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
// Slab layout: line (j, k) of level l occupies 2^l slots; from level 2 on the
// line is split by i mod 4 into four segments of Q = 2^(l-2) slots, node
// i = 4q + r at slot r Q + q (slot 0, i = 0, is the line's zero pad).  The
// colours (i + j + k) mod 4 are then segments: a colour launch of the
// Gauss-Seidel reads and writes one segment of its own line and reads the
// other colours' segments of its line and the neighbouring lines, instead of
// every cache line of x and b.  Level 1 (one node) keeps it at slot 0, the pad
// at slot 1.
//
// Kernels run one 64-lane wave per grid line (j, k) and time row (a
// grid-stride loop over the rows); the Gauss-Seidel launches put 64 / Q lines
// in one wave on levels below 8, one lane per node of the colour, and the
// residual, restriction and prolongation launches put 64 / pitch lines in one
// wave on levels below 6.  Neighbour values come straight from global memory, which the L2 caches; there is no LDS tiling as in the
// two-dimensional kernels.  Levels 4..1 of a V-cycle run in one launch with one
// workgroup per time row and every level in LDS (mg3_coarse_kernel).
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

constexpr int kMaxGridRows = 65535;

// Launch geometry: one 64-lane wave per grid line (j, k) of a slab and per
// time row (grid-stride over rows); lane t takes the line's nodes
// i = i0 + t * stride.  The line's position is uniform across the wave, so a
// node's 14 neighbours sit in 9 line offsets computed once per wave, and the
// lanes only check i against the grid.
constexpr int kLane = 64;

// slot of node i (1..n) within its line on level l, the pad's slot, and the
// node at a slot (0 or n + 1 for the pad)
__device__ __forceinline__ int pos3(int i, int l) {
  return l >= 2 ? (i & 3) * (1 << (l - 2)) + (i >> 2) : i - 1;
}
__device__ __forceinline__ int pad3(int l) { return l >= 2 ? 0 : 1; }
__device__ __forceinline__ int node_at3(int p, int l) {
  if (l < 2) return p + 1;
  const int q = p & ((1 << (l - 2)) - 1);
  return 4 * q + (p >> (l - 2));
}

struct Line3 {
  int j, k, n, pitch, l;
  int64_t off;  // slab offset of the line
};

__device__ __forceinline__ Line3 line3(int line, int l) {
  Line3 L;
  L.n = grid_n(l);
  L.pitch = line_pitch(l);
  L.l = l;
  L.j = line % L.n + 1;
  L.k = line / L.n + 1;
  L.off = (int64_t)line * L.pitch;
  return L;
}

// value of slab s at node (i + di, j + dj, k + dk) of the line, zero outside
template <typename T, int DI, int DJ, int DK>
__device__ __forceinline__ T nb3(const T* s, const Line3& L, int i) {
  const int ii = i + DI, jj = L.j + DJ, kk = L.k + DK;
  if (ii < 1 || ii > L.n || jj < 1 || jj > L.n || kk < 1 || kk > L.n) return T(0);
  return s[L.off + ((int64_t)DK * L.n + DJ) * L.pitch + pos3(ii, L.l)];
}

// Stencil weights of C = a A_x + sigma M_x on level l: centre, the six axis
// neighbours, the six face-diagonal and the two body-diagonal neighbours.
struct C3 {
  double c0, ax, fd, bd;
};
__device__ __forceinline__ C3 coef3(double a, double sigma, int l) {
  const double h = 1.0 / (double)(1 << l);
  const double m = sigma * h * h * h;
  return {a * 6.0 * h + 0.4 * m, -a * h + m / 20.0, m / 30.0, m / 20.0};
}

template <typename T>
__device__ __forceinline__ T axis_sum(const T* s, const Line3& L, int i) {
  return ((nb3<T, 1, 0, 0>(s, L, i) + nb3<T, -1, 0, 0>(s, L, i)) +
          (nb3<T, 0, 1, 0>(s, L, i) + nb3<T, 0, -1, 0>(s, L, i))) +
         (nb3<T, 0, 0, 1>(s, L, i) + nb3<T, 0, 0, -1>(s, L, i));
}
template <typename T>
__device__ __forceinline__ T face_sum(const T* s, const Line3& L, int i) {
  return ((nb3<T, 1, 1, 0>(s, L, i) + nb3<T, -1, -1, 0>(s, L, i)) +
          (nb3<T, 1, 0, 1>(s, L, i) + nb3<T, -1, 0, -1>(s, L, i))) +
         (nb3<T, 0, 1, 1>(s, L, i) + nb3<T, 0, -1, -1>(s, L, i));
}
template <typename T>
__device__ __forceinline__ T body_sum(const T* s, const Line3& L, int i) {
  return nb3<T, 1, 1, 1>(s, L, i) + nb3<T, -1, -1, -1>(s, L, i);
}

// (C x) at node i of the line without (off-centre part) or with the centre;
// DIAG: the mass couplings across the diagonals are present (sigma != 0).
template <typename T, bool DIAG>
__device__ __forceinline__ T off3(const T* s, const Line3& L, int i, const C3& c) {
  T v = T(c.ax) * axis_sum(s, L, i);
  if constexpr (DIAG) v += T(c.fd) * face_sum(s, L, i) + T(c.bd) * body_sum(s, L, i);
  return v;
}
template <typename T>
__device__ __forceinline__ T mass3(const T* s, const Line3& L, int i, const C3& c) {
  return (T(c.c0) * nb3<T, 0, 0, 0>(s, L, i) + T(c.ax) * axis_sum(s, L, i)) +
         (T(c.fd) * face_sum(s, L, i) + T(c.bd) * body_sum(s, L, i));
}

// grid: x = lines of the level (n^2), y = rows (grid-stride), one wave each
inline dim3 grid3(int l, int rows) {
  return dim3((unsigned)(grid_n(l) * grid_n(l)), (unsigned)std::min(rows, kMaxGridRows));
}
#define FOR_LINE_ROWS(l, rows)                    \
  const Line3 L = line3(blockIdx.x, l);            \
  for (int row = blockIdx.y; row < (rows); row += gridDim.y)
// lanes over the slots of the line; i: the slot's node, skipped at the pad
#define FOR_NODES(L)                                                   \
  for (int p = threadIdx.x; p < (L).pitch; p += kLane)                 \
    if (const int i = node_at3(p, (L).l); i >= 1 && i <= (L).n)

// Packed lines: lines shorter than a wave share it (64 / pitch lines per
// wave, one lane per slot); a line of 64 slots or more takes a wave to
// itself, its lanes striding over the slots.  grid3p is the matching grid.
struct Packed {
  int line, p0, pstep;
};
__device__ __forceinline__ Packed packed_line(int l) {
  const int pitch = line_pitch(l);
  if (pitch >= kLane) return {(int)blockIdx.x, (int)threadIdx.x, kLane};
  return {(int)blockIdx.x * (kLane / pitch) + (int)threadIdx.x / pitch,
          (int)threadIdx.x % pitch, pitch};
}
inline dim3 grid3p(int l, int rows) {
  const int n = grid_n(l), pitch = line_pitch(l), per = pitch >= kLane ? 1 : kLane / pitch;
  return dim3((unsigned)((n * n + per - 1) / per), (unsigned)std::min(rows, kMaxGridRows));
}
#define FOR_PACKED_NODES(L, pk)                                        \
  for (int p = (pk).p0; p < (L).pitch; p += (pk).pstep)                \
    if (const int i = node_at3(p, (L).l); i >= 1 && i <= (L).n)

// writes the pad of a line and the slab tail zero
template <typename T>
__device__ __forceinline__ void zero_pads(T* slab_base, const Line3& L, int l, int line) {
  if (threadIdx.x == 0) slab_base[L.off + pad3(l)] = T(0);
  const int64_t used = (int64_t)L.n * L.n * L.pitch;
  if (line == L.n * L.n - 1)
    for (int64_t e = used + threadIdx.x; e < slab3_elems(l); e += kLane) slab_base[e] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kLane) void pack3_kernel(const double* __restrict__ src,
                                                      T* __restrict__ dst, int K, int rows) {
  const int64_t nx = (int64_t)grid_n(K) * grid_n(K) * grid_n(K);
  FOR_LINE_ROWS(K, rows) {
    T* d = dst + row * slab3_elems(K);
    const double* sr = src + row * nx + (int64_t)blockIdx.x * L.n;
    FOR_NODES(L) d[L.off + p] = (T)sr[i - 1];
    zero_pads(d, L, K, blockIdx.x);
  }
}

template <typename T>
__global__ __launch_bounds__(kLane) void unpack3_kernel(const T* __restrict__ src,
                                                        double* __restrict__ dst, int K,
                                                        int rows) {
  const int64_t nx = (int64_t)grid_n(K) * grid_n(K) * grid_n(K);
  FOR_LINE_ROWS(K, rows) {
    const T* s = src + row * slab3_elems(K);
    double* dr = dst + row * nx + (int64_t)blockIdx.x * L.n;
    FOR_NODES(L) dr[i - 1] = (double)s[L.off + p];
  }
}

// y = (a A + sigma M) x per row (A: a = 1, sigma = 0; M: a = 0, sigma = 1)
template <typename T>
__global__ __launch_bounds__(kLane) void apply3_kernel(const T* __restrict__ x,
                                                       T* __restrict__ y, int K, int rows,
                                                       double a, double sigma) {
  const C3 c = coef3(a, sigma, K);
  FOR_LINE_ROWS(K, rows) {
    const T* xr = x + row * slab3_elems(K);
    T* yr = y + row * slab3_elems(K);
    FOR_NODES(L) yr[L.off + p] = mass3(xr, L, i, c);
    zero_pads(yr, L, K, blockIdx.x);
  }
}

// Weights of the four time combinations of Lemma 4.2 on time rows i - 1, i,
// i + 1 (exact hat integrals, one-sided at t = 0 and t = 1): A_t, M_t, L and
// L^T applied to a function of time are w[0] x_{i-1} + w[1] x_i + w[2] x_{i+1}.
struct TW3 {
  double At[3], Mt[3], L[3], LT[3];
};
__device__ __forceinline__ TW3 time_weights3(int i, int N) {
  const double n = (double)N, m6 = 1.0 / (6.0 * (double)N);
  if (i == 0) return {{0.0, n, -n}, {0.0, 2.0 * m6, m6}, {0.0, -0.5, 0.5}, {0.0, -0.5, -0.5}};
  if (i == N) return {{-n, n, 0.0}, {m6, 2.0 * m6, 0.0}, {-0.5, 0.5, 0.0}, {0.5, 0.5, 0.0}};
  return {{-n, 2.0 * n, -n}, {m6, 4.0 * m6, m6}, {-0.5, 0.0, 0.5}, {0.5, 0.0, -0.5}};
}

// MODE 0: y1 = M (A_t X) + A (L^T X), y2 = A (M_t X) + M (L X)
// MODE 1: G1 = M (L^T g), G0 = M (M_t g)
// The time combinations are linear in the three time rows, so each output is
// a weighted sum of A x and M x of rows i - 1, i, i + 1: a lane forms those
// spatial products one time row after another (15 loads each) and
// accumulates them.
template <typename T, int MODE>
__global__ __launch_bounds__(kLane) void time_pair3_kernel(const T* __restrict__ X,
                                                           T* __restrict__ y1,
                                                           T* __restrict__ y2, int J, int K,
                                                           int rows) {
  const int N = 1 << J;
  const int64_t slab = slab3_elems(K);
  const C3 ca = coef3(1.0, 0.0, K), cm = coef3(0.0, 1.0, K);
  FOR_LINE_ROWS(K, rows) {
    const int rhs = row / (N + 1), ti = row - rhs * (N + 1);
    const TW3 w = time_weights3(ti, N);
    const T* x0 = X + (int64_t)row * slab;
    FOR_NODES(L) {
      T o1 = T(0), o2 = T(0);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        if ((t == 0 && ti == 0) || (t == 2 && ti == N)) continue;
        const T* xs = x0 + (t - 1) * slab;
        const T axis = axis_sum(xs, L, i);
        const T Mx = (T(cm.c0) * nb3<T, 0, 0, 0>(xs, L, i) + T(cm.ax) * axis) +
                     (T(cm.fd) * face_sum(xs, L, i) + T(cm.bd) * body_sum(xs, L, i));
        if constexpr (MODE == 0) {
          const T Ax = T(ca.c0) * nb3<T, 0, 0, 0>(xs, L, i) + T(ca.ax) * axis;
          o1 += T(w.At[t]) * Mx + T(w.LT[t]) * Ax;
          o2 += T(w.Mt[t]) * Ax + T(w.L[t]) * Mx;
        } else {
          o1 += T(w.LT[t]) * Mx;
          o2 += T(w.Mt[t]) * Mx;
        }
      }
      y1[(int64_t)row * slab + L.off + p] = o1;
      y2[(int64_t)row * slab + L.off + p] = o2;
    }
    zero_pads(y1 + (int64_t)row * slab, L, K, blockIdx.x);
    zero_pads(y2 + (int64_t)row * slab, L, K, blockIdx.x);
  }
}

// out = M z1 + A z2, plus M e_b in row 0 of right-hand side b
template <typename T>
__global__ __launch_bounds__(kLane) void combine3_kernel(const T* __restrict__ z1,
                                                        const T* __restrict__ z2,
                                                        const T* __restrict__ extra,
                                                        int64_t extra_stride, T* __restrict__ out,
                                                        int J, int K, int rows) {
  const int N = 1 << J;
  const int64_t slab = slab3_elems(K);
  const C3 ca = coef3(1.0, 0.0, K), cm = coef3(0.0, 1.0, K);
  FOR_LINE_ROWS(K, rows) {
    const int rhs = row / (N + 1), ti = row - rhs * (N + 1);
    const T* a1 = z1 + (int64_t)row * slab;
    const T* a2 = z2 + (int64_t)row * slab;
    const T* e = (ti == 0 && extra) ? extra + (int64_t)rhs * extra_stride : nullptr;
    T* o = out + (int64_t)row * slab;
    FOR_NODES(L) {
      T v = mass3(a1, L, i, cm) + (T(ca.c0) * nb3<T, 0, 0, 0>(a2, L, i) + off3<T, false>(a2, L, i, ca));
      if (e) v += mass3(e, L, i, cm);
      o[L.off + p] = v;
    }
    zero_pads(o, L, K, blockIdx.x);
  }
}

// XCD-aware order of the Gauss-Seidel tiles.  Workgroups are dealt to the 8
// XCDs in turn in the order of their linear index, and each XCD has its own
// L2.  The linear index is renumbered so that each XCD takes one contiguous
// range of (line group, row) tiles: the lines next to a tile (j +- 1, k +- 1)
// are then mostly ones its own L2 has just fetched.  A bijection of the grid
// onto itself.
struct Tile {
  int x, y;
};
__device__ __forceinline__ Tile xcd_tile() {
  constexpr int kXcd = 8;
  const int64_t gx = gridDim.x, total = gx * gridDim.y;
  const int64_t id = (int64_t)blockIdx.y * gx + blockIdx.x;
  const int64_t per = total / kXcd, rem = total % kXcd, x = id % kXcd;
  const int64_t t = x * per + (x < rem ? x : rem) + id / kXcd;
  return {(int)(t % gx), (int)(t / gx)};
}

// One colour of Gauss-Seidel on level l >= 2 for C = a A + sigma_row M.  A
// wave takes 64 / Q lines (Q = 2^(l-2) slots per segment, at most 64) and
// one lane per slot of each line's colour segment: line (j, k) holds colour
// c in segment r = (c - j - k) mod 4, node i = 4q + r.
template <typename T, bool DIAG>
__global__ __launch_bounds__(kLane) void relax3_kernel(T* __restrict__ x,
                                                       const T* __restrict__ b, int l, int rows,
                                                       double a, const double* __restrict__ sigma,
                                                       int colour) {
  const int n = grid_n(l), Q = 1 << (l - 2);
  const Tile tile = xcd_tile();
  const int line = tile.x * (kLane / Q) + threadIdx.x / Q;
  const int q = threadIdx.x & (Q - 1);
  if (line >= n * n) return;
  const Line3 L = line3(line, l);
  const int r = (colour - L.j - L.k) & 3;
  const int i = 4 * q + r;
  if (i < 1 || i > n) return;
  const int64_t at = L.off + r * Q + q;
  for (int row = tile.y; row < rows; row += gridDim.y) {
    const C3 c = coef3(a, sigma ? sigma[row] : 0.0, l);
    T* xr = x + row * slab3_elems(l);
    const T* br = b + row * slab3_elems(l);
    xr[at] = (br[at] - off3<T, DIAG>(xr, L, i, c)) * T(1.0 / c.c0);
  }
}

template <typename T, bool DIAG>
__global__ __launch_bounds__(kLane) void residual3_kernel(const T* __restrict__ x,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ r, int l, int rows,
                                                          double a,
                                                          const double* __restrict__ sigma) {
  const Packed pk = packed_line(l);
  if (pk.line >= grid_n(l) * grid_n(l)) return;
  const Line3 L = line3(pk.line, l);
  for (int row = blockIdx.y; row < rows; row += gridDim.y) {
    const C3 c = coef3(a, sigma ? sigma[row] : 0.0, l);
    const T* xr = x + row * slab3_elems(l);
    const T* br = b + row * slab3_elems(l);
    T* rr = r + row * slab3_elems(l);
    FOR_PACKED_NODES(L, pk)
      rr[L.off + p] = br[L.off + p] - (T(c.c0) * nb3<T, 0, 0, 0>(xr, L, i) +
                                       off3<T, DIAG>(xr, L, i, c));
  }
}

// bc (level l - 1) = P^T r (level l): the coarse node's own fine value plus
// half of each of its 14 fine neighbours along the edge directions.  The
// wave runs over a coarse line; Lf addresses the fine line through 2J, 2K.
template <typename T>
__global__ __launch_bounds__(kLane) void restrict3_kernel(const T* __restrict__ r,
                                                          T* __restrict__ bc, int l, int rows) {
  const int lc = l - 1, nc = grid_n(lc), pc = line_pitch(lc);
  const Packed pk = packed_line(lc);
  if (pk.line >= nc * nc) return;
  const int line = pk.line, p0 = pk.p0, pstep = pk.pstep;
  const Line3 L = line3(line, lc);
  Line3 Lf;
  Lf.n = grid_n(l);
  Lf.pitch = line_pitch(l);
  Lf.l = l;
  Lf.j = 2 * L.j;
  Lf.k = 2 * L.k;
  Lf.off = ((int64_t)(Lf.k - 1) * Lf.n + (Lf.j - 1)) * Lf.pitch;
  const int64_t used = (int64_t)nc * nc * pc;
  for (int row = blockIdx.y; row < rows; row += gridDim.y) {
    const T* rr = r + row * slab3_elems(l);
    T* o = bc + row * slab3_elems(lc);
    for (int p = p0; p < pc; p += pstep) {
      const int i = node_at3(p, lc);
      if (i >= 1 && i <= nc) {
        const int f = 2 * i;  // the fine node under coarse node i
        const T half = (axis_sum(rr, Lf, f) + face_sum(rr, Lf, f)) + body_sum(rr, Lf, f);
        o[L.off + p] = nb3<T, 0, 0, 0>(rr, Lf, f) + T(0.5) * half;
      } else {
        o[L.off + p] = T(0);  // the line's pad
      }
    }
    if (line == nc * nc - 1)  // the slab's tail
      for (int64_t e = used + p0; e < slab3_elems(lc); e += pstep) o[e] = T(0);
  }
}

// x (level l) += P e (e on level l - 1): fine node (2I + a, 2J + b, 2K + c)
// takes the mean of the coarse ends of the edge it bisects.
template <typename T>
__global__ __launch_bounds__(kLane) void prolong_add3_kernel(const T* __restrict__ e,
                                                             T* __restrict__ x, int l, int rows) {
  const Packed pk = packed_line(l);
  if (pk.line >= grid_n(l) * grid_n(l)) return;
  const Line3 L = line3(pk.line, l);
  for (int row = blockIdx.y; row < rows; row += gridDim.y) {
    const int nc = grid_n(l - 1), pc = line_pitch(l - 1), lc = l - 1;
    const T* ee = e + row * slab3_elems(l - 1);
    T* xr = x + row * slab3_elems(l);
    const int bb = L.j & 1, cc = L.k & 1, J = L.j >> 1, Kc = L.k >> 1;
    // slab index of coarse node (I, Jn, Kn), -1 outside the grid
    auto idx = [&](int I, int Jn, int Kn) -> int64_t {
      const bool in = I >= 1 && I <= nc && Jn >= 1 && Jn <= nc && Kn >= 1 && Kn <= nc;
      return in ? ((int64_t)(Kn - 1) * nc + (Jn - 1)) * pc + pos3(I, lc) : -1;
    };
    FOR_PACKED_NODES(L, pk) {
      const int aa = i & 1, I = i >> 1;
      const int64_t q0 = idx(I, J, Kc), q1 = idx(I + aa, J + bb, Kc + cc);
      // the three loads are issued before any value is used: an end outside
      // the grid loads element 0 and is then replaced by zero.  A node on a
      // coarse node has q1 = q0, and the mean of a value with itself is that
      // value exactly, so every node takes the same branch-free form.
      const T e0 = ee[q0 < 0 ? 0 : q0], e1 = ee[q1 < 0 ? 0 : q1];
      const T xo = xr[L.off + p];
      const T v = T(0.5) * ((q0 < 0 ? T(0) : e0) + (q1 < 0 ? T(0) : e1));
      xr[L.off + p] = xo + v;
    }
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
  x[row * s] = b[row * s] / T(c.c0);
}

template <typename T>
__global__ __launch_bounds__(256) void zero3_kernel(T* __restrict__ x, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) x[i] = T(0);
}

// ---- V-cycles on levels L..1 (L <= kCoarse3) of one time row per workgroup,
// every level in LDS.  Each level is a cube of (n + 2)^3 values with a zero
// border, node (i, j, k) at (k p + j) p + i, p = n + 2; the schedule and the
// arithmetic are those of the launches above (relax3_kernel, residual3_kernel,
// restrict3_kernel, prolong_add3_kernel, coarsest3_kernel), one barrier per
// colour step instead of one launch.
constexpr int kCoarse3 = 4;
constexpr int kCoarse3Threads = 512;

template <int l>
struct Cube {
  static constexpr int n = (1 << l) - 1;
  static constexpr int p = n + 2;
  static constexpr int size = p * p * p;
  static constexpr int m = (n + 3) / 4;  // nodes of one colour per grid line, at most
};

// LDS layout for top level L: x_l then b_l for l = L..1, then level L's residual
template <int L>
struct Layout3 {
  static constexpr int x(int l) {
    int o = 0;
    for (int k = L; k > l; --k) o += 2 * ((1 << k) + 1) * ((1 << k) + 1) * ((1 << k) + 1);
    return o;
  }
  static constexpr int b(int l) { return x(l) + ((1 << l) + 1) * ((1 << l) + 1) * ((1 << l) + 1); }
  static constexpr int r = x(0);
  static constexpr int total = r + ((1 << L) + 1) * ((1 << L) + 1) * ((1 << L) + 1);
};

template <int l, int DI, int DJ, int DK, typename T>
__device__ __forceinline__ T cnb(const T* x, int q) {
  constexpr int p = Cube<l>::p;
  return x[q + (DK * p + DJ) * p + DI];
}
template <int l, typename T>
__device__ __forceinline__ T caxis(const T* x, int q) {
  return ((cnb<l, 1, 0, 0>(x, q) + cnb<l, -1, 0, 0>(x, q)) +
          (cnb<l, 0, 1, 0>(x, q) + cnb<l, 0, -1, 0>(x, q))) +
         (cnb<l, 0, 0, 1>(x, q) + cnb<l, 0, 0, -1>(x, q));
}
template <int l, typename T>
__device__ __forceinline__ T cface(const T* x, int q) {
  return ((cnb<l, 1, 1, 0>(x, q) + cnb<l, -1, -1, 0>(x, q)) +
          (cnb<l, 1, 0, 1>(x, q) + cnb<l, -1, 0, -1>(x, q))) +
         (cnb<l, 0, 1, 1>(x, q) + cnb<l, 0, -1, -1>(x, q));
}
template <int l, typename T>
__device__ __forceinline__ T cbody(const T* x, int q) {
  return cnb<l, 1, 1, 1>(x, q) + cnb<l, -1, -1, -1>(x, q);
}
template <int l, bool DIAG, typename T>
__device__ __forceinline__ T coff(const T* x, int q, const C3& c) {
  T v = T(c.ax) * caxis<l>(x, q);
  if constexpr (DIAG) v += T(c.fd) * cface<l>(x, q) + T(c.bd) * cbody<l>(x, q);
  return v;
}

template <int l, bool DIAG, typename T>
__device__ __forceinline__ void crelax(T* x, const T* b, int colour, const C3& c) {
  constexpr int n = Cube<l>::n, p = Cube<l>::p, m = Cube<l>::m;
  const T inv = T(1.0 / c.c0);
  for (int t = threadIdx.x; t < n * n * m; t += kCoarse3Threads) {
    const int line = t / m, qq = t - line * m;
    const int j = line % n + 1, k = line / n + 1;
    const int i = 4 * qq + ((colour - j - k) & 3);
    if (i < 1 || i > n) continue;
    const int q = (k * p + j) * p + i;
    x[q] = (b[q] - coff<l, DIAG>(x, q, c)) * inv;
  }
}

template <int l, bool DIAG, typename T>
__device__ void csweeps(T* x, const T* b, const C3& c, bool forward) {
  for (int s = 0; s < 3; ++s)
    for (int k = 0; k < 4; ++k) {
      crelax<l, DIAG>(x, b, forward ? k : 3 - k, c);
      __syncthreads();
    }
}

template <int L, int l, bool DIAG, typename T>
__device__ void cvcycle(T* sh, double a, double sg) {
  T* x = sh + Layout3<L>::x(l);
  T* bl = sh + Layout3<L>::b(l);
  if constexpr (l == 1) {
    if (threadIdx.x == 0) {
      constexpr int q = (Cube<1>::p + 1) * Cube<1>::p + 1;
      x[q] = bl[q] / T(coef3(a, sg, 1).c0);
    }
    __syncthreads();
  } else {
    constexpr int n = Cube<l>::n, p = Cube<l>::p;
    constexpr int nc = Cube<l - 1>::n, pc = Cube<l - 1>::p;
    T* r = sh + Layout3<L>::r;
    {
      const C3 c = coef3(a, sg, l);
      csweeps<l, DIAG>(x, bl, c, true);
      for (int t = threadIdx.x; t < n * n * n; t += kCoarse3Threads) {
        const int i = t % n + 1, j = (t / n) % n + 1, k = t / (n * n) + 1;
        const int q = (k * p + j) * p + i;
        r[q] = bl[q] - (T(c.c0) * x[q] + coff<l, DIAG>(x, q, c));
      }
    }
    __syncthreads();
    T* bc = sh + Layout3<L>::b(l - 1);
    T* xc = sh + Layout3<L>::x(l - 1);
    for (int t = threadIdx.x; t < nc * nc * nc; t += kCoarse3Threads) {
      const int I = t % nc + 1, J = (t / nc) % nc + 1, K = t / (nc * nc) + 1;
      const int q = (2 * K * p + 2 * J) * p + 2 * I;
      const T half = (caxis<l>(r, q) + cface<l>(r, q)) + cbody<l>(r, q);
      const int qc = (K * pc + J) * pc + I;
      bc[qc] = r[q] + T(0.5) * half;
      xc[qc] = T(0);
    }
    __syncthreads();
    cvcycle<L, l - 1, DIAG>(sh, a, sg);
    for (int t = threadIdx.x; t < n * n * n; t += kCoarse3Threads) {
      const int i = t % n + 1, j = (t / n) % n + 1, k = t / (n * n) + 1;
      const int aa = i & 1, bb = j & 1, cc = k & 1;
      const int q0 = ((k >> 1) * pc + (j >> 1)) * pc + (i >> 1);
      T v = xc[q0];
      if (aa | bb | cc) v = T(0.5) * (v + xc[q0 + (cc * pc + bb) * pc + aa]);
      x[(k * p + j) * p + i] += v;
    }
    __syncthreads();
    csweeps<l, DIAG>(x, bl, coef3(a, sg, l), false);
  }
}

// `cycles` V-cycles from xin (NULL: zero) on one time row per workgroup; the
// result, or A_x applied to it, to xout (the whole slab, pads zero).
template <typename T, int L, bool DIAG>
__global__ __launch_bounds__(kCoarse3Threads) void mg3_coarse_kernel(
    const T* __restrict__ xin, const T* __restrict__ b, T* __restrict__ xout, double a,
    const double* __restrict__ sigma, int write_Ax, int cycles) {
  __shared__ T sh[Layout3<L>::total];
  constexpr int n = Cube<L>::n, p = Cube<L>::p, pitch = 1 << L;
  for (int t = threadIdx.x; t < Layout3<L>::total; t += kCoarse3Threads) sh[t] = T(0);
  __syncthreads();
  const int row = blockIdx.x;
  const double sg = sigma ? sigma[row] : 0.0;
  const int64_t base = (int64_t)row * slab3_elems(L);
  T* x = sh + Layout3<L>::x(L);
  T* bl = sh + Layout3<L>::b(L);
  for (int t = threadIdx.x; t < n * n * n; t += kCoarse3Threads) {
    const int i = t % n + 1, line = t / n;
    const int64_t g = base + (int64_t)line * pitch + pos3(i, L);
    const int q = ((line / n + 1) * p + (line % n + 1)) * p + i;
    bl[q] = b[g];
    if (xin) x[q] = xin[g];
  }
  __syncthreads();
  for (int c = 0; c < cycles; ++c) cvcycle<L, L, DIAG>(sh, a, sg);
  const C3 ac = coef3(1.0, 0.0, L);  // A_x itself
  for (int64_t e = threadIdx.x; e < slab3_elems(L); e += kCoarse3Threads) {
    const int line = (int)(e / pitch), slot = (int)(e - (int64_t)line * pitch);
    const int i = node_at3(slot, L);
    T v = T(0);
    if (line < n * n && i >= 1 && i <= n) {
      const int q = ((line / n + 1) * p + (line % n + 1)) * p + i;
      v = x[q];
      if (write_Ax)
        v = (T(ac.c0) * v + T(ac.ax) * caxis<L>(x, q)) +
            (T(ac.fd) * cface<L>(x, q) + T(ac.bd) * cbody<L>(x, q));
    }
    xout[base + e] = v;
  }
}

template <typename T, bool DIAG>
hipError_t launch_coarse3(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows,
                          double a, const double* sigma, bool write_Ax, int cycles) {
  const int wa = write_Ax ? 1 : 0;
  switch (L) {
    case 2: mg3_coarse_kernel<T, 2, DIAG><<<rows, kCoarse3Threads, 0, s>>>(xin, b, xout, a, sigma, wa, cycles); break;
    case 3: mg3_coarse_kernel<T, 3, DIAG><<<rows, kCoarse3Threads, 0, s>>>(xin, b, xout, a, sigma, wa, cycles); break;
    case 4: mg3_coarse_kernel<T, 4, DIAG><<<rows, kCoarse3Threads, 0, s>>>(xin, b, xout, a, sigma, wa, cycles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t coarse3(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows, double a,
                   const double* sigma, bool write_Ax, int cycles) {
  return sigma ? launch_coarse3<T, true>(s, xin, b, xout, L, rows, a, sigma, write_Ax, cycles)
               : launch_coarse3<T, false>(s, xin, b, xout, L, rows, a, sigma, write_Ax, cycles);
}

}  // namespace

template <typename T>
hipError_t pack3(hipStream_t s, const double* src, T* dst, int K, int rows) {
  pack3_kernel<T><<<grid3(K, rows), kLane, 0, s>>>(src, dst, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t unpack3(hipStream_t s, const T* src, double* dst, int K, int rows) {
  unpack3_kernel<T><<<grid3(K, rows), kLane, 0, s>>>(src, dst, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t apply_A3(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply3_kernel<T><<<grid3(K, rows), kLane, 0, s>>>(x, y, K, rows, 1.0, 0.0);
  return hipGetLastError();
}
template <typename T>
hipError_t apply_M3(hipStream_t s, const T* x, T* y, int K, int rows) {
  apply3_kernel<T><<<grid3(K, rows), kLane, 0, s>>>(x, y, K, rows, 0.0, 1.0);
  return hipGetLastError();
}
template <typename T>
hipError_t time_stencil_pair3(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  time_pair3_kernel<T, 0><<<grid3(K, rows), kLane, 0, s>>>(X, y1, y2, J, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t rhs_stencil_pair3(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  time_pair3_kernel<T, 1><<<grid3(K, rows), kLane, 0, s>>>(g, G1, G0, J, K, rows);
  return hipGetLastError();
}
template <typename T>
hipError_t combine3(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                    T* out, int J, int K, int nrhs) {
  const int rows = nrhs * ((1 << J) + 1);
  combine3_kernel<T><<<grid3(K, rows), kLane, 0, s>>>(z1, z2, extra, extra_stride, out, J, K,
                                                        rows);
  return hipGetLastError();
}

// V-cycle on level l for x (in place), b; w: level-l residual buffer.
template <typename T>
hipError_t vcycle3(hipStream_t s, const Mg3Work<T>& w, T* x, const T* b, int l, int rows,
                   double a, const double* sigma) {
  const dim3 g = grid3p(l, rows);  // residual, prolongation
  // Gauss-Seidel launches: 64 / Q lines per wave (l >= 2; l is at least 2 here)
  const int n = grid_n(l), per = kLane / (1 << (l - 2));
  const dim3 gr((unsigned)((n * n + per - 1) / per), (unsigned)std::min(rows, kMaxGridRows));
  auto relax = [&](int c) {
    if (sigma)
      relax3_kernel<T, true><<<gr, kLane, 0, s>>>(x, b, l, rows, a, sigma, c);
    else
      relax3_kernel<T, false><<<gr, kLane, 0, s>>>(x, b, l, rows, a, sigma, c);
  };
  for (int sw = 0; sw < 3; ++sw)
    for (int c = 0; c < 4; ++c) relax(c);
  if (sigma)
    residual3_kernel<T, true><<<g, kLane, 0, s>>>(x, b, w.r[l], l, rows, a, sigma);
  else
    residual3_kernel<T, false><<<g, kLane, 0, s>>>(x, b, w.r[l], l, rows, a, sigma);
  restrict3_kernel<T><<<grid3p(l - 1, rows), kLane, 0, s>>>(w.r[l], w.b[l - 1], l, rows);
  if (l - 1 <= kCoarse3) {
    // levels l - 1 .. 1 from zero in one launch, every level in LDS
    const hipError_t e =
        coarse3<T>(s, nullptr, w.b[l - 1], w.x[l - 1], l - 1, rows, a, sigma, false, 1);
    if (e != hipSuccess) return e;
  } else {
    const int64_t cnt = (int64_t)rows * slab3_elems(l - 1);
    zero3_kernel<T><<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(w.x[l - 1], cnt);
    const hipError_t e = vcycle3<T>(s, w, w.x[l - 1], w.b[l - 1], l - 1, rows, a, sigma);
    if (e != hipSuccess) return e;
  }
  prolong_add3_kernel<T><<<g, kLane, 0, s>>>(w.x[l - 1], x, l, rows);
  for (int sw = 0; sw < 3; ++sw)
    for (int c = 3; c >= 0; --c) relax(c);
  return hipGetLastError();
}

template <typename T>
hipError_t mg3_apply(hipStream_t s, const Mg3Work<T>& w, const T* b, T* x, int K, int rows,
                     double a, const double* sigma, int vcycles, bool write_Ax) {
  if (K >= 2 && K <= kCoarse3)  // every cycle in one launch, every level in LDS
    return coarse3<T>(s, nullptr, b, x, K, rows, a, sigma, write_Ax, vcycles);
  T* xk = write_Ax ? w.x[K] : x;
  const int64_t cnt = (int64_t)rows * slab3_elems(K);
  zero3_kernel<T><<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(xk, cnt);
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
