// The wavelet transforms along time in one pass over the rows (gfx950).
//
// One thread per slab column (two adjacent columns in FP32).  The analysis
// W^T (Section 3.3, eq. (10), fine to coarse) is a cascade of per-level
// lifting steps: level l consumes the values of its rows (multiples of
// s = N / 2^l) in increasing row order, and every second value it consumes
// completes one of its odd rows (written out: final) and one of its even
// rows, which it passes on to level l - 1 as that level's next value.  Each
// level keeps three values in registers (the old and the accumulating value
// of its current even row, the pending odd row), so the input is read once,
// in row order, and every row is written once, when it becomes final.  Each
// level performs the operations of a level-by-level sweep over the column,
// in the same order; only the interleaving of the levels differs.
//
// Rows are read in batches of 8 per thread, all issued before the first is
// used.  The level structure is unrolled at compile time (the kernel
// is instantiated per J), so the level states are plain registers.
//
// The dot product that PCG needs after the analysis, p^T (W^T y) with y the
// operator applied to X = W p, is taken as X^T y = (W p)^T y, the same number
// in exact arithmetic: X is still resident, and X^T y sums over the rows in
// the order they are read, where p^T (W^T y) would pair every output row with
// a row of p in the scattered order in which the outputs become final.
//
// The synthesis W (coarse to fine) runs the same way in the other direction:
// level 0 hands rows 0 and N to level 1, and level l, on receiving the value
// of its even row m + s, reads the coefficient of its odd row m and hands the
// finished rows m - s and m to level l + 1; level J's rows are final and are
// written in row order.  The coefficients are consumed in a fixed order of the
// rows (the order in which this cascade first needs them, the same for every
// column), which the host computes once per J by running the cascade; the
// kernel reads them in that order, in batches, so the reads are prefetched
// like the analysis's although they are not in row order.  With the update,
// the batch forms p = z + beta p and writes p back as it loads.
#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.h"

namespace stp {

namespace {

constexpr int kStreamBlock = 256;
// rows per batch in both precisions (16 FP32 rows measured slower: the
// registers cost more occupancy than the deeper batch gains)
template <typename T>
constexpr int stream_batch() {
  return 8;
}

// What a thread carries: one FP64 column, or two adjacent FP32 columns, so
// that every load and store moves 8 bytes per lane in both precisions.  The
// two FP32 columns go through the same operations, component by component.
typedef float F2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Lane {
  using V = T;
  static constexpr int W = 1;
  static __device__ __forceinline__ V zero() { return T(0); }
  // p = z + beta p, in FP64 and rounded to T
  static __device__ __forceinline__ V upd(V z, V p, double beta) {
    return (T)((double)z + beta * (double)p);
  }
  static __device__ __forceinline__ double dot(V x, V y) { return (double)x * (double)y; }
};
template <>
struct Lane<float> {
  using V = F2;
  static constexpr int W = 2;
  static __device__ __forceinline__ V zero() { return V{0.0f, 0.0f}; }
  static __device__ __forceinline__ V upd(V z, V p, double beta) {
    return V{(float)((double)z.x + beta * (double)p.x), (float)((double)z.y + beta * (double)p.y)};
  }
  static __device__ __forceinline__ double dot(V a, V b) {
    return (double)a.x * (double)b.x + (double)a.y * (double)b.y;
  }
};

// The analysis keeps the state of its kAnaRegLevels finest levels in
// registers; a coarser level acts once per 64 or more input rows, and its
// state lives in LDS (one slot per thread and value).  With the state of all
// levels in registers the kernel needed up to 198 VGPRs (two waves per SIMD);
// this way about 100, and four to five waves per SIMD up to J = 12.
constexpr int kAnaRegLevels = 6;

template <typename T, int J>
struct AnaState {
  using V = typename Lane<T>::V;
  static constexpr int R = J < kAnaRegLevels ? J : kAnaRegLevels;
  V reo[R];  // old value of the level's current even row
  V rea[R];  // its value with the contributions of the odd rows seen so far
  V ryo[R];  // the pending odd row
  int k[J];  // values consumed by the level
  V* lds;    // levels t >= R: lds[(3 (t - R) + q) kStreamBlock + thread], q = eo, ea, yo

  template <int t, int q>
  __device__ __forceinline__ V& at() {
    if constexpr (t < R) {
      if constexpr (q == 0) return reo[t];
      else if constexpr (q == 1) return rea[t];
      else return ryo[t];
    } else {
      return lds[(3 * (t - R) + q) * kStreamBlock + threadIdx.x];
    }
  }
  template <int t> __device__ __forceinline__ V& eo() { return at<t, 0>(); }
  template <int t> __device__ __forceinline__ V& ea() { return at<t, 1>(); }
  template <int t> __device__ __forceinline__ V& yo() { return at<t, 2>(); }
};

// Writes the final value v of row r.
template <typename T, bool DOT>
struct AnaOut {
  using V = typename Lane<T>::V;
  V* x;
  int64_t slab;  // row stride in units of V
  __device__ __forceinline__ void operator()(int r, V v) { x[(int64_t)r * slab] = v; }
};

// Level J - t consumes value x (its k-th, row k s).
template <typename T, bool DOT, int J, int t>
__device__ __forceinline__ void ana_feed(AnaState<T, J>& st, typename Lane<T>::V x,
                                         AnaOut<T, DOT>& out) {
  using V = typename Lane<T>::V;
  constexpr int l = J - t;
  constexpr int N = 1 << J;
  constexpr int s = 1 << t;
  constexpr int last = 1 << l;
  const int i = st.k[t]++;
  if (i == 0) {
    st.template eo<t>() = x;
    st.template ea<t>() = x;
    return;
  }
  if (i & 1) {
    st.template yo<t>() = x;
    return;
  }
  // x is the old value of the even row i s; the odd row (i - 1) s is final
  const T c = (T)exp2(0.5 * (double)l);
  const V yo = st.template yo<t>();
  const T wl = i == 2 ? T(1) : T(0.5);     // boundary weights of rows 0 and N
  const T wr = i == last ? T(1) : T(0.5);
  out((i - 1) * s, c * ((yo - wl * st.template eo<t>()) - wr * x));
  const V e = st.template ea<t>() + T(0.5) * yo;  // the even row (i - 2) s, done at this level
  const V e2 = x + T(0.5) * yo;
  st.template eo<t>() = x;
  st.template ea<t>() = e2;
  if constexpr (l == 1) {
    out(0, e);
    out(N, e2);
  } else {
    ana_feed<T, DOT, J, t + 1>(st, e, out);
  }
}

// After the last input row: level J - t passes its last even row (row N) on.
template <typename T, bool DOT, int J, int t>
__device__ __forceinline__ void ana_flush(AnaState<T, J>& st, AnaOut<T, DOT>& out) {
  if constexpr (t + 1 < J) {
    ana_feed<T, DOT, J, t + 1>(st, st.template ea<t>(), out);
    ana_flush<T, DOT, J, t + 1>(st, out);
  }
}

__device__ double stream_block_sum(double v) {
  __shared__ double part[kStreamBlock / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kStreamBlock / 64; ++k) t += part[k];
  __syncthreads();
  return t;
}

// In place on Y (nrhs blocks of N + 1 slabs); with DOT the block's share of
// Xs^T Y (Y before the transform) goes to partials[rhs * gridDim.x + block].
template <typename T, bool DOT, int J>
__global__ __launch_bounds__(kStreamBlock) void wavelet_ana_stream_kernel(
    T* __restrict__ Y, const T* __restrict__ Xs, double* __restrict__ partials, int64_t slab) {
  using L = Lane<T>;
  using V = typename L::V;
  constexpr int N = 1 << J;
  const int64_t vslab = slab / L::W;  // row stride in units of V
  const int64_t col = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
  double acc = 0.0;
  if (col < vslab) {
    const int64_t off = (int64_t)blockIdx.y * (N + 1) * vslab + col;
    AnaOut<T, DOT> out;
    out.x = reinterpret_cast<V*>(Y) + off;
    out.slab = vslab;
    const V* xs = DOT ? reinterpret_cast<const V*>(Xs) + off : nullptr;
    AnaState<T, J> st;
    constexpr int LL = J > AnaState<T, J>::R ? J - AnaState<T, J>::R : 1;
    __shared__ V lds_state[3 * LL * kStreamBlock];
    st.lds = lds_state;
#pragma unroll
    for (int t = 0; t < J; ++t) st.k[t] = 0;
    constexpr int B = stream_batch<T>();
#pragma unroll 1
    for (int r0 = 0; r0 <= N; r0 += B) {
      V v[B], w[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        v[b] = r0 + b <= N ? out.x[(int64_t)(r0 + b) * vslab] : L::zero();
        if constexpr (DOT) w[b] = r0 + b <= N ? xs[(int64_t)(r0 + b) * vslab] : L::zero();
      }
      const int nb = min(B, N + 1 - r0);
      if constexpr (DOT) {
#pragma unroll
        for (int b = 0; b < B; ++b) acc += L::dot(w[b], v[b]);  // 0 past N
      }
#pragma unroll 1
      for (int b = 0; b < nb; ++b) {
        const V x = v[0];
#pragma unroll
        for (int q = 0; q + 1 < B; ++q) v[q] = v[q + 1];
        ana_feed<T, DOT, J, 0>(st, x, out);
      }
    }
    ana_flush<T, DOT, J, 0>(st, out);
  }
  if constexpr (DOT) {
    acc = stream_block_sum(acc);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
  }
}

// J = 0: W is the identity on the two rows; only the dot.
template <typename T>
__global__ __launch_bounds__(kStreamBlock) void dot_rows2_kernel(const T* __restrict__ Y,
                                                                  const T* __restrict__ Xs,
                                                                  double* __restrict__ partials,
                                                                  int64_t slab) {
  const int64_t col = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
  double acc = 0.0;
  if (col < slab) {
    const int64_t off = (int64_t)blockIdx.y * 2 * slab + col;
    acc = (double)Xs[off] * (double)Y[off] + (double)Xs[off + slab] * (double)Y[off + slab];
  }
  acc = stream_block_sum(acc);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// ---------------------------------------------------------------- synthesis

template <typename T, bool UPD, int J>
struct SynState {
  using L = Lane<T>;
  using V = typename L::V;
  V eo[J + 1];  // level l: old value of its current even row
  V ea[J + 1];  // and that value with the contributions of the odd rows seen
  int k[J + 1]; // values received by level l
  // coefficients in the read order, B at a time
  static constexpr int B = stream_batch<T>();
  V ring[B];
  int left;     // coefficients in the ring
  int next;     // position in the read order of the next batch
  int orow;     // next output row
  const int* order;
  const V* src;
  V* p;
  const V* z;
  double beta;
  V* dst;
  int64_t slab;  // row stride in units of V

  __device__ __forceinline__ V input() {
    if (left == 0) {
      constexpr int N = 1 << J;
      V a[B], b[B];
      int rows[B];
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const bool ok = next + q <= N;
        rows[q] = ok ? order[next + q] : 0;
        if constexpr (UPD) {
          a[q] = ok ? z[(int64_t)rows[q] * slab] : L::zero();
          b[q] = ok ? p[(int64_t)rows[q] * slab] : L::zero();
        } else {
          a[q] = ok ? src[(int64_t)rows[q] * slab] : L::zero();
        }
      }
#pragma unroll
      for (int q = 0; q < B; ++q) {
        if constexpr (UPD) {
          ring[q] = L::upd(a[q], b[q], beta);
          if (next + q <= N) p[(int64_t)rows[q] * slab] = ring[q];
        } else {
          ring[q] = a[q];
        }
      }
      left = min(B, N + 1 - next);
      next += B;
    }
    const V x = ring[0];
#pragma unroll
    for (int q = 0; q + 1 < B; ++q) ring[q] = ring[q + 1];
    --left;
    return x;
  }
  __device__ __forceinline__ void output(V v) { dst[(int64_t)(orow++) * slab] = v; }
};

// Level l receives x, the value of its k-th even row (row 2 k s, s = N / 2^l).
template <typename T, bool UPD, int J, int l>
__device__ __forceinline__ void syn_feed(SynState<T, UPD, J>& st, typename Lane<T>::V x) {
  using V = typename Lane<T>::V;
  if constexpr (l > J) {
    st.output(x);
  } else {
    constexpr int N = 1 << J;
    constexpr int s = N >> l;
    const int i = st.k[l]++;
    if (i == 0) {
      st.eo[l] = x;
      st.ea[l] = x;
      return;
    }
    // x is the old value of the even row m + s; the odd row m comes in now
    const int m = (2 * i - 1) * s;
    const T c = (T)exp2(0.5 * (double)l);
    const V d = st.input();
    const T wl = m - s == 0 ? T(1) : T(0.5);  // boundary weights of rows 0 and N
    const T wr = m + s == N ? T(1) : T(0.5);
    const V odd = T(0.5) * (st.eo[l] + x) + c * d;
    const V even = st.ea[l] - (c * wl) * d;    // row m - s, done at this level
    st.eo[l] = x;
    st.ea[l] = x - (c * wr) * d;
#pragma unroll 1
    for (int q = 0; q < 2; ++q) syn_feed<T, UPD, J, l + 1>(st, q == 0 ? even : odd);
  }
}

// After the coarsest values: level l passes its last even row (row N) on.
template <typename T, bool UPD, int J, int l>
__device__ __forceinline__ void syn_flush(SynState<T, UPD, J>& st) {
  if constexpr (l <= J) {
    syn_feed<T, UPD, J, l + 1>(st, st.ea[l]);
    syn_flush<T, UPD, J, l + 1>(st);
  }
}

// dst = W src for nrhs blocks of N + 1 slabs (src == dst allowed); with UPD
// the coefficients are p = z + beta_rhs p, written back to p (src unused).
template <typename T, bool UPD, int J>
__global__ __launch_bounds__(kStreamBlock) void wavelet_syn_stream_kernel(
    const T* src, T* dst, T* p, const T* __restrict__ z, const double* __restrict__ beta,
    const int* __restrict__ order, int64_t slab) {
  using V = typename Lane<T>::V;
  constexpr int N = 1 << J;
  const int64_t vslab = slab / Lane<T>::W;  // row stride in units of V
  const int64_t col = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
  if (col >= vslab) return;
  const int64_t off = (int64_t)blockIdx.y * (N + 1) * vslab + col;
  SynState<T, UPD, J> st;
#pragma unroll
  for (int l = 0; l <= J; ++l) st.k[l] = 0;
  st.left = 0;
  st.next = 0;
  st.orow = 0;
  st.order = order;
  st.slab = vslab;
  st.dst = reinterpret_cast<V*>(dst) + off;
  if constexpr (UPD) {
    st.p = reinterpret_cast<V*>(p) + off;
    st.z = reinterpret_cast<const V*>(z) + off;
    st.beta = beta[blockIdx.y];
  } else {
    st.src = reinterpret_cast<const V*>(src) + off;
  }
  // level 0: rows 0 and N
#pragma unroll 1
  for (int q = 0; q < 2; ++q) syn_feed<T, UPD, J, 1>(st, st.input());
  syn_flush<T, UPD, J, 1>(st);
}

template <typename T, bool UPD, int J>
hipError_t launch_syn_stream_j(hipStream_t s, const T* src, T* dst, T* p, const T* z,
                               const double* beta, const int* order, int64_t slab, int nrhs) {
  const int64_t threads = slab / Lane<T>::W;
  const dim3 grid((unsigned)((threads + kStreamBlock - 1) / kStreamBlock), nrhs);
  wavelet_syn_stream_kernel<T, UPD, J><<<grid, kStreamBlock, 0, s>>>(src, dst, p, z, beta, order,
                                                                     slab);
  return hipGetLastError();
}

template <typename T, bool DOT, int J>
hipError_t launch_ana_stream_j(hipStream_t s, T* X, const T* p, double* partials, int64_t slab,
                               int nrhs, int* nblk) {
  const int64_t threads = slab / Lane<T>::W;
  const dim3 grid((unsigned)((threads + kStreamBlock - 1) / kStreamBlock), nrhs);
  *nblk = (int)grid.x;
  wavelet_ana_stream_kernel<T, DOT, J><<<grid, kStreamBlock, 0, s>>>(X, p, partials, slab);
  return hipGetLastError();
}

}  // namespace

template <typename T, bool DOT>
hipError_t wavelet_ana_stream(hipStream_t s, T* X, const T* p, double* partials, int J,
                              int64_t slab, int nrhs, int* nblk) {
  if (J == 0) {
    const dim3 grid((unsigned)((slab + kStreamBlock - 1) / kStreamBlock), nrhs);
    *nblk = (int)grid.x;
    if constexpr (DOT) dot_rows2_kernel<T><<<grid, kStreamBlock, 0, s>>>(X, p, partials, slab);
    return hipGetLastError();
  }
  switch (J) {
#define STP_J(j) \
  case j: return launch_ana_stream_j<T, DOT, j>(s, X, p, partials, slab, nrhs, nblk);
    STP_J(1) STP_J(2) STP_J(3) STP_J(4) STP_J(5) STP_J(6) STP_J(7)
    STP_J(8) STP_J(9) STP_J(10) STP_J(11) STP_J(12) STP_J(13) STP_J(14)
#undef STP_J
    default: return hipErrorInvalidValue;
  }
}

int wavelet_stream_blocks(int64_t slab) { return (int)((slab + kStreamBlock - 1) / kStreamBlock); }

template <typename T, bool UPD>
hipError_t wavelet_syn_stream(hipStream_t s, const T* src, T* dst, T* p, const T* z,
                              const double* beta, const int* order, int J, int64_t slab,
                              int nrhs) {
  switch (J) {
#define STP_J(j) \
  case j: return launch_syn_stream_j<T, UPD, j>(s, src, dst, p, z, beta, order, slab, nrhs);
    STP_J(0) STP_J(1) STP_J(2) STP_J(3) STP_J(4) STP_J(5) STP_J(6) STP_J(7)
    STP_J(8) STP_J(9) STP_J(10) STP_J(11) STP_J(12) STP_J(13) STP_J(14)
#undef STP_J
    default: return hipErrorInvalidValue;
  }
}

// The rows in the order the synthesis cascade consumes their coefficients:
// the kernel's cascade run on row numbers.
std::vector<int> synthesis_read_order(int J) {
  const int N = 1 << J;
  std::vector<int> order, k(J + 2, 0);
  order.reserve(N + 1);
  // level l receives its next even row `row`
  auto feed = [&](auto&& self, int l, int row) -> void {
    if (l > J) return;
    const int i = k[l]++;
    if (i == 0) return;
    const int s = N >> l, m = row - s;
    order.push_back(m);
    self(self, l + 1, m - s);
    self(self, l + 1, m);
  };
  order.push_back(0);
  feed(feed, 1, 0);
  order.push_back(N);
  feed(feed, 1, N);
  for (int l = 1; l <= J; ++l) feed(feed, l + 1, N);
  return order;
}

template hipError_t wavelet_syn_stream<double, false>(hipStream_t, const double*, double*, double*,
                                                      const double*, const double*, const int*,
                                                      int, int64_t, int);
template hipError_t wavelet_syn_stream<double, true>(hipStream_t, const double*, double*, double*,
                                                     const double*, const double*, const int*, int,
                                                     int64_t, int);
template hipError_t wavelet_syn_stream<float, false>(hipStream_t, const float*, float*, float*,
                                                     const float*, const double*, const int*, int,
                                                     int64_t, int);
template hipError_t wavelet_syn_stream<float, true>(hipStream_t, const float*, float*, float*,
                                                    const float*, const double*, const int*, int,
                                                    int64_t, int);
template hipError_t wavelet_ana_stream<double, false>(hipStream_t, double*, const double*, double*,
                                                      int, int64_t, int, int*);
template hipError_t wavelet_ana_stream<double, true>(hipStream_t, double*, const double*, double*,
                                                     int, int64_t, int, int*);
template hipError_t wavelet_ana_stream<float, false>(hipStream_t, float*, const float*, double*,
                                                     int, int64_t, int, int*);
template hipError_t wavelet_ana_stream<float, true>(hipStream_t, float*, const float*, double*, int,
                                                    int64_t, int, int*);

}  // namespace stp
