// Streaming multigrid smoothing kernels (gfx950): the fine-grid work of one
// V-cycle level, three-colour Gauss-Seidel, with every operand in registers.
//
// Work decomposition.  One wavefront (64 lanes) owns one vertical strip of one
// time row (slab): 192 consecutive columns, three per lane (lane t holds
// columns gxs + 3t + {0, 1, 2}), and walks up the rows of the grid.  Holding
// three adjacent columns per lane makes the colour (i + j) mod 3 of "the
// column to relax" the same for every lane, so no lane idles in a colour
// phase.  Horizontal neighbours in other lanes come over DPP wave shifts.
//
// Schedule.  The 9 colour phases of 3 Gauss-Seidel steps are skewed by one
// row: at step s the wave loads row s + 1, then applies phase p to row s - p
// for p = 0..8 in increasing p.  When phase p touches row r, row r + 1 has
// just had phase p - 1 and row r - 1 had phase p one step earlier, so every
// neighbour holds exactly the value a global colour sweep would see: the
// result equals the global three-colour ordering bit for bit, with no halo
// along the rows.  A window of 12 rows per column lives in registers; the
// step loop is unrolled by 12 so every register index is a compile-time
// constant.
//
// Strips.  Neighbouring strips overlap: a strip needs H valid columns on each
// side of the columns it outputs (9 phases, plus one column for the residual
// and one for the restriction in the pre-smoothing kernel).  Strip starts are
// rounded down to 1 (mod 3) so that the active column of a phase is also a
// compile-time constant.  At the domain boundary no halo is needed.
//
// Kernels.  pre:  x <- forward steps from xin (or zero), residual, restriction
//                 b_c <- P^T (b - C x);   writes x and b_c.
//           post: x <- backward steps from xin + P e_c;   writes x.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace stp {

namespace {

constexpr int kStripCols = 192;  // 64 lanes x 3 columns
constexpr int kWin = 12;         // rows held per column
constexpr int kPhases = 9;       // 3 steps x 3 colours
constexpr int kHaloPre = 11;
constexpr int kHaloPost = 9;
constexpr int kWavesPerBlock = 4;

// DPP wave shifts: value held by lane t-1 (from_left) / lane t+1 (from_right);
// the lanes at the wave's edges receive 0.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

__device__ __forceinline__ int dpp_shr(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kDppWaveShr1, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kDppWaveShl1, 0xf, 0xf, false);
}
__device__ __forceinline__ double from_left(double v) {
  return __hiloint2double(dpp_shr(__double2hiint(v)), dpp_shr(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v) {
  return __hiloint2double(dpp_shl(__double2hiint(v)), dpp_shl(__double2loint(v)));
}
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(dpp_shr(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(dpp_shl(__float_as_int(v)));
}

template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    static_for<Begin + 1, End>(f);
  }
}

constexpr int mod(int a, int m) { return ((a % m) + m) % m; }

// A wave-uniform 64-bit offset, forced into scalar registers.  Row offsets go
// through here so that each load address is "scalar base + lane offset" and
// the compiler keeps no per-access 64-bit pointers in vector registers.
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

template <typename T>
struct State {
  T x[kWin][3];  // iterate, row r in slot r mod kWin
  T b[kWin][3];  // right-hand side
  T r[3][3];     // residual rows (pre-smoothing), row r in slot r mod 3
};

template <typename T>
struct StateP : State<T> {
  T px[2][3];  // prefetched iterate rows (2 = rows ahead)
  T pb[2][3];  // prefetched right-hand-side rows
  T ce[2][3];  // post: coarse correction rows J (slot J mod 2), coarse columns cI0 .. cI0 + 2
  T pce[3];    // post: prefetched coarse row
};

}  // namespace

// Strip s of a level with n columns and halo H: first column gxs (1 mod 3),
// output columns [lo, hi].  Returns false past the last strip.
__host__ __device__ inline bool strip_geometry(int s, int n, int H, int& gxs, int& lo, int& hi) {
  gxs = 1;
  lo = 1;
  for (int k = 0;; ++k) {
    const int right = gxs + kStripCols - 1;
    hi = right >= n ? n : right - H;
    if (k == s) return true;
    if (hi >= n) return false;
    lo = hi + 1;
    int g = lo - H;
    g -= mod(g - 1, 3);
    gxs = g;
  }
}

__host__ __device__ inline int strip_count(int n, int H) {
  int s = 0, gxs, lo, hi;
  while (strip_geometry(s, n, H, gxs, lo, hi) && hi < n) ++s;
  return s + 1;
}

namespace {

constexpr int kPf = 2;  // rows prefetched ahead of the one being assembled

// One Gauss-Seidel update of the column with in-lane index K in the row held
// in slot SR (neighbour rows in slots SN above, SS below).  Columns outside
// the grid have cinv = 0 and b = 0, so they stay exactly zero.
template <typename T, int K, int SR, int SN, int SS>
__device__ __forceinline__ void relax(State<T>& st, const T* cinv, T c1, T c2) {
  T xe, xw, xne, xsw;
  if constexpr (K < 2) {
    xe = st.x[SR][K + 1];
    xne = st.x[SN][K + 1];
  } else {
    xe = from_right(st.x[SR][0]);
    xne = from_right(st.x[SN][0]);
  }
  if constexpr (K > 0) {
    xw = st.x[SR][K - 1];
    xsw = st.x[SS][K - 1];
  } else {
    xw = from_left(st.x[SR][2]);
    xsw = from_left(st.x[SS][2]);
  }
  const T off = c1 * (((xe + xw) + st.x[SN][K]) + st.x[SS][K]) + c2 * (xne + xsw);
  st.x[SR][K] = (st.b[SR][K] - off) * cinv[K];
}

// residual of all three columns of the row in slot SR, stored in residual slot RS
template <typename T, int SR, int SN, int SS, int RS>
__device__ __forceinline__ void residual(State<T>& st, const bool* in, T c0, T c1, T c2) {
  const T e2 = from_right(st.x[SR][0]);
  const T ne2 = from_right(st.x[SN][0]);
  const T w0 = from_left(st.x[SR][2]);
  const T sw0 = from_left(st.x[SS][2]);
  static_for<0, 3>([&](auto KK) {
    constexpr int K = decltype(KK)::value;
    const T xe = K < 2 ? st.x[SR][K < 2 ? K + 1 : 0] : e2;
    const T xne = K < 2 ? st.x[SN][K < 2 ? K + 1 : 0] : ne2;
    const T xw = K > 0 ? st.x[SR][K > 0 ? K - 1 : 0] : w0;
    const T xsw = K > 0 ? st.x[SS][K > 0 ? K - 1 : 0] : sw0;
    const T off = c1 * (((xe + xw) + st.x[SN][K]) + st.x[SS][K]) + c2 * (xne + xsw);
    const T rv = st.b[SR][K] - (c0 * st.x[SR][K] + off);
    st.r[RS][K] = in[K] ? rv : T(0);
  });
}

// Everything a wave needs besides the register state.
template <typename T>
struct Args {
  const T* xin;
  const T* b;
  const T* ec;
  T* xout;
  T* bc;
  int64_t off, off_c;  // slab offsets of this row (fine, coarse)
  int n, pitch, nc, pitch_c;
  int gxc[3];   // this lane's columns, clamped into [1, n] (for loads)
  bool in[3];   // column inside the grid
  bool out[3];  // column written by this strip
  int gx[3];
  T cinv[3];    // 1/centre inside the grid, 0 outside
  T c0, c1, c2;
  // post: coarse columns cI0 .. cI0 + 2 of this lane, clamped, and masks
  int cic[3];
  bool cin[3];
  bool gx0_even;
};

// Prefetch row q (fine) into prefetch slot PS: x (unless x starts at zero) and b.
template <typename T, bool XIN, bool CHK, int PS>
__device__ __forceinline__ void prefetch_fine(StateP<T>& st, const Args<T>& A, int q) {
  if (CHK && (q < 1 || q > A.n)) {
    static_for<0, 3>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      if constexpr (XIN) st.px[PS][K] = T(0);
      st.pb[PS][K] = T(0);
    });
    return;
  }
  const int64_t ro = uniform(A.off + (int64_t)(q - 1) * A.pitch - 1);
  static_for<0, 3>([&](auto KK) {
    constexpr int K = decltype(KK)::value;
    if constexpr (XIN) st.px[PS][K] = A.xin[ro + A.gxc[K]];
    st.pb[PS][K] = A.b[ro + A.gxc[K]];
  });
}

// Prefetch coarse row J (post-smoothing) into the coarse prefetch slot.
template <typename T, bool CHK>
__device__ __forceinline__ void prefetch_coarse(StateP<T>& st, const Args<T>& A, int J) {
  if (CHK && (J < 1 || J > A.nc)) {
    static_for<0, 3>([&](auto KK) { st.pce[decltype(KK)::value] = T(0); });
    return;
  }
  const int64_t ro = uniform(A.off_c + (int64_t)(J - 1) * A.pitch_c - 1);
  static_for<0, 3>([&](auto KK) {
    constexpr int K = decltype(KK)::value;
    st.pce[K] = A.ec[ro + A.cic[K]];
  });
}

template <typename T, bool PRE, bool XIN, bool CHK, int U>
__device__ __forceinline__ void step(StateP<T>& st, const Args<T>& A, int s0) {
  const int s = s0 + U;
  const int n = A.n;
  // ---- assemble row s + 1 from its prefetched values
  {
    constexpr int SL = mod(U + 1, kWin);
    constexpr int PS = mod(U + 1, kPf);
    if constexpr (!PRE) {
      constexpr bool odd_row = mod(U + 1, 2) == 1;  // s0 is even
      // coarse rows: J0 = (s+1) >> 1 in ring slot J0 mod 2; for an odd fine
      // row the row above (J0 + 1) arrives now from the coarse prefetch slot
      const int gy = s + 1;
      // coarse row J0 = (s + 1) >> 1 = s0 / 2 + ((U + 1) >> 1); s0 / 2 is even
      constexpr int j0par = ((U + 1) >> 1) & 1;
      if constexpr (odd_row) {
        // coarse row J0 + 1 (first needed now) leaves the prefetch slot for
        // ring slot (J0 + 1) mod 2; columns outside the coarse grid are zero
        static_for<0, 3>([&](auto KK) {
          constexpr int K = decltype(KK)::value;
          st.ce[1 - j0par][K] = A.cin[K] ? st.pce[K] : T(0);
        });
      }
      T e0[3], e1[3];  // coarse rows J0 and J0 + 1 at coarse columns cI0 .. cI0 + 2
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        e0[K] = st.ce[j0par][K];
        e1[K] = st.ce[1 - j0par][K];
      });
      // P1 interpolation on the "/" mesh (see the tiled post kernel)
      T pe[3];
      if constexpr (!odd_row) {
        // even fine row: coarse row J0 only
        const T a0 = e0[0], a1 = T(0.5) * (e0[0] + e0[1]), a2 = e0[1];   // gx0 even
        const T b0 = T(0.5) * (e0[0] + e0[1]), b1 = e0[1], b2 = T(0.5) * (e0[1] + e0[2]);  // odd
        pe[0] = A.gx0_even ? a0 : b0;
        pe[1] = A.gx0_even ? a1 : b1;
        pe[2] = A.gx0_even ? a2 : b2;
      } else {
        // odd fine row: even column -> mean of rows J0, J0+1 in that column;
        // odd column -> mean of (left column, row J0) and (right column, row J0+1)
        const T a0 = T(0.5) * (e0[0] + e1[0]);
        const T a1 = T(0.5) * (e0[0] + e1[1]);
        const T a2 = T(0.5) * (e0[1] + e1[1]);
        const T b0 = T(0.5) * (e0[0] + e1[1]);
        const T b1 = T(0.5) * (e0[1] + e1[1]);
        const T b2 = T(0.5) * (e0[1] + e1[2]);
        pe[0] = A.gx0_even ? a0 : b0;
        pe[1] = A.gx0_even ? a1 : b1;
        pe[2] = A.gx0_even ? a2 : b2;
      }
      const bool rowin = !CHK || (gy >= 1 && gy <= n);
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const T xv = st.px[PS][K] + pe[K];
        st.x[SL][K] = (rowin && A.in[K]) ? xv : T(0);
        st.b[SL][K] = A.in[K] ? st.pb[PS][K] : T(0);
      });
    } else {
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        if constexpr (XIN) st.x[SL][K] = A.in[K] ? st.px[PS][K] : T(0);
        else st.x[SL][K] = T(0);
        st.b[SL][K] = A.in[K] ? st.pb[PS][K] : T(0);
      });
    }
    // ---- prefetch row s + 1 + kPf into the slot just emptied
    prefetch_fine<T, XIN || !PRE, CHK, PS>(st, A, s + 1 + kPf);
    if constexpr (!PRE) {
      if constexpr (mod(U, 2) == 0) prefetch_coarse<T, CHK>(st, A, (s + 4) >> 1);
    }
  }
  // ---- phases: p at row s - p.  Slots and the active column are compile-time.
  static_for<0, kPhases>([&](auto PP) {
    constexpr int P = decltype(PP)::value;
    constexpr int colour = PRE ? (P % 3) : (2 - P % 3);
    // row r = s0 + U - P; s0 = 0 mod 12 and strip starts = 1 mod 3:
    // (gx + r) mod 3 = colour  <=>  K = colour - 1 - (U - P)  (mod 3)
    constexpr int K = mod(colour - 1 - (U - P), 3);
    constexpr int SR = mod(U - P, kWin);
    constexpr int SN = mod(U - P + 1, kWin);
    constexpr int SS = mod(U - P - 1, kWin);
    const int r = s - P;
    if (!CHK || (r >= 1 && r <= n)) relax<T, K, SR, SN, SS>(st, A.cinv, A.c1, A.c2);
  });
  // ---- row s - 8 has had all nine phases: write it
  {
    constexpr int SW = mod(U - 8, kWin);
    const int r = s - 8;
    if (!CHK || (r >= 1 && r <= n)) {
      const int64_t ro = uniform(A.off + (int64_t)(r - 1) * A.pitch - 1);
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        if (A.out[K]) A.xout[ro + A.gx[K]] = st.x[SW][K];
      });
    }
  }
  if constexpr (PRE) {
    // ---- residual of row s - 9 (rows s - 10 .. s - 8 are final)
    constexpr int SR = mod(U - 9, kWin);
    constexpr int SN = mod(U - 8, kWin);
    constexpr int SS = mod(U - 10, kWin);
    constexpr int RS = mod(U - 9, 3);
    const int rr = s - 9;
    if (!CHK || (rr >= 1 && rr <= n)) {
      residual<T, SR, SN, SS, RS>(st, A.in, A.c0, A.c1, A.c2);
    } else {
      static_for<0, 3>([&](auto KK) { st.r[RS][decltype(KK)::value] = T(0); });
    }
    // ---- restriction of coarse row J once fine rows 2J-1, 2J, 2J+1 have residuals
    if constexpr (mod(U - 9, 2) == 1) {  // rr odd (s0 is even)
      if (!CHK || (rr >= 3 && rr <= n)) {
        const int J = (rr - 1) >> 1;
        constexpr int R1 = mod(U - 9, 3);   // row 2J + 1
        constexpr int R0 = mod(U - 10, 3);  // row 2J
        constexpr int Rm = mod(U - 11, 3);  // row 2J - 1
        const T e2 = from_right(st.r[R0][0]);
        const T ne2 = from_right(st.r[R1][0]);
        const T w0 = from_left(st.r[R0][2]);
        const T sw0 = from_left(st.r[Rm][2]);
        const int64_t ro = uniform(A.off_c + (int64_t)(J - 1) * A.pitch_c - 1);
        static_for<0, 3>([&](auto KK) {
          constexpr int K = decltype(KK)::value;
          const T re = K < 2 ? st.r[R0][K < 2 ? K + 1 : 0] : e2;
          const T rne = K < 2 ? st.r[R1][K < 2 ? K + 1 : 0] : ne2;
          const T rw = K > 0 ? st.r[R0][K > 0 ? K - 1 : 0] : w0;
          const T rsw = K > 0 ? st.r[Rm][K > 0 ? K - 1 : 0] : sw0;
          const T half = ((((re + rw) + st.r[R1][K]) + st.r[Rm][K]) + rne) + rsw;
          const int gx = A.gx[K];
          if (A.out[K] && !(gx & 1)) A.bc[ro + (gx >> 1)] = st.r[R0][K] + T(0.5) * half;
        });
      }
    }
  }
}

template <typename T, bool PRE, bool XIN, bool CHK, int... Us>
__device__ __forceinline__ void chunk(StateP<T>& st, const Args<T>& A, int s0,
                                      std::integer_sequence<int, Us...>) {
  // each step is a scheduling region of its own: the explicit prefetch already
  // hides the load latency, and letting the scheduler hoist loads across steps
  // only inflates register pressure
  ((step<T, PRE, XIN, CHK, Us>(st, A, s0), __builtin_amdgcn_sched_barrier(0)), ...);
}

template <typename T, bool PRE, bool XIN>
__global__ __launch_bounds__(64 * kWavesPerBlock) void mg_stream_kernel(
    const T* __restrict__ xin, const T* __restrict__ b, const T* __restrict__ ec,
    T* __restrict__ xout, T* __restrict__ bc, int l, int nstrips, int rows, double a,
    const double* __restrict__ sigma) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * kWavesPerBlock + wave;
  if (task >= rows * nstrips) return;  // whole wavefronts only
  const int row = task / nstrips;
  const int strip = task - row * nstrips;

  Args<T> A;
  A.xin = xin;
  A.b = b;
  A.ec = ec;
  A.xout = xout;
  A.bc = bc;
  A.n = grid_n(l);
  A.pitch = line_pitch(l);
  A.nc = grid_n(l - 1);
  A.pitch_c = line_pitch(l - 1);
  A.off = (int64_t)row * slab_elems(l);
  A.off_c = (int64_t)row * slab_elems(l - 1);
  int gxs, lo, hi;
  strip_geometry(strip, A.n, PRE ? kHaloPre : kHaloPost, gxs, lo, hi);

  const double sg = sigma ? sigma[row] : 0.0;
  const double h = 1.0 / (double)(1 << l);
  const double m = h * h / 12.0;
  const double c0d = 4.0 * a + 6.0 * m * sg;
  A.c0 = (T)c0d;
  A.c1 = (T)(-a + m * sg);
  A.c2 = (T)(m * sg);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int gx = gxs + 3 * lane + k;
    A.gx[k] = gx;
    A.in[k] = gx >= 1 && gx <= A.n;
    A.out[k] = gx >= lo && gx <= hi;
    A.gxc[k] = gx < 1 ? 1 : (gx > A.n ? A.n : gx);
    A.cinv[k] = A.in[k] ? (T)(1.0 / c0d) : T(0);
  }
  const int cI0 = (gxs + 3 * lane) >> 1;
  A.gx0_even = ((gxs + 3 * lane) & 1) == 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int I = cI0 + k;
    A.cin[k] = I >= 1 && I <= A.nc;
    A.cic[k] = I < 1 ? 1 : (I > A.nc ? (A.nc > 0 ? A.nc : 1) : I);
  }

  StateP<T> st;
#pragma unroll
  for (int i = 0; i < kWin; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      st.x[i][k] = T(0);
      st.b[i][k] = T(0);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) st.r[i][k] = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    st.ce[0][k] = T(0);
    st.ce[1][k] = T(0);
  }
  // prime the pipeline: fine rows 1 .. kPf; for post, coarse row 1 (first
  // needed by fine row 1; coarse row 0 is the zero boundary)
  prefetch_fine<T, XIN || !PRE, true, 1>(st, A, 1);
  prefetch_fine<T, XIN || !PRE, true, 0>(st, A, 2);
  if constexpr (!PRE) prefetch_coarse<T, true>(st, A, 1);
  // three loops over chunks of kWin steps: the first and last touch rows
  // outside [1, n] and check every row; the middle ones run check-free
  const int last = A.n + (PRE ? 9 : 8);
  int s0 = 0;
  chunk<T, PRE, XIN, true>(st, A, s0, std::make_integer_sequence<int, kWin>{});
  for (s0 = kWin; s0 + 16 <= A.n; s0 += kWin)
    chunk<T, PRE, XIN, false>(st, A, s0, std::make_integer_sequence<int, kWin>{});
  for (; s0 <= last; s0 += kWin)
    chunk<T, PRE, XIN, true>(st, A, s0, std::make_integer_sequence<int, kWin>{});
}

}  // namespace

template <typename T>
hipError_t mg_pre_stream(hipStream_t s, const T* xin, const T* b, T* xout, T* bc, int l, int rows,
                         double a, const double* sigma) {
  const int ns = strip_count(grid_n(l), kHaloPre);
  const int64_t tasks = (int64_t)rows * ns;
  const unsigned blocks = (unsigned)((tasks + kWavesPerBlock - 1) / kWavesPerBlock);
  if (xin)
    mg_stream_kernel<T, true, true><<<blocks, 64 * kWavesPerBlock, 0, s>>>(xin, b, nullptr, xout, bc,
                                                                           l, ns, rows, a, sigma);
  else
    mg_stream_kernel<T, true, false><<<blocks, 64 * kWavesPerBlock, 0, s>>>(xin, b, nullptr, xout, bc,
                                                                            l, ns, rows, a, sigma);
  return hipGetLastError();
}

template <typename T>
hipError_t mg_post_stream(hipStream_t s, const T* xin, const T* b, const T* ec, T* xout, int l,
                          int rows, double a, const double* sigma) {
  const int ns = strip_count(grid_n(l), kHaloPost);
  const int64_t tasks = (int64_t)rows * ns;
  const unsigned blocks = (unsigned)((tasks + kWavesPerBlock - 1) / kWavesPerBlock);
  mg_stream_kernel<T, false, true><<<blocks, 64 * kWavesPerBlock, 0, s>>>(xin, b, ec, xout, nullptr,
                                                                           l, ns, rows, a, sigma);
  return hipGetLastError();
}

template hipError_t mg_pre_stream<double>(hipStream_t, const double*, const double*, double*,
                                          double*, int, int, double, const double*);
template hipError_t mg_pre_stream<float>(hipStream_t, const float*, const float*, float*, float*,
                                         int, int, double, const double*);
template hipError_t mg_post_stream<double>(hipStream_t, const double*, const double*,
                                           const double*, double*, int, int, double,
                                           const double*);
template hipError_t mg_post_stream<float>(hipStream_t, const float*, const float*, const float*,
                                          float*, int, int, double, const double*);

}  // namespace stp
