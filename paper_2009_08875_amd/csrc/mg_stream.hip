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
// row: at step s the wave assembles row s + 1, then applies phase p to row
// s - p for p = 0..8 in increasing p.  When phase p touches row r, row r + 1
// has just had phase p - 1 and row r - 1 had phase p one step earlier, so
// every neighbour holds exactly the value a global colour sweep would see:
// the result equals the global three-colour ordering, with no halo along the
// rows.  A window of 12 rows per column lives in registers; the step loop is
// unrolled by 12 so every register index is a compile-time constant; rows are
// prefetched two steps ahead.
//
// Within a step, phase p reads one value written by phase p - 1 (the
// north-east neighbour in a forward sweep, the north neighbour in a backward
// sweep).  That value enters last, through one fused multiply-add, so the
// dependency chain through a step is one FMA per phase; without the mass term
// (sigma = 0) the north-east coefficient is zero and forward steps have no
// chain at all.
//
// Strips.  Neighbouring strips overlap: a strip needs H valid columns on each
// side of the columns it outputs (9 phases, plus one column for the residual
// and one for the restriction in the pre-smoothing kernel, one for A x in the
// fused post-smoothing variant).  Strip starts are rounded down to 1 (mod 3)
// so that the active column of a phase is also a compile-time constant.  At
// the domain boundary no halo is needed.
//
// Balance.  The (row, strip) tasks are cut into segments of consecutive grid
// rows so that every resident wave gets the same number of row steps; a
// segment that does not start at the bottom of the grid restarts the
// pipeline H rows lower (rounded down to the 12-row unroll), recomputing
// those rows without writing them.  How many segments (one per time row, or
// about as many as fit the resident waves) is picked per level and row count
// by the launch autotuner; all give the same result.
//
// Kernels.  pre:  x <- forward steps from xin (or zero), residual, restriction
//                 b_c <- P^T (b - C x);   writes x and b_c.
//           post: x <- backward steps from xin + P e_c;   writes x, or A x.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "tune.h"

namespace stp {

namespace {

constexpr int kStripCols = 192;  // 64 lanes x 3 columns
constexpr int kWin = 12;         // rows held per column
constexpr int kPhases = 9;       // 3 steps x 3 colours
constexpr int kHaloPre = 11;
constexpr int kHaloPost = 9;
constexpr int kHaloPostA = 10;
constexpr int kWavesPerBlock = 4;
constexpr int kPf = 2;           // rows prefetched ahead of the one being assembled

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

// Buffer resources: global memory is accessed through a per-row descriptor
// whose record count covers exactly the valid elements; lanes outside it read
// zero and their stores are dropped by the hardware range check, so no access
// needs a branch or a mask.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw (untyped) access
constexpr int kCachePolicyNT = 2;       // non-temporal (streaming) store

__device__ __forceinline__ Rsrc rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
template <typename T>
__device__ __forceinline__ T buf_load(Rsrc r, int voff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
// Stores carry the non-temporal cache policy: a written row is not read again
// by this kernel, and streaming it out keeps the L2 for the rows in flight.
template <typename T>
__device__ __forceinline__ void buf_store(T v, Rsrc r, int voff) {
  if constexpr (sizeof(T) == 8) {
    using V2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, voff, 0, kCachePolicyNT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, 0,
                                         kCachePolicyNT);
  }
}

template <typename T>
struct State {
  T x[kWin][3];  // iterate, row r in slot r mod kWin
  T* bl;         // right-hand side window in LDS: bl[(slot * 3 + column) * 64 + lane]
  T r[3][3];     // residual rows (pre-smoothing), row r in slot r mod 3
  T* stg;        // per-wave LDS staging row (192 elements) for coalesced global access
  T px[kPf][3];  // prefetched iterate rows, element layout: [j] = strip column t + 64 j
  T pb[kPf][3];  // prefetched right-hand-side rows, element layout
  T ce[2][3];    // post: coarse correction rows J (slot J mod 2), coarse columns cI0 .. cI0 + 2
  T pce[3];      // post: prefetched coarse row
};

// The right-hand side of a row stays in LDS while the row is in flight: each
// lane only ever reads its own three columns, laid out lane-contiguous so that
// the accesses are conflict-free.
template <typename T, int SLOT, int K>
__device__ __forceinline__ T bget(const State<T>& st) {
  return st.bl[(SLOT * 3 + K) * 64 + (threadIdx.x & 63)];
}
template <typename T, int SLOT, int K>
__device__ __forceinline__ void bset(State<T>& st, T v) {
  st.bl[(SLOT * 3 + K) * 64 + (threadIdx.x & 63)] = v;
}

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

// Everything a wave needs for one (row, strip) task besides the register state.
template <typename T>
struct Args {
  const T* xin;
  const T* b;
  const T* ec;
  T* xout;
  T* bc;
  int64_t off, off_c;  // slab offsets of this row (fine, coarse)
  int n, pitch, nc, pitch_c;
  int ys, ye;   // rows of this segment that are written
  // Global memory is accessed in the coalesced element layout: lane t handles
  // strip elements e_j = t + 64 j (columns gxs + e_j), and LDS moves values
  // between that layout and the register layout (columns gxs + 3t + k).
  int eld[3];   // byte offset of element e_j from column 1 (negative = outside)
  int kld[3];   // byte offset of register column k from column 1
  int est[3];   // byte offset of element e_j from column lo (store range [lo, hi])
  int eslot[3]; // LDS offset of element e_j in the [column mod 3][column / 3] layout
  int cld[3];   // post: byte offsets of coarse columns cI0 .. cI0 + 2 from coarse column 1
  int cst[2];   // pre: byte offsets of staged coarse values lane + 64 j from coarse column Ilo
  int Ilo, Ihi; // pre: coarse columns written by this strip
  bool in[3];   // column inside the grid
  bool out[3];  // column written by this strip
  int gx[3];
  // The right-hand side is stored scaled by 1 / centre, b' = b / c0, and the
  // update reads x = b' - qx (E + W) - qy (N + S) - q2 (NE + SW) with
  // q = c / c0, one fused multiply-add per neighbour; the q are zero outside
  // the grid so those columns stay exactly zero.  qx = qy unless the
  // diffusion tensor is anisotropic (Section 4).
  T qx[3];
  T qy[3];
  T q2[3];
  T cinv;       // 1 / c0 (scales b when it enters the window)
  T c0;
  // A_x itself (the fused A x output): heat equation (5 points, -1 and 4) or
  // the stencil of A_D + c M (centre, x, y, "/" diagonal)
  bool heat;
  T a0, ax, ay, ad;
  int lo, hi;   // output columns of this strip
  int cI0;      // pre: first coarse column of the strip, (gxs + 1) / 2
  bool gx0_even;
};

// One Gauss-Seidel update of the column with in-lane index K in the row held
// in slot SR (neighbour rows in slots SN above, SS below); t is its scaled
// right-hand side b / c0.  Columns outside
// the grid have cinv = qx = qy = q2 = 0 and b = 0, so they stay exactly zero.
// FWD: the value written by the previous phase is the north-east neighbour
// (it only matters with the mass term, DIAG); backward: the north neighbour.
template <typename T, bool FWD, bool DIAG, int K, int SR, int SN, int SS>
__device__ __forceinline__ void relax(State<T>& st, const Args<T>& A, T t) {
  T xe, xw, xne = T(0), xsw = T(0);
  if constexpr (K < 2) {
    xe = st.x[SR][K + 1];
    if constexpr (DIAG) xne = st.x[SN][K + 1];
  } else {
    xe = from_right(st.x[SR][0]);
    if constexpr (DIAG) xne = from_right(st.x[SN][0]);
  }
  if constexpr (K > 0) {
    xw = st.x[SR][K - 1];
    if constexpr (DIAG) xsw = st.x[SS][K - 1];
  } else {
    xw = from_left(st.x[SR][2]);
    if constexpr (DIAG) xsw = from_left(st.x[SS][2]);
  }
  const T xn = st.x[SN][K], xs = st.x[SS][K];
  const T m1 = -A.qx[K], m1y = -A.qy[K], m2 = -A.q2[K];
  if constexpr (FWD) {
    // the north-east neighbour was written by the previous phase: it goes last
    t = fma(m1, xe, t);
    t = fma(m1, xw, t);
    t = fma(m1y, xn, t);
    t = fma(m1y, xs, t);
    if constexpr (DIAG) {
      t = fma(m2, xsw, t);
      t = fma(m2, xne, t);
    }
  } else {
    // the north neighbour was written by the previous phase: it goes last
    t = fma(m1, xe, t);
    t = fma(m1, xw, t);
    t = fma(m1y, xs, t);
    if constexpr (DIAG) {
      t = fma(m2, xne, t);
      t = fma(m2, xsw, t);
    }
    t = fma(m1y, xn, t);
  }
  st.x[SR][K] = t;
}

// residual of all three columns of the row in slot SR, stored in residual slot RS
template <typename T, bool DIAG, int SR, int SN, int SS, int RS>
__device__ __forceinline__ void residual(State<T>& st, const Args<T>& A) {
  const T e2 = from_right(st.x[SR][0]);
  const T w0 = from_left(st.x[SR][2]);
  T ne2 = T(0), sw0 = T(0);
  if constexpr (DIAG) {
    ne2 = from_right(st.x[SN][0]);
    sw0 = from_left(st.x[SS][2]);
  }
  static_for<0, 3>([&](auto KK) {
    constexpr int K = decltype(KK)::value;
    const T xe = K < 2 ? st.x[SR][K < 2 ? K + 1 : 0] : e2;
    const T xw = K > 0 ? st.x[SR][K > 0 ? K - 1 : 0] : w0;
    T t = bget<T, SR, K>(st) - st.x[SR][K];
    const T m1 = -A.qx[K], m1y = -A.qy[K];
    t = fma(m1, xe, t);
    t = fma(m1, xw, t);
    t = fma(m1y, st.x[SN][K], t);
    t = fma(m1y, st.x[SS][K], t);
    if constexpr (DIAG) {
      const T xne = K < 2 ? st.x[SN][K < 2 ? K + 1 : 0] : ne2;
      const T xsw = K > 0 ? st.x[SS][K > 0 ? K - 1 : 0] : sw0;
      const T m2 = -A.q2[K];
      t = fma(m2, xne, t);
      t = fma(m2, xsw, t);
    }
    const T rv = A.c0 * t;
    st.r[RS][K] = A.in[K] ? rv : T(0);
  });
}

// Prefetch fine row q into prefetch slot PS: b coalesced (element layout; it
// goes to LDS), x directly in the register layout (it is needed as soon as
// the row is assembled).  Rows outside [1, n] and columns outside the grid
// read as zero.
template <typename T, bool XLOAD, bool CHK, int PS>
__device__ __forceinline__ void prefetch_fine(State<T>& st, const Args<T>& A, int q) {
  const bool ok = !CHK || (q >= 1 && q <= A.n);
  const int64_t ro = A.off + (int64_t)(ok ? q - 1 : 0) * A.pitch;
  const uint32_t bytes = ok ? (uint32_t)(A.n * sizeof(T)) : 0u;
  const Rsrc rb = rsrc(A.b + ro, bytes);
  static_for<0, 3>([&](auto JJ) {
    constexpr int J = decltype(JJ)::value;
    st.pb[PS][J] = buf_load<T>(rb, A.eld[J]);
  });
  if constexpr (XLOAD) {
    const Rsrc rx = rsrc(A.xin + ro, bytes);
    static_for<0, 3>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      st.px[PS][K] = buf_load<T>(rx, A.kld[K]);
    });
  }
}

// Prefetch coarse row J (post-smoothing) into the coarse prefetch slot; rows
// and columns outside the coarse grid read as zero.
template <typename T, bool CHK>
__device__ __forceinline__ void prefetch_coarse(State<T>& st, const Args<T>& A, int J) {
  const bool ok = !CHK || (J >= 1 && J <= A.nc);
  const int64_t ro = A.off_c + (int64_t)(ok ? J - 1 : 0) * A.pitch_c;
  const Rsrc re = rsrc(A.ec + ro, ok ? (uint32_t)(A.nc * sizeof(T)) : 0u);
  static_for<0, 3>([&](auto KK) {
    constexpr int K = decltype(KK)::value;
    st.pce[K] = buf_load<T>(re, A.cld[K]);
  });
}

template <typename T, bool PRE, bool XIN, bool DIAG, bool WRITE_A, bool CHK, int U>
__device__ __forceinline__ void step(State<T>& st, const Args<T>& A, int s0) {
  const int s = s0 + U;
  const int n = A.n;
  // ---- the right-hand sides of the nine rows this step relaxes (rows s - 8
  // .. s, all in the LDS window already) are read first, so that their LDS
  // latency overlaps the assembly of row s + 1 instead of stalling each phase
  T bv[kPhases];
  static_for<0, kPhases>([&](auto PP) {
    constexpr int P = decltype(PP)::value;
    constexpr int colour = PRE ? (P % 3) : (2 - P % 3);
    bv[P] = bget<T, mod(U - P, kWin), mod(colour - 1 - (U - P), 3)>(st);
  });
  __builtin_amdgcn_sched_barrier(0);
  // ---- assemble row s + 1 from its prefetched values
  {
    constexpr int SL = mod(U + 1, kWin);
    constexpr int PS = mod(U + 1, kPf);
    if constexpr (!PRE) {
      constexpr bool odd_row = mod(U + 1, 2) == 1;  // s0 is a multiple of 12
      // coarse row J0 = (s + 1) >> 1 = s0 / 2 + ((U + 1) >> 1); s0 / 2 is even
      constexpr int j0par = ((U + 1) >> 1) & 1;
      if constexpr (odd_row) {
        // coarse row J0 + 1 (first needed now) leaves the prefetch slot for
        // ring slot (J0 + 1) mod 2; columns outside the coarse grid are zero
        static_for<0, 3>([&](auto KK) {
          constexpr int K = decltype(KK)::value;
          st.ce[1 - j0par][K] = st.pce[K];
        });
      }
      T e0[3], e1[3];  // coarse rows J0 and J0 + 1 at coarse columns cI0 .. cI0 + 2
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        e0[K] = st.ce[j0par][K];
        e1[K] = st.ce[1 - j0par][K];
      });
      // P1 interpolation of the coarse correction on the "/" mesh
      T pe[3];
      if constexpr (!odd_row) {
        // even fine row: coarse row J0 only (a: first column even, b: odd)
        const T a0 = e0[0], a1 = T(0.5) * (e0[0] + e0[1]), a2 = e0[1];
        const T b0 = T(0.5) * (e0[0] + e0[1]), b1 = e0[1], b2 = T(0.5) * (e0[1] + e0[2]);
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
      // out-of-grid columns and rows read zero from both x and the coarse grid
      static_for<0, 3>([&](auto JJ) {
        constexpr int J = decltype(JJ)::value;
        st.bl[SL * 192 + A.eslot[J]] = st.pb[PS][J] * A.cinv;
      });
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        st.x[SL][K] = st.px[PS][K] + pe[K];
      });
    } else {
      static_for<0, 3>([&](auto JJ) {
        constexpr int J = decltype(JJ)::value;
        st.bl[SL * 192 + A.eslot[J]] = st.pb[PS][J] * A.cinv;
      });
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        st.x[SL][K] = XIN ? st.px[PS][K] : T(0);
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
    if (!CHK || (r >= 1 && r <= n)) relax<T, PRE, DIAG, K, SR, SN, SS>(st, A, bv[P]);
  });
  if constexpr (!WRITE_A) {
    // ---- row s - 8 has had all nine phases: write it (coalesced, via LDS;
    // rows outside [ys, ye] and columns outside [lo, hi] are dropped)
    constexpr int SW = mod(U - 8, kWin);
    const int r = s - 8;
    const int lane = threadIdx.x & 63;
    static_for<0, 3>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      st.stg[K * 64 + lane] = st.x[SW][K];
    });
    const bool ok = r >= A.ys && r <= A.ye;
    const int64_t ro = A.off + (int64_t)(ok ? r - 1 : 0) * A.pitch + (A.lo - 1);
    const Rsrc rs = rsrc(A.xout + ro, ok ? (uint32_t)((A.hi - A.lo + 1) * sizeof(T)) : 0u);
    static_for<0, 3>([&](auto JJ) {
      constexpr int J = decltype(JJ)::value;
      buf_store<T>(st.stg[A.eslot[J]], rs, A.est[J]);
    });
  } else {
    // ---- A x of row s - 9 (rows s - 10 .. s - 8 are final)
    constexpr int SR = mod(U - 9, kWin);
    constexpr int SN = mod(U - 8, kWin);
    constexpr int SS = mod(U - 10, kWin);
    const int r = s - 9;
    const T e2 = from_right(st.x[SR][0]);
    const T w0 = from_left(st.x[SR][2]);
    const int lane = threadIdx.x & 63;
    if (A.heat) {
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const T xe = K < 2 ? st.x[SR][K < 2 ? K + 1 : 0] : e2;
        const T xw = K > 0 ? st.x[SR][K > 0 ? K - 1 : 0] : w0;
        st.stg[K * 64 + lane] = (((T(4) * st.x[SR][K] - xe) - xw) - st.x[SN][K]) - st.x[SS][K];
      });
    } else {
      // A_D + c M (Section 4): the 7-point stencil, "/" neighbours included
      const T ne2 = from_right(st.x[SN][0]);
      const T sw0 = from_left(st.x[SS][2]);
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const T xe = K < 2 ? st.x[SR][K < 2 ? K + 1 : 0] : e2;
        const T xw = K > 0 ? st.x[SR][K > 0 ? K - 1 : 0] : w0;
        const T xne = K < 2 ? st.x[SN][K < 2 ? K + 1 : 0] : ne2;
        const T xsw = K > 0 ? st.x[SS][K > 0 ? K - 1 : 0] : sw0;
        st.stg[K * 64 + lane] = ((A.a0 * st.x[SR][K] + A.ax * (xe + xw)) +
                                 A.ay * (st.x[SN][K] + st.x[SS][K])) +
                                A.ad * (xne + xsw);
      });
    }
    const bool ok = r >= A.ys && r <= A.ye;
    const int64_t ro = A.off + (int64_t)(ok ? r - 1 : 0) * A.pitch + (A.lo - 1);
    const Rsrc rs = rsrc(A.xout + ro, ok ? (uint32_t)((A.hi - A.lo + 1) * sizeof(T)) : 0u);
    static_for<0, 3>([&](auto JJ) {
      constexpr int J = decltype(JJ)::value;
      buf_store<T>(st.stg[A.eslot[J]], rs, A.est[J]);
    });
  }
  if constexpr (PRE) {
    // ---- residual of row s - 9 (rows s - 10 .. s - 8 are final)
    constexpr int SR = mod(U - 9, kWin);
    constexpr int SN = mod(U - 8, kWin);
    constexpr int SS = mod(U - 10, kWin);
    constexpr int RS = mod(U - 9, 3);
    const int rr = s - 9;
    if (!CHK || (rr >= 1 && rr <= n)) {
      residual<T, DIAG, SR, SN, SS, RS>(st, A);
    } else {
      static_for<0, 3>([&](auto KK) { st.r[RS][decltype(KK)::value] = T(0); });
    }
    // ---- restriction of coarse row J once fine rows 2J-1, 2J, 2J+1 have residuals;
    // the segment holding fine row 2J writes it
    if constexpr (mod(U - 9, 2) == 1) {  // rr odd (s0 is even)
      const int J = (rr - 1) >> 1;
      constexpr int R1 = mod(U - 9, 3);   // row 2J + 1
      constexpr int R0 = mod(U - 10, 3);  // row 2J
      constexpr int Rm = mod(U - 11, 3);  // row 2J - 1
      const T e2 = from_right(st.r[R0][0]);
      const T ne2 = from_right(st.r[R1][0]);
      const T w0 = from_left(st.r[R0][2]);
      const T sw0 = from_left(st.r[Rm][2]);
      const int lane = threadIdx.x & 63;
      // coarse node I = gx / 2 of an even column goes to staging slot
      // I - cI0 (cI0 = (gxs + 1) / 2, the strip's first coarse column; odd
      // columns write a slot that is never read), then the wave stores the
      // strip's coarse values coalesced
      static_for<0, 3>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const T re = K < 2 ? st.r[R0][K < 2 ? K + 1 : 0] : e2;
        const T rne = K < 2 ? st.r[R1][K < 2 ? K + 1 : 0] : ne2;
        const T rw = K > 0 ? st.r[R0][K > 0 ? K - 1 : 0] : w0;
        const T rsw = K > 0 ? st.r[Rm][K > 0 ? K - 1 : 0] : sw0;
        const T half = ((((re + rw) + st.r[R1][K]) + st.r[Rm][K]) + rne) + rsw;
        const int gx = A.gx[K];
        const int slot = (gx & 1) ? 96 + lane : (gx >> 1) - A.cI0;
        st.stg[slot] = st.r[R0][K] + T(0.5) * half;
      });
      // the segment holding fine row 2J writes coarse row J
      const bool ok = rr >= 3 && rr - 1 >= A.ys && rr - 1 <= A.ye && A.Ihi >= A.Ilo;
      const int64_t ro = A.off_c + (int64_t)(ok ? J - 1 : 0) * A.pitch_c + (A.Ilo - 1);
      const Rsrc rc = rsrc(A.bc + ro, ok ? (uint32_t)((A.Ihi - A.Ilo + 1) * sizeof(T)) : 0u);
      static_for<0, 2>([&](auto JJ) {
        constexpr int Jc = decltype(JJ)::value;
        buf_store<T>(st.stg[lane + 64 * Jc], rc, A.cst[Jc]);
      });
    }
  }
}

template <typename T, bool PRE, bool XIN, bool DIAG, bool WRITE_A, bool CHK, int... Us>
__device__ __forceinline__ void chunk(State<T>& st, const Args<T>& A, int s0,
                                      std::integer_sequence<int, Us...>) {
  // one scheduling region per step, so that the two-row prefetch stays where
  // it was issued
  ((step<T, PRE, XIN, DIAG, WRITE_A, CHK, Us>(st, A, s0), __builtin_amdgcn_sched_barrier(0)), ...);
}

// Run rows [ys, ye] of task (row, strip).
template <typename T, bool PRE, bool XIN, bool DIAG, bool WRITE_A>
__device__ __forceinline__ void run_segment(const T* __restrict__ xin, const T* __restrict__ b,
                                            const T* __restrict__ ec, T* __restrict__ xout,
                                            T* __restrict__ bc, int l, int row, int strip, int ys,
                                            int ye, double a, const double* __restrict__ sigma,
                                            const SpaceOp& op, T* bwin, T* stg) {
  const int lane = threadIdx.x & 63;
  constexpr int H = PRE ? kHaloPre : (WRITE_A ? kHaloPostA : kHaloPost);
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
  A.ys = ys;
  A.ye = ye;
  int gxs, lo, hi;
  strip_geometry(strip, A.n, H, gxs, lo, hi);

  const double sg = sigma ? sigma[row] : 0.0;
  const Stencil sc = stencil_of(op, a, sg, l);
  const double c0d = sc.c0;
  A.c0 = (T)c0d;
  A.cinv = (T)(1.0 / c0d);
  A.heat = op.heat();
  {
    const Stencil as = stencil_of(op, 1.0, 0.0, l);
    A.a0 = (T)as.c0;
    A.ax = (T)as.cx;
    A.ay = (T)as.cy;
    A.ad = (T)as.cd;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int gx = gxs + 3 * lane + k;
    A.gx[k] = gx;
    A.in[k] = gx >= 1 && gx <= A.n;
    A.out[k] = gx >= lo && gx <= hi;
    A.qx[k] = A.in[k] ? (T)(sc.cx / c0d) : T(0);
    A.qy[k] = A.in[k] ? (T)(sc.cy / c0d) : T(0);
    A.q2[k] = A.in[k] ? (T)(sc.cd / c0d) : T(0);
    A.kld[k] = (gx - 1) * (int)sizeof(T);
  }
  A.lo = lo;
  A.hi = hi;
  A.cI0 = (gxs + 1) >> 1;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int e = lane + 64 * j;
    const int c = gxs + e;
    A.eld[j] = (int)((c - 1) * (int)sizeof(T));  // negative (out of range) left of the grid
    A.est[j] = (int)((c - lo) * (int)sizeof(T));
    A.eslot[j] = (e % 3) * 64 + e / 3;
  }
  // coarse columns written by this strip: fine column 2I in [lo, hi]
  A.Ilo = (lo + 1) >> 1;
  A.Ihi = hi >> 1;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = lane + 64 * j;  // staged coarse value: column cI0 + i (valid for i < 96)
    A.cst[j] = i < 96 ? (A.cI0 + i - A.Ilo) * (int)sizeof(T) : -1;
  }
  const int cI0 = (gxs + 3 * lane) >> 1;
  A.gx0_even = ((gxs + 3 * lane) & 1) == 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) A.cld[k] = (cI0 + k - 1) * (int)sizeof(T);

  State<T> st;
  st.bl = bwin;
  st.stg = stg;
#pragma unroll
  for (int i = 0; i < kWin; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      st.x[i][k] = T(0);
      st.bl[(i * 3 + k) * 64 + lane] = T(0);
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
  // first step: far enough below ys that the rows it cannot see (treated as
  // zero) no longer influence rows >= ys, and a multiple of the unroll
  int s0 = ys - H - 1;
  s0 = s0 <= 0 ? 0 : (s0 / kWin) * kWin;
  // prime the pipeline: fine rows s0 + 1 .. s0 + kPf; for post, coarse row
  // s0 / 2 into ring slot 0 (s0 / 2 is even) and coarse row s0 / 2 + 1 into
  // the prefetch slot (both zero beyond the coarse grid)
  prefetch_fine<T, XIN || !PRE, true, mod(1, kPf)>(st, A, s0 + 1);
  prefetch_fine<T, XIN || !PRE, true, mod(2, kPf)>(st, A, s0 + 2);
  if constexpr (!PRE) {
    if (s0 > 0) {
      prefetch_coarse<T, true>(st, A, s0 / 2);
#pragma unroll
      for (int k = 0; k < 3; ++k) st.ce[0][k] = st.pce[k];
    }
    prefetch_coarse<T, true>(st, A, s0 / 2 + 1);
  }
  // chunks of kWin steps: those touching rows outside [1, n] check every row,
  // the others run check-free
  const int last = ye + (PRE || WRITE_A ? 10 : 8);
  for (; s0 <= last && s0 < kWin; s0 += kWin)
    chunk<T, PRE, XIN, DIAG, WRITE_A, true>(st, A, s0, std::make_integer_sequence<int, kWin>{});
  for (; s0 <= last && s0 + 16 <= A.n; s0 += kWin)
    chunk<T, PRE, XIN, DIAG, WRITE_A, false>(st, A, s0, std::make_integer_sequence<int, kWin>{});
  for (; s0 <= last; s0 += kWin)
    chunk<T, PRE, XIN, DIAG, WRITE_A, true>(st, A, s0, std::make_integer_sequence<int, kWin>{});
}

// Waves come in groups of nstrips, one wave per strip of a time row; group g
// handles grid rows [g * units / groups, (g + 1) * units / groups) of the
// concatenation of all time rows (n grid rows each), and all waves of a group
// walk the same rows side by side, so that the strips of one grid line are
// read and written together.
template <typename T, bool PRE, bool XIN, bool DIAG, bool WRITE_A>
__global__ __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(2))) void mg_stream_kernel(
    const T* __restrict__ xin, const T* __restrict__ b, const T* __restrict__ ec,
    T* __restrict__ xout, T* __restrict__ bc, int l, int nstrips, int rows, int groups, double a,
    const double* __restrict__ sigma, SpaceOp op) {
  __shared__ T bwin[kWavesPerBlock][kWin * 3 * 64];
  __shared__ T stg[kWavesPerBlock][kStripCols];
  // the wave index is uniform across the wave: say so, so that every row and
  // segment quantity derived from it lives in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
  const int g = w / nstrips;
  const int strip = w - g * nstrips;
  if (g >= groups) return;  // whole wavefronts only (no barriers below)
  const int n = grid_n(l);
  const int64_t units = (int64_t)rows * n;
  const int64_t ua = units * g / groups;
  const int64_t ub = units * (g + 1) / groups;
  for (int64_t u = ua; u < ub;) {
    const int row = (int)(u / n);
    const int ys = (int)(u - (int64_t)row * n) + 1;
    const int64_t rend = (int64_t)(row + 1) * n;
    const int ye = (int)((ub < rend ? ub : rend) - (int64_t)row * n);
    run_segment<T, PRE, XIN, DIAG, WRITE_A>(xin, b, ec, xout, bc, l, row, strip, ys, ye, a,
                                            sigma, op, bwin[threadIdx.x >> 6],
                                            stg[threadIdx.x >> 6]);
    u = (int64_t)row * n + ye;
  }
}

// Resident wavefronts of one kernel on this device.
template <typename K>
int resident_waves(K kernel) {
  int dev = 0, cus = 0, blocks = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 64 * kWavesPerBlock, 0) !=
          hipSuccess ||
      blocks <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  return cus * blocks * kWavesPerBlock;
}

template <typename T, bool PRE, bool XIN, bool DIAG, bool WRITE_A>
hipError_t launch(hipStream_t s, const T* xin, const T* b, const T* ec, T* xout, T* bc, int l,
                  int rows, double a, const double* sigma, const SpaceOp& op) {
  constexpr int H = PRE ? kHaloPre : (WRITE_A ? kHaloPostA : kHaloPost);
  auto kernel = mg_stream_kernel<T, PRE, XIN, DIAG, WRITE_A>;
  // per kernel instantiation (the library drives one device type); a
  // function-local static is initialised exactly once even when the server's
  // worker and caller threads launch concurrently
  static const int slots = resident_waves(kernel);
  const int n = grid_n(l);
  const int ns = strip_count(n, H);
  // Candidate group counts (all give the same result): G groups that split
  // the rows into equal segments, for G = the groups that fit in the
  // resident slots (the first candidate, used untuned), 3/4, 1/2, 1/4 and
  // twice that, as long as the segments stay long compared with the restart
  // halo; and one group per time row.  Fewer groups than resident slots can
  // win: fewer grid lines are then streamed at once.
  std::vector<int64_t> cand;
  const int64_t fit = slots > 0 ? slots / ns : 0;
  for (int64_t g : {fit, 3 * fit / 4, fit / 2, fit / 4, 2 * fit}) {
    if (g > 0 && rows > g && (int64_t)rows * n / g >= 8 * (H + kWin) &&
        std::find(cand.begin(), cand.end(), g) == cand.end())
      cand.push_back(g);
  }
  cand.push_back(rows);
  auto go = [&](int c) -> hipError_t {
    const int64_t groups = cand[c];
    const int64_t waves = groups * ns;
    const unsigned blocks = (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    kernel<<<blocks, 64 * kWavesPerBlock, 0, s>>>(xin, b, ec, xout, bc, l, ns, rows, (int)groups,
                                                  a, sigma, op);
    return hipGetLastError();
  };
  const uint64_t variant = (sizeof(T) == 8 ? 16 : 0) | (PRE ? 8 : 0) | (XIN ? 4 : 0) |
                           (DIAG ? 2 : 0) | (WRITE_A ? 1 : 0);
  const int c = tuned(tune_key(1, variant, (uint64_t)l, (uint64_t)rows), (int)cand.size(), 0, s,
                      go);
  return go(c);
}

}  // namespace

// The "/"-diagonal couplings vanish only for the heat equation's K_x (no
// mass term, no reaction, no mixed diffusion): then the kernels skip them.
inline bool has_diag(const double* sigma, const SpaceOp& op) {
  return sigma != nullptr || op.c != 0.0 || op.dxy != 0.0;
}

template <typename T>
hipError_t mg_pre_stream(hipStream_t s, const T* xin, const T* b, T* xout, T* bc, int l, int rows,
                         double a, const double* sigma, const SpaceOp& op) {
  const bool d = has_diag(sigma, op);
  if (xin) {
    return d ? launch<T, true, true, true, false>(s, xin, b, nullptr, xout, bc, l, rows, a, sigma,
                                                  op)
             : launch<T, true, true, false, false>(s, xin, b, nullptr, xout, bc, l, rows, a, sigma,
                                                   op);
  }
  return d ? launch<T, true, false, true, false>(s, xin, b, nullptr, xout, bc, l, rows, a, sigma,
                                                 op)
           : launch<T, true, false, false, false>(s, xin, b, nullptr, xout, bc, l, rows, a, sigma,
                                                  op);
}

template <typename T>
hipError_t mg_post_stream(hipStream_t s, const T* xin, const T* b, const T* ec, T* xout, int l,
                          int rows, double a, const double* sigma, bool write_Ax,
                          const SpaceOp& op) {
  const bool d = has_diag(sigma, op);
  if (write_Ax) {
    return d ? launch<T, false, true, true, true>(s, xin, b, ec, xout, nullptr, l, rows, a, sigma,
                                                  op)
             : launch<T, false, true, false, true>(s, xin, b, ec, xout, nullptr, l, rows, a, sigma,
                                                   op);
  }
  return d ? launch<T, false, true, true, false>(s, xin, b, ec, xout, nullptr, l, rows, a, sigma,
                                                 op)
           : launch<T, false, true, false, false>(s, xin, b, ec, xout, nullptr, l, rows, a, sigma,
                                                  op);
}

template hipError_t mg_pre_stream<double>(hipStream_t, const double*, const double*, double*,
                                          double*, int, int, double, const double*,
                                          const SpaceOp&);
template hipError_t mg_pre_stream<float>(hipStream_t, const float*, const float*, float*, float*,
                                         int, int, double, const double*, const SpaceOp&);
template hipError_t mg_post_stream<double>(hipStream_t, const double*, const double*,
                                           const double*, double*, int, int, double,
                                           const double*, bool, const SpaceOp&);
template hipError_t mg_post_stream<float>(hipStream_t, const float*, const float*, const float*,
                                          float*, int, int, double, const double*, bool,
                                          const SpaceOp&);

}  // namespace stp
