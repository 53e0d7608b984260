// Host-side launchers of the solver's HIP kernels (gfx950).
//
// Every launcher enqueues on `stream`, returns the launch status, and checks
// nothing about pointer validity: the driver allocates every buffer with the
// sizes stated next to each launcher and validates sizes before calling.
// T is the storage and arithmetic type (double, or float for the FP32 inner
// solve); reductions always accumulate in double.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "layout.h"

namespace stp {

// ---- the spatial operator of Section 4: A_x = A_D + c M_x, the P1 stiffness
// of int D grad u . grad v for the constant symmetric positive definite
// D = [[dxx, dxy], [dxy, dyy]] plus the reaction c >= 0.  The heat equation
// is D = Id, c = 0.
struct SpaceOp {
  double dxx = 1.0, dyy = 1.0, dxy = 0.0, c = 0.0;
  __host__ __device__ bool heat() const {
    return dxx == 1.0 && dyy == 1.0 && dxy == 0.0 && c == 0.0;
  }
};

// Stencil of C = a A_x + sigma M_x on the level with mesh width 2^-l, on the
// "/" mesh: centre, the x-neighbours (i +- 1, j), the y-neighbours
// (i, j +- 1), the two neighbours across the "/" diagonal (i + 1, j + 1),
// (i - 1, j - 1).  The element integrals of A_D: centre 2 (dxx + dyy - dxy),
// x: dxy - dxx, y: dxy - dyy, diagonal: -dxy; of M_x: h^2/12 (6; 1 at each
// of the six neighbours).
struct Stencil {
  double c0, cx, cy, cd;
};
__host__ __device__ inline Stencil stencil_of(const SpaceOp& op, double a, double sigma, int l) {
  const double h = 1.0 / (double)(1 << l);
  const double m = h * h / 12.0;
  if (op.heat()) return {4.0 * a + 6.0 * m * sigma, -a + m * sigma, -a + m * sigma, m * sigma};
  const double s = sigma + a * op.c;
  return {2.0 * a * (op.dxx + op.dyy - op.dxy) + 6.0 * m * s, a * (op.dxy - op.dxx) + m * s,
          a * (op.dxy - op.dyy) + m * s, -a * op.dxy + m * s};
}

// ---- multigrid for C = a A_x + sigma M_x on level l (Section 3.1, Theorem 3.1,
// Section 5.1: 3 Gauss-Seidel steps per grid).  Arrays hold `rows` slabs of
// level l (slab_elems(l) elements each); `sigma` has one value per row (NULL
// means sigma = 0 for every row).

// Forward smoothing from xin (or from zero when xin == NULL), then the
// residual restricted to level l-1:  xout <- S_f^3(xin, b),  bc <- P^T (b - C xout).
// xout must not alias xin; bc holds `rows` slabs of level l-1.  Streaming
// wavefront kernels (mg_stream.hip): rows held in registers, no halo along rows.
template <typename T>
hipError_t mg_pre_stream(hipStream_t s, const T* xin, const T* b, T* xout, T* bc, int l, int rows,
                         double a, const double* sigma, const SpaceOp& op);
// Coarse correction then backward smoothing: xout <- S_b^3(xin + P ec, b);
// ec holds `rows` slabs of level l-1.  write_Ax: store A_x x (the stiffness
// applied to the smoothed iterate) instead of x.
template <typename T>
hipError_t mg_post_stream(hipStream_t s, const T* xin, const T* b, const T* ec, T* xout, int l,
                          int rows, double a, const double* sigma, bool write_Ax,
                          const SpaceOp& op);

// The analysis W^T in one pass over the rows (wavelet_stream.hip): in place
// on X, 0 <= J <= 14; with DOT the first pass of p^T X (X before the
// transform), one partial per block of wavelet_stream_blocks(slab) and
// right-hand side, to partials.
template <typename T, bool UPD>
hipError_t wavelet_syn_stream(hipStream_t s, const T* src, T* dst, T* p, const T* z,
                              const double* beta, const int* order, int J, int64_t slab,
                              int nrhs);
template <typename T, bool DOT>
hipError_t wavelet_ana_stream(hipStream_t s, T* X, const T* p, double* partials, int J,
                              int64_t slab, int nrhs, int* nblk);
int wavelet_stream_blocks(int64_t slab);

// `cycles` V-cycles on levels L..1 (L <= coarse_levels<T>()) per row, each row
// in one workgroup with all levels in LDS (mg_coarse.hip): xout =
// V^cycles(L, b, xin) (xin NULL: from zero), or A_x applied to it when
// write_Ax.  xout may alias xin.  Level 6 would fit LDS too (62.6 KB in FP32),
// but one workgroup per row on 3969 nodes is slower than streaming that
// level: at 64 right-hand sides of N = 2^8, h = 2^-7 the level-6 cycle took
// 1.73 ms per launch against about 1.0 ms for the two level-6 streaming
// launches and the level-5 cycle.
template <typename T>
constexpr int coarse_levels() {
  return 5;
}
template <typename T>
hipError_t mg_coarse_cycle(hipStream_t s, const T* xin, const T* b, T* xout, int L, int rows,
                           double a, const double* sigma, bool write_Ax, const SpaceOp& op,
                           int cycles = 1);

// ---- space-time stencils (Lemma 4.2 and Lemma 4.1, applied row-wise through
// the Kronecker identity, eq. (15) of Section 5.2).  X has nrhs * (2^J+1) slabs
// of level K; outputs likewise.

// y1 = M (A_t X) + A (L^T X),  y2 = A (M_t X) + M (L X)   (first half of S).
template <typename T>
hipError_t time_stencil_pair(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs,
                             const SpaceOp& op);

// G1 = M (L^T g),  G0 = M (M_t g)   (the data terms of f in Lemma 4.1).
template <typename T>
hipError_t rhs_stencil_pair(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs);

// out_i = M z1_i + A z2_i, plus M e_b in row 0 of right-hand side b, where
// e_b = extra + b * extra_stride (one slab); extra == NULL adds nothing.
template <typename T>
hipError_t combine(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                   T* out, int J, int K, int nrhs, const SpaceOp& op);

// y = A_x x or y = M_x x on every one of `rows` slabs of level K.
template <typename T>
hipError_t apply_A(hipStream_t s, const T* x, T* y, int K, int rows, const SpaceOp& op);
template <typename T>
hipError_t apply_M(hipStream_t s, const T* x, T* y, int K, int rows);

// ---- three-point wavelet transform along time, in place (Section 3.3).  It
// acts on every element of a time row alike, so it takes the row length
// (slab: slab_elems(K) in 2D, slab3_elems(K) in 3D).
template <typename T>
hipError_t wavelet(hipStream_t s, T* X, int J, int64_t slab, int nrhs, bool synthesis,
                   const int* order);
// dst = W src (src == dst allowed; for J = 0 a copy).  `order`: the device
// copy of synthesis_read_order(J).
template <typename T>
hipError_t synthesis(hipStream_t s, const T* src, T* dst, int J, int64_t slab, int nrhs,
                     const int* order);
// X = W p after the conjugate-gradient update p = z + beta_b p (p is updated
// in place; X must not alias p, z).
template <typename T>
hipError_t synthesis_update(hipStream_t s, T* p, const T* z, const double* beta, T* X, int J,
                            int64_t slab, int nrhs, const int* order);
// The rows 0..2^J in the order in which the one-pass synthesis reads their
// coefficients (wavelet_stream.hip).
std::vector<int> synthesis_read_order(int J);
// Y = W^T Y in place, and out_b = Ws_b^T Y_b with Y before the transform
// (FP64, deterministic).  With Ws = W p this is p^T (W^T Y), the dot PCG
// needs.  partials holds nrhs * analysis_dot_blocks(slab) values.
int analysis_dot_blocks(int64_t slab);
template <typename T>
hipError_t analysis_dot(hipStream_t s, T* Y, const T* Ws, double* partials, double* out, int J,
                        int64_t slab, int nrhs);

// ---- vector operations over `nrhs` segments of `n` elements (segment b at
// offset b * n).  Dots are deterministic: a fixed block decomposition of each
// segment and a fixed-order second pass, independent of nrhs.
int dot_blocks(int64_t n);
template <typename T>
hipError_t dot(hipStream_t s, const T* a, const T* b, int64_t n, int nrhs, double* partials,
               double* out);

template <typename T>
hipError_t copy(hipStream_t s, const T* src, T* dst, int64_t count);

// w += gamma_b p, r -= gamma_b q (per segment b).
template <typename T>
hipError_t update_wr(hipStream_t s, T* w, T* r, const T* p, const T* q, const double* gamma,
                     int64_t n, int nrhs);
// p = z + beta_b p.
template <typename T>
hipError_t update_p(hipStream_t s, T* p, const T* z, const double* beta, int64_t n, int nrhs);

// PCG scalars per right-hand side (all device arrays of length nrhs).
struct PcgScalars {
  double* rho;     // r^T z of the current iterate
  double* rho0;    // r_0^T z_0
  double* pq;      // p^T q
  double* rhonew;  // r^T z after the update
  double* gamma;
  double* beta;
  double* target;  // converged once sqrt(r^T z) <= target (0: never, run to maxit)
  int* active;     // 1 while iterating
  int* its;        // iterations performed
  int* status;     // 0 ok/running, 1 converged, -3 breakdown
};
// start: rho = rho0 = rhonew, target = tol_b * sqrt(rho0) (tol: device array of
// nrhs relative tolerances, or NULL for 0 = run to maxit), its = 0, active
// unless rho0 == 0 (nothing to solve) or non-finite (breakdown).
// ref (NULL: the first residual's rho): f-hat^T K_X f-hat per right-hand
// side, the reference of the stopping test and of rho0 from an initial guess.
hipError_t pcg_start(hipStream_t s, PcgScalars sc, int nrhs, const double* tol,
                     const double* ref = nullptr);
// The convergence state the host reads after a unit of work, packed per
// right-hand side b as out[5b .. 5b+4] = active, its, rho, rho0, target.
hipError_t pack_flags(hipStream_t s, PcgScalars sc, int nrhs, double* out);
// gamma = rho / p^T q for active right-hand sides (breakdown if p^T q <= 0).
hipError_t pcg_gamma(hipStream_t s, PcgScalars sc, int nrhs);
// beta = rhonew / rho, rho = rhonew, its += 1, convergence test against target;
// a right-hand side that reaches maxit iterations stops (status stays 0).
hipError_t pcg_beta(hipStream_t s, PcgScalars sc, int nrhs, int maxit);

// State of the FP32-inner / FP64-outer form per right-hand side (device arrays).
struct MixedState {
  double* rho0_first;  // r^T K_X r of the first outer step
  double* rel;         // sqrt(rho0 / rho0_first) at the latest outer step
  int* done;           // 1 once converged or broken down
  int* status;         // 0 converged, -3 breakdown, 1 still running
  int* outer;          // index of the latest outer step
  int* inner_its;      // inner iterations, summed
};
hipError_t mixed_reset(hipStream_t s, MixedState ms, int nrhs);
// after the inner PCG start of outer step k: convergence test of the FP64
// residual against tol_b, inner target max(inner_tol sqrt(rho0), tol_b/2 sqrt(rho0_first));
// last: no further inner solve (the right-hand sides not converged stop unconverged)
hipError_t mixed_adjust(hipStream_t s, PcgScalars sc, MixedState ms, int nrhs, const double* tol,
                        double inner_tol, int k, bool last);
// after an inner solve: inner_its += its, breakdown marks the right-hand side done
hipError_t mixed_inner_done(hipStream_t s, PcgScalars sc, MixedState ms, int nrhs);

// ---- layout conversion and precision casts.
// Compact FP64 rows of (2^K-1)^2 values <-> slabs of level K in type T.
template <typename T>
hipError_t pack(hipStream_t s, const double* src, T* dst, int K, int rows);
template <typename T>
hipError_t unpack(hipStream_t s, const T* src, double* dst, int K, int rows);
template <typename Tin, typename Tout>
hipError_t cast(hipStream_t s, const Tin* in, Tout* out, int64_t count);
// r = f - q (FP64).
hipError_t residual64(hipStream_t s, const double* f, const double* q, double* r, int64_t count);
// w += (double) d per segment of n elements, except segments with status[b] == -3.
hipError_t add_correction(hipStream_t s, double* w, const float* d, int64_t n, int nrhs,
                          const int* status);
// sigma[b * (N+1) + i] = 2^row_level(i, J)
hipError_t fill_level_sigma(hipStream_t s, double* sigma, int J, int nrhs);

// ---- three space dimensions (Section 5.2's 3D problem, space3d.hip): slabs
// of slab3_elems(l) elements, the Kuhn tetrahedral mesh of the unit cube.
// Same contracts as the two-dimensional launchers above.
template <typename T>
hipError_t pack3(hipStream_t s, const double* src, T* dst, int K, int rows);
template <typename T>
hipError_t unpack3(hipStream_t s, const T* src, double* dst, int K, int rows);
template <typename T>
hipError_t apply_A3(hipStream_t s, const T* x, T* y, int K, int rows);
template <typename T>
hipError_t apply_M3(hipStream_t s, const T* x, T* y, int K, int rows);
template <typename T>
hipError_t time_stencil_pair3(hipStream_t s, const T* X, T* y1, T* y2, int J, int K, int nrhs);
template <typename T>
hipError_t rhs_stencil_pair3(hipStream_t s, const T* g, T* G1, T* G0, int J, int K, int nrhs);
template <typename T>
hipError_t combine3(hipStream_t s, const T* z1, const T* z2, const T* extra, int64_t extra_stride,
                    T* out, int J, int K, int nrhs);
// Multigrid work space for `rows` slabs: per level l, x[l] and b[l] (l < K)
// and the residual r[l] (l >= 2); x[K] holds the iterate when write_Ax.
template <typename T>
struct Mg3Work {
  T* x[kMaxK3 + 1] = {};
  T* b[kMaxK3 + 1] = {};
  T* r[kMaxK3 + 1] = {};
};
// x = K[a, sigma] b (vcycles V-cycles from zero) on `rows` slabs of level K,
// or A_x of it when write_Ax; x must not alias b.
template <typename T>
hipError_t mg3_apply(hipStream_t s, const Mg3Work<T>& w, const T* b, T* x, int K, int rows,
                     double a, const double* sigma, int vcycles, bool write_Ax);

// ---- nested iteration (Section 4.2).
// Data on a coarser mesh: dst (nrhs x rows_c slabs of level Kf - d) takes
// the values of src (nrhs x rows_f slabs of level Kf) at its nodes: row i
// from row i * tstride, node (a, b) from node (2^d a, 2^d b).
hipError_t inject(hipStream_t s, const double* src, double* dst, int Kf, int d, int rows_f,
                  int rows_c, int tstride, int nrhs);
// wf (nrhs x (2^J + 1) slabs of level K) = the coefficients wc of mesh
// (J - 1, K - 1) expressed on mesh (J, K): even rows from coarse rows by P1
// interpolation in space, odd rows zero.
hipError_t prolong_w(hipStream_t s, const double* wc, double* wf, int J, int K, int nrhs);

}  // namespace stp
