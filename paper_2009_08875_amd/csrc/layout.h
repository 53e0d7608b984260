// Device data layout shared by the kernels and the host driver.
//
// A spatial grid on multigrid level l (mesh width 2^-l) has n_l = 2^l - 1
// interior nodes per side.  One time row ("slab") stores them line by line
// with a line pitch of 2^l elements: node (a, b), 1 <= a, b <= n_l, is at
// offset (b - 1) * 2^l + (a - 1); the last element of each line (a = 2^l)
// is padding and always zero.  The slab length is rounded up to a multiple
// of 64 elements (also zero), so every slab starts 256-byte aligned in FP32
// and 512-byte aligned in FP64.  A space-time array is `rows` consecutive
// slabs, time-major: row = rhs * (2^J + 1) + i.
#pragma once
#include <cstddef>
#include <cstdint>

namespace stp {

inline constexpr int kMaxJ = 14;
inline constexpr int kMaxK = 10;
inline constexpr int kMaxK3 = 8;  // three space dimensions

__host__ __device__ inline int grid_n(int l) { return (1 << l) - 1; }
__host__ __device__ inline int line_pitch(int l) { return 1 << l; }
__host__ __device__ inline int64_t slab_elems(int l) {
  int64_t e = (int64_t)grid_n(l) * line_pitch(l);
  return (e + 63) & ~(int64_t)63;
}

// Three space dimensions (the unit cube): a slab stores the n_l^3 interior
// nodes plane by plane and line by line with line pitch 2^l: node (a, b, c)
// at ((c - 1) n_l + (b - 1)) 2^l + (a - 1); rounded up to 64 elements.
__host__ __device__ inline int64_t slab3_elems(int l) {
  int64_t e = (int64_t)grid_n(l) * grid_n(l) * line_pitch(l);
  return (e + 63) & ~(int64_t)63;
}

// Wavelet level |lambda| of the coefficient stored at time row i (0..N):
// level 0 at both ends, J - ctz(i) inside.
__host__ __device__ inline int row_level(int i, int J) {
  int N = 1 << J;
  if (i == 0 || i == N) return 0;
  int tz = 0;
  while (((i >> tz) & 1) == 0) ++tz;
  return J - tz;
}

}  // namespace stp
