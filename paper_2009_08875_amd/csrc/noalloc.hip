// K_x on caller buffers with every intermediate in a fixed device array:
// the entry point for callers that cannot allocate device memory.
//
// The array `scratch` below is a file-scope device variable.  In host code
// its name is only a host-side stand-in, so the host never passes it to a
// kernel or a copy: on first use on a device (with that device current)
// hipGetSymbolAddress gives the device's own copy of the array, and that
// address, kept per device, is what the kernels receive.
//
// Layout of one chunk of R rows of level K inside the array (every part at
// a multiple of 512 bytes from the array's start): the input slabs (R slabs
// of level K), the output slabs (R), then the multigrid work space of
// mg_apply: xb[K] (R slabs of level K) and, for each coarser level
// l = K-1 .. 1, xa[l], xb[l], b[l] (R slabs of level l each).  R is at most
// 65535, the launch grid's limit along the rows.  No element of it needs to start at zero: the pack kernel
// writes every element of the input slabs, padding included, and every
// multigrid kernel reads only interior nodes that an earlier launch of the
// same call has written.  The array is cleared once per device anyway, so
// its contents are defined from the start.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "solver.h"
#include "tune.h"

constexpr size_t kScratchBytes = size_t(256) << 20;  // STP_STATIC_SCRATCH_BYTES
static_assert(kScratchBytes == STP_STATIC_SCRATCH_BYTES, "stp.h states the array size");

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
constexpr int64_t kMaxChunkRows = 65535;  // grid.y of the row-wise launches

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

__global__ void clear_kernel(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

size_t round512(size_t b) { return (b + 511) & ~size_t(511); }

// Bytes of one row's share of a chunk at level K (see the layout above).
size_t row_bytes(int K) {
  size_t b = 3 * round512(sizeof(double) * (size_t)stp::slab_elems(K));
  for (int l = 1; l < K; ++l) b += 3 * round512(sizeof(double) * (size_t)stp::slab_elems(l));
  return b;
}

// The current device's copy of `scratch` (set up on first use: address
// lookup and one clear, on the caller's stream).
stp_status device_scratch(hipStream_t s, double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    stp::set_error("stp_kspace_apply_static: no usable current HIP device");
    return STP_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      stp::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return STP_E_DEVICE;
    }
    const size_t n = kScratchBytes / sizeof(double);
    clear_kernel<<<1024, 256, 0, s>>>((double*)p, n);
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) {
      stp::set_error(std::string("clearing the static scratch: ") + hipGetErrorString(e2));
      return STP_E_DEVICE;
    }
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return STP_OK;
}

}  // namespace

extern "C" stp_status stp_kspace_apply_static(int K, int rows, const double* in, double* out,
                                              void* hip_stream) {
  using namespace stp;
  if (K < 1 || K > kMaxK || rows < 0 || (rows > 0 && (!in || !out))) {
    set_error("stp_kspace_apply_static: need 1 <= K <= 10, rows >= 0 and device buffers");
    return STP_E_INVALID_ARG;
  }
  const size_t per_row = row_bytes(K);
  if (per_row > kScratchBytes) {
    set_error("stp_kspace_apply_static: one row of level " + std::to_string(K) + " needs " +
              std::to_string(per_row) + " bytes, more than the " +
              std::to_string(kScratchBytes) + "-byte static array");
    return STP_E_INVALID_ARG;
  }
  if (rows == 0) return STP_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  double* base = nullptr;
  STP_TRY(device_scratch(s, &base));

  const int64_t chunk =
      std::min<int64_t>({(int64_t)(kScratchBytes / per_row), (int64_t)rows, kMaxChunkRows});
  const int64_t nn = (int64_t)grid_n(K) * grid_n(K);
  // carve one chunk's buffers out of the array
  char* q = (char*)base;
  auto take = [&](int l) {
    double* p = (double*)q;
    q += chunk * round512(sizeof(double) * (size_t)slab_elems(l));
    return p;
  };
  double* bin = take(K);
  double* xout = take(K);
  MgScratch<double> mg;
  mg.K = K;
  mg.chunk_rows = chunk;
  mg.xb[K] = take(K);
  for (int l = 1; l < K; ++l) {
    mg.xa[l] = take(l);
    mg.xb[l] = take(l);
    mg.b[l] = take(l);
  }
  // chunk * round512(...) per buffer == chunk * per_row in all: inside the array
  NoTuning no_tuning;  // launch shapes: remembered choices or defaults, no trial runs
  for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
    const int nr = (int)std::min<int64_t>(chunk, rows - r0);
    HIP_TRY(pack<double>(s, in + r0 * nn, bin, K, nr));
    STP_TRY(kspace_apply_slabs(s, mg, bin, xout, K, nr, 2));
    HIP_TRY(unpack<double>(s, xout, out + r0 * nn, K, nr));
  }
  return STP_OK;
}
