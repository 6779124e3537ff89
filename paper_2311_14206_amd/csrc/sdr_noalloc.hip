// Allocation-free batched sketch: Y = S X with the sparse-sign operator of
// Section 3 (eq. (3.1)), for callers that cannot allocate device memory.
//
// The kernels are those of sdr_sketch (k_sketch_cols, then the fixed-order
// column reduction); their partial sums live in a file-scope device array
// instead of a handle's buffers.  Each GPU holds its own copy of the array
// until the process ends; its address on a device is looked up once, with
// that device current, and kept per device.  Host code never passes the
// array's own name to a kernel: that name is a host-side stand-in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/sdr.h"
#include "sdr_kernels.h"

using namespace sdr;

static constexpr size_t kScratchBytes = (size_t)16 << 20;  // SDR_NOALLOC_SCRATCH_BYTES in sdr.h

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array, looked up on first use.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_last_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return SDR_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("device ordinal beyond the scratch table");
    return SDR_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SDR_EDEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SDR_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch bytes for cc columns: partials [(cc*s + cc) x nb], then the
// reduced column [cc*s + cc].
template <class A>
size_t scratch_need(int cc, int s, int nb) {
  const size_t rows = (size_t)cc * s + cc;
  return align256(rows * nb * sizeof(A)) + rows * sizeof(A);
}

template <class A>
int sketch_static(int n, SketchSpec sk, const A* X, int ncols, A* Y, hipStream_t st, char* base) {
  const int s = sk.s;
  const int nb = (n + kRowsUpdate - 1) / kRowsUpdate;
  // columns per launch: as sdr_sketch (the per-wave bins within 48 KiB, at
  // most 8), and as many as the scratch holds
  int cc = std::max(1, std::min(8, (int)(48 * 1024 / ((size_t)kWaves * s * sizeof(A)))));
  while (cc > 1 && scratch_need<A>(cc, s, nb) > kScratchBytes) --cc;
  A* part = reinterpret_cast<A*>(base);
  const double scl = 1.0 / std::sqrt((double)sk.zeta);
  for (int c0 = 0; c0 < ncols; c0 += cc) {
    const int c = std::min(cc, ncols - c0);
    A* red = reinterpret_cast<A*>(base + align256(((size_t)c * s + c) * nb * sizeof(A)));
    launch_sketch_cols<A>(st, n, X + (size_t)c0 * n, (int64_t)n, c, sk, part, nb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
      launch_reduce_cols<A>(st, part, nb, c * s + c, c * s, scl, red, nullptr);
      e = hipGetLastError();
    }
    // S X(:, c0 .. c0+c-1) is contiguous in red (the norms follow it)
    if (e == hipSuccess)
      e = hipMemcpyAsync(Y + (size_t)c0 * s, red, sizeof(A) * (size_t)c * s, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      set_last_error(std::string("sdr_sketch_noalloc: ") + hipGetErrorString(e));
      return SDR_EDEVICE;
    }
  }
  return SDR_OK;
}

}  // namespace

extern "C" int sdr_sketch_noalloc(int64_t n, int s_dim, int zeta, uint64_t seed, sdr_dtype dtype,
                                  const void* X, int ncols, void* Y, void* hip_stream) {
  if (n <= 0 || n > (int64_t)0x7fffffff || ncols < 0 || zeta < 1 || s_dim < zeta ||
      s_dim % zeta != 0 || (ncols > 0 && (!X || !Y))) {
    set_last_error("sdr_sketch_noalloc: bad argument (n >= 1, ncols >= 0, s_dim a multiple of zeta)");
    return SDR_EINVAL;
  }
  if (dtype != SDR_F64 && dtype != SDR_C128) {
    set_last_error("sdr_sketch_noalloc: dtype must be SDR_F64 or SDR_C128");
    return SDR_EINVAL;
  }
  const size_t esz = dtype == SDR_C128 ? 16 : 8;
  if ((size_t)kWaves * s_dim * esz > 64 * 1024) {
    set_last_error("sdr_sketch_noalloc: s_dim too large (at most 2048 real, 1024 complex)");
    return SDR_EINVAL;
  }
  const int nb = (int)((n + kRowsUpdate - 1) / kRowsUpdate);
  const size_t need = dtype == SDR_C128 ? scratch_need<cx<double>>(1, s_dim, nb) : scratch_need<double>(1, s_dim, nb);
  if (need > kScratchBytes) {
    set_last_error("sdr_sketch_noalloc: n = " + std::to_string(n) + " with s_dim = " + std::to_string(s_dim) +
                   " needs " + std::to_string(need) + " bytes of partial sums, more than the " +
                   std::to_string(kScratchBytes >> 20) + " MiB scratch");
    return SDR_EINVAL;
  }
  if (ncols == 0) return SDR_OK;
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != SDR_OK) return rc;
  SketchSpec sk;
  sk.seed = seed;
  sk.s = s_dim;
  sk.zeta = zeta;
  sk.bsz = s_dim / zeta;
  sk.words = (zeta + 3) / 4;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (dtype == SDR_C128)
    return sketch_static<cx<double>>((int)n, sk, static_cast<const cx<double>*>(X), ncols,
                                     static_cast<cx<double>*>(Y), st, static_cast<char*>(base));
  return sketch_static<double>((int)n, sk, static_cast<const double*>(X), ncols, static_cast<double*>(Y),
                               st, static_cast<char*>(base));
}
