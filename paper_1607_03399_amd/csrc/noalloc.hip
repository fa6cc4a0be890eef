// Allocation-free variant of the right-hand-side evaluation of libwdg
// (wdg_eval_rhs_noalloc), for callers that cannot allocate device memory.
//
// wdg_eval_rhs stages the caller's four FP64 field blocks into two device
// buffers it allocates per call.  This variant stages them through one
// file-scope device array instead:
//   region A: 4 n FP64 values (the caller's p, u_x, u_y, u_z blocks; reused
//             for the result on its way back),
//   region B: n node 4-vectors (p, u_z, u_x, u_y) of the context precision
//             (the input state of the stage kernels),
//   region C: n node 4-vectors (their right-hand side),
// each region starting on a 256-byte boundary.  Calls on one GPU share the
// array; calls that overlap on one GPU (several host threads, or streams of
// contexts that are not synchronised against each other) race on it.  The
// entry point waits for its own stream before returning, so consecutive
// calls do not overlap.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.hpp"
#include "wdg.h"

namespace {

// Largest staging the array holds: 32 MiB.  In FP32 that is 524 288 nodes
// (64 bytes per node), in FP64 349 525 nodes (96 bytes per node).
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of scratch on each device (the array's host-side name is
// not a device address), looked up once per device with that device current.
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// FP64 field blocks (p, u_x, u_y, u_z; n values each) to node 4-vectors (p, u_z, u_x, u_y) of type T
template <typename T>
__global__ void __launch_bounds__(256) blocks_to_nodes(const double* __restrict__ a, int64_t n, T* __restrict__ b) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= n) return;
  b[4 * m] = T(a[m]);
  b[4 * m + 1] = T(a[3 * n + m]);
  b[4 * m + 2] = T(a[n + m]);
  b[4 * m + 3] = T(a[2 * n + m]);
}

// node 4-vectors (p, u_z, u_x, u_y) of type T to FP64 field blocks (p, u_x, u_y, u_z)
template <typename T>
__global__ void __launch_bounds__(256) nodes_to_blocks(const T* __restrict__ b, int64_t n, double* __restrict__ a) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= n) return;
  a[m] = double(b[4 * m]);
  a[3 * n + m] = double(b[4 * m + 1]);
  a[n + m] = double(b[4 * m + 2]);
  a[2 * n + m] = double(b[4 * m + 3]);
}

int scratch_on_device(wdg_ctx* ctx, int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return wdg::ctx_fail(ctx, WDG_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return wdg::ctx_fail(ctx, WDG_ERR_HIP, "hipGetSymbolAddress(scratch) failed");
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return WDG_OK;
}

#define NACHK(expr)                                                                          \
  do {                                                                                       \
    const hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return wdg::ctx_fail(ctx, WDG_ERR_HIP, #expr " failed");           \
  } while (0)

template <typename T>
int run(wdg_ctx* ctx, const wdg::RhsView& v, unsigned char* base, double t, const double* in4, double* out4) {
  const int64_t n = v.nodes;
  double* A = reinterpret_cast<double*>(base);
  T* B = reinterpret_cast<T*>(base + round256(size_t(n) * 4 * sizeof(double)));
  T* Cq = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(B) + round256(size_t(n) * 4 * sizeof(T)));
  const unsigned grid = unsigned((n + 255) / 256);
  NACHK(hipMemcpyAsync(A, in4, size_t(n) * 4 * sizeof(double), hipMemcpyHostToDevice, v.stream));
  hipLaunchKernelGGL(blocks_to_nodes<T>, dim3(grid), dim3(256), 0, v.stream, A, n, B);
  NACHK(hipGetLastError());
  const int rc = wdg::ctx_eval_rhs_device(ctx, t, B, Cq);
  if (rc != WDG_OK) {
    (void)hipStreamSynchronize(v.stream);
    return rc;
  }
  hipLaunchKernelGGL(nodes_to_blocks<T>, dim3(grid), dim3(256), 0, v.stream, Cq, n, A);
  NACHK(hipGetLastError());
  NACHK(hipMemcpyAsync(out4, A, size_t(n) * 4 * sizeof(double), hipMemcpyDeviceToHost, v.stream));
  NACHK(hipStreamSynchronize(v.stream));
  return WDG_OK;
}

}  // namespace

extern "C" int wdg_eval_rhs_noalloc_max_nodes(int precision_bits, int64_t* n) {
  if (!n || (precision_bits != 32 && precision_bits != 64)) return WDG_ERR_ARG;
  const size_t per = 4 * sizeof(double) + 2 * 4 * size_t(precision_bits / 8);
  // the two 256-byte roundings cost at most 512 bytes
  *n = int64_t((kScratchBytes - 512) / per);
  return WDG_OK;
}

extern "C" int wdg_eval_rhs_noalloc(wdg_ctx* ctx, double t, const double* in4, double* out4) {
  if (!ctx) return WDG_ERR_ARG;
  wdg::RhsView v{};
  int rc = wdg::ctx_rhs_view(ctx, &v);
  if (rc != WDG_OK) return rc;
  if (!in4 || !out4) return wdg::ctx_fail(ctx, WDG_ERR_ARG, "null array");
  const size_t ts = v.bits == 32 ? 4 : 8;
  const size_t need = round256(size_t(v.nodes) * 4 * sizeof(double)) + round256(size_t(v.nodes) * 4 * ts) +
                      size_t(v.nodes) * 4 * ts;
  if (need > kScratchBytes)
    return wdg::ctx_fail(ctx, WDG_ERR_ARG,
                         "wdg_eval_rhs_noalloc: the mesh needs more staging than the 32 MiB device array "
                         "(see wdg_eval_rhs_noalloc_max_nodes)");
  NACHK(hipSetDevice(v.device));
  void* p = nullptr;
  rc = scratch_on_device(ctx, v.device, &p);
  if (rc != WDG_OK) return rc;
  unsigned char* base = static_cast<unsigned char*>(p);
  return v.bits == 32 ? run<float>(ctx, v, base, t, in4, out4) : run<double>(ctx, v, base, t, in4, out4);
}
