// Batch stage records of libwdg: many independent wedge meshes advanced by
// one launch per order and stage.  The per-problem stage records live in
// device memory; before every stage one small kernel writes their
// stage-dependent fields (buffers of the ping-pong pair, Runge-Kutta
// coefficients, source amplitudes at the problem's own time from a table)
// from a step counter in device memory, so that a captured graph of one step
// can be replayed without host work.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace wdg {
namespace {

__global__ void __launch_bounds__(64) batch_prepare_kernel(int nprob, StageLaunch* __restrict__ probs,
                                                           const BatchParam* __restrict__ par,
                                                           const int64_t* __restrict__ counter, int s, double a,
                                                           double b, const double* __restrict__ amp) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= nprob) return;
  const BatchParam& P = par[p];
  StageLaunch& A = probs[p];
  const int64_t n = *counter;
  const int parity = int((P.cur0 + 5 * n + s) & 1);
  A.Uin = P.U[parity];
  A.Uout = P.U[1 - parity];
  A.a = a;
  A.b = b;
  A.dt = P.dt;
  A.g = 1.0;
  A.flags = P.flags | (s == 0 ? 0 : kReadRes) | kWriteU;
  const double* am = amp + ((n * 5 + s) * nprob + p) * kMaxSources;
  for (int k = 0; k < P.nsrc; ++k) A.src_amp[k] = am[k];
}

__global__ void batch_advance_kernel(int64_t* counter) {
  if (threadIdx.x == 0) *counter += 1;
}

}  // namespace

hipError_t launch_batch_prepare(int nprob, StageLaunch* probs, const BatchParam* par, const int64_t* counter, int s,
                                double a, double b, const double* amp, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_prepare_kernel, dim3(unsigned((nprob + 63) / 64)), dim3(64), 0, st, nprob, probs, par,
                     counter, s, a, b, amp);
  return hipGetLastError();
}

hipError_t launch_batch_advance(int64_t* counter, hipStream_t st) {
  hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

}  // namespace wdg
