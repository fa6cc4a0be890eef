// Adjoint-gradient kernels of libwdg (meshes of wedges, exact mass).
//
// The semi-discrete operator is A = E^-1 G with the block-diagonal energy
// matrix E = diag(M/kappa, rho M, rho M, rho M) of eq. (estab) and
// G = (skew central part) + (symmetric penalty part) (Sec. 2); flipping the
// velocity sign (T) negates only the skew part, so A^T = E T A T E^-1.  In the
// variables sig = T E^-1 (adjoint), the reverse sweep of the low-storage
// Runge-Kutta stages runs the forward stage kernel on sig, and the derivative
// of one stage with respect to an element's material is
//   dt sig^T T (dG/dtheta Us - dE/dtheta Rs)
// with Us the forward stage input and Rs its right-hand side (sources
// included: E Rs = G Us + b with b independent of the material).  The mass
// terms are summed over a step's stages through the forward residuals
// (dt Rs = res_s - a_s res_{s-1}), so the forward keeps those and never
// stores Rs.
//   dE/dc:   pressure block -2/(c kappa) M
//   dE/drho: pressure block -1/(rho kappa) M, velocity blocks M
//   dG/dZ:   the penalties tau_p = 2/(Z- + Z+), tau_u = (Z- + Z+)/2 of every
//            face touching the element (upwind flux only)
// The stage kernel (its gradient epilogue) accumulates, per wedge and stage,
// the mass terms and the face integrals; grad_combine_kernel applies the
// penalty derivatives, which need the face integrals of both sides of a face;
// inject_kernel adds the receivers' adjoint sources between steps.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.hpp"

namespace wdg {
namespace {

// Per-wedge accumulator slots (state precision): 0 dJ/dc and 1 dJ/drho of
// the mass terms; 2..6 per face (bottom, top, quadrilaterals 0..2) the sum of
// dt (-tau_p^2/2 1/2 int sig_p [p] - 1/2 1/2 int sig_un [u_n]), the own side's
// share of dJ/dZ; FP32 records then hold the Kahan compensations of the same
// slots (the sums are read as they are: the compensation is below their last
// bit).
static_assert(kGradStride == 7, "gradient record layout");

// dJ/dZ of a wedge: every face's penalties depend on the impedances of both
// sides (both are the own one on the boundary) alike, so the face's share
// from both sides adds up; Z = rho c gives dZ/dc = rho, dZ/drho = c.
// Arithmetic in the state precision; the results are stored as FP64.
template <typename T>
__global__ void __launch_bounds__(256) grad_combine_kernel(int64_t K, const T* __restrict__ gacc,
                                                           const T* __restrict__ geo, const int* __restrict__ conn,
                                                           int flags, double* __restrict__ gc,
                                                           double* __restrict__ grho) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= K) return;
  const T* ga = gacc + k * kGradRecord<T>;
  const T* g = geo + k * kGeoStride;
  T gZ = 0;
  if (!(flags & kCentral)) {
    const int* cn = conn + k * kConnStride;
    const int code = cn[5];
    for (int f = 0; f < 5; ++f) {
      const T own = ga[2 + f];
      T other = own;
      const int nbr = cn[f];
      if (nbr >= 0) {
        const int nf = f < 2 ? ((code >> (6 + f)) & 1) : 2 + ((code >> (8 + 2 * (f - 2))) & 3);
        other = gacc[int64_t(nbr) * kGradRecord<T> + 2 + nf];
      }
      gZ += own + other;
    }
  }
  const T kap = g[9], irho = g[10];
  const T rho = T(1) / irho, c = std::sqrt(kap * irho);
  gc[k] = double(ga[0] + rho * gZ);
  grho[k] = double(ga[1] + c * gZ);
}

// One thread per node index; the receivers are visited in order by every
// thread, so receivers in the same element never race.
template <typename T>
__global__ void __launch_bounds__(128) inject_kernel(int NP, int nrec, const int64_t* __restrict__ base,
                                                     const double* __restrict__ vec, const double* __restrict__ w,
                                                     double sb, V4<T>* __restrict__ U, V4<T>* __restrict__ S) {
  const int i = threadIdx.x;
  if (i >= NP) return;
  for (int r = 0; r < nrec; ++r) {
    const T v = T(w[r]) * T(vec[int64_t(r) * NP + i]);
    U[base[r] + i].p += v;
    S[base[r] + i].p += T(sb) * v;
  }
}

}  // namespace

hipError_t launch_grad_combine(int bits, int64_t K, const void* gacc, const void* geo, const int* conn, int flags,
                               double* gc, double* grho, hipStream_t st) {
  const unsigned nb = unsigned((K + 255) / 256);
  if (nb == 0) return hipSuccess;
  if (bits == 32)
    hipLaunchKernelGGL(grad_combine_kernel<float>, dim3(nb), dim3(256), 0, st, K, static_cast<const float*>(gacc),
                       static_cast<const float*>(geo), conn, flags, gc, grho);
  else
    hipLaunchKernelGGL(grad_combine_kernel<double>, dim3(nb), dim3(256), 0, st, K, static_cast<const double*>(gacc),
                       static_cast<const double*>(geo), conn, flags, gc, grho);
  return hipGetLastError();
}

hipError_t launch_inject(int bits, int NP, int nrec, const int64_t* base, const double* vec, const double* w,
                         double sb, void* U, void* S, hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  if (NP > 128) return hipErrorInvalidValue;
  if (bits == 32)
    hipLaunchKernelGGL(inject_kernel<float>, dim3(1), dim3(128), 0, st, NP, nrec, base, vec, w, sb,
                       static_cast<V4<float>*>(U), static_cast<V4<float>*>(S));
  else
    hipLaunchKernelGGL(inject_kernel<double>, dim3(1), dim3(128), 0, st, NP, nrec, base, vec, w, sb,
                       static_cast<V4<double>*>(U), static_cast<V4<double>*>(S));
  return hipGetLastError();
}

}  // namespace wdg
