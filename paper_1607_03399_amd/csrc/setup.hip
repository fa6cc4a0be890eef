// Setup and diagnostic kernels of libwdg: FP64 geometric factors and
// triangular operators of the wedges (Lemma 1, Sec. 4.2), material records,
// receiver sampling and the discrete energies.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace wdg {
namespace {

// ---------------------------------------------------------------------------
// FP64 setup: one wavefront per element
// ---------------------------------------------------------------------------
constexpr int kMaxNT = 21;

template <typename T>
__global__ void __launch_bounds__(64) setup_kernel(int NT, int LS, int64_t K, const double* __restrict__ X,
                                                   const double* __restrict__ Mv, const double* __restrict__ Mtri,
                                                   T* __restrict__ geo, T* __restrict__ L, double* __restrict__ aux) {
  const bool packed = Mtri == nullptr;  // store (M^{tri,k})^-1 packed, else L^{tri,k}
  __shared__ double Aug[kMaxNT * 2 * kMaxNT];
  __shared__ double fac[kMaxNT];
  const int tid = threadIdx.x;
  const int W = 2 * NT;
  for (int64_t k = blockIdx.x; k < K; k += gridDim.x) {
    const double* x = X + k * 18;
    double xb[3], yb[3], zb[3], zt[3];
    for (int v = 0; v < 3; ++v) {
      xb[v] = x[3 * v];
      yb[v] = x[3 * v + 1];
      zb[v] = x[3 * v + 2];
      zt[v] = x[3 * (v + 3) + 2];
    }
    const double xr = 0.5 * (xb[1] - xb[0]), xs = 0.5 * (xb[2] - xb[0]);
    const double yr = 0.5 * (yb[1] - yb[0]), ys = 0.5 * (yb[2] - yb[0]);
    const double Jt = xr * ys - xs * yr;
    double cw[3];
    for (int v = 0; v < 3; ++v) cw[v] = 0.5 * Jt * (zt[v] - zb[v]);

    if (tid == 0) {
      double gf[kGeoStride];
      for (int i = 0; i < kGeoStride; ++i) gf[i] = 0.0;
      gf[0] = ys / Jt;
      gf[1] = -xs / Jt;
      gf[2] = -yr / Jt;
      gf[3] = xr / Jt;
      gf[4] = Jt;
      const double zr_lo = 0.5 * (zb[1] - zb[0]), zs_lo = 0.5 * (zb[2] - zb[0]);
      const double zr_hi = 0.5 * (zt[1] - zt[0]), zs_hi = 0.5 * (zt[2] - zt[0]);
      gf[5] = yr * zs_lo - zr_lo * ys;
      gf[6] = yr * zs_hi - zr_hi * ys;
      gf[7] = zr_lo * xs - xr * zs_lo;
      gf[8] = zr_hi * xs - xr * zs_hi;
      gf[9] = 1.0;
      gf[10] = 1.0;
      gf[11] = 1.0;
      for (int f = 0; f < 5; ++f) gf[32 + f] = 2.0;  // rho = c = 1 until the material is set
      for (int face = 0; face < 2; ++face) {
        const double* zz = face == 0 ? zb : zt;
        const double ax = xb[1] - xb[0], ay = yb[1] - yb[0], az = zz[1] - zz[0];
        const double bx = xb[2] - xb[0], by = yb[2] - yb[0], bz = zz[2] - zz[0];
        const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        const double nrm = sqrt(cx * cx + cy * cy + cz * cz);
        const double sgn = face == 0 ? -1.0 : 1.0;
        gf[12 + 4 * face] = 0.25 * nrm;
        gf[13 + 4 * face] = sgn * cx / nrm;
        gf[14 + 4 * face] = sgn * cy / nrm;
        gf[15 + 4 * face] = sgn * cz / nrm;
      }
      for (int ed = 0; ed < 3; ++ed) {
        const int a = ed, b = (ed + 1) % 3;
        const double dx = xb[b] - xb[a], dy = yb[b] - yb[a];
        const double ell = sqrt(dx * dx + dy * dy);
        gf[20 + 4 * ed] = 0.25 * ell * (zt[a] - zb[a]);
        gf[21 + 4 * ed] = 0.25 * ell * (zt[b] - zb[b]);
        gf[22 + 4 * ed] = dy / ell;
        gf[23 + 4 * ed] = -dx / ell;
      }
      // M^{tri,k} = sum_v cw_v M_v: its weights (the adjoint's mass terms)
      gf[37] = cw[0];
      gf[38] = cw[1];
      gf[39] = cw[2];
      for (int i = 0; i < kGeoStride; ++i) geo[k * kGeoStride + i] = T(gf[i]);
      double* ax = aux + k * kAuxStride;
      ax[0] = cw[0];
      ax[1] = cw[1];
      ax[2] = cw[2];
      ax[3] = Jt;
      ax[4] = 1.0;
      ax[5] = 1.0;
      ax[6] = 0.0;
      ax[7] = 0.0;
    }
    // [ M^{tri,k} | I ] (packed) or [ M^{tri,k} | M^tri ],
    // M^{tri,k} = sum_v (J_tri h_v / 2) int l_a l_b lambda_v
    for (int idx = tid; idx < NT * W; idx += 64) {
      const int r = idx / W, c = idx - r * W;
      double v;
      if (c < NT) {
        v = cw[0] * Mv[r * NT + c] + cw[1] * Mv[NT * NT + r * NT + c] + cw[2] * Mv[2 * NT * NT + r * NT + c];
      } else {
        v = packed ? ((c - NT == r) ? 1.0 : 0.0) : Mtri[r * NT + (c - NT)];
      }
      Aug[idx] = v;
    }
    __syncthreads();
    // Gauss-Jordan elimination (M^{tri,k} is symmetric positive definite: no pivoting)
    for (int p = 0; p < NT; ++p) {
      const double piv = Aug[p * W + p];
      __syncthreads();
      for (int c = tid; c < W; c += 64) Aug[p * W + c] /= piv;
      __syncthreads();
      for (int r = tid; r < NT; r += 64) fac[r] = Aug[r * W + p];
      __syncthreads();
      for (int idx = tid; idx < NT * W; idx += 64) {
        const int r = idx / W, c = idx - r * W;
        if (r != p) Aug[idx] -= fac[r] * Aug[p * W + c];
      }
      __syncthreads();
    }
    // (M^{tri,k})^-1 is symmetric: its lower triangle, row by row; or L^{tri,k} column by column
    for (int idx = tid; idx < LS; idx += 64) {
      double v = 0.0;
      if (packed && idx < NT * (NT + 1) / 2) {
        const int r = tri_row(idx), c = idx - r * (r + 1) / 2;
        v = 0.5 * (Aug[r * W + NT + c] + Aug[c * W + NT + r]);
      } else if (!packed && idx < NT * NT) {
        const int c = idx / NT, r = idx - c * NT;
        v = Aug[r * W + NT + c];
      }
      L[k * LS + idx] = T(v);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void material_kernel(int64_t K, const double* __restrict__ c, const double* __restrict__ rho,
                                const int* __restrict__ conn, T* __restrict__ geo, double* __restrict__ aux) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double kap = rho[k] * c[k] * c[k];
  const double Z = rho[k] * c[k];
  geo[k * kGeoStride + 9] = T(kap);
  geo[k * kGeoStride + 10] = T(1.0 / rho[k]);
  geo[k * kGeoStride + 11] = T(Z);
  for (int f = 0; f < 5; ++f) {
    const int nb = conn[k * kConnStride + f];
    geo[k * kGeoStride + 32 + f] = T(Z + (nb >= 0 ? rho[nb] * c[nb] : Z));
  }
  aux[k * kAuxStride + 4] = kap;
  aux[k * kAuxStride + 5] = rho[k];
}

// receiver traces: p at each receiver by its element's interpolation row, in
// the state precision (the trace buffer holds them widened to double)
template <typename T>
__global__ void sample_receivers(int ld, int nrec, const T* __restrict__ U, const int64_t* __restrict__ base,
                                 const int* __restrict__ nn, const T* __restrict__ rows, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const T* Ue = U + base[r] * 4;
  T acc = T(0);
  for (int n = 0; n < nn[r]; ++n) acc += rows[int64_t(r) * ld + n] * Ue[4 * n];
  out[r] = double(acc);
}

template <int N, typename T>
__global__ void __launch_bounds__(256) energy_kernel(int64_t K, const T* __restrict__ U, const double* __restrict__ aux,
                                                     const double* __restrict__ Mv, const double* __restrict__ M1,
                                                     double* __restrict__ partial) {
  constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < K; k += int64_t(gridDim.x) * 256) {
    const double* ax = aux + k * kAuxStride;
    const double c0 = ax[0], c1 = ax[1], c2 = ax[2], kap = ax[4], rho = ax[5];
    const T* Ue = U + k * NP * 4;
    for (int f = 0; f < 4; ++f) {
      const double w = f == 0 ? 1.0 / kap : rho;
      double ef = 0.0;
      for (int j = 0; j < Nq; ++j)
        for (int i = 0; i < NT; ++i) {
          // y = (M^{tri,k} v_j')_i summed with M^1D weights
          double yi = 0.0;
          for (int jj = 0; jj < Nq; ++jj) {
            const double m1 = M1[j * Nq + jj];
            double t = 0.0;
            for (int ii = 0; ii < NT; ++ii) {
              const double mt = c0 * Mv[i * NT + ii] + c1 * Mv[NT * NT + i * NT + ii] + c2 * Mv[2 * NT * NT + i * NT + ii];
              t += mt * double(Ue[4 * (jj * NT + ii) + f]);
            }
            yi += m1 * t;
          }
          ef += double(Ue[4 * (j * NT + i) + f]) * yi;
        }
      acc += 0.5 * w * ef;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// E_k = 1/2 J (p^T M p / kappa + rho sum_d u_d^T M u_d) for affine tetrahedra
template <int N, typename T>
__global__ void __launch_bounds__(256) energy_tet_kernel(int64_t Kt, const T* __restrict__ U,
                                                         const double* __restrict__ aux, const double* __restrict__ Mt,
                                                         double* __restrict__ partial) {
  constexpr int NP = TDim<N>::NP;
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < Kt; k += int64_t(gridDim.x) * 256) {
    const double J = aux[k * kTetAuxStride], kap = aux[k * kTetAuxStride + 1], rho = aux[k * kTetAuxStride + 2];
    const T* Ue = U + k * NP * 4;
    for (int f = 0; f < 4; ++f) {
      double ef = 0.0;
      for (int i = 0; i < NP; ++i) {
        double y = 0.0;
        for (int m = 0; m < NP; ++m) y += Mt[i * NP + m] * double(Ue[4 * m + f]);
        ef += double(Ue[4 * i + f]) * y;
      }
      acc += 0.5 * J * (f == 0 ? 1.0 / kap : rho) * ef;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <int N, typename T>
hipError_t launch_energy_t(int64_t K, const void* U, const double* aux, const double* Mv, const double* M1,
                           double* partial, int* nblocks, hipStream_t st) {
  int nb = int((K + 255) / 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  *nblocks = nb;
  hipLaunchKernelGGL((energy_kernel<N, T>), dim3(nb), dim3(256), 0, st, K, static_cast<const T*>(U), aux, Mv, M1,
                     partial);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_energy_tet_t(int64_t Kt, const void* U, const double* aux, const double* Mt, double* partial,
                               int* nblocks, hipStream_t st) {
  int nb = int((Kt + 255) / 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  *nblocks = nb;
  hipLaunchKernelGGL((energy_tet_kernel<N, T>), dim3(nb), dim3(256), 0, st, Kt, static_cast<const T*>(U), aux, Mt,
                     partial);
  return hipGetLastError();
}

}  // namespace

int lift_stride(int N) {
  const int NT = (N + 1) * (N + 2) / 2;
  return ((lift_packed(N) ? NT * (NT + 1) / 2 : NT * NT) + 3) / 4 * 4;
}

hipError_t launch_setup(int N, int bits, int64_t K, const double* dX, const double* dMv, const double* dMtri,
                        void* dGeo, void* dL, double* dAux, hipStream_t st) {
  if (lift_packed(N)) dMtri = nullptr;
  else if (!dMtri) return hipErrorInvalidValue;
  const int NT = (N + 1) * (N + 2) / 2;
  const int LS = lift_stride(N);
  int64_t nb = K < 65536 ? K : 65536;
  if (nb <= 0) return hipSuccess;
  if (bits == 32)
    hipLaunchKernelGGL(setup_kernel<float>, dim3(unsigned(nb)), dim3(64), 0, st, NT, LS, K, dX, dMv, dMtri,
                       static_cast<float*>(dGeo), static_cast<float*>(dL), dAux);
  else
    hipLaunchKernelGGL(setup_kernel<double>, dim3(unsigned(nb)), dim3(64), 0, st, NT, LS, K, dX, dMv, dMtri,
                       static_cast<double*>(dGeo), static_cast<double*>(dL), dAux);
  return hipGetLastError();
}

hipError_t launch_material(int bits, int64_t K, const double* dc, const double* drho, const int* dConn, void* dGeo,
                           double* dAux, hipStream_t st) {
  const unsigned nb = unsigned((K + 255) / 256);
  if (nb == 0) return hipSuccess;
  if (bits == 32)
    hipLaunchKernelGGL(material_kernel<float>, dim3(nb), dim3(256), 0, st, K, dc, drho, dConn,
                       static_cast<float*>(dGeo), dAux);
  else
    hipLaunchKernelGGL(material_kernel<double>, dim3(nb), dim3(256), 0, st, K, dc, drho, dConn,
                       static_cast<double*>(dGeo), dAux);
  return hipGetLastError();
}

hipError_t launch_receivers(int bits, int ld, int nrec, const void* U, const int64_t* base, const int* nn,
                            const void* rows, double* out, hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  const unsigned nb = unsigned((nrec + 63) / 64);
  if (bits == 32)
    hipLaunchKernelGGL(sample_receivers<float>, dim3(nb), dim3(64), 0, st, ld, nrec, static_cast<const float*>(U), base,
                       nn, static_cast<const float*>(rows), out);
  else
    hipLaunchKernelGGL(sample_receivers<double>, dim3(nb), dim3(64), 0, st, ld, nrec, static_cast<const double*>(U),
                       base, nn, static_cast<const double*>(rows), out);
  return hipGetLastError();
}

hipError_t launch_energy(int N, int bits, int64_t K, const void* U, const double* aux, const double* Mv,
                         const double* M1, double* partial, int* nblocks, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_EN(n, T) err = launch_energy_t<n, T>(K, U, aux, Mv, M1, partial, nblocks, st)
  WDG_DISPATCH_N(N, bits, WDG_EN)
#undef WDG_EN
  return err;
}

hipError_t launch_energy_tet(int N, int bits, int64_t Kt, const void* U, const double* auxT, const double* Mt,
                             double* partial, int* nblocks, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_ENT(n, T) err = launch_energy_tet_t<n, T>(Kt, U, auxT, Mt, partial, nblocks, st)
  WDG_DISPATCH_N(N, bits, WDG_ENT)
#undef WDG_ENT
  return err;
}

}  // namespace wdg
