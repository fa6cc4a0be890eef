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
// included: E Rs = G Us + b with b independent of the material).
//   dE/dc:   pressure block -2/(c kappa) M
//   dE/drho: pressure block -1/(rho kappa) M, velocity blocks M
//   dG/dZ:   the penalties tau_p = 2/(Z- + Z+), tau_u = (Z- + Z+)/2 of every
//            face touching the element (upwind flux only)
// grad_stage_kernel accumulates, per wedge, the mass terms and the face
// integrals of every stage; grad_combine_kernel applies the penalty
// derivatives, which need the face integrals of both sides of a face.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.hpp"
#include "ref_tables.inc"

namespace wdg {
namespace {

// Per-wedge accumulator slots (FP64): 0 dJ/dc and 1 dJ/drho of the mass
// terms; 2..6 sum dt 1/2 int sig_p [p], 7..11 sum dt 1/2 int sig_un [u_n]
// over the faces (bottom, top, quadrilaterals 0..2).
static_assert(kGradStride == 12, "gradient record layout");

template <typename T>
__device__ __forceinline__ void constexpr_or_skip(double c, T& acc, T x) {
  if (c != 0.0) acc += T(c) * x;
}

// entry of a reference table selected by the lane's level j (j < Nq)
template <int Nq, typename T>
__device__ __forceinline__ T pick(const double* tab, int j, int stride, int col) {
  T v = T(tab[col]);
#pragma unroll
  for (int jj = 1; jj < Nq; ++jj) v = (j == jj) ? T(tab[jj * stride + col]) : v;
  return v;
}

// One wavefront per EPB wedges, lane = (wedge, level j) as in the stage
// kernel; the chunk's adjoint vectors, stage inputs and right-hand sides are
// staged in LDS with coalesced loads.  The masses (M_v, reference triangle,
// 1D, edge) are compile-time literals.
template <int N, typename T>
__global__ void __launch_bounds__(64) grad_stage_kernel(int64_t K, const V4<T>* __restrict__ sig,
                                                        const V4<T>* __restrict__ Us, const V4<T>* __restrict__ Rs,
                                                        const T* __restrict__ geo, const int* __restrict__ conn,
                                                        const double* __restrict__ aux, double dt, int flags,
                                                        double* __restrict__ gacc) {
  using RT = gen::RefTables<N>;
  constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  constexpr int EPB = 64 / Nq;
  constexpr int NS = (EPB * NP + 63) / 64;
  constexpr int V4B = 4 * int(sizeof(T));
  // staging buffer: the adjoint vectors (copied to registers), then the stage
  // inputs, then the per-lane partial sums
  constexpr int BUF = (EPB * NP + 1) * V4B > EPB * Nq * kGradStride * 8 ? (EPB * NP + 1) * V4B
                                                                        : EPB * Nq * kGradStride * 8;
  __shared__ __align__(16) unsigned char sBuf[BUF];
  __shared__ V4<T> sR[EPB * NP + 1];
  __shared__ T sJ[EPB * 3 * Nq * Nq * 2];  // quadrilateral-face jumps [wedge][edge][level][node][p, u_n]
  V4<T>* const sV = reinterpret_cast<V4<T>*>(sBuf);
  double* const sPart = reinterpret_cast<double*>(sBuf);

  // XCD-aware chunk order (face neighbours share an L2), as in the stage kernel
  const int nb = gridDim.x, bid = blockIdx.x;
  const int qd = nb / 8, rm = nb % 8, xcd = bid % 8, kk = bid / 8;
  const int chunk = xcd < rm ? xcd * (qd + 1) + kk : rm * (qd + 1) + (xcd - rm) * qd + kk;
  const int64_t e0 = int64_t(chunk) * EPB;
  const int64_t left = K - e0;
  const int nE = left < EPB ? int(left) : EPB;
  const int tid = threadIdx.x, le = tid / Nq, j = tid - le * Nq;
  const bool lane_ok = le < EPB;
  const bool active = lane_ok && le < nE;
  const int64_t e = e0 + (active ? le : 0);  // idle lanes shadow a valid wedge
  const T bsign = (flags & kDirichlet) ? T(-1) : T(1);
  const int64_t bytes = int64_t(nE) * NP * V4B;
  const int lb = (lane_ok ? le : 0) * NP + j * NT;  // this lane's level in the staged chunk
  V4<T> sg[NT];
  {
    const auto bs = chunk_rsrc(sig + e0 * NP, bytes);
    const auto br = chunk_rsrc(Rs + e0 * NP, bytes);
    V4<T> a[NS], c[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      a[k] = bload<T>(bs, tid + 64 * k);
      c[k] = bload<T>(br, tid + 64 * k);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int idx = tid + 64 * k < EPB * NP ? tid + 64 * k : EPB * NP;
      sV[idx] = a[k];
      sR[idx] = c[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NT; ++i) sg[i] = sV[lb + i];
  __syncthreads();
  {
    const auto bu = chunk_rsrc(Us + e0 * NP, bytes);
    V4<T> b[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) b[k] = bload<T>(bu, tid + 64 * k);
#pragma unroll
    for (int k = 0; k < NS; ++k) sV[tid + 64 * k < EPB * NP ? tid + 64 * k : EPB * NP] = b[k];
  }
  const V4<T>* const sU = sV;
  const T* g = geo + e * kGeoStride;
  const int* cn = conn + e * kConnStride;
  const int code = cn[5];
  __syncthreads();

  double part[kGradStride];
#pragma unroll
  for (int k = 0; k < kGradStride; ++k) part[k] = 0.0;

  // triangular faces: lane 0 the bottom, lane N the top (own level)
  if (j == 0 || j == N) {
    const int face = j == 0 ? 0 : 1;
    const int nbr = cn[face];
    const int pc = (code >> (3 * face)) & 7;
    const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
    const T Jf = g[12 + 4 * face], nx = g[13 + 4 * face], ny = g[14 + 4 * face], nz = g[15 + 4 * face];
    T jp[NT], jn[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const V4<T> own = sU[lb + i];
      const T pm = own.p, unm = nx * own.ux + ny * own.uy + nz * own.uz;
      T pp = bsign * pm, unp = -bsign * unm;  // mirror state
      if (nbr >= 0) {
        const V4<T> v = Us[int64_t(nbr) * NP + nlev * NT + face_perm<N>(pc, i)];
        pp = v.p;
        unp = nx * v.ux + ny * v.uy + nz * v.uz;
      }
      jp[i] = pp - pm;
      jn[i] = unp - unm;
    }
    T sp = 0, sn = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T mp = 0, mn = 0;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        constexpr_or_skip(RT::Mtri[i * NT + k], mp, jp[k]);
        constexpr_or_skip(RT::Mtri[i * NT + k], mn, jn[k]);
      }
      const V4<T> a = sg[i];
      sp += a.p * mp;
      sn += (nx * a.ux + ny * a.uy + nz * a.uz) * mn;
    }
    part[2 + face] = 0.5 * double(Jf) * double(sp);
    part[7 + face] = 0.5 * double(Jf) * double(sn);
  }

  // quadrilateral faces: jumps of this level to LDS; the adjoint trace times
  // the edge mass stays in registers
  T ap[3][Nq], an[3][Nq];
#pragma unroll
  for (int ed = 0; ed < 3; ++ed) {
    const int nbr = cn[2 + ed];
    const int ned = (code >> (8 + 2 * ed)) & 3;
    const T Ja = g[20 + 4 * ed], Jb = g[21 + 4 * ed], nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
    T sp[Nq], sn[Nq];
#pragma unroll
    for (int q = 0; q < Nq; ++q) {
      const int i = edge_node(N, ed, q);
      const V4<T> own = sU[lb + i];
      const T pm = own.p, unm = nx * own.ux + ny * own.uy;
      T pp = bsign * pm, unp = -bsign * unm;
      if (nbr >= 0) {
        const int ni = ned == 0 ? edge_node(N, 0, N - q) : (ned == 1 ? edge_node(N, 1, N - q) : edge_node(N, 2, N - q));
        const V4<T> v = Us[int64_t(nbr) * NP + j * NT + ni];
        pp = v.p;
        unp = nx * v.ux + ny * v.uy;
      }
      if (lane_ok) {
        T* sj = sJ + (((le * 3 + ed) * Nq + j) * Nq + q) * 2;
        sj[0] = pp - pm;
        sj[1] = unp - unm;
      }
      const V4<T> a = sg[i];
      sp[q] = a.p;
      sn[q] = nx * a.ux + ny * a.uy;
    }
#pragma unroll
    for (int qq = 0; qq < Nq; ++qq) {
      T vpa = 0, vna = 0, vpb = 0, vnb = 0;
#pragma unroll
      for (int q = 0; q < Nq; ++q) {
        constexpr_or_skip(RT::Ma[q * Nq + qq], vpa, sp[q]);
        constexpr_or_skip(RT::Ma[q * Nq + qq], vna, sn[q]);
        constexpr_or_skip(RT::Mb[q * Nq + qq], vpb, sp[q]);
        constexpr_or_skip(RT::Mb[q * Nq + qq], vnb, sn[q]);
      }
      ap[ed][qq] = Ja * vpa + Jb * vpb;
      an[ed][qq] = Ja * vna + Jb * vnb;
    }
  }
  __syncthreads();

  if (lane_ok) {
    T m1[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) m1[m] = pick<Nq, T>(RT::M1, j, Nq, m);
    // mass terms: sig_f^T (M^{tri,k} (x) M^1D) R_f on this level
    const double* ax = aux + e * kAuxStride;
    const T w0 = T(ax[0]), w1 = T(ax[1]), w2 = T(ax[2]);
    T y[4][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        const V4<T> r = sR[le * NP + m * NT + i];
        a0 += m1[m] * r.p;
        a1 += m1[m] * r.ux;
        a2 += m1[m] * r.uy;
        a3 += m1[m] * r.uz;
      }
      y[0][i] = a0;
      y[1][i] = a1;
      y[2][i] = a2;
      y[3][i] = a3;
    }
    T mp = 0, mu = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T z0 = 0, z1 = 0, z2 = 0, z3 = 0;
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        T m = 0;
        constexpr_or_skip(RT::Mv[i * NT + k], m, w0);
        constexpr_or_skip(RT::Mv[NT * NT + i * NT + k], m, w1);
        constexpr_or_skip(RT::Mv[2 * NT * NT + i * NT + k], m, w2);
        z0 += m * y[0][k];
        z1 += m * y[1][k];
        z2 += m * y[2][k];
        z3 += m * y[3][k];
      }
      const V4<T> a = sg[i];
      mp += a.p * z0;
      mu += a.ux * z1 + a.uy * z2 + a.uz * z3;
    }
    part[0] = double(mp);
    part[1] = double(mu);
    // quadrilateral faces: couple the levels through M^1D
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      T sp = 0, sn = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        const T* sj = sJ + ((le * 3 + ed) * Nq + m) * Nq * 2;
        T tp = 0, tn = 0;
#pragma unroll
        for (int qq = 0; qq < Nq; ++qq) {
          tp += ap[ed][qq] * sj[2 * qq];
          tn += an[ed][qq] * sj[2 * qq + 1];
        }
        sp += m1[m] * tp;
        sn += m1[m] * tn;
      }
      part[4 + ed] = 0.5 * double(sp);
      part[9 + ed] = 0.5 * double(sn);
    }
  }
  __syncthreads();  // the stage inputs in the staging buffer are consumed
  if (lane_ok) {
#pragma unroll
    for (int k = 0; k < kGradStride; ++k) sPart[(le * Nq + j) * kGradStride + k] = part[k];
  }
  __syncthreads();
  if (active && j == 0) {
    double tot[kGradStride];
#pragma unroll
    for (int k = 0; k < kGradStride; ++k) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < Nq; ++l) s += sPart[(le * Nq + l) * kGradStride + k];
      tot[k] = s;
    }
    const double kap = aux[e * kAuxStride + 4], rho = aux[e * kAuxStride + 5];
    const double c = std::sqrt(kap / rho);
    double* ga = gacc + e * kGradStride;
    ga[0] += dt * 2.0 / (c * kap) * tot[0];
    ga[1] += dt * (tot[0] / (rho * kap) + tot[1]);
#pragma unroll
    for (int k = 2; k < kGradStride; ++k) ga[k] += dt * tot[k];
  }
}

// dJ/dZ of a wedge: every face's penalties depend on the impedances of both
// sides (both are the own one on the boundary), with dtau_p/dZ = -tau_p^2/2
// and dtau_u/dZ = 1/2; Z = rho c gives dZ/dc = rho, dZ/drho = c.
template <typename T>
__global__ void __launch_bounds__(256) grad_combine_kernel(int64_t K, const double* __restrict__ gacc,
                                                           const T* __restrict__ geo, const int* __restrict__ conn,
                                                           const double* __restrict__ aux, int flags,
                                                           double* __restrict__ gc, double* __restrict__ grho) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= K) return;
  const double* ga = gacc + k * kGradStride;
  double gZ = 0.0;
  if (!(flags & kCentral)) {
    const int* cn = conn + k * kConnStride;
    const int code = cn[5];
    for (int f = 0; f < 5; ++f) {
      const double zs = double(geo[k * kGeoStride + 32 + f]);
      const double tp = 2.0 / zs;
      const double own = -0.5 * tp * tp * ga[2 + f] - 0.5 * ga[7 + f];
      double other = own;
      const int nbr = cn[f];
      if (nbr >= 0) {
        const int nf = f < 2 ? ((code >> (6 + f)) & 1) : 2 + ((code >> (8 + 2 * (f - 2))) & 3);
        const double* gn = gacc + int64_t(nbr) * kGradStride;
        other = -0.5 * tp * tp * gn[2 + nf] - 0.5 * gn[7 + nf];
      }
      gZ += own + other;
    }
  }
  const double kap = aux[k * kAuxStride + 4], rho = aux[k * kAuxStride + 5];
  const double c = std::sqrt(kap / rho);
  gc[k] = ga[0] + rho * gZ;
  grho[k] = ga[1] + c * gZ;
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
    const double v = w[r] * vec[int64_t(r) * NP + i];
    U[base[r] + i].p += T(v);
    S[base[r] + i].p += T(sb * v);
  }
}

template <int N, typename T>
hipError_t launch_grad_stage_t(int64_t K, const void* sig, const void* Us, const void* Rs, const void* geo,
                               const int* conn, const double* aux, double dt, int flags, double* gacc,
                               hipStream_t st) {
  constexpr int EPB = 64 / Dim<N>::Nq;
  const int64_t nb = (K + EPB - 1) / EPB;
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL((grad_stage_kernel<N, T>), dim3(unsigned(nb)), dim3(64), 0, st, K,
                     static_cast<const V4<T>*>(sig), static_cast<const V4<T>*>(Us), static_cast<const V4<T>*>(Rs),
                     static_cast<const T*>(geo), conn, aux, dt, flags, gacc);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grad_stage(int N, int bits, int64_t K, const void* sig, const void* Us, const void* Rs,
                             const void* geo, const int* conn, const double* aux, double dt, int flags, double* gacc,
                             hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_grad_stage_t<n, T>(K, sig, Us, Rs, geo, conn, aux, dt, flags, gacc, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

hipError_t launch_grad_combine(int bits, int64_t K, const double* gacc, const void* geo, const int* conn,
                               const double* aux, int flags, double* gc, double* grho, hipStream_t st) {
  const unsigned nb = unsigned((K + 255) / 256);
  if (nb == 0) return hipSuccess;
  if (bits == 32)
    hipLaunchKernelGGL(grad_combine_kernel<float>, dim3(nb), dim3(256), 0, st, K, gacc,
                       static_cast<const float*>(geo), conn, aux, flags, gc, grho);
  else
    hipLaunchKernelGGL(grad_combine_kernel<double>, dim3(nb), dim3(256), 0, st, K, gacc,
                       static_cast<const double*>(geo), conn, aux, flags, gc, grho);
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
