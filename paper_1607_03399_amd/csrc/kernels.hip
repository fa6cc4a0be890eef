// HIP kernels of libwdg for CDNA4 (gfx950).
//
//   setup_kernel     FP64 geometric factors (Lemma 1), face Jacobians and normals,
//                    triangular lift L^{tri,k} = (M^{tri,k})^-1 M^tri (Sec. 4.2)
//   wedge_stage      one Runge-Kutta stage: volume term, surface fluxes, lifts,
//                    L^{tri,k} application and the low-storage update, fused
//   sample_receivers pressure at receiver points
//   energy_kernel    discrete energy with M^k = M^{tri,k} (x) M^1D
#include <hip/hip_runtime.h>

#include <cstring>

#include "kernels.hpp"

namespace wdg {
namespace {

template <int N>
struct Dim {
  static constexpr int NT = (N + 1) * (N + 2) / 2;
  static constexpr int Nq = N + 1;
  static constexpr int NP = NT * Nq;
  // per-element stride of L^{tri,k}: padded to whole 4-vectors
  static constexpr int LS = (NT * NT + 3) / 4 * 4;
};

__host__ __device__ constexpr int tri_idx(int N, int a, int b) { return b * (N + 1) - b * (b - 1) / 2 + a; }
// triangle node q (0..N) along edge e, from its first to its second vertex
__host__ __device__ constexpr int edge_node(int N, int e, int q) {
  return e == 0 ? tri_idx(N, q, 0) : (e == 1 ? tri_idx(N, N - q, q) : tri_idx(N, 0, N - q));
}

template <int N, typename T>
struct Ops {
  static constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq;
  T Dr[NT * NT];
  T Ds[NT * NT];
  T Ea[3][NT * Nq];
  T Eb[3][NT * Nq];
  T Dt[Nq * Nq];
  T g0[Nq];
  T gN[Nq];
  T tlo[Nq];  // (1 - t_j) / 2
  T thi[Nq];  // (1 + t_j) / 2
  int perm[6 * NT];
};

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

// Block size: 256 threads unless the staged state would exceed 64 KiB of LDS.
template <int N, typename T>
struct Cfg {
  static constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  static constexpr int lds(int bs) {
    return (bs / Nq) * NP * 4 * int(sizeof(T)) + (bs / Nq) * 2 * NT * 2 * int(sizeof(T));
  }
  static constexpr int BS = lds(256) <= 65536 ? 256 : (lds(128) <= 65536 ? 128 : 64);
  static constexpr int EPB = BS / Nq;
};

// ---------------------------------------------------------------------------
// Fused stage kernel
//
// Lane (element, level j) owns the triangular slice j of its element: the
// reference triangle operators are then the same for every lane (scalar
// operands), and only the vertical derivative and the triangle-face lift
// couple lanes of one element, through LDS.
// ---------------------------------------------------------------------------
template <int N, typename T>
__global__ void __launch_bounds__((Cfg<N, T>::BS)) wedge_stage(StageLaunch A) {
  using C = Cfg<N, T>;
  constexpr int NT = C::NT, Nq = C::Nq, NP = C::NP, EPB = C::EPB, BS = C::BS;
  constexpr int LS = Dim<N>::LS;
  __shared__ V4<T> sU[EPB * NP];
  __shared__ T sF[EPB * 2 * NT * 2];

  const Ops<N, T>* __restrict__ op = static_cast<const Ops<N, T>*>(A.ops);
  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  V4<T>* __restrict__ Uout = static_cast<V4<T>*>(A.Uout);
  V4<T>* __restrict__ res = static_cast<V4<T>*>(A.res);
  const T* __restrict__ geo = static_cast<const T*>(A.geo);
  const T* __restrict__ Lm = static_cast<const T*>(A.L);
  const int* __restrict__ conn = A.conn;

  // XCD-aware mapping: consecutive workgroups go to different XCDs, so give
  // every XCD one contiguous range of chunks (face neighbours share its L2).
  const int nb = gridDim.x, bid = blockIdx.x;
  const int qd = nb / 8, rm = nb % 8, xcd = bid % 8, kk = bid / 8;
  const int chunk = xcd < rm ? xcd * (qd + 1) + kk : rm * (qd + 1) + (xcd - rm) * qd + kk;
  const int64_t e0 = int64_t(chunk) * EPB;
  const int64_t left = A.K - e0;
  const int nE = left < EPB ? int(left) : EPB;
  const int tid = threadIdx.x;

  {
    const V4<T>* src = Uin + e0 * NP;
    for (int idx = tid; idx < nE * NP; idx += BS) sU[idx] = src[idx];
  }
  __syncthreads();

  const int le = tid / Nq;
  const int j = tid - le * Nq;
  const bool active = le < nE;
  const int64_t e = e0 + le;
  const bool dirichlet = (A.flags & kDirichlet) != 0;
  const bool central = (A.flags & kCentral) != 0;

  T Bp[NT], Bx[NT], By[NT], Bz[NT];

  if (active) {
    const T* g = geo + e * kGeoStride;
    const T tzJ = g[4];
    const T tlo = op->tlo[j], thi = op->thi[j];
    const T txJ = g[5] * tlo + g[6] * thi;
    const T tyJ = g[7] * tlo + g[8] * thi;
    const T Zm = g[11];
    const V4<T>* el = sU + le * NP;

    T p[NT], ux[NT], uy[NT], uz[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      V4<T> v = el[j * NT + i];
      p[i] = v.x;
      ux[i] = v.y;
      uy[i] = v.z;
      uz[i] = v.w;
    }

    // vertical part of D_x, D_y, D_z (before L^{tri,k}): W = t_dJ(t_j) D_t U
    T dtrow[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) dtrow[m] = op->Dt[j * Nq + m];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T dP = 0, dX = 0, dY = 0, dZ = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        V4<T> v = el[m * NT + i];
        dP += dtrow[m] * v.x;
        dX += dtrow[m] * v.y;
        dY += dtrow[m] * v.z;
        dZ += dtrow[m] * v.w;
      }
      Bp[i] = -(txJ * dX + tyJ * dY + tzJ * dZ);
      Bx[i] = -txJ * dP;
      By[i] = -tyJ * dP;
      Bz[i] = -tzJ * dP;
    }

    const int* cn = conn + e * kConnStride;
    const int code = cn[5];

    // quadrilateral faces: nodes of edge e on this lane's level j
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      const int nbr = cn[2 + ed];
      const int ned = (code >> (8 + 2 * ed)) & 3;
      const T Ja = g[20 + 4 * ed], Jb = g[21 + 4 * ed];
      const T nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
      const T Zp = nbr >= 0 ? geo[int64_t(nbr) * kGeoStride + 11] : Zm;
      const T taup = central ? T(0) : T(2) / (Zm + Zp);
      const T tauu = central ? T(0) : (Zm + Zp) * T(0.5);
      const V4<T>* nb_el = Uin + int64_t(nbr >= 0 ? nbr : 0) * NP + j * NT;
      T fap[Nq], fbp[Nq], fau[Nq], fbu[Nq];
#pragma unroll
      for (int q = 0; q < Nq; ++q) {
        const int i = edge_node(N, ed, q);
        const T pm = p[i];
        const T unm = nx * ux[i] + ny * uy[i];
        T pp, unp;
        if (nbr >= 0) {
          const int ni = ned == 0 ? edge_node(N, 0, N - q) : (ned == 1 ? edge_node(N, 1, N - q) : edge_node(N, 2, N - q));
          const V4<T> v = nb_el[ni];
          pp = v.x;
          unp = nx * v.y + ny * v.z;
        } else if (dirichlet) {
          pp = -pm;
          unp = unm;
        } else {
          pp = pm;
          unp = -unm;
        }
        const T jp = pp - pm, jun = unp - unm;
        const T Fp = T(0.5) * (taup * jp - jun);
        const T Fu = T(0.5) * (tauu * jun - jp);
        fap[q] = Ja * Fp;
        fbp[q] = Jb * Fp;
        fau[q] = Ja * Fu;
        fbu[q] = Jb * Fu;
      }
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        T sp = 0, su = 0;
#pragma unroll
        for (int q = 0; q < Nq; ++q) {
          const T ea = op->Ea[ed][i * Nq + q], eb = op->Eb[ed][i * Nq + q];
          sp += ea * fap[q] + eb * fbp[q];
          su += ea * fau[q] + eb * fbu[q];
        }
        Bp[i] += sp;
        Bx[i] += nx * su;
        By[i] += ny * su;
      }
    }

    // triangular faces: the bottom level computes the bottom face, the top level the top face
    if (j == 0 || j == N) {
      const int face = j == 0 ? 0 : 1;
      const int nbr = cn[face];
      const int pc = (code >> (3 * face)) & 7;
      const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
      const T Jf = g[12 + 4 * face];
      const T nx = g[13 + 4 * face], ny = g[14 + 4 * face], nz = g[15 + 4 * face];
      const T Zp = nbr >= 0 ? geo[int64_t(nbr) * kGeoStride + 11] : Zm;
      const T taup = central ? T(0) : T(2) / (Zm + Zp);
      const T tauu = central ? T(0) : (Zm + Zp) * T(0.5);
      const V4<T>* nb_el = Uin + int64_t(nbr >= 0 ? nbr : 0) * NP + nlev * NT;
      T* f = sF + (le * 2 + face) * NT * 2;
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const T pm = p[i];
        const T unm = nx * ux[i] + ny * uy[i] + nz * uz[i];
        T pp, unp;
        if (nbr >= 0) {
          const V4<T> v = nb_el[op->perm[pc * NT + i]];
          pp = v.x;
          unp = nx * v.y + ny * v.z + nz * v.w;
        } else if (dirichlet) {
          pp = -pm;
          unp = unm;
        } else {
          pp = pm;
          unp = -unm;
        }
        const T jp = pp - pm, jun = unp - unm;
        f[2 * i] = Jf * T(0.5) * (taup * jp - jun);
        f[2 * i + 1] = Jf * T(0.5) * (tauu * jun - jp);
      }
    }
  }
  __syncthreads();
  if (!active) return;

  const T* g = geo + e * kGeoStride;
  const V4<T>* el = sU + le * NP;
  // triangular-face lifts: flux spread over all levels by (M^1D)^-1 e_{0,N}
  {
    const T g0j = op->g0[j], gNj = op->gN[j];
    const T bx = g[13], by = g[14], bz = g[15], tx = g[17], ty = g[18], tz = g[19];
    const T* fb = sF + (le * 2 + 0) * NT * 2;
    const T* ft = sF + (le * 2 + 1) * NT * 2;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      Bp[i] += g0j * fb[2 * i] + gNj * ft[2 * i];
      const T wb = g0j * fb[2 * i + 1], wt = gNj * ft[2 * i + 1];
      Bx[i] += wb * bx + wt * tx;
      By[i] += wb * by + wt * ty;
      Bz[i] += wb * bz + wt * tz;
    }
  }

  // horizontal part: (r_x D_r + s_x D_s) etc. on the own slice
  T Rp[NT], Rx[NT], Ry[NT], Rz[NT];
  {
    const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
    T P[NT], Ar[NT], As[NT];
#pragma unroll
    for (int m = 0; m < NT; ++m) {
      const V4<T> v = el[j * NT + m];
      P[m] = v.x;
      Ar[m] = rx * v.y + ry * v.z;
      As[m] = sx * v.y + sy * v.z;
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T dA = 0, dPr = 0, dPs = 0;
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const T dr = op->Dr[i * NT + m], ds = op->Ds[i * NT + m];
        dA += dr * Ar[m] + ds * As[m];
        dPr += dr * P[m];
        dPs += ds * P[m];
      }
      Rp[i] = -dA;
      Rx[i] = -(rx * dPr + sx * dPs);
      Ry[i] = -(ry * dPr + sy * dPs);
      Rz[i] = 0;
    }
  }

  // triangular lift L^{tri,k} applied to every field on this level
  {
    const V4<T>* Lv = reinterpret_cast<const V4<T>*>(Lm + e * LS);
#pragma unroll
    for (int c = 0; c < LS / 4; ++c) {
      const V4<T> l4 = Lv[c];
      const T lv[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int f = 4 * c + k;
        if (f < NT * NT) {
          const int i = f / NT, m = f % NT;
          Rp[i] += lv[k] * Bp[m];
          Rx[i] += lv[k] * Bx[m];
          Ry[i] += lv[k] * By[m];
          Rz[i] += lv[k] * Bz[m];
        }
      }
    }
  }

  const T kap = g[9], irho = g[10];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    Rp[i] *= kap;
    Rx[i] *= irho;
    Ry[i] *= irho;
    Rz[i] *= irho;
  }
  for (int s = 0; s < A.nsrc; ++s) {
    if (A.src_elem[s] == e) {
      const T* sv = static_cast<const T*>(A.srcvec) + s * NP + j * NT;
      const T amp = T(A.src_amp[s]);
#pragma unroll
      for (int i = 0; i < NT; ++i) Rp[i] += amp * sv[i];
    }
  }

  // low-storage Runge-Kutta update
  const T ca = T(A.a), cb = T(A.b), dt = T(A.dt);
  const bool rd = (A.flags & kReadRes) != 0, wu = (A.flags & kWriteU) != 0;
  V4<T>* rr = res + e * NP + j * NT;
  V4<T>* uo = Uout + e * NP + j * NT;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    V4<T> r;
    if (rd) {
      r = rr[i];
      r.x = ca * r.x + dt * Rp[i];
      r.y = ca * r.y + dt * Rx[i];
      r.z = ca * r.z + dt * Ry[i];
      r.w = ca * r.w + dt * Rz[i];
    } else {
      r.x = dt * Rp[i];
      r.y = dt * Rx[i];
      r.z = dt * Ry[i];
      r.w = dt * Rz[i];
    }
    rr[i] = r;
    if (wu) {
      V4<T> u = el[j * NT + i];
      u.x += cb * r.x;
      u.y += cb * r.y;
      u.z += cb * r.z;
      u.w += cb * r.w;
      uo[i] = u;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 setup: one wavefront per element
// ---------------------------------------------------------------------------
constexpr int kMaxNT = 21;

template <typename T>
__global__ void __launch_bounds__(64) setup_kernel(int NT, int LS, int64_t K, const double* __restrict__ X,
                                                   const double* __restrict__ Mv, const double* __restrict__ Mtri,
                                                   T* __restrict__ geo, T* __restrict__ L, double* __restrict__ aux) {
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
    // [ M^{tri,k} | M^tri ], M^{tri,k} = sum_v (J_tri h_v / 2) int l_a l_b lambda_v
    for (int idx = tid; idx < NT * W; idx += 64) {
      const int r = idx / W, c = idx - r * W;
      double v;
      if (c < NT) {
        v = cw[0] * Mv[r * NT + c] + cw[1] * Mv[NT * NT + r * NT + c] + cw[2] * Mv[2 * NT * NT + r * NT + c];
      } else {
        v = Mtri[r * NT + (c - NT)];
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
    for (int idx = tid; idx < LS; idx += 64) {
      double v = 0.0;
      if (idx < NT * NT) {
        const int r = idx / NT, c = idx - r * NT;
        v = Aug[r * W + NT + c];
      }
      L[k * LS + idx] = T(v);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void material_kernel(int64_t K, const double* __restrict__ c, const double* __restrict__ rho,
                                T* __restrict__ geo, double* __restrict__ aux) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double kap = rho[k] * c[k] * c[k];
  geo[k * kGeoStride + 9] = T(kap);
  geo[k * kGeoStride + 10] = T(1.0 / rho[k]);
  geo[k * kGeoStride + 11] = T(rho[k] * c[k]);
  aux[k * kAuxStride + 4] = kap;
  aux[k * kAuxStride + 5] = rho[k];
}

template <typename T>
__global__ void sample_receivers(int NP, int nrec, const T* __restrict__ U, const int* __restrict__ elem,
                                 const double* __restrict__ rows, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const T* Ue = U + int64_t(elem[r]) * NP * 4;
  double acc = 0.0;
  for (int n = 0; n < NP; ++n) acc += rows[int64_t(r) * NP + n] * double(Ue[4 * n]);
  out[r] = acc;
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

template <int N, typename T>
void fill_ops_t(void* dst, const double* Dr, const double* Ds, const double* const* Ea, const double* const* Eb,
                const double* Dt, const double* g0, const double* gN, const double* t, const int* perm) {
  using O = Ops<N, T>;
  constexpr int NT = O::NT, Nq = O::Nq;
  O* o = static_cast<O*>(dst);
  std::memset(o, 0, sizeof(O));
  for (int i = 0; i < NT * NT; ++i) {
    o->Dr[i] = T(Dr[i]);
    o->Ds[i] = T(Ds[i]);
  }
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < NT * Nq; ++i) {
      o->Ea[e][i] = T(Ea[e][i]);
      o->Eb[e][i] = T(Eb[e][i]);
    }
  for (int i = 0; i < Nq * Nq; ++i) o->Dt[i] = T(Dt[i]);
  for (int j = 0; j < Nq; ++j) {
    o->g0[j] = T(g0[j]);
    o->gN[j] = T(gN[j]);
    o->tlo[j] = T(0.5 * (1.0 - t[j]));
    o->thi[j] = T(0.5 * (1.0 + t[j]));
  }
  for (int i = 0; i < 6 * NT; ++i) o->perm[i] = perm[i];
}

template <int N, typename T>
hipError_t launch_stage_t(const StageLaunch& a, hipStream_t st) {
  using C = Cfg<N, T>;
  const int64_t nchunks = (a.K + C::EPB - 1) / C::EPB;
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL((wedge_stage<N, T>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  return hipGetLastError();
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

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define WDG_DISPATCH_N(N_, BITS_, CALL)                    \
  switch (N_) {                                            \
    case 1: if (BITS_ == 32) { CALL(1, float); } else { CALL(1, double); } break; \
    case 2: if (BITS_ == 32) { CALL(2, float); } else { CALL(2, double); } break; \
    case 3: if (BITS_ == 32) { CALL(3, float); } else { CALL(3, double); } break; \
    case 4: if (BITS_ == 32) { CALL(4, float); } else { CALL(4, double); } break; \
    case 5: if (BITS_ == 32) { CALL(5, float); } else { CALL(5, double); } break; \
    default: break;                                        \
  }

size_t ops_bytes(int N, int bits) {
  size_t out = 0;
#define WDG_SZ(n, T) out = sizeof(Ops<n, T>)
  WDG_DISPATCH_N(N, bits, WDG_SZ)
#undef WDG_SZ
  return out;
}

void fill_ops(int N, int bits, void* dst, const double* Dr, const double* Ds, const double* const* Ea,
              const double* const* Eb, const double* Dt, const double* g0, const double* gN, const double* t,
              const int* perm) {
#define WDG_FILL(n, T) fill_ops_t<n, T>(dst, Dr, Ds, Ea, Eb, Dt, g0, gN, t, perm)
  WDG_DISPATCH_N(N, bits, WDG_FILL)
#undef WDG_FILL
}

int lift_stride(int N) {
  const int NT = (N + 1) * (N + 2) / 2;
  return (NT * NT + 3) / 4 * 4;
}

hipError_t launch_setup(int N, int bits, int64_t K, const double* dX, const double* dMv, const double* dMtri,
                        void* dGeo, void* dL, double* dAux, hipStream_t st) {
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

hipError_t launch_material(int bits, int64_t K, const double* dc, const double* drho, void* dGeo, double* dAux,
                           hipStream_t st) {
  const unsigned nb = unsigned((K + 255) / 256);
  if (nb == 0) return hipSuccess;
  if (bits == 32)
    hipLaunchKernelGGL(material_kernel<float>, dim3(nb), dim3(256), 0, st, K, dc, drho, static_cast<float*>(dGeo), dAux);
  else
    hipLaunchKernelGGL(material_kernel<double>, dim3(nb), dim3(256), 0, st, K, dc, drho, static_cast<double*>(dGeo),
                       dAux);
  return hipGetLastError();
}

hipError_t launch_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

hipError_t launch_receivers(int bits, int NP, int nrec, const void* U, const int* elem, const double* rows,
                            double* out, hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  const unsigned nb = unsigned((nrec + 63) / 64);
  if (bits == 32)
    hipLaunchKernelGGL(sample_receivers<float>, dim3(nb), dim3(64), 0, st, NP, nrec, static_cast<const float*>(U), elem,
                       rows, out);
  else
    hipLaunchKernelGGL(sample_receivers<double>, dim3(nb), dim3(64), 0, st, NP, nrec, static_cast<const double*>(U),
                       elem, rows, out);
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

}  // namespace wdg
