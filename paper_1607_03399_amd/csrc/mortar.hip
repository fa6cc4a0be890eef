// Mortar kernel of libwdg: wedge quadrilateral faces covered by two
// tetrahedron triangles, coupled on the common refinement.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace wdg {
namespace {

// ---------------------------------------------------------------------------
// Only the pressure and the normal velocity enter the flux, so both traces of
// a mortar are carried as (p, u.n) with the wedge's outward normal.  On side s
// of the diagonal the traces are z_s = [wedge face nodes (level-major,
// Nq x Nq); tetrahedron face nodes (Np_tri)], and every integral the flux
// needs is a product with the symmetric matrix
//   C_s = int_{side s} b b^T dA,   b = (wedge face basis, tetrahedron face basis),
// which depends on the geometry only: the host integrates it once per mesh in
// FP64 (mort_nx(N) Gauss points along the edge times Nq in t on each side of
// the diagonal, exact in t) and stores its lower triangle.  With the wedge
// part of z_s negated, C_s z_s holds the moments of the jump (tetrahedron
// trace minus wedge trace) against both bases; the upwind / central flux
// combinations follow, then
//   wedge:       pre-lift contributions, (M^1D)^-1 in t and (M^tri)^-1
//                restricted to the edge nodes, applied to the wedge moments
//   tetrahedra:  equivalent nodal face flux (M^tri)^-1 (moments) / (area / 2)
// One wavefront per mortar.
// ---------------------------------------------------------------------------
template <int N>
struct MortTab {
  static constexpr int NT = (N + 1) * (N + 2) / 2, Nq = N + 1;
  static constexpr int MI1 = 0, ME = Nq * Nq, MTI = ME + 3 * NT * Nq, SIZE = MTI + NT * NT;
};

// Cache policy of the coupling-matrix loads: each value is read once per
// stage, so they stream (non-temporal) instead of evicting the state vectors
// that the wedge and tetrahedron kernels read next (on the 39 312-wedge +
// 29 520-tetrahedron N = 4 hybrid mesh the default
// policy cost those kernels 14 and 4 us per stage)
#ifndef WDG_MORT_CORE_AUX
#define WDG_MORT_CORE_AUX 2
#endif
// 4-vector idx of a buffer resource; past its end the hardware returns zeros
template <typename T>
__device__ __forceinline__ V4<T> core_load(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(V4<T>, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16, 0, WDG_MORT_CORE_AUX));
  } else {
    struct H2 {
      u32x4 lo, hi;
    } h{__builtin_amdgcn_raw_buffer_load_b128(r, idx * 32, 0, WDG_MORT_CORE_AUX),
        __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32 + 16, 0, WDG_MORT_CORE_AUX)};
    return __builtin_bit_cast(V4<T>, h);
  }
}

// packed lower triangle by columns: entry (r, c), r >= c
template <int n>
__device__ __forceinline__ constexpr int pk(int c, int r) {
  return c * n - (c * (c - 1)) / 2 + (r - c);
}

template <int N, typename T>
__global__ void __launch_bounds__(64) mortar_kernel(StageLaunch A) {
  using TB = MortTab<N>;
  constexpr int NT = TB::NT, Nq = TB::Nq;
  constexpr int NPW = Dim<N>::NP, NPT = TDim<N>::NP;
  constexpr int NW = Nq * Nq, n = mort_core_n(N), NPK = n * (n + 1) / 2, CS = mort_core_stride(N);
  constexpr int CV = CS / 4, CVL = (CV + 63) / 64;  // 4-vectors of the coupling matrices, per lane
  constexpr int NST = NW + 2 * NT, NSL = (NST + 63) / 64;
  constexpr int NTP = (NT + 3) / 4 * 4;
  static_assert(n <= 64 && 2 * NTP <= 64, "one lane per matrix row and per wedge output column");
  __shared__ V4<T> sC[CV];       // the mortar's coupling matrices, both sides
  __shared__ T sZ[2 * 2 * n];    // [side][field][-wedge ; tetrahedron of the side]
  __shared__ T sMW[2 * NW];      // wedge flux moments [field][level * Nq + edge node]
  __shared__ T sMT[2 * 2 * NT];  // tetrahedron flux moments [side][field][face node]

  const T* __restrict__ tab = static_cast<const T*>(A.mortTab);
  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const int tid = threadIdx.x;
  const int64_t mo = blockIdx.x;
  const int* mi = A.mortI + mo * kMortIntStride;
  const double* mg = static_cast<const double*>(A.mortG) + mo * kMortGeoStride;
  // Loads in the order their results are needed, each issued before any
  // wait: the mortar's record, its coupling matrices (which do not depend on
  // the record), then the node gathers addressed from the record.  The
  // vector-memory counter completes in order, so waiting for the record does
  // not wait for the matrices.
  const int wel = mi[0], e = mi[1], t0 = mi[3], f0 = mi[4], t1 = mi[5], f1 = mi[6];
  const double mgx = mg[5], mgy = mg[6], mz0 = mg[27], mz1 = mg[28], ms0 = mg[25], ms1 = mg[26];
  V4<T> cv[CVL];
  {
    const auto rc = chunk_rsrc(static_cast<const V4<T>*>(A.mortC) + mo * CV, int64_t(CV) * 4 * int64_t(sizeof(T)));
#pragma unroll
    for (int l = 0; l < CVL; ++l) cv[l] = core_load<T>(rc, tid + 64 * l);
  }

  // node values: the wedge face (Nq x Nq, level-major), then both tetrahedron
  // faces; lanes past them read node 0 (a valid address, never used)
  V4<T> nv[NSL];
#pragma unroll
  for (int l = 0; l < NSL; ++l) {
    const int idx = tid + 64 * l;
    const int lev = idx / Nq, q = idx - lev * Nq;
    const int r = idx - NW, side = r >= NT ? 1 : 0, i = r - side * NT;
    const int64_t aw = int64_t(wel) * NPW + lev * NT + edge_node(N, e, q < Nq ? q : 0);
    const int64_t at = A.Kw * NPW + (int64_t(side ? t1 : t0) - A.Kw) * NPT +
                       tet_face_node<N>(side ? f1 : f0, i >= 0 && i < NT ? i : 0);
    nv[l] = Uin[idx < NW ? aw : (idx < NST ? at : 0)];
  }
  const T nx = T(mgx), ny = T(mgy);
#pragma unroll
  for (int l = 0; l < NSL; ++l) {
    const int idx = tid + 64 * l;
    const T vp = nv[l].p, vn = nx * nv[l].ux + ny * nv[l].uy;
    if (idx < NW) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        sZ[(2 * s + 0) * n + idx] = -vp;
        sZ[(2 * s + 1) * n + idx] = -vn;
      }
    } else if (idx < NST) {
      const int r = idx - NW, side = r / NT, i = r - side * NT;
      sZ[(2 * side + 0) * n + NW + i] = vp;
      sZ[(2 * side + 1) * n + NW + i] = vn;
    }
  }
#pragma unroll
  for (int l = 0; l < CVL; ++l)
    if (tid + 64 * l < CV) sC[tid + 64 * l] = cv[l];
  __syncthreads();

  // jump moments J = (C_s z_s) / 2 (lane = matrix row), then the fluxes:
  //   wedge        F_p = taup J_p - J_u,   F_u = tauu J_u - J_p
  //   tetrahedron  F_p = -taup J_p - J_u,  F_u = tauu J_u + J_p  (the jump seen from its side)
  const T tau_on = (A.flags & kCentral) ? T(0) : T(1);
  if (tid < n) {
    const T* C = reinterpret_cast<const T*>(sC);
    T wp = 0, wn = 0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* Cs = C + s * NPK;
      const T* zp = sZ + (2 * s) * n;
      const T* zn = zp + n;
      T dp = 0, dn = 0;
#pragma unroll
      for (int c = 0; c < n; ++c) {
        const T cc = Cs[c <= tid ? pk<n>(c, tid) : pk<n>(tid, c)];
        dp += cc * zp[c];
        dn += cc * zn[c];
      }
      const T zs = T(s == 0 ? mz0 : mz1);
      const T taup = tau_on * T(2) / zs, tauu = tau_on * zs * T(0.5);
      if (tid < NW) {
        wp += T(0.5) * (taup * dp - dn);
        wn += T(0.5) * (tauu * dn - dp);
      } else {
        sMT[(2 * s + 0) * NT + tid - NW] = T(0.5) * (-taup * dp - dn);
        sMT[(2 * s + 1) * NT + tid - NW] = T(0.5) * (tauu * dn + dp);
      }
    }
    if (tid < NW) {
      sMW[tid] = wp;
      sMW[NW + tid] = wn;
    }
  }
  __syncthreads();

  // wedge pre-lift contributions [field][level j][node i] (i padded to NTP):
  //   sum_m (M^1D)^-1[j][m] sum_q (M^tri)^-1[i][node q of edge e] moments[m][q]
  if (tid < 2 * NTP) {
    const int f = tid / NTP, i = tid - f * NTP;
    T G[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) {
      T acc = 0;
      if (i < NT) {
#pragma unroll
        for (int q = 0; q < Nq; ++q) acc += tab[TB::ME + (e * NT + i) * Nq + q] * sMW[f * NW + m * Nq + q];
      }
      G[m] = acc;
    }
    T* outB = static_cast<T*>(A.mortB) + mo * (2 * Nq * NTP) + f * Nq * NTP + i;
#pragma unroll
    for (int j = 0; j < Nq; ++j) {
      T acc = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) acc += tab[TB::MI1 + j * Nq + m] * G[m];
      outB[j * NTP] = acc;
    }
  }
  // equivalent nodal flux of both tetrahedron faces [side][field][node]
  for (int o = tid; o < 4 * NT; o += 64) {
    const int side = o / (2 * NT), r = o - side * 2 * NT, f = r / NT, i = r - f * NT;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < NT; ++k) acc += tab[TB::MTI + i * NT + k] * sMT[(2 * side + f) * NT + k];
    static_cast<T*>(A.mortF)[(mo * 2 + side) * 2 * NT + f * NT + i] = acc * T(side ? ms1 : ms0);
  }
}

template <int N, typename T>
hipError_t launch_mortar_stage_t(const StageLaunch& a, hipStream_t st) {
  if (a.nmort <= 0) return hipSuccess;
  if (a.nmort > int64_t(0x7fffffff) || !a.mortC) return hipErrorInvalidValue;
  hipLaunchKernelGGL((mortar_kernel<N, T>), dim3(unsigned(a.nmort)), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mortar_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_mortar_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

int mortar_table_size(int N) {
  switch (N) {
    case 1: return MortTab<1>::SIZE;
    case 2: return MortTab<2>::SIZE;
    case 3: return MortTab<3>::SIZE;
    case 4: return MortTab<4>::SIZE;
    case 5: return MortTab<5>::SIZE;
    default: return 0;
  }
}

}  // namespace wdg
