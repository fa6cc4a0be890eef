// Mortar kernel of libwdg: wedge quadrilateral faces covered by two
// tetrahedron triangles, coupled on the common refinement.
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace wdg {
namespace {

// ---------------------------------------------------------------------------
// Mortar kernel: wedge quadrilateral faces covered by two tetrahedron triangles
//
// The flux is integrated on the common refinement in the wedge face's
// coordinates (edge parameter xi, vertical t): mort_nx(N) Gauss points in xi
// times Nq Gauss points in t on each side of the diagonal (exact in t).  Only
// the pressure and the normal velocity enter the flux, so both traces are
// carried as (p, u.n) with the wedge's outward normal.  One wavefront per
// mortar (persistent over mortars):
//   0. the wedge face interpolated to the edge points at every GLL level
//      (sum factorisation: per point only the Nq-term sum in t remains), and
//      the Legendre-product modal coefficients of both tetrahedron faces
//   per side of the diagonal:
//   1. per point: the GLL basis in t, both traces, the jumps
//   2. tetrahedron moments int phi_md F' (modes recomputed from the point's
//      face coordinates; the points are split over lane groups) and the wedge
//      sums H_f[a][m] = sum_g w F_f l_m(t_g) of each edge point a
//   3. wedge pre-lift contributions sum_a A[e][a][i] H_f[a][m]; the equivalent
//      nodal flux of the tetrahedron face, (M^tri)^-1 Vinv^T moments / (area/2)
//   and at the end the levels resolved by (M^1D)^-1.
// ---------------------------------------------------------------------------
template <int N, int BITS>
struct MortTab {
  static constexpr int NT = (N + 1) * (N + 2) / 2, Nq = N + 1, NX = mort_nx(N, BITS);
  static constexpr int XG = 0, WG = NX, TG = 2 * NX, WT = TG + Nq, TGLL = WT + Nq, DEN = TGLL + Nq;
  static constexpr int MI1 = DEN + Nq * Nq, E = MI1 + Nq * Nq, A = E + NX * Nq, VI = A + 3 * NT * NX;
  static constexpr int P = VI + NT * NT;
  static constexpr int SIZE = P + NT * NT;
};

// The mortar arithmetic runs in FP64 for either state precision: the
// tetrahedron trace goes through a Legendre-product Vandermonde whose
// conditioning would cost FP32 digits at high order; tables and records are
// FP64 as well.  The tables are read through the vector caches (they are
// small and shared by every wavefront of a CU); LDS holds only per-mortar data.
template <int N, typename T>
__global__ void __launch_bounds__(64) mortar_kernel(StageLaunch A) {
  using TB = MortTab<N, int(sizeof(T)) * 8>;
  using D = double;
  constexpr int NT = TB::NT, Nq = TB::Nq, NX = TB::NX;
  constexpr int NPW = Dim<N>::NP, NPT = TDim<N>::NP;
  constexpr int NQ1 = NX * Nq;          // points on one side of the diagonal
  constexpr int PPL = (NQ1 + 63) / 64;  // points per lane
  constexpr int NTP = (NT + 3) / 4 * 4;
  constexpr int NB = 2 * Nq * NTP;      // wedge outputs per mortar [field][level][node]
  constexpr int NBL = (NB + 63) / 64;   // ... per lane
  constexpr int CH = 64 / NT;           // lane groups of the moment sums
  constexpr int QC = (NQ1 + CH - 1) / CH;
  constexpr int NWH = 2 * NX * Nq;      // interpolated wedge face [field][a][m]
  __shared__ V4<T> sW[Nq * Nq];   // wedge face nodes [level][edge node]
  __shared__ V4<T> sTF[2 * NT];   // tetrahedron face nodes [side][face node]
  __shared__ D sWh[NWH];          // wedge face at the edge points [field][a][level]
  __shared__ D sCT[4 * NT];       // tetrahedron modal coefficients [side][field][mode]
  __shared__ D sLT[NQ1 * Nq];     // per point: GLL basis in t
  __shared__ D sJ[NQ1 * 2];       // per point: w [p] / 2, w [u.n] / 2
  __shared__ D sRS[NQ1 * 2];      // per point: tetrahedron face coordinates
  __shared__ D sH[2 * NX * Nq];   // [field][a][level]
  __shared__ D sRed[CH * 2 * NT]; // partial moments [group][field][mode]
  __shared__ D sB[NB];            // wedge outputs before (M^1D)^-1

  // constant address space: the tables are read-only for the whole launch, so
  // wave-uniform reads go through scalar loads
  using CD = __attribute__((address_space(4))) const D;
  // constant address space: the tables are read-only for the whole launch, so
  // wave-uniform reads go through scalar loads
  using CD = __attribute__((address_space(4))) const D;
  CD* tab = (CD*)(A.mortTab);
  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const D tau_on = (A.flags & kCentral) ? 0.0 : 1.0;
  const int tid = threadIdx.x;
  const int64_t tb = A.Kw * NPW;
  // mode (aa, bb) of a lane's moment sums
  const int mmd = tid % NT, mgr = tid / NT;
  int maa = 0, mbb = mmd;
#pragma unroll
  for (int aa = 0; aa < N; ++aa)
    if (maa == aa && mbb > N - aa) {
      mbb -= N - aa + 1;
      maa = aa + 1;
    }

  // node values a mortar reads: the wedge face (Nq x Nq) and both tetrahedron
  // faces (2 x NT); each lane loads at most NSL of them, one mortar ahead
  constexpr int NST = Nq * Nq + 2 * NT, NSL = (NST + 63) / 64;
  auto node_index = [&](int64_t m, int idx) -> int64_t {
    const int* mm = A.mortI + m * kMortIntStride;
    if (idx < Nq * Nq) {
      const int lev = idx / Nq, q = idx - lev * Nq;
      return int64_t(mm[0]) * NPW + lev * NT + edge_node(N, mm[1], q);
    }
    const int r = idx - Nq * Nq, side = r / NT, i = r - side * NT;
    return tb + (int64_t(mm[3 + 2 * side]) - A.Kw) * NPT + tet_face_node<N>(mm[4 + 2 * side], i);
  };
  V4<T> pre[NSL];
#pragma unroll
  for (int l = 0; l < NSL; ++l) pre[l] = V4<T>{T(0), T(0), T(0), T(0)};
  if (blockIdx.x < A.nmort) {
#pragma unroll
    for (int l = 0; l < NSL; ++l)
      if (tid + 64 * l < NST) pre[l] = Uin[node_index(blockIdx.x, tid + 64 * l)];
  }

  for (int64_t mo = blockIdx.x; mo < A.nmort; mo += gridDim.x) {
    const int* mi = A.mortI + mo * kMortIntStride;
    const D* mg = static_cast<const D*>(A.mortG) + mo * kMortGeoStride;
    const int e = mi[1], diag = mi[2];
    __syncthreads();  // the previous mortar is done with LDS
#pragma unroll
    for (int l = 0; l < NSL; ++l) {
      const int idx = tid + 64 * l;
      if (idx < Nq * Nq)
        sW[idx] = pre[l];
      else if (idx < NST)
        sTF[idx - Nq * Nq] = pre[l];
    }
    // the next mortar's node values load while this one computes
    if (mo + gridDim.x < A.nmort) {
#pragma unroll
      for (int l = 0; l < NSL; ++l)
        if (tid + 64 * l < NST) pre[l] = Uin[node_index(mo + gridDim.x, tid + 64 * l)];
    }
    const D zba = mg[0], zbb = mg[1], zta = mg[2], ztb = mg[3], ell = mg[4], nx = mg[5], ny = mg[6];
    __syncthreads();
    // 0. wedge face at the edge points; tetrahedron modal coefficients
    for (int o = tid; o < NWH + 4 * NT; o += 64) {
      D acc = 0;
      if (o < NWH) {
        const int f = o / (NX * Nq), rem = o - f * NX * Nq, a = rem / Nq, m = rem - a * Nq;
#pragma unroll
        for (int qq = 0; qq < Nq; ++qq) {
          const V4<T> v = sW[m * Nq + qq];
          const D val = f == 0 ? D(v.p) : nx * D(v.ux) + ny * D(v.uy);
          acc += tab[TB::E + a * Nq + qq] * val;
        }
        sWh[o] = acc;
      } else {
        const int r = o - NWH, side = r / (2 * NT), f = (r / NT) & 1, md = r % NT;
#pragma unroll 5
        for (int i = 0; i < NT; ++i) {
          const V4<T> v = sTF[side * NT + i];
          const D val = f == 0 ? D(v.p) : nx * D(v.ux) + ny * D(v.uy);
          acc += tab[TB::VI + md * NT + i] * val;
        }
        sCT[r] = acc;
      }
    }
    D accB[NBL];
#pragma unroll
    for (int r = 0; r < NBL; ++r) accB[r] = 0.0;

    for (int side = 0; side < 2; ++side) {
      __syncthreads();
      // 1. traces and jumps at the points of this side
#pragma unroll 1
      for (int pp = 0; pp < PPL; ++pp) {
        const int q = tid + 64 * pp;
        if (q >= NQ1) break;
        const int a = q / Nq, g = q - a * Nq;
        const D xi = tab[TB::XG + a];
        const D zb = zba * 0.5 * (1.0 - xi) + zbb * 0.5 * (1.0 + xi);
        const D zt = zta * 0.5 * (1.0 - xi) + ztb * 0.5 * (1.0 + xi);
        const D h = zt - zb;
        const D zd = diag == 0 ? zba * 0.5 * (1.0 - xi) + ztb * 0.5 * (1.0 + xi)
                               : zbb * 0.5 * (1.0 + xi) + zta * 0.5 * (1.0 - xi);
        const D td = (2.0 * zd - zb - zt) / h;
        const D lo = side == 0 ? -1.0 : td, hi = side == 0 ? td : 1.0;
        const D t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * tab[TB::TG + g];
        const D w = tab[TB::WG + a] * tab[TB::WT + g] * 0.5 * (hi - lo) * 0.25 * ell * h;
        const D z = zb * 0.5 * (1.0 - t) + zt * 0.5 * (1.0 + t);
        D wp = 0, wn = 0;
#pragma unroll
        for (int m = 0; m < Nq; ++m) {
          D v = 1.0;
#pragma unroll
          for (int mm = 0; mm < Nq; ++mm)
            if (mm != m) v *= (t - tab[TB::TGLL + mm]) * tab[TB::DEN + m * Nq + mm];
          sLT[q * Nq + m] = v;
          wp += v * sWh[a * Nq + m];
          wn += v * sWh[NX * Nq + a * Nq + m];
        }
        const D* lm = mg + 7 + 9 * side;
        const D l1 = lm[3] * xi + lm[4] * z + lm[5];
        const D l2 = lm[6] * xi + lm[7] * z + lm[8];
        const D rr = 2.0 * l1 - 1.0, ss = 2.0 * l2 - 1.0;
        D Pr[Nq], Ps[Nq];
        Pr[0] = Ps[0] = 1.0;
        Pr[1] = rr;
        Ps[1] = ss;
#pragma unroll
        for (int n = 1; n < N; ++n) {
          Pr[n + 1] = ((2 * n + 1) * rr * Pr[n] - n * Pr[n - 1]) * (1.0 / (n + 1));
          Ps[n + 1] = ((2 * n + 1) * ss * Ps[n] - n * Ps[n - 1]) * (1.0 / (n + 1));
        }
        D tp = 0, tn = 0;
        {
          int md = 0;
#pragma unroll
          for (int aa = 0; aa <= N; ++aa)
#pragma unroll
            for (int bb = 0; bb + aa <= N; ++bb) {
              const D ph = Pr[aa] * Ps[bb];
              tp += ph * sCT[side * 2 * NT + md];
              tn += ph * sCT[side * 2 * NT + NT + md];
              ++md;
            }
        }
        sRS[q * 2 + 0] = rr;
        sRS[q * 2 + 1] = ss;
        sJ[q * 2 + 0] = 0.5 * w * (tp - wp);
        sJ[q * 2 + 1] = 0.5 * w * (tn - wn);
      }
      const D zs = mg[27 + side];
      const D taup = tau_on * 2.0 / zs, tauu = tau_on * zs * 0.5;
      __syncthreads();
      // 2a. tetrahedron moments over one group of points.  Seen from the
      // tetrahedron [p]' = -[p], [u.n]' = [u.n]:
      //   F'_p = -taup w[p]/2 - w[u.n]/2,  F'_u = tauu w[u.n]/2 + w[p]/2
      if (mgr < CH) {
        D m0 = 0, m1 = 0;
        const int q0 = mgr * QC, q1 = q0 + QC < NQ1 ? q0 + QC : NQ1;
        for (int q = q0; q < q1; ++q) {
          const D rr = sRS[q * 2 + 0], ss = sRS[q * 2 + 1];
          D pa0 = 1.0, pa1 = rr, pb0 = 1.0, pb1 = ss;
          D Pa = maa == 0 ? 1.0 : rr, Pb = mbb == 0 ? 1.0 : ss;
#pragma unroll
          for (int n = 1; n < N; ++n) {
            const D na = ((2 * n + 1) * rr * pa1 - n * pa0) * (1.0 / (n + 1));
            const D nb = ((2 * n + 1) * ss * pb1 - n * pb0) * (1.0 / (n + 1));
            pa0 = pa1;
            pa1 = na;
            pb0 = pb1;
            pb1 = nb;
            Pa = maa == n + 1 ? na : Pa;
            Pb = mbb == n + 1 ? nb : Pb;
          }
          const D ph = Pa * Pb;
          const D jp = sJ[q * 2 + 0], jn = sJ[q * 2 + 1];
          m0 += ph * (-taup * jp - jn);
          m1 += ph * (tauu * jn + jp);
        }
        sRed[(mgr * 2 + 0) * NT + mmd] = m0;
        sRed[(mgr * 2 + 1) * NT + mmd] = m1;
      }
      // 2b. wedge sums over the t points of each edge point:
      //   F_p = taup w[p]/2 - w[u.n]/2,  F_u = tauu w[u.n]/2 - w[p]/2
      for (int o = tid; o < 2 * NX * Nq; o += 64) {
        const int f = o / (NX * Nq), rem = o - f * NX * Nq, a = rem / Nq, m = rem - a * Nq;
        D acc = 0;
#pragma unroll
        for (int g = 0; g < Nq; ++g) {
          const int q = a * Nq + g;
          const D jp = sJ[q * 2 + 0], jn = sJ[q * 2 + 1];
          const D F = f == 0 ? taup * jp - jn : tauu * jn - jp;
          acc += F * sLT[q * Nq + m];
        }
        sH[o] = acc;
      }
      __syncthreads();
      // 3a. wedge pre-lift contributions [field][level m][node i], both sides summed
#pragma unroll
      for (int r = 0; r < NBL; ++r) {
        const int o = tid + 64 * r;
        const int f = o / (Nq * NTP), rem = o - f * Nq * NTP, m = rem / NTP, i = rem - m * NTP;
        if (o < NB && i < NT) {
          CD* Ae = tab + TB::A + e * NX * NT + i;
          const D* Hf = sH + f * NX * Nq + m;
          D acc = 0;
#pragma unroll 4
          for (int a = 0; a < NX; ++a) acc += Ae[a * NT] * Hf[a * Nq];
          accB[r] += acc;
        }
      }
      // 3b. equivalent nodal flux of this side's tetrahedron face
      if (tid < 2 * NT) {
        const int f = tid / NT, i = tid - f * NT;
        D acc = 0;
        for (int md = 0; md < NT; ++md) {
          D mm = 0;
#pragma unroll
          for (int c = 0; c < CH; ++c) mm += sRed[(c * 2 + f) * NT + md];
          acc += tab[TB::P + i * NT + md] * mm;
        }
        static_cast<T*>(A.mortF)[(mo * 2 + side) * 2 * NT + tid] = T(acc * mg[25 + side]);
      }
    }
    // levels resolved by (M^1D)^-1
#pragma unroll
    for (int r = 0; r < NBL; ++r) {
      const int o = tid + 64 * r;
      if (o < NB) sB[o] = accB[r];
    }
    __syncthreads();
    T* outB = static_cast<T*>(A.mortB) + mo * NB;
#pragma unroll
    for (int r = 0; r < NBL; ++r) {
      const int o = tid + 64 * r;
      const int f = o / (Nq * NTP), rem = o - f * Nq * NTP, j = rem / NTP, i = rem - j * NTP;
      if (o < NB) {
        D acc = 0;
#pragma unroll
        for (int m = 0; m < Nq; ++m) acc += tab[TB::MI1 + j * Nq + m] * sB[f * Nq * NTP + m * NTP + i];
        outB[o] = T(acc);
      }
    }
  }
}

template <int N, typename T>
hipError_t launch_mortar_stage_t(const StageLaunch& a, hipStream_t st) {
  if (a.nmort <= 0) return hipSuccess;
  const unsigned grid = unsigned(a.nmort < 8192 ? a.nmort : 8192);
  hipLaunchKernelGGL((mortar_kernel<N, T>), dim3(grid), dim3(64), 0, st, a);
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

int mortar_table_size(int N, int bits) {
  switch (N) {
    case 1: return bits == 32 ? MortTab<1, 32>::SIZE : MortTab<1, 64>::SIZE;
    case 2: return bits == 32 ? MortTab<2, 32>::SIZE : MortTab<2, 64>::SIZE;
    case 3: return bits == 32 ? MortTab<3, 32>::SIZE : MortTab<3, 64>::SIZE;
    case 4: return bits == 32 ? MortTab<4, 32>::SIZE : MortTab<4, 64>::SIZE;
    case 5: return bits == 32 ? MortTab<5, 32>::SIZE : MortTab<5, 64>::SIZE;
    default: return 0;
  }
}

}  // namespace wdg
