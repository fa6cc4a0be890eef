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
// times Nq Gauss points in t on each side of the diagonal (exact in t).  One
// wavefront per mortar (persistent over mortars):
//   A. per point: wedge trace (GLL tensor interpolation of the face nodes),
//      tetrahedron trace (Lagrange basis of the tetrahedron face at the
//      point's barycentrics), upwind / central flux seen from both sides
//   B. wedge: pre-lift contributions (M^tri)^-1 int l_i l_j F, resolved into
//      the GLL levels by (M^1D)^-1, added by the wedge kernel before L^{tri,k};
//      tetrahedra: face moments int l_i F', returned as the equivalent nodal
//      face flux (M^tri)^-1 moments / (area/2) that the tetrahedron kernel lifts
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
// FP64 as well.
template <int N, typename T>
__global__ void __launch_bounds__(64) mortar_kernel(StageLaunch A) {
  using TB = MortTab<N, int(sizeof(T)) * 8>;
  using D = double;
  constexpr int NT = TB::NT, Nq = TB::Nq, NX = TB::NX;
  constexpr int NPW = Dim<N>::NP, NPT = TDim<N>::NP;
  constexpr int NQ1 = NX * Nq;  // points on one side of the diagonal
  constexpr int PPL = (NQ1 + 63) / 64;  // points per lane
  constexpr int NTP = (NT + 3) / 4 * 4;
  constexpr int NB = 2 * Nq * NTP;       // wedge outputs per mortar
  constexpr int NBL = (NB + 63) / 64;    // ... per lane
  __shared__ D tab[TB::SIZE];
  __shared__ V4<T> sW[Nq * Nq];   // wedge face nodes [level][edge node]
  __shared__ V4<T> sTF[2 * NT];   // tetrahedron face nodes [side][face node]
  __shared__ D sCT[3 * NT];       // modal coefficients of one side's tetrahedron trace (p, u_x, u_y)
  __shared__ D sC[NQ1 * 2];       // per point: w Fp, w Fu (wedge side)
  __shared__ D sG[NQ1 * Nq];      // per point: ((M^1D)^-1 l(t))_j
  __shared__ D sH[2 * NX * Nq];   // sums over the t points of one edge point: [field][a][j]
  __shared__ D sRed[64 * 2 * NT]; // per-lane partial modal moments of the tetrahedron side
  __shared__ D sMM[2 * NT];       // modal moments [field][mode]

  const D* __restrict__ gtab = static_cast<const D*>(A.mortTab);
  for (int idx = threadIdx.x; idx < TB::SIZE; idx += 64) tab[idx] = gtab[idx];
  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const D tau_on = (A.flags & kCentral) ? 0.0 : 1.0;
  const int tid = threadIdx.x;
  const int64_t tb = A.Kw * NPW;

  for (int64_t mo = blockIdx.x; mo < A.nmort; mo += gridDim.x) {
    const int* mi = A.mortI + mo * kMortIntStride;
    const D* mg = static_cast<const D*>(A.mortG) + mo * kMortGeoStride;
    const int64_t k = mi[0];
    const int e = mi[1], diag = mi[2];
    __syncthreads();  // tables loaded; the previous mortar is done with LDS
    // stage the wedge face nodes and both tetrahedron faces (one load per lane)
    for (int idx = tid; idx < Nq * Nq + 2 * NT; idx += 64) {
      if (idx < Nq * Nq) {
        const int lev = idx / Nq, q = idx - lev * Nq;
        sW[idx] = Uin[k * NPW + lev * NT + edge_node(N, e, q)];
      } else {
        const int r = idx - Nq * Nq, side = r / NT, i = r - side * NT;
        sTF[r] = Uin[tb + (int64_t(mi[3 + 2 * side]) - A.Kw) * NPT + tet_face_node<N>(mi[4 + 2 * side], i)];
      }
    }
    const D zba = mg[0], zbb = mg[1], zta = mg[2], ztb = mg[3], ell = mg[4], nx = mg[5], ny = mg[6];
    D accB[NBL];
#pragma unroll
    for (int r = 0; r < NBL; ++r) accB[r] = 0.0;

    for (int side = 0; side < 2; ++side) {
      __syncthreads();  // staged nodes ready; the previous side's data consumed
      if (tid < 3 * NT) {
        const int f = tid / NT, md = tid - f * NT;
        D acc = 0;
        for (int i = 0; i < NT; ++i) {
          const V4<T> v = sTF[side * NT + i];
          acc += tab[TB::VI + md * NT + i] * D(f == 0 ? v.p : (f == 1 ? v.ux : v.uy));
        }
        sCT[tid] = acc;
      }
      __syncthreads();
      // A. fluxes at the points of this side; partial modal moments per lane
      D pm[2 * NT];
#pragma unroll
      for (int md = 0; md < 2 * NT; ++md) pm[md] = 0.0;
#pragma unroll
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
        // GLL Lagrange basis in t (inverse denominators tabulated), then the wedge trace
        D lt[Nq];
#pragma unroll
        for (int m = 0; m < Nq; ++m) {
          D v = 1.0;
#pragma unroll
          for (int mm = 0; mm < Nq; ++mm)
            if (mm != m) v *= (t - tab[TB::TGLL + mm]) * tab[TB::DEN + m * Nq + mm];
          lt[m] = v;
        }
        D wp = 0, wx = 0, wy = 0;
#pragma unroll
        for (int qq = 0; qq < Nq; ++qq) {
          const D eq = tab[TB::E + a * Nq + qq];
#pragma unroll
          for (int m = 0; m < Nq; ++m) {
            const V4<T> v = sW[m * Nq + qq];
            const D c = eq * lt[m];
            wp += c * D(v.p);
            wx += c * D(v.ux);
            wy += c * D(v.uy);
          }
        }
#pragma unroll
        for (int j = 0; j < Nq; ++j) {
          D gj = 0;
#pragma unroll
          for (int m = 0; m < Nq; ++m) gj += tab[TB::MI1 + j * Nq + m] * lt[m];
          sG[q * Nq + j] = gj;
        }
        // tetrahedron face: barycentrics -> Legendre-product modes -> trace
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
        D phi[NT];
        D tp = 0, tx = 0, ty = 0;
        {
          int md = 0;
#pragma unroll
          for (int aa = 0; aa <= N; ++aa)
#pragma unroll
            for (int bb = 0; bb + aa <= N; ++bb) {
              const D ph = Pr[aa] * Ps[bb];
              phi[md] = ph;
              tp += ph * sCT[md];
              tx += ph * sCT[NT + md];
              ty += ph * sCT[2 * NT + md];
              ++md;
            }
        }
        const D zs = mg[27 + side];
        const D taup = tau_on * 2.0 / zs, tauu = tau_on * zs * 0.5;
        const D jp = tp - wp;
        const D jun = nx * (tx - wx) + ny * (ty - wy);
        sC[q * 2 + 0] = w * 0.5 * (taup * jp - jun);
        sC[q * 2 + 1] = w * 0.5 * (tauu * jun - jp);
        // seen from the tetrahedron: [p]' = -[p], [u.n]' = [u.n]
        const D fp = w * 0.5 * (-taup * jp - jun), fu = w * 0.5 * (tauu * jun + jp);
#pragma unroll
        for (int md = 0; md < NT; ++md) {
          pm[md] += fp * phi[md];
          pm[NT + md] += fu * phi[md];
        }
      }
#pragma unroll
      for (int md = 0; md < 2 * NT; ++md) sRed[md * 64 + tid] = pm[md];
      __syncthreads();
      // B. H_f[a][j] = sum over the t points of edge point a; reduce the modal moments
      for (int o = tid; o < 2 * NX * Nq; o += 64) {
        const int f = o / (NX * Nq), rem = o - f * NX * Nq, a = rem / Nq, j = rem - a * Nq;
        D acc = 0;
#pragma unroll
        for (int g = 0; g < Nq; ++g) acc += sC[(a * Nq + g) * 2 + f] * sG[(a * Nq + g) * Nq + j];
        sH[o] = acc;
      }
      if (tid < 2 * NT) {
        D acc = 0;
        for (int l = 0; l < 64; ++l) acc += sRed[tid * 64 + l];
        sMM[tid] = acc;
      }
      __syncthreads();
      // wedge pre-lift contributions [field][level j][node i], summed over both sides
#pragma unroll
      for (int r = 0; r < NBL; ++r) {
        const int o = tid + 64 * r;
        const int f = o / (Nq * NTP), rem = o - f * Nq * NTP, j = rem / NTP, i = rem - j * NTP;
        if (o < NB && i < NT) {
          const D* Ai = tab + TB::A + (e * NT + i) * NX;
          const D* Hf = sH + f * NX * Nq + j;
          D acc = 0;
#pragma unroll 4
          for (int a = 0; a < NX; ++a) acc += Ai[a] * Hf[a * Nq];
          accB[r] += acc;
        }
      }
      // equivalent nodal flux of this side's tetrahedron face: (M^tri)^-1 Vinv^T mm / (area/2)
      if (tid < 2 * NT) {
        const int f = tid / NT, i = tid - f * NT;
        D acc = 0;
        for (int md = 0; md < NT; ++md) acc += tab[TB::P + i * NT + md] * sMM[f * NT + md];
        static_cast<T*>(A.mortF)[(mo * 2 + side) * 2 * NT + tid] = T(acc * mg[25 + side]);
      }
    }
    T* outB = static_cast<T*>(A.mortB) + mo * NB;
#pragma unroll
    for (int r = 0; r < NBL; ++r) {
      const int o = tid + 64 * r;
      if (o < NB) outB[o] = T(accB[r]);
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
