// Fused wedge stage kernel of libwdg for CDNA4 (gfx950): volume term,
// surface fluxes and lifts, L^{tri,k} application and the low-storage
// Runge-Kutta update of one stage (Sec. 4.2-4.3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "device_common.hpp"
#include "ref_tables.inc"

namespace wdg {
namespace {

// Launch shape: one wavefront per block, lane = (element, level j), so a block
// holds EPB = 64 / Nq elements (fewer where the LDS would exceed 64 KiB).  LDS
// holds the staged state (per-element stride NPP, odd in 4-vectors, so that the
// elements of a wavefront fall on different banks) and a second region that
// first holds the inverse triangular masses, geometry records and triangular-face
// fluxes, and afterwards the right-hand side on its way to the coalesced
// update.
template <int N, typename T>
struct Cfg {
  static constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  static constexpr int NPP = NP | 1;
  // N <= 3: the element's triangular mass M^{tri,k} = sum_v w_v M_v is factored
  // (Cholesky) in the block from the vertex weights of the geometry record
  // instead of reading a stored inverse
  static constexpr bool CHOL = Dim<N>::PACKED;
  static constexpr int VL = Dim<N>::LS / 4, VG = kGeoStride / 4, VF = NT;  // 4-vectors per element
  static constexpr int XPE = (VL + VG + VF) > NPP ? (VL + VG + VF) : NPP;
  static constexpr int per_elem = (NPP + XPE) * 4 * int(sizeof(T));
  static constexpr int EPB_FULL = 64 / Nq;
  static constexpr int EPB_LDS = EPB_FULL * per_elem <= 65536 ? EPB_FULL : 65536 / per_elem;
  // Kernels that run one wavefront per SIMD (N >= 4; N = 3 in FP64, by its
  // registers) keep all four SIMDs of a CU busy only if four blocks fit in the
  // 160 KiB of LDS: at most 40 KiB per block (N = 5 FP32: 10 -> 9 elements,
  // 740 -> 620 us per stage on 73 728 wedges; N = 3 FP64: 16 -> 15, 497 -> 459 us
  // on 262 144 wedges).  With two wavefronts per SIMD (N <= 3, FP32) the same rule cost
  // 2 % at N = 3, so there the block keeps 64 / Nq elements.
  static constexpr bool ONE_WAVE = N >= 4 || (N == 3 && sizeof(T) == 8);
  static constexpr int EPB_CAP = ONE_WAVE ? 40960 / per_elem : 64;
  static constexpr int EPB = EPB_LDS < EPB_CAP ? EPB_LDS : EPB_CAP;
  static constexpr int BS = 64;
  // 4-vectors of the chunk each lane carries through the coalesced update
  static constexpr int UPD = (EPB * NP + BS - 1) / BS;
  // Prefetch the previous residual into registers when that costs at most 40
  // of them, or 80 for the one-wavefront-per-SIMD kernels, which have 512
  // (per stage: N = 4 on 73 728 wedges 145 -> 131 us, N = 5 621 -> 581 us,
  // N = 3 FP64 on 262 144 wedges 460 -> 387 us)
#ifndef WDG_PREFETCH_REGS
#define WDG_PREFETCH_REGS 40
#endif
#ifndef WDG_PREFETCH_REGS_ONE_WAVE
#define WDG_PREFETCH_REGS_ONE_WAVE 80
#endif
  static constexpr bool PREFETCH =
      UPD * 4 * int(sizeof(T)) / 4 <= (ONE_WAVE ? WDG_PREFETCH_REGS_ONE_WAVE : WDG_PREFETCH_REGS);
};

// acc1 += c x1; acc2 += c x2 for a reference-operator entry c known at
// compile time; exact zeros of the operator cost nothing
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

// The same selection where it is needed late in a kernel: the compiler turns
// the selection above into one load at a selected address in global memory,
// which is harmless next to the chunk's first loads but, issued late, comes
// with a wait for every load still in flight.  Here the entry is the sum of the
// entries times 0/1 masks of the lane's level (exact: one term is non-zero),
// the masks hidden from the compiler by an empty asm statement, so that every
// entry is read at a constant address (a scalar load).
template <int Nq, typename T>
struct LevelMask {
  T m[Nq];
  __device__ __forceinline__ explicit LevelMask(int j) {
#pragma unroll
    for (int jj = 0; jj < Nq; ++jj) {
      m[jj] = j == jj ? T(1) : T(0);
      asm volatile("" : "+v"(m[jj]));
    }
  }
  __device__ __forceinline__ T pick(const double* tab, int stride, int col) const {
    T v = T(0);
#pragma unroll
    for (int jj = 0; jj < Nq; ++jj) v += m[jj] * T(tab[jj * stride + col]);
    return v;
  }
};


// A wedge's accumulators across the reverse sweep: FP64 sums; FP32 Kahan
// (compensated) sums, the record holding the sums, then their compensations.
// Read early (grad_record_load), then one stage's terms x[kGradStride] added
// and written back (grad_record_add).
template <typename T>
struct GradRecord {
  T v[kGradRecord<T>];
};
template <typename T>
__device__ __forceinline__ void grad_record_load(const void* gacc, int64_t e, GradRecord<T>& r) {
  const T* ga = static_cast<const T*>(gacc) + e * kGradRecord<T>;
#pragma unroll
  for (int k = 0; k < kGradRecord<T>; ++k) r.v[k] = ga[k];
}
template <typename T>
__device__ __forceinline__ void grad_record_add(void* gacc, int64_t e, const GradRecord<T>& r, const T* x) {
  T* ga = static_cast<T*>(gacc) + e * kGradRecord<T>;
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int k = 0; k < kGradStride; ++k) ga[k] = r.v[k] + x[k];
  } else {
#pragma unroll
    for (int k = 0; k < kGradStride; ++k) {
      const T y = x[k] - r.v[kGradStride + k];
      const T t = r.v[k] + y;
      ga[kGradStride + k] = (t - r.v[k]) - y;
      ga[k] = t;
    }
  }
}

// Gradient terms of one reverse stage of the adjoint sweep (MODE 4), run by
// the stage kernel after its update.  The stage input (the adjoint stage
// vector sig) is still staged in sU and the incoming adjoint state U~ in the
// second region; the forward residual res_s after stage s, then the forward
// stage input Us, are staged into them as they free up.  Per wedge it
// accumulates the mass terms b_s U~_p^T M res_p, b_s U~_u^T M res_u (their sum
// over a step's stages is that of dt sig_p^T M R_p, dt sig_u^T M R_u with R_s
// the stage's right-hand side; as dJ/dc = 2/(c kappa) m_p, dJ/drho =
// m_p/(rho kappa) + m_u) and per face dt times the face integrals 1/2 int
// sig_p [p], 1/2 int sig_un [u_n] of Us weighted by the penalties'
// derivatives (gacc slots 2..6), which the combine kernel adds up over both
// sides of every face.  M^k = (sum_v w_v M_v) (x) M^1D and the face masses
// are literals (reference triangle, 1D, edge masses).
// FP32 up to N = 3 the gradient epilogue takes the element's connectivity
// and geometry from the stage's registers and issues its gathers first and its
// chunk loads before its first barrier: reloading them from memory after the
// update's stores would wait for the stores.  Beyond, the extra live registers
// spill, and it reads them from memory where they are used.
template <int N, typename T>
constexpr bool grad_early() {
  return sizeof(T) == 4 && N <= 3;
}
// the geometry the epilogue uses, copied out of the stage's LDS before the
// right-hand side overwrites it: the lane's triangular face (bottom for level
// 0, else top), the three quadrilateral faces, kappa, 1/rho, the vertex weights
template <typename T>
struct EpiGeo {
  T tJf, tnx, tny, tnz, kap, irho, w0, w1, w2;
  T qg[3][4];
};

// the epilogue's global loads: the quadrilateral-face neighbour nodes of Us
// on this level, the chunk's Us (a) and forward residual (b), coalesced
template <int N, typename T>
struct EpiLoads {
  static constexpr int SU = (Cfg<N, T>::EPB * Cfg<N, T>::NP + 63) / 64;
  V4<T> gq[3][Cfg<N, T>::Nq];
  V4<T> a[SU], b[SU];
};
template <int N, typename T>
__device__ __forceinline__ void grad_load_q(const StageLaunch& A, int j, int64_t e, const int* cv, EpiLoads<N, T>& L) {
  constexpr int NT = Cfg<N, T>::NT, Nq = Cfg<N, T>::Nq, NP = Cfg<N, T>::NP;
  const V4<T>* __restrict__ Us = static_cast<const V4<T>*>(A.gUs);
  const int code = cv[5];
#pragma unroll
  for (int ed = 0; ed < 3; ++ed) {
    const int nbr = cv[2 + ed];
    const int ned = (code >> (8 + 2 * ed)) & 3;
    const V4<T>* nb_el = Us + (nbr >= 0 ? int64_t(nbr) : e) * NP + j * NT;
#pragma unroll
    for (int q = 0; q < Nq; ++q) {
      const int ni = ned == 0 ? edge_node(N, 0, N - q) : (ned == 1 ? edge_node(N, 1, N - q) : edge_node(N, 2, N - q));
      L.gq[ed][q] = nb_el[ni];
    }
  }
}
template <int N, typename T>
__device__ __forceinline__ void grad_load_chunk(const void* src, int64_t e0, int nE, int tid, V4<T>* out) {
  constexpr int NP = Cfg<N, T>::NP, V4B = 4 * int(sizeof(T));
  const auto br = chunk_rsrc(static_cast<const V4<T>*>(src) + e0 * NP, int64_t(nE) * NP * V4B);
#pragma unroll
  for (int k = 0; k < EpiLoads<N, T>::SU; ++k) out[k] = bload<T>(br, tid + 64 * k);
}

template <int N, typename T>
__device__ __forceinline__ void grad_epilogue(const StageLaunch& A, int64_t e0, int nE, int tid, int le, int j,
                                              bool active, int64_t e, V4<T>* sU, V4<T>* sX, const int* cn,
                                              const EpiGeo<T>& eg) {
  using C = Cfg<N, T>;
  using RT = gen::RefTables<N>;
  constexpr int NT = C::NT, Nq = C::Nq, NP = C::NP, NPP = C::NPP, EPB = C::EPB;
  constexpr int SU = EpiLoads<N, T>::SU;
  constexpr int GS = kGradTerms + 1;  // partial sums per lane (odd: fewer bank conflicts)
  static_assert(EPB * 3 * Nq * Nq * 2 <= EPB * NPP * 4, "jump scratch fits the state region");
  static_assert(EPB * Nq * GS <= EPB * C::XPE * 4, "partial sums fit the second region");
  const bool lane_ok = le < EPB;
  const T bsign = (A.flags & kDirichlet) ? T(-1) : T(1);
  const int lb = (lane_ok ? le : 0) * NPP + j * NT;
  const V4<T>* __restrict__ Us = static_cast<const V4<T>*>(A.gUs);
  constexpr bool early = grad_early<N, T>();
  const int* __restrict__ gcn = A.conn + e * kConnStride;
  const T* __restrict__ gm = static_cast<const T*>(A.geo) + e * kGeoStride;
  int cv[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) cv[k] = early ? cn[k] : gcn[k];
  const int code = cv[5];
  // the quadrilateral-face gathers first; FP32 up to N = 3 the chunk loads
  // too, before the first barrier (beyond, holding them across it spills).
  // Issuing them before the update's stores instead, so that waiting for them
  // would not wait for the stores, measured slower (522 against 492 us per
  // stage on 524 288 wedges)
  EpiLoads<N, T> L;
  grad_load_q<N, T>(A, j, e, cv, L);
  if constexpr (early) {
    grad_load_chunk<N, T>(A.gUs, e0, nE, tid, L.a);
    grad_load_chunk<N, T>(A.gRs, e0, nE, tid, L.b);
  }
  auto slot = [&](int k) {
    const int idx = tid + 64 * k;
    return idx < EPB * NP ? idx + (idx / NP) * (NPP - NP) : EPB * NPP;
  };
  V4<T> sg[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) sg[i] = sU[lb + i];
  __syncthreads();  // the update and the reads of sig are done
  if constexpr (!early) grad_load_chunk<N, T>(A.gRs, e0, nE, tid, L.b);
#pragma unroll
  for (int k = 0; k < SU; ++k) sU[slot(k)] = L.b[k];  // res_s over sig
  __syncthreads();
  T part[kGradTerms];
#pragma unroll
  for (int k = 0; k < kGradTerms; ++k) part[k] = T(0);

  // Mass terms.  The stage's right-hand side R_s enters as sig_s^T M R_s; with
  // dt R_s = res_s - a_s res_{s-1} (a_1 = 0) the sum over a step's stages equals
  // the sum of (sig_s - a_{s+1} sig_{s+1})^T M res_s / dt, and the reverse sweep
  // has sig_s - a_{s+1} sig_{s+1} = b_s U~, U~ the adjoint state this stage
  // reads (left in the second LDS region by the update).  So the forward
  // keeps its residuals instead of writing every right-hand side.
  // On this level: U~^T (M^{tri,k} (x) M^1D) res_s, M^{tri,k} = sum_v w_v M_v.
  T m1[Nq];
  {
    const LevelMask<Nq, T> lm(j);
#pragma unroll
    for (int m = 0; m < Nq; ++m) m1[m] = lm.pick(RT::M1, Nq, m);
  }
  if (lane_ok) {
    const V4<T>* sRs = sU;
    const V4<T>* sUa = sX;
    const T w0 = early ? eg.w0 : gm[37], w1 = early ? eg.w1 : gm[38], w2 = early ? eg.w2 : gm[39];
    T y[4][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        const V4<T> r = sRs[le * NPP + m * NT + i];
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
      const V4<T> ua = sUa[lb + i];
      mp += ua.p * z0;
      mu += ua.ux * z1 + ua.uy * z2 + ua.uz * z3;
    }
    part[0] = mp;
    part[1] = mu;
  }
  if constexpr (!early) grad_load_chunk<N, T>(A.gUs, e0, nE, tid, L.a);
  __syncthreads();  // U~ and res_s in LDS are consumed
#pragma unroll
  for (int k = 0; k < SU; ++k) sX[slot(k)] = L.a[k];  // Us
  __syncthreads();
  const V4<T>* sUs = sX;

  // triangular faces: lane 0 the bottom, lane N the top (own level).  The
  // neighbour's face nodes are gathered here, unconditionally (the other
  // lanes, and boundary faces, read the own element: a valid address), and
  // used after the quadrilateral faces, which need no memory
  const bool tri = lane_ok && (j == 0 || j == N);
  const int face = j == 0 ? 0 : 1;
  const int tnbr = face ? cv[1] : cv[0];
  const bool inner = tnbr >= 0;
  const int pc = (code >> (3 * face)) & 7;
  const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
  const int64_t src = (tri && inner) ? int64_t(tnbr) : e;
  V4<T> vn[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) vn[i] = Us[src * NP + nlev * NT + face_perm<N>(pc, i)];

  // quadrilateral faces: jumps of this level (to LDS below); the adjoint
  // trace times the edge mass stays in registers
  T jq[3][Nq][2], ap[3][Nq], an[3][Nq];
#pragma unroll
  for (int ed = 0; ed < 3; ++ed) {
    const int nbr = cv[2 + ed];
    const T Ja = early ? eg.qg[ed][0] : gm[20 + 4 * ed], Jb = early ? eg.qg[ed][1] : gm[21 + 4 * ed];
    const T nx = early ? eg.qg[ed][2] : gm[22 + 4 * ed], ny = early ? eg.qg[ed][3] : gm[23 + 4 * ed];
    T sp[Nq], sn[Nq];
#pragma unroll
    for (int q = 0; q < Nq; ++q) {
      const int i = edge_node(N, ed, q);
      const V4<T> own = sUs[lb + i];
      const T pm = own.p, unm = nx * own.ux + ny * own.uy;
      T pp = bsign * pm, unp = -bsign * unm;
      if (nbr >= 0) {
        pp = L.gq[ed][q].p;
        unp = nx * L.gq[ed][q].ux + ny * L.gq[ed][q].uy;
      }
      jq[ed][q][0] = pp - pm;
      jq[ed][q][1] = unp - unm;
      sp[q] = sg[i].p;
      sn[q] = nx * sg[i].ux + ny * sg[i].uy;
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

  if (tri) {
    const T Jf = early ? eg.tJf : gm[12 + 4 * face], nx = early ? eg.tnx : gm[13 + 4 * face];
    const T ny = early ? eg.tny : gm[14 + 4 * face], nz = early ? eg.tnz : gm[15 + 4 * face];
    T jp[NT], jn[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const V4<T> own = sUs[lb + i];
      const T pm = own.p, unm = nx * own.ux + ny * own.uy + nz * own.uz;
      const T pp = inner ? vn[i].p : bsign * pm;  // else the mirror state
      const T unp = inner ? nx * vn[i].ux + ny * vn[i].uy + nz * vn[i].uz : -bsign * unm;
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
      sp += sg[i].p * mp;
      sn += (nx * sg[i].ux + ny * sg[i].uy + nz * sg[i].uz) * mn;
    }
    part[2 + face] = T(0.5) * Jf * sp;
    part[7 + face] = T(0.5) * Jf * sn;
  }

  // the wedge's accumulator record, read before the level coupling below
  // (idle lanes read the wedge they shadow)
  GradRecord<T> rec;
  grad_record_load<T>(A.gacc, e, rec);
  T zsum[5];  // Z- + Z+ per face
#pragma unroll
  for (int f = 0; f < 5; ++f) zsum[f] = gm[32 + f];
  __syncthreads();  // Us in LDS is consumed
  T* const sJ = reinterpret_cast<T*>(sU);  // quadrilateral-face jumps [wedge][edge][level][node][p, u_n]
  if (lane_ok) {
#pragma unroll
    for (int ed = 0; ed < 3; ++ed)
#pragma unroll
      for (int q = 0; q < Nq; ++q) {
        T* sj = sJ + (((le * 3 + ed) * Nq + j) * Nq + q) * 2;
        sj[0] = jq[ed][q][0];
        sj[1] = jq[ed][q][1];
      }
  }
  __syncthreads();
  T* const sPart = reinterpret_cast<T*>(sX);
  if (lane_ok) {
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
      part[4 + ed] = T(0.5) * sp;
      part[9 + ed] = T(0.5) * sn;
    }
#pragma unroll
    for (int k = 0; k < kGradTerms; ++k) sPart[(le * Nq + j) * GS + k] = part[k];
  }
  __syncthreads();
  if (active && j == 0) {
    T tot[kGradTerms];
#pragma unroll
    for (int k = 0; k < kGradTerms; ++k) {
      T s = 0;
#pragma unroll
      for (int l = 0; l < Nq; ++l) s += sPart[(le * Nq + l) * GS + k];
      tot[k] = s;
    }
    const T kap = early ? eg.kap : gm[9], irho = early ? eg.irho : gm[10];
    const T c = std::sqrt(kap * irho);
    const T dt = T(A.dt);
    T x[kGradStride];
    const T gb = T(A.gb);  // dt times the mass terms' factor b_s / dt
    x[0] = gb * T(2) / (c * kap) * tot[0];
    x[1] = gb * (tot[0] * irho / kap + tot[1]);
    // per face dtau_p/dZ = -tau_p^2 / 2, dtau_u/dZ = 1/2 (upwind, tau_p = 2 / (Z- + Z+);
    // the central flux has no penalties)
    const bool upwind = !(A.flags & kCentral);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const T tp = T(2) / zsum[f];
      x[2 + f] = upwind ? dt * (-T(0.5) * tp * tp * tot[2 + f] - T(0.5) * tot[7 + f]) : T(0);
    }
    grad_record_add<T>(A.gacc, e, rec, x);
  }
}

// ---------------------------------------------------------------------------
// Fused stage kernel
//
// Lane (element, level j) owns the triangular slice j of its element for all
// four equations.  The reference triangle and 1D operators are compile-time
// constants (instruction literals).  The chunk's state, lifts, geometry and
// connectivity are staged in LDS with coalesced loads; the vertical derivative
// and the triangle-face lifts couple the levels of one element through it.
//   phase 1: B = -W (vertical part of D_x, D_y, D_z, before L^{tri,k}) plus the
//            quadrilateral-face lifts of this level; triangular-face fluxes
//   phase 2: B += triangular-face lifts; R = L^{tri,k} B + H (horizontal part);
//            scale by kappa, 1/rho; sources
//   update:  R goes through LDS so that the low-storage Runge-Kutta update
//            reads and writes res and U with fully coalesced accesses
// highest order whose quadrilateral-face fluxes are added after M^tri (edge masses)
#ifndef WDG_QM_MAX_N
#define WDG_QM_MAX_N 4
#endif
#ifndef WDG_STAGE_WAVES_PER_EU
#define WDG_STAGE_WAVES_PER_EU 2
#endif
// MODE 0: wedges only; 1: tetrahedra across triangular faces; 2: also mortars;
// 3: wedges only, vertical neighbours inside the chunk read from LDS (layer marching);
// 4: wedges only, adjoint stage with its gradient terms (grad_epilogue);
// 5: as 3 for one chunk of a column marched from the bottom (wedge_column_stage):
//    the wedge below the chunk's first one is the previous chunk's last, whose
//    top level the previous call left in carry (when has_carry); this call
//    leaves its own last wedge's top level there.
// The chunk holds wedges e0 .. e0 + nE - 1 (nE <= EPB).
template <int N, typename T, int MODE>
__device__ __forceinline__ void wedge_stage_chunk(const StageLaunch& A, int64_t e0, int nE, V4<T>* carry = nullptr,
                                                  bool has_carry = false) {
  constexpr bool HYB = MODE == 1 || MODE == 2;
  constexpr bool MARCH = MODE == 3 || MODE == 5;
  using C = Cfg<N, T>;
  using RT = gen::RefTables<N>;
  constexpr int NT = C::NT, Nq = C::Nq, NP = C::NP, NPP = C::NPP, EPB = C::EPB;
  constexpr int VL = C::VL, VG = C::VG;
  // one spare 4-vector at the end of each array takes the stores of lanes
  // past the end of a staged stream
  __shared__ V4<T> sU[EPB * NPP + 1];
  __shared__ V4<T> sX[EPB * C::XPE + 1];
  V4<T>* const sL = sX;
  V4<T>* const sG = sX + EPB * VL;
  T* const sF = reinterpret_cast<T*>(sG + EPB * VG);
  V4<T>* const sR = sX;

  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const T* __restrict__ geo = static_cast<const T*>(A.geo);
  const T* __restrict__ Lm = static_cast<const T*>(A.L);
  const int* __restrict__ conn = A.conn;

  int tid = threadIdx.x;
  // marching a column, each chunk derives its lane constants anew: hoisted
  // out of the column loop they would stay live across chunks and spill
  if constexpr (MODE == 5) asm volatile("" : "+v"(tid));

  const int le = tid / Nq;
  const int j = tid - le * Nq;
  const bool active = tid < EPB * Nq && le < nE;
  const int64_t e = e0 + (active ? le : 0);  // idle lanes shadow a valid element
  const T bsign = (A.flags & kDirichlet) ? T(-1) : T(1);
  const T tau_on = (A.flags & kCentral) ? T(0) : T(1);
  constexpr int per = (2 * NT + Nq - 1) / Nq;  // triangular-face nodes per lane

  // The lane's own connectivity is read first and the neighbour gathers are
  // issued as soon as it arrives, while the chunk's coalesced staging loads
  // are still in flight: both memory latencies overlap.
  int cn[6];
  {
    const int4* cp = reinterpret_cast<const int4*>(conn + e * kConnStride);
    const int4 c0 = cp[0], c1 = cp[1];
    cn[0] = c0.x;
    cn[1] = c0.y;
    cn[2] = c0.z;
    cn[3] = c0.w;
    cn[4] = c1.x;
    cn[5] = c1.y;
  }
  constexpr int SU = (EPB * NP + 63) / 64, SL = C::CHOL ? 0 : (EPB * VL + 63) / 64, SG = (EPB * VG + 63) / 64;
  constexpr int V4B = 4 * int(sizeof(T));
  V4<T> rU[SU], rL[SL > 0 ? SL : 1], rG[SG];
  {
    const auto bu = chunk_rsrc(Uin + e0 * NP, int64_t(nE) * NP * V4B);
    const auto bl = chunk_rsrc(Lm + e0 * Dim<N>::LS, int64_t(nE) * VL * V4B);
    const auto bg = chunk_rsrc(geo + e0 * kGeoStride, int64_t(nE) * VG * V4B);
#pragma unroll
    for (int k = 0; k < SU; ++k) rU[k] = bload<T>(bu, tid + 64 * k);
#pragma unroll
    for (int k = 0; k < SL; ++k) rL[k] = bload<T>(bl, tid + 64 * k);
#pragma unroll
    for (int k = 0; k < SG; ++k) rG[k] = bload<T>(bg, tid + 64 * k);
  }
  const int code = cn[5];
  // quadrilateral-face neighbour nodes on this level (boundary faces read the
  // own element, a valid address; the mirror state is blended in later)
  V4<T> gq[3][Nq];
#pragma unroll
  for (int ed = 0; ed < 3; ++ed) {
    const int nbr = cn[2 + ed];
    const int ned = (code >> (8 + 2 * ed)) & 3;
    const V4<T>* nb_el = Uin + (nbr >= 0 ? int64_t(nbr) : e) * NP + j * NT;
#pragma unroll
    for (int q = 0; q < Nq; ++q) {
      const int ni = ned == 0 ? edge_node(N, 0, N - q) : (ned == 1 ? edge_node(N, 1, N - q) : edge_node(N, 2, N - q));
      gq[ed][q] = nb_el[ni];
    }
  }
  // triangular-face neighbour nodes: the 2 NT face nodes of the element are
  // shared out over its Nq lanes (surplus slots redo the last node)
  // Layer marching (MODE 3): a chunk is a run of consecutive layers of one
  // column, so the wedge below or above usually sits in the same chunk; its
  // face nodes are then read from the staged chunk after the barrier instead
  // of being gathered from memory.
  V4<T> gt[per];
#pragma unroll
  for (int t = 0; t < per; ++t) {
    const int fraw = j * per + t;
    const int fnode = fraw < 2 * NT ? fraw : 2 * NT - 1;
    const int face = fnode >= NT ? 1 : 0;
    const int i = fnode - face * NT;
    const int nbr = face ? cn[1] : cn[0];
    const int pc = (code >> (3 * face)) & 7;
    const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
    const int64_t src = nbr >= 0 ? int64_t(nbr) : e;
    const int fn = face_perm<N>(pc, i);
    if constexpr (HYB) {
      // a tetrahedron neighbour: its nodes follow all wedge nodes
      const int tf = (code >> (14 + 2 * face)) & 3;
      const bool tet = src >= A.Kw;
      gt[t] = Uin[tet ? A.Kw * NP + (src - A.Kw) * TDim<N>::NP + tet_face_node<N>(tf, fn) : src * NP + nlev * NT + fn];
    } else {
      const bool in_chunk = MARCH && nbr >= 0 && src >= e0 && src < e0 + nE;
      const bool carried = MODE == 5 && has_carry && nbr >= 0 && src == e0 - 1 && nlev == N;
      gt[t] = V4<T>{T(0), T(0), T(0), T(0)};
      if (!in_chunk && !carried) gt[t] = Uin[src * NP + nlev * NT + fn];
    }
  }
#pragma unroll
  for (int k = 0; k < SU; ++k) {
    const int idx = tid + 64 * k;
    sU[idx < EPB * NP ? idx + (idx / NP) * (NPP - NP) : EPB * NPP] = rU[k];
  }
#pragma unroll
  for (int k = 0; k < SL; ++k) {
    const int idx = tid + 64 * k;
    sX[idx < EPB * VL ? idx : EPB * C::XPE] = rL[k];
  }
#pragma unroll
  for (int k = 0; k < SG; ++k) {
    const int idx = tid + 64 * k;
    sX[idx < EPB * VG ? EPB * VL + idx : EPB * C::XPE] = rG[k];
  }
  __syncthreads();
  if constexpr (C::CHOL) {
    // M^{tri,k} = L L^T, row by row into the element's triangular-operator
    // slots (entry (i, m) at i (i + 1) / 2 + m, the diagonal holding 1 / L_ii);
    // read after the barrier that follows the triangular-face fluxes
    if (active && j == 0) {
      constexpr int NK = Dim<N>::NPK;
      const T* gw = reinterpret_cast<const T*>(sG) + le * kGeoStride;
      const T w0 = gw[37], w1 = gw[38], w2 = gw[39];
      T a[NK];
#pragma unroll
      for (int f = 0; f < NK; ++f) {
        const int i = tri_row(f), m = f - i * (i + 1) / 2;
        T v = 0;
        constexpr_or_skip(RT::Mv[i * NT + m], v, w0);
        constexpr_or_skip(RT::Mv[NT * NT + i * NT + m], v, w1);
        constexpr_or_skip(RT::Mv[2 * NT * NT + i * NT + m], v, w2);
        a[f] = v;
      }
#pragma unroll
      for (int f = 0; f < NK; ++f) {
        const int i = tri_row(f), m = f - i * (i + 1) / 2;
        T sm = a[f];
#pragma unroll
        for (int k = 0; k < m; ++k) sm -= a[i * (i + 1) / 2 + k] * a[m * (m + 1) / 2 + k];
        a[f] = m < i ? sm * a[m * (m + 1) / 2 + m] : T(1) / std::sqrt(sm);
      }
      T* lo = reinterpret_cast<T*>(sL + le * VL);
#pragma unroll
      for (int f = 0; f < NK; ++f) lo[f] = a[f];
    }
  }
  if constexpr (MARCH) {
#pragma unroll
    for (int t = 0; t < per; ++t) {
      const int fraw = j * per + t;
      const int fnode = fraw < 2 * NT ? fraw : 2 * NT - 1;
      const int face = fnode >= NT ? 1 : 0;
      const int nbr = face ? cn[1] : cn[0];
      const int64_t ln = int64_t(nbr) - e0;
      const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
      const int fn = face_perm<N>((code >> (3 * face)) & 7, fnode - face * NT);
      if (nbr >= 0 && ln >= 0 && ln < nE) {
        gt[t] = sU[int(ln) * NPP + nlev * NT + fn];
      } else if (MODE == 5 && has_carry && nbr >= 0 && ln == -1 && nlev == N) {
        gt[t] = carry[fn];
      }
    }
  }

  const V4<T>* el = sU + le * NPP;
  const T* g = reinterpret_cast<const T*>(sG) + le * kGeoStride;

  // pre-lift accumulators of the four equations on this level
  T Bp[NT], Bz[NT], Bx[NT], By[NT];
  // Quadrilateral-face fluxes: lifted by E_e (dense Np_tri x Nq) into the
  // pre-lift sums, or (QM) kept as (F_p, F_u) per edge node and added after the
  // reference mass M^tri is applied, where E_e becomes the Nq x Nq edge mass
  // on the edge's own nodes (M^tri E_e = int_edge l l_q (1 -+ xi) / 2).  QM
  // saves VALU work where the registers for the kept fluxes are free.
  constexpr bool QM = Dim<N>::PACKED && N <= WDG_QM_MAX_N;
  T qf[QM ? 3 : 1][QM ? Nq : 1][2];

  if (active) {
    const T tzJ = g[4];
    const LevelMask<Nq, T> lm(j);
    const T tj = lm.pick(RT::t, 1, 0);
    const T tl = T(0.5) * (T(1) - tj);
    const T th = T(0.5) * (T(1) + tj);
    const T txJ = g[5] * tl + g[6] * th;
    const T tyJ = g[7] * tl + g[8] * th;
    T dtr[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) dtr[m] = lm.pick(RT::Dt, Nq, m);

    // vertical part: W = t_dJ(t_j) (D_t U)(level j)
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      T dP = 0, dX = 0, dY = 0, dZ = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        const V4<T> v = el[m * NT + i];
        dP += dtr[m] * v.p;
        dX += dtr[m] * v.ux;
        dY += dtr[m] * v.uy;
        dZ += dtr[m] * v.uz;
      }
      T w = txJ * dX;
      w += tyJ * dY;
      w += tzJ * dZ;
      Bp[i] = -w;
      Bx[i] = -(txJ * dP);
      By[i] = -(tyJ * dP);
      Bz[i] = -(tzJ * dP);
    }

    // quadrilateral faces (normals horizontal, so they reach p, u_x, u_y only);
    // the mirror state of a boundary face is blended in without branches
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      const T w_in = cn[2 + ed] >= 0 ? T(1) : T(0);
      // a mortar face (-2 - m) takes its flux from the mortar kernel instead
      const T Ja = MODE == 2 && cn[2 + ed] <= -2 ? T(0) : g[20 + 4 * ed];
      const T Jb = MODE == 2 && cn[2 + ed] <= -2 ? T(0) : g[21 + 4 * ed];
      const T nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
      const T zs = g[34 + ed];  // Z- + Z+ (= 2 Z- on the boundary)
      const T taup = tau_on * T(2) / zs;
      const T tauu = tau_on * zs * T(0.5);
      T fpa[Nq], fpb[Nq], fua[Nq], fub[Nq];
#pragma unroll
      for (int q = 0; q < Nq; ++q) {
        const V4<T> own = el[j * NT + edge_node(N, ed, q)];
        const V4<T> v = gq[ed][q];
        const T pm = own.p;
        const T unm = nx * own.ux + ny * own.uy;
        // mirror state: p+ = s p-, u_n+ = -s u_n- (s = -1 Dirichlet, +1 rigid)
        const T pb = bsign * pm, ub = -bsign * unm;
        const T pp = pb + w_in * (v.p - pb);
        // (u_z enters with weight zero, which keeps the gather one 16-byte load)
        const T unp = ub + w_in * ((nx * v.ux + ny * v.uy + T(0) * v.uz) - ub);
        const T jp = pp - pm, jun = unp - unm;
        const T Fp = T(0.5) * (taup * jp - jun);
        const T Fu = T(0.5) * (tauu * jun - jp);
        if constexpr (QM) {
          qf[ed][q][0] = Fp;
          qf[ed][q][1] = Fu;
        } else {
          fpa[q] = Ja * Fp;
          fpb[q] = Jb * Fp;
          fua[q] = Ja * Fu;
          fub[q] = Jb * Fu;
        }
      }
      if constexpr (!QM) {
#pragma unroll
        for (int i = 0; i < NT; ++i) {
          T sp = 0, su = 0;
#pragma unroll
          for (int q = 0; q < Nq; ++q) {
            constexpr_or_skip(RT::Ea[(ed * NT + i) * Nq + q], sp, fpa[q]);
            constexpr_or_skip(RT::Eb[(ed * NT + i) * Nq + q], sp, fpb[q]);
            constexpr_or_skip(RT::Ea[(ed * NT + i) * Nq + q], su, fua[q]);
            constexpr_or_skip(RT::Eb[(ed * NT + i) * Nq + q], su, fub[q]);
          }
          Bp[i] += sp;
          Bx[i] += nx * su;
          By[i] += ny * su;
        }
      }
    }

    // triangular-face fluxes (premultiplied by J_f) go to LDS for every level
#pragma unroll
    for (int t = 0; t < per; ++t) {
      const int fraw = j * per + t;
      const int fnode = fraw < 2 * NT ? fraw : 2 * NT - 1;
      const int face = fnode >= NT ? 1 : 0;
      const int i = fnode - face * NT;
      const T w_in = (face ? cn[1] : cn[0]) >= 0 ? T(1) : T(0);
      const T* gf = g + 12 + 4 * face;
      const T Jf = gf[0], nx = gf[1], ny = gf[2], nz = gf[3];
      const T zs = g[32 + face];
      const T taup = tau_on * T(2) / zs;
      const T tauu = tau_on * zs * T(0.5);
      const V4<T> own = el[face * N * NT + i];
      const V4<T> v = gt[t];
      const T pm = own.p;
      const T unm = nx * own.ux + ny * own.uy + nz * own.uz;
      const T pb = bsign * pm, ub = -bsign * unm;
      const T pp = pb + w_in * (v.p - pb);
      const T unp = ub + w_in * ((nx * v.ux + ny * v.uy + nz * v.uz) - ub);
      const T jp = pp - pm, jun = unp - unm;
      if (fraw < 2 * NT) {
        T* f = sF + ((le * 2 + face) * NT + i) * 2;
        f[0] = Jf * T(0.5) * (taup * jp - jun);
        f[1] = Jf * T(0.5) * (tauu * jun - jp);
      }
    }
  }
  __syncthreads();

  const bool rd = (A.flags & kReadRes) != 0, wu = (A.flags & kWriteU) != 0;
  // residual of the previous stage, in the coalesced layout of the update.
  // The first stage reads none: its resource has an empty range, so the
  // loads return zeros without touching memory and need no branch.
  V4<T>* const res_chunk = static_cast<V4<T>*>(A.res) + e0 * NP;
  const auto bres_in = chunk_rsrc(res_chunk, rd ? int64_t(nE) * NP * V4B : 0);
  const auto bres = chunk_rsrc((A.flags & kResOut) ? static_cast<V4<T>*>(A.rout) + e0 * NP : res_chunk,
                               int64_t(nE) * NP * V4B);
  V4<T> rprev[C::PREFETCH ? C::UPD : 1];
  if constexpr (C::PREFETCH) {
#pragma unroll
    for (int k = 0; k < C::UPD; ++k) rprev[k] = bload<T>(bres_in, tid + 64 * k);
  }

  T Rp[NT], Rz[NT], Rx[NT], Ry[NT];
  if (active) {
    // triangular-face lifts: flux spread over all levels by (M^1D)^-1 e_{0,N}
    {
      // exact mass: (M^1D)^-1 e_{0,N}; lumped mass (Gauss-Lobatto weights w): e_{0,N} / w_{0,N}
      const T wend = T(0.5 * N * (N + 1));  // 1 / w_0 = 1 / w_N
      const bool lumped = (A.flags & kLumped) != 0;
      const LevelMask<Nq, T> lm(j);
      const T g0j = lumped ? (j == 0 ? wend : T(0)) : lm.pick(RT::g0, 1, 0);
      const T gNj = lumped ? (j == N ? wend : T(0)) : lm.pick(RT::gN, 1, 0);
      const T* fbt = sF + (le * 2 + 0) * NT * 2;
      const T* ftp = sF + (le * 2 + 1) * NT * 2;
      const T bx = g[13], by = g[14], bz = g[15], tx = g[17], ty = g[18], tz = g[19];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        Bp[i] += g0j * fbt[2 * i];
        Bp[i] += gNj * ftp[2 * i];
        const T wb = g0j * fbt[2 * i + 1], wt = gNj * ftp[2 * i + 1];
        Bx[i] += wb * bx;
        Bx[i] += wt * tx;
        By[i] += wb * by;
        By[i] += wt * ty;
        Bz[i] += wb * bz;
        Bz[i] += wt * tz;
      }
    }

    if constexpr (MODE == 2) {
      // mortar faces: pre-lift contributions of the common refinement; the
      // buffer's range check returns zeros for the other faces
      constexpr int NTP = (NT + 3) / 4 * 4;
      const auto rb = chunk_rsrc(A.mortB, A.nmort * 2 * Nq * NTP * int64_t(sizeof(T)));
#pragma unroll
      for (int ed = 0; ed < 3; ++ed) {
        const int nbr = cn[2 + ed];
        const T nxe = g[22 + 4 * ed], nye = g[23 + 4 * ed];
        const int64_t mo = nbr <= -2 ? int64_t(-2 - nbr) : int64_t(A.nmort);
        const int idx0 = int((mo * 2 * Nq + j) * NTP / 4);
#pragma unroll
        for (int c = 0; c < NTP / 4; ++c) {
          const V4<T> sp = bload<T>(rb, idx0 + c);
          const V4<T> su = bload<T>(rb, idx0 + Nq * NTP / 4 + c);
          const T vp[4] = {sp.p, sp.uz, sp.ux, sp.uy}, vu[4] = {su.p, su.uz, su.ux, su.uy};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            if (4 * c + kk < NT) {
              Bp[4 * c + kk] += vp[kk];
              Bx[4 * c + kk] += nxe * vu[kk];
              By[4 * c + kk] += nye * vu[kk];
            }
          }
        }
      }
    }

    // triangular lift on this level, R = L^{tri,k} B with L^{tri,k} = (M^{tri,k})^-1 M^tri
    // (Sec. 4.2).  N <= 4: the reference mass as literals, then the element's
    // inverse mass, stored as its lower triangle (symmetric: each off-diagonal
    // entry serves two rows); N = 5: the stored L^{tri,k}.
    if constexpr (Dim<N>::PACKED) {
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        T sp = 0, sz = 0, sx = 0, sy = 0;
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          constexpr_or_skip(RT::Mtri[i * NT + m], sp, Bp[m]);
          constexpr_or_skip(RT::Mtri[i * NT + m], sz, Bz[m]);
          constexpr_or_skip(RT::Mtri[i * NT + m], sx, Bx[m]);
          constexpr_or_skip(RT::Mtri[i * NT + m], sy, By[m]);
        }
        Rp[i] = sp;
        Rz[i] = sz;
        Rx[i] = sx;
        Ry[i] = sy;
      }
      if constexpr (QM) {
#pragma unroll
        for (int ed = 0; ed < 3; ++ed) {
          const T Ja = MODE == 2 && cn[2 + ed] <= -2 ? T(0) : g[20 + 4 * ed];
          const T Jb = MODE == 2 && cn[2 + ed] <= -2 ? T(0) : g[21 + 4 * ed];
          const T nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
#pragma unroll
          for (int qq = 0; qq < Nq; ++qq) {
            T pa = 0, pb = 0, ua = 0, ub = 0;
#pragma unroll
            for (int q = 0; q < Nq; ++q) {
              constexpr_or_skip(RT::Ma[qq * Nq + q], pa, qf[ed][q][0]);
              constexpr_or_skip(RT::Mb[qq * Nq + q], pb, qf[ed][q][0]);
              constexpr_or_skip(RT::Ma[qq * Nq + q], ua, qf[ed][q][1]);
              constexpr_or_skip(RT::Mb[qq * Nq + q], ub, qf[ed][q][1]);
            }
            const T vp = Ja * pa + Jb * pb, vu = Ja * ua + Jb * ub;
            const int i = edge_node(N, ed, qq);
            Rp[i] += vp;
            Rx[i] += nx * vu;
            Ry[i] += ny * vu;
          }
        }
      }
      {
        static_assert(C::CHOL, "the packed orders factor the triangular mass");
        // R = L^-T L^-1 R: forward substitution row by row, then the
        // transposed solve column by column (the factor's entries in reverse)
        const V4<T>* Lv = sL + le * VL;
#pragma unroll
        for (int c = 0; c < VL; ++c) {
          const V4<T> l4 = Lv[c];
          const T lv[4] = {l4.p, l4.uz, l4.ux, l4.uy};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int f = 4 * c + k;
            if (f < Dim<N>::NPK) {
              const int i = tri_row(f), m = f - i * (i + 1) / 2;
              if (m < i) {
                Rp[i] -= lv[k] * Rp[m];
                Rz[i] -= lv[k] * Rz[m];
                Rx[i] -= lv[k] * Rx[m];
                Ry[i] -= lv[k] * Ry[m];
              } else {
                Rp[i] *= lv[k];
                Rz[i] *= lv[k];
                Rx[i] *= lv[k];
                Ry[i] *= lv[k];
              }
            }
          }
        }
#pragma unroll
        for (int c = VL - 1; c >= 0; --c) {
          const V4<T> l4 = Lv[c];
          const T lv[4] = {l4.p, l4.uz, l4.ux, l4.uy};
#pragma unroll
          for (int k = 3; k >= 0; --k) {
            const int f = 4 * c + k;
            if (f < Dim<N>::NPK) {
              const int i = tri_row(f), m = f - i * (i + 1) / 2;
              if (m < i) {
                Rp[m] -= lv[k] * Rp[i];
                Rz[m] -= lv[k] * Rz[i];
                Rx[m] -= lv[k] * Rx[i];
                Ry[m] -= lv[k] * Ry[i];
              } else {
                Rp[i] *= lv[k];
                Rz[i] *= lv[k];
                Rx[i] *= lv[k];
                Ry[i] *= lv[k];
              }
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NT; ++i) Rp[i] = Rz[i] = Rx[i] = Ry[i] = T(0);
      const V4<T>* Lv = sL + le * VL;
#pragma unroll
      for (int c = 0; c < VL; ++c) {
        const V4<T> l4 = Lv[c];
        const T lv[4] = {l4.p, l4.uz, l4.ux, l4.uy};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int f = 4 * c + k;
          if (f < NT * NT) {
            const int m = f / NT, i = f % NT;  // the record holds L^{tri,k} column by column
            Rp[i] += lv[k] * Bp[m];
            Rz[i] += lv[k] * Bz[m];
            Rx[i] += lv[k] * Bx[m];
            Ry[i] += lv[k] * By[m];
          }
        }
      }
    }

    // horizontal part on the own slice:
    //   R_p -= D_r (r_x u_x + r_y u_y) + D_s (s_x u_x + s_y u_y)
    //   R_x -= r_x D_r p + s_x D_s p ;  R_y -= r_y D_r p + s_y D_s p
    {
      const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
      T Ar[NT], As[NT], P[NT];
#pragma unroll
      for (int m = 0; m < NT; ++m) {
        const V4<T> v = el[j * NT + m];
        Ar[m] = rx * v.ux + ry * v.uy;
        As[m] = sx * v.ux + sy * v.uy;
        P[m] = v.p;
      }
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        T dA = 0, dB = 0, dPr = 0, dPs = 0;
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          constexpr_or_skip(RT::Dr[i * NT + m], dA, Ar[m]);
          constexpr_or_skip(RT::Ds[i * NT + m], dB, As[m]);
          constexpr_or_skip(RT::Dr[i * NT + m], dPr, P[m]);
          constexpr_or_skip(RT::Ds[i * NT + m], dPs, P[m]);
        }
        Rp[i] -= dA;
        Rp[i] -= dB;
        Rx[i] -= rx * dPr;
        Rx[i] -= sx * dPs;
        Ry[i] -= ry * dPr;
        Ry[i] -= sy * dPs;
      }
    }

    const T kap = g[9], irho = g[10];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      Rp[i] *= kap;
      Rz[i] *= irho;
      Rx[i] *= irho;
      Ry[i] *= irho;
    }
    for (int s = 0; s < A.nsrc; ++s) {
      if (A.src_elem[s] == e) {
        const T* sv = static_cast<const T*>(A.srcvec) + s * NP + j * NT;
        const T amp = T(A.src_amp[s]);
#pragma unroll
        for (int i = 0; i < NT; ++i) Rp[i] += amp * sv[i];
      }
    }
  }
  // the gradient epilogue's geometry, before the right-hand side replaces it
  [[maybe_unused]] EpiGeo<T> eg{};
  if constexpr (MODE == 4 && grad_early<N, T>()) {
    const T* gl = reinterpret_cast<const T*>(sG) + (le < EPB ? le : 0) * kGeoStride;
    const int tf = j == 0 ? 0 : 1;
    eg.tJf = gl[12 + 4 * tf];
    eg.tnx = gl[13 + 4 * tf];
    eg.tny = gl[14 + 4 * tf];
    eg.tnz = gl[15 + 4 * tf];
#pragma unroll
    for (int ed = 0; ed < 3; ++ed)
#pragma unroll
      for (int k = 0; k < 4; ++k) eg.qg[ed][k] = gl[20 + 4 * ed + k];
    eg.kap = gl[9];
    eg.irho = gl[10];
    eg.w0 = gl[37];
    eg.w1 = gl[38];
    eg.w2 = gl[39];
  }
  // the right-hand side replaces lifts, geometry and fluxes in LDS
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < NT; ++i) sR[le * NPP + j * NT + i] = V4<T>{Rp[i], Rz[i], Rx[i], Ry[i]};
  }
  __syncthreads();

  // low-storage Runge-Kutta update, coalesced over the chunk
  const T ca = T(A.a), cb = T(A.b), dt = T(A.dt), cg = T(A.g);
  const auto bout = chunk_rsrc(static_cast<V4<T>*>(A.Uout) + e0 * NP, int64_t(nE) * NP * V4B);
  // U' = g U + b res' with g = 1 except in the adjoint sweep: two copies of the loop
  auto update = [&](auto with_g) {
    constexpr bool G = decltype(with_g)::value;
#pragma unroll
    for (int k = 0; k < C::UPD; ++k) {
      const int idx = tid + 64 * k;
      const int l = idx < nE * NP ? idx + (idx / NP) * (NPP - NP) : 0;
      const V4<T> R = sR[l];
      V4<T> q;
      if constexpr (C::PREFETCH)
        q = rprev[k];
      else
        q = bload<T>(bres_in, idx);
      const V4<T> r{ca * q.p + dt * R.p, ca * q.uz + dt * R.uz, ca * q.ux + dt * R.ux, ca * q.uy + dt * R.uy};
      bstore<T>(bres, idx, r);
      // the adjoint sweep's mass terms take the incoming adjoint state from
      // here (each slot is read above by the lane that writes it; the lanes
      // past the chunk write the spare slot)
      if constexpr (MODE == 4) sR[idx < nE * NP ? l : EPB * C::XPE] = q;
      if (wu) {
        V4<T> u = sU[l];
        if constexpr (G) u = V4<T>{cg * u.p, cg * u.uz, cg * u.ux, cg * u.uy};
        bstore<T>(bout, idx, V4<T>{u.p + cb * r.p, u.uz + cb * r.uz, u.ux + cb * r.ux, u.uy + cb * r.uy});
      }
    }
  };
  if (A.flags & kGamma)
    update(std::true_type{});
  else
    update(std::false_type{});
  if constexpr (MODE == 4) grad_epilogue<N, T>(A, e0, nE, tid, le, j, active, e, sU, sX, cn, eg);
  if constexpr (MODE == 5) {
    __syncthreads();  // the update's reads of the staged state are done
    if (tid < NT) carry[tid] = sU[(nE - 1) * NPP + N * NT + tid];
    __syncthreads();  // the next chunk may restage
  }
}

// chunk c of a mesh: wedges c EPB .. min((c + 1) EPB, Kw) - 1
template <int N, typename T, int MODE>
__device__ __forceinline__ void wedge_stage_chunk_at(const StageLaunch& A, int chunk) {
  constexpr int EPB = Cfg<N, T>::EPB;
  const int64_t e0 = int64_t(chunk) * EPB;
  const int64_t left = A.Kw - e0;
  wedge_stage_chunk<N, T, MODE>(A, e0, left < EPB ? int(left) : EPB);
}

// XCD-aware mapping: consecutive workgroups go to different XCDs, so give
// every XCD one contiguous range of chunks (face neighbours share its L2).
__device__ __forceinline__ int xcd_chunk(int bid, int nb) {
  const int qd = nb / 8, rm = nb % 8, xcd = bid % 8, kk = bid / 8;
  return xcd < rm ? xcd * (qd + 1) + kk : rm * (qd + 1) + (xcd - rm) * qd + kk;
}

// From N = 4 on, one wavefront per SIMD: the lane's triangle slice (15+
// nodes x 4 equations, twice) then fits in registers instead of spilling.
template <int N, typename T, int MODE>
__global__ void __launch_bounds__(64, (N >= 4 ? 1 : WDG_STAGE_WAVES_PER_EU)) wedge_stage(StageLaunch A) {
  wedge_stage_chunk_at<N, T, MODE>(A, xcd_chunk(blockIdx.x, gridDim.x));
}

// Column marching (the layer-by-layer reuse the paper proposes as future
// work, Sec. 7): block b walks the wedges of column segment b (a run of at
// most 2 EPB consecutive elements stacked bottom to top, from A.cols; the
// host splits taller columns) in two chunks of EPB layers from the bottom;
// vertical neighbours inside a chunk come from its staged state, the wedge
// below the second chunk's first one from the first chunk's top level kept
// in LDS, so no triangular face inside the segment is gathered from memory.
// (Straight-line code for the two chunks: a loop over chunks keeps values
// live across its back edge and spills.)
template <int N, typename T>
__global__ void __launch_bounds__(64, (N >= 4 ? 1 : WDG_STAGE_WAVES_PER_EU)) wedge_column_stage(StageLaunch A) {
  constexpr int EPB = Cfg<N, T>::EPB;
  __shared__ V4<T> carry[Dim<N>::NT];
  const int2 col = A.cols[xcd_chunk(blockIdx.x, gridDim.x)];
  wedge_stage_chunk<N, T, 5>(A, int64_t(col.x), col.y < EPB ? col.y : EPB, carry, false);
  if (col.y > EPB) {
    const int left = col.y - EPB;
    wedge_stage_chunk<N, T, 5>(A, int64_t(col.x) + EPB, left < EPB ? left : EPB, carry, true);
  }
}

// Many independent meshes of one order in one launch: block b takes chunk
// w = (problem, chunk) of a problem-major list, every XCD one contiguous range
// of it (face neighbours share an L2).  The stage record of each problem
// (buffers, coefficients, time step, source amplitudes) is in device memory,
// written by the batch preparation kernel of the stage.  WPE is the
// occupancy the register allocation aims at (1: up to 512 registers, no
// spills at high order; 2: as the single-problem kernel), chosen per order by
// the batch autotuner.
template <int N, typename T, int WPE>
__global__ void __launch_bounds__(64, WPE)
    wedge_batch_stage(const StageLaunch* __restrict__ probs, const int2* __restrict__ work, int nwork) {
  const int w = xcd_chunk(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const int2 it = work[w];
  wedge_stage_chunk_at<N, T, 0>(probs[it.x], it.y);  // the record is wave-uniform: scalar loads
}

template <int N, typename T>
hipError_t launch_wedge_batch_t(const StageLaunch* probs, const int2* work, int nwork, int wpe, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  if (wpe == 1)
    hipLaunchKernelGGL((wedge_batch_stage<N, T, 1>), dim3(unsigned(nwork)), dim3(Cfg<N, T>::BS), 0, st, probs, work,
                       nwork);
  else
    hipLaunchKernelGGL((wedge_batch_stage<N, T, 2>), dim3(unsigned(nwork)), dim3(Cfg<N, T>::BS), 0, st, probs, work,
                       nwork);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_wedge_stage_t(const StageLaunch& a, hipStream_t st) {
  using C = Cfg<N, T>;
  const int64_t nchunks = (a.Kw + C::EPB - 1) / C::EPB;
  if (nchunks <= 0) return hipSuccess;
  if (a.nmort > 0)
    hipLaunchKernelGGL((wedge_stage<N, T, 2>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else if (a.Kt == 0 && (a.flags & kGrad))
    hipLaunchKernelGGL((wedge_stage<N, T, 4>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else if (a.Kt == 0 && (a.flags & kColumnMarch) && a.cols && a.ncols > 0)
    hipLaunchKernelGGL((wedge_column_stage<N, T>), dim3(unsigned(a.ncols)), dim3(C::BS), 0, st, a);
  else if (a.Kt == 0 && (a.flags & kLayerMarch))
    hipLaunchKernelGGL((wedge_stage<N, T, 3>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else if (a.Kt > 0)
    hipLaunchKernelGGL((wedge_stage<N, T, 1>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else
    hipLaunchKernelGGL((wedge_stage<N, T, 0>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  return hipGetLastError();
}

}  // namespace

int wedge_chunk_elems(int N, int bits) {
  int epb = 0;
#define WDG_EPB(n, T) epb = Cfg<n, T>::EPB
  WDG_DISPATCH_N(N, bits, WDG_EPB)
#undef WDG_EPB
  return epb;
}

hipError_t launch_wedge_batch(int N, int bits, const StageLaunch* probs, const int2* work, int nwork, int wpe,
                              hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_wedge_batch_t<n, T>(probs, work, nwork, wpe, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

hipError_t launch_wedge_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_wedge_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

}  // namespace wdg
