// HIP kernels of libwdg for CDNA4 (gfx950).
//
//   setup_kernel     FP64 geometric factors (Lemma 1), face Jacobians and normals,
//                    triangular lift L^{tri,k} = (M^{tri,k})^-1 M^tri (Sec. 4.2)
//   wedge_stage      one Runge-Kutta stage on the wedges: volume term, surface
//                    fluxes, lifts, L^{tri,k} application and the low-storage
//                    update, fused
//   tet_stage        the same stage on the affine tetrahedra of hybrid meshes
//                    (standard nodal DG; they meet wedges at triangular faces)
//   sample_receivers pressure at receiver points
//   energy_kernel    discrete energy with M^k = M^{tri,k} (x) M^1D
#include <hip/hip_runtime.h>

#include <cstring>

#include "kernels.hpp"
#include "ref_tables.inc"

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

// Node-interleaved state: one 4-vector per node in the order (p, u_z, u_x, u_y).
template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T p, uz, ux, uy;
};

// Launch shape: one wavefront per block, lane = (element, level j), so a block
// holds EPB = 64 / Nq elements (fewer where the LDS would exceed 64 KiB).  LDS
// holds the staged state (per-element stride NPP, odd in 4-vectors, so that the
// elements of a wavefront fall on different banks) and a second region that
// first holds the triangular lifts, geometry records and triangular-face
// fluxes, and afterwards the right-hand side on its way to the coalesced
// update.
template <int N, typename T>
struct Cfg {
  static constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  static constexpr int NPP = NP | 1;
  static constexpr int VL = Dim<N>::LS / 4, VG = kGeoStride / 4, VF = NT;  // 4-vectors per element
  static constexpr int XPE = (VL + VG + VF) > NPP ? (VL + VG + VF) : NPP;
  static constexpr int per_elem = (NPP + XPE) * 4 * int(sizeof(T));
  static constexpr int EPB_FULL = 64 / Nq;
  static constexpr int EPB = EPB_FULL * per_elem <= 65536 ? EPB_FULL : 65536 / per_elem;
  static constexpr int BS = 64;
  // 4-vectors of the chunk each lane carries through the coalesced update
  static constexpr int UPD = (EPB * NP + BS - 1) / BS;
  // prefetch the previous residual into registers when that costs at most 40 of them
#ifndef WDG_PREFETCH_REGS
#define WDG_PREFETCH_REGS 40
#endif
  static constexpr bool PREFETCH = UPD * 4 * int(sizeof(T)) / 4 <= WDG_PREFETCH_REGS;
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

// Node of the neighbour's triangular face that coincides with node i of this
// element's face, for vertex permutation code p: node i has lattice indices
// (N-a-b, a, b); the permutation reorders them.  Selector of the neighbour's
// second / third index for each p, two bits per code (see the host's table of
// the six vertex permutations).
template <int N>
__device__ __forceinline__ int face_perm(int p, int i) {
  int b = 0;
#pragma unroll
  for (int bb = 1; bb <= N; ++bb) b += i >= tri_idx(N, 0, bb) ? 1 : 0;
  const int a = i - (b * (N + 1) - b * (b - 1) / 2);
  const int c = N - a - b;
  const int s1 = (417 >> (2 * p)) & 3, s2 = (2118 >> (2 * p)) & 3;
  const int j1 = s1 == 0 ? c : (s1 == 1 ? a : b);
  const int j2 = s2 == 0 ? c : (s2 == 1 ? a : b);
  return j2 * (N + 1) - j2 * (j2 - 1) / 2 + j1;
}

template <int N>
struct TDim {
  static constexpr int NT = (N + 1) * (N + 2) / 2;
  static constexpr int NP = (N + 1) * (N + 2) * (N + 3) / 6;
};
__host__ __device__ constexpr int tet_np(int n) { return (n + 1) * (n + 2) * (n + 3) / 6; }

// Tetrahedron node of face f's triangle node m.  The face node has integer
// barycentrics (N-a-b, a, b) relative to the face's vertices (faces
// (V0,V1,V2), (V0,V1,V3), (V1,V2,V3), (V0,V2,V3)); the tetrahedron orders its
// lattice (l1, l2, l3) by l3, then l2, then l1.
template <int N>
__device__ __forceinline__ int tet_face_node(int f, int m) {
  int b = 0;
#pragma unroll
  for (int bb = 1; bb <= N; ++bb) b += m >= tri_idx(N, 0, bb) ? 1 : 0;
  const int a = m - (b * (N + 1) - b * (b - 1) / 2);
  const int c = N - a - b;
  const int l1 = f == 0 ? a : (f == 1 ? a : (f == 2 ? c : 0));
  const int l2 = f == 0 ? b : (f == 1 ? 0 : a);
  const int l3 = f == 0 ? 0 : b;
  const int n = N - l3;  // the slice l3 is a triangle lattice of order n
  return tet_np(N) - tet_np(n) + l2 * (n + 1) - l2 * (l2 - 1) / 2 + l1;
}

// Raw buffer access to one chunk of a stream.  Loads past the resource's
// byte count return zeros and stores there are dropped by the hardware, so
// the ragged last chunk needs no branches around memory operations (a branch
// lets the compiler sink a load next to its use and serialise the latencies).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), kRsrcWord3);
}
template <typename T>
__device__ __forceinline__ V4<T> bload(__amdgpu_buffer_rsrc_t r, int idx) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(V4<T>, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16, 0, 0));
  } else {
    struct H2 {
      u32x4 lo, hi;
    } h{__builtin_amdgcn_raw_buffer_load_b128(r, idx * 32, 0, 0), __builtin_amdgcn_raw_buffer_load_b128(r, idx * 32 + 16, 0, 0)};
    return __builtin_bit_cast(V4<T>, h);
  }
}
// Stores of the stage outputs are streaming (cache policy: non-temporal):
// the next stage reads them back from HBM anyway.
constexpr int kStreamStore = 2;
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int idx, const V4<T>& v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, idx * 16, 0, kStreamStore);
  } else {
    struct H2 {
      u32x4 lo, hi;
    };
    const H2 h = __builtin_bit_cast(H2, v);
    __builtin_amdgcn_raw_buffer_store_b128(h.lo, r, idx * 32, 0, kStreamStore);
    __builtin_amdgcn_raw_buffer_store_b128(h.hi, r, idx * 32 + 16, 0, kStreamStore);
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
// ---------------------------------------------------------------------------
#ifndef WDG_STAGE_WAVES_PER_EU
#define WDG_STAGE_WAVES_PER_EU 2
#endif
// MODE 0: wedges only; 1: tetrahedra across triangular faces; 2: also mortars
template <int N, typename T, int MODE>
__global__ void __launch_bounds__(64, WDG_STAGE_WAVES_PER_EU) wedge_stage(StageLaunch A) {
  constexpr bool HYB = MODE >= 1;
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

  // XCD-aware mapping: consecutive workgroups go to different XCDs, so give
  // every XCD one contiguous range of chunks (face neighbours share its L2).
  const int nb = gridDim.x, bid = blockIdx.x;
  const int qd = nb / 8, rm = nb % 8, xcd = bid % 8, kk = bid / 8;
  const int chunk = xcd < rm ? xcd * (qd + 1) + kk : rm * (qd + 1) + (xcd - rm) * qd + kk;
  const int64_t e0 = int64_t(chunk) * EPB;
  const int64_t left = A.Kw - e0;
  const int nE = left < EPB ? int(left) : EPB;
  const int tid = threadIdx.x;

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
  constexpr int SU = (EPB * NP + 63) / 64, SL = (EPB * VL + 63) / 64, SG = (EPB * VG + 63) / 64;
  constexpr int V4B = 4 * int(sizeof(T));
  V4<T> rU[SU], rL[SL], rG[SG];
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
      gt[t] = Uin[src * NP + nlev * NT + fn];
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

  const V4<T>* el = sU + le * NPP;
  const T* g = reinterpret_cast<const T*>(sG) + le * kGeoStride;

  // pre-lift accumulators of the four equations on this level
  T Bp[NT], Bz[NT], Bx[NT], By[NT];

  if (active) {
    const T tzJ = g[4];
    const T tl = T(0.5) * (T(1) - pick<Nq, T>(RT::t, j, 1, 0));
    const T th = T(0.5) * (T(1) + pick<Nq, T>(RT::t, j, 1, 0));
    const T txJ = g[5] * tl + g[6] * th;
    const T tyJ = g[7] * tl + g[8] * th;
    T dtr[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) dtr[m] = pick<Nq, T>(RT::Dt, j, Nq, m);

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
        fpa[q] = Ja * Fp;
        fpb[q] = Jb * Fp;
        fua[q] = Ja * Fu;
        fub[q] = Jb * Fu;
      }
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
  const auto bres = chunk_rsrc(res_chunk, int64_t(nE) * NP * V4B);
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
      const T g0j = lumped ? (j == 0 ? wend : T(0)) : pick<Nq, T>(RT::g0, j, 1, 0);
      const T gNj = lumped ? (j == N ? wend : T(0)) : pick<Nq, T>(RT::gN, j, 1, 0);
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

    // triangular lift L^{tri,k} on this level: R = L B
#pragma unroll
    for (int i = 0; i < NT; ++i) Rp[i] = Rz[i] = Rx[i] = Ry[i] = T(0);
    {
      const V4<T>* Lv = sL + le * VL;
#pragma unroll
      for (int c = 0; c < VL; ++c) {
        const V4<T> l4 = Lv[c];
        const T lv[4] = {l4.p, l4.uz, l4.ux, l4.uy};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int f = 4 * c + k;
          if (f < NT * NT) {
            const int i = f / NT, m = f % NT;
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
  // the right-hand side replaces lifts, geometry and fluxes in LDS
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < NT; ++i) sR[le * NPP + j * NT + i] = V4<T>{Rp[i], Rz[i], Rx[i], Ry[i]};
  }
  __syncthreads();

  // low-storage Runge-Kutta update, coalesced over the chunk
  const T ca = T(A.a), cb = T(A.b), dt = T(A.dt);
  const auto bout = chunk_rsrc(static_cast<V4<T>*>(A.Uout) + e0 * NP, int64_t(nE) * NP * V4B);
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
    if (wu) {
      const V4<T> u = sU[l];
      bstore<T>(bout, idx, V4<T>{u.p + cb * r.p, u.uz + cb * r.uz, u.ux + cb * r.ux, u.uy + cb * r.uy});
    }
  }
}

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

// ---------------------------------------------------------------------------
// Tetrahedron stage kernel (affine tetrahedra, standard nodal DG)
//
// Lane (element, node i); a block of 256 lanes holds EPB = 256 / Np
// tetrahedra per chunk and loops over chunks (persistent), so the reference
// operators Dr, Ds, Dt and LIFT are staged in LDS once per block where they
// fit (read from memory otherwise).  Per chunk:
//   1. node i stores (p, r.u, s.u, t.u) with r.u = r_x u_x + r_y u_y + r_z u_z
//      (and likewise s, t), so that div u = D_r(r.u) + D_s(s.u) + D_t(t.u);
//      the 4 Np_tri face nodes are shared out over the lanes, whose fluxes
//      (scaled by J_f / J) go to LDS
//   2. node i: volume terms, LIFT of the fluxes, material scaling, sources and
//      the low-storage update (node-contiguous, coalesced)
// ---------------------------------------------------------------------------
template <int N, typename T>
struct TCfg {
  static constexpr int NT = TDim<N>::NT, NP = TDim<N>::NP;
  static constexpr int BS = 256;
  static constexpr int EPB = BS / NP;
  static constexpr int NOPS = 3 * NP * NP + NP * 4 * NT;
  static constexpr bool OPS_LDS = NOPS * int(sizeof(T)) <= 40960;
  static constexpr int SLOTS = (4 * NT + NP - 1) / NP;  // face nodes per lane
};

template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T p, ar, as, at;
};

template <int N, typename T>
__global__ void __launch_bounds__(256) tet_stage(StageLaunch A) {
  using C = TCfg<N, T>;
  constexpr int NT = C::NT, NP = C::NP, EPB = C::EPB;
  constexpr int NPW = Dim<N>::NP;
  __shared__ T sOps[C::OPS_LDS ? C::NOPS : 1];
  __shared__ V4<T> sU[EPB * NP];
  __shared__ Q4<T> sW[EPB * NP];
  __shared__ T sF[EPB * 4 * NT * 2];
  __shared__ T sG[EPB * kTetGeoStride];
  __shared__ int sC[EPB * kTetConnStride];

  const T* gops = static_cast<const T*>(A.opsT);
  if constexpr (C::OPS_LDS) {
    for (int idx = threadIdx.x; idx < C::NOPS; idx += C::BS) sOps[idx] = gops[idx];
  }
  const T* ops = C::OPS_LDS ? static_cast<const T*>(sOps) : gops;
  const T* Dr = ops;
  const T* Ds = ops + NP * NP;
  const T* Dt = ops + 2 * NP * NP;
  const T* LIFT = ops + 3 * NP * NP;

  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  V4<T>* __restrict__ res = static_cast<V4<T>*>(A.res);
  V4<T>* __restrict__ Uout = static_cast<V4<T>*>(A.Uout);
  const T* __restrict__ geo = static_cast<const T*>(A.geoT);
  const int* __restrict__ conn = A.connT;
  const int64_t tb = A.Kw * NPW;  // first tetrahedron node
  const int tid = threadIdx.x;
  const int le = tid / NP, i = tid - le * NP;
  const T bsign = (A.flags & kDirichlet) ? T(-1) : T(1);
  const T tau_on = (A.flags & kCentral) ? T(0) : T(1);
  const bool rd = (A.flags & kReadRes) != 0, wu = (A.flags & kWriteU) != 0;
  const int64_t nchunks = (A.Kt + EPB - 1) / EPB;

  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const int64_t e0 = chunk * EPB;
    const int nE = int(A.Kt - e0 < EPB ? A.Kt - e0 : EPB);
    __syncthreads();  // the previous chunk is done with LDS
    for (int idx = tid; idx < nE * NP; idx += C::BS) sU[idx] = Uin[tb + e0 * NP + idx];
    for (int idx = tid; idx < nE * kTetGeoStride; idx += C::BS) sG[idx] = geo[e0 * kTetGeoStride + idx];
    for (int idx = tid; idx < nE * kTetConnStride; idx += C::BS) sC[idx] = conn[e0 * kTetConnStride + idx];
    __syncthreads();

    const bool active = tid < EPB * NP && le < nE;
    const T* g = sG + le * kTetGeoStride;
    const int* cn = sC + le * kTetConnStride;
    const int64_t e = e0 + le;
    if (active) {
      const V4<T> v = sU[le * NP + i];
      sW[le * NP + i] = Q4<T>{v.p, g[0] * v.ux + g[1] * v.uy + g[2] * v.uz, g[3] * v.ux + g[4] * v.uy + g[5] * v.uz,
                              g[6] * v.ux + g[7] * v.uy + g[8] * v.uz};
      const int code = cn[4];
#pragma unroll
      for (int sl = 0; sl < C::SLOTS; ++sl) {
        const int q = i + NP * sl;
        if (q < 4 * NT) {
          const int f = q / NT, m = q - f * NT;
          const int nbr = cn[f];
          const T w_in = nbr >= 0 ? T(1) : T(0);
          const int pc = (code >> (5 * f)) & 7, nf = (code >> (5 * f + 3)) & 3;
          const int fn = face_perm<N>(pc, m);
          const int64_t src = nbr >= 0 ? int64_t(nbr) : A.Kw + e;
          const int64_t gi = src >= A.Kw ? tb + (src - A.Kw) * NP + tet_face_node<N>(nf, fn)
                                         : src * NPW + (nf == 1 ? N * NT : 0) + fn;
          const V4<T> own = sU[le * NP + tet_face_node<N>(f, m)];
          const V4<T> nb = Uin[gi];
          const T Fs = g[12 + 4 * f], nx = g[13 + 4 * f], ny = g[14 + 4 * f], nz = g[15 + 4 * f];
          const T zs = g[28 + f];
          const T taup = tau_on * T(2) / zs;
          const T tauu = tau_on * zs * T(0.5);
          const T pm = own.p;
          const T unm = nx * own.ux + ny * own.uy + nz * own.uz;
          const T pb = bsign * pm, ub = -bsign * unm;
          const T pp = pb + w_in * (nb.p - pb);
          const T unp = ub + w_in * ((nx * nb.ux + ny * nb.uy + nz * nb.uz) - ub);
          const T jp = pp - pm, jun = unp - unm;
          T Fp = T(0.5) * (taup * jp - jun), Fu = T(0.5) * (tauu * jun - jp);
          if (nbr <= -2) {
            // mortar side: the equivalent nodal flux of the common refinement
            const T* mf = static_cast<const T*>(A.mortF) + int64_t(-2 - nbr) * 2 * NT;
            Fp = mf[m];
            Fu = mf[NT + m];
          }
          sF[(le * 4 * NT + q) * 2] = Fs * Fp;
          sF[(le * 4 * NT + q) * 2 + 1] = Fs * Fu;
        }
      }
    }
    __syncthreads();
    if (!active) continue;

    T dpr = 0, dps = 0, dpt = 0, div = 0;
#pragma unroll 5
    for (int m = 0; m < NP; ++m) {
      const Q4<T> w = sW[le * NP + m];
      const T dr = Dr[i * NP + m], ds = Ds[i * NP + m], dt = Dt[i * NP + m];
      dpr += dr * w.p;
      dps += ds * w.p;
      dpt += dt * w.p;
      div += dr * w.ar;
      div += ds * w.as;
      div += dt * w.at;
    }
    T lp = 0, lx = 0, ly = 0, lz = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      T su = 0;
#pragma unroll 3
      for (int m = 0; m < NT; ++m) {
        const T l = LIFT[i * 4 * NT + f * NT + m];
        lp += l * sF[(le * 4 * NT + f * NT + m) * 2];
        su += l * sF[(le * 4 * NT + f * NT + m) * 2 + 1];
      }
      lx += g[13 + 4 * f] * su;
      ly += g[14 + 4 * f] * su;
      lz += g[15 + 4 * f] * su;
    }
    const T kap = g[9], irho = g[10];
    T Rp = kap * (lp - div);
    const T Rx = irho * (lx - (g[0] * dpr + g[3] * dps + g[6] * dpt));
    const T Ry = irho * (ly - (g[1] * dpr + g[4] * dps + g[7] * dpt));
    const T Rz = irho * (lz - (g[2] * dpr + g[5] * dps + g[8] * dpt));
    for (int s = 0; s < A.nsrc; ++s)
      if (A.src_elem[s] == A.Kw + e) Rp += T(A.src_amp[s]) * static_cast<const T*>(A.srcvec)[s * NPW + i];

    const int64_t gi = tb + e * NP + i;
    const T ca = T(A.a), cb = T(A.b), dtt = T(A.dt);
    V4<T> r{dtt * Rp, dtt * Rz, dtt * Rx, dtt * Ry};
    if (rd) {
      const V4<T> q = res[gi];
      r.p += ca * q.p;
      r.uz += ca * q.uz;
      r.ux += ca * q.ux;
      r.uy += ca * q.uy;
    }
    res[gi] = r;
    if (wu) {
      const V4<T> u = sU[le * NP + i];
      Uout[gi] = V4<T>{u.p + cb * r.p, u.uz + cb * r.uz, u.ux + cb * r.ux, u.uy + cb * r.uy};
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

template <typename T>
__global__ void sample_receivers(int ld, int nrec, const T* __restrict__ U, const int64_t* __restrict__ base,
                                 const int* __restrict__ nn, const double* __restrict__ rows, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const T* Ue = U + base[r] * 4;
  double acc = 0.0;
  for (int n = 0; n < nn[r]; ++n) acc += rows[int64_t(r) * ld + n] * double(Ue[4 * n]);
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
hipError_t launch_wedge_stage_t(const StageLaunch& a, hipStream_t st) {
  using C = Cfg<N, T>;
  const int64_t nchunks = (a.Kw + C::EPB - 1) / C::EPB;
  if (nchunks <= 0) return hipSuccess;
  if (a.nmort > 0)
    hipLaunchKernelGGL((wedge_stage<N, T, 2>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else if (a.Kt > 0)
    hipLaunchKernelGGL((wedge_stage<N, T, 1>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else
    hipLaunchKernelGGL((wedge_stage<N, T, 0>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_mortar_stage_t(const StageLaunch& a, hipStream_t st) {
  if (a.nmort <= 0) return hipSuccess;
  const unsigned grid = unsigned(a.nmort < 8192 ? a.nmort : 8192);
  hipLaunchKernelGGL((mortar_kernel<N, T>), dim3(grid), dim3(64), 0, st, a);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_tet_stage_t(const StageLaunch& a, hipStream_t st) {
  if (a.Kt <= 0) return hipSuccess;
  using TC = TCfg<N, T>;
  const int64_t tchunks = (a.Kt + TC::EPB - 1) / TC::EPB;
  const unsigned grid = unsigned(tchunks < 2048 ? tchunks : 2048);
  hipLaunchKernelGGL((tet_stage<N, T>), dim3(grid), dim3(TC::BS), 0, st, a);
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

hipError_t launch_wedge_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_wedge_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

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

hipError_t launch_tet_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_tet_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

hipError_t launch_receivers(int bits, int ld, int nrec, const void* U, const int64_t* base, const int* nn,
                            const double* rows, double* out, hipStream_t st) {
  if (nrec <= 0) return hipSuccess;
  const unsigned nb = unsigned((nrec + 63) / 64);
  if (bits == 32)
    hipLaunchKernelGGL(sample_receivers<float>, dim3(nb), dim3(64), 0, st, ld, nrec, static_cast<const float*>(U), base,
                       nn, rows, out);
  else
    hipLaunchKernelGGL(sample_receivers<double>, dim3(nb), dim3(64), 0, st, ld, nrec, static_cast<const double*>(U),
                       base, nn, rows, out);
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
