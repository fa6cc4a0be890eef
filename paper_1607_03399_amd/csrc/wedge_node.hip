// Wedge stage kernel of libwdg for high orders, one lane per triangle node
// (Sec. 4.2-4.3: the same stage as wedge_stage.hip, fused volume term,
// surface fluxes and lifts, L^{tri,k} application and low-storage update).
//
// wedge_stage gives each lane a GLL level of an element and keeps the whole
// triangular slice of the four equations in registers (twice: pre-lift sums
// and right-hand side), which at N >= 4 pins it to one wavefront per SIMD.
// Here lane (element, triangle node i) owns the vertical line of node i:
// its N+1 levels of the four equations (4 (N+1) values), so the kernel runs
// several wavefronts per SIMD.  The element's state, pre-lift sums and the
// quadrilateral-face fluxes are shared through LDS; a lane reads the other
// nodes' values as broadcasts (all lanes of an element read the same address).
//   1. staging: state (coalesced), geometry, reference rows D_r, D_s, E^{a,b}
//      (block-shared, LDS); the lane's row of L^{tri,k} (the record is stored
//      column by column, so these loads coalesce across the element's lanes);
//      neighbour gathers of the node's two triangular-face traces and of the
//      lane's share of the quadrilateral-face nodes
//   2. quadrilateral-face fluxes (per face node, to LDS); vertical part
//      -t_dJ D_t U along the node's line; triangular-face fluxes of the node
//      and their lift (M^1D)^-1 e_{0,N}; quadrilateral lifts J^a E^a + J^b E^b
//      from LDS -> pre-lift sums B (to LDS)
//   3. R = L^{tri,k} B for the node's row, all levels and fields; horizontal
//      part -(r_x D_r + s_x D_s) ... with the node's rows of D_r, D_s
//   4. material scaling, sources, low-storage update of the node's line
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "ref_tables.inc"

namespace wdg {
namespace {

template <int N, typename T, int EPB_>
struct NCfg {
  static constexpr int NT = Dim<N>::NT, Nq = Dim<N>::Nq, NP = Dim<N>::NP;
  static constexpr int NPP = NP | 1;  // odd 4-vector stride per element (banks)
  static constexpr int EPB = EPB_;
  static constexpr int LANES = EPB * NT;
  static constexpr int BS = (LANES + 63) / 64 * 64;
  static constexpr int NQF = 3 * Nq * Nq;           // quadrilateral-face nodes per element
  static constexpr int QSL = (NQF + NT - 1) / NT;   // of them per lane
  static constexpr int NOPS = 2 * NT * NT + 6 * NT * Nq;  // D_r, D_s, E^a, E^b
  static constexpr int LS = (NT * NT + 3) / 4 * 4;  // record of L^{tri,k} (column-major)
  static constexpr int LV = LS / 4;                 // its 4-vectors
  // per element, one region holds the quadrilateral-face fluxes and later the pre-lift sums
  static constexpr int XV = (2 * NQF + 3) / 4 > NPP ? (2 * NQF + 3) / 4 : NPP;
  static constexpr int SU = (EPB * NP + BS - 1) / BS;
  static constexpr int SL = (EPB * LV + BS - 1) / BS;
  static constexpr int SGV = kGeoStride / 4;        // geometry 4-vectors per element
  static constexpr int SG = (EPB * SGV + BS - 1) / BS;
  static constexpr int SO = (NOPS + BS - 1) / BS;
};

template <int N, typename T, int MODE, int EPB>
__device__ __forceinline__ void wedge_node_chunk(const StageLaunch& A, int chunk) {
  constexpr bool HYB = MODE == 1 || MODE == 2;
  using C = NCfg<N, T, EPB>;
  using RT = gen::RefTables<N>;
  constexpr int NT = C::NT, Nq = C::Nq, NP = C::NP, NPP = C::NPP, BS = C::BS;
  constexpr int V4B = 4 * int(sizeof(T));
  __shared__ T sOp[C::NOPS];
  __shared__ V4<T> sU[EPB * NPP + 1];
  __shared__ V4<T> sX[EPB * C::XV];  // quadrilateral-face fluxes, then pre-lift sums
  __shared__ V4<T> sL4[EPB * C::LV + 1];
  __shared__ V4<T> sG4[EPB * C::SGV + 1];
  T* const sFq = reinterpret_cast<T*>(sX);
  V4<T>* const sB = sX;
  const T* sDr = sOp;
  const T* sDs = sOp + NT * NT;
  const T* sEa = sOp + 2 * NT * NT;            // [edge][i][q]
  const T* sEb = sOp + 2 * NT * NT + 3 * NT * Nq;

  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const int64_t e0 = int64_t(chunk) * EPB;
  const int64_t left = A.Kw - e0;
  const int nE = left < EPB ? int(left) : EPB;
  const int tid = threadIdx.x;
  const int le_raw = tid / NT;
  const bool active = le_raw < nE;
  const int le = active ? le_raw : 0;  // idle lanes shadow the chunk's first element
  const int i = active ? tid - le_raw * NT : 0;
  const int64_t e = e0 + le;
  const T bsign = (A.flags & kDirichlet) ? T(-1) : T(1);
  const T tau_on = (A.flags & kCentral) ? T(0) : T(1);

  // ---- 1. loads: connectivity first, then the coalesced staging, then the gathers
  // (named values, not an array: a lane-dependent selection from a private
  // array becomes a scratch load, whose wait also waits for every gather
  // issued before it)
  const int4* cp = reinterpret_cast<const int4*>(A.conn + e * kConnStride);
  const int4 c0 = cp[0], c1 = cp[1];
  // the chunk's coalesced staging loads, issued before the connectivity is
  // waited for (the vector-memory counter completes in order: waiting for
  // the connectivity does not wait for these)
  V4<T> rU[C::SU], rG[C::SG], rL[C::SL];
  T rO[C::SO];
  {
    const auto bu = chunk_rsrc(Uin + e0 * NP, int64_t(nE) * NP * V4B);
    const auto bl = chunk_rsrc(static_cast<const T*>(A.L) + e0 * C::LS, int64_t(nE) * C::LV * V4B);
    const auto bg = chunk_rsrc(static_cast<const T*>(A.geo) + e0 * kGeoStride, int64_t(nE) * C::SGV * V4B);
#pragma unroll
    for (int k = 0; k < C::SU; ++k) rU[k] = bload<T>(bu, tid + BS * k);
#pragma unroll
    for (int k = 0; k < C::SL; ++k) rL[k] = bload<T>(bl, tid + BS * k);
#pragma unroll
    for (int k = 0; k < C::SG; ++k) rG[k] = bload<T>(bg, tid + BS * k);
    const T* ops = static_cast<const T*>(A.opsW);
#pragma unroll
    for (int k = 0; k < C::SO; ++k) {
      const int idx = tid + BS * k;
      rO[k] = ops[idx < C::NOPS ? idx : 0];
    }
  }
  const int tri_nb0 = c0.x, tri_nb1 = c0.y, quad_nb0 = c0.z, quad_nb1 = c0.w, quad_nb2 = c1.x;
  const int code = c1.y;
  // neighbour across triangular face (0 bottom, 1 top) and quadrilateral face ed
  auto tri_nbr = [&](int face) { return face == 0 ? tri_nb0 : tri_nb1; };
  auto quad_nbr = [&](int ed) { return ed == 0 ? quad_nb0 : (ed == 1 ? quad_nb1 : quad_nb2); };
  // the node's traces on the neighbours across the bottom and top triangles
  V4<T> gt[2];
#pragma unroll
  for (int face = 0; face < 2; ++face) {
    const int nbr = tri_nbr(face);
    const int pc = (code >> (3 * face)) & 7;
    const int nlev = ((code >> (6 + face)) & 1) ? N : 0;
    const int64_t src = nbr >= 0 ? int64_t(nbr) : e;
    const int fn = face_perm<N>(pc, i);
    if constexpr (HYB) {
      const int tf = (code >> (14 + 2 * face)) & 3;
      const bool tet = src >= A.Kw;
      gt[face] = Uin[tet ? A.Kw * NP + (src - A.Kw) * TDim<N>::NP + tet_face_node<N>(tf, fn) : src * NP + nlev * NT + fn];
    } else {
      gt[face] = Uin[src * NP + nlev * NT + fn];
    }
  }
  // the lane's quadrilateral-face nodes: slot s covers face node f = i + NT s,
  // f = (edge, level j, edge node q); surplus slots redo the last face node
  V4<T> gq[C::QSL];
#pragma unroll
  for (int s = 0; s < C::QSL; ++s) {
    const int f0 = i + NT * s;
    const int f = f0 < C::NQF ? f0 : C::NQF - 1;
    const int ed = f / (Nq * Nq), jq = f - ed * Nq * Nq, j = jq / Nq, q = jq - j * Nq;
    const int nbr = quad_nbr(ed);
    const int ned = (code >> (8 + 2 * ed)) & 3;
    const int ni = ned == 0 ? edge_node(N, 0, N - q) : (ned == 1 ? edge_node(N, 1, N - q) : edge_node(N, 2, N - q));
    gq[s] = Uin[(nbr >= 0 ? int64_t(nbr) : e) * NP + j * NT + ni];
  }
#pragma unroll
  for (int k = 0; k < C::SU; ++k) {
    const int idx = tid + BS * k;
    sU[idx < EPB * NP ? idx + (idx / NP) * (NPP - NP) : EPB * NPP] = rU[k];
  }
#pragma unroll
  for (int k = 0; k < C::SL; ++k) {
    const int idx = tid + BS * k;
    sL4[idx < EPB * C::LV ? idx : EPB * C::LV] = rL[k];
  }
#pragma unroll
  for (int k = 0; k < C::SG; ++k) {
    const int idx = tid + BS * k;
    sG4[idx < EPB * C::SGV ? idx : EPB * C::SGV] = rG[k];
  }
#pragma unroll
  for (int k = 0; k < C::SO; ++k) {
    const int idx = tid + BS * k;
    if (idx < C::NOPS) sOp[idx] = rO[k];
  }
  __syncthreads();

  const V4<T>* el = sU + le * NPP;
  const T* g = reinterpret_cast<const T*>(sG4) + le * kGeoStride;
  T* const fq = sFq + le * C::XV * 4;

  // ---- 2a. quadrilateral-face fluxes (F_p, F_u) of the lane's face nodes;
  // the mirror state of a boundary face is blended in without branches
  if (active) {
#pragma unroll
    for (int s = 0; s < C::QSL; ++s) {
      const int f = i + NT * s;
      if (f < C::NQF) {
        const int ed = f / (Nq * Nq), jq = f - ed * Nq * Nq, j = jq / Nq, q = jq - j * Nq;
        const T w_in = quad_nbr(ed) >= 0 ? T(1) : T(0);
        const T nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
        const T zs = g[34 + ed];
        const T taup = tau_on * T(2) / zs;
        const T tauu = tau_on * zs * T(0.5);
        const V4<T> own = el[j * NT + edge_node(N, ed, q)];
        const V4<T> v = gq[s];
        const T pm = own.p;
        const T unm = nx * own.ux + ny * own.uy;
        const T pb = bsign * pm, ub = -bsign * unm;
        const T pp = pb + w_in * (v.p - pb);
        const T unp = ub + w_in * ((nx * v.ux + ny * v.uy + T(0) * v.uz) - ub);
        const T jp = pp - pm, jun = unp - unm;
        fq[2 * f] = T(0.5) * (taup * jp - jun);
        fq[2 * f + 1] = T(0.5) * (tauu * jun - jp);
      }
    }
  }

  // ---- 2b. vertical part and triangular faces of the node's line
  T Bp[Nq], Bz[Nq], Bx[Nq], By[Nq];
  {
    const T tzJ = g[4];
    V4<T> col[Nq];
#pragma unroll
    for (int m = 0; m < Nq; ++m) col[m] = el[m * NT + i];
#pragma unroll
    for (int j = 0; j < Nq; ++j) {
      const T tl = T(0.5 * (1.0 - RT::t[j])), th = T(0.5 * (1.0 + RT::t[j]));
      const T txJ = g[5] * tl + g[6] * th;
      const T tyJ = g[7] * tl + g[8] * th;
      T dP = 0, dX = 0, dY = 0, dZ = 0;
#pragma unroll
      for (int m = 0; m < Nq; ++m) {
        const T d = T(RT::Dt[j * Nq + m]);
        dP += d * col[m].p;
        dX += d * col[m].ux;
        dY += d * col[m].uy;
        dZ += d * col[m].uz;
      }
      T w = txJ * dX;
      w += tyJ * dY;
      w += tzJ * dZ;
      Bp[j] = -w;
      Bx[j] = -(txJ * dP);
      By[j] = -(tyJ * dP);
      Bz[j] = -(tzJ * dP);
    }
    // triangular faces: flux at the node (scaled by J_f), spread over the
    // levels by (M^1D)^-1 e_{0,N} (exact mass) or e_{0,N} / w_{0,N} (lumped)
    const bool lumped = (A.flags & kLumped) != 0;
#pragma unroll
    for (int face = 0; face < 2; ++face) {
      const T w_in = tri_nbr(face) >= 0 ? T(1) : T(0);
      const T* gf = g + 12 + 4 * face;
      const T Jf = gf[0], nx = gf[1], ny = gf[2], nz = gf[3];
      const T zs = g[32 + face];
      const T taup = tau_on * T(2) / zs;
      const T tauu = tau_on * zs * T(0.5);
      const V4<T> own = col[face * N];
      const V4<T> v = gt[face];
      const T pm = own.p;
      const T unm = nx * own.ux + ny * own.uy + nz * own.uz;
      const T pb = bsign * pm, ub = -bsign * unm;
      const T pp = pb + w_in * (v.p - pb);
      const T unp = ub + w_in * ((nx * v.ux + ny * v.uy + nz * v.uz) - ub);
      const T jp = pp - pm, jun = unp - unm;
      const T Fp = Jf * T(0.5) * (taup * jp - jun);
      const T Fu = Jf * T(0.5) * (tauu * jun - jp);
      const T wend = T(0.5 * N * (N + 1));  // 1 / w_0 = 1 / w_N of the GLL rule
#pragma unroll
      for (int j = 0; j < Nq; ++j) {
        const T gj = lumped ? ((face == 0 ? j == 0 : j == N) ? wend : T(0))
                            : T(face == 0 ? RT::g0[j] : RT::gN[j]);
        const T wu = gj * Fu;
        Bp[j] += gj * Fp;
        Bx[j] += wu * nx;
        By[j] += wu * ny;
        Bz[j] += wu * nz;
      }
    }
  }
  __syncthreads();  // quadrilateral-face fluxes complete

  // ---- 2c. quadrilateral-face lifts J^a E^a + J^b E^b (J_f linear along the edge)
  // (a rolled loop over the edges: unrolled, the scheduler hoists all their
  // LDS reads at once)
#pragma unroll 1
  for (int ed = 0; ed < 3; ++ed) {
    const int nbr = quad_nbr(ed);
    const T Ja = MODE == 2 && nbr <= -2 ? T(0) : g[20 + 4 * ed];
    const T Jb = MODE == 2 && nbr <= -2 ? T(0) : g[21 + 4 * ed];
    const T nx = g[22 + 4 * ed], ny = g[23 + 4 * ed];
    T c[Nq];
#pragma unroll
    for (int q = 0; q < Nq; ++q) c[q] = Ja * sEa[(ed * NT + i) * Nq + q] + Jb * sEb[(ed * NT + i) * Nq + q];
#pragma unroll
    for (int j = 0; j < Nq; ++j) {
      T sp = 0, su = 0;
#pragma unroll
      for (int q = 0; q < Nq; ++q) {
        const T* f = fq + 2 * ((ed * Nq + j) * Nq + q);
        sp += c[q] * f[0];
        su += c[q] * f[1];
      }
      Bp[j] += sp;
      Bx[j] += nx * su;
      By[j] += ny * su;
    }
  }
  if constexpr (MODE == 2) {
    // mortar faces: the mortar kernel's pre-lift contributions of the common
    // refinement (the buffer's range check returns zeros for other faces)
    constexpr int NTP = (NT + 3) / 4 * 4;
    const T* mb = static_cast<const T*>(A.mortB);
#pragma unroll
    for (int ed = 0; ed < 3; ++ed) {
      const int nbr = quad_nbr(ed);
      if (nbr <= -2) {
        const int64_t mo = int64_t(-2 - nbr);
        const T nxe = g[22 + 4 * ed], nye = g[23 + 4 * ed];
#pragma unroll
        for (int j = 0; j < Nq; ++j) {
          const T vp = mb[(mo * 2 * Nq + j) * NTP + i];
          const T vu = mb[(mo * 2 * Nq + Nq + j) * NTP + i];
          Bp[j] += vp;
          Bx[j] += nxe * vu;
          By[j] += nye * vu;
        }
      }
    }
  }
  // previous residual of the node's line, read while the lifts are applied
  const bool rd = (A.flags & kReadRes) != 0, wu = (A.flags & kWriteU) != 0;
  V4<T>* const res_el = static_cast<V4<T>*>(A.res) + e * NP;
  V4<T> rprev[Nq];
#pragma unroll
  for (int j = 0; j < Nq; ++j) rprev[j] = (rd && active) ? res_el[j * NT + i] : V4<T>{T(0), T(0), T(0), T(0)};
  __syncthreads();  // the fluxes are read: their region takes the pre-lift sums
  if (active) {
#pragma unroll
    for (int j = 0; j < Nq; ++j) sB[le * C::XV + j * NT + i] = V4<T>{Bp[j], Bz[j], Bx[j], By[j]};
  }
  __syncthreads();  // pre-lift sums complete

  // ---- 3. R = L^{tri,k} B on the node's row, then the horizontal part
  T Rp[Nq], Rz[Nq], Rx[Nq], Ry[Nq];
#pragma unroll
  for (int j = 0; j < Nq; ++j) Rp[j] = Rz[j] = Rx[j] = Ry[j] = T(0);
  {
    // over the columns m, unrolled three times (NT is a multiple of 3 at
    // orders 4 and 5): each step reads L[i][m] and the element's column m of
    // B at all levels (a broadcast); fully unrolled, the scheduler would hoist
    // every column's reads at once and spill
    const V4<T>* bl = sB + le * C::XV;
    const T* lc = reinterpret_cast<const T*>(sL4) + le * C::LS + i;
#pragma unroll 3
    for (int m = 0; m < NT; ++m) {
      const T l = lc[m * NT];
#pragma unroll
      for (int j = 0; j < Nq; ++j) {
        const V4<T> b = bl[j * NT + m];
        Rp[j] += l * b.p;
        Rz[j] += l * b.uz;
        Rx[j] += l * b.ux;
        Ry[j] += l * b.uy;
      }
    }
  }
  {
    //   R_p -= D_r (r_x u_x + r_y u_y) + D_s (s_x u_x + s_y u_y)
    //   R_x -= r_x D_r p + s_x D_s p ;  R_y -= r_y D_r p + s_y D_s p
    T aPr[Nq], aPs[Nq], aXr[Nq], aXs[Nq], aYr[Nq], aYs[Nq];
#pragma unroll
    for (int j = 0; j < Nq; ++j) aPr[j] = aPs[j] = aXr[j] = aXs[j] = aYr[j] = aYs[j] = T(0);
#pragma unroll 3
    for (int m = 0; m < NT; ++m) {
      const T dr = sDr[i * NT + m], ds = sDs[i * NT + m];
#pragma unroll
      for (int j = 0; j < Nq; ++j) {
        const V4<T> u = el[j * NT + m];
        aPr[j] += dr * u.p;
        aPs[j] += ds * u.p;
        aXr[j] += dr * u.ux;
        aXs[j] += ds * u.ux;
        aYr[j] += dr * u.uy;
        aYs[j] += ds * u.uy;
      }
    }
    const T rx = g[0], ry = g[1], sx = g[2], sy = g[3];
#pragma unroll
    for (int j = 0; j < Nq; ++j) {
      Rp[j] -= rx * aXr[j] + ry * aYr[j] + sx * aXs[j] + sy * aYs[j];
      Rx[j] -= rx * aPr[j] + sx * aPs[j];
      Ry[j] -= ry * aPr[j] + sy * aPs[j];
    }
  }

  // ---- 4. scaling, sources, update of the node's line
  if (!active) return;
  const T kap = g[9], irho = g[10];
#pragma unroll
  for (int j = 0; j < Nq; ++j) {
    Rp[j] *= kap;
    Rz[j] *= irho;
    Rx[j] *= irho;
    Ry[j] *= irho;
  }
  for (int s = 0; s < A.nsrc; ++s) {
    if (A.src_elem[s] == e) {
      const T* sv = static_cast<const T*>(A.srcvec) + s * NP + i;
      const T amp = T(A.src_amp[s]);
#pragma unroll
      for (int j = 0; j < Nq; ++j) Rp[j] += amp * sv[j * NT];
    }
  }
  const T ca = T(A.a), cb = T(A.b), dt = T(A.dt), cg = (A.flags & kGamma) ? T(A.g) : T(1);
  V4<T>* const out_el = static_cast<V4<T>*>(A.Uout) + e * NP;
  V4<T>* const rout_el = ((A.flags & kResOut) ? static_cast<V4<T>*>(A.rout) : static_cast<V4<T>*>(A.res)) + e * NP;
#pragma unroll
  for (int j = 0; j < Nq; ++j) {
    const V4<T> q = rprev[j];
    const V4<T> r{ca * q.p + dt * Rp[j], ca * q.uz + dt * Rz[j], ca * q.ux + dt * Rx[j], ca * q.uy + dt * Ry[j]};
    rout_el[j * NT + i] = r;
    if (wu) {
      const V4<T> u = el[j * NT + i];
      out_el[j * NT + i] =
          V4<T>{cg * u.p + cb * r.p, cg * u.uz + cb * r.uz, cg * u.ux + cb * r.ux, cg * u.uy + cb * r.uy};
    }
  }
}

// XCD-aware mapping of blocks to chunks (each XCD one contiguous range, so
// face neighbours share its L2)
__device__ __forceinline__ int xcd_chunk_n(int bid, int nb) {
  const int qd = nb / 8, rm = nb % 8, xcd = bid % 8, kk = bid / 8;
  return xcd < rm ? xcd * (qd + 1) + kk : rm * (qd + 1) + (xcd - rm) * qd + kk;
}

// at least two wavefronts per SIMD (at most 256 registers per lane)
template <int N, typename T, int MODE, int EPB>
__global__ void __launch_bounds__((NCfg<N, T, EPB>::BS), 2) wedge_node_stage(StageLaunch A) {
  wedge_node_chunk<N, T, MODE, EPB>(A, xcd_chunk_n(blockIdx.x, gridDim.x));
}

template <int N, typename T, int EPB>
__global__ void __launch_bounds__((NCfg<N, T, EPB>::BS), 2)
    wedge_node_batch(const StageLaunch* __restrict__ probs, const int2* __restrict__ work, int nwork) {
  const int w = xcd_chunk_n(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const int2 it = work[w];
  wedge_node_chunk<N, T, 0, EPB>(probs[it.x], it.y);
}

template <int N, typename T, int EPB>
hipError_t launch_node_t(const StageLaunch& a, hipStream_t st) {
  using C = NCfg<N, T, EPB>;
  const int64_t nchunks = (a.Kw + EPB - 1) / EPB;
  if (nchunks <= 0) return hipSuccess;
  if (a.nmort > 0)
    hipLaunchKernelGGL((wedge_node_stage<N, T, 2, EPB>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else if (a.Kt > 0)
    hipLaunchKernelGGL((wedge_node_stage<N, T, 1, EPB>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  else
    hipLaunchKernelGGL((wedge_node_stage<N, T, 0, EPB>), dim3(unsigned(nchunks)), dim3(C::BS), 0, st, a);
  return hipGetLastError();
}

template <int N, typename T, int EPB>
hipError_t launch_node_batch_t(const StageLaunch* probs, const int2* work, int nwork, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL((wedge_node_batch<N, T, EPB>), dim3(unsigned(nwork)), dim3(NCfg<N, T, EPB>::BS), 0, st, probs,
                     work, nwork);
  return hipGetLastError();
}

}  // namespace

// Elements per block of the node-lane kernel (FP32): the candidates the batch
// autotuner tries (index 0 is the single-problem kernel's), lane counts
// EPB Np_tri close to whole wavefronts.
int wedge_node_epb(int N, int bits, int idx) {
  // index 0 is the default: the fastest shape measured for one problem (order 4
  // on 73 728 wedges: 121 / 125 / 125 / 124 us for 8 / 17 / 12 / 4 elements
  // per block, and 8 also beside tetrahedra; order 5: 213 us at 12, 239-244 at
  // 9, 6, 3)
  static const int e4[kNodeEpbVariants] = {8, 17, 12, 4}, e5[kNodeEpbVariants] = {12, 9, 6, 3};
  if (bits != 32 || idx < 0 || idx >= kNodeEpbVariants) return 0;
  return N == 4 ? e4[idx] : (N == 5 ? e5[idx] : 0);
}

#define WDG_NODE_EPB(n, CALL)                          \
  switch (epb) {                                       \
    case (n == 4 ? 12 : 9): CALL(n, (n == 4 ? 12 : 9)); break;   \
    case (n == 4 ? 8 : 6): CALL(n, (n == 4 ? 8 : 6)); break;     \
    case (n == 4 ? 4 : 3): CALL(n, (n == 4 ? 4 : 3)); break;     \
    case (n == 4 ? 17 : 12): CALL(n, (n == 4 ? 17 : 12)); break; \
    default: break;                                    \
  }

hipError_t launch_wedge_node_stage(int N, int bits, int epb, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  if (bits != 32) return err;
#define WDG_CALL(n, E) err = launch_node_t<n, float, E>(a, st)
  if (N == 4) {
    WDG_NODE_EPB(4, WDG_CALL)
  } else if (N == 5) {
    WDG_NODE_EPB(5, WDG_CALL)
  }
#undef WDG_CALL
  return err;
}

hipError_t launch_wedge_node_batch(int N, int bits, int epb, const StageLaunch* probs, const int2* work, int nwork,
                                   hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
  if (bits != 32) return err;
#define WDG_CALL(n, E) err = launch_node_batch_t<n, float, E>(probs, work, nwork, st)
  if (N == 4) {
    WDG_NODE_EPB(4, WDG_CALL)
  } else if (N == 5) {
    WDG_NODE_EPB(5, WDG_CALL)
  }
#undef WDG_CALL
  return err;
}
#undef WDG_NODE_EPB

}  // namespace wdg
