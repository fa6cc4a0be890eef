// Tetrahedron stage kernel of libwdg: affine tetrahedra of hybrid meshes
// (standard nodal DG; they meet wedges at triangular faces, Sec. 3.1).
#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace wdg {
namespace {

// ---------------------------------------------------------------------------
// Tetrahedron stage kernel (affine tetrahedra, standard nodal DG)
//
// Lane (element, node i); a block of 256 lanes holds EPB = 256 / Np
// tetrahedra per chunk and loops over chunks (persistent), so the reference
// operators Dr, Ds, Dt and LIFT are staged in LDS once per block where they
// fit (read from memory otherwise).  Each lane loads its share of the next
// chunk's state, geometry and connectivity, and its node's previous residual,
// before the current chunk's work.  Per chunk:
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
    // eight loads in flight per lane before their stores: a few L2 round trips
    // instead of one per value
    constexpr int OPL = (C::NOPS + C::BS - 1) / C::BS;
    for (int b = 0; b < OPL; b += 8) {
      T v[8];
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        const int idx = threadIdx.x + C::BS * (b + l);
        v[l] = gops[idx < C::NOPS ? idx : 0];
      }
#pragma unroll
      for (int l = 0; l < 8; ++l) {
        const int idx = threadIdx.x + C::BS * (b + l);
        if (idx < C::NOPS) sOps[idx] = v[l];
      }
    }
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
  // A chunk's state, geometry and connectivity are loaded one chunk ahead,
  // while the current chunk computes (one node, GL geometry and CL
  // connectivity values per lane).
  static_assert(EPB * NP <= C::BS, "one node per lane");
  constexpr int GL = (EPB * kTetGeoStride + C::BS - 1) / C::BS, CL = (EPB * kTetConnStride + C::BS - 1) / C::BS;
  struct Pre {
    V4<T> u;
    T g[GL];
    int c[CL];
  };
  // (indices past the chunk read its first value, a valid address; those
  // values are never stored)
  auto fetch = [&](int64_t c) -> Pre {
    const int64_t f0 = c * EPB;
    const int n = int(A.Kt - f0 < EPB ? A.Kt - f0 : EPB);
    Pre p;
    p.u = Uin[tb + f0 * NP + (tid < n * NP ? tid : 0)];
#pragma unroll
    for (int l = 0; l < GL; ++l) {
      const int idx = tid + C::BS * l;
      p.g[l] = geo[f0 * kTetGeoStride + (idx < n * kTetGeoStride ? idx : 0)];
    }
#pragma unroll
    for (int l = 0; l < CL; ++l) {
      const int idx = tid + C::BS * l;
      p.c[l] = conn[f0 * kTetConnStride + (idx < n * kTetConnStride ? idx : 0)];
    }
    return p;
  };
  Pre pre{};
  if (int64_t(blockIdx.x) < nchunks) pre = fetch(blockIdx.x);

  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const int64_t e0 = chunk * EPB;
    const int nE = int(A.Kt - e0 < EPB ? A.Kt - e0 : EPB);
    const bool active = tid < EPB * NP && le < nE;
    const int64_t e = e0 + le;
    const int64_t gi = tb + e * NP + i;
    // the previous residual of this lane's node, read early
    V4<T> rprev{T(0), T(0), T(0), T(0)};
    if (rd && active) rprev = res[gi];
    __syncthreads();  // the previous chunk is done with LDS
    if (tid < nE * NP) sU[tid] = pre.u;
#pragma unroll
    for (int l = 0; l < GL; ++l)
      if (tid + C::BS * l < nE * kTetGeoStride) sG[tid + C::BS * l] = pre.g[l];
#pragma unroll
    for (int l = 0; l < CL; ++l)
      if (tid + C::BS * l < nE * kTetConnStride) sC[tid + C::BS * l] = pre.c[l];
    if (chunk + gridDim.x < nchunks) pre = fetch(chunk + gridDim.x);
    __syncthreads();

    const T* g = sG + le * kTetGeoStride;
    const int* cn = sC + le * kTetConnStride;
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

    const T ca = T(A.a), cb = T(A.b), dtt = T(A.dt), cg = T(A.g);
    V4<T> r{dtt * Rp, dtt * Rz, dtt * Rx, dtt * Ry};
    if (rd) {
      r.p += ca * rprev.p;
      r.uz += ca * rprev.uz;
      r.ux += ca * rprev.ux;
      r.uy += ca * rprev.uy;
    }
    res[gi] = r;
    if (wu) {
      const V4<T> u = sU[le * NP + i];
      const T gg = (A.flags & kGamma) ? cg : T(1);
      Uout[gi] = V4<T>{gg * u.p + cb * r.p, gg * u.uz + cb * r.uz, gg * u.ux + cb * r.ux, gg * u.uy + cb * r.uy};
    }
  }
}

// ---------------------------------------------------------------------------
// Tetrahedron stage kernel on the matrix cores (default)
//
// The same stage as tet_stage, with the reference-operator products of a chunk
// of EPB tetrahedra done as dense contractions on MFMA (16x16x4, FP32 or
// FP64):
//   [D_r p, D_r(r.u)], [D_s p, D_s(s.u)], [D_t p, D_t(t.u)]
//       = D_o (Np x Np) times the chunk's (p, o.u) column pairs (2 EPB columns),
//   LIFT (Np x 4 Np_tri) times the chunk's face fluxes
//       (J_f/J) (F_p, F_u n_x, F_u n_y, F_u n_z) (4 EPB columns).
// A block holds one wavefront per 16-row tile of the operators (Np rows
// padded to a multiple of 16); each wavefront keeps its rows of D_r, D_s, D_t
// and LIFT in registers (the MFMA A operand) for the whole persistent kernel,
// so only the chunk's data (the B operand) is read from LDS: one value per
// lane per MFMA, against three operator values and a 4-vector per node and
// operator column in the per-node dot products of tet_stage.  The pointwise
// parts (geometry, fluxes, scaling, sources, update) run over the chunk's
// nodes on all lanes.
// ---------------------------------------------------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  using type = f32x4_t;
};
template <>
struct MfmaAcc<double> {
  using type = f64x4_t;
};

// D += A B for a 16x4 A and a 4x16 B: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[mfma_row<T>(l / 16, r)][l % 16], r = 0..3
// (FP32: rows 4 (l / 16) + r; FP64: rows 4 r + l / 16)
template <typename T>
__device__ __forceinline__ int mfma_row(int lk, int r) {
  return sizeof(T) == 4 ? 4 * lk + r : 4 * r + lk;
}
template <typename T>
__device__ __forceinline__ typename MfmaAcc<T>::type mfma16x16x4(T a, T b, typename MfmaAcc<T>::type c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int N, typename T>
struct MCfg {
  static constexpr int NT = TDim<N>::NT, NP = TDim<N>::NP, FN = 4 * NT;
  static constexpr int RT = (NP + 15) / 16;  // row tiles: one wavefront each
  static constexpr int BS = 64 * RT;
  // tetrahedra per chunk: the (p, o.u) column pairs fill whole 16-column tiles
  static constexpr int EPB = N <= 2 ? 16 : 8;
  static constexpr int KV = (NP + 3) / 4, KL = (FN + 3) / 4;  // k-steps
  static constexpr int VCT = 2 * EPB / 16, LCT = 4 * EPB / 16;  // column tiles
  static constexpr int NN = EPB * NP, NPL = (NN + BS - 1) / BS;  // nodes per lane
  static constexpr int NF = EPB * FN, FPL = (NF + BS - 1) / BS;  // face nodes per lane
  static constexpr int GL = (EPB * kTetGeoStride + BS - 1) / BS, CL = (EPB * kTetConnStride + BS - 1) / BS;
  static_assert(2 * EPB % 16 == 0, "whole column tiles");
};

template <int N, typename T>
__global__ void __launch_bounds__((MCfg<N, T>::BS)) tet_stage_mfma(StageLaunch A) {
  using C = MCfg<N, T>;
  using Acc = typename MfmaAcc<T>::type;
  constexpr int NT = C::NT, NP = C::NP, EPB = C::EPB, BS = C::BS, FN = C::FN;
  constexpr int NPW = Dim<N>::NP;
  constexpr int V4B = 4 * int(sizeof(T));
  __shared__ V4<T> sU[C::NN];
  __shared__ Q4<T> sW[C::NN];
  __shared__ V4<T> sF[C::NF];
  __shared__ V4<T> sD[2 * C::NN];  // per node: D_r p, D_s p, D_t p, div u; lifted F_p, F_u n_x, F_u n_y, F_u n_z
  __shared__ T sG[EPB * kTetGeoStride];
  __shared__ int sC[2][EPB * kTetConnStride];  // connectivity of this chunk and of the next one

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  // this wavefront's 16 operator rows as MFMA A operands, kept for the whole kernel
  const T* __restrict__ gops = static_cast<const T*>(A.opsT);
  const int orow = wave * 16 + lr;
  T aD[3][C::KV], aL[C::KL];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
#pragma unroll
    for (int ks = 0; ks < C::KV; ++ks) {
      const int col = 4 * ks + lk;
      const bool ok = orow < NP && col < NP;
      const T v = gops[ok ? o * NP * NP + orow * NP + col : 0];
      aD[o][ks] = ok ? v : T(0);
    }
  }
#pragma unroll
  for (int ks = 0; ks < C::KL; ++ks) {
    const int col = 4 * ks + lk;
    const bool ok = orow < NP && col < FN;
    const T v = gops[ok ? 3 * NP * NP + orow * FN + col : 0];
    aL[ks] = ok ? v : T(0);
  }

  const V4<T>* __restrict__ Uin = static_cast<const V4<T>*>(A.Uin);
  const T* __restrict__ geo = static_cast<const T*>(A.geoT);
  const int* __restrict__ conn = A.connT;
  const int64_t tb = A.Kw * NPW;  // first tetrahedron node
  const T bsign = (A.flags & kDirichlet) ? T(-1) : T(1);
  const T tau_on = (A.flags & kCentral) ? T(0) : T(1);
  const bool rd = (A.flags & kReadRes) != 0, wu = (A.flags & kWriteU) != 0;
  const int64_t nchunks = (A.Kt + EPB - 1) / EPB;

  // Loads run ahead of their use: a chunk's state and geometry one chunk
  // ahead (through the buffer's range check: zeros past the last
  // tetrahedron; geometry indices past the chunk read its first value, never
  // stored), its connectivity two chunks ahead, so that its neighbour states
  // and mortar fluxes can be gathered during the previous chunk.
  struct Pre {
    V4<T> u[C::NPL];
    T g[C::GL];
  };
  auto fetch = [&](int64_t ch) -> Pre {
    const int64_t f0 = ch * EPB;
    const int n = int(A.Kt - f0 < EPB ? A.Kt - f0 : EPB);
    Pre p;
    const auto bu = chunk_rsrc(Uin + tb + f0 * NP, int64_t(n) * NP * V4B);
#pragma unroll
    for (int l = 0; l < C::NPL; ++l) p.u[l] = bload<T>(bu, tid + BS * l);
#pragma unroll
    for (int l = 0; l < C::GL; ++l) {
      const int idx = tid + BS * l;
      p.g[l] = geo[f0 * kTetGeoStride + (idx < n * kTetGeoStride ? idx : 0)];
    }
    return p;
  };
  struct PreC {
    int c[C::CL];
  };
  auto fetch_conn = [&](int64_t ch) -> PreC {
    PreC p;
    const int64_t f0 = ch < nchunks ? ch * EPB : 0;
    const int n = int(A.Kt - f0 < EPB ? A.Kt - f0 : EPB);
#pragma unroll
    for (int l = 0; l < C::CL; ++l) {
      const int idx = tid + BS * l;
      p.c[l] = conn[f0 * kTetConnStride + (idx < n * kTetConnStride ? idx : 0)];
    }
    return p;
  };
  auto put_conn = [&](int buf, const PreC& p) {
#pragma unroll
    for (int l = 0; l < C::CL; ++l)
      if (tid + BS * l < EPB * kTetConnStride) sC[buf][tid + BS * l] = p.c[l];
  };
  // Neighbour state at every face node of chunk ch (connectivity in sC[buf])
  // and, on mortar faces, the mortar's nodal flux: issued without branches
  // (lanes past the chunk read node 0 and the state as a stand-in flux).
  V4<T> nbg[C::FPL];
  T mfp[C::FPL], mfu[C::FPL];
  const T* __restrict__ mortF = static_cast<const T*>(A.mortF);
  auto gather = [&](int64_t ch, int buf) {
    const int64_t f0 = ch * EPB;
    const int n = int(A.Kt - f0 < EPB ? A.Kt - f0 : EPB);
#pragma unroll
    for (int l = 0; l < C::FPL; ++l) {
      const int q0 = tid + BS * l;
      const bool ok = q0 < C::NF && q0 / FN < n;
      const int q = ok ? q0 : 0;
      const int le = q / FN, qq = q - le * FN;
      const int f = qq / NT, m = qq - f * NT;
      const int* cn = sC[buf] + le * kTetConnStride;
      const int code = cn[4];
      const int nbr = cn[f];
      const int pc = (code >> (5 * f)) & 7, nf = (code >> (5 * f + 3)) & 3;
      const int fn = face_perm<N>(pc, m);
      const int64_t src = nbr >= 0 ? int64_t(nbr) : A.Kw + f0 + le;
      const int64_t gi = src >= A.Kw ? tb + (src - A.Kw) * NP + tet_face_node<N>(nf, fn)
                                     : src * NPW + (nf == 1 ? N * NT : 0) + fn;
      nbg[l] = Uin[ok ? gi : 0];
      const bool mort = ok && nbr <= -2;
      const T* mf = mort ? mortF + int64_t(-2 - nbr) * 2 * NT + m : reinterpret_cast<const T*>(Uin);
      mfp[l] = mf[0];
      mfu[l] = mf[mort ? NT : 0];
    }
  };
  // the sources in this launch's elements (applied in the update of the chunks that hold them)
  int64_t src_lo = INT64_MAX, src_hi = -1;
  for (int s = 0; s < A.nsrc; ++s) {
    const int64_t se = A.src_elem[s];
    src_lo = se < src_lo ? se : src_lo;
    src_hi = se > src_hi ? se : src_hi;
  }

  Pre pre{};
  PreC prec{};
  if (int64_t(blockIdx.x) < nchunks) {
    pre = fetch(blockIdx.x);
    put_conn(0, fetch_conn(blockIdx.x));
    prec = fetch_conn(int64_t(blockIdx.x) + gridDim.x);
    __syncthreads();
    gather(blockIdx.x, 0);
  }

  int buf = 0;
  for (int64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x, buf ^= 1) {
    const int64_t e0 = chunk * EPB;
    const int nE = int(A.Kt - e0 < EPB ? A.Kt - e0 : EPB);
    const int64_t next = chunk + gridDim.x;
    const int nn = nE * NP;
    V4<T>* const res_chunk = static_cast<V4<T>*>(A.res) + tb + e0 * NP;
    const auto bres_in = chunk_rsrc(res_chunk, rd ? int64_t(nn) * V4B : 0);
    const auto bres = chunk_rsrc(res_chunk, int64_t(nn) * V4B);
    const auto bout = chunk_rsrc(static_cast<V4<T>*>(A.Uout) + tb + e0 * NP, int64_t(nn) * V4B);
    // the previous residual of this lane's nodes, read early (zeros in the first stage)
    V4<T> rprev[C::NPL];
#pragma unroll
    for (int l = 0; l < C::NPL; ++l) rprev[l] = bload<T>(bres_in, tid + BS * l);
    __syncthreads();  // the previous chunk is done with LDS
#pragma unroll
    for (int l = 0; l < C::NPL; ++l)
      if (tid + BS * l < C::NN) sU[tid + BS * l] = pre.u[l];
#pragma unroll
    for (int l = 0; l < C::GL; ++l)
      if (tid + BS * l < EPB * kTetGeoStride) sG[tid + BS * l] = pre.g[l];
    // the next chunk's connectivity, loaded one chunk ago
    put_conn(buf ^ 1, prec);
    if (next < nchunks) {
      pre = fetch(next);
      prec = fetch_conn(next + gridDim.x);
    }
    __syncthreads();

    // (p, r.u, s.u, t.u) per node: div u = D_r (r.u) + D_s (s.u) + D_t (t.u)
#pragma unroll
    for (int l = 0; l < C::NPL; ++l) {
      const int n = tid + BS * l;
      if (n < C::NN) {
        const T* g = sG + (n / NP) * kTetGeoStride;
        const V4<T> v = sU[n];
        sW[n] = Q4<T>{v.p, g[0] * v.ux + g[1] * v.uy + g[2] * v.uz, g[3] * v.ux + g[4] * v.uy + g[5] * v.uz,
                      g[6] * v.ux + g[7] * v.uy + g[8] * v.uz};
      }
    }
    // face fluxes (J_f / J) (F_p, F_u n) at the 4 Np_tri face nodes of every tetrahedron
#pragma unroll
    for (int l = 0; l < C::FPL; ++l) {
      const int q = tid + BS * l;
      if (q < C::NF) {
        const int le = q / FN, qq = q - le * FN;
        const int f = qq / NT, m = qq - f * NT;
        V4<T> out{T(0), T(0), T(0), T(0)};
        if (le < nE) {
          const T* g = sG + le * kTetGeoStride;
          const int nbr = sC[buf][le * kTetConnStride + f];
          const T w_in = nbr >= 0 ? T(1) : T(0);
          const V4<T> own = sU[le * NP + tet_face_node<N>(f, m)];
          const V4<T> nb = nbg[l];
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
            Fp = mfp[l];
            Fu = mfu[l];
          }
          const T su = Fs * Fu;
          out = V4<T>{Fs * Fp, su * nx, su * ny, su * nz};
        }
        sF[q] = out;
      }
    }
    __syncthreads();

    // reference-operator products on the matrix cores: this wavefront's rows
    // 16 w .. 16 w + 15 of every column tile
    {
      const T* sWf = reinterpret_cast<const T*>(sW);
      const T* sFf = reinterpret_cast<const T*>(sF);
      T* sDf = reinterpret_cast<T*>(sD);
#pragma unroll
      for (int ct = 0; ct < C::VCT; ++ct) {
        const int col = ct * 16 + lr;  // column (tetrahedron, p or o.u) of this lane's B and D values
        const int ce = col >> 1, which = col & 1;
        Acc acc[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) acc[o] = Acc{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < C::KV; ++ks) {
          const int k = 4 * ks + lk;
          // rows k >= Np of B meet zero columns of A: any finite value will do
          const int base = (ce * NP + (k < NP ? k : 0)) * 4;
#pragma unroll
          for (int o = 0; o < 3; ++o) acc[o] = mfma16x16x4<T>(aD[o][ks], sWf[base + (which ? 1 + o : 0)], acc[o]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wave * 16 + mfma_row<T>(lk, r);
          if (i < NP) {
            T* d = sDf + (ce * NP + i) * 8;
            if (which == 0) {
              d[0] = acc[0][r];
              d[1] = acc[1][r];
              d[2] = acc[2][r];
            } else {
              d[3] = acc[0][r] + acc[1][r] + acc[2][r];
            }
          }
        }
      }
#pragma unroll
      for (int ct = 0; ct < C::LCT; ++ct) {
        const int col = ct * 16 + lr;  // column (tetrahedron, component) of the fluxes
        const int ce = col >> 2, cc = col & 3;
        Acc acc = Acc{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < C::KL; ++ks) {
          const int k = 4 * ks + lk;
          acc = mfma16x16x4<T>(aL[ks], sFf[(ce * FN + (k < FN ? k : 0)) * 4 + cc], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wave * 16 + mfma_row<T>(lk, r);
          if (i < NP) sDf[(ce * NP + i) * 8 + 4 + cc] = acc[r];
        }
      }
    }
    // the next chunk's neighbour gathers, in flight during this update and
    // the next chunk's staging (its connectivity went to LDS before the
    // barrier ahead of the flux phase)
    if (next < nchunks) gather(next, buf ^ 1);
    __syncthreads();

    // right-hand side, sources and the low-storage update, node-contiguous
    const T ca = T(A.a), cb = T(A.b), dtt = T(A.dt), cg = (A.flags & kGamma) ? T(A.g) : T(1);
    const bool src_here = src_hi >= A.Kw + e0 && src_lo < A.Kw + e0 + nE;
#pragma unroll
    for (int l = 0; l < C::NPL; ++l) {
      const int n = tid + BS * l;
      if (n < nn) {
        const int le = n / NP, i = n - le * NP;
        const int64_t e = e0 + le;
        const T* g = sG + le * kTetGeoStride;
        const T* d = reinterpret_cast<const T*>(sD) + n * 8;
        const T kap = g[9], irho = g[10];
        T Rp = kap * (d[4] - d[3]);
        const T Rx = irho * (d[5] - (g[0] * d[0] + g[3] * d[1] + g[6] * d[2]));
        const T Ry = irho * (d[6] - (g[1] * d[0] + g[4] * d[1] + g[7] * d[2]));
        const T Rz = irho * (d[7] - (g[2] * d[0] + g[5] * d[1] + g[8] * d[2]));
        if (src_here)
          for (int s = 0; s < A.nsrc; ++s)
            if (A.src_elem[s] == A.Kw + e) Rp += T(A.src_amp[s]) * static_cast<const T*>(A.srcvec)[s * NPW + i];
        const V4<T> q = rprev[l];
        const V4<T> r{ca * q.p + dtt * Rp, ca * q.uz + dtt * Rz, ca * q.ux + dtt * Rx, ca * q.uy + dtt * Ry};
        bstore<T>(bres, n, r);
        if (wu) {
          const V4<T> u = sU[n];
          bstore<T>(bout, n, V4<T>{cg * u.p + cb * r.p, cg * u.uz + cb * r.uz, cg * u.ux + cb * r.ux,
                                   cg * u.uy + cb * r.uy});
        }
      }
    }
  }
}

#ifndef WDG_TET_BLOCKS
#define WDG_TET_BLOCKS 2048
#endif
constexpr int64_t kTetBlocks = WDG_TET_BLOCKS;

template <int N, typename T>
hipError_t launch_tet_stage_t(const StageLaunch& a, hipStream_t st) {
  if (a.Kt <= 0) return hipSuccess;
  using TC = TCfg<N, T>;
  const int64_t tchunks = (a.Kt + TC::EPB - 1) / TC::EPB;
  // persistent over chunks: each block stages the operators once (1024 blocks,
  // the resident count at four per CU, measured 1 us slower on the N = 4
  // hybrid mesh of 29 520 tetrahedra)
  const int64_t cap = a.tet_blocks > 0 ? int64_t(a.tet_blocks) : kTetBlocks;
  if (a.flags & kTetValu) {
    const unsigned grid = unsigned(tchunks < cap ? tchunks : cap);
    hipLaunchKernelGGL((tet_stage<N, T>), dim3(grid), dim3(TC::BS), 0, st, a);
  } else {
    using MC = MCfg<N, T>;
    const int64_t mchunks = (a.Kt + MC::EPB - 1) / MC::EPB;
    // every block loads its wavefronts' operator rows once: by default launch
    // only the blocks that are resident at once on the device
    static const int64_t resident = [] {
      int per_cu = 0, dev = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tet_stage_mfma<N, T>, MC::BS, 0) != hipSuccess ||
          hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return kTetBlocks;
      return int64_t(per_cu > 0 ? per_cu : 1) * int64_t(cus > 0 ? cus : 1);
    }();
    const int64_t mcap = a.tet_blocks > 0 ? int64_t(a.tet_blocks) : resident;
    const unsigned grid = unsigned(mchunks < mcap ? mchunks : mcap);
    hipLaunchKernelGGL((tet_stage_mfma<N, T>), dim3(grid), dim3(MC::BS), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tet_stage(int N, int bits, const StageLaunch& a, hipStream_t st) {
  hipError_t err = hipErrorInvalidValue;
#define WDG_STAGE(n, T) err = launch_tet_stage_t<n, T>(a, st)
  WDG_DISPATCH_N(N, bits, WDG_STAGE)
#undef WDG_STAGE
  return err;
}

}  // namespace wdg
