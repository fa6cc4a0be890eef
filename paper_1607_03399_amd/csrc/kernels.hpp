// Internal interface between the host runtime and the HIP kernels of libwdg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct wdg_ctx;

namespace wdg {

using wdg_ctx_fwd = ::wdg_ctx;

// Per-element record of geometric factors and material (values of type T):
//   0 r_x, 1 r_y, 2 s_x, 3 s_y, 4 t_zJ, 5/6 t_xJ at t=-1/+1, 7/8 t_yJ at t=-1/+1,
//   9 kappa, 10 1/rho, 11 rho c, 12..15 bottom (J_f, n), 16..19 top (J_f, n),
//   20+4e.. quad face e: J_f at first/second edge vertex, n_x, n_y,
//   32..36 rho c + (rho c of the neighbour, or own on the boundary) per face
//   (bottom, top, quad 0..2), 37..39 J_tri h_v / 2 (the M^{tri,k} weights).
constexpr int kGeoStride = 40;
// Per-element FP64 auxiliary record: 0..2 J_tri h_v / 2 (M^{tri,k} weights), 3 J_tri, 4 kappa, 5 rho.
constexpr int kAuxStride = 8;
// Per-element connectivity (int32): 0..4 neighbour of bottom, top, quad 0..2 (-1: boundary);
// 5 packed codes: bits 0-2 / 3-5 vertex permutation of the bottom / top neighbour face,
// bit 6 / 7 set when that neighbour face is the neighbour's top triangle, bits 8+2e..9+2e
// neighbour edge of quad face e, bits 14-15 / 16-17 the neighbour's face when the bottom /
// top neighbour is a tetrahedron (global id >= number of wedges).
constexpr int kConnStride = 8;
constexpr int kMaxSources = 8;
// Per-tetrahedron record (values of type T): 0..8 r_x r_y r_z s_x s_y s_z t_x t_y t_z,
// 9 kappa, 10 1/rho, 11 rho c, 12+4f.. face f: J_f / J, n_x, n_y, n_z,
// 28+f rho c + (rho c of the neighbour, or own on the boundary) across face f.
constexpr int kTetGeoStride = 32;
// Per-tetrahedron connectivity (int32): 0..3 neighbour across face f (global element id,
// wedges first; -1 boundary); 4 packed codes, 5 bits per face: bits 5f..5f+2 vertex
// permutation, 5f+3..5f+4 the neighbour's face (wedge: 0 bottom, 1 top; tetrahedron: 0..3).
constexpr int kTetConnStride = 8;
// Per-tetrahedron FP64 auxiliary record: 0 J, 1 kappa, 2 rho.
constexpr int kTetAuxStride = 4;
// Mortars: a wedge quadrilateral face covered by two tetrahedron triangles
// (wedge conn slot 2+e = -2 - m; tetrahedron conn slot f = -2 - (2 m + side)).
// Integer record: 0 wedge, 1 edge e, 2 diagonal (0: A0-A2, 1: A1-A3), 3/5 tetrahedron
// below/above the diagonal (global id), 4/6 its face.
constexpr int kMortIntStride = 8;
// Value record (FP64): 0..3 heights zb_a zb_b zt_a zt_b of the corners, 4 edge length,
// 5/6 outward normal of the wedge, 7..15 / 16..24 barycentrics of the tetrahedron faces
// below / above the diagonal as affine functions of (xi, z) (3 per vertex: xi, z, 1),
// 25/26 1/(area/2) of those faces, 27/28 rho c of the wedge plus that of the tetrahedron.
constexpr int kMortGeoStride = 32;
// Gauss points along the edge of a mortar face (the host's integration of the
// coupling matrices): the integrand is rational in the edge parameter; on
// layered meshes with interfaces perturbed by 0.3 of the layer thickness
// 4N + 8 points reach FP64 rounding.
constexpr int mort_nx(int N) { return 4 * N + 8; }
// Coupling matrix of one side of a mortar: the (N+1)^2 wedge face nodes
// (level-major) and the Np_tri tetrahedron face nodes; both sides' lower
// triangles (packed by columns) per mortar, padded to a multiple of 4 values.
__host__ __device__ constexpr int mort_core_n(int N) { return (N + 1) * (N + 1) + (N + 1) * (N + 2) / 2; }
__host__ __device__ constexpr int mort_core_stride(int N) {
  return (mort_core_n(N) * (mort_core_n(N) + 1) + 3) / 4 * 4;
}

enum StageFlags : int {
  kReadRes = 1,    // res = a res + dt rhs (else res = dt rhs)
  kWriteU = 2,     // U_out = U_in + b res
  kDirichlet = 4,  // else rigid wall
  kCentral = 8,    // else upwind flux
  kLumped = 16,    // Gauss-Lobatto mass in t: (M^1D)^-1 e_{0,N} becomes e_{0,N} / w_{0,N}
  kResOut = 32,    // res' goes to rout instead of back into res, which is then only read (wedges)
  kGamma = 64,     // U_out = g U_in + b res' (else g = 1)
  kLayerMarch = 128,  // wedge meshes: vertical neighbours inside a chunk from LDS
  kGrad = 256,        // wedge meshes, adjoint sweep: also accumulate the stage's gradient terms
  kTetValu = 512,     // tetrahedra: per-node dot products on the vector units (else MFMA)
  kColumnMarch = 1024,  // wedge meshes: one block marches each column (cols), with kLayerMarch
};

// One stage over the whole mesh.  State buffers hold wedges first (Kw x Np_wedge
// nodes), then tetrahedra (Kt x Np_tet nodes), one 4-vector per node.
struct StageLaunch {
  const void* Uin;
  void* Uout;
  void* res;
  const void* geo;   // wedges
  const void* L;     // wedges: triangular operator record (lift_packed, lift_stride)
  const int* conn;
  const void* geoT;  // tetrahedra
  const int* connT;
  const void* opsT;  // tetrahedron operators: Dr, Ds, Dt (Np x Np each), LIFT (Np x 4 Np_tri)
  const void* opsW;  // N >= 4 wedges: reference rows D_r, D_s (Np_tri x Np_tri), E^a, E^b ([edge][Np_tri][N+1])
  const void* srcvec;  // kMaxSources x Np_wedge (a tetrahedron source uses the first Np_tet)
  const int* mortI;    // mortars: kMortIntStride ints each
  const void* mortG;   // kMortGeoStride FP64 values each
  const void* mortTab; // reference tables of the mortar outputs, type T (see mortar_table_size)
  const void* mortC;   // per mortar: mort_core_stride values of type T (coupling matrices)
  void* mortB;         // per mortar: wedge pre-lift contributions [p, u][Nq][Np_tri padded to 4]
  void* mortF;         // per mortar side: equivalent nodal tetrahedron-face flux [p, u][Np_tri]
  int64_t nmort;
  int src_elem[kMaxSources];
  double src_amp[kMaxSources];
  int nsrc;
  // res' = a res + dt rhs;  U_out = g U_in + b res'  (the forward stages use g = 1)
  double a, b, dt, g;
  void* rout;  // kResOut: the updated residual, same layout as res
  // kGrad: the forward stage input U_s and the forward residual res_s after that
  // stage, the forward stage's coefficient b_s, gradient accumulators
  const void* gUs;
  const void* gRs;
  double gb;
  void* gacc;  // kGrad: gradient accumulators (kGradRecord values of the state precision per wedge)
  int64_t Kw, Kt;
  int flags;
  int tet_blocks;  // tetrahedron kernel: number of persistent blocks (0: default)
  // kColumnMarch: the column segments (first element, number of layers, at
  // most two chunks of the stage kernel; elements consecutive from the
  // bottom, each the one below's top neighbour)
  const int2* cols;
  int ncols;
};

// Whether order N stores (M^{tri,k})^-1 as its lower triangle (N <= 3: kept
// for wdg_element_data; the stage kernels factor M^{tri,k} from the geometry
// record's vertex weights instead of reading it) instead of the lift
// L^{tri,k} = (M^{tri,k})^-1 M^tri (Np_tri^2 values, column by column: entry
// (r, c) at c Np_tri + r).
constexpr bool lift_packed(int N) { return N <= 3; }
// Per-element stride (values) of that record, padded to a multiple of 4.
int lift_stride(int N);

hipError_t launch_setup(int N, int bits, int64_t K, const double* dX, const double* dMv, const double* dMtri,
                        void* dGeo, void* dL, double* dAux, hipStream_t st);
hipError_t launch_material(int bits, int64_t K, const double* dc, const double* drho, const int* dConn, void* dGeo,
                           double* dAux, hipStream_t st);
// One stage: the mortar kernel (meshes with mortars), the wedge kernel, then
// (hybrid meshes) the tetrahedron kernel, on the same stream.
hipError_t launch_mortar_stage(int N, int bits, const StageLaunch& a, hipStream_t st);
hipError_t launch_wedge_stage(int N, int bits, const StageLaunch& a, hipStream_t st);
hipError_t launch_tet_stage(int N, int bits, const StageLaunch& a, hipStream_t st);
// N >= 4, FP32: the wedge stage with one lane per triangle node
// (wedge_node.hip), epb elements per block, one of
// wedge_node_epb(N, bits, 0..kNodeEpbVariants-1) (index 0: the default; 0
// returned where there is no such kernel).  Not for layer marching or the
// adjoint sweep.
constexpr int kNodeEpbVariants = 4;
int wedge_node_epb(int N, int bits, int idx);
hipError_t launch_wedge_node_stage(int N, int bits, int epb, const StageLaunch& a, hipStream_t st);
hipError_t launch_wedge_node_batch(int N, int bits, int epb, const StageLaunch* probs, const int2* work, int nwork,
                                   hipStream_t st);
// Number of values of the mortar reference tables of order N, in this order:
// Minv1 (Nq x Nq, (M^1D)^-1), ME (3 x Np_tri x Nq: (M^tri)^-1 restricted to the
// columns of edge e's nodes, [e][i][q]), MTI (Np_tri x Np_tri, (M^tri)^-1).
int mortar_table_size(int N);
// Batches of independent wedge meshes (one launch per order and stage).
// Per-problem parameters of the stage records written on the device.
struct BatchParam {
  void* U[2];        // the problem's ping-pong state buffers
  int64_t cur0;      // buffer index holding the state at batch step 0
  double dt, t0;     // time step; time at batch step 0
  int flags;         // boundary / flux / mass flags
  int nsrc;
};
// Elements per chunk of the wedge stage kernel (work granularity).
int wedge_chunk_elems(int N, int bits);
// One stage of every problem of order N: one block per chunk (problem, chunk)
// of work; wpe (1 or 2) selects the register budget of the kernel.
hipError_t launch_wedge_batch(int N, int bits, const StageLaunch* probs, const int2* work, int nwork, int wpe,
                              hipStream_t st);
// Stage s (coefficients a, b) of batch step *counter: writes the
// stage-dependent fields of every problem's stage record; source amplitudes
// come from amp[((step * 5 + s) * nprob + problem) * kMaxSources + source],
// tabulated on the host with the single-problem driver's own arithmetic.
hipError_t launch_batch_prepare(int nprob, StageLaunch* probs, const BatchParam* par, const int64_t* counter, int s,
                                double a, double b, const double* amp, hipStream_t st);
hipError_t launch_batch_advance(int64_t* counter, hipStream_t st);

// Adjoint gradient (wedge meshes).  Per reverse stage the stage kernel (kGrad)
// accumulates into gacc (per wedge: kGradStride values of the state precision;
// FP32 also their kGradStride Kahan compensations): the mass terms' dJ/dc and
// dJ/drho, and per face (bottom, top, quadrilaterals 0..2) the own side's
// share of dJ/dZ, dt (dtau_p/dZ 1/2 int sig_p [p] + dtau_u/dZ 1/2 int sig_un
// [u_n]) of the forward stage input Us (the penalties' derivatives are fixed
// during the sweep).  kGradTerms: the partial sums behind them.
constexpr int kGradStride = 7;
constexpr int kGradTerms = 12;
template <typename T>
constexpr int kGradRecord = sizeof(T) == 4 ? 2 * kGradStride : kGradStride;  // values per wedge
// Gradient with respect to c and rho from the accumulated terms and the penalty
// derivatives, in the state precision; written to gc and grho as FP64.
hipError_t launch_grad_combine(int bits, int64_t K, const void* gacc, const void* geo, const int* conn, int flags,
                               double* gc, double* grho, hipStream_t st);
// Receiver injection: for receiver r (first node base[r], vector vec[r] of NP values),
// U += w[r] vec[r] and S += sb w[r] vec[r] on the pressure.
hipError_t launch_inject(int bits, int NP, int nrec, const int64_t* base, const double* vec, const double* w,
                         double sb, void* U, void* S, hipStream_t st);
// Pressure at receivers: receiver r reads nn[r] nodes from 4-vector index base[r] with row stride ld.
hipError_t launch_receivers(int bits, int ld, int nrec, const void* U, const int64_t* base, const int* nn,
                            const void* rows, double* out, hipStream_t st);
// Per-block partial energies; returns the number of partials written.
hipError_t launch_energy(int N, int bits, int64_t K, const void* U, const double* aux, const double* Mv,
                         const double* M1, double* partial, int* nblocks, hipStream_t st);
// Tetrahedron energies (U points at the first tetrahedron node), added to the same partial sums layout.
hipError_t launch_energy_tet(int N, int bits, int64_t Kt, const void* U, const double* auxT, const double* Mt,
                             double* partial, int* nblocks, hipStream_t st);

// Hooks of the host runtime for entry points defined outside api.cpp.
struct RhsView {
  int device;
  int bits;
  int64_t nodes;
  hipStream_t stream;
};
// Fills *v for a device context that may evaluate its right-hand side (state
// at least material); else returns the WDG_ERR_* code with the context message set.
int ctx_rhs_view(wdg_ctx_fwd* ctx, RhsView* v);
// The right-hand side of the device state dIn (node 4-vectors of the
// context's precision) at time t into dOut (same layout), sources included,
// enqueued on the context stream; neither buffer may alias the context state.
int ctx_eval_rhs_device(wdg_ctx_fwd* ctx, double t, const void* dIn, void* dOut);
// Sets the context message and returns code.
int ctx_fail(wdg_ctx_fwd* ctx, int code, const char* msg);

}  // namespace wdg
