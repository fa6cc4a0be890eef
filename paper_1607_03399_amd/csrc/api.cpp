// Host runtime and C ABI of libwdg.
//
// Mesh validation (Definition of vertically mapped wedges, Sec. 3.2),
// face matching, node coordinates, point location, sources/receivers and the
// Runge-Kutta driver loop.  All arithmetic of the right-hand side runs in the
// HIP kernels (wedge_stage.hip, tet_stage.hip, mortar.hip, setup.hip); the host
// only prepares data and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "refops.hpp"
#include "wdg.h"

using wdg::RefOps;
using wdg::TetOps;

namespace {

// five-stage fourth-order 2N-storage Runge-Kutta (Carpenter & Kennedy 1994)
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

struct Source {
  double xyz[3];
  double f0, t0, amp;
  int64_t elem;
  std::vector<double> vec;  // kappa (M^k)^-1 l(xs), NP values
  double value(double t) const {
    const double a = M_PI * M_PI * f0 * f0 * (t - t0) * (t - t0);
    return amp * (1.0 - 2.0 * a) * std::exp(-a);
  }
};

// A wedge quadrilateral face covered by two tetrahedron triangles (the
// common refinement of a column-split hybrid mesh).
struct MortarHost {
  int64_t k = 0;          // wedge
  int e = 0, diag = 0;    // quadrilateral face (edge e) and its diagonal (0: A0-A2, 1: A1-A3)
  int64_t t[2] = {0, 0};  // tetrahedra below / above the diagonal (global ids)
  int tf[2] = {0, 0};     // their faces
  double zba = 0, zbb = 0, zta = 0, ztb = 0, ell = 0, nx = 0, ny = 0;
  double lam[2][9] = {};  // tetrahedron face barycentrics as affine functions of (xi, z)
  double Jft[2] = {0, 0};  // tetrahedron face area / 2
};

enum State { kCreated = 0, kMesh = 1, kMaterial = 2, kFields = 3 };

}  // namespace

struct wdg_ctx {
  int N = 0, bits = 64, device = -1;
  bool host_only = true;
  std::unique_ptr<RefOps> ref;
  std::unique_ptr<TetOps> tref;  // built on first use (meshes with tetrahedra)
  mutable std::string err;
  int state = kCreated;
  int64_t K = 0, Kw = 0, Kt = 0;  // elements: wedges first, then tetrahedra
  std::vector<double> X;      // Kw x 6 x 3 wedge vertex coordinates
  std::vector<double> Xt;     // Kt x 4 x 3 tetrahedron vertex coordinates
  std::vector<int32_t> conn;  // Kw x kConnStride
  std::vector<int32_t> connT;  // Kt x kTetConnStride
  std::vector<double> geoT;   // Kt x kTetGeoStride (FP64 master copy)
  std::vector<double> c, rho;
  int bc = WDG_BC_RIGID, flux = WDG_FLUX_UPWIND, mass = WDG_MASS_EXACT;
  int layer_march = WDG_MARCH_OFF;
  int2* dCols = nullptr;  // columns of the wedge mesh: (first element, layers)
  int ncols = 0;
  int tet_blocks = 0;  // persistent blocks of the tetrahedron kernel (0: default)
  bool tet_valu = false;  // tetrahedron products as per-node dot products (else MFMA)
  int wedge_kernel = WDG_WEDGE_AUTO;  // which wedge stage kernel (wdg_set_wedge_kernel)
  int wedge_block = 0;  // elements per block of the node-lane kernel (0: default; wdg_set_wedge_block)
  // Hybrid meshes, optionally: after the mortar kernel the tetrahedron kernel
  // runs on a second stream beside the wedge kernel (they read the same input
  // and write disjoint nodes), joined back before the stage ends
  // (wdg_set_overlap; off by default: measured slower with the current kernels).
  bool overlap = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double time = 0.0;

  hipStream_t stream = nullptr;
  void* dU[2] = {nullptr, nullptr};
  void* dRes = nullptr;
  bool own_state = true;
  int cur = 0;
  void* dGeo = nullptr;
  void* dL = nullptr;
  void* dSrcVec = nullptr;
  double* dAux = nullptr;
  double* dMv = nullptr;
  double* dM1 = nullptr;
  double* dPartial = nullptr;
  int32_t* dConn = nullptr;
  void* dGeoT = nullptr;
  void* dOpsT = nullptr;
  void* dOpsW = nullptr;  // N >= 4: reference rows of the node-lane wedge kernel
  double* dAuxT = nullptr;
  double* dMt = nullptr;
  int32_t* dConnT = nullptr;
  std::vector<MortarHost> mort;
  int32_t* dMortI = nullptr;
  void* dMortG = nullptr;
  void* dMortTab = nullptr;
  void* dMortC = nullptr;
  void* dMortB = nullptr;
  void* dMortF = nullptr;
  std::vector<Source> src;
  int64_t nrec = 0;
  std::vector<double> rec_xyz;  // nrec x 3
  int64_t* dRecBase = nullptr;
  int* dRecNN = nullptr;
  void* dRecRows = nullptr;  // receiver interpolation rows, in the state precision
  double* dRecBuf = nullptr;
  int64_t rec_cap = 0, rec_steps = 0;
  bool timing = false;
  // forward recording for the adjoint (wdg_adjoint_record): the state at the
  // start of every adj_every-th step since the recording began
  bool recording = false;
  int64_t adj_every = 0, adj_ncap = 0, adj_steps = 0;
  double adj_t0 = 0.0, adj_dt = 0.0;
  void* dAdjCp = nullptr;
  size_t adj_cp_bytes = 0;
  size_t adj_mem_limit = 0;  // 0: automatic
  // state buffers of the reverse sweep, kept for later gradient calls (a
  // fresh allocation of this size costs more than the sweep on some drivers)
  void* dAdjStore = nullptr;
  size_t adj_store_bytes = 0;
  // the recorded forward writes each segment's stage inputs and residuals
  // into the store (set when a recording starts with the store already kept
  // in the whole-segment layout; cleared once a sweep overwrites it)
  bool adj_tail = false;
  // per stage: start, after the mortar kernel, after the wedge kernel, after the tet kernel
  std::vector<std::array<hipEvent_t, 4>> events;
  size_t events_used = 0;

  size_t tsize() const { return bits == 32 ? 4 : 8; }
  int NT() const { return ref->NT; }
  int NP() const { return ref->NP; }  // nodes of a wedge
  int NPt() const { return (N + 1) * (N + 2) * (N + 3) / 6; }
  int NPof(int64_t k) const { return k < Kw ? NP() : NPt(); }
  // first node of element k in the node-major state layout
  int64_t node_base(int64_t k) const { return k < Kw ? k * NP() : Kw * NP() + (k - Kw) * NPt(); }
  int64_t nodes() const { return Kw * NP() + Kt * NPt(); }
};

namespace {

int fail(const wdg_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      return fail(ctx, e_ == hipErrorOutOfMemory ? WDG_ERR_OOM : WDG_ERR_HIP,                    \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                            \
    }                                                                                            \
  } while (0)

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void release_device(wdg_ctx* ctx) {
  if (ctx->host_only) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  if (ctx->own_state) {
    dfree(ctx->dU[0]);
    dfree(ctx->dU[1]);
    dfree(ctx->dRes);
  }
  ctx->dU[0] = ctx->dU[1] = nullptr;
  ctx->dRes = nullptr;
  ctx->own_state = true;
  dfree(ctx->dGeo);
  dfree(ctx->dL);
  dfree(ctx->dAdjCp);
  dfree(ctx->dAdjStore);
  ctx->adj_store_bytes = 0;
  ctx->adj_tail = false;
  ctx->adj_cp_bytes = 0;
  dfree(ctx->dSrcVec);
  dfree(ctx->dAux);
  dfree(ctx->dMv);
  dfree(ctx->dM1);
  dfree(ctx->dPartial);
  dfree(ctx->dConn);
  dfree(ctx->dGeoT);
  dfree(ctx->dOpsT);
  dfree(ctx->dOpsW);
  dfree(ctx->dCols);
  ctx->ncols = 0;
  dfree(ctx->dAuxT);
  dfree(ctx->dMt);
  dfree(ctx->dConnT);
  dfree(ctx->dMortI);
  dfree(ctx->dMortG);
  dfree(ctx->dMortTab);
  dfree(ctx->dMortC);
  dfree(ctx->dMortB);
  dfree(ctx->dMortF);
  dfree(ctx->dRecBase);
  dfree(ctx->dRecNN);
  dfree(ctx->dRecRows);
  dfree(ctx->dRecBuf);
  ctx->rec_cap = 0;
  for (auto& ev : ctx->events)
    for (auto& e : ev) (void)hipEventDestroy(e);
  ctx->events.clear();
  ctx->events_used = 0;
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  ctx->side = nullptr;
  ctx->ev_fork = ctx->ev_join = nullptr;
}

// reference coordinates of physical point x in wedge k (closed form for a
// vertically mapped wedge: affine in (x, y), then linear in t along the vertical)
void wedge_ref_coords(const double* Xk, const double* x, double& r, double& s, double& t) {
  const double xr = 0.5 * (Xk[3] - Xk[0]), xs = 0.5 * (Xk[6] - Xk[0]);
  const double yr = 0.5 * (Xk[4] - Xk[1]), ys = 0.5 * (Xk[7] - Xk[1]);
  const double J = xr * ys - xs * yr;
  const double dx = x[0] - Xk[0], dy = x[1] - Xk[1];
  r = -1.0 + (ys * dx - xs * dy) / J;
  s = -1.0 + (-yr * dx + xr * dy) / J;
  const double lam[3] = {-(r + s) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0};
  double zb = 0, zt = 0;
  for (int v = 0; v < 3; ++v) {
    zb += lam[v] * Xk[3 * v + 2];
    zt += lam[v] * Xk[3 * (v + 3) + 2];
  }
  t = 2.0 * (x[2] - zb) / (zt - zb) - 1.0;
}

// barycentric reference coordinates of x in affine tetrahedron k (r = 2 lambda_1 - 1, ...)
void tet_ref_coords(const double* Xk, const double* x, double& r, double& s, double& t) {
  double A[9], b[3];
  for (int d = 0; d < 3; ++d) {
    for (int v = 0; v < 3; ++v) A[d * 3 + v] = Xk[3 * (v + 1) + d] - Xk[d];
    b[d] = x[d] - Xk[d];
  }
  std::vector<double> Am(A, A + 9), bv(b, b + 3);
  if (!wdg::solve_dense(3, 1, Am, bv)) {
    r = s = t = 1e300;
    return;
  }
  r = 2.0 * bv[0] - 1.0;
  s = 2.0 * bv[1] - 1.0;
  t = 2.0 * bv[2] - 1.0;
}

// element containing x (lowest global id), with reference coordinates
int64_t locate(const wdg_ctx* ctx, const double* x, double& r, double& s, double& t) {
  const double tol = 1e-12;
  for (int64_t k = 0; k < ctx->Kw; ++k) {
    double rr, ss, tt;
    wedge_ref_coords(&ctx->X[k * 18], x, rr, ss, tt);
    if (rr >= -1 - tol && ss >= -1 - tol && rr + ss <= tol && std::fabs(tt) <= 1 + tol) {
      r = rr;
      s = ss;
      t = tt;
      return k;
    }
  }
  for (int64_t k = 0; k < ctx->Kt; ++k) {
    double rr, ss, tt;
    tet_ref_coords(&ctx->Xt[k * 12], x, rr, ss, tt);
    if (rr >= -1 - tol && ss >= -1 - tol && tt >= -1 - tol && rr + ss + tt <= -1 + tol) {
      r = rr;
      s = ss;
      t = tt;
      return ctx->Kw + k;
    }
  }
  return -1;
}

// wedge basis l_{ij}(r,s,t) = l^tri_i(r,s) l^1D_j(t)
void wedge_basis(const RefOps& R, double r, double s, double t, std::vector<double>& out) {
  std::vector<double> lt(R.NT), l1(R.Nq);
  R.tri_basis(r, s, lt.data());
  R.line_basis(t, l1.data());
  out.resize(R.NP);
  for (int j = 0; j < R.Nq; ++j)
    for (int i = 0; i < R.NT; ++i) out[j * R.NT + i] = lt[i] * l1[j];
}

double tet_jacobian(const double* Xk) {
  double a[3], b[3], c[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = 0.5 * (Xk[3 + d] - Xk[d]);
    b[d] = 0.5 * (Xk[6 + d] - Xk[d]);
    c[d] = 0.5 * (Xk[9 + d] - Xk[d]);
  }
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
}

// kappa (M^k)^-1 l(x_s): wedges M^k = M^{tri,k} (x) M^1D (Sec. 4.2); tetrahedra M^k = J M
std::vector<double> mass_inverse_times(const wdg_ctx* ctx, int64_t k, double kappa, double r, double s, double t) {
  if (k >= ctx->Kw) {
    const TetOps& Tt = *ctx->tref;
    std::vector<double> l(Tt.NP);
    Tt.basis(r, s, t, l.data());
    wdg::solve_dense(Tt.NP, 1, Tt.M, l);
    const double J = tet_jacobian(&ctx->Xt[(k - ctx->Kw) * 12]);
    for (auto& v : l) v *= kappa / J;
    return l;
  }
  const RefOps& R = *ctx->ref;
  const double* Xk = &ctx->X[k * 18];
  const double xr = 0.5 * (Xk[3] - Xk[0]), xs = 0.5 * (Xk[6] - Xk[0]);
  const double yr = 0.5 * (Xk[4] - Xk[1]), ys = 0.5 * (Xk[7] - Xk[1]);
  const double Jt = xr * ys - xs * yr;
  std::vector<double> Mt(R.NT * R.NT, 0.0);
  for (int v = 0; v < 3; ++v) {
    const double cw = 0.5 * Jt * (Xk[3 * (v + 3) + 2] - Xk[3 * v + 2]);
    for (int i = 0; i < R.NT * R.NT; ++i) Mt[i] += cw * R.Mv[v][i];
  }
  std::vector<double> lt(R.NT), l1(R.Nq);
  R.tri_basis(r, s, lt.data());
  R.line_basis(t, l1.data());
  wdg::solve_dense(R.NT, 1, Mt, lt);
  if (ctx->mass == WDG_MASS_LUMPED) {
    for (int j = 0; j < R.Nq; ++j) l1[j] /= R.wgll[j];
  } else {
    wdg::solve_dense(R.Nq, 1, R.M1, l1);
  }
  std::vector<double> out(R.NP);
  for (int j = 0; j < R.Nq; ++j)
    for (int i = 0; i < R.NT; ++i) out[j * R.NT + i] = kappa * lt[i] * l1[j];
  return out;
}

template <typename T>
void to_interleaved(const wdg_ctx* ctx, const double* p, const double* ux, const double* uy, const double* uz,
                    std::vector<unsigned char>& buf) {
  const int64_t n = ctx->nodes();
  buf.resize(size_t(n) * 4 * sizeof(T));
  T* o = reinterpret_cast<T*>(buf.data());
  for (int64_t m = 0; m < n; ++m) {  // device node layout: (p, u_z, u_x, u_y)
    o[4 * m] = T(p[m]);
    o[4 * m + 1] = T(uz[m]);
    o[4 * m + 2] = T(ux[m]);
    o[4 * m + 3] = T(uy[m]);
  }
}

template <typename T>
void from_interleaved(const wdg_ctx* ctx, const std::vector<unsigned char>& buf, double* p, double* ux, double* uy,
                      double* uz) {
  const int64_t n = ctx->nodes();
  const T* o = reinterpret_cast<const T*>(buf.data());
  for (int64_t m = 0; m < n; ++m) {
    if (p) p[m] = double(o[4 * m]);
    if (uz) uz[m] = double(o[4 * m + 1]);
    if (ux) ux[m] = double(o[4 * m + 2]);
    if (uy) uy[m] = double(o[4 * m + 3]);
  }
}

int upload_state(wdg_ctx* ctx, void* dst, const double* p, const double* ux, const double* uy, const double* uz) {
  std::vector<unsigned char> buf;
  if (ctx->bits == 32) to_interleaved<float>(ctx, p, ux, uy, uz, buf);
  else to_interleaved<double>(ctx, p, ux, uy, uz, buf);
  HIPCHK(hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

int download_state(const wdg_ctx* ctx, const void* src, double* p, double* ux, double* uy, double* uz) {
  std::vector<unsigned char> buf(size_t(ctx->nodes()) * 4 * ctx->tsize());
  HIPCHK(hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->bits == 32) from_interleaved<float>(ctx, buf, p, ux, uy, uz);
  else from_interleaved<double>(ctx, buf, p, ux, uy, uz);
  return WDG_OK;
}

int upload_sources(wdg_ctx* ctx) {
  if (ctx->host_only || ctx->src.empty()) return WDG_OK;
  const int NP = ctx->NP();
  std::vector<unsigned char> buf(size_t(wdg::kMaxSources) * NP * ctx->tsize(), 0);
  for (size_t s = 0; s < ctx->src.size(); ++s)
    for (int n = 0; n < int(ctx->src[s].vec.size()); ++n) {
      if (ctx->bits == 32) reinterpret_cast<float*>(buf.data())[s * NP + n] = float(ctx->src[s].vec[n]);
      else reinterpret_cast<double*>(buf.data())[s * NP + n] = ctx->src[s].vec[n];
    }
  HIPCHK(hipMemcpyAsync(ctx->dSrcVec, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

// one Runge-Kutta stage (or, with a = 0, dt = 1, no U write, a plain RHS)
// Whether the wedges of a stage with these flags run on the node-lane kernel:
// it exists for orders 4 and 5 in FP32, without layer marching and outside
// the adjoint sweep (which only the level-lane kernel implements); by default
// it is the default wherever it exists (measured faster at orders 4 and 5:
// 122 against 137 us and 209 against 309 us per stage on 73 728 wedges).
bool node_kernel(const wdg_ctx* ctx, int flags) {
  if (ctx->N < 4 || ctx->bits != 32 || (flags & (wdg::kLayerMarch | wdg::kGrad))) return false;
  return ctx->wedge_kernel == WDG_WEDGE_NODE || ctx->wedge_kernel == WDG_WEDGE_AUTO;
}

hipError_t launch_wedges(const wdg_ctx* ctx, const wdg::StageLaunch& L) {
  if (node_kernel(ctx, L.flags))
    return wdg::launch_wedge_node_stage(ctx->N, ctx->bits,
                                        ctx->wedge_block ? ctx->wedge_block : wdg::wedge_node_epb(ctx->N, ctx->bits, 0),
                                        L, ctx->stream);
  return wdg::launch_wedge_stage(ctx->N, ctx->bits, L, ctx->stream);
}

int launch_stage(wdg_ctx* ctx, const void* Uin, void* Uout, void* res, double a, double b, double dt, double tstage,
                 int flags, double g = 1.0, void* rout = nullptr, bool sources = true, const void* gUs = nullptr,
                 const void* gRs = nullptr, void* gacc = nullptr, double gb = 0.0) {
  wdg::StageLaunch L{};
  L.Uin = Uin;
  L.Uout = Uout;
  L.res = res;
  L.geo = ctx->dGeo;
  L.L = ctx->dL;
  L.conn = ctx->dConn;
  L.geoT = ctx->dGeoT;
  L.connT = ctx->dConnT;
  L.opsT = ctx->dOpsT;
  L.opsW = ctx->dOpsW;
  L.srcvec = ctx->dSrcVec;
  L.mortI = ctx->dMortI;
  L.mortG = ctx->dMortG;
  L.mortTab = ctx->dMortTab;
  L.mortC = ctx->dMortC;
  L.mortB = ctx->dMortB;
  L.mortF = ctx->dMortF;
  L.nmort = int64_t(ctx->mort.size());
  L.nsrc = sources ? int(ctx->src.size()) : 0;
  for (int s = 0; s < L.nsrc; ++s) {
    L.src_elem[s] = int(ctx->src[s].elem);
    L.src_amp[s] = ctx->src[s].value(tstage);
  }
  L.a = a;
  L.b = b;
  L.dt = dt;
  L.g = g;
  L.rout = rout;
  L.gUs = gUs;
  L.gRs = gRs;
  L.gb = gb;
  L.gacc = gacc;
  L.Kw = ctx->Kw;
  L.Kt = ctx->Kt;
  L.tet_blocks = ctx->tet_blocks;
  L.cols = ctx->dCols;
  L.ncols = ctx->ncols;
  L.flags = flags | (g != 1.0 ? wdg::kGamma : 0) | (ctx->layer_march != WDG_MARCH_OFF ? wdg::kLayerMarch : 0) |
            (ctx->layer_march == WDG_MARCH_COLUMN ? wdg::kColumnMarch : 0) | (ctx->tet_valu ? wdg::kTetValu : 0) | (ctx->bc == WDG_BC_DIRICHLET_P0 ? wdg::kDirichlet : 0) |
            (ctx->flux == WDG_FLUX_CENTRAL ? wdg::kCentral : 0) | (ctx->mass == WDG_MASS_LUMPED ? wdg::kLumped : 0);
  if (ctx->timing) {
    // events only between kernels that actually run (an event adds a gap to the stream)
    if (ctx->events_used == ctx->events.size()) {
      std::array<hipEvent_t, 4> ev;
      for (auto& e : ev) HIPCHK(hipEventCreate(&e));
      ctx->events.push_back(ev);
    }
    auto& ev = ctx->events[ctx->events_used++];
    const bool has_m = !ctx->mort.empty(), has_t = ctx->Kt > 0;
    HIPCHK(hipEventRecord(ev[0], ctx->stream));
    if (has_m) {
      HIPCHK(wdg::launch_mortar_stage(ctx->N, ctx->bits, L, ctx->stream));
      HIPCHK(hipEventRecord(ev[1], ctx->stream));
    }
    HIPCHK(launch_wedges(ctx, L));
    if (has_t) {
      HIPCHK(hipEventRecord(ev[2], ctx->stream));
      HIPCHK(wdg::launch_tet_stage(ctx->N, ctx->bits, L, ctx->stream));
    }
    HIPCHK(hipEventRecord(ev[3], ctx->stream));
    return WDG_OK;
  }
  HIPCHK(wdg::launch_mortar_stage(ctx->N, ctx->bits, L, ctx->stream));
  if (ctx->overlap && ctx->side && ctx->Kw > 0 && ctx->Kt > 0) {
    // fork: the tetrahedra on the side stream once the mortar fluxes are
    // written, the wedges on the solver stream; join before the next stage
    HIPCHK(hipEventRecord(ctx->ev_fork, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    HIPCHK(wdg::launch_tet_stage(ctx->N, ctx->bits, L, ctx->side));
    HIPCHK(launch_wedges(ctx, L));
    HIPCHK(hipEventRecord(ctx->ev_join, ctx->side));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
    return WDG_OK;
  }
  HIPCHK(launch_wedges(ctx, L));
  HIPCHK(wdg::launch_tet_stage(ctx->N, ctx->bits, L, ctx->stream));
  return WDG_OK;
}

int ensure_receiver_capacity(wdg_ctx* ctx, int64_t steps_needed) {
  if (ctx->nrec == 0 || steps_needed <= ctx->rec_cap) return WDG_OK;
  int64_t cap = std::max<int64_t>(steps_needed, 2 * ctx->rec_cap);
  cap = std::max<int64_t>(cap, 64);
  double* nb = nullptr;
  HIPCHK(hipMalloc(&nb, size_t(cap * ctx->nrec) * sizeof(double)));
  if (ctx->dRecBuf && ctx->rec_steps > 0)
    HIPCHK(hipMemcpyAsync(nb, ctx->dRecBuf, size_t(ctx->rec_steps * ctx->nrec) * sizeof(double),
                          hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dfree(ctx->dRecBuf);
  ctx->dRecBuf = nb;
  ctx->rec_cap = cap;
  return WDG_OK;
}

// vertical mass used by the energy: exact M^1D, or the Gauss-Lobatto weights when lumped
int upload_vertical_mass(wdg_ctx* ctx) {
  if (ctx->host_only || !ctx->dM1) return WDG_OK;
  const RefOps& R = *ctx->ref;
  std::vector<double> M1 = R.M1;
  if (ctx->mass == WDG_MASS_LUMPED) {
    std::fill(M1.begin(), M1.end(), 0.0);
    for (int j = 0; j < R.Nq; ++j) M1[j * R.Nq + j] = R.wgll[j];
  }
  HIPCHK(hipMemcpyAsync(ctx->dM1, M1.data(), M1.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

// classical Legendre polynomials P_0..P_N at x
void legendre_all(int N, double x, double* P) {
  P[0] = 1.0;
  if (N >= 1) P[1] = x;
  for (int n = 1; n < N; ++n) P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
}

// Reference tables of the mortar outputs, in the layout of wdg::mortar_table_size
std::vector<double> mortar_tables(const RefOps& R) {
  const int NT = R.NT, Nq = R.Nq;
  std::vector<double> out;
  std::vector<double> Minv1(Nq * Nq, 0.0);
  for (int i = 0; i < Nq; ++i) Minv1[i * Nq + i] = 1.0;
  wdg::solve_dense(Nq, Nq, R.M1, Minv1);
  out.insert(out.end(), Minv1.begin(), Minv1.end());
  std::vector<double> MtriInv(NT * NT, 0.0);
  for (int i = 0; i < NT; ++i) MtriInv[i * NT + i] = 1.0;
  wdg::solve_dense(NT, NT, R.Mtri, MtriInv);
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < NT; ++i)
      for (int q = 0; q < Nq; ++q) out.push_back(MtriInv[i * NT + R.edge_nodes[e][q]]);
  out.insert(out.end(), MtriInv.begin(), MtriInv.end());
  return out;
}

// Coupling matrices of the mortars (FP64, once per mesh).  Per mortar and side
// of the diagonal, C = int b b^T dA over that side of the quadrilateral, with
// b = (wedge face Lagrange basis l_q(xi) l_m(t), level-major; the tetrahedron
// face's Lagrange basis) and dA the physical area element of the wedge face.
// The side is integrated in the wedge face's (xi, t) coordinates: mort_nx(N)
// Gauss points in xi times Nq Gauss points in t between the bottom (top) and
// the diagonal, exact in t at fixed xi (degree <= 2N); lower triangles packed
// by columns, both sides per mortar, wdg::mort_core_stride values each.
std::vector<double> mortar_cores(const RefOps& R, const std::vector<MortarHost>& mort) {
  const int N = R.N, NT = R.NT, Nq = R.Nq, NW = Nq * Nq, n = wdg::mort_core_n(N), NX = wdg::mort_nx(N);
  const int CS = wdg::mort_core_stride(N), NPK = n * (n + 1) / 2;
  std::vector<double> xg, wg, tg, wt;
  wdg::gauss_legendre(NX, xg, wg);
  wdg::gauss_legendre(Nq, tg, wt);
  // tetrahedron face nodal basis = Legendre products P_a(r) P_b(s) (a + b <= N)
  // combined by the inverse of their Vandermonde at the triangle nodes
  std::vector<double> V(NT * NT), Vinv(NT * NT, 0.0), Pr(N + 1), Ps(N + 1);
  for (int i = 0; i < NT; ++i) {
    legendre_all(N, R.r[i], Pr.data());
    legendre_all(N, R.s[i], Ps.data());
    int md = 0;
    for (int a = 0; a <= N; ++a)
      for (int b = 0; a + b <= N; ++b) V[i * NT + md++] = Pr[a] * Ps[b];
  }
  for (int i = 0; i < NT; ++i) Vinv[i * NT + i] = 1.0;
  wdg::solve_dense(NT, NT, V, Vinv);  // Vinv[md][i]
  std::vector<double> lxi(size_t(NX) * Nq);
  for (int a = 0; a < NX; ++a) R.line_basis(xg[a], &lxi[size_t(a) * Nq]);
  const size_t nm = mort.size();
  std::vector<double> out(nm * CS, 0.0);
  auto work = [&](size_t m0, size_t m1) {
    std::vector<double> b(n), lt(Nq), pr(N + 1), ps(N + 1), ph(NT);
    for (size_t m = m0; m < m1; ++m) {
      const MortarHost& M = mort[m];
      for (int side = 0; side < 2; ++side) {
        double* C = &out[m * CS + size_t(side) * NPK];
        const double* lm = M.lam[side];
        for (int a = 0; a < NX; ++a) {
          const double xi = xg[a];
          const double zb = M.zba * 0.5 * (1.0 - xi) + M.zbb * 0.5 * (1.0 + xi);
          const double zt = M.zta * 0.5 * (1.0 - xi) + M.ztb * 0.5 * (1.0 + xi);
          const double h = zt - zb;
          const double zd = M.diag == 0 ? M.zba * 0.5 * (1.0 - xi) + M.ztb * 0.5 * (1.0 + xi)
                                        : M.zbb * 0.5 * (1.0 + xi) + M.zta * 0.5 * (1.0 - xi);
          const double td = (2.0 * zd - zb - zt) / h;
          const double lo = side == 0 ? -1.0 : td, hi = side == 0 ? td : 1.0;
          for (int g = 0; g < Nq; ++g) {
            const double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * tg[g];
            const double w = wg[a] * wt[g] * 0.5 * (hi - lo) * 0.25 * M.ell * h;
            const double z = zb * 0.5 * (1.0 - t) + zt * 0.5 * (1.0 + t);
            R.line_basis(t, lt.data());
            for (int lev = 0; lev < Nq; ++lev)
              for (int q = 0; q < Nq; ++q) b[lev * Nq + q] = lt[lev] * lxi[size_t(a) * Nq + q];
            const double l1 = lm[3] * xi + lm[4] * z + lm[5], l2 = lm[6] * xi + lm[7] * z + lm[8];
            legendre_all(N, 2.0 * l1 - 1.0, pr.data());
            legendre_all(N, 2.0 * l2 - 1.0, ps.data());
            int md = 0;
            for (int aa = 0; aa <= N; ++aa)
              for (int bb = 0; aa + bb <= N; ++bb) ph[md++] = pr[aa] * ps[bb];
            for (int i = 0; i < NT; ++i) {
              double v = 0.0;
              for (int k = 0; k < NT; ++k) v += Vinv[k * NT + i] * ph[k];
              b[NW + i] = v;
            }
            int o = 0;
            for (int c = 0; c < n; ++c) {
              const double wc = w * b[c];
              for (int r = c; r < n; ++r) C[o++] += wc * b[r];
            }
          }
        }
      }
    }
  };
  const size_t nthr = std::min<size_t>(std::max(1u, std::thread::hardware_concurrency()), 16);
  if (nm < 256 || nthr == 1) {
    work(0, nm);
  } else {
    std::vector<std::thread> pool;
    const size_t per = (nm + nthr - 1) / nthr;
    for (size_t t = 0; t < nthr; ++t) {
      const size_t m0 = t * per, m1 = std::min(nm, m0 + per);
      if (m0 < m1) pool.emplace_back(work, m0, m1);
    }
    for (auto& th : pool) th.join();
  }
  return out;
}

// FP64 values in the device precision
std::vector<unsigned char> to_precision(const std::vector<double>& v, int bits) {
  std::vector<unsigned char> buf(v.size() * size_t(bits / 8));
  for (size_t i = 0; i < v.size(); ++i) {
    if (bits == 32) reinterpret_cast<float*>(buf.data())[i] = float(v[i]);
    else reinterpret_cast<double*>(buf.data())[i] = v[i];
  }
  return buf;
}

// mortar value records (geometry, and the impedance sums of the current material)
int upload_mortar_geometry(wdg_ctx* ctx) {
  if (ctx->host_only || ctx->mort.empty()) return WDG_OK;
  std::vector<double> g(ctx->mort.size() * wdg::kMortGeoStride, 0.0);
  for (size_t m = 0; m < ctx->mort.size(); ++m) {
    const MortarHost& M = ctx->mort[m];
    double* o = &g[m * wdg::kMortGeoStride];
    o[0] = M.zba;
    o[1] = M.zbb;
    o[2] = M.zta;
    o[3] = M.ztb;
    o[4] = M.ell;
    o[5] = M.nx;
    o[6] = M.ny;
    for (int side = 0; side < 2; ++side) {
      for (int i = 0; i < 9; ++i) o[7 + 9 * side + i] = M.lam[side][i];
      o[25 + side] = 1.0 / M.Jft[side];
      o[27 + side] = ctx->rho[M.k] * ctx->c[M.k] + ctx->rho[M.t[side]] * ctx->c[M.t[side]];
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->dMortG, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

// tetrahedron geometry and material records (FP64 master copy -> device precision)
int upload_tet_geometry(wdg_ctx* ctx) {
  if (ctx->host_only || ctx->Kt == 0) return WDG_OK;
  const size_t n = ctx->geoT.size();
  std::vector<unsigned char> buf(n * ctx->tsize());
  for (size_t i = 0; i < n; ++i) {
    if (ctx->bits == 32) reinterpret_cast<float*>(buf.data())[i] = float(ctx->geoT[i]);
    else reinterpret_cast<double*>(buf.data())[i] = ctx->geoT[i];
  }
  std::vector<double> aux(size_t(ctx->Kt) * wdg::kTetAuxStride, 0.0);
  for (int64_t k = 0; k < ctx->Kt; ++k) {
    const int64_t g = ctx->Kw + k;
    aux[k * wdg::kTetAuxStride] = tet_jacobian(&ctx->Xt[k * 12]);
    aux[k * wdg::kTetAuxStride + 1] = ctx->rho[g] * ctx->c[g] * ctx->c[g];
    aux[k * wdg::kTetAuxStride + 2] = ctx->rho[g];
  }
  HIPCHK(hipMemcpyAsync(ctx->dGeoT, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->dAuxT, aux.data(), aux.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

namespace wdg {

int ctx_rhs_view(wdg_ctx* ctx, RhsView* v) {
  if (!ctx || !v) return WDG_ERR_ARG;
  if (ctx->state < kMaterial || ctx->host_only) return fail(ctx, WDG_ERR_STATE, "eval_rhs before set_material");
  v->device = ctx->device;
  v->bits = ctx->bits;
  v->nodes = ctx->nodes();
  v->stream = ctx->stream;
  return WDG_OK;
}

int ctx_eval_rhs_device(wdg_ctx* ctx, double t, const void* dIn, void* dOut) {
  return launch_stage(ctx, dIn, nullptr, dOut, 0.0, 0.0, 1.0, t, 0);
}

int ctx_fail(wdg_ctx* ctx, int code, const char* msg) { return fail(ctx, code, msg); }

}  // namespace wdg

extern "C" {

int wdg_create(int order_N, int precision_bits, int device, wdg_ctx** out) {
  if (!out) return WDG_ERR_ARG;
  *out = nullptr;
  if (order_N < 1 || order_N > 5) return WDG_ERR_ARG;
  if (precision_bits != 32 && precision_bits != 64) return WDG_ERR_ARG;
  if (device < -1) return WDG_ERR_ARG;
  wdg_ctx* ctx = new (std::nothrow) wdg_ctx();
  if (!ctx) return WDG_ERR_OOM;
  ctx->N = order_N;
  ctx->bits = precision_bits;
  ctx->device = device;
  ctx->host_only = device < 0;
  try {
    ctx->ref = std::make_unique<RefOps>(order_N);
  } catch (...) {
    delete ctx;
    return WDG_ERR_ARG;
  }
  *out = ctx;
  return WDG_OK;
}

int wdg_destroy(wdg_ctx* ctx) {
  if (!ctx) return WDG_ERR_ARG;
  if (!ctx->host_only && ctx->dGeo) {
    (void)hipSetDevice(ctx->device);
    release_device(ctx);
  }
  delete ctx;
  return WDG_OK;
}

const char* wdg_last_error(const wdg_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int wdg_set_mesh(wdg_ctx* ctx, int64_t nv, const double* vxyz, int64_t nw, const int64_t* wedge_v, int64_t nt,
                 const int64_t* tet_v) {
  if (!ctx) return WDG_ERR_ARG;
  if (nv <= 0 || !vxyz || nw < 0 || nt < 0 || nw + nt <= 0 || (nw > 0 && !wedge_v) || (nt > 0 && !tet_v))
    return fail(ctx, WDG_ERR_ARG, "bad mesh arguments");
  if (nw + nt > (int64_t(1) << 31) / 8) return fail(ctx, WDG_ERR_ARG, "too many elements");
  for (int64_t i = 0; i < nv * 3; ++i)
    if (!std::isfinite(vxyz[i])) return fail(ctx, WDG_ERR_ARG, "non-finite vertex coordinate");
  const int64_t Kw = nw, Kt = nt, K = nw + nt;
  std::vector<double> X(size_t(Kw) * 18), Xt(size_t(Kt) * 12);
  for (int64_t k = 0; k < Kw; ++k) {
    for (int v = 0; v < 6; ++v) {
      const int64_t id = wedge_v[k * 6 + v];
      if (id < 0 || id >= nv) return fail(ctx, WDG_ERR_ARG, "vertex id out of range in wedge " + std::to_string(k));
      for (int d = 0; d < 3; ++d) X[k * 18 + 3 * v + d] = vxyz[id * 3 + d];
    }
    const double* x = &X[k * 18];
    double h = 0.0;
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) d2 += (x[3 * a + d] - x[3 * b + d]) * (x[3 * a + d] - x[3 * b + d]);
        h = std::max(h, std::sqrt(d2));
      }
    for (int v = 0; v < 3; ++v)
      if (std::fabs(x[3 * v] - x[3 * (v + 3)]) > 1e-12 * h || std::fabs(x[3 * v + 1] - x[3 * (v + 3) + 1]) > 1e-12 * h)
        return fail(ctx, WDG_ERR_NOT_VERTICAL, "wedge " + std::to_string(k) + " is not vertically mapped");
    const double xr = 0.5 * (x[3] - x[0]), xs = 0.5 * (x[6] - x[0]);
    const double yr = 0.5 * (x[4] - x[1]), ys = 0.5 * (x[7] - x[1]);
    const double Jt = xr * ys - xs * yr;
    if (std::fabs(Jt) <= 1e-14 * h * h) return fail(ctx, WDG_ERR_JACOBIAN, "wedge " + std::to_string(k) + " has a degenerate base");
    if (Jt < 0) return fail(ctx, WDG_ERR_ORIENTATION, "wedge " + std::to_string(k) + " bottom triangle is clockwise");
    for (int v = 0; v < 3; ++v)
      if (x[3 * (v + 3) + 2] - x[3 * v + 2] <= 1e-14 * h)
        return fail(ctx, WDG_ERR_JACOBIAN, "wedge " + std::to_string(k) + " has a non-positive vertical edge");
  }
  for (int64_t k = 0; k < Kt; ++k) {
    for (int v = 0; v < 4; ++v) {
      const int64_t id = tet_v[k * 4 + v];
      if (id < 0 || id >= nv) return fail(ctx, WDG_ERR_ARG, "vertex id out of range in tetrahedron " + std::to_string(k));
      for (int d = 0; d < 3; ++d) Xt[k * 12 + 3 * v + d] = vxyz[id * 3 + d];
    }
    const double* x = &Xt[k * 12];
    double h = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        double d2 = 0;
        for (int d = 0; d < 3; ++d) d2 += (x[3 * a + d] - x[3 * b + d]) * (x[3 * a + d] - x[3 * b + d]);
        h = std::max(h, std::sqrt(d2));
      }
    const double J = tet_jacobian(x);
    if (std::fabs(J) <= 1e-14 * h * h * h)
      return fail(ctx, WDG_ERR_JACOBIAN, "tetrahedron " + std::to_string(k) + " is degenerate");
    if (J < 0) return fail(ctx, WDG_ERR_ORIENTATION, "tetrahedron " + std::to_string(k) + " is negatively oriented");
  }

  // face matching by sorted vertex ids; face id = element * 5 + local face
  static const int kFaceVerts[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
  auto face_vertex = [&](int64_t k, int f, int m) -> int64_t {
    return k < Kw ? wedge_v[k * 6 + kFaceVerts[f][m]] : tet_v[(k - Kw) * 4 + wdg::kTetFaceVerts[f][m]];
  };
  struct FaceKey {
    std::array<int64_t, 4> key;
    int64_t id;
  };
  std::vector<FaceKey> faces;
  faces.reserve(size_t(Kw) * 5 + size_t(Kt) * 4);
  for (int64_t k = 0; k < K; ++k) {
    const int nf = k < Kw ? 5 : 4;
    for (int f = 0; f < nf; ++f) {
      std::array<int64_t, 4> kk{-1, -1, -1, -1};
      const int nvf = (k < Kw && f >= 2) ? 4 : 3;
      for (int m = 0; m < nvf; ++m) kk[m] = face_vertex(k, f, m);
      std::sort(kk.begin(), kk.begin() + nvf);
      if (nvf == 3) kk = {-1, kk[0], kk[1], kk[2]};
      faces.push_back({kk, k * 5 + f});
    }
  }
  std::sort(faces.begin(), faces.end(), [](const FaceKey& a, const FaceKey& b) { return a.key < b.key; });
  std::vector<int32_t> conn(size_t(Kw) * wdg::kConnStride, 0), connT(size_t(Kt) * wdg::kTetConnStride, 0);
  for (int64_t k = 0; k < Kw; ++k)
    for (int f = 0; f < 5; ++f) conn[k * wdg::kConnStride + f] = -1;
  for (int64_t k = 0; k < Kt; ++k)
    for (int f = 0; f < 4; ++f) connT[k * wdg::kTetConnStride + f] = -1;
  std::vector<std::pair<std::array<int64_t, 4>, int64_t>> open_tri;  // unmatched triangular faces (key, face id)
  for (size_t a = 0; a < faces.size();) {
    size_t b = a + 1;
    while (b < faces.size() && faces[b].key == faces[a].key) ++b;
    if (b - a > 2) return fail(ctx, WDG_ERR_NONCONFORMING, "a face is shared by more than two elements");
    if (b - a == 1 && faces[a].key[0] < 0) open_tri.push_back({faces[a].key, faces[a].id});
    if (b - a == 2) {
      for (int side = 0; side < 2; ++side) {
        const int64_t me = faces[a + side].id, other = faces[a + 1 - side].id;
        const int64_t k1 = me / 5, k2 = other / 5;
        const int f1 = int(me % 5), f2 = int(other % 5);
        const bool tri = k1 >= Kw || f1 < 2;
        if (tri) {
          // vertex permutation between the two numberings of the shared triangle
          int pi[3];
          for (int v = 0; v < 3; ++v) {
            const int64_t gid = face_vertex(k1, f1, v);
            pi[v] = -1;
            for (int m = 0; m < 3; ++m)
              if (face_vertex(k2, f2, m) == gid) pi[v] = m;
          }
          int code = -1;
          for (int p = 0; p < 6; ++p)
            if (wdg::kPerm[p][0] == pi[0] && wdg::kPerm[p][1] == pi[1] && wdg::kPerm[p][2] == pi[2]) code = p;
          if (code < 0) return fail(ctx, WDG_ERR_NONCONFORMING, "triangular face vertex mismatch");
          if (k1 < Kw) {
            int32_t* cn = &conn[k1 * wdg::kConnStride];
            cn[f1] = int32_t(k2);
            cn[5] |= code << (3 * f1);
            if (k2 < Kw) {
              if (f2 == 1) cn[5] |= 1 << (6 + f1);
            } else {
              cn[5] |= f2 << (14 + 2 * f1);
            }
          } else {
            int32_t* cn = &connT[(k1 - Kw) * wdg::kTetConnStride];
            cn[f1] = int32_t(k2);
            cn[4] |= (code | (f2 << 3)) << (5 * f1);
          }
        } else {
          int32_t* cn = &conn[k1 * wdg::kConnStride];
          cn[f1] = int32_t(k2);
          const int e1 = f1 - 2, e2 = f2 - 2;
          const int64_t A = wedge_v[k1 * 6 + e1], B = wedge_v[k1 * 6 + (e1 + 1) % 3];
          const int64_t A2 = wedge_v[k2 * 6 + e2], B2 = wedge_v[k2 * 6 + (e2 + 1) % 3];
          if (!(A2 == B && B2 == A))
            return fail(ctx, WDG_ERR_NONCONFORMING, "quadrilateral face orientation mismatch");
          cn[5] |= e2 << (8 + 2 * e1);
        }
      }
    }
    a = b;
  }
  // A wedge's quadrilateral face left open next to open tetrahedron triangles:
  // when two of them cover it (split along a diagonal) the face is integrated
  // on that common refinement (a mortar); anything else is not conforming.
  // Corners of the quadrilateral: A0, A1 the bottom edge from its first to
  // its second vertex, A2, A3 above A1, A0; diagonal 0 joins A0-A2, 1 A1-A3.
  std::vector<MortarHost> mortars;
  if (Kt > 0 && !open_tri.empty()) {
    std::sort(open_tri.begin(), open_tri.end());
    std::vector<char> used(open_tri.size(), 0);
    auto find_tri = [&](int64_t p, int64_t q, int64_t r) -> int64_t {
      std::array<int64_t, 4> t{-1, p, q, r};
      std::sort(t.begin() + 1, t.end());
      auto it = std::lower_bound(open_tri.begin(), open_tri.end(), std::make_pair(t, int64_t(-1)));
      if (it == open_tri.end() || it->first != t) return -1;
      return int64_t(it - open_tri.begin());
    };
    static const int kDiagTris[2][2][3] = {{{0, 1, 2}, {0, 2, 3}}, {{0, 1, 3}, {1, 2, 3}}};
    for (int64_t k = 0; k < Kw; ++k)
      for (int f = 2; f < 5; ++f) {
        if (conn[k * wdg::kConnStride + f] >= 0) continue;
        int64_t A[4];
        for (int m = 0; m < 4; ++m) A[m] = face_vertex(k, f, m);
        int found = -1;
        int64_t hit[2] = {-1, -1};
        int partial = 0;
        for (int d = 0; d < 2; ++d) {
          const int64_t i0 = find_tri(A[kDiagTris[d][0][0]], A[kDiagTris[d][0][1]], A[kDiagTris[d][0][2]]);
          const int64_t i1 = find_tri(A[kDiagTris[d][1][0]], A[kDiagTris[d][1][1]], A[kDiagTris[d][1][2]]);
          partial += (i0 >= 0) + (i1 >= 0);
          if (i0 >= 0 && i1 >= 0 && !used[i0] && !used[i1]) {
            found = d;
            hit[0] = i0;
            hit[1] = i1;
          }
        }
        if (found < 0) {
          if (partial > 0)
            return fail(ctx, WDG_ERR_NONCONFORMING,
                        "wedge " + std::to_string(k) + " has a quadrilateral face against triangular faces");
          continue;
        }
        used[hit[0]] = used[hit[1]] = 1;
        MortarHost M;
        M.k = k;
        M.e = f - 2;
        M.diag = found;
        for (int side = 0; side < 2; ++side) {
          const int64_t id = open_tri[hit[side]].second;
          M.t[side] = id / 5;
          M.tf[side] = int(id % 5);
        }
        mortars.push_back(M);
      }
  }
  const int64_t nmort = int64_t(mortars.size());
  for (int64_t m = 0; m < nmort; ++m) {
    MortarHost& M = mortars[m];
    conn[M.k * wdg::kConnStride + 2 + M.e] = int32_t(-2 - m);
    for (int side = 0; side < 2; ++side)
      connT[(M.t[side] - Kw) * wdg::kTetConnStride + M.tf[side]] = int32_t(-2 - (2 * m + side));
    // geometry of the quadrilateral in its (edge parameter xi, height z) plane
    const double* x = &X[M.k * 18];
    const int a = M.e, b = (M.e + 1) % 3;
    M.zba = x[3 * a + 2];
    M.zbb = x[3 * b + 2];
    M.zta = x[3 * (a + 3) + 2];
    M.ztb = x[3 * (b + 3) + 2];
    const double dx = x[3 * b] - x[3 * a], dy = x[3 * b + 1] - x[3 * a + 1];
    M.ell = std::sqrt(dx * dx + dy * dy);
    M.nx = dy / M.ell;
    M.ny = -dx / M.ell;
    const int64_t corner_id[4] = {wedge_v[M.k * 6 + a], wedge_v[M.k * 6 + b], wedge_v[M.k * 6 + b + 3],
                                  wedge_v[M.k * 6 + a + 3]};
    const double cxi[4] = {-1.0, 1.0, 1.0, -1.0};
    const double cz[4] = {M.zba, M.zbb, M.ztb, M.zta};
    for (int side = 0; side < 2; ++side) {
      const int64_t tl = M.t[side] - Kw;
      // barycentrics of the tetrahedron face (its own vertex order) as affine functions of (xi, z)
      std::vector<double> Am(9), Binv(9, 0.0);
      double P[3][3];
      for (int v = 0; v < 3; ++v) {
        const int64_t gid = tet_v[tl * 4 + wdg::kTetFaceVerts[M.tf[side]][v]];
        int c = -1;
        for (int q = 0; q < 4; ++q)
          if (corner_id[q] == gid) c = q;
        if (c < 0) return fail(ctx, WDG_ERR_NONCONFORMING, "mortar face corner mismatch");
        Am[0 * 3 + v] = cxi[c];
        Am[1 * 3 + v] = cz[c];
        Am[2 * 3 + v] = 1.0;
        for (int d = 0; d < 3; ++d) P[v][d] = vxyz[gid * 3 + d];
      }
      for (int i = 0; i < 3; ++i) Binv[i * 3 + i] = 1.0;
      if (!wdg::solve_dense(3, 3, Am, Binv)) return fail(ctx, WDG_ERR_NONCONFORMING, "degenerate mortar triangle");
      for (int i = 0; i < 9; ++i) M.lam[side][i] = Binv[i];  // lambda_v = B[v][0] xi + B[v][1] z + B[v][2]
      double u[3], w[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = P[1][d] - P[0][d];
        w[d] = P[2][d] - P[0][d];
      }
      const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz2 = u[0] * w[1] - u[1] * w[0];
      M.Jft[side] = 0.25 * std::sqrt(cx * cx + cy * cy + cz2 * cz2);  // area / 2
    }
  }

  // tetrahedron geometry (affine: constant metric, planar faces)
  std::vector<double> geoT(size_t(Kt) * wdg::kTetGeoStride, 0.0);
  for (int64_t k = 0; k < Kt; ++k) {
    const double* x = &Xt[k * 12];
    double Jm[3][3];  // d x_d / d (r, s, t)
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) Jm[d][c] = 0.5 * (x[3 * (c + 1) + d] - x[d]);
    const double J = tet_jacobian(x);
    double* g = &geoT[k * wdg::kTetGeoStride];
    // inverse metric: row c of the inverse is grad of reference coordinate c
    for (int c = 0; c < 3; ++c)
      for (int d = 0; d < 3; ++d) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3, d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        g[3 * c + d] = (Jm[d1][c1] * Jm[d2][c2] - Jm[d1][c2] * Jm[d2][c1]) / J;
      }
    g[9] = g[10] = g[11] = 1.0;
    for (int f = 0; f < 4; ++f) {
      const int* fv = wdg::kTetFaceVerts[f];
      int opp = 0 + 1 + 2 + 3 - fv[0] - fv[1] - fv[2];
      double u[3], w[3], n[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = x[3 * fv[1] + d] - x[3 * fv[0] + d];
        w[d] = x[3 * fv[2] + d] - x[3 * fv[0] + d];
      }
      n[0] = u[1] * w[2] - u[2] * w[1];
      n[1] = u[2] * w[0] - u[0] * w[2];
      n[2] = u[0] * w[1] - u[1] * w[0];
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double side = 0;
      for (int d = 0; d < 3; ++d) side += n[d] * (x[3 * opp + d] - x[3 * fv[0] + d]);
      const double sg = side > 0 ? -1.0 : 1.0;  // outward
      g[12 + 4 * f] = (0.25 * nn) / J;          // J_f / J, J_f = area / 2
      for (int d = 0; d < 3; ++d) g[13 + 4 * f + d] = sg * n[d] / nn;
      g[28 + f] = 2.0;
    }
  }

  // accept: replace any previous mesh
  if (!ctx->host_only && (ctx->dGeo || ctx->dGeoT)) {
    (void)hipSetDevice(ctx->device);
    release_device(ctx);
  }
  if (Kt > 0 && !ctx->tref) ctx->tref = std::make_unique<TetOps>(ctx->N);
  ctx->K = K;
  ctx->Kw = Kw;
  ctx->Kt = Kt;
  ctx->X.swap(X);
  ctx->Xt.swap(Xt);
  ctx->conn.swap(conn);
  ctx->connT.swap(connT);
  ctx->mort.swap(mortars);
  ctx->geoT.swap(geoT);
  ctx->c.assign(size_t(K), 1.0);
  ctx->rho.assign(size_t(K), 1.0);
  ctx->src.clear();
  ctx->nrec = 0;
  ctx->rec_steps = 0;
  ctx->time = 0.0;
  ctx->cur = 0;
  ctx->state = kMesh;

  if (ctx->host_only) return WDG_OK;
  ctx->state = kCreated;  // until the device side is complete
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= ctx->device)
    return fail(ctx, WDG_ERR_HIP, "no HIP device " + std::to_string(ctx->device));
  HIPCHK(hipSetDevice(ctx->device));
  const RefOps& R = *ctx->ref;
  const size_t ts = ctx->tsize();
  const size_t nstate = size_t(ctx->nodes()) * 4 * ts;
  const int LS = wdg::lift_stride(ctx->N);
  const size_t kw1 = size_t(std::max<int64_t>(Kw, 1));
  HIPCHK(hipMalloc(&ctx->dU[0], nstate));
  HIPCHK(hipMalloc(&ctx->dU[1], nstate));
  HIPCHK(hipMalloc(&ctx->dRes, nstate));
  HIPCHK(hipMalloc(&ctx->dGeo, kw1 * wdg::kGeoStride * ts));
  HIPCHK(hipMalloc(&ctx->dL, kw1 * LS * ts));
  HIPCHK(hipMalloc(&ctx->dAux, kw1 * wdg::kAuxStride * sizeof(double)));
  HIPCHK(hipMalloc(&ctx->dConn, kw1 * wdg::kConnStride * sizeof(int32_t)));
  HIPCHK(hipMalloc(&ctx->dMv, 3 * size_t(R.NT) * R.NT * sizeof(double)));
  HIPCHK(hipMalloc(&ctx->dM1, size_t(R.Nq) * R.Nq * sizeof(double)));
  HIPCHK(hipMalloc(&ctx->dPartial, 2048 * sizeof(double)));
  HIPCHK(hipMalloc(&ctx->dSrcVec, size_t(wdg::kMaxSources) * R.NP * ts));
  HIPCHK(hipMemsetAsync(ctx->dU[0], 0, nstate, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->dU[1], 0, nstate, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->dRes, 0, nstate, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->dSrcVec, 0, size_t(wdg::kMaxSources) * R.NP * ts, ctx->stream));

  std::vector<double> Mv(3 * size_t(R.NT) * R.NT);
  for (int v = 0; v < 3; ++v) std::copy(R.Mv[v].begin(), R.Mv[v].end(), Mv.begin() + v * R.NT * R.NT);
  HIPCHK(hipMemcpyAsync(ctx->dMv, Mv.data(), Mv.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  {
    int rc = upload_vertical_mass(ctx);
    if (rc) return rc;
  }
  if (Kw > 0) {
    double *dX = nullptr, *dMtri = nullptr;
    HIPCHK(hipMalloc(&dX, ctx->X.size() * sizeof(double)));
    HIPCHK(hipMalloc(&dMtri, R.Mtri.size() * sizeof(double)));
    HIPCHK(hipMemcpyAsync(dX, ctx->X.data(), ctx->X.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(dMtri, R.Mtri.data(), R.Mtri.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->dConn, ctx->conn.data(), ctx->conn.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(wdg::launch_setup(ctx->N, ctx->bits, Kw, dX, ctx->dMv, dMtri, ctx->dGeo, ctx->dL, ctx->dAux, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipFree(dX));
    HIPCHK(hipFree(dMtri));
  }
  if (Kw > 0) {
    // column segments for marching: runs of consecutive wedges, each the top
    // neighbour of the one before (element = column x layers + layer on
    // layered meshes; any other numbering gives shorter runs), of at most two
    // chunks of the stage kernel (the march kernel's straight-line reach)
    const int seg = 2 * wdg::wedge_chunk_elems(ctx->N, ctx->bits);
    std::vector<int2> cols;
    for (int64_t k = 0; k < Kw; ++k) {
      const bool stacked = k > 0 && ctx->conn[size_t(k - 1) * wdg::kConnStride + 1] == k &&
                           ctx->conn[size_t(k) * wdg::kConnStride] == k - 1 && cols.back().y < seg;
      if (stacked) {
        cols.back().y += 1;
      } else {
        cols.push_back(make_int2(int(k), 1));
      }
    }
    ctx->ncols = int(cols.size());
    HIPCHK(hipMalloc(&ctx->dCols, cols.size() * sizeof(int2)));
    HIPCHK(hipMemcpyAsync(ctx->dCols, cols.data(), cols.size() * sizeof(int2), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  if (Kw > 0 && ctx->N >= 4) {
    // node-lane kernel: D_r, D_s, then E^a and E^b of the three edges ([edge][i][q])
    std::vector<double> ops;
    ops.insert(ops.end(), R.Dr.begin(), R.Dr.end());
    ops.insert(ops.end(), R.Ds.begin(), R.Ds.end());
    for (int e = 0; e < 3; ++e) ops.insert(ops.end(), R.Ea[e].begin(), R.Ea[e].end());
    for (int e = 0; e < 3; ++e) ops.insert(ops.end(), R.Eb[e].begin(), R.Eb[e].end());
    std::vector<unsigned char> buf(ops.size() * ts);
    for (size_t i = 0; i < ops.size(); ++i) {
      if (ctx->bits == 32) reinterpret_cast<float*>(buf.data())[i] = float(ops[i]);
      else reinterpret_cast<double*>(buf.data())[i] = ops[i];
    }
    HIPCHK(hipMalloc(&ctx->dOpsW, buf.size()));
    HIPCHK(hipMemcpyAsync(ctx->dOpsW, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  if (Kt > 0 && Kw > 0) {
    // the second stream of the hybrid stage (non-blocking: ordered with the
    // solver stream only through the fork and join events)
    HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  if (Kt > 0) {
    const TetOps& Tt = *ctx->tref;
    const int NPt = Tt.NP, NT = R.NT;
    HIPCHK(hipMalloc(&ctx->dGeoT, size_t(Kt) * wdg::kTetGeoStride * ts));
    HIPCHK(hipMalloc(&ctx->dConnT, size_t(Kt) * wdg::kTetConnStride * sizeof(int32_t)));
    HIPCHK(hipMalloc(&ctx->dAuxT, size_t(Kt) * wdg::kTetAuxStride * sizeof(double)));
    const size_t nops = 3 * size_t(NPt) * NPt + size_t(NPt) * 4 * NT;
    HIPCHK(hipMalloc(&ctx->dOpsT, nops * ts));
    HIPCHK(hipMalloc(&ctx->dMt, size_t(NPt) * NPt * sizeof(double)));
    std::vector<double> ops;
    ops.reserve(nops);
    ops.insert(ops.end(), Tt.Dr.begin(), Tt.Dr.end());
    ops.insert(ops.end(), Tt.Ds.begin(), Tt.Ds.end());
    ops.insert(ops.end(), Tt.Dt.begin(), Tt.Dt.end());
    ops.insert(ops.end(), Tt.LIFT.begin(), Tt.LIFT.end());
    std::vector<unsigned char> buf(nops * ts);
    for (size_t i = 0; i < nops; ++i) {
      if (ctx->bits == 32) reinterpret_cast<float*>(buf.data())[i] = float(ops[i]);
      else reinterpret_cast<double*>(buf.data())[i] = ops[i];
    }
    HIPCHK(hipMemcpyAsync(ctx->dOpsT, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->dMt, Tt.M.data(), Tt.M.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->dConnT, ctx->connT.data(), ctx->connT.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int rc = upload_tet_geometry(ctx);
    if (rc) return rc;
  }
  if (!ctx->mort.empty()) {
    const size_t nm = ctx->mort.size();
    const int NT = R.NT, Nq = R.Nq, NTP = (NT + 3) / 4 * 4;
    std::vector<int32_t> mi(nm * wdg::kMortIntStride, 0);
    for (size_t m = 0; m < nm; ++m) {
      const MortarHost& M = ctx->mort[m];
      int32_t* o = &mi[m * wdg::kMortIntStride];
      o[0] = int32_t(M.k);
      o[1] = M.e;
      o[2] = M.diag;
      o[3] = int32_t(M.t[0]);
      o[4] = M.tf[0];
      o[5] = int32_t(M.t[1]);
      o[6] = M.tf[1];
    }
    const std::vector<double> tabs = mortar_tables(R);
    if (int(tabs.size()) != wdg::mortar_table_size(ctx->N)) return fail(ctx, WDG_ERR_HIP, "mortar table layout");
    const std::vector<unsigned char> tabT = to_precision(tabs, ctx->bits);
    const std::vector<unsigned char> cores = to_precision(mortar_cores(R, ctx->mort), ctx->bits);
    HIPCHK(hipMalloc(&ctx->dMortI, mi.size() * sizeof(int32_t)));
    HIPCHK(hipMalloc(&ctx->dMortG, nm * wdg::kMortGeoStride * sizeof(double)));
    HIPCHK(hipMalloc(&ctx->dMortTab, tabT.size()));
    HIPCHK(hipMalloc(&ctx->dMortC, cores.size()));
    HIPCHK(hipMalloc(&ctx->dMortB, nm * 2 * Nq * NTP * ts));
    HIPCHK(hipMalloc(&ctx->dMortF, nm * 2 * 2 * NT * ts));
    HIPCHK(hipMemcpyAsync(ctx->dMortI, mi.data(), mi.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->dMortTab, tabT.data(), tabT.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->dMortC, cores.data(), cores.size(), hipMemcpyHostToDevice, ctx->stream));
    int rc = upload_mortar_geometry(ctx);
    if (rc) return rc;
  }
  ctx->state = kMesh;
  return WDG_OK;
}

int wdg_set_material(wdg_ctx* ctx, const double* c, const double* rho) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "set_material before set_mesh");
  if (!c || !rho) return fail(ctx, WDG_ERR_ARG, "null material array");
  for (int64_t k = 0; k < ctx->K; ++k)
    if (!(c[k] > 0) || !(rho[k] > 0) || !std::isfinite(c[k]) || !std::isfinite(rho[k]))
      return fail(ctx, WDG_ERR_ARG, "material must be positive and finite");
  ctx->c.assign(c, c + ctx->K);
  ctx->rho.assign(rho, rho + ctx->K);
  for (auto& s : ctx->src) {
    double r, ss, t;
    if (s.elem < ctx->Kw) wedge_ref_coords(&ctx->X[s.elem * 18], s.xyz, r, ss, t);
    else tet_ref_coords(&ctx->Xt[(s.elem - ctx->Kw) * 12], s.xyz, r, ss, t);
    s.vec = mass_inverse_times(ctx, s.elem, ctx->rho[s.elem] * ctx->c[s.elem] * ctx->c[s.elem], r, ss, t);
  }
  // tetrahedron material slots: kappa, 1/rho, rho c and the impedance sums per face
  for (int64_t k = 0; k < ctx->Kt; ++k) {
    const int64_t gk = ctx->Kw + k;
    double* g = &ctx->geoT[k * wdg::kTetGeoStride];
    const double Z = ctx->rho[gk] * ctx->c[gk];
    g[9] = ctx->rho[gk] * ctx->c[gk] * ctx->c[gk];
    g[10] = 1.0 / ctx->rho[gk];
    g[11] = Z;
    for (int f = 0; f < 4; ++f) {
      const int nb = ctx->connT[k * wdg::kTetConnStride + f];
      g[28 + f] = Z + (nb >= 0 ? ctx->rho[nb] * ctx->c[nb] : Z);
    }
  }
  if (!ctx->host_only) {
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->Kw > 0) {
      double *dc = nullptr, *dr = nullptr;
      HIPCHK(hipMalloc(&dc, ctx->K * sizeof(double)));
      HIPCHK(hipMalloc(&dr, ctx->K * sizeof(double)));
      HIPCHK(hipMemcpyAsync(dc, c, ctx->K * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(dr, rho, ctx->K * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(wdg::launch_material(ctx->bits, ctx->Kw, dc, dr, ctx->dConn, ctx->dGeo, ctx->dAux, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipFree(dc));
      HIPCHK(hipFree(dr));
    }
    int rc = upload_tet_geometry(ctx);
    if (!rc) rc = upload_mortar_geometry(ctx);
    if (!rc) rc = upload_sources(ctx);
    if (rc) return rc;
  }
  ctx->state = std::max(ctx->state, int(kMaterial));
  return WDG_OK;
}

int wdg_set_boundary(wdg_ctx* ctx, int bc) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (bc != WDG_BC_DIRICHLET_P0 && bc != WDG_BC_RIGID) return fail(ctx, WDG_ERR_ARG, "unknown boundary condition");
  ctx->bc = bc;
  return WDG_OK;
}

int wdg_set_flux(wdg_ctx* ctx, int flux) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (flux != WDG_FLUX_UPWIND && flux != WDG_FLUX_CENTRAL) return fail(ctx, WDG_ERR_ARG, "unknown flux");
  ctx->flux = flux;
  return WDG_OK;
}

int wdg_set_mass(wdg_ctx* ctx, int mass) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (mass != WDG_MASS_EXACT && mass != WDG_MASS_LUMPED) return fail(ctx, WDG_ERR_ARG, "unknown mass treatment");
  ctx->mass = mass;
  // source vectors kappa (M^k)^-1 l(x_s) follow the mass treatment
  for (auto& s : ctx->src) {
    double r, ss, t;
    if (s.elem < ctx->Kw) wedge_ref_coords(&ctx->X[s.elem * 18], s.xyz, r, ss, t);
    else tet_ref_coords(&ctx->Xt[(s.elem - ctx->Kw) * 12], s.xyz, r, ss, t);
    s.vec = mass_inverse_times(ctx, s.elem, ctx->rho[s.elem] * ctx->c[s.elem] * ctx->c[s.elem], r, ss, t);
  }
  if (!ctx->host_only && ctx->state >= kMesh) {
    HIPCHK(hipSetDevice(ctx->device));
    int rc = upload_vertical_mass(ctx);
    if (rc) return rc;
    return upload_sources(ctx);
  }
  return WDG_OK;
}

int wdg_set_layer_march(wdg_ctx* ctx, int mode) {
  if (!ctx) return WDG_ERR_ARG;
  if (mode != WDG_MARCH_OFF && mode != WDG_MARCH_CHUNK && mode != WDG_MARCH_COLUMN)
    return fail(ctx, WDG_ERR_ARG, "unknown layer marching mode");
  ctx->layer_march = mode;
  return WDG_OK;
}

int wdg_set_overlap(wdg_ctx* ctx, int enable) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->overlap = enable != 0;
  return WDG_OK;
}

int wdg_set_tet_blocks(wdg_ctx* ctx, int blocks) {
  if (!ctx) return WDG_ERR_ARG;
  if (blocks < 0) return fail(ctx, WDG_ERR_ARG, "negative block count");
  ctx->tet_blocks = blocks;
  return WDG_OK;
}

int wdg_set_wedge_kernel(wdg_ctx* ctx, int variant) {
  if (!ctx) return WDG_ERR_ARG;
  if (variant != WDG_WEDGE_AUTO && variant != WDG_WEDGE_LEVEL && variant != WDG_WEDGE_NODE)
    return fail(ctx, WDG_ERR_ARG, "unknown wedge kernel");
  ctx->wedge_kernel = variant;
  return WDG_OK;
}

int wdg_set_wedge_block(wdg_ctx* ctx, int elements) {
  if (!ctx) return WDG_ERR_ARG;
  if (elements != 0) {
    bool ok = false;
    for (int k = 0; k < wdg::kNodeEpbVariants; ++k) ok = ok || wdg::wedge_node_epb(ctx->N, ctx->bits, k) == elements;
    if (!ok) return fail(ctx, WDG_ERR_ARG, "no node-lane wedge kernel with that many elements per block");
  }
  ctx->wedge_block = elements;
  return WDG_OK;
}

int wdg_set_tet_kernel(wdg_ctx* ctx, int variant) {
  if (!ctx) return WDG_ERR_ARG;
  if (variant != WDG_TET_MFMA && variant != WDG_TET_VALU) return fail(ctx, WDG_ERR_ARG, "unknown tetrahedron kernel");
  ctx->tet_valu = variant == WDG_TET_VALU;
  return WDG_OK;
}

int wdg_num_nodes(const wdg_ctx* ctx, int64_t* n) {
  if (!ctx || !n) return WDG_ERR_ARG;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "no mesh");
  *n = ctx->nodes();
  return WDG_OK;
}

int wdg_get_node_coords(const wdg_ctx* ctx, double* xyz) {
  if (!ctx || !xyz) return WDG_ERR_ARG;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "no mesh");
  const RefOps& R = *ctx->ref;
  for (int64_t k = 0; k < ctx->Kt; ++k) {
    const TetOps& Tt = *ctx->tref;
    const double* x = &ctx->Xt[k * 12];
    for (int i = 0; i < Tt.NP; ++i) {
      const double lam[4] = {-(1.0 + Tt.r[i] + Tt.s[i] + Tt.t[i]) / 2.0, (1.0 + Tt.r[i]) / 2.0, (1.0 + Tt.s[i]) / 2.0,
                             (1.0 + Tt.t[i]) / 2.0};
      double* o = xyz + 3 * (ctx->node_base(ctx->Kw + k) + i);
      for (int d = 0; d < 3; ++d) {
        double acc = 0;
        for (int v = 0; v < 4; ++v) acc += lam[v] * x[3 * v + d];
        o[d] = acc;
      }
    }
  }
  for (int64_t k = 0; k < ctx->Kw; ++k) {
    const double* x = &ctx->X[k * 18];
    for (int j = 0; j < R.Nq; ++j)
      for (int i = 0; i < R.NT; ++i) {
        const double r = R.r[i], s = R.s[i], t = R.t[j];
        const double lam[3] = {-(r + s) / 2.0, (1.0 + r) / 2.0, (1.0 + s) / 2.0};
        double* o = xyz + 3 * (k * R.NP + j * R.NT + i);
        for (int d = 0; d < 3; ++d) {
          double acc = 0;
          for (int v = 0; v < 3; ++v) acc += lam[v] * (x[3 * v + d] * (1 - t) / 2 + x[3 * (v + 3) + d] * (1 + t) / 2);
          o[d] = acc;
        }
      }
  }
  return WDG_OK;
}

int wdg_set_fields(wdg_ctx* ctx, const double* p, const double* ux, const double* uy, const double* uz) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (ctx->state < kMaterial) return fail(ctx, WDG_ERR_STATE, "set_fields before set_material");
  if (!p || !ux || !uy || !uz) return fail(ctx, WDG_ERR_ARG, "null field array");
  if (ctx->host_only) return fail(ctx, WDG_ERR_STATE, "host-only context cannot hold fields");
  const int64_t n = ctx->nodes();
  if (!finite_all(p, n) || !finite_all(ux, n) || !finite_all(uy, n) || !finite_all(uz, n))
    return fail(ctx, WDG_ERR_UNSTABLE, "non-finite field values");
  HIPCHK(hipSetDevice(ctx->device));
  int rc = upload_state(ctx, ctx->dU[ctx->cur], p, ux, uy, uz);
  if (rc) return rc;
  ctx->rec_steps = 0;
  ctx->state = kFields;
  return WDG_OK;
}

int wdg_get_fields(const wdg_ctx* ctx, double* p, double* ux, double* uy, double* uz) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->state < kFields) return fail(ctx, WDG_ERR_STATE, "no fields");
  HIPCHK(hipSetDevice(ctx->device));
  return download_state(ctx, ctx->dU[ctx->cur], p, ux, uy, uz);
}

int wdg_bind_device_state(wdg_ctx* ctx, void* d_U, void* d_res, void* hip_stream) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->host_only || ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "bind before set_mesh");
  if ((d_U == nullptr) != (d_res == nullptr)) return fail(ctx, WDG_ERR_ARG, "bind both state buffers or none");
  if ((reinterpret_cast<uintptr_t>(d_U) | reinterpret_cast<uintptr_t>(d_res)) & 255)
    return fail(ctx, WDG_ERR_ARG, "state buffers must be 256-byte aligned");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (!d_U) return WDG_OK;
  const size_t nstate = size_t(ctx->nodes()) * 4 * ctx->tsize();
  HIPCHK(hipMemcpyAsync(d_U, ctx->dU[ctx->cur], nstate, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(d_res, ctx->dRes, nstate, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->own_state) {
    dfree(ctx->dU[0]);
    dfree(ctx->dU[1]);
    dfree(ctx->dRes);
  }
  ctx->dU[0] = d_U;
  ctx->dU[1] = static_cast<unsigned char*>(d_U) + nstate;
  ctx->dRes = d_res;
  ctx->cur = 0;
  ctx->own_state = false;
  return WDG_OK;
}

int wdg_add_ricker_source(wdg_ctx* ctx, const double xyz[3], double f0, double t0, double amp, int* id) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;  // the recorded forward no longer matches the problem
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "source before set_mesh");
  if (!xyz || !(f0 > 0) || !std::isfinite(t0) || !std::isfinite(amp)) return fail(ctx, WDG_ERR_ARG, "bad source");
  if (ctx->src.size() >= size_t(wdg::kMaxSources)) return fail(ctx, WDG_ERR_ARG, "too many sources");
  double r, s, t;
  const int64_t k = locate(ctx, xyz, r, s, t);
  if (k < 0) return fail(ctx, WDG_ERR_OUTSIDE, "source outside the mesh");
  Source S;
  std::copy(xyz, xyz + 3, S.xyz);
  S.f0 = f0;
  S.t0 = t0;
  S.amp = amp;
  S.elem = k;
  S.vec = mass_inverse_times(ctx, k, ctx->rho[k] * ctx->c[k] * ctx->c[k], r, s, t);
  ctx->src.push_back(S);
  if (id) *id = int(ctx->src.size()) - 1;
  if (!ctx->host_only) {
    HIPCHK(hipSetDevice(ctx->device));
    return upload_sources(ctx);
  }
  return WDG_OK;
}

int wdg_set_receivers(wdg_ctx* ctx, int64_t n, const double* xyz) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "receivers before set_mesh");
  if (n < 0 || (n > 0 && !xyz)) return fail(ctx, WDG_ERR_ARG, "bad receivers");
  const RefOps& R = *ctx->ref;
  std::vector<int64_t> base(static_cast<size_t>(n));
  std::vector<int> nn(static_cast<size_t>(n));
  std::vector<double> rows(static_cast<size_t>(n) * R.NP, 0.0);
  for (int64_t q = 0; q < n; ++q) {
    double r, s, t;
    const int64_t k = locate(ctx, xyz + 3 * q, r, s, t);
    if (k < 0) return fail(ctx, WDG_ERR_OUTSIDE, "receiver " + std::to_string(q) + " outside the mesh");
    base[q] = ctx->node_base(k);
    nn[q] = ctx->NPof(k);
    std::vector<double> b;
    if (k < ctx->Kw) {
      wedge_basis(R, r, s, t, b);
    } else {
      b.resize(ctx->tref->NP);
      ctx->tref->basis(r, s, t, b.data());
    }
    std::copy(b.begin(), b.end(), rows.begin() + q * R.NP);
  }
  ctx->rec_steps = 0;
  ctx->rec_xyz.assign(xyz, xyz + 3 * n);
  if (ctx->host_only) {
    ctx->nrec = n;
    return WDG_OK;
  }
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dfree(ctx->dRecBase);
  dfree(ctx->dRecNN);
  dfree(ctx->dRecRows);
  dfree(ctx->dRecBuf);
  ctx->rec_cap = 0;
  ctx->nrec = n;
  if (n == 0) return WDG_OK;
  HIPCHK(hipMalloc(&ctx->dRecBase, base.size() * sizeof(int64_t)));
  HIPCHK(hipMalloc(&ctx->dRecNN, nn.size() * sizeof(int)));
  HIPCHK(hipMalloc(&ctx->dRecRows, rows.size() * ctx->tsize()));
  HIPCHK(hipMemcpyAsync(ctx->dRecBase, base.data(), base.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->dRecNN, nn.data(), nn.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  if (ctx->bits == 32) {
    const std::vector<float> rf(rows.begin(), rows.end());
    HIPCHK(hipMemcpyAsync(ctx->dRecRows, rf.data(), rf.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  } else {
    HIPCHK(hipMemcpyAsync(ctx->dRecRows, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  return WDG_OK;
}

int wdg_read_receivers(const wdg_ctx* ctx, double* out, int64_t* steps) {
  if (!ctx || !steps) return WDG_ERR_ARG;
  *steps = ctx->rec_steps;
  if (!out || ctx->rec_steps == 0 || ctx->nrec == 0) return WDG_OK;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipMemcpyAsync(out, ctx->dRecBuf, size_t(ctx->rec_steps * ctx->nrec) * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

int wdg_stable_dt(const wdg_ctx* ctx, double cfl, double* dt) {
  if (!ctx || !dt) return WDG_ERR_ARG;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "no mesh");
  if (!(cfl > 0)) return fail(ctx, WDG_ERR_ARG, "cfl must be positive");
  const int N = ctx->N;
  double worst = 0.0;
  for (int64_t k = 0; k < ctx->Kt; ++k) {
    // affine tetrahedron: J and J_f constant; J_f / J is stored per face
    double ratio = 0.0;
    for (int f = 0; f < 4; ++f) ratio = std::max(ratio, ctx->geoT[k * wdg::kTetGeoStride + 12 + 4 * f]);
    worst = std::max(worst, ctx->c[ctx->Kw + k] * (N + 1.0) * (N + 3.0) / 3.0 * ratio);
  }
  for (int64_t k = 0; k < ctx->Kw; ++k) {
    const double* x = &ctx->X[k * 18];
    const double xr = 0.5 * (x[3] - x[0]), xs = 0.5 * (x[6] - x[0]);
    const double yr = 0.5 * (x[4] - x[1]), ys = 0.5 * (x[7] - x[1]);
    const double Jt = xr * ys - xs * yr;
    double h[3], Jmin = 1e300, Jf = 0.0;
    for (int v = 0; v < 3; ++v) {
      h[v] = x[3 * (v + 3) + 2] - x[3 * v + 2];
      Jmin = std::min(Jmin, 0.5 * Jt * h[v]);
    }
    for (int face = 0; face < 2; ++face) {
      const int o = face == 0 ? 0 : 9;
      const double ax = x[o + 3] - x[o], ay = x[o + 4] - x[o + 1], az = x[o + 5] - x[o + 2];
      const double bx = x[o + 6] - x[o], by = x[o + 7] - x[o + 1], bz = x[o + 8] - x[o + 2];
      const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
      Jf = std::max(Jf, 0.25 * std::sqrt(cx * cx + cy * cy + cz * cz));
    }
    for (int e = 0; e < 3; ++e) {
      const int a = e, b = (e + 1) % 3;
      const double ell = std::hypot(x[3 * b] - x[3 * a], x[3 * b + 1] - x[3 * a + 1]);
      Jf = std::max(Jf, 0.25 * ell * std::max(h[a], h[b]));
    }
    worst = std::max(worst, ctx->c[k] * (N + 1.0) * (N + 3.0) / 3.0 * Jf / Jmin);
  }
  *dt = cfl / worst;
  return WDG_OK;
}

int wdg_step(wdg_ctx* ctx, int64_t nsteps, double dt) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->state < kFields) return fail(ctx, WDG_ERR_STATE, "step before set_fields");
  if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(ctx, WDG_ERR_ARG, "bad step arguments");
  HIPCHK(hipSetDevice(ctx->device));
  int rc = ensure_receiver_capacity(ctx, ctx->rec_steps + nsteps);
  if (rc) return rc;
  const double t0 = ctx->time;
  const size_t SB = size_t(ctx->nodes()) * 4 * ctx->tsize();
  // X: the current state.  A recorded forward with the reverse sweep's store
  // kept writes step i of each segment into its slots as the sweep lays them
  // out (start state 10 i, stage inputs 10 i + 1..4, residuals 10 i + 5..9),
  // the next step's start into the next step's slot (the segment's first
  // slot after its last step: the sweep starts a segment from its checkpoint); the
  // state returns to the solver's buffers when that stops and at the end.
  void* X = ctx->dU[ctx->cur];
  auto settle = [&]() -> int {
    if (X != ctx->dU[ctx->cur]) {
      HIPCHK(hipMemcpyAsync(ctx->dU[ctx->cur], X, SB, hipMemcpyDeviceToDevice, ctx->stream));
      X = ctx->dU[ctx->cur];
    }
    return WDG_OK;
  };
  for (int64_t n = 0; n < nsteps; ++n) {
    if (ctx->recording) {
      // checkpoint at the start of every adj_every-th recorded step
      if (ctx->adj_steps == 0) ctx->adj_dt = dt;
      const int64_t g = ctx->adj_steps / ctx->adj_every;
      if (dt != ctx->adj_dt || ctx->adj_steps >= ctx->adj_ncap * ctx->adj_every) {
        ctx->recording = false;
      } else if (g > 0 && ctx->adj_steps % ctx->adj_every == 0) {
        HIPCHK(hipMemcpyAsync(static_cast<unsigned char*>(ctx->dAdjCp) + size_t(g) * SB, X, SB,
                              hipMemcpyDeviceToDevice, ctx->stream));
      }
    }
    // a recorded step's time as the reverse sweep computes it when it
    // recomputes the step (the same bits whichever calls the steps came in)
    const double tn = ctx->recording ? ctx->adj_t0 + double(ctx->adj_steps) * dt : t0 + double(n) * dt;
    if (ctx->recording && ctx->adj_tail) {
      const int64_t i = ctx->adj_steps % ctx->adj_every;
      auto slot = [&](int64_t ii, int k) -> void* {
        return static_cast<unsigned char*>(ctx->dAdjStore) + size_t(10 * ii + k) * SB;
      };
      void* outs[5] = {slot(i, 1), slot(i, 2), slot(i, 3), slot(i, 4), slot((i + 1) % ctx->adj_every, 0)};
      const void* in = X;
      for (int s = 0; s < 5; ++s) {
        const int flags = (s == 0 ? 0 : wdg::kReadRes) | wdg::kWriteU | wdg::kResOut;
        rc = launch_stage(ctx, in, outs[s], slot(i, s > 0 ? 4 + s : 5), kRkA[s], kRkB[s], dt, tn + kRkC[s] * dt,
                          flags, 1.0, slot(i, 5 + s));
        if (rc) return rc;
        in = outs[s];
      }
      X = outs[4];
    } else {
      rc = settle();
      if (rc) return rc;
      for (int s = 0; s < 5; ++s) {
        const int flags = (s == 0 ? 0 : wdg::kReadRes) | wdg::kWriteU;
        rc = launch_stage(ctx, ctx->dU[ctx->cur], ctx->dU[1 - ctx->cur], ctx->dRes, kRkA[s], kRkB[s], dt,
                          tn + kRkC[s] * dt, flags);
        if (rc) return rc;
        ctx->cur = 1 - ctx->cur;
      }
      X = ctx->dU[ctx->cur];
    }
    if (ctx->nrec > 0) {
      HIPCHK(wdg::launch_receivers(ctx->bits, ctx->NP(), int(ctx->nrec), X, ctx->dRecBase, ctx->dRecNN,
                                   ctx->dRecRows, ctx->dRecBuf + ctx->rec_steps * ctx->nrec, ctx->stream));
      ctx->rec_steps += 1;
    }
    if (ctx->recording) ctx->adj_steps += 1;
  }
  rc = settle();
  if (rc) return rc;
  ctx->time = t0 + double(nsteps) * dt;
  return WDG_OK;
}

namespace {

// device buffers of one call, freed on every return path
struct DeviceScratch {
  std::vector<void*> p;
  hipError_t alloc(size_t bytes, void** out) {
    *out = nullptr;
    const hipError_t e = hipMalloc(out, bytes ? bytes : 1);
    if (e == hipSuccess) p.push_back(*out);
    return e;
  }
  ~DeviceScratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

}  // namespace

namespace {

int adjoint_supported(wdg_ctx* ctx) {
  if (ctx->state < kFields) return fail(ctx, WDG_ERR_STATE, "adjoint before set_fields");
  if (ctx->Kt > 0 || !ctx->mort.empty()) return fail(ctx, WDG_ERR_UNSUPPORTED, "adjoint: meshes of wedges only");
  if (ctx->mass != WDG_MASS_EXACT) return fail(ctx, WDG_ERR_UNSUPPORTED, "adjoint: exact mass only");
  if (ctx->nrec == 0) return fail(ctx, WDG_ERR_STATE, "adjoint without receivers");
  return WDG_OK;
}

// Reverse sweep of the solve of nsteps steps from time t0 whose states at the
// start of steps 0, C, 2C, ... are the states of cp.  Per segment (last
// first) the forward is recomputed from its checkpoint; when the memory
// budget allows, that pass keeps every stage input and stage right-hand side
// of the segment, otherwise it keeps the step-start states and every step
// recomputes its stages before its reverse stages.
// Memory plan of the reverse sweep's store: the stage store (keep: a whole
// segment's stage inputs and residuals, 10 states per step; else the
// step-start states and one step's stage data, C + 9), then the forward
// ping-pong pair and residual (3), then the adjoint state and the ping-pong
// pair of stage vectors (3).  Keep if it fits 85 % of the free memory (the
// kept store counts as free) or the set limit.
struct StorePlan {
  bool keep = false, reusable = false;
  size_t nstore = 0, need = 0;
};
int store_plan(wdg_ctx* ctx, int64_t C, int64_t nsteps, StorePlan& plan) {
  const size_t SB = size_t(ctx->nodes()) * 4 * ctx->tsize();
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  const size_t small = size_t(ctx->Kw) * (wdg::kGradStride + 2) * sizeof(double) +
                       (size_t(nsteps) * ctx->nrec + size_t(ctx->nrec) * ctx->NP()) * sizeof(double) +
                       size_t(ctx->nrec) * sizeof(int64_t);
  const size_t fixed = small + (size_t(256) << 20);
  const size_t avail = free_b + ctx->adj_store_bytes;
  const size_t budget = ctx->adj_mem_limit ? ctx->adj_mem_limit : size_t(0.85 * double(avail));
  plan.keep = fixed + size_t(10 * C + 6) * SB <= budget;
  plan.nstore = size_t(plan.keep ? 10 * C : C + 9);
  plan.need = (plan.nstore + 6) * SB;
  plan.reusable = ctx->dAdjStore && ctx->adj_store_bytes >= plan.need && ctx->adj_store_bytes <= plan.need + plan.need / 2;
  return WDG_OK;
}

// tail: the recorded forward kept its last segment's stage inputs and
// residuals in the store (valid only if the store is kept as it is)
int adjoint_backward(wdg_ctx* ctx, const void* cp, int64_t C, int64_t nsteps, double dt, double t0,
                     const double* weights, double* grad_c, double* grad_rho, bool tail) {
  const int N = ctx->N, NP = ctx->NP(), nrec = int(ctx->nrec);
  const int64_t K = ctx->Kw;
  const size_t SB = size_t(ctx->nodes()) * 4 * ctx->tsize();
  const int64_t ncp = (nsteps + C - 1) / C;
  const int mflags = (ctx->bc == WDG_BC_DIRICHLET_P0 ? wdg::kDirichlet : 0) |
                     (ctx->flux == WDG_FLUX_CENTRAL ? wdg::kCentral : 0);
  hipStream_t st = ctx->stream;

  // receivers become point sources of the adjoint: kappa (M^k)^-1 l(x_r)
  std::vector<int64_t> rbase(nrec);
  std::vector<double> rvec(size_t(nrec) * NP);
  for (int r = 0; r < nrec; ++r) {
    double rr, ss, tt;
    const int64_t k = locate(ctx, &ctx->rec_xyz[3 * r], rr, ss, tt);
    if (k < 0 || k >= ctx->Kw) return fail(ctx, WDG_ERR_OUTSIDE, "receiver outside the wedges");
    rbase[r] = ctx->node_base(k);
    const std::vector<double> v = mass_inverse_times(ctx, k, ctx->rho[k] * ctx->c[k] * ctx->c[k], rr, ss, tt);
    std::copy(v.begin(), v.end(), rvec.begin() + size_t(r) * NP);
  }
  // memory: keep the whole segment's stage data (10 states per step) if it fits
  StorePlan plan;
  int rc0 = store_plan(ctx, C, nsteps, plan);
  if (rc0) return rc0;
  const bool keep = plan.keep;
  const size_t nstore = plan.nstore;
  const bool fresh = !plan.reusable;
  if (fresh) {
    HIPCHK(hipStreamSynchronize(st));
    dfree(ctx->dAdjStore);
    ctx->adj_store_bytes = 0;
    HIPCHK(hipMalloc(&ctx->dAdjStore, plan.need));
    ctx->adj_store_bytes = plan.need;
  }
  // the recorded forward left the last segment's stage data in the store
  const bool use_tail = tail && keep && !fresh;
  ctx->adj_tail = false;  // the sweep overwrites the store

  DeviceScratch ds;
  void *pg, *pw, *pv, *pb;
  void* const store = ctx->dAdjStore;
  void* const tmp = static_cast<unsigned char*>(store) + nstore * SB;
  void* const adj = static_cast<unsigned char*>(tmp) + 3 * SB;
  HIPCHK(ds.alloc(size_t(K) * (wdg::kGradStride + 2) * sizeof(double), &pg));
  HIPCHK(ds.alloc(size_t(nsteps) * nrec * sizeof(double), &pw));
  HIPCHK(ds.alloc(rvec.size() * sizeof(double), &pv));
  HIPCHK(ds.alloc(rbase.size() * sizeof(int64_t), &pb));
  auto at = [SB](const void* base, int64_t i) -> void* {
    return const_cast<unsigned char*>(static_cast<const unsigned char*>(base)) + size_t(i) * SB;
  };
  // gradient accumulators: kGradStride FP64 slots per wedge hold the FP64
  // record or the FP32 record (sums and compensations) alike
  void* gacc = pg;
  double* gout = static_cast<double*>(pg) + K * wdg::kGradStride;
  const double* dw = static_cast<const double*>(pw);
  HIPCHK(hipMemcpyAsync(pw, weights, size_t(nsteps) * nrec * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pv, rvec.data(), rvec.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pb, rbase.data(), rbase.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(gacc, 0, size_t(K) * wdg::kGradStride * sizeof(double), st));
  HIPCHK(hipMemsetAsync(adj, 0, SB * 3, st));

  // store slots: keep: step i of the segment holds its start state (0; unused
  // for the first step), stage inputs 1..4 (1..4) and the residuals after
  // stages 0..4 (5..9); otherwise the step-start states (0..C-1), then one
  // step's stage inputs and residuals
  auto slot = [&](int64_t i, int k) -> void* {
    if (keep) return at(store, 10 * i + k);
    return k == 0 ? at(store, i) : at(store, C + k - 1);
  };
  // one forward step from X; stage s writes outs[s] (null: no state output)
  // and, if routs, keeps its residual in routs[s] (read back by stage s + 1)
  // instead of updating one residual in place
  auto forward_step = [&](const void* X, void* const* outs, void* const* routs, double tn) -> int {
    const void* in = X;
    for (int s = 0; s < 5; ++s) {
      const int flags = (s == 0 ? 0 : wdg::kReadRes) | (outs[s] ? wdg::kWriteU : 0) | (routs ? wdg::kResOut : 0);
      void* res = routs ? (s > 0 ? routs[s - 1] : routs[0]) : at(tmp, 2);
      const int rc = launch_stage(ctx, in, outs[s], res, kRkA[s], kRkB[s], dt, tn + kRkC[s] * dt, flags, 1.0,
                                  routs ? routs[s] : nullptr, true);
      if (rc) return rc;
      in = outs[s];
    }
    return WDG_OK;
  };

  void* Ua = at(adj, 0);
  int sc = 1;
  HIPCHK(wdg::launch_inject(ctx->bits, NP, nrec, static_cast<const int64_t*>(pb), static_cast<const double*>(pv),
                            dw + (nsteps - 1) * nrec, kRkB[4], Ua, at(adj, sc), st));
  for (int64_t g = ncp - 1; g >= 0; --g) {
    const int64_t n0 = g * C, n1 = std::min(n0 + C, nsteps);
    // step-start states: the segment's first is its checkpoint, read in place
    auto start = [&](int64_t i) -> void* { return i == 0 ? at(cp, g) : slot(i, 0); };
    for (int64_t n = n0; n < n1 && !(use_tail && g == ncp - 1); ++n) {
      const int64_t i = n - n0;
      void* next = n + 1 < n1 ? slot(i + 1, 0) : nullptr;
      int rc;
      if (keep) {
        void* outs[5] = {slot(i, 1), slot(i, 2), slot(i, 3), slot(i, 4), next};
        void* routs[5] = {slot(i, 5), slot(i, 6), slot(i, 7), slot(i, 8), slot(i, 9)};
        rc = forward_step(start(i), outs, routs, t0 + double(n) * dt);
      } else {
        if (!next) break;
        void* outs[5] = {at(tmp, 0), at(tmp, 1), at(tmp, 0), at(tmp, 1), next};
        rc = forward_step(start(i), outs, nullptr, t0 + double(n) * dt);
      }
      if (rc) return rc;
    }
    for (int64_t n = n1 - 1; n >= n0; --n) {
      const int64_t i = n - n0;
      void* Us[5];
      void* Rs[5];
      if (keep) {
        for (int s = 0; s < 5; ++s) {
          Us[s] = s ? slot(i, s) : start(i);
          Rs[s] = slot(i, 5 + s);
        }
      } else {
        // the stage data of this step go to the shared slots 1..9
        void* outs[5] = {slot(0, 1), slot(0, 2), slot(0, 3), slot(0, 4), nullptr};
        void* routs[5] = {slot(0, 5), slot(0, 6), slot(0, 7), slot(0, 8), slot(0, 9)};
        const int rc = forward_step(start(i), outs, routs, t0 + double(n) * dt);
        if (rc) return rc;
        Us[0] = start(i);
        for (int s = 1; s < 5; ++s) Us[s] = outs[s - 1];
        for (int s = 0; s < 5; ++s) Rs[s] = routs[s];
      }
      for (int s = 4; s >= 0; --s) {
        void* sig = at(adj, sc);
        // U~ += dt A sig;  sig <- a_s sig + b_{s-1} U~  (b of the previous step's last stage at s = 0);
        // the same kernel accumulates the stage's gradient terms from Us[s] and the
        // forward residual Rs[s] (mass terms weighted by b_s)
        const int rc = launch_stage(ctx, sig, at(adj, 3 - sc), Ua, 1.0, s > 0 ? kRkB[s - 1] : kRkB[4], dt, 0.0,
                                    wdg::kReadRes | wdg::kWriteU | wdg::kGrad, kRkA[s], nullptr, false, Us[s], Rs[s],
                                    gacc, kRkB[s]);
        if (rc) return rc;
        sc = 3 - sc;
      }
      if (n > 0)
        HIPCHK(wdg::launch_inject(ctx->bits, NP, nrec, static_cast<const int64_t*>(pb),
                                  static_cast<const double*>(pv), dw + (n - 1) * nrec, kRkB[4], Ua, at(adj, sc), st));
    }
  }
  HIPCHK(wdg::launch_grad_combine(ctx->bits, K, gacc, ctx->dGeo, ctx->dConn, mflags, gout, gout + K, st));
  HIPCHK(hipMemcpyAsync(grad_c, gout, size_t(K) * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(grad_rho, gout + K, size_t(K) * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return WDG_OK;
}

// stage timing off for the duration of an adjoint call
struct TimingOff {
  wdg_ctx* c;
  bool t;
  explicit TimingOff(wdg_ctx* ctx) : c(ctx), t(ctx->timing) { ctx->timing = false; }
  ~TimingOff() { c->timing = t; }
};

}  // namespace

int wdg_adjoint_gradient(wdg_ctx* ctx, int64_t nsteps, double dt, const double* weights, int64_t checkpoint_every,
                         double* grad_c, double* grad_rho) {
  if (!ctx) return WDG_ERR_ARG;
  if (nsteps < 1 || !(dt > 0) || !std::isfinite(dt) || checkpoint_every < 1 || !weights || !grad_c || !grad_rho)
    return fail(ctx, WDG_ERR_ARG, "bad adjoint arguments");
  int rc = adjoint_supported(ctx);
  if (rc) return rc;
  if (!finite_all(weights, nsteps * ctx->nrec)) return fail(ctx, WDG_ERR_ARG, "non-finite adjoint weights");
  HIPCHK(hipSetDevice(ctx->device));
  TimingOff off(ctx);
  const size_t SB = size_t(ctx->nodes()) * 4 * ctx->tsize();
  const int64_t C = std::min(checkpoint_every, nsteps);
  const int64_t ncp = (nsteps + C - 1) / C;
  const double t0 = ctx->time;
  hipStream_t st = ctx->stream;
  DeviceScratch ds;
  void *cp, *tmp;
  HIPCHK(ds.alloc(SB * size_t(ncp), &cp));
  HIPCHK(ds.alloc(SB * 4, &tmp));  // stage ping-pong pair, residual, step state
  auto at = [SB](void* base, int64_t i) -> void* { return static_cast<unsigned char*>(base) + size_t(i) * SB; };
  // forward sweep: checkpoint g holds the state at the start of step g C
  HIPCHK(hipMemcpyAsync(cp, ctx->dU[ctx->cur], SB, hipMemcpyDeviceToDevice, st));
  const void* x = cp;
  for (int64_t n = 0; n < (ncp - 1) * C; ++n) {
    const bool ck = (n + 1) % C == 0;
    void* outs[5] = {at(tmp, 0), at(tmp, 1), at(tmp, 0), at(tmp, 1), ck ? at(cp, (n + 1) / C) : at(tmp, 3)};
    const void* in = x;
    for (int s = 0; s < 5; ++s) {
      rc = launch_stage(ctx, in, outs[s], at(tmp, 2), kRkA[s], kRkB[s], dt, t0 + double(n) * dt + kRkC[s] * dt,
                        (s == 0 ? 0 : wdg::kReadRes) | wdg::kWriteU);
      if (rc) return rc;
      in = outs[s];
    }
    x = outs[4];
  }
  return adjoint_backward(ctx, cp, C, nsteps, dt, t0, weights, grad_c, grad_rho, false);
}

int wdg_adjoint_record(wdg_ctx* ctx, int64_t checkpoint_every, int64_t max_steps) {
  if (!ctx) return WDG_ERR_ARG;
  ctx->recording = false;
  if (checkpoint_every < 1 || max_steps < 1) return fail(ctx, WDG_ERR_ARG, "bad recording arguments");
  int rc = adjoint_supported(ctx);
  if (rc) return rc;
  HIPCHK(hipSetDevice(ctx->device));
  const size_t SB = size_t(ctx->nodes()) * 4 * ctx->tsize();
  const int64_t ncap = (max_steps + checkpoint_every - 1) / checkpoint_every;
  if (!ctx->dAdjCp || ctx->adj_cp_bytes != SB * size_t(ncap)) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    dfree(ctx->dAdjCp);
    ctx->adj_cp_bytes = 0;
    HIPCHK(hipMalloc(&ctx->dAdjCp, SB * size_t(ncap)));
    ctx->adj_cp_bytes = SB * size_t(ncap);
  }
  HIPCHK(hipMemcpyAsync(ctx->dAdjCp, ctx->dU[ctx->cur], SB, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->adj_every = checkpoint_every;
  ctx->adj_ncap = ncap;
  ctx->adj_steps = 0;
  ctx->adj_t0 = ctx->time;
  ctx->adj_dt = 0.0;
  // with the reverse sweep's store already kept in the whole-segment layout
  // (an earlier gradient call), the forward writes into it what the sweep
  // would recompute for the last segment
  StorePlan plan;
  rc = store_plan(ctx, checkpoint_every, max_steps, plan);
  if (rc) return rc;
  ctx->adj_tail = plan.keep && plan.reusable;
  ctx->recording = true;
  return WDG_OK;
}

int wdg_adjoint_gradient_recorded(wdg_ctx* ctx, const double* weights, double* grad_c, double* grad_rho,
                                  int64_t* nsteps) {
  if (!ctx) return WDG_ERR_ARG;
  if (!ctx->recording || ctx->adj_steps < 1) return fail(ctx, WDG_ERR_STATE, "no valid forward recording");
  if (nsteps) *nsteps = ctx->adj_steps;
  if (!weights || !grad_c || !grad_rho) return fail(ctx, WDG_ERR_ARG, "bad adjoint arguments");
  int rc = adjoint_supported(ctx);
  if (rc) return rc;
  if (!finite_all(weights, ctx->adj_steps * ctx->nrec)) return fail(ctx, WDG_ERR_ARG, "non-finite adjoint weights");
  HIPCHK(hipSetDevice(ctx->device));
  TimingOff off(ctx);
  return adjoint_backward(ctx, ctx->dAdjCp, ctx->adj_every, ctx->adj_steps, ctx->adj_dt, ctx->adj_t0, weights,
                          grad_c, grad_rho, ctx->adj_tail);
}

int wdg_set_adjoint_memory_limit(wdg_ctx* ctx, int64_t bytes) {
  if (!ctx || bytes < 0) return WDG_ERR_ARG;
  ctx->adj_mem_limit = size_t(bytes);
  ctx->adj_tail = false;
  if (ctx->dAdjStore) {
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    dfree(ctx->dAdjStore);
    ctx->adj_store_bytes = 0;
  }
  return WDG_OK;
}

int wdg_get_time(const wdg_ctx* ctx, double* t) {
  if (!ctx || !t) return WDG_ERR_ARG;
  *t = ctx->time;
  return WDG_OK;
}

int wdg_set_time(wdg_ctx* ctx, double t) {
  if (!ctx || !std::isfinite(t)) return WDG_ERR_ARG;
  ctx->recording = false;
  ctx->time = t;
  return WDG_OK;
}

int wdg_synchronize(wdg_ctx* ctx) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->host_only || ctx->state < kMesh) return WDG_OK;
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return WDG_OK;
}

int wdg_eval_rhs(wdg_ctx* ctx, double t, const double* in4, double* out4) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->state < kMaterial || ctx->host_only) return fail(ctx, WDG_ERR_STATE, "eval_rhs before set_material");
  if (!in4 || !out4) return fail(ctx, WDG_ERR_ARG, "null array");
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t n = ctx->nodes();
  const size_t nstate = size_t(n) * 4 * ctx->tsize();
  void *dIn = nullptr, *dOut = nullptr;
  HIPCHK(hipMalloc(&dIn, nstate));
  HIPCHK(hipMalloc(&dOut, nstate));
  int rc = upload_state(ctx, dIn, in4, in4 + n, in4 + 2 * n, in4 + 3 * n);
  if (!rc) rc = launch_stage(ctx, dIn, nullptr, dOut, 0.0, 0.0, 1.0, t, 0);
  if (!rc) rc = download_state(ctx, dOut, out4, out4 + n, out4 + 2 * n, out4 + 3 * n);
  (void)hipFree(dIn);
  (void)hipFree(dOut);
  return rc;
}

int wdg_energy(wdg_ctx* ctx, double* E) {
  if (!ctx || !E) return WDG_ERR_ARG;
  if (ctx->state < kFields) return fail(ctx, WDG_ERR_STATE, "energy before set_fields");
  HIPCHK(hipSetDevice(ctx->device));
  double acc = 0.0;
  if (ctx->Kw > 0) {
    int nb = 0;
    HIPCHK(wdg::launch_energy(ctx->N, ctx->bits, ctx->Kw, ctx->dU[ctx->cur], ctx->dAux, ctx->dMv, ctx->dM1,
                              ctx->dPartial, &nb, ctx->stream));
    std::vector<double> part(nb);
    HIPCHK(hipMemcpyAsync(part.data(), ctx->dPartial, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (double v : part) acc += v;
  }
  if (ctx->Kt > 0) {
    int nb = 0;
    const void* Ut = static_cast<const unsigned char*>(ctx->dU[ctx->cur]) + size_t(ctx->Kw) * ctx->NP() * 4 * ctx->tsize();
    HIPCHK(wdg::launch_energy_tet(ctx->N, ctx->bits, ctx->Kt, Ut, ctx->dAuxT, ctx->dMt, ctx->dPartial + 1024, &nb,
                                  ctx->stream));
    std::vector<double> part(nb);
    HIPCHK(hipMemcpyAsync(part.data(), ctx->dPartial + 1024, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (double v : part) acc += v;
  }
  *E = acc;
  return WDG_OK;
}

int wdg_kernel_timing(wdg_ctx* ctx, int enable) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->host_only || ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "timing needs a device mesh");
  ctx->timing = enable != 0;
  ctx->events_used = 0;
  return WDG_OK;
}

int wdg_read_kernel_timing_split(wdg_ctx* ctx, double* ms3, int64_t* launches) {
  if (!ctx || !ms3 || !launches) return WDG_ERR_ARG;
  if (ctx->host_only || ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "timing needs a device mesh");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double acc[3] = {0.0, 0.0, 0.0};
  const bool has_m = !ctx->mort.empty(), has_t = ctx->Kt > 0;
  for (size_t i = 0; i < ctx->events_used; ++i) {
    const auto& ev = ctx->events[i];
    const hipEvent_t wedge_start = has_m ? ev[1] : ev[0];
    const hipEvent_t wedge_end = has_t ? ev[2] : ev[3];
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, wedge_start, wedge_end));
    acc[0] += ms;  // wedge kernel
    if (has_t) {
      HIPCHK(hipEventElapsedTime(&ms, ev[2], ev[3]));
      acc[1] += ms;  // tetrahedron kernel
    }
    if (has_m) {
      HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
      acc[2] += ms;  // mortar kernel
    }
  }
  for (int i = 0; i < 3; ++i) ms3[i] = acc[i];
  *launches = int64_t(ctx->events_used);
  ctx->events_used = 0;
  return WDG_OK;
}

int wdg_read_kernel_timing(wdg_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!total_ms) return WDG_ERR_ARG;
  double ms3[3] = {0.0, 0.0, 0.0};
  const int rc = wdg_read_kernel_timing_split(ctx, ms3, launches);
  if (rc == WDG_OK) *total_ms = ms3[0] + ms3[1] + ms3[2];
  return rc;
}

int wdg_mortar_couplings(const wdg_ctx* ctx, int64_t cap, int64_t* faces, double* couplings, int64_t* count) {
  if (!ctx || !count || cap < 0) return WDG_ERR_ARG;
  if (ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "no mesh");
  const int64_t nm = int64_t(ctx->mort.size());
  *count = nm;
  const int64_t take = std::min(cap, nm);
  if (faces)
    for (int64_t m = 0; m < take; ++m) {
      const MortarHost& M = ctx->mort[m];
      int64_t* o = faces + 7 * m;
      o[0] = M.k;
      o[1] = M.e;
      o[2] = M.diag;
      o[3] = M.t[0];
      o[4] = M.tf[0];
      o[5] = M.t[1];
      o[6] = M.tf[1];
    }
  if (couplings && take > 0) {
    const int n = wdg::mort_core_n(ctx->N), npk = n * (n + 1) / 2, CS = wdg::mort_core_stride(ctx->N);
    const std::vector<MortarHost> part(ctx->mort.begin(), ctx->mort.begin() + take);
    const std::vector<double> c = mortar_cores(*ctx->ref, part);
    for (int64_t m = 0; m < take; ++m)
      std::copy(c.begin() + m * CS, c.begin() + m * CS + 2 * npk, couplings + m * 2 * npk);
  }
  return WDG_OK;
}

int wdg_get_element_data(const wdg_ctx* ctx, double* geo, double* lift) {
  if (!ctx) return WDG_ERR_ARG;
  if (ctx->host_only || ctx->state < kMesh) return fail(ctx, WDG_ERR_STATE, "no device mesh");
  HIPCHK(hipSetDevice(ctx->device));
  const int NT = ctx->NT();
  const int LS = wdg::lift_stride(ctx->N);
  auto fetch = [&](const void* src, size_t count, double* dst, int stride, int used) -> int {
    std::vector<unsigned char> buf(count * ctx->tsize());
    HIPCHK(hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < ctx->Kw; ++k)
      for (int i = 0; i < used; ++i) {
        const size_t m = size_t(k) * stride + i;
        dst[k * used + i] = ctx->bits == 32 ? double(reinterpret_cast<float*>(buf.data())[m])
                                            : reinterpret_cast<double*>(buf.data())[m];
      }
    return WDG_OK;
  };
  if (geo) {
    int rc = fetch(ctx->dGeo, size_t(ctx->Kw) * wdg::kGeoStride, geo, wdg::kGeoStride, wdg::kGeoStride);
    if (rc) return rc;
  }
  if (lift && !wdg::lift_packed(ctx->N)) {
    // the record holds L^{tri,k} column by column
    std::vector<double> cm(size_t(ctx->Kw) * NT * NT);
    int rc = fetch(ctx->dL, size_t(ctx->Kw) * LS, cm.data(), LS, NT * NT);
    if (rc) return rc;
    for (int64_t k = 0; k < ctx->Kw; ++k)
      for (int r = 0; r < NT; ++r)
        for (int c = 0; c < NT; ++c) lift[(size_t(k) * NT + r) * NT + c] = cm[(size_t(k) * NT + c) * NT + r];
  } else if (lift) {
    // L^{tri,k} = (M^{tri,k})^-1 M^tri from the stored lower triangle of the inverse
    const int NPK = NT * (NT + 1) / 2;
    std::vector<double> pk(size_t(ctx->Kw) * NPK);
    int rc = fetch(ctx->dL, size_t(ctx->Kw) * LS, pk.data(), LS, NPK);
    if (rc) return rc;
    const RefOps& R = *ctx->ref;
    std::vector<double> Mi(size_t(NT) * NT);
    for (int64_t k = 0; k < ctx->Kw; ++k) {
      for (int r = 0; r < NT; ++r)
        for (int c = 0; c <= r; ++c) Mi[r * NT + c] = Mi[c * NT + r] = pk[size_t(k) * NPK + r * (r + 1) / 2 + c];
      for (int r = 0; r < NT; ++r)
        for (int c = 0; c < NT; ++c) {
          double v = 0.0;
          for (int m = 0; m < NT; ++m) v += Mi[r * NT + m] * R.Mtri[m * NT + c];
          lift[(size_t(k) * NT + r) * NT + c] = v;
        }
    }
  }
  return WDG_OK;
}

int wdg_reference_operator(int order_N, const char* name, double* out, int64_t cap, int64_t* count) {
  if (!name || !count || order_N < 1 || order_N > 5 || cap < 0) return WDG_ERR_ARG;
  std::vector<double> v;
  const std::string n(name);
  if (n.rfind("tet_", 0) == 0) {
    const wdg::TetOps Tt(order_N);
    const std::string m = n.substr(4);
    if (m == "r") v = Tt.r;
    else if (m == "s") v = Tt.s;
    else if (m == "t") v = Tt.t;
    else if (m == "Dr") v = Tt.Dr;
    else if (m == "Ds") v = Tt.Ds;
    else if (m == "Dt") v = Tt.Dt;
    else if (m == "M") v = Tt.M;
    else if (m == "LIFT") v = Tt.LIFT;
    else if (m.size() == 5 && m.substr(0, 4) == "face" && m[4] >= '0' && m[4] <= '3') {
      for (int id : Tt.face_nodes[m[4] - '0']) v.push_back(id);
    } else {
      return WDG_ERR_ARG;
    }
    *count = int64_t(v.size());
    if (out) std::copy(v.begin(), v.begin() + std::min<int64_t>(cap, int64_t(v.size())), out);
    return WDG_OK;
  }
  RefOps R(order_N);
  if (n == "r") v = R.r;
  else if (n == "s") v = R.s;
  else if (n == "t") v = R.t;
  else if (n == "Dr") v = R.Dr;
  else if (n == "Ds") v = R.Ds;
  else if (n == "Dt") v = R.Dt;
  else if (n == "M1") v = R.M1;
  else if (n == "Mtri") v = R.Mtri;
  else if (n == "g0") v = R.g0;
  else if (n == "gN") v = R.gN;
  else if (n.size() == 3 && (n.substr(0, 2) == "Mv" || n.substr(0, 2) == "Ea" || n.substr(0, 2) == "Eb") &&
           n[2] >= '0' && n[2] <= '2') {
    const int e = n[2] - '0';
    v = n[0] == 'M' ? R.Mv[e] : (n[1] == 'a' ? R.Ea[e] : R.Eb[e]);
  } else if (n.size() == 5 && n.substr(0, 4) == "edge" && n[4] >= '0' && n[4] <= '2') {
    for (int id : R.edge_nodes[n[4] - '0']) v.push_back(id);
  } else {
    return WDG_ERR_ARG;
  }
  *count = int64_t(v.size());
  if (out) std::copy(v.begin(), v.begin() + std::min<int64_t>(cap, int64_t(v.size())), out);
  return WDG_OK;
}


// ---------------------------------------------------------------------------
// Batches of independent problems
// ---------------------------------------------------------------------------

}  // extern "C"

struct wdg_batch {
  int device = 0, bits = 32;
  hipStream_t stream = nullptr;
  std::vector<wdg_ctx*> probs;
  std::vector<double> dts;
  struct Trial {
    bool node;  // node-lane kernel, else level-lane
    int epb, wpe;
    float us;  // median stage time of the order's launch, microseconds
  };
  struct Group {
    int N = 0;
    std::vector<int> members;  // problem indices
    bool node = false;         // node-lane kernel (orders 4, 5 in FP32), else level-lane
    int epb = 0, wpe = 2, nwork = 0;
    int2* dWork = nullptr;
    float tuned_us = 0.0f;
    std::vector<Trial> trials;  // the autotuner's candidates, in the order tried
  };
  std::vector<Group> groups;
  wdg::StageLaunch* dProbs = nullptr;
  wdg::BatchParam* dParam = nullptr;
  int64_t* dCounter = nullptr;
  double* dAmp = nullptr;  // source amplitudes [step][stage][problem][source]
  int64_t amp_steps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // one side stream per further order: the orders of a stage run concurrently
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  bool ready = false;
  bool concurrent = true;  // the orders of a stage on side streams, else one after another
  mutable std::string err;
};

namespace {

int bfail(const wdg_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define BHIPCHK(expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      return bfail(b, e_ == hipErrorOutOfMemory ? WDG_ERR_OOM : WDG_ERR_HIP,                     \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                           \
    }                                                                                            \
  } while (0)

void batch_release(wdg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
  for (hipStream_t q : b->side) (void)hipStreamDestroy(q);
  b->events.clear();
  b->side.clear();
  for (auto& g : b->groups) dfree(g.dWork);
  dfree(b->dProbs);
  dfree(b->dParam);
  dfree(b->dCounter);
  dfree(b->dAmp);
  b->amp_steps = 0;
  b->ready = false;
}

// work list of group g at epb elements per chunk: (problem, chunk), problem-major
std::vector<int2> batch_work(const wdg_batch* b, const wdg_batch::Group& g, int epb) {
  std::vector<int2> w;
  for (int p : g.members) {
    const int nch = int((b->probs[p]->Kw + epb - 1) / epb);
    for (int c = 0; c < nch; ++c) w.push_back(make_int2(p, c));
  }
  return w;
}

// the stage records of every problem (static fields) and the per-problem parameters
int batch_upload_records(wdg_batch* b) {
  const size_t np = b->probs.size();
  std::vector<wdg::StageLaunch> L(np);
  std::vector<wdg::BatchParam> P(np);
  for (size_t i = 0; i < np; ++i) {
    wdg_ctx* ctx = b->probs[i];
    wdg::StageLaunch& A = L[i];
    A = wdg::StageLaunch{};
    A.Uin = ctx->dU[ctx->cur];
    A.Uout = nullptr;
    A.res = ctx->dRes;
    A.geo = ctx->dGeo;
    A.L = ctx->dL;
    A.conn = ctx->dConn;
    A.opsW = ctx->dOpsW;
    A.srcvec = ctx->dSrcVec;
    A.nsrc = int(ctx->src.size());
    for (int s = 0; s < A.nsrc; ++s) A.src_elem[s] = int(ctx->src[s].elem);
    A.dt = b->dts[i];
    A.g = 1.0;
    A.Kw = ctx->Kw;
    const int flags = (ctx->bc == WDG_BC_DIRICHLET_P0 ? wdg::kDirichlet : 0) |
                      (ctx->flux == WDG_FLUX_CENTRAL ? wdg::kCentral : 0) |
                      (ctx->mass == WDG_MASS_LUMPED ? wdg::kLumped : 0);
    A.flags = flags;  // a stage-1 launch without U write: the state of the autotuning runs
    wdg::BatchParam& Q = P[i];
    Q = wdg::BatchParam{};
    Q.U[0] = ctx->dU[0];
    Q.U[1] = ctx->dU[1];
    Q.cur0 = ctx->cur;
    Q.dt = b->dts[i];
    Q.t0 = ctx->time;
    Q.flags = flags;
    Q.nsrc = A.nsrc;
  }
  BHIPCHK(hipMemcpyAsync(b->dProbs, L.data(), np * sizeof(wdg::StageLaunch), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(hipMemcpyAsync(b->dParam, P.data(), np * sizeof(wdg::BatchParam), hipMemcpyHostToDevice, b->stream));
  const int64_t zero = 0;
  BHIPCHK(hipMemcpyAsync(b->dCounter, &zero, sizeof(zero), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  return WDG_OK;
}

// one stage of group g's problems on stream st with the given kernel shape
hipError_t launch_group(const wdg_batch* b, const wdg_batch::Group& g, bool node, int epb, int wpe, const int2* work,
                        int nwork, hipStream_t st) {
  if (node) return wdg::launch_wedge_node_batch(g.N, b->bits, epb, b->dProbs, work, nwork, st);
  return wdg::launch_wedge_batch(g.N, b->bits, b->dProbs, work, nwork, wpe, st);
}

}  // namespace

extern "C" {

int wdg_batch_create(int device, int precision_bits, wdg_batch** out) {
  if (!out) return WDG_ERR_ARG;
  *out = nullptr;
  if (precision_bits != 32 && precision_bits != 64) return WDG_ERR_ARG;
  wdg_batch* b = new (std::nothrow) wdg_batch;
  if (!b) return WDG_ERR_OOM;
  b->device = device;
  b->bits = precision_bits;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&b->stream) != hipSuccess) {
    delete b;
    return WDG_ERR_HIP;
  }
  *out = b;
  return WDG_OK;
}

int wdg_batch_destroy(wdg_batch* b) {
  if (!b) return WDG_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return WDG_OK;
}

const char* wdg_batch_last_error(const wdg_batch* b) { return b ? b->err.c_str() : "null batch"; }

int wdg_batch_add(wdg_batch* b, wdg_ctx* ctx, double dt, int* index) {
  if (!b || !ctx) return WDG_ERR_ARG;
  if (b->ready) return bfail(b, WDG_ERR_STATE, "add after prepare");
  if (ctx->host_only || ctx->device != b->device || ctx->bits != b->bits)
    return bfail(b, WDG_ERR_ARG, "problem on another device or precision");
  if (ctx->state < kFields) return bfail(b, WDG_ERR_STATE, "problem without fields");
  if (ctx->Kt > 0 || !ctx->mort.empty() || ctx->Kw == 0) return bfail(b, WDG_ERR_UNSUPPORTED, "batch: wedge meshes only");
  if (!(dt > 0) || !std::isfinite(dt)) return bfail(b, WDG_ERR_ARG, "bad time step");
  for (wdg_ctx* q : b->probs)
    if (q == ctx) return bfail(b, WDG_ERR_ARG, "problem added twice");
  b->probs.push_back(ctx);
  b->dts.push_back(dt);
  if (index) *index = int(b->probs.size()) - 1;
  return WDG_OK;
}

int wdg_batch_prepare(wdg_batch* b, int autotune) {
  if (!b) return WDG_ERR_ARG;
  if (b->probs.empty()) return bfail(b, WDG_ERR_STATE, "empty batch");
  BHIPCHK(hipSetDevice(b->device));
  // the autotuner's launches rewrite every problem's residual on the batch
  // stream: work still queued on a problem's own stream must finish first
  for (wdg_ctx* q : b->probs) BHIPCHK(hipStreamSynchronize(q->stream));
  batch_release(b);
  b->groups.clear();
  for (size_t i = 0; i < b->probs.size(); ++i) {
    const int N = b->probs[i]->N;
    auto it = std::find_if(b->groups.begin(), b->groups.end(), [N](const wdg_batch::Group& g) { return g.N == N; });
    if (it == b->groups.end()) {
      b->groups.emplace_back();
      b->groups.back().N = N;
      it = b->groups.end() - 1;
    }
    it->members.push_back(int(i));
  }
  std::sort(b->groups.begin(), b->groups.end(),
            [](const wdg_batch::Group& x, const wdg_batch::Group& y) { return x.N > y.N; });
  const size_t np = b->probs.size();
  BHIPCHK(hipMalloc(&b->dProbs, np * sizeof(wdg::StageLaunch)));
  BHIPCHK(hipMalloc(&b->dParam, np * sizeof(wdg::BatchParam)));
  BHIPCHK(hipMalloc(&b->dCounter, sizeof(int64_t)));
  int rc = batch_upload_records(b);
  if (rc) return rc;

  // autotuner (the paper tunes its elements per block, Sec. 6.3): per order,
  // the kernel shapes that exist for it -- the node-lane kernel (orders 4, 5
  // in FP32) at kNodeEpbVariants element counts per block, the level-lane
  // kernel at its register budgets (occupancy 2 as the single-problem kernel,
  // or 1: no spills at high order) -- each timed on the real data as the
  // median of kTuneReps launches that only rewrite the residual (harmless at
  // a step boundary, where the next stage overwrites it before reading)
  constexpr int kTuneReps = 5;
  std::array<hipEvent_t, kTuneReps + 1> ev{};
  for (auto& e : ev) BHIPCHK(hipEventCreate(&e));
  int2* dTry = nullptr;
  size_t try_cap = 0;
  for (auto& g : b->groups) {
    struct Cand {
      bool node;
      int epb, wpe;
    };
    // the kernel family the problems of this order use alone (so that batch
    // results equal theirs bit for bit): node-lane only if every one does;
    // first the single-problem kernel's shape (the choice without autotuning)
    bool node = true;
    for (int p : g.members) node = node && node_kernel(b->probs[p], 0);
    std::vector<Cand> cand;
    if (node) {
      for (int k = 0; k < wdg::kNodeEpbVariants; ++k) cand.push_back({true, wdg::wedge_node_epb(g.N, b->bits, k), 2});
    } else {
      cand.push_back({false, wdg::wedge_chunk_elems(g.N, b->bits), 2});
      cand.push_back({false, wdg::wedge_chunk_elems(g.N, b->bits), 1});
    }
    g.trials.clear();
    size_t pick = 0;
    if (autotune) {
      float best = 1e30f;
      for (size_t c = 0; c < cand.size(); ++c) {
        const std::vector<int2> w = batch_work(b, g, cand[c].epb);
        if (w.size() > try_cap) {
          BHIPCHK(hipStreamSynchronize(b->stream));
          dfree(dTry);
          try_cap = 0;
          BHIPCHK(hipMalloc(&dTry, w.size() * sizeof(int2)));
          try_cap = w.size();
        }
        BHIPCHK(hipMemcpyAsync(dTry, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
        const int nw = int(w.size());
        BHIPCHK(launch_group(b, g, cand[c].node, cand[c].epb, cand[c].wpe, dTry, nw, b->stream));  // warm-up
        BHIPCHK(hipEventRecord(ev[0], b->stream));
        for (int r = 0; r < kTuneReps; ++r) {
          BHIPCHK(launch_group(b, g, cand[c].node, cand[c].epb, cand[c].wpe, dTry, nw, b->stream));
          BHIPCHK(hipEventRecord(ev[r + 1], b->stream));
        }
        BHIPCHK(hipEventSynchronize(ev[kTuneReps]));
        std::array<float, kTuneReps> t{};
        for (int r = 0; r < kTuneReps; ++r) BHIPCHK(hipEventElapsedTime(&t[r], ev[r], ev[r + 1]));
        std::sort(t.begin(), t.end());
        const float med = t[kTuneReps / 2];
        g.trials.push_back({cand[c].node, cand[c].epb, cand[c].wpe, med * 1e3f});
        if (med < best) {
          best = med;
          pick = c;
        }
      }
      g.tuned_us = best * 1e3f;
    } else {
      g.tuned_us = 0.0f;
    }
    g.node = cand[pick].node;
    g.epb = cand[pick].epb;
    g.wpe = cand[pick].wpe;
    const std::vector<int2> w = batch_work(b, g, g.epb);
    g.nwork = int(w.size());
    BHIPCHK(hipMalloc(&g.dWork, w.size() * sizeof(int2)));
    BHIPCHK(hipMemcpyAsync(g.dWork, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
  }
  BHIPCHK(hipStreamSynchronize(b->stream));
  dfree(dTry);
  for (auto& e : ev) BHIPCHK(hipEventDestroy(e));

  b->ready = true;
  return WDG_OK;
}

}  // extern "C"

namespace {

// one step as a graph: per stage the record kernel, then one launch per order;
// then the step counter.  The amplitude table pointer is part of the graph.
int batch_capture(wdg_batch* b) {
  if (b->exec) BHIPCHK(hipGraphExecDestroy(b->exec));
  if (b->graph) BHIPCHK(hipGraphDestroy(b->graph));
  b->exec = nullptr;
  b->graph = nullptr;
  const int np = int(b->probs.size());
  const int ng = int(b->groups.size());
  // side streams (default priority) and fork/join events, per stage and order
  while (int(b->side.size()) < ng - 1) {
    hipStream_t q = nullptr;
    BHIPCHK(hipStreamCreate(&q));
    b->side.push_back(q);
  }
  while (int(b->events.size()) < 5 * (ng + 1)) {
    hipEvent_t e = nullptr;
    BHIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->events.push_back(e);
  }
  BHIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t cap = hipSuccess;
  auto ok = [&cap](hipError_t e) {
    if (cap == hipSuccess) cap = e;
  };
  for (int s = 0; s < 5 && cap == hipSuccess; ++s) {
    ok(wdg::launch_batch_prepare(np, b->dProbs, b->dParam, b->dCounter, s, kRkA[s], kRkB[s], b->dAmp, b->stream));
    if (!b->concurrent) {
      for (const auto& g : b->groups) ok(launch_group(b, g, g.node, g.epb, g.wpe, g.dWork, g.nwork, b->stream));
      continue;
    }
    hipEvent_t fork = b->events[s * (ng + 1)];
    ok(hipEventRecord(fork, b->stream));
    // the orders are independent within a stage: all but the first on side streams
    for (int gi = 1; gi < ng; ++gi) {
      const auto& g = b->groups[gi];
      ok(hipStreamWaitEvent(b->side[gi - 1], fork, 0));
      ok(launch_group(b, g, g.node, g.epb, g.wpe, g.dWork, g.nwork, b->side[gi - 1]));
      ok(hipEventRecord(b->events[s * (ng + 1) + gi], b->side[gi - 1]));
    }
    const auto& g0 = b->groups[0];
    ok(launch_group(b, g0, g0.node, g0.epb, g0.wpe, g0.dWork, g0.nwork, b->stream));
    for (int gi = 1; gi < ng; ++gi) ok(hipStreamWaitEvent(b->stream, b->events[s * (ng + 1) + gi], 0));
  }
  if (cap == hipSuccess) cap = wdg::launch_batch_advance(b->dCounter, b->stream);
  hipGraph_t graph = nullptr;
  const hipError_t end = hipStreamEndCapture(b->stream, &graph);
  BHIPCHK(cap);
  BHIPCHK(end);
  b->graph = graph;
  BHIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return WDG_OK;
}

}  // namespace

extern "C" {

int wdg_batch_set_concurrent(wdg_batch* b, int enable) {
  if (!b) return WDG_ERR_ARG;
  BHIPCHK(hipSetDevice(b->device));
  if (b->concurrent == (enable != 0)) return WDG_OK;
  BHIPCHK(hipStreamSynchronize(b->stream));
  b->concurrent = enable != 0;
  // the next step captures the graph again
  if (b->exec) BHIPCHK(hipGraphExecDestroy(b->exec));
  if (b->graph) BHIPCHK(hipGraphDestroy(b->graph));
  b->exec = nullptr;
  b->graph = nullptr;
  return WDG_OK;
}

int wdg_batch_step(wdg_batch* b, int64_t nsteps) {
  if (!b) return WDG_ERR_ARG;
  if (!b->ready) return bfail(b, WDG_ERR_STATE, "step before prepare");
  if (nsteps < 0) return bfail(b, WDG_ERR_ARG, "negative step count");
  BHIPCHK(hipSetDevice(b->device));
  for (wdg_ctx* ctx : b->probs) {
    BHIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->recording = false;
  }
  // the problems' current buffers and times (the graph reads them from device memory)
  int rc = batch_upload_records(b);
  if (rc) return rc;
  if (nsteps == 0) return WDG_OK;
  // source amplitudes of every stage, evaluated as wdg_step does
  const int np = int(b->probs.size());
  if (nsteps > b->amp_steps || !b->exec) {
    BHIPCHK(hipStreamSynchronize(b->stream));
    dfree(b->dAmp);
    b->amp_steps = 0;
    BHIPCHK(hipMalloc(&b->dAmp, size_t(nsteps) * 5 * np * wdg::kMaxSources * sizeof(double)));
    b->amp_steps = nsteps;
    rc = batch_capture(b);
    if (rc) return rc;
  }
  std::vector<double> amp(size_t(nsteps) * 5 * np * wdg::kMaxSources, 0.0);
  for (int p = 0; p < np; ++p) {
    const wdg_ctx* ctx = b->probs[p];
    const double t0 = ctx->time, dt = b->dts[p];
    for (int64_t n = 0; n < nsteps; ++n) {
      const double tn = t0 + double(n) * dt;
      for (int s = 0; s < 5; ++s)
        for (size_t k = 0; k < ctx->src.size(); ++k)
          amp[((size_t(n) * 5 + s) * np + p) * wdg::kMaxSources + k] = ctx->src[k].value(tn + kRkC[s] * dt);
    }
  }
  BHIPCHK(hipMemcpyAsync(b->dAmp, amp.data(), amp.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
  for (int64_t n = 0; n < nsteps; ++n) BHIPCHK(hipGraphLaunch(b->exec, b->stream));
  BHIPCHK(hipStreamSynchronize(b->stream));
  for (size_t i = 0; i < b->probs.size(); ++i) {
    wdg_ctx* ctx = b->probs[i];
    ctx->cur = int((ctx->cur + 5 * nsteps) & 1);
    ctx->time = ctx->time + double(nsteps) * b->dts[i];
  }
  return WDG_OK;
}

int wdg_batch_config(const wdg_batch* b, int N, int* elems_per_block, int* waves_per_simd, double* tuned_us) {
  if (!b) return WDG_ERR_ARG;
  for (const auto& g : b->groups)
    if (g.N == N) {
      if (elems_per_block) *elems_per_block = g.epb;
      if (waves_per_simd) *waves_per_simd = g.wpe;
      if (tuned_us) *tuned_us = g.tuned_us;
      return WDG_OK;
    }
  return bfail(b, WDG_ERR_ARG, "no problem of that order in the batch");
}

int wdg_batch_trials(const wdg_batch* b, int N, int64_t cap, int* kernel, int* elems_per_block, int* waves_per_simd,
                     double* stage_us, int64_t* count) {
  if (!b || !count || cap < 0) return WDG_ERR_ARG;
  for (const auto& g : b->groups)
    if (g.N == N) {
      *count = int64_t(g.trials.size());
      for (int64_t k = 0; k < cap && k < *count; ++k) {
        if (kernel) kernel[k] = g.trials[k].node ? WDG_WEDGE_NODE : WDG_WEDGE_LEVEL;
        if (elems_per_block) elems_per_block[k] = g.trials[k].epb;
        if (waves_per_simd) waves_per_simd[k] = g.trials[k].wpe;
        if (stage_us) stage_us[k] = g.trials[k].us;
      }
      return WDG_OK;
    }
  return bfail(b, WDG_ERR_ARG, "no problem of that order in the batch");
}

}  // extern "C"
