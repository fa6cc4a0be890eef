// Internal interface between the host runtime and the HIP kernels of libwdg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wdg {

// Per-element record of geometric factors and material (values of type T):
//   0 r_x, 1 r_y, 2 s_x, 3 s_y, 4 t_zJ, 5/6 t_xJ at t=-1/+1, 7/8 t_yJ at t=-1/+1,
//   9 kappa, 10 1/rho, 11 rho c, 12..15 bottom (J_f, n), 16..19 top (J_f, n),
//   20+4e.. quad face e: J_f at first/second edge vertex, n_x, n_y,
//   32..36 rho c + (rho c of the neighbour, or own on the boundary) per face
//   (bottom, top, quad 0..2), 37..39 unused.
constexpr int kGeoStride = 40;
// Per-element FP64 auxiliary record: 0..2 J_tri h_v / 2 (M^{tri,k} weights), 3 J_tri, 4 kappa, 5 rho.
constexpr int kAuxStride = 8;
// Per-element connectivity (int32): 0..4 neighbour of bottom, top, quad 0..2 (-1: boundary);
// 5 packed codes: bits 0-2 / 3-5 vertex permutation of the bottom / top neighbour face,
// bit 6 / 7 set when that neighbour face is the neighbour's top triangle, bits 8+2e..9+2e
// neighbour edge of quad face e.
constexpr int kConnStride = 8;
constexpr int kMaxSources = 8;

enum StageFlags : int {
  kReadRes = 1,    // res = a res + dt rhs (else res = dt rhs)
  kWriteU = 2,     // U_out = U_in + b res
  kDirichlet = 4,  // else rigid wall
  kCentral = 8,    // else upwind flux
};

struct StageLaunch {
  const void* Uin;
  void* Uout;
  void* res;
  const void* geo;
  const void* L;
  const int* conn;
  const void* ops;
  const void* srcvec;
  int src_elem[kMaxSources];
  double src_amp[kMaxSources];
  int nsrc;
  double a, b, dt;
  int64_t K;
  int flags;
};

// Per-element stride (values) of the stored triangular lift: Np_tri^2 padded to a multiple of 4.
int lift_stride(int N);
// Size in bytes of the device face-permutation table of order N (the only
// operator data the stage kernel reads from memory; the reference triangle
// and 1D operators are compiled into the kernel).
size_t ops_bytes(int N);
// Fill that table (host memory of ops_bytes(N)) from the 6 x Np_tri permutation list.
void fill_ops(int N, void* dst, const int* perm);

hipError_t launch_setup(int N, int bits, int64_t K, const double* dX, const double* dMv, const double* dMtri,
                        void* dGeo, void* dL, double* dAux, hipStream_t st);
hipError_t launch_material(int bits, int64_t K, const double* dc, const double* drho, const int* dConn, void* dGeo,
                           double* dAux, hipStream_t st);
hipError_t launch_stage(int N, int bits, const StageLaunch& a, hipStream_t st);
hipError_t launch_receivers(int bits, int NP, int nrec, const void* U, const int* elem, const double* rows,
                            double* out, hipStream_t st);
// Per-block partial energies; returns the number of partials written.
hipError_t launch_energy(int N, int bits, int64_t K, const void* U, const double* aux, const double* Mv,
                         const double* M1, double* partial, int* nblocks, hipStream_t st);

}  // namespace wdg
