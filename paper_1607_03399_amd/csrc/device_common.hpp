// Device-side helpers shared by the HIP kernels of libwdg (gfx950): node
// numbering of the reference triangle and tetrahedron, the node-interleaved
// 4-vector, face-node maps across shared triangles, raw buffer access, and
// the order/precision dispatch of the host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace wdg {
namespace {

template <int N>
struct Dim {
  static constexpr int NT = (N + 1) * (N + 2) / 2;
  static constexpr int Nq = N + 1;
  static constexpr int NP = NT * Nq;
  // Per-element triangular operator: for N <= 3 (M^{tri,k})^-1, stored as its
  // lower triangle row by row (symmetric; the stage kernel does not read it:
  // it factors M^{tri,k} itself into the same LDS slots and solves after the
  // literal M^tri); for N >= 4 the lift L^{tri,k} = (M^{tri,k})^-1 M^tri
  // itself, column by column (the node-lane kernel reads a row per lane,
  // coalesced across the element's lanes).  Padded to whole 4-vectors.
  static constexpr bool PACKED = N <= 3;
  static constexpr int NPK = NT * (NT + 1) / 2;
  static constexpr int LS = ((PACKED ? NPK : NT * NT) + 3) / 4 * 4;
};

// row of entry f of a lower triangle stored row by row (entry (r, c) at r (r + 1) / 2 + c)
__host__ __device__ constexpr int tri_row(int f) {
  int r = 0;
  while ((r + 1) * (r + 2) / 2 <= f) ++r;
  return r;
}

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

}  // namespace
}  // namespace wdg

// order and precision dispatch of the host launchers
#define WDG_DISPATCH_N(N_, BITS_, CALL)                    \
  switch (N_) {                                            \
    case 1: if (BITS_ == 32) { CALL(1, float); } else { CALL(1, double); } break; \
    case 2: if (BITS_ == 32) { CALL(2, float); } else { CALL(2, double); } break; \
    case 3: if (BITS_ == 32) { CALL(3, float); } else { CALL(3, double); } break; \
    case 4: if (BITS_ == 32) { CALL(4, float); } else { CALL(4, double); } break; \
    case 5: if (BITS_ == 32) { CALL(5, float); } else { CALL(5, double); } break; \
    default: break;                                        \
  }
