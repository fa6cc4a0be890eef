// Reference-element operators of the wedge DG method, built on the host in FP64.
//
// Reference domains are bi-unit: triangle {r,s >= -1, r+s <= 0} with vertices
// V1=(-1,-1), V2=(1,-1), V3=(-1,1); vertical interval t in [-1,1].
// Wedge nodes are triangle Warp & Blend nodes (alpha = 0) times the N+1
// Gauss-Legendre-Lobatto points (Sec. 3.1); wedge node n = j*NT + i.
//
// Triangle node ordering: lattice (a,b), a+b <= N, index b*(N+1) - b(b-1)/2 + a,
// integer barycentrics (N-a-b, a, b) relative to (V1, V2, V3).
#pragma once

#include <array>
#include <vector>

namespace wdg {

struct RefOps {
  int N = 0, NT = 0, Nq = 0, NP = 0;
  // 1D (GLL)
  std::vector<double> t;      // Nq nodes
  std::vector<double> wgll;   // Nq GLL weights
  std::vector<double> Dt;     // Nq x Nq, Dt[j*Nq+m] = l_m'(t_j)
  std::vector<double> M1;     // Nq x Nq exact 1D mass
  std::vector<double> g0, gN; // (M1)^-1 e_0, (M1)^-1 e_N
  // triangle
  std::vector<double> r, s;   // NT nodes
  std::vector<double> Dr, Ds; // NT x NT, row = output node
  std::vector<double> Mtri;   // NT x NT exact reference mass
  std::vector<double> Mv[3];  // NT x NT, int l_a l_b lambda_v
  std::vector<double> Ea[3], Eb[3];  // per edge: NT x Nq, (Mtri)^-1 int_edge l_i l_q (1-xi)/2 resp. (1+xi)/2
  std::array<std::vector<int>, 3> edge_nodes;  // per edge, N+1 triangle node ids from its first to its second vertex
  std::vector<int> perm;      // 6 x NT: node index after permuting the face vertices (see face_perm_index)

  explicit RefOps(int N);

  // Lagrange basis of the triangle at (r,s): NT values.
  void tri_basis(double rr, double ss, double* out) const;
  // 1D Lagrange basis at t: Nq values.
  void line_basis(double tt, double* out) const;

 private:
  std::vector<double> Vinv_;  // inverse Dubiner Vandermonde (NT x NT)
};

int tri_index(int N, int a, int b);

// Tetrahedron reference operators for the affine tetrahedra of hybrid meshes
// (standard nodal DG on simplices).  Bi-unit tetrahedron with vertices
// V0=(-1,-1,-1), V1=(1,-1,-1), V2=(-1,1,-1), V3=(-1,-1,1).  Nodes: Warp &
// Blend (alpha = 0); lattice (a,b,c), a+b+c <= N, integer barycentrics
// (N-a-b-c, a, b, c) relative to (V0..V3), index tet_index(N,a,b,c).  The
// nodes of each face coincide with the triangle nodes, so tetrahedra and the
// wedges' triangular faces share face nodes (Sec. 3.1).
// Faces: 0 = (V0,V1,V2), 1 = (V0,V1,V3), 2 = (V1,V2,V3), 3 = (V0,V2,V3); the
// nodes of a face are numbered as the triangle's, with barycentrics relative
// to the face's vertices in that order.
struct TetOps {
  int N = 0, NT = 0, NP = 0;
  std::vector<double> r, s, t;          // NP nodes
  std::vector<double> Dr, Ds, Dt;       // NP x NP, row = output node
  std::vector<double> M;                // NP x NP exact reference mass
  std::vector<double> LIFT;             // NP x 4 NT: M^-1 [E_0 .. E_3], E_f = reference face mass
  std::array<std::vector<int>, 4> face_nodes;  // NT tetrahedron node ids per face

  explicit TetOps(int N);
  // Lagrange basis of the tetrahedron at (r,s,t): NP values.
  void basis(double rr, double ss, double tt, double* out) const;

 private:
  std::vector<double> Vinv_;
};

int tet_index(int N, int a, int b, int c);
extern const int kTetFaceVerts[4][3];

// The six permutations of three face vertices; permutation p maps own face
// vertex k to neighbour face vertex kPerm[p][k].
extern const int kPerm[6][3];

// Gauss-Legendre rule on [-1,1] with n points.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// Solve A X = B in place (A: n x n row-major, B: n x m), Gaussian elimination with partial pivoting.
bool solve_dense(int n, int m, std::vector<double> A, std::vector<double>& B);

}  // namespace wdg
