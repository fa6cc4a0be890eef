// Host construction of the reference operators (FP64).
//
// Orthonormal bases: normalised Legendre polynomials on the interval and the
// Dubiner (collapsed Jacobi) basis on the triangle; Lagrange bases follow by
// inverting their Vandermonde matrices at the nodes.  Quadrature nodes come
// from Newton iteration on Jacobi polynomials.
#include "refops.hpp"

#include <cmath>
#include <stdexcept>

namespace wdg {

const int kPerm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};

int tri_index(int N, int a, int b) { return b * (N + 1) - b * (b - 1) / 2 + a; }

int tet_index(int N, int a, int b, int c) {
  int off = 0;
  for (int cc = 0; cc < c; ++cc) off += (N - cc + 1) * (N - cc + 2) / 2;
  return off + tri_index(N - c, a, b);
}

const int kTetFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

namespace {

// Orthonormal Jacobi polynomial P_n^{(al,be)}(x) w.r.t. (1-x)^al (1+x)^be on [-1,1].
double jacobi(int n, double al, double be, double x) {
  const double g0 = std::pow(2.0, -(al + be + 1.0)) * std::tgamma(al + be + 2.0) /
                    (std::tgamma(al + 1.0) * std::tgamma(be + 1.0));
  double p0 = std::sqrt(g0);
  if (n == 0) return p0;
  double p1 = p0 * ((al + be + 2.0) * x / 2.0 + (al - be) / 2.0) *
              std::sqrt((al + be + 3.0) / ((al + 1.0) * (be + 1.0)));
  if (n == 1) return p1;
  auto a_coef = [&](int k) {  // a_k of x P_{k-1} = a_k P_k + b P_{k-1} + a_{k-1} P_{k-2}
    double h = 2.0 * k + al + be;
    return 2.0 / h * std::sqrt(k * (k + al + be) * (k + al) * (k + be) / ((h - 1.0) * (h + 1.0)));
  };
  double aold = a_coef(1);
  for (int k = 1; k < n; ++k) {
    double h = 2.0 * k + al + be;
    double anew = a_coef(k + 1);
    double bk = -(al * al - be * be) / (h * (h + 2.0));
    double p2 = (x * p1 - bk * p1 - aold * p0) / anew;
    p0 = p1;
    p1 = p2;
    aold = anew;
  }
  return p1;
}

double djacobi(int n, double al, double be, double x) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + al + be + 1.0)) * jacobi(n - 1, al + 1.0, be + 1.0, x);
}

// classical (unnormalised) Legendre P_n and derivative by recurrence
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1.0) * std::pow(x, n - 1);
}

void gll(int N, std::vector<double>& x, std::vector<double>& w) {
  x.assign(N + 1, 0.0);
  w.assign(N + 1, 0.0);
  x[0] = -1.0;
  x[N] = 1.0;
  // interior nodes: roots of P_{N-1}^{(1,1)} (proportional to P_N')
  for (int k = 1; k < N; ++k) {
    double xi = -std::cos(M_PI * k / N);
    for (int it = 0; it < 100; ++it) {
      double f = jacobi(N - 1, 1.0, 1.0, xi);
      double df = djacobi(N - 1, 1.0, 1.0, xi);
      double dx = f / df;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[k] = xi;
  }
  for (int k = 0; k <= N; ++k) {
    double p, dp;
    legendre(N, x[k], p, dp);
    w[k] = 2.0 / (N * (N + 1.0) * p * p);
  }
}

// Dubiner orthonormal basis on the bi-unit triangle and its gradient.
void dubiner(int N, double r, double s, double* psi, double* pr, double* ps) {
  double a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  double b = s;
  int m = 0;
  for (int i = 0; i <= N; ++i) {
    for (int j = 0; j <= N - i; ++j, ++m) {
      double fa = jacobi(i, 0, 0, a), dfa = djacobi(i, 0, 0, a);
      double gb = jacobi(j, 2.0 * i + 1.0, 0, b), dgb = djacobi(j, 2.0 * i + 1.0, 0, b);
      double omb_i = std::pow(1.0 - b, i);
      psi[m] = std::sqrt(2.0) * fa * gb * omb_i;
      if (pr) {
        double omb_im1 = (i >= 1) ? std::pow(1.0 - b, i - 1) : 0.0;
        pr[m] = std::sqrt(2.0) * dfa * gb * 2.0 * omb_im1;
        // d/ds: through a (da/ds = (1+a)/(1-b)) and through b directly
        double t1 = dfa * gb * (1.0 + a) * omb_im1;
        double t2 = fa * (dgb * omb_i - i * gb * omb_im1);
        ps[m] = std::sqrt(2.0) * (t1 + t2);
      }
    }
  }
}

// Orthonormal Proriol-Koornwinder-Dubiner basis on the bi-unit tetrahedron
// and its gradient.  Collapsed coordinates a = 2(1+r)/(-s-t) - 1,
// b = 2(1+s)/(1-t) - 1, c = t, and
//   psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j).
// The gradient follows from the chain rule with -s-t = (1-b)(1-c)/2 and
// 1-t = 1-c; the powers (1-b)^(i-1), (1-c)^(i+j-1) stay finite where the
// collapse is singular, because the factor in front vanishes when the power
// would be negative.
void pkd3(int N, double r, double s, double t, double* psi, double* pr, double* ps, double* pt) {
  const double mst = -s - t, omt = 1.0 - t;
  const double a = std::fabs(mst) > 1e-14 ? 2.0 * (1.0 + r) / mst - 1.0 : -1.0;
  const double b = std::fabs(omt) > 1e-14 ? 2.0 * (1.0 + s) / omt - 1.0 : -1.0;
  const double c = t;
  const double k0 = 2.0 * std::sqrt(2.0);
  auto pw = [](double x, int e) { return e <= 0 ? (e == 0 ? 1.0 : 0.0) : std::pow(x, e); };
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m) {
        const double F = jacobi(i, 0, 0, a), dF = djacobi(i, 0, 0, a);
        const double G = jacobi(j, 2.0 * i + 1.0, 0, b), dG = djacobi(j, 2.0 * i + 1.0, 0, b);
        const double H = jacobi(k, 2.0 * (i + j) + 2.0, 0, c), dH = djacobi(k, 2.0 * (i + j) + 2.0, 0, c);
        const double bi = pw(1.0 - b, i), bi1 = pw(1.0 - b, i - 1);
        const double cij = pw(1.0 - c, i + j), cij1 = pw(1.0 - c, i + j - 1);
        psi[m] = k0 * F * G * bi * H * cij;
        if (!pr) continue;
        // d/da, d/db, d/dc of psi with one power of (1-b) resp. (1-c) taken out
        const double da_red = (i > 0) ? k0 * dF * G * bi1 * H * cij1 : 0.0;     // psi_a / ((1-b)(1-c))
        const double gb = dG * bi - (i > 0 ? i * G * bi1 : 0.0);                 // d/db [G (1-b)^i]
        const double db_red = (i + j > 0) ? k0 * F * gb * H * cij1 : 0.0;       // psi_b / (1-c)
        const double hc = dH * cij - (i + j > 0 ? (i + j) * H * cij1 : 0.0);    // d/dc [H (1-c)^(i+j)]
        const double dc = k0 * F * G * bi * hc;                                  // psi_c
        pr[m] = 4.0 * da_red;
        ps[m] = 2.0 * (1.0 + a) * da_red + 2.0 * db_red;
        pt[m] = 2.0 * (1.0 + a) * da_red + (1.0 + b) * db_red + dc;
      }
}

void invert(int n, const std::vector<double>& A, std::vector<double>& Ainv) {
  Ainv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1.0;
  if (!solve_dense(n, n, A, Ainv)) throw std::runtime_error("singular reference matrix");
}

// out = A (n x k) * B (k x m)
std::vector<double> matmul(int n, int k, int m, const std::vector<double>& A, const std::vector<double>& B) {
  std::vector<double> C(n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l)
      for (int j = 0; j < m; ++j) C[i * m + j] += A[i * k + l] * B[l * m + j];
  return C;
}

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double xi = -std::cos(M_PI * (k + 0.75) / (n + 0.5));
    double p = 0, dp = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, p, dp);
      double dx = p / dp;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(n, xi, p, dp);
    x[k] = xi;
    w[k] = 2.0 / ((1.0 - xi * xi) * dp * dp);
  }
}

bool solve_dense(int n, int m, std::vector<double> A, std::vector<double>& B) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      for (int j = 0; j < m; ++j) std::swap(B[k * m + j], B[piv * m + j]);
    }
    double d = 1.0 / A[k * n + k];
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      double f = A[i * n + k] * d;
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      for (int j = 0; j < m; ++j) B[i * m + j] -= f * B[k * m + j];
    }
  }
  for (int k = 0; k < n; ++k) {
    double d = 1.0 / A[k * n + k];
    for (int j = 0; j < m; ++j) B[k * m + j] *= d;
  }
  return true;
}

RefOps::RefOps(int N_) : N(N_) {
  if (N < 1 || N > 5) throw std::invalid_argument("order out of range");
  NT = (N + 1) * (N + 2) / 2;
  Nq = N + 1;
  NP = NT * Nq;

  // ---- 1D ----
  gll(N, t, wgll);
  std::vector<double> V1(Nq * Nq), V1t(Nq * Nq);
  for (int j = 0; j < Nq; ++j)
    for (int m = 0; m < Nq; ++m) {
      V1[j * Nq + m] = jacobi(m, 0, 0, t[j]);
      V1t[j * Nq + m] = djacobi(m, 0, 0, t[j]);
    }
  std::vector<double> V1inv;
  invert(Nq, V1, V1inv);
  Dt = matmul(Nq, Nq, Nq, V1t, V1inv);
  {
    std::vector<double> VVt(Nq * Nq, 0.0);
    for (int i = 0; i < Nq; ++i)
      for (int j = 0; j < Nq; ++j)
        for (int m = 0; m < Nq; ++m) VVt[i * Nq + j] += V1[i * Nq + m] * V1[j * Nq + m];
    invert(Nq, VVt, M1);
    std::vector<double> Minv1;
    invert(Nq, M1, Minv1);  // = V V^T
    g0.resize(Nq);
    gN.resize(Nq);
    for (int j = 0; j < Nq; ++j) {
      g0[j] = Minv1[j * Nq + 0];
      gN[j] = Minv1[j * Nq + N];
    }
  }

  // ---- triangle nodes: Warp & Blend, alpha = 0 ----
  const double s3 = std::sqrt(3.0);
  const double E[3][2] = {{-1.0, -1.0 / s3}, {1.0, -1.0 / s3}, {0.0, 2.0 / s3}};
  std::vector<double> xeq(Nq);
  for (int k = 0; k <= N; ++k) xeq[k] = -1.0 + 2.0 * k / N;
  auto warp = [&](double x) {
    if (std::fabs(x) >= 1.0 - 1e-10) return 0.0;
    double acc = 0.0;
    for (int i = 0; i <= N; ++i) {
      double li = 1.0;
      for (int m = 0; m <= N; ++m)
        if (m != i) li *= (x - xeq[m]) / (xeq[i] - xeq[m]);
      acc += li * (t[i] - xeq[i]);
    }
    return acc / (1.0 - x * x);
  };
  r.assign(NT, 0.0);
  s.assign(NT, 0.0);
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) {
      double lam[3] = {double(N - a - b) / N, double(a) / N, double(b) / N};
      double X = 0, Y = 0;
      for (int v = 0; v < 3; ++v) {
        X += lam[v] * E[v][0];
        Y += lam[v] * E[v][1];
      }
      const int ed[3][2] = {{0, 1}, {1, 2}, {2, 0}};
      double dX = 0, dY = 0;
      for (auto& e : ed) {
        double ux = E[e[1]][0] - E[e[0]][0], uy = E[e[1]][1] - E[e[0]][1];
        double len = std::sqrt(ux * ux + uy * uy);
        double amt = 4.0 * lam[e[0]] * lam[e[1]] * warp(lam[e[1]] - lam[e[0]]);
        dX += amt * ux / len;
        dY += amt * uy / len;
      }
      X += dX;
      Y += dY;
      double l3 = (s3 * Y + 1.0) / 3.0;
      int idx = tri_index(N, a, b);
      r[idx] = X - l3;
      s[idx] = 2.0 * l3 - 1.0;
    }

  // ---- triangle operators ----
  std::vector<double> V(NT * NT), Vr(NT * NT), Vs(NT * NT);
  for (int i = 0; i < NT; ++i) dubiner(N, r[i], s[i], &V[i * NT], &Vr[i * NT], &Vs[i * NT]);
  invert(NT, V, Vinv_);
  Dr = matmul(NT, NT, NT, Vr, Vinv_);
  Ds = matmul(NT, NT, NT, Vs, Vinv_);
  {
    std::vector<double> VVt(NT * NT, 0.0);
    for (int i = 0; i < NT; ++i)
      for (int j = 0; j < NT; ++j)
        for (int m = 0; m < NT; ++m) VVt[i * NT + j] += V[i * NT + m] * V[j * NT + m];
    invert(NT, VVt, Mtri);
  }
  // J-weight masses by collapsed Gauss quadrature (exact to degree 2N+2)
  {
    std::vector<double> xg, wg;
    gauss_legendre(N + 2, xg, wg);
    for (int v = 0; v < 3; ++v) Mv[v].assign(NT * NT, 0.0);
    std::vector<double> ell(NT);
    for (size_t ia = 0; ia < xg.size(); ++ia)
      for (size_t ib = 0; ib < xg.size(); ++ib) {
        double aa = xg[ia], bb = xg[ib];
        double rr = (1.0 + aa) * (1.0 - bb) / 2.0 - 1.0, ss = bb;
        double w = wg[ia] * wg[ib] * (1.0 - bb) / 2.0;
        tri_basis(rr, ss, ell.data());
        double lam[3] = {-(rr + ss) / 2.0, (1.0 + rr) / 2.0, (1.0 + ss) / 2.0};
        for (int v = 0; v < 3; ++v)
          for (int i = 0; i < NT; ++i)
            for (int j = 0; j < NT; ++j) Mv[v][i * NT + j] += w * lam[v] * ell[i] * ell[j];
      }
  }
  // edges: node lists and lift pieces
  for (int q = 0; q <= N; ++q) {
    edge_nodes[0].push_back(tri_index(N, q, 0));
    edge_nodes[1].push_back(tri_index(N, N - q, q));
    edge_nodes[2].push_back(tri_index(N, 0, N - q));
  }
  {
    std::vector<double> xg, wg;
    gauss_legendre(N + 2, xg, wg);
    std::vector<double> ell(NT), l1(Nq);
    for (int e = 0; e < 3; ++e) {
      std::vector<double> Ta(NT * Nq, 0.0), Tb(NT * Nq, 0.0);
      for (size_t k = 0; k < xg.size(); ++k) {
        double xi = xg[k];
        double rr = e == 0 ? xi : (e == 1 ? -xi : -1.0);
        double ss = e == 0 ? -1.0 : (e == 1 ? xi : -xi);
        tri_basis(rr, ss, ell.data());
        line_basis(xi, l1.data());
        for (int i = 0; i < NT; ++i)
          for (int q = 0; q < Nq; ++q) {
            Ta[i * Nq + q] += wg[k] * ell[i] * l1[q] * (1.0 - xi) / 2.0;
            Tb[i * Nq + q] += wg[k] * ell[i] * l1[q] * (1.0 + xi) / 2.0;
          }
      }
      Ea[e] = Ta;
      Eb[e] = Tb;
      if (!solve_dense(NT, Nq, Mtri, Ea[e]) || !solve_dense(NT, Nq, Mtri, Eb[e]))
        throw std::runtime_error("edge lift");
    }
  }
  // face permutations of triangle nodes
  perm.assign(6 * NT, 0);
  for (int p = 0; p < 6; ++p)
    for (int b = 0; b <= N; ++b)
      for (int a = 0; a + b <= N; ++a) {
        int I[3] = {N - a - b, a, b}, J[3];
        for (int k = 0; k < 3; ++k) J[kPerm[p][k]] = I[k];
        perm[p * NT + tri_index(N, a, b)] = tri_index(N, J[1], J[2]);
      }
}

void RefOps::tri_basis(double rr, double ss, double* out) const {
  std::vector<double> psi(NT);
  dubiner(N, rr, ss, psi.data(), nullptr, nullptr);
  for (int j = 0; j < NT; ++j) {
    double acc = 0.0;
    for (int m = 0; m < NT; ++m) acc += Vinv_[m * NT + j] * psi[m];
    out[j] = acc;
  }
}

void RefOps::line_basis(double tt, double* out) const {
  for (int j = 0; j < Nq; ++j) {
    double l = 1.0;
    for (int m = 0; m < Nq; ++m)
      if (m != j) l *= (tt - t[m]) / (t[j] - t[m]);
    out[j] = l;
  }
}

// ---------------------------------------------------------------------------
// tetrahedron
// ---------------------------------------------------------------------------
TetOps::TetOps(int N_) : N(N_) {
  if (N < 1 || N > 5) throw std::invalid_argument("order out of range");
  NT = (N + 1) * (N + 2) / 2;
  NP = (N + 1) * (N + 2) * (N + 3) / 6;

  // Warp & Blend nodes (alpha = 0) built on the equilateral tetrahedron:
  // every face adds its triangle warp (edge warps of the face, as for the
  // triangle nodes) times the face blend b c d / ((b + a/2)(c + a/2)(d + a/2))
  // (a: barycentric of the opposite vertex, b c d those of the face); a node
  // on an edge gets exactly that edge's warp.
  const double s3 = std::sqrt(3.0), s6 = std::sqrt(6.0);
  const double E[4][3] = {{-1.0, -1.0 / s3, -1.0 / s6}, {1.0, -1.0 / s3, -1.0 / s6}, {0.0, 2.0 / s3, -1.0 / s6},
                          {0.0, 0.0, 3.0 / s6}};
  const int faces[4][4] = {{3, 0, 1, 2}, {2, 0, 1, 3}, {0, 1, 2, 3}, {1, 0, 2, 3}};  // opposite, face vertices
  std::vector<double> xgll, wgll_;
  gll(N, xgll, wgll_);
  std::vector<double> xeq(N + 1);
  for (int k = 0; k <= N; ++k) xeq[k] = -1.0 + 2.0 * k / N;
  auto warp = [&](double x) {
    if (std::fabs(x) >= 1.0 - 1e-10) return 0.0;
    double acc = 0.0;
    for (int i = 0; i <= N; ++i) {
      double li = 1.0;
      for (int m = 0; m <= N; ++m)
        if (m != i) li *= (x - xeq[m]) / (xeq[i] - xeq[m]);
      acc += li * (xgll[i] - xeq[i]);
    }
    return acc / (1.0 - x * x);
  };
  r.assign(NP, 0.0);
  s.assign(NP, 0.0);
  t.assign(NP, 0.0);
  const double tol = 1e-10;
  for (int c = 0; c <= N; ++c)
    for (int b = 0; b + c <= N; ++b)
      for (int a = 0; a + b + c <= N; ++a) {
        const double lam[4] = {double(N - a - b - c) / N, double(a) / N, double(b) / N, double(c) / N};
        double X[3] = {0, 0, 0};
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 3; ++d) X[d] += lam[v] * E[v][d];
        int nonzero = 0;
        for (int v = 0; v < 4; ++v) nonzero += lam[v] > tol;
        double shift[3] = {0, 0, 0};
        for (const auto& f : faces) {
          const int va = f[0];
          const int fv[3] = {f[1], f[2], f[3]};
          double w[3] = {0, 0, 0};
          for (int e = 0; e < 3; ++e) {
            const int u = fv[e], v = fv[(e + 1) % 3];
            double dir[3], len = 0;
            for (int d = 0; d < 3; ++d) {
              dir[d] = E[v][d] - E[u][d];
              len += dir[d] * dir[d];
            }
            len = std::sqrt(len);
            const double amt = 4.0 * lam[u] * lam[v] * warp(lam[v] - lam[u]);
            for (int d = 0; d < 3; ++d) w[d] += amt * dir[d] / len;
          }
          const double la = lam[va], lb = lam[fv[0]], lc = lam[fv[1]], ld = lam[fv[2]];
          const double den = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la);
          const double beta = den > tol ? lb * lc * ld / den : 0.0;
          for (int d = 0; d < 3; ++d) shift[d] += beta * w[d];
          if (la < tol && nonzero == 2)
            for (int d = 0; d < 3; ++d) shift[d] = w[d];
        }
        for (int d = 0; d < 3; ++d) X[d] += shift[d];
        // back to barycentrics of the equilateral tetrahedron, then bi-unit
        double A4[16], rhs[4] = {X[0], X[1], X[2], 1.0};
        for (int d = 0; d < 3; ++d)
          for (int v = 0; v < 4; ++v) A4[d * 4 + v] = E[v][d];
        for (int v = 0; v < 4; ++v) A4[12 + v] = 1.0;
        std::vector<double> Am(A4, A4 + 16), bv(rhs, rhs + 4);
        if (!solve_dense(4, 1, Am, bv)) throw std::runtime_error("tet node map");
        const int idx = tet_index(N, a, b, c);
        r[idx] = -1.0 + 2.0 * bv[1];
        s[idx] = -1.0 + 2.0 * bv[2];
        t[idx] = -1.0 + 2.0 * bv[3];
      }

  // operators
  std::vector<double> V(NP * NP), Vr(NP * NP), Vs(NP * NP), Vt(NP * NP);
  for (int i = 0; i < NP; ++i) pkd3(N, r[i], s[i], t[i], &V[i * NP], &Vr[i * NP], &Vs[i * NP], &Vt[i * NP]);
  invert(NP, V, Vinv_);
  Dr = matmul(NP, NP, NP, Vr, Vinv_);
  Ds = matmul(NP, NP, NP, Vs, Vinv_);
  Dt = matmul(NP, NP, NP, Vt, Vinv_);
  {
    std::vector<double> VVt(NP * NP, 0.0);
    for (int i = 0; i < NP; ++i)
      for (int j = 0; j < NP; ++j)
        for (int m = 0; m < NP; ++m) VVt[i * NP + j] += V[i * NP + m] * V[j * NP + m];
    invert(NP, VVt, M);
  }

  // face node lists: face-local triangle node (a', b') has barycentrics
  // (N-a'-b', a', b') relative to the face's vertices
  for (int f = 0; f < 4; ++f) {
    face_nodes[f].assign(NT, 0);
    for (int bb = 0; bb <= N; ++bb)
      for (int aa = 0; aa + bb <= N; ++aa) {
        int L[4] = {0, 0, 0, 0};
        L[kTetFaceVerts[f][0]] = N - aa - bb;
        L[kTetFaceVerts[f][1]] = aa;
        L[kTetFaceVerts[f][2]] = bb;
        face_nodes[f][tri_index(N, aa, bb)] = tet_index(N, L[1], L[2], L[3]);
      }
  }
  // LIFT = M^-1 [E_0 .. E_3]: on its face a tetrahedron basis function is the
  // triangle basis function of the face node (or zero), so E_f holds the
  // reference triangle mass in the rows of the face's nodes
  RefOps tri(N);
  std::vector<double> Ef(NP * 4 * NT, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int m = 0; m < NT; ++m)
      for (int q = 0; q < NT; ++q) Ef[face_nodes[f][m] * 4 * NT + f * NT + q] = tri.Mtri[m * NT + q];
  LIFT = Ef;
  if (!solve_dense(NP, 4 * NT, M, LIFT)) throw std::runtime_error("tet lift");
}

void TetOps::basis(double rr, double ss, double tt, double* out) const {
  std::vector<double> psi(NP);
  pkd3(N, rr, ss, tt, psi.data(), nullptr, nullptr, nullptr);
  for (int j = 0; j < NP; ++j) {
    double acc = 0.0;
    for (int m = 0; m < NP; ++m) acc += Vinv_[m * NP + j] * psi[m];
    out[j] = acc;
  }
}

}  // namespace wdg
