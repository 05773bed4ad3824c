// Host runtime of the LxW-DG library: reference tables, mesh connectivity and geometry, solver
// state, step sequencing, diagnostics and the C interface declared in include/lxw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/lxw.h"
#include "lxw_internal.hpp"

using namespace lxw;

namespace {

thread_local std::string g_err;

lxw_status fail(lxw_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail(e_ == hipErrorOutOfMemory ? LXW_ERR_OOM : LXW_ERR_DEVICE,       \
                                      std::string("HIP error: ") + hipGetErrorString(e_) + " at " + #expr); \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Reference elements.  Quadrature: Gauss-Legendre with 3 nodes on [-1,1] for edges and 1D, its
// 3x3 tensor product on the square, and the symmetric 7-point degree-5 rule on the triangle
// (centroid plus two three-point orbits).  Basis: on the line and the square the orthonormal
// Legendre polynomials sqrt(2n+1) P_n and their products; on the triangle the monomials
// 1, x, y, x^2, xy, y^2 (and at degree 3 x^3, x^2 y, x y^2, y^3) orthonormalised through the
// Cholesky factor of their Gram matrix, which is Gram-Schmidt in that order.
// ---------------------------------------------------------------------------------------------
struct Rule {
  std::vector<double> x, w;  // points (n x dim), weights summing to 1
};

const double GL_S[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};  // sqrt(3/5)
const double GL_W[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};

Rule rule_line() {
  Rule r;
  for (int i = 0; i < 3; ++i) { r.x.push_back(GL_S[i]); r.w.push_back(GL_W[i] / 2.0); }
  return r;
}
Rule rule_quad() {
  Rule r;
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) {
      r.x.push_back(GL_S[i]);
      r.x.push_back(GL_S[j]);
      r.w.push_back(GL_W[i] * GL_W[j] / 4.0);
    }
  return r;
}
Rule rule_tri() {
  Rule r;
  const double s15 = std::sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, b1 = 1.0 - 2.0 * a1, w1 = (155.0 - s15) / 1200.0;
  const double a2 = (6.0 + s15) / 21.0, b2 = 1.0 - 2.0 * a2, w2 = (155.0 + s15) / 1200.0;
  auto pt = [&](double x, double y, double w) { r.x.push_back(x); r.x.push_back(y); r.w.push_back(w); };
  pt(1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0);
  pt(a1, a1, w1); pt(b1, a1, w1); pt(a1, b1, w1);
  pt(a2, a2, w2); pt(b2, a2, w2); pt(a2, b2, w2);
  return r;
}

// Degree 3: four-point Gauss-Legendre, nodes +-sqrt(3/7 -+ (2/7) sqrt(6/5)) with weights
// (18 +- sqrt 30)/36, on the edges and in 1D; on the triangle the collapsed product rule
// (xi, eta) = ((1 + s)/2 (1 - t), t), t = (1 + x)/2, of the four Gauss-Legendre nodes s and the
// four Gauss-Jacobi nodes x of the weight 1 - x (the Jacobian 1 - t of the collapse), 16 points
// exact to degree 7.  The Gauss-Jacobi nodes and weights are the eigenvalues and squared first
// eigenvector components (times int (1 - x) dx = 2) of the symmetric Jacobi matrix of the
// three-term recurrence (Golub-Welsch), found by cyclic Jacobi rotations.
double GL4_S[4], GL4_W[4];
struct GL4Init {
  GL4Init() {
    const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(6.0 / 5.0));
    const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
    const double s[4] = {-b, -a, a, b}, w[4] = {wb, wa, wa, wb};
    for (int i = 0; i < 4; ++i) { GL4_S[i] = s[i]; GL4_W[i] = w[i]; }
  }
} gl4_init;

// n-point Gauss rule (n <= 4) for the weight (1 - x)^al on [-1, 1].
void gauss_jacobi(int npt, double al, double* x, double* w) {
  const double be = 0.0;
  double A[4][4] = {}, Z[4][4] = {};
  for (int n = 0; n < npt; ++n) {
    const double s = 2.0 * n + al + be;
    A[n][n] = (s == 0.0) ? 0.0 : (be * be - al * al) / (s * (s + 2.0));
    Z[n][n] = 1.0;
    if (n + 1 < npt) {
      const double m = n + 1.0, t = 2.0 * m + al + be;
      const double off = std::sqrt(4.0 * m * (m + al) * (m + be) * (m + al + be) / (t * t * (t + 1.0) * (t - 1.0)));
      A[n][n + 1] = A[n + 1][n] = off;
    }
  }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double offn = 0.0;
    for (int p = 0; p < npt; ++p)
      for (int q = p + 1; q < npt; ++q) offn += A[p][q] * A[p][q];
    if (offn < 1e-40) break;
    for (int p = 0; p < npt; ++p)
      for (int q = p + 1; q < npt; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < npt; ++k) {  // A <- A G (columns p, q)
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < npt; ++k) {  // A <- G^T A (rows p, q)
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < npt; ++k) {  // eigenvectors
          const double zkp = Z[k][p], zkq = Z[k][q];
          Z[k][p] = c * zkp - sn * zkq;
          Z[k][q] = sn * zkp + c * zkq;
        }
      }
  }
  int idx[4] = {0, 1, 2, 3};
  std::sort(idx, idx + npt, [&](int i, int j) { return A[i][i] < A[j][j]; });
  const double mu0 = std::pow(2.0, al + 1.0) / (al + 1.0);  // int_{-1}^{1} (1 - x)^al dx
  for (int k = 0; k < npt; ++k) {
    x[k] = A[idx[k]][idx[k]];
    w[k] = mu0 * Z[0][idx[k]] * Z[0][idx[k]];
  }
}

Rule rule_line4() {
  Rule r;
  for (int i = 0; i < 4; ++i) { r.x.push_back(GL4_S[i]); r.w.push_back(GL4_W[i] / 2.0); }
  return r;
}
Rule rule_tri16() {
  double xj[4], wj[4];
  gauss_jacobi(4, 1.0, xj, wj);
  Rule r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const double t = 0.5 * (1.0 + xj[j]);
      r.x.push_back(0.5 * (1.0 + GL4_S[i]) * (1.0 - t));
      r.x.push_back(t);
      r.w.push_back(0.25 * GL4_W[i] * wj[j]);  // (1/8) int (1 - x) ds dx over the area 1/2
    }
  return r;
}

// Tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1): the collapsed product rule
// (xi, eta, zeta) = (u (1 - v)(1 - w), v (1 - w), w), u, v, w = (1 + t)/2 at the 3-point Gauss rules
// for the weights 1, (1 - t) and (1 - t)^2, 27 points exact to degree 5; faces: the 7-point
// triangle rule on each face (barycentric coordinates on the face's vertices).
Rule rule_tet27() {
  double x0[4], w0[4], x1[4], w1[4], x2[4], w2[4];
  gauss_jacobi(3, 0.0, x0, w0);
  gauss_jacobi(3, 1.0, x1, w1);
  gauss_jacobi(3, 2.0, x2, w2);
  Rule r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        const double u = 0.5 * (1.0 + x0[i]), v = 0.5 * (1.0 + x1[j]), w = 0.5 * (1.0 + x2[k]);
        r.x.push_back(u * (1.0 - v) * (1.0 - w));
        r.x.push_back(v * (1.0 - w));
        r.x.push_back(w);
        r.w.push_back(6.0 / 64.0 * w0[i] * w1[j] * w2[k]);  // (1/|T0|) int over 1/64 of the t-cube
      }
  return r;
}
// face k of the tetrahedron is opposite vertex k; vertex order with (b - a) x (c - a) outward
const int TET_FACE[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
// the six orderings of a face's three vertices (index 0 the identity)
const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Legendre, orthonormal on [-1,1] under (1/2) int: sqrt(2n+1) P_n, n <= 3, and its derivatives.
double leg(int n, double x, int der) {
  const double s3 = std::sqrt(3.0), s5 = std::sqrt(5.0), s7 = std::sqrt(7.0);
  if (n == 0) return der == 0 ? 1.0 : 0.0;
  if (n == 1) return der == 0 ? s3 * x : (der == 1 ? s3 : 0.0);
  if (n == 2) {
    if (der == 0) return 0.5 * s5 * (3.0 * x * x - 1.0);
    if (der == 1) return 3.0 * s5 * x;
    return der == 2 ? 3.0 * s5 : 0.0;
  }
  if (der == 0) return 0.5 * s7 * (5.0 * x * x * x - 3.0 * x);
  if (der == 1) return 0.5 * s7 * (15.0 * x * x - 3.0);
  if (der == 2) return 15.0 * s7 * x;
  return der == 3 ? 15.0 * s7 : 0.0;
}

const int QUAD_I[9] = {0, 1, 0, 2, 1, 0, 2, 1, 2};
const int QUAD_J[9] = {0, 0, 1, 0, 1, 2, 1, 2, 2};
const int TRI_EX[10] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
const int TRI_EY[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};

double dmono(double x, int n, int k) {
  if (k > n) return 0.0;
  double c = 1.0;
  for (int i = 0; i < k; ++i) c *= (n - i);
  double r = c;
  for (int i = 0; i < n - k; ++i) r *= x;
  return r;
}

// The first ML of the monomials above (6 for P2, 10 for P3) orthonormalised on the triangle
// through the Cholesky factor of their Gram matrix, whose entries are the exact moments
// (1/|T0|) int x^a y^b = 2 a! b! / (a + b + 2)!.
template <int ML>
struct TriBasis {
  double C[ML][ML];  // phi_l = sum_j C[l][j] x^ex_j y^ey_j
  TriBasis() {
    auto fact = [](int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; };
    double G[ML][ML];
    for (int a = 0; a < ML; ++a)
      for (int b = 0; b < ML; ++b) {
        const int px = TRI_EX[a] + TRI_EX[b], py = TRI_EY[a] + TRI_EY[b];
        G[a][b] = 2.0 * fact(px) * fact(py) / fact(px + py + 2);
      }
    double L[ML][ML] = {};
    for (int i = 0; i < ML; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = G[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        L[i][j] = (i == j) ? std::sqrt(s) : s / L[j][j];
      }
    // C = L^{-1} (lower triangular)
    for (int i = 0; i < ML; ++i)
      for (int j = 0; j < ML; ++j) C[i][j] = 0.0;
    for (int col = 0; col < ML; ++col)
      for (int i = col; i < ML; ++i) {
        double s = (i == col) ? 1.0 : 0.0;
        for (int k = col; k < i; ++k) s -= L[i][k] * C[k][col];
        C[i][col] = s / L[i][i];
      }
  }
};

// Tetrahedron: 1, x, y, z, x^2, xy, xz, y^2, yz, z^2 orthonormalised through the Cholesky factor
// of their Gram matrix of exact moments (1/|T0|) int x^a y^b z^c = 6 a! b! c! / (a + b + c + 3)!.
const int TET_E[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                          {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
struct TetBasis {
  double C[10][10];
  TetBasis() {
    auto fact = [](int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; };
    double G[10][10];
    for (int a = 0; a < 10; ++a)
      for (int b = 0; b < 10; ++b) {
        const int px = TET_E[a][0] + TET_E[b][0], py = TET_E[a][1] + TET_E[b][1], pz = TET_E[a][2] + TET_E[b][2];
        G[a][b] = 6.0 * fact(px) * fact(py) * fact(pz) / fact(px + py + pz + 3);
      }
    double L[10][10] = {};
    for (int i = 0; i < 10; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = G[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        L[i][j] = (i == j) ? std::sqrt(s) : s / L[j][j];
      }
    for (int i = 0; i < 10; ++i)
      for (int j = 0; j < 10; ++j) C[i][j] = 0.0;
    for (int col = 0; col < 10; ++col)
      for (int i = col; i < 10; ++i) {
        double s = (i == col) ? 1.0 : 0.0;
        for (int k = col; k < i; ++k) s -= L[i][k] * C[k][col];
        C[i][col] = s / L[i][i];
      }
  }
};

// basis value / derivative at polynomial degree deg (2, or 3 on the line and the triangle): dx, dy,
// dz derivative orders
double basis(int kind, int deg, int l, const double* xi, int dx, int dy, int dz = 0) {
  if (kind == LXW_TET) {
    static const TetBasis tb;
    double s = 0.0;
    for (int j = 0; j < 10; ++j)
      s += tb.C[l][j] * dmono(xi[0], TET_E[j][0], dx) * dmono(xi[1], TET_E[j][1], dy) * dmono(xi[2], TET_E[j][2], dz);
    return s;
  }
  if (dz) return 0.0;
  if (kind == LXW_LINE) return dy ? 0.0 : leg(l, xi[0], dx);
  if (kind == LXW_QUAD) return leg(QUAD_I[l], xi[0], dx) * leg(QUAD_J[l], xi[1], dy);
  static const TriBasis<6> tb2;
  static const TriBasis<10> tb3;
  double s = 0.0;
  if (deg == 3)
    for (int j = 0; j < 10; ++j) s += tb3.C[l][j] * dmono(xi[0], TRI_EX[j], dx) * dmono(xi[1], TRI_EY[j], dy);
  else
    for (int j = 0; j < 6; ++j) s += tb2.C[l][j] * dmono(xi[0], TRI_EX[j], dx) * dmono(xi[1], TRI_EY[j], dy);
  return s;
}

int nverts(int kind) { return kind == LXW_LINE ? 2 : (kind == LXW_QUAD || kind == LXW_TET ? 4 : 3); }

void ref_vertex(int kind, int a, double* xi) {
  static const double line[2] = {-1, 1};
  static const double quad[8] = {-1, -1, 1, -1, 1, 1, -1, 1};
  static const double tri[6] = {0, 0, 1, 0, 0, 1};
  static const double tet[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (kind == LXW_TET) { for (int d = 0; d < 3; ++d) xi[d] = tet[3 * a + d]; return; }
  if (kind == LXW_LINE) xi[0] = line[a];
  else if (kind == LXW_QUAD) { xi[0] = quad[2 * a]; xi[1] = quad[2 * a + 1]; }
  else { xi[0] = tri[2 * a]; xi[1] = tri[2 * a + 1]; }
}

template <class E>
Rule rule_of() {
  if constexpr (E::DEG == 3) return E::kind == LXW_LINE ? rule_line4() : rule_tri16();
  else if constexpr (E::kind == LXW_TET) return rule_tet27();
  else return E::kind == LXW_LINE ? rule_line() : (E::kind == LXW_QUAD ? rule_quad() : rule_tri());
}
// Gauss-Legendre node j of the edges and its weight on [-1, 1]
template <class E>
double edge_s(int j) { return E::DEG == 3 ? GL4_S[j] : GL_S[j]; }
template <class E>
double edge_w(int j) {
  if constexpr (E::DIM == 3) return 2.0 * rule_tri().w[j];  // face rule, weights summing to 2
  else return E::DIM == 1 ? 2.0 : (E::DEG == 3 ? GL4_W[j] : GL_W[j]);
}

// limiter / update points: interior rule, then edge k Gauss point j (counter-clockwise)
template <class E>
std::vector<double> all_points() {
  std::vector<double> pts = rule_of<E>().x;
  for (int k = 0; k < E::K; ++k)
    for (int j = 0; j < E::NQE; ++j) {
      double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
      if constexpr (E::DIM == 3) {  // face k: the triangle rule's point j on the face's vertices
        const Rule f = rule_tri();
        const double lam[3] = {1.0 - f.x[2 * j] - f.x[2 * j + 1], f.x[2 * j], f.x[2 * j + 1]};
        double x[3] = {0, 0, 0};
        for (int m = 0; m < 3; ++m) {
          double vm[3];
          ref_vertex(E::kind, TET_FACE[k][m], vm);
          for (int d = 0; d < 3; ++d) x[d] += lam[m] * vm[d];
        }
        for (int d = 0; d < 3; ++d) pts.push_back(x[d]);
        continue;
      }
      ref_vertex(E::kind, k, a);
      ref_vertex(E::kind, (k + 1) % nverts(E::kind), b);
      if (E::DIM == 1) { pts.push_back(a[0]); continue; }
      const double t = 0.5 * (1.0 + edge_s<E>(j));
      pts.push_back(a[0] + t * (b[0] - a[0]));
      pts.push_back(a[1] + t * (b[1] - a[1]));
    }
  return pts;
}

template <class E, class R>
void fill_tab(RefTab<E, R>& T) {
  std::memset(&T, 0, sizeof(T));
  Rule r = rule_of<E>();
  std::vector<double> pts = all_points<E>();
  auto B = [](int l, const double* xi, int dx, int dy, int dz = 0) { return basis(E::kind, E::DEG, l, xi, dx, dy, dz); };
  // (dx, dy, dz) of the second derivatives in table order (3D: xx, xy, xz, yy, yz, zz)
  static const int D2[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
  for (int p = 0; p < E::NP; ++p) {
    double xi[3] = {pts[p * E::DIM], E::DIM >= 2 ? pts[p * E::DIM + 1] : 0.0, E::DIM == 3 ? pts[p * E::DIM + 2] : 0.0};
    if constexpr (E::DIM == 3) {
      for (int l = 0; l < E::ML; ++l) {
        T.phi[p][l] = R(B(l, xi, 0, 0, 0));
        for (int a = 0; a < 3; ++a) T.dphi[p][a][l] = R(B(l, xi, a == 0, a == 1, a == 2));
        for (int k = 0; k < 6; ++k) T.d2phi[p][k][l] = R(B(l, xi, D2[k][0], D2[k][1], D2[k][2]));
      }
      continue;
    }
    for (int l = 0; l < E::ML; ++l) {
      T.phi[p][l] = R(B(l, xi, 0, 0));
      T.dphi[p][0][l] = R(B(l, xi, 1, 0));
      T.d2phi[p][0][l] = R(B(l, xi, 2, 0));
      if constexpr (E::DIM == 2) {
        T.dphi[p][1][l] = R(B(l, xi, 0, 1));
        T.d2phi[p][1][l] = R(B(l, xi, 1, 1));
        T.d2phi[p][2][l] = R(B(l, xi, 0, 2));
      }
    }
  }
  for (int p = 0; p < E::NP; ++p)
    for (int d = 0; d < E::DIM; ++d) T.xr[p][d] = R(pts[p * E::DIM + d]);
  if constexpr (E::DIM == 3) {
    const double o[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < E::ML; ++l) {
      for (int a = 0; a < 3; ++a) T.dphi0[a][l] = R(B(l, o, a == 0, a == 1, a == 2));
      for (int k = 0; k < 6; ++k) T.d2c[k][l] = R(B(l, o, D2[k][0], D2[k][1], D2[k][2]));
    }
  } else {
    const double o[2] = {0.0, 0.0};
    for (int l = 0; l < E::ML; ++l) {
      T.dphi0[0][l] = R(B(l, o, 1, 0));
      T.d2c[0][l] = R(B(l, o, 2, 0));
      if constexpr (E::DIM == 2) {
        T.dphi0[1][l] = R(B(l, o, 0, 1));
        T.d2c[1][l] = R(B(l, o, 1, 1));
        T.d2c[2][l] = R(B(l, o, 0, 2));
      }
      if constexpr (E::DEG == 3)  // third derivatives, j of them in eta
        for (int j = 0; j < E::ND3; ++j) T.d3c[j][l] = R(B(l, o, 3 - j, j));
    }
  }
  for (int m = 0; m < E::NI; ++m)
    for (int l = 0; l < E::ML; ++l) {
      double xi[3] = {pts[m * E::DIM], E::DIM >= 2 ? pts[m * E::DIM + 1] : 0.0, E::DIM == 3 ? pts[m * E::DIM + 2] : 0.0};
      T.wphi[m][l] = R(r.w[m] * B(l, xi, 0, 0));
      for (int a = 0; a < E::DIM; ++a) T.wdphi[m][a][l] = R(r.w[m] * B(l, xi, a == 0, a == 1, a == 2));
    }
  // the projection composed with div F^h and its gradient at the reference origin, in float64
  // before rounding: kd0[m][a] = sum_l w_m phi_l(x_m) d_a phi_l(0), kd1[m][a][b] likewise with d_a d_b
  for (int m = 0; m < E::NI; ++m) {
    double xi[3] = {pts[m * E::DIM], E::DIM >= 2 ? pts[m * E::DIM + 1] : 0.0, E::DIM == 3 ? pts[m * E::DIM + 2] : 0.0};
    const double o[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < E::DIM; ++a) {
      double s0 = 0.0;
      for (int l = 0; l < E::ML; ++l) s0 += r.w[m] * B(l, xi, 0, 0) * B(l, o, a == 0, a == 1, a == 2);
      T.kd0[m][a] = R(s0);
      for (int b2 = 0; b2 < E::DIM; ++b2) {
        double s1 = 0.0;
        for (int l = 0; l < E::ML; ++l)
          s1 += r.w[m] * B(l, xi, 0, 0) * B(l, o, (a == 0) + (b2 == 0), (a == 1) + (b2 == 1), (a == 2) + (b2 == 2));
        T.kd1[m][a][b2] = R(s1);
      }
      if constexpr (E::DEG == 3)
        for (int j = 0; j < 2 * E::DIM - 1; ++j) {
          double s2 = 0.0;  // third derivative with a + j of its three in eta (1D: xxx)
          for (int l = 0; l < E::ML; ++l) s2 += r.w[m] * B(l, xi, 0, 0) * B(l, o, 3 - (a + j), a + j);
          T.kd2[m][a][j] = R(s2);
        }
    }
  }
  // in 1D a face is a point with the single weight 2, so that (1/2) sum omega = 1
  for (int j = 0; j < E::NQE; ++j) T.om[j] = R(edge_w<E>(j));
  for (int k = 0; k < E::K; ++k)
    for (int j = 0; j < E::NQE; ++j) {
      const int p = E::NI + k * E::NQE + j;
      double xi[3] = {pts[p * E::DIM], E::DIM >= 2 ? pts[p * E::DIM + 1] : 0.0, E::DIM == 3 ? pts[p * E::DIM + 2] : 0.0};
      for (int l = 0; l < E::ML; ++l) T.ephi[k][j][l] = R(0.5 * edge_w<E>(j) * B(l, xi, 0, 0));
    }
  // tetrahedron faces: point jl of a face whose vertex m is the first element's face vertex
  // PERM3[p][m] has barycentric coordinates lam'_{PERM3[p][m]} = lam_m in the first element's order
  for (int p = 0; p < 6; ++p)
    for (int j = 0; j < E::NQE; ++j) T.pperm[p][j] = j;
  if constexpr (E::DIM == 3) {
    const Rule f = rule_tri();
    auto bary = [&](int j, double* lam) { lam[0] = 1.0 - f.x[2 * j] - f.x[2 * j + 1]; lam[1] = f.x[2 * j]; lam[2] = f.x[2 * j + 1]; };
    for (int p = 0; p < 6; ++p)
      for (int jl = 0; jl < E::NQE; ++jl) {
        double mu[3], lam[3];
        bary(jl, mu);
        for (int m = 0; m < 3; ++m) lam[PERM3[p][m]] = mu[m];
        int best = -1;
        double bd = 1e300;
        for (int jj = 0; jj < E::NQE; ++jj) {
          double c[3];
          bary(jj, c);
          const double d = std::fabs(c[0] - lam[0]) + std::fabs(c[1] - lam[1]) + std::fabs(c[2] - lam[2]);
          if (d < bd) { bd = d; best = jj; }
        }
        T.pperm[p][jl] = best;
      }
  }
}

std::mutex g_init_mu;
int g_init_state = 0;  // 0 not done, 1 ok, -1 failed

lxw_status ensure_init() {
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_init_state == 1) return LXW_OK;
  std::unique_ptr<HostTabs> t(new HostTabs);
  fill_tab(t->line_d); fill_tab(t->line_f);
  fill_tab(t->quad_d); fill_tab(t->quad_f);
  fill_tab(t->tri_d); fill_tab(t->tri_f);
  fill_tab(t->line3_d); fill_tab(t->line3_f);
  fill_tab(t->tri3_d); fill_tab(t->tri3_f);
  fill_tab(t->tet_d); fill_tab(t->tet_f);
  hipError_t e = upload_tables(*t);
  if (e != hipSuccess) {
    g_init_state = -1;
    return fail(LXW_ERR_DEVICE, std::string("uploading reference tables: ") + hipGetErrorString(e));
  }
  // device address of the fixed workspace of lxw_indicator_grad_noalloc on the current device
  // (other devices look theirs up on their first such call)
  float* ws = nullptr;
  e = ind_static_scratch(&ws);
  if (e != hipSuccess) {
    g_init_state = -1;
    return fail(LXW_ERR_DEVICE, std::string("workspace address: ") + hipGetErrorString(e));
  }
  g_init_state = 1;
  return LXW_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Mesh: connectivity in the caller's order, then a Hilbert-curve renumbering of 2D elements by
// centroid for locality, then edges numbered in the new element order (i_e = the first element
// to visit the edge), geometry and the per-element edge slots.
// ---------------------------------------------------------------------------------------------
struct lxw_mesh {
  int kind = 0, dim = 0, N = 0, E = 0, K = 0, V = 0, ML = 0;
  int deg = 2;                      // polynomial degree (3 only in a degree-3 solver's own copy)
  std::vector<int> perm, iperm;     // internal -> caller, caller -> internal
  std::vector<double> vx;           // internal order: N x nv x dim
  std::vector<double> area, perim, Jinv, nout, hsz;  // N; N; N*dim*dim; N*K*dim; N
  std::vector<int> nbr, nbr_k, bcode;                // N*K (internal indices); bcode LXW_BC_* or -1
  std::vector<int> eslot;                            // N*K
  std::vector<unsigned char> fperm;                  // tetrahedra, N*K: order of the face's vertices
                                                     //   relative to the face's first element
  std::vector<int> e_i, e_j, e_bc;
  std::vector<int> e_ki, e_kj;                       // local edge index in i_e and j_e (-1)
  std::vector<double> e_n;                           // E*dim
  double geo = 0.0;
};

namespace {

// Gauss points per face: one in 1D, degree + 1 on the sides of 2D elements.
int nqe_of(const lxw_mesh& M) { return M.kind == LXW_LINE ? 1 : (M.kind == LXW_TET ? 7 : M.deg + 1); }

// Element configuration of a mesh: its kind, or 4 + kind at degree 3 (line and triangle).
enum { EK_LINE = LXW_LINE, EK_QUAD = LXW_QUAD, EK_TRI = LXW_TRI, EK_TET = LXW_TET, EK_LINE3 = 4 + LXW_LINE,
       EK_TRI3 = 4 + LXW_TRI };
int ekind(const lxw_mesh& M) { return M.deg == 3 ? 4 + M.kind : M.kind; }

int bc_to_slot(int bc) {
  switch (bc) {
    case LXW_BC_TRANSPARENT: return SB_TRANSPARENT;
    case LXW_BC_REFLECTIVE: return SB_REFLECTIVE;
    case LXW_BC_INFLOW: return SB_INFLOW;
    default: return SB_INTERIOR;
  }
}

// Index of (x, y) along a Hilbert curve over a 2^16 x 2^16 grid: consecutive indices are grid
// neighbours, so elements close in the order are close in space (fewer long jumps than a Z-order).
uint64_t hilbert2(uint32_t x, uint32_t y) {
  uint64_t d = 0;
  for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {  // rotate the quadrant (bits below s) so the sub-curve is traversed in order
      if (rx == 1) {
        x = s - 1 - (x & (s - 1)) + (x & ~(s - 1));
        y = s - 1 - (y & (s - 1)) + (y & ~(s - 1));
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Finish a mesh given, in caller order: vertex coordinates cvx (N x nv x dim), neighbours cnb /
// cnk (N x K, -1 on the boundary) and boundary codes cbc (N x K).
// Index of (x, y, z) along the Morton (Z-order) curve over a 2^21 grid per axis: elements close in
// the order are close in space (3D locality of the element numbering).
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t d = 0;
  for (int b = 20; b >= 0; --b)
    d = (d << 3) | ((uint64_t)((x >> b) & 1u) << 2) | ((uint64_t)((y >> b) & 1u) << 1) | (uint64_t)((z >> b) & 1u);
  return d;
}

lxw_status finish_mesh(lxw_mesh* M, const std::vector<double>& cvx, const std::vector<int>& cnb,
                       const std::vector<int>& cnk, const std::vector<int>& cbc, double alpha_unused,
                       const std::vector<unsigned char>* csig = nullptr) {
  (void)alpha_unused;
  const int N = M->N, K = M->K, dim = M->dim, nv = nverts(M->kind);
  // renumbering
  M->perm.resize(N);
  for (int i = 0; i < N; ++i) M->perm[i] = i;
  if (dim == 3 && N > 1) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    std::vector<double> cen(3 * (size_t)N);
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 3; ++d) {
        double c = 0.0;
        for (int a = 0; a < nv; ++a) c += cvx[((size_t)i * nv + a) * 3 + d];
        cen[3 * (size_t)i + d] = c / nv;
        lo[d] = std::min(lo[d], cen[3 * (size_t)i + d]);
        hi[d] = std::max(hi[d], cen[3 * (size_t)i + d]);
      }
    std::vector<uint64_t> code(N);
    for (int i = 0; i < N; ++i) {
      uint32_t q[3];
      for (int d = 0; d < 3; ++d) {
        double f = (hi[d] > lo[d]) ? (cen[3 * (size_t)i + d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
        q[d] = (uint32_t)std::min(2097151.0, std::max(0.0, f * 2097151.0));
      }
      code[i] = morton3(q[0], q[1], q[2]);
    }
    std::stable_sort(M->perm.begin(), M->perm.end(), [&](int a, int b) { return code[a] < code[b]; });
  }
  if (dim == 2 && N > 1) {
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    std::vector<double> cen(2 * N);
    for (int i = 0; i < N; ++i)
      for (int d = 0; d < 2; ++d) {
        double c = 0.0;
        for (int a = 0; a < nv; ++a) c += cvx[(i * nv + a) * 2 + d];
        cen[2 * i + d] = c / nv;
        lo[d] = std::min(lo[d], cen[2 * i + d]);
        hi[d] = std::max(hi[d], cen[2 * i + d]);
      }
    std::vector<uint64_t> code(N);
    for (int i = 0; i < N; ++i) {
      uint32_t q[2];
      for (int d = 0; d < 2; ++d) {
        double f = (hi[d] > lo[d]) ? (cen[2 * i + d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
        q[d] = (uint32_t)std::min(65535.0, std::max(0.0, f * 65535.0));
      }
      code[i] = hilbert2(q[0], q[1]);
    }
    std::stable_sort(M->perm.begin(), M->perm.end(), [&](int a, int b) { return code[a] < code[b]; });
  }
  M->iperm.resize(N);
  for (int i = 0; i < N; ++i) M->iperm[M->perm[i]] = i;
  M->vx.resize((size_t)N * nv * dim);
  M->nbr.assign((size_t)N * K, -1);
  M->nbr_k.assign((size_t)N * K, -1);
  M->bcode.assign((size_t)N * K, -1);
  std::vector<unsigned char> sig;  // internal order, per (element, face): permutation to the partner
  if (csig) sig.assign((size_t)N * K, 0);
  for (int i = 0; i < N; ++i) {
    const int c = M->perm[i];
    for (int x = 0; x < nv * dim; ++x) M->vx[(size_t)i * nv * dim + x] = cvx[(size_t)c * nv * dim + x];
    for (int k = 0; k < K; ++k) {
      const int j = cnb[(size_t)c * K + k];
      M->nbr[(size_t)i * K + k] = j >= 0 ? M->iperm[j] : -1;
      M->nbr_k[(size_t)i * K + k] = cnk[(size_t)c * K + k];
      M->bcode[(size_t)i * K + k] = j >= 0 ? -1 : cbc[(size_t)c * K + k];
      if (csig) sig[(size_t)i * K + k] = (*csig)[(size_t)c * K + k];
    }
  }
  // geometry
  M->area.resize(N);
  M->perim.resize(N);
  M->Jinv.resize((size_t)N * dim * dim);
  M->nout.resize((size_t)N * K * dim);
  M->hsz.resize(N);
  double geo = 0.0;
  for (int i = 0; i < N; ++i) {
    const double* v = &M->vx[(size_t)i * nv * dim];
    if (M->kind == LXW_LINE) {
      const double h = v[1] - v[0];
      if (!(h > 0.0)) return fail(LXW_ERR_MESH, "non-positive cell length");
      M->area[i] = h;
      M->perim[i] = 2.0;
      M->Jinv[i] = 2.0 / h;
      M->nout[(size_t)i * K + 0] = -1.0;
      M->nout[(size_t)i * K + 1] = 1.0;
      M->hsz[i] = h;
    } else if (M->kind == LXW_TET) {
      // J[a][b] = d x_a / d xi_b = (v_{b+1} - v_0)_a; Jinv = adj(J) / det
      double J[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = v[3 * (b + 1) + a] - v[a];
      double cof[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
          cof[a][b] = J[a1][b1] * J[a2][b2] - J[a1][b2] * J[a2][b1];
        }
      const double det = J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
      if (!(det > 0.0)) {
        char buf[128];
        snprintf(buf, sizeof buf, "element %d is negatively oriented or degenerate", M->perm[i]);
        return fail(LXW_ERR_MESH, buf);
      }
      double* Ji = &M->Jinv[(size_t)i * 9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ji[a * 3 + b] = cof[b][a] / det;
      M->area[i] = det / 6.0;
      double P = 0.0;
      for (int k = 0; k < K; ++k) {
        const double* A = &v[3 * TET_FACE[k][0]];
        const double* B = &v[3 * TET_FACE[k][1]];
        const double* C = &v[3 * TET_FACE[k][2]];
        const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        const double n[3] = {0.5 * (u[1] * w[2] - u[2] * w[1]), 0.5 * (u[2] * w[0] - u[0] * w[2]), 0.5 * (u[0] * w[1] - u[1] * w[0])};
        for (int d = 0; d < 3; ++d) M->nout[((size_t)i * K + k) * 3 + d] = n[d];
        P += std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      }
      M->perim[i] = P;
      M->hsz[i] = std::cbrt(6.0 * M->area[i]);  // the lattice spacing of a cube split into six
    } else {
      double J[2][2];
      if (M->kind == LXW_TRI) {
        J[0][0] = v[2] - v[0]; J[0][1] = v[4] - v[0];
        J[1][0] = v[3] - v[1]; J[1][1] = v[5] - v[1];
      } else {
        J[0][0] = 0.5 * (v[2] - v[0]); J[0][1] = 0.5 * (v[6] - v[0]);
        J[1][0] = 0.5 * (v[3] - v[1]); J[1][1] = 0.5 * (v[7] - v[1]);
      }
      const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      if (!(det > 0.0)) {
        char buf[128];
        snprintf(buf, sizeof buf, "element %d is clockwise or degenerate", M->perm[i]);
        return fail(LXW_ERR_MESH, buf);
      }
      double* Ji = &M->Jinv[(size_t)i * 4];
      Ji[0] = J[1][1] / det; Ji[1] = -J[0][1] / det;
      Ji[2] = -J[1][0] / det; Ji[3] = J[0][0] / det;
      M->area[i] = det * (M->kind == LXW_TRI ? 0.5 : 4.0);
      double P = 0.0;
      for (int k = 0; k < K; ++k) {
        const int b = (k + 1) % nv;
        const double dx = v[2 * b] - v[2 * k], dy = v[2 * b + 1] - v[2 * k + 1];
        M->nout[((size_t)i * K + k) * 2 + 0] = dy;
        M->nout[((size_t)i * K + k) * 2 + 1] = -dx;
        P += std::sqrt(dx * dx + dy * dy);
      }
      M->perim[i] = P;
      M->hsz[i] = M->kind == LXW_TRI ? std::sqrt(2.0 * M->area[i]) : std::sqrt(M->area[i]);
    }
    geo = std::max(geo, M->perim[i] / (2.0 * M->area[i]));
  }
  M->geo = geo;
  // edges in internal element order
  M->eslot.assign((size_t)N * K, -1);
  M->e_i.clear(); M->e_j.clear(); M->e_bc.clear(); M->e_n.clear(); M->e_ki.clear(); M->e_kj.clear();
  int E = 0;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < K; ++k) {
      if (M->eslot[(size_t)i * K + k] >= 0) continue;
      const int j = M->nbr[(size_t)i * K + k], kj = M->nbr_k[(size_t)i * K + k];
      const int e = E++;
      const int bc = j >= 0 ? SB_INTERIOR : bc_to_slot(M->bcode[(size_t)i * K + k]);
      M->e_i.push_back(i);
      M->e_j.push_back(j);
      M->e_ki.push_back(k);
      M->e_kj.push_back(j >= 0 ? kj : -1);
      M->e_bc.push_back(bc);
      for (int d = 0; d < dim; ++d) M->e_n.push_back(M->nout[((size_t)i * K + k) * dim + d]);
      M->eslot[(size_t)i * K + k] = e * 8 + 0 * 4 + bc;
      if (j >= 0) {
        if (M->eslot[(size_t)j * K + kj] >= 0) return fail(LXW_ERR_MESH, "an edge is shared by more than two elements");
        M->eslot[(size_t)j * K + kj] = e * 8 + 1 * 4 + SB_INTERIOR;
        // the second element takes the edge's normal negated (its own cross product or vertex
        // differences can differ by rounding, on periodic sides and on faces): both sides of an
        // edge then form the same |n_e| for the Lax-Friedrichs part of F*
        for (int d = 0; d < dim; ++d) M->nout[((size_t)j * K + kj) * dim + d] = -M->nout[((size_t)i * K + k) * dim + d];
      }
    }
  M->E = E;
  // tetrahedra: the first element of a face reads its points in its own order (permutation 0),
  // the second one through the permutation of its face's vertices onto the first one's
  if (csig) {
    M->fperm.assign((size_t)N * K, 0);
    for (int e = 0; e < E; ++e)
      if (M->e_j[e] >= 0) M->fperm[(size_t)M->e_j[e] * K + M->e_kj[e]] = sig[(size_t)M->e_j[e] * K + M->e_kj[e]];
  }
  return LXW_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// Solver
// ---------------------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct lxw_solver {
  const lxw_mesh* M = nullptr;
  std::unique_ptr<lxw_mesh> own_mesh;  // degree 3: M is this copy of the caller's mesh
  lxw_params P{};
  hipStream_t st = nullptr;
  bool fp32 = false;
  std::vector<DevBuf> bufs;
  View<double> vd{};
  View<float> vf{};
  Scalars* sc = nullptr;
  DevError* err = nullptr;
  Scalars hsc{};
  bool debug = false;
  // diagnostics copies
  double* dq_upd_bar = nullptr;
  void* dq_upd_h = nullptr;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<int> ev_kid;
  size_t ev_used = 0;
  double kms[LXW_K_COUNT] = {};
  int64_t kcount[LXW_K_COUNT] = {};
  // launch shapes
  LaunchCfg cfg{};
  // batched form: n_mesh meshes concatenated into M (elements of mesh b at [eoff[b], eoff[b+1]))
  int n_mesh = 1;
  bool batch = false;
  std::vector<int> eoff{0, 0};
  std::vector<int> mesh_of, e_mesh;  // host copies uploaded by setup_view (batched form only)
  std::vector<double> geo_m;         // per mesh max |dT|/(2|T|)
  std::vector<Scalars> hscv;         // per-mesh scalars after the last sync
  // one step captured in a HIP graph (replayed by lxw_run_steps)
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  // learned troubled-cell indicator (triangles): decisions per element, decision counts
  const lxw_indicator* ind = nullptr;
  unsigned char* ind_flag = nullptr;
  unsigned long long* ind_counts = nullptr;
  double t_end = std::numeric_limits<double>::infinity();  // end time last set on the device
  float tau_lo = 0.0f, tau_hi = 1.0f;
  ~lxw_solver() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto& b : bufs) if (b.p) (void)hipFree(b.p);
    for (auto& e : ev_pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }
  template <class T>
  lxw_status alloc(T** out, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return fail(LXW_ERR_OOM, std::string("device allocation failed: ") + hipGetErrorString(e));
    bufs.push_back({p, count * sizeof(T)});
    *out = (T*)p;
    return LXW_OK;
  }
};

// Learned troubled-cell indicator: FP32 master parameters with Adam moments, and the bf16 /
// FP32 arrays the inference kernel reads (packed from the master parameters).
struct lxw_indicator {
  hipStream_t st = nullptr;
  float* theta = nullptr;  // [IND_NPARAM]
  float* m = nullptr;
  float* v = nullptr;
  int64_t t = 0;           // Adam updates so far
  uint16_t* A1 = nullptr;  // [2][3][64][8]
  uint16_t* A2 = nullptr;  // [2][4][64][8]
  float* b1p = nullptr;    // [2][2][16]
  float* b2p = nullptr;
  float* w3p = nullptr;    // [2][2][16] + b3
  float* part = nullptr;   // [part_blocks][IND_PART]
  int part_blocks = 0;
  float* scal = nullptr;   // [1] loss
  std::vector<void*> bufs;
  ~lxw_indicator() {
    if (st) (void)hipStreamSynchronize(st);
    for (void* p : bufs) (void)hipFree(p);
  }
};

// A batch: independent meshes of one kind concatenated into one internal mesh, advanced by one
// solver whose kernels cover all of them (each mesh keeps its own s, dt and t).
struct lxw_batch {
  std::vector<const lxw_mesh*> ms;  // caller's meshes (outlive the batch)
  lxw_mesh merged;
  lxw_solver* S = nullptr;
  ~lxw_batch() { delete S; }
};

namespace {

template <class T>
lxw_status upload(lxw_solver* S, const T** dst, const std::vector<T>& host) {
  T* p = nullptr;
  lxw_status s = S->alloc(&p, host.size());
  if (s) return s;
  hipError_t e = hipMemcpy(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(LXW_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e));
  *dst = p;
  return LXW_OK;
}

// Upload geometry and allocate the work arrays for precision R.
template <class R>
lxw_status setup_view(lxw_solver* S, View<R>& v) {
  const lxw_mesh& M = *S->M;
  const int N = M.N, E = M.E, K = M.K, dim = M.dim, V = M.V, ML = M.ML;
  const int NQE = nqe_of(M);
  std::memset(&v, 0, sizeof(v));
  v.N = N;
  v.E = E;
  lxw_status st;
  // SoA transposes
  std::vector<double> Ji((size_t)dim * dim * N), no((size_t)K * dim * N), delta(N);
  std::vector<int> es((size_t)K * N), nb((size_t)K * N);
  for (int i = 0; i < N; ++i) {
    for (int x = 0; x < dim * dim; ++x) Ji[(size_t)x * N + i] = M.Jinv[(size_t)i * dim * dim + x];
    for (int k = 0; k < K; ++k) {
      for (int d = 0; d < dim; ++d) no[((size_t)k * dim + d) * N + i] = M.nout[((size_t)i * K + k) * dim + d];
      es[(size_t)k * N + i] = M.eslot[(size_t)i * K + k];
      nb[(size_t)k * N + i] = M.nbr[(size_t)i * K + k];
    }
    delta[i] = S->P.alpha0 * std::pow(M.hsz[i], 1.5);
  }
  std::vector<R> JiR(Ji.begin(), Ji.end()), noR(no.begin(), no.end());
  std::vector<double> en((size_t)dim * E);
  for (int e = 0; e < E; ++e)
    for (int d = 0; d < dim; ++d) en[(size_t)d * E + e] = M.e_n[(size_t)e * dim + d];
  if ((st = upload(S, &v.area, M.area))) return st;
  if ((st = upload(S, &v.Jinv, JiR))) return st;
  if ((st = upload(S, &v.nout, noR))) return st;
  if ((st = upload(S, &v.eslot, es))) return st;
  if ((st = upload(S, &v.nbr, nb))) return st;
  if (!M.fperm.empty()) {
    std::vector<unsigned char> fp((size_t)K * N);
    for (int i = 0; i < N; ++i)
      for (int k = 0; k < K; ++k) fp[(size_t)k * N + i] = M.fperm[(size_t)i * K + k];
    if ((st = upload(S, &v.fperm, fp))) return st;
  }
  if ((st = upload(S, &v.delta, delta))) return st;
  if ((st = upload(S, &v.e_i, M.e_i))) return st;
  if ((st = upload(S, &v.e_j, M.e_j))) return st;
  if ((st = upload(S, &v.e_bc, M.e_bc))) return st;
  if ((st = upload(S, &v.e_n, en))) return st;
  v.mesh_of = nullptr;
  v.e_mesh = nullptr;
  if (S->batch) {
    if ((st = upload(S, &v.mesh_of, S->mesh_of))) return st;
    if ((st = upload(S, &v.e_mesh, S->e_mesh))) return st;
  }
  if ((st = S->alloc(&v.Qbar, (size_t)V * N))) return st;
  if ((st = S->alloc(&v.Qh, (size_t)V * (ML - 1) * N))) return st;
  if ((st = S->alloc(&v.theta, (size_t)N))) return st;
  if ((st = S->alloc(&v.spart, (size_t)egrid_blocks(N, 64)))) return st;  // smallest tunable workgroup
  if ((st = S->alloc(&v.tr, (size_t)2 * NQE * V * E))) return st;
  if ((st = S->alloc(&v.fstar, (size_t)NQE * V * E))) return st;
  if ((st = S->alloc(&v.fLxW, (size_t)V * E))) return st;
  if ((st = S->alloc(&v.fLxF, (size_t)V * E))) return st;
  if ((st = S->alloc(&v.cedge, (size_t)2 * E))) return st;
  {
    std::vector<double> ones((size_t)2 * E, 1.0);
    HIPCHK(hipMemcpy(v.cedge, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  v.sc = S->sc;
  v.err = S->err;
  v.gamma = S->P.gamma;
  v.eps0 = S->P.eps0;
  for (int c = 0; c < 4; ++c) v.inflow[c] = S->P.inflow[c];
  v.shock = S->P.shock;
  v.theta_exact = S->P.theta_exact;
  v.s_avg = S->P.wave_speed;
  return LXW_OK;
}

template <class E, class R>
hipError_t launch_one(lxw_solver* S, const View<R>& v, KernelId k, int mode) {
  const int pub = (k == K_SHOCK) ? LXW_K_PRE : (int)k;
  hipEvent_t a = nullptr, b = nullptr;
  if (S->timing) {
    if (S->ev_used == S->ev_pool.size()) {
      hipEvent_t x, y;
      if (hipEventCreate(&x) != hipSuccess || hipEventCreate(&y) != hipSuccess) return hipErrorOutOfMemory;
      S->ev_pool.push_back({x, y});
      S->ev_kid.push_back(0);
    }
    a = S->ev_pool[S->ev_used].first;
    b = S->ev_pool[S->ev_used].second;
    S->ev_kid[S->ev_used] = pub;
    S->ev_used++;
    hipError_t e = hipEventRecord(a, S->st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch<E, R>(k, v, S->cfg, S->st, S->n_mesh, mode);
  if (e != hipSuccess) return e;
  if (S->timing) e = hipEventRecord(b, S->st);
  return e;
}

IndW ind_weights(const lxw_solver* S) {
  const lxw_indicator* I = S->ind;
  IndW W{};
  W.A1 = I->A1; W.A2 = I->A2; W.b1 = I->b1p; W.b2 = I->b2p; W.w3 = I->w3p;
  W.tau_lo = S->tau_lo;
  W.tau_hi = S->tau_hi;
  return W;
}

// The learned indicator's decisions for the pending shock-capturing limiter (triangles only).
template <class E, class R>
hipError_t launch_ind_step(lxw_solver* S, const View<R>& v, bool in_step) {
  if constexpr (E::kind == ElTri::kind) {
    if (!S->ind) return hipSuccess;
    hipEvent_t a = nullptr, b = nullptr;
    if (S->timing) {
      if (S->ev_used == S->ev_pool.size()) {
        hipEvent_t x, y;
        if (hipEventCreate(&x) != hipSuccess || hipEventCreate(&y) != hipSuccess) return hipErrorOutOfMemory;
        S->ev_pool.push_back({x, y});
        S->ev_kid.push_back(0);
      }
      a = S->ev_pool[S->ev_used].first;
      b = S->ev_pool[S->ev_used].second;
      S->ev_kid[S->ev_used] = LXW_K_IND;
      S->ev_used++;
      hipError_t e = hipEventRecord(a, S->st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = launch_indicator<R>(v, ind_weights(S), S->ind_flag, S->ind_counts, in_step, S->st);
    if (e == hipSuccess && S->timing) e = hipEventRecord(b, S->st);
    return e;
  } else {
    (void)S; (void)v;
    return hipSuccess;
  }
}

template <class E, class R>
lxw_status enqueue_step_t(lxw_solver* S, const View<R>& v) {
  const lxw_mesh& M = *S->M;
  const int V = M.V, ML = M.ML, N = M.N;
  HIPCHK((launch_ind_step<E, R>(S, v, true)));
  HIPCHK((launch_one<E, R>(S, v, K_PRE, 0)));
  HIPCHK((launch_one<E, R>(S, v, K_DT, 0)));
  HIPCHK((launch_one<E, R>(S, v, K_ELEM, 0)));
  HIPCHK((launch_one<E, R>(S, v, K_EDGE, 0)));
  HIPCHK((launch_one<E, R>(S, v, K_FLIM, 0)));
  HIPCHK((launch_one<E, R>(S, v, K_UPDATE, 0)));
  if (S->debug) {
    HIPCHK(hipMemcpyAsync(S->dq_upd_bar, v.Qbar, (size_t)V * N * sizeof(double), hipMemcpyDeviceToDevice, S->st));
    HIPCHK(hipMemcpyAsync(S->dq_upd_h, v.Qh, (size_t)V * (ML - 1) * N * sizeof(R), hipMemcpyDeviceToDevice, S->st));
  }
  return LXW_OK;
}

template <class E, class R>
lxw_status enqueue_shock_t(lxw_solver* S, const View<R>& v) {
  HIPCHK((launch_ind_step<E, R>(S, v, false)));
  HIPCHK((launch_one<E, R>(S, v, K_SHOCK, 1)));
  HIPCHK((launch_one<E, R>(S, v, K_FINAL, 1)));
  return LXW_OK;
}

lxw_status enqueue_step(lxw_solver* S) {
  switch (ekind(*S->M)) {
    case EK_LINE: return S->fp32 ? enqueue_step_t<ElLine, float>(S, S->vf) : enqueue_step_t<ElLine, double>(S, S->vd);
    case EK_QUAD: return S->fp32 ? enqueue_step_t<ElQuad, float>(S, S->vf) : enqueue_step_t<ElQuad, double>(S, S->vd);
    case EK_LINE3: return S->fp32 ? enqueue_step_t<ElLine3, float>(S, S->vf) : enqueue_step_t<ElLine3, double>(S, S->vd);
    case EK_TRI3: return S->fp32 ? enqueue_step_t<ElTri3, float>(S, S->vf) : enqueue_step_t<ElTri3, double>(S, S->vd);
    case EK_TET: return S->fp32 ? enqueue_step_t<ElTet, float>(S, S->vf) : enqueue_step_t<ElTet, double>(S, S->vd);
    default: return S->fp32 ? enqueue_step_t<ElTri, float>(S, S->vf) : enqueue_step_t<ElTri, double>(S, S->vd);
  }
}

lxw_status enqueue_shock(lxw_solver* S) {
  switch (ekind(*S->M)) {
    case EK_LINE: return S->fp32 ? enqueue_shock_t<ElLine, float>(S, S->vf) : enqueue_shock_t<ElLine, double>(S, S->vd);
    case EK_QUAD: return S->fp32 ? enqueue_shock_t<ElQuad, float>(S, S->vf) : enqueue_shock_t<ElQuad, double>(S, S->vd);
    case EK_LINE3: return S->fp32 ? enqueue_shock_t<ElLine3, float>(S, S->vf) : enqueue_shock_t<ElLine3, double>(S, S->vd);
    case EK_TRI3: return S->fp32 ? enqueue_shock_t<ElTri3, float>(S, S->vf) : enqueue_shock_t<ElTri3, double>(S, S->vd);
    case EK_TET: return S->fp32 ? enqueue_shock_t<ElTet, float>(S, S->vf) : enqueue_shock_t<ElTet, double>(S, S->vd);
    default: return S->fp32 ? enqueue_shock_t<ElTri, float>(S, S->vf) : enqueue_shock_t<ElTri, double>(S, S->vd);
  }
}

// Wait for the stream, read the scalars and the error record, accumulate kernel timings.
lxw_status sync_check(lxw_solver* S) {
  HIPCHK(hipStreamSynchronize(S->st));
  if (S->timing) {
    for (size_t x = 0; x < S->ev_used; ++x) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, S->ev_pool[x].first, S->ev_pool[x].second));
      S->kms[S->ev_kid[x]] += ms;
      S->kcount[S->ev_kid[x]] += 1;
    }
    S->ev_used = 0;
  }
  S->hscv.resize(S->n_mesh);
  HIPCHK(hipMemcpy(S->hscv.data(), S->sc, S->n_mesh * sizeof(Scalars), hipMemcpyDeviceToHost));
  S->hsc = S->hscv[0];
  DevError de{};
  HIPCHK(hipMemcpy(&de, S->err, sizeof(DevError), hipMemcpyDeviceToHost));
  if (de.code != 0) {
    const int caller = (de.elem >= 0 && de.elem < S->M->N) ? S->M->perm[de.elem] : -1;
    const char* what = de.code == LXW_ERR_CFL ? "Lax-Friedrichs update not positive: time step too large"
                       : de.code == LXW_ERR_NONFINITE ? "non-finite value"
                                                      : "cell-average density or pressure not positive";
    char buf[240];
    if (S->batch && caller >= 0) {
      const int b = (int)(std::upper_bound(S->eoff.begin(), S->eoff.end(), caller) - S->eoff.begin()) - 1;
      snprintf(buf, sizeof buf, "%s (mesh %d, element %d, t = %.17g)", what, b, caller - S->eoff[b], S->hscv[b].t);
    } else {
      snprintf(buf, sizeof buf, "%s (element %d, t = %.17g)", what, caller, S->hsc.t);
    }
    DevError z{};
    HIPCHK(hipMemcpy(S->err, &z, sizeof(DevError), hipMemcpyHostToDevice));
    return fail(de.code, buf);
  }
  return LXW_OK;
}

// Checks a caller state of mesh Mloc (rho_bar >= eps0, p_bar > 0, finite) and uploads it, in the
// internal order, into elements [off, off + Mloc.N) of the solver's state.
lxw_status load_state(lxw_solver* S, const lxw_mesh& Mloc, int off, const double* Q, int32_t flags) {
  const int N = Mloc.N, V = Mloc.V, ML = Mloc.ML, dim = Mloc.dim, Nt = S->M->N;
  const size_t n = (size_t)N * V * ML;
  std::vector<double> h(n);
  HIPCHK(hipStreamSynchronize(S->st));
  if (flags & LXW_DEVICE_PTR) {
    HIPCHK(hipMemcpy(h.data(), Q, n * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(h.data(), Q, n * sizeof(double));
  }
  for (int c = 0; c < N && !(flags & LXW_STATE_UNCHECKED); ++c) {
    const double* q = &h[(size_t)c * V * ML];
    double qb[4];
    bool fin = true;
    for (int v = 0; v < V; ++v) { qb[v] = q[v * ML]; for (int l = 0; l < ML; ++l) fin = fin && std::isfinite(q[v * ML + l]); }
    double k = 0.0;
    for (int d = 0; d < dim; ++d) k += qb[1 + d] * qb[1 + d];
    const double pb = (S->P.gamma - 1.0) * (qb[V - 1] - 0.5 * k / qb[0]);
    if (!fin || !(qb[0] >= S->P.eps0) || !(pb > 0.0)) {
      char buf[160];
      snprintf(buf, sizeof buf, "initial state violates rho_bar >= eps0, p_bar > 0 or is not finite (element %d)", c);
      return fail(LXW_ERR_STATE, buf);
    }
  }
  std::vector<double> qbar((size_t)V * N);  // [N][V]
  std::vector<double> qh((size_t)V * (ML - 1) * N);
  for (int i = 0; i < N; ++i) {
    const double* q = &h[(size_t)Mloc.perm[i] * V * ML];
    for (int v = 0; v < V; ++v) {
      qbar[(size_t)i * V + v] = q[v * ML];
      for (int l = 1; l < ML; ++l) qh[((size_t)v * (ML - 1) + l - 1) * N + i] = q[v * ML + l];
    }
  }
  double* dbar = S->fp32 ? S->vf.Qbar : S->vd.Qbar;
  HIPCHK(hipMemcpy(dbar + (size_t)off * V, qbar.data(), qbar.size() * sizeof(double), hipMemcpyHostToDevice));
  const int rows = V * (ML - 1);
  if (S->fp32) {
    std::vector<float> f(qh.begin(), qh.end());
    for (int r = 0; r < rows; ++r)
      HIPCHK(hipMemcpy(S->vf.Qh + (size_t)r * Nt + off, &f[(size_t)r * N], N * sizeof(float), hipMemcpyHostToDevice));
  } else {
    for (int r = 0; r < rows; ++r)
      HIPCHK(hipMemcpy(S->vd.Qh + (size_t)r * Nt + off, &qh[(size_t)r * N], N * sizeof(double), hipMemcpyHostToDevice));
  }
  return LXW_OK;
}

// Time t0, no step taken, no limiter pending, for mesh b.
lxw_status reset_scalars(lxw_solver* S, int b, double t0) {
  Scalars z{};
  z.geo = S->geo_m[b];
  z.cfl = S->P.cfl;
  z.t = t0;
  z.T = std::numeric_limits<double>::infinity();
  HIPCHK(hipMemcpy(S->sc + b, &z, sizeof z, hipMemcpyHostToDevice));
  S->t_end = z.T;
  if ((int)S->hscv.size() != S->n_mesh) S->hscv.assign(S->n_mesh, Scalars{});
  S->hscv[b] = z;
  S->hsc = S->hscv[0];
  return LXW_OK;
}

// Device state of elements [off, off + Mloc.N) -> caller layout of mesh Mloc (float64).
lxw_status store_state(lxw_solver* S, const lxw_mesh& Mloc, int off, bool upd_copy, std::vector<double>& out) {
  const int N = Mloc.N, V = Mloc.V, ML = Mloc.ML, Nt = S->M->N;
  std::vector<double> qbar((size_t)V * N), qh((size_t)V * (ML - 1) * N);
  const double* src_bar = upd_copy ? S->dq_upd_bar : (S->fp32 ? S->vf.Qbar : S->vd.Qbar);
  const char* src_h = (const char*)(upd_copy ? S->dq_upd_h : (S->fp32 ? (const void*)S->vf.Qh : (const void*)S->vd.Qh));
  HIPCHK(hipMemcpy(qbar.data(), src_bar + (size_t)off * V, qbar.size() * sizeof(double), hipMemcpyDeviceToHost));
  const int rows = V * (ML - 1);
  if (S->fp32) {
    std::vector<float> f(qh.size());
    for (int r = 0; r < rows; ++r)
      HIPCHK(hipMemcpy(&f[(size_t)r * N], src_h + ((size_t)r * Nt + off) * sizeof(float), N * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t x = 0; x < f.size(); ++x) qh[x] = f[x];
  } else {
    for (int r = 0; r < rows; ++r)
      HIPCHK(hipMemcpy(&qh[(size_t)r * N], src_h + ((size_t)r * Nt + off) * sizeof(double), N * sizeof(double), hipMemcpyDeviceToHost));
  }
  out.assign((size_t)N * V * ML, 0.0);
  for (int i = 0; i < N; ++i) {
    double* q = &out[(size_t)Mloc.perm[i] * V * ML];
    for (int v = 0; v < V; ++v) {
      q[v * ML] = qbar[(size_t)i * V + v];
      for (int l = 1; l < ML; ++l) q[v * ML + l] = qh[((size_t)v * (ML - 1) + l - 1) * N + i];
    }
  }
  return LXW_OK;
}

// Capture one step (no final time) on the library's own stream into a graph.
lxw_status capture_step(lxw_solver* S) {
  if (!S->cap) HIPCHK(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
  hipStream_t user = S->st;
  S->st = S->cap;
  lxw_status s = enqueue_step(S);
  S->st = user;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(S->cap, &g);
  if (s) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(LXW_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    S->gexec = nullptr;
    return fail(LXW_ERR_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(e));
  }
  return LXW_OK;
}

void drop_graph(lxw_solver* S) {
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  S->gexec = nullptr;
}

lxw_status check_params(const lxw_params* p) {
  if (p->degree != 2 && p->degree != 3) return fail(LXW_ERR_UNSUPPORTED, "polynomial degree 2 or 3");
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->cfl <= 1.0) || !(p->eps0 > 0.0) || !(p->alpha0 >= 0.0))
    return fail(LXW_ERR_ARG, "need gamma > 1, 0 < cfl <= 1, eps0 > 0, alpha0 >= 0");
  if (p->precision != LXW_FP64 && p->precision != LXW_FP32_MIXED) return fail(LXW_ERR_ARG, "bad precision");
  if (p->shock != LXW_SHOCK_OFF && p->shock != LXW_SHOCK_PLAIN) return fail(LXW_ERR_UNSUPPORTED, "bad shock-limiter mode");
  if (p->theta_exact != 0 && p->theta_exact != 1) return fail(LXW_ERR_ARG, "theta_exact must be 0 or 1");
  if (p->wave_speed != LXW_SPEED_POINTS && p->wave_speed != LXW_SPEED_AVERAGES)
    return fail(LXW_ERR_ARG, "wave_speed must be LXW_SPEED_POINTS or LXW_SPEED_AVERAGES");
  return LXW_OK;
}

// Solver over mesh m.  With `batch` (the merged mesh of a batch, m == batch->mesh), the per-mesh
// offsets, element and edge mesh indices and geometry factors come from it.
struct BatchLayout {
  std::vector<int> eoff, mesh_of, e_mesh;
  std::vector<double> geo;
};

// Concatenate meshes (each already in its internal order) into one: elements of mesh b occupy
// [eoff[b], eoff[b+1]), its edges a contiguous range in the same order; caller order of the merged
// mesh is the concatenation of the meshes' caller orders.
lxw_status merge_meshes(const std::vector<const lxw_mesh*>& ms, lxw_mesh& M, BatchLayout& bl) {
  const lxw_mesh& m0 = *ms[0];
  M.kind = m0.kind; M.dim = m0.dim; M.K = m0.K; M.V = m0.V; M.ML = m0.ML;
  int64_t Nt = 0, Et = 0;
  for (const lxw_mesh* m : ms) { Nt += m->N; Et += m->E; }
  if (Nt > (int64_t)INT32_MAX / 8 || Et > (int64_t)INT32_MAX / 8) return fail(LXW_ERR_ARG, "batch too large for 32-bit indices");
  M.N = (int)Nt;
  M.E = (int)Et;
  const int K = M.K, nvd = nverts(M.kind) * M.dim;
  bl.eoff.assign(1, 0);
  bl.geo.clear();
  bl.mesh_of.resize(Nt);
  bl.e_mesh.resize(Et);
  M.geo = 0.0;
  int eo = 0, go = 0;
  for (size_t b = 0; b < ms.size(); ++b) {
    const lxw_mesh& m = *ms[b];
    for (int i = 0; i < m.N; ++i) {
      M.perm.push_back(eo + m.perm[i]);
      bl.mesh_of[eo + i] = (int)b;
    }
    for (int i = 0; i < m.N; ++i) M.iperm.push_back(eo + m.iperm[i]);
    M.vx.insert(M.vx.end(), m.vx.begin(), m.vx.begin() + (size_t)m.N * nvd);
    M.area.insert(M.area.end(), m.area.begin(), m.area.end());
    M.perim.insert(M.perim.end(), m.perim.begin(), m.perim.end());
    M.Jinv.insert(M.Jinv.end(), m.Jinv.begin(), m.Jinv.end());
    M.nout.insert(M.nout.end(), m.nout.begin(), m.nout.end());
    M.hsz.insert(M.hsz.end(), m.hsz.begin(), m.hsz.end());
    for (size_t x = 0; x < (size_t)m.N * K; ++x) {
      M.nbr.push_back(m.nbr[x] >= 0 ? m.nbr[x] + eo : -1);
      M.nbr_k.push_back(m.nbr_k[x]);
      M.bcode.push_back(m.bcode[x]);
      M.eslot.push_back(((m.eslot[x] >> 3) + go) * 8 + (m.eslot[x] & 7));
    }
    for (int e = 0; e < m.E; ++e) {
      M.e_i.push_back(m.e_i[e] + eo);
      M.e_j.push_back(m.e_j[e] >= 0 ? m.e_j[e] + eo : -1);
      M.e_bc.push_back(m.e_bc[e]);
      M.e_ki.push_back(m.e_ki[e]);
      M.e_kj.push_back(m.e_kj[e]);
      bl.e_mesh[go + e] = (int)b;
    }
    M.e_n.insert(M.e_n.end(), m.e_n.begin(), m.e_n.end());
    bl.geo.push_back(m.geo);
    M.geo = std::max(M.geo, m.geo);
    eo += m.N;
    go += m.E;
    bl.eoff.push_back(eo);
  }
  return LXW_OK;
}

lxw_status create_solver(const lxw_mesh* m, const lxw_params* p, void* stream, BatchLayout* bl, lxw_solver** out) {
  if (!p || !out) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  lxw_status s = check_params(p);
  if (s) return s;
  if ((s = ensure_init())) return s;
  std::unique_ptr<lxw_mesh> own;
  if (p->degree == 3) {
    if (bl) return fail(LXW_ERR_UNSUPPORTED, "degree 3 is for single-mesh solvers");
    if (m->kind == LXW_QUAD || m->kind == LXW_TET) return fail(LXW_ERR_UNSUPPORTED, "degree 3 is for line and triangle meshes");
    // the solver's own copy of the mesh at degree 3 (more modes; the geometry is the same)
    own.reset(new (std::nothrow) lxw_mesh(*m));
    if (!own) return fail(LXW_ERR_OOM, "host allocation");
    own->deg = 3;
    own->ML = m->kind == LXW_LINE ? ElLine3::ML : ElTri3::ML;
    m = own.get();
  }
  {
    // device arrays are indexed with 32-bit integers: the largest per-element array has V*ML
    // columns of N entries, the largest per-edge array 3*V columns of E entries
    const int64_t nqe = nqe_of(*m);
    if ((int64_t)m->V * m->ML * m->N > INT32_MAX || 2 * nqe * m->V * (int64_t)m->E > INT32_MAX)
      return fail(LXW_ERR_ARG, "mesh too large for one solver (32-bit device indices)");
  }
  std::unique_ptr<lxw_solver> S(new (std::nothrow) lxw_solver);
  if (!S) return fail(LXW_ERR_OOM, "host allocation");
  S->own_mesh = std::move(own);
  S->M = m;
  S->P = *p;
  S->st = (hipStream_t)stream;
  S->fp32 = p->precision == LXW_FP32_MIXED;
  if (bl) {
    S->batch = true;
    S->n_mesh = (int)bl->geo.size();
    S->eoff = std::move(bl->eoff);
    S->mesh_of = std::move(bl->mesh_of);
    S->e_mesh = std::move(bl->e_mesh);
    S->geo_m = std::move(bl->geo);
  } else {
    S->eoff = {0, m->N};
    S->geo_m = {m->geo};
  }
  if ((s = S->alloc(&S->sc, S->n_mesh))) return s;
  if ((s = S->alloc(&S->err, 1))) return s;
  for (int b = 0; b < S->n_mesh; ++b)
    if ((s = reset_scalars(S.get(), b, 0.0))) return s;
  DevError ze{};
  HIPCHK(hipMemcpy(S->err, &ze, sizeof ze, hipMemcpyHostToDevice));
  if (S->fp32) s = setup_view<float>(S.get(), S->vf);
  else s = setup_view<double>(S.get(), S->vd);
  if (s) return s;
  *out = S.release();
  return LXW_OK;
}

// Sets the end time on the device if it differs from the one last set (stream-ordered).
lxw_status set_end_time(lxw_solver* S, double T) {
  if (S->t_end == T) return LXW_OK;
  HIPCHK(launch_set_end(S->sc, S->n_mesh, T, S->st));
  S->t_end = T;
  return LXW_OK;
}

// Steps of a batch by the persistent kernel, at most 1024 per cooperative launch.
template <class E, class R>
lxw_status persistent_steps_t(lxw_solver* S, const View<R>& v, int64_t n_steps) {
  for (int64_t k = 0; k < n_steps; k += 1024)
    HIPCHK((launch_persistent<E, R>(v, S->cfg.persistent, S->st, S->n_mesh, (int)std::min<int64_t>(1024, n_steps - k))));
  return LXW_OK;
}

lxw_status persistent_steps(lxw_solver* S, int64_t n_steps) {
  if (S->M->deg != 2) return fail(LXW_ERR_UNSUPPORTED, "the persistent kernel is for degree-2 batches");
  switch (S->M->kind) {
    case LXW_LINE: return S->fp32 ? persistent_steps_t<ElLine, float>(S, S->vf, n_steps) : persistent_steps_t<ElLine, double>(S, S->vd, n_steps);
    case LXW_QUAD: return S->fp32 ? persistent_steps_t<ElQuad, float>(S, S->vf, n_steps) : persistent_steps_t<ElQuad, double>(S, S->vd, n_steps);
    default: return S->fp32 ? persistent_steps_t<ElTri, float>(S, S->vf, n_steps) : persistent_steps_t<ElTri, double>(S, S->vd, n_steps);
  }
}

// Enqueues n steps: the persistent kernel (a batch with that launch shape), replays of the captured
// step graph, or eager launches while timing, stage read-out or graphs are off.
lxw_status replay_steps(lxw_solver* S, int64_t n_steps) {
  if (S->batch && S->cfg.persistent && !S->timing && !S->debug && !S->ind) return persistent_steps(S, n_steps);
  if (S->timing || S->debug || !S->use_graph) {
    for (int64_t k = 0; k < n_steps; ++k) {
      lxw_status s = enqueue_step(S);
      if (s) return s;
    }
    return LXW_OK;
  }
  if (!S->gexec) {
    lxw_status s = capture_step(S);
    if (s) return s;
  }
  for (int64_t k = 0; k < n_steps; ++k) HIPCHK(hipGraphLaunch(S->gexec, S->st));
  return LXW_OK;
}

lxw_status run_steps_impl(lxw_solver* S, int64_t n_steps) {
  if (n_steps < 0) return fail(LXW_ERR_ARG, "negative step count");
  if (n_steps == 0) return LXW_OK;
  lxw_status s = set_end_time(S, std::numeric_limits<double>::infinity());
  if (s) return s;
  return replay_steps(S, n_steps);
}

// ---- learned indicator: host helpers ---------------------------------------------------------

uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

// Pack the master parameters into the inference kernel's lane layout (see lxw_indicator.hip).
lxw_status ind_pack(lxw_indicator* I) {
  std::vector<float> th(IND_NPARAM);
  HIPCHK(hipStreamSynchronize(I->st));
  HIPCHK(hipMemcpy(th.data(), I->theta, IND_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  const float* W1 = &th[IND_OFF_W1];
  const float* W2 = &th[IND_OFF_W2];
  std::vector<uint16_t> A1(2 * 3 * 64 * 8), A2(2 * 4 * 64 * 8);
  for (int mt = 0; mt < 2; ++mt)
    for (int st = 0; st < 3; ++st)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int k = 16 * st + 8 * (l / 32) + e, m = 32 * mt + l % 32;
          A1[((mt * 3 + st) * 64 + l) * 8 + e] = bf16_bits(W1[k * IND_NH + m]);
        }
  for (int mt2 = 0; mt2 < 2; ++mt2)
    for (int mt = 0; mt < 2; ++mt)
      for (int g = 0; g < 2; ++g)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int kin = 32 * mt + 8 * (2 * g + e / 4) + 4 * (l / 32) + e % 4, mout = 32 * mt2 + l % 32;
            A2[((mt2 * 4 + mt * 2 + g) * 64 + l) * 8 + e] = bf16_bits(W2[kin * IND_NH + mout]);
          }
  std::vector<float> b1p(64), b2p(64), w3p(65);
  for (int mt = 0; mt < 2; ++mt)
    for (int h = 0; h < 2; ++h)
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * mt + 8 * (r / 4) + 4 * h + r % 4;
        b1p[(mt * 2 + h) * 16 + r] = th[IND_OFF_B1 + m];
        b2p[(mt * 2 + h) * 16 + r] = th[IND_OFF_B2 + m];
        w3p[(mt * 2 + h) * 16 + r] = th[IND_OFF_W3 + m];
      }
  w3p[64] = th[IND_OFF_B3];
  HIPCHK(hipMemcpy(I->A1, A1.data(), A1.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->A2, A2.data(), A2.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->b1p, b1p.data(), 64 * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->b2p, b2p.data(), 64 * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->w3p, w3p.data(), 65 * 4, hipMemcpyHostToDevice));
  return LXW_OK;
}

template <class T>
lxw_status ind_alloc(lxw_indicator* I, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (n ? n : 1) * sizeof(T));
  if (e != hipSuccess) return fail(LXW_ERR_OOM, "indicator allocation");
  I->bufs.push_back(q);
  *p = (T*)q;
  return LXW_OK;
}

lxw_status ind_part(lxw_indicator* I, int nblk) {
  if (nblk <= I->part_blocks) return LXW_OK;
  lxw_status s = ind_alloc(I, &I->part, (size_t)nblk * IND_PART);
  if (s) return s;
  I->part_blocks = nblk;
  return LXW_OK;
}

lxw_status ind_set_theta(lxw_indicator* I, const float* p) {
  for (int j = 0; j < IND_NPARAM; ++j)
    if (!std::isfinite(p[j])) return fail(LXW_ERR_ARG, "non-finite indicator parameter " + std::to_string(j));
  std::vector<float> z(IND_NPARAM, 0.0f);
  HIPCHK(hipStreamSynchronize(I->st));
  HIPCHK(hipMemcpy(I->theta, p, IND_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->m, z.data(), IND_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(I->v, z.data(), IND_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  I->t = 0;
  return ind_pack(I);
}

template <class E, class R>
lxw_status collect_t(lxw_solver* S, const View<R>& v, float* Xd, double* thd) {
  HIPCHK(launch_features<R>(v, Xd, S->st));
  View<R> w = v;
  w.theta = thd;  // k_pre mode 2 stores the factor there
  HIPCHK((launch<E, R>(K_SHOCK, w, S->cfg, S->st, S->n_mesh, 2)));
  HIPCHK(hipStreamSynchronize(S->st));
  return LXW_OK;
}

lxw_status check_solver(lxw_solver* s) {
  if (!s) return fail(LXW_ERR_ARG, "null solver");
  return LXW_OK;
}

}  // namespace

// =============================================================================================
// C interface
// =============================================================================================
extern "C" {

lxw_status lxw_params_default(lxw_params* p) {
  if (!p) return fail(LXW_ERR_ARG, "null params");
  p->gamma = 1.4;
  p->degree = 2;
  p->cfl = 0.08;
  p->eps0 = 1e-12;
  p->alpha0 = 500.0;
  p->precision = LXW_FP64;
  p->shock = LXW_SHOCK_PLAIN;
  p->theta_exact = 0;
  p->wave_speed = LXW_SPEED_POINTS;
  p->inflow[0] = 1.0; p->inflow[1] = 0.0; p->inflow[2] = 0.0; p->inflow[3] = 2.5;
  return LXW_OK;
}

const char* lxw_last_error(void) { return g_err.c_str(); }

lxw_status lxw_mesh_create_1d(int32_t n, double x0, double x1, int32_t bcl, int32_t bcr, lxw_mesh** out) {
  if (!out) return fail(LXW_ERR_ARG, "null output");
  *out = nullptr;
  if (n < 2 || !(x1 > x0)) return fail(LXW_ERR_ARG, "need n >= 2 and x1 > x0");
  if (bcl < 0 || bcl > 3 || bcr < 0 || bcr > 3) return fail(LXW_ERR_ARG, "bad boundary code");
  if ((bcl == LXW_BC_PERIODIC) != (bcr == LXW_BC_PERIODIC)) return fail(LXW_ERR_ARG, "periodic must be set on both ends");
  std::unique_ptr<lxw_mesh> M(new (std::nothrow) lxw_mesh);
  if (!M) return fail(LXW_ERR_OOM, "host allocation");
  M->kind = LXW_LINE; M->dim = 1; M->N = n; M->K = 2; M->V = 3; M->ML = 3;
  const double h = (x1 - x0) / n;
  std::vector<double> cvx(2 * (size_t)n);
  std::vector<int> nb(2 * (size_t)n, -1), nk(2 * (size_t)n, -1), bc(2 * (size_t)n, -1);
  const bool per = bcl == LXW_BC_PERIODIC;
  for (int i = 0; i < n; ++i) {
    cvx[2 * i] = x0 + i * h;
    cvx[2 * i + 1] = (i == n - 1) ? x1 : x0 + (i + 1) * h;
    if (i > 0 || per) { nb[2 * i] = (i - 1 + n) % n; nk[2 * i] = 1; } else bc[2 * i] = bcl;
    if (i < n - 1 || per) { nb[2 * i + 1] = (i + 1) % n; nk[2 * i + 1] = 0; } else bc[2 * i + 1] = bcr;
  }
  lxw_status s = finish_mesh(M.get(), cvx, nb, nk, bc, 0.0);
  if (s) return s;
  *out = M.release();
  return LXW_OK;
}

lxw_status lxw_mesh_create_cart(int32_t nx, int32_t ny, double x0, double x1, double y0, double y1, const int32_t bc[4],
                                lxw_mesh** out) {
  return lxw_mesh_create_cart_masked(nx, ny, x0, x1, y0, y1, bc, nullptr, LXW_BC_REFLECTIVE, out);
}

lxw_status lxw_mesh_create_cart_masked(int32_t nx, int32_t ny, double x0, double x1, double y0, double y1,
                                       const int32_t bc[4], const uint8_t* keep, int32_t wall_bc, lxw_mesh** out) {
  if (!out || !bc) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  if (nx < 2 || ny < 2 || !(x1 > x0) || !(y1 > y0)) return fail(LXW_ERR_ARG, "need nx, ny >= 2 and a non-empty box");
  if ((int64_t)nx * ny > INT32_MAX) return fail(LXW_ERR_ARG, "too many cells");
  for (int s = 0; s < 4; ++s)
    if (bc[s] < 0 || bc[s] > 3) return fail(LXW_ERR_ARG, "bad boundary code");
  if ((bc[0] == LXW_BC_PERIODIC) != (bc[1] == LXW_BC_PERIODIC) || (bc[2] == LXW_BC_PERIODIC) != (bc[3] == LXW_BC_PERIODIC))
    return fail(LXW_ERR_ARG, "periodic must be set on both sides of a direction");
  if (wall_bc != LXW_BC_REFLECTIVE && wall_bc != LXW_BC_TRANSPARENT && wall_bc != LXW_BC_INFLOW)
    return fail(LXW_ERR_ARG, "wall_bc must be reflective, transparent or inflow");
  // caller index of every kept cell, -1 for a removed one
  std::vector<int> id((size_t)nx * ny, -1);
  int N = 0;
  for (size_t c = 0; c < id.size(); ++c)
    if (!keep || keep[c]) id[c] = N++;
  if (N == 0) return fail(LXW_ERR_ARG, "the mask keeps no cell");
  std::unique_ptr<lxw_mesh> M(new (std::nothrow) lxw_mesh);
  if (!M) return fail(LXW_ERR_OOM, "host allocation");
  M->kind = LXW_QUAD; M->dim = 2; M->N = N; M->K = 4; M->V = 4; M->ML = 9;
  const double hx = (x1 - x0) / nx, hy = (y1 - y0) / ny;
  std::vector<double> cvx((size_t)N * 8);
  std::vector<int> nb((size_t)N * 4, -1), nk((size_t)N * 4, -1), bcv((size_t)N * 4, -1);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int e = id[(size_t)i + (size_t)nx * j];
      if (e < 0) continue;
      const double xa = x0 + i * hx, xb = (i == nx - 1) ? x1 : x0 + (i + 1) * hx;
      const double ya = y0 + j * hy, yb = (j == ny - 1) ? y1 : y0 + (j + 1) * hy;
      const double v[8] = {xa, ya, xb, ya, xb, yb, xa, yb};
      for (int x = 0; x < 8; ++x) cvx[(size_t)e * 8 + x] = v[x];
      struct L { int k, ii, jj, kk, code; } links[4] = {
          {0, i, j - 1, 2, bc[2]}, {1, i + 1, j, 3, bc[1]}, {2, i, j + 1, 0, bc[3]}, {3, i - 1, j, 1, bc[0]}};
      for (auto& l : links) {
        const bool outside = l.ii < 0 || l.ii >= nx || l.jj < 0 || l.jj >= ny;
        if (outside && l.code != LXW_BC_PERIODIC) { bcv[(size_t)e * 4 + l.k] = l.code; continue; }
        const int ii = (l.ii + nx) % nx, jj = (l.jj + ny) % ny;
        const int n = id[(size_t)ii + (size_t)nx * jj];
        if (n < 0) { bcv[(size_t)e * 4 + l.k] = wall_bc; continue; }  // face of a removed cell
        nb[(size_t)e * 4 + l.k] = n;
        nk[(size_t)e * 4 + l.k] = l.kk;
      }
    }
  lxw_status s = finish_mesh(M.get(), cvx, nb, nk, bcv, 0.0);
  if (s) return s;
  *out = M.release();
  return LXW_OK;
}

lxw_status lxw_mesh_create_tri(int32_t n_nodes, const double* xy, int32_t n_tri, const int32_t* tri,
                               const int32_t* bnd_tag, const double* period, lxw_mesh** out) {
  if (!out || !xy || !tri) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  if (n_nodes < 3 || n_tri < 1) return fail(LXW_ERR_ARG, "need at least one triangle");
  std::unique_ptr<lxw_mesh> M(new (std::nothrow) lxw_mesh);
  if (!M) return fail(LXW_ERR_OOM, "host allocation");
  const int N = n_tri;
  M->kind = LXW_TRI; M->dim = 2; M->N = N; M->K = 3; M->V = 4; M->ML = 6;
  std::vector<double> cvx((size_t)N * 6);
  for (int t = 0; t < N; ++t)
    for (int a = 0; a < 3; ++a) {
      const int v = tri[3 * t + a];
      if (v < 0 || v >= n_nodes) return fail(LXW_ERR_ARG, "node index out of range in triangle " + std::to_string(t));
      cvx[(size_t)t * 6 + 2 * a] = xy[2 * v];
      cvx[(size_t)t * 6 + 2 * a + 1] = xy[2 * v + 1];
    }
  std::vector<int> nb((size_t)N * 3, -1), nk((size_t)N * 3, -1), bcv((size_t)N * 3, -1);
  std::unordered_map<uint64_t, int64_t> open;  // vertex pair -> t*3+k
  open.reserve((size_t)N * 2);
  for (int t = 0; t < N; ++t)
    for (int k = 0; k < 3; ++k) {
      const uint32_t a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      const uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
      auto it = open.find(key);
      if (it == open.end()) {
        open.emplace(key, (int64_t)t * 3 + k);
      } else {
        if (it->second < 0) return fail(LXW_ERR_MESH, "an edge is shared by more than two triangles");
        const int t2 = (int)(it->second / 3), k2 = (int)(it->second % 3);
        nb[(size_t)t * 3 + k] = t2; nk[(size_t)t * 3 + k] = k2;
        nb[(size_t)t2 * 3 + k2] = t; nk[(size_t)t2 * 3 + k2] = k;
        it->second = -1;
      }
    }
  // boundary edges and periodic pairing by midpoint modulo the period
  std::map<std::pair<int64_t, int64_t>, int64_t> pmap;
  for (auto& kv : open) {
    if (kv.second < 0) continue;
    const int t = (int)(kv.second / 3), k = (int)(kv.second % 3);
    const int code = bnd_tag ? bnd_tag[3 * t + k] : LXW_BC_TRANSPARENT;
    if (code < 0 || code > 3) return fail(LXW_ERR_ARG, "bad boundary code on triangle " + std::to_string(t));
    if (code != LXW_BC_PERIODIC) { bcv[(size_t)t * 3 + k] = code; continue; }
    if (!period) return fail(LXW_ERR_ARG, "periodic edges need a period");
    const double* v = &cvx[(size_t)t * 6];
    const int b = (k + 1) % 3;
    double m[2] = {0.5 * (v[2 * k] + v[2 * b]), 0.5 * (v[2 * k + 1] + v[2 * b + 1])};
    int64_t q[2];
    for (int d = 0; d < 2; ++d) {
      const double L = period[d];
      const int64_t Q = 1ll << 24;
      if (L > 0) {
        int64_t x = (int64_t)std::llround(m[d] / L * (double)Q);
        q[d] = ((x % Q) + Q) % Q;
      } else {
        q[d] = (int64_t)std::llround(m[d] * 1e9);
      }
    }
    auto key = std::make_pair(q[0], q[1]);
    auto it = pmap.find(key);
    if (it == pmap.end()) {
      pmap.emplace(key, (int64_t)t * 3 + k);
    } else {
      const int t2 = (int)(it->second / 3), k2 = (int)(it->second % 3);
      nb[(size_t)t * 3 + k] = t2; nk[(size_t)t * 3 + k] = k2;
      nb[(size_t)t2 * 3 + k2] = t; nk[(size_t)t2 * 3 + k2] = k;
      pmap.erase(it);
    }
  }
  if (!pmap.empty()) return fail(LXW_ERR_MESH, "unpaired periodic edge");
  lxw_status s = finish_mesh(M.get(), cvx, nb, nk, bcv, 0.0);
  if (s) return s;
  *out = M.release();
  return LXW_OK;
}

lxw_status lxw_mesh_create_tet(int32_t n_nodes, const double* xyz, int32_t n_tet, const int32_t* tet,
                               const int32_t* bnd_tag, const double* period, lxw_mesh** out) {
  if (!out || !xyz || !tet) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  if (n_nodes < 4 || n_tet < 1) return fail(LXW_ERR_ARG, "need at least one tetrahedron");
  std::unique_ptr<lxw_mesh> M(new (std::nothrow) lxw_mesh);
  if (!M) return fail(LXW_ERR_OOM, "host allocation");
  const int N = n_tet;
  M->kind = LXW_TET; M->dim = 3; M->N = N; M->K = 4; M->V = 5; M->ML = 10;
  std::vector<double> cvx((size_t)N * 12);
  for (int t = 0; t < N; ++t)
    for (int a = 0; a < 4; ++a) {
      const int v = tet[4 * t + a];
      if (v < 0 || v >= n_nodes) return fail(LXW_ERR_ARG, "node index out of range in tetrahedron " + std::to_string(t));
      for (int d = 0; d < 3; ++d) cvx[(size_t)t * 12 + 3 * a + d] = xyz[3 * (size_t)v + d];
    }
  std::vector<int> nb((size_t)N * 4, -1), nk((size_t)N * 4, -1), bcv((size_t)N * 4, -1);
  std::vector<unsigned char> sig((size_t)N * 4, 0);
  auto face_nodes = [&](int t, int k, int* f) { for (int m = 0; m < 3; ++m) f[m] = tet[4 * t + TET_FACE[k][m]]; };
  // sigma[m] = the partner's face vertex equal to this face's vertex m
  auto perm_index = [](const int* sigma) {
    for (int p = 0; p < 6; ++p)
      if (PERM3[p][0] == sigma[0] && PERM3[p][1] == sigma[1] && PERM3[p][2] == sigma[2]) return p;
    return -1;
  };
  auto link = [&](int t, int k, int t2, int k2, const int* sig_t) {
    nb[(size_t)t * 4 + k] = t2; nk[(size_t)t * 4 + k] = k2;
    nb[(size_t)t2 * 4 + k2] = t; nk[(size_t)t2 * 4 + k2] = k;
    int inv[3];
    for (int m = 0; m < 3; ++m) inv[sig_t[m]] = m;
    sig[(size_t)t * 4 + k] = (unsigned char)perm_index(sig_t);
    sig[(size_t)t2 * 4 + k2] = (unsigned char)perm_index(inv);
  };
  // interior faces: the sorted node triple
  std::vector<std::tuple<int, int, int, int>> faces;  // (a, b, c, t*4 + k), a < b < c
  faces.reserve((size_t)N * 4);
  for (int t = 0; t < N; ++t)
    for (int k = 0; k < 4; ++k) {
      int f[3];
      face_nodes(t, k, f);
      std::sort(f, f + 3);
      faces.emplace_back(f[0], f[1], f[2], t * 4 + k);
    }
  std::sort(faces.begin(), faces.end());
  std::vector<int> open;
  for (size_t x = 0; x < faces.size();) {
    size_t y = x + 1;
    while (y < faces.size() && std::get<0>(faces[y]) == std::get<0>(faces[x]) && std::get<1>(faces[y]) == std::get<1>(faces[x]) &&
           std::get<2>(faces[y]) == std::get<2>(faces[x]))
      ++y;
    if (y - x > 2) return fail(LXW_ERR_MESH, "a face is shared by more than two tetrahedra");
    if (y - x == 2) {
      const int a = std::get<3>(faces[x]), b = std::get<3>(faces[x + 1]);
      int fa[3], fb[3], sg[3];
      face_nodes(a / 4, a % 4, fa);
      face_nodes(b / 4, b % 4, fb);
      for (int m = 0; m < 3; ++m) sg[m] = (int)(std::find(fb, fb + 3, fa[m]) - fb);
      link(a / 4, a % 4, b / 4, b % 4, sg);
    } else {
      open.push_back(std::get<3>(faces[x]));
    }
    x = y;
  }
  // boundary faces; periodic faces paired by their centroid modulo the period
  std::map<std::tuple<int64_t, int64_t, int64_t>, int> pmap;
  for (int tk : open) {
    const int t = tk / 4, k = tk % 4;
    const int code = bnd_tag ? bnd_tag[4 * t + k] : LXW_BC_TRANSPARENT;
    if (code < 0 || code > 3) return fail(LXW_ERR_ARG, "bad boundary code on tetrahedron " + std::to_string(t));
    if (code == LXW_BC_INFLOW) return fail(LXW_ERR_UNSUPPORTED, "inflow sides are not supported on tetrahedra");
    if (code != LXW_BC_PERIODIC) { bcv[(size_t)t * 4 + k] = code; continue; }
    if (!period) return fail(LXW_ERR_ARG, "periodic faces need a period");
    const double* v = &cvx[(size_t)t * 12];
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = (v[3 * TET_FACE[k][0] + d] + v[3 * TET_FACE[k][1] + d] + v[3 * TET_FACE[k][2] + d]) / 3.0;
    int64_t q[3];
    for (int d = 0; d < 3; ++d) {
      const double L = period[d];
      const int64_t Q = 1ll << 24;
      if (L > 0) {
        int64_t x = (int64_t)std::llround(c[d] / L * (double)Q);
        q[d] = ((x % Q) + Q) % Q;
      } else {
        q[d] = (int64_t)std::llround(c[d] * 1e9);
      }
    }
    auto key = std::make_tuple(q[0], q[1], q[2]);
    auto it = pmap.find(key);
    if (it == pmap.end()) {
      pmap.emplace(key, tk);
    } else {
      const int t2 = it->second / 4, k2 = it->second % 4;
      // vertices matched by position after removing the shift between the two faces
      const double* v2 = &cvx[(size_t)t2 * 12];
      double c2[3];
      for (int d = 0; d < 3; ++d) c2[d] = (v2[3 * TET_FACE[k2][0] + d] + v2[3 * TET_FACE[k2][1] + d] + v2[3 * TET_FACE[k2][2] + d]) / 3.0;
      int sg[3];
      for (int m = 0; m < 3; ++m) {
        double best = 1e300;
        sg[m] = -1;
        for (int m2 = 0; m2 < 3; ++m2) {
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            const double dd = (v[3 * TET_FACE[k][m] + d] - c[d]) - (v2[3 * TET_FACE[k2][m2] + d] - c2[d]);
            d2 += dd * dd;
          }
          if (d2 < best) { best = d2; sg[m] = m2; }
        }
      }
      if (perm_index(sg) < 0) return fail(LXW_ERR_MESH, "periodic faces whose vertices do not match");
      link(t, k, t2, k2, sg);
      pmap.erase(it);
    }
  }
  if (!pmap.empty()) return fail(LXW_ERR_MESH, "unpaired periodic face");
  lxw_status s = finish_mesh(M.get(), cvx, nb, nk, bcv, 0.0, &sig);
  if (s) return s;
  *out = M.release();
  return LXW_OK;
}

lxw_status lxw_mesh_destroy(lxw_mesh* m) {
  delete m;
  return LXW_OK;
}

lxw_status lxw_mesh_get_info(const lxw_mesh* m, lxw_mesh_info* out) {
  if (!m || !out) return fail(LXW_ERR_ARG, "null argument");
  out->kind = m->kind; out->dim = m->dim; out->n_elem = m->N; out->n_edge = m->E;
  out->n_var = m->V; out->n_modes = m->ML; out->n_faces = m->K;
  out->min_area = m->N ? *std::min_element(m->area.begin(), m->area.end()) : 0.0;
  out->max_area = m->N ? *std::max_element(m->area.begin(), m->area.end()) : 0.0;
  return LXW_OK;
}

lxw_status lxw_refelem_info_deg(int32_t kind, int32_t degree, int32_t* n_pts, double* xi, double* w, double* phi) {
  if (kind < 0 || kind > 3 || !n_pts) return fail(LXW_ERR_ARG, "bad kind or null n_pts");
  if (degree != 2 && (degree != 3 || kind == LXW_QUAD || kind == LXW_TET))
    return fail(LXW_ERR_UNSUPPORTED, "degree 2, or 3 on lines and triangles");
  Rule r = degree == 3 ? (kind == LXW_LINE ? rule_line4() : rule_tri16())
                       : (kind == LXW_LINE ? rule_line()
                                           : (kind == LXW_QUAD ? rule_quad() : (kind == LXW_TET ? rule_tet27() : rule_tri())));
  const int dim = kind == LXW_LINE ? 1 : (kind == LXW_TET ? 3 : 2);
  const int ML = degree == 3 ? (kind == LXW_LINE ? 4 : 10)
                             : (kind == LXW_LINE ? 3 : (kind == LXW_QUAD ? 9 : (kind == LXW_TET ? 10 : 6)));
  const int n = (int)r.w.size();
  *n_pts = n;
  if (xi) for (int x = 0; x < n * dim; ++x) xi[x] = r.x[x];
  if (w) for (int m = 0; m < n; ++m) w[m] = r.w[m];
  if (phi)
    for (int m = 0; m < n; ++m) {
      double p[3] = {r.x[m * dim], dim >= 2 ? r.x[m * dim + 1] : 0.0, dim == 3 ? r.x[m * dim + 2] : 0.0};
      for (int l = 0; l < ML; ++l) phi[m * ML + l] = basis(kind, degree, l, p, 0, 0);
    }
  return LXW_OK;
}

lxw_status lxw_refelem_info(int32_t kind, int32_t* n_pts, double* xi, double* w, double* phi) {
  return lxw_refelem_info_deg(kind, 2, n_pts, xi, w, phi);
}

lxw_status lxw_solver_create(const lxw_mesh* m, const lxw_params* p, void* stream, lxw_solver** out) {
  if (!m) return fail(LXW_ERR_ARG, "null argument");
  return create_solver(m, p, stream, nullptr, out);
}

lxw_status lxw_solver_destroy(lxw_solver* s) {
  if (s) (void)hipStreamSynchronize(s->st);
  delete s;
  return LXW_OK;
}

lxw_status lxw_set_state(lxw_solver* S, const double* Q, double t0, int32_t flags) {
  if (check_solver(S) || !Q) return fail(LXW_ERR_ARG, "null argument");
  if (S->batch) return fail(LXW_ERR_UNSUPPORTED, "a batch's state is set per mesh (lxw_batch_set_state)");
  lxw_status s = load_state(S, *S->M, 0, Q, flags);
  if (s) return s;
  if ((s = reset_scalars(S, 0, t0))) return s;
  DevError ze{};
  HIPCHK(hipMemcpy(S->err, &ze, sizeof ze, hipMemcpyHostToDevice));
  return LXW_OK;
}

lxw_status lxw_get_state(lxw_solver* S, double* Q, double* t, int32_t flags) {
  if (check_solver(S) || !Q) return fail(LXW_ERR_ARG, "null argument");
  if (S->batch) return fail(LXW_ERR_UNSUPPORTED, "a batch's state is read per mesh (lxw_batch_get_state)");
  lxw_status s = sync_check(S);
  if (s) return s;
  if (S->hsc.shock_pending && S->P.shock) {
    if ((s = enqueue_shock(S))) return s;
    if ((s = sync_check(S))) return s;
  }
  std::vector<double> h;
  if ((s = store_state(S, *S->M, 0, false, h))) return s;
  if (flags & LXW_DEVICE_PTR) {
    HIPCHK(hipMemcpyAsync(Q, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
  } else {
    std::memcpy(Q, h.data(), h.size() * sizeof(double));
  }
  if (t) *t = S->hsc.t;
  return LXW_OK;
}

lxw_status lxw_step(lxw_solver* S, double T, double* dt_taken) {
  if (check_solver(S)) return LXW_ERR_ARG;
  if (S->batch) return fail(LXW_ERR_UNSUPPORTED, "a batch advances by step counts (lxw_batch_advance_steps)");
  if (!(S->hsc.t < T)) return fail(LXW_ERR_ARG, "t >= T");
  lxw_status s = set_end_time(S, T);
  if (!s) s = enqueue_step(S);
  if (s) return s;
  s = sync_check(S);
  if (dt_taken) *dt_taken = S->hsc.dt;
  return s;
}

lxw_status lxw_advance(lxw_solver* S, double T, int64_t max_steps, lxw_stats* out) {
  if (check_solver(S)) return LXW_ERR_ARG;
  if (S->batch) return fail(LXW_ERR_UNSUPPORTED, "a batch advances by step counts (lxw_batch_advance_steps)");
  // Steps in chunks (graph replays) with one synchronisation per chunk: the end time sits on
  // the device, every step is clipped to it and a step at t = T changes nothing, so a chunk may
  // run past T.  Chunks grow to 256 steps and shrink to the number the last dt predicts.
  const int64_t steps0 = S->hsc.steps;
  int64_t n = 0, chunk = 1;
  lxw_status s = set_end_time(S, T);
  while (!s && S->hsc.t < T && n < max_steps) {
    int64_t k = std::min(chunk, max_steps - n);
    if (S->hsc.dt > 0.0) {
      const double est = std::ceil((T - S->hsc.t) / S->hsc.dt);
      if (est >= 1.0 && est < (double)k) k = (int64_t)est;
    }
    s = replay_steps(S, k);
    if (!s) s = sync_check(S);
    n = S->hsc.steps - steps0;
    chunk = std::min<int64_t>(2 * chunk, 256);
  }
  if (out) { out->steps = n; out->t = S->hsc.t; out->last_dt = S->hsc.dt; out->last_s = S->hsc.s; }
  return s;
}

lxw_status lxw_run_steps(lxw_solver* S, int64_t n_steps) {
  if (check_solver(S)) return LXW_ERR_ARG;
  return run_steps_impl(S, n_steps);
}

lxw_status lxw_set_graph(lxw_solver* S, int32_t enable) {
  if (check_solver(S)) return LXW_ERR_ARG;
  S->use_graph = enable != 0;
  return LXW_OK;
}

lxw_status lxw_sync(lxw_solver* S) {
  if (check_solver(S)) return LXW_ERR_ARG;
  return sync_check(S);
}

lxw_status lxw_set_debug(lxw_solver* S, int32_t keep) {
  if (check_solver(S)) return LXW_ERR_ARG;
  if (S->batch) return fail(LXW_ERR_UNSUPPORTED, "stage read-out is for single meshes");
  S->debug = keep != 0;
  if (!S->debug) return LXW_OK;
  const lxw_mesh& M = *S->M;
  const int N = M.N, V = M.V, ML = M.ML, K = M.K;
  if (!S->dq_upd_bar) {
    lxw_status s;
    const size_t rs = S->fp32 ? sizeof(float) : sizeof(double);
    if ((s = S->alloc(&S->dq_upd_bar, (size_t)V * N))) return s;
    char* p2 = nullptr;
    if ((s = S->alloc(&p2, (size_t)V * (ML - 1) * N * rs))) return s;
    S->dq_upd_h = p2;
    double *a, *b, *c, *d, *q;
    if ((s = S->alloc(&q, (size_t)V * ML * N))) return s;
    if ((s = S->alloc(&a, N))) return s;
    if ((s = S->alloc(&b, N))) return s;
    if ((s = S->alloc(&c, (size_t)V * ML * N))) return s;
    if ((s = S->alloc(&d, (size_t)K * N))) return s;
    std::vector<double> ones(N, 1.0);
    HIPCHK(hipMemcpy(b, ones.data(), N * sizeof(double), hipMemcpyHostToDevice));
    auto set = [&](auto& v) { v.dbg_theta = a; v.dbg_theta_sc = b; v.dbg_vol = c; v.dbg_lame = d; v.dbg_qlim = q; };
    set(S->vd);
    set(S->vf);
  }
  return LXW_OK;
}

lxw_status lxw_debug_stage(lxw_solver* S, int32_t stage, double* out) {
  if (check_solver(S) || !out) return fail(LXW_ERR_ARG, "null argument");
  if (!S->debug || !S->dq_upd_bar) return fail(LXW_ERR_ARG, "stages are kept only after lxw_set_debug(s, 1)");
  lxw_status s = sync_check(S);
  if (s) return s;
  const lxw_mesh& M = *S->M;
  const int N = M.N, V = M.V, ML = M.ML, K = M.K, E = M.E;
  auto dget = [&](const double* src, size_t n, std::vector<double>& h) -> lxw_status {
    h.resize(n);
    HIPCHK(hipMemcpy(h.data(), src, n * sizeof(double), hipMemcpyDeviceToHost));
    return LXW_OK;
  };
  std::vector<double> h;
  const double* vol = S->fp32 ? S->vf.dbg_vol : S->vd.dbg_vol;
  switch (stage) {
    case LXW_STAGE_QLIM: {
      if ((s = dget(S->fp32 ? S->vf.dbg_qlim : S->vd.dbg_qlim, (size_t)V * ML * N, h))) return s;
      for (int i = 0; i < N; ++i)
        for (int v = 0; v < V; ++v)
          for (int l = 0; l < ML; ++l) out[((size_t)M.perm[i] * V + v) * ML + l] = h[((size_t)v * ML + l) * N + i];
      return LXW_OK;
    }
    case LXW_STAGE_QUPD: {
      std::vector<double> qbar((size_t)V * N), qh((size_t)V * (ML - 1) * N);
      HIPCHK(hipMemcpy(qbar.data(), S->dq_upd_bar, qbar.size() * sizeof(double), hipMemcpyDeviceToHost));
      const void* src = S->dq_upd_h;
      if (S->fp32) {
        std::vector<float> f(qh.size());
        HIPCHK(hipMemcpy(f.data(), src, f.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t x = 0; x < f.size(); ++x) qh[x] = f[x];
      } else {
        HIPCHK(hipMemcpy(qh.data(), src, qh.size() * sizeof(double), hipMemcpyDeviceToHost));
      }
      for (int i = 0; i < N; ++i) {
        double* q = &out[(size_t)M.perm[i] * V * ML];
        for (int v = 0; v < V; ++v) {
          q[v * ML] = qbar[(size_t)i * V + v];
          for (int l = 1; l < ML; ++l) q[v * ML + l] = qh[((size_t)v * (ML - 1) + l - 1) * N + i];
        }
      }
      return LXW_OK;
    }
    case LXW_STAGE_THETA:
    case LXW_STAGE_THETA_SC: {
      if ((s = dget(stage == LXW_STAGE_THETA ? S->vd.dbg_theta ? S->vd.dbg_theta : S->vf.dbg_theta
                                             : (S->vd.dbg_theta_sc ? S->vd.dbg_theta_sc : S->vf.dbg_theta_sc),
                    N, h))) return s;
      for (int i = 0; i < N; ++i) out[M.perm[i]] = h[i];
      return LXW_OK;
    }
    case LXW_STAGE_VOL: {
      if ((s = dget(vol, (size_t)V * ML * N, h))) return s;
      for (int i = 0; i < N; ++i)
        for (int v = 0; v < V; ++v)
          for (int l = 0; l < ML; ++l) out[((size_t)M.perm[i] * V + v) * ML + l] = h[((size_t)v * ML + l) * N + i];
      return LXW_OK;
    }
    case LXW_STAGE_FLXW:
    case LXW_STAGE_FLXF: {
      const bool w = stage == LXW_STAGE_FLXW;
      if ((s = dget(S->fp32 ? (w ? S->vf.fLxW : S->vf.fLxF) : (w ? S->vd.fLxW : S->vd.fLxF), (size_t)V * E, h))) return s;
      for (int i = 0; i < N; ++i)
        for (int k = 0; k < K; ++k) {
          const int slot = M.eslot[(size_t)i * K + k];
          const int e = slot >> 3;
          const double ep = ((slot >> 2) & 1) ? -1.0 : 1.0;
          for (int v = 0; v < V; ++v) out[((size_t)M.perm[i] * K + k) * V + v] = ep * h[(size_t)e * V + v];
        }
      return LXW_OK;
    }
    case LXW_STAGE_C: {
      if ((s = dget(S->fp32 ? S->vf.cedge : S->vd.cedge, (size_t)2 * E, h))) return s;
      for (int i = 0; i < N; ++i)
        for (int k = 0; k < K; ++k) {
          const int slot = M.eslot[(size_t)i * K + k];
          out[(size_t)M.perm[i] * K + k] = h[(size_t)(slot >> 3) * 2 + ((slot >> 2) & 1)];
        }
      return LXW_OK;
    }
    case LXW_STAGE_LAME: {
      if ((s = dget(S->fp32 ? S->vf.dbg_lame : S->vd.dbg_lame, (size_t)K * N, h))) return s;
      for (int i = 0; i < N; ++i)
        for (int k = 0; k < K; ++k) out[(size_t)M.perm[i] * K + k] = h[(size_t)k * N + i];
      return LXW_OK;
    }
    case LXW_STAGE_SDT:
      out[0] = S->hsc.s;
      out[1] = S->hsc.dt;
      return LXW_OK;
    default:
      return fail(LXW_ERR_ARG, "unknown stage");
  }
}

lxw_status lxw_set_timing(lxw_solver* S, int32_t enable) {
  if (check_solver(S)) return LXW_ERR_ARG;
  lxw_status s = sync_check(S);
  if (s) return s;
  S->timing = enable != 0;
  for (int k = 0; k < LXW_K_COUNT; ++k) { S->kms[k] = 0.0; S->kcount[k] = 0; }
  return LXW_OK;
}

lxw_status lxw_kernel_times(lxw_solver* S, double* ms, int64_t* launches) {
  if (check_solver(S) || !ms || !launches) return fail(LXW_ERR_ARG, "null argument");
  lxw_status s = sync_check(S);
  if (s) return s;
  for (int k = 0; k < LXW_K_COUNT; ++k) { ms[k] = S->kms[k]; launches[k] = S->kcount[k]; }
  return LXW_OK;
}

// ---- launch shapes and the autotuner --------------------------------------------------------

lxw_status lxw_get_tune(const lxw_solver* S, lxw_tune* out) {
  if (!S || !out) return fail(LXW_ERR_ARG, "null argument");
  for (int k = 0; k < LXW_K_COUNT; ++k) out->block[k] = S->cfg.bs[k];
  out->persistent = S->cfg.persistent;
  return LXW_OK;
}

lxw_status lxw_set_tune(lxw_solver* S, const lxw_tune* t) {
  if (check_solver(S) || !t) return fail(LXW_ERR_ARG, "null argument");
  LaunchCfg c = S->cfg;
  for (int k = 0; k < LXW_K_COUNT; ++k) {
    if (!tunable(k)) continue;
    const int b = t->block[k];
    if (b != 64 && b != 128 && b != 256) return fail(LXW_ERR_ARG, "workgroup sizes must be 64, 128 or 256");
    c.bs[k] = b;
  }
  const int pw = t->persistent;
  if (pw != 0 && pw != 128 && pw != 256) return fail(LXW_ERR_ARG, "persistent must be 0, 128 or 256");
  if (pw && (!S->batch || S->M->kind != LXW_TRI))
    return fail(LXW_ERR_UNSUPPORTED, "the persistent kernel runs batches of triangle meshes only");
  c.persistent = pw;
  lxw_status s = sync_check(S);
  if (s) return s;
  S->cfg = c;
  drop_graph(S);
  return LXW_OK;
}

lxw_status lxw_autotune(lxw_solver* S, int32_t trial_steps, lxw_tune* out) {
  if (check_solver(S)) return LXW_ERR_ARG;
  if (trial_steps < 1) return fail(LXW_ERR_ARG, "trial_steps must be >= 1");
  if (S->debug) return fail(LXW_ERR_ARG, "switch stage read-out off before tuning");
  lxw_status s = sync_check(S);
  if (s) return s;
  const lxw_mesh& M = *S->M;
  const size_t nbar = (size_t)M.V * M.N * sizeof(double);
  const size_t nh = (size_t)M.V * (M.ML - 1) * M.N * (S->fp32 ? sizeof(float) : sizeof(double));
  void* dbar = S->fp32 ? (void*)S->vf.Qbar : (void*)S->vd.Qbar;
  void* dh = S->fp32 ? (void*)S->vf.Qh : (void*)S->vd.Qh;
  // snapshot of the state and the scalars, restored afterwards
  void *sbar = nullptr, *sh = nullptr;
  HIPCHK(hipMalloc(&sbar, nbar ? nbar : 1));
  if (hipMalloc(&sh, nh ? nh : 1) != hipSuccess) { (void)hipFree(sbar); return fail(LXW_ERR_OOM, "tuning snapshot"); }
  std::vector<Scalars> ssc(S->n_mesh);
  auto cleanup = [&]() { (void)hipFree(sbar); (void)hipFree(sh); };
  if (hipMemcpy(sbar, dbar, nbar, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(sh, dh, nh, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(ssc.data(), S->sc, S->n_mesh * sizeof(Scalars), hipMemcpyDeviceToHost) != hipSuccess) {
    cleanup();
    return fail(LXW_ERR_DEVICE, "tuning snapshot copy failed");
  }
  const bool timing0 = S->timing;
  double kms0[LXW_K_COUNT];
  int64_t kc0[LXW_K_COUNT];
  std::memcpy(kms0, S->kms, sizeof kms0);
  std::memcpy(kc0, S->kcount, sizeof kc0);
  S->timing = true;
  LaunchCfg best = S->cfg;
  const int sizes[3] = {64, 128, 256};
  const int order[5] = {K_ELEM, K_PRE, K_EDGE, K_UPDATE, K_FLIM};
  const double inf = std::numeric_limits<double>::infinity();
  for (int k : order) {
    double best_ms = inf;
    int best_bs = best.bs[k];
    for (int bs : sizes) {
      S->cfg = best;
      S->cfg.bs[k] = bs;
      s = enqueue_step(S);  // warm-up with this shape
      if (!s) s = sync_check(S);
      S->kms[k] = 0.0;
      S->kcount[k] = 0;
      for (int t = 0; t < trial_steps && !s; ++t) s = enqueue_step(S);
      if (!s) s = sync_check(S);
      if (s) break;
      const double ms = S->kms[k] / (double)std::max<int64_t>(S->kcount[k], 1);
      if (ms < best_ms) { best_ms = ms; best_bs = bs; }
    }
    if (s) break;
    best.bs[k] = best_bs;
  }
  S->cfg = best;
  if (!s && S->batch && S->M->kind == LXW_TRI && !S->ind) {
    // whole steps: per-phase launches replayed from the graph against the persistent kernel
    S->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) s = fail(LXW_ERR_DEVICE, "tuning events");
    float best_ms = std::numeric_limits<float>::infinity();
    int best_p = 0;
    for (int pw : {0, 128, 256}) {
      if (s) break;
      drop_graph(S);
      S->cfg = best;
      S->cfg.persistent = pw;
      s = replay_steps(S, 1);  // warm-up (captures the graph of the per-phase launches)
      if (!s) s = sync_check(S);
      if (s) {
        if (pw == 0) break;
        s = LXW_OK;  // this launch shape cannot run here (e.g. too few resident workgroups)
        (void)hipGetLastError();
        continue;
      }
      if (hipEventRecord(e0, S->st) != hipSuccess) { s = fail(LXW_ERR_DEVICE, "tuning events"); break; }
      s = replay_steps(S, trial_steps);
      if (!s && hipEventRecord(e1, S->st) != hipSuccess) s = fail(LXW_ERR_DEVICE, "tuning events");
      if (!s) s = sync_check(S);
      float ms = 0.0f;
      if (!s && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(LXW_ERR_DEVICE, "tuning events");
      if (!s && ms < best_ms) { best_ms = ms; best_p = pw; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    best.persistent = best_p;
    S->cfg = best;
  }
  S->timing = timing0;
  std::memcpy(S->kms, kms0, sizeof kms0);
  std::memcpy(S->kcount, kc0, sizeof kc0);
  drop_graph(S);
  (void)hipStreamSynchronize(S->st);
  hipError_t e1 = hipMemcpy(dbar, sbar, nbar, hipMemcpyDeviceToDevice);
  hipError_t e2 = hipMemcpy(dh, sh, nh, hipMemcpyDeviceToDevice);
  hipError_t e3 = hipMemcpy(S->sc, ssc.data(), S->n_mesh * sizeof(Scalars), hipMemcpyHostToDevice);
  cleanup();
  if (s) return s;
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(LXW_ERR_DEVICE, "tuning restore failed");
  S->hscv = ssc;
  S->hsc = ssc[0];
  if (out) {
    for (int k = 0; k < LXW_K_COUNT; ++k) out->block[k] = S->cfg.bs[k];
    out->persistent = S->cfg.persistent;
  }
  return LXW_OK;
}

// ---- batched form -------------------------------------------------------------------------

lxw_status lxw_batch_create(int32_t n, const lxw_mesh* const* meshes, const lxw_params* p, void* stream, lxw_batch** out) {
  if (!meshes || !p || !out) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  if (n < 1) return fail(LXW_ERR_ARG, "a batch needs at least one mesh");
  for (int b = 0; b < n; ++b) {
    if (!meshes[b]) return fail(LXW_ERR_ARG, "null mesh " + std::to_string(b));
    if (meshes[b]->kind != meshes[0]->kind) return fail(LXW_ERR_ARG, "all meshes of a batch must be of one kind");
    if (meshes[b]->kind == LXW_TET) return fail(LXW_ERR_UNSUPPORTED, "batches are for 1D and 2D meshes");
  }
  lxw_status s = check_params(p);
  if (s) return s;
  std::unique_ptr<lxw_batch> B(new (std::nothrow) lxw_batch);
  if (!B) return fail(LXW_ERR_OOM, "host allocation");
  B->ms.assign(meshes, meshes + n);
  BatchLayout bl;
  if ((s = merge_meshes(B->ms, B->merged, bl))) return s;
  if ((s = create_solver(&B->merged, p, stream, &bl, &B->S))) return s;
  *out = B.release();
  return LXW_OK;
}

lxw_status lxw_batch_destroy(lxw_batch* b) {
  if (b && b->S) (void)hipStreamSynchronize(b->S->st);
  delete b;
  return LXW_OK;
}

lxw_solver* lxw_batch_solver(lxw_batch* b) { return b ? b->S : nullptr; }

lxw_status lxw_batch_set_state(lxw_batch* B, int32_t i, const double* Q, double t0, int32_t flags) {
  if (!B || !Q) return fail(LXW_ERR_ARG, "null argument");
  if (i < 0 || i >= (int)B->ms.size()) return fail(LXW_ERR_ARG, "mesh index out of range");
  lxw_solver* S = B->S;
  lxw_status s = sync_check(S);
  if (s) return s;
  if ((s = load_state(S, *B->ms[i], S->eoff[i], Q, flags))) return s;
  return reset_scalars(S, i, t0);
}

lxw_status lxw_batch_get_state(lxw_batch* B, int32_t i, double* Q, double* t, int32_t flags) {
  if (!B || !Q) return fail(LXW_ERR_ARG, "null argument");
  if (i < 0 || i >= (int)B->ms.size()) return fail(LXW_ERR_ARG, "mesh index out of range");
  lxw_solver* S = B->S;
  lxw_status s = sync_check(S);
  if (s) return s;
  bool pending = false;
  for (const Scalars& x : S->hscv) pending = pending || x.shock_pending;
  if (pending && S->P.shock) {
    if ((s = enqueue_shock(S))) return s;
    if ((s = sync_check(S))) return s;
  }
  std::vector<double> h;
  if ((s = store_state(S, *B->ms[i], S->eoff[i], false, h))) return s;
  if (flags & LXW_DEVICE_PTR) {
    HIPCHK(hipMemcpy(Q, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::memcpy(Q, h.data(), h.size() * sizeof(double));
  }
  if (t) *t = S->hscv[i].t;
  return LXW_OK;
}

lxw_status lxw_batch_advance_steps(lxw_batch* B, int64_t n_steps) {
  if (!B) return fail(LXW_ERR_ARG, "null batch");
  return run_steps_impl(B->S, n_steps);
}

lxw_status lxw_batch_stats(lxw_batch* B, int32_t i, lxw_stats* out) {
  if (!B || !out) return fail(LXW_ERR_ARG, "null argument");
  if (i < 0 || i >= (int)B->ms.size()) return fail(LXW_ERR_ARG, "mesh index out of range");
  lxw_status s = sync_check(B->S);
  if (s) return s;
  const Scalars& x = B->S->hscv[i];
  out->steps = x.steps;
  out->t = x.t;
  out->last_dt = x.dt;
  out->last_s = x.s;
  return LXW_OK;
}

// ---- learned troubled-cell indicator --------------------------------------------------------

lxw_status lxw_indicator_create(const float* params, void* stream, lxw_indicator** out) {
  if (!params || !out) return fail(LXW_ERR_ARG, "null argument");
  *out = nullptr;
  lxw_status s = ensure_init();
  if (s) return s;
  std::unique_ptr<lxw_indicator> I(new (std::nothrow) lxw_indicator);
  if (!I) return fail(LXW_ERR_OOM, "host allocation");
  I->st = (hipStream_t)stream;
  if ((s = ind_alloc(I.get(), &I->theta, IND_NPARAM)) || (s = ind_alloc(I.get(), &I->m, IND_NPARAM)) ||
      (s = ind_alloc(I.get(), &I->v, IND_NPARAM)) || (s = ind_alloc(I.get(), &I->A1, 2 * 3 * 64 * 8)) ||
      (s = ind_alloc(I.get(), &I->A2, 2 * 4 * 64 * 8)) || (s = ind_alloc(I.get(), &I->b1p, 64)) ||
      (s = ind_alloc(I.get(), &I->b2p, 64)) || (s = ind_alloc(I.get(), &I->w3p, 65)) ||
      (s = ind_alloc(I.get(), &I->scal, 1)))
    return s;
  if ((s = ind_set_theta(I.get(), params))) return s;
  *out = I.release();
  return LXW_OK;
}

lxw_status lxw_indicator_destroy(lxw_indicator* ind) {
  delete ind;
  return LXW_OK;
}

lxw_status lxw_indicator_get_params(const lxw_indicator* I, float* out) {
  if (!I || !out) return fail(LXW_ERR_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(I->st));
  HIPCHK(hipMemcpy(out, I->theta, IND_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return LXW_OK;
}

lxw_status lxw_indicator_set_params(lxw_indicator* I, const float* p) {
  if (!I || !p) return fail(LXW_ERR_ARG, "null argument");
  return ind_set_theta(I, p);
}

static const char IND_MAGIC[8] = {'L', 'X', 'W', 'I', 'N', 'D', '0', '1'};

lxw_status lxw_indicator_save(const lxw_indicator* I, const char* path) {
  if (!I || !path) return fail(LXW_ERR_ARG, "null argument");
  std::vector<float> th(IND_NPARAM);
  lxw_status s = lxw_indicator_get_params(I, th.data());
  if (s) return s;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(LXW_ERR_ARG, std::string("cannot open ") + path);
  const int32_t n = IND_NPARAM;
  bool ok = std::fwrite(IND_MAGIC, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 &&
            std::fwrite(th.data(), 4, IND_NPARAM, f) == (size_t)IND_NPARAM;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? LXW_OK : fail(LXW_ERR_ARG, std::string("write failed: ") + path);
}

lxw_status lxw_indicator_load(lxw_indicator* I, const char* path) {
  if (!I || !path) return fail(LXW_ERR_ARG, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(LXW_ERR_ARG, std::string("cannot open ") + path);
  char mg[8];
  int32_t n = 0;
  std::vector<float> th(IND_NPARAM);
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, IND_MAGIC, 8) == 0 && std::fread(&n, 4, 1, f) == 1 &&
            n == IND_NPARAM && std::fread(th.data(), 4, IND_NPARAM, f) == (size_t)IND_NPARAM;
  std::fclose(f);
  if (!ok) return fail(LXW_ERR_ARG, std::string("not an indicator parameter file: ") + path);
  return ind_set_theta(I, th.data());
}

lxw_status lxw_indicator_predict(lxw_indicator* I, const float* X, int32_t n, float* p) {
  if (!I || (n > 0 && (!X || !p))) return fail(LXW_ERR_ARG, "null argument");
  if (n < 0) return fail(LXW_ERR_ARG, "negative sample count");
  IndW W{};
  W.A1 = I->A1; W.A2 = I->A2; W.b1 = I->b1p; W.b2 = I->b2p; W.w3 = I->w3p;
  W.tau_lo = 0.0f; W.tau_hi = 1.0f;
  HIPCHK(launch_predict(W, X, n, p, I->st));
  HIPCHK(hipStreamSynchronize(I->st));
  return LXW_OK;
}

lxw_status lxw_indicator_grad(lxw_indicator* I, const float* X, const float* y, int32_t n, double w_pos, double w_neg,
                              float* grad, double* loss) {
  if (!I || !X || !y || !grad) return fail(LXW_ERR_ARG, "null argument");
  if (n < 1) return fail(LXW_ERR_ARG, "need at least one sample");
  const int nblk = mlp_blocks(n);
  lxw_status s = ind_part(I, nblk);
  if (s) return s;
  float* gd = nullptr;
  HIPCHK(hipMalloc(&gd, IND_NPARAM * sizeof(float)));
  TrainArgs a{X, y, nullptr, n, 0, n, (float)w_pos, (float)w_neg, 1.0f / (float)n, I->theta, I->part};
  hipError_t e = launch_mlp_grad(a, I->st);
  if (e == hipSuccess) e = launch_mlp_reduce(nblk, I->part, I->theta, I->m, I->v, gd, I->scal, 0, 0, 0, 0, 0, 1, 1, I->st);
  if (e == hipSuccess) e = hipStreamSynchronize(I->st);
  float lf = 0.0f;
  if (e == hipSuccess) e = hipMemcpy(grad, gd, IND_NPARAM * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&lf, I->scal, sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(gd);
  HIPCHK(e);
  if (loss) *loss = lf;
  return LXW_OK;
}

static_assert(LXW_IND_NOALLOC_MAX == IND_STATIC_MAX_SAMPLES, "public and internal workspace limits differ");

lxw_status lxw_indicator_grad_noalloc(lxw_indicator* I, const float* X, const float* y, int32_t n, double w_pos,
                                      double w_neg, float* grad, float* loss) {
  if (!I || !X || !y || !grad) return fail(LXW_ERR_ARG, "null argument");
  if (n < 1 || n > IND_STATIC_MAX_SAMPLES)
    return fail(LXW_ERR_ARG, "lxw_indicator_grad_noalloc takes 1 to " + std::to_string(IND_STATIC_MAX_SAMPLES) +
                                 " samples, got " + std::to_string(n));
  float* part = nullptr;
  HIPCHK(ind_static_scratch(&part));
  const int nblk = mlp_blocks(n);
  TrainArgs a{X, y, nullptr, n, 0, n, (float)w_pos, (float)w_neg, 1.0f / (float)n, I->theta, part};
  HIPCHK(launch_mlp_grad(a, I->st));
  HIPCHK(launch_mlp_reduce(nblk, part, I->theta, I->m, I->v, grad, loss, 0, 0, 0, 0, 0, 1, 1, I->st));
  return LXW_OK;
}

lxw_status lxw_indicator_train(lxw_indicator* I, const float* X, const float* y, int32_t n_samples,
                               const int32_t* order, int32_t n_updates, int32_t batch, const lxw_adam* hp,
                               double* last_loss) {
  if (!I || !X || !y || !order || !hp) return fail(LXW_ERR_ARG, "null argument");
  if (n_samples < 1 || batch < 1 || n_updates < 0) return fail(LXW_ERR_ARG, "need n_samples >= 1, batch >= 1, n_updates >= 0");
  if (!(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) || !(hp->eps > 0) ||
      !(hp->w_pos > 0) || !(hp->w_neg > 0))
    return fail(LXW_ERR_ARG, "bad Adam or class-weight parameters");
  const int nblk = mlp_blocks(batch);
  lxw_status s = ind_part(I, nblk);
  if (s) return s;
  for (int32_t u = 0; u < n_updates; ++u) {
    TrainArgs a{X, y, order, n_samples, u * batch, batch, (float)hp->w_pos, (float)hp->w_neg, 1.0f / (float)batch,
                I->theta, I->part};
    I->t += 1;
    const double bc1 = 1.0 - std::pow(hp->beta1, (double)I->t), bc2 = 1.0 - std::pow(hp->beta2, (double)I->t);
    HIPCHK(launch_mlp_grad(a, I->st));
    HIPCHK(launch_mlp_reduce(nblk, I->part, I->theta, I->m, I->v, nullptr, I->scal, 1, (float)hp->lr, (float)hp->beta1,
                             (float)hp->beta2, (float)hp->eps, (float)bc1, (float)bc2, I->st));
  }
  HIPCHK(hipStreamSynchronize(I->st));
  if (last_loss) {
    float lf = 0.0f;
    HIPCHK(hipMemcpy(&lf, I->scal, sizeof(float), hipMemcpyDeviceToHost));
    *last_loss = n_updates > 0 ? lf : 0.0;
  }
  return ind_pack(I);
}

lxw_status lxw_indicator_collect(lxw_solver* S, float* X, double* theta_sc, int32_t flags) {
  if (check_solver(S) || !X || !theta_sc) return fail(LXW_ERR_ARG, "null argument");
  if (S->M->kind != LXW_TRI || S->M->deg != 2 || S->batch)
    return fail(LXW_ERR_UNSUPPORTED, "the indicator is for single degree-2 triangle meshes");
  lxw_status s = sync_check(S);
  if (s) return s;
  if (!S->hsc.shock_pending || !S->P.shock)
    return fail(LXW_ERR_ARG, "no shock-capturing limiter pending: take a step first (and read no state in between)");
  const int N = S->M->N;
  float* Xd = nullptr;
  double* td = nullptr;
  HIPCHK(hipMalloc(&Xd, (size_t)N * IND_NIN * sizeof(float)));
  if (hipMalloc(&td, (size_t)(N ? N : 1) * sizeof(double)) != hipSuccess) {
    (void)hipFree(Xd);
    return fail(LXW_ERR_OOM, "collect buffers");
  }
  s = S->fp32 ? collect_t<ElTri, float>(S, S->vf, Xd, td) : collect_t<ElTri, double>(S, S->vd, Xd, td);
  std::vector<float> xh((size_t)N * IND_NIN);
  std::vector<double> th(N);
  hipError_t e = hipSuccess;
  if (!s) e = hipMemcpy(xh.data(), Xd, xh.size() * sizeof(float), hipMemcpyDeviceToHost);
  if (!s && e == hipSuccess) e = hipMemcpy(th.data(), td, th.size() * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(Xd);
  (void)hipFree(td);
  if (s) return s;
  HIPCHK(e);
  std::vector<float> xo(xh.size());
  std::vector<double> to(N);
  for (int i = 0; i < N; ++i) {
    const int c = S->M->perm[i];
    std::memcpy(&xo[(size_t)c * IND_NIN], &xh[(size_t)i * IND_NIN], IND_NIN * sizeof(float));
    to[c] = th[i];
  }
  if (flags & LXW_DEVICE_PTR) {
    HIPCHK(hipMemcpy(X, xo.data(), xo.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(theta_sc, to.data(), to.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::memcpy(X, xo.data(), xo.size() * sizeof(float));
    std::memcpy(theta_sc, to.data(), to.size() * sizeof(double));
  }
  return LXW_OK;
}

lxw_status lxw_solver_set_indicator(lxw_solver* S, const lxw_indicator* ind, double tau_lo, double tau_hi) {
  if (check_solver(S)) return LXW_ERR_ARG;
  if (ind && (S->M->kind != LXW_TRI || S->M->deg != 2))
    return fail(LXW_ERR_UNSUPPORTED, "the indicator is for degree-2 triangle meshes");
  if (ind && !(tau_lo >= 0.0 && tau_lo <= tau_hi && tau_hi <= 1.0))
    return fail(LXW_ERR_ARG, "need 0 <= tau_lo <= tau_hi <= 1");
  lxw_status s = sync_check(S);
  if (s) return s;
  if (ind && !S->ind_flag) {
    if ((s = S->alloc(&S->ind_flag, (size_t)S->M->N))) return s;
    if ((s = S->alloc(&S->ind_counts, (size_t)3 * IND_GRID_MAX))) return s;
  }
  if (ind) HIPCHK(hipMemset(S->ind_counts, 0, sizeof(unsigned long long) * 3 * IND_GRID_MAX));
  S->ind = ind;
  S->tau_lo = (float)tau_lo;
  S->tau_hi = (float)tau_hi;
  S->vd.ind_flag = ind ? S->ind_flag : nullptr;
  S->vf.ind_flag = ind ? S->ind_flag : nullptr;
  drop_graph(S);
  return LXW_OK;
}

lxw_status lxw_indicator_decisions(lxw_solver* S, int64_t* counts, uint8_t* flags) {
  if (check_solver(S) || !counts) return fail(LXW_ERR_ARG, "null argument");
  if (!S->ind) return fail(LXW_ERR_ARG, "no indicator set on this solver");
  lxw_status s = sync_check(S);
  if (s) return s;
  std::vector<unsigned long long> c((size_t)3 * IND_GRID_MAX);
  HIPCHK(hipMemcpy(c.data(), S->ind_counts, c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  for (int k = 0; k < 3; ++k) {
    unsigned long long t = 0;
    for (int b = 0; b < IND_GRID_MAX; ++b) t += c[(size_t)b * 3 + k];
    counts[k] = (int64_t)t;
  }
  if (flags) {
    std::vector<unsigned char> f(S->M->N);
    HIPCHK(hipMemcpy(f.data(), S->ind_flag, f.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < S->M->N; ++i) flags[S->M->perm[i]] = f[i];
  }
  return LXW_OK;
}

}  // extern "C"
