// TEST INFRASTRUCTURE ONLY -- the oracle.
//
// A plain, slow, FP64 CPU implementation of one time step of the positivity-preserving
// Lax-Wendroff discontinuous Galerkin (LxW-DG) method of Moe, Rossmanith and Seal,
// "Positivity-preserving discontinuous Galerkin methods with Lax-Wendroff time
// discretizations" (arXiv:1601.08145), for the compressible Euler equations in 1D, on 2D
// Cartesian (tensor Q2) meshes and on 2D triangle (P2) meshes.
//
// It exists to check the GPU library against.  Only the test-suite, the smoke entry point and
// the CPU-baseline leg of the benchmark may load it.  It shares no code, header, table or
// helper with the GPU library: its own reference elements, its own mesh connectivity, its own
// flux derivatives (by hyper-dual automatic differentiation instead of hand-written Jacobian and
// Hessian products), and its own limiter arithmetic, written for clarity, not speed.
//
// The step follows the per-loop algorithm of Sec. 3.3 ("Putting it all together"): element loop
// (Steps 1-2), edge loop (Step 3), element loop (Steps 4-5), element loop (Step 6), followed by
// the shock-capturing limiter of Sec. 1.5 Step 5.  Where the paper is silent or its printed
// formulas disagree with each other, the reading taken is stated at the place it is used.
//
// Pins: every function here is checked in tests/ against something other than itself
// (closed forms, exactness of quadrature, finite differences, exact Riemann solutions,
// convergence order, conservation, positivity, reduction to first-order Lax-Friedrichs).
// The shock-capturing limiter (shock_limit below) is a reading of a limiter that the paper cites
// but does not define, so its fidelity to that limiter's source cannot be checked from the paper;
// the reading itself is pinned by its defining properties (bounds after limiting, maximality of
// the factor, the neighbour averages it uses, the cell size in the relaxation, hand-computed
// cases) in tests/test_oracle_shock_limiter.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace ora {

// ------------------------------------------------------------------------------------------
// Hyper-dual numbers: v + a e1 + b e2 + ab e1 e2 with e1^2 = e2^2 = 0.  Evaluating F(q + e1 x
// + e2 y) gives F(q), F'(q)x, F'(q)y and F''(q)(x, y) exactly (no truncation error).  Used for
// the flux Jacobian-vector and Hessian-vector products of Eqs. (fluxderivs-a), (fluxderivs-b).
// ------------------------------------------------------------------------------------------
struct HD {
  double v, a, b, ab;
};
static inline HD hd(double v) { return {v, 0.0, 0.0, 0.0}; }
static inline HD operator+(HD x, HD y) { return {x.v + y.v, x.a + y.a, x.b + y.b, x.ab + y.ab}; }
static inline HD operator-(HD x, HD y) { return {x.v - y.v, x.a - y.a, x.b - y.b, x.ab - y.ab}; }
static inline HD operator*(HD x, HD y) {
  return {x.v * y.v, x.v * y.a + x.a * y.v, x.v * y.b + x.b * y.v,
          x.v * y.ab + x.a * y.b + x.b * y.a + x.ab * y.v};
}
static inline HD operator*(double s, HD x) { return {s * x.v, s * x.a, s * x.b, s * x.ab}; }
static inline HD operator+(HD x, double s) { return {x.v + s, x.a, x.b, x.ab}; }
static inline HD recip(HD x) {
  // d(1/v) = -dv/v^2 ; d2(1/v) = 2 dv1 dv2 / v^3 - d2v / v^2
  double r = 1.0 / x.v;
  return {r, -x.a * r * r, -x.b * r * r, 2.0 * x.a * x.b * r * r * r - x.ab * r * r};
}
static inline HD operator/(HD x, HD y) { return x * recip(y); }

// Triple-dual numbers: coefficients c[S] of the products e_S of the infinitesimals in S (bit i of S
// for e_{i+1}, e_i^2 = 0).  Evaluating F(q + e1 x + e2 y + e3 z) gives the third derivative
// F^(3)(q)(x, y, z) exactly as the e1 e2 e3 coefficient (the third time derivative of the flux,
// for the fourth-order time-averaged flux).
struct TD {
  double c[8];
};
static inline TD td(double v) { TD r{}; r.c[0] = v; return r; }
static inline TD operator+(TD x, TD y) { for (int k = 0; k < 8; ++k) x.c[k] += y.c[k]; return x; }
static inline TD operator-(TD x, TD y) { for (int k = 0; k < 8; ++k) x.c[k] -= y.c[k]; return x; }
static inline TD operator*(TD x, TD y) {
  TD r{};
  for (int S = 0; S < 8; ++S)
    for (int T = S;; T = (T - 1) & S) {  // every subset T of S
      r.c[S] += x.c[T] * y.c[S ^ T];
      if (T == 0) break;
    }
  return r;
}
static inline TD operator*(double s, TD x) { for (int k = 0; k < 8; ++k) x.c[k] *= s; return x; }
static inline TD operator+(TD x, double s) { x.c[0] += s; return x; }
static inline TD recip(TD x) {
  // 1/(v + n) = (1/v) (1 - n/v + (n/v)^2 - (n/v)^3) with n nilpotent (n^4 = 0)
  const double r = 1.0 / x.c[0];
  TD n = x;
  n.c[0] = 0.0;
  n = r * n;
  TD n2 = n * n, n3 = n2 * n;
  TD out = td(1.0) - n + n2 - n3;
  return r * out;
}
static inline TD operator/(TD x, TD y) { return x * recip(y); }

// ------------------------------------------------------------------------------------------
// Physics: Eq. (euler-eqns) with the equation of state Eq. (eos); the flux in direction d as
// written in Sec. 1.5.  Conserved variables q = (rho, M, E) in 1D, (rho, Mx, My, E) in 2D and
// (rho, Mx, My, Mz, E) in 3D.
// ------------------------------------------------------------------------------------------
template <class T>
static void euler_flux(int dim, double gam, const T* q, int d, T* F) {
  if (dim == 1) {
    T rho = q[0], m = q[1], E = q[2];
    T u = m / rho;
    T p = (gam - 1.0) * (E - 0.5 * (m * u));
    F[0] = m;
    F[1] = m * u + p;
    F[2] = u * (E + p);
  } else if (dim == 2) {
    T rho = q[0], mx = q[1], my = q[2], E = q[3];
    T u = mx / rho, v = my / rho;
    T p = (gam - 1.0) * (E - 0.5 * (mx * u + my * v));
    if (d == 0) {
      F[0] = mx;
      F[1] = mx * u + p;
      F[2] = my * u;
      F[3] = u * (E + p);
    } else {
      F[0] = my;
      F[1] = mx * v;
      F[2] = my * v + p;
      F[3] = v * (E + p);
    }
  } else {
    T rho = q[0], E = q[4];
    T m[3] = {q[1], q[2], q[3]};
    T u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
    T p = (gam - 1.0) * (E - 0.5 * (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]));
    F[0] = m[d];
    for (int k = 0; k < 3; ++k) F[1 + k] = m[k] * u[d];
    F[1 + d] = F[1 + d] + p;
    F[4] = u[d] * (E + p);
  }
}

template <>
void euler_flux<double>(int dim, double gam, const double* q, int d, double* F) {
  HD qh[5] = {}, Fh[5] = {};
  int V = dim + 2;
  for (int i = 0; i < V; ++i) qh[i] = hd(q[i]);
  euler_flux<HD>(dim, gam, qh, d, Fh);
  for (int i = 0; i < V; ++i) F[i] = Fh[i].v;
}

// A_d(q) x  (flux Jacobian times a vector), Eq. (fluxderivs-a)
static void flux_jvp(int dim, double gam, const double* q, int d, const double* x, double* out) {
  HD qh[5] = {}, Fh[5] = {};
  int V = dim + 2;
  for (int i = 0; i < V; ++i) qh[i] = {q[i], x[i], 0.0, 0.0};
  euler_flux<HD>(dim, gam, qh, d, Fh);
  for (int i = 0; i < V; ++i) out[i] = Fh[i].a;
}

// H_d(q)(x, y)  (flux Hessian applied to two vectors), Eq. (fluxderivs-b)
static void flux_hvp(int dim, double gam, const double* q, int d, const double* x, const double* y,
                     double* out) {
  HD qh[5] = {}, Fh[5] = {};
  int V = dim + 2;
  for (int i = 0; i < V; ++i) qh[i] = {q[i], x[i], y[i], 0.0};
  euler_flux<HD>(dim, gam, qh, d, Fh);
  for (int i = 0; i < V; ++i) out[i] = Fh[i].ab;
}

// F^(3)_d(q)(x, y, z)  (third derivative of the flux applied to three vectors)
static void flux_3vp(int dim, double gam, const double* q, int d, const double* x, const double* y,
                     const double* z, double* out) {
  TD qh[5] = {}, Fh[5] = {};
  int V = dim + 2;
  for (int i = 0; i < V; ++i) {
    qh[i] = td(q[i]);
    qh[i].c[1] = x[i];
    qh[i].c[2] = y[i];
    qh[i].c[4] = z[i];
  }
  euler_flux<TD>(dim, gam, qh, d, Fh);
  for (int i = 0; i < V; ++i) out[i] = Fh[i].c[7];
}

// Pressure from conserved variables, Eq. (eos) / Eq. (ave_press).
static double pressure(int dim, double gam, const double* q) {
  if (dim == 1) return (gam - 1.0) * (q[2] - 0.5 * q[1] * q[1] / q[0]);
  if (dim == 2) return (gam - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
  return (gam - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// ------------------------------------------------------------------------------------------
// Reference elements (Sec. 1.2).  The basis is the Gram-Schmidt orthonormalisation of the
// monomials listed below, in that order, under (1/|T0|) int_{T0} f g, using exact monomial
// integrals; phi_1 == 1 so that Q^(1) is the cell average (Sec. 1.2).  Line: Legendre P0..P2 on
// [-1,1].  Quad: the same procedure on [-1,1]^2 with the graded list below, which yields the
// tensor-product Legendre basis (Q2, 9 modes).  Triangle: reference triangle (0,0),(1,0),(0,1),
// P2 (6 modes).  Tetrahedron (Sec. 3.3 remark: the construction carries over face by face):
// reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1), P2 (10 modes).
// ------------------------------------------------------------------------------------------
enum Kind { LINE = 0, QUAD = 1, TRI = 2, TET = 3 };

struct RefElem {
  int kind = 0, deg = 2, dim = 0, ML = 0, K = 0, NI = 0, NQE = 0, NV = 0;
  double T0 = 0.0;                 // |T0|
  std::vector<int> ex, ey, ez;     // monomial exponents
  std::vector<double> C;           // ML x ML: phi_l = sum_j C[l*ML+j] * mono_j
  std::vector<double> xi_int;      // NI x dim interior quadrature points
  std::vector<double> w_int;       // NI weights, normalised to sum 1
  std::vector<double> s_edge, om_edge;  // NQE Gauss-Legendre nodes on [-1,1], weights sum 2
                                   // (tetrahedron: om_edge the face rule's weights, sum 2)
  std::vector<double> fb;          // tetrahedron: NQE x 3 barycentric coordinates of the face points
  std::vector<double> xv;          // NV x dim reference vertices (CCW)
};

static double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// (1/|T0|) int_{T0} xi^a eta^b zeta^c
static double mono_moment(int kind, int a, int b, int c = 0) {
  auto line = [](int n) { return (n % 2) ? 0.0 : 1.0 / (n + 1); };  // (1/2) int_{-1}^1 x^n
  if (kind == LINE) return line(a);
  if (kind == QUAD) return line(a) * line(b);
  if (kind == TET) return 6.0 * fact(a) * fact(b) * fact(c) / fact(a + b + c + 3);  // |T0| = 1/6
  return 2.0 * fact(a) * fact(b) / fact(a + b + 2);  // |T0| = 1/2
}

// Faces of the reference tetrahedron: face k is opposite vertex k, its vertices ordered so that
// (b - a) x (c - a) points outward.
static const int TET_FACE[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

static double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}
// d^k/dx^k x^n
static double dpow(double x, int n, int k) {
  if (k > n) return 0.0;
  double c = 1.0;
  for (int i = 0; i < k; ++i) c *= (n - i);
  return c * ipow(x, n - k);
}

// n-point Gauss rule on [-1, 1] for the weight (1 - x)^a (a = 0: Gauss-Legendre, a = 1:
// Gauss-Jacobi with alpha = 1, beta = 0): the roots of the orthogonal polynomial of degree n,
// found by Newton's method on the three-term recurrence from the Chebyshev points, and the weights
// 2^(a+1) / ((1 - x^2) P_n'(x)^2).
static void gauss_rule(int n, int a, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  auto poly = [&](double t, double& p, double& dp) {
    // Jacobi P_k^(a,0): 2k(k+a)(2k+a-2) P_k = (2k+a-1)[(2k+a)(2k+a-2) t + a^2] P_{k-1}
    //                                         - 2(k+a-1)(k-1)(2k+a) P_{k-2}
    double p0 = 1.0, p1 = 0.5 * ((a + 2) * t + a);
    if (n == 0) { p = p0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
      const double c1 = 2.0 * k * (k + a) * (2.0 * k + a - 2.0);
      const double c2 = (2.0 * k + a - 1.0) * ((2.0 * k + a) * (2.0 * k + a - 2.0) * t + a * a);
      const double c3 = 2.0 * (k + a - 1.0) * (k - 1.0) * (2.0 * k + a);
      const double p2 = (c2 * p1 - c3 * p0) / c1;
      p0 = p1;
      p1 = p2;
    }
    p = p1;
    // (2n + a)(1 - t^2) P_n' = n [(a - (2n + a) t) P_n + 2 (n + a) P_{n-1}]   (Jacobi, beta = 0)
    dp = n * ((a - (2.0 * n + a) * t) * p1 + 2.0 * (n + a) * p0) / ((2.0 * n + a) * (1.0 - t * t));
  };
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      poly(t, p, dp);
      const double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p, dp;
    poly(t, p, dp);
    x[n - 1 - i] = t;
    w[n - 1 - i] = std::pow(2.0, a + 1) / ((1.0 - t * t) * dp * dp);
  }
}

static RefElem make_ref(int kind, int deg = 2) {
  RefElem R;
  R.kind = kind;
  R.deg = deg;
  const double g = std::sqrt(3.0 / 5.0);
  R.s_edge = {-g, 0.0, g};
  R.om_edge = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
  if (deg == 3) {
    // P3: 4-point Gauss-Legendre on the edges and in 1D; on the triangle the collapsed product of
    // 4-point Gauss-Legendre in s and 4-point Gauss-Jacobi (weight 1 - t) in t, at
    // (xi, eta) = (s (1 - t), t): 16 points, exact to degree 7 (the products phi_l phi_m of
    // degree 6 of the projection included).
    std::vector<double> xl, wl, xj, wj;
    gauss_rule(4, 0, xl, wl);
    gauss_rule(4, 1, xj, wj);
    R.s_edge = xl;
    R.om_edge = wl;
    if (kind == LINE) {
      R.dim = 1; R.ML = 4; R.K = 2; R.NV = 2; R.NQE = 1; R.T0 = 2.0;
      R.ex = {0, 1, 2, 3}; R.ey = {0, 0, 0, 0};
      R.xv = {-1.0, 1.0};
      for (int i = 0; i < 4; ++i) { R.xi_int.push_back(xl[i]); R.w_int.push_back(wl[i] / 2.0); }
      R.s_edge = {0.0}; R.om_edge = {2.0};
    } else if (kind == TRI) {
      R.dim = 2; R.ML = 10; R.K = 3; R.NV = 3; R.NQE = 4; R.T0 = 0.5;
      R.ex = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0}; R.ey = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
      R.xv = {0, 0, 1, 0, 0, 1};
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) {
          const double sv = 0.5 * (xl[i] + 1.0), tv = 0.5 * (xj[j] + 1.0);
          R.xi_int.push_back(sv * (1.0 - tv));
          R.xi_int.push_back(tv);
          // (1/|T0|) int = 2 int_0^1 int_0^1 f (1 - t) ds dt; ds = dx/2, (1 - t) dt = (1 - x) dx / 4
          R.w_int.push_back(2.0 * (wl[i] / 2.0) * (wj[j] / 4.0));
        }
    } else {
      return R;  // no degree-3 element of this kind (R.ML == 0)
    }
    R.NI = (int)R.w_int.size();
  } else if (kind == LINE) {
    R.dim = 1; R.ML = 3; R.K = 2; R.NV = 2; R.NQE = 1; R.T0 = 2.0;
    R.ex = {0, 1, 2}; R.ey = {0, 0, 0};
    R.xv = {-1.0, 1.0};
    for (int i = 0; i < 3; ++i) { R.xi_int.push_back(R.s_edge[i]); R.w_int.push_back(R.om_edge[i] / 2.0); }
    R.s_edge = {0.0}; R.om_edge = {2.0};  // a face in 1D is a point; half the weight sum is 1
  } else if (kind == QUAD) {
    R.dim = 2; R.ML = 9; R.K = 4; R.NV = 4; R.NQE = 3; R.T0 = 4.0;
    R.ex = {0, 1, 0, 2, 1, 0, 2, 1, 2}; R.ey = {0, 0, 1, 0, 1, 2, 1, 2, 2};
    R.xv = {-1, -1, 1, -1, 1, 1, -1, 1};
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        R.xi_int.push_back(R.s_edge[i]); R.xi_int.push_back(R.s_edge[j]);
        R.w_int.push_back(R.om_edge[i] * R.om_edge[j] / 4.0);
      }
  } else if (kind == TET) {
    R.dim = 3; R.ML = 10; R.K = 4; R.NV = 4; R.T0 = 1.0 / 6.0;
    R.ex = {0, 1, 0, 0, 2, 1, 1, 0, 0, 0};
    R.ey = {0, 0, 1, 0, 0, 1, 0, 2, 1, 0};
    R.ez = {0, 0, 0, 1, 0, 0, 1, 0, 1, 2};
    R.xv = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    // Interior: the collapsed (Duffy) product rule (xi, eta, zeta) = (u (1 - v)(1 - w), v (1 - w), w)
    // with u, v, w = (1 + t)/2 at the 3-point Gauss rules for the weights 1, (1 - t) and (1 - t)^2
    // (the Jacobian (1 - v)(1 - w)^2 of the collapse): 27 points, exact to degree 5.
    std::vector<double> x0, w0, x1, w1, x2, w2;
    gauss_rule(3, 0, x0, w0);
    gauss_rule(3, 1, x1, w1);
    gauss_rule(3, 2, x2, w2);
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          const double u = 0.5 * (1.0 + x0[i]), v = 0.5 * (1.0 + x1[j]), w = 0.5 * (1.0 + x2[k]);
          R.xi_int.push_back(u * (1.0 - v) * (1.0 - w));
          R.xi_int.push_back(v * (1.0 - w));
          R.xi_int.push_back(w);
          // (1/|T0|) int = 6 int u,v,w f (1 - v)(1 - w)^2 = (6/64) int f (1 - t1)(1 - t2)^2 dt0 dt1 dt2
          R.w_int.push_back(6.0 / 64.0 * w0[i] * w1[j] * w2[k]);
        }
    // Faces: the same 7-point degree-5 rule as the triangle interior, in barycentric coordinates
    // (fully symmetric, so both sides of a face see the same point set); weights scaled to sum 2.
    const double r15 = std::sqrt(15.0);
    const double a1 = (6.0 - r15) / 21.0, b1 = (9.0 + 2.0 * r15) / 21.0, v1 = (155.0 - r15) / 1200.0;
    const double a2 = (6.0 + r15) / 21.0, b2 = (9.0 - 2.0 * r15) / 21.0, v2 = (155.0 + r15) / 1200.0;
    R.om_edge.clear();
    auto addf = [&](double l0, double l1, double l2, double w) {
      R.fb.push_back(l0); R.fb.push_back(l1); R.fb.push_back(l2); R.om_edge.push_back(2.0 * w);
    };
    addf(1.0 / 3, 1.0 / 3, 1.0 / 3, 9.0 / 40.0);
    addf(b1, a1, a1, v1); addf(a1, b1, a1, v1); addf(a1, a1, b1, v1);
    addf(b2, a2, a2, v2); addf(a2, b2, a2, v2); addf(a2, a2, b2, v2);
    R.NQE = 7;
    R.s_edge.assign(7, 0.0);
  } else {
    R.dim = 2; R.ML = 6; R.K = 3; R.NV = 3; R.NQE = 3; R.T0 = 0.5;
    R.ex = {0, 1, 0, 2, 1, 0}; R.ey = {0, 0, 1, 0, 1, 2};
    R.xv = {0, 0, 1, 0, 0, 1};
    // Degree-5, 7-point symmetric rule (Radon): centroid plus two orbits (a,a,b).
    const double r15 = std::sqrt(15.0);
    const double a1 = (6.0 - r15) / 21.0, b1 = (9.0 + 2.0 * r15) / 21.0, w1 = (155.0 - r15) / 1200.0;
    const double a2 = (6.0 + r15) / 21.0, b2 = (9.0 - 2.0 * r15) / 21.0, w2 = (155.0 + r15) / 1200.0;
    auto add = [&](double l1, double l2, double l3, double w) {
      (void)l1;
      R.xi_int.push_back(l2); R.xi_int.push_back(l3); R.w_int.push_back(w);
    };
    add(1.0 / 3, 1.0 / 3, 1.0 / 3, 9.0 / 40.0);
    add(a1, a1, b1, w1); add(a1, b1, a1, w1); add(b1, a1, a1, w1);
    add(a2, a2, b2, w2); add(a2, b2, a2, w2); add(b2, a2, a2, w2);
  }
  R.NI = (int)R.w_int.size();
  if (R.ez.empty()) R.ez.assign(R.ML, 0);
  // Gram-Schmidt in the monomial coordinates with the exact Gram matrix G.
  int ML = R.ML;
  std::vector<double> G(ML * ML);
  for (int a = 0; a < ML; ++a)
    for (int b = 0; b < ML; ++b)
      G[a * ML + b] = mono_moment(kind, R.ex[a] + R.ex[b], R.ey[a] + R.ey[b], R.ez[a] + R.ez[b]);
  auto ip = [&](const double* u, const double* v) {
    double s = 0.0;
    for (int a = 0; a < ML; ++a)
      for (int b = 0; b < ML; ++b) s += u[a] * G[a * ML + b] * v[b];
    return s;
  };
  R.C.assign(ML * ML, 0.0);
  for (int l = 0; l < ML; ++l) {
    std::vector<double> u(ML, 0.0);
    u[l] = 1.0;
    for (int k = 0; k < l; ++k) {
      double c = ip(u.data(), &R.C[k * ML]);
      for (int a = 0; a < ML; ++a) u[a] -= c * R.C[k * ML + a];
    }
    double nrm = std::sqrt(ip(u.data(), u.data()));
    for (int a = 0; a < ML; ++a) R.C[l * ML + a] = u[a] / nrm;
  }
  return R;
}

// phi_l and its reference derivatives at xi.  da, db, dc count derivatives in xi, eta, zeta.
static double phi(const RefElem& R, int l, const double* xi, int da = 0, int db = 0, int dc = 0) {
  double s = 0.0;
  double x = xi[0], y = (R.dim >= 2) ? xi[1] : 0.0, z = (R.dim == 3) ? xi[2] : 0.0;
  for (int j = 0; j < R.ML; ++j) {
    double c = R.C[l * R.ML + j];
    if (c == 0.0) continue;
    double t = c * dpow(x, R.ex[j], da) * dpow(y, R.ey[j], db);
    if (R.dim == 3) t *= dpow(z, R.ez[j], dc);
    else if (dc) t = 0.0;
    s += t;
  }
  return s;
}

// Reference coordinates of edge point j on local edge k.  Edge k runs from vertex k to vertex
// k+1 (counter-clockwise); in 1D local edge k is vertex k.
static void edge_point(const RefElem& R, int k, int j, double* xi) {
  if (R.dim == 1) { xi[0] = R.xv[k]; return; }
  if (R.dim == 3) {  // face k: barycentric combination of its three vertices
    for (int a = 0; a < 3; ++a) {
      xi[a] = 0.0;
      for (int m = 0; m < 3; ++m) xi[a] += R.fb[j * 3 + m] * R.xv[TET_FACE[k][m] * 3 + a];
    }
    return;
  }
  int a = k, b = (k + 1) % R.NV;
  double t = 0.5 * (1.0 + R.s_edge[j]);
  xi[0] = R.xv[2 * a] + t * (R.xv[2 * b] - R.xv[2 * a]);
  xi[1] = R.xv[2 * a + 1] + t * (R.xv[2 * b + 1] - R.xv[2 * a + 1]);
}

// ------------------------------------------------------------------------------------------
// Mesh: elements, edges e with normal n_e (|n_e| = edge length), the element i_e out of which
// n_e points, the element j_e into which it points, and eps_ik = +1/-1 (Sec. 3.3, Eq. (epsik)).
// Boundary edges have i_e = the interior element and j_e = -1 (a ghost, Sec. 2.4).
// ------------------------------------------------------------------------------------------
enum BC { BC_INTERIOR = -1, BC_PERIODIC = 0, BC_TRANSPARENT = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3 };

struct Mesh {
  RefElem R;
  int N = 0, E = 0;
  std::vector<double> vx;          // N x NV x dim
  std::vector<double> Jinv;        // N x dim x dim, Jinv[a][d] = d xi_a / d x_d
  std::vector<double> area, perim;
  std::vector<int> nbr, nbr_k;     // N x K, -1 on the boundary
  std::vector<int> ebc;            // N x K boundary type of local edge (BC_INTERIOR inside)
  std::vector<int> eid, eps;       // N x K
  std::vector<int> e_i, e_ki, e_j, e_kj, e_bc;
  std::vector<double> e_n, e_len;  // E x 3 (unused components zero); |n_e| = edge length / face area
  // Point order on an edge or face: local point jl of (element i, local edge k) is point
  // fmap[(i K + k) NQE + jl] in the order of i_e; finv is the inverse.
  std::vector<int> fmap, finv;
};

static void map_point(const Mesh& M, int i, const double* xi, double* x);
static void build_point_order(Mesh& M);

static void finish_mesh(Mesh& M) {
  const RefElem& R = M.R;
  int N = M.N, K = R.K, dim = R.dim;
  M.Jinv.assign(N * dim * dim, 0.0);
  M.area.assign(N, 0.0);
  M.perim.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    const double* v = &M.vx[i * R.NV * dim];
    if (R.kind == LINE) {
      double J = 0.5 * (v[1] - v[0]);
      M.Jinv[i] = 1.0 / J;
      M.area[i] = v[1] - v[0];
      M.perim[i] = 2.0;
    } else if (R.kind == TET) {
      // J[a][b] = d x_a / d xi_b = (v_{b+1} - v_0)_a; Jinv by the adjugate
      double J[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = v[3 * (b + 1) + a] - v[a];
      double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                   J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      double* Ji = &M.Jinv[i * 9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          // inverse[a][b] = cofactor[b][a] / det
          int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
          Ji[a * 3 + b] = (J[r0][c0] * J[r1][c1] - J[r0][c1] * J[r1][c0]) / det;
        }
      M.area[i] = det * R.T0;
      double P = 0.0;
      for (int k = 0; k < 4; ++k) {
        const double* A = &v[3 * TET_FACE[k][0]];
        const double* B = &v[3 * TET_FACE[k][1]];
        const double* C = &v[3 * TET_FACE[k][2]];
        double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        P += 0.5 * std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      }
      M.perim[i] = P;
    } else {
      double J[2][2];
      if (R.kind == TRI) {
        J[0][0] = v[2] - v[0]; J[0][1] = v[4] - v[0];
        J[1][0] = v[3] - v[1]; J[1][1] = v[5] - v[1];
      } else {
        J[0][0] = 0.5 * (v[2] - v[0]); J[0][1] = 0.5 * (v[6] - v[0]);
        J[1][0] = 0.5 * (v[3] - v[1]); J[1][1] = 0.5 * (v[7] - v[1]);
      }
      double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      double* Ji = &M.Jinv[i * 4];
      Ji[0] = J[1][1] / det; Ji[1] = -J[0][1] / det;
      Ji[2] = -J[1][0] / det; Ji[3] = J[0][0] / det;
      M.area[i] = det * R.T0;
      double P = 0.0;
      for (int k = 0; k < K; ++k) {
        int b = (k + 1) % R.NV;
        P += std::hypot(v[2 * b] - v[2 * k], v[2 * b + 1] - v[2 * k + 1]);
      }
      M.perim[i] = P;
    }
  }
  // Edges: one per boundary (i,k), one per interior pair, i_e = the lexicographically first.
  M.eid.assign(N * K, -1);
  M.eps.assign(N * K, 0);
  M.E = 0;
  M.e_i.clear(); M.e_ki.clear(); M.e_j.clear(); M.e_kj.clear(); M.e_bc.clear();
  M.e_n.clear(); M.e_len.clear();
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < K; ++k) {
      if (M.eid[i * K + k] >= 0) continue;
      int j = M.nbr[i * K + k], kj = M.nbr_k[i * K + k];
      int e = M.E++;
      M.e_i.push_back(i); M.e_ki.push_back(k); M.e_j.push_back(j); M.e_kj.push_back(kj);
      M.e_bc.push_back(M.ebc[i * K + k]);
      M.eid[i * K + k] = e; M.eps[i * K + k] = +1;
      if (j >= 0) { M.eid[j * K + kj] = e; M.eps[j * K + kj] = -1; }
      const double* v = &M.vx[i * R.NV * dim];
      if (dim == 1) {
        M.e_n.push_back(k == 0 ? -1.0 : 1.0); M.e_n.push_back(0.0); M.e_n.push_back(0.0);
        M.e_len.push_back(1.0);
      } else if (dim == 2) {
        int b = (k + 1) % R.NV;
        double dx = v[2 * b] - v[2 * k], dy = v[2 * b + 1] - v[2 * k + 1];
        M.e_n.push_back(dy); M.e_n.push_back(-dx); M.e_n.push_back(0.0);
        M.e_len.push_back(std::hypot(dx, dy));
      } else {  // face k: n = (1/2)(B - A) x (C - A), outward, |n| = face area
        const double* A = &v[3 * TET_FACE[k][0]];
        const double* B = &v[3 * TET_FACE[k][1]];
        const double* C = &v[3 * TET_FACE[k][2]];
        double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, w[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        double n[3] = {0.5 * (u[1] * w[2] - u[2] * w[1]), 0.5 * (u[2] * w[0] - u[0] * w[2]), 0.5 * (u[0] * w[1] - u[1] * w[0])};
        for (int a = 0; a < 3; ++a) M.e_n.push_back(n[a]);
        M.e_len.push_back(std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
      }
    }
  build_point_order(M);
}

// Point order across each edge: in 1D and 2D the second element visits the edge's points in
// reverse.  On tetrahedron faces the points of the j_e side are located among those of the
// i_e side by their physical coordinates (shifted by the difference of the face centroids,
// which is the period on periodic faces).
static void build_point_order(Mesh& M) {
  const RefElem& R = M.R;
  const int N = M.N, K = R.K, dim = R.dim, NQ = R.NQE;
  M.fmap.assign((size_t)N * K * NQ, 0);
  M.finv.assign((size_t)N * K * NQ, 0);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < K; ++k)
      for (int jl = 0; jl < NQ; ++jl) {
        int jj = (M.eps[i * K + k] > 0 || dim < 3) ? ((M.eps[i * K + k] > 0) ? jl : NQ - 1 - jl) : -1;
        if (jj < 0) {
          const int e = M.eid[i * K + k], ie = M.e_i[e], ke = M.e_ki[e];
          double xj[3], ci[3] = {0, 0, 0}, cj[3] = {0, 0, 0}, xi_[3];
          for (int q = 0; q < NQ; ++q) {
            double a[3], b[3];
            edge_point(R, ke, q, xi_); map_point(M, ie, xi_, a);
            edge_point(R, k, q, xi_); map_point(M, i, xi_, b);
            for (int c = 0; c < 3; ++c) { ci[c] += a[c] / NQ; cj[c] += b[c] / NQ; }
          }
          edge_point(R, k, jl, xi_);
          map_point(M, i, xi_, xj);
          double best = 1e300;
          for (int q = 0; q < NQ; ++q) {
            double a[3];
            edge_point(R, ke, q, xi_);
            map_point(M, ie, xi_, a);
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) d2 += (xj[c] - (cj[c] - ci[c]) - a[c]) * (xj[c] - (cj[c] - ci[c]) - a[c]);
            if (d2 < best) { best = d2; jj = q; }
          }
        }
        M.fmap[((size_t)i * K + k) * NQ + jl] = jj;
        M.finv[((size_t)i * K + k) * NQ + jj] = jl;
      }
}

static Mesh* mesh_1d(int n, double x0, double x1, int bcl, int bcr) {
  Mesh* M = new Mesh;
  M->R = make_ref(LINE);
  M->N = n;
  double h = (x1 - x0) / n;
  for (int i = 0; i < n; ++i) { M->vx.push_back(x0 + i * h); M->vx.push_back(x0 + (i + 1) * h); }
  M->nbr.assign(2 * n, -1); M->nbr_k.assign(2 * n, -1); M->ebc.assign(2 * n, BC_INTERIOR);
  bool per = (bcl == BC_PERIODIC);
  for (int i = 0; i < n; ++i) {
    // local edge 0 = left end, 1 = right end
    if (i > 0) { M->nbr[2 * i] = i - 1; M->nbr_k[2 * i] = 1; }
    else if (per) { M->nbr[0] = n - 1; M->nbr_k[0] = 1; }
    else M->ebc[0] = bcl;
    if (i < n - 1) { M->nbr[2 * i + 1] = i + 1; M->nbr_k[2 * i + 1] = 0; }
    else if (per) { M->nbr[2 * i + 1] = 0; M->nbr_k[2 * i + 1] = 0; }
    else M->ebc[2 * i + 1] = bcr;
  }
  finish_mesh(*M);
  return M;
}

// bc[4] = {x-low, x-high, y-low, y-high}.  keep (nullable, nx*ny flags, cell (i, j) at i + nx*j)
// removes the cells whose flag is 0: the remaining cells are numbered in that row-major order and
// their edges facing a removed cell get the boundary type wall_bc (the solid of the paper's
// Cartesian step problem, Sec. 4).
static Mesh* mesh_cart(int nx, int ny, double x0, double x1, double y0, double y1, const int* bc,
                       const unsigned char* keep, int wall_bc) {
  Mesh* M = new Mesh;
  M->R = make_ref(QUAD);
  std::vector<int> id(nx * ny, -1);
  int N = 0;
  for (int c = 0; c < nx * ny; ++c)
    if (!keep || keep[c]) id[c] = N++;
  M->N = N;
  double hx = (x1 - x0) / nx, hy = (y1 - y0) / ny;
  M->nbr.assign(4 * N, -1); M->nbr_k.assign(4 * N, -1); M->ebc.assign(4 * N, BC_INTERIOR);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int e = id[i + nx * j];
      if (e < 0) continue;
      double xa = x0 + i * hx, xb = x0 + (i + 1) * hx, ya = y0 + j * hy, yb = y0 + (j + 1) * hy;
      double v[8] = {xa, ya, xb, ya, xb, yb, xa, yb};
      for (double c : v) M->vx.push_back(c);
      // local edges: 0 bottom, 1 right, 2 top, 3 left
      auto link = [&](int k, int ii, int jj, int kk, int bcode) {
        bool out = (ii < 0 || ii >= nx || jj < 0 || jj >= ny);
        if (out && bcode != BC_PERIODIC) { M->ebc[4 * e + k] = bcode; return; }
        ii = (ii + nx) % nx; jj = (jj + ny) % ny;
        int n = id[ii + nx * jj];
        if (n < 0) { M->ebc[4 * e + k] = wall_bc; return; }
        M->nbr[4 * e + k] = n; M->nbr_k[4 * e + k] = kk;
      };
      link(0, i, j - 1, 2, bc[2]);
      link(1, i + 1, j, 3, bc[1]);
      link(2, i, j + 1, 0, bc[3]);
      link(3, i - 1, j, 1, bc[0]);
    }
  finish_mesh(*M);
  return M;
}

// Triangles given by node coordinates and counter-clockwise vertex triples.  Boundary edges get
// the type bnd[3*t+k] (transparent when bnd is null).  Boundary edges marked periodic are paired
// with the boundary edge whose midpoint differs by one period in x or y.
static Mesh* mesh_tri(int nn, const double* xy, int nt, const int* tri, const int* bnd,
                      const double* period, std::string* err) {
  Mesh* M = new Mesh;
  M->R = make_ref(TRI);
  M->N = nt;
  for (int t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a) {
      int v = tri[3 * t + a];
      if (v < 0 || v >= nn) { *err = "node index out of range"; delete M; return nullptr; }
      M->vx.push_back(xy[2 * v]); M->vx.push_back(xy[2 * v + 1]);
    }
  M->nbr.assign(3 * nt, -1); M->nbr_k.assign(3 * nt, -1); M->ebc.assign(3 * nt, BC_INTERIOR);
  std::map<std::pair<int, int>, std::pair<int, int>> open;
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      auto key = std::make_pair(std::min(a, b), std::max(a, b));
      auto it = open.find(key);
      if (it == open.end()) open[key] = {t, k};
      else {
        int t2 = it->second.first, k2 = it->second.second;
        M->nbr[3 * t + k] = t2; M->nbr_k[3 * t + k] = k2;
        M->nbr[3 * t2 + k2] = t; M->nbr_k[3 * t2 + k2] = k;
        open.erase(it);
      }
    }
  std::vector<std::pair<int, int>> per;
  for (auto& kv : open) {
    int t = kv.second.first, k = kv.second.second;
    int code = bnd ? bnd[3 * t + k] : BC_TRANSPARENT;
    if (code == BC_PERIODIC) per.push_back({t, k});
    else M->ebc[3 * t + k] = code;
  }
  if (!per.empty()) {
    if (!period) { *err = "periodic edges without a period"; delete M; return nullptr; }
    // pair periodic edges by midpoint modulo the period
    auto mid = [&](int t, int k, double* m) {
      const double* v = &M->vx[6 * t];
      int b = (k + 1) % 3;
      m[0] = 0.5 * (v[2 * k] + v[2 * b]); m[1] = 0.5 * (v[2 * k + 1] + v[2 * b + 1]);
    };
    std::vector<int> used(per.size(), 0);
    for (size_t p = 0; p < per.size(); ++p) {
      if (used[p]) continue;
      double mp[2]; mid(per[p].first, per[p].second, mp);
      bool found = false;
      for (size_t q = p + 1; q < per.size() && !found; ++q) {
        if (used[q]) continue;
        double mq[2]; mid(per[q].first, per[q].second, mq);
        double dx = mq[0] - mp[0], dy = mq[1] - mp[1];
        double tol = 1e-9 * (std::fabs(period[0]) + std::fabs(period[1]));
        bool mx = period[0] > 0 && std::fabs(std::fabs(dx) - period[0]) < tol && std::fabs(dy) < tol;
        bool my = period[1] > 0 && std::fabs(std::fabs(dy) - period[1]) < tol && std::fabs(dx) < tol;
        if (mx || my) {
          int t = per[p].first, k = per[p].second, t2 = per[q].first, k2 = per[q].second;
          M->nbr[3 * t + k] = t2; M->nbr_k[3 * t + k] = k2;
          M->nbr[3 * t2 + k2] = t; M->nbr_k[3 * t2 + k2] = k;
          used[p] = used[q] = 1; found = true;
        }
      }
      if (!found) { *err = "unpaired periodic edge"; delete M; return nullptr; }
    }
  }
  finish_mesh(*M);
  for (int t = 0; t < nt; ++t)
    if (!(M->area[t] > 0.0)) { *err = "triangle not counter-clockwise or degenerate"; delete M; return nullptr; }
  return M;
}

// Tetrahedral mesh: nodes xyz (nn x 3), tetrahedra tet (nt x 4, positively oriented), boundary
// codes per (tetrahedron, face k opposite vertex k) (null: transparent), period (3 lengths, 0 for
// a non-periodic axis) for periodic faces, which are paired by their centroids.  Inflow sides are
// not supported on tetrahedra.
static Mesh* mesh_tet(int nn, const double* xyz, int nt, const int* tet, const int* bnd, const double* period,
                      std::string* err) {
  Mesh* M = new Mesh;
  M->R = make_ref(TET);
  M->N = nt;
  for (int t = 0; t < nt; ++t)
    for (int a = 0; a < 4; ++a) {
      int v = tet[4 * t + a];
      if (v < 0 || v >= nn) { *err = "node index out of range"; delete M; return nullptr; }
      for (int c = 0; c < 3; ++c) M->vx.push_back(xyz[3 * v + c]);
    }
  M->nbr.assign(4 * nt, -1); M->nbr_k.assign(4 * nt, -1); M->ebc.assign(4 * nt, BC_INTERIOR);
  std::map<std::tuple<int, int, int>, std::pair<int, int>> open;
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 4; ++k) {
      int f[3];
      for (int m = 0; m < 3; ++m) f[m] = tet[4 * t + TET_FACE[k][m]];
      std::sort(f, f + 3);
      auto key = std::make_tuple(f[0], f[1], f[2]);
      auto it = open.find(key);
      if (it == open.end()) open[key] = {t, k};
      else {
        int t2 = it->second.first, k2 = it->second.second;
        M->nbr[4 * t + k] = t2; M->nbr_k[4 * t + k] = k2;
        M->nbr[4 * t2 + k2] = t; M->nbr_k[4 * t2 + k2] = k;
        open.erase(it);
      }
    }
  std::vector<std::pair<int, int>> per;
  for (auto& kv : open) {
    int t = kv.second.first, k = kv.second.second;
    int code = bnd ? bnd[4 * t + k] : BC_TRANSPARENT;
    if (code == BC_INFLOW) { *err = "inflow boundaries are not supported on tetrahedra"; delete M; return nullptr; }
    if (code == BC_PERIODIC) per.push_back({t, k});
    else M->ebc[4 * t + k] = code;
  }
  if (!per.empty()) {
    if (!period) { *err = "periodic faces without a period"; delete M; return nullptr; }
    auto cen = [&](int t, int k, double* c) {
      const double* v = &M->vx[12 * t];
      for (int a = 0; a < 3; ++a)
        c[a] = (v[3 * TET_FACE[k][0] + a] + v[3 * TET_FACE[k][1] + a] + v[3 * TET_FACE[k][2] + a]) / 3.0;
    };
    const double tol = 1e-9 * (std::fabs(period[0]) + std::fabs(period[1]) + std::fabs(period[2]));
    std::vector<int> used(per.size(), 0);
    for (size_t p = 0; p < per.size(); ++p) {
      if (used[p]) continue;
      double cp[3]; cen(per[p].first, per[p].second, cp);
      bool found = false;
      for (size_t q = p + 1; q < per.size() && !found; ++q) {
        if (used[q]) continue;
        double cq[3]; cen(per[q].first, per[q].second, cq);
        int shifted = 0, same = 0;
        for (int a = 0; a < 3; ++a) {
          const double d = std::fabs(cq[a] - cp[a]);
          if (d < tol) ++same;
          else if (period[a] > 0 && std::fabs(d - period[a]) < tol) ++shifted;
        }
        if (shifted == 1 && same == 2) {
          int t = per[p].first, k = per[p].second, t2 = per[q].first, k2 = per[q].second;
          M->nbr[4 * t + k] = t2; M->nbr_k[4 * t + k] = k2;
          M->nbr[4 * t2 + k2] = t; M->nbr_k[4 * t2 + k2] = k;
          used[p] = used[q] = 1; found = true;
        }
      }
      if (!found) { *err = "unpaired periodic face"; delete M; return nullptr; }
    }
  }
  finish_mesh(*M);
  for (int t = 0; t < nt; ++t)
    if (!(M->area[t] > 0.0)) { *err = "tetrahedron not positively oriented or degenerate"; delete M; return nullptr; }
  return M;
}

// ------------------------------------------------------------------------------------------
// Solver state and the step.
// ------------------------------------------------------------------------------------------
struct Params {
  double gamma = 1.4, cfl = 0.08, eps0 = 1e-12, alpha0 = 500.0;
  int shock = 1;
  double inflow[4] = {1, 0, 0, 1};
  double force_theta = -1.0;  // test hook: when >= 0, every Lambda_e is replaced by this value
  int exact_theta = 0;        // moment limiter Step 2 by the exact root instead of concavity
  int s_avg = 0;              // global wave speed from the cell averages only
};

enum Status { OK = 0, ERR_ARG = -1, ERR_STATE = -4, ERR_POSITIVITY = -5, ERR_NONFINITE = -6, ERR_CFL = -7 };

struct Solver {
  Mesh* M;
  Params P;
  double t = 0.0;
  std::vector<double> Q;  // N x V x ML
  // Intermediate quantities of the last step, for stage-by-stage comparison.
  double s = 0.0, dt = 0.0;
  std::vector<double> theta_mom, theta_sc, Qlim, Vol, Qupd;
  std::vector<double> fLxW_ik, fLxF_ik, Lam_ik, c_ik, Lam_e_ik;  // per (element, local edge)
  std::vector<double> qderiv;  // q_t, q_tt, q_ttt (zero below degree 3) at the interior points: N x NI x 3 x V
  // Cells the shock-capturing limiter may act on (empty: all).  A learned troubled-cell
  // indicator replaces only the detection of that limiter; this mask carries its decisions.
  std::vector<unsigned char> shock_mask;
  int err_elem = -1;
  std::string err;
};

static inline int NVAR(const Mesh& M) { return M.R.dim + 2; }

// Physical coordinates of a reference point in element i.
static void map_point(const Mesh& M, int i, const double* xi, double* x) {
  const RefElem& R = M.R;
  const double* v = &M.vx[i * R.NV * R.dim];
  if (R.kind == LINE) { x[0] = v[0] + 0.5 * (xi[0] + 1.0) * (v[1] - v[0]); return; }
  if (R.kind == TET) {
    for (int a = 0; a < 3; ++a)
      x[a] = v[a] + xi[0] * (v[3 + a] - v[a]) + xi[1] * (v[6 + a] - v[a]) + xi[2] * (v[9 + a] - v[a]);
    return;
  }
  if (R.kind == TRI) {
    x[0] = v[0] + xi[0] * (v[2] - v[0]) + xi[1] * (v[4] - v[0]);
    x[1] = v[1] + xi[0] * (v[3] - v[1]) + xi[1] * (v[5] - v[1]);
  } else {
    x[0] = v[0] + 0.5 * (xi[0] + 1.0) * (v[2] - v[0]) + 0.5 * (xi[1] + 1.0) * (v[6] - v[0]);
    x[1] = v[1] + 0.5 * (xi[0] + 1.0) * (v[3] - v[1]) + 0.5 * (xi[1] + 1.0) * (v[7] - v[1]);
  }
}

// Physical gradient of phi_l: d phi / d x_d = sum_a Jinv[a][d] d phi / d xi_a.
static void grad_phi(const Mesh& M, int i, int l, const double* xi, double* g) {
  const RefElem& R = M.R;
  const double* Ji = &M.Jinv[i * R.dim * R.dim];
  if (R.dim == 1) { g[0] = Ji[0] * phi(R, l, xi, 1, 0); return; }
  if (R.dim == 3) {
    const double r[3] = {phi(R, l, xi, 1, 0, 0), phi(R, l, xi, 0, 1, 0), phi(R, l, xi, 0, 0, 1)};
    for (int d = 0; d < 3; ++d) g[d] = Ji[0 * 3 + d] * r[0] + Ji[1 * 3 + d] * r[1] + Ji[2 * 3 + d] * r[2];
    return;
  }
  double d0 = phi(R, l, xi, 1, 0), d1 = phi(R, l, xi, 0, 1);
  g[0] = Ji[0] * d0 + Ji[2] * d1;
  g[1] = Ji[1] * d0 + Ji[3] * d1;
}

// Physical Hessian of phi_l: H[d][e] = sum_ab Jinv[a][d] Jinv[b][e] d2 phi / dxi_a dxi_b.
static void hess_phi(const Mesh& M, int i, int l, const double* xi, double* H) {
  const RefElem& R = M.R;
  const double* Ji = &M.Jinv[i * R.dim * R.dim];
  if (R.dim == 1) { H[0] = Ji[0] * Ji[0] * phi(R, l, xi, 2, 0); return; }
  if (R.dim == 3) {
    double r[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        r[a][b] = phi(R, l, xi, (a == 0) + (b == 0), (a == 1) + (b == 1), (a == 2) + (b == 2));
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e) {
        double t = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) t += Ji[a * 3 + d] * Ji[b * 3 + e] * r[a][b];
        H[d * 3 + e] = t;
      }
    return;
  }
  double r[2][2] = {{phi(R, l, xi, 2, 0), phi(R, l, xi, 1, 1)}, {phi(R, l, xi, 1, 1), phi(R, l, xi, 0, 2)}};
  for (int d = 0; d < 2; ++d)
    for (int e = 0; e < 2; ++e) {
      double s = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += Ji[a * 2 + d] * Ji[b * 2 + e] * r[a][b];
      H[d * 2 + e] = s;
    }
}

// Physical third derivatives of phi_l: T[(d dim + e) dim + f] = sum_abc Jinv[a][d] Jinv[b][e]
// Jinv[c][f] d3 phi / dxi_a dxi_b dxi_c (affine elements).
static void d3_phi(const Mesh& M, int i, int l, const double* xi, double* T) {
  const RefElem& R = M.R;
  const double* Ji = &M.Jinv[i * R.dim * R.dim];
  if (R.dim == 1) { T[0] = Ji[0] * Ji[0] * Ji[0] * phi(R, l, xi, 3, 0); return; }
  double r[2][2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) r[a][b][c] = phi(R, l, xi, (a == 0) + (b == 0) + (c == 0), (a == 1) + (b == 1) + (c == 1));
  for (int d = 0; d < 2; ++d)
    for (int e = 0; e < 2; ++e)
      for (int f = 0; f < 2; ++f) {
        double t = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) t += Ji[a * 2 + d] * Ji[b * 2 + e] * Ji[c * 2 + f] * r[a][b][c];
        T[(d * 2 + e) * 2 + f] = t;
      }
}

// q^h(xi) on element i (Sec. 1.2)
static void eval_q(const Mesh& M, const double* Qi, const double* xi, double* q) {
  const RefElem& R = M.R;
  int V = NVAR(M);
  for (int v = 0; v < V; ++v) {
    double s = 0.0;
    for (int l = 0; l < R.ML; ++l) s += Qi[v * R.ML + l] * phi(R, l, xi);
    q[v] = s;
  }
}

// The limiter points: interior quadrature points and edge quadrature points (Sec. 3.1).
static std::vector<std::vector<double>> limiter_points(const RefElem& R) {
  std::vector<std::vector<double>> pts;
  for (int m = 0; m < R.NI; ++m) {
    std::vector<double> x(3, 0.0);
    for (int a = 0; a < R.dim; ++a) x[a] = R.xi_int[m * R.dim + a];
    pts.push_back(x);
  }
  for (int k = 0; k < R.K; ++k)
    for (int j = 0; j < R.NQE; ++j) {
      double xi[3] = {0, 0, 0};
      edge_point(R, k, j, xi);
      pts.push_back({xi[0], xi[1], xi[2]});
    }
  return pts;
}

// Moment limiter of Sec. 3.1 for one element (Steps 0-2).  Returns theta and scales modes l>=2.
//  Step 0 reading: a cell whose average density is below eps0 (the flux limiter only guarantees
//  rho_bar >= 0) or whose average pressure is not positive is flattened (theta = 0).
//  Step 1: theta^rho = largest theta in [0,1] with rho_bar + theta*rho~_m >= eps0 at all points;
//  the closed form is (rho_bar - eps0)/(rho_bar - rho_m) over the points with rho_m < eps0.
//  Step 2 reading: pressure target eps_p = min(eps0, p_bar); by concavity of p in theta,
//  theta_m = theta^rho if p(q_bar + theta^rho q~_m) >= eps_p, otherwise
//  theta^rho (p_bar - eps_p)/(p_bar - p(q_bar + theta^rho q~_m)); theta = min_m theta_m.
//  Exact variant (the paper notes the optimal theta could be computed at the cost of more
//  arithmetic): along the segment q(s) = q_bar + s D, D = q(theta^rho) - q_bar, the function
//  g(s) = rho (p - eps_p) = (gamma-1)(E rho - |M|^2/2) - eps_p rho is the quadratic A s^2 + B s + C,
//    A = (gamma-1)(D_E D_rho - |D_M|^2/2),
//    B = (gamma-1)(D_E rho_bar + E_bar D_rho - D_M . M_bar) - eps_p D_rho,
//    C = (gamma-1)(E_bar rho_bar - |M_bar|^2/2) - eps_p rho_bar,
//  (the paper's a_m, b_m and c of the quadratic in theta, shifted by the target eps_p) is
//  non-negative at s = 0 and negative at s = 1; its root in (0, 1) is taken in the
//  cancellation-free form s* = 2C / (-B + sqrt(B^2 - 4AC)) (s* = 0 when C <= 0) and moved inside
//  by a relative 1e-10, so that p(q(s)) >= eps_p holds in floating point with a margin; where
//  that check still fails the concavity value is kept.  theta_m = theta^rho max(s_c, s).
static double exact_segment_root(int dim, double gam, const double* qbar, const double* qt, double eps_p,
                                 double s_c) {
  const int V = dim + 2;
  double D[5];
  for (int v = 0; v < V; ++v) D[v] = qt[v] - qbar[v];
  const double gm1 = gam - 1.0;
  double dMdM = 0.0, dMM = 0.0, MM = 0.0;
  for (int d = 0; d < dim; ++d) {
    dMdM += D[1 + d] * D[1 + d];
    dMM += D[1 + d] * qbar[1 + d];
    MM += qbar[1 + d] * qbar[1 + d];
  }
  const double A = gm1 * (D[V - 1] * D[0] - 0.5 * dMdM);
  const double B = gm1 * (D[V - 1] * qbar[0] + qbar[V - 1] * D[0] - dMM) - eps_p * D[0];
  const double C = gm1 * (qbar[V - 1] * qbar[0] - 0.5 * MM) - eps_p * qbar[0];
  double sr = 0.0;
  if (C > 0.0) {
    const double den = -B + std::sqrt(std::max(B * B - 4.0 * A * C, 0.0));
    sr = den > 0.0 ? 2.0 * C / den : 1.0;
  }
  sr = std::min(sr, 1.0) * (1.0 - 1e-10);
  double q[5];
  for (int v = 0; v < V; ++v) q[v] = qbar[v] + sr * D[v];
  if (!(q[0] > 0.0) || !(pressure(dim, gam, q) >= eps_p)) return s_c;
  return std::max(s_c, sr);
}

static double moment_limit(const Mesh& M, const Params& P, double* Qi) {
  const RefElem& R = M.R;
  int V = NVAR(M), ML = R.ML, dim = R.dim;
  double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int v = 0; v < V; ++v) qbar[v] = Qi[v * ML + 0];
  double rbar = qbar[0];
  double pbar = pressure(dim, P.gamma, qbar);
  double theta;
  if (!(rbar >= P.eps0) || !(pbar > 0.0)) {
    theta = 0.0;
  } else {
    auto pts = limiter_points(R);
    std::vector<std::vector<double>> dev;  // q~_m
    for (auto& x : pts) {
      double q[5];
      eval_q(M, Qi, x.data(), q);
      std::vector<double> d(V);
      for (int v = 0; v < V; ++v) d[v] = q[v] - qbar[v];
      dev.push_back(d);
    }
    double th_rho = 1.0;
    for (auto& d : dev) {
      double rm = rbar + d[0];
      if (rm < P.eps0) th_rho = std::min(th_rho, (rbar - P.eps0) / (rbar - rm));
    }
    double eps_p = std::min(P.eps0, pbar);
    theta = th_rho;
    for (auto& d : dev) {
      double qt[5];
      for (int v = 0; v < V; ++v) qt[v] = qbar[v] + th_rho * d[v];
      double pt = pressure(dim, P.gamma, qt);
      double thm = th_rho;
      if (pt < eps_p) {
        const double s_c = (pbar - eps_p) / (pbar - pt);
        thm = P.exact_theta ? th_rho * exact_segment_root(dim, P.gamma, qbar, qt, eps_p, s_c) : th_rho * s_c;
      }
      theta = std::min(theta, thm);
    }
  }
  if (theta < 1.0)
    for (int v = 0; v < V; ++v)
      for (int l = 1; l < ML; ++l) Qi[v * ML + l] *= theta;
  return theta;
}

// |u| + c at a state (rho > 0, p > 0 assumed by the caller).
static double wave_speed(int dim, double gam, const double* q) {
  double rho = q[0];
  double p = pressure(dim, gam, q);
  double u2 = 0.0;
  for (int d = 0; d < dim; ++d) u2 += (q[1 + d] / rho) * (q[1 + d] / rho);
  return std::sqrt(u2) + std::sqrt(gam * p / rho);
}

// Boundary operator of Sec. 2.4 on a state or on a time derivative of it: tangential momentum
// kept, normal momentum kept (transparent) or negated (reflective).  nhat is the unit normal.
static void bc_reflect(int dim, const double* q, const double* nhat, double* out) {
  int V = dim + 2;
  for (int v = 0; v < V; ++v) out[v] = q[v];
  if (dim == 1) { out[1] = -q[1]; return; }
  double mn = 0.0;
  for (int d = 0; d < dim; ++d) mn += q[1 + d] * nhat[d];
  for (int d = 0; d < dim; ++d) out[1 + d] = q[1 + d] - 2.0 * mn * nhat[d];
}

// F_T of Eq. (taylor3-flux) from q, q_t, q_tt at a point (chain rule for F_t and F_tt).
static void ft_from_derivs(int dim, double gam, double dt, const double* q, const double* qt,
                           const double* qtt, double* FT /* dim x V */) {
  int V = dim + 2;
  for (int d = 0; d < dim; ++d) {
    double F[5], Ft[5], H[5], Aqtt[5];
    euler_flux<double>(dim, gam, q, d, F);
    flux_jvp(dim, gam, q, d, qt, Ft);
    flux_hvp(dim, gam, q, d, qt, qt, H);
    flux_jvp(dim, gam, q, d, qtt, Aqtt);
    for (int v = 0; v < V; ++v)
      FT[d * V + v] = F[v] + 0.5 * dt * Ft[v] + (dt * dt / 6.0) * (H[v] + Aqtt[v]);
  }
}

// Degree 3: the time-averaged flux to fourth order (Sec. 2.2, the Taylor series one term further),
//   F_T = F + dt/2 F_t + dt^2/6 F_tt + dt^3/24 F_ttt,
//   F_ttt = F^(3)(q_t, q_t, q_t) + 3 H(q_t, q_tt) + A q_ttt.
static void ft4_from_derivs(int dim, double gam, double dt, const double* q, const double* qt,
                            const double* qtt, const double* qttt, double* FT /* dim x V */) {
  int V = dim + 2;
  for (int d = 0; d < dim; ++d) {
    double F[5], Ft[5], H[5], Aqtt[5], T3[5], H2[5], Aqttt[5];
    euler_flux<double>(dim, gam, q, d, F);
    flux_jvp(dim, gam, q, d, qt, Ft);
    flux_hvp(dim, gam, q, d, qt, qt, H);
    flux_jvp(dim, gam, q, d, qtt, Aqtt);
    flux_3vp(dim, gam, q, d, qt, qt, qt, T3);
    flux_hvp(dim, gam, q, d, qt, qtt, H2);
    flux_jvp(dim, gam, q, d, qttt, Aqttt);
    for (int v = 0; v < V; ++v)
      FT[d * V + v] = F[v] + 0.5 * dt * Ft[v] + (dt * dt / 6.0) * (H[v] + Aqtt[v]) +
                      (dt * dt * dt / 24.0) * (T3[v] + 3.0 * H2[v] + Aqttt[v]);
  }
}

struct Trace {  // per element, local edge, edge point: q and its time derivatives, F_T (dim x V)
  double q[5], qt[5], qtt[5], qttt[5], FT[15];
};

// The shock-capturing limiter (Sec. 1.5 Step 5, Sec. 4.1).  The paper cites this limiter but does
// not define it; the reading implemented here works on the primitive variables w in
// {rho, u, (v, w), p}, with relaxation delta = alpha0 h^1.5 (alpha0 = 500; h = Delta x in 1D,
// sqrt|T| on quads, sqrt(2|T|) on triangles, cbrt(6|T|) on tetrahedra: the lattice spacing of
// the split square and cube).  Bounds: M_w = max(w_bar_i + delta, max over edge
// neighbours of w_bar_j), m_w = min(w_bar_i - delta, min_j w_bar_j); neighbour averages across
// boundary edges are the boundary operator applied to the own average.  theta^w shrinks the
// deviation from w_bar_i at the limiter points so that the extremes meet the bounds; velocity and
// pressure are only sampled at points with positive density.  theta = min_w theta^w scales
// modes l >= 2.  It runs on the updated state, before the next step's moment limiter.
static double shock_limit(const Solver& S, const std::vector<double>& Qold, int i, double* Qi) {
  const Mesh& M = *S.M;
  const RefElem& R = M.R;
  int V = NVAR(M), ML = R.ML, dim = R.dim, K = R.K;
  double gam = S.P.gamma;
  auto prim = [&](const double* q, double* w) {  // (rho, u[, v], p)
    w[0] = q[0];
    for (int d = 0; d < dim; ++d) w[1 + d] = q[1 + d] / q[0];
    w[dim + 1] = pressure(dim, gam, q);
  };
  double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int v = 0; v < V; ++v) qbar[v] = Qi[v * ML];
  if (!(qbar[0] >= S.P.eps0) || !(pressure(dim, gam, qbar) > 0.0)) return 1.0;
  double wbar[5];
  prim(qbar, wbar);
  double h = (R.kind == LINE) ? M.area[i]
             : (R.kind == QUAD ? std::sqrt(M.area[i])
                               : (R.kind == TET ? std::cbrt(6.0 * M.area[i]) : std::sqrt(2.0 * M.area[i])));
  double delta = S.P.alpha0 * std::pow(h, 1.5);
  double Mx[5], Mn[5];
  for (int w = 0; w < V; ++w) { Mx[w] = wbar[w] + delta; Mn[w] = wbar[w] - delta; }
  for (int k = 0; k < K; ++k) {
    double qn[5];
    int j = M.nbr[i * K + k];
    if (j >= 0) {
      for (int v = 0; v < V; ++v) qn[v] = Qold[(size_t)j * V * ML + v * ML];
    } else {
      int bc = M.ebc[i * K + k];
      int e = M.eid[i * K + k];
      double nh[3] = {M.e_n[3 * e] / M.e_len[e], M.e_n[3 * e + 1] / M.e_len[e], M.e_n[3 * e + 2] / M.e_len[e]};
      if (bc == BC_REFLECTIVE) bc_reflect(dim, qbar, nh, qn);
      else if (bc == BC_INFLOW) for (int v = 0; v < V; ++v) qn[v] = (dim == 1 && v == 2) ? S.P.inflow[3] : S.P.inflow[v];
      else for (int v = 0; v < V; ++v) qn[v] = qbar[v];
    }
    double wn[5];
    prim(qn, wn);
    for (int w = 0; w < V; ++w) { Mx[w] = std::max(Mx[w], wn[w]); Mn[w] = std::min(Mn[w], wn[w]); }
  }
  double wmax[5], wmin[5];
  for (int w = 0; w < V; ++w) { wmax[w] = wbar[w]; wmin[w] = wbar[w]; }
  for (auto& x : limiter_points(R)) {
    double q[5], wv[5];
    eval_q(M, Qi, x.data(), q);
    wmax[0] = std::max(wmax[0], q[0]); wmin[0] = std::min(wmin[0], q[0]);
    if (q[0] > 0.0) {
      prim(q, wv);
      for (int w = 1; w < V; ++w) { wmax[w] = std::max(wmax[w], wv[w]); wmin[w] = std::min(wmin[w], wv[w]); }
    }
  }
  double theta = 1.0;
  for (int w = 0; w < V; ++w) {
    if (wmax[w] > Mx[w]) theta = std::min(theta, (Mx[w] - wbar[w]) / (wmax[w] - wbar[w]));
    if (wmin[w] < Mn[w]) theta = std::min(theta, (wbar[w] - Mn[w]) / (wbar[w] - wmin[w]));
  }
  theta = std::max(0.0, std::min(1.0, theta));
  if (theta < 1.0)
    for (int v = 0; v < V; ++v)
      for (int l = 1; l < ML; ++l) Qi[v * ML + l] *= theta;
  return theta;
}

// Largest mu in [0,1] with p(qL + mu (qa - qL)) >= eps_p and positive density (Sec. 3.3 Step 5b).
// Along the segment, (gamma-1)(rho E - |M|^2/2) - eps_p rho is the quadratic a mu^2 + b mu + c
// with c = rho_L (p_L - eps_p) >= 0; its first crossing of zero is 2c / (-b + sqrt(b^2 - 4ac)).
// The root is then stepped down by ulps until the condition holds in floating point.
static double mu_solve(int dim, double gam, double eps_p, const double* qL, const double* qa) {
  int V = dim + 2;
  auto ok = [&](double mu) {
    double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) q[v] = qL[v] + mu * (qa[v] - qL[v]);
    return q[0] > 0.0 && pressure(dim, gam, q) >= eps_p;
  };
  if (ok(1.0)) return 1.0;
  double d[5];
  for (int v = 0; v < V; ++v) d[v] = qa[v] - qL[v];
  double mL2 = 0.0, mLd = 0.0, dd2 = 0.0;
  for (int k = 1; k <= dim; ++k) { mL2 += qL[k] * qL[k]; mLd += qL[k] * d[k]; dd2 += d[k] * d[k]; }
  int iE = dim + 1;
  double a = (gam - 1.0) * (d[0] * d[iE] - 0.5 * dd2);
  double b = (gam - 1.0) * (qL[0] * d[iE] + d[0] * qL[iE] - mLd) - eps_p * d[0];
  double c = (gam - 1.0) * (qL[0] * qL[iE] - 0.5 * mL2) - eps_p * qL[0];
  if (!(c > 0.0)) return 0.0;
  // The target is the LxF corner's own pressure (p(q^LxF) <= eps0): c vanishes in exact
  // arithmetic, g(mu) = mu (a mu + b), and with b <= 0 no mu > 0 keeps p >= eps_p; c > 0 here
  // is rounding, and the ulp search below would only end at 0.
  if (b <= 0.0 && pressure(dim, gam, qL) <= eps_p) return 0.0;
  double disc = std::max(0.0, b * b - 4.0 * a * c);
  double den = -b + std::sqrt(disc);
  double mu = (den > 0.0) ? 2.0 * c / den : 0.0;
  mu = std::min(1.0, std::max(0.0, mu));
  for (int it = 0; it < 64 && mu > 0.0 && !ok(mu); ++it) mu = std::nextafter(mu, 0.0);
  if (!ok(mu)) mu = 0.0;
  return mu;
}

static int set_err(Solver& S, int code, int elem, const char* msg) {
  if (S.err_elem < 0) {
    S.err_elem = elem;
    char buf[256];
    snprintf(buf, sizeof buf, "%s (element %d)", msg, elem);
    S.err = buf;
  }
  return code;
}

// One LxW-DG step to min(t + dt_CFL, T).  Returns a status code.
static int step(Solver& S, double T) {
  Mesh& M = *S.M;
  const RefElem& R = M.R;
  const int N = M.N, V = NVAR(M), ML = R.ML, K = R.K, dim = R.dim, NQE = R.NQE, NI = R.NI;
  const double gam = S.P.gamma;
  const size_t QS = (size_t)V * ML;
  S.err_elem = -1; S.err.clear();
  // threads only where the loops are long enough to pay for them (results do not depend on it);
  // a tetrahedron's step costs about 30 times a triangle's
  const bool par = N >= (dim == 3 ? 64 : 4096);
  (void)par;
  for (double x : S.Q)
    if (!std::isfinite(x)) return set_err(S, ERR_NONFINITE, -1, "non-finite state");

  // ---- Element loop, Step 1: moment limiter (Sec. 3.1) -------------------------------------
  S.theta_mom.assign(N, 1.0);
  int bad = -1;
#pragma omp parallel for schedule(static) if (par)
  for (int i = 0; i < N; ++i) {
    double* Qi = &S.Q[i * QS];
    double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) qbar[v] = Qi[v * ML];
    if (!(qbar[0] > 0.0) || !(pressure(dim, gam, qbar) > 0.0)) {
#pragma omp critical
      if (bad < 0 || i < bad) bad = i;
    }
    S.theta_mom[i] = moment_limit(M, S.P, Qi);
  }
  if (bad >= 0) return set_err(S, ERR_POSITIVITY, bad, "cell average density or pressure not positive");
  S.Qlim = S.Q;

  // ---- Global wave speed s and the time step (reading of Sec. 4.1: CFL 0.08 means
  //      dt * s * max_i |dT_i| / (2|T_i|) = CFL; the last step is clipped to reach T).  s is the
  //      largest |u| + c over the cell averages and every limited point, or over the cell
  //      averages only when s_avg is set -------------------------------------------------------
  auto pts = limiter_points(R);
  double s = 0.0, geo = 0.0;
#pragma omp parallel for reduction(max : s, geo) schedule(static) if (par)
  for (int i = 0; i < N; ++i) {
    const double* Qi = &S.Q[i * QS];
    double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) qbar[v] = Qi[v * ML];
    double si = wave_speed(dim, gam, qbar);
    if (!S.P.s_avg) for (auto& x : pts) {
      double q[5];
      eval_q(M, Qi, x.data(), q);
      si = std::max(si, wave_speed(dim, gam, q));
    }
    s = std::max(s, si);
    geo = std::max(geo, M.perim[i] / (2.0 * M.area[i]));
  }
  double dt = S.P.cfl / (s * geo);
  if (S.t + dt > T) dt = T - S.t;
  S.s = s; S.dt = dt;

  // ---- Element loop, Step 2: time-averaged flux F_T at every quadrature point --------------
  // Sec. 2.3 Step 1: project F(q^h) onto the basis with the interior rule (normalised weights).
  // Sec. 2.3 Step 2: from q^h and F^h form q, grad q, D = div F^h, grad D, then (Sec. 2.2)
  //   q_t = -D, F_t = A q_t, q_tt = sum_d [H_d(d_d q, D) + A_d d_d D], F_tt = H(q_t,q_t) + A q_tt,
  //   F_T = F + dt/2 F_t + dt^2/6 F_tt.
  // Sec. 2.3 Step 3 (signs from integrating by parts, which the printed Eq. (EulerStepExact)
  // has flipped; the printed cell-average update fixes them): the volume term
  //   V_l = (1/|T|) int grad phi_l . F_T  ~  sum_m w_m grad phi_l(x_m) . F_T(x_m).
  std::vector<Trace> tr((size_t)N * K * NQE);
  S.Vol.assign((size_t)N * QS, 0.0);
  S.qderiv.assign((size_t)N * NI * 3 * V, 0.0);
#pragma omp parallel for schedule(static) if (par)
  for (int i = 0; i < N; ++i) {
    const double* Qi = &S.Q[i * QS];
    double Fh[3][5][10];
    for (int d = 0; d < dim; ++d)
      for (int v = 0; v < V; ++v)
        for (int l = 0; l < ML; ++l) Fh[d][v][l] = 0.0;
    for (int m = 0; m < NI; ++m) {
      const double* xi = &R.xi_int[m * dim];
      double q[5];
      eval_q(M, Qi, xi, q);
      for (int d = 0; d < dim; ++d) {
        double F[5];
        euler_flux<double>(dim, gam, q, d, F);
        for (int v = 0; v < V; ++v)
          for (int l = 0; l < ML; ++l) Fh[d][v][l] += R.w_int[m] * F[v] * phi(R, l, xi);
      }
    }
    auto at_point = [&](const double* xi, double* q, double* qt, double* qtt, double* qttt, double* FT) {
      double dq[3][5], D[5], dD[3][5];
      eval_q(M, Qi, xi, q);
      for (int v = 0; v < V; ++v) {
        for (int a = 0; a < dim; ++a) { dq[a][v] = 0.0; dD[a][v] = 0.0; }
        D[v] = 0.0;
      }
      for (int l = 0; l < ML; ++l) {
        double g[3], H[9];
        grad_phi(M, i, l, xi, g);
        hess_phi(M, i, l, xi, H);
        for (int v = 0; v < V; ++v) {
          for (int a = 0; a < dim; ++a) dq[a][v] += Qi[v * ML + l] * g[a];
          for (int d = 0; d < dim; ++d) {
            D[v] += Fh[d][v][l] * g[d];
            for (int a = 0; a < dim; ++a) dD[a][v] += Fh[d][v][l] * H[d * dim + a];
          }
        }
      }
      for (int v = 0; v < V; ++v) qt[v] = -D[v];
      for (int v = 0; v < V; ++v) qtt[v] = 0.0;
      for (int d = 0; d < dim; ++d) {
        double h[5], a[5];
        flux_hvp(dim, gam, q, d, dq[d], D, h);
        flux_jvp(dim, gam, q, d, dD[d], a);
        for (int v = 0; v < V; ++v) qtt[v] += h[v] + a[v];
      }
      if (R.deg != 3) {
        for (int v = 0; v < V; ++v) qttt[v] = 0.0;
        ft_from_derivs(dim, gam, dt, q, qt, qtt, FT);
        return;
      }
      // Degree 3 (the same chain rule one derivative further):
      //   q_ttt = -sum_d d_d F_tt,d = -sum_d [F3_d(d_d q, q_t, q_t) + 2 H_d(d_d q_t, q_t)
      //                                       + H_d(d_d q, q_tt) + A_d d_d q_tt],
      //   d_e q_t = -d_e D,
      //   d_e q_tt = sum_d [F3_d(d_e q, d_d q, D) + H_d(d_e d_d q, D) + H_d(d_d q, d_e D)
      //                     + H_d(d_e q, d_d D) + A_d d_e d_d D],
      // with the Hessian of q and that of D = div F^h (third derivatives of F^h).
      double Hq[2][2][4], HD[2][2][4];
      for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b)
          for (int v = 0; v < V; ++v) { Hq[a][b][v] = 0.0; HD[a][b][v] = 0.0; }
      for (int l = 0; l < ML; ++l) {
        double H[4], T3[8];
        hess_phi(M, i, l, xi, H);
        d3_phi(M, i, l, xi, T3);
        for (int v = 0; v < V; ++v)
          for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
              Hq[a][b][v] += Qi[v * ML + l] * H[a * dim + b];
              for (int d = 0; d < dim; ++d) HD[a][b][v] += Fh[d][v][l] * T3[(d * dim + a) * dim + b];
            }
      }
      double dqtt[2][4];
      for (int e = 0; e < dim; ++e) {
        for (int v = 0; v < V; ++v) dqtt[e][v] = 0.0;
        for (int d = 0; d < dim; ++d) {
          double t1[4], t2[4], t3[4], t4[4], t5[4];
          flux_3vp(dim, gam, q, d, dq[e], dq[d], D, t1);
          flux_hvp(dim, gam, q, d, Hq[e][d], D, t2);
          flux_hvp(dim, gam, q, d, dq[d], dD[e], t3);
          flux_hvp(dim, gam, q, d, dq[e], dD[d], t4);
          flux_jvp(dim, gam, q, d, HD[e][d], t5);
          for (int v = 0; v < V; ++v) dqtt[e][v] += t1[v] + t2[v] + t3[v] + t4[v] + t5[v];
        }
      }
      for (int v = 0; v < V; ++v) qttt[v] = 0.0;
      for (int d = 0; d < dim; ++d) {
        double dqt[4], t1[4], t2[4], t3[4], t4[4];
        for (int v = 0; v < V; ++v) dqt[v] = -dD[d][v];
        flux_3vp(dim, gam, q, d, dq[d], qt, qt, t1);
        flux_hvp(dim, gam, q, d, dqt, qt, t2);
        flux_hvp(dim, gam, q, d, dq[d], qtt, t3);
        flux_jvp(dim, gam, q, d, dqtt[d], t4);
        for (int v = 0; v < V; ++v) qttt[v] -= t1[v] + 2.0 * t2[v] + t3[v] + t4[v];
      }
      ft4_from_derivs(dim, gam, dt, q, qt, qtt, qttt, FT);
    };
    double* Vi = &S.Vol[i * QS];
    for (int m = 0; m < NI; ++m) {
      const double* xi = &R.xi_int[m * dim];
      double q[5], qt[5], qtt[5], qttt[5], FT[15];
      at_point(xi, q, qt, qtt, qttt, FT);
      for (int v = 0; v < V; ++v) {
        S.qderiv[(((size_t)i * NI + m) * 3 + 0) * V + v] = qt[v];
        S.qderiv[(((size_t)i * NI + m) * 3 + 1) * V + v] = qtt[v];
        S.qderiv[(((size_t)i * NI + m) * 3 + 2) * V + v] = qttt[v];
      }
      for (int l = 0; l < ML; ++l) {
        double g[3];
        grad_phi(M, i, l, xi, g);
        for (int v = 0; v < V; ++v) {
          double dot = 0.0;
          for (int d = 0; d < dim; ++d) dot += g[d] * FT[d * V + v];
          Vi[v * ML + l] += R.w_int[m] * dot;
        }
      }
    }
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < NQE; ++j) {
        double xi[3] = {0, 0, 0};
        edge_point(R, k, j, xi);
        Trace& T_ = tr[((size_t)i * K + k) * NQE + j];
        at_point(xi, T_.q, T_.qt, T_.qtt, T_.qttt, T_.FT);
      }
  }

  // ---- Edge loop, Step 3: F_T^* . n_e at the edge points (Eq. (LLF) with |n_e| the length),
  //      f^LxW_e = (1/2) sum omega F^*.n_e, f^LxF_e from the cell averages, Lambda_e = 1 --------
  const int E = M.E;
  std::vector<double> Fstar((size_t)E * NQE * V), fLxW((size_t)E * V), fLxF((size_t)E * V), Lam_e(E, 1.0);
#pragma omp parallel for schedule(static) if (par)
  for (int e = 0; e < E; ++e) {
    int i = M.e_i[e], ki = M.e_ki[e], j = M.e_j[e], kj = M.e_kj[e];
    const double* n = &M.e_n[3 * e];
    double len = M.e_len[e];
    double nh[3] = {n[0] / len, n[1] / len, n[2] / len};
    int bc = M.e_bc[e];
    double qbi[5], qbj[5];
    for (int v = 0; v < V; ++v) qbi[v] = S.Q[i * QS + v * ML];
    if (j >= 0) for (int v = 0; v < V; ++v) qbj[v] = S.Q[j * QS + v * ML];
    else if (bc == BC_REFLECTIVE) bc_reflect(dim, qbi, nh, qbj);
    else if (bc == BC_INFLOW) for (int v = 0; v < V; ++v) qbj[v] = (dim == 1 && v == 2) ? S.P.inflow[3] : S.P.inflow[v];
    else for (int v = 0; v < V; ++v) qbj[v] = qbi[v];
    for (int jj = 0; jj < NQE; ++jj) {
      const Trace& Tm = tr[((size_t)i * K + ki) * NQE + jj];
      double qp[5], FTp[15];
      if (j >= 0) {
        const Trace& Tp = tr[((size_t)j * K + kj) * NQE + M.finv[((size_t)j * K + kj) * NQE + jj]];
        for (int v = 0; v < V; ++v) qp[v] = Tp.q[v];
        for (int x = 0; x < dim * V; ++x) FTp[x] = Tp.FT[x];
      } else if (bc == BC_REFLECTIVE) {
        double qt[5], qtt[5], qttt[5];
        bc_reflect(dim, Tm.q, nh, qp);
        bc_reflect(dim, Tm.qt, nh, qt);
        bc_reflect(dim, Tm.qtt, nh, qtt);
        if (R.deg == 3) {
          bc_reflect(dim, Tm.qttt, nh, qttt);
          ft4_from_derivs(dim, gam, dt, qp, qt, qtt, qttt, FTp);
        } else {
          ft_from_derivs(dim, gam, dt, qp, qt, qtt, FTp);
        }
      } else if (bc == BC_INFLOW) {
        double z[5] = {0, 0, 0, 0, 0};
        for (int v = 0; v < V; ++v) qp[v] = qbj[v];
        if (R.deg == 3) ft4_from_derivs(dim, gam, dt, qp, z, z, z, FTp);
        else ft_from_derivs(dim, gam, dt, qp, z, z, FTp);
      } else {
        for (int v = 0; v < V; ++v) qp[v] = Tm.q[v];
        for (int x = 0; x < dim * V; ++x) FTp[x] = Tm.FT[x];
      }
      double* fs = &Fstar[((size_t)e * NQE + jj) * V];
      for (int v = 0; v < V; ++v) {
        double nFp = 0.0, nFm = 0.0;
        for (int d = 0; d < dim; ++d) { nFp += n[d] * FTp[d * V + v]; nFm += n[d] * Tm.FT[d * V + v]; }
        fs[v] = 0.5 * (nFp + nFm) - 0.5 * s * len * (qp[v] - Tm.q[v]);
      }
    }
    for (int v = 0; v < V; ++v) {
      double acc = 0.0;
      for (int jj = 0; jj < NQE; ++jj) acc += R.om_edge[jj] * Fstar[((size_t)e * NQE + jj) * V + v];
      fLxW[e * V + v] = 0.5 * acc;
    }
    double Fi[5], Fj[5];
    for (int v = 0; v < V; ++v) fLxF[e * V + v] = 0.0;
    for (int d = 0; d < dim; ++d) {
      euler_flux<double>(dim, gam, qbi, d, Fi);
      euler_flux<double>(dim, gam, qbj, d, Fj);
      for (int v = 0; v < V; ++v) fLxF[e * V + v] += 0.5 * n[d] * (Fj[v] + Fi[v]);
    }
    for (int v = 0; v < V; ++v) fLxF[e * V + v] -= 0.5 * s * len * (qbj[v] - qbi[v]);
  }

  // ---- Element loop, Steps 4-5: the flux limiter ------------------------------------------
  // Step 4 (with eps_ik applied to every edge flux of the element, as in the printed Step 4):
  //   Gamma_i = |T_i| rho_bar_i / dt - sum_k eps_ik f^{LxF,rho}_k,
  //   Delta f_k = eps_ik (f^LxF - f^LxW)^rho_k.  Cases 1-4 of the sorted Delta f all say: every
  //   edge with Delta f_k < 0 gets Lambda_ik = min(1, Gamma_i / |sum of the negative Delta f|),
  //   the others get 1 (no sort needed).
  // Step 5 (reading: in the corner states the edges switched off keep the Lax-Friedrichs flux,
  //   so that c = 000 is the pure LxF update the text describes):
  //   q^LxF = q_bar - dt/|T| sum_k eps_ik f^LxF_k,
  //   q^c   = q_bar - dt/|T| sum_k eps_ik [alpha_k Lam_ik f^LxW_k + (1 - alpha_k Lam_ik) f^LxF_k],
  //   mu_c  = largest mu in [0,1] with positive pressure (target eps_p = min(eps0, p(q^LxF)))
  //           on mu q^c + (1 - mu) q^LxF,
  //   Lambda_{e_ik} = min(Lambda_{e_ik}, Lam_ik * min over corners with alpha_k = 1 of mu_c).
  S.Lam_ik.assign((size_t)N * K, 1.0);
  S.c_ik.assign((size_t)N * K, 1.0);
  int cfl_bad = -1;
  for (int i = 0; i < N; ++i) {
    double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) qbar[v] = S.Q[i * QS + v * ML];
    double area = M.area[i];
    double Gam = area * qbar[0] / dt;
    double df[4], fW[4][5], fF[4][5];
    for (int k = 0; k < K; ++k) {
      int e = M.eid[i * K + k];
      double ep = M.eps[i * K + k];
      for (int v = 0; v < V; ++v) { fW[k][v] = ep * fLxW[e * V + v]; fF[k][v] = ep * fLxF[e * V + v]; }
      Gam -= fF[k][0];
      df[k] = fF[k][0] - fW[k][0];
    }
    double Sneg = 0.0;
    for (int k = 0; k < K; ++k)
      if (df[k] < 0.0) Sneg += df[k];
    if (Gam < 0.0 && cfl_bad < 0) cfl_bad = i;
    double Lam[4];
    for (int k = 0; k < K; ++k) {
      Lam[k] = 1.0;
      if (df[k] < 0.0) Lam[k] = std::max(0.0, std::min(1.0, Gam / std::fabs(Sneg)));
      S.Lam_ik[i * K + k] = Lam[k];
    }
    double qL[5];
    for (int v = 0; v < V; ++v) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += fF[k][v];
      qL[v] = qbar[v] - dt / area * acc;
    }
    double pL = (qL[0] > 0.0) ? pressure(dim, gam, qL) : -1.0;
    if (!(pL > 0.0) && cfl_bad < 0) cfl_bad = i;
    double eps_p = std::min(S.P.eps0, pL);
    double mmin[4] = {1.0, 1.0, 1.0, 1.0};
    for (int a = 1; a < (1 << K); ++a) {
      double qa[5];
      for (int v = 0; v < V; ++v) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
          double th = ((a >> k) & 1) ? Lam[k] : 0.0;
          acc += th * fW[k][v] + (1.0 - th) * fF[k][v];
        }
        qa[v] = qbar[v] - dt / area * acc;
      }
      double mu = (pL > 0.0) ? mu_solve(dim, gam, eps_p, qL, qa) : 0.0;
      for (int k = 0; k < K; ++k)
        if ((a >> k) & 1) mmin[k] = std::min(mmin[k], mu);
    }
    for (int k = 0; k < K; ++k) {
      double c = Lam[k] * mmin[k];
      S.c_ik[i * K + k] = c;
      int e = M.eid[i * K + k];
      Lam_e[e] = std::min(Lam_e[e], c);
    }
  }
  if (cfl_bad >= 0) return set_err(S, ERR_CFL, cfl_bad, "Lax-Friedrichs update not positive (time step too large)");
  if (S.P.force_theta >= 0.0)
    for (int e = 0; e < E; ++e) Lam_e[e] = S.P.force_theta;

  // ---- Element loop, Step 6: update ---------------------------------------------------------
  //   Q^(1) -= dt/|T| sum_k eps_ik [theta_k f^LxW + (1 - theta_k) f^LxF],  theta_k = Lambda_{e_ik}
  //   Q^(l) += dt V_l - dt/|T| sum_k eps_ik (1/2) sum_j omega_j phi_l(x_kj) F^*_kj . n_e,  l >= 2
  //   (the higher moments use the unblended flux, as printed).
  S.fLxW_ik.assign((size_t)N * K * V, 0.0);
  S.fLxF_ik.assign((size_t)N * K * V, 0.0);
  S.Lam_e_ik.assign((size_t)N * K, 1.0);
  std::vector<double> Qnew(S.Q.size());
#pragma omp parallel for schedule(static) if (par)
  for (int i = 0; i < N; ++i) {
    const double* Qi = &S.Q[i * QS];
    double* Qn = &Qnew[i * QS];
    double area = M.area[i];
    for (size_t x = 0; x < QS; ++x) Qn[x] = Qi[x];
    for (int k = 0; k < K; ++k) {
      int e = M.eid[i * K + k];
      double ep = M.eps[i * K + k];
      double th = Lam_e[e];
      S.Lam_e_ik[i * K + k] = th;
      for (int v = 0; v < V; ++v) {
        S.fLxW_ik[(i * K + k) * V + v] = ep * fLxW[e * V + v];
        S.fLxF_ik[(i * K + k) * V + v] = ep * fLxF[e * V + v];
        Qn[v * ML] -= dt / area * ep * (th * fLxW[e * V + v] + (1.0 - th) * fLxF[e * V + v]);
      }
      for (int jl = 0; jl < NQE; ++jl) {
        // local point jl of element i corresponds to edge point jj in i_e's ordering
        int jj = M.fmap[((size_t)i * K + k) * NQE + jl];
        double xi[3] = {0, 0, 0};
        edge_point(R, k, jl, xi);
        for (int l = 1; l < ML; ++l) {
          double ph = phi(R, l, xi);
          for (int v = 0; v < V; ++v)
            Qn[v * ML + l] -= dt / area * ep * 0.5 * R.om_edge[jl] * ph * Fstar[((size_t)e * NQE + jj) * V + v];
        }
      }
    }
    for (int v = 0; v < V; ++v)
      for (int l = 1; l < ML; ++l) Qn[v * ML + l] += dt * S.Vol[i * QS + v * ML + l];
  }
  S.Qupd = Qnew;

  // ---- Shock-capturing limiter on the updated state ---------------------------------------
  S.theta_sc.assign(N, 1.0);
  if (S.P.shock) {
    std::vector<double> Qs = Qnew;
#pragma omp parallel for schedule(static) if (par)
    for (int i = 0; i < N; ++i)
      if (S.shock_mask.empty() || S.shock_mask[i]) S.theta_sc[i] = shock_limit(S, Qnew, i, &Qs[i * QS]);
    Qnew.swap(Qs);
  }
  S.Q.swap(Qnew);
  S.t += dt;

  // ---- Positivity of the new cell averages (guaranteed by Sec. 3.2-3.3) ---------------------
  for (int i = 0; i < N; ++i) {
    double qbar[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < V; ++v) qbar[v] = S.Q[i * QS + v * ML];
    for (int v = 0; v < V; ++v)
      if (!std::isfinite(qbar[v])) return set_err(S, ERR_NONFINITE, i, "non-finite cell average");
    if (!(qbar[0] > 0.0) || !(pressure(dim, gam, qbar) > 0.0))
      return set_err(S, ERR_POSITIVITY, i, "cell average density or pressure not positive after update");
  }
  return OK;
}

}  // namespace ora

// ==========================================================================================
// C interface for the test harness (ctypes).
// ==========================================================================================
using namespace ora;

extern "C" {

void* ora_mesh_1d(int n, double x0, double x1, int bcl, int bcr) { return mesh_1d(n, x0, x1, bcl, bcr); }
// Number of threads the element and edge loops run on.
void ora_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
int ora_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void* ora_mesh_cart(int nx, int ny, double x0, double x1, double y0, double y1, const int* bc,
                    const unsigned char* keep, int wall_bc) {
  return mesh_cart(nx, ny, x0, x1, y0, y1, bc, keep, wall_bc);
}
static std::string g_err;
void* ora_mesh_tri(int nn, const double* xy, int nt, const int* tri, const int* bnd, const double* period) {
  g_err.clear();
  return mesh_tri(nn, xy, nt, tri, bnd, period, &g_err);
}
void* ora_mesh_tet(int nn, const double* xyz, int nt, const int* tet, const int* bnd, const double* period) {
  g_err.clear();
  return mesh_tet(nn, xyz, nt, tet, bnd, period, &g_err);
}
const char* ora_last_error() { return g_err.c_str(); }
void ora_mesh_free(void* m) { delete (Mesh*)m; }

// kind, dim, N, E, ML, K, NI, NQE
void ora_mesh_info(void* m, int* out) {
  Mesh* M = (Mesh*)m;
  out[0] = M->R.kind; out[1] = M->R.dim; out[2] = M->N; out[3] = M->E;
  out[4] = M->R.ML; out[5] = M->R.K; out[6] = M->R.NI; out[7] = M->R.NQE;
}
void ora_mesh_geom(void* m, double* area, double* perim, int* nbr, int* nbr_k) {
  Mesh* M = (Mesh*)m;
  for (int i = 0; i < M->N; ++i) { area[i] = M->area[i]; perim[i] = M->perim[i]; }
  for (int x = 0; x < M->N * M->R.K; ++x) { nbr[x] = M->nbr[x]; nbr_k[x] = M->nbr_k[x]; }
}

// Edges (faces in 3D): i_e, its local index, j_e (-1 on the boundary), its local index, and n_e
// (E x 3, |n_e| the edge length or face area); the point order of every (element, local edge).
void ora_mesh_edges(void* m, int* ei, int* ki, int* ej, int* kj, double* n) {
  Mesh* M = (Mesh*)m;
  for (int e = 0; e < M->E; ++e) {
    ei[e] = M->e_i[e]; ki[e] = M->e_ki[e]; ej[e] = M->e_j[e]; kj[e] = M->e_kj[e];
    for (int a = 0; a < 3; ++a) n[3 * e + a] = M->e_n[3 * e + a];
  }
}
void ora_mesh_point_order(void* m, int* fmap) {
  Mesh* M = (Mesh*)m;
  for (size_t x = 0; x < M->fmap.size(); ++x) fmap[x] = M->fmap[x];
}

void* ora_solver_new(void* m, double gamma, double cfl, double eps0, double alpha0, int shock, const double* inflow) {
  Solver* S = new Solver;
  S->M = (Mesh*)m;
  S->P.gamma = gamma; S->P.cfl = cfl; S->P.eps0 = eps0; S->P.alpha0 = alpha0; S->P.shock = shock;
  if (inflow) for (int v = 0; v < 4; ++v) S->P.inflow[v] = inflow[v];
  S->Q.assign((size_t)S->M->N * NVAR(*S->M) * S->M->R.ML, 0.0);
  return S;
}
void ora_solver_free(void* s) { delete (Solver*)s; }
void ora_force_theta(void* s, double th) { ((Solver*)s)->P.force_theta = th; }
void ora_set_exact_theta(void* s, int on) { ((Solver*)s)->P.exact_theta = on; }
void ora_set_s_avg(void* s, int on) { ((Solver*)s)->P.s_avg = on; }
void ora_set_shock_mask(void* s, const unsigned char* mask) {
  Solver* S = (Solver*)s;
  if (mask) S->shock_mask.assign(mask, mask + S->M->N);
  else S->shock_mask.clear();
}
void ora_set_state(void* s, const double* Q, double t) {
  Solver* S = (Solver*)s;
  std::memcpy(S->Q.data(), Q, S->Q.size() * sizeof(double));
  S->t = t;
}
void ora_get_state(void* s, double* Q, double* t) {
  Solver* S = (Solver*)s;
  std::memcpy(Q, S->Q.data(), S->Q.size() * sizeof(double));
  *t = S->t;
}
int ora_step(void* s, double T, double* dt) {
  Solver* S = (Solver*)s;
  int st = step(*S, T);
  *dt = S->dt;
  return st;
}
int ora_error_elem(void* s) { return ((Solver*)s)->err_elem; }
const char* ora_error_msg(void* s) { return ((Solver*)s)->err.c_str(); }

// Intermediates of the last step.  stage: 0 Q after limiters (start of step), 1 theta_moment,
// 2 volume term, 3 f^LxW (outward, per element and local edge), 4 f^LxF, 5 Lambda_ik (density),
// 6 c_ik, 7 Lambda_e per (element, local edge), 8 Q after update before the shock limiter,
// 9 theta_shock, 10 {s, dt}, 11 q_t and q_tt at the interior points (N x NI x 2 x V).
int ora_stage(void* s, int stage, double* out) {
  Solver* S = (Solver*)s;
  const std::vector<double>* src = nullptr;
  switch (stage) {
    case 0: src = &S->Qlim; break;
    case 1: src = &S->theta_mom; break;
    case 2: src = &S->Vol; break;
    case 3: src = &S->fLxW_ik; break;
    case 4: src = &S->fLxF_ik; break;
    case 5: src = &S->Lam_ik; break;
    case 6: src = &S->c_ik; break;
    case 7: src = &S->Lam_e_ik; break;
    case 8: src = &S->Qupd; break;
    case 9: src = &S->theta_sc; break;
    case 10: out[0] = S->s; out[1] = S->dt; return 0;
    case 11: src = &S->qderiv; break;
    default: return -1;
  }
  std::memcpy(out, src->data(), src->size() * sizeof(double));
  return 0;
}

// Reference element tables, for tests: basis monomial coefficients, interior points and weights,
// edge points (reference coordinates), and basis values/derivatives at an arbitrary point.
// Polynomial degree of a mesh's elements (2 by default; 3 for lines and triangles).  Returns 0, or
// -1 for a degree the element kind does not have here.
int ora_mesh_set_degree(void* m, int deg) {
  Mesh* M = (Mesh*)m;
  if (deg != 2 && deg != 3) return -1;
  RefElem R = make_ref(M->R.kind, deg);
  if (R.ML == 0) return -1;
  M->R = R;
  build_point_order(*M);
  return 0;
}
void ora_ref_info(int kind, int deg, int* out) {
  RefElem R = make_ref(kind, deg);
  out[0] = R.dim; out[1] = R.ML; out[2] = R.K; out[3] = R.NI; out[4] = R.NQE;
}
void ora_ref_tables(int kind, int deg, double* C, double* xi_int, double* w_int, double* xi_edge, double* om_edge) {
  RefElem R = make_ref(kind, deg);
  for (size_t x = 0; x < R.C.size(); ++x) C[x] = R.C[x];
  for (size_t x = 0; x < R.xi_int.size(); ++x) xi_int[x] = R.xi_int[x];
  for (int m = 0; m < R.NI; ++m) w_int[m] = R.w_int[m];
  int c = 0;
  for (int k = 0; k < R.K; ++k)
    for (int j = 0; j < R.NQE; ++j) {
      double xi[3] = {0, 0, 0};
      edge_point(R, k, j, xi);
      for (int d = 0; d < R.dim; ++d) xi_edge[c++] = xi[d];
    }
  for (int j = 0; j < R.NQE; ++j) om_edge[j] = R.om_edge[j];
}
double ora_phi(int kind, int deg, int l, const double* xi, int da, int db, int dc) {
  static RefElem R[2][4] = {{make_ref(0), make_ref(1), make_ref(2), make_ref(3)},
                            {make_ref(0, 3), make_ref(1, 3), make_ref(2, 3), make_ref(3, 3)}};
  return phi(R[deg == 3 ? 1 : 0][kind], l, xi, da, db, dc);
}
// Third derivative of the flux applied to three vectors, and F_T to fourth order, for tests.
void ora_flux_3vp(int dim, double gam, const double* q, int d, const double* x, const double* y, const double* z,
                  double* out) {
  flux_3vp(dim, gam, q, d, x, y, z, out);
}
void ora_ft4(int dim, double gam, double dt, const double* q, const double* qt, const double* qtt, const double* qttt,
             double* FT) {
  ft4_from_derivs(dim, gam, dt, q, qt, qtt, qttt, FT);
}

// Flux, Jacobian-vector and Hessian-vector products, for tests.
void ora_flux(int dim, double gam, const double* q, int d, double* F) { euler_flux<double>(dim, gam, q, d, F); }
void ora_flux_jvp(int dim, double gam, const double* q, int d, const double* x, double* out) { flux_jvp(dim, gam, q, d, x, out); }
void ora_flux_hvp(int dim, double gam, const double* q, int d, const double* x, const double* y, double* out) {
  flux_hvp(dim, gam, q, d, x, y, out);
}
// F_T at a point from (q, q_t, q_tt), for tests.
void ora_ft(int dim, double gam, double dt, const double* q, const double* qt, const double* qtt, double* FT) {
  ft_from_derivs(dim, gam, dt, q, qt, qtt, FT);
}
double ora_mu_solve(int dim, double gam, double eps_p, const double* qL, const double* qa) {
  return mu_solve(dim, gam, eps_p, qL, qa);
}
// Moment limiter on one element's coefficients (V x ML), for tests.
double ora_moment_limit(void* s, double* Qi) {
  Solver* S = (Solver*)s;
  return moment_limit(*S->M, S->P, Qi);
}

// Shock-capturing limiter on one element's coefficients Qi (V x ML), with the neighbours' averages
// taken from Qall (N x V x ML), for tests.  Returns theta.
double ora_shock_limit(void* s, const double* Qall, int i, double* Qi) {
  Solver* S = (Solver*)s;
  const RefElem& R = S->M->R;
  std::vector<double> Q(Qall, Qall + (size_t)S->M->N * NVAR(*S->M) * R.ML);
  return shock_limit(*S, Q, i, Qi);
}

// Physical coordinates of the interior quadrature points of every element (N x NI x dim) and
// the L2 projection of point values there (N x NI x V) onto the basis (N x V x ML).
void ora_quad_points(void* m, double* xq) {
  Mesh* M = (Mesh*)m;
  const RefElem& R = M->R;
  for (int i = 0; i < M->N; ++i)
    for (int q = 0; q < R.NI; ++q) map_point(*M, i, &R.xi_int[q * R.dim], &xq[((size_t)i * R.NI + q) * R.dim]);
}
void ora_project(void* m, const double* vals, double* Q) {
  Mesh* M = (Mesh*)m;
  const RefElem& R = M->R;
  int V = NVAR(*M);
  for (int i = 0; i < M->N; ++i)
    for (int v = 0; v < V; ++v)
      for (int l = 0; l < R.ML; ++l) {
        double acc = 0.0;
        for (int q = 0; q < R.NI; ++q) acc += R.w_int[q] * vals[((size_t)i * R.NI + q) * V + v] * phi(R, l, &R.xi_int[q * R.dim]);
        Q[((size_t)i * V + v) * R.ML + l] = acc;
      }
}
// Evaluate q^h at given reference points of every element: xi (P x dim) -> out (N x P x V),
// and the physical coordinates of those points (N x P x dim).
void ora_eval(void* s, int P, const double* xi, double* out, double* x) {
  Solver* S = (Solver*)s;
  Mesh* M = S->M;
  const RefElem& R = M->R;
  int V = NVAR(*M);
  size_t QS = (size_t)V * R.ML;
  for (int i = 0; i < M->N; ++i)
    for (int p = 0; p < P; ++p) {
      eval_q(*M, &S->Q[i * QS], &xi[p * R.dim], &out[((size_t)i * P + p) * V]);
      map_point(*M, i, &xi[p * R.dim], &x[((size_t)i * P + p) * R.dim]);
    }
}

}  // extern "C"
