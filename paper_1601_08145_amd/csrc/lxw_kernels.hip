// HIP kernels (gfx950) of the positivity-preserving Lax-Wendroff DG step
// (Moe, Rossmanith, Seal, arXiv:1601.08145).
//
// One step is six launches on one stream (grid-wide dependencies separate them):
//   k_pre    per element: pending shock-capturing limiter of the previous step (Sec. 1.5 Step 5),
//            moment limiter (Sec. 3.1), cell-average checks, and the global wave speed s
//            (one partial maximum per workgroup for a single mesh; in a batch one atomic maximum
//            per wavefront and mesh);
//   k_dt     per mesh: dt = CFL / (s max_i |dT_i|/(2|T_i|)), clipped to reach T (for a single
//            mesh it first reduces the workgroup partials);
//   k_elem   per element: Galerkin projection of F (Sec. 2.3 Step 1), the time-averaged flux F_T
//            of Eq. (taylor3-flux) at every interior and edge point (Sec. 2.2, 2.3 Step 2), the
//            volume term (Sec. 2.3 Step 3) added to the higher modes, and the edge traces (each
//            side's half of Eq. (LLF), which is linear in the two sides' values);
//   k_edge   per edge: Lax-Friedrichs flux of F_T at the edge points (Eq. (LLF)), the
//            edge-averaged high-order flux f^LxW and the low-order flux f^LxF (Sec. 3.3 Step 3);
//   k_flim   per element, float64: the flux limiter of Sec. 3.3 Steps 4-5 (Gamma, Lambda_ik, the
//            corner states and the damping-factor solve mu_c), one candidate per (element, edge);
//   k_update per element: Lambda_e = min over the two sides, the blended cell-average update and
//            the higher-moment update of Sec. 3.3 Step 6, and the positivity check; the first
//            element of each mesh then ends the mesh's step (t += dt);
//   k_final  per mesh, after a state read-out applied the pending shock limiter: marks it done.
// Thread-per-element (or per-edge) mapping; reference tables sit in __constant__ memory and are
// read through the scalar cache (every lane of a wave reads the same entry).  State is stored as
// cell averages Qbar[N][V] (float64, one record per element: also gathered by neighbour index) and
// higher modes as structure-of-arrays Qh[V][ML-1][N].
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "lxw_internal.hpp"

namespace lxw {

__constant__ RefTab<ElLine, double> c_line_d;
__constant__ RefTab<ElLine, float> c_line_f;
__constant__ RefTab<ElQuad, double> c_quad_d;
__constant__ RefTab<ElQuad, float> c_quad_f;
__constant__ RefTab<ElTri, double> c_tri_d;
__constant__ RefTab<ElTri, float> c_tri_f;
__constant__ RefTab<ElLine3, double> c_line3_d;
__constant__ RefTab<ElLine3, float> c_line3_f;
__constant__ RefTab<ElTri3, double> c_tri3_d;
__constant__ RefTab<ElTri3, float> c_tri3_f;
__constant__ RefTab<ElTet, double> c_tet_d;
__constant__ RefTab<ElTet, float> c_tet_f;

template <class E, class R>
struct TabSel;
template <> struct TabSel<ElLine, double> { static __device__ __forceinline__ const RefTab<ElLine, double>& get() { return c_line_d; } };
template <> struct TabSel<ElLine, float> { static __device__ __forceinline__ const RefTab<ElLine, float>& get() { return c_line_f; } };
template <> struct TabSel<ElQuad, double> { static __device__ __forceinline__ const RefTab<ElQuad, double>& get() { return c_quad_d; } };
template <> struct TabSel<ElQuad, float> { static __device__ __forceinline__ const RefTab<ElQuad, float>& get() { return c_quad_f; } };
template <> struct TabSel<ElTri, double> { static __device__ __forceinline__ const RefTab<ElTri, double>& get() { return c_tri_d; } };
template <> struct TabSel<ElTri, float> { static __device__ __forceinline__ const RefTab<ElTri, float>& get() { return c_tri_f; } };
template <> struct TabSel<ElLine3, double> { static __device__ __forceinline__ const RefTab<ElLine3, double>& get() { return c_line3_d; } };
template <> struct TabSel<ElLine3, float> { static __device__ __forceinline__ const RefTab<ElLine3, float>& get() { return c_line3_f; } };
template <> struct TabSel<ElTri3, double> { static __device__ __forceinline__ const RefTab<ElTri3, double>& get() { return c_tri3_d; } };
template <> struct TabSel<ElTri3, float> { static __device__ __forceinline__ const RefTab<ElTri3, float>& get() { return c_tri3_f; } };
template <> struct TabSel<ElTet, double> { static __device__ __forceinline__ const RefTab<ElTet, double>& get() { return c_tet_d; } };
template <> struct TabSel<ElTet, float> { static __device__ __forceinline__ const RefTab<ElTet, float>& get() { return c_tet_f; } };

hipError_t upload_tables(const HostTabs& t) {
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_line_d), &t.line_d, sizeof(t.line_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_line_f), &t.line_f, sizeof(t.line_f));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_quad_d), &t.quad_d, sizeof(t.quad_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_quad_f), &t.quad_f, sizeof(t.quad_f));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri_d), &t.tri_d, sizeof(t.tri_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri_f), &t.tri_f, sizeof(t.tri_f));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_line3_d), &t.line3_d, sizeof(t.line3_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_line3_f), &t.line3_f, sizeof(t.line3_f));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri3_d), &t.tri3_d, sizeof(t.tri3_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tri3_f), &t.tri3_f, sizeof(t.tri3_f));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tet_d), &t.tet_d, sizeof(t.tet_d));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_tet_f), &t.tet_f, sizeof(t.tet_f));
  return e;
}

// Error codes (public values, see lxw.h).
enum { E_POSITIVITY = -5, E_NONFINITE = -6, E_CFL = -7 };

__device__ __forceinline__ void report(DevError* err, int code, int elem) {
  if (atomicCAS(&err->code, 0, code) == 0) err->elem = elem;
}

// ---------------------------------------------------------------------------------------------
// Physics.  q = (rho, M_1..M_DIM, E); F_d(q) = (M_d, M u_d + p e_d, u_d (E + p)) (Sec. 1.5) with
// p from Eq. (eos).  Jacobian and Hessian products (Eqs. (fluxderivs-a), (fluxderivs-b)) are
// written as first and second directional variations through the variations of u and p:
//   du_k = (a_Mk - u_k a_rho)/rho,  dp = (gamma-1)(a_E - u.a_M + |u|^2 a_rho / 2),
//   d2u_k = -(du_k[a] b_rho + du_k[b] a_rho)/rho,  d2p = -(gamma-1) rho du[a].du[b].
// ---------------------------------------------------------------------------------------------
template <int DIM, class R>
struct St {
  R rho, r, u[DIM], m[DIM], E, p, Ep, u2;
};

// 1/rho: in the float32 bulk the hardware reciprocal refined by one Newton-Raphson step,
// r + r (1 - x r) with the residual formed exactly by a fused multiply-add (the estimate is within
// 1 ulp; the refined value is within an ulp and almost always the correctly rounded quotient, in 3
// instructions instead of the division's 10; rho is positive and far above the denormal range
// wherever it is used), in float64 the correctly rounded quotient.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __fmaf_rn(r, __fmaf_rn(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <int DIM, class R>
__device__ __forceinline__ St<DIM, R> base_state(const R* q, R gm1) {
  St<DIM, R> s;
  s.rho = q[0];
  s.r = recip(q[0]);
  R mu = R(0), u2 = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    s.m[d] = q[1 + d];
    s.u[d] = s.m[d] * s.r;
    mu += s.m[d] * s.u[d];
    u2 += s.u[d] * s.u[d];
  }
  s.u2 = u2;
  s.E = q[DIM + 1];
  s.p = gm1 * (s.E - R(0.5) * mu);
  s.Ep = s.E + s.p;
  return s;
}

template <int DIM, class R>
struct Var {
  R du[DIM];
  R dp;
};

template <int DIM, class R>
__device__ __forceinline__ Var<DIM, R> var1(const St<DIM, R>& s, const R* a, R gm1) {
  Var<DIM, R> v;
  R t = a[DIM + 1] + R(0.5) * s.u2 * a[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    v.du[d] = (a[1 + d] - s.u[d] * a[0]) * s.r;
    t -= s.u[d] * a[1 + d];
  }
  v.dp = gm1 * t;
  return v;
}

template <int DIM, class R>
__device__ __forceinline__ void flux(const St<DIM, R>& s, int d, R* F) {
  F[0] = s.m[d];
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = s.m[k] * s.u[d] + (k == d ? s.p : R(0));
  F[DIM + 1] = s.u[d] * s.Ep;
}

// A_d a
template <int DIM, class R>
__device__ __forceinline__ void dflux(const St<DIM, R>& s, int d, const R* a, const Var<DIM, R>& va, R* F) {
  F[0] = a[1 + d];
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = a[1 + k] * s.u[d] + s.m[k] * va.du[d] + (k == d ? va.dp : R(0));
  F[DIM + 1] = va.du[d] * s.Ep + s.u[d] * (a[DIM + 1] + va.dp);
}

// H_d(a, b); d2p = -(gamma-1) rho du[a].du[b] is shared by all d and passed in.
template <int DIM, class R>
__device__ __forceinline__ void d2flux(const St<DIM, R>& s, int d, const R* a, const Var<DIM, R>& va, const R* b,
                                       const Var<DIM, R>& vb, R d2p, R* F) {
  R d2u = -(va.du[d] * b[0] + vb.du[d] * a[0]) * s.r;
  F[0] = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = a[1 + k] * vb.du[d] + b[1 + k] * va.du[d] + s.m[k] * d2u + (k == d ? d2p : R(0));
  F[DIM + 1] = d2u * s.Ep + va.du[d] * (b[DIM + 1] + vb.dp) + vb.du[d] * (a[DIM + 1] + va.dp) + s.u[d] * d2p;
}

// H_d(a, a), the same terms with the two symmetric ones gathered
template <int DIM, class R>
__device__ __forceinline__ void d2flux_sym(const St<DIM, R>& s, int d, const R* a, const Var<DIM, R>& va, R d2p, R* F) {
  const R du2 = R(2) * va.du[d];
  const R d2u = -du2 * a[0] * s.r;
  F[0] = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = a[1 + k] * du2 + s.m[k] * d2u + (k == d ? d2p : R(0));
  F[DIM + 1] = d2u * s.Ep + du2 * (a[DIM + 1] + va.dp) + s.u[d] * d2p;
}

template <int DIM, class R>
__device__ __forceinline__ R d2p_of(const St<DIM, R>& s, const Var<DIM, R>& va, const Var<DIM, R>& vb, R gm1) {
  R t = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) t += va.du[d] * vb.du[d];
  return -gm1 * s.rho * t;
}

// F_T = F + dt/2 A q_t + dt^2/6 (H(q_t, q_t) + A q_tt) for every direction d (Eq. (taylor3-flux)
// with the chain rule of Sec. 2.2; also the ghost-state flux of Sec. 2.4).  A is linear, so its two
// products are formed as one, A (dt/2 q_t + dt^2/6 q_tt).  The caller passes the state s of q and
// the variation vt of q_t (the element kernel has them from the time derivatives).
template <int DIM, class R>
__device__ __forceinline__ void ft_core(const St<DIM, R>& s, const R* qt, const Var<DIM, R>& vt, const R* qtt, R gm1,
                                        R dt, R FT[DIM][DIM + 2]) {
  constexpr int V = DIM + 2;
  const R c1 = R(0.5) * dt, c2 = dt * dt * R(1.0 / 6.0);
  R qc[V];
#pragma unroll
  for (int c = 0; c < V; ++c) qc[c] = c1 * qt[c] + c2 * qtt[c];
  const Var<DIM, R> vc = var1<DIM, R>(s, qc, gm1);
  const R d2p = d2p_of<DIM, R>(s, vt, vt, gm1);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    R F[V], A[V], H[V];
    flux<DIM, R>(s, d, F);
    dflux<DIM, R>(s, d, qc, vc, A);
    d2flux_sym<DIM, R>(s, d, qt, vt, d2p, H);
#pragma unroll
    for (int c = 0; c < V; ++c) FT[d][c] = F[c] + A[c] + c2 * H[c];
  }
}
template <int DIM, class R>
__device__ __forceinline__ void ft_from(const R* q, const R* qt, const R* qtt, R gm1, R dt, R FT[DIM][DIM + 2]) {
  const St<DIM, R> s = base_state<DIM, R>(q, gm1);
  ft_core<DIM, R>(s, qt, var1<DIM, R>(s, qt, gm1), qtt, gm1, dt, FT);
}

// n . F_T for an edge normal n (length included), from the flux along n, F_n = sum_d n_d F_d, and
// its variations (the directional formulas above summed over d with weights n_d: only u.n, M.n and
// p n enter), so an edge point forms one normal flux instead of DIM fluxes and a dot product.
template <int DIM, class R>
__device__ __forceinline__ R dot_n(const R* x, const R* n) {
  R t = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) t += x[d] * n[d];
  return t;
}
template <int DIM, class R>
__device__ __forceinline__ void ftn_core(const St<DIM, R>& s, const R* qt, const Var<DIM, R>& vt, const R* qtt,
                                         const R* n, R gm1, R dt, R* FTn) {
  constexpr int V = DIM + 2;
  const R c1 = R(0.5) * dt, c2 = dt * dt * R(1.0 / 6.0);
  R qc[V];  // one Jacobian product A_n (dt/2 q_t + dt^2/6 q_tt), as in ft_core
#pragma unroll
  for (int c = 0; c < V; ++c) qc[c] = c1 * qt[c] + c2 * qtt[c];
  const Var<DIM, R> vc = var1<DIM, R>(s, qc, gm1);
  const R d2p = d2p_of<DIM, R>(s, vt, vt, gm1);
  const R un = dot_n<DIM, R>(s.u, n), mn = dot_n<DIM, R>(s.m, n);
  const R dun = dot_n<DIM, R>(vt.du, n), dcn = dot_n<DIM, R>(vc.du, n);
  const R d2un = -R(2) * dun * qt[0] * s.r;  // (d2u[qt, qt]) . n
  R an = R(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) an += qc[1 + d] * n[d];
  // F_n + A_n qc + dt^2/6 H_n(q_t, q_t)
  FTn[0] = mn + an;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const R F = s.m[k] * un + s.p * n[k];
    const R A = qc[1 + k] * un + s.m[k] * dcn + vc.dp * n[k];
    const R H = R(2) * qt[1 + k] * dun + s.m[k] * d2un + d2p * n[k];
    FTn[1 + k] = F + A + c2 * H;
  }
  {
    const R F = un * s.Ep;
    const R A = dcn * s.Ep + un * (qc[V - 1] + vc.dp);
    const R H = d2un * s.Ep + R(2) * dun * (qt[V - 1] + vt.dp) + un * d2p;
    FTn[V - 1] = F + A + c2 * H;
  }
}
template <int DIM, class R>
__device__ __forceinline__ void ftn_from(const R* q, const R* qt, const R* qtt, const R* n, R gm1, R dt, R* FTn) {
  const St<DIM, R> s = base_state<DIM, R>(q, gm1);
  ftn_core<DIM, R>(s, qt, var1<DIM, R>(s, qt, gm1), qtt, n, gm1, dt, FTn);
}

// Degree 3: the third variation F^(3)_d(a, b, c), through the third variations of u and p (the
// first and second are those above):
//   d3u_k[a,b,c] = -(d2u_k[a,b] c_rho + d2u_k[a,c] b_rho + d2u_k[b,c] a_rho)/rho,
//   d3p[a,b,c]   = (gamma-1)(a_rho du[b].du[c] + b_rho du[a].du[c] + c_rho du[a].du[b]);
// M_k u_d picks up a_Mk d2u_d[b,c] (and its two permutations) + M_k d3u_d, and u_d (E + p) the full
// product rule with first, second and third variations a_E + dp, d2p and d3p of E + p.
template <int DIM, class R>
__device__ __forceinline__ void d3flux(const St<DIM, R>& s, int d, const R* a, const Var<DIM, R>& va, const R* b,
                                       const Var<DIM, R>& vb, const R* c, const Var<DIM, R>& vc, R gm1, R* F) {
  constexpr int V = DIM + 2;
  R ab = R(0), ac = R(0), bc = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    ab += va.du[k] * vb.du[k];
    ac += va.du[k] * vc.du[k];
    bc += vb.du[k] * vc.du[k];
  }
  const R pab = -gm1 * s.rho * ab, pac = -gm1 * s.rho * ac, pbc = -gm1 * s.rho * bc;
  const R p3 = gm1 * (a[0] * bc + b[0] * ac + c[0] * ab);
  const R uab = -(va.du[d] * b[0] + vb.du[d] * a[0]) * s.r;
  const R uac = -(va.du[d] * c[0] + vc.du[d] * a[0]) * s.r;
  const R ubc = -(vb.du[d] * c[0] + vc.du[d] * b[0]) * s.r;
  const R u3 = -(uab * c[0] + uac * b[0] + ubc * a[0]) * s.r;
  F[0] = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = a[1 + k] * ubc + b[1 + k] * uac + c[1 + k] * uab + s.m[k] * u3 + (k == d ? p3 : R(0));
  F[V - 1] = u3 * s.Ep + uab * (c[V - 1] + vc.dp) + uac * (b[V - 1] + vb.dp) + ubc * (a[V - 1] + va.dp) +
             va.du[d] * pbc + vb.du[d] * pac + vc.du[d] * pab + s.u[d] * p3;
}

// F^(3)_d(a, a, a): the terms of d3flux with the three directions equal, gathered (the three
// pairwise products are one, and each permuted sum becomes three times one term).
template <int DIM, class R>
__device__ __forceinline__ void d3flux_sym(const St<DIM, R>& s, int d, const R* a, const Var<DIM, R>& va, R gm1, R* F) {
  constexpr int V = DIM + 2;
  R aa = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) aa += va.du[k] * va.du[k];
  const R paa = -gm1 * s.rho * aa;
  const R p3 = R(3) * gm1 * a[0] * aa;
  const R uaa = -R(2) * va.du[d] * a[0] * s.r;
  const R u3 = -R(3) * uaa * a[0] * s.r;
  F[0] = R(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = R(3) * a[1 + k] * uaa + s.m[k] * u3 + (k == d ? p3 : R(0));
  F[V - 1] = u3 * s.Ep + R(3) * (uaa * (a[V - 1] + va.dp) + va.du[d] * paa) + s.u[d] * p3;
}

// Degree 3: F_T one Taylor term further, + dt^3/24 (F^(3)(q_t, q_t, q_t) + 3 H(q_t, q_tt) + A q_ttt).
// A is linear and H bilinear, so the terms are gathered as
//   F + A (c1 q_t + c2 q_tt + c3 q_ttt) + H(q_t, c2 q_t + 3 c3 q_tt) + c3 F^(3)(q_t, q_t, q_t)
// with c1 = dt/2, c2 = dt^2/6, c3 = dt^3/24: one Jacobian and one Hessian product per direction.
template <int DIM, class R>
__device__ __forceinline__ void ft4_core(const St<DIM, R>& s, const R* qt, const Var<DIM, R>& vt, const R* qtt,
                                         const R* qttt, R gm1, R dt, R FT[DIM][DIM + 2]) {
  constexpr int V = DIM + 2;
  const R c1 = R(0.5) * dt, c2 = dt * dt * R(1.0 / 6.0), c3 = dt * dt * dt * R(1.0 / 24.0);
  const R c33 = R(3) * c3;
  R qc[V], qh[V];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    qc[c] = c1 * qt[c] + c2 * qtt[c] + c3 * qttt[c];
    qh[c] = c2 * qt[c] + c33 * qtt[c];
  }
  const Var<DIM, R> vc = var1<DIM, R>(s, qc, gm1);
  const Var<DIM, R> vh = var1<DIM, R>(s, qh, gm1);
  const R d2p = d2p_of<DIM, R>(s, vt, vh, gm1);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    R F[V], A[V], H[V], T3[V];
    flux<DIM, R>(s, d, F);
    dflux<DIM, R>(s, d, qc, vc, A);
    d2flux<DIM, R>(s, d, qt, vt, qh, vh, d2p, H);
    d3flux_sym<DIM, R>(s, d, qt, vt, gm1, T3);
#pragma unroll
    for (int c = 0; c < V; ++c) FT[d][c] = F[c] + A[c] + H[c] + c3 * T3[c];
  }
}
template <int DIM, class R>
__device__ __forceinline__ void ft4_from(const R* q, const R* qt, const R* qtt, const R* qttt, R gm1, R dt,
                                         R FT[DIM][DIM + 2]) {
  const St<DIM, R> s = base_state<DIM, R>(q, gm1);
  ft4_core<DIM, R>(s, qt, var1<DIM, R>(s, qt, gm1), qtt, qttt, gm1, dt, FT);
}

// Pressure and wave speed (double, for the limiters and s).
template <int DIM>
__device__ __forceinline__ double pressure(const double* q, double gam) {
  double k = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) k += q[1 + d] * q[1 + d];
  return (gam - 1.0) * (q[DIM + 1] - 0.5 * k / q[0]);
}

template <int DIM>
__device__ __forceinline__ double wave_speed(const double* q, double gam) {
  double u2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) u2 += (q[1 + d] / q[0]) * (q[1 + d] / q[0]);
  return sqrt(u2) + sqrt(gam * pressure<DIM>(q, gam) / q[0]);
}

// Boundary operator of Sec. 2.4: keep the tangential momentum, negate the normal one.
template <int DIM, class T>
__device__ __forceinline__ void reflect(const T* q, const T* nh, T* out) {
  constexpr int V = DIM + 2;
#pragma unroll
  for (int c = 0; c < V; ++c) out[c] = q[c];
  if constexpr (DIM == 1) {
    out[1] = -q[1];
  } else if constexpr (DIM == 2) {
    T mn = q[1] * nh[0] + q[DIM] * nh[DIM - 1];
    out[1] = q[1] - T(2) * mn * nh[0];
    out[DIM] = q[DIM] - T(2) * mn * nh[DIM - 1];
  } else {
    T mn = q[1] * nh[0] + q[2] * nh[1] + q[3] * nh[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) out[1 + d] = q[1 + d] - T(2) * mn * nh[d];
  }
}

template <int DIM, class T>
__device__ __forceinline__ void inflow_state(const double* inflow, T* out) {
  if constexpr (DIM == 1) { out[0] = T(inflow[0]); out[1] = T(inflow[1]); out[2] = T(inflow[3]); }
  else if constexpr (DIM == 2) { out[0] = T(inflow[0]); out[1] = T(inflow[1]); out[DIM] = T(inflow[2]); out[DIM + 1] = T(inflow[3]); }
  else { out[0] = T(inflow[0]); out[1] = T(inflow[1]); out[2] = T(inflow[2]); out[3] = T(0); out[4] = T(inflow[3]); }  // not used: no inflow sides on tetrahedra
}

template <class R>
__device__ __forceinline__ int mesh_id(const int* mesh_of, int i) { return mesh_of ? mesh_of[i] : 0; }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Elements (and
// edges, numbered in element order) are in space-filling-curve order, so neighbouring work items
// share data; give every XCD one contiguous range of blocks (the grid is padded to a multiple of 8
// blocks) so that shared lines are reused within one L2.
__device__ __forceinline__ int xcd_item() {
  const int nb = (int)gridDim.x;  // multiple of 8
  const int b = (int)blockIdx.x;
  return ((b & 7) * (nb >> 3) + (b >> 3)) * (int)blockDim.x + (int)threadIdx.x;
}

// Per-mesh maximum of a non-negative double: wavefront reduction when the wavefront lies in one
// mesh, else one atomic per lane.
__device__ __forceinline__ void atomic_max_per_mesh(Scalars* sc, int mid, double val, bool valid) {
  int lane = threadIdx.x & 63;
  int m0 = __shfl(mid, 0);
  bool uniform = __all(!valid || mid == m0);
  if (uniform) {
    double x = valid ? val : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    if (lane == 0 && __any(valid)) atomicMax(&sc[m0].s_bits, (unsigned long long)__double_as_longlong(x));
  } else if (valid) {
    atomicMax(&sc[mid].s_bits, (unsigned long long)__double_as_longlong(val));
  }
}

// ---------------------------------------------------------------------------------------------
// k_pre: pending shock-capturing limiter, moment limiter, checks, wave speed.
//   mode 0: computes the element's total limiter factor theta = theta_shock * theta_moment and
//           stores it (k_elem applies it to the higher modes); wave speed and checks.
//   mode 1: applies only the pending shock-capturing limiter to the stored modes (state read-out).
//   mode 2: stores the pending shock-capturing limiter's factor in theta, changing nothing else
//           (training data for the learned indicator).
// With a learned indicator, elements it clears (ind_flag 0) skip the shock-capturing limiter in
// modes 0 and 1; the positivity limiter is never skipped.
// All limiter arithmetic is float64 on the stored state, evaluated as q_bar + theta sum_l Q_l phi_l,
// the same expression k_elem uses for its point states, so the positivity the limiter establishes
// holds for the states the time-averaged flux is built from.
// ---------------------------------------------------------------------------------------------
// 1/x in float64 for the limiter passes of k_pre (x a positive normal number: a point density
// checked > 0 first, or a cell average >= eps0): the hardware estimate (about 2^-23 relative) and
// two Newton-Raphson steps r <- r + r (1 - x r), each squaring the relative error, to within an ulp
// of the quotient, in 5 instructions instead of the correctly rounded division's 10.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __fma_rn(r, __fma_rn(-x, r, 1.0), r);
  return __fma_rn(r, __fma_rn(-x, r, 1.0), r);
}

template <int DIM>
__device__ __forceinline__ double pressure_r(const double* q, double r, double gam) {
  double k = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) k += q[1 + d] * q[1 + d];
  return (gam - 1.0) * (q[DIM + 1] - 0.5 * k * r);
}

// |u| + c from u2 = |u|^2 and c2 = gamma p / rho (both float64) for the global wave speed s.
// Float64 form: in float64.  FP32-mixed form: both square roots by the hardware float32 square
// root (a float64 square root, or a correctly rounded float32 one, is a sequence of a dozen
// instructions, and k_pre takes two per limiter point), the sum enlarged by a relative 2^-21 in
// float64.  The float32 rounding of u2 and c2 (2^-24 each, halved by the root), the roots (up to
// two ulp, 2^-22) and the sum (2^-24) stay below that margin for u2 and c2 within the float32
// normal range, so the result is never below the float64 value: the condition on s of the
// positivity argument (s at least the largest |u| + c) still holds.
template <class R>
__device__ __forceinline__ double speed_of(double u2, double c2) {
  if constexpr (sizeof(R) == sizeof(double)) {
    return sqrt(u2) + sqrt(c2);
  } else {
    return double(__builtin_amdgcn_sqrtf(float(u2)) + __builtin_amdgcn_sqrtf(float(c2))) * (1.0 + 0x1p-21);
  }
}

template <int DIM, class R>
__device__ __forceinline__ double speed_r(const double* q, double gam) {
  const double r = rcp_nr(q[0]);
  double u2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) u2 += (q[1 + d] * r) * (q[1 + d] * r);
  return speed_of<R>(u2, gam * pressure_r<DIM>(q, r, gam) * r);
}

// deviation of variable c from the cell average at point p, float64, from the stored modes
template <class E, class R>
__device__ __forceinline__ double point_dev(const RefTab<E, double>& T, const R (&Qh)[E::V][E::ML - 1], int p, int c) {
  double acc = 0.0;
#pragma unroll
  for (int l = 1; l < E::ML; ++l) acc += double(Qh[c][l - 1]) * T.phi[p][l];
  return acc;
}

// Exact variant of the moment limiter's pressure step (Sec. 3.1; the paper notes the optimal factor
// could be computed at the cost of more arithmetic).  Along the segment q(s) = qb + s D from the
// average to the point state at the density factor, D = q - qb, g(s) = rho (p - eps_p) =
// (gamma-1)(E rho - |M|^2/2) - eps_p rho is the quadratic A s^2 + B s + C (the paper's a_m, b_m, c
// shifted by the target eps_p), with g(0) >= 0 > g(1).  Its root in (0, 1) in the cancellation-free
// form 2C / (-B + sqrt(B^2 - 4AC)) (0 when C <= 0), moved inside by a relative 1e-10 and accepted
// only where p(q(s)) >= eps_p then holds in float64; the result is never below the concavity
// value s_c.
template <int DIM>
__device__ __forceinline__ double exact_segment(const double* qb, const double* q, double epsp, double gam, double s_c) {
  constexpr int V = DIM + 2;
  double D[V];
#pragma unroll
  for (int c = 0; c < V; ++c) D[c] = q[c] - qb[c];
  const double gm1 = gam - 1.0;
  double dMdM = 0.0, dMM = 0.0, MM = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    dMdM += D[1 + d] * D[1 + d];
    dMM += D[1 + d] * qb[1 + d];
    MM += qb[1 + d] * qb[1 + d];
  }
  const double A = gm1 * (D[V - 1] * D[0] - 0.5 * dMdM);
  const double B = gm1 * (D[V - 1] * qb[0] + qb[V - 1] * D[0] - dMM) - epsp * D[0];
  const double C = gm1 * (qb[V - 1] * qb[0] - 0.5 * MM) - epsp * qb[0];
  double sr = 0.0;
  if (C > 0.0) {
    const double den = -B + sqrt(fmax(B * B - 4.0 * A * C, 0.0));
    sr = den > 0.0 ? 2.0 * C / den : 1.0;
  }
  sr = fmin(sr, 1.0) * (1.0 - 1e-10);
  double qs[V];
#pragma unroll
  for (int c = 0; c < V; ++c) qs[c] = qb[c] + sr * D[c];
  if (!(qs[0] > 0.0) || !(pressure<DIM>(qs, gam) >= epsp)) return s_c;
  return fmax(s_c, sr);
}

// The mode is a template argument: each mode's kernel holds only its own path, so the read-out and
// collection paths do not raise the register allocation of the per-step kernel.  Modes: 0 step,
// 1 read-out (pending shock-capturing limiter applied), 2 collection (its factor recorded), 3 step
// with the exact pressure factor of the moment limiter, 4 step with the wave speed from the cell
// averages only, 5 both.
// Element i of k_pre (i may be past the last element: every lane of a wavefront takes part in the
// wave-speed reduction).
template <class E, class R, int mode>
__device__ __forceinline__ void pre_item(View<R> v, const int i) {
  constexpr int V = E::V, ML = E::ML, DIM = E::DIM, NP = E::NP, K = E::K;
  constexpr bool kStep = mode == 0 || mode >= 3;
  constexpr bool kExact = mode == 3 || mode == 5;  // exact pressure factor of the moment limiter
  constexpr bool kSavg = mode >= 4;                // wave speed from the cell averages only
  const RefTab<E, double>& T = TabSel<E, double>::get();
  const int N = v.N;
  const bool valid = i < N;
  const double gam = v.gamma, eps0 = v.eps0;
  double smax = 0.0;
  int mid = 0;
  if (valid) {
    mid = mesh_id<R>(v.mesh_of, i);
    double qb[V];
    R Qh[V][ML - 1];
#pragma unroll
    for (int c = 0; c < V; ++c) {
      qb[c] = v.Qbar[(size_t)i * V + c];
#pragma unroll
      for (int l = 0; l < ML - 1; ++l) Qh[c][l] = at(v.Qh + (size_t)(c * (ML - 1) + l) * N, i);
    }
    const double rb = rcp_nr(qb[0]);
    const double pb = pressure_r<DIM>(qb, rb, gam);
    bool finite = true;
#pragma unroll
    for (int c = 0; c < V; ++c) finite = finite && isfinite(qb[c]);
    if (kStep) {
      if (!finite) report(v.err, E_NONFINITE, i);
      else if (!(qb[0] > 0.0) || !(pb > 0.0)) report(v.err, E_POSITIVITY, i);
    }
    const bool ok = finite && qb[0] >= eps0 && pb > 0.0;

    // ---- one pass over the points of the unlimited state: the shock-capturing limiter on the
    // primitive variables (bounds from the edge neighbours' averages relaxed by alpha0 h^1.5;
    // velocity and pressure sampled where the density is positive) when it is due, and the
    // smallest point density and pressure and the largest wave speed, which settle the moment
    // limiter and the wave speed at once when nothing needs limiting
    double th_sc = 1.0;
    double rmin = INFINITY;  // smallest point density of the unlimited state
    double pmin = INFINITY;  // smallest point pressure of the unlimited state (points with rho > 0)
    double smax0 = 0.0;      // largest point wave speed of the unlimited state (points with rho > 0)
    bool have_rmin = false;
    const bool detect = mode == 2 || !v.ind_flag || at(v.ind_flag, i) != 0;
    const bool shock_on = v.shock && v.sc[mid].shock_pending && ok && detect;
    if (shock_on || (kStep && ok)) {
      have_rmin = true;
      // primitive variables of the average (formed again after the point pass, so that they are
      // not live across it)
      auto prim_avg = [&](double* w) {
        w[0] = qb[0];
#pragma unroll
        for (int d = 0; d < DIM; ++d) w[1 + d] = qb[1 + d] * rb;
        w[DIM + 1] = pb;
      };
      // the point pass before the bounds: neither the neighbour states nor the relaxed bounds are
      // live across it (fewer registers)
      double wmax[V], wmin[V];
      prim_avg(wmax);
      prim_avg(wmin);
      // a loop at run time (the table rows are scalar loads): unrolled, the point states of all
      // points were scheduled together and the kernel needed 160 registers (three waves per SIMD
      // instead of four on triangles; 1.5x the time on tetrahedra)
#pragma unroll 1
      for (int p = 0; p < NP; ++p) {
        double q[V];
#pragma unroll
        for (int c = 0; c < V; ++c) q[c] = qb[c] + point_dev<E, R>(T, Qh, p, c);
        wmax[0] = fmax(wmax[0], q[0]);
        wmin[0] = fmin(wmin[0], q[0]);
        rmin = fmin(rmin, q[0]);
        if (q[0] > 0.0) {
          const double r = rcp_nr(q[0]);
          double u2 = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const double u = q[1 + d] * r;
            wmax[1 + d] = fmax(wmax[1 + d], u);
            wmin[1 + d] = fmin(wmin[1 + d], u);
            u2 += u * u;
          }
          const double pp = pressure_r<DIM>(q, r, gam);
          wmax[DIM + 1] = fmax(wmax[DIM + 1], pp);
          wmin[DIM + 1] = fmin(wmin[DIM + 1], pp);
          pmin = fmin(pmin, pp);
          smax0 = fmax(smax0, speed_of<R>(u2, gam * pp * r));  // = speed_r of this point
        }
      }
      double wb[V], Mx[V], Mn[V];
      prim_avg(wb);
      const double dl = at(v.delta, i);
#pragma unroll
      for (int c = 0; c < V; ++c) { Mx[c] = wb[c] + dl; Mn[c] = wb[c] - dl; }
#pragma unroll
      for (int k = 0; k < K && shock_on; ++k) {
        double qn[V], wn[V];
        const int j = at(v.nbr + (size_t)k * N, i);
        if (j >= 0) {
#pragma unroll
          for (int c = 0; c < V; ++c) qn[c] = v.Qbar[(size_t)j * V + c];
        } else {
          const int bc = at(v.eslot + (size_t)k * N, i) & 3;
          if (bc == SB_REFLECTIVE) {
            double nh[DIM], len2 = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) { nh[d] = double(at(v.nout + (size_t)(k * DIM + d) * N, i)); len2 += nh[d] * nh[d]; }
            const double il = 1.0 / sqrt(len2);
#pragma unroll
            for (int d = 0; d < DIM; ++d) nh[d] *= il;
            reflect<DIM, double>(qb, nh, qn);
          } else if (bc == SB_INFLOW) {
            inflow_state<DIM, double>(v.inflow, qn);
          } else {
#pragma unroll
            for (int c = 0; c < V; ++c) qn[c] = qb[c];
          }
        }
        const double rn = rcp_nr(qn[0]);
        wn[0] = qn[0];
#pragma unroll
        for (int d = 0; d < DIM; ++d) wn[1 + d] = qn[1 + d] * rn;
        wn[DIM + 1] = pressure_r<DIM>(qn, rn, gam);
#pragma unroll
        for (int c = 0; c < V; ++c) { Mx[c] = fmax(Mx[c], wn[c]); Mn[c] = fmin(Mn[c], wn[c]); }
      }
      if (shock_on) {
#pragma unroll
        for (int c = 0; c < V; ++c) {
          if (wmax[c] > Mx[c]) th_sc = fmin(th_sc, (Mx[c] - wb[c]) / (wmax[c] - wb[c]));
          if (wmin[c] < Mn[c]) th_sc = fmin(th_sc, (wb[c] - Mn[c]) / (wb[c] - wmin[c]));
        }
        th_sc = fmax(0.0, fmin(1.0, th_sc));
      }
    }

    if (mode == 2) {
      at(v.theta, i) = th_sc;  // the factor the limiter would apply; the state is left as it is
    } else if (mode == 1) {
      if (th_sc < 1.0) {
#pragma unroll
        for (int c = 0; c < V; ++c)
#pragma unroll
          for (int l = 0; l < ML - 1; ++l) at(v.Qh + (size_t)(c * (ML - 1) + l) * N, i) = R(th_sc * double(Qh[c][l]));
      }
      if (v.dbg_theta_sc && v.shock && v.sc[mid].shock_pending) v.dbg_theta_sc[i] = th_sc;
    } else {
      // ---- moment limiter (Sec. 3.1): Step 0 flattens cells below eps0 or with p_bar <= 0;
      // Step 1 density (closed form of the largest theta); Step 2 pressure by concavity, target
      // eps_p = min(eps0, p_bar).
      // When neither the shock limiter nor the density step limits (the common case), the point
      // states of the density, pressure and wave-speed passes are the same; those passes then share
      // one loop.  Every value is computed by the same operations as in the separate passes.
      double th = 1.0;
      double smax1 = 0.0;
      bool fused = false;
      if (!ok) {
        th = 0.0;
      } else if (have_rmin && th_sc == 1.0 && rmin >= eps0 && pmin >= fmin(eps0, pb)) {
        // nothing limits: the shock pass already evaluated every point's pressure and speed
        fused = true;
        smax1 = smax0;
      } else {
        double thr = 1.0;
        if (have_rmin && th_sc == 1.0) {
          // the density factor is a decreasing function of the point density: its minimum over
          // the points is its value at the smallest point density
          if (rmin < eps0) thr = fmin(thr, (qb[0] - eps0) / (qb[0] - rmin));
        } else {
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            const double rm = qb[0] + th_sc * point_dev<E, R>(T, Qh, p, 0);
            if (rm < eps0) thr = fmin(thr, (qb[0] - eps0) / (qb[0] - rm));
          }
        }
        const double epsp = fmin(eps0, pb);
        const double ts = thr * th_sc;
        th = thr;
        fused = ts == 1.0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          double q[V];
#pragma unroll
          for (int c = 0; c < V; ++c) q[c] = qb[c] + ts * point_dev<E, R>(T, Qh, p, c);
          const double pt = pressure_r<DIM>(q, rcp_nr(q[0]), gam);
          if (pt < epsp) {
            if (kExact) th = fmin(th, thr * exact_segment<DIM>(qb, q, epsp, gam, (pb - epsp) / (pb - pt)));
            else th = fmin(th, thr * (pb - epsp) / (pb - pt));
          }
          if (fused) smax1 = fmax(smax1, speed_r<DIM, R>(q, gam));
        }
      }
      const double tt = th_sc * th;
      at(v.theta, i) = tt;
      if (finite && qb[0] > 0.0 && pb > 0.0) {
        smax = speed_r<DIM, R>(qb, gam);
        if (kSavg) {
          // the cell average's speed only
        } else if (fused && tt == 1.0) {
          smax = fmax(smax, smax1);
        } else if (tt > 0.0) {
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            double q[V];
#pragma unroll
            for (int c = 0; c < V; ++c) q[c] = qb[c] + tt * point_dev<E, R>(T, Qh, p, c);
            smax = fmax(smax, speed_r<DIM, R>(q, gam));
          }
        }
      }
      if (!isfinite(smax)) {  // fmax-based reductions would drop a NaN: report it here
        report(v.err, E_NONFINITE, i);
        smax = INFINITY;
      }
      if (v.dbg_theta) v.dbg_theta[i] = th;
      if (v.dbg_theta_sc && v.shock && v.sc[mid].shock_pending) v.dbg_theta_sc[i] = th_sc;
      if (v.dbg_qlim) {
#pragma unroll
        for (int c = 0; c < V; ++c) {
          v.dbg_qlim[(c * ML) * N + i] = qb[c];
#pragma unroll
          for (int l = 1; l < ML; ++l) v.dbg_qlim[(c * ML + l) * N + i] = tt * double(Qh[c][l - 1]);
        }
      }
    }
  }
  if (kStep) {
    if (v.mesh_of) {
      atomic_max_per_mesh(v.sc, mid, smax, valid);
    } else {
      // one partial maximum per block (k_dt reduces them): no contended atomics on one address
      __shared__ double red[4];
      double x = valid ? smax : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
      __syncthreads();
      if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        v.spart[blockIdx.x] = m;
      }
    }
  }
}

template <class E, class R, int mode>
__global__ __launch_bounds__(256) void k_pre(View<R> v) {
  constexpr bool kStep = mode == 0 || mode >= 3;
  // a single mesh at its end time: the step changes nothing (every lane leaves together)
  if (kStep && !v.mesh_of && !(v.sc[0].t < v.sc[0].T)) return;
  pre_item<E, R, mode>(v, xcd_item());
}

// ---------------------------------------------------------------------------------------------
// k_dt: per mesh, dt from the CFL condition (reading of Sec. 4.1, "CFL 0.08"), clipped to T.
// ---------------------------------------------------------------------------------------------
// Single mesh: one workgroup of 1024 lanes reduces the per-workgroup maxima of k_pre.
__global__ __launch_bounds__(1024) void k_dt_single(Scalars* sc, DevError* err, const double* spart, int nparts) {
  __shared__ double red[16];
  double x = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) x = fmax(x, spart[b]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, red[w]);
  Scalars& S = sc[0];
  S.idle = !(S.t < S.T);  // the end time is reached: this step changes nothing
  if (S.idle) return;
  S.s = s;
  if (!(s > 0.0) || !isfinite(s)) {
    report(err, E_NONFINITE, -1);
    S.dt = 0.0;
    return;
  }
  double dt = S.cfl / (s * S.geo);
  if (S.t + dt > S.T) dt = S.T - S.t;
  S.dt = dt;
}

__device__ __forceinline__ void dt_mesh(Scalars* sc, DevError* err, const int m) {
  Scalars& S = sc[m];
  S.idle = !(S.t < S.T);
  if (S.idle) return;
  const double s = __longlong_as_double((long long)S.s_bits);
  S.s = s;
  if (!(s > 0.0) || !isfinite(s)) {
    report(err, E_NONFINITE, -1);
    S.dt = 0.0;
    return;
  }
  double dt = S.cfl / (s * S.geo);
  if (S.t + dt > S.T) dt = S.T - S.t;
  S.dt = dt;
}

__global__ void k_dt(Scalars* sc, DevError* err, int n_mesh) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n_mesh) dt_mesh(sc, err, m);
}

// ---------------------------------------------------------------------------------------------
// k_elem: projection of F onto the basis, F_T at all points, volume term, edge traces.
// F^h is projected in contravariant form Fc_a = sum_d Jinv[a][d] F_d, so that div F^h =
// sum_a d/dxi_a Fc_a^h and grad D follows from reference second derivatives (affine elements).
// ---------------------------------------------------------------------------------------------
// Waves per SIMD the register allocation of k_elem targets: two for float32 triangles (measured
// faster: latency of the trace stores is hidden), one elsewhere (float64 would spill at two).
// Stores V values of one record (consecutive, 16-byte aligned when V values fill whole 16-byte
// words) with vector stores.
template <class R, int V>
__device__ __forceinline__ void store_rec(R* p, const R (&x)[V]) {
  if constexpr ((V * sizeof(R)) % 16 == 0) {
    typedef R vec __attribute__((ext_vector_type(V)));
    vec t;
#pragma unroll
    for (int c = 0; c < V; ++c) t[c] = x[c];
    *reinterpret_cast<vec*>(p) = t;
  } else {
#pragma unroll
    for (int c = 0; c < V; ++c) p[c] = x[c];
  }
}

// Index of the second reference derivative d/dxi_a d/dxi_b in the tables (2D: xx, xy, yy; 3D:
// xx, xy, xz, yy, yz, zz).
template <int DIM>
__device__ __forceinline__ constexpr int sidx(int a, int b) {
  if (a > b) { const int t = a; a = b; b = t; }
  return DIM == 3 ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : a + b;
}

template <class E, class R>
struct ElemOcc { static constexpr int waves = (E::kind == ElTri::kind && E::DEG == 2 && sizeof(R) == 4) ? 2 : 1; };

template <class E, class R>
__device__ __forceinline__ void elem_item2(View<R> v, const int i) {
  constexpr int V = E::V, ML = E::ML, DIM = E::DIM, NI = E::NI, K = E::K, NQE = E::NQE;
  const RefTab<E, R>& T = TabSel<E, R>::get();
  const RefTab<E, double>& TD = TabSel<E, double>::get();
  const int N = v.N, NE = v.E;
  if (i >= N) return;
  const int mid = mesh_id<R>(v.mesh_of, i);
  // At the end time the step changes nothing: the stored modes are written back as they were.
  // The flag is applied at the store (not by an early return), so its load overlaps the others.
  const bool idle = v.sc[mid].idle;
  const R dt = R(v.sc[mid].dt);
  const R gm1 = R(v.gamma - 1.0);

  // stored modes (before the limiter) and the limiter factor theta of this step
  double qb[V];
  R Qr[V][ML - 1];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    qb[c] = v.Qbar[(size_t)i * V + c];
#pragma unroll
    for (int l = 1; l < ML; ++l) Qr[c][l - 1] = v.Qh[(c * (ML - 1) + l - 1) * N + i];
  }
  const double th = v.theta[i];
  const R thR = R(th);
  R Ji[DIM][DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int d = 0; d < DIM; ++d) Ji[a][d] = v.Jinv[(a * DIM + d) * N + i];

  // point state of the limited polynomial in float64, q_bar + theta sum_l Q_l phi_l (the
  // expression the moment limiter made positive), then rounded to the bulk precision
  auto state_at = [&](int p, R* q) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int l = 1; l < ML; ++l) acc += double(Qr[c][l - 1]) * TD.phi[p][l];
      q[c] = R(qb[c] + th * acc);
    }
  };

  // Complete P2 on an affine element (line, triangle, tetrahedron): grad q and div F^h are linear
  // and their derivatives constant, so they are formed once per element from their values at the
  // reference origin and the constant reference Hessians, and each point costs a few multiply-adds.
  // In 2D and 3D F^h itself is never needed: Step 1's projection composed with div (and its
  // gradient) at the origin is a fixed table (kd0, kd1), and D0 = div F^h(0) and gDr = grad div F^h
  // accumulate directly from the quadrature values.  (1D, three modes, forms F^h as before; on the
  // tensor Q2 quadrilateral they are not linear, and those points contract F^h and the modes
  // directly.)
  constexpr bool AFF = E::kind != ElQuad::kind;
  constexpr bool KD = AFF && DIM >= 2;
  // Sec. 2.3 Step 1: Fc^h_a = sum_m w_m Fc_a(q(x_m)) phi_l(x_m)
  R Fh[DIM][V][ML];
  R D0[V], gDr[V][DIM];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    D0[c] = R(0);
#pragma unroll
    for (int b = 0; b < DIM; ++b) gDr[c][b] = R(0);
  }
  if constexpr (!KD) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c)
#pragma unroll
        for (int l = 0; l < ML; ++l) Fh[a][c][l] = R(0);
  }
  for (int m = 0; m < NI; ++m) {
    R q[V];
    state_at(m, q);
    St<DIM, R> s = base_state<DIM, R>(q, gm1);
    R F[DIM][V];
#pragma unroll
    for (int d = 0; d < DIM; ++d) flux<DIM, R>(s, d, F[d]);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R fc = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) fc += Ji[a][d] * F[d][c];
        if constexpr (KD) {
          D0[c] += T.kd0[m][a] * fc;
#pragma unroll
          for (int b = 0; b < DIM; ++b) gDr[c][b] += T.kd1[m][a][b] * fc;
        } else {
#pragma unroll
          for (int l = 0; l < ML; ++l) Fh[a][c][l] += T.wphi[m][l] * fc;
        }
      }
  }

  R vol[V][ML - 1];
#pragma unroll
  for (int c = 0; c < V; ++c)
#pragma unroll
    for (int l = 0; l < ML - 1; ++l) vol[c][l] = R(0);

  R g0[V][DIM], Hq[V][E::ND2], gDx[DIM][V];
  if constexpr (AFF) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      if constexpr (!KD) {  // 1D: div F^h and its derivative at the origin from F^h
        R dd = R(0), h = R(0);
#pragma unroll
        for (int l = 0; l < ML; ++l) {
          dd += Fh[0][c][l] * T.dphi0[0][l];
          h += Fh[0][c][l] * T.d2c[0][l];
        }
        D0[c] = dd;
        gDr[c][0] = h;
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        R acc = R(0);
#pragma unroll
        for (int l = 1; l < ML; ++l) acc += Qr[c][l - 1] * T.dphi0[a][l];
        g0[c][a] = thR * acc;
      }
#pragma unroll
      for (int k = 0; k < E::ND2; ++k) {
        R acc = R(0);
#pragma unroll
        for (int l = 1; l < ML; ++l) acc += Qr[c][l - 1] * T.d2c[k][l];
        Hq[c][k] = thR * acc;
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        R sh = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) sh += Ji[a][d] * gDr[c][a];
        gDx[d][c] = sh;
      }
    }
  }

  // Sec. 2.3 Step 2 at point p: q, grad q, D = div F^h, grad D, then q_t, q_tt and F_T; also the
  // state s of q and the variation vt of q_t, which F_T needs.
  auto derivs = [&](int p, R* q, R* qt, R* qtt, St<DIM, R>& s, Var<DIM, R>& vt) {
    R gq[DIM][V], D[V], gD[DIM][V];
    state_at(p, q);
    if constexpr (AFF) {
      R x[DIM];
#pragma unroll
      for (int a = 0; a < DIM; ++a) x[a] = T.xr[p][a];
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R g[DIM];
        if constexpr (DIM == 1) {
          g[0] = g0[c][0] + Hq[c][0] * x[0];
          D[c] = D0[c] + gDr[c][0] * x[0];
        } else if constexpr (DIM == 2) {
          g[0] = g0[c][0] + Hq[c][0] * x[0] + Hq[c][1] * x[1];
          g[1] = g0[c][1] + Hq[c][1] * x[0] + Hq[c][2] * x[1];
          D[c] = D0[c] + gDr[c][0] * x[0] + gDr[c][1] * x[1];
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a)
            g[a] = g0[c][a] + Hq[c][sidx<3>(a, 0)] * x[0] + Hq[c][sidx<3>(a, 1)] * x[1] + Hq[c][sidx<3>(a, 2)] * x[2];
          D[c] = D0[c] + gDr[c][0] * x[0] + gDr[c][1] * x[1] + gDr[c][2] * x[2];
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          R sg = R(0);
#pragma unroll
          for (int a = 0; a < DIM; ++a) sg += Ji[a][d] * g[a];
          gq[d][c] = sg;
          gD[d][c] = gDx[d][c];
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R g[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) g[a] = R(0);
        R dd = R(0);
        R h[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) h[a] = R(0);
#pragma unroll
        for (int l = 0; l < ML; ++l) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            if (l > 0) g[a] += Qr[c][l - 1] * T.dphi[p][a][l];
            dd += Fh[a][c][l] * T.dphi[p][a][l];
          }
          // d/dxi_b sum_a d/dxi_a Fc_a: b = 0 uses (xx, xy), b = 1 uses (xy, yy)
          h[0] += Fh[0][c][l] * T.d2phi[p][0][l] + Fh[DIM - 1][c][l] * T.d2phi[p][1][l];
          h[DIM - 1] += Fh[0][c][l] * T.d2phi[p][1][l] + Fh[DIM - 1][c][l] * T.d2phi[p][DIM][l];
        }
        D[c] = dd;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          R sg = R(0), sh = R(0);
#pragma unroll
          for (int a = 0; a < DIM; ++a) { sg += Ji[a][d] * g[a]; sh += Ji[a][d] * h[a]; }
          gq[d][c] = thR * sg;
          gD[d][c] = sh;
        }
      }
    }
    s = base_state<DIM, R>(q, gm1);
    const Var<DIM, R> vD = var1<DIM, R>(s, D, gm1);
#pragma unroll
    for (int d = 0; d < DIM; ++d) vt.du[d] = -vD.du[d];  // var1 is linear: q_t = -D
    vt.dp = -vD.dp;
#pragma unroll
    for (int c = 0; c < V; ++c) { qt[c] = -D[c]; qtt[c] = R(0); }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      Var<DIM, R> vq = var1<DIM, R>(s, gq[d], gm1);
      Var<DIM, R> vg = var1<DIM, R>(s, gD[d], gm1);
      R d2p = d2p_of<DIM, R>(s, vq, vD, gm1);
      R H[V], A[V];
      d2flux<DIM, R>(s, d, gq[d], vq, D, vD, d2p, H);
      dflux<DIM, R>(s, d, gD[d], vg, A);
#pragma unroll
      for (int c = 0; c < V; ++c) qtt[c] += H[c] + A[c];
    }
  };
  // In 3D the state and q_t's variation are formed again from q and q_t instead of being held across
  // the call: at one wave per SIMD the float64 tetrahedron kernel then spills less (820 instead of
  // 924 bytes per lane).
  auto point = [&](int p, R* q, R* qt, R* qtt, R FT[DIM][V]) {
    St<DIM, R> s;
    Var<DIM, R> vt;
    derivs(p, q, qt, qtt, s, vt);
    if constexpr (DIM == 3) ft_from<DIM, R>(q, qt, qtt, gm1, dt, FT);
    else ft_core<DIM, R>(s, qt, vt, qtt, gm1, dt, FT);
  };

  // interior points: volume term V_l = sum_m w_m grad phi_l . F_T
  for (int m = 0; m < NI; ++m) {
    R q[V], qt[V], qtt[V], FT[DIM][V];
    point(m, q, qt, qtt, FT);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R fc = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) fc += Ji[a][d] * FT[d][c];
#pragma unroll
        for (int l = 1; l < ML; ++l) vol[c][l - 1] += T.wdphi[m][a][l] * fc;
      }
  }

  // Sec. 2.3 Step 3 / Sec. 3.3 Step 6, volume part: Q^(l) += dt V_l for l >= 2.  Stored before the
  // edge points (which use the modes held in registers), so the accumulators are free for them.
#pragma unroll
  for (int c = 0; c < V; ++c)
#pragma unroll
    for (int l = 1; l < ML; ++l)
      v.Qh[(c * (ML - 1) + l - 1) * N + i] = idle ? Qr[c][l - 1] : thR * Qr[c][l - 1] + dt * vol[c][l - 1];
  if (v.dbg_vol) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      v.dbg_vol[(c * ML) * N + i] = 0.0;
#pragma unroll
      for (int l = 1; l < ML; ++l) v.dbg_vol[(c * ML + l) * N + i] = double(vol[c][l - 1]);
    }
  }

  // edge points: the trace n_out . F_T / 2 + hs q (and the ghost side's on boundary edges)
  const double hs0 = 0.5 * v.sc[mid].s;
  for (int k = 0; k < K; ++k) {
    const int slot = v.eslot[k * N + i];
    const int e = slot >> 3, side = (slot >> 2) & 1, bc = slot & 3;
    const int perm = (DIM == 3) ? v.fperm[k * N + i] : 0;
    R n[DIM], len2 = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) { n[d] = v.nout[(k * DIM + d) * N + i]; len2 += n[d] * n[d]; }
    // s |n_e| / 2: both elements of an edge hold the same normal up to sign, so they form it alike
    const R hs = R(hs0 * double(sqrt(len2)));
    for (int jl = 0; jl < NQE; ++jl) {
      const int p = NI + k * NQE + jl;
      // point order of i_e along the edge (reversed on the other side), or on the face
      const int jj = (DIM == 3) ? T.pperm[perm][jl] : (side ? (NQE - 1 - jl) : jl);
      // the normal flux directly (3D: 5% faster), or both directions and a dot product (1D/2D:
      // measured faster there, the two directions' independent chains hide latency at two waves)
      R q[V], qt[V], qtt[V], fn[V];
      if constexpr (DIM == 3) {
        St<DIM, R> s;
        Var<DIM, R> vt;
        derivs(p, q, qt, qtt, s, vt);
        ftn_from<DIM, R>(q, qt, qtt, n, gm1, dt, fn);
      } else {
        R FT[DIM][V];
        point(p, q, qt, qtt, FT);
#pragma unroll
        for (int c = 0; c < V; ++c) {
          fn[c] = R(0);
#pragma unroll
          for (int d = 0; d < DIM; ++d) fn[c] += n[d] * FT[d][c];
        }
      }
      R b[V];
#pragma unroll
      for (int c = 0; c < V; ++c) b[c] = R(0.5) * fn[c] + hs * q[c];
      store_rec<R, V>(v.tr + (((size_t)side * NE + e) * NQE + jj) * V, b);
      if (bc != SB_INTERIOR) {
        R qg[V], fgn[V];
        if (bc == SB_TRANSPARENT) {
#pragma unroll
          for (int c = 0; c < V; ++c) { qg[c] = q[c]; fgn[c] = fn[c]; }
        } else if (bc == SB_REFLECTIVE) {
          R nh[DIM];
          const R il = R(1) / sqrt(len2);
#pragma unroll
          for (int d = 0; d < DIM; ++d) nh[d] = n[d] * il;
          R qtg[V], qttg[V];
          reflect<DIM, R>(q, nh, qg);
          reflect<DIM, R>(qt, nh, qtg);
          reflect<DIM, R>(qtt, nh, qttg);
          ftn_from<DIM, R>(qg, qtg, qttg, n, gm1, dt, fgn);
        } else {
          R z[V];
#pragma unroll
          for (int c = 0; c < V; ++c) z[c] = R(0);
          inflow_state<DIM, R>(v.inflow, qg);
          ftn_from<DIM, R>(qg, z, z, n, gm1, dt, fgn);
        }
        // the ghost is side 1: its outward normal is -n
        R bg[V];
#pragma unroll
        for (int c = 0; c < V; ++c) bg[c] = hs * qg[c] - R(0.5) * fgn[c];
        store_rec<R, V>(v.tr + (((size_t)NE + e) * NQE + jj) * V, bg);
      }
    }
  }
}

// k_elem at degree 3 (P3 on the line and on triangles, affine elements).  The same steps as above
// with the Taylor series of Sec. 2.2 carried one term further: F_T needs q_ttt = -div F_tt, which
// takes the gradient of q_tt, hence the Hessians of q and of D = div F^h (constant for cubic F^h).
// With D_e = d/dx_e D and q_e = d/dx_e q:
//   q_t = -D,  q_tt = sum_d [H_d(q_d, D) + A_d D_d],
//   d/dx_e q_tt = sum_d [F3_d(q_e, q_d, D) + H_d(q_ed, D) + H_d(q_d, D_e) + H_d(q_e, D_d) + A_d D_ed],
//   q_ttt = -sum_d [F3_d(q_d, q_t, q_t) - 2 H_d(D_d, q_t) + H_d(q_d, q_tt) + A_d d/dx_d q_tt].
// Gradients and Hessians are contracted per point from the reference tables (quadratic and linear
// in the reference coordinates), the Hessian of D once per element.
template <class E, class R>
__device__ __forceinline__ void elem_item3(View<R> v, const int i) {
  constexpr int V = E::V, ML = E::ML, DIM = E::DIM, NI = E::NI, K = E::K, NQE = E::NQE;
  const RefTab<E, R>& T = TabSel<E, R>::get();
  const RefTab<E, double>& TD = TabSel<E, double>::get();
  const int N = v.N, NE = v.E;
  if (i >= N) return;
  const int mid = mesh_id<R>(v.mesh_of, i);
  const bool idle = v.sc[mid].idle;
  const R dt = R(v.sc[mid].dt);
  const R gm1 = R(v.gamma - 1.0);

  double qb[V];
  R Qr[V][ML - 1];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    qb[c] = v.Qbar[(size_t)i * V + c];
#pragma unroll
    for (int l = 1; l < ML; ++l) Qr[c][l - 1] = v.Qh[(c * (ML - 1) + l - 1) * N + i];
  }
  const double th = v.theta[i];
  const R thR = R(th);
  R Ji[DIM][DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a)
#pragma unroll
    for (int d = 0; d < DIM; ++d) Ji[a][d] = v.Jinv[(a * DIM + d) * N + i];

  auto state_at = [&](int p, R* q) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int l = 1; l < ML; ++l) acc += double(Qr[c][l - 1]) * TD.phi[p][l];
      q[c] = R(qb[c] + th * acc);
    }
  };
  // physical second derivatives from the reference ones (xx[, xy, yy] at index a + b)
  auto map2 = [&](const R* hr, R out[DIM][DIM]) {
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int e = 0; e < DIM; ++e) {
        R t = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
          for (int b = 0; b < DIM; ++b) t += Ji[a][d] * Ji[b][e] * hr[a + b];
        out[d][e] = t;
      }
  };

  // Sec. 2.3 Step 1: Fc^h_a = sum_m w_m Fc_a(q(x_m)) phi_l(x_m).  Only D = div F^h is needed, and
  // it is quadratic: on triangles its value, gradient and Hessian at the reference origin accumulate
  // straight from the quadrature values through the tables kd0, kd1, kd2 (the projection composed
  // with div and its derivatives); in 1D F^h is formed.
  constexpr int N2 = 2 * DIM - 1;
  constexpr bool KD = DIM >= 2;
  R Fh[DIM][V][ML];
  R D0[V], gD0[V][DIM], HDr[V][N2];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    D0[c] = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) gD0[c][a] = R(0);
#pragma unroll
    for (int j = 0; j < N2; ++j) HDr[c][j] = R(0);
  }
  if constexpr (!KD) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c)
#pragma unroll
        for (int l = 0; l < ML; ++l) Fh[a][c][l] = R(0);
  }
  for (int m = 0; m < NI; ++m) {
    R q[V];
    state_at(m, q);
    St<DIM, R> s = base_state<DIM, R>(q, gm1);
    R F[DIM][V];
#pragma unroll
    for (int d = 0; d < DIM; ++d) flux<DIM, R>(s, d, F[d]);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R fc = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) fc += Ji[a][d] * F[d][c];
        if constexpr (KD) {
          D0[c] += T.kd0[m][a] * fc;
#pragma unroll
          for (int b = 0; b < DIM; ++b) gD0[c][b] += T.kd1[m][a][b] * fc;
#pragma unroll
          for (int j = 0; j < N2; ++j) HDr[c][j] += T.kd2[m][a][j] * fc;
        } else {
#pragma unroll
          for (int l = 0; l < ML; ++l) Fh[a][c][l] += T.wphi[m][l] * fc;
        }
      }
  }

  // The point derivatives come from Taylor coefficients at the reference origin, formed once per
  // element (reference derivative indices count the eta derivatives: second xx, xy, yy; third xxx,
  // xxy, xyy, yyy): q is cubic, so its reference gradient is g0 + H0 x + T3[x, x]/2 and its
  // reference Hessian H0 + T3 x; D = div F^h is quadratic, D0 + gD0 . x + x^T HDr x / 2, with
  // reference gradient gD0 + HDr x and constant Hessian HDr (the physical HD).  The limiter
  // factor theta is folded into q's coefficients.
  R qg0[V][DIM], qH0[V][N2], qT3[V][E::ND3];
  R HD[DIM][DIM][V];
#pragma unroll
  for (int c = 0; c < V; ++c) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      R t = R(0), u = R(0);
#pragma unroll
      for (int l = 1; l < ML; ++l) t += Qr[c][l - 1] * T.dphi0[a][l];
      qg0[c][a] = thR * t;
      if constexpr (!KD) {
#pragma unroll
        for (int l = 0; l < ML; ++l)
#pragma unroll
          for (int b = 0; b < DIM; ++b) u += Fh[b][c][l] * T.d2c[a + b][l];
        gD0[c][a] = u;
      }
    }
#pragma unroll
    for (int j = 0; j < N2; ++j) {
      R t = R(0), u = R(0);
#pragma unroll
      for (int l = 1; l < ML; ++l) t += Qr[c][l - 1] * T.d2c[j][l];
      qH0[c][j] = thR * t;
      if constexpr (!KD) {
#pragma unroll
        for (int l = 0; l < ML; ++l)
#pragma unroll
          for (int a = 0; a < DIM; ++a) u += Fh[a][c][l] * T.d3c[a + j][l];
        HDr[c][j] = u;
      }
    }
#pragma unroll
    for (int j = 0; j < E::ND3; ++j) {
      R t = R(0);
#pragma unroll
      for (int l = 1; l < ML; ++l) t += Qr[c][l - 1] * T.d3c[j][l];
      qT3[c][j] = thR * t;
    }
    if constexpr (!KD) {
      R t = R(0);
#pragma unroll
      for (int l = 0; l < ML; ++l)
#pragma unroll
        for (int a = 0; a < DIM; ++a) t += Fh[a][c][l] * T.dphi0[a][l];
      D0[c] = t;
    }
    R h[DIM][DIM];
    map2(HDr[c], h);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int e = 0; e < DIM; ++e) HD[d][e][c] = h[d][e];
  }

  auto point = [&](int p, R* q, R* qt, R* qtt, R* qttt, R FT[DIM][V]) {
    R gq[DIM][V], Hq[DIM][DIM][V], D[V], gD[DIM][V];
    state_at(p, q);
    // the point's reference coordinates x and the quadratic monomials m2[j] (j eta factors), with
    // the factor 1/2 of the Taylor series and the two orderings of a mixed product
    R x[DIM], m2[N2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = T.xr[p][a];
    if constexpr (DIM == 1) {
      m2[0] = R(0.5) * x[0] * x[0];
    } else {
      m2[0] = R(0.5) * x[0] * x[0];
      m2[1] = x[0] * x[1];
      m2[2] = R(0.5) * x[1] * x[1];
    }
#pragma unroll
    for (int c = 0; c < V; ++c) {
      R g[DIM], hq[N2], gd[DIM];
      R dd = D0[c];
#pragma unroll
      for (int j = 0; j < N2; ++j) dd += HDr[c][j] * m2[j];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        R t = qg0[c][a], u = gD0[c][a];
#pragma unroll
        for (int b = 0; b < DIM; ++b) { t += qH0[c][a + b] * x[b]; u += HDr[c][a + b] * x[b]; }
#pragma unroll
        for (int j = 0; j < N2; ++j) t += qT3[c][a + j] * m2[j];
        g[a] = t;
        gd[a] = u;
        dd += gD0[c][a] * x[a];
      }
#pragma unroll
      for (int j = 0; j < N2; ++j) {
        R t = qH0[c][j];
#pragma unroll
        for (int e = 0; e < DIM; ++e) t += qT3[c][j + e] * x[e];
        hq[j] = t;
      }
      D[c] = dd;
      R h[DIM][DIM];
      map2(hq, h);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        R sg = R(0), sd = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) { sg += Ji[a][d] * g[a]; sd += Ji[a][d] * gd[a]; }
        gq[d][c] = sg;
        gD[d][c] = sd;
#pragma unroll
        for (int e = 0; e < DIM; ++e) Hq[d][e][c] = h[d][e];
      }
    }
    St<DIM, R> s = base_state<DIM, R>(q, gm1);
    Var<DIM, R> vD = var1<DIM, R>(s, D, gm1);
    Var<DIM, R> vq[DIM], vg[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      vq[d] = var1<DIM, R>(s, gq[d], gm1);
      vg[d] = var1<DIM, R>(s, gD[d], gm1);
    }
#pragma unroll
    for (int c = 0; c < V; ++c) { qt[c] = -D[c]; qtt[c] = R(0); qttt[c] = R(0); }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      R H[V], A[V];
      d2flux<DIM, R>(s, d, gq[d], vq[d], D, vD, d2p_of<DIM, R>(s, vq[d], vD, gm1), H);
      dflux<DIM, R>(s, d, gD[d], vg[d], A);
#pragma unroll
      for (int c = 0; c < V; ++c) qtt[c] += H[c] + A[c];
    }
    Var<DIM, R> vt;  // the variation of q_t = -D (var1 is linear)
#pragma unroll
    for (int d = 0; d < DIM; ++d) vt.du[d] = -vD.du[d];
    vt.dp = -vD.dp;
    Var<DIM, R> vtt = var1<DIM, R>(s, qtt, gm1);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // d/dx_d q_tt
      R dq2[V];
#pragma unroll
      for (int c = 0; c < V; ++c) dq2[c] = R(0);
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        R t1[V], t2[V], t3[V], t4[V], t5[V];
        Var<DIM, R> vH = var1<DIM, R>(s, Hq[d][k], gm1);
        Var<DIM, R> vHD = var1<DIM, R>(s, HD[d][k], gm1);
        d3flux<DIM, R>(s, k, gq[d], vq[d], gq[k], vq[k], D, vD, gm1, t1);
        d2flux<DIM, R>(s, k, Hq[d][k], vH, D, vD, d2p_of<DIM, R>(s, vH, vD, gm1), t2);
        d2flux<DIM, R>(s, k, gq[k], vq[k], gD[d], vg[d], d2p_of<DIM, R>(s, vq[k], vg[d], gm1), t3);
        d2flux<DIM, R>(s, k, gq[d], vq[d], gD[k], vg[k], d2p_of<DIM, R>(s, vq[d], vg[k], gm1), t4);
        dflux<DIM, R>(s, k, HD[d][k], vHD, t5);
#pragma unroll
        for (int c = 0; c < V; ++c) dq2[c] += t1[c] + t2[c] + t3[c] + t4[c] + t5[c];
      }
      R t1[V], t2[V], t3[V], t4[V];
      Var<DIM, R> v2 = var1<DIM, R>(s, dq2, gm1);
      d3flux<DIM, R>(s, d, gq[d], vq[d], qt, vt, qt, vt, gm1, t1);
      d2flux<DIM, R>(s, d, gD[d], vg[d], qt, vt, d2p_of<DIM, R>(s, vg[d], vt, gm1), t2);
      d2flux<DIM, R>(s, d, gq[d], vq[d], qtt, vtt, d2p_of<DIM, R>(s, vq[d], vtt, gm1), t3);
      dflux<DIM, R>(s, d, dq2, v2, t4);
#pragma unroll
      for (int c = 0; c < V; ++c) qttt[c] -= t1[c] - R(2) * t2[c] + t3[c] + t4[c];
    }
    ft4_core<DIM, R>(s, qt, vt, qtt, qttt, gm1, dt, FT);
  };

  R vol[V][ML - 1];
#pragma unroll
  for (int c = 0; c < V; ++c)
#pragma unroll
    for (int l = 0; l < ML - 1; ++l) vol[c][l] = R(0);
  for (int m = 0; m < NI; ++m) {
    R q[V], qt[V], qtt[V], qttt[V], FT[DIM][V];
    point(m, q, qt, qtt, qttt, FT);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int c = 0; c < V; ++c) {
        R fc = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) fc += Ji[a][d] * FT[d][c];
#pragma unroll
        for (int l = 1; l < ML; ++l) vol[c][l - 1] += T.wdphi[m][a][l] * fc;
      }
  }
#pragma unroll
  for (int c = 0; c < V; ++c)
#pragma unroll
    for (int l = 1; l < ML; ++l)
      v.Qh[(c * (ML - 1) + l - 1) * N + i] = idle ? Qr[c][l - 1] : thR * Qr[c][l - 1] + dt * vol[c][l - 1];
  if (v.dbg_vol) {
#pragma unroll
    for (int c = 0; c < V; ++c) {
      v.dbg_vol[(c * ML) * N + i] = 0.0;
#pragma unroll
      for (int l = 1; l < ML; ++l) v.dbg_vol[(c * ML + l) * N + i] = double(vol[c][l - 1]);
    }
  }

  // edge points: the trace n_out . F_T / 2 + hs q (and the ghost side's on boundary edges)
  const double hs0 = 0.5 * v.sc[mid].s;
  for (int k = 0; k < K; ++k) {
    const int slot = v.eslot[k * N + i];
    const int e = slot >> 3, side = (slot >> 2) & 1, bc = slot & 3;
    R n[DIM], len2 = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) { n[d] = v.nout[(k * DIM + d) * N + i]; len2 += n[d] * n[d]; }
    const R hs = R(hs0 * double(sqrt(len2)));
    for (int jl = 0; jl < NQE; ++jl) {
      const int p = NI + k * NQE + jl;
      const int jj = side ? (NQE - 1 - jl) : jl;
      R q[V], qt[V], qtt[V], qttt[V], FT[DIM][V];
      point(p, q, qt, qtt, qttt, FT);
      R fn[V];
#pragma unroll
      for (int c = 0; c < V; ++c) {
        fn[c] = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) fn[c] += n[d] * FT[d][c];
      }
      R b[V];
#pragma unroll
      for (int c = 0; c < V; ++c) b[c] = R(0.5) * fn[c] + hs * q[c];
      store_rec<R, V>(v.tr + (((size_t)side * NE + e) * NQE + jj) * V, b);
      if (bc != SB_INTERIOR) {
        R qg[V], FTg[DIM][V];
        if (bc == SB_TRANSPARENT) {
#pragma unroll
          for (int c = 0; c < V; ++c) qg[c] = q[c];
#pragma unroll
          for (int d = 0; d < DIM; ++d)
#pragma unroll
            for (int c = 0; c < V; ++c) FTg[d][c] = FT[d][c];
        } else if (bc == SB_REFLECTIVE) {
          R nh[DIM];
          const R il = R(1) / sqrt(len2);
#pragma unroll
          for (int d = 0; d < DIM; ++d) nh[d] = n[d] * il;
          R qtg[V], qttg[V], q3g[V];
          reflect<DIM, R>(q, nh, qg);
          reflect<DIM, R>(qt, nh, qtg);
          reflect<DIM, R>(qtt, nh, qttg);
          reflect<DIM, R>(qttt, nh, q3g);
          ft4_from<DIM, R>(qg, qtg, qttg, q3g, gm1, dt, FTg);
        } else {
          R z[V];
#pragma unroll
          for (int c = 0; c < V; ++c) z[c] = R(0);
          inflow_state<DIM, R>(v.inflow, qg);
          ft4_from<DIM, R>(qg, z, z, z, gm1, dt, FTg);
        }
        R bg[V];  // the ghost is side 1: its outward normal is -n
#pragma unroll
        for (int c = 0; c < V; ++c) {
          R f = R(0);
#pragma unroll
          for (int d = 0; d < DIM; ++d) f += n[d] * FTg[d][c];
          bg[c] = hs * qg[c] - R(0.5) * f;
        }
        store_rec<R, V>(v.tr + (((size_t)NE + e) * NQE + jj) * V, bg);
      }
    }
  }
}

template <class E, class R>
__device__ __forceinline__ void elem_item(View<R> v, const int i) {
  if constexpr (E::DEG == 3) elem_item3<E, R>(v, i);
  else elem_item2<E, R>(v, i);
}

template <class E, class R>
__global__ __launch_bounds__(256, (ElemOcc<E, R>::waves)) void k_elem(View<R> v) {
  elem_item<E, R>(v, xcd_item());
}

// ---------------------------------------------------------------------------------------------
// k_edge: F*_T . n_e = (1/2)(n_e.F_T(q+) + n_e.F_T(q-)) - (s |n_e| / 2)(q+ - q-) at each edge point
// (Eq. (LLF) with the scaled normal; the flux is linear in the two sides' values, so each element
// wrote its half n_out.F_T/2 + (s |n_e|/2) q and F* is side 0 minus side 1),
// f^LxW_e = (1/2) sum_j omega_j F*_j (float64 sum), and
// f^LxF_e = (1/2) n_e.(F(q_bar_j) + F(q_bar_i)) - (s |n_e| / 2)(q_bar_j - q_bar_i) in float64.
// ---------------------------------------------------------------------------------------------
// Copies nbytes (a multiple of 4) from LDS to global memory with the whole workgroup, 16 bytes per
// lane and store where both ends allow it: consecutive lanes write consecutive addresses.
template <int ALIGN16>
__device__ __forceinline__ void lds_to_global(unsigned char* dst, const unsigned char* src, int nbytes) {
  if constexpr (ALIGN16) {
    for (int o = (int)threadIdx.x * 16; o < nbytes; o += (int)blockDim.x * 16)
      *reinterpret_cast<uint4*>(dst + o) = *reinterpret_cast<const uint4*>(src + o);
  } else {
    for (int o = (int)threadIdx.x * 4; o < nbytes; o += (int)blockDim.x * 4)
      *reinterpret_cast<unsigned*>(dst + o) = *reinterpret_cast<const unsigned*>(src + o);
  }
}

// f^LxW_e = (1/2) sum_j omega_j F*_j in float64, summed in the edge's point order with explicit
// fused multiply-adds: k_edge stores it for the flux limiter and k_update forms it again from the
// F* record, and the two agree bit for bit.
template <class E, class R>
__device__ __forceinline__ void lxw_average(const RefTab<E, R>& T, const R (&fs)[E::NQE][E::V], double (&W)[E::V]) {
#pragma unroll
  for (int c = 0; c < E::V; ++c) W[c] = 0.0;
#pragma unroll
  for (int jj = 0; jj < E::NQE; ++jj) {
    const double w = 0.5 * double(T.om[jj]);
#pragma unroll
    for (int c = 0; c < E::V; ++c) W[c] = __fma_rn(w, double(fs[jj][c]), W[c]);
  }
}

// Edge e of k_edge; every lane of the workgroup calls it with the edges e0 + threadIdx.x of one
// contiguous tile (the records are staged through LDS and written together).
template <class E, class R>
__device__ __forceinline__ void edge_tile(View<R> v, const int e) {
  constexpr int V = E::V, DIM = E::DIM, NQE = E::NQE;
  // per-edge records: F* at the edge points, f^LxW and f^LxF; each lane writes its edge's records
  // into LDS as it computes them
  constexpr int FS = NQE * V * (int)sizeof(R), FL = V * (int)sizeof(double);
  __shared__ __align__(16) unsigned char rec_fs[256 * FS];
  __shared__ __align__(16) unsigned char rec_fw[256 * FL];
  __shared__ __align__(16) unsigned char rec_ff[256 * FL];
  const RefTab<E, R>& T = TabSel<E, R>::get();
  const int NE = v.E;
  const bool valid = e < NE;
  const int e0 = e - (int)threadIdx.x;  // first edge of the workgroup (its edges are consecutive)
  const int nrec = max(0, min((int)blockDim.x, NE - e0));
  R* fsr = reinterpret_cast<R*>(rec_fs + threadIdx.x * FS);
  double* fwr = reinterpret_cast<double*>(rec_fw + threadIdx.x * FL);
  double* ffr = reinterpret_cast<double*>(rec_ff + threadIdx.x * FL);
  if (valid) {
    const int mid = v.e_mesh ? at(v.e_mesh, e) : 0;
    const double s = v.sc[mid].s;
    const double gam = v.gamma;
    double n[DIM], len2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) { n[d] = at(v.e_n + (size_t)d * NE, e); len2 += n[d] * n[d]; }
    const double len = sqrt(len2);
    const int ie = at(v.e_i, e), je = at(v.e_j, e);
    R fs[NQE][V];
#pragma unroll
    for (int jj = 0; jj < NQE; ++jj) {
#pragma unroll
      for (int c = 0; c < V; ++c) {
        // (n.F_T(q-) + n.F_T(q+))/2 - hs (q+ - q-), from the two sides' traces
        fs[jj][c] = v.tr[((size_t)e * NQE + jj) * V + c] - v.tr[(((size_t)NE + e) * NQE + jj) * V + c];
        fsr[jj * V + c] = fs[jj][c];
      }
    }
    double W[V];
    lxw_average<E, R>(T, fs, W);
#pragma unroll
    for (int c = 0; c < V; ++c) fwr[c] = W[c];

    const int i = ie, j = je;
    double qi[V], qj[V];
#pragma unroll
    for (int c = 0; c < V; ++c) qi[c] = v.Qbar[(size_t)i * V + c];
    if (j >= 0) {
#pragma unroll
      for (int c = 0; c < V; ++c) qj[c] = v.Qbar[(size_t)j * V + c];
    } else {
      const int bc = at(v.e_bc, e);
      if (bc == SB_REFLECTIVE) {
        double nh[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) nh[d] = n[d] / len;
        reflect<DIM, double>(qi, nh, qj);
      } else if (bc == SB_INFLOW) {
        inflow_state<DIM, double>(v.inflow, qj);
      } else {
#pragma unroll
        for (int c = 0; c < V; ++c) qj[c] = qi[c];
      }
    }
    St<DIM, double> si = base_state<DIM, double>(qi, gam - 1.0);
    St<DIM, double> sj = base_state<DIM, double>(qj, gam - 1.0);
    double Lf[V];
#pragma unroll
    for (int c = 0; c < V; ++c) Lf[c] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      double Fi[V], Fj[V];
      flux<DIM, double>(si, d, Fi);
      flux<DIM, double>(sj, d, Fj);
#pragma unroll
      for (int c = 0; c < V; ++c) Lf[c] += 0.5 * n[d] * (Fj[c] + Fi[c]);
    }
#pragma unroll
    for (int c = 0; c < V; ++c) ffr[c] = Lf[c] - 0.5 * s * len * (qj[c] - qi[c]);
  }
  // The records of the workgroup's edges are one contiguous range: staged in LDS, they are written
  // with coalesced stores (written straight from the lanes, every store instruction would touch a
  // cache line per lane).
  __syncthreads();
  lds_to_global<FS % 16 == 0>(reinterpret_cast<unsigned char*>(v.fstar) + (size_t)max(e0, 0) * FS, rec_fs, nrec * FS);
  lds_to_global<FL % 16 == 0>(reinterpret_cast<unsigned char*>(v.fLxW) + (size_t)max(e0, 0) * FL, rec_fw, nrec * FL);
  lds_to_global<FL % 16 == 0>(reinterpret_cast<unsigned char*>(v.fLxF) + (size_t)max(e0, 0) * FL, rec_ff, nrec * FL);
  // the staging area is free again only when every lane has copied its part out (a workgroup of
  // the persistent kernel goes on to its next tile)
  __syncthreads();
}

template <class E, class R>
__global__ __launch_bounds__(256) void k_edge(View<R> v) {
  edge_tile<E, R>(v, xcd_item());
}

// ---------------------------------------------------------------------------------------------
// Damping factor mu (Sec. 3.3 Step 5b): the largest mu in [0,1] with positive density and
// pressure >= eps_p on qL + mu (qa - qL).  Along the segment (gamma-1)(rho E - |M|^2/2) - eps_p rho
// is a quadratic a mu^2 + b mu + c with c >= 0; its first zero is 2c/(-b + sqrt(b^2 - 4ac)),
// which is then lowered by ulps until the condition holds in float64.
// ---------------------------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ bool mu_ok(const double* qL, const double* qa, double mu, double gam, double epsp) {
  constexpr int V = DIM + 2;
  double q[V];
#pragma unroll
  for (int c = 0; c < V; ++c) q[c] = qL[c] + mu * (qa[c] - qL[c]);
  return q[0] > 0.0 && pressure<DIM>(q, gam) >= epsp;
}

template <int DIM>
__device__ double mu_solve(const double* qL, const double* qa, double gam, double epsp) {
  constexpr int V = DIM + 2;
  if (mu_ok<DIM>(qL, qa, 1.0, gam, epsp)) return 1.0;
  double dq[V];
#pragma unroll
  for (int c = 0; c < V; ++c) dq[c] = qa[c] - qL[c];
  double mL2 = 0.0, mLd = 0.0, dd2 = 0.0;
#pragma unroll
  for (int k = 1; k <= DIM; ++k) { mL2 += qL[k] * qL[k]; mLd += qL[k] * dq[k]; dd2 += dq[k] * dq[k]; }
  const double g1 = gam - 1.0;
  const double a = g1 * (dq[0] * dq[V - 1] - 0.5 * dd2);
  const double b = g1 * (qL[0] * dq[V - 1] + dq[0] * qL[V - 1] - mLd) - epsp * dq[0];
  const double c = g1 * (qL[0] * qL[V - 1] - 0.5 * mL2) - epsp * qL[0];
  if (!(c > 0.0)) return 0.0;
  // target equal to the LxF corner's own pressure (p(q^LxF) <= eps0): c is zero up to rounding,
  // g(mu) = mu (a mu + b), and with b <= 0 only mu = 0 is feasible (the ulp search would end there)
  if (b <= 0.0 && pressure<DIM>(qL, gam) <= epsp) return 0.0;
  const double den = -b + sqrt(fmax(0.0, b * b - 4.0 * a * c));
  double mu = den > 0.0 ? 2.0 * c / den : 0.0;
  mu = fmin(1.0, fmax(0.0, mu));
  for (int it = 0; it < 64 && mu > 0.0 && !mu_ok<DIM>(qL, qa, mu, gam, epsp); ++it) mu = nextafter(mu, 0.0);
  if (!mu_ok<DIM>(qL, qa, mu, gam, epsp)) mu = 0.0;
  return mu;
}

// ---------------------------------------------------------------------------------------------
// k_flim: the flux limiter of Sec. 3.3 Steps 4-5, float64, per element.  Readings: every edge flux
// of the element carries eps_ik (as in the printed Step 4); Cases 1-4 of the sorted Delta f are
// evaluated as "each edge with Delta f_k < 0 gets min(1, Gamma / |sum of the negative Delta f|)"
// (no sort); the corner states keep the Lax-Friedrichs flux on the edges switched off, so that
// corner 000 is the pure LxF update; the pressure target is eps_p = min(eps0, p(q^LxF)).
// ---------------------------------------------------------------------------------------------
template <class E, class R>
__device__ __forceinline__ void flim_item(View<R> v, const int i) {
  constexpr int V = E::V, DIM = E::DIM, K = E::K;
  const int N = v.N;
  if (i >= N) return;
  const int mid = mesh_id<R>(v.mesh_of, i);
  const double dt = v.sc[mid].dt;
  const bool idle = v.sc[mid].idle;  // at the end time nothing is reported (the step is discarded)
  const double gam = v.gamma;
  const double area = at(v.area, i);
  const double r = dt / area;
  double qb[V];
#pragma unroll
  for (int c = 0; c < V; ++c) qb[c] = v.Qbar[(size_t)i * V + c];
  double fW[K][V], fF[K][V], df[K];
  int eidx[K], sd[K];
  double Gam = area * qb[0] / dt;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int slot = at(v.eslot + (size_t)k * N, i);
    eidx[k] = slot >> 3;
    sd[k] = (slot >> 2) & 1;
    const double ep = sd[k] ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < V; ++c) {
      fW[k][c] = ep * v.fLxW[(size_t)eidx[k] * V + c];
      fF[k][c] = ep * v.fLxF[(size_t)eidx[k] * V + c];
    }
    Gam -= fF[k][0];
    df[k] = fF[k][0] - fW[k][0];
  }
  double Sneg = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (df[k] < 0.0) Sneg += df[k];
  bool bad = Gam < 0.0;
  double Lam[K];
#pragma unroll
  for (int k = 0; k < K; ++k) Lam[k] = df[k] < 0.0 ? fmax(0.0, fmin(1.0, Gam / fabs(Sneg))) : 1.0;
  double qL[V];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc += fF[k][c];
    qL[c] = qb[c] - r * acc;
  }
  const double pL = qL[0] > 0.0 ? pressure<DIM>(qL, gam) : -1.0;
  bad = bad || !(pL > 0.0);
  const double epsp = fmin(v.eps0, pL);
  double mm[K];
#pragma unroll
  for (int k = 0; k < K; ++k) mm[k] = 1.0;
#pragma unroll
  for (int a = 1; a < (1 << K); ++a) {
    double qa[V];
#pragma unroll
    for (int c = 0; c < V; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double th = ((a >> k) & 1) ? Lam[k] : 0.0;
        acc += th * fW[k][c] + (1.0 - th) * fF[k][c];
      }
      qa[c] = qb[c] - r * acc;
    }
    const double mu = pL > 0.0 ? mu_solve<DIM>(qL, qa, gam, epsp) : 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if ((a >> k) & 1) mm[k] = fmin(mm[k], mu);
  }
  if (bad && !idle) report(v.err, E_CFL, i);
#pragma unroll
  for (int k = 0; k < K; ++k) v.cedge[(size_t)eidx[k] * 2 + sd[k]] = Lam[k] * mm[k];
}

template <class E, class R>
__global__ __launch_bounds__(256) void k_flim(View<R> v) {
  flim_item<E, R>(v, xcd_item());
}

// ---------------------------------------------------------------------------------------------
// k_update: Sec. 3.3 Step 6 with theta_k = Lambda_{e_ik} = min(1, both sides' candidates):
//   Q^(1) -= dt/|T| sum_k eps_ik [theta_k f^LxW + (1 - theta_k) f^LxF]            (float64)
//   Q^(l) -= dt/|T| sum_k eps_ik (1/2) sum_j omega_j phi_l(x_kj) F*_kj . n_e,  l >= 2
// (the volume part of the higher moments was added by k_elem), then the positivity check of the
// new cell average.
// ---------------------------------------------------------------------------------------------
template <class E, class R>
__device__ __forceinline__ void update_item(View<R> v, const int i) {
  constexpr int V = E::V, ML = E::ML, DIM = E::DIM, K = E::K, NQE = E::NQE;
  const RefTab<E, R>& T = TabSel<E, R>::get();
  const int N = v.N;
  if (i >= N) return;
  const int mid = mesh_id<R>(v.mesh_of, i);
  // at the end time the step changes nothing: the flag is read here and applied at the stores
  const bool idle = v.sc[mid].idle;
  const double dt = v.sc[mid].dt;
  const double r = dt / at(v.area, i);
  double qb[V];
  R Qh[V][ML - 1];
#pragma unroll
  for (int c = 0; c < V; ++c) {
    qb[c] = v.Qbar[(size_t)i * V + c];
#pragma unroll
    for (int l = 0; l < ML - 1; ++l) Qh[c][l] = at(v.Qh + (size_t)(c * (ML - 1) + l) * N, i);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int slot = at(v.eslot + (size_t)k * N, i);
    const int e = slot >> 3, side = (slot >> 2) & 1;
    const double ep = side ? -1.0 : 1.0;
    const double th = fmin(1.0, fmin(v.cedge[(size_t)e * 2], v.cedge[(size_t)e * 2 + 1]));
    if (v.dbg_lame) v.dbg_lame[k * N + i] = th;
    // 1D and 2D: the edge's F* record in registers, and f^LxW formed from it as k_edge formed the
    // one the limiter used (one record read instead of two); 3D: f^LxW as stored (a face record of
    // 7 points per face, four faces in flight, would not fit the registers)
    R fsr[NQE][V];
    double W[V];
    if constexpr (DIM == 3) {
#pragma unroll
      for (int c = 0; c < V; ++c) W[c] = v.fLxW[(size_t)e * V + c];
    } else {
#pragma unroll
      for (int jj = 0; jj < NQE; ++jj)
#pragma unroll
        for (int c = 0; c < V; ++c) fsr[jj][c] = v.fstar[(size_t)e * (NQE * V) + jj * V + c];
      lxw_average<E, R>(T, fsr, W);
    }
#pragma unroll
    for (int c = 0; c < V; ++c) qb[c] -= r * ep * (th * W[c] + (1.0 - th) * v.fLxF[(size_t)e * V + c]);
    const R re = R(r * ep);
    const int perm = (DIM == 3) ? at(v.fperm + (size_t)k * N, i) : 0;
#pragma unroll
    for (int jl = 0; jl < NQE; ++jl) {
      const int jj = (DIM == 3) ? T.pperm[perm][jl] : (side ? (NQE - 1 - jl) : jl);
#pragma unroll
      for (int c = 0; c < V; ++c) {
        const R fs = re * ((DIM == 3) ? v.fstar[(size_t)e * (NQE * V) + jj * V + c] : fsr[jj][c]);
#pragma unroll
        for (int l = 1; l < ML; ++l) Qh[c][l - 1] -= T.ephi[k][jl][l] * fs;
      }
    }
  }
  if (idle) return;
  bool finite = true;
#pragma unroll
  for (int c = 0; c < V; ++c) {
    v.Qbar[(size_t)i * V + c] = qb[c];
    finite = finite && isfinite(qb[c]);
#pragma unroll
    for (int l = 0; l < ML - 1; ++l) at(v.Qh + (size_t)(c * (ML - 1) + l) * N, i) = Qh[c][l];
  }
  if (!finite) report(v.err, E_NONFINITE, i);
  else if (!(qb[0] > 0.0) || !(pressure<DIM>(qb, v.gamma) > 0.0)) report(v.err, E_POSITIVITY, i);
  // The first element of each mesh ends the mesh's step: t += dt, the wave-speed maximum is reset
  // and the shock-capturing limiter becomes due.  Every lane has read dt above and no kernel of
  // this step reads the fields written here.
  if (i == 0 || (v.mesh_of && at(v.mesh_of, i - 1) != mid)) {
    Scalars& S = v.sc[mid];
    S.t += dt;
    S.steps += 1;
    S.s_bits = 0ull;
    S.shock_pending = v.shock ? 1 : 0;
  }
}

template <class E, class R>
__global__ __launch_bounds__(256) void k_update(View<R> v) {
  update_item<E, R>(v, xcd_item());
}

// ---------------------------------------------------------------------------------------------
// k_persist: n_steps whole steps of a batch of meshes in one cooperative launch.  Every workgroup
// stays resident and runs each phase of the step (the bodies of k_pre, k_dt, k_elem, k_edge,
// k_flim, k_update) over tiles of elements or edges, with a grid-wide barrier where the separate
// launches have a kernel boundary; the arithmetic is that of the separate kernels, so the results
// are the same bit for bit.  The grid is a multiple of 8 workgroups: workgroup b runs on XCD b mod 8,
// and the tiles of each XCD are one contiguous range of the space-filling-curve order.
// ---------------------------------------------------------------------------------------------
template <class E, class R, int pmode>
__global__ __launch_bounds__(256, (ElemOcc<E, R>::waves)) void k_persist(View<R> v, int n_mesh, int n_steps) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int bs = (int)blockDim.x, nb = (int)gridDim.x;
  const int x = (int)blockIdx.x & 7, r = (int)blockIdx.x >> 3, per = nb >> 3;
  auto tiles = [&](int n_items, auto&& body) {
    const int nt = (n_items + bs - 1) / bs;
    const int t0 = (int)((long long)nt * x / 8), t1 = (int)((long long)nt * (x + 1) / 8);
    for (int t = t0 + r; t < t1; t += per) body(t * bs + (int)threadIdx.x);
  };
  for (int step = 0; step < n_steps; ++step) {
    tiles(v.N, [&](int i) { pre_item<E, R, pmode>(v, i); });
    grid.sync();
    for (int m = (int)(blockIdx.x * blockDim.x + threadIdx.x); m < n_mesh; m += nb * bs) dt_mesh(v.sc, v.err, m);
    grid.sync();
    tiles(v.N, [&](int i) { elem_item<E, R>(v, i); });
    grid.sync();
    tiles(v.E, [&](int e) { edge_tile<E, R>(v, e); });
    grid.sync();
    tiles(v.N, [&](int i) { flim_item<E, R>(v, i); });
    grid.sync();
    tiles(v.N, [&](int i) { update_item<E, R>(v, i); });
    grid.sync();
  }
}

template <class E, class R>
hipError_t launch_persistent(const View<R>& v, int bs, hipStream_t st, int n_mesh, int n_steps) {
  if (bs != 128 && bs != 256) return hipErrorInvalidConfiguration;
  if (!v.mesh_of || n_steps < 1 || E::kind != ElTri::kind) return hipErrorInvalidValue;
  const void* fn = nullptr;
  switch ((v.theta_exact ? 1 : 0) + (v.s_avg ? 2 : 0)) {
    case 0: fn = reinterpret_cast<const void*>(&k_persist<E, R, 0>); break;
    case 1: fn = reinterpret_cast<const void*>(&k_persist<E, R, 3>); break;
    case 2: fn = reinterpret_cast<const void*>(&k_persist<E, R, 4>); break;
    default: fn = reinterpret_cast<const void*>(&k_persist<E, R, 5>); break;
  }
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, bs, 0);
  if (e != hipSuccess) return e;
  // every workgroup must be resident for the grid barriers; a multiple of 8 for the XCD mapping
  const int nb = per_cu * prop.multiProcessorCount / 8 * 8;
  if (nb < 8) return hipErrorCooperativeLaunchTooLarge;
  View<R> vv = v;
  void* args[] = {&vv, &n_mesh, &n_steps};
  return hipLaunchCooperativeKernel(fn, dim3((unsigned)nb), dim3((unsigned)bs), args, 0, st);
}

// Sets the end time of every mesh (a kernel, so that it is ordered on the stream and may be
// captured).
__global__ void k_set_end(Scalars* sc, int n_mesh, double T) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n_mesh) sc[m].T = T;
}

hipError_t launch_set_end(Scalars* sc, int n_mesh, double T, hipStream_t st) {
  hipLaunchKernelGGL(k_set_end, dim3((unsigned)((n_mesh + 63) / 64)), dim3(64), 0, st, sc, n_mesh, T);
  return hipGetLastError();
}

// k_final: marks the pending shock-capturing limiter as applied (after a state read-out applied
// it).
__global__ void k_final(Scalars* sc, int n_mesh) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_mesh) return;
  sc[m].shock_pending = 0;
}

template <class E, class R>
hipError_t launch(KernelId k, const View<R>& v, const LaunchCfg& cfg, hipStream_t st, int n_mesh, int mode) {
  auto grid = [](int n, int b) { return dim3((unsigned)((n + b - 1) / b)); };
  // element and edge kernels: grid padded to a multiple of 8 blocks (XCD-contiguous block order)
  auto egrid = [](int n, int b) { return dim3((unsigned)egrid_blocks(n, b)); };
  const int bs = (k == K_SHOCK) ? cfg.bs[K_PRE] : (tunable(k) ? cfg.bs[k] : 0);
  if (tunable(k == K_SHOCK ? K_PRE : k) && bs != 64 && bs != 128 && bs != 256) return hipErrorInvalidConfiguration;
  switch (k) {
    case K_PRE:
      if (v.N > 0) {
        switch ((v.theta_exact ? 1 : 0) + (v.s_avg ? 2 : 0)) {
          case 0: hipLaunchKernelGGL((k_pre<E, R, 0>), egrid(v.N, bs), dim3(bs), 0, st, v); break;
          case 1: hipLaunchKernelGGL((k_pre<E, R, 3>), egrid(v.N, bs), dim3(bs), 0, st, v); break;
          case 2: hipLaunchKernelGGL((k_pre<E, R, 4>), egrid(v.N, bs), dim3(bs), 0, st, v); break;
          default: hipLaunchKernelGGL((k_pre<E, R, 5>), egrid(v.N, bs), dim3(bs), 0, st, v); break;
        }
      }
      break;
    case K_SHOCK:
      if (mode != 1 && mode != 2) return hipErrorInvalidValue;
      if (v.N > 0) {
        if (mode == 1) hipLaunchKernelGGL((k_pre<E, R, 1>), egrid(v.N, bs), dim3(bs), 0, st, v);
        else hipLaunchKernelGGL((k_pre<E, R, 2>), egrid(v.N, bs), dim3(bs), 0, st, v);
      }
      break;
    case K_IND:
      return hipErrorInvalidValue;  // launched through launch_indicator
    case K_DT:
      if (v.mesh_of) hipLaunchKernelGGL(k_dt, grid(n_mesh, 64), dim3(64), 0, st, v.sc, v.err, n_mesh);
      else hipLaunchKernelGGL(k_dt_single, dim3(1), dim3(1024), 0, st, v.sc, v.err, v.spart,
                              v.N > 0 ? egrid_blocks(v.N, cfg.bs[K_PRE]) : 0);
      break;
    case K_ELEM:
      if (v.N > 0) hipLaunchKernelGGL((k_elem<E, R>), egrid(v.N, bs), dim3(bs), 0, st, v);
      break;
    case K_EDGE:
      if (v.E > 0) hipLaunchKernelGGL((k_edge<E, R>), egrid(v.E, bs), dim3(bs), 0, st, v);
      break;
    case K_FLIM:
      if (v.N > 0) hipLaunchKernelGGL((k_flim<E, R>), egrid(v.N, bs), dim3(bs), 0, st, v);
      break;
    case K_UPDATE:
      if (v.N > 0) hipLaunchKernelGGL((k_update<E, R>), egrid(v.N, bs), dim3(bs), 0, st, v);
      break;
    case K_FINAL:
      if (mode != 1) return hipErrorInvalidValue;  // the step itself ends in k_update
      hipLaunchKernelGGL(k_final, grid(n_mesh, 64), dim3(64), 0, st, v.sc, n_mesh);
      break;
  }
  return hipGetLastError();
}

template hipError_t launch_persistent<ElLine, double>(const View<double>&, int, hipStream_t, int, int);
template hipError_t launch_persistent<ElLine, float>(const View<float>&, int, hipStream_t, int, int);
template hipError_t launch_persistent<ElQuad, double>(const View<double>&, int, hipStream_t, int, int);
template hipError_t launch_persistent<ElQuad, float>(const View<float>&, int, hipStream_t, int, int);
template hipError_t launch_persistent<ElTri, double>(const View<double>&, int, hipStream_t, int, int);
template hipError_t launch_persistent<ElTri, float>(const View<float>&, int, hipStream_t, int, int);
template hipError_t launch<ElLine, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElLine, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElQuad, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElQuad, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTri, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTri, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElLine3, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElLine3, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTri3, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTri3, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTet, double>(KernelId, const View<double>&, const LaunchCfg&, hipStream_t, int, int);
template hipError_t launch<ElTet, float>(KernelId, const View<float>&, const LaunchCfg&, hipStream_t, int, int);

}  // namespace lxw
