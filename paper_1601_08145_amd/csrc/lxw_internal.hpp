// Internal declarations shared by the host runtime (lxw_host.cpp) and the kernels
// (lxw_kernels.hip) of the LxW-DG library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lxw {

// ---- Element configurations (Sec. 1.2): P2 on the line, tensor Q2 on quads, P2 on triangles,
// and the degree-3 forms P3 on the line and on triangles (the construction of Sec. 2.2 carried one
// order further).  NI interior quadrature points, K faces with NQE Gauss points each; NP = NI +
// K*NQE limiter points (Sec. 3.1 uses exactly the points of the update); NC = 2^K - 1 pressure
// corners (Sec. 3.3 Step 5a); ND2 / ND3 independent second / third reference derivatives.
struct ElLine {
  static constexpr int kind = 0, DEG = 2, DIM = 1, V = 3, ML = 3, K = 2, NI = 3, NQE = 1;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 1, ND3 = 1;
};
struct ElQuad {
  static constexpr int kind = 1, DEG = 2, DIM = 2, V = 4, ML = 9, K = 4, NI = 9, NQE = 3;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 3, ND3 = 1;
};
struct ElTri {
  static constexpr int kind = 2, DEG = 2, DIM = 2, V = 4, ML = 6, K = 3, NI = 7, NQE = 3;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 3, ND3 = 1;
};
struct ElLine3 {
  static constexpr int kind = 0, DEG = 3, DIM = 1, V = 3, ML = 4, K = 2, NI = 4, NQE = 1;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 1, ND3 = 1;
};
struct ElTri3 {
  static constexpr int kind = 2, DEG = 3, DIM = 2, V = 4, ML = 10, K = 3, NI = 16, NQE = 4;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 3, ND3 = 4;
};
// P2 on tetrahedra (3D; the paper's closing remark of Sec. 3.3): 27 interior points, four faces of
// 7 points, 15 pressure corners, second derivatives xx, xy, xz, yy, yz, zz.
struct ElTet {
  static constexpr int kind = 3, DEG = 2, DIM = 3, V = 5, ML = 10, K = 4, NI = 27, NQE = 7;
  static constexpr int NP = NI + K * NQE, NC = (1 << K) - 1, ND2 = 6, ND3 = 1;
};

// Reference tables of one element kind in one precision, kept in __constant__ memory so that
// every lane of a wave (one element per lane) reads the same entry through the scalar cache.
// Points are ordered interior first, then edge k, Gauss point j (counter-clockwise along k).
template <class E, class R>
struct RefTab {
  R phi[E::NP][E::ML];             // basis values
  R dphi[E::NP][E::DIM][E::ML];    // reference gradient
  R d2phi[E::NP][E::ND2][E::ML];   // reference second derivatives (xx[, xy, yy])
  R wphi[E::NI][E::ML];            // w_m phi_l(x_m): projection onto the basis
  R wdphi[E::NI][E::DIM][E::ML];   // w_m grad phi_l(x_m): volume term
  R kd0[E::NI][E::DIM];            // sum_l w_m phi_l(x_m) d phi_l/d xi_a (origin): the projection of
                                   // Step 1 composed with div at the reference origin
  R kd1[E::NI][E::DIM][E::DIM];    // sum_l w_m phi_l(x_m) d2 phi_l/d xi_a d xi_b (origin): the same
                                   // with the gradient of div (complete P2, affine elements)
  R kd2[E::DEG == 3 ? E::NI : 1][E::DIM][2 * E::DIM - 1];  // degree 3: the same with the (constant)
                                   // second derivatives of div, index j = eta derivatives of the pair
  R ephi[E::K][E::NQE][E::ML];     // (1/2) omega_j phi_l(x_kj): edge term of the update
  R om[E::NQE];                    // Gauss-Legendre weights on [-1, 1]
  R xr[E::NP][E::DIM];             // reference coordinates of the points
  R dphi0[E::DIM][E::ML];          // reference gradient at the reference origin
  R d2c[E::ND2][E::ML];            // reference second derivatives at the origin (constant for
                                   // complete P2 on the line and the triangle)
  R d3c[E::ND3][E::ML];            // reference third derivatives (xxx[, xxy, xyy, yyy]): constant
                                   // for complete P3, unused at degree 2
  int pperm[6][E::NQE];            // tetrahedron faces: point jl of a face whose vertices are those
                                   // of the first element's face permuted by permutation p is that
                                   // face's point pperm[p][jl] (p = 0 the identity); unused in 1D/2D
};

// Per-mesh device scalars (one record per mesh; the batched form holds many).
struct Scalars {
  unsigned long long s_bits;  // global wave speed as the bit pattern of a non-negative double
  double s, dt, t;
  double T;                   // end time: dt is clipped to reach it; at t >= T a step changes nothing
  double geo;                 // max_i |dT_i| / (2|T_i|)
  double cfl;
  int shock_pending;          // the shock-capturing limiter of the previous step is still due
  int idle;                   // set by k_dt when t >= T: the rest of the step changes nothing
  long long steps;
};

// Device error record: first error wins (atomicCAS on code).
struct DevError {
  int code;
  int elem;
};

// Boundary codes stored in an element's edge slot (slot = edge*8 + side*4 + bc).
enum { SB_INTERIOR = 0, SB_TRANSPARENT = 1, SB_REFLECTIVE = 2, SB_INFLOW = 3 };

// Everything a kernel needs, passed by value.  R is the arithmetic of the bulk (double for
// LXW_FP64, float for LXW_FP32_MIXED); cell averages and the flux limiter are always double.
template <class R>
struct View {
  int N, E;
  // elements (internal order)
  const double* area;     // [N]
  const R* Jinv;          // [DIM*DIM][N], Jinv[a][d] = d xi_a / d x_d
  const R* nout;          // [K][DIM][N] outward normal of local edge k, length = edge length
  const int* eslot;       // [K][N] edge*8 + side*4 + boundary code
  const unsigned char* fperm;  // tetrahedra: [K][N] permutation of the face's vertices relative to
                               //   the face's first element (RefTab::pperm); null in 1D/2D
  const int* nbr;         // [K][N] neighbour element or -1
  const double* delta;    // [N] shock-limiter relaxation alpha0 h^1.5
  const int* mesh_of;     // [N] mesh index (batched form) or null
  // edges
  const int* e_i;         // [E] element i_e (n_e points out of it)
  const int* e_j;         // [E] element j_e or -1
  const int* e_bc;        // [E] boundary code (SB_*)
  const double* e_n;      // [DIM][E] n_e, |n_e| = edge length
  const int* e_mesh;      // [E] mesh index or null
  // state
  double* Qbar;           // [N][V] cell averages (array of structures: the kernels also gather
                          //   them by neighbour index, and one element's averages then share
                          //   a cache line)
  R* Qh;                  // [V][ML-1][N] modes 2..ML
  // work
  double* theta;          // [N] limiter factor of the step (shock x moment), applied by k_elem
  R* tr;                  // [2][E][NQE][V] one trace per edge side (side 0 = i_e, side 1 = j_e or
                          //   the ghost state), n_out . F_T / 2 + (s |n_e| / 2) q of that side,
                          //   so that F*_T . n_e = side 0 - side 1; points in i_e's order along
                          //   the edge: one record per edge side, written by the element with
                          //   vector stores, read by k_edge with coalesced vector loads
  // Per-edge records (array of structures): the element kernels gather them by edge index, and
  // one record spans one or two cache lines instead of one line per component.
  R* fstar;               // [E][NQE][V] F*_T . n_e at the edge points
  double* fLxW;           // [E][V] f^LxW of edge e (read by the flux limiter; k_update forms it
                          //   again from the F* record, bit for bit)
  double* fLxF;           // [E][V] f^LxF of edge e
  double* cedge;          // [E][2] damping candidate of each side (1 on a ghost side)
  const unsigned char* ind_flag;  // [N] learned indicator decision (0: the shock-capturing limiter
                                 //   is skipped) or null (plain detection everywhere)
  Scalars* sc;
  DevError* err;
  double* spart;          // [blocks of k_pre] per-block maximum wave speed (single-mesh form)
  // parameters
  double gamma, eps0;
  double inflow[4];
  int shock;
  int theta_exact;        // moment limiter Step 2 by the exact root (k_pre modes 3, 5) instead of concavity
  int s_avg;              // global wave speed from the cell averages only (k_pre modes 4, 5)
  // diagnostics (null unless requested)
  double* dbg_theta;      // [N]
  double* dbg_theta_sc;   // [N]
  double* dbg_vol;        // [V][ML][N]
  double* dbg_lame;       // [K][N]
  double* dbg_qlim;       // [V][ML][N] limited state at the start of the step
};

// Entry i of a structure-of-arrays column that starts at `col` (a pointer the whole wavefront
// shares).  The byte offset is formed in 32 bits (i < 2^29, and no column reaches 4 GiB), so the
// address is the shared base plus the lane's offset: without this the compiler keeps one 64-bit
// vector address per column live across a burst of loads, which costs more registers than the
// data itself.
template <class T>
__device__ __forceinline__ T& at(T* col, int i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(col) + (unsigned)i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T& at(const T* col, int i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(col) + (unsigned)i * (unsigned)sizeof(T));
}

// All reference tables in both precisions (built on the host by lxw_host.cpp).
struct HostTabs {
  RefTab<ElLine, double> line_d;
  RefTab<ElLine, float> line_f;
  RefTab<ElQuad, double> quad_d;
  RefTab<ElQuad, float> quad_f;
  RefTab<ElTri, double> tri_d;
  RefTab<ElTri, float> tri_f;
  RefTab<ElLine3, double> line3_d;
  RefTab<ElLine3, float> line3_f;
  RefTab<ElTri3, double> tri3_d;
  RefTab<ElTri3, float> tri3_f;
  RefTab<ElTet, double> tet_d;
  RefTab<ElTet, float> tet_f;
};
// Constant memory on gfx950 is ordinary device memory read through the scalar cache (there is no
// 64 KiB constant bank); the tables are kept well within a few hundred KiB.
static_assert(sizeof(HostTabs) <= 256 * 1024, "reference tables larger than intended");

// ---- host-side launchers implemented in lxw_kernels.hip -----------------------------------
hipError_t upload_tables(const HostTabs& t);
// End time of every mesh (stream-ordered): steps are clipped to reach it and change nothing after.
hipError_t launch_set_end(Scalars* sc, int n_mesh, double T, hipStream_t st);

enum KernelId { K_PRE = 0, K_DT = 1, K_ELEM = 2, K_EDGE = 3, K_FLIM = 4, K_UPDATE = 5, K_FINAL = 6, K_IND = 7,
                K_SHOCK = 8 };

// Workgroup size (one lane per element or edge, so also elements or edges per workgroup) of each
// kernel, indexed by KernelId; the scalar kernels (K_DT, K_FINAL) and the indicator (K_IND, one
// wavefront per 64 elements) have fixed shapes.  Every
// tunable kernel accepts 64, 128 or 256.
struct LaunchCfg {
  int bs[8] = {256, 0, 128, 256, 256, 256, 0, 0};
  int persistent = 0;  // batches: 0 per-phase launches (graph replay), else k_persist with this workgroup size
};
inline bool tunable(int k) { return k == K_PRE || k == K_ELEM || k == K_EDGE || k == K_FLIM || k == K_UPDATE; }
// Number of workgroups of an element or edge kernel: padded to a multiple of 8 (one contiguous
// range of workgroups per XCD).
inline int egrid_blocks(int n, int bs) { return ((n + bs - 1) / bs + 7) / 8 * 8; }

template <class E, class R>
hipError_t launch(KernelId k, const View<R>& v, const LaunchCfg& cfg, hipStream_t st, int n_mesh, int mode);
// n_steps whole steps of a batch (v.mesh_of set) in one cooperative launch of workgroups of bs
// lanes (64, 128 or 256), as many as stay resident together; same results as the separate kernels.
template <class E, class R>
hipError_t launch_persistent(const View<R>& v, int bs, hipStream_t st, int n_mesh, int n_steps);

// ---- learned troubled-cell indicator (lxw_indicator.hip) ------------------------------------
// Network 48 -> 64 (ReLU) -> 64 (ReLU) -> 1 (sigmoid); flat FP32 parameters W1[48][64], b1[64],
// W2[64][64], b2[64], w3[64], b3.
constexpr int IND_NIN = 48, IND_NH = 64;
constexpr int IND_NPARAM = IND_NIN * IND_NH + IND_NH + IND_NH * IND_NH + IND_NH + IND_NH + 1;  // 7361
constexpr int IND_OFF_W1 = 0, IND_OFF_B1 = 3072, IND_OFF_W2 = 3136, IND_OFF_B2 = 7232, IND_OFF_W3 = 7296,
              IND_OFF_B3 = 7360;
constexpr int IND_PART = 7368;  // stride of one block's partial gradient (7361 gradients, loss, pad)

// Inference weights in the lane layout of the 32x32x16 bf16 matrix instruction (packed on the
// host from the FP32 parameters).  uint16_t holds bfloat16 bit patterns.
struct IndW {
  const uint16_t* A1;  // [2 row tiles][3 k-steps][64 lanes][8]
  const uint16_t* A2;  // [2 row tiles][4 k-steps][64 lanes][8]
  const float* b1;     // [2 row tiles][2 lane halves][16 accumulator registers]
  const float* b2;     // same layout
  const float* w3;     // same layout, then b3 at index 64
  float tau_lo, tau_hi;
};

// Inference over the solver's elements: decisions flag[N] and per-workgroup decision counts
// counts[IND_GRID_MAX][3], each workgroup adding to its own row (no two workgroups share a
// counter); the caller sums the rows.
constexpr int IND_GRID_MAX = 2048;
template <class R>
hipError_t launch_indicator(const View<R>& v, const IndW& W, unsigned char* flag, unsigned long long* counts,
                            bool in_step, hipStream_t st);
template <class R>
hipError_t launch_features(const View<R>& v, float* X, hipStream_t st);
hipError_t launch_predict(const IndW& W, const float* X, int n, float* p, hipStream_t st);
// Training: per-block partial gradients of the class-weighted cross-entropy over samples
// order[base + s] (s < n; order null: base + s), then the in-order reduction and, with adam != 0,
// the Adam update of theta / m / v (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t).
struct TrainArgs {
  const float* X;       // [n_samples][48]
  const float* y;       // [n_samples]
  const int* order;     // sample indices (clamped to [0, n_samples))
  int n_samples;
  int base, n;
  float w_pos, w_neg, inv_n;
  const float* theta;
  float* part;
};
hipError_t launch_mlp_grad(const TrainArgs& a, hipStream_t st);
hipError_t launch_mlp_reduce(int nblk, const float* part, float* theta, float* m, float* v, float* grad_out,
                             float* loss_out, int adam, float lr, float b1, float b2, float eps, float bc1,
                             float bc2, hipStream_t st);
inline int mlp_blocks(int n) { return (n + 63) / 64; }

// Fixed device workspace of the gradient entry point that allocates nothing: the per-workgroup
// partial gradients of at most IND_STATIC_MAX_SAMPLES samples (one workgroup per 64 samples).
constexpr int IND_STATIC_MAX_SAMPLES = 8192;
constexpr int IND_STATIC_BLOCKS = IND_STATIC_MAX_SAMPLES / 64;
constexpr size_t IND_STATIC_FLOATS = (size_t)IND_STATIC_BLOCKS * IND_PART;  // 3.6 MiB
// Device address of that workspace on the current device (looked up once per device with
// hipGetSymbolAddress and kept).
hipError_t ind_static_scratch(float** out);

}  // namespace lxw
