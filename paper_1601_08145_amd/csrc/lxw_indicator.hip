// Learned troubled-cell indicator for P2 triangles: features, inference on the bf16 matrix cores,
// and the FP32 training kernels (forward, backward, in-order gradient reduction, Adam).
//
// The paper detects troubled cells with the shock-capturing limiter it cites (Sec. 1.5 Step 5,
// Sec. 4.1).  Here a multilayer perceptron 48 -> 64 (ReLU) -> 64 (ReLU) -> 1 (sigmoid) predicts
// whether that limiter will act on a cell; cells it clears skip the limiter, every other cell runs
// it unchanged, and the positivity limiters of Secs. 3.1-3.3 always run.
//
// Features of cell i: cells c = (i, n_0, n_1, n_2) (n_k the neighbour across local edge k, i on
// the boundary); for rho and E the 24 modal coefficients Q[c][var][l] with the centre average
// subtracted from the mode-1 entries, divided by (max |value| + delta_i + 1e-6 |centre average| +
// 1e-30) with delta_i = alpha0 h_i^1.5 the shock-capturing limiter's relaxation; index
// var*24 + c*6 + l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "lxw_internal.hpp"

namespace lxw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// ---- features ---------------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void cell_features(const View<R>& v, int i, float (&F)[IND_NIN]) {
  constexpr int ML = ElTri::ML;
  const int N = v.N;
  int cells[4] = {i, i, i, i};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int j = at(v.nbr + (size_t)k * N, i);
    cells[k + 1] = j >= 0 ? j : i;
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int c = g == 0 ? 0 : 3;  // rho, E
    const double avg = v.Qbar[(size_t)i * ElTri::V + c];
    float vals[24];
    float mx = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cell = cells[q];
      vals[q * 6] = float(v.Qbar[(size_t)cell * ElTri::V + c] - avg);
#pragma unroll
      for (int l = 1; l < ML; ++l) vals[q * 6 + l] = float(at(v.Qh + (size_t)(c * (ML - 1) + l - 1) * N, cell));
    }
#pragma unroll
    for (int x = 0; x < 24; ++x) mx = fmaxf(mx, fabsf(vals[x]));
    // floor: the shock-capturing limiter's relaxation delta_i (variations far below it give
    // features near zero) and a relative 1e-6 (a uniform region's round-off stays near zero)
    const float rs = 1.0f / (mx + float(at(v.delta, i) + 1e-6 * fabs(avg)) + 1e-30f);
#pragma unroll
    for (int x = 0; x < 24; ++x) F[g * 24 + x] = vals[x] * rs;
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_feat(View<R> v, float* X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.N) return;
  float F[IND_NIN];
  cell_features<R>(v, i, F);
#pragma unroll
  for (int f = 0; f < IND_NIN; ++f) X[(size_t)i * IND_NIN + f] = F[f];
}

// ---- inference: one wavefront evaluates the network for 64 cells ------------------------------
// 32x32x16 bf16 matrix instruction, lane l (half h = l / 32):
//   A operand (32 rows x 16 k): row l % 32, k = 8h .. 8h+7;  B operand (16 k x 32 columns): column
//   l % 32, k = 8h .. 8h+7;  accumulator register r: row 8(r/4) + 4h + r%4, column l % 32.
// Cells are the columns: cell 32t + n of the wave is column n of column tile t.  Hidden units are
// rows (two row tiles of 32).  The first layer's k runs over the 48 features in three steps; the
// second layer's k runs over the first layer's accumulator registers in the order they sit in the
// lanes, and its weights are packed in that order, so no data moves between lanes there.
__device__ __forceinline__ bf16x8 swap_halves(bf16x8 x) {
  i32x4 w = __builtin_bit_cast(i32x4, x);
  w.x = __shfl_xor(w.x, 32);
  w.y = __shfl_xor(w.y, 32);
  w.z = __shfl_xor(w.z, 32);
  w.w = __shfl_xor(w.w, 32);
  return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p) {
  const i32x4 w = *reinterpret_cast<const i32x4*>(p);
  return __builtin_bit_cast(bf16x8, w);
}

// The packed weights, staged in LDS once per workgroup (14.8 KB).
struct IndLds {
  uint16_t A1[2 * 3 * 64 * 8];
  uint16_t A2[2 * 4 * 64 * 8];
  float b1[64], b2[64], w3[65];
};

__device__ __forceinline__ void stage_weights(IndLds& L, const IndW& W) {
  const int t = threadIdx.x, nt = blockDim.x;
  const i32x4* a1 = reinterpret_cast<const i32x4*>(W.A1);
  const i32x4* a2 = reinterpret_cast<const i32x4*>(W.A2);
  i32x4* l1 = reinterpret_cast<i32x4*>(L.A1);
  i32x4* l2 = reinterpret_cast<i32x4*>(L.A2);
  for (int x = t; x < 2 * 3 * 64 * 8 / 8; x += nt) l1[x] = a1[x];
  for (int x = t; x < 2 * 4 * 64 * 8 / 8; x += nt) l2[x] = a2[x];
  for (int x = t; x < 64; x += nt) { L.b1[x] = W.b1[x]; L.b2[x] = W.b2[x]; }
  for (int x = t; x < 65; x += nt) L.w3[x] = W.w3[x];
  __syncthreads();
}

// Logit of the lane's own cell (all 64 lanes must call this together).
__device__ __forceinline__ float mlp_logit(const float (&F)[IND_NIN], const IndLds& W) {
  const int l = threadIdx.x & 63, h = l >> 5;
  bf16x8 own[3], other[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    bf16x8 mine, send;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float lo = F[16 * s + e], hi = F[16 * s + 8 + e];  // static indices: F stays in registers
      mine[e] = (__bf16)(h ? hi : lo);
      send[e] = (__bf16)(h ? lo : hi);
    }
    own[s] = mine;
    other[s] = swap_halves(send);  // the partner cell's features for this lane's k range
  }
  // layer 1, one 32 x 32 tile at a time, each followed by its bias, ReLU and bf16 rounding (the
  // second layer's B operands): only one accumulator tile is live
  bf16x8 H[2][2][2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const float* bb = W.b1 + (mt * 2 + h) * 16;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x16 a = {};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const bf16x8 A = load_bf16x8(W.A1 + ((mt * 3 + s) * 64 + l) * 8);
        const bf16x8 B = (t == h) ? own[s] : other[s];
        a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, a, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) H[mt][t][r >> 3][r & 7] = (__bf16)fmaxf(a[r] + bb[r], 0.0f);
    }
  }
  // layer 2
  float part[2] = {0.0f, 0.0f};
#pragma unroll 1  // unrolled, the two row tiles' weight, bias and output loads all stay live
  for (int mt2 = 0; mt2 < 2; ++mt2) {
    const float* bb = W.b2 + (mt2 * 2 + h) * 16;
    const float* ww = W.w3 + (mt2 * 2 + h) * 16;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x16 a = {};
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          const bf16x8 A = load_bf16x8(W.A2 + ((mt2 * 4 + mt * 2 + g) * 64 + l) * 8);
          a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, H[mt][t][g], a, 0, 0, 0);
        }
      // layer 3 on the lane's 16 hidden units of this row tile
#pragma unroll
      for (int r = 0; r < 16; ++r) part[t] += ww[r] * fmaxf(a[r] + bb[r], 0.0f);
    }
  }
  const float z0 = part[0] + __shfl_xor(part[0], 32);
  const float z1 = part[1] + __shfl_xor(part[1], 32);
  return (h == 0 ? z0 : z1) + W.w3[64];
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

// Decisions for the solver's elements: 0 skip the shock-capturing limiter (p < tau_lo), 2 flagged
// (p >= tau_hi), 1 otherwise.  Workgroups of 256 lanes stage the weights once and then walk over
// chunks of 256 elements (every lane of a workgroup runs the same number of chunks, as the matrix
// instructions need full wavefronts).  Workgroup b adds its decision counts to row b of
// counts[][3]: atomics of every wavefront on three shared counters serialise (about 8 ns each,
// over 100 us at a million cells).
// Three wavefronts per SIMD (168 registers, no spills): the feature gathers are latency-bound.
template <class R>
__global__ __launch_bounds__(256, 3) void k_ind(View<R> v, IndW W, unsigned char* flag, unsigned long long* counts,
                                                int in_step) {
  // a step of a single mesh at its end time changes nothing (the state read-out still decides)
  if (in_step && !v.mesh_of && !(v.sc[0].t < v.sc[0].T)) return;
  __shared__ IndLds Ls;
  stage_weights(Ls, W);
  const int nchunk = (v.N + 255) / 256;
  unsigned long long n0 = 0, n1 = 0, n2 = 0;
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int i = ch * 256 + threadIdx.x;
    const bool valid = i < v.N;
    float F[IND_NIN];
    if (valid) {
      cell_features<R>(v, i, F);
    } else {
#pragma unroll
      for (int f = 0; f < IND_NIN; ++f) F[f] = 0.0f;
    }
    const float p = sigmoidf(mlp_logit(F, Ls));
    const int d = p < W.tau_lo ? 0 : (p >= W.tau_hi ? 2 : 1);
    if (valid) flag[i] = (unsigned char)d;
    n0 += __popcll(__ballot(valid && d == 0));
    n1 += __popcll(__ballot(valid && d == 1));
    n2 += __popcll(__ballot(valid && d == 2));
  }
  __shared__ unsigned long long red[4][3];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[w][0] = n0; red[w][1] = n1; red[w][2] = n2; }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long s = 0;
    for (int x = 0; x < (int)(blockDim.x >> 6); ++x) s += red[x][threadIdx.x];
    counts[blockIdx.x * 3 + threadIdx.x] += s;
  }
}

__global__ __launch_bounds__(256, 3) void k_predict(IndW W, const float* X, int n, float* p) {
  __shared__ IndLds Ls;
  stage_weights(Ls, W);
  const int nchunk = (n + 255) / 256;
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int i = ch * 256 + threadIdx.x;
    const bool valid = i < n;
    float F[IND_NIN];
#pragma unroll
    for (int f = 0; f < IND_NIN; ++f) F[f] = valid ? X[(size_t)i * IND_NIN + f] : 0.0f;
    const float z = mlp_logit(F, Ls);
    if (valid) p[i] = sigmoidf(z);
  }
}

// ---- training: one wavefront of 64 samples per workgroup --------------------------------------
// Forward and backward per sample in FP32 registers (weights read uniformly by all lanes), then
// the weight gradients as sums over the workgroup's samples: g_W2 = H1^T DA2, g_W1 = X^T DA1,
// staged through LDS (rows padded by one word against bank conflicts).  Each workgroup writes
// its partial gradient and loss; k_mlp_reduce adds the partials in workgroup order.
__device__ __forceinline__ float softplusf(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

__global__ __launch_bounds__(64) void k_mlp_grad(TrainArgs a) {
  __shared__ float sX[64][IND_NIN + 1];
  __shared__ float sH1[64][IND_NH + 1];   // h1, later da1
  __shared__ float sDA2[64][IND_NH + 1];
  __shared__ float sS[64][IND_NH + 1];    // dz * h2
  __shared__ float sDZ[64];
  __shared__ float sL[64];
  const int tid = threadIdx.x;
  const int idx = a.base + blockIdx.x * 64 + tid;
  const bool valid = blockIdx.x * 64 + tid < a.n;
  int smp = valid ? (a.order ? a.order[idx] : idx) : 0;
  smp = smp < 0 ? 0 : (smp >= a.n_samples ? a.n_samples - 1 : smp);
  const float* th = a.theta;
  float x[IND_NIN];
#pragma unroll
  for (int k = 0; k < IND_NIN; ++k) {
    x[k] = valid ? a.X[(size_t)smp * IND_NIN + k] : 0.0f;
    sX[tid][k] = x[k];
  }
  const float yv = valid ? a.y[smp] : 0.0f;
  // forward
  float a1[IND_NH];
#pragma unroll
  for (int m = 0; m < IND_NH; ++m) a1[m] = th[IND_OFF_B1 + m];
#pragma unroll 4
  for (int k = 0; k < IND_NIN; ++k)
#pragma unroll
    for (int m = 0; m < IND_NH; ++m) a1[m] += x[k] * th[IND_OFF_W1 + k * IND_NH + m];
  float a2[IND_NH];
#pragma unroll
  for (int m = 0; m < IND_NH; ++m) a2[m] = th[IND_OFF_B2 + m];
#pragma unroll 4
  for (int k = 0; k < IND_NH; ++k) {
    const float hk = fmaxf(a1[k], 0.0f);
    sH1[tid][k] = hk;
#pragma unroll
    for (int m = 0; m < IND_NH; ++m) a2[m] += hk * th[IND_OFF_W2 + k * IND_NH + m];
  }
  float z = th[IND_OFF_B3];
#pragma unroll
  for (int m = 0; m < IND_NH; ++m) z += th[IND_OFF_W3 + m] * fmaxf(a2[m], 0.0f);
  const float p = 1.0f / (1.0f + expf(-z));
  // loss and dL/dz: log p = -softplus(-z), log(1 - p) = -softplus(z)
  const float loss = valid ? (a.w_pos * yv * softplusf(-z) + a.w_neg * (1.0f - yv) * softplusf(z)) * a.inv_n : 0.0f;
  const float dz = valid ? (a.w_pos * yv * (p - 1.0f) + a.w_neg * (1.0f - yv) * p) * a.inv_n : 0.0f;
  sDZ[tid] = dz;
  sL[tid] = loss;
  float da2[IND_NH];
#pragma unroll
  for (int m = 0; m < IND_NH; ++m) {
    sS[tid][m] = dz * fmaxf(a2[m], 0.0f);
    da2[m] = a2[m] > 0.0f ? dz * th[IND_OFF_W3 + m] : 0.0f;
    sDA2[tid][m] = da2[m];
  }
  float da1[IND_NH];
#pragma unroll 4
  for (int k = 0; k < IND_NH; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int m = 0; m < IND_NH; ++m) acc += th[IND_OFF_W2 + k * IND_NH + m] * da2[m];
    da1[k] = a1[k] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  float* out = a.part + (size_t)blockIdx.x * IND_PART;
  // g_W2[tid][m] = sum_b h1[b][tid] da2[b][m]
  {
    float g[IND_NH];
#pragma unroll
    for (int m = 0; m < IND_NH; ++m) g[m] = 0.0f;
    for (int b = 0; b < 64; ++b) {
      const float hv = sH1[b][tid];
#pragma unroll
      for (int m = 0; m < IND_NH; ++m) g[m] += hv * sDA2[b][m];
    }
#pragma unroll
    for (int m = 0; m < IND_NH; ++m) out[IND_OFF_W2 + tid * IND_NH + m] = g[m];
  }
  {
    float gb2 = 0.0f, gw3 = 0.0f;
    for (int b = 0; b < 64; ++b) { gb2 += sDA2[b][tid]; gw3 += sS[b][tid]; }
    out[IND_OFF_B2 + tid] = gb2;
    out[IND_OFF_W3 + tid] = gw3;
  }
  if (tid == 0) {
    float gb3 = 0.0f, ls = 0.0f;
    for (int b = 0; b < 64; ++b) { gb3 += sDZ[b]; ls += sL[b]; }
    out[IND_OFF_B3] = gb3;
    out[IND_NPARAM] = ls;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < IND_NH; ++k) sH1[tid][k] = da1[k];
  __syncthreads();
  // g_W1[k][tid] = sum_b x[b][k] da1[b][tid]; g_b1[tid] = sum_b da1[b][tid]
  {
    float g[IND_NIN];
#pragma unroll
    for (int k = 0; k < IND_NIN; ++k) g[k] = 0.0f;
    float gb1 = 0.0f;
    for (int b = 0; b < 64; ++b) {
      const float d = sH1[b][tid];
      gb1 += d;
#pragma unroll
      for (int k = 0; k < IND_NIN; ++k) g[k] += sX[b][k] * d;
    }
#pragma unroll
    for (int k = 0; k < IND_NIN; ++k) out[IND_OFF_W1 + k * IND_NH + tid] = g[k];
    out[IND_OFF_B1 + tid] = gb1;
  }
}

// Sum of the workgroup partials in workgroup order (deterministic); optional gradient output and
// Adam update (Kingma & Ba) of the FP32 master parameters.
__global__ __launch_bounds__(256) void k_mlp_reduce(int nblk, const float* part, float* theta, float* m, float* v,
                                                    float* grad_out, float* loss_out, int adam, float lr, float b1,
                                                    float b2, float eps, float bc1, float bc2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > IND_NPARAM) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += part[(size_t)b * IND_PART + j];
  if (j == IND_NPARAM) {
    if (loss_out) *loss_out = g;
    return;
  }
  if (grad_out) grad_out[j] = g;
  if (adam) {
    const float mj = b1 * m[j] + (1.0f - b1) * g;
    const float vj = b2 * v[j] + (1.0f - b2) * g * g;
    m[j] = mj;
    v[j] = vj;
    theta[j] -= lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
  }
}

// ---- fixed workspace of the no-allocation gradient entry point ---------------------------------
// Partial gradients of up to IND_STATIC_BLOCKS workgroups.  Every device the library runs on holds
// its own copy until the process ends.  Host code must not pass the array's name to a kernel (on
// the host it is only a stand-in for the symbol): its device address is looked up per device with
// hipGetSymbolAddress and kept, and that address is what the kernels get.  k_mlp_grad writes every
// entry k_mlp_reduce reads, so nothing needs clearing between calls; calls that overlap on one
// device share the array and race.
static __device__ __align__(256) float scratch[IND_STATIC_FLOATS];

hipError_t ind_static_scratch(float** out) {
  static std::mutex mu;
  static std::vector<float*> addr;  // per device, null until looked up
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<float*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// ---- launchers --------------------------------------------------------------------------------
template <class R>
hipError_t launch_indicator(const View<R>& v, const IndW& W, unsigned char* flag, unsigned long long* counts,
                            bool in_step, hipStream_t st) {
  if (v.N > 0)
    hipLaunchKernelGGL(k_ind<R>, dim3(std::min((v.N + 255) / 256, IND_GRID_MAX)), dim3(256), 0, st, v, W, flag, counts,
                       in_step ? 1 : 0);
  return hipGetLastError();
}

template <class R>
hipError_t launch_features(const View<R>& v, float* X, hipStream_t st) {
  if (v.N > 0) hipLaunchKernelGGL(k_feat<R>, dim3((v.N + 255) / 256), dim3(256), 0, st, v, X);
  return hipGetLastError();
}

hipError_t launch_predict(const IndW& W, const float* X, int n, float* p, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_predict, dim3(std::min((n + 255) / 256, 2048)), dim3(256), 0, st, W, X, n, p);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const TrainArgs& a, hipStream_t st) {
  if (a.n > 0) hipLaunchKernelGGL(k_mlp_grad, dim3(mlp_blocks(a.n)), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(int nblk, const float* part, float* theta, float* m, float* v, float* grad_out,
                             float* loss_out, int adam, float lr, float b1, float b2, float eps, float bc1,
                             float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3((IND_NPARAM + 1 + 255) / 256), dim3(256), 0, st, nblk, part, theta, m, v,
                     grad_out, loss_out, adam, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

template hipError_t launch_indicator<double>(const View<double>&, const IndW&, unsigned char*, unsigned long long*, bool,
                                             hipStream_t);
template hipError_t launch_indicator<float>(const View<float>&, const IndW&, unsigned char*, unsigned long long*, bool,
                                            hipStream_t);
template hipError_t launch_features<double>(const View<double>&, float*, hipStream_t);
template hipError_t launch_features<float>(const View<float>&, float*, hipStream_t);

}  // namespace lxw
