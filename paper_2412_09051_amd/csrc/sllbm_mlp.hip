// Learned post-collision correction on tensor-product meshes (gfx950).
//
// Node features (moments and their interpolant gradients), the network's forward pass on
// BF16 MFMA with FP32 accumulation, the projected correction added in place (one network per
// wave on v_mfma_f32_16x16x32_bf16, optionally fused with the relaxation of a tiled step),
// one-step training targets, restriction by injection, and training: a fused forward / loss /
// backward kernel per 32-row tile (v_mfma_f32_16x16x16_bf16) whose weight gradients are again
// MFMA products, written as per-workgroup partials and summed in a fixed order, then Adam on
// the FP32 master weights.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "sllbm_device_common.h"
#include "sllbm_internal.h"
#include "sllbm_kernels.h"

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess) return fail(SLLBM_EHIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

using namespace sllbm;

namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int R = 32;        // rows (nodes) per workgroup tile
constexpr int KIN = 32;      // inputs, padded
constexpr int HW = 64;       // hidden width
constexpr int NOUTP = 256;   // outputs, padded
constexpr int NT = 256;      // threads per workgroup (4 waves)
constexpr int WBF_W1 = 0, WBF_W2 = KIN * HW, WBF_W3 = KIN * HW + HW * HW, WBF_W4 = KIN * HW + 2 * HW * HW;
constexpr int WBF_N = KIN * HW + 2 * HW * HW + HW * NOUTP;
constexpr int kMaxPartialBlocks = 512;
// The correction kernels' LDS (about 76 KB) admits two workgroups per compute unit: a grid of
// two per CU stages the weights twice per CU and walks the node groups from there.
constexpr int64_t kCorrectGrid = 512;

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- MFMA tiles
// One wave computes a 16x16 tile D += A B over K (a multiple of 16).  Operand layout of
// v_mfma_f32_16x16x16_bf16 (wave64): lane l holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16]
// for j < 4, and receives D[4(l/16)+j][l%16].
__device__ inline float4_t mma_ab(const uint16_t *A, int lda, const uint16_t *B, int ldb, int K, float4_t acc) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    short4_t a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      a[j] = (short)A[r * lda + k0 + 4 * g + j];
      b[j] = (short)B[(k0 + 4 * g + j) * ldb + r];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}
// B given transposed: B(k, n) = Bt[n ldb + k]
__device__ inline float4_t mma_abt(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, int K, float4_t acc) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    short4_t a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      a[j] = (short)A[r * lda + k0 + 4 * g + j];
      b[j] = (short)Bt[r * ldb + k0 + 4 * g + j];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}
// A given transposed: A(m, k) = At[k lda + m]
__device__ inline float4_t mma_atb(const uint16_t *At, int lda, const uint16_t *B, int ldb, int K, float4_t acc) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    short4_t a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      a[j] = (short)At[(k0 + 4 * g + j) * lda + r];
      b[j] = (short)B[(k0 + 4 * g + j) * ldb + r];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// sum of v over the 16-row tile's rows for this lane's column (lanes r, r+16, r+32, r+48)
__device__ inline float tile_colsum(float4_t acc) {
  float s = acc[0] + acc[1] + acc[2] + acc[3];
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

struct MlpArgs {
  int n_in, n_out;
  const float *theta;     // master weights (biases read from here)
  const uint16_t *wbf;    // padded BF16 weights, each layer [in][out]
  const uint16_t *wbt;    // the correction kernels' stored layout (k_refresh_corr)
  int off[8];
};

struct FwdShared {
  uint16_t W[WBF_N];
  uint16_t X[R * KIN];
  uint16_t H[3][R * HW];
  float A[3][R * HW];
};

__device__ void stage_weights(const MlpArgs &m, uint16_t *W) {
  const uint32_t *src = (const uint32_t *)m.wbf;
  uint32_t *dst = (uint32_t *)W;
  for (int e = threadIdx.x; e < WBF_N / 2; e += NT) dst[e] = src[e];
}

__device__ void stage_x(const MlpArgs &m, const uint16_t *x, int64_t row0, int64_t rows, uint16_t *X) {
  for (int e = threadIdx.x; e < R * KIN; e += NT) {
    int r = e / KIN, c = e % KIN;
    int64_t gr = row0 + r;
    X[e] = (gr < rows && c < m.n_in) ? x[gr * m.n_in + c] : (uint16_t)0;
  }
}

// hidden layers: H[l] = tanh(in W_l + b_l), 2 x 4 tiles over 4 waves
__device__ void hidden_layers(const MlpArgs &m, FwdShared &S) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  for (int layer = 0; layer < 3; layer++) {
    const uint16_t *in = layer == 0 ? S.X : S.H[layer - 1];
    const int lda = layer == 0 ? KIN : HW, K = lda;
    const uint16_t *Wl = S.W + (layer == 0 ? WBF_W1 : (layer == 1 ? WBF_W2 : WBF_W3));
    const float *b = m.theta + m.off[2 * layer + 1];
    for (int t = wave; t < 8; t += 4) {
      const int rt = t & 1, ct = t >> 1;
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = mma_ab(in + rt * 16 * lda, lda, Wl + ct * 16, HW, K, acc);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
        float a = tanhf(acc[j] + b[col]);
        S.A[layer][row * HW + col] = a;
        S.H[layer][row * HW + col] = f2bf(a);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- forward only
__global__ void __launch_bounds__(NT) k_mlp_forward(MlpArgs m, const uint16_t *x, int64_t rows, float *y) {
  __shared__ FwdShared S;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  stage_weights(m, S.W);
  stage_x(m, x, row0, rows, S.X);
  __syncthreads();
  hidden_layers(m, S);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  const float *b4 = m.theta + m.off[7];
  for (int t = wave; t < 2 * (NOUTP / 16); t += 4) {
    const int rt = t & 1, ct = t >> 1;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma_ab(S.H[2] + rt * 16 * HW, HW, S.W + WBF_W4 + ct * 16, NOUTP, HW, acc);
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
      int64_t gr = row0 + row;
      if (gr < rows && col < m.n_out) y[gr * m.n_out + col] = acc[j] + b4[col];
    }
  }
}

// ---------------------------------------------------------------- correction in place
struct ProjArgs {
  int Q, D;
  const double *vel;       // [Q][8]: zeta xyz, xi xyz, |xi|^2, w
  double G[25];            // (M W M^T)^-1, (D+2) x (D+2)
};

// A node lies in a boundary layer of a bounded face (the gather kernel's nodes, relaxed
// there) if its index along the face axis is within the face's depth.
__device__ inline bool in_layer(const DevTensorPlan &pl, int64_t k) {
  const int Nx = pl.ax[0].N, Ny = pl.ax[1].N;
  for (int fc = 0; fc < pl.nfaces; fc++) {
    const DevFace &F = pl.face[fc];
    const int64_t n3 = F.axis == 0 ? k % Nx : (F.axis == 1 ? (k / Nx) % Ny : k / ((int64_t)Nx * Ny));
    const int64_t l = F.side == 0 ? n3 : pl.ax[F.axis].N - 1 - n3;
    if (l < F.depth) return true;
  }
  return false;
}

// Post-collision node fields (rho, u, T) [D+2][N] of a 3D tile step whose relaxation is still
// to come: for the tile's nodes from the node state the streaming launch stored (the
// collision keeps rho and T and Kupershtokh's difference adds F dt / rho to u), for the
// boundary layers (already relaxed by the gather launch) from their populations.
template <typename T>
__global__ void k_step_fields(const DevTensorPlan pl, const StepArgs sa, const double *nstate, const T *pop,
                              double *fld) {
  const int64_t N = pl.N;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double rho, u[3], Tk;
  if (in_layer(pl, k)) {
    const int Q = pl.Q;
    double j[3] = {0, 0, 0}, E = 0;
    rho = 0;
    for (int i = 0; i < Q; i++) {
      const double *vi = pl.vel + 8 * i;
      const double f = (double)pop[(size_t)i * N + k], g = (double)pop[((size_t)Q + i) * N + k];
      rho += f;
      double z2 = 0;
      for (int a = 0; a < 3; a++) {
        j[a] += vi[a] * f;
        z2 += vi[a] * vi[a];
      }
      E += z2 * f + g;
    }
    double uu = 0;
    for (int a = 0; a < 3; a++) {
      u[a] = j[a] / rho;
      uu += u[a] * u[a];
    }
    Tk = (E - rho * uu) / (2.0 * rho * sa.cv);
  } else {
    rho = nstate[k];
    Tk = nstate[4 * N + k];
    double F[3] = {0, 0, 0};
    if (sa.has_force) {
      for (int a = 0; a < 3; a++) F[a] = sa.force_dev ? sa.force_dev[a] : sa.force[a];
    }
    for (int a = 0; a < 3; a++) u[a] = nstate[(size_t)(1 + a) * N + k] + F[a] * sa.dt / rho;
  }
  fld[k] = rho;
  for (int a = 0; a < 3; a++) fld[(size_t)(1 + a) * N + k] = u[a];
  fld[4 * (size_t)N + k] = Tk;
}

// The correction kernels run one independent network per wave, 16 nodes at a time, on
// v_mfma_f32_16x16x32_bf16 with the layers evaluated transposed (D = W^T H^T, nodes as
// columns).  Lane l (r = l % 16, g = l / 16) supplies A[r][k(g, j)] and B[k(g, j)][r] for
// j < 8 and receives D[4 g + j][r] for j < 4, so after a layer it holds units 16 t + 4 g + j
// of node r for each 16-unit tile t.  Those eight values of tiles 2 b and 2 b + 1 are its B
// operand of the next layer's 32-deep K block b once the next layer's weight columns are
// stored in the matching order (hid_unit_of_col): activations never leave registers.  The
// output layer's rows are ordered so that a lane's four outputs of tile t are f and g of the
// velocities 8 t + 2 g and 8 t + 2 g + 1 (out_of_row), so that the population pass updates
// both populations of a velocity from one equilibrium evaluation.  The output layer runs
// twice, for the projection's invariant sums and again in the population pass (two MFMAs a
// tile, cheaper than holding 2Q outputs per node).  The weights (rows padded by 16 B against
// LDS bank conflicts), biases and velocity constants are staged once per workgroup; the waves
// then run without barriers.
// 8 waves per workgroup, two workgroups per CU (4 waves per SIMD, at most 128 VGPRs; the
// variants with both the Prandtl-number term and forcing spill a few registers, still faster
// than 6 waves without spills).  Population loads run PD tiles ahead of the tile computed.
// 64^3 cells p = 2 (2.1M nodes), FP32, per launch: correction alone 1.31 ms (D3V125) and
// 0.55 ms (D3Q45); fused with the relaxation 1.38 ms (D3V125), 0.65 / 0.99 ms (D3Q45 at
// Pr 1 / 0.71); 6 waves: 1.44, 0.73, 1.77 ms; one tile ahead: within 5 %.
constexpr int NTC = 512;
constexpr int PD = 2;
constexpr int KP1 = KIN + 8, KPH = HW + 8;    // LDS row strides (bf16) of layer 1 and of layers 2-4
constexpr int WC_W2 = HW * KP1, WC_W3 = WC_W2 + HW * KPH, WC_W4 = WC_W3 + HW * KPH;
constexpr int WC_N = WC_W4 + NOUTP * KPH;

// hidden unit held in stored column c (c = 32 b + 8 g + j) of a layer fed by a hidden layer
__host__ __device__ inline int hid_unit_of_col(int c) {
  const int b = c >> 5, g = (c >> 3) & 3, j = c & 7;
  return 32 * b + 16 * (j >> 2) + 4 * g + (j & 3);
}
// network output of the output layer's row R = 16 t + 4 g + j for Q velocities (f_v: v,
// g_v: Q + v), -1 for a padding row
__host__ __device__ inline int out_of_row(int R, int Q) {
  const int t = R >> 4, g = (R >> 2) & 3, j = R & 3;
  const int v = 8 * t + 2 * g + (j & 1);
  if (v >= Q) return -1;
  return (j >> 1) ? Q + v : v;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ inline float4_t mfma32(u32x4_t a, u32x4_t b, float4_t acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                 acc, 0, 0, 0);
}
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
// two values rounded to BF16 (nearest even, as f2bf) and packed, low half first
__device__ inline uint32_t pack_bf(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2_t{a, b}, bf16x2_t));
}
// An offset of zero the compiler cannot see through: LDS reads indexed with it are not hoisted
// out of the node-group loop or merged across its passes (the staged weights would otherwise
// be held in registers, well beyond the register budget, and spilled).
__device__ inline int opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// Population access of the correction kernels through buffer resources: the base (eight
// population planes from a wave-uniform plane) stays in scalar registers, each lane supplies
// a 32-bit byte offset, and an offset past the range (kOutOfRange) reads 0 and drops a store.
// Lanes without a population thus need no branch: loads under divergent branches would make
// the compiler wait for every load in flight before the next use, voiding the prefetch.
constexpr int kOutOfRange = 0x7ffffff0;
template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(T *pop, int64_t plane0, int64_t N) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)(pop + plane0 * N), (short)0, (int)(8 * N * (int64_t)sizeof(T)),
                                           0x00020000);
}
template <typename T> struct PopBuf;
template <> struct PopBuf<float> {
  __device__ static float load(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  __device__ static void store(__amdgpu_buffer_rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
  }
};
template <> struct PopBuf<double> {
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
  __device__ static double load(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  __device__ static void store(__amdgpu_buffer_rsrc_t r, int off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
  }
};

// tanh in FP32 for the correction kernels (the result is rounded to BF16 next): for |x| >=
// 1/8, sign(x) (1 - e) / (1 + e) with e = exp(-2 |x|) from the hardware exp2 and reciprocal
// (a few ulp); below, where 1 - e loses digits, the Taylor series to x^7 (truncation under
// 2e-10 relative at 1/8).
__device__ inline float tanh_fast(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * ax);   // 2 log2(e)
  const float big = (1.f - e) * __builtin_amdgcn_rcpf(1.f + e);
  const float x2 = x * x;
  const float small = ax * (1.f + x2 * (-1.f / 3.f + x2 * (2.f / 15.f + x2 * (-17.f / 315.f))));
  return copysignf(ax < 0.125f ? small : big, x);
}

// One tanh layer of 64 units: in[b] the B operands of the KB 32-deep K blocks, Wl the stored
// weights (row = unit, stride ld), out the B operands of the next layer.
template <int KB>
__device__ inline void corr_hidden(const uint16_t *Wl, int ld, const float *bias, const u32x4_t (&in)[KB],
                                   u32x4_t (&out)[2], int r, int g) {
#pragma unroll
  for (int t = 0; t < 4; t++) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < KB; b++) acc = mfma32(*(const u32x4_t *)(Wl + (16 * t + r) * ld + 32 * b + 8 * g), in[b], acc);
    const float4_t bb = *(const float4_t *)(bias + 16 * t + 4 * g);
    out[t >> 1][2 * (t & 1)] = pack_bf(tanh_fast(acc[0] + bb[0]), tanh_fast(acc[1] + bb[1]));
    out[t >> 1][2 * (t & 1) + 1] = pack_bf(tanh_fast(acc[2] + bb[2]), tanh_fast(acc[3] + bb[3]));
  }
}

// output tile t: this lane's rows 16 t + 4 g + j (f, f, g, g of velocities 8 t + 2 g + 0, 1)
__device__ inline float4_t corr_out(const uint16_t *W4, const float *b4, const u32x4_t (&h)[2], int t, int r, int g) {
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
  acc = mfma32(*(const u32x4_t *)(W4 + (16 * t + r) * KPH + 8 * g), h[0], acc);
  acc = mfma32(*(const u32x4_t *)(W4 + (16 * t + r) * KPH + 32 + 8 * g), h[1], acc);
  const float4_t bb = *(const float4_t *)(b4 + 16 * t + 4 * g);
  return float4_t{acc[0] + bb[0], acc[1] + bb[1], acc[2] + bb[2], acc[3] + bb[3]};
}

struct CorrShared {
  uint16_t W[WC_N] __attribute__((aligned(16)));   // stored weights, layers 1-4
  float B[3 * HW + NOUTP] __attribute__((aligned(16)));   // biases (output layer in row order)
  double V[kMaxQ][8];                              // zeta, xi, |xi|^2, w
  double PW[kMaxQ][6];                             // w zeta, w |zeta|^2, |zeta|^2 (zeta: D components)
};

// RELAX = 0: the correction alone, in place on post-collision populations (fld: the node
// fields of those populations).  RELAX = 1: the relaxation of a 3D tile step fused with the
// correction: the tile's nodes hold their stored streamed values and node state (nstate) and
// are relaxed (BGK against the equilibrium of their node state, the Prandtl-number term when
// PR = 1, Kupershtokh forcing when FORCE = 1) exactly as the relaxation launch does, then
// corrected; boundary-layer nodes arrive relaxed by the gather launch and are only corrected.
template <typename T, int RELAX, int PR, int FORCE, int D>
__global__ void __launch_bounds__(NTC, 4) k_correct(MlpArgs m, ProjArgs pa, const DevTensorPlan pl,
                                                    const StepArgs sa, int64_t N, const uint16_t *feat,
                                                    const double *fld, const double *nstate, T *pop) {
  __shared__ CorrShared S;
  constexpr int NQ = D + 2;
  const int Q = pa.Q;
  const int ntile = (Q + 7) / 8;   // output tiles, 8 velocities (16 outputs) each
  {  // weights (the output layer's used rows only), biases and velocity constants
    const int nw = (WC_W4 + 16 * ntile * KPH) / 8;
    const u32x4_t *src = (const u32x4_t *)m.wbt;
    u32x4_t *dst = (u32x4_t *)S.W;
    for (int e = threadIdx.x; e < nw; e += NTC) dst[e] = src[e];
    for (int e = threadIdx.x; e < 3 * HW + NOUTP; e += NTC) {
      const int layer = e < 3 * HW ? e / HW : 3, c = e - layer * HW;
      const int o = layer < 3 ? c : out_of_row(c, Q);
      S.B[e] = o >= 0 ? m.theta[m.off[2 * layer + 1] + o] : 0.f;
    }
    for (int e = threadIdx.x; e < Q * 8; e += NTC) S.V[e >> 3][e & 7] = pa.vel[e];
    for (int v = threadIdx.x; v < Q; v += NTC) {
      const double *z = pa.vel + 8 * v, w = z[7];
      double z2 = 0.0;
      for (int a = 0; a < D; a++) z2 += z[a] * z[a];
      for (int a = 0; a < 3; a++) S.PW[v][a] = a < D ? w * z[a] : 0.0;
      S.PW[v][3] = w * z2;
      S.PW[v][4] = z2;
      S.PW[v][5] = 0.0;
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const uint16_t *W4 = S.W + WC_W4;
  const float *b4 = S.B + 3 * HW;
  const bool vec_feat = (m.n_in & 3) == 0;
  const int64_t ngroups = (N + 15) / 16, nwaves = (int64_t)gridDim.x * (NTC / 64);
  // features 8 g .. 8 g + 7 of node kk (zero past N)
  auto load_x = [&](int64_t kk) {
    u32x4_t x = {0u, 0u, 0u, 0u};
    if (vec_feat) {   // branch-free: out-of-range lanes read row 0 and drop it
      const uint16_t *fr = feat + (kk < N ? kk : 0) * m.n_in;
#pragma unroll
      for (int q = 0; q < 2; q++) {
        const int c0 = 8 * g + 4 * q;
        const bool ok = kk < N && c0 + 4 <= m.n_in;
        const uint2 v = *(const uint2 *)(fr + (ok ? c0 : 0));
        x[2 * q] = ok ? v.x : 0u;
        x[2 * q + 1] = ok ? v.y : 0u;
      }
    } else if (kk < N) {
      const uint16_t *fr = feat + kk * m.n_in;
      for (int c = 8 * g; c < 8 * g + 8 && c < m.n_in; c++)
        x[(c - 8 * g) >> 1] |= (uint32_t)fr[c] << (16 * ((c - 8 * g) & 1));
    }
    return x;
  };
  for (int64_t grp = (int64_t)blockIdx.x * (NTC / 64) + wave; grp < ngroups; grp += nwaves) {
    const int64_t k = grp * 16 + r;
    const bool valid = k < N;
    const int z1 = opaque_zero();
    // ---- network: three tanh layers on the node's features
    u32x4_t h[2];
    {
      u32x4_t x1[1] = {load_x(k)}, h1[2];
      corr_hidden<1>(S.W + z1, KP1, S.B + z1, x1, h1, r, g);
      corr_hidden<2>(S.W + z1 + WC_W2, KPH, S.B + z1 + HW, h1, h, r, g);
      corr_hidden<2>(S.W + z1 + WC_W3, KPH, S.B + z1 + 2 * HW, h, h1, r, g);
      h[0] = h1[0];
      h[1] = h1[1];
    }
    const double rk = valid ? fld[k] : 0.0;
    // ---- relaxation coefficients of node k
    bool act = false;
    EqNode eq{}, ef{};
    double itau = 0.0, gT = 0.0, uk[3] = {0.0, 0.0, 0.0};
    if constexpr (RELAX) {
      if (valid && sa.relax_mode != 2 && !in_layer(pl, k)) {
        act = true;
        const double rho = nstate[k], Tn = nstate[4 * N + k];
        uk[0] = nstate[N + k];
        uk[1] = nstate[2 * N + k];
        uk[2] = nstate[3 * N + k];
        itau = nstate[5 * N + k];
        eq = eq_prepare(rho, uk[0], uk[1], uk[2], Tn, sa, D);
        if constexpr (FORCE) ef = eq_forced(rho, uk[0], uk[1], uk[2], Tn, sa, D);
        gT = Tn * sa.gbase;
      }
    }
    // byte offset of velocity 8 t + 2 g + e (e < 2) of node k in the planes of tile t, or
    // out of range for a lane without that population
    auto pop_off = [&](int t, int e) {
      const int v = 8 * t + 2 * g + e;
      int off = (valid && v < Q) ? (int)(((int64_t)(2 * g + e) * N + k) * (int64_t)sizeof(T)) : kOutOfRange;
      asm volatile("" : "+v"(off));   // one offset in a register: keeps the access out of branches
      return off;
    };
    auto load_tile = [&](int t, T (&d)[4]) {
      const __amdgpu_buffer_rsrc_t rf = plane_rsrc(pop, 8 * t, N), rg = plane_rsrc(pop, Q + 8 * t, N);
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int off = pop_off(t, e);
        d[e] = PopBuf<T>::load(rf, off);
        d[2 + e] = PopBuf<T>::load(rg, off);
      }
    };
    T B[PD + 1][4];
    // ---- pass 1: invariant sums of w y over this lane's outputs (and the heat flux of the
    // streamed values when PR = 1), then over the node's four lanes
    double sm[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) sm[q] = 0.0;
    HeatFlux hq = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int t = 0; t < ntile; t++) {
      const float4_t y = corr_out(W4 + z1, b4 + z1, h, t, r, g);
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const bool has = 8 * t + 2 * g + e < Q;        // lanes past Q add zeros
        const int v = min(8 * t + 2 * g + e, Q - 1);
        const double *pw = S.PW[v] + z1;
        const double w = S.V[v][7 + z1], yf = has ? (double)y[e] : 0.0, yg = has ? (double)y[2 + e] : 0.0;
        sm[0] += w * yf;
#pragma unroll
        for (int a = 0; a < D; a++) sm[1 + a] += pw[a] * yf;
        sm[NQ - 1] += pw[3] * yf + w * yg;
        if constexpr (RELAX && PR) {
          const int off = act ? pop_off(t, e) : kOutOfRange;
          const double f = (double)PopBuf<T>::load(plane_rsrc(pop, 8 * t, N), off);
          const double gv = (double)PopBuf<T>::load(plane_rsrc(pop, Q + 8 * t, N), off);
          heat_flux_add(hq, S.V[v] + z1, uk[0], uk[1], uk[2], f, gv);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      sm[q] += __shfl_xor(sm[q], 16);
      sm[q] += __shfl_xor(sm[q], 32);
    }
    double cc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      double v = 0.0;
#pragma unroll
      for (int q2 = 0; q2 < NQ; q2++) v += pa.G[q * NQ + q2] * (rk * sm[q2]);
      cc[q] = v;
    }
    PrTerm pt{};
    if constexpr (RELAX && PR) {
      double hv[6] = {hq.f0, hq.f1, hq.f2, hq.g0, hq.g1, hq.g2};
#pragma unroll
      for (int q = 0; q < 6; q++) {
        hv[q] += __shfl_xor(hv[q], 16);
        hv[q] += __shfl_xor(hv[q], 32);
      }
      pt = pr_term(HeatFlux{hv[0], hv[1], hv[2], hv[3], hv[4], hv[5]}, itau, sa, D);
    }
    const int z2 = opaque_zero();
    // ---- pass 2: pop = relax(pop) + w (rho y - M^T c) for this lane's velocities, the next
    // tile's four populations in flight while the current one is computed.  Every lane stays
    // in the loop (the MFMAs take their operands from the whole wave); loads and stores are
    // guarded per lane.
#pragma unroll
    for (int p = 0; p < PD; p++) load_tile(p, B[p]);
#pragma unroll 1
    for (int t = 0; t < ntile; t++) {
      load_tile(t + PD, B[PD]);
      const float4_t y = corr_out(W4 + z2, b4 + z2, h, t, r, g);
      const __amdgpu_buffer_rsrc_t rf = plane_rsrc(pop, 8 * t, N), rg = plane_rsrc(pop, Q + 8 * t, N);
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int v = min(8 * t + 2 * g + e, Q - 1);   // lanes past Q compute on a valid row, store nothing
        const double *vi = S.V[v] + z2;
        double fo = (double)B[0][e], go = (double)B[0][2 + e];
        if constexpr (RELAX) {
          if (act) {
            const double fe = eq_f(eq, vi);
            fo = fo - (fo - fe) * itau;
            go = go - (go - gT * fe) * itau;
            if constexpr (PR) pr_add(pt, vi, fo, go);
            if constexpr (FORCE) {
              const double df = eq_f(ef, vi) - fe;
              fo += df;
              go += gT * df;
            }
          }
        }
        double mt = cc[0];
#pragma unroll
        for (int a = 0; a < D; a++) mt += cc[1 + a] * vi[a];
        mt += cc[NQ - 1] * S.PW[v][4 + z2];
        const double w = vi[7];
        const int off = pop_off(t, e);
        PopBuf<T>::store(rf, off, (T)(fo + w * (rk * (double)y[e] - mt)));
        PopBuf<T>::store(rg, off, (T)(go + w * (rk * (double)y[2 + e] - cc[NQ - 1])));
      }
#pragma unroll
      for (int p = 0; p < PD; p++)
#pragma unroll
        for (int j = 0; j < 4; j++) B[p][j] = B[p + 1][j];
    }
  }
}

// ---------------------------------------------------------------- training
struct TrainShared {
  FwdShared F;
  uint16_t DY[R * NOUTP];
  uint16_t DZ[2][R * HW];
  float bias[2][NOUTP];
  double red[NT / 64];
};

// Forward, loss, backward for the workgroup's row tiles (tile = blockIdx.x, + gridDim.x,
// ...): the parameter gradient of sum over rows of the loss, accumulated into this
// workgroup's partial slot part[blockIdx.x][nparam]; the loss sum into lpart[blockIdx.x].
__global__ void __launch_bounds__(NT) k_mlp_train(MlpArgs m, const uint16_t *x, const float *tgt, int64_t rows,
                                                  float inv_n, int64_t nparam, float *part, double *lpart) {
  __shared__ TrainShared S;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  float *P = part + (size_t)blockIdx.x * nparam;
  stage_weights(m, S.F.W);
  double lsum = 0.0;
  const int64_t ntiles = (rows + R - 1) / R;
  bool first = true;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, first = false) {
    const int64_t row0 = tile * R;
    __syncthreads();
    stage_x(m, x, row0, rows, S.F.X);
    __syncthreads();
    hidden_layers(m, S.F);
    // ---- output layer, loss, dY
    const float *b4 = m.theta + m.off[7];
    for (int t = wave; t < 2 * (NOUTP / 16); t += 4) {
      const int rt = t & 1, ct = t >> 1;
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = mma_ab(S.F.H[2] + rt * 16 * HW, HW, S.F.W + WBF_W4 + ct * 16, NOUTP, HW, acc);
      float4_t dyv;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
        const int64_t gr = row0 + row;
        float d = 0.f;
        if (gr < rows && col < m.n_out) d = acc[j] + b4[col] - tgt[gr * m.n_out + col];
        lsum += (double)d * (double)d;
        const float dy = 2.f * d * inv_n;
        dyv[j] = dy;
        S.DY[row * NOUTP + col] = f2bf(dy);
      }
      const float cs = tile_colsum(dyv);
      if (g == 0) S.bias[rt][ct * 16 + r] = cs;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < m.n_out; c += NT) {
      float v = S.bias[0][c] + S.bias[1][c];
      float *d = P + m.off[7] + c;
      *d = first ? v : *d + v;
    }
    __syncthreads();   // S.bias is rewritten by the first backward layer
    // dW4 = H3^T dY: 4 x 16 tiles
    for (int t = wave; t < 4 * (NOUTP / 16); t += 4) {
      const int mt = t & 3, nt = t >> 2;
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = mma_atb(S.F.H[2] + mt * 16, HW, S.DY + nt * 16, NOUTP, R, acc);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int mm = mt * 16 + 4 * g + j, n = nt * 16 + r;
        if (n < m.n_out) {
          float *d = P + m.off[6] + (size_t)mm * m.n_out + n;
          *d = first ? acc[j] : *d + acc[j];
        }
      }
    }
    // hidden layers backwards: layer index 2, 1, 0 (dZ of layer L into DZ[L & 1])
    for (int L = 2; L >= 0; L--) {
      // dH_L = dZ_{L+1} W_{L+1}^T ; dZ_L = dH_L (1 - a_L^2)
      const uint16_t *dzn = L == 2 ? S.DY : S.DZ[(L + 1) & 1];
      const int ldz = L == 2 ? NOUTP : HW;
      const uint16_t *Wn = S.F.W + (L == 2 ? WBF_W4 : (L == 1 ? WBF_W3 : WBF_W2));
      uint16_t *dz = S.DZ[L & 1];
      for (int t = wave; t < 8; t += 4) {
        const int rt = t & 1, ct = t >> 1;
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_abt(dzn + rt * 16 * ldz, ldz, Wn + ct * 16 * ldz, ldz, ldz, acc);
        float4_t dzv;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
          const float a = S.F.A[L][row * HW + col];
          const float v = acc[j] * (1.f - a * a);
          dzv[j] = v;
          dz[row * HW + col] = f2bf(v);
        }
        const float cs = tile_colsum(dzv);
        if (g == 0) S.bias[rt][ct * 16 + r] = cs;
      }
      __syncthreads();
      for (int c = threadIdx.x; c < HW; c += NT) {
        float v = S.bias[0][c] + S.bias[1][c];
        float *d = P + m.off[2 * L + 1] + c;
        *d = first ? v : *d + v;
      }
      // dW_L = H_{L-1}^T dZ_L (H_{-1} = X)
      const uint16_t *hin = L == 0 ? S.F.X : S.F.H[L - 1];
      const int ldh = L == 0 ? KIN : HW, nin = L == 0 ? m.n_in : HW;
      const int mtiles = L == 0 ? KIN / 16 : HW / 16;
      for (int t = wave; t < mtiles * 4; t += 4) {
        const int mt = t % mtiles, nt = t / mtiles;
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_atb(hin + mt * 16, ldh, dz + nt * 16, HW, R, acc);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int mm = mt * 16 + 4 * g + j, n = nt * 16 + r;
          if (mm < nin) {
            float *d = P + m.off[2 * L] + (size_t)mm * HW + n;
            *d = first ? acc[j] : *d + acc[j];
          }
        }
      }
      __syncthreads();
    }
  }
  // loss of this workgroup: waves -> LDS -> one value
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  __syncthreads();
  if (l == 0) S.red[wave] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = S.red[0] + S.red[1] + S.red[2] + S.red[3];
}

// grad[p] = sum over workgroups of the partials (fixed order), in double
__global__ void k_grad_reduce(const float *part, int nblk, int64_t nparam, float *grad, const double *lpart,
                              double *loss) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nparam) {
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += (double)part[(size_t)b * nparam + p];
    grad[p] = (float)s;
  }
  if (p == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += lpart[b];
    *loss = s;
  }
}

__global__ void k_adam(int64_t nparam, float *theta, float *mm, float *vv, const float *grad, float lr, float bc1,
                       float bc2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nparam) return;
  const float gr = grad[p];
  const float m1 = 0.9f * mm[p] + 0.1f * gr;
  const float v1 = 0.999f * vv[p] + 0.001f * gr * gr;
  mm[p] = m1;
  vv[p] = v1;
  const float mh = m1 / bc1, vh = v1 / bc2;
  theta[p] = theta[p] - lr * mh / (sqrtf(vh) + 1e-8f);
}

// padded BF16 copies of the weights from the master copy
__global__ void k_refresh_bf16(MlpArgs m, uint16_t *wbf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= WBF_N) return;
  float v = 0.f;
  if (e < WBF_W2) {
    int i = e / HW, o = e % HW;
    if (i < m.n_in) v = m.theta[m.off[0] + i * HW + o];
  } else if (e < WBF_W3) {
    int q = e - WBF_W2;
    v = m.theta[m.off[2] + q];
  } else if (e < WBF_W4) {
    int q = e - WBF_W3;
    v = m.theta[m.off[4] + q];
  } else {
    int q = e - WBF_W4, i = q / NOUTP, o = q % NOUTP;
    if (o < m.n_out) v = m.theta[m.off[6] + i * m.n_out + o];
  }
  wbf[e] = f2bf(v);
}

// the BF16 weights as the correction kernels stage them: each layer [unit][input] with rows
// padded to KP1 / KPH, the inputs of layers 2-4 in the order hid_unit_of_col gives and the
// output layer's rows in the order out_of_row gives
__global__ void k_refresh_corr(MlpArgs m, uint16_t *wc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= WC_N) return;
  float v = 0.f;
  if (e < WC_W2) {
    const int o = e / KP1, i = e % KP1;
    if (i < m.n_in) v = m.theta[m.off[0] + i * HW + o];
  } else if (e < WC_W4) {
    const int L = e < WC_W3 ? 1 : 2, q = e - (L == 1 ? WC_W2 : WC_W3), o = q / KPH, c = q % KPH;
    if (c < HW) v = m.theta[m.off[2 * L] + hid_unit_of_col(c) * HW + o];
  } else {
    const int q = e - WC_W4, R = q / KPH, c = q % KPH;
    const int o = out_of_row(R, m.n_out / 2);
    if (c < HW && o >= 0) v = m.theta[m.off[6] + hid_unit_of_col(c) * m.n_out + o];
  }
  wc[e] = f2bf(v);
}

// ---------------------------------------------------------------- features
struct FeatArgs {
  int D, p, nf;             // nf = D + 2 fields
  int64_t N;
  int Na[3];
  const int32_t *didx[3];   // [Na][2][p+1] node index along the axis, -1: unused slot
  const double *dw[3];      // matching weights: (h_mean / cells) (2 / h_cell) l_m'(x_j)
  double inv_sqrtT0, T0;
};

template <typename T>
__global__ void k_node_fields(int64_t N, int Q, int D, const double *vel, double cv, const T *pop, double *fld) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double rho = 0, j[3] = {0, 0, 0}, E = 0;
  for (int i = 0; i < Q; i++) {
    const double *vi = vel + 8 * i;
    const double f = (double)pop[(size_t)i * N + k], g = (double)pop[((size_t)Q + i) * N + k];
    rho += f;
    double z2 = 0;
    for (int a = 0; a < D; a++) {
      j[a] += vi[a] * f;
      z2 += vi[a] * vi[a];
    }
    E += z2 * f + g;
  }
  double u2 = 0;
  fld[k] = rho;
  for (int a = 0; a < D; a++) {
    double u = j[a] / rho;
    fld[(size_t)(1 + a) * N + k] = u;
    u2 += u * u;
  }
  fld[(size_t)(D + 1) * N + k] = (E - rho * u2) / (2.0 * rho * cv);
}

__device__ inline double scaled_field(const FeatArgs &fa, const double *fld, int q, int64_t k) {
  double v = fld[(size_t)q * fa.N + k];
  if (q == 0) return v - 1.0;
  if (q == fa.D + 1) return v / fa.T0 - 1.0;
  return v * fa.inv_sqrtT0;
}

// One node per thread: the D + 2 scaled fields, then their derivatives along each axis (the
// per-axis table rows loaded once for all fields), stored 8 bytes at a time.
template <int D>
__global__ void k_features(FeatArgs fa, const double *fld, uint16_t *feat) {
  constexpr int NF = D + 2, NFEAT = NF * (1 + D);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= fa.N) return;
  const int P1 = fa.p + 1;
  int n[3] = {0, 0, 0};
  const int64_t stride[3] = {1, fa.Na[0], (int64_t)fa.Na[0] * fa.Na[1]};
  n[0] = (int)(k % fa.Na[0]);
  if (D > 1) n[1] = (int)((k / fa.Na[0]) % fa.Na[1]);
  if (D > 2) n[2] = (int)(k / ((int64_t)fa.Na[0] * fa.Na[1]));
  uint16_t o[NFEAT];
#pragma unroll
  for (int q = 0; q < NF; q++) o[q] = f2bf((float)scaled_field(fa, fld, q, k));
#pragma unroll
  for (int a = 0; a < D; a++) {
    double s[NF];
#pragma unroll
    for (int q = 0; q < NF; q++) s[q] = 0.0;
    const int64_t base = k - (int64_t)n[a] * stride[a];
    for (int slot = 0; slot < 2; slot++) {
      const int32_t *id = fa.didx[a] + ((size_t)n[a] * 2 + slot) * P1;
      const double *w = fa.dw[a] + ((size_t)n[a] * 2 + slot) * P1;
      if (id[0] < 0) continue;
      for (int mm = 0; mm < P1; mm++) {
        const int64_t kk = base + (int64_t)id[mm] * stride[a];
        const double wm = w[mm];
#pragma unroll
        for (int q = 0; q < NF; q++) s[q] += wm * scaled_field(fa, fld, q, kk);
      }
    }
#pragma unroll
    for (int q = 0; q < NF; q++) o[NF + q * D + a] = f2bf((float)s[q]);
  }
  static_assert(NFEAT % 4 == 0, "feature rows are stored 8 bytes at a time");
  uint2 *out = (uint2 *)(feat + k * NFEAT);
#pragma unroll
  for (int c = 0; c < NFEAT / 4; c++)
    out[c] = make_uint2((uint32_t)o[4 * c] | ((uint32_t)o[4 * c + 1] << 16),
                        (uint32_t)o[4 * c + 2] | ((uint32_t)o[4 * c + 3] << 16));
}

// ---------------------------------------------------------------- targets, restriction
template <typename T>
__global__ void k_targets(ProjArgs pa, int64_t N, const T *plain, const T *truth, float *t) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int Q = pa.Q, D = pa.D, NQ = D + 2, Q2 = 2 * Q;
  double rho = 0.0, s[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < Q2; c++) {
    const int i = c < Q ? c : c - Q;
    const double *vi = pa.vel + 8 * i;
    const double pl = (double)plain[(size_t)c * N + k];
    const double d = (double)truth[(size_t)c * N + k] - pl;
    if (c < Q) {
      rho += pl;
      s[0] += d;
      double z2 = 0.0;
      for (int a = 0; a < D; a++) {
        s[1 + a] += vi[a] * d;
        z2 += vi[a] * vi[a];
      }
      s[NQ - 1] += z2 * d;
    } else {
      s[NQ - 1] += d;
    }
  }
  double cc[5];
  for (int q = 0; q < NQ; q++) {
    cc[q] = 0.0;
    for (int q2 = 0; q2 < NQ; q2++) cc[q] += pa.G[q * NQ + q2] * s[q2];
  }
  for (int c = 0; c < Q2; c++) {
    const int i = c < Q ? c : c - Q;
    const double *vi = pa.vel + 8 * i;
    const double d = (double)truth[(size_t)c * N + k] - (double)plain[(size_t)c * N + k];
    double mt;
    if (c < Q) {
      double z2 = 0.0;
      mt = cc[0];
      for (int a = 0; a < D; a++) {
        mt += cc[1 + a] * vi[a];
        z2 += vi[a] * vi[a];
      }
      mt += cc[NQ - 1] * z2;
    } else {
      mt = cc[NQ - 1];
    }
    t[k * Q2 + c] = (float)((d - vi[7] * mt) / (vi[7] * rho));
  }
}

template <typename T>
__global__ void k_restrict(int64_t Nc, int Q2, int Ncx, int Ncy, int Nfx, int Nfy, int64_t Nf, int r, const T *fine,
                           T *coarse) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Nc) return;
  const int64_t jx = k % Ncx, jy = (k / Ncx) % Ncy, jz = k / ((int64_t)Ncx * Ncy);
  const int64_t kf = r * jx + (int64_t)Nfx * (r * jy + (int64_t)Nfy * (r * jz));
  for (int c = 0; c < Q2; c++) coarse[(size_t)c * Nc + k] = fine[(size_t)c * Nf + kf];
}

}  // namespace

// ================================================================== host side

struct sllbm_mlp_s {
  sllbm::DevAllocator dalloc;   // allocator of this network's device memory
  int n_in = 0, n_out = 0, device = -1;
  int64_t nparam = 0;
  int off[8] = {};
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  uint16_t *wbf = nullptr, *wbt = nullptr;
  float *part = nullptr;
  double *lpart = nullptr, *loss = nullptr;
  int64_t step = 0;
  MlpArgs args() const {
    MlpArgs a;
    a.n_in = n_in;
    a.n_out = n_out;
    a.theta = theta;
    a.wbf = wbf;
    a.wbt = wbt;
    for (int k = 0; k < 8; k++) a.off[k] = off[k];
    return a;
  }
};

namespace {

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int refresh(sllbm_mlp m, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_bf16, dim3((WBF_N + 255) / 256), dim3(256), 0, s, m->args(), m->wbf);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_refresh_corr, dim3((WC_N + 255) / 256), dim3(256), 0, s, m->args(), m->wbt);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

// G = (M W M^T)^-1 of the plan's velocity set, by Gauss-Jordan elimination
int proj_args(sllbm_plan_s *P, ProjArgs &pa) {
  const int D = P->mesh.dim, Q = P->vel.Q, NQ = D + 2;
  double A[5][10] = {};
  auto row = [&](int q, int c, double *val) {  // M[q][c] (c over 2Q)
    const int i = c < Q ? c : c - Q;
    const double *z = &P->vel.zeta[(size_t)i * D];
    if (c < Q) {
      if (q == 0) return (*val = 1.0, 0);
      if (q <= D) return (*val = z[q - 1], 0);
      double z2 = 0;
      for (int a = 0; a < D; a++) z2 += z[a] * z[a];
      return (*val = z2, 0);
    }
    return (*val = (q == NQ - 1) ? 1.0 : 0.0, 0);
  };
  for (int q = 0; q < NQ; q++)
    for (int q2 = 0; q2 < NQ; q2++) {
      double s = 0;
      for (int c = 0; c < 2 * Q; c++) {
        double a, b;
        row(q, c, &a);
        row(q2, c, &b);
        s += a * P->vel.w[c < Q ? c : c - Q] * b;
      }
      A[q][q2] = s;
      A[q][NQ + q2] = q == q2 ? 1.0 : 0.0;
    }
  for (int c = 0; c < NQ; c++) {
    int piv = c;
    for (int r2 = c + 1; r2 < NQ; r2++)
      if (std::fabs(A[r2][c]) > std::fabs(A[piv][c])) piv = r2;
    if (std::fabs(A[piv][c]) < 1e-300) return fail(SLLBM_EINVAL, "learned: singular invariant Gram matrix");
    for (int k = 0; k < 2 * NQ; k++) std::swap(A[c][k], A[piv][k]);
    double d = A[c][c];
    for (int k = 0; k < 2 * NQ; k++) A[c][k] /= d;
    for (int r2 = 0; r2 < NQ; r2++)
      if (r2 != c) {
        double f = A[r2][c];
        for (int k = 0; k < 2 * NQ; k++) A[r2][k] -= f * A[c][k];
      }
  }
  pa.Q = Q;
  pa.D = D;
  pa.vel = nullptr;   // the callers point it at the plan's device velocity table
  for (int q = 0; q < NQ; q++)
    for (int q2 = 0; q2 < NQ; q2++) pa.G[q * NQ + q2] = A[q][NQ + q2];
  return SLLBM_OK;
}

int learned_ready(sllbm_plan_s *P) {
  if (!P) return fail(SLLBM_EINVAL, "learned: plan is NULL");
  if (!P->has_device) return fail(SLLBM_EHIP, "learned: the plan has no device");
  if (P->kernel != 0) return fail(SLLBM_EUNSUPPORTED, "learned correction: tensor-product plans only");
  HIP_TRY(hipSetDevice(P->device));
  if (P->lfield) return SLLBM_OK;
  const Mesh &m = P->mesh;
  const int D = m.dim, p = m.p, P1 = p + 1;
  HIP_TRY(P->dalloc.get((void **)&P->lfield, sizeof(double) * (D + 2) * (size_t)m.n_nodes));
  P->dev_allocs.push_back(P->lfield);
  // per-axis derivative tables
  std::vector<double> dm((size_t)P1 * P1);  // dm[j][mm] = l_mm'(x_j)
  for (int j = 0; j < P1; j++)
    for (int mm = 0; mm < P1; mm++) {
      const std::vector<double> &x = m.xref;
      double v;
      if (mm == j) {
        v = 0;
        for (int q = 0; q < P1; q++)
          if (q != j) v += 1.0 / (x[j] - x[q]);
      } else {
        v = 1.0 / (x[mm] - x[j]);
        for (int q = 0; q < P1; q++)
          if (q != mm && q != j) v *= (x[j] - x[q]) / (x[mm] - x[q]);
      }
      dm[(size_t)j * P1 + mm] = v;
    }
  for (int a = 0; a < D; a++) {
    const int Na = m.N[a], nc = m.ncell[a];
    const bool per = m.periodic(a);
    std::vector<int32_t> idx((size_t)Na * 2 * P1, -1);
    std::vector<double> w((size_t)Na * 2 * P1, 0.0);
    std::vector<int> cnt(Na, 0);
    std::vector<double> hs(Na, 0.0);
    for (int c = 0; c < nc; c++) {
      const double h = m.edges[a][c + 1] - m.edges[a][c];
      for (int j = 0; j < P1; j++) {
        int n = (c * p + j) % Na;
        cnt[n]++;
        hs[n] += h;
      }
    }
    std::vector<int> used(Na, 0);
    for (int c = 0; c < nc; c++) {
      const double h = m.edges[a][c + 1] - m.edges[a][c];
      for (int j = 0; j < P1; j++) {
        const int n = (c * p + j) % Na;
        const int slot = used[n]++;
        const double hm = hs[n] / cnt[n];
        for (int mm = 0; mm < P1; mm++) {
          idx[((size_t)n * 2 + slot) * P1 + mm] = (c * p + mm) % Na;
          w[((size_t)n * 2 + slot) * P1 + mm] = (hm / cnt[n]) * (2.0 / h) * dm[(size_t)j * P1 + mm];
        }
      }
    }
    (void)per;
    int32_t *di = nullptr;
    double *dw = nullptr;
    HIP_TRY(P->dalloc.get((void **)&di, idx.size() * sizeof(int32_t)));
    P->dev_allocs.push_back(di);
    HIP_TRY(P->dalloc.get((void **)&dw, w.size() * sizeof(double)));
    P->dev_allocs.push_back(dw);
    HIP_TRY(hipMemcpy(di, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
    P->ldidx[a] = di;
    P->ldw[a] = dw;
  }
  const int nfeat = (D + 2) * (D + 1);
  HIP_TRY(P->dalloc.get((void **)&P->lfeat, sizeof(uint16_t) * nfeat * (size_t)m.n_nodes));
  P->dev_allocs.push_back(P->lfeat);
  return SLLBM_OK;
}

int check_pop_ptr(const void *p, const char *what) {
  if (!p) return fail(SLLBM_EINVAL, "%s is NULL", what);
  if ((uintptr_t)p % 16) return fail(SLLBM_EINVAL, "%s must be 16-byte aligned", what);
  return SLLBM_OK;
}

void feature_args(const sllbm_plan_s *P, FeatArgs &fa) {
  const Mesh &m = P->mesh;
  fa.D = m.dim;
  fa.p = m.p;
  fa.nf = m.dim + 2;
  fa.N = m.n_nodes;
  for (int a = 0; a < 3; a++) {
    fa.Na[a] = a < m.dim ? m.N[a] : 1;
    fa.didx[a] = a < m.dim ? P->ldidx[a] : nullptr;
    fa.dw[a] = a < m.dim ? P->ldw[a] : nullptr;
  }
  fa.T0 = P->vel.T0;
  fa.inv_sqrtT0 = 1.0 / std::sqrt(P->vel.T0);
}

int run_features(sllbm_plan_s *P, const sllbm_params *prm, const void *pop, uint16_t *feat, hipStream_t s) {
  const Mesh &m = P->mesh;
  const int64_t N = m.n_nodes;
  const double cv = 1.0 / (prm->gamma - 1.0);
  const double *vel = P->tp.vel;
  dim3 grid((unsigned)((N + 255) / 256));
  {
    ProfScope ps(P, "k_node_fields", s);
    if (P->prec == SLLBM_F32)
      hipLaunchKernelGGL(k_node_fields<float>, grid, dim3(256), 0, s, N, P->vel.Q, m.dim, vel, cv,
                         (const float *)pop, P->lfield);
    else
      hipLaunchKernelGGL(k_node_fields<double>, grid, dim3(256), 0, s, N, P->vel.Q, m.dim, vel, cv,
                         (const double *)pop, P->lfield);
  }
  HIP_TRY(hipGetLastError());
  FeatArgs fa{};
  feature_args(P, fa);
  {
    ProfScope ps(P, "k_features", s);
    if (m.dim == 2) hipLaunchKernelGGL(k_features<2>, grid, dim3(256), 0, s, fa, (const double *)P->lfield, feat);
    else hipLaunchKernelGGL(k_features<3>, grid, dim3(256), 0, s, fa, (const double *)P->lfield, feat);
  }
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int check_params_basic(const sllbm_params *prm) {
  if (!prm) return fail(SLLBM_EINVAL, "params is NULL");
  if (!(prm->gamma > 1.0)) return fail(SLLBM_EINVAL, "gamma must be > 1");
  return SLLBM_OK;
}

int ensure_partials(sllbm_mlp m, int nblk) {
  if (m->part) return SLLBM_OK;
  HIP_TRY(m->dalloc.get((void **)&m->part, sizeof(float) * (size_t)kMaxPartialBlocks * m->nparam));
  HIP_TRY(m->dalloc.get((void **)&m->lpart, sizeof(double) * kMaxPartialBlocks));
  HIP_TRY(m->dalloc.get((void **)&m->loss, sizeof(double)));
  (void)nblk;
  return SLLBM_OK;
}

int gradient(sllbm_mlp m, const uint16_t *x, const float *t, int64_t rows, hipStream_t s) {
  if (!m) return fail(SLLBM_EINVAL, "mlp is NULL");
  if (!x || !t || rows <= 0) return fail(SLLBM_EINVAL, "mlp gradient: NULL data or rows <= 0");
  HIP_TRY(hipSetDevice(m->device));
  int rc = ensure_partials(m, 0);
  if (rc) return rc;
  const int64_t ntiles = (rows + R - 1) / R;
  const int nblk = (int)std::min<int64_t>(ntiles, kMaxPartialBlocks);
  const float inv_n = (float)(1.0 / ((double)rows * m->n_out));
  hipLaunchKernelGGL(k_mlp_train, dim3(nblk), dim3(NT), 0, s, m->args(), x, t, rows, inv_n, m->nparam, m->part,
                     m->lpart);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((m->nparam + 255) / 256)), dim3(256), 0, s,
                     (const float *)m->part, nblk, m->nparam, m->grad, (const double *)m->lpart, m->loss);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int read_loss(sllbm_mlp m, int64_t rows, float *loss_host, hipStream_t s) {
  if (!loss_host) return SLLBM_OK;
  double l = 0;
  HIP_TRY(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *loss_host = (float)(l / ((double)rows * m->n_out));
  return SLLBM_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" int sllbm_mlp_create(int n_in, int width, int depth, int n_out, uint64_t seed, sllbm_mlp *out) {
  if (!out) return fail(SLLBM_EINVAL, "mlp_create: out is NULL");
  *out = nullptr;
  if (width != HW || depth != 3) return fail(SLLBM_EUNSUPPORTED, "mlp_create: width 64 and depth 3 only");
  if (n_in < 1 || n_in > KIN || n_out < 1 || n_out > NOUTP)
    return fail(SLLBM_EUNSUPPORTED, "mlp_create: need 1 <= n_in <= %d and 1 <= n_out <= %d", KIN, NOUTP);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(SLLBM_EHIP, "mlp_create: no HIP device");
  sllbm_mlp m = new (std::nothrow) sllbm_mlp_s;
  if (!m) return fail(SLLBM_ENOMEM, "mlp_create");
  m->n_in = n_in;
  m->n_out = n_out;
  m->device = dev;
  m->dalloc = sllbm::current_allocator();
  const int64_t sizes[8] = {(int64_t)n_in * HW, HW, HW * HW, HW, HW * HW, HW, (int64_t)HW * n_out, n_out};
  int64_t o = 0;
  for (int k = 0; k < 8; k++) {
    m->off[k] = (int)o;
    o += sizes[k];
  }
  m->nparam = o;
  std::vector<float> th(o, 0.f);
  const int fan[4] = {n_in, HW, HW, HW};
  for (int layer = 0; layer < 4; layer++) {
    const double bound = 1.0 / std::sqrt((double)fan[layer]);
    for (int64_t q = 0; q < sizes[2 * layer]; q++) {
      const int64_t idx = m->off[2 * layer] + q;
      const double u = (double)(splitmix64(seed + (uint64_t)idx) >> 11) * (1.0 / 9007199254740992.0);
      th[idx] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  auto alloc = [&](void **p, size_t b) { return m->dalloc.get(p, b) == hipSuccess; };
  if (!alloc((void **)&m->theta, o * 4) || !alloc((void **)&m->m, o * 4) || !alloc((void **)&m->v, o * 4) ||
      !alloc((void **)&m->grad, o * 4) || !alloc((void **)&m->wbf, WBF_N * 2) || !alloc((void **)&m->wbt, WC_N * 2)) {
    sllbm_mlp_destroy(m);
    return fail(SLLBM_ENOMEM, "mlp_create: device allocation");
  }
  int rc = sllbm_mlp_set_params(m, th.data());
  if (rc) {
    sllbm_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return SLLBM_OK;
}

extern "C" void sllbm_mlp_destroy(sllbm_mlp m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  void *ptrs[] = {m->theta, m->m, m->v, m->grad, m->wbf, m->wbt, m->part, m->lpart, m->loss};
  for (void *p : ptrs) m->dalloc.put(p);
  delete m;
}

extern "C" int sllbm_mlp_num_params(sllbm_mlp m, int64_t *n) {
  if (!m || !n) return fail(SLLBM_EINVAL, "mlp_num_params: NULL argument");
  *n = m->nparam;
  return SLLBM_OK;
}

extern "C" int sllbm_mlp_get_params(sllbm_mlp m, float *host) {
  if (!m || !host) return fail(SLLBM_EINVAL, "mlp_get_params: NULL argument");
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host, m->theta, m->nparam * 4, hipMemcpyDeviceToHost));
  return SLLBM_OK;
}

extern "C" int sllbm_mlp_set_params(sllbm_mlp m, const float *host) {
  if (!m || !host) return fail(SLLBM_EINVAL, "mlp_set_params: NULL argument");
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(m->theta, host, m->nparam * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(m->m, 0, m->nparam * 4));
  HIP_TRY(hipMemset(m->v, 0, m->nparam * 4));
  m->step = 0;
  int rc = refresh(m, nullptr);
  if (rc) return rc;
  HIP_TRY(hipDeviceSynchronize());
  return SLLBM_OK;
}

extern "C" int sllbm_features(sllbm_plan P, const sllbm_params *prm, const void *pop, uint16_t *feat, void *stream) {
  int rc = learned_ready(P);
  if (rc) return rc;
  if ((rc = check_params_basic(prm)) || (rc = check_pop_ptr(pop, "features: pop"))) return rc;
  if (!feat) return fail(SLLBM_EINVAL, "features: output is NULL");
  if ((uintptr_t)feat % 8) return fail(SLLBM_EINVAL, "features: output must be 8-byte aligned");
  return run_features(P, prm, pop, feat, (hipStream_t)stream);
}

extern "C" int sllbm_mlp_forward(sllbm_mlp m, const uint16_t *x, int64_t rows, float *y, void *stream) {
  if (!m || !x || !y || rows <= 0) return fail(SLLBM_EINVAL, "mlp_forward: NULL argument or rows <= 0");
  HIP_TRY(hipSetDevice(m->device));
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + R - 1) / R)), dim3(NT), 0, (hipStream_t)stream,
                     m->args(), x, rows, y);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

int sllbm::learned_check(sllbm_plan_s *P, sllbm_mlp m) {
  int rc = learned_ready(P);
  if (rc) return rc;
  if (!m) return fail(SLLBM_EINVAL, "learned: mlp is NULL");
  const int D = P->mesh.dim;
  if (m->n_in != (D + 2) * (D + 1) || m->n_out != 2 * P->vel.Q)
    return fail(SLLBM_EINVAL, "learned: network is %d -> %d, the plan needs %d -> %d", m->n_in, m->n_out,
                (D + 2) * (D + 1), 2 * P->vel.Q);
  if (m->device != P->device) return fail(SLLBM_EINVAL, "learned: network and plan on different devices");
  const int64_t esz = P->prec == SLLBM_F32 ? 4 : 8;
  if (8 * P->mesh.n_nodes * esz > kOutOfRange)
    return fail(SLLBM_EUNSUPPORTED, "learned correction: at most %lld nodes in this precision",
                (long long)(kOutOfRange / (8 * esz)));
  return SLLBM_OK;
}

int sllbm::launch_relax_correct(sllbm_plan_s *P, const StepArgs &a, sllbm_mlp m, void *pop, hipStream_t s) {
  const int64_t N = P->mesh.n_nodes;
  const dim3 grid1((unsigned)((N + 255) / 256));
  {
    ProfScope ps(P, "k_step_fields", s);
    if (P->prec == SLLBM_F32)
      hipLaunchKernelGGL(k_step_fields<float>, grid1, dim3(256), 0, s, P->tp, a, (const double *)P->nstate,
                         (const float *)pop, P->lfield);
    else
      hipLaunchKernelGGL(k_step_fields<double>, grid1, dim3(256), 0, s, P->tp, a, (const double *)P->nstate,
                         (const double *)pop, P->lfield);
  }
  HIP_TRY(hipGetLastError());
  FeatArgs fa{};
  feature_args(P, fa);
  {
    ProfScope ps(P, "k_features", s);
    hipLaunchKernelGGL(k_features<3>, grid1, dim3(256), 0, s, fa, (const double *)P->lfield, P->lfeat);
  }
  HIP_TRY(hipGetLastError());
  ProjArgs pa{};
  int rc = proj_args(P, pa);
  if (rc) return rc;
  pa.vel = P->tp.vel;
  {
    ProfScope ps(P, "k_relax_correct", s);
#define RC_LAUNCH(TT, PRV, FV)                                                                                 \
  do {                                                                                                         \
    const dim3 grid((unsigned)std::min<int64_t>((N + NTC / 4 - 1) / (NTC / 4), kCorrectGrid));                \
    hipLaunchKernelGGL((k_correct<TT, 1, PRV, FV, 3>), grid, dim3(NTC), 0, s, m->args(), pa, P->tp, a, N,     \
                       (const uint16_t *)P->lfeat, (const double *)P->lfield, (const double *)P->nstate,       \
                       (TT *)pop);                                                                             \
  } while (0)
#define RC_LAUNCH_F(TT, PRV)           \
  do {                                 \
    if (a.has_force) RC_LAUNCH(TT, PRV, 1); \
    else RC_LAUNCH(TT, PRV, 0);        \
  } while (0)
    if (P->prec == SLLBM_F32) {
      if (a.pr_on) RC_LAUNCH_F(float, 1);
      else RC_LAUNCH_F(float, 0);
    } else {
      if (a.pr_on) RC_LAUNCH_F(double, 1);
      else RC_LAUNCH_F(double, 0);
    }
#undef RC_LAUNCH_F
#undef RC_LAUNCH
  }
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

extern "C" int sllbm_mlp_correct(sllbm_plan P, const sllbm_params *prm, sllbm_mlp m, void *pop, void *stream) {
  int rc = learned_check(P, m);
  if (rc) return rc;
  if ((rc = check_params_basic(prm)) || (rc = check_pop_ptr(pop, "mlp_correct: pop"))) return rc;
  return launch_mlp_correct(P, prm, m, pop, (hipStream_t)stream);
}

int sllbm::launch_mlp_correct(sllbm_plan_s *P, const sllbm_params *prm, sllbm_mlp m, void *pop, hipStream_t s) {
  int rc;
  if ((rc = run_features(P, prm, pop, P->lfeat, s))) return rc;
  ProjArgs pa{};
  if ((rc = proj_args(P, pa))) return rc;
  pa.vel = P->tp.vel;
  const int64_t N = P->mesh.n_nodes;
  // a persistent grid: each workgroup stages the weights once and walks several tiles
  dim3 grid((unsigned)std::min<int64_t>((N + NTC / 4 - 1) / (NTC / 4), kCorrectGrid));
  const StepArgs none{};
  {
    ProfScope ps(P, "k_mlp_correct", s);
#define MC_LAUNCH(TT, DD)                                                                                      \
  hipLaunchKernelGGL((k_correct<TT, 0, 0, 0, DD>), grid, dim3(NTC), 0, s, m->args(), pa, P->tp, none, N,        \
                     (const uint16_t *)P->lfeat, (const double *)P->lfield, (const double *)nullptr, (TT *)pop)
    if (P->prec == SLLBM_F32) {
      if (P->mesh.dim == 2) MC_LAUNCH(float, 2);
      else MC_LAUNCH(float, 3);
    } else {
      if (P->mesh.dim == 2) MC_LAUNCH(double, 2);
      else MC_LAUNCH(double, 3);
    }
#undef MC_LAUNCH
  }
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

extern "C" int sllbm_learned_targets(sllbm_plan P, const void *plain, const void *truth, float *t, void *stream) {
  int rc = learned_ready(P);
  if (rc) return rc;
  if ((rc = check_pop_ptr(plain, "targets: pop_plain")) || (rc = check_pop_ptr(truth, "targets: pop_true"))) return rc;
  if (!t) return fail(SLLBM_EINVAL, "targets: output is NULL");
  ProjArgs pa{};
  if ((rc = proj_args(P, pa))) return rc;
  pa.vel = P->tp.vel;
  const int64_t N = P->mesh.n_nodes;
  hipStream_t s = (hipStream_t)stream;
  dim3 grid((unsigned)((N + 255) / 256));
  if (P->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_targets<float>, grid, dim3(256), 0, s, pa, N, (const float *)plain, (const float *)truth, t);
  else
    hipLaunchKernelGGL(k_targets<double>, grid, dim3(256), 0, s, pa, N, (const double *)plain,
                       (const double *)truth, t);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

extern "C" int sllbm_restrict(sllbm_plan F, sllbm_plan C, int r, const void *pf, void *pc, void *stream) {
  if (!F || !C) return fail(SLLBM_EINVAL, "restrict: plan is NULL");
  if (!F->has_device || !C->has_device) return fail(SLLBM_EHIP, "restrict: plans need a device");
  if (F->kernel != 0 || C->kernel != 0) return fail(SLLBM_EUNSUPPORTED, "restrict: tensor-product plans only");
  int rc;
  if ((rc = check_pop_ptr(pf, "restrict: pop_fine")) || (rc = check_pop_ptr(pc, "restrict: pop_coarse"))) return rc;
  if (r < 1) return fail(SLLBM_EINVAL, "restrict: ratio must be >= 1");
  const Mesh &mf = F->mesh, &mc = C->mesh;
  if (mf.dim != mc.dim || F->vel.Q != C->vel.Q || F->prec != C->prec)
    return fail(SLLBM_EINVAL, "restrict: dimension, velocity set or precision differ");
  for (int a = 0; a < mc.dim; a++) {
    const bool per = mc.periodic(a);
    if (per != mf.periodic(a)) return fail(SLLBM_EINVAL, "restrict: axis %d boundary kinds differ", a);
    const int64_t need = per ? (int64_t)r * mc.N[a] : (int64_t)r * (mc.N[a] - 1) + 1;
    if (mf.N[a] != need) return fail(SLLBM_EINVAL, "restrict: axis %d has %d fine nodes, nesting needs %lld", a,
                                     mf.N[a], (long long)need);
    const double L = std::fabs(mc.edges[a].back() - mc.edges[a].front());
    for (int j = 0; j < mc.N[a]; j++) {
      double xc = tensor_node_coord(mc, a, j), xf = tensor_node_coord(mf, a, r * j);
      if (std::fabs(xc - xf) > 1e-12 * L)
        return fail(SLLBM_EINVAL, "restrict: node %d of axis %d is not a fine node (%g vs %g)", j, a, xc, xf);
    }
  }
  HIP_TRY(hipSetDevice(C->device));
  const int64_t Nc = mc.n_nodes;
  hipStream_t s = (hipStream_t)stream;
  dim3 grid((unsigned)((Nc + 255) / 256));
  const int Ncy = mc.dim > 1 ? mc.N[1] : 1, Nfy = mf.dim > 1 ? mf.N[1] : 1;
  if (C->prec == SLLBM_F32)
    hipLaunchKernelGGL(k_restrict<float>, grid, dim3(256), 0, s, Nc, 2 * C->vel.Q, mc.N[0], Ncy, mf.N[0], Nfy,
                       (int64_t)mf.n_nodes, r, (const float *)pf, (float *)pc);
  else
    hipLaunchKernelGGL(k_restrict<double>, grid, dim3(256), 0, s, Nc, 2 * C->vel.Q, mc.N[0], Ncy, mf.N[0], Nfy,
                       (int64_t)mf.n_nodes, r, (const double *)pf, (double *)pc);
  HIP_TRY(hipGetLastError());
  return SLLBM_OK;
}

extern "C" int sllbm_mlp_gradient(sllbm_mlp m, const uint16_t *x, const float *t, int64_t rows, float *grad_host,
                                  float *loss_host, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  int rc = gradient(m, x, t, rows, s);
  if (rc) return rc;
  if (grad_host) {
    HIP_TRY(hipMemcpyAsync(grad_host, m->grad, m->nparam * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return read_loss(m, rows, loss_host, s);
}

extern "C" int sllbm_mlp_train_step(sllbm_mlp m, const uint16_t *x, const float *t, int64_t rows, float lr,
                                    float *loss_host, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!(lr > 0.f)) return fail(SLLBM_EINVAL, "mlp_train_step: lr must be > 0");
  int rc = gradient(m, x, t, rows, s);
  if (rc) return rc;
  m->step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->nparam + 255) / 256)), dim3(256), 0, s, m->nparam, m->theta, m->m,
                     m->v, (const float *)m->grad, lr, bc1, bc2);
  HIP_TRY(hipGetLastError());
  if ((rc = refresh(m, s))) return rc;
  return read_loss(m, rows, loss_host, s);
}
