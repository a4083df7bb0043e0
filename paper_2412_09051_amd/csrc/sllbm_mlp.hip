// Learned post-collision correction on tensor-product meshes (gfx950).
//
// Node features (moments and their interpolant gradients), the network's forward pass on
// BF16 MFMA (v_mfma_f32_16x16x16_bf16, FP32 accumulation), the projected correction added
// in place, one-step training targets, restriction by injection, and training: a fused
// forward / loss / backward kernel per 32-row tile whose weight gradients are again MFMA
// products, written as per-workgroup partials and summed in a fixed order, then Adam on
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
// two per CU stages the weights twice per CU and walks the tiles from there.
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
  const uint16_t *wbt;    // the same transposed, each layer [out][in] (the correction kernels)
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

// The correction kernels: a persistent grid of 256-thread workgroups (4 waves), two per
// compute unit as their LDS allows (so that one workgroup's network runs while the other's
// population pass waits on memory), each walking 32-node tiles.  Per workgroup the hidden
// layers' transposed BF16 weights, the biases and the velocity constants are staged once;
// the output layer's weights (up to 32 KB) are read from the L1/L2-resident global copy.  Per
// tile: the network on the 32 nodes' features (16x16x16 BF16 MFMA tiles, operands read 4
// values at a time: the activations row-major, the weights transposed), the invariant sums
// of the scaled outputs, then one pass over the tile's populations, one node per lane and
// several populations in flight per lane.
constexpr int RC = 32;       // nodes per tile
constexpr int NTC = 256;     // threads per workgroup
constexpr int UB = 8;        // populations per lane in flight in the population pass
constexpr int WH_N = KIN * HW + 2 * HW * HW;   // hidden layers' weights

// D += A B over K, A (16 x K) row-major with leading dimension lda, B given transposed
// (Bt: 16 x K, row n holds column n of B); lane l reads A[l%16][k0+4(l/16) .. +3] and
// Bt[l%16][k0+4(l/16) .. +3] as single 8-byte loads (v_mfma_f32_16x16x16_bf16 layout), all
// k-steps' operands before the products.
template <int K>
__device__ inline float4_t mma_abt4(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, float4_t acc) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  short4_t a[K / 16], b[K / 16];
#pragma unroll
  for (int q = 0; q < K / 16; q++) {
    a[q] = *(const short4_t *)(A + r * lda + 16 * q + 4 * g);
    b[q] = *(const short4_t *)(Bt + r * ldb + 16 * q + 4 * g);
  }
#pragma unroll
  for (int q = 0; q < K / 16; q++) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[q], b[q], acc, 0, 0, 0);
  return acc;
}

// tanh from one exponential: tanh x = sign(x) (1 - e) / (1 + e), e = exp(-2 |x|) (FP32; the
// result is rounded to BF16 next)
__device__ inline float tanh_fast(float x) {
  const float e = __expf(-2.f * fabsf(x));
  return copysignf((1.f - e) / (1.f + e), x);
}

struct CorrShared {
  uint16_t W[WH_N];                       // hidden layers' transposed weights
  float B[3 * HW + NOUTP];                // biases
  union {
    struct {
      uint16_t X[RC * KIN];
      uint16_t H[2][RC * HW];
    } a;
    double hq[2 * NTC / 64][RC][6];       // heat-flux partials of the half-waves (Pr != 1)
  } u;
  float Y[RC * (NOUTP + 1)];              // rows padded to an odd stride (bank-conflict free
                                          // column reads)
  double C[RC * 5];
  double V[kMaxQ][8];                     // velocity constants: zeta, xi, |xi|^2, w
};

// RELAX = 0: the correction alone, in place on post-collision populations (fld: the node
// fields of those populations).  RELAX = 1: the relaxation of a 3D tile step fused with the
// correction: the tile's nodes hold their stored streamed values and node state (nstate) and
// are relaxed (BGK against the equilibrium of their node state, the Prandtl-number term when
// PR = 1, Kupershtokh forcing) exactly as the relaxation launch does, then corrected;
// boundary-layer nodes arrive relaxed by the gather launch and are only corrected.
template <typename T, int RELAX, int PR, int D>
__global__ void __launch_bounds__(NTC, 2) k_correct(MlpArgs m, ProjArgs pa, const DevTensorPlan pl,
                                                    const StepArgs sa, int64_t N, const uint16_t *feat,
                                                    const double *fld, const double *nstate, T *pop) {
  __shared__ CorrShared S;
  constexpr int NQ = D + 2;
  const int Q = pa.Q, Q2 = 2 * Q;
  {  // hidden weights, biases and velocity constants, once per workgroup
    const uint32_t *src = (const uint32_t *)m.wbt;
    uint32_t *dst = (uint32_t *)S.W;
    for (int e = threadIdx.x; e < WH_N / 2; e += NTC) dst[e] = src[e];
    for (int e = threadIdx.x; e < 3 * HW + NOUTP; e += NTC) {
      const int layer = e < 3 * HW ? e / HW : 3, c = e - layer * HW;
      S.B[e] = (layer < 3 || c < m.n_out) ? m.theta[m.off[2 * layer + 1] + c] : 0.f;
    }
    for (int e = threadIdx.x; e < Q * 8; e += NTC) S.V[e >> 3][e & 7] = pa.vel[e];
  }
  const uint16_t *W4t = m.wbt + WBF_W4;   // output layer, transposed [NOUTP][HW], global
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int nct = (m.n_out + 15) / 16;    // output column tiles
  // population passes: node `node` of the tile, half-wave `hw` of 8 (one population each)
  const int node = lane & (RC - 1), hw = 2 * wave + (lane >> 5);
  const int64_t ntiles = (N + RC - 1) / RC;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * RC;
    const int64_t k = row0 + node;
    const bool valid = k < N;
    // ---- relaxation coefficients of this lane's node
    bool act = false;
    EqNode eq{}, ef{};
    double itau = 0.0, gT = 0.0;
    if constexpr (RELAX) {
      if (valid && sa.relax_mode != 2 && !in_layer(pl, k)) {
        act = true;
        const double rho = nstate[k], u0 = nstate[N + k], u1 = nstate[2 * N + k], u2 = nstate[3 * N + k];
        const double Tn = nstate[4 * N + k];
        itau = nstate[5 * N + k];
        eq = eq_prepare(rho, u0, u1, u2, Tn, sa, D);
        ef = sa.has_force ? eq_forced(rho, u0, u1, u2, Tn, sa, D) : eq;
        gT = Tn * sa.gbase;
      }
    }
    __syncthreads();   // the previous tile's passes are done with every buffer
    PrTerm pt{};
    if constexpr (RELAX && PR) {  // Pr != 1: heat flux of the streamed values over the half-waves
      HeatFlux h = {0, 0, 0, 0, 0, 0};
      if (act) {
        const double u0 = nstate[N + k], u1 = nstate[2 * N + k], u2 = nstate[3 * N + k];
        for (int i = hw; i < Q; i += 2 * NTC / 64)
          heat_flux_add(h, S.V[i], u0, u1, u2, (double)pop[(size_t)i * N + k], (double)pop[((size_t)Q + i) * N + k]);
      }
      double *hp = S.u.hq[hw][node];
      hp[0] = h.f0;
      hp[1] = h.f1;
      hp[2] = h.f2;
      hp[3] = h.g0;
      hp[4] = h.g1;
      hp[5] = h.g2;
      __syncthreads();
      double t[6] = {0, 0, 0, 0, 0, 0};
      for (int w = 0; w < 2 * NTC / 64; w++)
#pragma unroll
        for (int q = 0; q < 6; q++) t[q] += S.u.hq[w][node][q];
      if (act) pt = pr_term(HeatFlux{t[0], t[1], t[2], t[3], t[4], t[5]}, itau, sa, D);
      __syncthreads();   // the partials share their space with X and H
    }
    // ---- network: features -> three tanh layers -> outputs
    for (int e = threadIdx.x; e < RC * KIN; e += NTC) {
      const int rr = e / KIN, c = e % KIN;
      const int64_t gr = row0 + rr;
      S.u.a.X[e] = (gr < N && c < m.n_in) ? feat[gr * m.n_in + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int layer = 0; layer < 3; layer++) {
      const uint16_t *in = layer == 0 ? S.u.a.X : S.u.a.H[(layer - 1) & 1];
      uint16_t *out = S.u.a.H[layer & 1];
      const uint16_t *Wt = S.W + (layer == 0 ? WBF_W1 : (layer == 1 ? WBF_W2 : WBF_W3));
      const float *b = S.B + layer * HW;
      // 8 output tiles of 16 x 16 over 4 waves: two each, their products issued together
      float4_t acc[2];
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int t = wave + 4 * h, rt = t & 1, ct = t >> 1;
        acc[h] = float4_t{0.f, 0.f, 0.f, 0.f};
        if (layer == 0) acc[h] = mma_abt4<KIN>(in + rt * 16 * KIN, KIN, Wt + ct * 16 * KIN, KIN, acc[h]);
        else acc[h] = mma_abt4<HW>(in + rt * 16 * HW, HW, Wt + ct * 16 * HW, HW, acc[h]);
      }
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int t = wave + 4 * h, rt = t & 1, ct = t >> 1;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
          out[row * HW + col] = f2bf(tanh_fast(acc[h][j] + b[col]));
        }
      }
      __syncthreads();
    }
    {
      const float *b4 = S.B + 3 * HW;
      const uint16_t *h3 = S.u.a.H[0];     // the third layer's output (layer 2 writes H[0])
      for (int t = wave; t < 2 * nct; t += NTC / 64) {
        const int rt = t & 1, ct = t >> 1;
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
        acc = mma_abt4<HW>(h3 + rt * 16 * HW, HW, W4t + ct * 16 * HW, HW, acc);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int row = rt * 16 + 4 * g + j, col = ct * 16 + r;
          S.Y[row * (NOUTP + 1) + col] = acc[j] + b4[col];
        }
      }
    }
    __syncthreads();
    {  // invariant sums s = M (w rho y) per node, then c = G s: 8 threads per node
      const int row = threadIdx.x >> 3, part = threadIdx.x & 7;
      const int64_t kr = row0 + row;
      const double rk = kr < N ? fld[kr] : 0.0;
      double sm[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) sm[q] = 0.0;
      for (int c = part; c < Q2; c += 8) {
        const bool isf = c < Q;
        const double *vi = S.V[isf ? c : c - Q];
        const double dy = vi[7] * rk * (double)S.Y[row * (NOUTP + 1) + c];
        if (isf) {
          sm[0] += dy;
          double z2 = 0.0;
#pragma unroll
          for (int a = 0; a < D; a++) {
            sm[1 + a] += vi[a] * dy;
            z2 += vi[a] * vi[a];
          }
          sm[NQ - 1] += z2 * dy;
        } else {
          sm[NQ - 1] += dy;
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; q++) {
        sm[q] += __shfl_xor(sm[q], 1);
        sm[q] += __shfl_xor(sm[q], 2);
        sm[q] += __shfl_xor(sm[q], 4);
      }
      if (part == 0)
#pragma unroll
        for (int q = 0; q < NQ; q++) {
          double v = 0.0;
#pragma unroll
          for (int q2 = 0; q2 < NQ; q2++) v += pa.G[q * NQ + q2] * sm[q2];
          S.C[row * 5 + q] = v;
        }
    }
    __syncthreads();
    // ---- populations: pop = relax(pop) + w rho y - w (M^T c), node `node`, c = hw + 8 n
    if (valid) {
      const double rk = fld[k];
      double cc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) cc[q] = S.C[node * 5 + q];
      for (int c0 = hw; c0 < Q2; c0 += UB * (2 * NTC / 64)) {
        T hv[UB];
#pragma unroll
        for (int b = 0; b < UB; b++) {
          const int c = c0 + b * (2 * NTC / 64);
          if (c < Q2) hv[b] = pop[(size_t)c * N + k];
        }
#pragma unroll
        for (int b = 0; b < UB; b++) {
          const int c = c0 + b * (2 * NTC / 64);
          if (c >= Q2) break;
          const bool isf = c < Q;
          const double *vi = S.V[isf ? c : c - Q];
          double mt;
          if (isf) {
            double z2 = 0.0;
            mt = cc[0];
#pragma unroll
            for (int a = 0; a < D; a++) {
              mt += cc[1 + a] * vi[a];
              z2 += vi[a] * vi[a];
            }
            mt += cc[NQ - 1] * z2;
          } else {
            mt = cc[NQ - 1];
          }
          double h = (double)hv[b];
          if constexpr (RELAX) {
            if (act) {
              const double fe = eq_f(eq, vi);
              if (isf) {
                double fo = h - (h - fe) * itau;
                if constexpr (PR) {
                  double unused = 0.0;
                  pr_add(pt, vi, fo, unused);
                }
                if (sa.has_force) fo += eq_f(ef, vi) - fe;
                h = fo;
              } else {
                double go = h - (h - gT * fe) * itau;
                if constexpr (PR) {
                  double unused = 0.0;
                  pr_add(pt, vi, unused, go);
                }
                if (sa.has_force) go += gT * (eq_f(ef, vi) - fe);
                h = go;
              }
            }
          }
          pop[(size_t)c * N + k] = (T)(h + vi[7] * (rk * (double)S.Y[node * (NOUTP + 1) + c] - mt));
        }
      }
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

// the same BF16 weights transposed: layer blocks at the same offsets, [out][in] (inputs
// padded to KIN, outputs of the last layer to NOUTP)
__global__ void k_refresh_bf16t(MlpArgs m, uint16_t *wbt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= WBF_N) return;
  float v = 0.f;
  if (e < WBF_W2) {
    int o = e / KIN, i = e % KIN;
    if (i < m.n_in) v = m.theta[m.off[0] + i * HW + o];
  } else if (e < WBF_W3) {
    int q = e - WBF_W2, o = q / HW, i = q % HW;
    v = m.theta[m.off[2] + i * HW + o];
  } else if (e < WBF_W4) {
    int q = e - WBF_W3, o = q / HW, i = q % HW;
    v = m.theta[m.off[4] + i * HW + o];
  } else {
    int q = e - WBF_W4, o = q / HW, i = q % HW;
    if (o < m.n_out) v = m.theta[m.off[6] + i * m.n_out + o];
  }
  wbt[e] = f2bf(v);
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

__global__ void k_features(FeatArgs fa, const double *fld, uint16_t *feat) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= fa.N) return;
  const int D = fa.D, nf = fa.nf, P1 = fa.p + 1;
  const int nfeat = nf * (1 + D);
  int n[3] = {0, 0, 0};
  int64_t stride[3] = {1, fa.Na[0], (int64_t)fa.Na[0] * fa.Na[1]};
  n[0] = (int)(k % fa.Na[0]);
  if (D > 1) n[1] = (int)((k / fa.Na[0]) % fa.Na[1]);
  if (D > 2) n[2] = (int)(k / ((int64_t)fa.Na[0] * fa.Na[1]));
  uint16_t *out = feat + k * nfeat;
  for (int q = 0; q < nf; q++) out[q] = f2bf((float)scaled_field(fa, fld, q, k));
  for (int q = 0; q < nf; q++)
    for (int a = 0; a < D; a++) {
      double s = 0.0;
      const int64_t base = k - (int64_t)n[a] * stride[a];
      for (int slot = 0; slot < 2; slot++) {
        const int32_t *id = fa.didx[a] + ((size_t)n[a] * 2 + slot) * P1;
        const double *w = fa.dw[a] + ((size_t)n[a] * 2 + slot) * P1;
        if (id[0] < 0) continue;
        for (int m = 0; m < P1; m++) s += w[m] * scaled_field(fa, fld, q, base + (int64_t)id[m] * stride[a]);
      }
      out[nf + q * D + a] = f2bf((float)s);
    }
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
  hipLaunchKernelGGL(k_refresh_bf16t, dim3((WBF_N + 255) / 256), dim3(256), 0, s, m->args(), m->wbt);
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
    hipLaunchKernelGGL(k_features, grid, dim3(256), 0, s, fa, (const double *)P->lfield, feat);
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
      !alloc((void **)&m->grad, o * 4) || !alloc((void **)&m->wbf, WBF_N * 2) || !alloc((void **)&m->wbt, WBF_N * 2)) {
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
    hipLaunchKernelGGL(k_features, grid1, dim3(256), 0, s, fa, (const double *)P->lfield, P->lfeat);
  }
  HIP_TRY(hipGetLastError());
  ProjArgs pa{};
  int rc = proj_args(P, pa);
  if (rc) return rc;
  pa.vel = P->tp.vel;
  const dim3 grid((unsigned)std::min<int64_t>((N + RC - 1) / RC, kCorrectGrid));
  {
    ProfScope ps(P, "k_relax_correct", s);
#define RC_LAUNCH(TT, PRV)                                                                                     \
  hipLaunchKernelGGL((k_correct<TT, 1, PRV, 3>), grid, dim3(NTC), 0, s, m->args(), pa, P->tp, a, N,             \
                     (const uint16_t *)P->lfeat, (const double *)P->lfield, (const double *)P->nstate, (TT *)pop)
    if (P->prec == SLLBM_F32) {
      if (a.pr_on) RC_LAUNCH(float, 1);
      else RC_LAUNCH(float, 0);
    } else {
      if (a.pr_on) RC_LAUNCH(double, 1);
      else RC_LAUNCH(double, 0);
    }
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
  dim3 grid((unsigned)std::min<int64_t>((N + RC - 1) / RC, kCorrectGrid));
  const StepArgs none{};
  {
    ProfScope ps(P, "k_mlp_correct", s);
#define MC_LAUNCH(TT, DD)                                                                                      \
  hipLaunchKernelGGL((k_correct<TT, 0, 0, DD>), grid, dim3(NTC), 0, s, m->args(), pa, P->tp, none, N,           \
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
