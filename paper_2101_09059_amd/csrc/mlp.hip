// Learned form: a fully connected GELU network that maps the leading
// Karhunen-Loeve coefficients of log E and log h to the per-node peak radial
// displacement, trained and evaluated with BF16 matrix-core (MFMA) kernels
// accumulating in FP32, plus the multifidelity control-variate combination.
//
// Storage: W_l [out][in] FP32 master copy + BF16 copy, biases FP32, Adam
// moments FP32; activations BF16 between layers, pre-activations FP32.
//
// GEMM: C[M x N] = sum_k A(m, k) B(k, n), 128 x 128 block tile, 32-deep
// K steps staged through two LDS buffers (both operands stored K-contiguous
// there; the next step's tiles are fetched while the current one is
// multiplied), 4 waves of 64 x 64, each a 4 x 4 grid of 16x16x32 BF16 MFMAs.  The
// operands may be K-contiguous or M/N-contiguous in global memory.
// Epilogues: bias + GELU (forward hidden), bias (forward output), FP32
// store with split-K partials (backward data / gradient check, Gram
// matrix), per-row quadratic form sum_n C(m, n) A(m, n) (moments), fused
// Adam update (backward weights).  All reductions run in a fixed order.
//
// Moments over many draws: the output layer is linear, y_r = W h_r + b, so
// per output j
//   sum_r y_rj   = w_j . s + M b_j,                     s = sum_r h_r
//   sum_r y_rj^2 = w_j^T G w_j + 2 b_j w_j . s + M b_j^2, G = sum_r h_r h_r^T
// with h_r the last hidden layer's (BF16) activations: the draws only pass
// through the hidden layers, and the output layer enters once, as the
// product W G (G split into two BF16 parts for the matrix cores) and the
// product W s in FP64.
#include "ensfem.h"
#include "ensfem_surrogate.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32, LDS_STRIDE = BK + 8;

enum Epi { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_BIAS_F32 = 2, EPI_QUAD = 3, EPI_ADAM = 4 };

struct GemmArgs {
  int M, N, K;
  const __bf16* A;
  int64_t a_sm, a_sk;  // A(m, k) = A[m * a_sm + k * a_sk]
  const __bf16* B;
  int64_t b_sk, b_sn;  // B(k, n) = B[k * b_sk + n * b_sn]
  int k_chunk;         // K range per blockIdx.z
  bool vec_ok;         // 16-byte operand loads are aligned
  // epilogue operands
  float* C32;
  int64_t ldc;
  int64_t split_stride;  // elements between split-K partial outputs
  const float* bias;
  float* Z32;
  __bf16* H16;
  float* Q;  // EPI_QUAD: [column tiles][M] per-row partial sums
  float* W32;
  float* M1;
  float* M2;
  __bf16* W16;
  float lr, b1, b2, eps, c1, c2;
  float wd;  // decoupled weight decay of the weight matrix
};

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// A BM x BK (or BN x BK) tile of an operand, global -> registers (two
// 8-element chunks per thread) and registers -> LDS [row][k].
// KC: the operand is contiguous along k in global memory.
template <bool KC>
__device__ __forceinline__ void load_tile(bf16x8 (&v)[2], const __bf16* __restrict__ P, int64_t s_row,
                                          int64_t s_k, int row0, int k0, int rows, int kend, bool vec_ok) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int c = t + 256 * it;
    if constexpr (KC) {
      // 128 rows x 4 chunks of 8 k
      const int r = c >> 2, kc = (c & 3) * 8;
      const int gr = row0 + r, gk = k0 + kc;
      if (gr < rows && gk + 8 <= kend && vec_ok) {
        v[it] = *reinterpret_cast<const bf16x8*>(P + (int64_t)gr * s_row + gk);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[it][e] = (gr < rows && gk + e < kend) ? P[(int64_t)gr * s_row + (int64_t)(gk + e) * s_k] : (__bf16)0.0f;
      }
    } else {
      // 32 k x 16 chunks of 8 rows
      const int kk = c >> 4, rc = (c & 15) * 8;
      const int gk = k0 + kk, gr = row0 + rc;
      if (gk < kend && gr + 8 <= rows && vec_ok) {
        v[it] = *reinterpret_cast<const bf16x8*>(P + (int64_t)gk * s_k + gr);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          v[it][e] = (gk < kend && gr + e < rows) ? P[(int64_t)(gr + e) * s_row + (int64_t)gk * s_k] : (__bf16)0.0f;
      }
    }
  }
}

template <bool KC>
__device__ __forceinline__ void store_tile(__bf16 (*S)[LDS_STRIDE], const bf16x8 (&v)[2]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int c = t + 256 * it;
    if constexpr (KC) {
      const int r = c >> 2, kc = (c & 3) * 8;
      *reinterpret_cast<bf16x8*>(&S[r][kc]) = v[it];
    } else {
      // transposed into [row][k]
      const int kk = c >> 4, rc = (c & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) S[rc + e][kk] = v[it][e];
    }
  }
}

// Two LDS buffers: the next K step's tiles are fetched from global memory
// into registers while the MFMAs run on the current buffer, then written to
// the other buffer; one barrier per K step.
template <bool AK, bool BKC, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __bf16 As[2][BM][LDS_STRIDE];
  __shared__ __bf16 Bs[2][BN][LDS_STRIDE];
  // Tile order: workgroup L runs on XCD L mod 8; each XCD takes every 8th
  // column tile and walks all row tiles of one column tile back to back, so
  // the row tiles that share a B tile read it through one L2.
  const int mt = (g.M + BM - 1) / BM;
  const int xcd = (int)(blockIdx.x & 7), idx = (int)(blockIdx.x >> 3);
  const int mtile = idx % mt, ntile = (idx / mt) * 8 + xcd;
  const int m0 = mtile * BM, n0 = ntile * BN;
  if (n0 >= g.N) return;  // column tiles padded to a multiple of 8 (whole workgroup)
  const int kbeg = blockIdx.z * g.k_chunk;
  const int kend = min(g.K, kbeg + g.k_chunk);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wm = w >> 1, wn = w & 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 va[2], vb[2];
  if (kbeg < kend) {
    load_tile<AK>(va, g.A, g.a_sm, g.a_sk, m0, kbeg, g.M, kend, g.vec_ok);
    load_tile<BKC>(vb, g.B, g.b_sn, g.b_sk, n0, kbeg, g.N, kend, g.vec_ok);
    store_tile<AK>(As[0], va);
    store_tile<BKC>(Bs[0], vb);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      load_tile<AK>(va, g.A, g.a_sm, g.a_sk, m0, k0 + BK, g.M, kend, g.vec_ok);
      load_tile<BKC>(vb, g.B, g.b_sn, g.b_sk, n0, k0 + BK, g.N, kend, g.vec_ok);
    }
    bf16x8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 64 + i * 16 + (l & 15)][8 * (l >> 4)]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * 64 + j * 16 + (l & 15)][8 * (l >> 4)]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (more) {
      store_tile<AK>(As[buf ^ 1], va);
      store_tile<BKC>(Bs[buf ^ 1], vb);
    }
    __syncthreads();
    buf ^= 1;
  }
  // lane l of a 16x16 output tile holds rows 4*(l/16) + r, column l % 16
  if constexpr (EPI == EPI_QUAD) {
    // per row m: sum over this tile's columns n of C(m, n) A(m, n) (A the
    // left operand itself, read again from global memory); lanes with the
    // same l / 16 share rows, a fixed butterfly adds their columns, then the
    // two column halves are added in wave order
    __shared__ float redq[2][BM];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ml = wm * 64 + i * 16 + 4 * (l >> 4) + r;
        const int m = m0 + ml;
        float a = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = n0 + wn * 64 + j * 16 + (l & 15);
          if (m < g.M && n < g.N) a = fmaf(acc[i][j][r], (float)g.A[(int64_t)m * g.a_sm + (int64_t)n * g.a_sk], a);
        }
        a += __shfl_xor(a, 1, 64);
        a += __shfl_xor(a, 2, 64);
        a += __shfl_xor(a, 4, 64);
        a += __shfl_xor(a, 8, 64);
        if ((l & 15) == 0) redq[wn][ml] = a;
      }
    __syncthreads();
    if (threadIdx.x < BM) {
      const int m = m0 + threadIdx.x;
      if (m < g.M) g.Q[(int64_t)(n0 / BN) * g.M + m] = redq[0][threadIdx.x] + redq[1][threadIdx.x];
    }
  } else {
    // j innermost: consecutive accesses cover 64 consecutive columns of a row
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = m0 + wm * 64 + i * 16 + 4 * (l >> 4) + r;
          const int n = n0 + wn * 64 + j * 16 + (l & 15);
          if (m >= g.M || n >= g.N) continue;
          const float v = acc[i][j][r];
          const int64_t idx = (int64_t)m * g.ldc + n;
          if constexpr (EPI == EPI_F32) {
            g.C32[blockIdx.z * g.split_stride + idx] = v;
          } else if constexpr (EPI == EPI_BIAS_GELU) {
            const float z = v + g.bias[n];
            if (g.Z32) g.Z32[idx] = z;  // pre-activations are kept for training only
            g.H16[idx] = (__bf16)gelu_f(z);
          } else if constexpr (EPI == EPI_BIAS_F32) {
            g.C32[idx] = v + g.bias[n];
          } else if constexpr (EPI == EPI_ADAM) {
            const float m1 = fmaf(g.b1, g.M1[idx], (1.f - g.b1) * v);
            const float m2 = fmaf(g.b2, g.M2[idx], (1.f - g.b2) * v * v);
            const float w0 = g.W32[idx];
            const float wv = w0 - g.lr * ((m1 * g.c1) / (sqrtf(m2 * g.c2) + g.eps) + g.wd * w0);
            g.M1[idx] = m1;
            g.M2[idx] = m2;
            g.W32[idx] = wv;
            g.W16[idx] = (__bf16)wv;
          }
        }
  }
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, __bf16* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) y[t] = (__bf16)x[t];
}

// sum of split-K partials in split order
__global__ void k_split_reduce(int64_t n, int splits, int64_t stride, const float* __restrict__ P,
                               float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += P[z * stride + t];
  out[t] = s;
}

// dZ = dH * GELU'(Z): FP32 copy (bias gradient) and BF16 copy (GEMMs)
__global__ void k_gelu_bwd(int64_t n, const float* __restrict__ dH, const float* __restrict__ Z,
                           float* __restrict__ dZ32, __bf16* __restrict__ dZ16) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float d = dH[t] * gelu_grad_f(Z[t]);
  dZ32[t] = d;
  dZ16[t] = (__bf16)d;
}

// MSE: dY = 2 (Y - T) / (B n) in BF16 and FP32; per-block partial loss sums.
__global__ void k_mse(int64_t n, float scale, const float* __restrict__ Y, const float* __restrict__ T,
                      __bf16* __restrict__ dY16, float* __restrict__ dY32, double* __restrict__ part) {
  __shared__ double red[256];
  double e2 = 0.0;
  // grid-stride: one partial per workgroup, at most kLossParts of them
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
    const float d = Y[t] - T[t];
    dY16[t] = (__bf16)(2.f * scale * d);
    if (dY32) dY32[t] = 2.f * scale * d;
    e2 += (double)d * (double)d;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One block of 256: each thread sums a fixed stride of the partials, then a
// fixed tree (deterministic order).
__global__ __launch_bounds__(256) void k_loss_final(int nparts, const double* __restrict__ part, double scale,
                                                    float* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] * scale);
}

// column sums of a [rows][cols] FP32 matrix: a workgroup takes 64 columns,
// its 4 waves sum every 4th row (in order), the 4 sums are added in wave
// order
__global__ __launch_bounds__(256) void k_colsum(int rows, int cols, const float* __restrict__ X,
                                                float* __restrict__ out) {
  __shared__ float red[256];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (c < cols)
    for (int r = g; r < rows; r += 4) s += X[(int64_t)r * cols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && c < cols) out[c] = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
}

__global__ void k_adam_vec(int n, const float* __restrict__ g, float* __restrict__ w, float* __restrict__ m1,
                           float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float a = fmaf(b1, m1[t], (1.f - b1) * g[t]);
  const float b = fmaf(b2, m2[t], (1.f - b2) * g[t] * g[t]);
  m1[t] = a;
  m2[t] = b;
  w[t] = w[t] - lr * (a * c1) / (sqrtf(b * c2) + eps);
}

__global__ void k_zero64(int64_t n, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = 0.0;
}

// Gram matrix update G += sum of the split-K partials [splits][n] (split
// order), in FP64.
__global__ void k_gram_acc(int64_t n, int splits, const float* __restrict__ part, double* __restrict__ G) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double a = 0.0;
  for (int z = 0; z < splits; ++z) a += (double)part[z * n + t];
  G[t] += a;
}

// Column sums of H (BF16 [rows][cols]) in kColGroups row groups:
// part[g][c] = sum over the rows of group g (in order).
constexpr int kColGroups = 16;
__global__ void k_colsum_part(int rows, int cols, const __bf16* __restrict__ H, double* __restrict__ part) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (c >= cols) return;
  const int per = (rows + kColGroups - 1) / kColGroups;
  const int r1 = min(rows, (g + 1) * per);
  double a = 0.0;
  for (int r = g * per; r < r1; ++r) a += (double)(float)H[(int64_t)r * cols + c];
  part[(int64_t)g * cols + c] = a;
}

// s[c] += the kColGroups partials of column c (group order).
__global__ void k_colsum_acc(int cols, const double* __restrict__ part, double* __restrict__ s) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  double a = 0.0;
  for (int g = 0; g < kColGroups; ++g) a += part[(int64_t)g * cols + c];
  s[c] += a;
}

// G (FP64) = hi + lo with hi = bf16(G) and lo = bf16(G - hi).
__global__ void k_split_hilo(int64_t n, const double* __restrict__ G, __bf16* __restrict__ hi,
                             __bf16* __restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const __bf16 h = (__bf16)(float)G[t];
  hi[t] = h;
  lo[t] = (__bf16)(float)(G[t] - (double)(float)h);
}

// ws[j] = sum_k W[j][k] s[k] in FP64 (W BF16 [rows][K]); one wave per row,
// lane-strided sums then a fixed butterfly.
__global__ __launch_bounds__(256) void k_rowdot64(int rows, int K, const __bf16* __restrict__ W,
                                                  const double* __restrict__ sv, double* __restrict__ ws) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (row >= rows) return;
  const __bf16* w = W + (int64_t)row * K;
  double a = 0.0;
  for (int k = l; k < K; k += 64) a = fma((double)(float)w[k], sv[k], a);
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if (l == 0) ws[row] = a;
}

// Output-layer moments from the hidden-layer sums: S1 = W s + M b,
// S2 = w^T G w + 2 b (W s) + M b^2, the quadratic forms from the per-tile
// partials of W G_hi and W G_lo (tile order).
__global__ void k_moments_final(int n_out, int tiles, double M, const float* __restrict__ qhi,
                                const float* __restrict__ qlo, const double* __restrict__ ws,
                                const float* __restrict__ bias, double* __restrict__ S1, double* __restrict__ S2) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_out) return;
  double q = 0.0;
  for (int t = 0; t < tiles; ++t) q += (double)qhi[(int64_t)t * n_out + j] + (double)qlo[(int64_t)t * n_out + j];
  const double b = (double)bias[j];
  S1[j] = fma(M, b, ws[j]);
  S2[j] = fma(M * b, b, fma(2.0 * b, ws[j], q));
}

// Squared error of the physical-unit predictions mu + sd y against Q over
// [rows][n_out] (FP64): per-workgroup partials in a fixed order.
__global__ __launch_bounds__(256) void k_sq_error(int64_t n, int n_out, const float* __restrict__ y,
                                                  const double* __restrict__ Q, const double* __restrict__ mu,
                                                  const double* __restrict__ sd, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int j = (int)(i % n_out);
    const double d = fma(sd[j], (double)y[i], mu[j]) - Q[i];
    acc = fma(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// *acc += the sum of the partials (fixed order, one workgroup)
__global__ __launch_bounds__(256) void k_parts_add(int nparts, const double* __restrict__ part,
                                                   double* __restrict__ acc) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) v += part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

// dst[r][:] = src[idx[r]][:] for FP32 rows of n_cols values.
__global__ __launch_bounds__(256) void k_gather_rows(int64_t n_cols, const int32_t* __restrict__ idx,
                                                     const float* __restrict__ src, float* __restrict__ dst) {
  const int64_t r = blockIdx.y;
  const float* from = src + (int64_t)idx[r] * n_cols;
  float* to = dst + r * n_cols;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n_cols; c += (int64_t)gridDim.x * 256)
    to[c] = from[c];
}

// Control-variate combination per node (FP64), see sur_cv_moments.
__global__ void k_cv(int64_t n, int N, const double* __restrict__ qH, const double* __restrict__ qL,
                     const double* __restrict__ sL, const double* __restrict__ sL2, double M,
                     double* __restrict__ mean, double* __restrict__ var, double* __restrict__ rho) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double* h = qH + i * N;
  const double* q = qL + i * N;
  // two estimators: the values (first moment) and their squares (second)
  double est[2];
  double rho1 = 0.0;
  for (int p = 0; p < 2; ++p) {
    double hm = 0.0, lm = 0.0;
    for (int s = 0; s < N; ++s) {
      const double a = p ? h[s] * h[s] : h[s];
      const double b = p ? q[s] * q[s] : q[s];
      hm += a;
      lm += b;
    }
    hm /= N;
    lm /= N;
    double cov = 0.0, vl = 0.0, vh = 0.0;
    for (int s = 0; s < N; ++s) {
      const double a = (p ? h[s] * h[s] : h[s]) - hm;
      const double b = (p ? q[s] * q[s] : q[s]) - lm;
      cov += a * b;
      vl += b * b;
      vh += a * a;
    }
    cov /= (N - 1);
    vl /= (N - 1);
    vh /= (N - 1);
    const double beta = vl > 0.0 ? cov / vl : 0.0;
    const double lM = (p ? sL2[i] : sL[i]) / M;
    est[p] = hm - beta * (lm - lM);
    if (p == 0) rho1 = (vl > 0.0 && vh > 0.0) ? cov / sqrt(vl * vh) : 0.0;
  }
  mean[i] = est[0];
  var[i] = est[1] - est[0] * est[0];
  rho[i] = rho1;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }
constexpr unsigned kLossParts = 2048;  // workgroups (and partial sums) of the loss
constexpr int kMomRows = 4096;         // rows per pass of the moments
constexpr int kGramSplits = 4;         // split-K partials of the Gram matrix

}  // namespace

struct sur_net {
  int device = 0;
  int n_in = 0, width = 0, n_hidden = 0, n_out = 0, max_batch = 0;
  std::string err;
  // layer geometry
  std::vector<int> fan_in, fan_out;
  std::vector<size_t> w_off, b_off;  // offsets into the parameter vector (floats)
  size_t n_params = 0;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t o_p32 = 0, o_m1 = 0, o_m2 = 0, o_w16 = 0, o_h0 = 0, o_z = 0, o_h = 0, o_y = 0, o_dy16 = 0,
         o_dh = 0, o_dz32 = 0, o_dz16 = 0, o_split = 0, o_db = 0, o_mx = 0, o_ma = 0, o_mb = 0, o_gpart = 0,
         o_g64 = 0, o_s64 = 0, o_cpart = 0, o_ghl = 0, o_qp = 0, o_ws = 0, o_s1 = 0, o_s2 = 0,
         o_lpart = 0, o_loss = 0, total = 0;
  int splits_max = 64;
  float wd = 0.0f;  // decoupled weight decay (weight matrices only)
  bool bound = false, have_params = false;
  int64_t t = 0;  // Adam steps taken
  int32_t fail(int32_t c, const std::string& m) {
    err = m;
    return c;
  }
  template <class T>
  T* p(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float* W32(int l) const { return p<float>(o_p32) + w_off[l]; }
  float* B32(int l) const { return p<float>(o_p32) + b_off[l]; }
  __bf16* W16(int l) const { return p<__bf16>(o_w16) + w_off[l]; }
  float* Z(int l) const { return p<float>(o_z) + (size_t)l * max_batch * width; }      // l = 0..n_hidden-1
  __bf16* H(int l) const {  // l = 0: input, l >= 1 hidden outputs
    return l == 0 ? p<__bf16>(o_h0) : p<__bf16>(o_h) + (size_t)(l - 1) * max_batch * width;
  }
};

#define SHIPC(expr)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return s->fail(ENS_EDEVICE, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr); \
  } while (0)

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

void plan(sur_net* s) {
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = al(off + b);
    return o;
  };
  const size_t B = s->max_batch, W = s->width;
  s->o_p32 = take(4 * s->n_params);
  s->o_m1 = take(4 * s->n_params);
  s->o_m2 = take(4 * s->n_params);
  s->o_w16 = take(2 * s->n_params);
  s->o_h0 = take(2 * B * s->n_in);
  s->o_z = take(4 * B * W * s->n_hidden);
  s->o_h = take(2 * B * W * s->n_hidden);
  s->o_y = take(4 * B * s->n_out);
  s->o_dy16 = take(2 * B * s->n_out);
  s->o_dh = take(4 * B * W);
  s->o_dz32 = take(4 * B * std::max<size_t>(W, s->n_out));
  s->o_dz16 = take(2 * B * W);
  s->o_split = take(4 * (size_t)s->splits_max * B * W);
  s->o_db = take(4 * std::max<size_t>(W, s->n_out));
  // moments: kMomRows rows per pass through the hidden layers (BF16 input
  // and two activation buffers), the Gram matrix as split-K partials and in
  // FP64, its BF16 halves, the quadratic-form partials of both halves, W s
  const size_t C = kMomRows, nt = (W + BN - 1) / BN;
  s->o_mx = take(2 * C * s->n_in);
  s->o_ma = take(2 * C * W);
  s->o_mb = take(2 * C * W);
  s->o_gpart = take(4 * (size_t)kGramSplits * W * W);
  s->o_g64 = take(8 * W * W);
  s->o_s64 = take(8 * W);
  s->o_cpart = take(8 * (size_t)kColGroups * W);
  s->o_ghl = take(2 * 2 * W * W);
  s->o_qp = take(4 * 2 * nt * (size_t)s->n_out);
  s->o_ws = take(8 * (size_t)s->n_out);
  s->o_s1 = take(8 * (size_t)s->n_out);
  s->o_s2 = take(8 * (size_t)s->n_out);
  s->o_lpart = take(8 * (size_t)kLossParts);
  s->o_loss = take(4);
  s->total = off;
}

template <bool AK, bool BKC, int EPI>
hipError_t gemm(GemmArgs g, int splits, hipStream_t st) {
  const unsigned mt = (unsigned)((g.M + BM - 1) / BM), nt = (unsigned)((g.N + BN - 1) / BN);
  dim3 grid(mt * ((nt + 7) / 8 * 8), 1, splits);
  k_gemm<AK, BKC, EPI><<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
}

GemmArgs base_gemm(int M, int N, int K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.M = M;
  g.N = N;
  g.K = K;
  g.k_chunk = K;
  return g;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Forward through the hidden layers for `batch` rows of X (FP32 [batch][n_in]).
int32_t forward_hidden(sur_net* s, const float* X, int batch, hipStream_t st) {
  SHIPC((k_to_bf16<<<blocks((int64_t)batch * s->n_in), 256, 0, st>>>((int64_t)batch * s->n_in, X, s->H(0)),
         hipGetLastError()));
  for (int l = 0; l < s->n_hidden; ++l) {
    const int in = s->fan_in[l], out = s->fan_out[l];
    GemmArgs g = base_gemm(batch, out, in);
    g.A = s->H(l);
    g.a_sm = in;
    g.a_sk = 1;
    g.B = s->W16(l);
    g.b_sk = 1;
    g.b_sn = in;
    g.vec_ok = (in % 8 == 0) && aligned16(g.A) && aligned16(g.B);
    g.ldc = out;
    g.bias = s->B32(l);
    g.Z32 = s->Z(l);
    g.H16 = s->H(l + 1);
    SHIPC((gemm<true, true, EPI_BIAS_GELU>(g, 1, st)));
  }
  return ENS_OK;
}

GemmArgs output_gemm(sur_net* s, int batch) {
  const int L = s->n_hidden, in = s->fan_in[L], out = s->fan_out[L];
  GemmArgs g = base_gemm(batch, out, in);
  g.A = s->H(L);
  g.a_sm = in;
  g.a_sk = 1;
  g.B = s->W16(L);
  g.b_sk = 1;
  g.b_sn = in;
  g.vec_ok = (in % 8 == 0) && aligned16(g.A) && aligned16(g.B);
  g.ldc = out;
  g.bias = s->B32(L);
  return g;
}

int split_count(const sur_net* s, int M, int N, int K) {
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int sp = std::max(1, 512 / std::max(1, tiles));
  sp = std::min(sp, s->splits_max);
  sp = std::min(sp, std::max(1, K / (4 * BK)));
  return sp;
}

// dH = dZ_next (bf16 [batch][out]) * W (bf16 [out][in]) -> FP32 [batch][in]
int32_t backward_data(sur_net* s, int layer, const __bf16* dZ, int batch, float* dH, hipStream_t st) {
  const int in = s->fan_in[layer], out = s->fan_out[layer];
  const int sp = split_count(s, batch, in, out);
  GemmArgs g = base_gemm(batch, in, out);
  g.A = dZ;
  g.a_sm = out;
  g.a_sk = 1;
  g.B = s->W16(layer);
  g.b_sk = in;
  g.b_sn = 1;
  g.vec_ok = (out % 8 == 0) && (in % 8 == 0) && aligned16(g.A) && aligned16(g.B);
  g.k_chunk = ((out + sp - 1) / sp + BK - 1) / BK * BK;
  const int splits = (out + g.k_chunk - 1) / g.k_chunk;
  g.ldc = in;
  g.split_stride = (int64_t)batch * in;
  g.C32 = s->p<float>(s->o_split);
  SHIPC((gemm<true, false, EPI_F32>(g, splits, st)));
  const int64_t n = (int64_t)batch * in;
  SHIPC((k_split_reduce<<<blocks(n), 256, 0, st>>>(n, splits, g.split_stride, g.C32, dH), hipGetLastError()));
  return ENS_OK;
}

// weight gradient dW = dZ^T H (dZ bf16 [batch][out], H bf16 [batch][in]),
// either stored (grad != null) or applied by Adam
int32_t backward_weight(sur_net* s, int layer, const __bf16* dZ, const __bf16* Hin, int batch, float* grad,
                        float lr, float c1, float c2, hipStream_t st) {
  const int in = s->fan_in[layer], out = s->fan_out[layer];
  GemmArgs g = base_gemm(out, in, batch);
  g.A = dZ;
  g.a_sm = 1;
  g.a_sk = out;
  g.B = Hin;
  g.b_sk = in;
  g.b_sn = 1;
  g.vec_ok = (out % 8 == 0) && (in % 8 == 0) && aligned16(g.A) && aligned16(g.B);
  g.ldc = in;
  if (grad) {
    g.C32 = grad;
    SHIPC((gemm<false, false, EPI_F32>(g, 1, st)));
  } else {
    g.W32 = s->W32(layer);
    g.M1 = s->p<float>(s->o_m1) + s->w_off[layer];
    g.M2 = s->p<float>(s->o_m2) + s->w_off[layer];
    g.W16 = s->W16(layer);
    g.lr = lr;
    g.b1 = 0.9f;
    g.b2 = 0.999f;
    g.eps = 1e-8f;
    g.c1 = c1;
    g.c2 = c2;
    g.wd = s->wd;
    SHIPC((gemm<false, false, EPI_ADAM>(g, 1, st)));
  }
  return ENS_OK;
}

// Full backward pass after a forward pass that left Y in o_y.  grad != null:
// store the gradient vector (layout of the parameters); else Adam step.
int32_t backward(sur_net* s, const float* T, int batch, float* grad, float* loss_dev, float lr,
                 hipStream_t st) {
  const int L = s->n_hidden;
  const int64_t ny = (int64_t)batch * s->n_out;
  const unsigned nb = std::min(blocks(ny), kLossParts);
  float* dY32 = s->p<float>(s->o_dz32);  // FP32 dY reuses the dZ32 buffer (sized for n_out)
  SHIPC((k_mse<<<nb, 256, 0, st>>>(ny, 1.0f / (float)ny, s->p<float>(s->o_y), T, s->p<__bf16>(s->o_dy16), dY32,
                                   s->p<double>(s->o_lpart)),
         hipGetLastError()));
  SHIPC((k_loss_final<<<1, 256, 0, st>>>((int)nb, s->p<double>(s->o_lpart), 1.0 / (double)ny,
                                        loss_dev ? loss_dev : s->p<float>(s->o_loss)),
         hipGetLastError()));
  const double t = (double)(s->t + 1);
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
  const __bf16* dZ = s->p<__bf16>(s->o_dy16);
  const float* dZf = dY32;
  for (int l = L; l >= 0; --l) {
    const int in = s->fan_in[l], out = s->fan_out[l];
    // bias gradient
    float* db = grad ? grad + s->b_off[l] : s->p<float>(s->o_db);
    SHIPC((k_colsum<<<(unsigned)((out + 63) / 64), 256, 0, st>>>(batch, out, dZf, db), hipGetLastError()));
    if (!grad) {
      float* m1 = s->p<float>(s->o_m1) + s->b_off[l];
      float* m2 = s->p<float>(s->o_m2) + s->b_off[l];
      SHIPC((k_adam_vec<<<blocks(out), 256, 0, st>>>(out, db, s->B32(l), m1, m2, lr, 0.9f, 0.999f, 1e-8f, c1, c2),
             hipGetLastError()));
    }
    // data gradient for the layer below (uses the weights before their update)
    if (l > 0) {
      float* dH = s->p<float>(s->o_dh);
      int32_t rc = backward_data(s, l, dZ, batch, dH, st);
      if (rc != ENS_OK) return rc;
      const int64_t n = (int64_t)batch * in;
      // the weight update below still reads dZ of this layer: write the next
      // dZ into the other half of the buffers
      rc = backward_weight(s, l, dZ, s->H(l), batch, grad ? grad + s->w_off[l] : nullptr, lr, c1, c2, st);
      if (rc != ENS_OK) return rc;
      SHIPC((k_gelu_bwd<<<blocks(n), 256, 0, st>>>(n, dH, s->Z(l - 1), s->p<float>(s->o_dz32),
                                                   s->p<__bf16>(s->o_dz16)),
             hipGetLastError()));
      dZ = s->p<__bf16>(s->o_dz16);
      dZf = s->p<float>(s->o_dz32);
    } else {
      const int32_t rc = backward_weight(s, 0, dZ, s->H(0), batch, grad ? grad + s->w_off[0] : nullptr, lr, c1,
                                         c2, st);
      if (rc != ENS_OK) return rc;
    }
  }
  if (!grad) s->t += 1;
  return ENS_OK;
}

}  // namespace

extern "C" {

int32_t sur_create(int32_t device, int32_t n_in, int32_t width, int32_t n_hidden, int32_t n_out,
                   int32_t max_batch, sur_net** out) {
  if (!out) return ENS_EINVAL;
  *out = nullptr;
  if (n_in < 1 || width < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1) return ENS_EINVAL;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return ENS_EDEVICE;
  sur_net* s = new (std::nothrow) sur_net();
  if (!s) return ENS_EINVAL;
  s->device = device;
  s->n_in = n_in;
  s->width = width;
  s->n_hidden = n_hidden;
  s->n_out = n_out;
  s->max_batch = max_batch;
  size_t off = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    const int in = l == 0 ? n_in : width;
    const int o = l == n_hidden ? n_out : width;
    s->fan_in.push_back(in);
    s->fan_out.push_back(o);
    s->w_off.push_back(off);
    off += (size_t)in * o;
    s->b_off.push_back(off);
    off += o;
  }
  s->n_params = off;
  plan(s);
  *out = s;
  return ENS_OK;
}

int32_t sur_destroy(sur_net* s) {
  if (!s) return ENS_EINVAL;
  if (s->bound) {  // teardown: nothing to report
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
  }
  delete s;
  return ENS_OK;
}

const char* sur_last_error(const sur_net* s) { return s ? s->err.c_str() : "null network"; }

int32_t sur_info(sur_net* s, int64_t* n_params, size_t* workspace_bytes) {
  if (!s) return ENS_EINVAL;
  if (n_params) *n_params = (int64_t)s->n_params;
  if (workspace_bytes) *workspace_bytes = s->total;
  return ENS_OK;
}

int32_t sur_bind_workspace(sur_net* s, void* dptr, size_t bytes) {
  if (!s) return ENS_EINVAL;
  if (!dptr || (reinterpret_cast<uintptr_t>(dptr) & 255) != 0)
    return s->fail(ENS_EWORKSPACE, "sur_bind_workspace: null or unaligned (256 B) buffer");
  if (bytes < s->total)
    return s->fail(ENS_EWORKSPACE, "sur_bind_workspace: need " + std::to_string(s->total) + " bytes");
  s->ws = static_cast<char*>(dptr);
  s->ws_bytes = bytes;
  s->bound = true;
  s->have_params = false;
  return ENS_OK;
}

int32_t sur_set_weight_decay(sur_net* s, float wd) {
  if (!s) return ENS_EINVAL;
  if (!(wd >= 0.0f) || !std::isfinite(wd)) return s->fail(ENS_EINVAL, "sur_set_weight_decay: need a finite wd >= 0");
  s->wd = wd;
  return ENS_OK;
}

int32_t sur_set_params(sur_net* s, const float* host) {
  if (!s || !host) return ENS_EINVAL;
  if (!s->bound) return s->fail(ENS_EWORKSPACE, "sur_set_params: bind a workspace first");
  for (size_t i = 0; i < s->n_params; ++i)
    if (!std::isfinite(host[i])) return s->fail(ENS_EINVAL, "sur_set_params: non-finite parameter");
  SHIPC(hipSetDevice(s->device));
  SHIPC(hipMemcpy(s->p<float>(s->o_p32), host, 4 * s->n_params, hipMemcpyHostToDevice));
  SHIPC(hipMemset(s->p<float>(s->o_m1), 0, 4 * s->n_params));
  SHIPC(hipMemset(s->p<float>(s->o_m2), 0, 4 * s->n_params));
  SHIPC((k_to_bf16<<<blocks((int64_t)s->n_params), 256>>>((int64_t)s->n_params, s->p<float>(s->o_p32),
                                                          s->p<__bf16>(s->o_w16)),
         hipGetLastError()));
  SHIPC(hipDeviceSynchronize());
  s->t = 0;
  s->have_params = true;
  return ENS_OK;
}

int32_t sur_get_params(sur_net* s, float* host) {
  if (!s || !host) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_get_params: no parameters");
  SHIPC(hipSetDevice(s->device));
  SHIPC(hipDeviceSynchronize());
  SHIPC(hipMemcpy(host, s->p<float>(s->o_p32), 4 * s->n_params, hipMemcpyDeviceToHost));
  return ENS_OK;
}

int32_t sur_get_params_device(sur_net* s, float* dptr, void* stream) {
  if (!s || !dptr) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_get_params_device: no parameters");
  SHIPC(hipSetDevice(s->device));
  SHIPC(hipMemcpyAsync(dptr, s->p<float>(s->o_p32), 4 * s->n_params, hipMemcpyDeviceToDevice,
                       static_cast<hipStream_t>(stream)));
  return ENS_OK;
}

int32_t sur_forward(sur_net* s, const float* X, int32_t batch, float* Y, void* stream) {
  if (!s || !X || !Y) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_forward: set the parameters first");
  if (batch < 1 || batch > s->max_batch) return s->fail(ENS_EINVAL, "sur_forward: batch out of range");
  SHIPC(hipSetDevice(s->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t rc = forward_hidden(s, X, batch, st);
  if (rc != ENS_OK) return rc;
  GemmArgs g = output_gemm(s, batch);
  g.C32 = Y;
  SHIPC((gemm<true, true, EPI_BIAS_F32>(g, 1, st)));
  return ENS_OK;
}

int32_t sur_gradients(sur_net* s, const float* X, const float* T, int32_t batch, float* grad, float* loss,
                      void* stream) {
  if (!s || !X || !T || !grad) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_gradients: set the parameters first");
  if (batch < 1 || batch > s->max_batch) return s->fail(ENS_EINVAL, "sur_gradients: batch out of range");
  SHIPC(hipSetDevice(s->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t rc = forward_hidden(s, X, batch, st);
  if (rc != ENS_OK) return rc;
  GemmArgs g = output_gemm(s, batch);
  g.C32 = s->p<float>(s->o_y);
  SHIPC((gemm<true, true, EPI_BIAS_F32>(g, 1, st)));
  return backward(s, T, batch, grad, loss, 0.f, st);
}

int32_t sur_train_step(sur_net* s, const float* X, const float* T, int32_t batch, float lr, float* loss,
                       void* stream) {
  if (!s || !X || !T) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_train_step: set the parameters first");
  if (batch < 1 || batch > s->max_batch) return s->fail(ENS_EINVAL, "sur_train_step: batch out of range");
  if (!(lr >= 0.f)) return s->fail(ENS_EINVAL, "sur_train_step: lr must be >= 0");
  SHIPC(hipSetDevice(s->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t rc = forward_hidden(s, X, batch, st);
  if (rc != ENS_OK) return rc;
  GemmArgs g = output_gemm(s, batch);
  g.C32 = s->p<float>(s->o_y);
  SHIPC((gemm<true, true, EPI_BIAS_F32>(g, 1, st)));
  return backward(s, T, batch, nullptr, loss, lr, st);
}

int32_t sur_moments(sur_net* s, const float* X, int64_t M, double* sum_host, double* sumsq_host,
                    void* stream) {
  if (!s || !X || !sum_host || !sumsq_host || M < 1) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_moments: set the parameters first");
  SHIPC(hipSetDevice(s->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int Wd = s->width, L = s->n_hidden, n_out = s->n_out;
  const int64_t WW = (int64_t)Wd * Wd;
  double* G = s->p<double>(s->o_g64);
  double* sv = s->p<double>(s->o_s64);
  SHIPC((k_zero64<<<blocks(WW), 256, 0, st>>>(WW, G), hipGetLastError()));
  SHIPC((k_zero64<<<blocks(Wd), 256, 0, st>>>(Wd, sv), hipGetLastError()));
  __bf16* buf[2] = {s->p<__bf16>(s->o_ma), s->p<__bf16>(s->o_mb)};
  for (int64_t r0 = 0; r0 < M; r0 += kMomRows) {
    const int rows = (int)std::min<int64_t>(kMomRows, M - r0);
    // hidden layers (no pre-activations kept)
    __bf16* X16 = s->p<__bf16>(s->o_mx);
    SHIPC((k_to_bf16<<<blocks((int64_t)rows * s->n_in), 256, 0, st>>>((int64_t)rows * s->n_in,
                                                                      X + r0 * s->n_in, X16),
           hipGetLastError()));
    const __bf16* Hin = X16;
    for (int l = 0; l < L; ++l) {
      const int in = s->fan_in[l], out = s->fan_out[l];
      GemmArgs g = base_gemm(rows, out, in);
      g.A = Hin;
      g.a_sm = in;
      g.a_sk = 1;
      g.B = s->W16(l);
      g.b_sk = 1;
      g.b_sn = in;
      g.vec_ok = (in % 8 == 0) && aligned16(g.A) && aligned16(g.B);
      g.ldc = out;
      g.bias = s->B32(l);
      g.Z32 = nullptr;
      g.H16 = buf[l & 1];
      SHIPC((gemm<true, true, EPI_BIAS_GELU>(g, 1, st)));
      Hin = g.H16;
    }
    // G += H^T H (split-K partials, then FP64 in split order), s += column sums
    GemmArgs g = base_gemm(Wd, Wd, rows);
    g.A = Hin;
    g.a_sm = 1;
    g.a_sk = Wd;
    g.B = Hin;
    g.b_sk = Wd;
    g.b_sn = 1;
    g.vec_ok = (Wd % 8 == 0) && aligned16(g.A);
    g.k_chunk = ((rows + kGramSplits - 1) / kGramSplits + BK - 1) / BK * BK;
    const int splits = (rows + g.k_chunk - 1) / g.k_chunk;
    g.ldc = Wd;
    g.split_stride = WW;
    g.C32 = s->p<float>(s->o_gpart);
    SHIPC((gemm<false, false, EPI_F32>(g, splits, st)));
    SHIPC((k_gram_acc<<<blocks(WW), 256, 0, st>>>(WW, splits, g.C32, G), hipGetLastError()));
    double* cpart = s->p<double>(s->o_cpart);
    SHIPC((k_colsum_part<<<dim3(blocks(Wd), kColGroups), 256, 0, st>>>(rows, Wd, Hin, cpart), hipGetLastError()));
    SHIPC((k_colsum_acc<<<blocks(Wd), 256, 0, st>>>(Wd, cpart, sv), hipGetLastError()));
  }
  // output layer: W G (both BF16 halves of G) as per-row quadratic forms,
  // W s in FP64, then the sums
  __bf16* Ghi = s->p<__bf16>(s->o_ghl);
  __bf16* Glo = Ghi + WW;
  SHIPC((k_split_hilo<<<blocks(WW), 256, 0, st>>>(WW, G, Ghi, Glo), hipGetLastError()));
  const int nt = (Wd + BN - 1) / BN;
  float* qp = s->p<float>(s->o_qp);
  for (int half = 0; half < 2; ++half) {
    GemmArgs g = base_gemm(n_out, Wd, Wd);
    g.A = s->W16(L);
    g.a_sm = Wd;
    g.a_sk = 1;
    g.B = half ? Glo : Ghi;  // symmetric: B(k, n) = G[n][k]
    g.b_sk = 1;
    g.b_sn = Wd;
    g.vec_ok = (Wd % 8 == 0) && aligned16(g.A) && aligned16(g.B);
    g.Q = qp + (int64_t)half * nt * n_out;
    SHIPC((gemm<true, true, EPI_QUAD>(g, 1, st)));
  }
  double* ws = s->p<double>(s->o_ws);
  SHIPC((k_rowdot64<<<(unsigned)((n_out + 3) / 4), 256, 0, st>>>(n_out, Wd, s->W16(L), sv, ws), hipGetLastError()));
  double* S1 = s->p<double>(s->o_s1);
  double* S2 = s->p<double>(s->o_s2);
  SHIPC((k_moments_final<<<blocks(n_out), 256, 0, st>>>(n_out, nt, (double)M, qp, qp + (int64_t)nt * n_out, ws,
                                                        s->B32(L), S1, S2),
         hipGetLastError()));
  SHIPC(hipStreamSynchronize(st));
  SHIPC(hipMemcpy(sum_host, S1, 8 * (size_t)n_out, hipMemcpyDeviceToHost));
  SHIPC(hipMemcpy(sumsq_host, S2, 8 * (size_t)n_out, hipMemcpyDeviceToHost));
  return ENS_OK;
}

int32_t sur_sq_error(sur_net* s, const float* X, int32_t batch, const double* Q, const double* mu, const double* sd,
                     double* acc, void* stream) {
  if (!s || !X || !Q || !mu || !sd || !acc) return ENS_EINVAL;
  if (!s->have_params) return s->fail(ENS_ESTATE, "sur_sq_error: set the parameters first");
  if (batch < 1 || batch > s->max_batch) return s->fail(ENS_EINVAL, "sur_sq_error: batch out of range");
  SHIPC(hipSetDevice(s->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t rc = forward_hidden(s, X, batch, st);
  if (rc != ENS_OK) return rc;
  GemmArgs g = output_gemm(s, batch);
  g.C32 = s->p<float>(s->o_y);
  SHIPC((gemm<true, true, EPI_BIAS_F32>(g, 1, st)));
  const int64_t n = (int64_t)batch * s->n_out;
  const unsigned nb = std::min(blocks(n), kLossParts);
  SHIPC((k_sq_error<<<nb, 256, 0, st>>>(n, s->n_out, s->p<float>(s->o_y), Q, mu, sd, s->p<double>(s->o_lpart)),
         hipGetLastError()));
  SHIPC((k_parts_add<<<1, 256, 0, st>>>((int)nb, s->p<double>(s->o_lpart), acc), hipGetLastError()));
  return ENS_OK;
}

int32_t sur_gather_rows(const float* src, int64_t n_cols, const int32_t* idx, int32_t n_rows, float* dst,
                        void* stream) {
  if (!src || !idx || !dst || n_cols < 1 || n_rows < 0 || n_rows > 65535) return ENS_EINVAL;
  if (n_rows == 0) return ENS_OK;
  const unsigned gx = (unsigned)std::min<int64_t>((n_cols + 255) / 256, 1024);
  k_gather_rows<<<dim3(gx, (unsigned)n_rows), 256, 0, static_cast<hipStream_t>(stream)>>>(n_cols, idx, src, dst);
  return hipGetLastError() == hipSuccess ? ENS_OK : ENS_EDEVICE;
}

int32_t sur_cv_moments(const double* qH, const double* qL, int64_t n, int32_t N, const double* sumL,
                       const double* sumsqL, int64_t M, double* mean, double* var, double* rho, void* stream) {
  if (!qH || !qL || !sumL || !sumsqL || !mean || !var || !rho || n < 1 || N < 2 || M < 1) return ENS_EINVAL;
  k_cv<<<blocks(n), 256, 0, static_cast<hipStream_t>(stream)>>>(n, N, qH, qL, sumL, sumsqL, (double)M, mean,
                                                                var, rho);
  return hipGetLastError() == hipSuccess ? ENS_OK : ENS_EDEVICE;
}

}  // extern "C"
