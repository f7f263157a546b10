// mlp.hpp -- learned tagging: per-patch statistics, and a small network
// (16 -> 64 -> 64 -> 3, GELU) that predicts refine / keep / coarsen tags,
// trained and evaluated with bfloat16 matrix-core (MFMA) products and FP32
// accumulation.  An extension of the criterion tagging of Sec. 5.
//
// Parameter vector (FP32 master copy, kMlpParams floats):
//   W1[16][64] b1[64] W2[64][64] b2[64] W3[64][3] b3[3]
// Normalisation (not trained): mu[16] then sigma[16]; x_n = (x - mu) / sigma.
// Every operand of a matrix product is rounded to bfloat16 (round to
// nearest even): the normalised inputs, the weights, the hidden activations
// after GELU, and in the backward pass the logit gradient and both
// pre-activation gradients.  Biases, GELU, its derivative and the softmax
// stay FP32.
//
// Matrix-core tile: v_mfma_f32_16x16x16_bf16 on one wavefront.  Lane l
// supplies A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16], and
// receives D[4 (l / 16) + i][l % 16], i = 0..3.  One wavefront owns a block
// of 16 rows; activations of the block are re-laid out through LDS between
// layers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace fcx {

constexpr int kMlpIn = 16, kMlpHid = 64, kMlpOut = 3;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid, kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid, kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;            // 5443

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return short(u >> 16);
}
__device__ __forceinline__ float bf16_float(short b) {
  return __uint_as_float(uint32_t(uint16_t(b)) << 16);
}

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights in LDS as bfloat16 bits; biases and normalisation FP32.
struct MlpLds {
  short w1[kMlpIn][kMlpHid];
  short w2[kMlpHid][kMlpHid];
  short w3[kMlpHid][16];                    // classes padded to 16
  float b1[kMlpHid], b2[kMlpHid], b3[16];
  float mu[kMlpIn], isg[kMlpIn];
};

__device__ __forceinline__ void mlp_load(MlpLds& L, const float* P,
                                         const float* norm) {
  for (int t = threadIdx.x; t < kMlpIn * kMlpHid; t += blockDim.x)
    L.w1[t / kMlpHid][t % kMlpHid] = bf16_bits(P[kOffW1 + t]);
  for (int t = threadIdx.x; t < kMlpHid * kMlpHid; t += blockDim.x)
    L.w2[t / kMlpHid][t % kMlpHid] = bf16_bits(P[kOffW2 + t]);
  for (int t = threadIdx.x; t < kMlpHid * 16; t += blockDim.x) {
    const int h = t / 16, c = t % 16;
    L.w3[h][c] = c < kMlpOut ? bf16_bits(P[kOffW3 + h * kMlpOut + c]) : short(0);
  }
  for (int t = threadIdx.x; t < kMlpHid; t += blockDim.x) {
    L.b1[t] = P[kOffB1 + t];
    L.b2[t] = P[kOffB2 + t];
  }
  for (int t = threadIdx.x; t < 16; t += blockDim.x) {
    L.b3[t] = t < kMlpOut ? P[kOffB3 + t] : 0.0f;
    L.mu[t] = norm[t];
    L.isg[t] = 1.0f / norm[kMlpIn + t];
  }
}

// Activations of one 16-row block (one wavefront).
struct MlpWave {
  float z1[16][kMlpHid], z2[16][kMlpHid];   // pre-activations
  short h1[16][kMlpHid], h2[16][kMlpHid];   // activations (bf16)
  short x[16][16];                          // normalised inputs (bf16)
  float g[16][16];                          // logits, then their gradient
};

// Forward of rows r0 .. r0 + 15 (rows >= M act as zero inputs and give
// zero activations); logits land in W.g[row][0..2].
__device__ __forceinline__ void mlp_forward_block(const MlpLds& L, MlpWave& W,
                                                  const float* x, int64_t M,
                                                  int64_t r0) {
  const int l = threadIdx.x & 63, lr = l & 15, lg = l >> 4;
  bf16x4 xa;
  for (int i = 0; i < 4; ++i) {
    const int f = 4 * lg + i;
    float v = 0.0f;
    if (r0 + lr < M) v = (x[(r0 + lr) * kMlpIn + f] - L.mu[f]) * L.isg[f];
    xa[i] = bf16_bits(v);
    W.x[lr][f] = xa[i];
  }
  for (int nb = 0; nb < 4; ++nb) {
    bf16x4 b;
    for (int i = 0; i < 4; ++i) b[i] = L.w1[4 * lg + i][16 * nb + lr];
    f32x4 d = {0, 0, 0, 0};
    d = mfma16(xa, b, d);
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * lg + i, col = 16 * nb + lr;
      const float z = d[i] + L.b1[col];
      W.z1[row][col] = z;
      W.h1[row][col] = (r0 + row < M) ? bf16_bits(gelu(z)) : short(0);
    }
  }
  wave_sync();
  for (int nb = 0; nb < 4; ++nb) {
    f32x4 d = {0, 0, 0, 0};
    for (int kb = 0; kb < 4; ++kb) {
      bf16x4 a, b;
      for (int i = 0; i < 4; ++i) {
        a[i] = W.h1[lr][16 * kb + 4 * lg + i];
        b[i] = L.w2[16 * kb + 4 * lg + i][16 * nb + lr];
      }
      d = mfma16(a, b, d);
    }
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * lg + i, col = 16 * nb + lr;
      const float z = d[i] + L.b2[col];
      W.z2[row][col] = z;
      W.h2[row][col] = (r0 + row < M) ? bf16_bits(gelu(z)) : short(0);
    }
  }
  wave_sync();
  f32x4 d = {0, 0, 0, 0};
  for (int kb = 0; kb < 4; ++kb) {
    bf16x4 a, b;
    for (int i = 0; i < 4; ++i) {
      a[i] = W.h2[lr][16 * kb + 4 * lg + i];
      b[i] = L.w3[16 * kb + 4 * lg + i][lr];
    }
    d = mfma16(a, b, d);
  }
  for (int i = 0; i < 4; ++i) W.g[4 * lg + i][lr] = d[i] + L.b3[lr];
  wave_sync();
}

// Inference: 4 wavefronts per workgroup, each striding over 16-row blocks.
__global__ void __launch_bounds__(256)
k_mlp_forward(const float* __restrict__ P, const float* __restrict__ norm,
              const float* __restrict__ x, int64_t M, float* __restrict__ logits) {
  __shared__ MlpLds L;
  __shared__ MlpWave Wv[4];
  mlp_load(L, P, norm);
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t nblk = (M + 15) / 16, nw = int64_t(gridDim.x) * 4;
  for (int64_t blk = int64_t(blockIdx.x) * 4 + w; blk < nblk; blk += nw) {
    const int64_t r0 = blk * 16;
    mlp_forward_block(L, Wv[w], x, M, r0);
    if (l < 48) {
      const int row = l / 3, c = l % 3;
      if (r0 + row < M) logits[(r0 + row) * kMlpOut + c] = Wv[w].g[row][c];
    }
    wave_sync();
  }
}

// Training: forward, weighted softmax cross-entropy
//   loss = scale * sum_r cw[y_r] * (-log softmax(z_r)[y_r]),
// and its gradient.  Weight gradients accumulate over a wavefront's row
// blocks in MFMA accumulators, then per workgroup in LDS, then into
// grad[] with one FP32 atomic per parameter and workgroup.  Rows with a
// label outside 0..2 contribute nothing.  grad and loss must be zero on
// entry.
__global__ void __launch_bounds__(256)
k_mlp_backward(const float* __restrict__ P, const float* __restrict__ norm,
               const float* __restrict__ x, const int32_t* __restrict__ y,
               const float* __restrict__ cw, float scale, int64_t M,
               float* __restrict__ grad, float* __restrict__ loss) {
  __shared__ MlpLds L;
  __shared__ MlpWave Wv[4];
  __shared__ short dz[4][16][kMlpHid];
  __shared__ float red[kMlpParams + 1];
  for (int t = threadIdx.x; t <= kMlpParams; t += blockDim.x) red[t] = 0.0f;
  mlp_load(L, P, norm);
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lg = l >> 4;
  MlpWave& W = Wv[w];
  short (*dzw)[kMlpHid] = dz[w];
  short (*dz1)[kMlpHid] = W.h2;             // H2 is dead once dW3 is formed
  f32x4 acc1[4], acc2[16], acc3[4];
  for (int t = 0; t < 4; ++t) acc1[t] = acc3[t] = f32x4{0, 0, 0, 0};
  for (int t = 0; t < 16; ++t) acc2[t] = f32x4{0, 0, 0, 0};
  float db1 = 0.0f, db2 = 0.0f, db3 = 0.0f, lsum = 0.0f;
  const int64_t nblk = (M + 15) / 16, nw = int64_t(gridDim.x) * 4;
  for (int64_t blk = int64_t(blockIdx.x) * 4 + w; blk < nblk; blk += nw) {
    const int64_t r0 = blk * 16;
    mlp_forward_block(L, W, x, M, r0);
    float gr[3] = {0.0f, 0.0f, 0.0f};
    if (l < 16 && r0 + l < M) {
      const int yy = y[r0 + l];
      if (yy >= 0 && yy < kMlpOut) {
        const float z0 = W.g[l][0], z1 = W.g[l][1], z2 = W.g[l][2];
        const float zm = fmaxf(z0, fmaxf(z1, z2));
        const float e0 = expf(z0 - zm), e1 = expf(z1 - zm), e2 = expf(z2 - zm);
        const float s = e0 + e1 + e2, is = 1.0f / s;
        const float wy = scale * cw[yy];
        const float pr[3] = {e0 * is, e1 * is, e2 * is};
        for (int c = 0; c < 3; ++c) gr[c] = wy * (pr[c] - (c == yy ? 1.0f : 0.0f));
        lsum += wy * (logf(s) + zm - (yy == 0 ? z0 : (yy == 1 ? z1 : z2)));
      }
    }
    wave_sync();
    if (l < 16)
      for (int c = 0; c < 16; ++c)
        W.g[l][c] = c < 3 ? bf16_float(bf16_bits(gr[c])) : 0.0f;
    wave_sync();
    // dW3 += H2^T G ; db3 += column sums of G
    for (int mb = 0; mb < 4; ++mb) {
      bf16x4 a, b;
      for (int i = 0; i < 4; ++i) {
        a[i] = W.h2[4 * lg + i][16 * mb + lr];
        b[i] = bf16_bits(W.g[4 * lg + i][lr]);
      }
      acc3[mb] = mfma16(a, b, acc3[mb]);
    }
    if (l < kMlpOut)
      for (int r = 0; r < 16; ++r) db3 += W.g[r][l];
    // dZ2 = (G W3^T) * gelu'(Z2)
    {
      bf16x4 a;
      for (int i = 0; i < 4; ++i) a[i] = bf16_bits(W.g[lr][4 * lg + i]);
      for (int nb = 0; nb < 4; ++nb) {
        bf16x4 b;
        for (int i = 0; i < 4; ++i) b[i] = L.w3[16 * nb + lr][4 * lg + i];
        f32x4 d = {0, 0, 0, 0};
        d = mfma16(a, b, d);
        for (int i = 0; i < 4; ++i) {
          const int row = 4 * lg + i, col = 16 * nb + lr;
          dzw[row][col] = bf16_bits(d[i] * gelu_d(W.z2[row][col]));
        }
      }
    }
    wave_sync();
    // dW2 += H1^T dZ2 ; db2 += column sums of dZ2
    for (int mb = 0; mb < 4; ++mb)
      for (int nb = 0; nb < 4; ++nb) {
        bf16x4 a, b;
        for (int i = 0; i < 4; ++i) {
          a[i] = W.h1[4 * lg + i][16 * mb + lr];
          b[i] = dzw[4 * lg + i][16 * nb + lr];
        }
        acc2[4 * mb + nb] = mfma16(a, b, acc2[4 * mb + nb]);
      }
    for (int r = 0; r < 16; ++r) db2 += bf16_float(dzw[r][l]);
    // dZ1 = (dZ2 W2^T) * gelu'(Z1)
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 d = {0, 0, 0, 0};
      for (int kb = 0; kb < 4; ++kb) {
        bf16x4 a, b;
        for (int i = 0; i < 4; ++i) {
          a[i] = dzw[lr][16 * kb + 4 * lg + i];
          b[i] = L.w2[16 * nb + lr][16 * kb + 4 * lg + i];
        }
        d = mfma16(a, b, d);
      }
      for (int i = 0; i < 4; ++i) {
        const int row = 4 * lg + i, col = 16 * nb + lr;
        dz1[row][col] = bf16_bits(d[i] * gelu_d(W.z1[row][col]));
      }
    }
    wave_sync();
    // dW1 += X^T dZ1 ; db1 += column sums of dZ1
    for (int nb = 0; nb < 4; ++nb) {
      bf16x4 a, b;
      for (int i = 0; i < 4; ++i) {
        a[i] = W.x[4 * lg + i][lr];
        b[i] = dz1[4 * lg + i][16 * nb + lr];
      }
      acc1[nb] = mfma16(a, b, acc1[nb]);
    }
    for (int r = 0; r < 16; ++r) db1 += bf16_float(dz1[r][l]);
    wave_sync();                            // block done: scratch is free
  }
  // workgroup reduction in LDS, then one global atomic per parameter
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * lg + i;
    for (int nb = 0; nb < 4; ++nb)
      atomicAdd(&red[kOffW1 + row * kMlpHid + 16 * nb + lr], acc1[nb][i]);
    for (int mb = 0; mb < 4; ++mb) {
      for (int nb = 0; nb < 4; ++nb)
        atomicAdd(&red[kOffW2 + (16 * mb + row) * kMlpHid + 16 * nb + lr],
                  acc2[4 * mb + nb][i]);
      if (lr < kMlpOut)
        atomicAdd(&red[kOffW3 + (16 * mb + row) * kMlpOut + lr], acc3[mb][i]);
    }
  }
  atomicAdd(&red[kOffB1 + l], db1);
  atomicAdd(&red[kOffB2 + l], db2);
  if (l < kMlpOut) atomicAdd(&red[kOffB3 + l], db3);
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if (l == 0) atomicAdd(&red[kMlpParams], lsum);
  __syncthreads();
  for (int t = threadIdx.x; t < kMlpParams; t += blockDim.x)
    if (red[t] != 0.0f) atomicAdd(&grad[t], red[t]);
  if (threadIdx.x == 0) atomicAdd(loss, red[kMlpParams]);
}

__global__ void k_zero_f32(float* a, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// Adam (Kingma and Ba 2015, Algorithm 1) with bias correction at step t.
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ g,
                       float* __restrict__ m1, float* __restrict__ m2, int64_t n,
                       int32_t t, float lr, float b1, float b2, float eps) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c1 = 1.0f - powf(b1, float(t)), c2 = 1.0f - powf(b2, float(t));
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  P[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Tags from logits with the criterion as fallback: +1 where the plain tag
// is +1; the plain tag where the largest softmax probability is below
// `conf`; otherwise 1 - argmax (class 0 refine, 1 keep, 2 coarsen; the
// lowest class wins ties).
__global__ void k_learned_tags(const float* __restrict__ z, const int8_t* __restrict__ plain,
                               int64_t M, float conf, int8_t* __restrict__ tags) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= M) return;
  const float z0 = z[3 * r], z1 = z[3 * r + 1], z2 = z[3 * r + 2];
  int best = 0;
  float zb = z0;
  if (z1 > zb) { best = 1; zb = z1; }
  if (z2 > zb) { best = 2; zb = z2; }
  const float pmax = 1.0f / (expf(z0 - zb) + expf(z1 - zb) + expf(z2 - zb));
  const int8_t pt = plain[r];
  tags[r] = (pt == 1 || pmax < conf) ? pt : int8_t(1 - best);
}

// Refinement buffer: a patch below lmax next to (face or corner) a patch
// tagged +1 is tagged +1 too; other tags are copied.
__global__ void k_dilate_tags(const int8_t* __restrict__ in, const PatchRec* __restrict__ rec,
                              int64_t P, int lmax, int8_t* __restrict__ out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int8_t t = in[p];
  if (t != 1 && rec[p].level < lmax)
    for (int s = 0; s < 12; ++s) {
      const int32_t n = rec[p].nbr[s];
      if (n >= 0 && in[n] == 1) t = 1;
    }
  out[p] = t;
}

// Per-patch statistics (one workgroup of 256 per patch, FP64 arithmetic):
// for k < 3 (zero beyond meqn) min, max, mean over the interior and
// log(1 + largest |grad q_k|) by central differences over the ghost-extended
// data; then the level; then zeros.  feats[p * 16 + f], FP32.  (Largest
// gradients span about four decades over a forest; the logarithm keeps those
// near the criterion threshold apart once standardised and rounded to
// bfloat16.)
template <typename R, int MEQN>
__global__ void __launch_bounds__(256)
k_features(const R* __restrict__ q, const R* __restrict__ ghost,
           const PatchRec* __restrict__ rec, int m, float* __restrict__ feats) {
  __shared__ double red[4][4][MEQN];
  const int p = blockIdx.x, tid = threadIdx.x;
  const double dx = ldexp(1.0, -rec[p].level) / m;
  const size_t G = size_t(8 * m + 16);
  double lo[MEQN], hi[MEQN], sum[MEQN], gm[MEQN];
  for (int k = 0; k < MEQN; ++k) { lo[k] = 1e300; hi[k] = -1e300; sum[k] = 0.0; gm[k] = 0.0; }
  auto at = [&](int k, int i, int j) -> double {
    if (i >= 1 && i <= m && j >= 1 && j <= m)
      return double(q[(size_t(p * MEQN + k) * m + (j - 1)) * m + (i - 1)]);
    return double(ghost[size_t(p * MEQN + k) * G + ghost_index(m, i, j)]);
  };
  for (int c = tid; c < m * m; c += 256) {
    const int i = c % m + 1, j = c / m + 1;
    for (int k = 0; k < MEQN; ++k) {
      const double v = at(k, i, j);
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
      sum[k] += v;
      const double gx = (at(k, i + 1, j) - at(k, i - 1, j)) / (2.0 * dx);
      const double gy = (at(k, i, j + 1) - at(k, i, j - 1)) / (2.0 * dx);
      gm[k] = fmax(gm[k], sqrt(gx * gx + gy * gy));
    }
  }
  for (int k = 0; k < MEQN; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fmin(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmax(hi[k], __shfl_xor(hi[k], off));
      sum[k] += __shfl_xor(sum[k], off);
      gm[k] = fmax(gm[k], __shfl_xor(gm[k], off));
    }
  if ((tid & 63) == 0)
    for (int k = 0; k < MEQN; ++k) {
      red[tid >> 6][0][k] = lo[k];
      red[tid >> 6][1][k] = hi[k];
      red[tid >> 6][2][k] = sum[k];
      red[tid >> 6][3][k] = gm[k];
    }
  __syncthreads();
  if (tid < 16) {
    float v = 0.0f;
    const int k = tid / 4, s = tid % 4;
    if (tid == 12) {
      v = float(rec[p].level);
    } else if (k < MEQN && k < 3) {
      double a = red[0][s][k];
      for (int w = 1; w < 4; ++w) {
        const double b = red[w][s][k];
        a = s == 0 ? fmin(a, b) : (s == 2 ? a + b : fmax(a, b));
      }
      v = float(s == 2 ? a / (double(m) * m) : (s == 3 ? log1p(a) : a));
    }
    feats[size_t(p) * 16 + tid] = v;
  }
}

}  // namespace fcx
