// Surrogate network kernels (BF16 matrix cores, FP32 accumulation) and the
// C ABI declared in include/sur.h.
//
// Every product of the network has the form
//     C[r][c] = sum_k X[r][k] * Y[c][k]
// with X and Y row-major BF16 and the reduction index k contiguous:
//   forward      Z = A W^T       X = A  [batch][in],   Y = W   [out][in]
//   data grad    dA = dZ W       X = dZ [batch][out],  Y = W^T [in][out]
//   weight grad  dW = dZ^T A     X = dZ^T [out][batch], Y = A^T [in][batch]
// A training step is 3 launches.  The work local to a batch row (the feature
// layer, the forward products, the loss gradient, the data gradients) runs in
// one kernel per 16-row tile with the activations in LDS (k_train_fb), which
// also writes each activation and gradient transposed for the weight
// gradients.  Those are split over the batch (k_gemm, the three products in
// one launch, one wave per 32 x 32 output tile, operands read as 16-byte vectors straight from global memory,
// a whole group of K steps at a time); bias gradients are column sums per
// 16-row tile; one kernel then reduces every partial sum in a fixed order, so
// every result is deterministic, and takes each parameter's Adam step on the
// FP32 master copy at once, refreshing both W and W^T in BF16.  The first layer is a fixed random
// Fourier-feature map of the two inputs (sin of x W1^T + b1, on the vector
// unit) and is not trained, so no gradient is propagated to it.  Inference
// runs the whole network in one kernel (k_fused).
//
// MFMA 16x16x32 BF16 operand layout (lane l, 64 lanes): A fragment = row
// (l mod 16), k = 8 (l / 16) + 0..7; B fragment = column (l mod 16), same k;
// accumulator element q = row 4 (l / 16) + q, column (l mod 16).
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "../../include/sur.h"
#include "ens_internal.h"

namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kIn = SUR_IN, kH = SUR_HIDDEN, kOut = SUR_OUT;
// packed parameter offsets: W1, b1, W2, b2, W3, b3, W4, b4
constexpr int64_t oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
                  oW3 = ob2 + kH, ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kOut * kH,
                  kNP = ob4 + kOut;
static_assert(kNP == SUR_N_PARAMS, "parameter count");

// Loss weight of output column c: the first output (the largest of the
// recorded maxima, the value the screen labels by) counts kW0 times, the
// others once, normalised to mean 1.
constexpr float kW0 = 32.0f;
__device__ __forceinline__ float out_weight(int c) {
  return (c == 0 ? kW0 : 1.0f) * ((float)kOut / (kW0 + (float)(kOut - 1)));
}

// The network's two nonlinear functions, in the form every kernel uses:
//
// Fourier feature sin(v): the hardware sine (v_sin_f32, which takes its
// argument in turns) of the fractional part of v / (2 pi).  Rounding v / (2 pi)
// to FP32 moves the angle by at most |v| 2^-24 (under 1e-5 for the |v| < 200
// the features reach), the size of the rounding of v itself, and far below
// the BF16 unit (2^-8) the feature is rounded to.
__device__ __forceinline__ float feature_sin(float v) {
  return __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(v * 0.15915494309189534f));
}

// GELU(z) = z Phi(z), Phi the standard normal CDF.  The tail
// T(z) = Phi(-|z|) = erfc(|z| / sqrt 2) / 2 comes from the rational-times-
// Gaussian approximation of Abramowitz and Stegun (eq. 7.1.26, after
// Hastings; |error in erfc| <= 1.5e-7):
//   erfc(u) ~ t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-u^2),
//   t = 1 / (1 + p u),
// evaluated with u' = u sqrt(log2 e) so that exp(-u^2) = 2^(-u'^2) (p scaled
// to match, the a_i halved).  Then GELU(z) = max(z, 0) - |z| T(z), which
// holds for either sign and forms the small negative tail without the
// cancellation of 1 + erf.  Branch-free: one reciprocal, one exp2.
constexpr float kTailU = 0.84932180028801907f;   // sqrt(log2 e / 2)
constexpr float kTailP = 0.27273748f;            // 0.3275911 / sqrt(log2 e)
constexpr float kTailA1 = 0.127414796f, kTailA2 = -0.142248368f, kTailA3 = 0.7107068705f,
                kTailA4 = -0.7265760135f, kTailA5 = 0.5307027145f;
__device__ __forceinline__ float normal_tail(float z, float *gauss = nullptr) {
  const float u = fabsf(z) * kTailU;
  const float t = __builtin_amdgcn_rcpf(fmaf(kTailP, u, 1.0f));
  float p = fmaf(t, kTailA5, kTailA4);
  p = fmaf(t, p, kTailA3);
  p = fmaf(t, p, kTailA2);
  p = fmaf(t, p, kTailA1);
  const float e = __builtin_amdgcn_exp2f(-(u * u));   // exp(-z^2 / 2)
  if (gauss) *gauss = e;
  return (t * p) * e;
}
__device__ __forceinline__ float gelu_f(float z) {
  return fmaf(-fabsf(z), normal_tail(z), fmaxf(z, 0.0f));
}
// d GELU / dz = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad_f(float z) {
  float e;
  const float tail = normal_tail(z, &e);
  const float cdf = z < 0.0f ? tail : 1.0f - tail;
  return fmaf(z, e * 0.39894228040143268f, cdf);
}

// ---------------------------------------------------------------- GEMM tile
// Weight-gradient products: C = sum_k X[r][k] Y[c][k] over one share of the
// batch (k), written as a partial sum.
struct GemmArgs {
  const bf16 *X;
  int64_t ldx;
  const bf16 *Y;
  int64_t ldy;
  int64_t R, C, K;       // C[R][C], reduction length K (split over gridDim.z)
  float *out_f32;        // [split][R][C] partial sums
};

constexpr int kTile = 32;  // output tile edge per wave

// Up to three products in one launch (a training step's weight gradients),
// each split over its K range in `split` equal parts.
struct GemmBatch {
  GemmArgs g[3];
  int64_t nblk[3];  // blocks of each product: (R/32) (C/32) split
  int split;
};

// One wave per 32 x 32 output tile (2 x 2 accumulators).  The blocks of the
// products follow each other; within one, the tile row runs fastest, then
// the tile column, then the K part, so consecutive blocks share the rows of
// X, and blocks are spread over the XCDs by block index, so each XCD reads
// its own share of X.  The K range is taken KG MFMA steps (32 each) at a
// time: all operand loads of a group are issued before its products, so one
// memory latency covers KG steps.
template <int KG>
__global__ __launch_bounds__(64) void k_gemm(GemmBatch bt) {
  int64_t bid = blockIdx.x;
  const int p = bid < bt.nblk[0] ? 0 : (bid < bt.nblk[0] + bt.nblk[1] ? 1 : 2);
  bid -= p == 0 ? 0 : (p == 1 ? bt.nblk[0] : bt.nblk[0] + bt.nblk[1]);
  const GemmArgs g = p == 0 ? bt.g[0] : (p == 1 ? bt.g[1] : bt.g[2]);
  const int64_t tr = g.R / kTile, tc = g.C / kTile;
  const int64_t bx = bid % tr, by = (bid / tr) % tc, bz = bid / (tr * tc);
  const int64_t r0 = bx * kTile, c0 = by * kTile;
  const int64_t kchunk = g.K / bt.split;
  const int64_t kb = bz * kchunk, ke = kb + kchunk;
  const int l = threadIdx.x & 63;
  const int64_t lr = l & 15, lk = (l >> 4) * 8;
  const int64_t lc = l & 15, lrow = (l >> 4) * 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16 *xp = g.X + (r0 + lr) * g.ldx + lk;
  const bf16 *yp = g.Y + (c0 + lr) * g.ldy + lk;
  for (int64_t k = kb; k < ke; k += 32 * KG) {
    bf16x8 a[KG][2], b[KG][2];
#pragma unroll
    for (int u = 0; u < KG; ++u) {
#pragma unroll
      for (int i = 0; i < 2; ++i) a[u][i] = *(const bf16x8 *)(xp + 16 * i * g.ldx + k + 32 * u);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[u][j] = *(const bf16x8 *)(yp + 16 * j * g.ldy + k + 32 * u);
    }
    // keep the whole group of loads ahead of the products
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < KG; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], b[u][j], acc[i][j], 0, 0, 0);
  }
  float *o = g.out_f32 + bz * g.R * g.C;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t c = c0 + 16 * j + lc;
      const int64_t rb = r0 + 16 * i + lrow;
#pragma unroll
      for (int q = 0; q < 4; ++q) o[(rb + q) * g.C + c] = acc[i][j][q];
    }
}

// ------------------------------------------------ fused training tile
// One training step's work that is local to a row of the batch, for a tile
// of 16 rows per block of 4 waves (a batch of 4096 rows fills every CU): the feature layer, the forward products
// of layers 2 to 4, the loss gradient of the output layer, and the data
// gradients back through layers 3 and 2.  The activations and gradients
// that feed the next product stay in LDS (two BF16 row-major tiles, rows
// padded to 264 so that the 16 rows of an operand fragment fall on
// different banks), and each product's weight operands are loaded into
// registers a layer ahead; each wave computes 64 output features of a 256-wide
// layer (4 accumulators), so it already holds, in the accumulator
// layout, the GELU derivatives of exactly the positions whose data gradient
// it forms on the way back.  What leaves the block is what the
// weight-gradient products and the reduction need: the activations and
// gradients transposed ([feature][batch row], BF16), the column sums of each
// gradient over the tile (bias gradients), and the tile's weighted squared
// error.  Activations and gradients are rounded to BF16 where they become
// operands; every product accumulates in FP32, its MFMA steps in increasing
// k.
constexpr int kTileLd = kH + 8;
constexpr int kTR = 16, kNI = kTR / 16;  // rows per tile, 16-row groups

struct TrainArgs {
  const float *x;          // inputs [*][2]: batch row r is dataset row rows[r] (or r)
  const int64_t *rows;     // dataset rows of the batch, or NULL
  const float *tgt;        // targets [*][64], indexed like x
  const float *P;          // FP32 parameters (W1, b1 .. b4 read here)
  const bf16 *W2, *W3, *W4;  // BF16 weights [out][in]
  const bf16 *W3T, *W4T;     // BF16 transposes [in][out]
  int64_t m;               // batch rows (a multiple of 16)
  bf16 *a1T, *a2T, *a3T;   // [256][m]
  bf16 *dz4T;              // [64][m]
  bf16 *dz3T, *dz2T;       // [256][m]
  float *cp4, *cp3, *cp2;  // [m/16][64], [m/16][256], [m/16][256]
  float *lpart;            // [m/16]
};

// The B operands of a tile product: weight rows c0 + 16 j + (l mod 16),
// k = 32 s + 8 (l / 16) + 0..7 for every MFMA step s of K, from the row-major
// weights (ld ldw).  Loaded a whole layer ahead: the weights do not depend on
// the activations, so a layer's loads are issued before the previous layer's
// epilogue and barrier, which hides their latency at one wave per SIMD.
template <int NJ, int K>
__device__ __forceinline__ void tile_weights(const bf16 *__restrict__ W, int64_t ldw, int c0,
                                             int l, bf16x8 (&b)[K / 32][NJ]) {
  const bf16 *wp = W + (int64_t)(c0 + (l & 15)) * ldw + (l >> 4) * 8;
#pragma unroll
  for (int s = 0; s < K / 32; ++s)
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[s][j] = *(const bf16x8 *)(wp + 16 * j * ldw + 32 * s);
}

// acc[i][j] = the tile's rows 16 i .. 16 i + 15 times the weight rows of
// b[.][j] over k = 0 .. K, the A operands from the LDS tile, the MFMA steps
// in increasing k.
template <int NJ, int K>
__device__ __forceinline__ void tile_product(const bf16 (*in)[kTileLd],
                                             const bf16x8 (&b)[K / 32][NJ], int l,
                                             f32x4 (&acc)[kNI][NJ]) {
  const int lr = l & 15, lk = (l >> 4) * 8;
#pragma unroll
  for (int i = 0; i < kNI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < K / 32; ++s) {
    bf16x8 a[kNI];
#pragma unroll
    for (int i = 0; i < kNI; ++i) a[i] = *(const bf16x8 *)&in[16 * i + lr][32 * s + lk];
#pragma unroll
    for (int i = 0; i < kNI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[s][j], acc[i][j], 0, 0, 0);
  }
}

// Column sums over the tile's rows of v (the accumulator layout: lane l
// holds rows 16 i + 4 (l / 16) + q of column l mod 16): the lane's rows,
// then the 4 lane groups, in a fixed order; lanes 0 .. 15 hold the sums.
__device__ __forceinline__ float tile_colsum(const float (&v)[kNI][4]) {
  float s0 = 0.f;
#pragma unroll
  for (int i = 0; i < kNI; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) s0 += v[i][q];
  s0 += __shfl_xor(s0, 16);
  s0 += __shfl_xor(s0, 32);
  return s0;
}

__global__ __launch_bounds__(256) void k_train_fb(TrainArgs g) {
  __shared__ bf16 act[2][kTR][kTileLd];
  __shared__ float xs[kTR][2];
  __shared__ float lw[4];
  const int64_t m = g.m, r0 = (int64_t)blockIdx.x * kTR;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int lc = l & 15, lrow = (l >> 4) * 4;
  bf16x8 bw[kH / 32][4];    // the next 256-wide product's weights
  tile_weights<4, kH>(g.W2, kH, 64 * w, l, bw);
  // biases and targets of the lane's output positions, loaded ahead
  float b23[2][4], tq[kNI][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    b23[0][j] = g.P[ob2 + 64 * w + 16 * j + lc];
    b23[1][j] = g.P[ob3 + 64 * w + 16 * j + lc];
  }
  const float b4c = g.P[ob4 + 16 * w + lc];
#pragma unroll
  for (int i = 0; i < kNI; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t rr = r0 + 16 * i + lrow + q;
      tq[i][q] = g.tgt[(g.rows ? g.rows[rr] : rr) * kOut + 16 * w + lc];
    }
  if (t < kTR) {
    const int64_t src = g.rows ? g.rows[r0 + t] : r0 + t;
    xs[t][0] = g.x[2 * src];
    xs[t][1] = g.x[2 * src + 1];
  }
  __syncthreads();
  // layer 1: thread t is feature t of the tile's rows
  {
    const float w0 = g.P[oW1 + 2 * t], w1 = g.P[oW1 + 2 * t + 1], bb = g.P[ob1 + t];
    bf16x8 col[kTR / 8];
#pragma unroll
    for (int k = 0; k < kTR; ++k) {
      const bf16 f = (bf16)feature_sin(fmaf(xs[k][1], w1, fmaf(xs[k][0], w0, bb)));
      act[0][k][t] = f;
      col[k >> 3][k & 7] = f;
    }
#pragma unroll
    for (int q = 0; q < kTR / 8; ++q) *(bf16x8 *)(g.a1T + (int64_t)t * m + r0 + 8 * q) = col[q];
  }
  __syncthreads();
  // layers 2 and 3: z = a W^T + b, a' = GELU(z); keep GELU'(z) for the way back
  float gp[2][kNI][4][4];  // [layer 2, 3][i][j][q]
  f32x4 acc[kNI][4];
  bf16x8 bw4[kH / 32][1];   // layer 4's weights
#pragma unroll
  for (int L = 0; L < 2; ++L) {
    bf16 *aT = L == 0 ? g.a2T : g.a3T;
    tile_product<4, kH>(act[L], bw, l, acc);
    if (L == 0)
      tile_weights<4, kH>(g.W3, kH, 64 * w, l, bw);
    else
      tile_weights<1, kH>(g.W4, kH, 16 * w, l, bw4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 64 * w + 16 * j + lc;
      const float bj = b23[L][j];
#pragma unroll
      for (int i = 0; i < kNI; ++i) {
        bf16x4 col;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float z = acc[i][j][q] + bj;
          gp[L][i][j][q] = gelu_grad_f(z);
          const bf16 a = (bf16)gelu_f(z);
          act[1 - L][16 * i + lrow + q][c] = a;
          col[q] = a;
        }
        *(bf16x4 *)(aT + (int64_t)c * m + r0 + 16 * i + lrow) = col;
      }
    }
    __syncthreads();
  }
  // layer 4 and the loss gradient 2 w_c (out - t) / (m * 64); wave w takes
  // the output columns 16 w .. 16 w + 15
  bf16x8 bwt[kOut / 32][4];  // W4^T for the first product back
  {
    f32x4 acc4[kNI][1];
    tile_product<1, kH>(act[0], bw4, l, acc4);
    tile_weights<4, kOut>(g.W4T, kOut, 64 * w, l, bwt);
    const int c = 16 * w + lc;
    const float bj = b4c;
    const float wc = out_weight(c);
    const float scale = 2.0f * wc / (float)(m * kOut);
    float gv[kNI][4];
    float sq = 0.f;
#pragma unroll
    for (int i = 0; i < kNI; ++i) {
      bf16x4 col;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = 16 * i + lrow + q;
        const float d = (acc4[i][0][q] + bj) - tq[i][q];
        sq = fmaf(wc * d, d, sq);
        gv[i][q] = scale * d;
        const bf16 gb = (bf16)gv[i][q];
        act[1][rr][c] = gb;
        col[q] = gb;
      }
      *(bf16x4 *)(g.dz4T + (int64_t)c * m + r0 + 16 * i + lrow) = col;
    }
    const float cs = tile_colsum(gv);
    if (l < 16) g.cp4[(int64_t)blockIdx.x * kOut + c] = cs;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (l == 0) lw[w] = sq;
  }
  __syncthreads();
  if (t == 0) g.lpart[blockIdx.x] = ((lw[0] + lw[1]) + lw[2]) + lw[3];
  // back through layer 3 (dA3 = dZ4 W4, K = 64), then layer 2 (dA2 = dZ3 W3)
#pragma unroll
  for (int L = 1; L >= 0; --L) {
    if (L == 1) {
      tile_product<4, kOut>(act[1], bwt, l, acc);
      tile_weights<4, kH>(g.W3T, kH, 64 * w, l, bw);
    } else {
      tile_product<4, kH>(act[0], bw, l, acc);
    }
    bf16 *dT = L == 1 ? g.dz3T : g.dz2T;
    float *cp = L == 1 ? g.cp3 : g.cp2;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 64 * w + 16 * j + lc;
      float dz[kNI][4];
#pragma unroll
      for (int i = 0; i < kNI; ++i) {
        bf16x4 col;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dz[i][q] = acc[i][j][q] * gp[L][i][j][q];
          const bf16 gb = (bf16)dz[i][q];
          if (L == 1) act[0][16 * i + lrow + q][c] = gb;
          col[q] = gb;
        }
        *(bf16x4 *)(dT + (int64_t)c * m + r0 + 16 * i + lrow) = col;
      }
      const float cs = tile_colsum(dz);
      if (l < 16) cp[(int64_t)blockIdx.x * kH + c] = cs;
    }
    if (L == 1) __syncthreads();
  }
}

// ---------------------------------------------------------------- small kernels
// Gradients of all parameters from the partial sums of one batch of m rows
// (T = m / 16 row tiles, S weight-gradient splits), each summed in a fixed
// order, and the batch loss; acc (optional) accumulates the loss.
struct GradParts {
  const float *w2, *w3;           // [S][256][256]
  const float *b2, *b3;           // [T][256]
  const float *w4;                // [S][64][256]
  const float *b4;                // [T][64]
  const float *lpart;             // [T]
};
constexpr int64_t kNW = 2 * kH * kH + kOut * kH;   // weights of the MFMA layers
constexpr int kNColSums = 5 * kH + kOut + 1;        // W1 (2 x 256), b1..b4, loss
constexpr int kReduceWBlocks = (int)((kNW + 255) / 256);
// Adam on the FP32 master parameters (Kingma and Ba, 2015); the BF16 copies
// of W2, W3, W4 and their transposes follow the updated values.  The step
// count is t = t_base + step + 1; with hyper != NULL the learning rate,
// betas, epsilon and t_base are read from device memory (hyper[0..4]), so a
// captured epoch replays with new values.
struct AdamArgs {
  float *P, *Mm, *V;
  const double *hyper;
  double lr, b1, b2, eps, t_base;
  int step;
  bf16 *W2, *W2T, *W3, *W3T, *W4, *W4T;
};

// The block's hyper-parameters and bias corrections (two FP64 powers, in
// thread 0): h = lr, b1, b2, eps, 1 / (1 - b1^t), 1 / (1 - b2^t).
__device__ __forceinline__ void adam_setup(const AdamArgs &a, float *h) {
  if (threadIdx.x == 0) {
    double lr = a.lr, b1 = a.b1, b2 = a.b2, eps = a.eps, t0 = a.t_base;
    if (a.hyper) {
      lr = a.hyper[0];
      b1 = a.hyper[1];
      b2 = a.hyper[2];
      eps = a.hyper[3];
      t0 = a.hyper[4];
    }
    const double t = t0 + (double)a.step + 1.0;
    h[0] = (float)lr;
    h[1] = (float)b1;
    h[2] = (float)b2;
    h[3] = (float)eps;
    h[4] = (float)(1.0 / (1.0 - pow(b1, t)));
    h[5] = (float)(1.0 / (1.0 - pow(b2, t)));
  }
  __syncthreads();
}

// One parameter i (a trained one: W2 onwards) with gradient gr.
__device__ __forceinline__ void adam_one(const AdamArgs &a, const float *h, int64_t i, float gr) {
  const float lr = h[0], b1 = h[1], b2 = h[2], eps = h[3], c1 = h[4], c2 = h[5];
  const float m = fmaf(b1, a.Mm[i], (1.0f - b1) * gr);
  const float v = fmaf(b2, a.V[i], (1.0f - b2) * gr * gr);
  a.Mm[i] = m;
  a.V[i] = v;
  const float w = a.P[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
  a.P[i] = w;
  const bf16 wb = (bf16)w;
  if (i >= oW2 && i < ob2) {
    const int64_t k = i - oW2, o = k / kH, in = k % kH;
    a.W2[k] = wb;
    a.W2T[in * kH + o] = wb;
  } else if (i >= oW3 && i < ob3) {
    const int64_t k = i - oW3, o = k / kH, in = k % kH;
    a.W3[k] = wb;
    a.W3T[in * kH + o] = wb;
  } else if (i >= oW4 && i < ob4) {
    const int64_t k = i - oW4, o = k / kH, in = k % kH;
    a.W4[k] = wb;
    a.W4T[in * kOut + o] = wb;
  }
}

// Blocks [0, kReduceWBlocks): one weight per thread (S partials).  The
// following blocks: one wave per tile-summed entry (T partials: lane l takes
// tiles l, l + 64, ..., then a butterfly over the wave).  ADAM: each summed
// gradient also takes its Adam step at once (the feature layer's entries,
// whose gradient is 0, and the loss excepted).
template <bool ADAM>
__global__ __launch_bounds__(256) void k_reduce_grads(GradParts p, int64_t T, int S,
                                                      float count, float *G, float *loss,
                                                      float *acc, int first, AdamArgs ad) {
  __shared__ float h[6];
  if (ADAM) adam_setup(ad, h);
  if ((int)blockIdx.x < kReduceWBlocks) {
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= kNW) return;
    const float *src;
    int64_t o, stride;
    if (w < kH * kH) {
      src = p.w2 + w; o = oW2 + w; stride = kH * kH;
    } else if (w < 2 * kH * kH) {
      src = p.w3 + (w - kH * kH); o = oW3 + (w - kH * kH); stride = kH * kH;
    } else {
      src = p.w4 + (w - 2 * kH * kH); o = oW4 + (w - 2 * kH * kH); stride = kOut * kH;
    }
    float g = 0.f;
    for (int k = 0; k < S; ++k) g += src[k * stride];
    G[o] = g;
    if (ADAM) adam_one(ad, h, o, g);
    return;
  }
  const int e = ((int)blockIdx.x - kReduceWBlocks) * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (e >= kNColSums) return;
  const float *src;
  int64_t ld;
  float *dst;
  if (e < kH) {          // the fixed feature layer: no partial sums, gradient 0
    src = nullptr; ld = 0; dst = G + oW1 + 2 * e;
  } else if (e < 2 * kH) {
    src = nullptr; ld = 0; dst = G + oW1 + 2 * (e - kH) + 1;
  } else if (e < 3 * kH) {
    src = nullptr; ld = 0; dst = G + ob1 + (e - 2 * kH);
  } else if (e < 4 * kH) {
    src = p.b2 + (e - 3 * kH); ld = kH; dst = G + ob2 + (e - 3 * kH);
  } else if (e < 5 * kH) {
    src = p.b3 + (e - 4 * kH); ld = kH; dst = G + ob3 + (e - 4 * kH);
  } else if (e < 5 * kH + kOut) {
    src = p.b4 + (e - 5 * kH); ld = kOut; dst = G + ob4 + (e - 5 * kH);
  } else {
    src = p.lpart; ld = 1; dst = nullptr;
  }
  float v = 0.f;
  if (src)
    for (int64_t t = l; t < T; t += 64) v += src[t * ld];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (l == 0) {
    if (dst) {
      *dst = v;
      if (ADAM && src) adam_one(ad, h, dst - G, v);
    } else {
      const float lv = v / count;
      *loss = lv;
      if (acc) *acc = first ? lv : *acc + lv;
    }
  }
}

// BF16 copies of W2, W3, W4 and their transposes from the master weights.
__global__ void k_refresh(const float *__restrict__ P, bf16 *W2, bf16 *W2T, bf16 *W3, bf16 *W3T,
                          bf16 *W4, bf16 *W4T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kH * kH) {
    const int64_t o = i / kH, in = i % kH;
    const bf16 a = (bf16)P[oW2 + i], b = (bf16)P[oW3 + i];
    W2[i] = a;
    W2T[in * kH + o] = a;
    W3[i] = b;
    W3T[in * kH + o] = b;
  }
  if (i < kOut * kH) {
    const int64_t o = i / kH, in = i % kH;
    const bf16 c = (bf16)P[oW4 + i];
    W4[i] = c;
    W4T[in * kOut + o] = c;
  }
}

// Sweep inputs -> normalised network inputs: (p_A, ln f) mapped to [-1, 1]
// (k_fused<true> normalises its inputs the same way).
__global__ void k_inputs(const double *__restrict__ prm, int64_t n, double lo0, double sc0,
                         double lo1, double sc1, float *x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  x[2 * r] = (float)(fma(prm[r] - lo0, sc0, -1.0));
  x[2 * r + 1] = (float)(fma(log(prm[n + r]) - lo1, sc1, -1.0));
}

// The recorded maxima of each point in decreasing order: one wave per point,
// lane j holding rec[j][i], sorted across the lanes by a bitonic network
// (the first output then is the point's largest maximum; the order does not
// depend on the phase of a periodic or chaotic response within the window).
__global__ __launch_bounds__(256) void k_sort_desc(const double *__restrict__ rec, int64_t n,
                                                   double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (i >= n) return;   // the whole wave shares i
  double v = rec[(int64_t)l * n + i];
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const double o = __shfl_xor(v, j);
      const bool keep_max = ((l & k) == 0) == ((l & j) == 0);
      v = keep_max ? fmax(v, o) : fmin(v, o);
    }
  }
  out[(int64_t)l * n + i] = v;
}

// Standardised targets: y[i][j] = (ln rec[j][i] - mean_j) / std_j.
__global__ void k_targets(const double *__restrict__ rec, int64_t n, const double *mean,
                          const double *stdv, float *y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * kOut) return;
  const int64_t i = idx / kOut, j = idx % kOut;
  y[idx] = (float)((log(rec[j * n + i]) - mean[j]) / stdv[j]);
}

// ---------------------------------------------------------------- fused inference
// The whole network for 32 points per wave in one kernel.  The products are
// taken transposed, Z^T = W A^T (MFMA rows = output features, columns =
// points), so the accumulator of feature block fb and point block j holds, in
// lane 16 g + i, features 16 fb + 4 g + q of point 16 j + i.  Packed pairwise
// ((fb, fb + 1) = (2c, 2c + 1)) these are already the B fragments of the next
// layer's k chunk c, in the permuted k order
//     k slot 8 g + s  <->  feature 32 c + 16 (s / 4) + 4 g + s mod 4,
// so the weights of layers 3 and 4 are read with their columns permuted the
// same way; the feature layer's fragments are formed directly in the standard
// order.  Weights come from L2 (288 KB in all) in fragment order (k_frag_layout),
// each fragment serving both point blocks; between layers the activations wait
// in the wave's slice of LDS.  The arithmetic of every element is the training
// path's (same features, GELU and roundings to BF16) except for the order of
// the FP32 sums: the bias starts the accumulation here, and the k order inside
// an MFMA differs for layers 3 and 4.

// The weights of one layer in fragment order, so that each wave load of an A
// fragment is 1 KB contiguous: Wf[((fb * 8 + c) * 64 + lane) * 8 + s] holds
// W[16 fb + lane mod 16][k], k = 32 c + 8 g + s in the standard order, or
// k = 32 c + 16 (s / 4) + 4 g + s mod 4 in the permuted one (g = lane / 16).
__global__ void k_frag_layout(const bf16 *__restrict__ W, int64_t rows, int permuted,
                              bf16 *__restrict__ Wf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * kH) return;
  const int s = (int)(e & 7), lane = (int)(e >> 3) & 63;
  const int64_t c = (e >> 9) & 7, fb = e >> 12;
  const int g = lane >> 4;
  const int64_t k = permuted ? 32 * c + 16 * (s >> 2) + 4 * g + (s & 3) : 32 * c + 8 * g + s;
  Wf[e] = W[(16 * fb + (lane & 15)) * kH + k];
}

struct FusedArgs {
  int64_t n;                       // points
  const double *prm;               // screen: sweep parameters [2][n] (p_A, f)
  double lo0, sc0, lo1, sc1;       //   and their normalisation
  const float *x;                  // forward: normalised inputs [n][2]
  float *out;                      // forward: network outputs [n][64]
  const float *P;                  // master parameters (W1, b1, b2, b3, b4)
  const bf16 *W2f, *W3f, *W4f;     // BF16 weights in fragment order (k_frag_layout;
                                   // 3 and 4 k-permuted)
  // screen epilogue (k_screen_epi's rule)
  const float *mean, *stdv;
  float margin, spread, flag_margin, label_margin;
  const int8_t *nlab;
  int GL;
  int8_t *label;
  uint8_t *resolve;
  float *pmax;
};

// One hidden layer, Z^T = W A^T, for the wave's 32 points: the input's B
// fragments in[c][j] (k chunk c, point block j) in registers, W's rows read in
// the permuted k order of the fragments (or the standard one for the feature
// layer).  Output feature blocks are taken in pairs (2c', 2c' + 1), each pair
// accumulated over the 8 k chunks (4 independent accumulators, starting from
// the bias) and at once turned into the next layer's chunk c' (GELU, BF16),
// which goes to the wave's slice of LDS, out[c'][j][lane].  A pair's 16
// weight fragments are loaded while the previous pair is computed (two
// register buffers), so one L2 latency is exposed per layer rather than per
// MFMA group.  The loop over pairs stays rolled (by two): the kernel is a few
// thousand instructions, which the waves of a CU share in the instruction
// cache.
// Wp: the pair's first fragment for this lane, fragments (fb, c) 8 KB x
// (fb - 2 cp) + 1 KB x c apart.
__device__ __forceinline__ void load_pair(const bf16 *__restrict__ Wp,
                                          const float *__restrict__ bp, bf16x8 (&w)[8][2],
                                          f32x4 (&bb)[2]) {
  // the bias first: the products wait for loads in issue order
  bb[0] = *(const f32x4 *)bp;
  bb[1] = *(const f32x4 *)(bp + 16);
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int h = 0; h < 2; ++h) w[c][h] = *(const bf16x8 *)(Wp + (h * 8 + c) * 512);
}

__device__ __forceinline__ void pair_out(const bf16x8 (&w)[8][2], const f32x4 (&bb)[2],
                                         const bf16x8 (&in)[8][2], int l, bf16x8 *out) {
  f32x4 acc[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[h][j] = bb[h];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[h][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[c][h], in[c][j], acc[h][j], 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    bf16x8 v;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[4 * h + q] = (bf16)gelu_f(acc[h][j][q]);
    out[j * 64 + l] = v;
  }
}

__device__ __forceinline__ void hidden_layer(const bf16 *__restrict__ W,
                                             const float *__restrict__ b, int g, int l,
                                             const bf16x8 (&in)[8][2], bf16x8 *out) {
  const bf16 *W0 = W + l * 8;
  const float *b0 = b + 4 * g;
  bf16x8 wa[8][2], wb[8][2];
  f32x4 ba[2], bb[2];
  load_pair(W0, b0, wa, ba);
#pragma unroll 1
  for (int cp = 0; cp < 8; cp += 2) {
    load_pair(W0 + (cp + 1) * 8192, b0 + 32 * (cp + 1), wb, bb);
    __builtin_amdgcn_sched_barrier(0);
    pair_out(wa, ba, in, l, out + 2 * cp * 64);
    // the last round reloads pair 0 (a harmless L2 hit) rather than branch
    load_pair(W0 + ((cp + 2) & 7) * 8192, b0 + 32 * ((cp + 2) & 7), wa, ba);
    __builtin_amdgcn_sched_barrier(0);
    pair_out(wb, bb, in, l, out + 2 * (cp + 1) * 64);
  }
}

__device__ __forceinline__ void load_act(const bf16x8 *act, int l, bf16x8 (&in)[8][2]) {
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int j = 0; j < 2; ++j) in[c][j] = act[(2 * c + j) * 64 + l];
}

template <bool SCREEN>
__global__ __launch_bounds__(256, 2) void k_fused(FusedArgs a) {
  // each wave's activations between layers: [chunk][point block][lane]
  __shared__ bf16x8 lds[4][8 * 2 * 64];
  const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
  if (r0 >= a.n) return;   // the whole wave
  bf16x8 *act = lds[threadIdx.x >> 6];
  const float *__restrict__ P = a.P;
  float x0[2], x1[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t r = r0 + 16 * j + i;
    x0[j] = x1[j] = 0.f;
    if (r < a.n) {
      if (SCREEN) {
        x0[j] = (float)(fma(a.prm[r] - a.lo0, a.sc0, -1.0));
        x1[j] = (float)(fma(log(a.prm[a.n + r]) - a.lo1, a.sc1, -1.0));
      } else {
        x0[j] = a.x[2 * r];
        x1[j] = a.x[2 * r + 1];
      }
    }
  }
  // the Fourier features, in the standard k order: chunk c, slot 8 g + s
  bf16x8 fa[8][2];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int f = 32 * c + 8 * g + s;
      const float w0 = P[oW1 + 2 * f], w1 = P[oW1 + 2 * f + 1], bb = P[ob1 + f];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        fa[c][j][s] = (bf16)feature_sin(fmaf(x1[j], w1, fmaf(x0[j], w0, bb)));
    }
  hidden_layer(a.W2f, P + ob2, g, l, fa, act);    // layer 2
  load_act(act, l, fa);
  hidden_layer(a.W3f, P + ob3, g, l, fa, act);    // layer 3
  load_act(act, l, fa);
  // output layer
  f32x4 o4[4][2];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const f32x4 bb = *(const f32x4 *)(P + ob4 + 16 * ob + 4 * g);
#pragma unroll
    for (int j = 0; j < 2; ++j) o4[ob][j] = bb;
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      const bf16x8 w = *(const bf16x8 *)(a.W4f + ((ob * 8 + c) * 64 + l) * 8);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        o4[ob][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, fa[c][j], o4[ob][j], 0, 0, 0);
    }
  if (!SCREEN) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t r = r0 + 16 * j + i;
      if (r < a.n)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) *(f32x4 *)(a.out + r * kOut + 16 * ob + 4 * g) = o4[ob][j];
    }
    return;
  }
  // de-standardised maximum and minimum over the 64 outputs of each point:
  // 16 in the lane, then across the four lane groups
  float mx[2], mn[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    mx[j] = -INFINITY;
    mn[j] = INFINITY;
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    const f32x4 sd = *(const f32x4 *)(a.stdv + 16 * ob + 4 * g);
    const f32x4 mu = *(const f32x4 *)(a.mean + 16 * ob + 4 * g);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float v = fmaf(o4[ob][j][q], sd[q], mu[q]);
        mx[j] = fmaxf(mx[j], v);
        mn[j] = fminf(mn[j], v);
      }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      mx[j] = fmaxf(mx[j], __shfl_xor(mx[j], off));
      mn[j] = fminf(mn[j], __shfl_xor(mn[j], off));
    }
  // lane group j (j < 2) finishes point 16 j + i
  if (g >= 2) return;
  const int64_t r = r0 + 16 * g + i;
  if (r >= a.n) return;
  const float xmx = g ? mx[1] : mx[0], xmn = g ? mn[1] : mn[0];
  const float u0f = g ? x0[1] : x0[0], v0f = g ? x1[1] : x1[0];
  const float ln2 = 0.69314718055994531f;
  const float d = fabsf(xmx - ln2);
  const bool unsure = d < a.margin;
  bool flag = (xmx - xmn > a.spread) && d < a.flag_margin;
  const int8_t lab = xmx >= ln2 ? 1 : 0;
  if (a.nlab) {
    const int GL = a.GL;
    const float u = (u0f + 1.0f) * 0.5f * (float)(GL - 1);
    const float v = (v0f + 1.0f) * 0.5f * (float)(GL - 1);
    int u0 = (int)floorf(u), v0 = (int)floorf(v);
    u0 = u0 < 0 ? 0 : (u0 > GL - 2 ? GL - 2 : u0);
    v0 = v0 < 0 ? 0 : (v0 > GL - 2 ? GL - 2 : v0);
    const int64_t b = (int64_t)u0 * GL + v0;
    const int k = (a.nlab[b] != lab) + (a.nlab[b + 1] != lab) + (a.nlab[b + GL] != lab) +
                  (a.nlab[b + GL + 1] != lab);
    flag = flag || k == 4 || (k > 0 && d < a.label_margin);
  }
  if (a.label) a.label[r] = lab;
  if (a.resolve) a.resolve[r] = (unsure || flag) ? 1 : 0;
  if (a.pmax) a.pmax[r] = xmx;
}

// Exact label of each training node: [max_j rec[j][i] >= 2], -1 if a record
// is NaN.
__global__ void k_node_label(const double *__restrict__ rec, int64_t n, int8_t *lab) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double mx = -INFINITY;
  bool bad = false;
  for (int j = 0; j < kOut; ++j) {
    const double v = rec[j * n + i];
    bad = bad || isnan(v);
    mx = v > mx ? v : mx;
  }
  lab[i] = bad ? -1 : (mx >= 2.0 ? 1 : 0);
}

// Deterministic compaction of the re-solve mask: block counts, one-block
// exclusive scan, ordered write.
constexpr int kScanBlock = 1024;
__global__ __launch_bounds__(kScanBlock) void k_count(const uint8_t *__restrict__ f, int64_t n,
                                                      int64_t *counts) {
  __shared__ int red[kScanBlock];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  red[threadIdx.x] = (i < n && f[i]) ? 1 : 0;
  __syncthreads();
  for (int s = kScanBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kScanBlock) void k_scan(int64_t *counts, int64_t nb, int64_t *total) {
  __shared__ int64_t part[kScanBlock];
  const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
  const int64_t b = threadIdx.x * per, e = b + per < nb ? b + per : nb;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += counts[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int k = 0; k < kScanBlock; ++k) {
      const int64_t v = part[k];
      part[k] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    const int64_t v = counts[i];
    counts[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_write_idx(const uint8_t *__restrict__ f, int64_t n,
                                                          const int64_t *offs, int64_t *idx) {
  __shared__ int pre[kScanBlock];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const int v = (i < n && f[i]) ? 1 : 0;
  pre[threadIdx.x] = v;
  __syncthreads();
  // inclusive Hillis--Steele scan over the block
  for (int s = 1; s < kScanBlock; s <<= 1) {
    const int add = threadIdx.x >= s ? pre[threadIdx.x - s] : 0;
    __syncthreads();
    pre[threadIdx.x] += add;
    __syncthreads();
  }
  if (v) idx[offs[blockIdx.x] + pre[threadIdx.x] - 1] = i;
}

// Mean of ln rec[j][i] over i (one block per output j, fixed-order tree).
__global__ __launch_bounds__(256) void k_logmean(const double *__restrict__ rec, int64_t n,
                                                 double *mean) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += log(rec[j * n + i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[j] = red[0] / (double)n;
}

// Standard deviation of ln rec[j][i] about the mean (second pass).
__global__ __launch_bounds__(256) void k_logstd(const double *__restrict__ rec, int64_t n,
                                                const double *mean, double *stdv) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const double mu = mean[j];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = log(rec[j * n + i]) - mu;
    s = fma(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) stdv[j] = sqrt(red[0] / (double)n);
}

// label[idx[i]] = [max_j rec[j][i] >= 2]; -1 if any record is NaN.
__global__ void k_exact_labels(const double *__restrict__ rec, int64_t k,
                               const int64_t *__restrict__ idx, int8_t *label) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double mx = -INFINITY;
  bool bad = false;
  for (int j = 0; j < kOut; ++j) {
    const double v = rec[j * k + i];
    bad = bad || isnan(v);
    mx = v > mx ? v : mx;
  }
  label[idx ? idx[i] : i] = bad ? -1 : (mx >= 2.0 ? 1 : 0);
}

}  // namespace

// ======================================================================== API

struct sur_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t max_batch = 0;
  std::string err;
  double lr = 1e-3, b1 = 0.9, b2 = 0.999, eps = 1e-8;
  int64_t t = 0;
  double in_lo[2] = {0, 0}, in_hi[2] = {1, 1};
  double out_mean[kOut], out_std[kOut];
  bool have_norm = false;
  // parameters and optimiser state
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *V = nullptr;
  bf16 *W2 = nullptr, *W2T = nullptr, *W3 = nullptr, *W3T = nullptr, *W4 = nullptr,
       *W4T = nullptr;
  float *d_mean = nullptr, *d_std = nullptr;
  double *d_dmean = nullptr, *d_dstd = nullptr;
  // one batch: inputs and targets, the activations and gradients
  // transposed ([feature][batch row]) for the weight-gradient products
  float *x = nullptr, *tgt = nullptr;
  bf16 *a1T = nullptr, *a2T = nullptr, *a3T = nullptr;
  bf16 *dz4bT = nullptr, *dz3bT = nullptr, *dz2bT = nullptr;
  // partial sums of the gradients: split-K weight products, per-16-row-tile
  // column sums (biases, layer-1 weights), loss
  float *part2 = nullptr, *part3 = nullptr, *part4 = nullptr;
  float *cp2 = nullptr, *cp3 = nullptr,
        *cp4 = nullptr;
  float *lpart = nullptr;     // loss partials
  float *loss = nullptr;      // device scalar
  float *loss_acc = nullptr;  // device scalar: sum of batch losses of an epoch
  int64_t *scan = nullptr;    // compaction scratch
  int64_t scan_cap = 0;
  int8_t *nlab = nullptr;     // exact labels of the training grid [G][G]
  double *srec = nullptr;     // records sorted per point (fit_norm, build_dataset)
  int64_t srec_n = 0;
  int nlab_G = 0;
  // captured training epoch (sur_train_epoch), replayed while the dataset,
  // row list and batch are the same
  hipStream_t cap_stream = nullptr;
  hipGraph_t ep_graph = nullptr;
  hipGraphExec_t ep_exec = nullptr;
  const float *ep_x = nullptr, *ep_y = nullptr;
  const int64_t *ep_perm = nullptr;
  int64_t ep_n = 0, ep_batch = 0;
  double *hyper = nullptr;   // device: lr, beta1, beta2, eps, t_base
  double hyper_host[5] = {0, 0, 0, 0, 0};
  // inference: W2, W3, W4 in fragment order (k_frag_layout), and staging of
  // host inputs and outputs (sur_forward from host memory: kInferRows rows,
  // allocated on first use)
  bf16 *W2f = nullptr, *W3f = nullptr, *W4f = nullptr;
  float *ix = nullptr, *iout = nullptr;
};

namespace {

constexpr int kSplit = 8;   // largest batch split of the weight-gradient products

// Batch split of a weight-gradient product: chunks of 256 rows where the
// batch allows (at most kSplit of them), else chunks of a multiple of 64 rows
// (m is a multiple of 64).
int wgrad_split(int64_t m) {
  for (int s = kSplit; s > 1; s >>= 1)
    if (m % (64 * s) == 0 && m / s >= 256) return s;
  return 1;
}

thread_local std::string g_serr;

int sfail(sur_ctx *s, int code, const std::string &m) {
  g_serr = m;
  if (s) s->err = m;
  return code;
}

#define SUR_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return sfail((ctx), e_ == hipErrorOutOfMemory ? ENS_E_NOMEM : ENS_E_HIP,          \
                   std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) == hipSuccess) (void)hipSetDevice(d);
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <class T>
hipError_t alloc(T **p, int64_t count) {
  return hipMalloc((void **)p, (size_t)(count > 0 ? count : 1) * sizeof(T));
}

unsigned nblk(int64_t count, int b) { return (unsigned)((count + b - 1) / b); }

// R, C multiples of 32; K / split a multiple of 64.
// The three products of bt.g in one launch (each R, C a multiple of 32, the
// same K with K / split a multiple of 64).
hipError_t gemm3(hipStream_t st, GemmBatch bt, int split) {
  bt.split = split;
  int64_t total = 0;
  for (int p = 0; p < 3; ++p) {
    bt.nblk[p] = (bt.g[p].R / kTile) * (bt.g[p].C / kTile) * split;
    total += bt.nblk[p];
  }
  if ((bt.g[0].K / split) % 256 == 0)
    hipLaunchKernelGGL((k_gemm<8>), dim3((unsigned)total), dim3(64), 0, st, bt);
  else
    hipLaunchKernelGGL((k_gemm<2>), dim3((unsigned)total), dim3(64), 0, st, bt);
  return hipGetLastError();
}

GemmArgs gargs(const bf16 *X, int64_t ldx, const bf16 *Y, int64_t ldy, int64_t R, int64_t C,
               int64_t K) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.X = X;
  g.ldx = ldx;
  g.Y = Y;
  g.ldy = ldy;
  g.R = R;
  g.C = C;
  g.K = K;
  return g;
}

constexpr int64_t kInferRows = 65536;

hipError_t ensure_infer(sur_ctx *s) {
  if (s->ix) return hipSuccess;
  hipError_t e = hipMalloc((void **)&s->ix, kInferRows * kIn * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&s->iout, kInferRows * kOut * sizeof(float));
  if (e != hipSuccess) {
    (void)hipFree(s->ix);
    (void)hipFree(s->iout);
    s->ix = s->iout = nullptr;
  }
  return e;
}

// Compaction scratch (block counts and their scan) for screens of up to n
// points, grown when a larger screen comes.
hipError_t reserve_scan(sur_ctx *s, int64_t n) {
  const int64_t need = (n + kScanBlock - 1) / kScanBlock + 1;
  if (need <= s->scan_cap) return hipSuccess;
  (void)hipFree(s->scan);
  s->scan = nullptr;
  s->scan_cap = 0;
  const hipError_t e = hipMalloc((void **)&s->scan, (size_t)need * sizeof(int64_t));
  if (e == hipSuccess) s->scan_cap = need;
  return e;
}

// The fragment-order weight copies of the current parameters, then the fused
// inference of n points (n > 0).
hipError_t fused(sur_ctx *s, FusedArgs a, bool screen) {
  hipStream_t st = s->stream;
  hipLaunchKernelGGL(k_frag_layout, dim3(nblk(kH * kH, 256)), dim3(256), 0, st, s->W2,
                     (int64_t)kH, 0, s->W2f);
  hipLaunchKernelGGL(k_frag_layout, dim3(nblk(kH * kH, 256)), dim3(256), 0, st, s->W3,
                     (int64_t)kH, 1, s->W3f);
  hipLaunchKernelGGL(k_frag_layout, dim3(nblk(kOut * kH, 256)), dim3(256), 0, st, s->W4,
                     (int64_t)kOut, 1, s->W4f);
  a.P = s->P;
  a.W2f = s->W2f;
  a.W3f = s->W3f;
  a.W4f = s->W4f;
  const dim3 grid(nblk(a.n, 128));   // 4 waves of 32 points
  if (screen)
    hipLaunchKernelGGL(k_fused<true>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_fused<false>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// Adam's arguments for the handle's parameters: hyper-parameters from
// device memory (hyper != NULL, a captured step `step`) or the handle's.
AdamArgs adam_args(sur_ctx *s, const double *hyper, int step) {
  AdamArgs a;
  a.P = s->P;
  a.Mm = s->Mm;
  a.V = s->V;
  a.hyper = hyper;
  a.lr = s->lr;
  a.b1 = s->b1;
  a.b2 = s->b2;
  a.eps = s->eps;
  a.t_base = (double)s->t;
  a.step = step;
  a.W2 = s->W2;
  a.W2T = s->W2T;
  a.W3 = s->W3;
  a.W3T = s->W3T;
  a.W4 = s->W4;
  a.W4T = s->W4T;
  return a;
}

// One batch's loss and gradients of all parameters into s->G and s->loss:
// the fused tile kernel (forward, loss gradient, data gradients), then the
// weight gradients (split over the batch) and the fixed-order reduction,
// which with ad != NULL also takes the Adam step.  Inputs: row r of x and
// tgt, or row rows[r] with rows; loss_acc (optional) accumulates the loss
// (first: starts it).
hipError_t train_batch(sur_ctx *s, int64_t m, const float *x, const float *tgt,
                       const int64_t *rows, float *loss_acc = nullptr, bool first = true,
                       const AdamArgs *ad = nullptr) {
  hipStream_t st = s->stream;
  hipError_t e;
  const int split = wgrad_split(m);
  const int64_t T = m / kTR;
  TrainArgs a;
  a.x = x;
  a.rows = rows;
  a.tgt = tgt;
  a.P = s->P;
  a.W2 = s->W2;
  a.W3 = s->W3;
  a.W4 = s->W4;
  a.W3T = s->W3T;
  a.W4T = s->W4T;
  a.m = m;
  a.a1T = s->a1T;
  a.a2T = s->a2T;
  a.a3T = s->a3T;
  a.dz4T = s->dz4bT;
  a.dz3T = s->dz3bT;
  a.dz2T = s->dz2bT;
  a.cp4 = s->cp4;
  a.cp3 = s->cp3;
  a.cp2 = s->cp2;
  a.lpart = s->lpart;
  hipLaunchKernelGGL(k_train_fb, dim3((unsigned)T), dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  GemmBatch bt;
  bt.g[0] = gargs(s->dz4bT, m, s->a3T, m, kOut, kH, m);
  bt.g[0].out_f32 = s->part4;
  bt.g[1] = gargs(s->dz3bT, m, s->a2T, m, kH, kH, m);
  bt.g[1].out_f32 = s->part3;
  bt.g[2] = gargs(s->dz2bT, m, s->a1T, m, kH, kH, m);
  bt.g[2].out_f32 = s->part2;
  if ((e = gemm3(st, bt, split)) != hipSuccess) return e;
  GradParts p{s->part2, s->part3, s->cp2, s->cp3, s->part4, s->cp4, s->lpart};
  const dim3 rg(kReduceWBlocks + (kNColSums + 3) / 4);
  if (ad)
    hipLaunchKernelGGL(k_reduce_grads<true>, rg, dim3(256), 0, st, p, T, split,
                       (float)(m * kOut), s->G, s->loss, loss_acc, first ? 1 : 0, *ad);
  else
    hipLaunchKernelGGL(k_reduce_grads<false>, rg, dim3(256), 0, st, p, T, split,
                       (float)(m * kOut), s->G, s->loss, loss_acc, first ? 1 : 0,
                       adam_args(s, nullptr, 0));
  return hipGetLastError();
}

void free_epoch_graph(sur_ctx *s) {
  if (s->ep_exec) (void)hipGraphExecDestroy(s->ep_exec);
  if (s->ep_graph) (void)hipGraphDestroy(s->ep_graph);
  s->ep_exec = nullptr;
  s->ep_graph = nullptr;
}

hipError_t refresh(sur_ctx *s) {
  hipLaunchKernelGGL(k_refresh, dim3(nblk(kH * kH, 256)), dim3(256), 0, s->stream, s->P, s->W2,
                     s->W2T, s->W3, s->W3T, s->W4, s->W4T);
  return hipGetLastError();
}

// The records [kOut][n] sorted in decreasing order per point, in the
// handle's scratch (grown as needed); NULL on allocation failure.
const double *sorted_records(sur_ctx *s, const double *rec, int64_t n, hipError_t *e) {
  *e = hipSuccess;
  if (n > s->srec_n) {
    (void)hipFree(s->srec);
    s->srec = nullptr;
    s->srec_n = 0;
    *e = alloc(&s->srec, n * kOut);
    if (*e != hipSuccess) return nullptr;
    s->srec_n = n;
  }
  hipLaunchKernelGGL(k_sort_desc, dim3(nblk(n, 4)), dim3(256), 0, s->stream, rec, n, s->srec);
  *e = hipGetLastError();
  return *e == hipSuccess ? s->srec : nullptr;
}

int check_batch(sur_ctx *s, int64_t m) {
  if (m <= 0 || m % 64 || m > s->max_batch)
    return sfail(s, ENS_E_INVAL, "batch must be a positive multiple of 64 <= max_batch");
  return ENS_OK;
}

int load_batch(sur_ctx *s, const float *x, const float *tgt, int64_t m, int where) {
  const hipMemcpyKind k = where == ENS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  SUR_HIP(s, hipMemcpyAsync(s->x, x, (size_t)m * kIn * sizeof(float), k, s->stream));
  if (tgt)
    SUR_HIP(s, hipMemcpyAsync(s->tgt, tgt, (size_t)m * kOut * sizeof(float), k, s->stream));
  return ENS_OK;
}

// Captures the launches of one epoch over perm[0 .. n) (once per dataset,
// row-list buffer and batch); replays read the hyper-parameters and the row
// list's contents from device memory.
int ensure_epoch_graph(sur_ctx *s, const float *x, const float *y, int64_t n, const int64_t *perm,
                       int64_t batch) {
  const int64_t nb = n / batch;
  if (s->ep_exec && s->ep_x == x && s->ep_y == y && s->ep_perm == perm && s->ep_n == n &&
      s->ep_batch == batch)
    return ENS_OK;
  free_epoch_graph(s);
  hipStream_t user = s->stream;
  s->stream = s->cap_stream;
  hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  for (int64_t b = 0; e == hipSuccess && b < nb; ++b) {
    const int64_t *rows = perm + b * batch;
    // the step's Adam update from the hyper-parameters in s->hyper
    const AdamArgs ad = adam_args(s, s->hyper, (int)b);
    e = train_batch(s, batch, x, y, rows, s->loss_acc, b == 0, &ad);
  }
  hipGraph_t gr = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &gr);
  s->stream = user;
  if (e != hipSuccess || e2 != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return sfail(s, ENS_E_HIP, std::string("training epoch capture: ") +
                                   hipGetErrorString(e != hipSuccess ? e : e2));
  }
  s->ep_graph = gr;
  SUR_HIP(s, hipGraphInstantiate(&s->ep_exec, gr, nullptr, nullptr, 0));
  s->ep_x = x;
  s->ep_y = y;
  s->ep_perm = perm;
  s->ep_n = n;
  s->ep_batch = batch;
  return ENS_OK;
}

// Epoch e's row order: the training rows sorted by a hash of (seed, e, i)
// (SplitMix64's output function of a Weyl sequence), i.e. a seeded uniformly
// random permutation; equal keys keep index order.
__global__ void k_epoch_keys(const int64_t *__restrict__ rows, int64_t n, uint64_t seed,
                             int64_t epoch, unsigned long long *key, int64_t *val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(epoch * n + i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  key[i] = (unsigned long long)(z ^ (z >> 31));
  val[i] = rows[i];
}

}  // namespace

extern "C" {

const char *sur_last_error(sur_t s) { return s ? s->err.c_str() : g_serr.c_str(); }

int sur_create(int32_t device, void *hip_stream, int64_t max_batch, sur_t *out) {
  if (!out) return sfail(nullptr, ENS_E_INVAL, "sur_create: out is NULL");
  *out = nullptr;
  if (max_batch <= 0 || max_batch % 64 || max_batch > 65536)
    return sfail(nullptr, ENS_E_INVAL, "sur_create: max_batch must be a multiple of 64 in [64, 65536]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return sfail(nullptr, ENS_E_HIP, "sur_create: no HIP device");
  if (device < 0 || device >= ndev) return sfail(nullptr, ENS_E_INVAL, "sur_create: bad device");
  sur_ctx *s = new (std::nothrow) sur_ctx();
  if (!s) return sfail(nullptr, ENS_E_NOMEM, "sur_create: out of host memory");
  s->device = device;
  s->stream = (hipStream_t)hip_stream;
  s->max_batch = max_batch;
  for (int j = 0; j < kOut; ++j) {
    s->out_mean[j] = 0.0;
    s->out_std[j] = 1.0;
  }
  DevGuard dg(device);
  const int64_t B = max_batch;
  hipError_t e = hipSuccess;
#define A(ptr, cnt) \
  if (e == hipSuccess) e = alloc(&s->ptr, (cnt))
  A(P, kNP); A(G, kNP); A(Mm, kNP); A(V, kNP);
  A(W2, kH * kH); A(W2T, kH * kH); A(W3, kH * kH); A(W3T, kH * kH);
  A(W4, kOut * kH); A(W4T, kOut * kH); A(W2f, kH * kH); A(W3f, kH * kH);
  A(W4f, kOut * kH);
  A(d_mean, kOut); A(d_std, kOut); A(d_dmean, kOut); A(d_dstd, kOut);
  A(x, B * kIn); A(tgt, B * kOut);
  A(a1T, B * kH); A(a2T, B * kH); A(a3T, B * kH);
  A(dz4bT, B * kOut); A(dz3bT, B * kH); A(dz2bT, B * kH);
  A(part2, (int64_t)kSplit * kH * kH); A(part3, (int64_t)kSplit * kH * kH);
  A(part4, (int64_t)kSplit * kOut * kH);
  A(cp2, B / kTR * kH);
  A(cp3, B / kTR * kH); A(cp4, B / kTR * kOut);
  A(lpart, B / kTR); A(loss, 1);
  A(loss_acc, 1);
  A(hyper, 5);
#undef A
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMemsetAsync(s->P, 0, kNP * sizeof(float), s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->Mm, 0, kNP * sizeof(float), s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->V, 0, kNP * sizeof(float), s->stream);
  if (e == hipSuccess) e = refresh(s);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    int code = sfail(nullptr, e == hipErrorOutOfMemory ? ENS_E_NOMEM : ENS_E_HIP,
                     std::string("sur_create: ") + hipGetErrorString(e));
    sur_destroy(s);
    return code;
  }
  *out = s;
  return ENS_OK;
}

int sur_destroy(sur_t s) {
  if (!s) return ENS_OK;
  DevGuard dg(s->device);
  (void)hipStreamSynchronize(s->stream);
  void *ptrs[] = {s->P, s->G, s->Mm, s->V, s->W2, s->W2T, s->W3, s->W3T, s->W4, s->W4T,
                  s->d_mean, s->d_std, s->d_dmean, s->d_dstd, s->x, s->tgt, s->a1T,
                  s->a2T, s->a3T, s->dz4bT, s->dz3bT, s->dz2bT, s->part2, s->part3,
                  s->part4, s->cp2, s->cp3, s->cp4, s->lpart,
                  s->loss, s->loss_acc, s->scan, s->nlab, s->srec, s->ix, s->iout, s->W2f,
                  s->W3f, s->W4f};
  for (void *p : ptrs) (void)hipFree(p);
  free_epoch_graph(s);
  (void)hipFree(s->hyper);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
  return ENS_OK;
}

int sur_set_params(sur_t s, const double *flat) {
  if (!s || !flat) return sfail(s, ENS_E_INVAL, "sur_set_params: NULL argument");
  std::vector<float> f(kNP);
  for (int64_t i = 0; i < kNP; ++i) {
    if (!std::isfinite(flat[i])) return sfail(s, ENS_E_INVAL, "sur_set_params: non-finite value");
    f[i] = (float)flat[i];
  }
  DevGuard dg(s->device);
  SUR_HIP(s, hipMemcpyAsync(s->P, f.data(), kNP * sizeof(float), hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipMemsetAsync(s->Mm, 0, kNP * sizeof(float), s->stream));
  SUR_HIP(s, hipMemsetAsync(s->V, 0, kNP * sizeof(float), s->stream));
  SUR_HIP(s, refresh(s));
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  s->t = 0;
  return ENS_OK;
}

int sur_get_params(sur_t s, double *flat) {
  if (!s || !flat) return sfail(s, ENS_E_INVAL, "sur_get_params: NULL argument");
  std::vector<float> f(kNP);
  DevGuard dg(s->device);
  SUR_HIP(s, hipMemcpyAsync(f.data(), s->P, kNP * sizeof(float), hipMemcpyDeviceToHost, s->stream));
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  for (int64_t i = 0; i < kNP; ++i) flat[i] = f[i];
  return ENS_OK;
}

int sur_set_norm(sur_t s, const double *in_lo, const double *in_hi, const double *out_mean,
                 const double *out_std) {
  if (!s || !in_lo || !in_hi || !out_mean || !out_std)
    return sfail(s, ENS_E_INVAL, "sur_set_norm: NULL argument");
  for (int i = 0; i < 2; ++i)
    if (!(in_hi[i] > in_lo[i]) || !std::isfinite(in_lo[i]) || !std::isfinite(in_hi[i]))
      return sfail(s, ENS_E_INVAL, "sur_set_norm: need finite in_lo < in_hi");
  for (int j = 0; j < kOut; ++j)
    if (!(out_std[j] > 0.0) || !std::isfinite(out_mean[j]) || !std::isfinite(out_std[j]))
      return sfail(s, ENS_E_INVAL, "sur_set_norm: need finite mean and std > 0");
  std::vector<float> m(kOut), sd(kOut);
  for (int i = 0; i < 2; ++i) {
    s->in_lo[i] = in_lo[i];
    s->in_hi[i] = in_hi[i];
  }
  for (int j = 0; j < kOut; ++j) {
    s->out_mean[j] = out_mean[j];
    s->out_std[j] = out_std[j];
    m[j] = (float)out_mean[j];
    sd[j] = (float)out_std[j];
  }
  DevGuard dg(s->device);
  SUR_HIP(s, hipMemcpyAsync(s->d_mean, m.data(), kOut * sizeof(float), hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipMemcpyAsync(s->d_std, sd.data(), kOut * sizeof(float), hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipMemcpyAsync(s->d_dmean, s->out_mean, kOut * sizeof(double), hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipMemcpyAsync(s->d_dstd, s->out_std, kOut * sizeof(double), hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  s->have_norm = true;
  return ENS_OK;
}

int sur_build_dataset(sur_t s, const double *params, const double *records, int64_t n, float *x,
                      float *y) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_build_dataset: NULL handle");
  if (!s->have_norm) return sfail(s, ENS_E_ORDER, "sur_build_dataset: call sur_set_norm first");
  if (n < 0 || (n > 0 && (!params || !records || !x || !y)))
    return sfail(s, ENS_E_INVAL, "sur_build_dataset: bad arguments");
  if (n == 0) return ENS_OK;
  DevGuard dg(s->device);
  const double sc0 = 2.0 / (s->in_hi[0] - s->in_lo[0]), sc1 = 2.0 / (s->in_hi[1] - s->in_lo[1]);
  hipLaunchKernelGGL(k_inputs, dim3(nblk(n, 256)), dim3(256), 0, s->stream, params, n,
                     s->in_lo[0], sc0, s->in_lo[1], sc1, x);
  SUR_HIP(s, hipGetLastError());
  hipError_t se;
  const double *sorted = sorted_records(s, records, n, &se);
  SUR_HIP(s, se);
  hipLaunchKernelGGL(k_targets, dim3(nblk(n * kOut, 256)), dim3(256), 0, s->stream, sorted, n,
                     s->d_dmean, s->d_dstd, y);
  SUR_HIP(s, hipGetLastError());
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}

int sur_set_adam(sur_t s, double lr, double beta1, double beta2, double eps) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_set_adam: NULL handle");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return sfail(s, ENS_E_INVAL, "sur_set_adam: bad hyper-parameters");
  s->lr = lr;
  s->b1 = beta1;
  s->b2 = beta2;
  s->eps = eps;
  return ENS_OK;
}

int sur_gradients(sur_t s, const float *x, const float *target, int64_t m, float *grads,
                  float *loss, int32_t where) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_gradients: NULL handle");
  if (int rc = check_batch(s, m)) return rc;
  if (!x || !target) return sfail(s, ENS_E_INVAL, "sur_gradients: NULL input");
  DevGuard dg(s->device);
  if (int rc = load_batch(s, x, target, m, where)) return rc;
  SUR_HIP(s, train_batch(s, m, s->x, s->tgt, nullptr));
  const hipMemcpyKind k = where == ENS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (grads) SUR_HIP(s, hipMemcpyAsync(grads, s->G, kNP * sizeof(float), k, s->stream));
  if (loss) SUR_HIP(s, hipMemcpyAsync(loss, s->loss, sizeof(float), k, s->stream));
  if (where == ENS_HOST) SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}

int sur_train_step(sur_t s, const float *x, const float *target, int64_t m, float *loss,
                   int32_t where) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_train_step: NULL handle");
  if (int rc = check_batch(s, m)) return rc;
  if (!x || !target) return sfail(s, ENS_E_INVAL, "sur_train_step: NULL input");
  DevGuard dg(s->device);
  if (int rc = load_batch(s, x, target, m, where)) return rc;
  const AdamArgs ad = adam_args(s, nullptr, 0);
  SUR_HIP(s, train_batch(s, m, s->x, s->tgt, nullptr, nullptr, true, &ad));
  s->t += 1;
  if (loss) {
    const hipMemcpyKind k = where == ENS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    SUR_HIP(s, hipMemcpyAsync(loss, s->loss, sizeof(float), k, s->stream));
    if (where == ENS_HOST) SUR_HIP(s, hipStreamSynchronize(s->stream));
  }
  return ENS_OK;
}

int sur_forward(sur_t s, const float *x, int64_t m, float *out, int32_t where) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_forward: NULL handle");
  if (m < 0 || (m > 0 && (!x || !out))) return sfail(s, ENS_E_INVAL, "sur_forward: bad arguments");
  DevGuard dg(s->device);
  if (m == 0) return ENS_OK;
  FusedArgs a;
  std::memset(&a, 0, sizeof(a));
  if (where == ENS_DEVICE) {
    a.n = m;
    a.x = x;
    a.out = out;
    SUR_HIP(s, fused(s, a, false));
    return ENS_OK;
  }
  // host buffers: staged through the handle's buffers kInferRows rows at a time
  SUR_HIP(s, ensure_infer(s));
  for (int64_t first = 0; first < m; first += kInferRows) {
    const int64_t rows = m - first < kInferRows ? m - first : kInferRows;
    SUR_HIP(s, hipMemcpyAsync(s->ix, x + first * kIn, rows * kIn * sizeof(float),
                              hipMemcpyHostToDevice, s->stream));
    a.n = rows;
    a.x = s->ix;
    a.out = s->iout;
    SUR_HIP(s, fused(s, a, false));
    SUR_HIP(s, hipMemcpyAsync(out + first * kOut, s->iout, rows * kOut * sizeof(float),
                              hipMemcpyDeviceToHost, s->stream));
  }
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}

int sur_reserve(sur_t s, int64_t n_screen) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_reserve: NULL handle");
  if (n_screen < 0) return sfail(s, ENS_E_INVAL, "sur_reserve: n_screen must be >= 0");
  DevGuard dg(s->device);
  SUR_HIP(s, reserve_scan(s, n_screen));
  return ENS_OK;
}

int sur_screen(sur_t s, const double *params, int64_t n, const sur_screen_opts *o, int8_t *label,
               uint8_t *resolve, float *pred_max, int64_t *resolve_idx, int64_t *n_resolve) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_screen: NULL handle");
  if (!o || !n_resolve || n < 0 || (n > 0 && !params))
    return sfail(s, ENS_E_INVAL, "sur_screen: bad arguments");
  if (resolve_idx && !resolve)
    return sfail(s, ENS_E_INVAL, "sur_screen: resolve_idx needs the resolve mask");
  if (!s->have_norm) return sfail(s, ENS_E_ORDER, "sur_screen: call sur_set_norm first");
  if (!(o->margin >= 0) || !(o->spread >= 0) || !(o->flag_margin >= 0) ||
      std::isnan(o->label_margin))
    return sfail(s, ENS_E_INVAL, "sur_screen: margins must be >= 0");
  *n_resolve = 0;
  if (n == 0) return ENS_OK;
  DevGuard dg(s->device);
  const double sc0 = 2.0 / (s->in_hi[0] - s->in_lo[0]), sc1 = 2.0 / (s->in_hi[1] - s->in_lo[1]);
  const bool use_labels = s->nlab && o->label_margin >= 0.0;
  FusedArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.prm = params;
  a.lo0 = s->in_lo[0];
  a.sc0 = sc0;
  a.lo1 = s->in_lo[1];
  a.sc1 = sc1;
  a.mean = s->d_mean;
  a.stdv = s->d_std;
  a.margin = (float)o->margin;
  a.spread = (float)o->spread;
  a.flag_margin = (float)o->flag_margin;
  a.label_margin = (float)o->label_margin;
  a.nlab = use_labels ? s->nlab : nullptr;
  a.GL = s->nlab_G;
  a.label = label;
  a.resolve = resolve;
  a.pmax = pred_max;
  SUR_HIP(s, fused(s, a, true));
  if (resolve) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    SUR_HIP(s, reserve_scan(s, n));
    hipLaunchKernelGGL(k_count, dim3((unsigned)nb), dim3(kScanBlock), 0, s->stream, resolve, n,
                       s->scan);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, s->stream, s->scan, nb,
                       s->scan + nb);
    if (resolve_idx)
      hipLaunchKernelGGL(k_write_idx, dim3((unsigned)nb), dim3(kScanBlock), 0, s->stream,
                         resolve, n, s->scan, resolve_idx);
    SUR_HIP(s, hipGetLastError());
    SUR_HIP(s, hipMemcpyAsync(n_resolve, s->scan + nb, sizeof(int64_t), hipMemcpyDeviceToHost,
                              s->stream));
  }
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}

int sur_fit_norm(sur_t s, const double *in_lo, const double *in_hi, const double *records,
                 int64_t n, double *out_mean, double *out_std) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_fit_norm: NULL handle");
  if (!in_lo || !in_hi || !records || n <= 0)
    return sfail(s, ENS_E_INVAL, "sur_fit_norm: bad arguments");
  DevGuard dg(s->device);
  hipError_t se;
  const double *sorted = sorted_records(s, records, n, &se);
  SUR_HIP(s, se);
  hipLaunchKernelGGL(k_logmean, dim3(kOut), dim3(256), 0, s->stream, sorted, n, s->d_dmean);
  hipLaunchKernelGGL(k_logstd, dim3(kOut), dim3(256), 0, s->stream, sorted, n, s->d_dmean,
                     s->d_dstd);
  SUR_HIP(s, hipGetLastError());
  double m[kOut], sd[kOut];
  SUR_HIP(s, hipMemcpyAsync(m, s->d_dmean, sizeof(m), hipMemcpyDeviceToHost, s->stream));
  SUR_HIP(s, hipMemcpyAsync(sd, s->d_dstd, sizeof(sd), hipMemcpyDeviceToHost, s->stream));
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  for (int j = 0; j < kOut; ++j)
    if (!(sd[j] > 0.0) || !std::isfinite(m[j]))
      return sfail(s, ENS_E_INVAL, "sur_fit_norm: records give a non-positive or non-finite spread");
  if (int rc = sur_set_norm(s, in_lo, in_hi, m, sd)) return rc;
  if (out_mean) std::memcpy(out_mean, m, sizeof(m));
  if (out_std) std::memcpy(out_std, sd, sizeof(sd));
  return ENS_OK;
}

int sur_train_epoch(sur_t s, const float *x, const float *y, int64_t n, const int64_t *perm,
                    int64_t batch, float *mean_loss) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_train_epoch: NULL handle");
  if (int rc = check_batch(s, batch)) return rc;
  if (!x || !y || !perm || n < batch) return sfail(s, ENS_E_INVAL, "sur_train_epoch: bad arguments");
  DevGuard dg(s->device);
  const int64_t nb = n / batch;
  if (int rc = ensure_epoch_graph(s, x, y, n, perm, batch)) return rc;
  s->hyper_host[0] = s->lr;
  s->hyper_host[1] = s->b1;
  s->hyper_host[2] = s->b2;
  s->hyper_host[3] = s->eps;
  s->hyper_host[4] = (double)s->t;
  SUR_HIP(s, hipMemcpyAsync(s->hyper, s->hyper_host, sizeof(s->hyper_host),
                            hipMemcpyHostToDevice, s->stream));
  SUR_HIP(s, hipGraphLaunch(s->ep_exec, s->stream));
  s->t += nb;
  if (mean_loss) {
    float acc = 0.f;
    SUR_HIP(s, hipMemcpyAsync(&acc, s->loss_acc, sizeof(float), hipMemcpyDeviceToHost, s->stream));
    SUR_HIP(s, hipStreamSynchronize(s->stream));
    *mean_loss = acc / (float)nb;
  }
  return ENS_OK;
}

int sur_train_epochs(sur_t s, const float *x, const float *y, const int64_t *rows, int64_t n,
                     int64_t batch, int64_t epochs, const double *lr, uint64_t seed,
                     float *losses) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_train_epochs: NULL handle");
  if (int rc = check_batch(s, batch)) return rc;
  if (!x || !y || !rows || n < batch || epochs < 0 || (epochs > 0 && !lr))
    return sfail(s, ENS_E_INVAL, "sur_train_epochs: bad arguments");
  for (int64_t e = 0; e < epochs; ++e)
    if (!(lr[e] > 0)) return sfail(s, ENS_E_INVAL, "sur_train_epochs: learning rates must be > 0");
  if (epochs == 0) return ENS_OK;
  DevGuard dg(s->device);
  const int64_t nb = n / batch;
  // device buffers of this call: sort keys and values, the epoch's order,
  // the per-epoch hyper-parameters, the per-epoch losses, sort scratch
  size_t tmp = 0;
  SUR_HIP(s, rocprim::radix_sort_pairs(nullptr, tmp, (const unsigned long long *)nullptr,
                                       (unsigned long long *)nullptr, (const int64_t *)nullptr,
                                       (int64_t *)nullptr, (size_t)n, 0u, 64u, s->stream));
  const size_t kb = ((size_t)n * 8 + 255) & ~(size_t)255;
  const size_t hb = ((size_t)epochs * 5 * sizeof(double) + 255) & ~(size_t)255;
  const size_t lb = ((size_t)epochs * sizeof(float) + 255) & ~(size_t)255;
  char *buf = nullptr;
  SUR_HIP(s, hipMalloc((void **)&buf, 4 * kb + hb + lb + tmp));
  auto *key_in = (unsigned long long *)buf;
  auto *key_out = (unsigned long long *)(buf + kb);
  auto *val_in = (int64_t *)(buf + 2 * kb);
  auto *order = (int64_t *)(buf + 3 * kb);
  auto *hyp = (double *)(buf + 4 * kb);
  auto *loss_d = (float *)(buf + 4 * kb + hb);
  void *sort_tmp = buf + 4 * kb + hb + lb;
  std::vector<double> h((size_t)epochs * 5);
  for (int64_t e = 0; e < epochs; ++e) {
    h[5 * e + 0] = lr[e];
    h[5 * e + 1] = s->b1;
    h[5 * e + 2] = s->b2;
    h[5 * e + 3] = s->eps;
    h[5 * e + 4] = (double)(s->t + e * nb);
  }
  hipError_t err = hipMemcpyAsync(hyp, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                                  s->stream);
  int rc = ENS_OK;
  if (err == hipSuccess) rc = ensure_epoch_graph(s, x, y, n, order, batch);
  for (int64_t e = 0; err == hipSuccess && rc == ENS_OK && e < epochs; ++e) {
    hipLaunchKernelGGL(k_epoch_keys, dim3(nblk(n, 256)), dim3(256), 0, s->stream, rows, n,
                       (uint64_t)seed, e, key_in, val_in);
    err = hipGetLastError();
    if (err == hipSuccess)
      err = rocprim::radix_sort_pairs(sort_tmp, tmp, key_in, key_out, val_in, order, (size_t)n,
                                      0u, 64u, s->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(s->hyper, hyp + 5 * e, 5 * sizeof(double), hipMemcpyDeviceToDevice,
                           s->stream);
    if (err == hipSuccess) err = hipGraphLaunch(s->ep_exec, s->stream);
    if (err == hipSuccess)
      err = hipMemcpyAsync(loss_d + e, s->loss_acc, sizeof(float), hipMemcpyDeviceToDevice,
                           s->stream);
  }
  std::vector<float> lh((size_t)epochs);
  if (err == hipSuccess && rc == ENS_OK)
    err = hipMemcpyAsync(lh.data(), loss_d, epochs * sizeof(float), hipMemcpyDeviceToHost, s->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(s->stream);
  // the epoch graph reads `order`, which is freed here: drop it
  free_epoch_graph(s);
  s->ep_perm = nullptr;
  (void)hipFree(buf);
  if (rc != ENS_OK) return rc;
  if (err != hipSuccess)
    return sfail(s, err == hipErrorOutOfMemory ? ENS_E_NOMEM : ENS_E_HIP,
                 std::string("sur_train_epochs: ") + hipGetErrorString(err));
  s->t += epochs * nb;
  if (losses)
    for (int64_t e = 0; e < epochs; ++e) losses[e] = lh[e] / (float)nb;
  return ENS_OK;
}

int sur_exact_labels(sur_t s, const double *records, int64_t k, const int64_t *idx,
                     int8_t *label) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_exact_labels: NULL handle");
  if (k < 0 || (k > 0 && (!records || !label)))
    return sfail(s, ENS_E_INVAL, "sur_exact_labels: bad arguments");
  if (k == 0) return ENS_OK;
  DevGuard dg(s->device);
  hipLaunchKernelGGL(k_exact_labels, dim3(nblk(k, 256)), dim3(256), 0, s->stream, records, k,
                     idx, label);
  SUR_HIP(s, hipGetLastError());
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}

int sur_fit_label_map(sur_t s, const double *records, int32_t G, int8_t *map_out) {
  if (!s) return sfail(nullptr, ENS_E_INVAL, "sur_fit_label_map: NULL handle");
  if (!records || G < 2 || G > 65536) return sfail(s, ENS_E_INVAL, "sur_fit_label_map: bad arguments");
  const int64_t n = (int64_t)G * G;
  DevGuard dg(s->device);
  if (s->nlab_G != G) {
    (void)hipFree(s->nlab);
    s->nlab = nullptr;
    s->nlab_G = 0;
    SUR_HIP(s, hipMalloc((void **)&s->nlab, n));
    s->nlab_G = G;
  }
  hipLaunchKernelGGL(k_node_label, dim3(nblk(n, 256)), dim3(256), 0, s->stream, records, n, s->nlab);
  SUR_HIP(s, hipGetLastError());
  if (map_out) SUR_HIP(s, hipMemcpyAsync(map_out, s->nlab, n, hipMemcpyDeviceToDevice, s->stream));
  SUR_HIP(s, hipStreamSynchronize(s->stream));
  return ENS_OK;
}


}  // extern "C"
