// Learned narrow-band cull (Sec. II.A.3: the interpolant is only needed in a
// narrow volume around the surface, where its zero level set is the
// reconstruction).  A network u -> 128 -> 128 -> 128 -> 128 -> 1 with SiLU
// after every hidden layer predicts f / tau from the position u, normalised
// as u = (x - centre) * scale; it is trained with Adam on (position, f)
// pairs that the interpolant itself supplies.  On a grid it keeps the exact
// sum only on the bricks where its sign may be wrong (a node within 3 steps
// of an opposite predicted sign, or a prediction below the held-out error);
// the other bricks of the support take tau * y.
//
// Matrix cores.  The three 128 x 128 layers run on
// v_mfma_f32_16x16x32_bf16 (bf16 operands, float32 accumulation).  Operand
// layouts of the instruction (checked on the GPU): lane l holds row (A) or
// column (B) l % 16 and k = 8 (l / 16) .. 8 (l / 16) + 7, eight consecutive
// bf16 in one 16-byte register quad; the 16 x 16 float32 result holds column
// l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3.  Every product here is written
// as rows of A times rows of B (B "stored by columns"), both with k
// contiguous, so each operand is one 16-byte load per lane.  A workgroup of
// four waves takes 64 samples; a wave owns 16 of them through every layer,
// their activations in LDS (bf16 rows padded to 136 entries, so that the
// 16 rows of a tile start in different banks).
//
// Training.  Forward (saving the pre-activations in float32), backward (one
// workgroup per 64 samples writes its whole gradient: the products
// dZ^T H and dZ W of the three wide layers on the matrix cores, the first
// and last layers on the VALU), then one thread per parameter sums the
// workgroups' gradients in a fixed order and takes the Adam step; the bf16
// copies (and their transposes, for dZ W) are refreshed after it.
#include <algorithm>
#include <vector>

#include "common.h"

namespace rbf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW = 128;                  // hidden width
constexpr int kTile = 64;                // samples per workgroup
constexpr int kNetThreads = 256;
constexpr int kLdh = kW + 8;             // padded bf16 row, samples x features
constexpr int kLdt = kTile + 8;          // padded bf16 row, features x samples
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + 3 * kW;
constexpr int kOffW2 = kOffB1 + kW, kOffB2 = kOffW2 + kW * kW;
constexpr int kOffW3 = kOffB2 + kW, kOffB3 = kOffW3 + kW * kW;
constexpr int kOffW4 = kOffB3 + kW, kOffB4 = kOffW4 + kW * kW;
constexpr int kOffW5 = kOffB4 + kW, kOffB5 = kOffW5 + kW;
constexpr int kParams = kOffB5 + 1;
static_assert(kParams == RBF_NET_PARAMS, "parameter count of the header");
constexpr int kOffW[3] = {kOffW2, kOffW3, kOffW4};
constexpr int kOffB[3] = {kOffB2, kOffB3, kOffB4};

struct NetView {
  const float* P;         // float32 parameters
  const __bf16* Wb;       // W2, W3, W4, [out][in], bf16
  const __bf16* WbT;      // their transposes, [in][out]
  double cx, cy, cz, scale;
};

// Sample positions: B x 3 float64 points, or the nodes of a brick list (16
// per brick, in the brick's node order; nodes outside the grid are invalid).
struct PosSrc {
  const double* X;
  const int64_t* bricks;
  GridDesc gd;
};

__device__ __forceinline__ bool sample_pos(const PosSrc& p, int64_t s, double* x) {
  if (p.X) {
    x[0] = p.X[3 * s];
    x[1] = p.X[3 * s + 1];
    x[2] = p.X[3 * s + 2];
    return true;
  }
  const int64_t b = p.bricks[s / kGroup];
  const int l = (int)(s % kGroup);
  const GridDesc& gd = p.gd;
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  const int64_t i = bx * 4 + (l & 3), j = by * 2 + ((l >> 2) & 1), k = bz * 2 + (l >> 3);
  x[0] = gd.o[0] + (double)i * gd.h[0];
  x[1] = gd.o[1] + (double)j * gd.h[1];
  x[2] = gd.o[2] + (double)k * gd.h[2];
  return i < gd.n[0] && j < gd.n[1] && k < gd.n[2];
}

// SiLU with the hardware exponential and reciprocal (about one ulp each:
// far below the bf16 rounding the activations then take).
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// acc[t] += A[16 rows][K] * B[16 t .. 16 t + 15][K]^T for t = 0..7: the 16
// rows of A at A + r lda, the 128 rows of B at B + n ldb, k contiguous.
__device__ __forceinline__ void mma_rows16(const __bf16* A, int lda, const __bf16* B, int ldb, int K,
                                           f32x4 (&acc)[8]) {
  const int l = threadIdx.x & 63;
  const __bf16* a = A + (l & 15) * lda + 8 * (l >> 4);
  const __bf16* b = B + (l & 15) * ldb + 8 * (l >> 4);
  for (int c = 0; c < K; c += 32) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + c);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + 16 * t * ldb + c);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
    }
  }
}

// Forward: a persistent launch, one workgroup of eight waves per compute
// unit; the three bf16 weight matrices are copied into its LDS once (rows
// padded like the activations) and the workgroup walks over tiles of 128
// samples, a wave taking 16 of them through every layer.  y, and with SAVE
// the pre-activations Z[layer][sample][feature].
constexpr int kFwdWaves = 8;
constexpr int kFwdTile = 16 * kFwdWaves;
template <bool SAVE>
__global__ __launch_bounds__(64 * kFwdWaves) void k_net_forward(NetView nv, PosSrc ps, int64_t B, float* __restrict__ y,
                                                                float* __restrict__ Z, int64_t zld) {
  __shared__ __align__(16) __bf16 Wl[3 * kW * kLdh];
  __shared__ __align__(16) __bf16 H[kFwdTile * kLdh];
  __shared__ float U[kFwdTile][3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < 3 * kW * kW / 8; e += 64 * kFwdWaves) {
    const int row = e / (kW / 8), c8 = e % (kW / 8);   // row = layer * 128 + out
    *reinterpret_cast<bf16x8*>(Wl + row * kLdh + 8 * c8) = *reinterpret_cast<const bf16x8*>(nv.Wb + row * kW + 8 * c8);
  }
  const int r0 = 16 * wave + 4 * (lane >> 4), c0 = lane & 15;
  const int64_t ntiles = ceil_div(B, kFwdTile);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t s0 = tile * kFwdTile;
    __syncthreads();   // the previous tile is done with U and H (and the weights are in)
    if (tid < kFwdTile) {
      const int64_t s = s0 + tid;
      double x[3] = {0.0, 0.0, 0.0};
      const bool ok = s < B && sample_pos(ps, s, x);
      U[tid][0] = ok ? (float)((x[0] - nv.cx) * nv.scale) : 0.0f;
      U[tid][1] = ok ? (float)((x[1] - nv.cy) * nv.scale) : 0.0f;
      U[tid][2] = ok ? (float)((x[2] - nv.cz) * nv.scale) : 0.0f;
    }
    __syncthreads();
    {
      const int j = tid & (kW - 1);
      const float w0 = nv.P[kOffW1 + 3 * j], w1 = nv.P[kOffW1 + 3 * j + 1], w2 = nv.P[kOffW1 + 3 * j + 2];
      const float bj = nv.P[kOffB1 + j];
      constexpr int kRowsPer = 64 * kFwdWaves / kW;
      for (int q = 0; q < kFwdTile / kRowsPer; ++q) {
        const int i = (tid >> 7) + kRowsPer * q;
        const float z = fmaf(w2, U[i][2], fmaf(w1, U[i][1], fmaf(w0, U[i][0], bj)));
        if (SAVE && s0 + i < B) Z[(s0 + i) * kW + j] = z;
        H[i * kLdh + j] = (__bf16)silu(z);
      }
    }
    __syncthreads();
    f32x4 acc[8];
    for (int L = 0; L < 3; ++L) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float b = nv.P[kOffB[L] + 16 * t + c0];
        acc[t] = f32x4{b, b, b, b};
      }
      mma_rows16(H + 16 * wave * kLdh, kLdh, Wl + L * kW * kLdh, kLdh, kW, acc);
      // the wave's own rows: nothing else reads them, and its reads are done
      // (every value stored below depends on all of them)
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int row = r0 + s, col = 16 * t + c0;
          const float z = acc[t][s];
          if (SAVE && s0 + row < B) Z[(int64_t)(L + 1) * zld + (s0 + row) * kW + col] = z;
          const float h = silu(z);
          if (L < 2) H[row * kLdh + col] = (__bf16)h;
          acc[t][s] = h;
        }
    }
    // output layer: the 16 lanes of a row hold its 128 features, 8 each
    float p[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float w = nv.P[kOffW5 + 16 * t + c0];
#pragma unroll
      for (int s = 0; s < 4; ++s) p[s] = fmaf(w, acc[t][s], p[s]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
      for (int off = 8; off > 0; off >>= 1) p[s] += __shfl_xor(p[s], off);
    if (c0 == 0) {
      const float b5 = nv.P[kOffB5];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s0 + r0 + s < B) y[s0 + r0 + s] = p[s] + b5;
    }
  }
}

// Backward over 64 samples per workgroup: the gradient of
// sum_i (y_i - t_i)^2 * w_loss over the workgroup's samples (w_loss = 1/B of
// the whole batch), written whole to G[blockIdx.x]; the workgroup's squared
// error to loss[blockIdx.x].
__global__ __launch_bounds__(kNetThreads) void k_net_backward(NetView nv, PosSrc ps, int64_t B, const float* __restrict__ Z,
                                                              int64_t zld, const float* __restrict__ y,
                                                              const double* __restrict__ f, double inv_tau, float w_loss,
                                                              float* __restrict__ G, float* __restrict__ loss) {
  __shared__ __align__(16) __bf16 dZ[kTile * kLdh];
  __shared__ __align__(16) __bf16 dZT[kW * kLdt];
  __shared__ __align__(16) __bf16 HT[kW * kLdt];
  __shared__ float dZf[kTile][kW + 1];
  __shared__ float U[kTile][3];
  __shared__ float g5[kTile];
  __shared__ float part[2][kW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t s0 = (int64_t)blockIdx.x * kTile;
  float* Gb = G + (int64_t)blockIdx.x * kParams;
  if (tid < kTile) {
    const int64_t s = s0 + tid;
    double x[3] = {0.0, 0.0, 0.0};
    const bool ok = s < B && sample_pos(ps, s, x);
    U[tid][0] = ok ? (float)((x[0] - nv.cx) * nv.scale) : 0.0f;
    U[tid][1] = ok ? (float)((x[1] - nv.cy) * nv.scale) : 0.0f;
    U[tid][2] = ok ? (float)((x[2] - nv.cz) * nv.scale) : 0.0f;
    const float e = s < B ? y[s] - (float)(f[s] * inv_tau) : 0.0f;
    g5[tid] = 2.0f * w_loss * e;
    dZf[tid][0] = e * e;     // scratch for the loss sum
  }
  __syncthreads();
  if (tid == 0) {
    float acc = 0.0f;
    for (int i = 0; i < kTile; ++i) acc += dZf[i][0];
    loss[blockIdx.x] = acc;
  }
  __syncthreads();
  auto zval = [&](int layer, int i, int j) -> float {
    return s0 + i < B ? Z[(int64_t)layer * zld + (s0 + i) * kW + j] : 0.0f;
  };
  // output layer: dW5, db5, and dZ4 = g5 w5 silu'(z4)
  {
    const int j = tid & (kW - 1), half = tid >> 7;
    const float w5 = nv.P[kOffW5 + j];
    float a = 0.0f;
    for (int q = 0; q < kTile / 2; ++q) {
      const int i = half + 2 * q;
      const float z = zval(3, i, j);
      a = fmaf(g5[i], silu(z), a);
      const float d = g5[i] * w5 * silu_grad(z);
      dZf[i][j] = d;
      dZ[i * kLdh + j] = (__bf16)d;
      dZT[j * kLdt + i] = (__bf16)d;
    }
    part[half][j] = a;
  }
  __syncthreads();
  if (tid < kW) Gb[kOffW5 + tid] = part[0][tid] + part[1][tid];
  if (tid == 0) {
    float a = 0.0f;
    for (int i = 0; i < kTile; ++i) a += g5[i];
    Gb[kOffB5] = a;
  }
  const int r0 = 16 * wave + 4 * (lane >> 4), c0 = lane & 15;
  for (int L = 2; L >= 0; --L) {          // weights W_{L+2}, input H_{L+1} = silu(Z_L)
    // db of this layer from the float32 dZ
    if (tid < kW) {
      float a = 0.0f;
      for (int i = 0; i < kTile; ++i) a += dZf[i][tid];
      Gb[kOffB[L] + tid] = a;
    }
    {
      const int k = tid & (kW - 1), half = tid >> 7;
      for (int q = 0; q < kTile / 2; ++q) {
        const int i = half + 2 * q;
        HT[k * kLdt + i] = (__bf16)silu(zval(L, i, k));
      }
    }
    __syncthreads();
    // dW = dZ^T H: rows j of dW in two halves of 64, K = the 64 samples
    for (int p = 0; p < 2; ++p) {
      f32x4 acc[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      mma_rows16(dZT + (64 * p + 16 * wave) * kLdt, kLdt, HT, kLdt, kTile, acc);
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) Gb[kOffW[L] + (64 * p + r0 + s) * kW + 16 * t + c0] = acc[t][s];
    }
    // dH = dZ W (W^T stored by rows), then dZ of the layer below
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    mma_rows16(dZ + 16 * wave * kLdh, kLdh, nv.WbT + L * kW * kW, kW, kW, acc);
    __syncthreads();   // every wave is done with dZT, HT and dZf of this layer
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = r0 + s, col = 16 * t + c0;
        const float d = acc[t][s] * silu_grad(zval(L, row, col));
        dZf[row][col] = d;
        dZ[row * kLdh + col] = (__bf16)d;
        dZT[col * kLdt + row] = (__bf16)d;
      }
    __syncthreads();
  }
  // first layer from the float32 dZ1
  if (tid < kW) {
    float a = 0.0f, w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
    for (int i = 0; i < kTile; ++i) {
      const float d = dZf[i][tid];
      a += d;
      w0 = fmaf(d, U[i][0], w0);
      w1 = fmaf(d, U[i][1], w1);
      w2 = fmaf(d, U[i][2], w2);
    }
    Gb[kOffB1 + tid] = a;
    Gb[kOffW1 + 3 * tid] = w0;
    Gb[kOffW1 + 3 * tid + 1] = w1;
    Gb[kOffW1 + 3 * tid + 2] = w2;
  }
}

// Sum of the workgroups' gradients (fixed order) into grad, and, when
// adam != 0, the Adam step on the parameters.
struct AdamArgs {
  float* P;
  float* m;
  float* v;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};
__global__ void k_net_reduce(const float* __restrict__ G, int nblk, float* __restrict__ grad, int adam, AdamArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += G[(int64_t)b * kParams + p];
  if (grad) grad[p] = g;
  if (adam) {
    const float m = a.b1 * a.m[p] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[p] + (1.0f - a.b2) * g * g;
    a.m[p] = m;
    a.v[p] = v;
    a.P[p] -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
  }
}

// bf16 copies of W2..W4 and their transposes.
__global__ void k_net_bf16(const float* __restrict__ P, __bf16* __restrict__ Wb, __bf16* __restrict__ WbT) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * kW * kW) return;
  const int L = e / (kW * kW), r = e % (kW * kW), j = r / kW, k = r % kW;
  const __bf16 v = (__bf16)P[kOffW[L] + r];
  Wb[e] = v;
  WbT[L * kW * kW + k * kW + j] = v;
}

// Learned cull: y over the nodes of the support bricks (NaN where no node),
// then the kept flag of every support brick.
__global__ void k_scatter_nodes(const float* __restrict__ ysup, const int64_t* __restrict__ bricks, int64_t nact,
                                GridDesc gd, float* __restrict__ ygrid) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nact * kGroup) return;
  const int64_t b = bricks[s / kGroup];
  const int l = (int)(s % kGroup);
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  const int64_t i = bx * 4 + (l & 3), j = by * 2 + ((l >> 2) & 1), k = bz * 2 + (l >> 3);
  if (i < gd.n[0] && j < gd.n[1] && k < gd.n[2]) ygrid[i + gd.n[0] * (j + gd.n[1] * k)] = ysup[s];
}

__global__ void k_fill_nan(float* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = __builtin_nanf("");
}

// The keep test in three separable passes.  Signs of the support nodes as
// bits (1 positive, 2 negative, 4 |y| < e_val; NaN nodes, outside the
// support, carry none); then, along x, y and z in turn, every node ORs the
// sign bits of the nodes within `reach` steps, so that after the three
// passes it holds the signs of its (2 reach + 1)^3 neighbourhood.
__global__ void k_sign_bits(const float* __restrict__ ygrid, int64_t total, float e_val, uint8_t* __restrict__ bits) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float v = ygrid[i];
  bits[i] = (uint8_t)((v > 0.0f ? 1 : 0) | (v < 0.0f ? 2 : 0) | (fabsf(v) < e_val ? 4 : 0));
}

// dir 0, 1, 2: x, y, z.  Only the two sign bits are spread.
__global__ void k_spread_signs(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, GridDesc gd, int dir,
                               int reach) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = gd.n[0] * gd.n[1] * gd.n[2];
  if (idx >= total) return;
  const int64_t stride = dir == 0 ? 1 : dir == 1 ? gd.n[0] : gd.n[0] * gd.n[1];
  const int64_t c = dir == 0 ? idx % gd.n[0] : dir == 1 ? (idx / gd.n[0]) % gd.n[1] : idx / (gd.n[0] * gd.n[1]);
  const int64_t lo = max<int64_t>(0, c - reach), hi = min<int64_t>(gd.n[dir] - 1, c + reach);
  uint8_t acc = 0;
  for (int64_t q = lo; q <= hi; ++q) acc |= in[idx + (q - c) * stride] & 3;
  out[idx] = acc;
}

// One thread per node of the support bricks: kept when |y| < e_val or a
// support node of the opposite sign lies in its neighbourhood.
__global__ void k_cull_keep(const uint8_t* __restrict__ own, const uint8_t* __restrict__ hood,
                            const int64_t* __restrict__ bricks, int64_t nact, GridDesc gd, int64_t* __restrict__ keep) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nact * kGroup) return;
  const int64_t b = bricks[s / kGroup];
  const int l = (int)(s % kGroup);
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  const int64_t i = bx * 4 + (l & 3), j = by * 2 + ((l >> 2) & 1), k = bz * 2 + (l >> 3);
  if (!(i < gd.n[0] && j < gd.n[1] && k < gd.n[2])) return;
  const int64_t n = i + gd.n[0] * (j + gd.n[1] * k);
  const uint8_t o = own[n], h = hood[n];
  const bool hit = (o & 4) || ((o & 1) && (h & 2)) || ((o & 2) && (h & 1));
  if (hit) keep[s / kGroup] = 1;   // benign race: every writer stores 1
}

// Culled support bricks take tau * y.
__global__ void k_cull_fill(const float* __restrict__ ysup, const int64_t* __restrict__ bricks,
                            const int64_t* __restrict__ keep, int64_t nact, GridDesc gd, float tau,
                            float* __restrict__ out) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nact * kGroup || keep[s / kGroup]) return;
  const int64_t b = bricks[s / kGroup];
  const int l = (int)(s % kGroup);
  const int64_t bx = b % gd.nb[0], by = (b / gd.nb[0]) % gd.nb[1], bz = b / (gd.nb[0] * gd.nb[1]);
  const int64_t i = bx * 4 + (l & 3), j = by * 2 + ((l >> 2) & 1), k = bz * 2 + (l >> 3);
  if (i < gd.n[0] && j < gd.n[1] && k < gd.n[2]) out[i + gd.n[0] * (j + gd.n[1] * k)] = tau * ysup[s];
}

__global__ void k_gather_kept(const int64_t* __restrict__ bricks, const int64_t* __restrict__ keep,
                              const int64_t* __restrict__ pos, int64_t nact, int64_t* __restrict__ kept) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < nact && keep[q]) kept[pos[q]] = bricks[q];
}

__global__ void k_fill_i64_m(int64_t* p, int64_t v, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

unsigned blocks_for(int64_t n, int t = 256) { return (unsigned)std::max<int64_t>(1, ceil_div(n, t)); }

// One forward workgroup per compute unit (its LDS holds the weights), or
// fewer when there are fewer tiles.
unsigned fwd_blocks(int64_t B) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    RBF_HIP(hipGetDevice(&dev));
    RBF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(B, kFwdTile), std::max(cus, 1)));
}

NetView view(const NetData& d) { return NetView{d.P, d.Wb, d.WbT, d.centre[0], d.centre[1], d.centre[2], d.scale}; }

}  // namespace

int net_param_count() { return kParams; }

NetData* net_create(const float* host_params, const double centre[3], double scale, double tau, hipStream_t s) {
  NetData* d = new NetData();
  d->P = dalloc<float>(kParams);
  d->m = dalloc<float>(kParams);
  d->v = dalloc<float>(kParams);
  d->Wb = reinterpret_cast<__bf16*>(dalloc<uint16_t>(3 * kW * kW));
  d->WbT = reinterpret_cast<__bf16*>(dalloc<uint16_t>(3 * kW * kW));
  for (int k = 0; k < 3; ++k) d->centre[k] = centre[k];
  d->scale = scale;
  d->tau = tau;
  RBF_HIP(hipMemcpyAsync(d->P, host_params, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
  fill_f32(d->m, 0.0f, kParams, s);
  fill_f32(d->v, 0.0f, kParams, s);
  hipLaunchKernelGGL(k_net_bf16, dim3(blocks_for(3 * kW * kW)), dim3(256), 0, s, d->P, d->Wb, d->WbT);
  RBF_HIP(hipGetLastError());
  return d;
}

void free_net(NetData* d) {
  if (!d) return;
  for (void* p : {(void*)d->P, (void*)d->m, (void*)d->v, (void*)d->Wb, (void*)d->WbT}) dfree(p);
  delete d;
}

void net_get(const NetData& d, float* host_params, hipStream_t s) {
  RBF_HIP(hipMemcpyAsync(host_params, d.P, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
}

void net_forward(const NetData& d, const double* X, int64_t B, float* y, hipStream_t s) {
  if (B <= 0) return;
  PosSrc ps{X, nullptr, GridDesc{}};
  hipLaunchKernelGGL(k_net_forward<false>, dim3(fwd_blocks(B)), dim3(64 * kFwdWaves), 0, s, view(d), ps, B, y,
                     (float*)nullptr, (int64_t)0);
  RBF_HIP(hipGetLastError());
}

// Gradient of the batch loss mean (y - f/tau)^2 into grad (device, kParams),
// and the loss itself; with adam, the Adam step too (step t counts from 1).
double net_step(NetData& d, const double* X, const double* f, int64_t B, float* grad, bool adam, double lr,
                hipStream_t s) {
  const int64_t nblk = ceil_div(B, kTile);
  float* Z = talloc<float>(4 * B * kW);
  float* y = talloc<float>(B);
  float* G = talloc<float>(nblk * kParams);
  float* loss = talloc<float>(nblk);
  PosSrc ps{X, nullptr, GridDesc{}};
  const NetView nv = view(d);
  hipLaunchKernelGGL(k_net_forward<true>, dim3(fwd_blocks(B)), dim3(64 * kFwdWaves), 0, s, nv, ps, B, y, Z, B * kW);
  hipLaunchKernelGGL(k_net_backward, dim3((unsigned)nblk), dim3(kNetThreads), 0, s, nv, ps, B, Z, B * kW, y, f,
                     1.0 / d.tau, (float)(1.0 / (double)B), G, loss);
  AdamArgs a{d.P, d.m, d.v, (float)lr, 0.9f, 0.999f, 1e-8f, 1.0f, 1.0f};
  if (adam) {
    d.step += 1;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)d.step));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)d.step));
  }
  hipLaunchKernelGGL(k_net_reduce, dim3(blocks_for(kParams)), dim3(256), 0, s, G, (int)nblk, grad, adam ? 1 : 0, a);
  if (adam) hipLaunchKernelGGL(k_net_bf16, dim3(blocks_for(3 * kW * kW)), dim3(256), 0, s, d.P, d.Wb, d.WbT);
  RBF_HIP(hipGetLastError());
  std::vector<float> hl((size_t)nblk);
  RBF_HIP(hipMemcpyAsync(hl.data(), loss, sizeof(float) * nblk, hipMemcpyDeviceToHost, s));
  RBF_HIP(hipStreamSynchronize(s));
  double L = 0.0;
  for (float v : hl) L += v;
  for (void* p : {(void*)Z, (void*)y, (void*)G, (void*)loss}) temp_free(p);
  return L / (double)B;
}

void net_eval_grid_culled(const Ctx& c, const NetData& d, const double* w_sorted, const rbf_grid& g, float* out,
                          double e_val, int reach, NetCullStats* st, hipStream_t s) {
  const GridDesc gd = grid_desc(g);
  const int64_t total = g.dims[0] * g.dims[1] * g.dims[2];
  fill_f32(out, 0.0f, total, s);
  int64_t* sup = nullptr;
  const int64_t nsup = support_bricks(c, g, &sup, s);
  int64_t* all = nullptr;
  if (!sup) {   // no cutoff: every brick
    std::vector<int64_t> h((size_t)nsup);
    for (int64_t b = 0; b < nsup; ++b) h[b] = b;
    all = talloc<int64_t>(nsup);
    RBF_HIP(hipMemcpyAsync(all, h.data(), sizeof(int64_t) * nsup, hipMemcpyHostToDevice, s));
    sup = all;
  }
  st->support_bricks = nsup;
  st->kept_bricks = 0;
  if (nsup > 0) {
    // the network on every node of the support
    float* ysup = talloc<float>(nsup * kGroup);
    PosSrc ps{nullptr, sup, gd};
    hipLaunchKernelGGL(k_net_forward<false>, dim3(fwd_blocks(nsup * kGroup)), dim3(64 * kFwdWaves), 0, s, view(d), ps,
                       nsup * kGroup, ysup, (float*)nullptr, (int64_t)0);
    float* ygrid = talloc<float>(total);
    hipLaunchKernelGGL(k_fill_nan, dim3(blocks_for(total)), dim3(256), 0, s, ygrid, total);
    hipLaunchKernelGGL(k_scatter_nodes, dim3(blocks_for(nsup * kGroup)), dim3(256), 0, s, ysup, sup, nsup, gd, ygrid);
    uint8_t* own = talloc<uint8_t>(total);
    uint8_t* t1 = talloc<uint8_t>(total);
    uint8_t* t2 = talloc<uint8_t>(total);
    hipLaunchKernelGGL(k_sign_bits, dim3(blocks_for(total)), dim3(256), 0, s, ygrid, total, (float)e_val, own);
    hipLaunchKernelGGL(k_spread_signs, dim3(blocks_for(total)), dim3(256), 0, s, own, t1, gd, 0, reach);
    hipLaunchKernelGGL(k_spread_signs, dim3(blocks_for(total)), dim3(256), 0, s, t1, t2, gd, 1, reach);
    hipLaunchKernelGGL(k_spread_signs, dim3(blocks_for(total)), dim3(256), 0, s, t2, t1, gd, 2, reach);
    int64_t* keep = talloc<int64_t>(nsup);
    hipLaunchKernelGGL(k_fill_i64_m, dim3(blocks_for(nsup)), dim3(256), 0, s, keep, (int64_t)0, nsup);
    hipLaunchKernelGGL(k_cull_keep, dim3(blocks_for(nsup * kGroup)), dim3(256), 0, s, own, t1, sup, nsup, gd, keep);
    hipLaunchKernelGGL(k_cull_fill, dim3(blocks_for(nsup * kGroup)), dim3(256), 0, s, ysup, sup, keep, nsup, gd,
                       (float)d.tau, out);
    RBF_HIP(hipGetLastError());
    // the exact sum on the kept bricks
    int64_t* pos = talloc<int64_t>(nsup);
    scan_exclusive_i64(keep, pos, nsup, s);
    int64_t last_pos = 0, last_keep = 0;
    RBF_HIP(hipMemcpyAsync(&last_pos, pos + (nsup - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipMemcpyAsync(&last_keep, keep + (nsup - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    const int64_t nkeep = last_pos + last_keep;
    st->kept_bricks = nkeep;
    int64_t* kept = talloc<int64_t>(nkeep);
    hipLaunchKernelGGL(k_gather_kept, dim3(blocks_for(nsup)), dim3(256), 0, s, sup, keep, pos, nsup, kept);
    RBF_HIP(hipGetLastError());
    if (brick_sum_applies(c, g)) {
      // the bricks walk their candidate sources directly, as in the plain grid
      brick_sum_f32(c, g, kept, nkeep, w_sorted, out, &st->useful_pairs, &st->examined_pairs, s);
    } else {
      TargetSet ts;
      brick_targets(c, g, kept, nkeep, ts, s);
      if (ts.n_groups > 0) pairsum_f32(c, ts, w_sorted, true, out, s);
      RBF_HIP(hipStreamSynchronize(s));
      st->useful_pairs = ts.useful;
      st->examined_pairs = ts.list_entries * kGroup;
      free_targets(ts);
    }
    for (void* p : {(void*)ysup, (void*)ygrid, (void*)own, (void*)t1, (void*)t2, (void*)keep, (void*)pos,
                    (void*)kept})
      temp_free(p);
  }
  temp_free(sup);
}

}  // namespace rbf
