// Learned prescreen: an ensemble of MLPs x -> GELU(W1 x + b1) -> GELU(W2 h1 +
// b2) -> w3 . h2 + b3, trained on the search's own evaluations with the
// mean-squared error and Adam (Kingma & Ba 2015, Alg. 1), then used to rank
// a large candidate pool by ensemble expected improvement (mean and
// population standard deviation over the members).
//
// Precision: float32 master weights and Adam moments; bfloat16 copies of the
// weights and bfloat16 activations as matrix-core operands, float32
// accumulation.  Rounding to bfloat16 happens at exactly these points: the
// inputs x, the weight copies W1/W2/w3, h1 = GELU(pre1), h2 = GELU(pre2), and
// in the backward pass dpre2 and dpre1 where they feed a product (bias
// gradients use the unrounded values).
//
// Layout: activations are sample-major [member][sample][feature]; weights are
// [member][out][in].  Every matrix-core product is an "NT" product
// C[M][N] = A[M][K] B[N][K]^T with K contiguous in both operands; the
// backward products that contract over samples read feature-major copies
// ([member][feature][sample]) written by the producing kernels.
#include <cmath>
#include <cstring>

#include "gpbo_internal.h"
#include "score_common.h"

namespace gpbo {

using namespace sc;

namespace {

constexpr int MT = 64;  // samples per forward / backward workgroup

__device__ __forceinline__ float bfr(float x) { return __uint_as_float((unsigned)f2bf(x) << 16); }
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// GELU u Phi(u) and its derivative Phi(u) + u phi(u).  The normal tail
// Phi(-a), a = |u|, is exp2(p(a)) with p the degree-5 polynomial, p(0) = -1
// (Phi(0) = 1/2 exactly), fitted to log2 Phi(-a) on [0, 6] for the smallest
// absolute error of Phi(-a) by gelu_tail_fit.py: absolute error <= 3.0e-7
// (relative <= 1.8e-6 for a <= 1, where most activations lie and where a
// relative error turns directly into bfloat16 rounding flips).  Beyond
// a = 6 p keeps decreasing (p(6) = -30.25; the float32 Horner value is
// monotone there and reaches -inf, never NaN, for finite a), so the tail
// needs no clamp: below 8e-10 there, where Phi(-a) < 1e-9.  One v_exp_f32
// and no reciprocal per activation.
__device__ __forceinline__ float normal_tail(float u) {
  const float m = fabsf(u);
  float p = fmaf(m, -0.0005204600165598094f, 0.0073975189588963985f);
  p = fmaf(m, p, -0.05256125330924988f);
  p = fmaf(m, p, -0.4592546820640564f);
  p = fmaf(m, p, -1.1510913372039795f);
  p = fmaf(m, p, -1.0f);
  return __builtin_amdgcn_exp2f(p);
}
struct NormalCdf {
  float Phi, e;  // Phi(u) and exp(-u^2 / 2)
};
__device__ __forceinline__ NormalCdf normal_cdf(float u) {
  const float tail = normal_tail(u);  // Phi(-|u|)
  const float e = __builtin_amdgcn_exp2f((u * (-0.5f * 1.44269504088896340736f)) * u);
  return {u >= 0.0f ? 1.0f - tail : tail, e};
}
// GELU u Phi(u) = max(u, 0) - |u| Phi(-|u|): the same value for either sign,
// without a select on the sign.
__device__ __forceinline__ float gelu(float u) {
  // the max needs a canonical operand (an accumulator value is not known to
  // be one)
  const float c = __builtin_canonicalizef(u);
  return fmaf(-fabsf(c), normal_tail(c), fmaxf(c, 0.0f));
}
// 2 GELU(u) = (u + |u|) - |u| 2Phi(-|u|), with 2Phi(-a) = exp2(p(a) + 1)
// (the same polynomial, its constant term -1 + 1 = 0): one instruction fewer
// than GELU and no canonicalisation (u + |u| needs none).  The prescreen
// pass uses it with the next layer's weights halved (exact in bfloat16), so
// every product of the next layer is the one of GELU times the full weight.
__device__ __forceinline__ float gelu2(float u) {
  const float m = fabsf(u);
  float p = fmaf(m, -0.0005204600165598094f, 0.0073975189588963985f);
  p = fmaf(m, p, -0.05256125330924988f);
  p = fmaf(m, p, -0.4592546820640564f);
  p = fmaf(m, p, -1.1510913372039795f);
  p = m * p;
  return fmaf(-m, __builtin_amdgcn_exp2f(p), u + m);
}
__device__ __forceinline__ float gelu_grad(float u) {
  const NormalCdf c = normal_cdf(u);
  return c.Phi + u * c.e * 0.39894228040143267794f;
}

// Two floats rounded to bfloat16 (round to nearest even, NaN kept) and packed,
// the first in the low half: one v_cvt_pk_bf16_f32.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

struct MlpDev {
  int E, D, H;
  int DP;                  // D rounded up to the matrix-core depth (32 or 64)
  int64_t P;               // parameters per member
  float* master;           // E x P
  float* mom1;             // E x P
  float* mom2;             // E x P
  unsigned short* W1b;     // E x H x DP (rows zero-padded from D to DP)
  unsigned short* W2b;     // E x H x H  [out][in]
  unsigned short* W2Tb;    // E x H x H  [in][out]
  unsigned short* w3b;     // E x H
  unsigned short* W2hb;    // E x H x H  [out][in], 0.5 W2 (the prescreen pass)
  unsigned short* w3hb;    // E x H, 0.5 w3 (the prescreen pass)
  int* step;               // [0] Adam steps taken, [1] steps taken before this training call
};

__device__ __forceinline__ const float* pW1(const MlpDev& M, int e) { return M.master + e * M.P; }
__device__ __forceinline__ int64_t off_b1(const MlpDev& M) { return (int64_t)M.H * M.D; }
__device__ __forceinline__ int64_t off_W2(const MlpDev& M) { return off_b1(M) + M.H; }
__device__ __forceinline__ int64_t off_b2(const MlpDev& M) { return off_W2(M) + (int64_t)M.H * M.H; }
__device__ __forceinline__ int64_t off_w3(const MlpDev& M) { return off_b2(M) + M.H; }
__device__ __forceinline__ int64_t off_b3(const MlpDev& M) { return off_w3(M) + M.H; }

// bfloat16 copies of the master weights (and the transposed W2).
__global__ void k_mlp_cast(MlpDev M) {
  const int e = blockIdx.y;
  const float* p = M.master + e * M.P;
  const int H = M.H, D = M.D;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H * H; i += gridDim.x * blockDim.x) {
    const int o = i / H, in = i % H;
    const unsigned short b = f2bf(p[off_W2(M) + i]);
    M.W2b[(int64_t)e * H * H + i] = b;
    M.W2Tb[(int64_t)e * H * H + (int64_t)in * H + o] = b;
    M.W2hb[(int64_t)e * H * H + i] = f2bf(0.5f * p[off_W2(M) + i]);
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H * M.DP; i += gridDim.x * blockDim.x) {
    const int h = i / M.DP, k = i % M.DP;
    M.W1b[(int64_t)e * H * M.DP + i] = k < D ? f2bf(p[h * D + k]) : (unsigned short)0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H; i += gridDim.x * blockDim.x) {
    M.w3b[(int64_t)e * H + i] = f2bf(p[off_w3(M) + i]);
    M.w3hb[(int64_t)e * H + i] = f2bf(0.5f * p[off_w3(M) + i]);
  }
}

// Forward of MT samples through one member (blockIdx.y), 256 threads, both
// dense layers on the bfloat16 matrix cores:
//   layer 1: pre1 = x W1^T + b1 (x and W1 staged in LDS, zero-padded to DP),
//   each wave 64 samples x 64 hidden units; h1 = bf16(GELU(pre1)) into an
//   LDS tile;
//   layer 2: pre2 = h1 W2^T + b2, each wave 64 samples x 64 outputs;
//   epilogue h2 = bf16(GELU(pre2)), out = w3 . h2 + b3.
// With TRAIN the kernel also writes pre1, h1 (feature-major, the operand of
// the layer-2 weight gradient) and pre2.
struct FwdOut {
  float* out;               // E x n
  float* pre1;              // E x n x H (TRAIN)
  unsigned short* h1T;      // E x H x ldt (TRAIN)
  float* pre2;              // E x n x H (TRAIN)
  int64_t ldt;              // row stride of the feature-major copies (elements)
};

__device__ __forceinline__ int fwd_ldx(int DP) { return DP + 8; }  // bf16 row stride of x / W1 tiles

// Work items: the E members of every 64-sample tile.  Workgroup b runs on
// XCD b % 8 (round-robin dispatch); item q takes XCD x = q % 8, member
// (q / 8) % E and tile 8 (q / 8E) + x, so the E members of a tile run back to
// back on one XCD and read its samples from that XCD's L2 once (all members'
// W2, 640 KB, stay resident there too).  Workgroup b takes items b, b +
// grid, ... (grid a multiple of 8); a grid of one workgroup per item is the
// plain launch, a smaller one keeps part of every compute unit free for
// other streams' work.  Items past the last tile are skipped.
__host__ __device__ inline int64_t fwd_items(int ntile, int E) {
  return ((int64_t)(ntile + 7) / 8) * 8 * E;
}
// bump (training steps that apply Adam): the first thread advances the step
// counter, which this step's Adam launch then reads (nothing in between
// does).
template <bool TRAIN>
__global__ void __launch_bounds__(256, 2) k_mlp_fwd(MlpDev M, int64_t n, const float* __restrict__ X,
                                                 FwdOut O, int ntile, int bump) {
  if (TRAIN && bump && blockIdx.x == 0 && threadIdx.x == 0) M.step[0] += 1;
  extern __shared__ __align__(16) unsigned char sm[];
  const int H = M.H, D = M.D, DP = M.DP;
  const int t = threadIdx.x, lane = t % 64, wave = wave_id();
  const int ldh = H + 8;  // bf16 row stride of the h1 tile (16-byte rows, skewed banks)
  const int ldx = fwd_ldx(DP);
  unsigned short* hA = (unsigned short*)sm;  // [MT][ldh]
  unsigned short* xb = hA + MT * ldh;        // [MT][ldx], samples in bfloat16, zero from column D
  float* red = (float*)(xb + MT * ldx);      // [4][MT]
  for (int q = t; q < MT * (DP - D); q += 256) xb[(q / (DP - D)) * ldx + D + q % (DP - D)] = 0;
  const int64_t items = fwd_items(ntile, M.E);
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const int64_t local = item / 8;
    const int e = (int)(local % M.E);
    const int64_t tile = (local / M.E) * 8 + item % 8;
    if (tile >= ntile) continue;
    const int64_t i0 = tile * MT;
    const float* p = M.master + e * M.P;
    // the item's samples, rounded to bfloat16 (four columns per store when
    // D is a multiple of 4; rows past n are zeros)
    if (D % 4 == 0) {
      const int D4 = D / 4;
      for (int q = t; q < MT * D4; q += 256) {
        const int r = q / D4, c = 4 * (q % D4);
        const int64_t i = i0 + r;
        const float4 v = i < n ? *(const float4*)(X + i * D + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        *(uint2*)(xb + r * ldx + c) = make_uint2(pack_bf16x2(v.x, v.y), pack_bf16x2(v.z, v.w));
      }
    } else {
      for (int q = t; q < MT * D; q += 256) {
        const int r = q / D, k = q % D;
        const int64_t i = i0 + r;
        xb[r * ldx + k] = i < n ? f2bf(X[i * D + k]) : (unsigned short)0;
      }
    }
    __syncthreads();
    // W1 (bfloat16, zero-padded rows of DP) is read as the matrix-core operand
    // straight from global memory: it is 16 KB per member and stays in L2
    const unsigned short* W1 = M.W1b + (int64_t)e * H * DP;
    const int ocol = wave * 64;  // this wave's 64 columns (hidden units / outputs)
    // the accumulators start from the biases: lane's entry r of block b is unit
    // ocol + 16b + 4(lane/16) + r for every sample block; the first
    // contraction step takes them as its addend, so they are not copied into
    // the accumulators first
    f4 bias[4];
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int h0 = ocol + b * 16 + 4 * (lane / 16);
      bias[b] = f4{p[off_b1(M) + h0], p[off_b1(M) + h0 + 1], p[off_b1(M) + h0 + 2],
                   p[off_b1(M) + h0 + 3]};
    }
    f4 acc[4][4];
    // layer 1, transposed: C[h][s] = sum_k W1[h][k] x[s][k] (A = W1 rows, B =
    // samples), so that a lane's four accumulators are four consecutive hidden
    // units of one sample: they round to bfloat16 in pairs and go to the
    // sample-major h1 tile as one 8-byte store
    auto step1 = [&](int k0, bool first) {
      us8 av[4], bv[4];
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        av[a] = *(const us8*)(xb + (a * 16 + lane % 16) * ldx + k0 + 8 * (lane / 16));
      #pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *(const us8*)(W1 + (ocol + b * 16 + lane % 16) * DP + k0 + 8 * (lane / 16));
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, bv[b]),
                                                              __builtin_bit_cast(bf8, av[a]),
                                                              first ? bias[b] : acc[a][b], 0, 0, 0);
    };
    step1(0, true);
    for (int k0 = 32; k0 < DP; k0 += 32) step1(k0, false);
    // layer-1 epilogue: lane holds hidden units h0 .. h0+3 (h0 = ocol + 16b +
    // 4(lane/16)) of sample 16a + lane%16
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int h0 = ocol + b * 16 + 4 * (lane / 16);
      #pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = a * 16 + lane % 16;
        // training: GELU (its h1 feeds the backward); prescreen: 2 GELU, the
        // next layer's weights halved
        float pre[4], g[4];
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
          pre[r] = acc[a][b][r];
          g[r] = TRAIN ? gelu(pre[r]) : gelu2(pre[r]);
        }
        const uint2 hb = make_uint2(pack_bf16x2(g[0], g[1]), pack_bf16x2(g[2], g[3]));
        *(uint2*)(hA + row * ldh + h0) = hb;
        if (TRAIN && i0 + row < n) {
          const int64_t o = ((int64_t)e * n + i0 + row) * H + h0;
          *(float4*)(O.pre1 + o) = make_float4(pre[0], pre[1], pre[2], pre[3]);
        }
      }
    }
    __syncthreads();
    if (TRAIN) {  // feature-major copy, coalesced along the samples
      for (int q = t; q < H * MT; q += 256) {
        const int h = q / MT, r = q % MT;
        if (i0 + r < n) O.h1T[((int64_t)e * H + h) * O.ldt + i0 + r] = hA[r * ldh + h];
      }
    }
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j0 = ocol + b * 16 + 4 * (lane / 16);
      bias[b] = f4{p[off_b2(M) + j0], p[off_b2(M) + j0 + 1], p[off_b2(M) + j0 + 2],
                   p[off_b2(M) + j0 + 3]};
    }
    // layer 2, transposed the same way: C[j][s] = sum_k W2[j][k] h1[s][k];
    // wave w computes outputs [64w, 64w + 64) for the MT samples
    const unsigned short* W2 = (TRAIN ? M.W2b : M.W2hb) + (int64_t)e * H * H;
    auto step2 = [&](int k0, bool first) {
      us8 av[4], bv[4];
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        av[a] = *(const us8*)(hA + (a * 16 + lane % 16) * ldh + k0 + 8 * (lane / 16));
      #pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *(const us8*)(W2 + (int64_t)(ocol + b * 16 + lane % 16) * H + k0 + 8 * (lane / 16));
      #pragma unroll
      for (int a = 0; a < 4; ++a)
        #pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, bv[b]),
                                                              __builtin_bit_cast(bf8, av[a]),
                                                              first ? bias[b] : acc[a][b], 0, 0, 0);
    };
    step2(0, true);
    for (int k0 = 32; k0 < H; k0 += 32) step2(k0, false);
    // epilogue: lane holds outputs j0 .. j0+3 (j0 = ocol + 16b + 4(lane/16)) of
    // sample 16a + lane%16; h2 = bf16(GELU(pre2)) and its dot with w3 stay in
    // the lane until the four lane groups are summed
    float rowsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j0 = ocol + b * 16 + 4 * (lane / 16);
      // w3 of the lane's four outputs as two bfloat16 pairs (halved for the
      // prescreen's 2 GELU)
      const uint2 w3p = *(const uint2*)((TRAIN ? M.w3b : M.w3hb) + (int64_t)e * H + j0);
      #pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = a * 16 + lane % 16;
        float pre[4], g[4];
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
          pre[r] = acc[a][b][r];
          g[r] = TRAIN ? gelu(pre[r]) : gelu2(pre[r]);
        }
        if (TRAIN && i0 + row < n)
          *(float4*)(O.pre2 + ((int64_t)e * n + i0 + row) * H + j0) =
              make_float4(pre[0], pre[1], pre[2], pre[3]);
        const unsigned lo = pack_bf16x2(g[0], g[1]), hi = pack_bf16x2(g[2], g[3]);
        // h2 . w3 on the bfloat16 pairs (the products are exact in float32):
        // one v_dot2c_f32_bf16 per pair
        float v = rowsum[a];
        v = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, lo),
                                            __builtin_bit_cast(bf16x2_t, w3p.x), v, false);
        v = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, hi),
                                            __builtin_bit_cast(bf16x2_t, w3p.y), v, false);
        rowsum[a] = v;
      }
    }
    // sum over the four lane groups, then over the four waves
    #pragma unroll
    for (int a = 0; a < 4; ++a) {
      float v = rowsum[a];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (lane < 16) red[wave * MT + a * 16 + lane] = v;
    }
    __syncthreads();
    if (t < MT && i0 + t < n) {
      const float o = red[t] + red[MT + t] + red[2 * MT + t] + red[3 * MT + t] + p[off_b3(M)];
      O.out[(int64_t)e * n + i0 + t] = o;
    }
    __syncthreads();  // the tiles are restaged for the next item
  }
}

// Output-layer backward for MT samples of one member: dout = 2 (out - y) / n,
// dpre2 = dout w3 GELU'(pre2) (bf16, both layouts), and per-block column sums
// for gb2 (unrounded dpre2), gw3 (dout h2) and gb3, and the squared error.
struct BwdBuf {
  unsigned short* dpre2;   // E x n x H
  unsigned short* dpre2T;  // E x H x ldt
  float* colpart;          // E x nblk x (2H + 2): gb2, gw3, gb3, loss
  int64_t ldt;
};
__global__ void __launch_bounds__(256) k_mlp_bwd_out(MlpDev M, int64_t n, const float* __restrict__ y,
                                                     const float* __restrict__ out,
                                                     const float* __restrict__ pre2, BwdBuf B) {
  __shared__ unsigned short tT[256][MT + 2];
  __shared__ float dout_s[MT];
  const int H = M.H;
  const int e = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * MT;
  const int t = threadIdx.x;
  const int nblk = gridDim.x;
  float* part = B.colpart + ((int64_t)e * nblk + blockIdx.x) * (2 * H + 2);
  if (t < MT) {
    const int64_t i = i0 + t;
    dout_s[t] = i < n ? 2.0f * (out[(int64_t)e * n + i] - y[i]) / (float)n : 0.0f;
  }
  __syncthreads();
  // gb3 and the squared error: the samples' terms formed in parallel (one
  // per thread of the first wave), summed in sample order by one thread
  static_assert(MT <= 64, "one sample per lane of the first wave");
  __shared__ float sq_s[MT];
  if (t < MT) {
    const int64_t i = i0 + t;
    float sq = 0.0f;
    if (i < n) {
      const float d = out[(int64_t)e * n + i] - y[i];
      sq = d * d;
    }
    sq_s[t] = sq;
  }
  __syncthreads();
  if (t == 0) {
    float g3 = 0.0f, ls = 0.0f;
    for (int r = 0; r < MT; ++r) {
      g3 += dout_s[r];
      ls += sq_s[r];
    }
    part[2 * H] = g3;
    part[2 * H + 1] = ls;
  }
  for (int j = t; j < H; j += 256) {
    const float w3 = bf2f(M.w3b[(int64_t)e * H + j]);
    float gb2 = 0.0f, gw3 = 0.0f;
    // eight samples' pre-activations requested before any is used
    constexpr int U = 8;
    for (int r0 = 0; r0 < MT; r0 += U) {
      float pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + r0 + u;
        pv[u] = i < n ? pre2[((int64_t)e * n + i) * H + j] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = r0 + u;
        const int64_t i = i0 + r;
        unsigned short db = 0;
        if (i < n) {
          const float pre = pv[u];
          const float d = dout_s[r] * w3 * gelu_grad(pre);
          gb2 += d;
          gw3 = fmaf(dout_s[r], bfr(gelu(pre)), gw3);
          db = f2bf(d);
          B.dpre2[((int64_t)e * n + i) * H + j] = db;
        }
        tT[j][r] = db;
      }
    }
    part[j] = gb2;
    part[H + j] = gw3;
  }
  __syncthreads();
  // feature-major copy, coalesced along the samples
  for (int q = t; q < H * MT; q += 256) {
    const int j = q / MT, r = q % MT;
    if (i0 + r < n) B.dpre2T[((int64_t)e * H + j) * B.ldt + i0 + r] = tT[j][r];
  }
}

// C[M][N] = A[M][K] B[N][K]^T on the bfloat16 matrix cores, batched over the
// members (blockIdx.z) and split over K (blockIdx.y); WM x WN waves per
// workgroup, a 32 x 32 tile per wave (waves of one workgroup share operand
// rows in L1), operands read straight from L2 (16 bytes per lane).  Epilogue: STORE writes C to out[split][member][M][N]; DPRE1 writes
// C * GELU'(pre1) to out[member][M][N] (one split).
enum { EPI_STORE = 0, EPI_DPRE1 = 1 };

struct Gemm {
  const unsigned short* A;
  const unsigned short* B;
  int64_t sA, sB;   // member strides (elements)
  int64_t lda, ldb; // row strides (elements, multiples of 8)
  int M, N, K;
  int kchunk;       // K per split
  float* out;
  const float* pre1;
  unsigned short* dpre1T;  // DPRE1: bf16(dpre1), feature-major [member][N][ldo]
  int64_t ldo;
  float* b1part;           // DPRE1: per 32-row block column sums of dpre1 [member][M/32][N]
};
template <int EPI, int WM, int WN, int KU>
__global__ void __launch_bounds__(64 * WM * WN) k_gemm_nt(Gemm g) {
  // XCD-aware order: workgroup b of the launch runs on XCD b % 8 (round-robin
  // dispatch); each XCD takes a contiguous range of the (tile, split,
  // member) order instead, so the tiles that share operand rows (one member
  // and split of a weight gradient, one row block of dh1) fetch them into
  // one L2 rather than into all eight (gW2 with one-wave workgroups fetched
  // 4.6 times its 21 MB of operands from HBM without it)
  const unsigned nwg = gridDim.x * gridDim.y * gridDim.z;
  unsigned wg = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (nwg % 8 == 0) wg = (wg % 8) * (nwg / 8) + wg / 8;
  const int bx = (int)(wg % gridDim.x), split = (int)((wg / gridDim.x) % gridDim.y),
            e = (int)(wg / (gridDim.x * gridDim.y));
  const int tilesN = g.N / (32 * WN);
  const int tm = bx / tilesN, tn = bx % tilesN;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int r0 = (tm * WM + wave / WN) * 32, c0 = (tn * WN + wave % WN) * 32;
  const unsigned short* A = g.A + (int64_t)e * g.sA;
  const unsigned short* Bm = g.B + (int64_t)e * g.sB;
  const int kb = split * g.kchunk, ke = min(g.K, kb + g.kchunk);
  f4 acc[2][2];
  #pragma unroll
  for (int a = 0; a < 2; ++a)
    #pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0, 0, 0, 0};
  // DPRE1: the pre-activations the epilogue scales by are requested before
  // the product, so their latency hides behind it
  float pre[2][2][4];
  if (EPI == EPI_DPRE1) {
    #pragma unroll
    for (int b = 0; b < 2; ++b)
      #pragma unroll
      for (int a = 0; a < 2; ++a)
        #pragma unroll
        for (int r = 0; r < 4; ++r)
          pre[b][a][r] = g.pre1[((int64_t)e * g.M + r0 + a * 16 + 4 * (lane / 16) + r) * g.N +
                                c0 + b * 16 + lane % 16];
  }
  // the operands of KU consecutive K steps are requested together (one
  // memory latency per KU steps instead of per step); the accumulation
  // order along K is the same for every KU.  The K range is a multiple of 32.
  for (int k0 = kb; k0 < ke; k0 += 32 * KU) {
    us8 av[KU][2], bv[KU][2];
    #pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k0 + 32 * u < ke) {
        const int k = k0 + 32 * u + 8 * (lane / 16);
        #pragma unroll
        for (int a = 0; a < 2; ++a)
          av[u][a] = *(const us8*)(A + (int64_t)(r0 + a * 16 + lane % 16) * g.lda + k);
        #pragma unroll
        for (int b = 0; b < 2; ++b)
          bv[u][b] = *(const us8*)(Bm + (int64_t)(c0 + b * 16 + lane % 16) * g.ldb + k);
      }
    }
    #pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k0 + 32 * u < ke) {
        #pragma unroll
        for (int a = 0; a < 2; ++a)
          #pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av[u][a]),
                                                                __builtin_bit_cast(bf8, bv[u][b]),
                                                                acc[a][b], 0, 0, 0);
      }
    }
  }
  if (EPI == EPI_STORE) {
    #pragma unroll
    for (int a = 0; a < 2; ++a)
      #pragma unroll
      for (int b = 0; b < 2; ++b)
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + a * 16 + 4 * (lane / 16) + r;
          const int col = c0 + b * 16 + lane % 16;
          const int64_t o = ((int64_t)e * g.M + row) * g.N + col;
          g.out[(int64_t)split * gridDim.z * g.M * g.N + o] = acc[a][b][r];
        }
    return;
  }
  // dpre1 = dh1 GELU'(pre1): rows are samples, columns hidden units.  The
  // bfloat16 value feeds the layer-1 weight gradient (an NT product over
  // samples, so it is stored feature-major: each lane's four consecutive
  // samples are one 8-byte store); the unrounded value feeds the bias
  // gradient as column sums over this wave's 32 samples.
  #pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int col = c0 + b * 16 + lane % 16;
    float csum = 0.0f;
    #pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int row0 = r0 + a * 16 + 4 * (lane / 16);
      unsigned short q[4];
      #pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[a][b][r] * gelu_grad(pre[b][a][r]);
        csum += v;
        q[r] = f2bf(v);
      }
      const uint2 pk = make_uint2((unsigned)q[0] | ((unsigned)q[1] << 16),
                                  (unsigned)q[2] | ((unsigned)q[3] << 16));
      *(uint2*)(g.dpre1T + ((int64_t)e * g.N + col) * g.ldo + row0) = pk;
    }
    csum += __shfl_xor(csum, 16);
    csum += __shfl_xor(csum, 32);
    if (lane < 16) g.b1part[((int64_t)e * (g.M / 32) + r0 / 32) * g.N + col] = csum;
  }
}

// Layer-1 inputs for the weight-gradient product: bf16(x) feature-major,
// xT[k][i] (row stride ldt) for k < D, zero rows up to DX (32 or 64: whole
// 32-column tiles).
__global__ void __launch_bounds__(256) k_mlp_xt(const float* __restrict__ X, int64_t n, int D,
                                                int DX, int64_t ldt, unsigned short* __restrict__ xT) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)DX * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / n, i = e % n;
    xT[k * ldt + i] = k < D ? f2bf(X[i * D + k]) : (unsigned short)0;
  }
}

// Adam on every parameter, gradients assembled from the partial sums in a
// fixed order; the threads that update a weight also refresh its bfloat16
// copies.
struct AdamIn {
  const float* gW2part;   // S2 x E x H x H
  int S2;
  const float* l1part;    // S1 x E x H x DX (weight sums, columns < D used)
  int S1, DX;
  const float* b1part;    // E x (n / 32) x H (bias sums of dpre1)
  int nb1;
  const float* colpart;   // E x nblk x (2H + 2)
  int nblk;
  double lr;
  float* grad_out;        // E x P (optional): the assembled gradient
  float* loss_hist;       // steps x E (optional)
  int64_t n;
  int apply;              // 0: assemble gradients only
};

// One Adam update of parameter q of member e with gradient g.
// One Adam update of parameter q of member e with gradient g; with apply,
// also the bfloat16 copies the kernels read (W1, W2 both ways, w3 and the
// halved W2 and w3 of the prescreen pass), which k_mlp_cast builds at
// creation.
__device__ __forceinline__ void adam_update(const MlpDev& M, const AdamIn& in, int e, int64_t q,
                                            float g, double c1, double c2) {
  const int64_t P = M.P;
  if (in.grad_out) in.grad_out[e * P + q] = g;
  if (!in.apply) return;
  float* w = M.master + e * P + q;
  float* m1 = M.mom1 + e * P + q;
  float* m2 = M.mom2 + e * P + q;
  const float mn = 0.9f * *m1 + 0.1f * g;
  const float vn = 0.999f * *m2 + 0.001f * g * g;
  *m1 = mn;
  *m2 = vn;
  const double mh = mn / c1, vh = vn / c2;
  const float wn = (float)(*w - in.lr * mh / (sqrt(vh) + 1e-8));
  *w = wn;
  const int H = M.H, D = M.D;
  if (q < off_b1(M)) {  // W1[h][d]
    M.W1b[((int64_t)e * H + q / D) * M.DP + q % D] = f2bf(wn);
  } else if (q >= off_W2(M) && q < off_b2(M)) {  // W2[o][in]
    const int64_t i = q - off_W2(M);
    const int o = (int)(i / H), c = (int)(i % H);
    const unsigned short b = f2bf(wn);
    M.W2b[(int64_t)e * H * H + i] = b;
    M.W2Tb[(int64_t)e * H * H + (int64_t)c * H + o] = b;
    M.W2hb[(int64_t)e * H * H + i] = f2bf(0.5f * wn);
  } else if (q >= off_w3(M) && q < off_b3(M)) {  // w3
    const int64_t j = q - off_w3(M);
    M.w3b[(int64_t)e * H + j] = f2bf(wn);
    M.w3hb[(int64_t)e * H + j] = f2bf(0.5f * wn);
  }
}

// Sum of nb partials src[b * stride], b = 0 .. nb - 1, added in that order
// (the order of a sequential loop) by lane 0 of the calling wave: the lanes
// first load them in parallel, 64 at a time, into the wave's LDS slice.
__device__ __forceinline__ float ordered_sum(const float* __restrict__ src, int64_t stride, int nb,
                                             float* slice) {
  const int lane = threadIdx.x % 64;
  float g = 0.0f;
  for (int b0 = 0; b0 < nb; b0 += 64) {
    const int cnt = min(64, nb - b0);
    if (lane < cnt) slice[lane] = src[(int64_t)(b0 + lane) * stride];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (lane == 0)
      for (int b = 0; b < cnt; ++b) g += slice[b];
    __builtin_amdgcn_wave_barrier();
  }
  return g;
}

// Workgroups 0 .. ADAM_BULK_WG(M) - 1 of member e (blockIdx.y): one weight
// of W1 or W2 per thread, its gradient the sum of the S1 or S2 chunk
// partials.  The others: one bias or output weight per wave (b1 over the
// n / 32 block sums, b2, w3, b3 over the nblk block sums: a column of
// partials, loaded lane-parallel and added in block order), and one wave
// for the loss history.
constexpr int ADAM_COLS_PER_WG = 4;  // waves per workgroup, one column each
__host__ __device__ __forceinline__ int adam_bulk_wg(int H, int D) {
  return (H * D + H * H + 255) / 256;
}
__host__ __device__ __forceinline__ int adam_grid_x(int H, int D) {
  return adam_bulk_wg(H, D) + (3 * H + 2 + ADAM_COLS_PER_WG - 1) / ADAM_COLS_PER_WG;
}
__global__ void __launch_bounds__(256) k_mlp_adam(MlpDev M, AdamIn in) {
  __shared__ double corr[2];
  __shared__ float slices[ADAM_COLS_PER_WG][64];
  const int e = blockIdx.y;
  const int H = M.H, D = M.D;
  // the step's training forward has advanced the counter already
  const int t = *M.step;
  // the bias corrections 1 - beta^t, evaluated once per workgroup
  if (threadIdx.x == 0) {
    corr[0] = 1.0 - pow(0.9, t);
    corr[1] = 1.0 - pow(0.999, t);
  }
  __syncthreads();
  const double c1 = corr[0], c2 = corr[1];
  const int nbulk = adam_bulk_wg(H, D);
  if ((int)blockIdx.x < nbulk) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)H * D + (int64_t)H * H) return;
    float g = 0.0f;
    int64_t q;
    if (i < (int64_t)H * D) {  // W1[h][d]
      q = i;
      const int h = (int)(i / D), d = (int)(i % D);
      const float* src = in.l1part + ((int64_t)e * H + h) * in.DX + d;
      const int64_t stride = (int64_t)M.E * H * in.DX;
#pragma unroll 8
      for (int s = 0; s < in.S1; ++s) g += src[s * stride];
    } else {  // W2
      const int64_t w = i - (int64_t)H * D;
      q = off_W2(M) + w;
      const float* src = in.gW2part + (int64_t)e * H * H + w;
      const int64_t stride = (int64_t)M.E * H * H;
#pragma unroll 8
      for (int s = 0; s < in.S2; ++s) g += src[s * stride];
    }
    adam_update(M, in, e, q, g, c1, c2);
    return;
  }
  const int lane = threadIdx.x % 64;
  const int c = ((int)blockIdx.x - nbulk) * ADAM_COLS_PER_WG + (int)threadIdx.x / 64;
  if (c > 3 * H + 1) return;
  float* slice = slices[threadIdx.x / 64];
  const int64_t cstride = 2 * H + 2;
  const float* cbase = in.colpart + (int64_t)e * in.nblk * cstride;
  if (c == 3 * H + 1) {  // the loss history row of this step
    if (!in.loss_hist) return;
    const float ls = ordered_sum(cbase + 2 * H + 1, cstride, in.nblk, slice);
    if (lane == 0) in.loss_hist[(int64_t)(t - 1 - M.step[1]) * M.E + e] = ls / (float)in.n;
    return;
  }
  float g;
  int64_t q;
  if (c < H) {  // b1
    q = off_b1(M) + c;
    g = ordered_sum(in.b1part + (int64_t)e * in.nb1 * H + c, H, in.nb1, slice);
  } else {  // b2 -> columns [0, H), w3 -> [H, 2H), b3 -> 2H of the block sums
    const int col = c - H;
    q = off_b2(M) + col;  // b2, w3, b3 are consecutive
    g = ordered_sum(cbase + col, cstride, in.nblk, slice);
  }
  if (lane == 0) adam_update(M, in, e, q, g, c1, c2);
}

__global__ void k_mlp_zero_step(MlpDev M) {
  M.step[0] = 0;
  M.step[1] = 0;
}
__global__ void k_mlp_mark(MlpDev M) { M.step[1] = M.step[0]; }

// Ensemble mean / population standard deviation over the members and EI.
// The member mean and spread, z and EI in float64 (a few dozen operations per
// candidate): when the members nearly agree the spread is a small difference
// of the outputs, and float32 would carry a relative error of ~eps |mean| /
// sd into z; only the result is rounded to float32.
__global__ void k_ens_ei(int E, int64_t m, const float* __restrict__ out, double fbest,
                         float* __restrict__ ei) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = 0; e < E; ++e) s += out[(int64_t)e * m + i];
    const double mean = s / E;
    double q = 0.0;
    for (int e = 0; e < E; ++e) {
      const double d = out[(int64_t)e * m + i] - mean;
      q += d * d;
    }
    ei[i] = (float)ei_of<double>(mean, sqrt(q / E), fbest);
  }
}

// Ensemble lower confidence bound as a score to maximise:
// score = -(mean - kappa * sd), mean and population sd over the members.
__global__ void k_ens_lcb(int E, int64_t m, const float* __restrict__ out, float kappa,
                          float* __restrict__ score) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int e = 0; e < E; ++e) s += out[(int64_t)e * m + i];
    const float mean = s / E;
    float q = 0.0f;
    for (int e = 0; e < E; ++e) {
      const float d = out[(int64_t)e * m + i] - mean;
      q += d * d;
    }
    score[i] = -(mean - kappa * sqrtf(q / E));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct MlpState {
  Ctx* ctx;
  MlpDev dev;
  // training workspace (for the n of the last call)
  int64_t ws_n = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // float32 training data taken from a fitted model (mlp_train_model)
  float* data = nullptr;
  size_t data_bytes = 0;
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
  int ncu = 256;           // compute units of the device
  int fwd_wg_per_cu = 0;   // forward grid: 0 = one workgroup per item, else this many per CU
};

void mlp_set_occupancy(MlpState* st, int wg_per_cu) { st->fwd_wg_per_cu = wg_per_cu; }

int mlp_dp(int D) { return D <= 32 ? 32 : 64; }

size_t mlp_fwd_smem(int D, int H) {
  const int ldx = mlp_dp(D) + 8;
  return (size_t)MT * (H + 8) * 2 + (size_t)MT * ldx * 2 + 4 * MT * 4;
}

MlpState* mlp_create(Ctx* c, int E, int D, int H, const float* init, hipStream_t s) {
  MlpState* st = new MlpState();
  st->ctx = c;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        ncu > 0)
      st->ncu = ncu;
  }
  MlpDev& M = st->dev;
  M.E = E;
  M.D = D;
  M.DP = mlp_dp(D);
  M.H = H;
  M.P = (int64_t)H * D + H + (int64_t)H * H + H + H + 1;
  const size_t pb = (size_t)E * M.P * sizeof(float);
  M.master = (float*)dmalloc(c, pb);
  M.mom1 = (float*)dmalloc(c, pb);
  M.mom2 = (float*)dmalloc(c, pb);
  M.W1b = (unsigned short*)dmalloc(c, (size_t)E * H * mlp_dp(D) * 2);
  M.W2b = (unsigned short*)dmalloc(c, (size_t)E * H * H * 2);
  M.W2Tb = (unsigned short*)dmalloc(c, (size_t)E * H * H * 2);
  M.w3b = (unsigned short*)dmalloc(c, (size_t)E * H * 2);
  M.W2hb = (unsigned short*)dmalloc(c, (size_t)E * H * H * 2);
  M.w3hb = (unsigned short*)dmalloc(c, (size_t)E * H * 2);
  M.step = (int*)dmalloc(c, 64);
  if (!M.master || !M.mom1 || !M.mom2 || !M.W1b || !M.W2b || !M.W2Tb || !M.w3b || !M.W2hb ||
      !M.w3hb || !M.step) {
    delete st;
    return nullptr;
  }
  (void)hipMemcpyAsync(M.master, init, pb, hipMemcpyDeviceToDevice, s);
  (void)hipMemsetAsync(M.mom1, 0, pb, s);
  (void)hipMemsetAsync(M.mom2, 0, pb, s);
  hipLaunchKernelGGL(k_mlp_zero_step, dim3(1), dim3(1), 0, s, M);
  hipLaunchKernelGGL(k_mlp_cast, dim3(64, E), dim3(256), 0, s, M);
  (void)hipFuncSetAttribute((const void*)k_mlp_fwd<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)mlp_fwd_smem(D, H));
  (void)hipFuncSetAttribute((const void*)k_mlp_fwd<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)mlp_fwd_smem(D, H));
  return st;
}

void mlp_destroy(MlpState* st) {
  Ctx* c = st->ctx;
  (void)hipStreamSynchronize(c->stream);
  if (st->graph) (void)hipGraphExecDestroy(st->graph);
  void* ps[] = {st->dev.master, st->dev.mom1, st->dev.mom2, st->dev.W1b, st->dev.W2b,
                st->dev.W2Tb, st->dev.w3b, st->dev.W2hb, st->dev.w3hb, st->dev.step, st->ws,
                st->data};
  for (void* p : ps) dfree(c, p);
  delete st;
}

const float* mlp_master(MlpState* st) { return st->dev.master; }
int64_t mlp_nparams(MlpState* st) { return st->dev.P; }

// Workspace layout for n training samples.
struct Ws {
  float *out, *pre1, *pre2, *b1part, *colpart, *gW2part, *l1part;
  unsigned short *h1T, *dpre2, *dpre2T, *dpre1T, *xT;
  int nblk, S2, S1, DX;
  int64_t ldt;  // row stride of the feature-major (sample-contiguous) buffers
};
static Ws carve(MlpState* st, int64_t n, size_t* total) {
  const MlpDev& M = st->dev;
  const int64_t E = M.E, H = M.H, D = M.D;
  Ws w{};
  w.nblk = (int)ceil_div(n, MT);
  w.S2 = (int)std::min<int64_t>(8, ceil_div(n, 512));
  w.S1 = (int)std::min<int64_t>(8, ceil_div(n, 512));
  w.DX = D <= 32 ? 32 : 64;  // the weight-gradient product's columns (D <= 64), whole tiles
  w.ldt = n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  const size_t o_out = take(E * n * 4), o_pre1 = take(E * n * H * 4), o_pre2 = take(E * n * H * 4),
               o_b1 = take(E * (n / 32) * H * 4), o_col = take(E * w.nblk * (2 * H + 2) * 4),
               o_gw2 = take((size_t)w.S2 * E * H * H * 4), o_l1 = take((size_t)w.S1 * E * H * w.DX * 4),
               o_h1T = take(E * H * w.ldt * 2), o_dp2 = take(E * n * H * 2),
               o_dp2T = take(E * H * w.ldt * 2), o_dp1T = take(E * H * w.ldt * 2),
               o_xT = take((size_t)w.DX * w.ldt * 2);
  *total = off;
  unsigned char* b = (unsigned char*)st->ws;
  if (b) {
    w.out = (float*)(b + o_out);
    w.pre1 = (float*)(b + o_pre1);
    w.pre2 = (float*)(b + o_pre2);
    w.b1part = (float*)(b + o_b1);
    w.colpart = (float*)(b + o_col);
    w.gW2part = (float*)(b + o_gw2);
    w.l1part = (float*)(b + o_l1);
    w.h1T = (unsigned short*)(b + o_h1T);
    w.dpre2 = (unsigned short*)(b + o_dp2);
    w.dpre2T = (unsigned short*)(b + o_dp2T);
    w.dpre1T = (unsigned short*)(b + o_dp1T);
    w.xT = (unsigned short*)(b + o_xT);
  }
  return w;
}

bool mlp_ensure_ws(MlpState* st, int64_t n) {
  if (st->ws && st->ws_n == n) return true;
  size_t bytes = 0;
  carve(st, n, &bytes);
  Ctx* c = st->ctx;
  (void)hipStreamSynchronize(c->stream);
  if (st->ws) dfree(c, st->ws);
  if (st->graph) {
    (void)hipGraphExecDestroy(st->graph);
    st->graph = nullptr;
    st->graph_key.clear();
  }
  st->ws = dmalloc(c, bytes);
  st->ws_bytes = st->ws ? bytes : 0;
  st->ws_n = st->ws ? n : 0;
  return st->ws != nullptr;
}

// One training step (apply = 1) or a gradient evaluation (apply = 0).
void mlp_step(MlpState* st, int64_t n, const float* X, const float* y, double lr, int apply,
              float* grad_out, float* loss_hist, hipStream_t s) {
  size_t bytes;
  Ws w = carve(st, n, &bytes);
  MlpDev& M = st->dev;
  const int E = M.E, H = M.H;
  FwdOut fo{w.out, w.pre1, w.h1T, w.pre2, w.ldt};
  hipLaunchKernelGGL(k_mlp_fwd<true>, dim3((unsigned)fwd_items((int)w.nblk, E)), dim3(256),
                     mlp_fwd_smem(M.D, H), s, M, n, X, fo, (int)w.nblk, apply);
  BwdBuf bb{w.dpre2, w.dpre2T, w.colpart, w.ldt};
  hipLaunchKernelGGL(k_mlp_bwd_out, dim3(w.nblk, E), dim3(256), 0, s, M, n, y, w.out, w.pre2, bb);
  // gW2 = dpre2^T h1 over the samples (split over S2 sample chunks; one
  // wave per workgroup measured faster than 2 x 2 for these grids)
  Gemm g1{};
  g1.A = w.dpre2T;
  g1.B = w.h1T;
  g1.sA = (int64_t)H * w.ldt;
  g1.sB = (int64_t)H * w.ldt;
  g1.lda = g1.ldb = w.ldt;
  g1.M = H;
  g1.N = H;
  g1.K = (int)n;
  g1.kchunk = (int)round_up(ceil_div(n, w.S2), 32);
  g1.out = w.gW2part;
  hipLaunchKernelGGL((k_gemm_nt<EPI_STORE, 1, 1, 8>), dim3((H / 32) * (H / 32), w.S2, E), dim3(64), 0, s,
                     g1);
  // dh1 = dpre2 W2 -> dpre1 = dh1 GELU'(pre1) (one wave per workgroup too;
  // the bias partials are per 32-row block, i.e. per wave, either way)
  Gemm g2{};
  g2.A = w.dpre2;
  g2.B = M.W2Tb;
  g2.sA = (int64_t)n * H;
  g2.sB = (int64_t)H * H;
  g2.lda = g2.ldb = H;
  g2.M = (int)n;
  g2.N = H;
  g2.K = H;
  g2.kchunk = H;
  g2.out = nullptr;
  g2.pre1 = w.pre1;
  g2.dpre1T = w.dpre1T;
  g2.ldo = w.ldt;
  g2.b1part = w.b1part;
  hipLaunchKernelGGL((k_gemm_nt<EPI_DPRE1, 1, 1, 8>), dim3((unsigned)(n / 32) * (H / 32), 1, E),
                     dim3(64), 0, s, g2);
  // gW1 = dpre1^T x over the samples (bf16 operands, split over S1 chunks);
  // x^T is shared by the members
  Gemm g3{};
  g3.A = w.dpre1T;
  g3.B = w.xT;
  g3.sA = (int64_t)H * w.ldt;
  g3.sB = 0;
  g3.lda = g3.ldb = w.ldt;
  g3.M = H;
  g3.N = w.DX;
  g3.K = (int)n;
  g3.kchunk = (int)round_up(ceil_div(n, w.S1), 32);
  g3.out = w.l1part;
  hipLaunchKernelGGL((k_gemm_nt<EPI_STORE, 1, 1, 8>), dim3((H / 32) * (w.DX / 32), w.S1, E), dim3(64), 0, s,
                     g3);
  AdamIn ai{w.gW2part, w.S2, w.l1part, w.S1, w.DX, w.b1part, (int)(n / 32), w.colpart, w.nblk,
            lr, grad_out, loss_hist, n, apply};
  hipLaunchKernelGGL(k_mlp_adam, dim3(adam_grid_x(H, st->dev.D), E), dim3(256), 0, s, M, ai);
}

// bf16(x) feature-major for the layer-1 weight gradient: the training data
// are fixed over the steps of a call, so this runs once per call, ahead of
// the (captured) steps.
static void mlp_prepare_x(MlpState* st, int64_t n, const float* X, hipStream_t s) {
  size_t bytes;
  Ws w = carve(st, n, &bytes);
  const unsigned g = (unsigned)std::min<int64_t>(1024, ceil_div((int64_t)w.DX * n, 256));
  hipLaunchKernelGGL(k_mlp_xt, dim3(g), dim3(256), 0, s, X, n, st->dev.D, w.DX, w.ldt, w.xT);
}

// Training: the step sequence is captured once per (n, inputs, lr, history)
// and the graph replayed `steps` times.
bool mlp_train(MlpState* st, int64_t n, const float* X, const float* y, int steps, double lr,
               float* loss_hist, bool use_graph, hipStream_t s) {
  if (steps <= 0) return true;
  if (!mlp_ensure_ws(st, n)) return false;
  mlp_prepare_x(st, n, X, s);
  hipLaunchKernelGGL(k_mlp_mark, dim3(1), dim3(1), 0, s, st->dev);
  std::vector<uint64_t> key = {(uint64_t)n, (uint64_t)(uintptr_t)X, (uint64_t)(uintptr_t)y,
                               (uint64_t)(uintptr_t)loss_hist, (uint64_t)(uintptr_t)s};
  uint64_t lrbits;
  memcpy(&lrbits, &lr, 8);
  key.push_back(lrbits);
  if (!use_graph || s == nullptr) {
    for (int k = 0; k < steps; ++k) mlp_step(st, n, X, y, lr, 1, nullptr, loss_hist, s);
    return true;
  }
  if (!st->graph || st->graph_key != key) {
    if (st->graph) (void)hipGraphExecDestroy(st->graph);
    st->graph = nullptr;
    // one eager step first: it also checks the launch configuration
    mlp_step(st, n, X, y, lr, 1, nullptr, loss_hist, s);
    --steps;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    mlp_step(st, n, X, y, lr, 1, nullptr, loss_hist, s);
    if (hipStreamEndCapture(s, &g) != hipSuccess) return false;
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return false;
    st->graph = ex;
    st->graph_key = key;
  }
  for (int k = 0; k < steps; ++k)
    if (hipGraphLaunch(st->graph, s) != hipSuccess) return false;
  return true;
}

// The model's observations as float32 training data: inputs X (n x d) and
// targets ytilde (the fit's normalised observations).
__global__ void __launch_bounds__(256) k_model_data(const double* __restrict__ X,
                                                    const double* __restrict__ yt, int64_t n, int d,
                                                    float* __restrict__ X32, float* __restrict__ y32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * (d + 1);
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n * d) X32[i] = (float)X[i];
    else y32[i - n * d] = (float)yt[i - n * d];
  }
}

bool mlp_train_model(MlpState* st, const Model* M, int steps, double lr, float* loss_hist,
                     bool use_graph, hipStream_t s) {
  const int64_t n = M->n;
  const int d = M->d;
  const size_t bytes = (size_t)(n * d + n) * sizeof(float);
  if (st->data_bytes < bytes) {
    if (st->data) {
      (void)hipStreamSynchronize(s);
      dfree(st->ctx, st->data);
    }
    st->data = (float*)dmalloc(st->ctx, bytes);
    st->data_bytes = st->data ? bytes : 0;
    if (!st->data) return false;
  }
  float* X32 = st->data;
  float* y32 = st->data + n * d;
  const unsigned grid = (unsigned)std::min<int64_t>(1024, ceil_div(n * (d + 1), 256));
  hipLaunchKernelGGL(k_model_data, dim3(grid), dim3(256), 0, s, M->X64, M->yt, n, d, X32, y32);
  return mlp_train(st, n, X32, y32, steps, lr, loss_hist, use_graph, s);
}

bool mlp_grads(MlpState* st, int64_t n, const float* X, const float* y, float* grad, float* loss,
               hipStream_t s) {
  if (!mlp_ensure_ws(st, n)) return false;
  mlp_prepare_x(st, n, X, s);
  // loss through a one-entry history at the current step: record it into a
  // scratch row, then copy out
  mlp_step(st, n, X, y, 0.0, 0, grad, nullptr, s);
  size_t bytes;
  Ws w = carve(st, n, &bytes);
  // loss = (1/n) sum of squared errors from the column partials
  const int E = st->dev.E, H = st->dev.H;
  std::vector<float> cp((size_t)E * w.nblk * (2 * H + 2));
  (void)hipMemcpyAsync(cp.data(), w.colpart, cp.size() * 4, hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  std::vector<float> ls(E, 0.0f);
  for (int e = 0; e < E; ++e)
    for (int b = 0; b < w.nblk; ++b) ls[e] += cp[((size_t)e * w.nblk + b) * (2 * H + 2) + 2 * H + 1];
  for (int e = 0; e < E; ++e) ls[e] /= (float)n;
  (void)hipMemcpyAsync(loss, ls.data(), E * 4, hipMemcpyHostToDevice, s);
  (void)hipStreamSynchronize(s);
  return true;
}

// Member outputs on m candidates, in chunks (out: E x m).
void mlp_forward(MlpState* st, int64_t m, const float* Xc, float* out, hipStream_t s) {
  MlpDev& M = st->dev;
  FwdOut fo{out, nullptr, nullptr, nullptr};
  const int ntile = (int)ceil_div(m, MT);
  int64_t grid = fwd_items(ntile, M.E);
  if (st->fwd_wg_per_cu > 0)
    grid = std::min<int64_t>(grid, round_up((int64_t)st->ncu * st->fwd_wg_per_cu, 8));
  hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((unsigned)grid), dim3(256), mlp_fwd_smem(M.D, M.H), s,
                     M, m, Xc, fo, ntile, 0);
}

void ens_score(int E, int64_t m, const float* out, bool lcb, double arg, float* score,
               hipStream_t s) {
  const int g = (int)std::min<int64_t>(8192, ceil_div(m, 256));
  if (lcb)
    hipLaunchKernelGGL(k_ens_lcb, dim3(std::max(g, 1)), dim3(256), 0, s, E, m, out, (float)arg,
                       score);
  else
    hipLaunchKernelGGL(k_ens_ei, dim3(std::max(g, 1)), dim3(256), 0, s, E, m, out, arg, score);
}

void mlp_ens_ei(MlpState* st, int64_t m, const float* out, double fbest, float* ei, hipStream_t s) {
  ens_score(st->dev.E, m, out, false, fbest, ei, s);
}

void mlp_ens_lcb(MlpState* st, int64_t m, const float* out, double kappa, float* score,
                 hipStream_t s) {
  ens_score(st->dev.E, m, out, true, kappa, score, s);
}

}  // namespace gpbo
