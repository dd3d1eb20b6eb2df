// Device-side building blocks shared by the scoring kernels (single-problem
// fused, large-n, batched): precision traits, the packed matrix-core block
// format, covariance, expected improvement, argmax ordering and reductions.
#pragma once

#include <cmath>

#include "gpbo_internal.h"

namespace gpbo {
namespace sc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr float kLog2e = 1.4426950408889634f;

template <int P>
struct PT;
template <>
struct PT<GPBO_FP64> {
  using In = double;   // candidate coordinates and outputs
  using C = double;    // cross-covariance arithmetic
  using K = double;    // LDS / matrix-core operand
  using Acc = double;  // accumulators
  using V4 = d4;
  static constexpr int KB = 16;
};
template <>
struct PT<GPBO_FP32> {
  using In = float;
  using C = float;
  using K = float;
  using Acc = float;
  using V4 = f4;
  static constexpr int KB = 16;
};
template <>
struct PT<GPBO_BF16> {
  using In = float;
  using C = float;
  using K = unsigned short;  // bfloat16 bits
  using Acc = float;
  using V4 = f4;
  static constexpr int KB = 32;
};

// Escalated float32 scoring (P_F64IO32): float64 arithmetic and operands,
// float32 candidate coordinates and outputs.
template <>
struct PT<P_F64IO32> {
  using In = float;
  using C = double;
  using K = double;
  using Acc = double;
  using V4 = d4;
  static constexpr int KB = 16;
};
// Float64 arithmetic (either input type).
__host__ __device__ constexpr bool arith64(int P) { return P == GPBO_FP64 || P == P_F64IO32; }

// float32 -> bfloat16 bits, round to nearest even (NaN kept quiet; an
// infinity, whose low bits are zero, passes the rounding unchanged).
// Branch-free: both results are formed and one is selected, so a wave does
// not split its execution mask per element.
__device__ __forceinline__ unsigned short f2bf(float f) {
  const unsigned int u = __float_as_uint(f);
  const unsigned int rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const unsigned int quiet = (u >> 16) | 0x40u;
  return (unsigned short)(f != f ? quiet : rounded);
}
// The same rounding by the hardware conversion (v_cvt_pk_bf16_f32).  Faster
// in the cross-covariance tile of the scoring kernels; measured slower than
// f2bf in the network's activation epilogue, which keeps f2bf.
__device__ __forceinline__ unsigned short f2bf_hw(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}

// Two float32 values as a pair of bfloat16 (round to nearest even, the
// first in the low half): one v_cvt_pk_bf16_f32.
__device__ __forceinline__ unsigned bf16_pair(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  const f2 v = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, b2));
}

template <typename K, typename C>
__device__ __forceinline__ K to_k(C v);
template <>
__device__ __forceinline__ double to_k<double, double>(double v) { return v; }
template <>
__device__ __forceinline__ float to_k<float, float>(float v) { return v; }
template <>
__device__ __forceinline__ unsigned short to_k<unsigned short, float>(float v) { return f2bf_hw(v); }

__device__ __forceinline__ void store_elem(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_elem(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_elem(unsigned short* p, double v) { *p = f2bf((float)v); }

// Matrix-core squared distances of the bfloat16 path: the contraction depth
// (d coordinates and two extra terms, rounded up to the 4 of one float32
// matrix-core step) and the largest number of steps taken that way (larger d
// form the distances on the vector ALU).
__host__ __device__ constexpr int dist_kp(int d) { return (d + 2 + 3) / 4 * 4; }
constexpr int DIST_SMAX = 8;
__host__ __device__ constexpr bool dist_mfma(int prec, int d) {
  return prec == GPBO_BF16 && dist_kp(d) <= 4 * DIST_SMAX;
}

// Covariance (without the signal variance) from the squared scaled distance.
// For the float kernels the squared-exponential coordinates carry the factor
// sqrt(log2(e) / 2), so exp(-r^2 / 2) becomes one hardware exp2.
template <int KERN>
__device__ __forceinline__ float cov_from_r2(float r2) {
  if (KERN == GPBO_KERNEL_SE) return __builtin_amdgcn_exp2f(-r2);
  const float r = __builtin_sqrtf(r2);
  const float s5r = 2.2360679774997896f * r;
  return (1.0f + s5r + (5.0f / 3.0f) * r2) * __builtin_amdgcn_exp2f(-s5r * kLog2e);
}
template <int KERN>
__device__ __forceinline__ double cov_from_r2(double r2) {
  if (KERN == GPBO_KERNEL_SE) return exp(-0.5 * r2);
  const double r = sqrt(r2);
  const double s5r = 2.23606797749978969641 * r;
  return (1.0 + s5r + (5.0 / 3.0) * r2) * exp(-s5r);
}

// Expected improvement for minimisation (Jones, Schonlau & Welch 1998):
// (f - mu) Phi(z) + sigma phi(z), z = (f - mu) / sigma; max(f - mu, 0) at
// sigma = 0.
template <typename T>
__device__ __forceinline__ T ei_of(T mu, T sigma, T fbest) {
  const T imp = fbest - mu;
  if (sigma > T(0)) {
    const T z = imp / sigma;
    const T Phi = T(0.5) * erfc(-z * T(0.70710678118654752440));
    const T phi = exp(T(-0.5) * z * z) * T(0.39894228040143267794);
    return imp * Phi + sigma * phi;
  }
  return imp > T(0) ? imp : T(0);
}
template <>
__device__ __forceinline__ float ei_of<float>(float mu, float sigma, float fbest) {
  const float imp = fbest - mu;
  if (sigma > 0.0f) {
    const float z = imp / sigma;
    const float Phi = 0.5f * erfcf(-z * 0.70710678118654752440f);
    const float phi = expf(-0.5f * z * z) * 0.39894228040143267794f;
    return imp * Phi + sigma * phi;
  }
  return imp > 0.0f ? imp : 0.0f;
}

// (value, index) ordering of the argmax: larger value wins, ties go to the
// lower index; index -1 marks "no candidate".  Callers map NaN to -inf.
__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  if (i < 0) return false;
  if (bi < 0) return true;
  return v > bv || (v == bv && i < bi);
}

// Packed inverse factor layout: row tile t (16 rows) needs column blocks
// 0 .. floor(t / R) (R = KB / 16) and stores that count rounded up to a
// multiple of the pipeline depth PF, the extra blocks being zero, so the
// matrix-core loop runs whole groups without branches.
__host__ __device__ __forceinline__ int tile_blocks(int t, int R, int PF) {
  return (t / R + 1 + PF - 1) / PF * PF;
}
__host__ __device__ __forceinline__ int prec_pf(int) { return 2; }

// One packed 16 x KB block of the inverse factor (A operand) or of the
// cross-covariance tile (B operand) as one lane holds it, and its
// matrix-core product.  Lane l holds KB/4 consecutive columns of row l % 16
// starting at (KB/4)(l / 16); the k-th matrix-core step of a block uses the
// k-th of those columns for both operands, so A and B agree on the order of
// the contraction index.  The 16 x 16 output tile leaves lane l with rows
// 4(l / 16) .. 4(l / 16) + 3 of column l % 16.
template <int P>
struct Blk;
template <>
struct Blk<GPBO_FP32> {
  using V = f4;
  using Acc = f4;
  static constexpr int EPB = 64 * 4;
  static constexpr int PF = 2;  // blocks per pipeline group (row tiles are padded to a multiple)
  static constexpr int KS = 4;  // matrix-core steps per block
  __device__ static __forceinline__ V load(const float* p) { return *(const f4*)p; }
  // step kk of the block product (callers interleave independent accumulators)
  __device__ static __forceinline__ void mma_k(Acc& c, const V& a, const V& b, int kk) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[kk], c, 0, 0, 0);
  }
  __device__ static __forceinline__ void mma(Acc& c, const V& a, const V& b) {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) mma_k(c, a, b, kk);
  }
};
template <>
struct Blk<GPBO_BF16> {
  using V = us8;
  using Acc = f4;
  static constexpr int EPB = 64 * 8;
  static constexpr int PF = 2;
  static constexpr int KS = 1;
  __device__ static __forceinline__ V load(const unsigned short* p) { return *(const us8*)p; }
  __device__ static __forceinline__ void mma_k(Acc& c, const V& a, const V& b, int) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  }
  __device__ static __forceinline__ void mma(Acc& c, const V& a, const V& b) { mma_k(c, a, b, 0); }
};
struct dq {
  double2 lo, hi;
};
template <>
struct Blk<GPBO_FP64> {
  using V = dq;
  using Acc = d4;
  static constexpr int EPB = 64 * 4;
  static constexpr int PF = 2;
  static constexpr int KS = 4;
  __device__ static __forceinline__ V load(const double* p) {
    return dq{*(const double2*)p, *(const double2*)(p + 2)};
  }
  __device__ static __forceinline__ void mma_k(Acc& c, const V& a, const V& b, int kk) {
    const double av = kk == 0 ? a.lo.x : kk == 1 ? a.lo.y : kk == 2 ? a.hi.x : a.hi.y;
    const double bv = kk == 0 ? b.lo.x : kk == 1 ? b.lo.y : kk == 2 ? b.hi.x : b.hi.y;
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
  }
  __device__ static __forceinline__ void mma(Acc& c, const V& a, const V& b) {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) mma_k(c, a, b, kk);
  }
};

template <>
struct Blk<P_F64IO32> : Blk<GPBO_FP64> {};

// Transpose-reduction of N per-lane partial sums over the 64 lanes of a wave:
// log2 N halving exchanges leave each lane with one entry summed over 64/N...
// lanes; the remaining low lane bits are folded by butterflies.  Entry e ends
// in the lanes whose bits 5..(6 - log2 N) spell e; the lane with the low bits
// clear writes it to dst[e].
template <typename A, int N>
__device__ __forceinline__ void lane_transpose_sum(A (&v)[N], A* dst) {
  const int lane = threadIdx.x % 64;
  constexpr int LOGN = N == 64 ? 6 : N == 32 ? 5 : N == 16 ? 4 : N == 8 ? 3 : N == 4 ? 2 : 0;
  static_assert(LOGN > 0, "N must be 4, 8, 16, 32 or 64");
  int width = N;
  int D = 32;
#pragma unroll
  for (int s = 0; s < LOGN; ++s) {
    const int half = width / 2;
    const bool upper = (lane & D) != 0;
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
      if (k < half) {
        // the empty asm keeps the two selects on registers: without it the
        // compiler folds them into one runtime-indexed read of v[], lowered
        // as a compare-and-select chain over the whole array
        A lo = v[k], hi = v[k + half];
        __asm__("" : "+v"(lo), "+v"(hi));
        const A keep = upper ? hi : lo;
        const A send = upper ? lo : hi;
        v[k] = keep + __shfl_xor(send, D);
      }
    }
    width = half;
    D >>= 1;
  }
  A r = v[0];
  for (int o = D; o > 0; o >>= 1) r += __shfl_xor(r, o);
  int idx = 0;
  int bitpos = 5;
#pragma unroll
  for (int s = 0; s < LOGN; ++s, --bitpos) idx = (idx << 1) | ((lane >> bitpos) & 1);
  if ((lane & ((1 << (6 - LOGN)) - 1)) == 0) dst[idx] = r;
}

// Wave index as a scalar (uniform) value, so loops over it stay scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Posterior, EI and argmax of one candidate from its mean and squared-norm
// partial sums.  Writes the outputs (each may be NULL) and folds (EI, gc)
// into the running maximum.
template <typename Acc, typename In>
__device__ __forceinline__ void finish_candidate(int64_t gc, Acc muz, Acc vv, double sf2,
                                                 const double* __restrict__ stats, In* mu_out,
                                                 In* sigma_out, In* ei_out, double& bv,
                                                 int64_t& bi) {
  Acc varz = (Acc)sf2 - vv;
  varz = varz > Acc(0) ? varz : Acc(0);
  const Acc ymean = (Acc)stats[S_YMEAN], sy = (Acc)stats[S_YSTD], fb = (Acc)stats[S_FBEST];
  const Acc mu = ymean + sy * muz;
  const Acc sg = sy * sqrt(varz);
  const Acc e = ei_of<Acc>(mu, sg, fb);
  if (mu_out) mu_out[gc] = (In)mu;
  if (sigma_out) sigma_out[gc] = (In)sg;
  if (ei_out) ei_out[gc] = (In)e;
  const double ev = e == e ? (double)e : -INFINITY;  // NaN never wins
  if (better(ev, gc, bv, bi)) {
    bv = ev;
    bi = gc;
  }
}

// Wave-wide (value, index) maximum.
__device__ __forceinline__ void wave_argmax(double& bv, int64_t& bi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const int64_t oi = __shfl_xor(bi, o);
    if (better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
}

}  // namespace sc
}  // namespace gpbo
