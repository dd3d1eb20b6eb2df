// Scoring kernels: posterior mean, standard deviation and expected
// improvement of candidate configurations under a fitted Gaussian process,
// with a per-tile argmax (the acquisition step of Sec. III-A of the paper;
// formulas from Rasmussen & Williams 2006, eqs. 2.25-2.26, and Jones et al.
// 1998, eq. 15):
//
//   k*_j   = k(x*, x_j)                      cross-covariance, VALU
//   mu_z   = sum_j (sf2 alpha_j) khat_j       in-register, transpose-reduced
//   v      = (sf2 L^-1) khat                  matrix cores, triangular
//   var_z  = max(sf2 - |v|^2, 0)              sum-of-squares epilogue
//   mu = ymean + s_y mu_z,  sigma = s_y sqrt(var_z),  EI(mu, sigma, f_best)
//
// One workgroup (four waves) owns TM candidates.
//   Phase 1: the scaled candidate tile sits in LDS; each lane owns one
//            training point (its coordinates in registers) and loops over the
//            TM candidates, writing khat[c][j] into an LDS tile and
//            accumulating alpha_j khat_cj in TM registers.
//   Phase 2: the waves split the 16-row tiles of the packed inverse factor
//            (streamed from L2 in the exact order the matrix-core lanes read
//            it), multiply against the LDS khat tile and fold the squares of
//            each finished output tile into per-lane partial sums.
//   Phase 3: one thread per candidate combines the partials, evaluates EI,
//            writes the outputs and the tile's (EI, index) maximum.
#include <cmath>
#include <cstdio>

#include "gpbo_internal.h"

namespace gpbo {

namespace {

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
  static constexpr int KB = 16;
};
template <>
struct PT<GPBO_FP32> {
  using In = float;
  using C = float;
  using K = float;
  using Acc = float;
  static constexpr int KB = 16;
};
template <>
struct PT<GPBO_BF16> {
  using In = float;
  using C = float;
  using K = unsigned short;  // bfloat16 bits
  using Acc = float;
  static constexpr int KB = 32;
};

// float32 -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0x7fffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <typename K, typename C>
__device__ __forceinline__ K to_k(C v);
template <>
__device__ __forceinline__ double to_k<double, double>(double v) { return v; }
template <>
__device__ __forceinline__ float to_k<float, float>(float v) { return v; }
template <>
__device__ __forceinline__ unsigned short to_k<unsigned short, float>(float v) { return f2bf(v); }

// Covariance from the squared scaled distance.  For the float kernels the
// squared-exponential coordinates carry the factor sqrt(log2(e) / 2), so
// exp(-r^2 / 2) becomes one hardware exp2.
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

// Expected improvement for minimisation.
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
// lower index, NaN never wins.
__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  if (i < 0) return false;
  if (bi < 0) return true;
  return v > bv || (v == bv && i < bi);
}

// Padded extents of the packed operand.
__host__ __device__ __forceinline__ int packed_rows(int n) { return (int)round_up(n, TI); }
// Offset (in blocks) of row tile t when row tile t holds floor(t / R) + 1
// column blocks (R = KB / TI).
__host__ __device__ __forceinline__ int64_t tile_offset(int t, int R) {
  if (R == 1) return (int64_t)t * (t + 1) / 2;
  const int64_t q = t / 2, r = t % 2;
  return t + q * (q - 1) + r * q;
}

__device__ __forceinline__ void store_elem(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_elem(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_elem(unsigned short* p, double v) { *p = f2bf((float)v); }

// Packed sf2 * Linv: row tile ti, column block tj holds a 16 x KB block; lane
// l (0..63) stores KB/4 consecutive entries of row 16 ti + l%16 starting at
// column KB tj + (KB/4) (l/16).
template <typename K>
__global__ void k_pack(const double* __restrict__ Linv, int npad, int n, double sf2, int KB,
                       K* __restrict__ out, int64_t total_blocks) {
  const int R = KB / TI;
  const int per = KB / 4;
  const int64_t cnt = total_blocks * 64 * per;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = e / (64 * per);
    const int w = (int)(e % (64 * per));
    const int lane = w / per, q = w % per;
    // find the row tile ti of this block
    int ti = (int)(R == 1 ? (sqrt(8.0 * blk + 1.0) - 1.0) * 0.5 : sqrt((double)blk));
    while (ti > 0 && tile_offset(ti, R) > blk) --ti;
    while (tile_offset(ti + 1, R) <= blk) ++ti;
    const int tj = (int)(blk - tile_offset(ti, R));
    const int i = ti * TI + lane % 16;
    const int j = tj * KB + per * (lane / 16) + q;
    double v = 0.0;
    if (i < n && j < n && j <= i) v = sf2 * Linv[(int64_t)i * npad + j];
    store_elem(out + e, v);
  }
}

// Scaled coordinates of the observations for the scoring kernels.
template <typename T>
__global__ void k_scale_obs(const double* __restrict__ X, const double* __restrict__ sc, int n,
                            int d, T* __restrict__ Xs) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * d;
       e += (int64_t)gridDim.x * blockDim.x)
    Xs[e] = (T)(X[e] * sc[e % d]);
}

template <typename T>
__global__ void k_scale_alpha(const double* __restrict__ a, int n, double sf2, T* __restrict__ o) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    o[i] = (T)(sf2 * a[i]);
}

// Transpose-reduction of TM per-lane partial sums over the 64 lanes: after
// the call, lane l holds the full sum of entry (l >> (6 - log2 TM))-th in a
// fixed lane order, returned through `out` for lanes with (l & mask) == 0.
template <typename A, int TM>
__device__ __forceinline__ void lane_transpose_sum(A (&v)[TM], A* dst /* LDS, TM entries */) {
  const int lane = threadIdx.x % 64;
  // Halving steps: at step with width W (values per lane), partner = lane ^ D
  // keeps the half selected by its own bit.
  constexpr int LOGTM = TM == 64 ? 6 : TM == 32 ? 5 : TM == 16 ? 4 : TM == 8 ? 3 : 0;
  static_assert(LOGTM > 0, "TM must be 8, 16, 32 or 64");
  int width = TM;
  int D = 32;
#pragma unroll
  for (int s = 0; s < LOGTM; ++s) {
    const int half = width / 2;
    const bool upper = (lane & D) != 0;
#pragma unroll
    for (int k = 0; k < TM / 2; ++k) {
      if (k < half) {
        // keep entry (upper ? k + half : k); send the other one
        const A keep = upper ? v[k + half] : v[k];
        const A send = upper ? v[k] : v[k + half];
        const A got = __shfl_xor(send, D);
        v[k] = keep + got;
      }
    }
    width = half;
    D >>= 1;
  }
  // remaining lanes that share the value: reduce over the low bits
  A r = v[0];
  for (int o = D; o > 0; o >>= 1) r += __shfl_xor(r, o);
  // entry index held by this lane: bits of the lane from bit 5 downwards
  int idx = 0;
  int bitpos = 5;
#pragma unroll
  for (int s = 0; s < LOGTM; ++s, --bitpos) idx = (idx << 1) | ((lane >> bitpos) & 1);
  if ((lane & ((1 << (6 - LOGTM)) - 1)) == 0) dst[idx] = r;
}

template <int P, int KERN, int TM, int DMAX>
__global__ void __launch_bounds__(256) k_score_fused(
    int n, int d, int npk, const typename PT<P>::K* __restrict__ pk,
    const typename PT<P>::Acc* __restrict__ alpha, const typename PT<P>::C* __restrict__ Xs,
    const typename PT<P>::C* __restrict__ sc, const double* __restrict__ stats, double sf2_d,
    int64_t m, const typename PT<P>::In* __restrict__ Xc, typename PT<P>::In* __restrict__ mu_out,
    typename PT<P>::In* __restrict__ sigma_out, typename PT<P>::In* __restrict__ ei_out,
    double* __restrict__ part_v, int64_t* __restrict__ part_i, int ldk) {
  using C = typename PT<P>::C;
  using K = typename PT<P>::K;
  using Acc = typename PT<P>::Acc;
  using In = typename PT<P>::In;
  constexpr int KB = PT<P>::KB;
  constexpr int R = KB / TI;
  constexpr int NCT = TM / 16;  // candidate tiles of 16 per workgroup

  extern __shared__ __align__(16) unsigned char smem[];
  K* kt = (K*)smem;                                     // [TM][ldk]
  C* xc = (C*)(smem + (size_t)TM * ldk * sizeof(K));    // [TM][DMAX]
  Acc* mu_part = (Acc*)(xc + TM * DMAX);                // [4][TM]
  Acc* ssq_part = mu_part + 4 * TM;                     // [4][TM]

  const int t = threadIdx.x;
  const int lane = t % 64, wave = t / 64;
  const int64_t c0 = (int64_t)blockIdx.x * TM;
  const int njb = (int)ceil_div(npk, KB);  // column blocks of the widest row tile
  const int npj = njb * KB;                // padded training-point extent

  // ---- scaled candidate tile ---------------------------------------------
  for (int e = t; e < TM * DMAX; e += 256) {
    const int c = e / DMAX, k = e % DMAX;
    C v = 0;
    if (k < d && c0 + c < m) v = (C)Xc[(c0 + c) * d + k] * sc[k];
    xc[e] = v;
  }
  __syncthreads();

  // ---- phase 1: cross-covariance tile + mean partials ----------------------
  // Candidates are taken CG at a time so their mean partials stay in
  // registers; each lane re-reads its training point's coordinates per group.
  constexpr int CG = TM < 16 ? TM : 16;
  for (int cg = 0; cg < TM; cg += CG) {
    Acc macc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) macc[c] = 0;
    for (int jb = wave * 64; jb < npj; jb += 256) {
      const int j = jb + lane;
      const bool valid = j < n;
      C xj[DMAX];
#pragma unroll
      for (int k = 0; k < DMAX; ++k) xj[k] = (valid && k < d) ? Xs[(int64_t)j * d + k] : C(0);
      const Acc aj = valid ? alpha[j] : Acc(0);
#pragma unroll
      for (int cc = 0; cc < CG; ++cc) {
        const int c = cg + cc;
        C r2 = 0;
#pragma unroll
        for (int k = 0; k < DMAX; k += 4) {
          if (k < d) {
            const C* xr = xc + c * DMAX + k;
            const C t0 = xj[k] - xr[0], t1 = xj[k + 1] - xr[1], t2 = xj[k + 2] - xr[2],
                    t3 = xj[k + 3] - xr[3];
            r2 = fma(t0, t0, r2);
            r2 = fma(t1, t1, r2);
            r2 = fma(t2, t2, r2);
            r2 = fma(t3, t3, r2);
          }
        }
        const C kv = valid ? cov_from_r2<KERN>(r2) : C(0);
        macc[cc] = fma((Acc)kv, aj, macc[cc]);
        if (j < npj) kt[c * ldk + j] = to_k<K, C>(kv);
      }
    }
    lane_transpose_sum<Acc, CG>(macc, mu_part + wave * TM + cg);
  }
  __syncthreads();

  // ---- phase 2: v = (sf2 Linv) khat on the matrix cores ----------------------
  Acc ssq[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) ssq[ct] = 0;
  const int ntiles = npk / TI;
  // balanced assignment: row tile t goes to wave (t mod 8 < 4 ? t mod 8 : 7 - t mod 8)
  for (int ti = 0; ti < ntiles; ++ti) {
    const int r8 = ti % 8;
    if ((r8 < 4 ? r8 : 7 - r8) != wave) continue;
    const int nblk = ti / R + 1;
    const K* ablk = pk + tile_offset(ti, R) * 64 * (KB / 4) + lane * (KB / 4);
    if constexpr (P == GPBO_BF16) {
      f4 acc[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[ct] = f4{0, 0, 0, 0};
      for (int tj = 0; tj < nblk; ++tj) {
        const us8 av = *(const us8*)(ablk + (int64_t)tj * 64 * 8);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const us8 bv = *(const us8*)(kt + (ct * 16 + lane % 16) * ldk + tj * KB + 8 * (lane / 16));
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av),
                                                            __builtin_bit_cast(bf8, bv), acc[ct],
                                                            0, 0, 0);
        }
      }
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        ssq[ct] += acc[ct][0] * acc[ct][0] + acc[ct][1] * acc[ct][1] + acc[ct][2] * acc[ct][2] +
                   acc[ct][3] * acc[ct][3];
    } else if constexpr (P == GPBO_FP32) {
      f4 acc[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[ct] = f4{0, 0, 0, 0};
      for (int tj = 0; tj < nblk; ++tj) {
        const f4 av = *(const f4*)(ablk + (int64_t)tj * 64 * 4);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const f4 bv = *(const f4*)(kt + (ct * 16 + lane % 16) * ldk + tj * KB + 4 * (lane / 16));
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], bv[0], acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], bv[1], acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], bv[2], acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], bv[3], acc[ct], 0, 0, 0);
        }
      }
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        ssq[ct] += acc[ct][0] * acc[ct][0] + acc[ct][1] * acc[ct][1] + acc[ct][2] * acc[ct][2] +
                   acc[ct][3] * acc[ct][3];
    } else {
      d4 acc[NCT];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[ct] = d4{0, 0, 0, 0};
      for (int tj = 0; tj < nblk; ++tj) {
        const double* ap = (const double*)(ablk + (int64_t)tj * 64 * 4);
        const double2 a01 = *(const double2*)ap;
        const double2 a23 = *(const double2*)(ap + 2);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const double* bp =
              (const double*)(kt + (ct * 16 + lane % 16) * ldk + tj * KB + 4 * (lane / 16));
          const double2 b01 = *(const double2*)bp;
          const double2 b23 = *(const double2*)(bp + 2);
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b01.x, acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b01.y, acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b23.x, acc[ct], 0, 0, 0);
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b23.y, acc[ct], 0, 0, 0);
        }
      }
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        ssq[ct] += acc[ct][0] * acc[ct][0] + acc[ct][1] * acc[ct][1] + acc[ct][2] * acc[ct][2] +
                   acc[ct][3] * acc[ct][3];
    }
  }
  // lanes l, l+16, l+32, l+48 hold rows of the same candidate column l % 16
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    Acc v = ssq[ct];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) ssq_part[wave * TM + ct * 16 + lane] = v;
  }
  __syncthreads();

  // ---- phase 3: outputs and the tile's argmax ------------------------------
  if (t < 64) {
    double bv = -INFINITY;
    int64_t bi = -1;
    for (int c = t; c < TM; c += 64) {
      const int64_t gc = c0 + c;
      if (gc >= m) continue;
      const Acc muz = mu_part[c] + mu_part[TM + c] + mu_part[2 * TM + c] + mu_part[3 * TM + c];
      const Acc vv = ssq_part[c] + ssq_part[TM + c] + ssq_part[2 * TM + c] + ssq_part[3 * TM + c];
      Acc varz = (Acc)sf2_d - vv;
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
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int64_t oi = __shfl_xor(bi, o);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (t == 0 && part_v) {
      part_v[blockIdx.x] = bv;
      part_i[blockIdx.x] = bi;
    }
  }
}

__global__ void __launch_bounds__(256) k_argmax_final(const double* __restrict__ pv,
                                                      const int64_t* __restrict__ pi, int64_t np,
                                                      int64_t* __restrict__ argmax,
                                                      double* __restrict__ ei_max) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double bv = -INFINITY;
  int64_t bi = -1;
  for (int64_t k = threadIdx.x; k < np; k += 256) {
    if (better(pv[k], pi[k], bv, bi)) {
      bv = pv[k];
      bi = pi[k];
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double ov = sv[threadIdx.x + s];
      const int64_t oi = si[threadIdx.x + s];
      if (better(ov, oi, sv[threadIdx.x], si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (argmax) *argmax = si[0];
    if (ei_max) *ei_max = si[0] >= 0 ? sv[0] : -INFINITY;
  }
}

template <int P, int KERN, int TM, int DMAX>
void launch_fused_t(const ScoreJob& j, int ldk, size_t smem, hipStream_t s) {
  using T = PT<P>;
  const int64_t grid = ceil_div(j.m, TM);
  if (smem > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)k_score_fused<P, KERN, TM, DMAX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  hipLaunchKernelGGL((k_score_fused<P, KERN, TM, DMAX>), dim3((unsigned)grid), dim3(256), smem, s,
                     j.n, j.d, j.npk, (const typename T::K*)j.pk, (const typename T::Acc*)j.alpha,
                     (const typename T::C*)j.Xs, (const typename T::C*)j.sc, j.stats, j.sf2, j.m,
                     (const typename T::In*)j.Xc, (typename T::In*)j.mu,
                     (typename T::In*)j.sigma, (typename T::In*)j.ei, j.part_v, j.part_i, ldk);
}

template <int P, int KERN, int TM>
void launch_fused_d(const ScoreJob& j, int ldk, size_t smem, hipStream_t s) {
  if (j.d <= 16)
    launch_fused_t<P, KERN, TM, 16>(j, ldk, smem, s);
  else
    launch_fused_t<P, KERN, TM, 64>(j, ldk, smem, s);
}

template <int P, int KERN>
void launch_fused_tm(const ScoreJob& j, int tm, int ldk, size_t smem, hipStream_t s) {
  switch (tm) {
    case 16: launch_fused_d<P, KERN, 16>(j, ldk, smem, s); break;
    case 32: launch_fused_d<P, KERN, 32>(j, ldk, smem, s); break;
    default: launch_fused_d<P, KERN, 64>(j, ldk, smem, s); break;
  }
}

size_t esize(int prec) { return prec == GPBO_FP64 ? 8 : prec == GPBO_FP32 ? 4 : 2; }

// LDS row stride (elements) of the khat tile: rows 16-byte aligned and
// offset by 16 bytes modulo 128 so the 16 rows read by one matrix-core
// operand load fall in different banks.
int kt_stride(int prec, int npk) {
  const int kb = score_kb(prec);
  const int64_t bytes = round_up(round_up(npk, kb) * (int64_t)esize(prec), 128) + 16;
  return (int)(bytes / esize(prec));
}

size_t fused_smem(int prec, int n, int d, int tm) {
  const int npk = packed_rows(n);
  const int dmax = d <= 16 ? 16 : 64;
  const size_t csz = prec == GPBO_FP64 ? 8 : 4;
  return (size_t)tm * kt_stride(prec, npk) * esize(prec) + (size_t)tm * dmax * csz +
         8 * (size_t)tm * csz;
}

}  // namespace

int score_kb(int prec) { return prec == GPBO_BF16 ? 32 : 16; }

static int64_t packed_blocks(int n, int prec) {
  const int R = score_kb(prec) / TI;
  return tile_offset(packed_rows(n) / TI, R);
}

void ensure_score_operands(Model* M, int prec, hipStream_t s) {
  Ctx* c = M->ctx;
  const int n = M->n, d = M->d;
  if (!M->sc64) {
    // coordinate scales: 1/l for float64 and Matern; sqrt(log2(e)/2)/l for
    // the float32 squared-exponential path (one exp2 per covariance)
    std::vector<double> s64(d), s32(d);
    for (int k = 0; k < d; ++k) {
      s64[k] = 1.0 / M->ls[k];
      s32[k] = (M->kernel == GPBO_KERNEL_SE ? std::sqrt(0.5 * 1.4426950408889634) : 1.0) / M->ls[k];
    }
    std::vector<float> s32f(s32.begin(), s32.end());
    M->sc64 = (double*)dmalloc(c, d * sizeof(double));
    M->sc32 = (float*)dmalloc(c, d * sizeof(float));
    double* s32d = (double*)dmalloc(c, d * sizeof(double));
    hipMemcpyAsync(M->sc64, s64.data(), d * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(M->sc32, s32f.data(), d * sizeof(float), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(s32d, s32.data(), d * sizeof(double), hipMemcpyHostToDevice, s);
    M->Xs64 = (double*)dmalloc(c, (size_t)n * d * sizeof(double));
    M->Xs32 = (float*)dmalloc(c, (size_t)n * d * sizeof(float));
    const int g = (int)std::min<int64_t>(4096, ceil_div((int64_t)n * d, 256));
    hipLaunchKernelGGL(k_scale_obs<double>, dim3(g), dim3(256), 0, s, M->X64, M->sc64, n, d,
                       M->Xs64);
    hipLaunchKernelGGL(k_scale_obs<float>, dim3(g), dim3(256), 0, s, M->X64, s32d, n, d, M->Xs32);
    hipStreamSynchronize(s);
    dfree(c, s32d);
  }
  if (!M->pk[prec]) {
    const int64_t blocks = packed_blocks(n, prec);
    const int kb = score_kb(prec);
    const int64_t count = blocks * TI * kb;
    M->pk[prec] = dmalloc(c, count * esize(prec));
    const int g = (int)std::min<int64_t>(8192, ceil_div(count, 256));
    if (prec == GPBO_FP64) {
      hipLaunchKernelGGL(k_pack<double>, dim3(g), dim3(256), 0, s, M->Linv, M->npad, n, M->sf2, kb,
                         (double*)M->pk[prec], blocks);
      M->alphaT[prec] = dmalloc(c, n * sizeof(double));
      hipLaunchKernelGGL(k_scale_alpha<double>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M->alpha,
                         n, M->sf2, (double*)M->alphaT[prec]);
    } else {
      if (prec == GPBO_FP32)
        hipLaunchKernelGGL(k_pack<float>, dim3(g), dim3(256), 0, s, M->Linv, M->npad, n, M->sf2,
                           kb, (float*)M->pk[prec], blocks);
      else
        hipLaunchKernelGGL(k_pack<unsigned short>, dim3(g), dim3(256), 0, s, M->Linv, M->npad, n,
                           M->sf2, kb, (unsigned short*)M->pk[prec], blocks);
      M->alphaT[prec] = dmalloc(c, n * sizeof(float));
      hipLaunchKernelGGL(k_scale_alpha<float>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M->alpha,
                         n, M->sf2, (float*)M->alphaT[prec]);
    }
  }
}

int score_tile_m(int prec, int n, int d) {
  // Largest tile whose LDS footprint fits; prefer two workgroups per CU.
  const size_t lds = 160 * 1024;
  for (int tm : {64, 32, 16})
    if (2 * fused_smem(prec, n, d, tm) <= lds) return tm;
  for (int tm : {64, 32, 16})
    if (fused_smem(prec, n, d, tm) <= lds) return tm;
  return 0;
}

void launch_score(const ScoreJob& j, int prec, int tm, hipStream_t s) {
  const int ldk = kt_stride(prec, j.npk);
  const size_t smem = fused_smem(prec, j.n, j.d, tm);
  const bool se = j.kernel == GPBO_KERNEL_SE;
  switch (prec) {
    case GPBO_FP64:
      if (se) launch_fused_tm<GPBO_FP64, GPBO_KERNEL_SE>(j, tm, ldk, smem, s);
      else launch_fused_tm<GPBO_FP64, GPBO_KERNEL_MATERN52>(j, tm, ldk, smem, s);
      break;
    case GPBO_FP32:
      if (se) launch_fused_tm<GPBO_FP32, GPBO_KERNEL_SE>(j, tm, ldk, smem, s);
      else launch_fused_tm<GPBO_FP32, GPBO_KERNEL_MATERN52>(j, tm, ldk, smem, s);
      break;
    default:
      if (se) launch_fused_tm<GPBO_BF16, GPBO_KERNEL_SE>(j, tm, ldk, smem, s);
      else launch_fused_tm<GPBO_BF16, GPBO_KERNEL_MATERN52>(j, tm, ldk, smem, s);
      break;
  }
}

void launch_argmax_final(const double* pv, const int64_t* pi, int64_t np, int64_t* argmax,
                         double* ei_max, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(256), 0, s, pv, pi, np, argmax, ei_max);
}

}  // namespace gpbo
