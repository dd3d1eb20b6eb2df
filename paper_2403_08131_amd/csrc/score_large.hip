// Large-n scoring path (float32).  When n is large the cross-covariance tile
// of a useful number of candidates no longer fits in LDS, so the inverse
// factor would be re-streamed for every few candidates.  Instead, per chunk
// of candidates (sized to stay resident in the last-level cache):
//   1. k_kstar:    khat[c][j] = k(x*_c, x_j) / sf2 in float32 (VALU, lanes
//                  over training points, as in the fused kernel) and partial
//                  sums of (sf2 alpha_j) khat_cj per 256-point block;
//   2. k_trigemm:  v = (sf2 L^-1) khat on the float32 matrix cores, only the
//                  lower-triangular blocks, with a sum-of-squares epilogue:
//                  one partial |v|^2 per (64-row block, candidate);
//   3. k_finish:   mean, variance, EI, outputs and per-block argmax partials.
// The GEMM maps workgroups to XCDs so that every row block of one candidate
// block runs on the same XCD and reads that block's khat rows from one L2.
#include <algorithm>
#include <cmath>
#include <functional>

#include "score_common.h"

namespace gpbo {

using namespace sc;

namespace {

constexpr int KS_CG = 32;    // candidates per k_kstar workgroup
constexpr int KS_J = 256;    // training points per k_kstar workgroup
constexpr int GM_I = 128;    // inverse-factor rows per GEMM workgroup (8 row tiles)
constexpr int GM_C = 128;    // candidates per GEMM workgroup

template <int KERN>
__global__ void __launch_bounds__(256) k_kstar(int n, int d, int npj, int nx,
                                               const float* __restrict__ XsT,
                                               const float* __restrict__ sc,
                                               const float* __restrict__ alpha, int64_t m,
                                               int64_t cbeg, const float* __restrict__ Xc,
                                               float* __restrict__ khat, int ldk,
                                               float* __restrict__ mu_part, int64_t mc_pad) {
  __shared__ __align__(16) float xcT[64 * KS_CG];  // [d][KS_CG], d <= 64
  __shared__ float red[4][KS_CG];
  const int t = threadIdx.x, lane = t % 64, wave = wave_id();
  const int64_t cl0 = (int64_t)blockIdx.x * KS_CG;  // chunk-local first candidate
  const int jb = blockIdx.y * KS_J;
  for (int e = t; e < KS_CG * d; e += 256) {
    const int c = e / d, k = e % d;
    const int64_t gc = cbeg + cl0 + c;
    xcT[k * KS_CG + c] = gc < m ? Xc[gc * d + k] * sc[k] : 0.0f;
  }
  __syncthreads();
  const int j = jb + t;
  const bool valid = j < n;
  const float* xcol = XsT + (valid ? j : 0);
  float r2[KS_CG];
#pragma unroll
  for (int c = 0; c < KS_CG; ++c) r2[c] = 0.0f;
  float xnext = xcol[0];
  for (int k = 0; k < d; ++k) {
    const float xk = xnext;
    if (k + 1 < d) xnext = xcol[(int64_t)(k + 1) * nx];
    const float* xr = xcT + k * KS_CG;
#pragma unroll
    for (int c = 0; c < KS_CG; c += 4) {
      const f4 x4 = *(const f4*)(xr + c);
      const float u0 = xk - x4[0], u1 = xk - x4[1], u2 = xk - x4[2], u3 = xk - x4[3];
      r2[c] = fmaf(u0, u0, r2[c]);
      r2[c + 1] = fmaf(u1, u1, r2[c + 1]);
      r2[c + 2] = fmaf(u2, u2, r2[c + 2]);
      r2[c + 3] = fmaf(u3, u3, r2[c + 3]);
    }
  }
  const float aj = valid ? alpha[j] : 0.0f;
  float macc[KS_CG];
#pragma unroll
  for (int c = 0; c < KS_CG; ++c) {
    const float kv = valid ? cov_from_r2<KERN>(r2[c]) : 0.0f;
    macc[c] = kv * aj;
    if (j < npj && cl0 + c < mc_pad) khat[(cl0 + c) * ldk + j] = kv;
  }
  lane_transpose_sum<float, KS_CG>(macc, red[wave]);
  __syncthreads();
  if (t < KS_CG && cl0 + t < mc_pad)
    mu_part[(int64_t)blockIdx.y * mc_pad + cl0 + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// Posterior mean and the nearest-observation bounds (no triangular product):
// per candidate mu_z = sum_j khat_j (sf2 alpha_j) and khat_max = max_j khat_j;
// conditioning on one noisy observation alone leaves the latent variance
// sf2 - k^2 / (sf2 + sn2), and more observations only lower it, so
// var_ub = sf2 - (sf2 khat_max)^2 / (sf2 + sn2) bounds the posterior variance
// from above and EI(mu, sigma_ub) bounds EI.  Workgroup: KS_CG candidates,
// 256 threads over the training points (one point per thread per pass,
// coordinates read coalesced from the transposed scaled observations),
// partial sums and maxima in registers, then across lanes and waves.
struct BoundArgs {
  int n, d, nx, kernel;
  const float* XsT;      // d x nx scaled observations (padding points beyond n)
  const float* sc;       // d candidate coordinate scales
  const float* alpha;    // sf2 * alpha, zero beyond n
  const double* stats;   // ymean, ystd, fbest
  double sf2, sn2;
  int64_t m;
  const float* Xc;
  float* mu;
  float* sigma_ub;
  float* ei_ub;
};
template <int KERN>
__global__ void __launch_bounds__(256) k_score_bound(BoundArgs A) {
  __shared__ __align__(16) float xcT[64 * KS_CG];  // [d][KS_CG], d <= 64
  __shared__ float red_s[4][KS_CG], red_m[4][KS_CG];
  const int t = threadIdx.x, lane = t % 64, wave = wave_id();
  const int d = A.d, nx = A.nx;
  const int64_t c0 = (int64_t)blockIdx.x * KS_CG;
  for (int e = t; e < KS_CG * d; e += 256) {
    const int c = e / d, k = e % d;
    const int64_t gc = c0 + c;
    xcT[k * KS_CG + c] = gc < A.m ? A.Xc[gc * d + k] * A.sc[k] : 0.0f;
  }
  __syncthreads();
  float macc[KS_CG], kmax[KS_CG];
#pragma unroll
  for (int c = 0; c < KS_CG; ++c) {
    macc[c] = 0.0f;
    kmax[c] = 0.0f;
  }
  // columns n .. round_up(n, 64) - 1 are padding points (zero covariance and
  // zero alpha) inside the row stride nx
  const int jend = (int)round_up(A.n, 64);
  for (int j = t; j < jend; j += 256) {
    const float* xcol = A.XsT + j;
    float r2[KS_CG];
#pragma unroll
    for (int c = 0; c < KS_CG; ++c) r2[c] = 0.0f;
    float xnext = xcol[0];
    for (int k = 0; k < d; ++k) {
      const float xk = xnext;
      if (k + 1 < d) xnext = xcol[(int64_t)(k + 1) * nx];
      const float* xr = xcT + k * KS_CG;
#pragma unroll
      for (int c = 0; c < KS_CG; c += 4) {
        const f4 x4 = *(const f4*)(xr + c);
        const float u0 = xk - x4[0], u1 = xk - x4[1], u2 = xk - x4[2], u3 = xk - x4[3];
        r2[c] = fmaf(u0, u0, r2[c]);
        r2[c + 1] = fmaf(u1, u1, r2[c + 1]);
        r2[c + 2] = fmaf(u2, u2, r2[c + 2]);
        r2[c + 3] = fmaf(u3, u3, r2[c + 3]);
      }
    }
    const float aj = A.alpha[j];
#pragma unroll
    for (int c = 0; c < KS_CG; ++c) {
      const float kv = cov_from_r2<KERN>(r2[c]);
      macc[c] = fmaf(kv, aj, macc[c]);
      kmax[c] = fmaxf(kmax[c], kv);
    }
  }
  // across the 64 lanes: sums by the transpose-reduction, maxima by butterflies
  lane_transpose_sum<float, KS_CG>(macc, red_s[wave]);
#pragma unroll
  for (int c = 0; c < KS_CG; ++c) {
    float v = kmax[c];
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    kmax[c] = v;
  }
  if (lane < KS_CG) {
    float v = 0.0f;
#pragma unroll
    for (int c = 0; c < KS_CG; ++c) v = lane == c ? kmax[c] : v;
    red_m[wave][lane] = v;
  }
  __syncthreads();
  if (t < KS_CG && c0 + t < A.m) {
    const float muz = (red_s[0][t] + red_s[1][t]) + (red_s[2][t] + red_s[3][t]);
    const float km = fmaxf(fmaxf(red_m[0][t], red_m[1][t]), fmaxf(red_m[2][t], red_m[3][t]));
    const float sf2 = (float)A.sf2;
    const float kk = sf2 * km;
    float var = sf2 - kk * kk / (sf2 + (float)A.sn2);
    var = var > 0.0f ? var : 0.0f;
    const float ymean = (float)A.stats[S_YMEAN], sy = (float)A.stats[S_YSTD];
    const float mu = ymean + sy * muz;
    const float sg = sy * __builtin_sqrtf(var);
    const int64_t gc = c0 + t;
    if (A.mu) A.mu[gc] = mu;
    if (A.sigma_ub) A.sigma_ub[gc] = sg;
    if (A.ei_ub) A.ei_ub[gc] = ei_of<float>(mu, sg, (float)A.stats[S_FBEST]);
  }
}

// Triangular product with sum-of-squares epilogue.  Workgroup: 128 rows of
// the inverse factor (eight 16-row tiles) x 128 candidates, eight waves; wave
// (wp, wc) owns row tiles 2wp, 2wp + 1 of the block and candidates
// 64wc .. 64wc + 63.  Per stage of two 16-column blocks of the contraction,
// the packed A blocks of the eight row tiles and the 128 x 32 khat block are
// staged in LDS (each loaded from L2 once per workgroup, not once per wave),
// double buffered: stage s + 1 is loaded from memory while the products of
// stage s run from LDS, then stored, one barrier per stage.
constexpr int TG_W = 8;          // waves per workgroup
constexpr int TG_LDB = 36;       // LDS row stride (floats) of a staged khat row: 32 + 4 (banks)
constexpr int TG_AS = 2 * 8 * 2 * 256;        // floats of staged A: [stage][tile][block][256]
constexpr int TG_BS = 2 * GM_C * TG_LDB;      // floats of staged khat: [stage][cand][TG_LDB]
constexpr size_t TG_LDS = (size_t)(TG_AS + TG_BS) * sizeof(float);
__global__ void __launch_bounds__(64 * TG_W) k_trigemm(const float* __restrict__ khat, int ldk,
                                                       const float* __restrict__ pk,
                                                       const int64_t* __restrict__ pk_off,
                                                       int ntiles, int nib, int ncb,
                                                       float* __restrict__ ssq_part,
                                                       int64_t mc_pad) {
  extern __shared__ __align__(16) float tg_lds[];
  float* as = tg_lds;           // [2][8][2][256]
  float* bs = tg_lds + TG_AS;   // [2][GM_C][TG_LDB]
  __shared__ float red[4][GM_C];
  const int t = threadIdx.x, lane = t % 64, wave = wave_id();
  const int wp = wave / 2, wc = wave % 2;
  // XCD-aware order: workgroup b runs on XCD b % 8; all row blocks of one
  // candidate block share an XCD, heaviest row blocks first.
  const int b = blockIdx.x;
  const int xcd = b % 8, local = b / 8;
  const int cb = (local / nib) * 8 + xcd;
  const int I = nib - 1 - local % nib;
  if (cb >= ncb) return;  // whole workgroup: no barrier is skipped by part of it
  const int tlast = min(I * 8 + 7, ntiles - 1);  // last column block any row of the block needs
  const int ti0 = I * 8 + 2 * wp, ti1 = ti0 + 1;
  const bool has0 = ti0 < ntiles, has1 = ti1 < ntiles;
  const int nl = has1 ? ti1 : ti0;  // this wave's last column block
  // staging roles: A -- tile sr = t / 64 of the block, lane t % 64, both
  // blocks of the stage; khat -- candidate row t / 4, columns 4(t % 4) of
  // each of the two blocks
  const int sr = t / 64, sti = I * 8 + sr;
  const float* ap = pk + (sti < ntiles ? pk_off[sti] * 256 : 0) + lane * 4;
  const float* bp = khat + ((int64_t)cb * GM_C + t / 4) * ldk + 4 * (t % 4);
  const f4 zero = {0, 0, 0, 0};
  // blocks past a tile's own (and khat blocks past the last) are zeros
  auto fetch = [&](int tj, f4 (&av)[2], f4 (&bv)[2]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int bj = tj + u;
      av[u] = (sti < ntiles && bj <= sti) ? *(const f4*)(ap + (int64_t)bj * 256) : zero;
      bv[u] = bj <= tlast ? *(const f4*)(bp + bj * 16) : zero;
    }
  };
  auto stage = [&](int q, const f4 (&av)[2], const f4 (&bv)[2]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      *(f4*)&as[((q * 8 + sr) * 2 + u) * 256 + lane * 4] = av[u];
      *(f4*)&bs[(q * GM_C + t / 4) * TG_LDB + 16 * u + 4 * (t % 4)] = bv[u];
    }
  };
  f4 acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[r][ct] = zero;
  // products of block u of the stage in buffer q (step-major: consecutive
  // matrix-core instructions update different accumulators)
  auto mma = [&](int q, int u) {
    const f4 a0 = *(const f4*)&as[((q * 8 + 2 * wp) * 2 + u) * 256 + lane * 4];
    const f4 a1 = *(const f4*)&as[((q * 8 + 2 * wp + 1) * 2 + u) * 256 + lane * 4];
    f4 bv[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      bv[ct] = *(const f4*)&bs[(q * GM_C + wc * 64 + ct * 16 + lane % 16) * TG_LDB + 16 * u +
                               4 * (lane / 16)];
#pragma unroll
    for (int kk = 0; kk < Blk<GPBO_FP32>::KS; ++kk)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        Blk<GPBO_FP32>::mma_k(acc[0][ct], a0, bv[ct], kk);
        Blk<GPBO_FP32>::mma_k(acc[1][ct], a1, bv[ct], kk);
      }
  };
  auto mma_stage = [&](int q, int tj) {
    if (has0 && tj <= nl) mma(q, 0);
    if (has0 && tj + 1 <= nl) mma(q, 1);
  };
  {
    f4 av[2], bv[2];
    fetch(0, av, bv);
    stage(0, av, bv);
  }
  __syncthreads();
  // two stages (four blocks) per iteration so the buffer index is a constant
  for (int tj = 0; tj <= tlast; tj += 4) {
    f4 av[2], bv[2];
    if (tj + 2 <= tlast) fetch(tj + 2, av, bv);
    mma_stage(0, tj);
    if (tj + 2 > tlast) break;
    stage(1, av, bv);
    __syncthreads();
    if (tj + 4 <= tlast) fetch(tj + 4, av, bv);
    mma_stage(1, tj + 2);
    if (tj + 4 <= tlast) stage(0, av, bv);
    __syncthreads();
  }
  // per candidate column: sum of squares over this wave's 32 rows
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    float v = 0.0f;
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (r == 0 ? has0 : has1)
        v += acc[r][ct][0] * acc[r][ct][0] + acc[r][ct][1] * acc[r][ct][1] +
             acc[r][ct][2] * acc[r][ct][2] + acc[r][ct][3] * acc[r][ct][3];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) red[wp][wc * 64 + ct * 16 + lane] = v;
  }
  __syncthreads();
  if (t < GM_C) {
    const int64_t c = (int64_t)cb * GM_C + t;
    if (c < mc_pad)
      ssq_part[(int64_t)I * mc_pad + c] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
  }
}

__global__ void __launch_bounds__(256) k_finish(int64_t mc, int64_t mc_pad, int64_t cbeg, int njb,
                                                int nib, const float* __restrict__ mu_part,
                                                const float* __restrict__ ssq_part, double sf2,
                                                const double* __restrict__ stats,
                                                float* __restrict__ mu_out,
                                                float* __restrict__ sigma_out,
                                                float* __restrict__ ei_out,
                                                double* __restrict__ part_v,
                                                int64_t* __restrict__ part_i, int64_t pbase) {
  __shared__ double wv[4];
  __shared__ int64_t wi_[4];
  const int64_t cl = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double bv = -INFINITY;
  int64_t bi = -1;
  if (cl < mc) {
    float muz = 0.0f, vv = 0.0f;
    for (int q = 0; q < njb; ++q) muz += mu_part[(int64_t)q * mc_pad + cl];
    for (int q = 0; q < nib; ++q) vv += ssq_part[(int64_t)q * mc_pad + cl];
    finish_candidate<float, float>(cbeg + cl, muz, vv, sf2, stats, mu_out, sigma_out, ei_out, bv,
                                   bi);
  }
  wave_argmax(bv, bi);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (lane == 0) {
    wv[w] = bv;
    wi_[w] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0 && part_v) {
    double v = wv[0];
    int64_t i = wi_[0];
    for (int q = 1; q < 4; ++q)
      if (better(wv[q], wi_[q], v, i)) {
        v = wv[q];
        i = wi_[q];
      }
    part_v[pbase + blockIdx.x] = v;
    part_i[pbase + blockIdx.x] = i;
  }
}

}  // namespace

// Candidates per chunk: khat of a chunk stays within about 128 MiB.
int64_t large_chunk(int npj, int64_t m) {
  int64_t mc = (128ll << 20) / ((int64_t)npj * 4);
  mc = std::max<int64_t>(GM_C, mc / GM_C * GM_C);
  return std::min<int64_t>(mc, round_up(m, GM_C));
}

// Scratch bytes and argmax partial count of the large path for m candidates.
size_t large_scratch_bytes(int n, int npj, int64_t m) {
  const int64_t mc = large_chunk(npj, m);
  const int njb = (int)ceil_div(npj, KS_J), nib = (int)ceil_div(round_up(n, 16) / 16, GM_I / 16);
  return (size_t)mc * npj * 4 + (size_t)(njb + nib) * mc * 4 + 256;
}
// Exactly the number of partials the launch sequence writes (one per
// 256-candidate block of every chunk).
int64_t large_partials(int npj, int64_t m) {
  const int64_t mc = large_chunk(npj, m);
  return (m / mc) * ceil_div(mc, 256) + ceil_div(m % mc, 256);
}

void launch_score_large(const ScoreArgs& a, void* scratch, hipStream_t s,
                        const std::function<void(int)>& mark) {
  const int n = a.n, d = a.d, npj = a.npj;
  const int64_t m = a.m;
  const int64_t mc = large_chunk(npj, m);
  const int njb = (int)ceil_div(npj, KS_J);
  const int ntiles = (int)round_up(n, 16) / 16;
  const int nib = (int)ceil_div(ntiles, GM_I / 16);
  float* khat = (float*)scratch;
  float* mu_part = khat + (size_t)mc * npj;
  float* ssq_part = mu_part + (size_t)njb * mc;
  int64_t pbase = 0;
  for (int64_t cbeg = 0; cbeg < m; cbeg += mc) {
    const int64_t mcur = std::min<int64_t>(mc, m - cbeg);
    const int64_t mc_pad = round_up(mcur, GM_C);
    const dim3 gk((unsigned)ceil_div(mc_pad, KS_CG), (unsigned)njb);
    if (a.kernel == GPBO_KERNEL_SE)
      hipLaunchKernelGGL(k_kstar<GPBO_KERNEL_SE>, gk, dim3(256), 0, s, n, d, npj, a.nx,
                         (const float*)a.Xs, (const float*)a.sc, (const float*)a.alpha, m, cbeg,
                         (const float*)a.Xc, khat, npj, mu_part, mc_pad);
    else
      hipLaunchKernelGGL(k_kstar<GPBO_KERNEL_MATERN52>, gk, dim3(256), 0, s, n, d, npj, a.nx,
                         (const float*)a.Xs, (const float*)a.sc, (const float*)a.alpha, m, cbeg,
                         (const float*)a.Xc, khat, npj, mu_part, mc_pad);
    const int ncb = (int)(mc_pad / GM_C);
    const int nwg = (int)round_up(ncb, 8) * nib;  // XCD-aware order pads to whole groups of 8
    mark(0);
    static const bool lds_set = [] {
      return hipFuncSetAttribute((const void*)k_trigemm, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)TG_LDS) == hipSuccess;
    }();
    (void)lds_set;
    hipLaunchKernelGGL(k_trigemm, dim3(nwg), dim3(64 * TG_W), TG_LDS, s, khat, npj, (const float*)a.pk,
                       a.pk_off, ntiles, nib, ncb, ssq_part, mc_pad);
    mark(1);
    const int nfb = (int)ceil_div(mcur, 256);
    hipLaunchKernelGGL(k_finish, dim3(nfb), dim3(256), 0, s, mcur, mc_pad, cbeg, njb, nib, mu_part,
                       ssq_part, a.sf2, a.stats, (float*)a.mu, (float*)a.sigma, (float*)a.ei,
                       a.part_v, a.part_i, pbase);
    pbase += nfb;
  }
}

void launch_score_bound(const Model* M, int64_t m, const float* Xc, float* mu, float* sigma_ub,
                        float* ei_ub, hipStream_t s) {
  BoundArgs a{};
  a.n = M->n;
  a.d = M->d;
  a.nx = M->nx;
  a.kernel = M->kernel;
  a.XsT = M->Xs32;
  a.sc = M->sc32;
  a.alpha = (const float*)M->alphaT[GPBO_FP32];
  a.stats = M->stats;
  a.sf2 = M->sf2;
  a.sn2 = M->sn2;
  a.m = m;
  a.Xc = Xc;
  a.mu = mu;
  a.sigma_ub = sigma_ub;
  a.ei_ub = ei_ub;
  const dim3 grid((unsigned)ceil_div(m, KS_CG));
  if (M->kernel == GPBO_KERNEL_SE)
    hipLaunchKernelGGL(k_score_bound<GPBO_KERNEL_SE>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_score_bound<GPBO_KERNEL_MATERN52>, grid, dim3(256), 0, s, a);
}

}  // namespace gpbo
