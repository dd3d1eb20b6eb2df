// Scoring kernels: posterior mean, standard deviation and expected
// improvement of candidate configurations under a fitted Gaussian process,
// with an argmax (the acquisition step of Sec. III-A of the paper; formulas
// from Rasmussen & Williams 2006, eqs. 2.25-2.26, and Jones et al. 1998,
// eq. 15):
//
//   khat_j = k(x*, x_j) / sf2                cross-covariance, VALU
//   mu_z   = sum_j (sf2 alpha_j) khat_j       in registers, transpose-reduced
//   v      = (sf2 L^-1) khat                  matrix cores, triangular
//   var_z  = max(sf2 - |v|^2, 0)              sum-of-squares epilogue
//   mu = ymean + s_y mu_z,  sigma = s_y sqrt(var_z),  EI(mu, sigma, f_best)
//
// One workgroup (eight waves) scores one tile of TM candidates:
//   Phase 1: the scaled candidate tile sits in LDS, transposed (dimension-
//            major).  Each lane owns one training point; a uniform loop over
//            the input dimensions reads that point's coordinate from the
//            transposed observation matrix (coalesced) and updates CG squared
//            distances at once.  The covariances go to an LDS tile khat[c][j]
//            and alpha_j khat_cj accumulates in CG registers.
//   Phase 2: the waves split the 16-row tiles of the packed inverse factor
//            (streamed from L2 in the order the matrix-core lanes read it,
//            one pipeline group ahead), multiply against the LDS khat tile
//            and fold the squares of each finished output tile into per-lane
//            partial sums.
//   Phase 3: one thread per candidate combines the partials, evaluates EI,
//            writes the outputs and the tile's (EI, index) maximum.
// The single-problem launch has one workgroup per tile.  The batched launch
// (independent sub-searches, run in parallel per Sec. IV-D) is persistent:
// the (problem, tile) items, largest problems first, are dealt cyclically
// over its workgroups.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <type_traits>

#include "score_common.h"

namespace gpbo {

using namespace sc;

size_t score_esize(int prec);
int packed_npj(int n, int prec);
int kt_stride(int prec, int npj);

namespace {

// Per-problem arguments of the score-operand preparation kernels (problem
// blockIdx.y of a launch).
struct PrepDesc {
  int n, d, npad, ntiles, kb, nx;
  int obs;             // build the scaled observations
  double sf2;
  const double* Linv;  // npad x npad
  const double* X;     // n x d
  const double* alpha; // n
  const double* sc;    // 2d: 1 / l, then the float32 kernels' scales
  double* Xs64;        // d x nx
  float* Xs32;         // d x nx
  float* Xp32;         // dist_kp(d) x nx
  const int64_t* off;  // ntiles + 1 row-tile block offsets (NULL: no packed operand)
  void* pk;            // packed blocks (+ PF zero slack blocks)
  int64_t blocks;      // stored blocks including the slack
  void* alphaT;        // sf2 * alpha, precision-typed, nx (zero padded)
};

// Scaled coordinate of the padding points (columns n .. nx-1 of the scaled
// observations): far enough that every covariance with them is exactly 0,
// small enough that squared distances over 64 dimensions stay finite.
constexpr double kPadCoord = 1e15;

// Packed sf2 * Linv: row tile ti, column block tj holds a 16 x KB block in
// the lane order of Blk (off[t] .. off[t+1] are the blocks of row tile t;
// blocks past off[ntiles] are zero slack for the pipelined loads); then
// sf2 * alpha.  K: element type of the packed operand, A: of alpha.
template <typename K, typename A>
__global__ void __launch_bounds__(256) k_prep_pack(const PrepDesc* __restrict__ D) {
  const PrepDesc& P = D[blockIdx.y];
  if (!P.off) return;
  const int per = P.kb / 4, n = P.n, ntiles = P.ntiles;
  const int64_t cnt = P.blocks * 64 * per;
  const int64_t* __restrict__ off = P.off;
  K* __restrict__ out = (K*)P.pk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt + P.nx;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e >= cnt) {
      const int j = (int)(e - cnt);
      ((A*)P.alphaT)[j] = j < n ? (A)(P.sf2 * P.alpha[j]) : A(0);
      continue;
    }
    const int64_t blk = e / (64 * per);
    const int w = (int)(e % (64 * per));
    const int lane = w / per, q = w % per;
    double v = 0.0;
    if (blk < off[ntiles]) {
      int lo = 0, hi = ntiles - 1;  // row tile: largest t with off[t] <= blk
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (off[mid] <= blk) lo = mid; else hi = mid - 1;
      }
      const int ti = lo;
      const int tj = (int)(blk - off[ti]);
      const int i = ti * TI + lane % 16;
      const int j = tj * P.kb + per * (lane / 16) + q;
      if (i < n && j < n && j <= i) v = P.sf2 * P.Linv[(int64_t)i * P.npad + j];
    }
    store_elem(out + e, v);
  }
}

// Centre of the coordinates of the matrix-core distances: the middle of the
// unit box the search parameters are normalised to.  The expansion's
// rounding error grows with |u|^2, which centring reduces about fourfold for
// points spread over the box; distances themselves are unchanged.
constexpr double kDistCentre = 0.5;

// Transposed scaled coordinates of the observations, both precisions:
// Xs64[k][j] = X[j][k] / l_k, Xs32[k][j] = X[j][k] sc[d + k]; padding points
// past n.  Then the observation operand of the matrix-core distances:
// p_j = (2 u_j, -|u_j|^2, -1, 0 ...) with u_j = (X[j] - kDistCentre) sc32
// rounded to float32 (the squared norm summed in float64 and rounded once), stored
// dimension-major with the points of each 64-point block permuted so that
// one 16-byte load gives a lane its point in all four 16-point tiles:
// Xp32[k][64 b + 4 r + t] = p_{64 b + 16 t + r}[k].  A padding point has
// -|u|^2 = -1e30 (covariance exactly 0) and zeros elsewhere.
__global__ void __launch_bounds__(256) k_prep_obs(const PrepDesc* __restrict__ D) {
  const PrepDesc& P = D[blockIdx.y];
  if (!P.obs) return;
  const int n = P.n, d = P.d, nx = P.nx, kp = dist_kp(d);
  const int64_t ns = (int64_t)nx * d;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ns + (int64_t)nx * kp;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e >= ns) {
      const int64_t f = e - ns;
      const int k = (int)(f / nx), col = (int)(f % nx);
      const int w = col % 64;
      const int j = col - w + 16 * (w % 4) + w / 4;  // the point stored at this column
      float v = 0.0f;
      if (j < n) {
        auto u = [&](int q) {
          return (float)((P.X[(int64_t)j * d + q] - kDistCentre) * P.sc[d + q]);
        };
        if (k < d) {
          v = 2.0f * u(k);
        } else if (k == d) {
          double s2 = 0.0;
          for (int q = 0; q < d; ++q) s2 += (double)u(q) * (double)u(q);
          v = (float)-s2;
        } else if (k == d + 1) {
          v = -1.0f;
        }
      } else if (k == d) {
        v = -1e30f;
      }
      P.Xp32[f] = v;
      continue;
    }
    const int64_t k = e / nx, j = e % nx;
    if (j < n) {
      const double x = P.X[j * d + k];
      P.Xs64[e] = x * P.sc[k];
      P.Xs32[e] = (float)(x * P.sc[d + k]);
    } else {
      P.Xs64[e] = kPadCoord;
      P.Xs32[e] = (float)kPadCoord;
    }
  }
}

// Eight waves share one LDS tile; LDS allows at most two workgroups per CU,
// i.e. four waves per SIMD, and the register budget is stated accordingly.
constexpr int FW = 8;        // waves per scoring workgroup
constexpr int FT = FW * 64;  // threads per scoring workgroup

// The three phases of scoring one tile of TM candidates, written for a group
// of NW waves (w: the wave's index in the group, 0 .. NW-1).

// Scaled candidate tile, dimension-major: xcT[k][c] = Xc[c0 + c][k] sc[k].
template <int P, int TM, int NW>
__device__ __forceinline__ void stage_candidates(const ScoreArgs& A, int64_t tile,
                                                 typename PT<P>::C* xcT, int tid) {
  using C = typename PT<P>::C;
  using In = typename PT<P>::In;
  const int d = A.d;
  const int64_t c0 = tile * TM, m = A.m;
  const In* __restrict__ Xc = (const In*)A.Xc;
  const C* __restrict__ sc = (const C*)A.sc;
  // the matrix-core distances take coordinates centred on the unit box
  const C z = dist_mfma(P, d) ? C(kDistCentre) : C(0);
  for (int e = tid; e < TM * d; e += NW * 64) {
    const int c = e / d, k = e % d;
    xcT[k * TM + c] = c0 + c < m ? ((C)Xc[(c0 + c) * d + k] - z) * sc[k] : C(0);
  }
}

// Waves of the cross-covariance phase that share a candidate group: the
// number of 64-point blocks of the tile, rounded up to a power of two, at
// most NW.  The other NW / WP wave slots take other candidate groups, so a
// small problem still keeps every wave busy.
template <int NW>
__device__ __forceinline__ int cross_wp(int npj) {
  const int pb = (npj + 63) / 64;
  int wp = 1;
  while (wp < pb && wp < NW) wp *= 2;
  return wp;
}

// Phase 1: cross-covariance tile kt[c][j] and the mean partials
// mu_part[r][c], r = the 64-point-block residue of the wave (rows
// 0 .. cross_wp - 1).  Wave w takes point blocks w mod WP (stride WP) of the
// candidate groups of CG candidates numbered w / WP (stride NW / WP).
// DMAX > 0: points of up to DMAX dimensions keep all coordinates in
// registers; larger d (and DMAX = 0) stream them DC at a time.
template <int P, int KERN, int TM, int NW, int DMAX, int CG0 = 0, bool SPLIT = false>
__device__ __forceinline__ void phase_cross(const ScoreArgs& A, typename PT<P>::K* kt,
                                            const typename PT<P>::C* xcT,
                                            typename PT<P>::Acc* mu_part, int w) {
  using C = typename PT<P>::C;
  using K = typename PT<P>::K;
  using Acc = typename PT<P>::Acc;
  using V4 = typename PT<P>::V4;
  // candidates per register group (float64 halves it to avoid spills)
  constexpr int CGD = arith64(P) ? 16 : 32;
  constexpr int CGM = CG0 > 0 ? CG0 : CGD;
  constexpr int CG = TM < CGM ? TM : CGM;
  const int d = A.d, npj = A.npj, ldk = A.ldk, nx = A.nx;
  const Acc* __restrict__ alpha = (const Acc*)A.alpha;
  const C* __restrict__ XsT = (const C*)A.Xs;
  const int lane = threadIdx.x % 64;
  const int wp = SPLIT ? cross_wp<NW>(npj) : NW;
  // (cg0, cgs): first candidate group and stride; (pr, wp): point-block
  // residue and stride.  The full-width case (wp == NW) is a separate copy
  // with the candidate loop known at compile time; SPLIT = false (one
  // problem per launch) keeps only that copy.
  auto body = [&](const int cg0, const int cgs, const int pr, const int pws) {
  for (int cg = cg0; cg < TM; cg += cgs) {
    Acc macc[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) macc[c] = 0;
    for (int jb = pr * 64; jb < npj; jb += pws * 64) {
      // columns past n are padding points (zero covariance, zero alpha)
      const int j = jb + lane;
      const C* xcol = XsT + j;
      C r2[CG];
#pragma unroll
      for (int c = 0; c < CG; ++c) r2[c] = 0;
      // squared distances to this lane's point, one input dimension at a time
      auto dim = [&](C xk, int k) {
        const C* xr = xcT + k * TM + cg;
#pragma unroll
        for (int c = 0; c < CG; c += 4) {
          const V4 x4 = *(const V4*)(xr + c);
          const C u0 = xk - x4[0], u1 = xk - x4[1], u2 = xk - x4[2], u3 = xk - x4[3];
          r2[c] = fma(u0, u0, r2[c]);
          r2[c + 1] = fma(u1, u1, r2[c + 1]);
          r2[c + 2] = fma(u2, u2, r2[c + 2]);
          r2[c + 3] = fma(u3, u3, r2[c + 3]);
        }
      };
      if (DMAX > 0 && d <= DMAX) {
        // all of the point's coordinates requested at once: one memory
        // latency per point
        C xp[DMAX > 0 ? DMAX : 1];
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
          if (k < d) xp[k] = xcol[(int64_t)k * nx];
#pragma unroll
        for (int k = 0; k < DMAX; ++k)
          if (k < d) dim(xp[k], k);
      } else {
        // DC coordinates at a time, the next DC requested before the
        // current ones are used (indices past d are clamped to a valid
        // address and never used)
        constexpr int DC = 8;
        C xa[DC];
#pragma unroll
        for (int u = 0; u < DC; ++u) xa[u] = xcol[(int64_t)min(u, d - 1) * nx];
        for (int k0 = 0; k0 < d; k0 += DC) {
          C xb[DC];
#pragma unroll
          for (int u = 0; u < DC; ++u) xb[u] = xcol[(int64_t)min(k0 + DC + u, d - 1) * nx];
#pragma unroll
          for (int u = 0; u < DC; ++u)
            if (k0 + u < d) dim(xa[u], k0 + u);
#pragma unroll
          for (int u = 0; u < DC; ++u) xa[u] = xb[u];
        }
      }
      const Acc aj = alpha[j];
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        const C kv = cov_from_r2<KERN>(r2[c]);
        macc[c] = fma((Acc)kv, aj, macc[c]);
        kt[(cg + c) * ldk + j] = to_k<K, C>(kv);  // rows hold whole 64-point blocks
      }
    }
    lane_transpose_sum<Acc, CG>(macc, mu_part + pr * TM + cg);
  }
  };
  if (!SPLIT || wp == NW)
    body(0, CG, w, NW);
  else
    body((w / wp) * CG, (NW / wp) * CG, w % wp, wp);
}

// Phase 1 of the bfloat16 path (d + 2 <= 4 DIST_SMAX): the squared distances
// on the float32 matrix cores.  With the observation operand
// p_j = (2 u_j, -|u_j|^2, -1, 0 ...) and the candidate operand
// q_c = (u_c, 1, |u_c|^2, 0 ...), p_j . q_c = -|u_j - u_c|^2: one
// 16 x 16 x 4 product per (16 points, 16 candidates, 4 terms).  The
// expansion loses to cancellation about eps_32 (|u_j|^2 + |u_c|^2) of
// absolute accuracy in the squared distance (relative to the covariance: the
// same times ln 2), below the bfloat16 rounding of the tile for scaled
// coordinates up to |u|^2 ~ 1e4.  Wave w takes candidate group w mod
// (TM / 16) and every (NW / (TM / 16))-th 64-point block from w / (TM / 16);
// lane l holds four consecutive points 4 (l / 16) .. of each 16-point tile
// for candidate l mod 16, so the covariances of a tile leave as one 8-byte
// LDS store and the mean partial as one accumulator per lane.  Rows
// 0 .. NW / (TM / 16) - 1 of mu_part are written.
template <int KERN, int TM, int NW>
__device__ __forceinline__ void phase_cross_mfma(const ScoreArgs& A, unsigned short* kt,
                                                 const float* xcT, float* mu_part, int w) {
  constexpr int NCG = TM / 16;   // candidate groups of 16
  constexpr int WPG = NW / NCG;  // waves per candidate group
  static_assert(NCG <= NW && NW % NCG == 0, "candidate groups must divide the waves");
  const int d = A.d, npj = A.npj, ldk = A.ldk, nx = A.nx;
  const int S = dist_kp(d) / 4;  // matrix-core steps
  const int lane = threadIdx.x % 64;
  const int r = lane % 16, kq = lane / 16;
  const int cg = w % NCG, pr = w / NCG;
  const int c = cg * 16 + r;
  // candidate operand of step s: q_c[4 s + l / 16], from the LDS tile
  float nrm = 0.0f;
  for (int k = 0; k < d; ++k) {
    const float u = xcT[k * TM + c];
    nrm = fmaf(u, u, nrm);
  }
  float qb[DIST_SMAX];
#pragma unroll
  for (int s = 0; s < DIST_SMAX; ++s) {
    const int k = 4 * s + kq;
    float v = 0.0f;
    if (k < d) v = xcT[k * TM + c];
    else if (k == d) v = 1.0f;
    else if (k == d + 1) v = nrm;
    qb[s] = v;
  }
  const float* __restrict__ Xp = A.Xp + kq * (int64_t)nx + 4 * r;
  const float* __restrict__ alpha = (const float*)A.alpha + 4 * kq;
  unsigned short* krow = kt + c * ldk + 4 * kq;
  float macc = 0.0f;
  // the observation operand in two halves of SH steps (the second only for
  // d + 2 > 4 SH), to bound the live registers (requesting the next block's
  // first half ahead of this block's covariances was measured: 12 % more
  // vector instructions, no gain)
  constexpr int SH = DIST_SMAX / 2;
  for (int jb = pr * 64; jb < npj; jb += WPG * 64) {
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h * SH >= S) break;
      f4 a[SH];
#pragma unroll
      for (int s = 0; s < SH; ++s)
        if (h * SH + s < S) a[s] = *(const f4*)(Xp + 4 * (h * SH + s) * (int64_t)nx + jb);
#pragma unroll
      for (int s = 0; s < SH; ++s)
        if (h * SH + s < S)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s][t], qb[h * SH + s], acc[t], 0, 0, 0);
    }
    f4 al[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) al[t] = *(const f4*)(alpha + jb + 16 * t);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float kv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        kv[i] = cov_from_r2<KERN>(fmaxf(-acc[t][i], 0.0f));
        macc = fmaf(kv[i], al[t][i], macc);
      }
      *(uint2*)(krow + jb + 16 * t) = make_uint2(bf16_pair(kv[0], kv[1]), bf16_pair(kv[2], kv[3]));
    }
  }
  // lanes l, l + 16, l + 32, l + 48 hold the same candidate
  macc += __shfl_xor(macc, 16);
  macc += __shfl_xor(macc, 32);
  if (lane < 16) mu_part[pr * TM + cg * 16 + lane] = macc;
}

// Phase 2: v = (sf2 Linv) khat on the matrix cores; ssq_part[w][c] receives
// this wave's sum of squares of v over its row tiles.  A wave takes RT
// consecutive row tiles per pass so that every B operand read from the LDS
// tile feeds RT products (with RT = 1 the LDS read rate, not the matrix
// cores, bounds the phase); RT = 1 keeps the register count low.
template <int P, int TM, int NW, int RT>
__device__ __forceinline__ void phase_variance(const ScoreArgs& A, const typename PT<P>::K* kt,
                                               typename PT<P>::Acc* ssq_part, int w) {
  using K = typename PT<P>::K;
  using Acc = typename PT<P>::Acc;
  constexpr int KB = PT<P>::KB;
  constexpr int NCT = TM / 16;  // candidate tiles of 16 per workgroup
  constexpr int PF = Blk<P>::PF;
  using V = typename Blk<P>::V;
  const int npk = A.npk, ldk = A.ldk;
  const int64_t* __restrict__ pk_off = A.pk_off;
  const K* __restrict__ pk = (const K*)A.pk;
  const int lane = threadIdx.x % 64;
  const K* bbase = kt + (lane % 16) * ldk + (KB / 4) * (lane / 16);
  Acc ssq[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) ssq[ct] = 0;
  const int ntiles = npk / TI;
  const int ngroups = (ntiles + RT - 1) / RT;
  // balanced assignment: group g goes to wave s or 2NW-1-s, s = g mod 2NW
  for (int g = 0; g < ngroups; ++g) {
    const int r = g % (2 * NW);
    if ((r < NW ? r : 2 * NW - 1 - r) != w) continue;
    // row tiles RT g .. RT g + RT - 1.  Block counts grow with the tile
    // index, so the last tile's count bounds the loop and every earlier
    // tile ends at a group boundary (counts are multiples of PF): a group
    // below the first tile's count multiplies every tile, one past it only
    // the last.  With RT = 2 and the second tile missing, the first tile
    // takes the last slot and the first slot stays empty.
    static_assert(RT == 1 || RT == 2, "one or two row tiles per group");
    constexpr int R = KB / TI;  // row tiles per column block
    const K* ablk[RT];
    int nfirst, nact[RT];  // nfirst: stored (PF-rounded) blocks of the first tile; nact: real blocks
    {
      const int t0 = RT * g;
      const int64_t o0 = pk_off[t0], o1 = pk_off[t0 + 1];
      if (RT == 1) {
        ablk[0] = pk + o0 * Blk<P>::EPB + lane * (KB / 4);
        nfirst = (int)(o1 - o0);
        nact[0] = t0 / R + 1;
      } else if (t0 + 1 < ntiles) {
        ablk[0] = pk + o0 * Blk<P>::EPB + lane * (KB / 4);
        ablk[RT - 1] = pk + o1 * Blk<P>::EPB + lane * (KB / 4);
        nfirst = (int)(o1 - o0);
        nact[0] = t0 / R + 1;
        nact[RT - 1] = (t0 + 1) / R + 1;
      } else {
        ablk[0] = ablk[RT - 1] = pk + o0 * Blk<P>::EPB + lane * (KB / 4);
        nfirst = 0;
        nact[0] = 0;
        nact[RT - 1] = t0 / R + 1;
      }
    }
    const int nlast = nact[RT - 1];
    typename Blk<P>::Acc acc[RT][NCT];
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[q][ct] = typename Blk<P>::Acc{0, 0, 0, 0};
    // one pipeline group: per block, the B operands from LDS, then the
    // products of tiles Q0 .. RT - 1; a group that reaches past a tile's real
    // blocks (the stored ones are rounded up to PF with zeros) skips them
    auto group = [&](const V (&a)[RT][PF], int tj0, auto q0, auto full) {
      constexpr int Q0 = decltype(q0)::value;
      constexpr bool FULL = decltype(full)::value;
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        V bv[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) bv[ct] = Blk<P>::load(bbase + ct * 16 * ldk + (tj0 + u) * KB);
#pragma unroll
        for (int kk = 0; kk < Blk<P>::KS; ++kk)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int q = Q0; q < RT; ++q)
              if (FULL || tj0 + u < nact[q]) Blk<P>::mma_k(acc[q][ct], a[q][u], bv[ct], kk);
      }
    };
    // The packed blocks stream from L2 one group ahead (a group past the
    // last tile's end reads the next tile or the zero slack and is not used).
    auto fetch = [&](V (&a)[RT][PF], int tj0, auto q0) {
      constexpr int Q0 = decltype(q0)::value;
#pragma unroll
      for (int q = Q0; q < RT; ++q)
#pragma unroll
        for (int u = 0; u < PF; ++u) a[q][u] = Blk<P>::load(ablk[q] + (int64_t)(tj0 + u) * Blk<P>::EPB);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
    };
    using All = std::integral_constant<int, 0>;
    using Last = std::integral_constant<int, RT - 1>;
    using Full = std::true_type;
    using Part = std::false_type;
    auto fetch_at = [&](V (&a)[RT][PF], int tj0) {
      if (tj0 < nfirst) fetch(a, tj0, All{}); else fetch(a, tj0, Last{});
    };
    auto group_at = [&](const V (&a)[RT][PF], int tj0) {
      if (tj0 < nfirst) {
        if (tj0 + PF <= nact[0]) group(a, tj0, All{}, Full{}); else group(a, tj0, All{}, Part{});
      } else {
        if (tj0 + PF <= nlast) group(a, tj0, Last{}, Full{}); else group(a, tj0, Last{}, Part{});
      }
    };
    V ra[RT][PF], rb[RT][PF];
    fetch_at(ra, 0);
    for (int tj0 = 0; tj0 < nlast; tj0 += 2 * PF) {
      fetch_at(rb, tj0 + PF);
      group_at(ra, tj0);
      if (tj0 + PF >= nlast) break;
      fetch_at(ra, tj0 + 2 * PF);
      group_at(rb, tj0 + PF);
    }
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        ssq[ct] += acc[q][ct][0] * acc[q][ct][0] + acc[q][ct][1] * acc[q][ct][1] +
                   acc[q][ct][2] * acc[q][ct][2] + acc[q][ct][3] * acc[q][ct][3];
  }
  // lanes l, l+16, l+32, l+48 hold rows of the same candidate column l % 16
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    Acc v = ssq[ct];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) ssq_part[w * TM + ct * 16 + lane] = v;
  }
}

// Phase 3 (one wave): outputs and the tile's argmax from the partials of
// NW waves.
template <int P, int TM, int NW>
__device__ __forceinline__ void phase_finish(const ScoreArgs& A, int64_t tile,
                                             const typename PT<P>::Acc* mu_part,
                                             const typename PT<P>::Acc* ssq_part, int wp) {
  using Acc = typename PT<P>::Acc;
  using In = typename PT<P>::In;
  const int lane = threadIdx.x % 64;
  const int64_t c0 = tile * TM, m = A.m;
  // wp: rows of mu_part written by phase 1
  double bv = -INFINITY;
  int64_t bi = -1;
  for (int c = lane; c < TM; c += 64) {
    const int64_t gc = c0 + c;
    if (gc >= m) continue;
    Acc muz = 0, vv = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (w < wp) muz += mu_part[w * TM + c];
      vv += ssq_part[w * TM + c];
    }
    finish_candidate<Acc, In>(gc, muz, vv, A.sf2, A.stats, (In*)A.mu, (In*)A.sigma, (In*)A.ei, bv,
                              bi);
  }
  wave_argmax(bv, bi);
  if (lane == 0 && A.part_v) {
    A.part_v[tile] = bv;
    A.part_i[tile] = bi;
  }
}

// Score candidate tile `tile` of problem A (TM candidates from tile * TM)
// with all FW waves of the workgroup in every phase.
// xc_off >= 0 (the batched kernel): the candidate tile and the partial sums
// sit at fixed byte offsets sized for the batch's largest row stride and d,
// so no area of one item depends on the problem of another.
template <int P, int KERN, int TM, int RT, int CG = 0, bool SPLIT = false>
__device__ __forceinline__ void score_tile(const ScoreArgs& A, int64_t tile,
                                           unsigned char* smem, int xc_off = -1,
                                           int part_off = -1) {
  using C = typename PT<P>::C;
  using K = typename PT<P>::K;
  using Acc = typename PT<P>::Acc;
  const int d = A.d, ldk = A.ldk;
  K* kt = (K*)smem;                                            // [TM][ldk]
  C* xcT = (C*)(smem + (xc_off >= 0 ? (size_t)xc_off : (size_t)TM * ldk * sizeof(K)));  // [d][TM]
  Acc* mu_part = part_off >= 0 ? (Acc*)(smem + part_off)
                               : (Acc*)(xcT + round_up((int64_t)d * TM, 4));  // [FW][TM]
  Acc* ssq_part = mu_part + FW * TM;                                          // [FW][TM]
  const int wave = wave_id();
  stage_candidates<P, TM, FW>(A, tile, xcT, threadIdx.x);
  __syncthreads();
  int mu_rows;
  if constexpr (P == GPBO_BF16) {
    if (dist_mfma(P, d)) {
      phase_cross_mfma<KERN, TM, FW>(A, kt, xcT, mu_part, wave);
      mu_rows = FW / (TM / 16);
    } else {
      phase_cross<P, KERN, TM, FW, 0, CG, SPLIT>(A, kt, xcT, mu_part, wave);
      mu_rows = SPLIT ? cross_wp<FW>(A.npj) : FW;
    }
  } else {
    phase_cross<P, KERN, TM, FW, 0, CG, SPLIT>(A, kt, xcT, mu_part, wave);
    mu_rows = SPLIT ? cross_wp<FW>(A.npj) : FW;
  }
  __syncthreads();
  phase_variance<P, TM, FW, RT>(A, kt, ssq_part, wave);
  __syncthreads();
  if (wave == 0) phase_finish<P, TM, FW>(A, tile, mu_part, ssq_part, mu_rows);
}

// Below 64 candidates per workgroup the LDS tile leaves room for a second
// workgroup per CU; at 128 registers or fewer (four waves per SIMD) it fits,
// and one workgroup's cross-covariance phase overlaps the other's products.
template <int P, int KERN, int TM>
__global__ void __launch_bounds__(FT)
    __attribute__((amdgpu_waves_per_eu((TM == 64 || arith64(P)) ? 1 : 4, 4)))
k_score_fused(ScoreArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the float32 path of a model whose escalation is decided here: the
  // kernel that does not apply returns at once
  if (A.gate && escalate_fp64(A.stats[S_KINV]) != (A.gate == 2)) return;
  // two float64 row tiles over 64 candidates exceed the register file
  constexpr int RT = (arith64(P) && TM == 64) ? 1 : 2;
  score_tile<P, KERN, TM, RT>(A, blockIdx.x, smem);
}

// Persistent batched scoring over the work items of one class of a plan:
// items 0 .. total-1 enumerate (problem, tile) pairs, the k-th problem of the
// class (descriptor idx[k]) owning items [begin[k], begin[k+1]).  Every
// workgroup leaves its loop once its next item index passes the total.
// Problem starts of up to BT_MAX problems are looked up in LDS.  Candidate
// groups of 16 keep every wave of the cross-covariance phase busy on the
// small problems of a batch.
constexpr int BT_MAX = 256;

// The same address, known to the compiler as device-global memory (a round
// trip through the global address space), so loads and stores through it are
// global rather than flat instructions.
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
  __attribute__((address_space(1))) T* g = (__attribute__((address_space(1))) T*)p;
  __asm__("" : "+s"(g));  // keeps the cast pair from being folded away
  return (T*)g;
}

// Device plan of a batched launch (batch_plan_bytes(B) bytes): per class c
// (0: the launch precision, 1: the float64 escalation of the float32 path)
// the number of problems and work items, the problems' descriptor indices
// and first items; per descriptor, the tile count of its argmax partials.
struct PlanHdr {
  int count[2];
  int pad[2];
  int64_t total[2];
};
struct PlanView {
  PlanHdr* hdr;
  int* idx;         // [2][B]
  int64_t* begin;   // [2][B]
  int64_t* nparts;  // [B]
};
__host__ __device__ inline PlanView plan_view(void* base, int B) {
  PlanView v;
  char* p = (char*)base;
  v.hdr = (PlanHdr*)p;
  p += sizeof(PlanHdr);
  v.idx = (int*)p;
  p += round_up(2 * (int64_t)B * sizeof(int), 16);
  v.begin = (int64_t*)p;
  p += 2 * (int64_t)B * sizeof(int64_t);
  v.nparts = (int64_t*)p;
  return v;
}

// One workgroup: each problem's class (escalate = 1: from its fit's
// conditioning statistic), then per class an ordered prefix sum of the work
// items over chunks of 256 problems (descriptor order, i.e. largest first,
// is kept within each class).
__global__ void __launch_bounds__(256) k_plan_batched(const ScoreArgs* __restrict__ dd, int B,
                                                      int tm0, int tm1, int escalate, void* plan) {
  __shared__ int64_t sc[2][256];
  __shared__ int sn[2][256];
  __shared__ int64_t run_items[2];
  __shared__ int run_count[2];
  const PlanView v = plan_view(plan, B);
  const int t = threadIdx.x;
  if (t < 2) {
    run_items[t] = 0;
    run_count[t] = 0;
  }
  __syncthreads();
  for (int k0 = 0; k0 < B; k0 += 256) {
    const int k = k0 + t;
    int cls = 0;
    int64_t items = 0;
    if (k < B) {
      const ScoreArgs& A = dd[k];
      cls = escalate && escalate_fp64(A.stats[S_KINV]) ? 1 : 0;
      items = (A.m + (cls ? tm1 : tm0) - 1) / (cls ? tm1 : tm0);
      v.nparts[k] = items;
    }
    // inclusive scans of (is in class c) and (items if in class c)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      sn[c][t] = (k < B && cls == c) ? 1 : 0;
      sc[c][t] = (k < B && cls == c) ? items : 0;
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int a0 = 0, a1 = 0;
      int64_t b0 = 0, b1 = 0;
      if (t >= o) {
        a0 = sn[0][t - o];
        a1 = sn[1][t - o];
        b0 = sc[0][t - o];
        b1 = sc[1][t - o];
      }
      __syncthreads();
      sn[0][t] += a0;
      sn[1][t] += a1;
      sc[0][t] += b0;
      sc[1][t] += b1;
      __syncthreads();
    }
    if (k < B) {
      const int pos = run_count[cls] + sn[cls][t] - 1;
      v.idx[cls * B + pos] = k;
      v.begin[cls * B + pos] = run_items[cls] + sc[cls][t] - items;
    }
    __syncthreads();
    if (t < 2) {
      run_count[t] += sn[t][255];
      run_items[t] += sc[t][255];
    }
    __syncthreads();
  }
  if (t < 2) {
    v.hdr->count[t] = run_count[t];
    v.hdr->total[t] = run_items[t];
  }
}

// Two workgroups per CU: the bfloat16 variant is held to the 128 registers
// of four waves per SIMD (its matrix-core distances would otherwise take
// more); the others stay there without a cap.
// A descriptor read from LDS, every 32-bit word made wave-uniform (scalar
// registers), as a scalar load from global memory would leave it.
__device__ __forceinline__ ScoreArgs uniform_args(const ScoreArgs* p) {
  static_assert(sizeof(ScoreArgs) % 4 == 0, "descriptor of whole words");
  ScoreArgs a;
  const int* src = (const int*)p;
  int* dst = (int*)&a;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ScoreArgs) / 4); ++i)
    dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return a;
}

// Items are dealt cyclically: workgroup g takes items g, g + G, g + 2G, ...
// (G workgroups).  The items enumerate (problem, tile) with the problems in
// decreasing n, so every round deals tiles of similar cost and the totals
// stay balanced; no shared counter is popped (8192 items over 512
// workgroups on one global atomic queued behind each other), and the next
// item's candidates are staged while wave 0 still finishes the current one.
// desc_off > 0: byte offset in the dynamic LDS (past the tile areas) where
// the workgroup keeps a copy of the class's descriptors, in class order,
// loaded once at its start; per item the descriptor then comes from LDS
// instead of a dependent pair of global loads (problem index, then
// descriptor).
template <int P, int TM>
__global__ void __launch_bounds__(FT)
    __attribute__((amdgpu_waves_per_eu(P == GPBO_BF16 ? 4 : 1, 4)))
k_score_batched(const ScoreArgs* __restrict__ descs, int B, int cls, const void* plan,
                int xc_off, int part_off, int desc_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t begin_s[BT_MAX];
  const PlanView v = plan_view(const_cast<void*>(plan), B);
  const int cnt = __builtin_amdgcn_readfirstlane(v.hdr->count[cls]);
  const int64_t total = v.hdr->total[cls];
  const int* __restrict__ idx = v.idx + cls * B;
  const int64_t* __restrict__ begin = v.begin + cls * B;
  const bool lds_table = cnt <= BT_MAX;
  if (lds_table)
    for (int b = threadIdx.x; b < cnt; b += FT) begin_s[b] = begin[b];
  ScoreArgs* desc_s = desc_off > 0 ? (ScoreArgs*)(smem + desc_off) : nullptr;
  if (desc_s) {
    constexpr int W = (int)(sizeof(ScoreArgs) / 4);
    for (int e = threadIdx.x; e < cnt * W; e += FT) {
      const int k = e / W, w = e % W;
      ((int*)(desc_s + k))[w] = ((const int*)(descs + idx[k]))[w];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x % 64;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int lo;  // largest k with begin[k] <= item (the starts increase)
    if (lds_table && cnt <= 64) {
      // one comparison per lane: the lanes whose start is reached form a prefix
      const bool reached = lane < cnt && begin_s[lane] <= item;
      lo = __popcll(__ballot(reached)) - 1;
    } else {
      int l = 0, hi = cnt - 1;
      while (l < hi) {
        const int mid = (l + hi + 1) / 2;
        const int64_t tb = lds_table ? begin_s[mid] : begin[mid];
        if (tb <= item) l = mid; else hi = mid - 1;
        l = __builtin_amdgcn_readfirstlane(l);
        hi = __builtin_amdgcn_readfirstlane(hi);
      }
      lo = l;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const int64_t tile = item - (lds_table ? begin_s[lo] : begin[lo]);
    ScoreArgs A = desc_s ? uniform_args(desc_s + lo)
                         : descs[__builtin_amdgcn_readfirstlane(idx[lo])];
    // the descriptor's pointers are device-global memory: loads through them
    // become global (not flat) loads, with their own wait counter
    A.Xc = global_ptr(A.Xc);
    A.mu = global_ptr(A.mu);
    A.sigma = global_ptr(A.sigma);
    A.Xs = global_ptr(A.Xs);
    A.Xp = global_ptr(A.Xp);
    A.sc = global_ptr(A.sc);
    A.alpha = global_ptr(A.alpha);
    A.pk = global_ptr(A.pk);
    A.pk_off = global_ptr(A.pk_off);
    A.stats = global_ptr(A.stats);
    A.ei = global_ptr(A.ei);
    A.part_v = global_ptr(A.part_v);
    A.part_i = global_ptr(A.part_i);
    if (A.kernel == GPBO_KERNEL_SE)
      score_tile<P, GPBO_KERNEL_SE, TM, 1, 16, true>(A, tile, smem, xc_off, part_off);
    else
      score_tile<P, GPBO_KERNEL_MATERN52, TM, 1, 16, true>(A, tile, smem, xc_off, part_off);
    // No barrier here: the waves that are done stage the next item's
    // candidates while wave 0 still finishes this one.  The finish reads only
    // the partial sums, at fixed offsets apart from the candidate tile; the
    // next item's first phase writes them (and the covariance tile) only
    // after the staging barrier, which wave 0 reaches when it is done.
  }
}

// Block-wide (value, index) maximum over np partials.
__device__ __forceinline__ void block_argmax(const double* __restrict__ pv,
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

__global__ void __launch_bounds__(256) k_argmax_final(const double* __restrict__ pv,
                                                      const int64_t* __restrict__ pi, int64_t np,
                                                      int64_t* __restrict__ argmax,
                                                      double* __restrict__ ei_max) {
  block_argmax(pv, pi, np, argmax, ei_max);
}

// The single float32 launch whose escalation was decided on the device:
// the partials of whichever kernel ran.
__global__ void __launch_bounds__(256) k_argmax_gated(const double* __restrict__ pv,
                                                      const int64_t* __restrict__ pi, int64_t np32,
                                                      int64_t np64, const double* __restrict__ stats,
                                                      int64_t* __restrict__ argmax,
                                                      double* __restrict__ ei_max) {
  block_argmax(pv, pi, escalate_fp64(stats[S_KINV]) ? np64 : np32, argmax, ei_max);
}

// One workgroup per problem of a batch (descriptor blockIdx.x; its tile
// count from the plan).
__global__ void __launch_bounds__(256) k_argmax_batched(const ScoreArgs* __restrict__ descs, int B,
                                                        const void* plan,
                                                        int64_t* __restrict__ argmax,
                                                        double* __restrict__ ei_max) {
  const ScoreArgs& A = descs[blockIdx.x];
  const PlanView v = plan_view(const_cast<void*>(plan), B);
  block_argmax(A.part_v, A.part_i, v.nparts[blockIdx.x], argmax ? argmax + A.slot : nullptr,
               ei_max ? ei_max + A.slot : nullptr);
}

template <typename F>
void allow_smem(F f, size_t smem) {
  if (smem > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)smem);
}

template <int P, int KERN, int TM>
void launch_fused_t(const ScoreArgs& a, size_t smem, hipStream_t s) {
  allow_smem(k_score_fused<P, KERN, TM>, smem);
  hipLaunchKernelGGL((k_score_fused<P, KERN, TM>), dim3((unsigned)ceil_div(a.m, TM)), dim3(FT),
                     smem, s, a);
}

template <int P, int KERN>
void launch_fused_tm(const ScoreArgs& a, int tm, size_t smem, hipStream_t s) {
  switch (tm) {
    case 16: launch_fused_t<P, KERN, 16>(a, smem, s); break;
    case 32: launch_fused_t<P, KERN, 32>(a, smem, s); break;
    default: launch_fused_t<P, KERN, 64>(a, smem, s); break;
  }
}

// The descriptor copy in LDS is taken when it keeps per_cu workgroups per
// CU (with the kernel's static LDS, ~2.1 KB).
constexpr size_t kBatchedStaticLds = 2560;
// The tile areas of the batch: the covariance tile for the largest row
// stride, then the candidate tile for the largest d, then the partial sums
// (score_smem of the largest n and d, the size the caller passes).
template <int P, int TM>
void launch_batched_t(const ScoreArgs* dd, int B, int cls, void* plan, int nmax, int dmax,
                      size_t smem, int grid, int per_cu, hipStream_t s) {
  const size_t xc_off = (size_t)TM * kt_stride(P, packed_npj(nmax, P)) * score_esize(P);
  const size_t part_off = xc_off + (size_t)round_up((int64_t)dmax * TM, 4) * (arith64(P) ? 8 : 4);
  const size_t off = round_up((int64_t)smem, 16);
  const size_t with = off + (size_t)B * sizeof(ScoreArgs);
  const bool cache = off > 0 && (size_t)per_cu * (with + kBatchedStaticLds) <= 160 * 1024;
  const size_t dyn = cache ? with : smem;
  allow_smem(k_score_batched<P, TM>, dyn);
  hipLaunchKernelGGL((k_score_batched<P, TM>), dim3(grid), dim3(FT), dyn, s, dd, B, cls,
                     (const void*)plan, (int)xc_off, (int)part_off, cache ? (int)off : 0);
}

template <int P>
void launch_batched_tm(const ScoreArgs* dd, int B, int cls, void* plan, int nmax, int dmax, int tm,
                       size_t smem, int grid, int per_cu, hipStream_t s) {
  switch (tm) {
    case 16: launch_batched_t<P, 16>(dd, B, cls, plan, nmax, dmax, smem, grid, per_cu, s); break;
    case 32: launch_batched_t<P, 32>(dd, B, cls, plan, nmax, dmax, smem, grid, per_cu, s); break;
    default: launch_batched_t<P, 64>(dd, B, cls, plan, nmax, dmax, smem, grid, per_cu, s); break;
  }
}

}  // namespace

size_t score_esize(int prec) { return arith64(prec) ? 8 : prec == GPBO_FP32 ? 4 : 2; }
int score_kb(int prec) { return prec == GPBO_BF16 ? 32 : 16; }

// Column extent of the packed operand: the widest (last) row tile's padded
// block count times the block width.
int packed_npj(int n, int prec) {
  const int ntiles = (int)round_up(n, TI) / TI;
  return tile_blocks(ntiles - 1, score_kb(prec) / TI, prec_pf(prec)) * score_kb(prec);
}

// LDS row stride (elements) of the khat tile: whole 64-point blocks (the
// cross-covariance phase writes every lane of a block), rows 16-byte aligned
// and offset by 16 bytes modulo 128 so the 16 rows read by one matrix-core
// operand load fall in different banks.
int kt_stride(int prec, int npj) {
  const int64_t bytes = round_up(round_up(npj, 64) * (int64_t)score_esize(prec), 128) + 16;
  return (int)(bytes / score_esize(prec));
}

size_t score_smem(int prec, int n, int d, int tm) {
  const size_t csz = arith64(prec) ? 8 : 4;
  return (size_t)tm * kt_stride(prec, packed_npj(n, prec)) * score_esize(prec) +
         (size_t)round_up((int64_t)d * tm, 4) * csz + 2 * FW * (size_t)tm * csz;
}

// Row-tile block offsets of the packed operand (ntiles + 1 entries).
std::vector<int64_t> packed_offsets(int n, int prec) {
  const int ntiles = (int)round_up(n, TI) / TI;
  const int R = score_kb(prec) / TI, PF = prec_pf(prec);
  std::vector<int64_t> off(ntiles + 1, 0);
  for (int t = 0; t < ntiles; ++t) off[t + 1] = off[t] + tile_blocks(t, R, PF);
  return off;
}

// Row stride of the scaled observations: n rounded up to whole 64-point
// blocks, plus one block, which covers the packed column extent of every
// precision rounded up to 64.
static int score_nx(int n) { return (int)round_up(n, 64) + 64; }

void ensure_score_operands(Ctx* c, Model* const* models, int B, int prec, hipStream_t s) {
  // what each model lacks
  std::vector<Model*> need;
  for (int b = 0; b < B; ++b) {
    Model* M = models[b];
    if (!M->blk_obs || !M->blk_score[prec])
      if (std::find(need.begin(), need.end(), M) == need.end()) need.push_back(M);
  }
  if (need.empty()) return;
  for (Model* M : need)
    if (M->alloc_stream != s) M->alloc_mixed = true;
  const int nb = (int)need.size();
  const int kb = score_kb(prec), PF = prec_pf(prec);
  const size_t es = score_esize(prec), as = prec == GPBO_FP64 ? sizeof(double) : sizeof(float);
  // Layout: the uploaded part (descriptors, coordinate scales, row-tile
  // offsets), then the built part (scaled observations, packed operand,
  // scaled alpha) of every model in one device allocation.
  Carve up;
  const size_t odesc = up.take(nb * sizeof(PrepDesc));
  struct Part {
    bool obs, score;
    std::vector<int64_t> off;
    size_t osc, ooff, oX64, oX32, oXp, opk, oal;
  };
  std::vector<Part> parts(nb);
  for (int k = 0; k < nb; ++k) {
    Model* M = need[k];
    Part& q = parts[k];
    q.obs = !M->blk_obs;
    q.score = !M->blk_score[prec];
    if (q.obs) q.osc = up.take(3 * M->d * sizeof(double));  // 2d doubles + d floats
    if (q.score) {
      q.off = packed_offsets(M->n, prec);
      q.ooff = up.take(q.off.size() * sizeof(int64_t));
    }
  }
  const size_t up_bytes = up.bytes;
  Carve cv = up;
  for (int k = 0; k < nb; ++k) {
    Model* M = need[k];
    Part& q = parts[k];
    const int nx = score_nx(M->n);
    if (q.obs) {
      q.oX64 = cv.take((size_t)nx * M->d * sizeof(double));
      q.oX32 = cv.take((size_t)nx * M->d * sizeof(float));
      q.oXp = cv.take((size_t)nx * dist_kp(M->d) * sizeof(float));
    }
    if (q.score) {
      q.opk = cv.take((size_t)(q.off.back() + PF) * TI * kb * es);
      q.oal = cv.take(nx * as);
    }
  }
  std::shared_ptr<void> grp = dshared(c, cv.bytes);
  if (!grp) return;  // the caller reports the missing operands
  char* g = (char*)grp.get();
  auto stage = std::make_shared<std::vector<unsigned char>>(up_bytes);
  unsigned char* h = stage->data();
  PrepDesc* hd = (PrepDesc*)(h + odesc);
  int64_t max_elems = 0;
  bool any_obs = false, any_score = false;
  for (int k = 0; k < nb; ++k) {
    Model* M = need[k];
    Part& q = parts[k];
    const int n = M->n, d = M->d;
    PrepDesc pd{};
    pd.n = n;
    pd.d = d;
    pd.nx = score_nx(n);
    pd.npad = M->npad;
    pd.kb = kb;
    pd.sf2 = M->sf2;
    pd.Linv = M->Linv;
    pd.X = M->X64;
    pd.alpha = M->alpha;
    if (q.obs) {
      // coordinate scales: 1/l for float64 and Matern; sqrt(log2(e)/2)/l for
      // the float32 squared-exponential path (one exp2 per covariance)
      double* sc = (double*)(h + q.osc);
      float* sc32 = (float*)(sc + 2 * d);
      for (int j = 0; j < d; ++j) {
        sc[j] = 1.0 / M->ls[j];
        sc[d + j] = (M->kernel == GPBO_KERNEL_SE ? std::sqrt(0.5 * 1.4426950408889634) : 1.0) / M->ls[j];
        sc32[j] = (float)sc[d + j];
      }
      M->nx = pd.nx;
      M->sc64 = (double*)(g + q.osc);
      M->sc32 = (float*)(M->sc64 + 2 * d);
      M->Xs64 = (double*)(g + q.oX64);
      M->Xs32 = (float*)(g + q.oX32);
      M->Xp32 = (float*)(g + q.oXp);
      M->blk_obs = std::shared_ptr<void>(grp, g + q.oX64);
      pd.obs = 1;
      pd.sc = M->sc64;
      pd.Xs64 = M->Xs64;
      pd.Xs32 = M->Xs32;
      pd.Xp32 = M->Xp32;
      max_elems = std::max<int64_t>(max_elems, (int64_t)pd.nx * (d + dist_kp(d)));
      any_obs = true;
    }
    if (q.score) {
      std::memcpy(h + q.ooff, q.off.data(), q.off.size() * sizeof(int64_t));
      M->pk[prec] = g + q.opk;
      M->pk_off[prec] = (int64_t*)(g + q.ooff);
      M->alphaT[prec] = g + q.oal;
      M->pk_npj[prec] = packed_npj(n, prec);
      M->blk_score[prec] = std::shared_ptr<void>(grp, g + q.opk);
      pd.ntiles = (int)q.off.size() - 1;
      pd.off = M->pk_off[prec];
      pd.pk = M->pk[prec];
      pd.blocks = q.off.back() + PF;  // + zero slack for the pipelined loads
      pd.alphaT = M->alphaT[prec];
      max_elems = std::max<int64_t>(max_elems, pd.blocks * TI * kb + pd.nx);
      any_score = true;
    }
    hd[k] = pd;
    M->host_stage = stage;  // the upload's source lives as long as the group
  }
  (void)hipMemcpyAsync(g, h, up_bytes, hipMemcpyHostToDevice, s);
  const PrepDesc* dd = (const PrepDesc*)(g + odesc);
  const dim3 grid((unsigned)std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(max_elems, 256))),
                  (unsigned)nb);
  if (any_obs) hipLaunchKernelGGL(k_prep_obs, grid, dim3(256), 0, s, dd);
  if (any_score) {
    if (prec == GPBO_FP64)
      hipLaunchKernelGGL((k_prep_pack<double, double>), grid, dim3(256), 0, s, dd);
    else if (prec == GPBO_FP32)
      hipLaunchKernelGGL((k_prep_pack<float, float>), grid, dim3(256), 0, s, dd);
    else
      hipLaunchKernelGGL((k_prep_pack<unsigned short, float>), grid, dim3(256), 0, s, dd);
  }
}

int score_tile_m64(int n, int d) { return score_tile_m(GPBO_FP64, n, d); }

int score_tile_m(int prec, int n, int d) {
  // Largest tile whose LDS footprint allows two workgroups per CU, else one.
  const size_t lds = 160 * 1024;
  for (int tm : {64, 32, 16})
    if (2 * score_smem(prec, n, d, tm) <= lds) return tm;
  for (int tm : {64, 32, 16})
    if (score_smem(prec, n, d, tm) <= lds) return tm;
  return 0;
}

ScoreArgs make_score_args(Model* M, int prec, int tm) {
  ScoreArgs a{};
  a.n = M->n;
  a.d = M->d;
  a.npk = (int)round_up(M->n, TI);
  a.npj = M->pk_npj[prec];
  a.nx = M->nx;
  a.kernel = M->kernel;
  a.ldk = kt_stride(prec, a.npj);
  a.pk_off = M->pk_off[prec];
  a.pk = M->pk[prec];
  a.alpha = M->alphaT[prec];
  a.Xs = prec == GPBO_FP64 ? (const void*)M->Xs64 : (const void*)M->Xs32;
  a.Xp = M->Xp32;
  a.sc = prec == GPBO_FP64 ? (const void*)M->sc64 : (const void*)M->sc32;
  a.stats = M->stats;
  a.sf2 = M->sf2;
  (void)tm;
  return a;
}

void launch_score(const ScoreArgs& a, int prec, int tm, hipStream_t s) {
  const size_t smem = score_smem(prec, a.n, a.d, tm);
  const bool se = a.kernel == GPBO_KERNEL_SE;
  switch (prec) {
    case GPBO_FP64:
      if (se) launch_fused_tm<GPBO_FP64, GPBO_KERNEL_SE>(a, tm, smem, s);
      else launch_fused_tm<GPBO_FP64, GPBO_KERNEL_MATERN52>(a, tm, smem, s);
      break;
    case GPBO_FP32:
      if (se) launch_fused_tm<GPBO_FP32, GPBO_KERNEL_SE>(a, tm, smem, s);
      else launch_fused_tm<GPBO_FP32, GPBO_KERNEL_MATERN52>(a, tm, smem, s);
      break;
    case P_F64IO32:
      if (se) launch_fused_tm<P_F64IO32, GPBO_KERNEL_SE>(a, tm, smem, s);
      else launch_fused_tm<P_F64IO32, GPBO_KERNEL_MATERN52>(a, tm, smem, s);
      break;
    default:
      if (se) launch_fused_tm<GPBO_BF16, GPBO_KERNEL_SE>(a, tm, smem, s);
      else launch_fused_tm<GPBO_BF16, GPBO_KERNEL_MATERN52>(a, tm, smem, s);
      break;
  }
}

void launch_score_escalated(const ScoreArgs& a32, int tm32, const ScoreArgs& a64, int tm64,
                            hipStream_t s) {
  ScoreArgs a = a32, b = a64;
  a.gate = 1;
  b.gate = 2;
  launch_score(a, GPBO_FP32, tm32, s);
  launch_score(b, P_F64IO32, tm64, s);
}

void launch_argmax_final(const double* pv, const int64_t* pi, int64_t np, int64_t* argmax,
                         double* ei_max, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(256), 0, s, pv, pi, np, argmax, ei_max);
}

void launch_argmax_gated(const double* pv, const int64_t* pi, int64_t np32, int64_t np64,
                         const double* stats, int64_t* argmax, double* ei_max, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax_gated, dim3(1), dim3(256), 0, s, pv, pi, np32, np64, stats, argmax,
                     ei_max);
}

__global__ void __launch_bounds__(256) k_check_finite(const void* __restrict__ p, int64_t count,
                                                      int is_double, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = is_double ? ((const double*)p)[i] : (double)((const float*)p)[i];
    bad |= !(v - v == 0.0);  // NaN and +-inf give NaN
  }
  if (__any(bad) && threadIdx.x % 64 == 0) atomicOr(flag, 1);
}

__global__ void k_clear_flag(int* flag) { *flag = 0; }

void launch_check_finite(const void* p, int64_t count, int is_double, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag);
  if (count <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(1024, ceil_div(count, 256));
  hipLaunchKernelGGL(k_check_finite, dim3(grid), dim3(256), 0, s, p, count, is_double, flag);
}

size_t batch_plan_bytes(int B) {
  return sizeof(PlanHdr) + round_up(2 * (int64_t)B * sizeof(int), 16) +
         3 * (int64_t)B * sizeof(int64_t);
}

void launch_score_batched(const BatchLaunch& L, hipStream_t s,
                          const std::function<void(int)>* mark) {
  const bool esc = L.dd64 != nullptr;
  hipLaunchKernelGGL(k_plan_batched, dim3(1), dim3(256), 0, s, L.dd, L.B, L.tm, L.tm64,
                     esc ? 1 : 0, L.plan);
  if (mark) (*mark)(0);
  switch (L.prec) {
    case GPBO_FP64:
      launch_batched_tm<GPBO_FP64>(L.dd, L.B, 0, L.plan, L.nmax, L.dmax, L.tm, L.smem, L.grid,
                                   L.per_cu, s);
      break;
    case GPBO_FP32:
      launch_batched_tm<GPBO_FP32>(L.dd, L.B, 0, L.plan, L.nmax, L.dmax, L.tm, L.smem, L.grid,
                                   L.per_cu, s);
      break;
    default:
      launch_batched_tm<GPBO_BF16>(L.dd, L.B, 0, L.plan, L.nmax, L.dmax, L.tm, L.smem, L.grid,
                                   L.per_cu, s);
      break;
  }
  if (esc)
    launch_batched_tm<P_F64IO32>(L.dd64, L.B, 1, L.plan, L.nmax, L.dmax, L.tm64, L.smem64,
                                 L.grid64, L.per_cu64, s);
  if (mark) (*mark)(1);
  if (L.argmax || L.ei_max)
    hipLaunchKernelGGL(k_argmax_batched, dim3(L.B), dim3(256), 0, s, L.dd, L.B,
                       (const void*)L.plan, L.argmax, L.ei_max);
}

}  // namespace gpbo
