// Float64 fit of Gaussian-process surrogates on the GPU: normalisation, Gram
// matrix, blocked Cholesky factorisation, inverse factor, weights alpha with
// iterative refinement, log marginal likelihood.  One launch sequence fits a
// whole batch of independent sub-searches (the paper runs them in parallel,
// Sec. IV-D); a single fit is a batch of one.
//
// The paper names the surrogate and its cubic training cost (Sec. IV-D); the
// formulas are the textbook ones (Rasmussen & Williams 2006, Alg. 2.1):
//   K = k(X,X) + sn2 I = L L^T,  alpha = L^-T L^-1 ytilde,
//   log p(ytilde) = -ytilde^T alpha / 2 - sum log L_ii - n/2 log 2 pi.
//
// Layout: every n x n matrix is row-major with leading dimension npad =
// round_up(n, 64) and is padded with the identity, so the blocked kernels
// work on whole 64 x 64 tiles without bounds checks.  The factorisation is
// right-looking: per 64-column block, one wave factors the diagonal tile
// (rows in registers) and inverts it, the panel below is multiplied by that
// inverse, and the trailing lower triangle receives a rank-64 update.  The
// inverse factor is formed the same way, as a blocked triangular solve
// against the identity.  Every kernel reads its problem's descriptor through
// blockIdx.z and returns at once when the problem has no work at that step or
// its factorisation has already failed.
#include <algorithm>
#include <climits>
#include <cmath>

#include "gpbo_internal.h"

namespace gpbo {

namespace {

constexpr int LDT = NB + 2;        // LDS row stride of a 64 x 64 float64 tile (16-byte rows)
constexpr int GRAM_DMAX = 64;      // largest supported input dimension
constexpr int GS = GRAM_DMAX + 1;  // LDS row stride of staged coordinates (odd: no bank conflicts)

__device__ __forceinline__ bool fit_failed(const int* info) {
  const volatile int* v = info;
  return v[0] != INT_MAX || v[1] != 0;
}

// A block-uniform reading of the failure flags (another workgroup of the
// same launch may set them while this one runs).
__device__ __forceinline__ bool block_failed(const int* info, int* flag) {
  if (threadIdx.x == 0) *flag = fit_failed(info) ? 1 : 0;
  __syncthreads();
  const bool f = *flag != 0;
  __syncthreads();
  return f;
}

// Workgroup reductions (256 threads): butterfly within each wave, then the
// four wave results through LDS.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// The same sum for a workgroup of NW waves.
template <int NW>
__device__ __forceinline__ double block_sum_w(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) r += red[q];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_min(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  const double r = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  __syncthreads();
  return r;
}

// The model's copy of the inverse lengthscales, normalisation statistics,
// finiteness check of y and the normalised targets (X is copied and checked
// by the Gram kernel's diagonal tiles).
__global__ void __launch_bounds__(256) k_fit_stats(const FitDesc* __restrict__ D) {
  __shared__ double red[256];
  __shared__ int bad;
  const FitDesc& P = D[blockIdx.z];
  const int n = P.n, d = P.d;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  int b = 0;
  for (int k = t; k < d; k += 256) P.il[k] = P.ilsrc[k];
  for (int i = t; i < n; i += 256) b |= !isfinite(P.y[i]);
  if (b) atomicOr(&bad, 1);
  double s = 0.0;
  for (int i = t; i < n; i += 256) s += P.y[i];
  const double mean = block_sum(s, red) / n;
  double q = 0.0;
  for (int i = t; i < n; i += 256) q += (P.y[i] - mean) * (P.y[i] - mean);
  double sy = sqrt(block_sum(q, red) / n);
  if (!P.normalize || sy == 0.0) sy = 1.0;
  double mn = INFINITY;
  for (int i = t; i < n; i += 256) mn = fmin(mn, P.y[i]);
  mn = block_min(mn, red);
  for (int i = t; i < P.npad; i += 256) P.yt[i] = i < n ? (P.y[i] - mean) / sy : 0.0;
  if (P.ymod != P.y)
    for (int i = t; i < n; i += 256) P.ymod[i] = P.y[i];
  if (t < S_COUNT) P.stats[t] = 0.0;
  __syncthreads();
  if (t == 0) {
    P.stats[S_YMEAN] = mean;
    P.stats[S_YSTD] = sy;
    P.stats[S_FBEST] = mn;
    if (!P.append) {
      P.info[0] = INT_MAX;
      P.info[1] = bad;
    } else if (bad) {
      P.info[1] = 1;
    }
  }
}

// Covariance at squared scaled distance r2 (coordinates pre-divided by the
// lengthscales).
__device__ __forceinline__ double cov_r2(int kernel, double r2, double sf2) {
  if (kernel == GPBO_KERNEL_SE) return sf2 * exp(-0.5 * r2);
  const double r = sqrt(r2);
  const double s5r = 2.23606797749978969641 * r;
  return sf2 * (1.0 + s5r + (5.0 / 3.0) * r2) * exp(-s5r);
}

// Squared distance of two LDS-staged coordinate rows zero-padded to a
// multiple of 4; four partial sums keep independent loads in flight.
__device__ __forceinline__ double sqdist4(const double* a, const double* b, int dp4) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k = 0; k < dp4; k += 4) {
    const double u0 = a[k] - b[k], u1 = a[k + 1] - b[k + 1], u2 = a[k + 2] - b[k + 2],
                 u3 = a[k + 3] - b[k + 3];
    s0 = fma(u0, u0, s0);
    s1 = fma(u1, u1, s1);
    s2 = fma(u2, u2, s2);
    s3 = fma(u3, u3, s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// Stage R scaled coordinate rows of X (n x d) starting at row r0 (rows >=
// lim are zero).
template <int R = NB>
__device__ __forceinline__ void stage_rows(const FitDesc& P, const double* X, int r0, int lim,
                                           double* dst) {
  const int dp4 = (P.d + 3) & ~3;
  for (int e = threadIdx.x; e < R * dp4; e += blockDim.x) {
    const int r = e / dp4, k = e % dp4;
    dst[r * GS + k] = (r0 + r < lim && k < P.d) ? X[(int64_t)(r0 + r) * P.d + k] * P.il[k] : 0.0;
  }
}

// Triangular enumeration of the tiles (I, J), J <= I.
__device__ __forceinline__ void tri_index(int b, int& I, int& J) {
  int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  while (i * (i + 1) / 2 > b) --i;
  I = i;
  J = b - i * (i + 1) / 2;
}

// Rows of a tile handled by one workgroup of the Gram and residual kernels:
// four workgroups per 64 x 64 tile keep four times as many waves busy on
// what is a latency-bound float64 loop.
constexpr int KR = 16;

// Lower triangle of K = sf2 k(X,X) + sn2 I (identity beyond n); the tile
// mirrored above the diagonal is zeroed so the factor's upper part is clean.
// The same entries also go to the model's symmetric copy of K (both
// triangles, rows and columns < n), which the residual of the alpha solve
// reads instead of evaluating the covariance again.
// Workgroup 4b + h covers rows 16h..16h+15 of tile b (I, J).  The
// coordinates are read from the caller's X; the diagonal tiles also copy
// their rows into the model and flag non-finite values.
__global__ void __launch_bounds__(256) k_gram(const FitDesc* __restrict__ D) {
  __shared__ double xi[KR * GS], xj[NB * GS], kt[KR * (NB + 1)];
  __shared__ int flag;
  const FitDesc& P = D[blockIdx.z];
  const int nb = P.npad / NB;
  const int tile = blockIdx.x / (NB / KR), h = blockIdx.x % (NB / KR);
  // (the diagonal tiles of this launch may flag non-finite X meanwhile: the
  // whole workgroup takes one reading)
  if (tile >= nb * (nb + 1) / 2 || block_failed(P.info, &flag)) return;
  const int n = P.n, npad = P.npad;
  int I, J;
  tri_index(tile, I, J);
  const int r0 = I * NB + KR * h;  // first row of this workgroup
  if (I == J) {
    const int64_t e0 = (int64_t)min(n, r0) * P.d, e1 = (int64_t)min(n, r0 + KR) * P.d;
    int bad = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      const double x = P.Xsrc[e];
      bad |= !isfinite(x);
      P.X[e] = x;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(P.info + 1, 1);
  }
  stage_rows<KR>(P, P.Xsrc, r0, n, xi);
  stage_rows(P, P.Xsrc, J * NB, n, xj);
  if (I != J) {
    // mirrored block: rows J*64 .. J*64+63, columns r0 .. r0+15
#pragma unroll
    for (int e = threadIdx.x; e < NB * KR; e += 256) {
      const int64_t o = (int64_t)(J * NB + e / KR) * npad + r0 + e % KR;
      P.L[o] = 0.0;
      P.Linv[o] = 0.0;
    }
  }
  __syncthreads();
  const int dp4 = (P.d + 3) & ~3;
#pragma unroll
  for (int e = threadIdx.x; e < KR * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    const int i = r0 + r, j = J * NB + c;
    double v;
    if (i < n && j < n) {
      v = (j <= i) ? cov_r2(P.kernel, sqdist4(xi + r * GS, xj + c * GS, dp4), P.sf2) : 0.0;
      if (i == j) v += P.sn2;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    if (j > i) v = 0.0;
    P.L[(int64_t)i * npad + j] = v;
    P.Linv[(int64_t)i * npad + j] = 0.0;  // the inverse factor starts from zero
    if (i < n && j <= i) P.K[(int64_t)i * npad + j] = v;
    kt[r * (NB + 1) + c] = v;
  }
  __syncthreads();
  // the strictly lower entries mirrored above the diagonal (rows of 16
  // consecutive columns per store group)
  for (int e = threadIdx.x; e < NB * KR; e += 256) {
    const int c = e / KR, r = e % KR;
    const int i = r0 + r, j = J * NB + c;
    if (i < n && j < i) P.K[(int64_t)j * npad + i] = kt[r * (NB + 1) + c];
  }
}

// ---- 64 x 64 float64 tile products staged in LDS ----------------------------

// dst[q][r] (stride LDT) = src[r][q] when transpose, else src[q][r].  All 16
// loads of a thread are issued before the first LDS store.
__device__ __forceinline__ void load_tile(const double* __restrict__ src, int ld, double* dst,
                                          bool transpose) {
  double v[NB * NB / 256];
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    v[q] = src[(int64_t)(e / NB) * ld + e % NB];  // src row e/64, column e%64 (coalesced)
  }
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int a = e / NB, b = e % NB;
    if (transpose)
      dst[b * LDT + a] = v[q];
    else
      dst[a * LDT + b] = v[q];
  }
}

// Broadcast of lane l's double (l a compile-time constant in the callers).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

typedef double d4x __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 float64 matrix-core step: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; lane l holds D[l / 16 + 4 r][l % 16] in element r (rows
// interleaved across the lane groups, unlike the 32-bit 16 x 16 forms).
__device__ __forceinline__ d4x mma64(double a, double b, d4x c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The 64 x 64 product C[r][c] = sum_q At[q][r] Bt[q][c] on the float64
// matrix cores: wave w forms rows 16w..16w+15 as four 16 x 16 blocks, column
// block c in acc[c] (80 LDS reads per lane instead of the 512 of an outer
// product on the vector ALUs).
__device__ __forceinline__ void tile_mac(const double* At, const double* Bt, d4x acc[4]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int mr = lane % 16, mk = lane / 16;
#pragma unroll 4
  for (int s = 0; s < NB / 4; ++s) {
    const int q = 4 * s + mk;
    const double a = At[q * LDT + 16 * w + mr];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = mma64(a, Bt[q * LDT + 16 * c + mr], acc[c]);
  }
}

// The C tile's entries in the product's register layout: lane l holds row
// 16w + l/16 + 4e, column 16c + l%16 in v[c][e].  An update loads them
// before its product, so the loads overlap the staging and the product.
__device__ __forceinline__ void load_acc(const double* __restrict__ C, int ld, double v[4][4]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int mr = lane % 16, mk = lane / 16;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) v[c][e] = C[(int64_t)(16 * w + mk + 4 * e) * ld + 16 * c + mr];
}

// C tile = acc, or C = old - acc when old is given (same layout).
__device__ __forceinline__ void store_tile(double* __restrict__ C, int ld, const d4x acc[4],
                                           const double (*old)[4] = nullptr) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int mr = lane % 16, mk = lane / 16;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      C[(int64_t)(16 * w + mk + 4 * e) * ld + 16 * c + mr] = old ? old[c][e] - acc[c][e] : acc[c][e];
}

constexpr int PW = 16;  // panel width of the blocked factorisation
// LDS of the diagonal-tile step, small arrays first, so that every address
// the factorisation's column reads use fits the 16-bit LDS instruction
// offset.  The panel columns (factorisation) and the block products
// (inverse) share their space: 78,352 bytes, two workgroups per CU.
struct DiagLds {
  union {
    double colb[PW][NB];             // the panel's unscaled columns, one slot each
    double Tb[NB / PW][PW][PW + 2];  // one block product per wave
  };
  double piv[NB];    // pivots d_j
  double pinv[NB];   // 1 / d_j
  double rdiag[NB];  // 1 / L_jj
  int bad;
  int npad_s;          // the row stride and the tile's address, for the
  double* tile_s;      // store after the factorisation (see there)
  double Ls[NB][LDT];  // the tile, then U, then L_kk
  double Xl[NB][LDT];  // the inverse, staged for a coalesced store
};
static_assert(sizeof(DiagLds) == 78352 && 2 * sizeof(DiagLds) <= 160 * 1024, "diagonal-step LDS");

// Factor the diagonal tile (k, k), write L_kk and its inverse D_k.  The 64
// column steps of the tile are a dependency chain; the kernel keeps the chain
// in one wave, trims that wave's instructions to the chain itself (a lone
// wave issues about one instruction per four cycles) and gives the rest to
// all four waves.
//   Factorisation A = U diag(d)^-1 U^T, blocked over four 16-column panels:
//   wave 0 factors the 64 x 16 panel with lane i holding row i's panel
//   entries in registers.  Step j reads the pivot d_j = U_jj from lane j and,
//   with 1/d_j from the hardware estimate and two Newton steps, updates the
//   remaining panel columns by A_iq -= (U_ij / d_j) U_qj; column j + 1 goes
//   to its own LDS slot as soon as its last update is done, so the LDS round
//   trip overlaps the rest of the step.  Then all waves apply the panel's
//   rank-16 update A_il -= sum_q U_iq U_lq / d_q to the trailing lower
//   triangle on the float64 matrix cores.  At the end L_ij = U_ij / sqrt(d_j)
//   (L_jj = sqrt(d_j)), one column per lane.
//   Inverse, blocked over 16 x 16 blocks (see below).
// With staged set, the caller has already written the tile to S.Ls (and
// synchronised the workgroup).
__device__ __forceinline__ void potrf_diag_tile(const FitDesc& P, int k, DiagLds& S,
                                                bool staged = false) {
  auto& colb = S.colb;
  auto& rdiag = S.rdiag;
  auto& bad_s = S.bad;
  auto& Ls = S.Ls;
  auto& Xl = S.Xl;
  auto& Tb = S.Tb;
  const int npad = P.npad;
  const int t = threadIdx.x, lane = t % 64;
  const int wave = __builtin_amdgcn_readfirstlane(t / 64);
  const int mr = lane % 16, mk = lane / 16;  // matrix-core operand row / k index
  {
    // coalesced rows into LDS, all loads in flight before the first store
    const double* Akk = P.L + (int64_t)k * NB * npad + k * NB;
    if (!staged) {
      double v[NB / 4];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) v[q] = Akk[(int64_t)(wave + 4 * q) * npad + lane];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) Ls[wave + 4 * q][lane] = v[q];
    }
    if (t == 0) {
      S.npad_s = npad;
      S.tile_s = P.L + (int64_t)k * NB * npad + k * NB;
    }
  }
  __syncthreads();
  int bad = -1;  // first pivot that is not positive and finite (uniform in wave 0)
  // The panel and inverse loops stay rolled: one copy of the loop body
  // reaches the instruction cache instead of four straight-line copies.
#pragma unroll 1
  for (int p0 = 0; p0 < NB; p0 += PW) {
    if (wave == 0) {
      const int i = lane;
      double r[PW];
#pragma unroll
      for (int q = 0; q < PW; q += 2) {
        const double2 v = *(const double2*)&Ls[i][p0 + q];
        r[q] = v.x;
        r[q + 1] = v.y;
      }
      // a pivot that is not positive and finite is found after the panel;
      // the arithmetic goes on meanwhile (the tile is then discarded)
      colb[0][i] = r[0];
#pragma unroll
      for (int jj = 0; jj + 1 < PW; ++jj) {
        const double d = readlane_f64(r[jj], p0 + jj);
        // one wave: a wave-scope fence orders the column's LDS store before
        // the reads below
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        double b[PW];
#pragma unroll
        for (int q = jj + 1; q < PW; ++q) b[q] = colb[jj][p0 + q];
        double inv = __builtin_amdgcn_rcp(d);
        inv = fma(inv, fma(-d, inv, 1.0), inv);
        inv = fma(inv, fma(-d, inv, 1.0), inv);
        const double ti = r[jj] * inv;
        r[jj + 1] = fma(-ti, b[jj + 1], r[jj + 1]);
        colb[jj + 1][i] = r[jj + 1];
#pragma unroll
        for (int q = jj + 2; q < PW; ++q) r[q] = fma(-ti, b[q], r[q]);
      }
#pragma unroll
      for (int q = 0; q < PW; q += 2) *(double2*)&Ls[i][p0 + q] = double2{r[q], r[q + 1]};
      // pivots and their reciprocals, one per diagonal lane
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const bool diag = i >= p0 && i < p0 + PW;
      const double dv = colb[diag ? i - p0 : 0][i];
      double inv = __builtin_amdgcn_rcp(dv);
      inv = fma(inv, fma(-dv, inv, 1.0), inv);
      inv = fma(inv, fma(-dv, inv, 1.0), inv);
      if (diag) {
        S.piv[i] = dv;
        S.pinv[i] = inv;
      }
      const unsigned long long badm = __ballot(diag && !(dv > 0.0 && isfinite(dv)));
      if (bad < 0 && badm != 0) bad = __builtin_ctzll(badm);  // lane i holds column i
    }
    __syncthreads();
    // rank-16 update of the trailing lower triangle, A_il -= sum_q U_iq U_lq
    // / d_q, one 16 x 16 block (I, J), I >= J, per wave and pass; the entries
    // above the diagonal of a diagonal block are updated too and never read
    const int nt = (NB - p0 - PW) / PW;
    if (nt > 0) {
      double w[PW / 4];
#pragma unroll
      for (int sk = 0; sk < PW / 4; ++sk) w[sk] = S.pinv[p0 + 4 * sk + mk];
      for (int b = wave; b < nt * (nt + 1) / 2; b += 4) {
        int I = 0, J = b;
        while (J > I) J -= ++I;
        const int r0 = p0 + PW * (I + 1), c0 = p0 + PW * (J + 1);
        d4x acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int sk = 0; sk < PW / 4; ++sk)
          acc = mma64(Ls[r0 + mr][p0 + 4 * sk + mk] * w[sk], Ls[c0 + mr][p0 + 4 * sk + mk], acc);
#pragma unroll
        for (int e = 0; e < 4; ++e) Ls[r0 + mk + 4 * e][c0 + mr] -= acc[e];
      }
    }
    __syncthreads();
  }
  if (t == 0) bad_s = bad;
  __syncthreads();
  if (bad_s >= 0) {
    if (t == 0) atomicMin(&P.info[0], k * NB + bad_s);
    return;
  }
  {
    // L = U diag(d)^-1/2: lane = column j, in LDS (stored to the factor at
    // the end: a barrier waits for the stores issued before it)
    const double d = S.piv[lane];
    double y = __builtin_amdgcn_rsq(d);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    double sq = d * y;
    sq = fma(0.5 * y, fma(-sq, sq, d), sq);  // sqrt(d), corrected
    if (wave == 0) rdiag[lane] = y;          // 1 / L_jj
    // all reads first and selects rather than branches: one LDS round trip
    // instead of one per row
    double u[NB / 4];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) u[q] = Ls[wave + 4 * q][lane];
#pragma unroll
    for (int q = 0; q < NB / 4; ++q) {
      const int r = wave + 4 * q;
      const double lo = u[q] * y, dg = r == lane ? sq : 0.0;
      Ls[r][lane] = r > lane ? lo : dg;
    }
  }
  // Inverse, blocked over 4 x 4 blocks of 16: the diagonal blocks by
  // forward substitution (wave s inverts block s, lane = column), then the
  // block diagonals d = 1, 2, 3 from
  //   X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ   (I - J = d),
  // wave J forming block (J + d, J) on the matrix cores, the inner sum
  // staged through LDS to become the second product's B operand.
#pragma unroll
  for (int q = 0; q < NB * NB / 256; ++q) Xl[wave + 4 * q][lane] = 0.0;
  __syncthreads();
  if (lane < PW) {
    const int b0 = wave * PW, cc = lane;
    double x[PW];
#pragma unroll
    for (int r = 0; r < PW; ++r) {
      double s0 = r == cc ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
      for (int q = 0; q + 1 < r; q += 2) {
        s0 = fma(-Ls[b0 + r][b0 + q], x[q], s0);
        s1 = fma(-Ls[b0 + r][b0 + q + 1], x[q + 1], s1);
      }
      if (r & 1) s0 = fma(-Ls[b0 + r][b0 + r - 1], x[r - 1], s0);
      x[r] = (s0 + s1) * rdiag[b0 + r];
      Xl[b0 + r][b0 + cc] = x[r];
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int dd = 1; dd < NB / PW; ++dd) {
    if (wave < NB / PW - dd) {
      const int J = wave, I = J + dd;
      d4x tacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
      for (int K = 0; K < dd; ++K)
#pragma unroll
        for (int sk = 0; sk < PW / 4; ++sk) {
          const int kc = (J + K) * PW + 4 * sk + mk;
          tacc = mma64(Ls[I * PW + mr][kc], Xl[kc][J * PW + mr], tacc);
        }
#pragma unroll
      for (int e = 0; e < 4; ++e) Tb[wave][mk + 4 * e][mr] = tacc[e];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      d4x xacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int sk = 0; sk < PW / 4; ++sk)
        xacc = mma64(Xl[I * PW + mr][I * PW + 4 * sk + mk], Tb[wave][4 * sk + mk][mr], xacc);
#pragma unroll
      for (int e = 0; e < 4; ++e) Xl[I * PW + mk + 4 * e][J * PW + mr] = -xacc[e];
    }
    __syncthreads();
  }
  // L_kk and D_k to memory (addresses formed only now: a volatile LDS read
  // keeps the compiler from holding them in registers across the
  // factorisation)
  const int np2 = *(const volatile int*)&S.npad_s;
  double* Akk = *(double* const volatile*)&S.tile_s;
  double* Dk = P.Dinv + (int64_t)k * NB * NB;
#pragma unroll
  for (int q = 0; q < NB / 4; ++q) {
    const int r = wave + 4 * q;
    Akk[(int64_t)r * np2 + lane] = Ls[r][lane];
    Dk[r * NB + lane] = Xl[r][lane];
  }
}

__global__ void __launch_bounds__(256) k_potrf_diag(const FitDesc* __restrict__ Ds, int k) {
  __shared__ __align__(16) DiagLds S;
  const FitDesc& P = Ds[blockIdx.z];
  if (k >= P.npad / NB || fit_failed(P.info)) return;
  potrf_diag_tile(P, k, S);
}

// The tile operations of the factorisation and of the inverse factor.  The
// inverse factor X = L^-1 is formed block row by block row in right-looking
// order: step I sets X_IJ = D_I B_IJ (J <= I; B_II = I) and then
// B_KJ -= L_KI X_IJ for K > I.  Step I needs only column block I of L and
// D_I, so it runs inside the launches of the factorisation's step I + 1,
// on workgroups of their own: no extra launch per step.

// One 16 x 16 block per wave of the product C[r][c] = sum_q At[q][r]
// Bt[q][c]: rows rb..rb+15, columns cb..cb+15 (register layout of
// load_acc).
__device__ __forceinline__ d4x block_mac(const double* At, const double* Bt, int rb, int cb) {
  const int lane = threadIdx.x % 64, mr = lane % 16, mk = lane / 16;
  d4x acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int s = 0; s < NB / 4; ++s) {
    const int q = 4 * s + mk;
    acc = mma64(At[q * LDT + rb + mr], Bt[q * LDT + cb + mr], acc);
  }
  return acc;
}

__device__ __forceinline__ void store_block(double* __restrict__ C, int ld, d4x acc, int rb, int cb) {
  const int lane = threadIdx.x % 64, mr = lane % 16, mk = lane / 16;
#pragma unroll
  for (int e = 0; e < 4; ++e) C[(int64_t)(rb + mk + 4 * e) * ld + cb + mr] = acc[e];
}

// The panel and the inverse's row multiply are split over four workgroups
// per tile (h = 0..3), so that their launches, which lie on the
// factorisation's critical path, each take a quarter of the matrix work.
// Each workgroup reads and writes only its own slice of the tile it
// overwrites.

// Panel: A_Ik <- A_Ik D_k^T for I > k; workgroup h takes rows 16h..16h+15.
__device__ __forceinline__ void panel_tile(const FitDesc& P, int k, int I, int h, double* sm) {
  const int npad = P.npad, t = threadIdx.x, w = t / 64;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  double* Pk = P.L + (int64_t)I * NB * npad + k * NB;
  double v[NB / 16];
#pragma unroll
  for (int q = 0; q < NB / 16; ++q) {  // rows 16h.. of A_Ik, transposed into At
    const int e = t + 256 * q, r = 16 * h + e / NB, c = e % NB;
    v[q] = Pk[(int64_t)r * npad + c];
  }
  load_tile(P.Dinv + (int64_t)k * NB * NB, NB, Bt, true);
#pragma unroll
  for (int q = 0; q < NB / 16; ++q) {
    const int e = t + 256 * q, r = 16 * h + e / NB, c = e % NB;
    At[c * LDT + r] = v[q];
  }
  __syncthreads();
  store_block(Pk, npad, block_mac(At, Bt, 16 * h, 16 * w), 16 * h, 16 * w);
}

// Trailing update: A_IJ -= A_Ik A_Jk^T for k < J <= I.
__device__ __forceinline__ void update_tile(const FitDesc& P, int k, int I, int J, double* sm) {
  const int npad = P.npad;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  double* C = P.L + (int64_t)I * NB * npad + J * NB;
  load_tile(P.L + (int64_t)I * NB * npad + k * NB, npad, At, true);
  load_tile(P.L + (int64_t)J * NB * npad + k * NB, npad, Bt, true);
  double old[4][4];
  load_acc(C, npad, old);
  __syncthreads();
  d4x acc[4] = {};
  tile_mac(At, Bt, acc);
  store_tile(C, npad, acc, old);
}

// Inverse factor, step I: X_IJ = D_I B_IJ for J < I, X_II = D_I;
// workgroup h takes columns 16h..16h+15.
__device__ __forceinline__ void rowmul_tile(const FitDesc& P, int I, int J, int h, double* sm) {
  const int npad = P.npad, t = threadIdx.x, w = t / 64;
  double* C = P.Linv + (int64_t)I * NB * npad + J * NB;
  const double* Dk = P.Dinv + (int64_t)I * NB * NB;
  if (J == I) {
    for (int e = t; e < NB * 16; e += 256) {
      const int r = e / 16, c = 16 * h + e % 16;
      C[(int64_t)r * npad + c] = Dk[r * NB + c];
    }
    return;
  }
  double* At = sm;
  double* Bt = sm + NB * LDT;
  double v[NB / 16];
#pragma unroll
  for (int q = 0; q < NB / 16; ++q) {  // columns 16h.. of B_IJ into Bt
    const int e = t + 256 * q, r = e / 16, c = 16 * h + e % 16;
    v[q] = C[(int64_t)r * npad + c];
  }
  load_tile(Dk, NB, At, true);
#pragma unroll
  for (int q = 0; q < NB / 16; ++q) {
    const int e = t + 256 * q, r = e / 16, c = 16 * h + e % 16;
    Bt[r * LDT + c] = v[q];
  }
  __syncthreads();
  store_block(C, npad, block_mac(At, Bt, 16 * w, 16 * h), 16 * w, 16 * h);
}

// Whole-tile variants (one workgroup per tile, each wave four 16 x 16
// blocks): D_k is read once per tile instead of once per quarter.  A batch
// of many problems has tiles enough to fill the GPU without the quarters,
// and then the four reads of D_k (32 KB each) per tile dominate the launch.
__device__ __forceinline__ void panel_tile_all(const FitDesc& P, int k, int I, double* sm) {
  const int npad = P.npad, t = threadIdx.x, w = t / 64;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  double* Pk = P.L + (int64_t)I * NB * npad + k * NB;
  for (int e = t; e < NB * NB; e += 256) {  // A_Ik transposed into At
    const int r = e / NB, c = e % NB;
    At[c * LDT + r] = Pk[(int64_t)r * npad + c];
  }
  load_tile(P.Dinv + (int64_t)k * NB * NB, NB, Bt, true);
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 4; ++h)
    store_block(Pk, npad, block_mac(At, Bt, 16 * h, 16 * w), 16 * h, 16 * w);
}

__device__ __forceinline__ void rowmul_tile_all(const FitDesc& P, int I, int J, double* sm) {
  const int npad = P.npad, t = threadIdx.x, w = t / 64;
  double* C = P.Linv + (int64_t)I * NB * npad + J * NB;
  const double* Dk = P.Dinv + (int64_t)I * NB * NB;
  if (J == I) {
    for (int e = t; e < NB * NB; e += 256) C[(int64_t)(e / NB) * npad + e % NB] = Dk[e];
    return;
  }
  double* At = sm;
  double* Bt = sm + NB * LDT;
  for (int e = t; e < NB * NB; e += 256) {  // B_IJ into Bt
    const int r = e / NB, c = e % NB;
    Bt[r * LDT + c] = C[(int64_t)r * npad + c];
  }
  load_tile(Dk, NB, At, true);
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 4; ++h)
    store_block(C, npad, block_mac(At, Bt, 16 * w, 16 * h), 16 * w, 16 * h);
}

// Inverse factor, step I: B_KJ -= L_KI X_IJ for K > I, J <= I.
__device__ __forceinline__ void trtri_update_tile(const FitDesc& P, int I, int K, int J, double* sm) {
  const int npad = P.npad;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  double* C = P.Linv + (int64_t)K * NB * npad + J * NB;
  load_tile(P.L + (int64_t)K * NB * npad + I * NB, npad, At, true);
  load_tile(P.Linv + (int64_t)I * NB * npad + J * NB, npad, Bt, false);
  double old[4][4];
  load_acc(C, npad, old);
  __syncthreads();
  d4x acc[4] = {};
  tile_mac(At, Bt, acc);
  store_tile(C, npad, acc, old);
}

// Launch of step k (k <= nbmax): panel tiles of the factorisation (the first
// npanel workgroups, npanel = nbmax - k - 1 for the largest problem) and the
// row-multiply tiles of inverse step k - 1.
// quarters = 4: four workgroups per tile (h = 0..3); 1: one per tile.
__global__ void __launch_bounds__(256) k_chol_panel(const FitDesc* __restrict__ Ds, int k,
                                                    int npanel, int quarters) {
  extern __shared__ double sm[];
  const FitDesc& P = Ds[blockIdx.z];
  if (fit_failed(P.info)) return;
  const int nb = P.npad / NB;
  const int bx = blockIdx.x / quarters, h = blockIdx.x % quarters;  // tile, quarter
  if (bx < npanel) {
    const int I = k + 1 + bx;
    if (I < nb) {
      if (quarters == 1) panel_tile_all(P, k, I, sm);
      else panel_tile(P, k, I, h, sm);
    }
  } else {
    const int I = k - 1, J = bx - npanel;
    if (I >= 0 && I < nb && J <= I) {
      if (quarters == 1) rowmul_tile_all(P, I, J, sm);
      else rowmul_tile(P, I, J, h, sm);
    }
  }
}

// Launch of step k: trailing-update tiles of the factorisation (the first
// nupd workgroups) and the update tiles of inverse step k - 1.  Look-ahead:
// the workgroup that updates the next diagonal tile (k + 1, k + 1) goes on to
// factor and invert it, so step k + 1 needs no launch of its own for it and
// starts as soon as that one tile is done.
__global__ void __launch_bounds__(256) k_chol_update(const FitDesc* __restrict__ Ds, int k,
                                                     int nupd) {
  extern __shared__ double sm[];
  const FitDesc& P = Ds[blockIdx.z];
  if (fit_failed(P.info)) return;
  const int nb = P.npad / NB;
  const int bx = blockIdx.x;
  if (bx < nupd) {
    // rest < 0 for a smaller problem of a batch whose factorisation has
    // ended (rest (rest + 1) / 2 would be positive again for rest <= -2).
    const int rest = nb - k - 1;
    if (rest <= 0 || bx >= rest * (rest + 1) / 2) return;
    if (bx == 0) {
      // tile (k + 1, k + 1): updated in registers and handed to the
      // diagonal step through LDS, never stored in between
      const int npad = P.npad, I = k + 1;
      double* At = sm;
      load_tile(P.L + (int64_t)I * NB * npad + k * NB, npad, At, true);
      double old[4][4];
      load_acc(P.L + (int64_t)I * NB * npad + I * NB, npad, old);
      __syncthreads();
      d4x acc[4] = {};
      tile_mac(At, At, acc);
      __syncthreads();  // the staging area becomes the diagonal step's LDS
      DiagLds& S = *reinterpret_cast<DiagLds*>(sm);
      const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          S.Ls[16 * w + lane / 16 + 4 * e][16 * c + lane % 16] = old[c][e] - acc[c][e];
      __syncthreads();
      potrf_diag_tile(P, I, S, true);
      return;
    }
    int I, J;
    tri_index(bx, I, J);
    update_tile(P, k, I + k + 1, J + k + 1, sm);
  } else {
    const int I = k - 1, b = bx - nupd;
    if (I < 0 || I >= nb - 1 || b >= (nb - I - 1) * (I + 1)) return;
    trtri_update_tile(P, I, I + 1 + b / (I + 1), b % (I + 1), sm);
  }
}

// The float32 copy of the inverse factor (refinement only).
__global__ void __launch_bounds__(256) k_cast_linv(const FitDesc* __restrict__ Ds) {
  const FitDesc& P = Ds[blockIdx.z];
  if (!P.refine || fit_failed(P.info)) return;
  const int64_t cnt = (int64_t)P.npad * P.npad;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    P.L32[i] = (float)P.Linv[i];
}

// Vectors of the alpha solve, by index into the work area (V_Q: the row
// sums of squares of the inverse factor).
enum { V_W = 0, V_R = 1, V_Q = 2, V_PART = 4 };
__device__ __forceinline__ double* wvec(const FitDesc& P, int v) {
  return v < 0 ? (v == -1 ? P.yt : P.alpha) : P.work + (int64_t)v * P.npad;
}

// y = Linv x (lower triangular; float64, or the float32 copy with float32
// accumulation when refining).  One wave per row.  With ssq = 1 the row's
// sum of squares sum_j Linv_ij^2 also goes to work vector V_Q: summed over
// the rows it is trace(K^-1) = |Linv|_F^2.
__global__ void __launch_bounds__(256) k_trmv(const FitDesc* __restrict__ Ds, int xv, int yv,
                                              int ssq) {
  const FitDesc& P = Ds[blockIdx.z];
  const int lane = threadIdx.x % 64;
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= P.npad || fit_failed(P.info)) return;
  const int n = P.n, npad = P.npad;
  const double* x = wvec(P, xv);
  double* y = wvec(P, yv);
  double r = 0.0, q = 0.0;
  if (P.refine) {
    float s = 0.0f, s2 = 0.0f;
    if (row < n)
#pragma unroll 8
      for (int j = lane; j <= row; j += 64) {
        const float l = P.L32[(int64_t)row * npad + j];
        s += l * (float)x[j];
        if (ssq) s2 = fmaf(l, l, s2);
      }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (ssq)
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    r = s;
    q = s2;
  } else {
    double s = 0.0, s2 = 0.0;
    if (row < n)
#pragma unroll 8
      for (int j = lane; j <= row; j += 64) {
        const double l = P.Linv[(int64_t)row * npad + j];
        s += l * x[j];
        if (ssq) s2 = fma(l, l, s2);
      }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (ssq)
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    r = s;
    q = s2;
  }
  if (lane == 0) {
    y[row] = row < n ? r : 0.0;
    if (ssq) P.work[(int64_t)V_Q * npad + row] = row < n ? q : 0.0;
  }
}

// y = Linv^T x: y_j = sum_{i >= j} Linv_ij x_i.  A workgroup owns 16
// columns; each load of a wave covers 4 rows x 16 columns (four 128-byte
// segments), the 64 row slots of the 16 waves take every 64th row from the
// block's first column on, and the slots are combined through LDS.  (The
// inverse factor is exactly zero above its diagonal, so the rows i < j of
// the first block add zeros and need no test.)
constexpr int TRMV_T_WAVES = 16, TT_COLS = 16, TT_SLOTS = TRMV_T_WAVES * 64 / TT_COLS;
// accumulate = 1: y += Linv^T x (the correction step of alpha).
__global__ void __launch_bounds__(64 * TRMV_T_WAVES) k_trmv_t(const FitDesc* __restrict__ Ds,
                                                              int xv, int yv, int accumulate) {
  __shared__ double red[TT_SLOTS][TT_COLS];
  const FitDesc& P = Ds[blockIdx.z];
  if ((int)blockIdx.x * TT_COLS >= P.npad || fit_failed(P.info)) return;
  const int n = P.n, npad = P.npad;
  const double* x = wvec(P, xv);
  double* y = wvec(P, yv);
  const int t = threadIdx.x, c = t % TT_COLS, g = t / TT_COLS;  // column, row slot
  const int j0 = blockIdx.x * TT_COLS, j = j0 + c;
  double s = 0.0;
  if (P.refine) {
    float sf = 0.0f;
#pragma unroll 4
    for (int i = j0 + g; i < n; i += TT_SLOTS) sf += P.L32[(int64_t)i * npad + j] * (float)x[i];
    s = sf;
  } else {
#pragma unroll 4
    for (int i = j0 + g; i < n; i += TT_SLOTS) s += P.Linv[(int64_t)i * npad + j] * x[i];
  }
  red[g][c] = s;
  __syncthreads();
  if (t < 64) {
    // lane (c, part) sums slots part*16 .. part*16+15, then the four parts
    const int part = t / TT_COLS;
    double u = 0.0;
#pragma unroll
    for (int q = 0; q < TT_SLOTS / 4; ++q) u += red[part * (TT_SLOTS / 4) + q][c];
    u += __shfl_xor(u, 16);
    u += __shfl_xor(u, 32);
    if (t < TT_COLS) y[j] = j < n ? (accumulate ? y[j] + u : u) : 0.0;
  }
}

// K alpha from the stored K (float64, rows < n, one wave per row, lanes over
// the columns), into work vector V_PART (one chunk).
__global__ void __launch_bounds__(256) k_residual(const FitDesc* __restrict__ Ds) {
  const FitDesc& P = Ds[blockIdx.z];
  const int lane = threadIdx.x % 64;
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= P.n || fit_failed(P.info)) return;
  const double* k = P.K + (int64_t)row * P.npad;
  double s0 = 0.0, s1 = 0.0;
  int j = lane;
  for (; j + 64 < P.n; j += 128) {
    s0 = fma(k[j], P.alpha[j], s0);
    s1 = fma(k[j + 64], P.alpha[j + 64], s1);
  }
  if (j < P.n) s0 = fma(k[j], P.alpha[j], s0);
  double v = s0 + s1;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) P.work[(int64_t)V_PART * P.npad + row] = v;
}

// r = ytilde - sum_y part[y], its norm into stats[slot].  One workgroup of
// 16 waves per problem (the partial columns of a row are summed by its
// thread).
// With lml = 1 it also writes the log marginal likelihood and log det K:
// LML = -ytilde^T alpha / 2 - sum log L_ii - n/2 log 2 pi, and the mean
// diagonal of sf2 K^-1 (sf2 trace(K^-1) / n, from the row sums of squares of
// the inverse factor): (K^-1)_ii is the reciprocal of the leave-one-out
// predictive variance at x_i, so the mean is large when observations are
// nearly redundant, i.e. when K is ill-conditioned.
constexpr int RESF_W = 16;
__global__ void __launch_bounds__(64 * RESF_W) k_res_finish(const FitDesc* __restrict__ Ds,
                                                            int slot, int lml) {
  __shared__ double red[RESF_W];
  const FitDesc& P = Ds[blockIdx.z];
  if (fit_failed(P.info)) return;
  // (each thread requests the values of U consecutive strides before it uses
  // any: the loops are a chain of memory latencies otherwise, on the fit's
  // critical path and slow to issue beside other streams' work)
  constexpr int NT = 64 * RESF_W, U = 4;
  if (lml) {
    double q = 0.0, ld = 0.0, tr = 0.0;
    for (int i0 = threadIdx.x; i0 < P.n; i0 += U * NT) {
      double yv[U], av[U], lv[U], tv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * NT;
        const bool in = i < P.n;
        yv[u] = in ? P.yt[i] : 0.0;
        av[u] = in ? P.alpha[i] : 0.0;
        lv[u] = in ? P.L[(int64_t)i * P.npad + i] : 1.0;
        tv[u] = in ? P.work[(int64_t)V_Q * P.npad + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        q += yv[u] * av[u];
        ld += log(lv[u]);
        tr += tv[u];
      }
    }
    q = block_sum_w<RESF_W>(q, red);
    ld = block_sum_w<RESF_W>(ld, red);
    tr = block_sum_w<RESF_W>(tr, red);
    if (threadIdx.x == 0) {
      P.stats[S_LOGDET] = 2.0 * ld;
      P.stats[S_LML] = -0.5 * q - ld - 0.5 * P.n * log(2.0 * 3.14159265358979323846);
      P.stats[S_KINV] = P.sf2 * tr / P.n;
    }
  }
  double* r = P.work + (int64_t)V_R * P.npad;
  double q = 0.0;
  for (int i0 = threadIdx.x; i0 < P.npad; i0 += U * NT) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      v[u] = 0.0;
      if (i < P.n) {
        double kv = 0.0;
        for (int c = 0; c < P.nchunks; ++c) kv += P.work[(int64_t)(V_PART + c) * P.npad + i];
        v[u] = P.yt[i] - kv;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      if (i < P.npad) {
        r[i] = v[u];
        q += v[u] * v[u];
      }
    }
  }
  q = block_sum_w<RESF_W>(q, red);
  if (threadIdx.x == 0) P.stats[slot] = sqrt(q);
}

// ---------------------------------------------------------------------------
// Rank-one append (the re-training step of the optimisation loop with fixed
// hyperparameters): K grows by one row and column, and so do L and L^-1.
// The descriptors of the first three kernels describe the models before the
// append (n = old number of observations).
// ---------------------------------------------------------------------------

// The new column of K, k_j = k(x_j, x_new) for j < n, into work vector V_W
// (coordinates scaled and distances summed as the Gram kernel does); the
// first workgroup also copies the configuration and its value into the
// model and flags a non-finite one.
__global__ void __launch_bounds__(256) k_append_k(const FitDesc* __restrict__ Ds) {
  __shared__ double xs[GRAM_DMAX + 4];
  __shared__ int flag;
  const FitDesc& P = Ds[blockIdx.z];
  const int n = P.n, d = P.d, t = threadIdx.x;
  if ((int)blockIdx.x * 256 >= max(n, 1) || block_failed(P.info, &flag)) return;
  const int dp4 = (d + 3) & ~3;
  for (int k = t; k < dp4; k += 256) xs[k] = k < d ? P.xnew[k] * P.il[k] : 0.0;
  if (blockIdx.x == 0) {
    int bad = 0;
    for (int k = t; k < d; k += 256) {
      const double v = P.xnew[k];
      P.X[(int64_t)n * d + k] = v;
      bad |= !isfinite(v);
    }
    if (t == 0) {
      const double v = *P.ynew;
      P.ymod[n] = v;
      bad |= !isfinite(v);
    }
    if (bad) atomicOr(&P.info[1], 1);
  }
  __syncthreads();
  const int j = blockIdx.x * 256 + t;
  if (j >= n) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const double* xj = P.X + (int64_t)j * d;
  for (int k = 0; k < dp4; k += 4) {
    const double u0 = (k < d ? xj[k] * P.il[k] : 0.0) - xs[k];
    const double u1 = (k + 1 < d ? xj[k + 1] * P.il[k + 1] : 0.0) - xs[k + 1];
    const double u2 = (k + 2 < d ? xj[k + 2] * P.il[k + 2] : 0.0) - xs[k + 2];
    const double u3 = (k + 3 < d ? xj[k + 3] * P.il[k + 3] : 0.0) - xs[k + 3];
    s0 = fma(u0, u0, s0);
    s1 = fma(u1, u1, s1);
    s2 = fma(u2, u2, s2);
    s3 = fma(u3, u3, s3);
  }
  P.work[(int64_t)V_W * P.npad + j] = cov_r2(P.kernel, (s0 + s1) + (s2 + s3), P.sf2);
}

// With l = L^-1 k (work V_R) and v = L^-T l (work V_Q), the bordered
// factor and its inverse gain the rows
//   L[n]    = [l^T, delta],           delta = sqrt(kappa - l^T l),
//   L^-1[n] = [-v^T / delta, 1/delta]  (block substitution),
// where kappa = sf2 + sn2 is K's new diagonal entry.  Every workgroup forms
// l^T l in the same order, so all of them take the same decision; a pivot
// that is not positive marks the model as failed at index n (NOT_PD).
__global__ void __launch_bounds__(256) k_append_row(const FitDesc* __restrict__ Ds) {
  __shared__ double red[4];
  __shared__ int flag;
  const FitDesc& P = Ds[blockIdx.z];
  const int n = P.n, npad = P.npad, t = threadIdx.x;
  if ((int)blockIdx.x * 256 > n || block_failed(P.info, &flag)) return;
  const double* l = P.work + (int64_t)V_R * npad;
  const double* v = P.work + (int64_t)V_Q * npad;
  double q = 0.0;
  for (int i = t; i < n; i += 256) q = fma(l[i], l[i], q);
  q = block_sum(q, red);
  const double d2 = (P.sf2 + P.sn2) - q;
  if (!(d2 > 0.0) || !isfinite(d2)) {
    if (blockIdx.x == 0 && t == 0) P.info[0] = n;
    return;
  }
  const double delta = sqrt(d2), rdelta = 1.0 / delta;
  const int j = blockIdx.x * 256 + t;
  if (j < n) {
    const double kj = P.work[(int64_t)V_W * npad + j];
    P.L[(int64_t)n * npad + j] = l[j];
    P.Linv[(int64_t)n * npad + j] = -v[j] * rdelta;
    P.K[(int64_t)n * npad + j] = kj;
    P.K[(int64_t)j * npad + n] = kj;
  } else if (j == n) {
    P.L[(int64_t)n * npad + n] = delta;
    P.Linv[(int64_t)n * npad + n] = rdelta;
    P.K[(int64_t)n * npad + n] = P.sf2 + P.sn2;
  }
}

// Copy of a model into larger buffers (see GrowDesc).
__global__ void __launch_bounds__(256) k_grow(const GrowDesc* __restrict__ Ds) {
  const GrowDesc& G = Ds[blockIdx.z];
  const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x, st = (int64_t)gridDim.x * 256;
  const int64_t nn = (int64_t)G.np_new * G.np_new;
  for (int64_t e = t0; e < nn; e += st) {
    const int64_t i = e / G.np_new, j = e % G.np_new;
    const bool in = i < G.np_old && j < G.np_old;
    const double id = i == j ? 1.0 : 0.0;
    G.L2[e] = in ? G.L[i * G.np_old + j] : id;
    G.Linv2[e] = in ? G.Linv[i * G.np_old + j] : id;
    G.K2[e] = in ? G.K[i * G.np_old + j] : 0.0;
  }
  for (int64_t e = t0; e < (int64_t)G.n * G.d; e += st) G.X2[e] = G.X[e];
  for (int64_t e = t0; e < G.n; e += st) G.y2[e] = G.y[e];
  for (int64_t e = t0; e < G.d; e += st) G.il2[e] = G.il[e];
  if (t0 < S_COUNT) G.stats2[t0] = G.stats[t0];
  if (t0 < 2) G.info2[t0] = G.info[t0];
}

// The statistics and flags of each model into one contiguous region (slot
// bytes apart) for a single read-back.
__global__ void __launch_bounds__(64) k_status_copy(const FitDesc* __restrict__ Ds,
                                                    unsigned char* out, int slot) {
  const FitDesc& P = Ds[blockIdx.x];
  double* st = (double*)(out + (int64_t)blockIdx.x * slot);
  int* inf = (int*)(st + S_COUNT);
  const int t = threadIdx.x;
  if (t < S_COUNT) st[t] = P.stats[t];
  if (t < 2) inf[t] = P.info[t];
}

// ---------------------------------------------------------------------------
// Gradient of the log marginal likelihood in the log hyperparameters
// theta = (log l_1 .. log l_d, log sf2, log sn2) of fitted models:
//   dLML/dtheta_j = 1/2 sum_il W_il dK_il/dtheta_j,   W = alpha alpha^T - K^-1,
//   dK_il/dlog l_k = g(r_il) (x_ik - x_lk)^2 / l_k^2  with g = k_f (SE) or
//                    sf2 (5/3)(1 + sqrt5 r) e^{-sqrt5 r} (Matern-5/2),
//   dK/dlog sf2 = k_f,  dK/dlog sn2 = sn2 I.
// Workgroup (tile, model) takes the 64 x 64 tile (I, J), J <= I, of the
// symmetric W: K^-1 = L^-T L^-1 on that tile is sum_{k >= 64 I} Linv[k, i]
// Linv[k, l] (the inverse factor is lower triangular), accumulated in float64
// from 16-row slabs of Linv staged in LDS, each thread owning 4 x 4 entries.
// The tile's d + 2 sums (off-diagonal tiles counted twice) go to
// part[model][tile][j]; a second kernel adds the tiles in order.
// ---------------------------------------------------------------------------
constexpr int GK = 16;  // Linv rows per slab
inline size_t grad_lds_bytes(int dmax) {
  return (size_t)(2 * GK * NB + 2 * NB * (dmax + 1) + 4 * (dmax + 2) + 8) * sizeof(double);
}

__global__ void __launch_bounds__(256) k_lml_grad_tiles(const FitDesc* __restrict__ Ds, int ldp,
                                                        int64_t tstride, double* __restrict__ part) {
  extern __shared__ __align__(16) double gsm[];
  const FitDesc& P = Ds[blockIdx.z];
  const int n = P.n, d = P.d, npad = P.npad, t = threadIdx.x, lane = t % 64, wave = t / 64;
  const int nb = npad / NB;
  const int tile = blockIdx.x;
  if (tile >= nb * (nb + 1) / 2 || fit_failed(P.info)) return;
  int I, J;
  tri_index(tile, I, J);
  const int ds = d + 1;  // LDS row stride of the staged coordinates
  double* A = gsm;                  // [GK][NB] Linv[k, 64 I + a]
  double* Bm = A + GK * NB;         // [GK][NB] Linv[k, 64 J + c]
  double* xi = Bm + GK * NB;        // [NB][ds] scaled coordinates of the tile's rows
  double* xl = xi + NB * ds;        // [NB][ds] ... of its columns
  double* red = xl + NB * ds;       // [4][d + 2]
  const int i0 = I * NB, l0 = J * NB;
  for (int e = t; e < NB * d; e += 256) {
    const int r = e / d, k = e % d;
    xi[r * ds + k] = i0 + r < n ? P.X[(int64_t)(i0 + r) * d + k] * P.il[k] : 0.0;
    xl[r * ds + k] = l0 + r < n ? P.X[(int64_t)(l0 + r) * d + k] * P.il[k] : 0.0;
  }
  for (int e = t; e < 4 * (d + 2); e += 256) red[e] = 0.0;
  const int ra = (t / 16) * 4, ca = (t % 16) * 4;  // this thread's 4 x 4 block of the tile
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = i0; k0 < n; k0 += GK) {
    __syncthreads();
    for (int e = t; e < GK * NB; e += 256) {
      const int kk = e / NB, c = e % NB, k = k0 + kk;
      A[e] = k < n ? P.Linv[(int64_t)k * npad + i0 + c] : 0.0;
      Bm[e] = k < n ? P.Linv[(int64_t)k * npad + l0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = A[kk * NB + ra + u];
        b[u] = Bm[kk * NB + ca + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
  }
  // W and the kernel factors of the thread's 16 entries
  double base[4][4];
  double gsf = 0.0, gsn = 0.0;
  const double s5 = 2.23606797749978969641;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ra + u, l = l0 + ca + v;
      base[u][v] = 0.0;
      if (i < n && l < n) {
        const double w = P.alpha[i] * P.alpha[l] - acc[u][v];
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
          const double q = xi[(ra + u) * ds + k] - xl[(ca + v) * ds + k];
          r2 = fma(q, q, r2);
        }
        const double kf = cov_r2(P.kernel, r2, P.sf2);
        double g;
        if (P.kernel == GPBO_KERNEL_SE) {
          g = kf;
        } else {
          const double r = sqrt(r2);
          g = P.sf2 * (5.0 / 3.0) * (1.0 + s5 * r) * exp(-s5 * r);
        }
        base[u][v] = w * g;
        gsf = fma(w, kf, gsf);
        if (i == l) gsn = fma(w, P.sn2, gsn);
      }
    }
  const double wt = I == J ? 1.0 : 2.0;  // the mirrored tile above the diagonal
  for (int k = 0; k < d + 2; ++k) {
    double v = 0.0;
    if (k < d) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double q = xi[(ra + u) * ds + k] - xl[(ca + c) * ds + k];
          v = fma(base[u][c], q * q, v);
        }
    } else {
      v = k == d ? gsf : gsn;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave * (d + 2) + k] = v;
  }
  __syncthreads();
  for (int k = t; k < d + 2; k += 256) {
    const double v = (red[k] + red[(d + 2) + k]) + (red[2 * (d + 2) + k] + red[3 * (d + 2) + k]);
    part[(int64_t)blockIdx.z * tstride + (int64_t)tile * ldp + k] = wt * v;
  }
}

// grad[b][j] = 1/2 sum over the tiles (in tile order) of part[b][tile][j];
// lml[b] from the fit's statistics.  NaN for a model whose fit failed.
__global__ void __launch_bounds__(64) k_lml_grad_finish(const FitDesc* __restrict__ Ds, int ldp,
                                                        int64_t tstride,
                                                        const double* __restrict__ part, int ldg,
                                                        double* __restrict__ grad,
                                                        double* __restrict__ lml) {
  const FitDesc& P = Ds[blockIdx.x];
  const int nb = P.npad / NB, nt = nb * (nb + 1) / 2;
  const bool failed = fit_failed(P.info);
  for (int j = threadIdx.x; j < ldg; j += 64) {
    double s = 0.0;
    if (j < P.d + 2 && !failed)
      for (int q = 0; q < nt; ++q) s += part[(int64_t)blockIdx.x * tstride + (int64_t)q * ldp + j];
    grad[(int64_t)blockIdx.x * ldg + j] =
        failed ? __builtin_nan("") : (j < P.d + 2 ? 0.5 * s : 0.0);
  }
  if (lml && threadIdx.x == 0) lml[blockIdx.x] = failed ? __builtin_nan("") : P.stats[S_LML];
}

// The two-tile kernels stage 2 x 64 x 66 doubles (66 KiB) of dynamic LDS;
// the update kernel takes the diagonal step's 76.5 KiB.
void allow_tile_lds() {
  static bool done = false;
  if (done) return;
  const int bytes = 2 * NB * LDT * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void*)k_chol_update, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(DiagLds));
  done = true;
}

}  // namespace

FitDesc make_fit_desc(Model* M, const double* X, const double* il, const double* y,
                      int normalize_y, int refine) {
  FitDesc f{};
  f.n = M->n;
  f.d = M->d;
  f.npad = M->npad;
  f.kernel = M->kernel;
  f.normalize = normalize_y;
  f.refine = refine;
  f.chunk = M->n;  // K alpha is one product over the stored K
  f.nchunks = 1;
  f.sf2 = M->sf2;
  f.sn2 = M->sn2;
  f.Xsrc = X;
  f.ilsrc = il;
  f.X = M->X64;
  f.il = M->il64;
  f.y = y;
  f.ymod = M->y64;
  f.xnew = nullptr;
  f.ynew = nullptr;
  f.append = 0;
  f.L = M->L;
  f.Linv = M->Linv;
  f.K = M->K;
  f.Dinv = M->Dinv;
  f.yt = M->yt;
  f.alpha = M->alpha;
  f.work = M->work;
  f.L32 = M->L32;
  f.stats = M->stats;
  f.info = M->info;
  return f;
}

std::vector<uint64_t> fit_launch_shape(const FitDesc* h, int B) {
  int nbmax = 0, nmax = 0, chmax = 1, refine = 0;
  int64_t npmax = 0;
  for (int b = 0; b < B; ++b) {
    nbmax = std::max(nbmax, h[b].npad / NB);
    nmax = std::max(nmax, h[b].n);
    npmax = std::max<int64_t>(npmax, h[b].npad);
    chmax = std::max(chmax, h[b].nchunks);
    refine |= h[b].refine != 0;
  }
  return {(uint64_t)B, (uint64_t)nbmax, (uint64_t)npmax, (uint64_t)ceil_div(nmax, KR),
          (uint64_t)chmax, (uint64_t)refine};
}

void launch_solve(const FitDesc* h, const FitDesc* dd, int B, hipStream_t s);

void launch_fit(const FitDesc* h, const FitDesc* dd, int B, hipStream_t s) {
  allow_tile_lds();
  int nbmax = 0;
  for (int b = 0; b < B; ++b) nbmax = std::max(nbmax, h[b].npad / NB);
  const size_t sm2 = 2 * NB * LDT * sizeof(double);
  const unsigned Bz = (unsigned)B;
  hipLaunchKernelGGL(k_fit_stats, dim3(1, 1, Bz), dim3(256), 0, s, dd);
  hipLaunchKernelGGL(k_gram, dim3(nbmax * (nbmax + 1) / 2 * (NB / KR), 1, Bz), dim3(256), 0, s, dd);
  // step k: diagonal tile k (a launch of its own for k = 0, else factored by
  // the update launch of step k - 1); panel k with row multiply of inverse
  // step k-1; trailing update k with the update of inverse step k-1 and the
  // diagonal tile k + 1; step nbmax finishes the inverse
  const size_t smu = sizeof(DiagLds);
  // the panel launch in quarters of a tile while its tiles alone would not
  // fill the GPU (one problem, or few); whole tiles otherwise
  auto quarters = [&](int tiles) { return (int64_t)Bz * tiles >= 512 ? 1 : 4; };
  for (int k = 0; k <= nbmax; ++k) {
    if (k == 0) hipLaunchKernelGGL(k_potrf_diag, dim3(1, 1, Bz), dim3(256), 0, s, dd, k);
    const int npanel = std::max(nbmax - k - 1, 0);
    const int nrow = k;  // inverse step k - 1 has k tiles in its row
    if (npanel + nrow > 0) {
      const int qt = quarters(npanel + nrow);
      hipLaunchKernelGGL(k_chol_panel, dim3(qt * (npanel + nrow), 1, Bz), dim3(256), sm2, s, dd, k,
                         npanel, qt);
    }
    const int nupd = npanel * (npanel + 1) / 2;
    const int ntri = k >= 1 ? (nbmax - k) * k : 0;  // inverse step k - 1: (nbmax-k) rows x k tiles
    if (nupd + ntri > 0)
      hipLaunchKernelGGL(k_chol_update, dim3(nupd + ntri, 1, Bz), dim3(256), smu, s, dd, k, nupd);
  }
  launch_solve(h, dd, B, s);
}

// alpha = K^-1 ytilde from the inverse factor with one refinement step, the
// log marginal likelihood and the statistics (the fit's last stage, and the
// whole recomputation after a rank-one append).
// The grids depend on the padded sizes only (workgroups past a problem's n
// return at once), so a search that grows inside its padding replays the
// same captured sequence.
void launch_solve(const FitDesc* h, const FitDesc* dd, int B, hipStream_t s) {
  int64_t npmax = 0;
  bool any_refine = false;
  for (int b = 0; b < B; ++b) {
    npmax = std::max<int64_t>(npmax, h[b].npad);
    any_refine |= h[b].refine != 0;
  }
  const unsigned Bz = (unsigned)B;
  const unsigned gz = (unsigned)std::min<int64_t>(1024, ceil_div(npmax * npmax, 256));
  if (any_refine) hipLaunchKernelGGL(k_cast_linv, dim3(gz, 1, Bz), dim3(256), 0, s, dd);
  const unsigned g_rows = (unsigned)ceil_div(npmax, 4), g_cols = (unsigned)ceil_div(npmax, TT_COLS);
  // alpha = Linv^T (Linv ytilde), then one residual-and-correction step
  hipLaunchKernelGGL(k_trmv, dim3(g_rows, 1, Bz), dim3(256), 0, s, dd, -1, (int)V_W, 1);
  hipLaunchKernelGGL(k_trmv_t, dim3(g_cols, 1, Bz), dim3(64 * TRMV_T_WAVES), 0, s, dd, (int)V_W, -2, 0);
  const dim3 g_res((unsigned)ceil_div(npmax, 4), 1, Bz);
  hipLaunchKernelGGL(k_residual, g_res, dim3(256), 0, s, dd);
  hipLaunchKernelGGL(k_res_finish, dim3(1, 1, Bz), dim3(64 * RESF_W), 0, s, dd, (int)S_RES0, 0);
  hipLaunchKernelGGL(k_trmv, dim3(g_rows, 1, Bz), dim3(256), 0, s, dd, (int)V_R, (int)V_W, 0);
  // alpha += Linv^T (Linv r)
  hipLaunchKernelGGL(k_trmv_t, dim3(g_cols, 1, Bz), dim3(64 * TRMV_T_WAVES), 0, s, dd, (int)V_W, -2, 1);
  hipLaunchKernelGGL(k_residual, g_res, dim3(256), 0, s, dd);
  hipLaunchKernelGGL(k_res_finish, dim3(1, 1, Bz), dim3(64 * RESF_W), 0, s, dd, (int)S_RES1, 1);
}

}  // namespace gpbo

namespace gpbo {

std::vector<uint64_t> append_launch_shape(const FitDesc* hnew, int B) {
  int chmax = 1, refine = 0;
  int64_t npmax = 0;
  for (int b = 0; b < B; ++b) {
    npmax = std::max<int64_t>(npmax, hnew[b].npad);
    chmax = std::max(chmax, hnew[b].nchunks);
    refine |= hnew[b].refine != 0;
  }
  return {0xA99E4Dull, (uint64_t)B, (uint64_t)npmax, (uint64_t)chmax, (uint64_t)refine};
}

// Grids from the padded sizes only, as in launch_solve (n + 1 <= npad).
void launch_append(const FitDesc* hold, const FitDesc* dold, const FitDesc* hnew,
                   const FitDesc* dnew, int B, hipStream_t s) {
  int64_t npmax = 0;
  for (int b = 0; b < B; ++b) npmax = std::max<int64_t>(npmax, hold[b].npad);
  const unsigned Bz = (unsigned)B;
  const unsigned gpad = (unsigned)ceil_div(npmax, 256);
  hipLaunchKernelGGL(k_append_k, dim3(gpad, 1, Bz), dim3(256), 0, s, dold);
  // l = L^-1 k, v = L^-T l (float64: the old descriptors never refine)
  hipLaunchKernelGGL(k_trmv, dim3((unsigned)ceil_div(npmax, 4), 1, Bz), dim3(256), 0, s, dold,
                     (int)V_W, (int)V_R, 0);
  hipLaunchKernelGGL(k_trmv_t, dim3((unsigned)ceil_div(npmax, TT_COLS), 1, Bz),
                     dim3(64 * TRMV_T_WAVES), 0, s, dold, (int)V_R, (int)V_Q, 0);
  hipLaunchKernelGGL(k_append_row, dim3(gpad, 1, Bz), dim3(256), 0, s, dold);
  // normalisation over the n + 1 values, then alpha, the LML and statistics
  hipLaunchKernelGGL(k_fit_stats, dim3(1, 1, Bz), dim3(256), 0, s, dnew);
  launch_solve(hnew, dnew, B, s);
}

void launch_grow(const GrowDesc* dd, int B, int np_new_max, hipStream_t s) {
  const unsigned gx =
      (unsigned)std::min<int64_t>(1024, ceil_div((int64_t)np_new_max * np_new_max, 256));
  hipLaunchKernelGGL(k_grow, dim3(gx, 1, (unsigned)B), dim3(256), 0, s, dd);
}

void launch_status_copy(const FitDesc* dd, int B, unsigned char* out, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_status_copy, dim3((unsigned)B), dim3(64), 0, s, dd, out, slot);
}

}  // namespace gpbo

namespace gpbo {

size_t lml_grad_part_doubles(const FitDesc* h, int B, int* ldp, int64_t* tstride) {
  int dmax = 1, nbmax = 1;
  for (int b = 0; b < B; ++b) {
    dmax = std::max(dmax, h[b].d);
    nbmax = std::max(nbmax, h[b].npad / NB);
  }
  *ldp = dmax + 2;
  *tstride = (int64_t)(nbmax * (nbmax + 1) / 2) * (dmax + 2);
  return (size_t)B * (size_t)*tstride;
}

void launch_lml_grad(const FitDesc* h, const FitDesc* dd, int B, double* part, int ldg,
                     double* grad, double* lml, hipStream_t s) {
  int ldp = 0;
  int64_t tstride = 0;
  (void)lml_grad_part_doubles(h, B, &ldp, &tstride);
  int dmax = 1, nbmax = 1;
  for (int b = 0; b < B; ++b) {
    dmax = std::max(dmax, h[b].d);
    nbmax = std::max(nbmax, h[b].npad / NB);
  }
  const size_t sm = grad_lds_bytes(dmax);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_lml_grad_tiles,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)grad_lds_bytes(64));
    attr = true;
  }
  hipLaunchKernelGGL(k_lml_grad_tiles, dim3((unsigned)(nbmax * (nbmax + 1) / 2), 1, (unsigned)B),
                     dim3(256), sm, s, dd, ldp, tstride, part);
  hipLaunchKernelGGL(k_lml_grad_finish, dim3((unsigned)B), dim3(64), 0, s, dd, ldp, tstride,
                     (const double*)part, ldg, grad, lml);
}

}  // namespace gpbo
