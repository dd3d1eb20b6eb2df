// Float64 fit of one Gaussian-process surrogate on the GPU: normalisation,
// Gram matrix, blocked Cholesky factorisation, inverse factor, weights alpha
// with iterative refinement, log marginal likelihood.
//
// The paper (Sec. IV-D) names the surrogate and its cubic training cost; the
// formulas are the textbook ones (Rasmussen & Williams 2006, Alg. 2.1):
//   K = k(X,X) + sn2 I = L L^T,  alpha = L^-T L^-1 ytilde,
//   log p(ytilde) = -ytilde^T alpha / 2 - sum log L_ii - n/2 log 2 pi.
//
// Layout: every n x n matrix is row-major with leading dimension npad =
// round_up(n, 64) and is padded with the identity, so the blocked kernels
// work on whole 64 x 64 tiles without bounds checks.  The factorisation is
// right-looking: per 64-column block, one workgroup factors the diagonal tile
// in LDS and inverts it, the panel below is multiplied by that inverse, and
// the trailing lower triangle receives a rank-64 update.  The inverse factor
// is formed the same way, as a blocked triangular solve against the identity.
#include <climits>
#include <cmath>

#include "gpbo_internal.h"

namespace gpbo {

namespace {

constexpr int LDT = NB + 2;  // LDS row stride of a 64 x 64 float64 tile (16-byte aligned rows)

__device__ __forceinline__ bool fit_failed(const int* info) {
  const volatile int* v = info;
  return v[0] != INT_MAX || v[1] != 0;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_min(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmin(red[t], red[t + s]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Normalisation statistics, finiteness check and the normalised targets.
__global__ void __launch_bounds__(256) k_fit_stats(int n, int d, const double* __restrict__ X,
                                                   const double* __restrict__ y, int normalize,
                                                   int npad, double* __restrict__ stats,
                                                   double* __restrict__ yt, int* __restrict__ info) {
  __shared__ double red[256];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  int b = 0;
  for (int64_t i = t; i < (int64_t)n * d; i += 256) b |= !isfinite(X[i]);
  for (int i = t; i < n; i += 256) b |= !isfinite(y[i]);
  if (b) atomicOr(&bad, 1);
  double s = 0.0;
  for (int i = t; i < n; i += 256) s += y[i];
  const double mean = block_sum(s, red) / n;
  double q = 0.0;
  for (int i = t; i < n; i += 256) q += (y[i] - mean) * (y[i] - mean);
  double sy = sqrt(block_sum(q, red) / n);
  if (!normalize || sy == 0.0) sy = 1.0;
  double mn = INFINITY;
  for (int i = t; i < n; i += 256) mn = fmin(mn, y[i]);
  mn = block_min(mn, red);
  for (int i = t; i < npad; i += 256) yt[i] = i < n ? (y[i] - mean) / sy : 0.0;
  if (t == 0) {
    stats[S_YMEAN] = mean;
    stats[S_YSTD] = sy;
    stats[S_FBEST] = mn;
    info[0] = INT_MAX;
    info[1] = bad;
  }
}

__device__ __forceinline__ double cov64(int kernel, int d, const double* __restrict__ a,
                                        const double* __restrict__ b, const double* __restrict__ il,
                                        double sf2) {
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = (a[k] - b[k]) * il[k];
    r2 = fma(t, t, r2);
  }
  if (kernel == GPBO_KERNEL_SE) return sf2 * exp(-0.5 * r2);
  const double r = sqrt(r2);
  const double s5r = 2.23606797749978969641 * r;
  return sf2 * (1.0 + s5r + (5.0 / 3.0) * r2) * exp(-s5r);
}

// Triangular enumeration of the tiles (I, J), J <= I.
__device__ __forceinline__ void tri_index(int b, int& I, int& J) {
  int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  while (i * (i + 1) / 2 > b) --i;
  I = i;
  J = b - i * (i + 1) / 2;
}

// Lower triangle of K = sf2 k(X,X) + sn2 I (identity beyond n); the tile
// mirrored above the diagonal is zeroed so the factor's upper part is clean.
__global__ void __launch_bounds__(256) k_gram(int n, int d, int npad, int kernel, double sf2,
                                              double sn2, const double* __restrict__ X,
                                              const double* __restrict__ il,
                                              double* __restrict__ A, const int* __restrict__ info) {
  if (fit_failed(info)) return;
  int I, J;
  tri_index(blockIdx.x, I, J);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    const int i = I * NB + r, j = J * NB + c;
    double v;
    if (i < n && j < n) {
      v = (j <= i) ? cov64(kernel, d, X + (int64_t)i * d, X + (int64_t)j * d, il, sf2) : 0.0;
      if (i == j) v += sn2;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    if (j > i) v = 0.0;
    A[(int64_t)i * npad + j] = v;
    if (I != J) A[(int64_t)(J * NB + c) * npad + (I * NB + r)] = 0.0;
  }
}

// ---- 64 x 64 float64 tile products staged in LDS ----------------------------

// dst[q][r] (stride LDT) = src[r][q] when transpose, else src[q][r].
__device__ __forceinline__ void load_tile(const double* __restrict__ src, int ld, double* dst,
                                          bool transpose) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int a = e / NB, b = e % NB;  // src row a, column b (coalesced)
    const double v = src[(int64_t)a * ld + b];
    if (transpose)
      dst[b * LDT + a] = v;
    else
      dst[a * LDT + b] = v;
  }
}

// acc[4][4] += sum_q At[q][r] * Bt[q][c] for r = 4*ty + i, c = 4*tx + j.
__device__ __forceinline__ void tile_mac(const double* At, const double* Bt, double acc[4][4]) {
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll 4
  for (int q = 0; q < NB; ++q) {
    const double2 a01 = *(const double2*)&At[q * LDT + 4 * ty];
    const double2 a23 = *(const double2*)&At[q * LDT + 4 * ty + 2];
    const double2 b01 = *(const double2*)&Bt[q * LDT + 4 * tx];
    const double2 b23 = *(const double2*)&Bt[q * LDT + 4 * tx + 2];
    const double a[4] = {a01.x, a01.y, a23.x, a23.y};
    const double b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
}

// C tile = acc (mode 0) or C -= acc (mode 1).
__device__ __forceinline__ void store_tile(double* __restrict__ C, int ld, const double acc[4][4],
                                           int mode) {
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double* p = &C[(int64_t)(4 * ty + i) * ld + 4 * tx + j];
      *p = mode == 0 ? acc[i][j] : *p - acc[i][j];
    }
}

// Factor the diagonal tile (k, k) in LDS, write L_kk and its inverse D_k.
__global__ void __launch_bounds__(256) k_potrf_diag(double* __restrict__ A, int npad, int k,
                                                    double* __restrict__ Dinv, int* __restrict__ info) {
  __shared__ double T[NB][NB + 1];
  __shared__ double U[NB][NB + 1];
  __shared__ double sq[NB];
  if (fit_failed(info)) return;
  const int t = threadIdx.x;
  double* Akk = A + (int64_t)k * NB * npad + k * NB;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    T[r][c] = c <= r ? Akk[(int64_t)r * npad + c] : 0.0;
    U[r][c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  // Right-looking elimination with unscaled columns: at step j the pivot is
  // p = S_jj and S_il -= S_ij S_lj / p for j < l <= i.
  for (int j = 0; j < NB; ++j) {
    const double p = T[j][j];
    if (!(p > 0.0) || !isfinite(p)) {
      if (t == 0) atomicMin(&info[0], k * NB + j);
      return;
    }
    const double ip = 1.0 / p;
    for (int e = t; e < NB * NB; e += 256) {
      const int i = e / NB, l = e % NB;
      if (l > j && l <= i) T[i][l] -= T[i][j] * T[l][j] * ip;
    }
    __syncthreads();
  }
  if (t < NB) sq[t] = sqrt(T[t][t]);
  __syncthreads();
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, j = e % NB;
    double v = 0.0;
    if (i == j) v = sq[j];
    else if (j < i) v = T[i][j] / sq[j];
    T[i][j] = v;  // each entry read and written by one thread only
  }
  __syncthreads();
  // Inverse of L_kk by eliminating against the identity, unscaled rows:
  // U_i -= (L_ij / L_jj) U_j for i > j, then row i is scaled by 1 / L_ii.
  for (int j = 0; j < NB; ++j) {
    const double ljj = T[j][j];
    for (int e = t; e < NB * NB; e += 256) {
      const int i = e / NB, c = e % NB;
      if (i > j && c <= j) U[i][c] -= (T[i][j] / ljj) * U[j][c];
    }
    __syncthreads();
  }
  double* D = Dinv + (int64_t)k * NB * NB;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Akk[(int64_t)r * npad + c] = T[r][c];
    D[e] = c <= r ? U[r][c] / T[r][r] : 0.0;
  }
}

// Panel: A_Ik <- A_Ik D_k^T for I > k.
__global__ void __launch_bounds__(256) k_chol_panel(double* __restrict__ A, int npad, int k,
                                                    const double* __restrict__ Dinv,
                                                    const int* __restrict__ info) {
  extern __shared__ double sm[];
  if (fit_failed(info)) return;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  const int I = k + 1 + blockIdx.x;
  double* P = A + (int64_t)I * NB * npad + k * NB;
  load_tile(P, npad, At, true);
  load_tile(Dinv + (int64_t)k * NB * NB, NB, Bt, true);
  __syncthreads();
  double acc[4][4] = {};
  tile_mac(At, Bt, acc);
  __syncthreads();
  store_tile(P, npad, acc, 0);
}

// Trailing update: A_IJ -= A_Ik A_Jk^T for k < J <= I.
__global__ void __launch_bounds__(256) k_chol_update(double* __restrict__ A, int npad, int k,
                                                     const int* __restrict__ info) {
  extern __shared__ double sm[];
  if (fit_failed(info)) return;
  double* At = sm;
  double* Bt = sm + NB * LDT;
  int I, J;
  tri_index(blockIdx.x, I, J);
  I += k + 1;
  J += k + 1;
  load_tile(A + (int64_t)I * NB * npad + k * NB, npad, At, true);
  load_tile(A + (int64_t)J * NB * npad + k * NB, npad, Bt, true);
  __syncthreads();
  double acc[4][4] = {};
  tile_mac(At, Bt, acc);
  store_tile(A + (int64_t)I * NB * npad + J * NB, npad, acc, 1);
}

// Inverse factor, step I: row block I of X = L^-1 becomes D_I B_I (B_II = I).
__global__ void __launch_bounds__(256) k_trtri_rowmul(double* __restrict__ Linv, int npad, int I,
                                                      const double* __restrict__ Dinv,
                                                      const int* __restrict__ info) {
  extern __shared__ double sm[];
  if (fit_failed(info)) return;
  const int J = blockIdx.x;
  double* C = Linv + (int64_t)I * NB * npad + J * NB;
  const double* D = Dinv + (int64_t)I * NB * NB;
  if (J == I) {
    for (int e = threadIdx.x; e < NB * NB; e += 256) C[(int64_t)(e / NB) * npad + e % NB] = D[e];
    return;
  }
  double* At = sm;
  double* Bt = sm + NB * LDT;
  load_tile(D, NB, At, true);
  load_tile(C, npad, Bt, false);
  __syncthreads();
  double acc[4][4] = {};
  tile_mac(At, Bt, acc);
  __syncthreads();
  store_tile(C, npad, acc, 0);
}

// Inverse factor, step I: B_KJ -= L_KI X_IJ for K > I, J <= I.
__global__ void __launch_bounds__(256) k_trtri_update(double* __restrict__ Linv,
                                                      const double* __restrict__ L, int npad, int I,
                                                      const int* __restrict__ info) {
  extern __shared__ double sm[];
  if (fit_failed(info)) return;
  const int K = I + 1 + blockIdx.x / (I + 1);
  const int J = blockIdx.x % (I + 1);
  double* At = sm;
  double* Bt = sm + NB * LDT;
  load_tile(L + (int64_t)K * NB * npad + I * NB, npad, At, true);
  load_tile(Linv + (int64_t)I * NB * npad + J * NB, npad, Bt, false);
  __syncthreads();
  double acc[4][4] = {};
  tile_mac(At, Bt, acc);
  store_tile(Linv + (int64_t)K * NB * npad + J * NB, npad, acc, 1);
}

__global__ void k_fill(double* __restrict__ p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// y = Linv x (lower triangular, float64 or float32 matrix; accumulation in
// AccT).  One wave per row.
template <typename MT, typename AccT>
__global__ void __launch_bounds__(256) k_trmv(const MT* __restrict__ Lm, int npad, int n,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              const int* __restrict__ info) {
  if (fit_failed(info)) return;
  const int lane = threadIdx.x % 64;
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= npad) return;
  AccT s = 0;
  if (row < n)
    for (int j = lane; j <= row; j += 64) s += (AccT)Lm[(int64_t)row * npad + j] * (AccT)x[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) y[row] = row < n ? (double)s : 0.0;
}

// y = Linv^T x: y_j = sum_{i >= j} Linv_ij x_i.  A workgroup owns 64 columns;
// its four waves split the rows and combine in LDS.
template <typename MT, typename AccT>
__global__ void __launch_bounds__(256) k_trmv_t(const MT* __restrict__ Lm, int npad, int n,
                                                const double* __restrict__ x,
                                                double* __restrict__ y, const int* __restrict__ info) {
  __shared__ AccT red[4][64];
  if (fit_failed(info)) return;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int j = blockIdx.x * 64 + lane;
  AccT s = 0;
  if (j < n)
    for (int i = j + w; i < n; i += 4) s += (AccT)Lm[(int64_t)i * npad + j] * (AccT)x[i];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    AccT r = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    y[j] = j < n ? (double)r : 0.0;
  }
}

// r = ytilde - K alpha, K recomputed in float64 (one wave per row).
__global__ void __launch_bounds__(256) k_residual(int n, int d, int kernel, double sf2,
                                                  double sn2, const double* __restrict__ X,
                                                  const double* __restrict__ il,
                                                  const double* __restrict__ yt,
                                                  const double* __restrict__ alpha,
                                                  double* __restrict__ r,
                                                  const int* __restrict__ info) {
  if (fit_failed(info)) return;
  const int lane = threadIdx.x % 64;
  const int i = blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) {
    double kij = cov64(kernel, d, X + (int64_t)i * d, X + (int64_t)j * d, il, sf2);
    if (i == j) kij += sn2;
    s = fma(kij, alpha[j], s);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) r[i] = yt[i] - s;
}

// a += b (n entries); optionally the norm of a vector into stats[slot].
__global__ void __launch_bounds__(256) k_axpy_norm(int n, double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ nv,
                                                   double* __restrict__ stats, int slot,
                                                   const int* __restrict__ info) {
  __shared__ double red[256];
  if (fit_failed(info)) return;
  if (a && b)
    for (int i = threadIdx.x; i < n; i += 256) a[i] += b[i];
  if (nv) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += nv[i] * nv[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) stats[slot] = sqrt(s);
  }
}

__global__ void __launch_bounds__(256) k_lml(int n, int npad, const double* __restrict__ L,
                                             const double* __restrict__ yt,
                                             const double* __restrict__ alpha,
                                             double* __restrict__ stats, const int* __restrict__ info) {
  __shared__ double red[256];
  if (fit_failed(info)) return;
  double q = 0.0, ld = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    q += yt[i] * alpha[i];
    ld += log(L[(int64_t)i * npad + i]);
  }
  q = block_sum(q, red);
  ld = block_sum(ld, red);
  if (threadIdx.x == 0) {
    stats[S_LOGDET] = 2.0 * ld;
    stats[S_LML] = -0.5 * q - ld - 0.5 * n * log(2.0 * 3.14159265358979323846);
  }
}

template <typename T>
__global__ void k_cast(const double* __restrict__ src, T* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (T)src[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t count, int block = 256) {
  int64_t g = ceil_div(count, block);
  return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

void launch_fit_prep(Model* M, const double* X, const double* y, int normalize_y, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_stats, dim3(1), dim3(256), 0, s, M->n, M->d, X, y, normalize_y,
                     M->npad, M->stats, M->yt, M->info);
}

void launch_gram(Model* M, double* A, hipStream_t s) {
  const int nb = M->npad / NB;
  hipLaunchKernelGGL(k_gram, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, M->n, M->d, M->npad,
                     M->kernel, M->sf2, M->sn2, M->X64, M->il64, A, M->info);
}

// The two-tile kernels stage 2 x 64 x 66 doubles (66 KiB) of dynamic LDS.
static void allow_tile_lds() {
  static bool done = false;
  if (done) return;
  const int bytes = 2 * NB * LDT * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_chol_panel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void*)k_chol_update, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void*)k_trtri_rowmul, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void*)k_trtri_update, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  done = true;
}

void launch_cholesky(Model* M, double* A, hipStream_t s) {
  allow_tile_lds();
  const int nb = M->npad / NB;
  const size_t sm2 = 2 * NB * LDT * sizeof(double);
  for (int k = 0; k < nb; ++k) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A, M->npad, k, M->Dinv, M->info);
    const int rest = nb - k - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3(rest), dim3(256), sm2, s, A, M->npad, k, M->Dinv,
                         M->info);
      hipLaunchKernelGGL(k_chol_update, dim3(rest * (rest + 1) / 2), dim3(256), sm2, s, A,
                         M->npad, k, M->info);
    }
  }
}

void launch_trtri(Model* M, hipStream_t s) {
  const int nb = M->npad / NB;
  const int64_t cnt = (int64_t)M->npad * M->npad;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(cnt)), dim3(256), 0, s, M->Linv, cnt, 0.0);
  const size_t sm2 = 2 * NB * LDT * sizeof(double);
  for (int I = 0; I < nb; ++I) {
    hipLaunchKernelGGL(k_trtri_rowmul, dim3(I + 1), dim3(256), sm2, s, M->Linv, M->npad, I,
                       M->Dinv, M->info);
    const int rest = nb - I - 1;
    if (rest > 0)
      hipLaunchKernelGGL(k_trtri_update, dim3(rest * (I + 1)), dim3(256), sm2, s, M->Linv, M->L,
                         M->npad, I, M->info);
  }
}

void launch_alpha(Model* M, int refine_f32, hipStream_t s) {
  const int n = M->n, np = M->npad;
  double* w = M->work;
  double* r = M->work + np;
  double* dlt = M->work + 2 * np;
  const int g_rows = (int)ceil_div(np, 4), g_cols = (int)ceil_div(np, 64);
  // float32 copy of the inverse factor for the low-precision solves
  const float* L32 = nullptr;
  if (refine_f32) {
    const int64_t cnt = (int64_t)np * np;
    hipLaunchKernelGGL(k_cast<float>, dim3(grid_for(cnt)), dim3(256), 0, s, M->Linv, M->L32, cnt);
    L32 = M->L32;
  }
  auto solve = [&](const double* rhs, double* out) {
    if (refine_f32) {
      hipLaunchKernelGGL((k_trmv<float, float>), dim3(g_rows), dim3(256), 0, s, L32, np, n, rhs,
                         w, M->info);
      hipLaunchKernelGGL((k_trmv_t<float, float>), dim3(g_cols), dim3(256), 0, s, L32, np, n, w,
                         out, M->info);
    } else {
      hipLaunchKernelGGL((k_trmv<double, double>), dim3(g_rows), dim3(256), 0, s, M->Linv, np, n,
                         rhs, w, M->info);
      hipLaunchKernelGGL((k_trmv_t<double, double>), dim3(g_cols), dim3(256), 0, s, M->Linv, np,
                         n, w, out, M->info);
    }
  };
  solve(M->yt, M->alpha);
  const int g_res = (int)ceil_div(n, 4);
  hipLaunchKernelGGL(k_residual, dim3(g_res), dim3(256), 0, s, n, M->d, M->kernel, M->sf2, M->sn2,
                     M->X64, M->il64, M->yt, M->alpha, r, M->info);
  hipLaunchKernelGGL(k_axpy_norm, dim3(1), dim3(256), 0, s, n, (double*)nullptr,
                     (const double*)nullptr, r, M->stats, (int)S_RES0, M->info);
  solve(r, dlt);
  hipLaunchKernelGGL(k_axpy_norm, dim3(1), dim3(256), 0, s, n, M->alpha, dlt,
                     (const double*)nullptr, M->stats, 0, M->info);
  hipLaunchKernelGGL(k_residual, dim3(g_res), dim3(256), 0, s, n, M->d, M->kernel, M->sf2, M->sn2,
                     M->X64, M->il64, M->yt, M->alpha, r, M->info);
  hipLaunchKernelGGL(k_axpy_norm, dim3(1), dim3(256), 0, s, n, (double*)nullptr,
                     (const double*)nullptr, r, M->stats, (int)S_RES1, M->info);
}

void launch_lml(Model* M, hipStream_t s) {
  hipLaunchKernelGGL(k_lml, dim3(1), dim3(256), 0, s, M->n, M->npad, M->L, M->yt, M->alpha,
                     M->stats, M->info);
}

}  // namespace gpbo
