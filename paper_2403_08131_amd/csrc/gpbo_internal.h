// Internal declarations of the gpbo library: device buffers of a fitted model,
// the context, and the host-side launchers of every kernel.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gpbo.h"

namespace gpbo {

// Blocking of the float64 factorisation kernels: 64 x 64 tiles.
constexpr int NB = 64;
// Blocking of the packed inverse factor consumed by the scoring kernels:
// 16 rows (one matrix-core output tile) by KB columns.
constexpr int TI = 16;

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Indices into the device statistics vector of a model.
enum StatIdx {
  S_YMEAN = 0,
  S_YSTD = 1,
  S_FBEST = 2,
  S_LML = 3,
  S_LOGDET = 4,
  S_RES0 = 5,
  S_RES1 = 6,
  S_COUNT = 8
};

struct Ctx;

struct Model {
  Ctx* ctx = nullptr;
  int n = 0, d = 0, npad = 0;  // npad = round_up(n, NB)
  int kernel = 0;
  double sf2 = 1, sn2 = 0;
  std::vector<double> ls;       // host lengthscales
  double* X64 = nullptr;        // n x d, the observations as given
  double* il64 = nullptr;       // d, 1 / lengthscale
  double* L = nullptr;          // npad x npad, lower Cholesky factor (identity padded)
  double* Linv = nullptr;       // npad x npad, lower inverse factor
  double* Dinv = nullptr;       // (npad/NB) x NB x NB inverses of the diagonal blocks
  double* yt = nullptr;         // npad, normalised observations (zero padded)
  double* alpha = nullptr;      // npad
  double* work = nullptr;       // npad x 4 scratch vectors
  float* L32 = nullptr;         // npad x npad float32 copy of Linv (refine_alpha = 1 only)
  double* stats = nullptr;      // S_COUNT scalars
  int* info = nullptr;          // first failing pivot (INT32_MAX when none) + nonfinite flag
  double host_stats[S_COUNT] = {0};
  // Score operands, built on first use per precision.
  float* Xs32 = nullptr;        // n x d, coordinates scaled for the float32 kernels
  float* sc32 = nullptr;        // d, coordinate scales for candidates (float32 kernels)
  double* sc64 = nullptr;       // d, coordinate scales (float64 kernels)
  double* Xs64 = nullptr;       // n x d, scaled coordinates (float64 kernels)
  void* pk[3] = {nullptr, nullptr, nullptr};   // packed sf2 * Linv per precision
  void* alphaT[3] = {nullptr, nullptr, nullptr};  // sf2 * alpha per precision (double / float)
};

struct Alloc {
  void* p;
  size_t bytes;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  gpbo_allocator alloc{};
  bool has_alloc = false;
  std::string last_error;
  int num_cu = 256;
  // Reusable scratch for score reductions (grown on demand).
  void* red = nullptr;
  size_t red_bytes = 0;
  // Batched-score graph cache.
  hipGraphExec_t batch_exec = nullptr;
  std::vector<uint64_t> batch_key;
  void* batch_buf = nullptr;
  size_t batch_buf_bytes = 0;
};

// Device memory through the context's allocator.
void* dmalloc(Ctx* c, size_t bytes);
void dfree(Ctx* c, void* p);

// ---------------------------------------------------------------------------
// Fit kernels (fit.hip)
// ---------------------------------------------------------------------------
void launch_fit_prep(Model* M, const double* X, const double* y, int normalize_y,
                     hipStream_t s);
void launch_gram(Model* M, double* A, hipStream_t s);
void launch_cholesky(Model* M, double* A, hipStream_t s);
void launch_trtri(Model* M, hipStream_t s);
void launch_alpha(Model* M, int refine_f32, hipStream_t s);
void launch_lml(Model* M, hipStream_t s);

// ---------------------------------------------------------------------------
// Score operands and kernels (score.hip)
// ---------------------------------------------------------------------------
// Packed layout of sf2 * Linv for the matrix cores: for row tile ti (TI rows)
// and column block tj <= ti*TI/KB ... see score.hip.
void ensure_score_operands(Model* M, int prec, hipStream_t s);
int score_kb(int prec);  // columns per packed block for a precision
// Per-launch description of one problem's scoring.
struct ScoreJob {
  int n, d, npk, kernel;           // npk: padded n of the packed operand
  const void* pk;                  // packed sf2 * Linv
  const void* alpha;               // sf2 * alpha (precision-typed)
  const void* Xs;                  // scaled observations
  const void* sc;                  // candidate coordinate scales
  const double* stats;             // device statistics (ymean, ystd, fbest)
  double sf2;
  int64_t m;
  const void* Xc;
  void* mu;
  void* sigma;
  void* ei;
  // argmax partials: one (value, index) pair per tile
  double* part_v;
  int64_t* part_i;
};
int score_tile_m(int prec, int n, int d);  // candidates per workgroup (0 = too large)
void launch_score(const ScoreJob& j, int prec, int tile_m, hipStream_t s);
void launch_argmax_final(const double* part_v, const int64_t* part_i, int64_t nparts,
                         int64_t* argmax, double* ei_max, hipStream_t s);
// Large-n path: cross-covariance materialised in chunks, then a triangular
// matrix-core product with a sum-of-squares epilogue.
void launch_score_large(Ctx* c, const ScoreJob& j, int prec, hipStream_t s);

// Batched scoring (batch.hip)
struct BatchDesc;
gpbo_status batched_score(Ctx* c, int B, Model* const* models, const int64_t* m,
                          const void* const* Xc, int prec, void* const* ei, int64_t* argmax,
                          double* ei_max);

// Top-k and gather (select.hip)
void launch_topk(Ctx* c, int64_t m, const float* v, int64_t k, int64_t* idx, hipStream_t s);
void launch_gather_rows(int64_t k, const int64_t* idx, int d, const float* Xc, float* out,
                        hipStream_t s);

}  // namespace gpbo
