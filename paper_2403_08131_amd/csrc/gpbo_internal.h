// Internal declarations of the gpbo library: device buffers of a fitted model,
// the context, and the host-side launchers of every kernel.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <memory>
#include <string>
#include <unordered_set>
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
  S_KINV = 7,  // mean diagonal of sf2 K^-1 (conditioning measure)
  S_COUNT = 8
};

// Precision escalation of the float32 scoring path.  Contractions in float32
// carry relative errors of a few units of 2^-24 in the cross-covariance and
// the inverse-factor products; the posterior mean and variance amplify them
// by the conditioning of K.  The fit measures that conditioning as the mean
// diagonal of sf2 K^-1 (stats[S_KINV]; each (K^-1)_ii is the reciprocal of
// the leave-one-out predictive variance at x_i).  Above the threshold the
// float32 path scores the problem with float64 arithmetic instead (same
// inputs and output types).  The threshold is calibrated against the float64
// definition on the seeded batched workloads (192 sub-searches, d = 2..12,
// n = 16..400, literal lengthscales): every problem below it stays within
// 2e-5 of the float64 posterior with float32 arithmetic, and every problem
// whose float32 error exceeds 3e-5 lies above it.
constexpr double kEscalateKinv = 8.0;
static_assert(kEscalateKinv == GPBO_ESCALATE_KINV, "escalation threshold of the header");
// Internal precision of an escalated float32 problem: float64 arithmetic and
// float64 operands (packed inverse factor, alpha, scaled observations), with
// the float32 candidate coordinates and outputs of the float32 path.
constexpr int P_F64IO32 = 3;
__host__ __device__ inline bool escalate_fp64(double kinv) { return kinv > kEscalateKinv; }

struct Ctx;

struct Model {
  Ctx* ctx = nullptr;
  int n = 0, d = 0, npad = 0;  // npad = round_up(n, NB)
  int kernel = 0;
  int normalize = 1, refine = 0;  // the fit's options (kept for rank-one appends)
  double sf2 = 1, sn2 = 0;
  std::vector<double> ls;       // host lengthscales
  double* X64 = nullptr;        // npad x d, the observations as given (n rows used)
  double* y64 = nullptr;        // npad, the observed values as given (n used)
  double* il64 = nullptr;       // d, 1 / lengthscale
  double* L = nullptr;          // npad x npad, lower Cholesky factor (identity padded)
  double* Linv = nullptr;       // npad x npad, lower inverse factor
  double* K = nullptr;          // npad x npad, K = sf2 k(X,X) + sn2 I, both triangles (n used)
  double* Dinv = nullptr;       // (npad/NB) x NB x NB inverses of the diagonal blocks
  double* yt = nullptr;         // npad, normalised observations (zero padded)
  double* alpha = nullptr;      // npad
  double* work = nullptr;       // npad x 5: four scratch vectors and K alpha
  float* L32 = nullptr;         // npad x npad float32 copy of Linv (refine_alpha = 1 only)
  double* stats = nullptr;      // S_COUNT scalars
  int* info = nullptr;          // first failing pivot (INT32_MAX when none) + nonfinite flag
  double host_stats[S_COUNT] = {0};
  int host_info[2] = {0, 0};
  bool pending = false;         // fitted asynchronously; host_stats / host_info not read yet
  // Stream the model's device buffers were allocated on, and whether a later
  // allocation for it used another one (then freeing it waits for the stream).
  hipStream_t alloc_stream = nullptr;
  bool alloc_mixed = false;
  // Status region of the asynchronous fit call this model came from (shared
  // by its models: the first status request reads all of them at once).
  struct GroupStatus {
    const unsigned char* dev = nullptr;  // nb slots on the device
    int nb = 0;
    bool read = false;
    std::vector<unsigned char> host;     // nb slots once read
    std::shared_ptr<void> hold;          // device region of the slots when it is not the fit's
    // The slots copied to pinned host memory right behind the fit, in stream
    // order, with an event after the copy: a status request then waits for
    // the event instead of starting a copy and a stream synchronisation
    // (pinned = nullptr: the request copies and synchronises).
    Ctx* ctx = nullptr;
    unsigned char* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t ev = nullptr;
    ~GroupStatus();  // returns the pinned chunk and the event to the context
  };
  std::shared_ptr<GroupStatus> gstat;
  int gslot = 0;
  // Score operands, built on first use per precision.
  int nx = 0;                   // row stride of Xs32 / Xs64 (n padded with far-away points)
  float* Xs32 = nullptr;        // d x nx, coordinates scaled for the float32 kernels
  float* Xp32 = nullptr;        // dist_kp(d) x nx, observation operand of the matrix-core
                                // squared distances (bfloat16 scoring)
  float* sc32 = nullptr;        // d, coordinate scales for candidates (float32 kernels)
  double* sc64 = nullptr;       // d, coordinate scales (float64 kernels)
  double* Xs64 = nullptr;       // d x nx, scaled coordinates (float64 kernels)
  void* pk[3] = {nullptr, nullptr, nullptr};   // packed sf2 * Linv per precision
  int64_t* pk_off[3] = {nullptr, nullptr, nullptr};  // block offset of each row tile (+ end)
  int pk_npj[3] = {0, 0, 0};                   // padded column extent of the packed operand
  void* alphaT[3] = {nullptr, nullptr, nullptr};  // sf2 * alpha per precision (double / float)
  // Every buffer above lives in one of these device allocations.  A batch of
  // models shares one allocation per group (fit; score operands), held by
  // reference: it is released with the last model that uses it.
  std::shared_ptr<void> blk_fit;          // X64 .. info, L32
  std::shared_ptr<void> blk_obs;          // scales and scaled coordinates
  std::shared_ptr<void> blk_score[3];     // pk, pk_off, alphaT per precision
  // Host sources of the asynchronous uploads of the group this model was
  // prepared with (kept until the last model of the group is freed).
  std::shared_ptr<std::vector<unsigned char>> host_stage;
};

// A device allocation released through the context's allocator when the last
// reference goes.
std::shared_ptr<void> dshared(Ctx* c, size_t bytes);

// Sub-buffers of one device allocation, each 256-byte aligned.
struct Carve {
  size_t bytes = 0;
  size_t take(size_t b) {
    const size_t o = bytes;
    bytes += (b + 255) / 256 * 256;
    return o;
  }
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
  // Device copies of fit / batch descriptors (grown on demand).
  void* desc_buf = nullptr;
  size_t desc_bytes = 0;
  // Optional timing of the scoring kernels (event pairs on the stream).
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<size_t, unsigned char*>> pinned_pool;  // free pinned chunks (size, ptr)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  bool no_graph = false;  // GPBO_NO_GRAPH=1: never capture batched launches
  bool debug = false;     // GPBO_DEBUG=1: scoring checks its candidates for non-finite values
  int score_path = 0;     // gpbo_score_path
  // Models and MLPs alive on this context (destroyed with it).
  std::unordered_set<Model*> live_models;
  std::unordered_set<void*> live_mlps;
  // Batched-score graph cache.
  // Batched-score graphs by launch shape (a few shapes alternate in a loop
  // over several batches), most recently captured last.
  std::vector<std::pair<std::vector<uint64_t>, hipGraphExec_t>> batch_graphs;
  std::vector<std::pair<std::vector<uint64_t>, hipGraphExec_t>> fit_graphs;
  void* batch_buf = nullptr;
  size_t batch_buf_bytes = 0;
};

// Device memory through the context's allocator.
void* dmalloc(Ctx* c, size_t bytes);
void dfree(Ctx* c, void* p);

// Autotuner (autotune.hip): the fastest of `cands` for `key`; `run(v)` queues
// one complete launch with configuration v on the context's stream.
int autotune_pick(Ctx* c, const std::string& key, const std::vector<int>& cands,
                  const std::function<void(int)>& run);

// ---------------------------------------------------------------------------
// Fit kernels (fit.hip)
// ---------------------------------------------------------------------------
// Per-problem arguments of the fit kernels.  A batch of problems is fitted by
// one launch sequence; every kernel finds its problem's descriptor through
// blockIdx.z and idles when the problem has no work at that step.
struct FitDesc {
  int n, d, npad, kernel;
  int normalize, refine, chunk, nchunks;  // residual column chunks
  double sf2, sn2;
  const double* Xsrc;   // n x d, the caller's observations (copied to X by the first kernel)
  const double* ilsrc;  // d, 1 / lengthscale staged with the descriptors (copied to il)
  double* X;            // n x d (the model's copy)
  double* il;           // d, 1 / lengthscale (the model's copy)
  const double* y;   // n, the caller's observations
  double* ymod;      // the model's copy of y (npad; written when it is not y itself)
  // Rank-one append (gpbo_append_batched): the new configuration (d) and
  // value, and append = 1 on the descriptor of the extended model (the
  // statistics kernel then keeps an earlier failure instead of clearing it).
  const double* xnew;
  const double* ynew;
  int append;
  double* L;         // npad x npad
  double* Linv;      // npad x npad
  double* K;         // npad x npad, K symmetric (rows and columns < n)
  double* Dinv;      // npad / NB inverse diagonal tiles
  double* yt;        // npad
  double* alpha;     // npad
  double* work;      // 5 npad
  float* L32;        // npad x npad (refine only)
  double* stats;
  int* info;
};
FitDesc make_fit_desc(Model* M, const double* X, const double* il, const double* y,
                      int normalize_y, int refine);
// Queue the whole fit of B problems (descriptors: host copy h, device copy dd).
void launch_fit(const FitDesc* h, const FitDesc* dd, int B, hipStream_t s);
// Queue the rank-one append of one configuration to each of B fitted models:
// dold describes the models as fitted (n = old size, float64 products),
// dnew the extended models (n + 1; the model's own X, y and refinement).
void launch_append(const FitDesc* hold, const FitDesc* dold, const FitDesc* hnew,
                   const FitDesc* dnew, int B, hipStream_t s);
// What that launch sequence depends on besides the descriptor pointers.
std::vector<uint64_t> append_launch_shape(const FitDesc* hnew, int B);
// Copy of a fitted model's buffers into larger ones (room for more rows):
// X, the inverse lengthscales, y and the status slot verbatim, L and L^-1
// into the wider row stride with the identity beyond the old padding.
struct GrowDesc {
  int n, d, np_old, np_new;
  const double *X, *il, *y, *L, *Linv, *K, *stats;
  const int* info;
  double *X2, *il2, *y2, *L2, *Linv2, *K2, *stats2;
  int* info2;
};
void launch_grow(const GrowDesc* dd, int B, int np_new_max, hipStream_t s);
// Gradient of the log marginal likelihood in (log l_1..d, log sf2, log sn2)
// of B fitted models: per-tile partial sums (lml_grad_part_doubles doubles of
// scratch) reduced in order into grad (B x ldg, zero beyond d + 2, NaN rows
// for failed fits) and lml (B, may be null).
size_t lml_grad_part_doubles(const FitDesc* h, int B, int* ldp, int64_t* tstride);
void launch_lml_grad(const FitDesc* h, const FitDesc* dd, int B, double* part, int ldg,
                     double* grad, double* lml, hipStream_t s);
// Each model's statistics and info words into out + b * slot.
void launch_status_copy(const FitDesc* dd, int B, unsigned char* out, int slot, hipStream_t s);
// What the grids and arguments of that launch sequence depend on besides the
// descriptor pointer: equal shapes launch identical sequences.
std::vector<uint64_t> fit_launch_shape(const FitDesc* h, int B);

// ---------------------------------------------------------------------------
// Score operands and kernels (score.hip)
// ---------------------------------------------------------------------------
// Packed layout of sf2 * Linv for the matrix cores: for row tile ti (TI rows)
// and column block tj <= ti*TI/KB ... see score.hip.
// Builds the missing score operands of `models` for `prec` (one device
// allocation and one upload for all of them); afterwards a model whose
// blk_obs / blk_score[prec] is still empty could not be allocated.
void ensure_score_operands(Ctx* c, Model* const* models, int B, int prec, hipStream_t s);
int score_kb(int prec);  // columns per packed block for a precision
// Arguments of one problem's scoring (kernel argument of the single-problem
// launch, and one entry of the descriptor array of a batched launch).
struct ScoreArgs {
  int n, d, npk, npj;              // npk: n rounded up to 16; npj: padded column extent
  int nx;                          // row stride of Xs; columns n .. nx-1 are padding points
  int kernel, ldk;                 // ldk: LDS row stride of the cross-covariance tile
  const int64_t* pk_off;           // row-tile block offsets of the packed operand
  const void* pk;                  // packed sf2 * Linv
  const void* alpha;               // sf2 * alpha (precision-typed)
  const void* Xs;                  // scaled observations, dimension-major (d x nx)
  const float* Xp;                 // observation operand of the matrix-core distances
  const void* sc;                  // candidate coordinate scales
  const double* stats;             // device statistics (ymean, ystd, fbest)
  double sf2;
  int64_t m;
  const void* Xc;
  void* mu;
  void* sigma;
  void* ei;
  double* part_v;                  // argmax partials, one (value, index) pair per tile
  int64_t* part_i;
  int slot;                        // batched launch: index of this problem's outputs
  int gate;                        // single launch: 0 = always score; 1 = only if the model
                                   // is not escalated to float64; 2 = only if it is
};
int score_tile_m(int prec, int n, int d);  // candidates per workgroup (0 = too large)
size_t score_smem(int prec, int n, int d, int tile_m);
ScoreArgs make_score_args(Model* M, int prec, int tile_m);
void launch_score(const ScoreArgs& a, int prec, int tile_m, hipStream_t s);
// Large-n float32 path (score_large.hip): workspace bytes, argmax partial
// count, and the launch sequence (a.part_v may be NULL).
size_t large_scratch_bytes(int n, int npj, int64_t m);
int64_t large_partials(int npj, int64_t m);
// mark(0) / mark(1) are called right before / after each launch of the
// triangular product (the dominant kernel), for timing.
void launch_score_large(const ScoreArgs& a, void* scratch, hipStream_t s,
                        const std::function<void(int)>& mark);
// Posterior mean, nearest-observation bound of sigma and the EI bound
// (float32; the model's float32 score operands must exist).
void launch_score_bound(const Model* M, int64_t m, const float* Xc, float* mu, float* sigma_ub,
                        float* ei_ub, hipStream_t s);
void launch_argmax_final(const double* part_v, const int64_t* part_i, int64_t nparts,
                         int64_t* argmax, double* ei_max, hipStream_t s);
// The float32 path escalated to float64 arithmetic on one problem (single
// launch, gate 0 or 2): candidates per workgroup and LDS bytes.
int score_tile_m64(int n, int d);
// Single launch of the float32 path when the model's escalation is decided
// on the device (its fit's statistics not read yet): the float32 kernel
// (gate 1) and the float64 kernel (gate 2) are both queued and each
// workgroup of the one that does not apply returns at once.
void launch_score_escalated(const ScoreArgs& a32, int tm32, const ScoreArgs& a64, int tm64,
                            hipStream_t s);
// Final argmax over the partials of whichever kernel ran.
void launch_argmax_gated(const double* part_v, const int64_t* part_i, int64_t np32, int64_t np64,
                         const double* stats, int64_t* argmax, double* ei_max, hipStream_t s);

// Batched scoring: a plan kernel sorts the problems into the launch
// precision's class and (float32 only) the float64 escalation class and
// numbers each class's (problem, tile) work items; one persistent launch per
// class pops them; a per-problem argmax follows.
struct BatchLaunch {
  const ScoreArgs* dd = nullptr;    // B descriptors in the launch precision (device)
  const ScoreArgs* dd64 = nullptr;  // B float64 descriptors of the same problems (device), or
                                    // NULL: no escalation
  int B = 0;
  int prec = GPBO_FP32;
  int tm = 32, tm64 = 16;           // candidates per work item of each class
  size_t smem = 0, smem64 = 0;      // dynamic LDS of each class's kernel
  int grid = 0, grid64 = 0;         // persistent workgroups of each class
  int per_cu = 2, per_cu64 = 1;     // their workgroups per CU (bounds the LDS of each)
  int nmax = 0, dmax = 0;           // largest n and d of the batch (the kernels' LDS layout)
  void* plan = nullptr;             // device plan area, batch_plan_bytes(B)
  int64_t* argmax = nullptr;        // device, B (may be NULL)
  double* ei_max = nullptr;         // device, B (may be NULL)
};
size_t batch_plan_bytes(int B);
// mark (may be NULL): (*mark)(0) / (*mark)(1) right before the first and
// after the last scoring kernel, for timing.
void launch_score_batched(const BatchLaunch& L, hipStream_t s,
                          const std::function<void(int)>* mark = nullptr);

// Sets *flag (device int, cleared by the launch) when any of the count
// values at p (float, or double when is_double) is a NaN or an infinity.
void launch_check_finite(const void* p, int64_t count, int is_double, int* flag, hipStream_t s);

// Top-k and gather (select.hip)
int topk_max_k();
size_t topk_scratch_bytes(int64_t m, int64_t k);
void launch_topk_into(int64_t m, const float* v, int64_t k, int64_t* idx, void* ws,
                      hipStream_t s);
// The top k as a set, in ascending index order (any k <= m): membership as
// in the sorted top-k (value descending, index ascending among ties).
size_t topk_set_scratch_bytes(int64_t m);
void launch_topk_set_into(int64_t m, const float* v, int64_t k, int64_t* idx, void* ws,
                          hipStream_t s);
// out[i] = outer[inner[i]] for i < k.
void launch_compose_idx(int64_t k, const int64_t* outer, const int64_t* inner, int64_t* out,
                        hipStream_t s);
// Pool index of a subset's argmax, its EI, and the certificate (see
// gpbo_score_subset); thr_key (the top-k set selection's threshold key in its
// scratch, launch_topk_set_threshold) may be NULL (every candidate scored).
void launch_subset_finish(const int64_t* am, const double* em, const int64_t* pool_idx,
                          const unsigned* thr_key, double tol, const double* stats, int64_t* next,
                          double* ei_max, int* certified, hipStream_t s);
// Where launch_topk_set_into leaves the order-preserving key of the k-th
// largest value (the selection threshold) in its scratch.
const unsigned* topk_set_threshold(const void* ws);
// Allocation-free top-k: the device address of the static scratch array on
// `device` (resolved by topk_noalloc_init with that device current, once per
// device; NULL before), and its size in bytes.
bool topk_noalloc_init(int device);
void* topk_noalloc_scratch(int device);
size_t topk_noalloc_bytes();
// Row argmax[b] of pool X[b] (m[b] rows of d[b] columns, float64 when dbl
// else float32) widened to float64 into row b of out (ldx columns, zero
// padded; NaN for an index outside the pool).  One launch per NEXT_MAX
// searches.
constexpr int NEXT_MAX = 64;
void launch_next_rows(int B, const void* const* X, const int64_t* m, const int* d, int dbl,
                      const int64_t* am, int ldx, double* out, hipStream_t s);
void launch_gather_rows(int64_t k, const int64_t* idx, int d, const float* Xc, float* out,
                        hipStream_t s);

// MLP ensemble (mlp.hip)
struct MlpState;
MlpState* mlp_create(Ctx* c, int E, int D, int H, const float* init, hipStream_t s);
void mlp_destroy(MlpState* st);
const float* mlp_master(MlpState* st);
int64_t mlp_nparams(MlpState* st);
bool mlp_train(MlpState* st, int64_t n, const float* X, const float* y, int steps, double lr,
               float* loss_hist, bool use_graph, hipStream_t s);
bool mlp_grads(MlpState* st, int64_t n, const float* X, const float* y, float* grad, float* loss,
               hipStream_t s);
// Training on a fitted model's own observations (its X and normalised y).
bool mlp_train_model(MlpState* st, const Model* M, int steps, double lr, float* loss_hist,
                     bool use_graph, hipStream_t s);
void mlp_forward(MlpState* st, int64_t m, const float* Xc, float* out, hipStream_t s);
// Forward grid: 0 = one workgroup per (sample tile, member); k > 0 = k
// workgroups per compute unit, each looping over items.
void mlp_set_occupancy(MlpState* st, int wg_per_cu);
void mlp_ens_ei(MlpState* st, int64_t m, const float* out, double fbest, float* ei, hipStream_t s);
void mlp_ens_lcb(MlpState* st, int64_t m, const float* out, double kappa, float* score,
                 hipStream_t s);
// Either rule on E member outputs (E x m): ensemble EI against arg = f_best,
// or the negated lower confidence bound with arg = kappa.
void ens_score(int E, int64_t m, const float* out, bool lcb, double arg, float* score,
               hipStream_t s);

}  // namespace gpbo
