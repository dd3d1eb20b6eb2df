// C ABI of the gpbo library (declared in include/gpbo.h): argument checks,
// device-memory management through the context's allocator, and the launch
// sequences of fit and scoring.  No C++ type or exception crosses the ABI.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gpbo_internal.h"

using namespace gpbo;

struct gpbo_ctx_s : Ctx {};
struct gpbo_model_s : Model {};

namespace {

thread_local std::string g_create_error;

gpbo_status fail(Ctx* c, gpbo_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->last_error = buf;
  else
    g_create_error = buf;
  return st;
}

#define HIP_TRY(c, call)                                                                \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail((c), GPBO_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

void free_model_buffers(Model* M) {
  Ctx* c = M->ctx;
  void* bufs[] = {M->X64, M->il64, M->L, M->Linv, M->Dinv, M->yt, M->alpha, M->work, M->L32,
                  M->stats, M->info, M->Xs32, M->sc32, M->sc64, M->Xs64};
  for (void* p : bufs)
    if (p) dfree(c, p);
  for (int i = 0; i < 3; ++i) {
    if (M->pk[i]) dfree(c, M->pk[i]);
    if (M->alphaT[i]) dfree(c, M->alphaT[i]);
  }
}

gpbo_status check_problem(Ctx* c, const gpbo_problem* p) {
  if (!p) return fail(c, GPBO_E_INVALID_ARG, "problem is NULL");
  if (p->n <= 0) return fail(c, GPBO_E_INVALID_ARG, "n must be positive (got %d)", p->n);
  if (p->d <= 0) return fail(c, GPBO_E_INVALID_ARG, "d must be positive (got %d)", p->d);
  if (p->d > 64) return fail(c, GPBO_E_UNSUPPORTED, "d > 64 is not supported (got %d)", p->d);
  if (p->n > 65536) return fail(c, GPBO_E_UNSUPPORTED, "n > 65536 is not supported (got %d)", p->n);
  if (!p->X || !p->y || !p->lengthscale) return fail(c, GPBO_E_INVALID_ARG, "X, y and lengthscale are required");
  if (p->kernel != GPBO_KERNEL_SE && p->kernel != GPBO_KERNEL_MATERN52)
    return fail(c, GPBO_E_INVALID_ARG, "unknown kernel %d", p->kernel);
  if (!(p->signal_var > 0.0) || !std::isfinite(p->signal_var))
    return fail(c, GPBO_E_INVALID_ARG, "signal_var must be positive and finite");
  if (!(p->noise_var >= 0.0) || !std::isfinite(p->noise_var))
    return fail(c, GPBO_E_INVALID_ARG, "noise_var must be non-negative and finite");
  for (int k = 0; k < p->d; ++k)
    if (!(p->lengthscale[k] > 0.0) || !std::isfinite(p->lengthscale[k]))
      return fail(c, GPBO_E_INVALID_ARG, "lengthscale[%d] must be positive and finite", k);
  return GPBO_OK;
}

// Allocate a model's buffers and queue its fit.  No synchronisation.
gpbo_status enqueue_fit(Ctx* c, const gpbo_problem* p, Model* M) {
  const int n = p->n, d = p->d;
  M->ctx = c;
  M->n = n;
  M->d = d;
  M->npad = (int)round_up(n, NB);
  M->kernel = p->kernel;
  M->sf2 = p->signal_var;
  M->sn2 = p->noise_var;
  M->ls.assign(p->lengthscale, p->lengthscale + d);
  const size_t np = M->npad;
  M->X64 = (double*)dmalloc(c, (size_t)n * d * sizeof(double));
  M->il64 = (double*)dmalloc(c, d * sizeof(double));
  M->L = (double*)dmalloc(c, np * np * sizeof(double));
  M->Linv = (double*)dmalloc(c, np * np * sizeof(double));
  M->Dinv = (double*)dmalloc(c, np * NB * sizeof(double));
  M->yt = (double*)dmalloc(c, np * sizeof(double));
  M->alpha = (double*)dmalloc(c, np * sizeof(double));
  M->work = (double*)dmalloc(c, 4 * np * sizeof(double));
  M->stats = (double*)dmalloc(c, S_COUNT * sizeof(double));
  M->info = (int*)dmalloc(c, 2 * sizeof(int));
  if (p->refine_alpha) M->L32 = (float*)dmalloc(c, np * np * sizeof(float));
  if (!M->X64 || !M->il64 || !M->L || !M->Linv || !M->Dinv || !M->yt || !M->alpha || !M->work ||
      !M->stats || !M->info || (p->refine_alpha && !M->L32))
    return fail(c, GPBO_E_OOM, "device allocation failed for a model with n=%d", n);
  hipStream_t s = c->stream;
  std::vector<double> il(d);
  for (int k = 0; k < d; ++k) il[k] = 1.0 / p->lengthscale[k];
  HIP_TRY(c, hipMemcpyAsync(M->X64, p->X, (size_t)n * d * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(M->il64, il.data(), d * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemsetAsync(M->stats, 0, S_COUNT * sizeof(double), s));
  launch_fit_prep(M, M->X64, p->y, p->normalize_y ? 1 : 0, s);
  launch_gram(M, M->L, s);
  launch_cholesky(M, M->L, s);
  launch_trtri(M, s);
  launch_alpha(M, p->refine_alpha ? 1 : 0, s);
  launch_lml(M, s);
  HIP_TRY(c, hipGetLastError());
  // the (small) synchronous copy of the coordinate scales needs the stream in
  // order anyway; build the float32 scoring operands eagerly
  return GPBO_OK;
}

gpbo_status finish_fit(Ctx* c, Model* M, int32_t* bad_pivot) {
  int info[2];
  HIP_TRY(c, hipMemcpyAsync(info, M->info, sizeof info, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(M->host_stats, M->stats, sizeof M->host_stats, hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (info[1]) return fail(c, GPBO_E_NONFINITE, "X or y holds a non-finite value");
  if (info[0] != INT_MAX) {
    if (bad_pivot) *bad_pivot = info[0];
    return fail(c, GPBO_E_NOT_PD, "K is not positive definite: pivot %d", info[0]);
  }
  if (bad_pivot) *bad_pivot = -1;
  return GPBO_OK;
}

}  // namespace

namespace gpbo {

void* dmalloc(Ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c->has_alloc) return c->alloc.alloc(bytes, c->stream, c->alloc.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dfree(Ctx* c, void* p) {
  if (!p) return;
  if (c->has_alloc)
    c->alloc.free(p, c->stream, c->alloc.user);
  else
    (void)hipFree(p);
}

}  // namespace gpbo

extern "C" {

const char* gpbo_status_string(gpbo_status s) {
  switch (s) {
    case GPBO_OK: return "ok";
    case GPBO_E_INVALID_ARG: return "invalid argument";
    case GPBO_E_NOT_PD: return "covariance matrix not positive definite";
    case GPBO_E_NONFINITE: return "non-finite input";
    case GPBO_E_OOM: return "out of device memory";
    case GPBO_E_HIP: return "HIP runtime error";
    case GPBO_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* gpbo_last_error(gpbo_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

int32_t gpbo_version(void) { return 10000; }

gpbo_status gpbo_ctx_create(int32_t device, void* stream, const gpbo_allocator* alloc,
                            gpbo_ctx* out) {
  if (!out) return fail(nullptr, GPBO_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(nullptr, GPBO_E_HIP, "no HIP device available (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "count is 0");
  }
  if (device < 0 || device >= count)
    return fail(nullptr, GPBO_E_INVALID_ARG, "device %d out of range (%d devices)", device, count);
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, GPBO_E_INVALID_ARG, "allocator needs both alloc and free");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(nullptr, GPBO_E_HIP, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, GPBO_E_UNSUPPORTED, "device %d is %s; this build targets gfx950", device,
                prop.gcnArchName);
  gpbo_ctx c = new (std::nothrow) gpbo_ctx_s();
  if (!c) return fail(nullptr, GPBO_E_OOM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->num_cu = prop.multiProcessorCount;
  if (alloc) {
    c->alloc = *alloc;
    c->has_alloc = true;
  }
  *out = c;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_destroy(gpbo_ctx c) {
  if (!c) return GPBO_OK;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
  if (c->red) dfree(c, c->red);
  if (c->batch_buf) dfree(c, c->batch_buf);
  delete c;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_set_stream(gpbo_ctx c, void* stream) {
  if (!c) return GPBO_E_INVALID_ARG;
  c->stream = (hipStream_t)stream;
  return GPBO_OK;
}

gpbo_status gpbo_fit(gpbo_ctx c, const gpbo_problem* p, gpbo_model* out, double* lml,
                     int32_t* bad_pivot) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!out) return fail(c, GPBO_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  gpbo_status st = check_problem(c, p);
  if (st != GPBO_OK) return st;
  DeviceGuard g(c->device);
  gpbo_model M = new (std::nothrow) gpbo_model_s();
  if (!M) return fail(c, GPBO_E_OOM, "host allocation failed");
  st = enqueue_fit(c, p, M);
  if (st == GPBO_OK) st = finish_fit(c, M, bad_pivot);
  if (st != GPBO_OK) {
    (void)hipStreamSynchronize(c->stream);
    free_model_buffers(M);
    delete M;
    return st;
  }
  if (lml) *lml = M->host_stats[S_LML];
  *out = M;
  return GPBO_OK;
}

gpbo_status gpbo_fit_batched(gpbo_ctx c, int32_t B, const gpbo_problem* probs, gpbo_model* out,
                             double* lml, int32_t* status) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!probs || !out || !status)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  DeviceGuard g(c->device);
  // Order by decreasing n^3 so the largest factorisations start first.
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].n > probs[b].n; });
  std::vector<gpbo_model> ms(B, nullptr);
  gpbo_status first = GPBO_OK;
  for (int b = 0; b < B; ++b) {
    out[b] = nullptr;
    status[b] = check_problem(c, &probs[b]);
  }
  for (int k = 0; k < B; ++k) {
    const int b = order[k];
    if (status[b] != GPBO_OK) continue;
    ms[b] = new (std::nothrow) gpbo_model_s();
    if (!ms[b]) {
      status[b] = GPBO_E_OOM;
      continue;
    }
    status[b] = enqueue_fit(c, &probs[b], ms[b]);
  }
  for (int b = 0; b < B; ++b) {
    if (ms[b] && status[b] == GPBO_OK) status[b] = finish_fit(c, ms[b], nullptr);
    if (status[b] != GPBO_OK) {
      if (first == GPBO_OK) first = (gpbo_status)status[b];
      if (ms[b]) {
        (void)hipStreamSynchronize(c->stream);
        free_model_buffers(ms[b]);
        delete ms[b];
        ms[b] = nullptr;
      }
    } else {
      out[b] = ms[b];
      if (lml) lml[b] = ms[b]->host_stats[S_LML];
    }
  }
  return first;
}

gpbo_status gpbo_model_free(gpbo_model M) {
  if (!M) return GPBO_OK;
  DeviceGuard g(M->ctx->device);
  (void)hipStreamSynchronize(M->ctx->stream);
  free_model_buffers(M);
  delete M;
  return GPBO_OK;
}

gpbo_status gpbo_model_stats(gpbo_model M, double* stats) {
  if (!M || !stats) return GPBO_E_INVALID_ARG;
  for (int i = 0; i < GPBO_NSTATS; ++i) stats[i] = M->host_stats[i];
  return GPBO_OK;
}

gpbo_status gpbo_model_shape(gpbo_model M, int32_t* n, int32_t* d) {
  if (!M) return GPBO_E_INVALID_ARG;
  if (n) *n = M->n;
  if (d) *d = M->d;
  return GPBO_OK;
}

gpbo_status gpbo_model_factors(gpbo_ctx c, gpbo_model M, double* L, double* Linv, double* alpha) {
  if (!c || !M) return GPBO_E_INVALID_ARG;
  DeviceGuard g(c->device);
  const size_t n = M->n, np = M->npad;
  if (L)
    HIP_TRY(c, hipMemcpy2DAsync(L, n * sizeof(double), M->L, np * sizeof(double), n * sizeof(double),
                                n, hipMemcpyDeviceToDevice, c->stream));
  if (Linv)
    HIP_TRY(c, hipMemcpy2DAsync(Linv, n * sizeof(double), M->Linv, np * sizeof(double),
                                n * sizeof(double), n, hipMemcpyDeviceToDevice, c->stream));
  if (alpha)
    HIP_TRY(c, hipMemcpyAsync(alpha, M->alpha, n * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
  return GPBO_OK;
}

static gpbo_status ensure_red(Ctx* c, size_t bytes) {
  if (c->red_bytes >= bytes) return GPBO_OK;
  if (c->red) {
    (void)hipStreamSynchronize(c->stream);
    dfree(c, c->red);
  }
  c->red = dmalloc(c, bytes);
  c->red_bytes = c->red ? bytes : 0;
  return c->red ? GPBO_OK : fail(c, GPBO_E_OOM, "scratch allocation of %zu bytes failed", bytes);
}

gpbo_status gpbo_score(gpbo_ctx c, gpbo_model M, int64_t m, const void* Xc, gpbo_precision prec,
                       void* mu, void* sigma, void* ei, int64_t* argmax, double* ei_max) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!M) return fail(c, GPBO_E_INVALID_ARG, "model is NULL");
  if (m < 0) return fail(c, GPBO_E_INVALID_ARG, "m must be >= 0");
  if (m > 0 && !Xc) return fail(c, GPBO_E_INVALID_ARG, "Xc is NULL");
  if (prec != GPBO_FP64 && prec != GPBO_FP32 && prec != GPBO_BF16)
    return fail(c, GPBO_E_INVALID_ARG, "unknown precision %d", (int)prec);
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  if (m == 0) {
    if (argmax || ei_max) launch_argmax_final(nullptr, nullptr, 0, argmax, ei_max, s);
    HIP_TRY(c, hipGetLastError());
    return GPBO_OK;
  }
  const int tm = score_tile_m(prec, M->n, M->d);
  if (tm == 0)
    return fail(c, GPBO_E_UNSUPPORTED, "n=%d is too large for the fused scoring kernel at this precision",
                M->n);
  ensure_score_operands(M, prec, s);
  const int64_t tiles = ceil_div(m, tm);
  double* pv = nullptr;
  int64_t* pi = nullptr;
  if (argmax || ei_max) {
    gpbo_status st = ensure_red(c, (size_t)tiles * 16);
    if (st != GPBO_OK) return st;
    pv = (double*)c->red;
    pi = (int64_t*)((double*)c->red + tiles);
  }
  ScoreJob j{};
  j.n = M->n;
  j.d = M->d;
  j.npk = (int)round_up(M->n, TI);
  j.kernel = M->kernel;
  j.pk = M->pk[prec];
  j.alpha = M->alphaT[prec];
  j.Xs = prec == GPBO_FP64 ? (const void*)M->Xs64 : (const void*)M->Xs32;
  j.sc = prec == GPBO_FP64 ? (const void*)M->sc64 : (const void*)M->sc32;
  j.stats = M->stats;
  j.sf2 = M->sf2;
  j.m = m;
  j.Xc = Xc;
  j.mu = mu;
  j.sigma = sigma;
  j.ei = ei;
  j.part_v = pv;
  j.part_i = pi;
  launch_score(j, prec, tm, s);
  if (pv) launch_argmax_final(pv, pi, tiles, argmax, ei_max, s);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_score_batched(gpbo_ctx c, int32_t B, const gpbo_model* models, const int64_t* m,
                               const void* const* Xc, gpbo_precision prec, void* const* ei,
                               int64_t* argmax, double* ei_max) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !m || !Xc)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  for (int b = 0; b < B; ++b) {
    gpbo_status st = gpbo_score(c, models[b], m[b], Xc[b], prec, nullptr, nullptr,
                                ei ? ei[b] : nullptr, argmax ? argmax + b : nullptr,
                                ei_max ? ei_max + b : nullptr);
    if (st != GPBO_OK) return st;
  }
  return GPBO_OK;
}

gpbo_status gpbo_topk(gpbo_ctx c, int64_t m, const float* v, int64_t k, int64_t* idx) {
  if (!c) return GPBO_E_INVALID_ARG;
  return fail(c, GPBO_E_UNSUPPORTED, "top-k is not built yet");
}

gpbo_status gpbo_gather_rows(gpbo_ctx c, int64_t k, const int64_t* idx, int32_t d, const float* Xc,
                             float* out) {
  if (!c) return GPBO_E_INVALID_ARG;
  return fail(c, GPBO_E_UNSUPPORTED, "gather is not built yet");
}

int64_t gpbo_mlp_nparams(int32_t d_in, int32_t hidden) {
  return (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + hidden + 1;
}

gpbo_status gpbo_mlp_create(gpbo_ctx c, int32_t, int32_t, int32_t, const float*, gpbo_mlp* out) {
  if (out) *out = nullptr;
  if (!c) return GPBO_E_INVALID_ARG;
  return fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet");
}
gpbo_status gpbo_mlp_free(gpbo_mlp) { return GPBO_OK; }
gpbo_status gpbo_mlp_params(gpbo_ctx c, gpbo_mlp, float*) {
  return c ? fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet") : GPBO_E_INVALID_ARG;
}
gpbo_status gpbo_mlp_grads(gpbo_ctx c, gpbo_mlp, int32_t, const float*, const float*, float*, float*) {
  return c ? fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet") : GPBO_E_INVALID_ARG;
}
gpbo_status gpbo_mlp_train(gpbo_ctx c, gpbo_mlp, int32_t, const float*, const float*, int32_t,
                           double, float*) {
  return c ? fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet") : GPBO_E_INVALID_ARG;
}
gpbo_status gpbo_mlp_forward(gpbo_ctx c, gpbo_mlp, int64_t, const float*, float*) {
  return c ? fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet") : GPBO_E_INVALID_ARG;
}
gpbo_status gpbo_mlp_prescreen(gpbo_ctx c, gpbo_mlp, int64_t, const float*, double, int64_t,
                               int64_t*, float*) {
  return c ? fail(c, GPBO_E_UNSUPPORTED, "MLP prescreen is not built yet") : GPBO_E_INVALID_ARG;
}

}  // extern "C"
