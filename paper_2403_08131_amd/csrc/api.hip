// C ABI of the gpbo library (declared in include/gpbo.h): argument checks,
// device-memory management through the context's allocator, and the launch
// sequences of fit and scoring.  No C++ type or exception crosses the ABI.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
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
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void free_model_buffers(Model* M) {
  M->blk_fit.reset();
  M->blk_obs.reset();
  for (int i = 0; i < 3; ++i) M->blk_score[i].reset();
  M->host_stage.reset();
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

// Byte offsets of one model's buffers inside its part of a fit allocation.
struct FitLayout {
  size_t oX, oy, oil, oL, oLi, oK, oD, oyt, oa, ow, o32, bytes;
};

// X and y take npad rows so that rank-one appends fill the padding before
// the buffers have to grow.
FitLayout fit_layout(int n, int d, bool refine) {
  const size_t np = round_up(n, NB);
  Carve cv;
  FitLayout f;
  f.oX = cv.take(np * d * sizeof(double));
  f.oy = cv.take(np * sizeof(double));
  f.oil = cv.take(d * sizeof(double));
  f.oL = cv.take(np * np * sizeof(double));
  f.oLi = cv.take(np * np * sizeof(double));
  f.oK = cv.take(np * np * sizeof(double));
  f.oD = cv.take(np * NB * sizeof(double));
  f.oyt = cv.take(np * sizeof(double));
  f.oa = cv.take(np * sizeof(double));
  f.ow = cv.take((4 + 1) * np * sizeof(double));  // 4 vectors + the product K alpha
  f.o32 = refine ? cv.take(np * np * sizeof(float)) : 0;
  f.bytes = cv.bytes;
  return f;
}

hipEvent_t timing_event(Ctx* c);

// A pinned host chunk of at least `bytes` from the context's pool (a new
// hipHostMalloc only when none fits); *got receives its size.
unsigned char* pinned_acquire(Ctx* c, size_t bytes, size_t* got) {
  for (size_t i = 0; i < c->pinned_pool.size(); ++i)
    if (c->pinned_pool[i].first >= bytes) {
      const auto pr = c->pinned_pool[i];
      c->pinned_pool.erase(c->pinned_pool.begin() + (std::ptrdiff_t)i);
      *got = pr.first;
      return pr.second;
    }
  const size_t sz = round_up(bytes, 4096);
  void* p = nullptr;
  if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  *got = sz;
  return (unsigned char*)p;
}

// The fit's launch sequence (descriptors already uploaded to dd in stream
// order).  On a created stream it is captured once per launch shape and
// replayed after that: the kernels read everything problem-specific from
// the descriptors, so the next fit of a search with the same sizes replays
// the 28-launch sequence (n = 512) as one graph launch.  The legacy default
// stream cannot be captured; there every call launches eagerly.
gpbo_status run_fit(Ctx* c, const FitDesc* h, const FitDesc* dd, int B, hipStream_t s) {
  std::vector<uint64_t> key = fit_launch_shape(h, B);
  key.push_back((uint64_t)(uintptr_t)dd);
  key.push_back((uint64_t)(uintptr_t)s);
  if (s != nullptr && !c->no_graph)
    for (auto& kv : c->fit_graphs)
      if (kv.first == key) {
        HIP_TRY(c, hipGraphLaunch(kv.second, s));
        return GPBO_OK;
      }
  // an eager launch (it also sets the kernels' LDS limits), then the capture
  launch_fit(h, dd, B, s);
  HIP_TRY(c, hipGetLastError());
  if (s == nullptr || c->no_graph) return GPBO_OK;
  constexpr size_t kMaxGraphs = 8;
  if (c->fit_graphs.size() >= kMaxGraphs) {
    // the oldest goes once every stream it may have been launched on has run it
    HIP_TRY(c, hipDeviceSynchronize());
    (void)hipGraphExecDestroy(c->fit_graphs.front().second);
    c->fit_graphs.erase(c->fit_graphs.begin());
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  launch_fit(h, dd, B, s);
  HIP_TRY(c, hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e == hipSuccess) c->fit_graphs.emplace_back(key, exec);
  return GPBO_OK;
}

// The rank-one append's launch sequence (descriptors of the models before
// and after at dd and dd + B), captured and replayed like the fit's: its
// grids depend on the padded sizes only, so the iterations of a search
// replay one graph until its padding fills.
gpbo_status run_append(Ctx* c, const FitDesc* h, const FitDesc* dd, int B, hipStream_t s) {
  std::vector<uint64_t> key = append_launch_shape(h + B, B);
  key.push_back((uint64_t)(uintptr_t)dd);
  key.push_back((uint64_t)(uintptr_t)s);
  if (s != nullptr && !c->no_graph)
    for (auto& kv : c->fit_graphs)
      if (kv.first == key) {
        HIP_TRY(c, hipGraphLaunch(kv.second, s));
        return GPBO_OK;
      }
  launch_append(h, dd, h + B, dd + B, B, s);
  HIP_TRY(c, hipGetLastError());
  if (s == nullptr || c->no_graph) return GPBO_OK;
  constexpr size_t kMaxGraphs = 8;
  if (c->fit_graphs.size() >= kMaxGraphs) {
    HIP_TRY(c, hipDeviceSynchronize());
    (void)hipGraphExecDestroy(c->fit_graphs.front().second);
    c->fit_graphs.erase(c->fit_graphs.begin());
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  launch_append(h, dd, h + B, dd + B, B, s);
  HIP_TRY(c, hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e == hipSuccess) c->fit_graphs.emplace_back(key, exec);
  return GPBO_OK;
}

// Per-model slot of the status region at the start of a fit allocation:
// S_COUNT statistics, then the two info words.
constexpr size_t STATUS_SLOT = 128;
static_assert(S_COUNT * sizeof(double) + 2 * sizeof(int) <= STATUS_SLOT, "status slot");

// Fit the models of `ms` (entries that are NULL are skipped) on problems
// `probs`, with one device allocation for all of them (a status region, then
// each model's buffers), one upload of the descriptors and staged inverse
// lengthscales, one launch sequence and one readback of every model's
// statistics.  status[b] receives each problem's result; on return the
// stream is synchronised.  Models whose status is not OK still hold their
// buffers (the caller frees them).
gpbo_status fit_group(Ctx* c, int B, const gpbo_problem* probs, Model* const* ms, int32_t* status,
                      bool sync = true) {
  std::vector<int> order;  // problems to fit, by decreasing n
  for (int b = 0; b < B; ++b)
    if (ms[b] && status[b] == GPBO_OK) order.push_back(b);
  if (order.empty()) return GPBO_OK;
  // the largest problems take the lowest workgroup indices (dispatched
  // first) in every batched launch
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].n > probs[b].n; });
  const int nb = (int)order.size();
  Carve cv;
  const size_t ostat = cv.take(nb * STATUS_SLOT);
  std::vector<FitLayout> lay(nb);
  std::vector<size_t> obase(nb);
  for (int k = 0; k < nb; ++k) {
    const gpbo_problem& p = probs[order[k]];
    lay[k] = fit_layout(p.n, p.d, p.refine_alpha != 0);
    obase[k] = cv.take(lay[k].bytes);
  }
  std::shared_ptr<void> grp = dshared(c, cv.bytes);
  if (!grp) {
    for (int b : order) status[b] = GPBO_E_OOM;
    return fail(c, GPBO_E_OOM, "device allocation of %zu bytes failed for %d models", cv.bytes, nb);
  }
  char* g = (char*)grp.get();
  // descriptors, then the inverse lengthscales of every problem
  size_t il_total = 0;
  for (int b : order) il_total += probs[b].d;
  const size_t desc_bytes = round_up(nb * sizeof(FitDesc), 256);
  const size_t up_bytes = desc_bytes + il_total * sizeof(double);
  if (c->desc_bytes < up_bytes) {
    if (c->desc_buf) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      dfree(c, c->desc_buf);
    }
    c->desc_buf = dmalloc(c, up_bytes);
    c->desc_bytes = c->desc_buf ? up_bytes : 0;
    if (!c->desc_buf) return fail(c, GPBO_E_OOM, "descriptor allocation failed");
  }
  std::vector<unsigned char> up(up_bytes);
  double* il_h = (double*)(up.data() + desc_bytes);
  const double* il_d = (const double*)((char*)c->desc_buf + desc_bytes);
  std::vector<FitDesc> hd(nb);
  size_t il_off = 0;
  for (int k = 0; k < nb; ++k) {
    const gpbo_problem& p = probs[order[k]];
    Model* M = ms[order[k]];
    const FitLayout& f = lay[k];
    char* b = g + obase[k];
    M->ctx = c;
    M->alloc_stream = c->stream;
    M->alloc_mixed = false;
    M->n = p.n;
    M->d = p.d;
    M->npad = (int)round_up(p.n, NB);
    M->kernel = p.kernel;
    M->normalize = p.normalize_y ? 1 : 0;
    M->refine = p.refine_alpha ? 1 : 0;
    M->sf2 = p.signal_var;
    M->sn2 = p.noise_var;
    M->ls.assign(p.lengthscale, p.lengthscale + p.d);
    M->X64 = (double*)(b + f.oX);
    M->y64 = (double*)(b + f.oy);
    M->il64 = (double*)(b + f.oil);
    M->L = (double*)(b + f.oL);
    M->Linv = (double*)(b + f.oLi);
    M->K = (double*)(b + f.oK);
    M->Dinv = (double*)(b + f.oD);
    M->yt = (double*)(b + f.oyt);
    M->alpha = (double*)(b + f.oa);
    M->work = (double*)(b + f.ow);
    M->L32 = p.refine_alpha ? (float*)(b + f.o32) : nullptr;
    M->stats = (double*)(g + ostat + k * STATUS_SLOT);
    M->info = (int*)(g + ostat + k * STATUS_SLOT + S_COUNT * sizeof(double));
    M->blk_fit = std::shared_ptr<void>(grp, b);  // shares the group's allocation
    for (int j = 0; j < p.d; ++j) il_h[il_off + j] = 1.0 / p.lengthscale[j];
    hd[k] = make_fit_desc(M, p.X, il_d + il_off, p.y, p.normalize_y ? 1 : 0, p.refine_alpha ? 1 : 0);
    il_off += p.d;
  }
  std::memcpy(up.data(), hd.data(), nb * sizeof(FitDesc));
  // a copy from pageable memory has consumed its source when it returns
  HIP_TRY(c, hipMemcpyAsync(c->desc_buf, up.data(), up_bytes, hipMemcpyHostToDevice, c->stream));
  {
    const gpbo_status st = run_fit(c, hd.data(), (const FitDesc*)c->desc_buf, nb, c->stream);
    if (st != GPBO_OK) return st;
  }
  if (!sync) {  // the statistics are read when the caller asks for a status
    auto gs = std::make_shared<Model::GroupStatus>();
    gs->dev = (const unsigned char*)(g + ostat);
    gs->nb = nb;
    gs->ctx = c;
    size_t got = 0;
    gs->pinned = pinned_acquire(c, (size_t)nb * STATUS_SLOT, &got);
    if (gs->pinned) {
      gs->pinned_bytes = got;
      HIP_TRY(c, hipMemcpyAsync(gs->pinned, gs->dev, (size_t)nb * STATUS_SLOT,
                                hipMemcpyDeviceToHost, c->stream));
      gs->ev = timing_event(c);
      if (gs->ev) HIP_TRY(c, hipEventRecord(gs->ev, c->stream));
    }
    for (int k = 0; k < nb; ++k) {
      Model* M = ms[order[k]];
      M->pending = true;
      M->gstat = gs;
      M->gslot = k;
    }
    HIP_TRY(c, hipGetLastError());
    return GPBO_OK;
  }
  std::vector<unsigned char> st_h(nb * STATUS_SLOT);
  HIP_TRY(c, hipMemcpyAsync(st_h.data(), g + ostat, st_h.size(), hipMemcpyDeviceToHost, c->stream));
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, GPBO_E_HIP, "fit: %s", hipGetErrorString(e));
  for (int k = 0; k < nb; ++k) {
    Model* M = ms[order[k]];
    std::memcpy(M->host_stats, st_h.data() + k * STATUS_SLOT, sizeof M->host_stats);
    std::memcpy(M->host_info, st_h.data() + k * STATUS_SLOT + S_COUNT * sizeof(double),
                sizeof M->host_info);
  }
  return GPBO_OK;
}

// Status of a fit whose readback has completed.
gpbo_status fit_status(Ctx* c, Model* M, int32_t* bad_pivot) {
  if (M->host_info[1]) return fail(c, GPBO_E_NONFINITE, "X or y holds a non-finite value");
  if (M->host_info[0] != INT_MAX) {
    if (bad_pivot) *bad_pivot = M->host_info[0];
    return fail(c, GPBO_E_NOT_PD, "K is not positive definite: pivot %d", M->host_info[0]);
  }
  if (bad_pivot) *bad_pivot = -1;
  return GPBO_OK;
}

// Read the statistics and status of an asynchronously fitted model
// (synchronises the context's stream).
gpbo_status resolve_pending(Ctx* c, Model* M) {
  if (!M->pending) return GPBO_OK;
  Model::GroupStatus& gs = *M->gstat;
  if (!gs.read) {  // every model of the fit call at once
    gs.host.resize((size_t)gs.nb * STATUS_SLOT);
    if (gs.pinned && gs.ev) {  // copied behind the fit already
      HIP_TRY(c, hipEventSynchronize(gs.ev));
      std::memcpy(gs.host.data(), gs.pinned, gs.host.size());
    } else {
      HIP_TRY(c, hipMemcpyAsync(gs.host.data(), gs.dev, gs.host.size(), hipMemcpyDeviceToHost,
                                c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    gs.read = true;
  }
  const unsigned char* slot = gs.host.data() + (size_t)M->gslot * STATUS_SLOT;
  std::memcpy(M->host_stats, slot, sizeof M->host_stats);
  std::memcpy(M->host_info, slot + S_COUNT * sizeof(double), sizeof M->host_info);
  M->pending = false;
  M->gstat.reset();
  return GPBO_OK;
}

hipEvent_t timing_event(Ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
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

// A later copy into a returned chunk is queued on the same stream behind
// any copy still in flight, and its reader waits for its own event.
Model::GroupStatus::~GroupStatus() {
  if (!ctx) return;
  // the copy into the chunk may still be in flight (a model freed without
  // asking for its status): the chunk is reused only once it has landed
  if (pinned && ev && hipEventQuery(ev) != hipSuccess) (void)hipEventSynchronize(ev);
  if (pinned && !ev) (void)hipStreamSynchronize(ctx->stream);
  if (pinned) {
    if (ctx->pinned_pool.size() < 64)
      ctx->pinned_pool.emplace_back(pinned_bytes, pinned);
    else
      (void)hipHostFree(pinned);
  }
  if (ev) ctx->ev_pool.push_back(ev);
}

std::shared_ptr<void> dshared(Ctx* c, size_t bytes) {
  void* p = dmalloc(c, bytes);
  if (!p) return nullptr;
  return std::shared_ptr<void>(p, [c](void* q) { dfree(c, q); });
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
  {
    // the allocation-free top-k's static scratch on this device: its device
    // address, resolved once per device with the device current
    DeviceGuard g(device);
    if (!topk_noalloc_init(device))
      return fail(nullptr, GPBO_E_HIP, "device %d: address of the static top-k scratch unavailable",
                  device);
  }
  gpbo_ctx c = new (std::nothrow) gpbo_ctx_s();
  if (!c) return fail(nullptr, GPBO_E_OOM, "host allocation failed");
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->num_cu = prop.multiProcessorCount;
  if (const char* ng = std::getenv("GPBO_NO_GRAPH")) c->no_graph = ng[0] == '1';
  if (const char* dbg = std::getenv("GPBO_DEBUG")) c->debug = dbg[0] == '1';
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
  // objects still alive on the context go with it
  for (void* p : std::vector<void*>(c->live_mlps.begin(), c->live_mlps.end()))
    (void)gpbo_mlp_free((gpbo_mlp)p);
  for (Model* M : std::vector<Model*>(c->live_models.begin(), c->live_models.end()))
    (void)gpbo_model_free((gpbo_model)M);
  for (auto& kv : c->batch_graphs) (void)hipGraphExecDestroy(kv.second);
  c->batch_graphs.clear();
  for (auto& kv : c->fit_graphs) (void)hipGraphExecDestroy(kv.second);
  c->fit_graphs.clear();
  for (auto& pr : c->ev_pending) {
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& pr : c->pinned_pool) (void)hipHostFree(pr.second);
  if (c->red) dfree(c, c->red);
  if (c->desc_buf) dfree(c, c->desc_buf);
  if (c->batch_buf) dfree(c, c->batch_buf);
  delete c;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_set_stream(gpbo_ctx c, void* stream) {
  if (!c) return GPBO_E_INVALID_ARG;
  // the work queued so far finishes first: the context's own buffers
  // (descriptor uploads, reduction scratch) and its objects' buffers are
  // then used on one stream at a time, and a release after the switch needs
  // no wait on the old stream
  if ((hipStream_t)stream != c->stream) {
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->stream = (hipStream_t)stream;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_enable_timing(gpbo_ctx c, int32_t enable) {
  if (!c) return GPBO_E_INVALID_ARG;
  c->timing = enable != 0;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_set_score_path(gpbo_ctx c, gpbo_score_path path) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (path != GPBO_PATH_AUTO && path != GPBO_PATH_FUSED && path != GPBO_PATH_LARGE)
    return fail(c, GPBO_E_INVALID_ARG, "unknown scoring path %d", (int)path);
  c->score_path = (int)path;
  return GPBO_OK;
}

gpbo_status gpbo_ctx_timing(gpbo_ctx c, int64_t* launches, double* total_ms) {
  if (!c) return GPBO_E_INVALID_ARG;
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (auto& pr : c->ev_pending) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  if (launches) *launches = (int64_t)c->ev_pending.size();
  if (total_ms) *total_ms = tot;
  c->ev_pending.clear();
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
  Model* ms[1] = {M};
  int32_t status[1] = {GPBO_OK};
  st = fit_group(c, 1, p, ms, status);
  if (st == GPBO_OK) st = (gpbo_status)status[0];
  if (st == GPBO_OK) st = fit_status(c, M, bad_pivot);
  if (st != GPBO_OK) {
    (void)hipStreamSynchronize(c->stream);
    free_model_buffers(M);
    delete M;
    return st;
  }
  if (lml) *lml = M->host_stats[S_LML];
  c->live_models.insert(M);
  *out = M;
  return GPBO_OK;
}

gpbo_status gpbo_fit_async(gpbo_ctx c, const gpbo_problem* p, gpbo_model* out) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!out) return fail(c, GPBO_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  gpbo_status st = check_problem(c, p);
  if (st != GPBO_OK) return st;
  DeviceGuard g(c->device);
  gpbo_model M = new (std::nothrow) gpbo_model_s();
  if (!M) return fail(c, GPBO_E_OOM, "host allocation failed");
  Model* ms[1] = {M};
  int32_t status[1] = {GPBO_OK};
  st = fit_group(c, 1, p, ms, status, false);
  if (st == GPBO_OK) st = (gpbo_status)status[0];
  if (st != GPBO_OK) {
    (void)hipStreamSynchronize(c->stream);
    free_model_buffers(M);
    delete M;
    return st;
  }
  c->live_models.insert(M);
  *out = M;
  return GPBO_OK;
}

gpbo_status gpbo_fit_batched_async(gpbo_ctx c, int32_t B, const gpbo_problem* probs,
                                   gpbo_model* out, int32_t* status) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!probs || !out || !status)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  DeviceGuard g(c->device);
  std::vector<gpbo_model> ms(B, nullptr);
  gpbo_status first = GPBO_OK;
  for (int b = 0; b < B; ++b) {
    out[b] = nullptr;
    status[b] = check_problem(c, &probs[b]);
    if (status[b] == GPBO_OK) {
      ms[b] = new (std::nothrow) gpbo_model_s();
      if (!ms[b]) status[b] = GPBO_E_OOM;
    }
  }
  std::vector<Model*> mp(ms.begin(), ms.end());
  gpbo_status gst = fit_group(c, B, probs, mp.data(), status, false);
  for (int b = 0; b < B; ++b) {
    if (ms[b] && status[b] == GPBO_OK && gst != GPBO_OK) status[b] = gst;
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
      c->live_models.insert(ms[b]);
    }
  }
  return first;
}

gpbo_status gpbo_model_status_batched(gpbo_ctx c, int32_t B, const gpbo_model* models,
                                      int32_t* status, double* lml) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !status)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  DeviceGuard g(c->device);
  gpbo_status first = GPBO_OK;
  for (int b = 0; b < B; ++b) {
    gpbo_status st = models[b] ? resolve_pending(c, models[b]) : GPBO_E_INVALID_ARG;
    if (st == GPBO_OK) st = fit_status(c, models[b], nullptr);
    status[b] = st;
    if (lml) lml[b] = st == GPBO_OK ? models[b]->host_stats[S_LML] : NAN;
    if (st != GPBO_OK && first == GPBO_OK) first = st;
  }
  return first;
}

gpbo_status gpbo_model_status(gpbo_ctx c, gpbo_model M, int32_t* bad_pivot, double* lml) {
  if (!c || !M) return GPBO_E_INVALID_ARG;
  DeviceGuard g(c->device);
  gpbo_status st = resolve_pending(c, M);
  if (st != GPBO_OK) return st;
  st = fit_status(c, M, bad_pivot);
  if (st == GPBO_OK && lml) *lml = M->host_stats[S_LML];
  return st;
}

gpbo_status gpbo_fit_batched(gpbo_ctx c, int32_t B, const gpbo_problem* probs, gpbo_model* out,
                             double* lml, int32_t* status) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!probs || !out || !status)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  DeviceGuard g(c->device);
  std::vector<gpbo_model> ms(B, nullptr);
  gpbo_status first = GPBO_OK;
  for (int b = 0; b < B; ++b) {
    out[b] = nullptr;
    status[b] = check_problem(c, &probs[b]);
    if (status[b] == GPBO_OK) {
      ms[b] = new (std::nothrow) gpbo_model_s();
      if (!ms[b]) status[b] = GPBO_E_OOM;
    }
  }
  std::vector<Model*> mp(ms.begin(), ms.end());
  gpbo_status gst = fit_group(c, B, probs, mp.data(), status);
  for (int b = 0; b < B; ++b) {
    if (ms[b] && status[b] == GPBO_OK) status[b] = gst != GPBO_OK ? gst : fit_status(c, ms[b], nullptr);
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
      c->live_models.insert(ms[b]);
      if (lml) lml[b] = ms[b]->host_stats[S_LML];
    }
  }
  return first;
}

gpbo_status gpbo_model_free(gpbo_model M) {
  if (!M) return GPBO_OK;
  DeviceGuard g(M->ctx->device);
  // With the context's allocator the buffers return in the order of the
  // stream they were allocated on, behind the work queued there.  A model
  // whose buffers were touched on another stream may still be read there
  // (the context may have moved back to the allocating stream since), so
  // it waits for the whole device; otherwise a wait on the context's
  // stream covers the case of a context moved to another stream, and
  // hipFree without an allocator.
  const Ctx* c = M->ctx;
  if (M->alloc_mixed)
    (void)hipDeviceSynchronize();
  else if (!c->has_alloc || M->alloc_stream != c->stream)
    (void)hipStreamSynchronize(c->stream);
  M->ctx->live_models.erase(M);
  free_model_buffers(M);
  delete M;
  return GPBO_OK;
}

gpbo_status gpbo_model_stats(gpbo_model M, double* stats) {
  if (!M || !stats) return GPBO_E_INVALID_ARG;
  if (M->pending) {
    DeviceGuard g(M->ctx->device);
    gpbo_status st = resolve_pending(M->ctx, M);
    if (st != GPBO_OK) return st;
  }
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
  if (M->alloc_stream != c->stream) M->alloc_mixed = true;
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

// Above this many observations gpbo_score takes the chunked float32 path.
static gpbo_status wait_before_release(Ctx* c, const Model* M);
static gpbo_status ensure_desc(Ctx* c, size_t bytes);

constexpr int LARGE_N_MIN = 1024;

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

// Whether a kernel may write to p: device (or managed) memory.  Anything else
// (pageable or pinned host memory) is written by a copy after the stream is
// synchronised.
static bool device_writable(const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // ordinary host memory: not known to HIP
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// A model touched on another stream than the one its buffers came from is
// freed only after a wait (gpbo_model_free).
static void note_stream(Model* M, hipStream_t s) {
  if (M->alloc_stream != s) M->alloc_mixed = true;
}

// Buffers of M that may still be read by queued work are released only
// after a wait when the stream order does not cover it (see gpbo_model_free).
static gpbo_status wait_before_release(Ctx* c, const Model* M) {
  if (M->alloc_mixed)
    HIP_TRY(c, hipDeviceSynchronize());
  else if (!c->has_alloc || M->alloc_stream != c->stream)
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  return GPBO_OK;
}

// The descriptor buffer holds at least `bytes` (a larger one replaces it
// once the work that reads the old one has run).
static gpbo_status ensure_desc(Ctx* c, size_t bytes) {
  if (c->desc_bytes >= bytes) return GPBO_OK;
  if (c->desc_buf) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c, c->desc_buf);
  }
  c->desc_buf = dmalloc(c, bytes);
  c->desc_bytes = c->desc_buf ? bytes : 0;
  return c->desc_buf ? GPBO_OK : fail(c, GPBO_E_OOM, "descriptor allocation failed");
}

gpbo_status gpbo_append_batched(gpbo_ctx c, int32_t B, const gpbo_model* models,
                                const double* x_new, int32_t ldx, const double* y_new) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !x_new || !y_new)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  if (!device_writable(x_new) || !device_writable(y_new))
    return fail(c, GPBO_E_INVALID_ARG, "x_new and y_new must be device memory");
  std::vector<Model*> ms(B);
  for (int b = 0; b < B; ++b) {
    Model* M = models[b];
    if (!M) return fail(c, GPBO_E_INVALID_ARG, "model %d is NULL", b);
    if (M->ctx != c) return fail(c, GPBO_E_INVALID_ARG, "model %d belongs to another context", b);
    for (int a = 0; a < b; ++a)
      if (ms[a] == M) return fail(c, GPBO_E_INVALID_ARG, "model %d appears twice in the batch", b);
    if (ldx < M->d)
      return fail(c, GPBO_E_INVALID_ARG, "ldx %d is smaller than model %d's d = %d", ldx, b, M->d);
    if (M->n + 1 > 65536)
      return fail(c, GPBO_E_UNSUPPORTED, "model %d would exceed n = 65536", b);
    ms[b] = M;
  }
  // Models whose padding is full move to buffers one tile larger (one
  // allocation for all of them, filled on the device).
  std::vector<int> grow;
  for (int b = 0; b < B; ++b)
    if (ms[b]->n + 1 > ms[b]->npad) grow.push_back(b);
  if (!grow.empty()) {
    const int ng = (int)grow.size();
    Carve cv;
    const size_t ostat = cv.take((size_t)ng * STATUS_SLOT);
    std::vector<FitLayout> lay(ng);
    std::vector<size_t> base(ng);
    for (int k = 0; k < ng; ++k) {
      const Model* M = ms[grow[k]];
      lay[k] = fit_layout(M->npad + 1, M->d, M->refine != 0);
      base[k] = cv.take(lay[k].bytes);
    }
    std::shared_ptr<void> grp = dshared(c, cv.bytes);
    if (!grp) return fail(c, GPBO_E_OOM, "device allocation of %zu bytes failed", cv.bytes);
    char* gb = (char*)grp.get();
    std::vector<GrowDesc> gd(ng);
    int np_max = 0;
    for (int k = 0; k < ng; ++k) {
      const Model* M = ms[grow[k]];
      const FitLayout& f = lay[k];
      char* p = gb + base[k];
      GrowDesc& G = gd[k];
      G.n = M->n;
      G.d = M->d;
      G.np_old = M->npad;
      G.np_new = (int)round_up(M->npad + 1, NB);
      np_max = std::max(np_max, G.np_new);
      G.X = M->X64;
      G.il = M->il64;
      G.y = M->y64;
      G.L = M->L;
      G.Linv = M->Linv;
      G.K = M->K;
      G.stats = M->stats;
      G.info = M->info;
      G.X2 = (double*)(p + f.oX);
      G.il2 = (double*)(p + f.oil);
      G.y2 = (double*)(p + f.oy);
      G.L2 = (double*)(p + f.oL);
      G.Linv2 = (double*)(p + f.oLi);
      G.K2 = (double*)(p + f.oK);
      G.stats2 = (double*)(gb + ostat + k * STATUS_SLOT);
      G.info2 = (int*)(gb + ostat + k * STATUS_SLOT + S_COUNT * sizeof(double));
    }
    {
      const gpbo_status st = ensure_desc(c, ng * sizeof(GrowDesc));
      if (st != GPBO_OK) return st;
    }
    HIP_TRY(c, hipMemcpyAsync(c->desc_buf, gd.data(), ng * sizeof(GrowDesc), hipMemcpyHostToDevice,
                              c->stream));
    launch_grow((const GrowDesc*)c->desc_buf, ng, np_max, c->stream);
    HIP_TRY(c, hipGetLastError());
    for (int k = 0; k < ng; ++k) {
      Model* M = ms[grow[k]];
      const FitLayout& f = lay[k];
      char* p = gb + base[k];
      {
        const gpbo_status st = wait_before_release(c, M);
        if (st != GPBO_OK) return st;
      }
      M->npad = gd[k].np_new;
      M->X64 = gd[k].X2;
      M->y64 = gd[k].y2;
      M->il64 = gd[k].il2;
      M->L = gd[k].L2;
      M->Linv = gd[k].Linv2;
      M->K = gd[k].K2;
      M->Dinv = (double*)(p + f.oD);
      M->yt = (double*)(p + f.oyt);
      M->alpha = (double*)(p + f.oa);
      M->work = (double*)(p + f.ow);
      M->L32 = M->refine ? (float*)(p + f.o32) : nullptr;
      M->stats = gd[k].stats2;
      M->info = gd[k].info2;
      M->blk_fit = std::shared_ptr<void>(grp, p);
      M->alloc_stream = c->stream;
    }
  }
  // Descriptors of the models as they are (float64 products, no
  // refinement), then of the extended models.
  std::vector<FitDesc> hd(2 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    Model* M = ms[b];
    FitDesc o = make_fit_desc(M, M->X64, M->il64, M->y64, M->normalize, 0);
    o.xnew = x_new + (int64_t)b * ldx;
    o.ynew = y_new + b;
    hd[b] = o;
    M->n += 1;
    FitDesc nw = make_fit_desc(M, M->X64, M->il64, M->y64, M->normalize, M->refine);
    nw.append = 1;
    hd[B + b] = nw;
  }
  {
    const gpbo_status st = ensure_desc(c, hd.size() * sizeof(FitDesc));
    if (st != GPBO_OK) return st;
  }
  const FitDesc* dd = (const FitDesc*)c->desc_buf;
  HIP_TRY(c, hipMemcpyAsync(c->desc_buf, hd.data(), hd.size() * sizeof(FitDesc),
                            hipMemcpyHostToDevice, c->stream));
  {
    const gpbo_status st = run_append(c, hd.data(), dd, B, c->stream);
    if (st != GPBO_OK) return st;
  }
  // The statistics of the extended models, read when a status is asked for.
  std::shared_ptr<void> sreg = dshared(c, (size_t)B * STATUS_SLOT);
  if (!sreg) return fail(c, GPBO_E_OOM, "status allocation failed");
  launch_status_copy(dd + B, B, (unsigned char*)sreg.get(), (int)STATUS_SLOT, c->stream);
  HIP_TRY(c, hipGetLastError());
  auto gs = std::make_shared<Model::GroupStatus>();
  gs->dev = (const unsigned char*)sreg.get();
  gs->nb = B;
  gs->ctx = c;
  gs->hold = sreg;
  size_t got = 0;
  gs->pinned = pinned_acquire(c, (size_t)B * STATUS_SLOT, &got);
  if (gs->pinned) {
    gs->pinned_bytes = got;
    HIP_TRY(c, hipMemcpyAsync(gs->pinned, gs->dev, (size_t)B * STATUS_SLOT, hipMemcpyDeviceToHost,
                              c->stream));
    gs->ev = timing_event(c);
    if (gs->ev) HIP_TRY(c, hipEventRecord(gs->ev, c->stream));
  }
  for (int b = 0; b < B; ++b) {
    Model* M = ms[b];
    // the score operands describe the old observations: rebuilt on next use
    if (M->blk_obs || M->blk_score[0] || M->blk_score[1] || M->blk_score[2]) {
      const gpbo_status st = wait_before_release(c, M);
      if (st != GPBO_OK) return st;
      M->blk_obs.reset();
      for (int i = 0; i < 3; ++i) M->blk_score[i].reset();
    }
    note_stream(M, c->stream);
    M->pending = true;
    M->gstat = gs;
    M->gslot = b;
  }
  return GPBO_OK;
}

// GPBO_DEBUG: reject candidate pools that hold NaN or infinity
// (synchronises).  flag: a device int of scratch.
static gpbo_status debug_check_pool(Ctx* c, const void* Xc, int64_t count, bool dbl, int* flag,
                                    int which) {
  launch_check_finite(Xc, count, dbl ? 1 : 0, flag, c->stream);
  int h = 0;
  HIP_TRY(c, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h) {
    if (which >= 0)
      return fail(c, GPBO_E_NONFINITE, "candidate pool %d holds a non-finite value", which);
    return fail(c, GPBO_E_NONFINITE, "the candidate pool holds a non-finite value");
  }
  return GPBO_OK;
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
  note_stream(M, s);
  // argmax / ei_max in host memory: the reduction writes device scratch,
  // copied out after a synchronisation
  const bool host_am = argmax && !device_writable(argmax);
  const bool host_em = ei_max && !device_writable(ei_max);
  const bool host_out = host_am || host_em;
  if (m == 0) {  // argmax -1, EI maximum -inf
    if (!argmax && !ei_max) return GPBO_OK;
    gpbo_status st = ensure_red(c, 256);
    if (st != GPBO_OK) return st;
    int64_t* am0 = host_am ? (int64_t*)c->red : argmax;
    double* em0 = host_em ? (double*)((char*)c->red + 8) : ei_max;
    launch_argmax_final(nullptr, nullptr, 0, am0, em0, s);
    HIP_TRY(c, hipGetLastError());
    if (host_out) {
      if (host_am) HIP_TRY(c, hipMemcpyAsync(argmax, am0, 8, hipMemcpyDeviceToHost, s));
      if (host_em) HIP_TRY(c, hipMemcpyAsync(ei_max, em0, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(c, hipStreamSynchronize(s));
    }
    return GPBO_OK;
  }
  // Path: the chunked path for float32 once n is large (the fused kernel's
  // LDS tile then holds too few candidates to amortise the inverse factor).
  const int tm = score_tile_m(prec, M->n, M->d);
  int path = c->score_path;
  if (path == GPBO_PATH_AUTO)
    path = prec == GPBO_FP32 && (tm == 0 || M->n > LARGE_N_MIN) ? GPBO_PATH_LARGE : GPBO_PATH_FUSED;
  if (path == GPBO_PATH_LARGE && prec != GPBO_FP32)
    return fail(c, GPBO_E_UNSUPPORTED, "the large-n scoring path is float32 only");
  if (path == GPBO_PATH_FUSED && tm == 0)
    return fail(c, GPBO_E_UNSUPPORTED, "n=%d is too large for the fused scoring kernel at this precision",
                M->n);
  const bool large = path == GPBO_PATH_LARGE;
  // Escalation of the fused float32 path to float64 arithmetic on an
  // ill-conditioned K: decided here when the fit's statistics are known,
  // else on the device (both kernels queued, one of them idles).
  const int tm64 = prec == GPBO_FP32 && !large ? score_tile_m64(M->n, M->d) : 0;
  int esc = 0;  // 0: float32 only; 1: float64 only; 2: decided on the device
  if (tm64 > 0) esc = M->pending ? 2 : (escalate_fp64(M->host_stats[S_KINV]) ? 1 : 0);
  {
    Model* one[1] = {M};
    if (esc != 1) ensure_score_operands(c, one, 1, prec, s);
    if (esc != 0) ensure_score_operands(c, one, 1, GPBO_FP64, s);
  }
  if (!M->blk_obs || (esc != 1 && !M->blk_score[prec]) || (esc != 0 && !M->blk_score[GPBO_FP64]))
    return fail(c, GPBO_E_OOM, "device allocation of the score operands failed (n=%d)", M->n);
  const int npj = M->pk_npj[esc == 1 ? GPBO_FP64 : prec];
  const int64_t tiles32 = large ? large_partials(npj, m) : (esc == 1 ? 0 : ceil_div(m, tm));
  const int64_t tiles64 = esc != 0 ? ceil_div(m, tm64) : 0;
  const int64_t tiles = std::max(tiles32, tiles64);
  const size_t part_bytes = round_up((size_t)tiles * 16, 256);
  const size_t ws_bytes = large ? large_scratch_bytes(M->n, npj, m) : 0;
  const size_t tail_bytes = 256;  // host-output staging and the debug flag
  gpbo_status st = ensure_red(c, part_bytes + ws_bytes + tail_bytes);
  if (st != GPBO_OK) return st;
  char* tail = (char*)c->red + part_bytes + ws_bytes;
  int64_t* am_dev = host_am ? (int64_t*)tail : argmax;
  double* em_dev = host_em ? (double*)(tail + 8) : ei_max;
  if (c->debug && m > 0) {
    st = debug_check_pool(c, Xc, m * M->d, prec == GPBO_FP64, (int*)(tail + 16), -1);
    if (st != GPBO_OK) return st;
  }
  auto finish_host = [&]() -> gpbo_status {
    if (!host_out) return GPBO_OK;
    if (host_am) HIP_TRY(c, hipMemcpyAsync(argmax, am_dev, 8, hipMemcpyDeviceToHost, s));
    if (host_em) HIP_TRY(c, hipMemcpyAsync(ei_max, em_dev, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return GPBO_OK;
  };
  double* pv = nullptr;
  int64_t* pi = nullptr;
  if (am_dev || em_dev) {
    pv = (double*)c->red;
    pi = (int64_t*)((double*)c->red + tiles);
  }
  auto args = [&](int p, int t) {
    ScoreArgs j = make_score_args(M, p, t);
    j.m = m;
    j.Xc = Xc;
    j.mu = mu;
    j.sigma = sigma;
    j.ei = ei;
    j.part_v = pv;
    j.part_i = pi;
    return j;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing && !large) {
    e0 = timing_event(c);
    e1 = timing_event(c);
    HIP_TRY(c, hipEventRecord(e0, s));
  }
  if (large) {
    launch_score_large(args(prec, 0), (char*)c->red + part_bytes, s, [&](int w) {
      if (!c->timing) return;
      if (w == 0) {
        e0 = timing_event(c);
        e1 = timing_event(c);
        (void)hipEventRecord(e0, s);
      } else {
        (void)hipEventRecord(e1, s);
        c->ev_pending.emplace_back(e0, e1);
      }
    });
  } else {
    if (esc == 0) launch_score(args(prec, tm), prec, tm, s);
    else if (esc == 1) launch_score(args(GPBO_FP64, tm64), P_F64IO32, tm64, s);
    else launch_score_escalated(args(prec, tm), tm, args(GPBO_FP64, tm64), tm64, s);
    if (c->timing) {
      HIP_TRY(c, hipEventRecord(e1, s));
      c->ev_pending.emplace_back(e0, e1);
    }
  }
  if (pv) {
    if (esc == 2) launch_argmax_gated(pv, pi, tiles32, tiles64, M->stats, am_dev, em_dev, s);
    else launch_argmax_final(pv, pi, esc == 1 ? tiles64 : tiles32, am_dev, em_dev, s);
  }
  HIP_TRY(c, hipGetLastError());
  return finish_host();
}

gpbo_status gpbo_score_prepare_batched(gpbo_ctx c, int32_t B, const gpbo_model* models,
                                       gpbo_precision prec) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && !models)) return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (prec != GPBO_FP64 && prec != GPBO_FP32 && prec != GPBO_BF16)
    return fail(c, GPBO_E_INVALID_ARG, "unknown precision %d", (int)prec);
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  for (int b = 0; b < B; ++b)
    if (!models[b]) return fail(c, GPBO_E_INVALID_ARG, "model %d is NULL", b);
  for (int b = 0; b < B; ++b) note_stream(models[b], s);
  std::vector<Model*> mp(models, models + B);
  ensure_score_operands(c, mp.data(), B, prec, s);
  for (int b = 0; b < B; ++b)
    if (!models[b]->blk_obs || !models[b]->blk_score[prec])
      return fail(c, GPBO_E_OOM, "device allocation of the score operands failed (problem %d)", b);
  return GPBO_OK;
}

gpbo_status gpbo_score_batched(gpbo_ctx c, int32_t B, const gpbo_model* models, const int64_t* m,
                               const void* const* Xc, gpbo_precision prec, void* const* mu,
                               void* const* sigma, void* const* ei, int64_t* argmax,
                               double* ei_max) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !m || !Xc)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (prec != GPBO_FP64 && prec != GPBO_FP32 && prec != GPBO_BF16)
    return fail(c, GPBO_E_INVALID_ARG, "unknown precision %d", (int)prec);
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  for (int b = 0; b < B; ++b) {
    if (!models[b]) return fail(c, GPBO_E_INVALID_ARG, "model %d is NULL", b);
    if (m[b] < 0 || (m[b] > 0 && !Xc[b])) return fail(c, GPBO_E_INVALID_ARG, "pool %d is invalid", b);
  }
  for (int b = 0; b < B; ++b) note_stream(models[b], s);
  const bool host_am = argmax && !device_writable(argmax);
  const bool host_em = ei_max && !device_writable(ei_max);
  // Tile size: every candidate tile size whose LDS footprint fits the largest
  // problem is a candidate; the autotuner times them on this batch shape once.
  int nmax = 0, dmax = 0;
  for (int b = 0; b < B; ++b) {
    nmax = std::max(nmax, models[b]->n);
    dmax = std::max(dmax, models[b]->d);
  }
  std::vector<int> cands;
  // (the batched kernel also holds a 2 KB table of problem starts in LDS)
  for (int tm : {64, 32, 16})
    if (score_smem(prec, nmax, dmax, tm) + 4096 <= 160 * 1024) cands.push_back(tm);
  if (cands.empty())
    return fail(c, GPBO_E_UNSUPPORTED, "n=%d is too large for the batched scoring kernel", nmax);
  // The float32 path escalates ill-conditioned problems to float64
  // arithmetic (a second persistent launch over those problems, chosen on
  // the device from each fit's conditioning statistic): its tile size is the
  // largest with two workgroups per CU, else one.
  int tm64 = 0, per_cu64 = 0;
  size_t smem64 = 0;
  if (prec == GPBO_FP32) {
    for (int pc : {2, 1}) {
      for (int tm : {32, 16})
        if (pc * (score_smem(GPBO_FP64, nmax, dmax, tm) + 4096) <= 160 * 1024) {
          tm64 = tm;
          per_cu64 = pc;
          break;
        }
      if (tm64) break;
    }
  }
  const bool esc = tm64 > 0;
  {
    std::vector<Model*> mp(models, models + B);
    ensure_score_operands(c, mp.data(), B, prec, s);
    if (esc) ensure_score_operands(c, mp.data(), B, GPBO_FP64, s);
  }
  for (int b = 0; b < B; ++b)
    if (!models[b]->blk_obs || !models[b]->blk_score[prec] ||
        (esc && !models[b]->blk_score[GPBO_FP64]))
      return fail(c, GPBO_E_OOM, "device allocation of the score operands failed (problem %d)", b);
  // problems in decreasing n: the costliest tiles are dispatched first
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return models[a]->n > models[b]->n; });
  // argmax partials: room for the smallest tile (16 candidates) of every problem
  std::vector<int64_t> poff(B + 1, 0);
  for (int k = 0; k < B; ++k) poff[k + 1] = poff[k] + ceil_div(m[order[k]], 16);
  const int64_t max_tiles = poff[B];
  const size_t desc_bytes = round_up(B * sizeof(ScoreArgs), 256);
  const size_t plan_bytes = round_up(batch_plan_bytes(B), 256);
  const size_t out_bytes = round_up((size_t)B * 16 + 16, 256);  // host-output staging, debug flag
  const size_t need = 2 * desc_bytes + 256 + plan_bytes + out_bytes + (size_t)max_tiles * 16;
  if (c->batch_buf_bytes < need) {
    HIP_TRY(c, hipStreamSynchronize(s));
    if (c->batch_buf) dfree(c, c->batch_buf);
    c->batch_buf = dmalloc(c, need);
    c->batch_buf_bytes = c->batch_buf ? need : 0;
    if (!c->batch_buf) return fail(c, GPBO_E_OOM, "batch buffer allocation failed");
  }
  unsigned char* base = (unsigned char*)c->batch_buf;
  ScoreArgs* dd = (ScoreArgs*)base;
  ScoreArgs* dd64 = (ScoreArgs*)(base + desc_bytes);
  void* plan = base + 2 * desc_bytes + 256;
  unsigned char* outs = base + 2 * desc_bytes + 256 + plan_bytes;
  double* pv = (double*)(outs + out_bytes);
  int64_t* pi = (int64_t*)(pv + max_tiles);
  int64_t* am_dev = host_am ? (int64_t*)outs : argmax;
  double* em_dev = host_em ? (double*)(outs + 8 * (size_t)B) : ei_max;
  if (c->debug)
    for (int b = 0; b < B; ++b)
      if (m[b] > 0) {
        const gpbo_status st = debug_check_pool(c, Xc[b], m[b] * models[b]->d, prec == GPBO_FP64,
                                                (int*)(outs + 16 * (size_t)B), b);
        if (st != GPBO_OK) return st;
      }
  auto build = [&](int tm, std::vector<ScoreArgs>& h, std::vector<ScoreArgs>& h64, size_t& smem) {
    h.clear();
    h64.clear();
    smem = 0;
    for (int k = 0; k < B; ++k) {
      const int b = order[k];
      ScoreArgs a = make_score_args(models[b], prec, tm);
      a.m = m[b];
      a.Xc = Xc[b];
      a.mu = mu ? mu[b] : nullptr;
      a.sigma = sigma ? sigma[b] : nullptr;
      a.ei = ei ? ei[b] : nullptr;
      a.part_v = pv + poff[k];
      a.part_i = pi + poff[k];
      a.slot = b;
      // the batched kernel lays its tile areas out for the largest n and d
      smem = std::max(smem, score_smem(prec, nmax, dmax, tm));
      h.push_back(a);
      if (esc) {
        ScoreArgs a64 = make_score_args(models[b], GPBO_FP64, tm64);
        a64.m = a.m;
        a64.Xc = a.Xc;
        a64.mu = a.mu;
        a64.sigma = a.sigma;
        a64.ei = a.ei;
        a64.part_v = a.part_v;
        a64.part_i = a.part_i;
        a64.slot = b;
        smem64 = std::max(smem64, score_smem(GPBO_FP64, nmax, dmax, tm64));
        h64.push_back(a64);
      }
    }
  };
  const int per_cu = 2;  // LDS-limited residency of the scoring workgroup
  BatchLaunch L;
  L.dd = dd;
  L.dd64 = esc ? dd64 : nullptr;
  L.B = B;
  L.prec = prec;
  L.tm64 = esc ? tm64 : 16;
  L.grid = c->num_cu * per_cu;
  L.grid64 = c->num_cu * std::max(per_cu64, 1);
  L.per_cu = per_cu;
  L.per_cu64 = std::max(per_cu64, 1);
  L.nmax = nmax;
  L.dmax = dmax;
  L.plan = plan;
  L.argmax = am_dev;
  L.ei_max = em_dev;
  {
    int64_t max_items = 0;
    for (int b = 0; b < B; ++b) max_items += ceil_div(m[b], 16);
    if (max_items + std::max(L.grid, L.grid64) >= (int64_t)INT_MAX)
      return fail(c, GPBO_E_UNSUPPORTED, "too many candidate tiles in one batch (%lld)",
                  (long long)max_items);
  }
  char kbuf[160];
  snprintf(kbuf, sizeof kbuf, "batched:gfx950:hip%d:p%d:B%d:n%d:d%d", HIP_VERSION, (int)prec, B,
           (int)round_up(nmax, 64), dmax);
  std::vector<ScoreArgs> hh, hh64;  // sources of the descriptor copies of the timing runs
  bool tuned = false;
  const int tm = autotune_pick(c, kbuf, cands, [&](int cand) {
    size_t sm;
    (void)hipStreamSynchronize(s);  // hh is reused by the next run
    build(cand, hh, hh64, sm);
    (void)hipMemcpyAsync(dd, hh.data(), hh.size() * sizeof(ScoreArgs), hipMemcpyHostToDevice, s);
    if (esc)
      (void)hipMemcpyAsync(dd64, hh64.data(), hh64.size() * sizeof(ScoreArgs),
                           hipMemcpyHostToDevice, s);
    BatchLaunch T = L;
    T.tm = cand;
    T.smem = sm;
    T.smem64 = smem64;
    launch_score_batched(T, s);
    tuned = true;
  });
  if (tuned) HIP_TRY(c, hipStreamSynchronize(s));
  // The descriptors go to device memory ahead of the launch, in stream order
  // (a pageable-memory copy has consumed the host vector when it returns).
  // The launch sequence reads everything problem-specific from them, so its
  // graph depends only on the batch shape below: calls with new models or
  // pools of the same shape (the next iteration of a search) replay it.
  std::vector<ScoreArgs> h, h64;
  size_t smem = 0;
  build(tm, h, h64, smem);
  L.tm = tm;
  L.smem = smem;
  L.smem64 = smem64;
  HIP_TRY(c, hipMemcpyAsync(dd, h.data(), h.size() * sizeof(ScoreArgs), hipMemcpyHostToDevice, s));
  if (esc)
    HIP_TRY(c, hipMemcpyAsync(dd64, h64.data(), h64.size() * sizeof(ScoreArgs),
                              hipMemcpyHostToDevice, s));
  auto finish_host = [&]() -> gpbo_status {
    if (!host_am && !host_em) return GPBO_OK;
    if (host_am) HIP_TRY(c, hipMemcpyAsync(argmax, am_dev, 8 * (size_t)B, hipMemcpyDeviceToHost, s));
    if (host_em) HIP_TRY(c, hipMemcpyAsync(ei_max, em_dev, 8 * (size_t)B, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return GPBO_OK;
  };
  const std::vector<uint64_t> key = {(uint64_t)B, (uint64_t)prec, (uint64_t)tm, (uint64_t)tm64,
                                     (uint64_t)max_tiles, (uint64_t)smem, (uint64_t)smem64,
                                     (uint64_t)L.grid, (uint64_t)L.grid64,
                                     (uint64_t)(uintptr_t)am_dev, (uint64_t)(uintptr_t)em_dev,
                                     (uint64_t)(uintptr_t)s, (uint64_t)(uintptr_t)base};
  // With kernel timing on, every call launches eagerly so that events can
  // bracket the scoring kernels alone.
  if (!c->timing)
    for (auto& kv : c->batch_graphs)
      if (kv.first == key) {
        HIP_TRY(c, hipGraphLaunch(kv.second, s));
        return finish_host();
      }
  // an eager launch (it also sets the kernels' LDS limits), then the capture
  hipEvent_t e0 = nullptr;
  const std::function<void(int)> mark = [&](int w) {
    if (w == 0) {
      e0 = timing_event(c);
      (void)hipEventRecord(e0, s);
    } else {
      hipEvent_t e1 = timing_event(c);
      (void)hipEventRecord(e1, s);
      c->ev_pending.emplace_back(e0, e1);
    }
  };
  launch_score_batched(L, s, c->timing ? &mark : nullptr);
  HIP_TRY(c, hipGetLastError());
  if (c->timing || s == nullptr || c->no_graph) return finish_host();
  constexpr size_t kMaxGraphs = 8;
  if (c->batch_graphs.size() >= kMaxGraphs) {
    // the oldest goes once every stream it may have been launched on has run it
    HIP_TRY(c, hipDeviceSynchronize());
    (void)hipGraphExecDestroy(c->batch_graphs.front().second);
    c->batch_graphs.erase(c->batch_graphs.begin());
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  launch_score_batched(L, s);
  HIP_TRY(c, hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e == hipSuccess) {
    c->batch_graphs.emplace_back(key, exec);
  }
  return finish_host();
}

gpbo_status gpbo_topk(gpbo_ctx c, int64_t m, const float* v, int64_t k, int64_t* idx) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (m < 0 || k < 0 || (m > 0 && !v) || (k > 0 && !idx))
    return fail(c, GPBO_E_INVALID_ARG, "invalid top-k arguments");
  if (k > m) return fail(c, GPBO_E_INVALID_ARG, "k (%lld) exceeds m (%lld)", (long long)k, (long long)m);
  if (k > topk_max_k()) return fail(c, GPBO_E_UNSUPPORTED, "k > %d is not supported", topk_max_k());
  if (m > 0xffffffffLL) return fail(c, GPBO_E_UNSUPPORTED, "m >= 2^32 is not supported");
  if (k == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  void* scratch = dmalloc(c, topk_scratch_bytes(m, k));
  if (!scratch) return fail(c, GPBO_E_OOM, "top-k scratch allocation failed");
  launch_topk_into(m, v, k, idx, scratch, c->stream);
  HIP_TRY(c, hipGetLastError());
  dfree(c, scratch);  // stream-ordered with the torch allocator; hipFree waits otherwise
  return GPBO_OK;
}

gpbo_status gpbo_topk_set(gpbo_ctx c, int64_t m, const float* v, int64_t k, int64_t* idx) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (m < 0 || k < 0 || (m > 0 && !v) || (k > 0 && !idx))
    return fail(c, GPBO_E_INVALID_ARG, "invalid top-k arguments");
  if (k > m) return fail(c, GPBO_E_INVALID_ARG, "k (%lld) exceeds m (%lld)", (long long)k, (long long)m);
  if (m > 0xffffffffLL) return fail(c, GPBO_E_UNSUPPORTED, "m >= 2^32 is not supported");
  if (k == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  void* ws = dmalloc(c, topk_set_scratch_bytes(m));
  if (!ws) return fail(c, GPBO_E_OOM, "top-k scratch allocation failed");
  launch_topk_set_into(m, v, k, idx, ws, c->stream);
  HIP_TRY(c, hipGetLastError());
  dfree(c, ws);  // stream-ordered with the torch allocator; hipFree waits otherwise
  return GPBO_OK;
}

gpbo_status gpbo_score_bound(gpbo_ctx c, gpbo_model M, int64_t m, const float* Xc, float* mu,
                             float* sigma_ub, float* ei_ub) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!M) return fail(c, GPBO_E_INVALID_ARG, "model is NULL");
  if (m < 0 || (m > 0 && !Xc)) return fail(c, GPBO_E_INVALID_ARG, "invalid candidate pool");
  if (m == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  note_stream(M, s);
  {
    Model* one[1] = {M};
    ensure_score_operands(c, one, 1, GPBO_FP32, s);
  }
  if (!M->blk_obs || !M->blk_score[GPBO_FP32])
    return fail(c, GPBO_E_OOM, "device allocation of the score operands failed (n=%d)", M->n);
  launch_score_bound(M, m, Xc, mu, sigma_ub, ei_ub, s);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_score_subset(gpbo_ctx c, gpbo_model M, int64_t m, const float* Xc, int64_t k1,
                              const int64_t* idx, int64_t k2, int64_t* next, double* ei_max,
                              int32_t* certified) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!M) return fail(c, GPBO_E_INVALID_ARG, "model is NULL");
  if (m <= 0 || !Xc || k1 <= 0 || k1 > m || !idx || k2 <= 0 || !next)
    return fail(c, GPBO_E_INVALID_ARG, "invalid subset arguments");
  if (k2 > k1) k2 = k1;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  note_stream(M, s);
  const int d = M->d;
  const bool all = k2 == k1;  // every candidate of the subset scored exactly
  Carve cv;
  const size_t o_rows1 = cv.take((size_t)k1 * d * sizeof(float));
  const size_t o_bound = cv.take((size_t)k1 * sizeof(float));
  const size_t o_pos = cv.take((size_t)k2 * sizeof(int64_t));
  const size_t o_idx2 = cv.take((size_t)k2 * sizeof(int64_t));
  const size_t o_rows2 = cv.take((size_t)k2 * d * sizeof(float));
  const size_t o_res = cv.take(64);
  const size_t o_ws = cv.take(topk_set_scratch_bytes(k1));
  char* b = (char*)dmalloc(c, cv.bytes);
  if (!b) return fail(c, GPBO_E_OOM, "subset scratch allocation failed");
  float* rows1 = (float*)(b + o_rows1);
  float* bound = (float*)(b + o_bound);
  int64_t* pos = (int64_t*)(b + o_pos);
  int64_t* idx2 = (int64_t*)(b + o_idx2);
  float* rows2 = (float*)(b + o_rows2);
  int64_t* am = (int64_t*)(b + o_res);
  double* em = (double*)(b + o_res + 8);
  int64_t* next_d = (int64_t*)(b + o_res + 16);
  double* emax_d = (double*)(b + o_res + 24);
  int* cert_d = (int*)(b + o_res + 32);
  if (all) {
    // no narrowing: the subset itself is scored exactly, in the given order
    HIP_TRY(c, hipMemcpyAsync(idx2, idx, (size_t)k2 * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  } else {
    // the k2 largest EI bounds among the subset (as a set; the selection's
    // threshold, the k2-th largest bound, certifies: no unscored bound is
    // above it)
    launch_gather_rows(k1, idx, d, Xc, rows1, s);
    {
      Model* one[1] = {M};
      ensure_score_operands(c, one, 1, GPBO_FP32, s);
    }
    if (!M->blk_obs || !M->blk_score[GPBO_FP32]) {
      dfree(c, b);
      return fail(c, GPBO_E_OOM, "device allocation of the score operands failed (n=%d)", M->n);
    }
    launch_score_bound(M, k1, rows1, nullptr, nullptr, bound, s);
    launch_topk_set_into(k1, bound, k2, pos, b + o_ws, s);
    launch_compose_idx(k2, idx, pos, idx2, s);
  }
  launch_gather_rows(k2, idx2, d, Xc, rows2, s);
  gpbo_status st = gpbo_score(c, M, k2, rows2, GPBO_FP32, nullptr, nullptr, nullptr, am, em);
  if (st != GPBO_OK) {
    dfree(c, b);
    return st;
  }
  // float32 errors of the exact EI and of the bound: 2e-4 of the prior
  // standard deviation s_y sqrt(sf2) (s_y is read on the device)
  launch_subset_finish(am, em, idx2, all ? nullptr : topk_set_threshold(b + o_ws),
                       2e-4 * std::sqrt(M->sf2), M->stats, next_d, emax_d, cert_d, s);
  HIP_TRY(c, hipGetLastError());
  if (device_writable(next)) {
    HIP_TRY(c, hipMemcpyAsync(next, next_d, 8, hipMemcpyDeviceToDevice, s));
  } else {
    HIP_TRY(c, hipMemcpyAsync(next, next_d, 8, hipMemcpyDeviceToHost, s));
  }
  if (ei_max)
    HIP_TRY(c, hipMemcpyAsync(ei_max, emax_d, 8,
                              device_writable(ei_max) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              s));
  if (certified)
    HIP_TRY(c, hipMemcpyAsync(certified, cert_d, 4,
                              device_writable(certified) ? hipMemcpyDeviceToDevice
                                                         : hipMemcpyDeviceToHost,
                              s));
  const bool host = !device_writable(next) || (ei_max && !device_writable(ei_max)) ||
                    (certified && !device_writable(certified));
  dfree(c, b);  // stream-ordered with the torch allocator; hipFree waits otherwise
  if (host) HIP_TRY(c, hipStreamSynchronize(s));
  return GPBO_OK;
}

gpbo_status gpbo_topk_noalloc(gpbo_ctx c, int64_t m, const float* v, int64_t k, int64_t* idx) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (m < 0 || k < 0 || (m > 0 && !v) || (k > 0 && !idx))
    return fail(c, GPBO_E_INVALID_ARG, "invalid top-k arguments");
  if (k > m) return fail(c, GPBO_E_INVALID_ARG, "k (%lld) exceeds m (%lld)", (long long)k, (long long)m);
  if (k > topk_max_k()) return fail(c, GPBO_E_UNSUPPORTED, "k > %d is not supported", topk_max_k());
  if (m > 0xffffffffLL) return fail(c, GPBO_E_UNSUPPORTED, "m >= 2^32 is not supported");
  const size_t need = topk_scratch_bytes(m, k);
  if (need > topk_noalloc_bytes())
    return fail(c, GPBO_E_UNSUPPORTED, "top-k needs %zu bytes of scratch; the static array holds %zu",
                need, topk_noalloc_bytes());
  if (k == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  void* ws = topk_noalloc_scratch(c->device);
  if (!ws) return fail(c, GPBO_E_HIP, "static top-k scratch not resolved on device %d", c->device);
  launch_topk_into(m, v, k, idx, ws, c->stream);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_gather_rows(gpbo_ctx c, int64_t k, const int64_t* idx, int32_t d, const float* Xc,
                             float* out) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (k < 0 || d <= 0 || (k > 0 && (!idx || !Xc || !out)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid gather arguments");
  if (k == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  launch_gather_rows(k, idx, d, Xc, out, c->stream);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_next_batched(gpbo_ctx c, int32_t B, const gpbo_model* models, const int64_t* m,
                              const void* const* Xc, gpbo_precision prec, const int64_t* argmax,
                              int32_t ldx, double* x_next) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !m || !Xc || !argmax || !x_next)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (prec != GPBO_FP64 && prec != GPBO_FP32 && prec != GPBO_BF16)
    return fail(c, GPBO_E_INVALID_ARG, "unknown precision %d", (int)prec);
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  if (!device_writable(argmax) || !device_writable(x_next))
    return fail(c, GPBO_E_INVALID_ARG, "argmax and x_next must be device memory");
  std::vector<int> d(B);
  for (int b = 0; b < B; ++b) {
    if (!models[b]) return fail(c, GPBO_E_INVALID_ARG, "model %d is NULL", b);
    if (m[b] < 0 || (m[b] > 0 && !Xc[b])) return fail(c, GPBO_E_INVALID_ARG, "pool %d is invalid", b);
    d[b] = models[b]->d;
    if (ldx < d[b]) return fail(c, GPBO_E_INVALID_ARG, "ldx %d is smaller than model %d's d", ldx, b);
  }
  launch_next_rows(B, Xc, m, d.data(), prec == GPBO_FP64 ? 1 : 0, argmax, ldx, x_next, c->stream);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

int64_t gpbo_mlp_nparams(int32_t d_in, int32_t hidden) {
  return (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + hidden + 1;
}

struct gpbo_mlp_s {
  Ctx* ctx;
  MlpState* st;
  int E, D, H;
  // Workspace of the pass over a pool (member outputs, scores, top-k
  // scratch), kept between calls on the network's own context so that a
  // step allocates nothing; grown when a larger pool comes.
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

gpbo_status gpbo_mlp_create(gpbo_ctx c, int32_t members, int32_t d_in, int32_t hidden,
                            const float* init, gpbo_mlp* out) {
  if (out) *out = nullptr;
  if (!c) return GPBO_E_INVALID_ARG;
  if (!out || !init) return fail(c, GPBO_E_INVALID_ARG, "init and out are required");
  if (members < 1 || members > 64 || d_in < 1 || d_in > 64)
    return fail(c, GPBO_E_INVALID_ARG, "members must be 1..64 and d_in 1..64");
  if (hidden != 256)
    return fail(c, GPBO_E_UNSUPPORTED, "hidden width %d: this build supports 256", hidden);
  DeviceGuard g(c->device);
  MlpState* st = mlp_create(c, members, d_in, hidden, init, c->stream);
  if (!st) return fail(c, GPBO_E_OOM, "MLP allocation failed");
  HIP_TRY(c, hipGetLastError());
  *out = new gpbo_mlp_s{c, st, members, d_in, hidden};
  c->live_mlps.insert(*out);
  return GPBO_OK;
}

gpbo_status gpbo_mlp_free(gpbo_mlp mlp) {
  if (!mlp) return GPBO_OK;
  DeviceGuard g(mlp->ctx->device);
  // the network's buffers may be in use on any stream the context has
  // queued on since they were allocated: wait for the device first
  (void)hipDeviceSynchronize();
  mlp->ctx->live_mlps.erase(mlp);
  if (mlp->ws) dfree(mlp->ctx, mlp->ws);
  mlp_destroy(mlp->st);
  delete mlp;
  return GPBO_OK;
}

gpbo_status gpbo_mlp_params(gpbo_ctx c, gpbo_mlp mlp, float* out) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!mlp || !out) return fail(c, GPBO_E_INVALID_ARG, "mlp and out are required");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipMemcpyAsync(out, mlp_master(mlp->st),
                            (size_t)mlp->E * mlp_nparams(mlp->st) * sizeof(float),
                            hipMemcpyDeviceToDevice, c->stream));
  return GPBO_OK;
}

// Network forward on the context's stream, bracketed by timing events when
// kernel timing is enabled.
static void timed_mlp_forward(Ctx* c, MlpState* st, int64_t m, const float* Xc, float* out) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    e0 = timing_event(c);
    e1 = timing_event(c);
    (void)hipEventRecord(e0, c->stream);
  }
  mlp_forward(st, m, Xc, out, c->stream);
  if (c->timing) {
    (void)hipEventRecord(e1, c->stream);
    c->ev_pending.emplace_back(e0, e1);
  }
}

static gpbo_status check_train_args(Ctx* c, gpbo_mlp mlp, int32_t n, const float* X,
                                    const float* y) {
  if (!mlp || !X || !y) return fail(c, GPBO_E_INVALID_ARG, "mlp, X and y are required");
  if (n <= 0 || n % 64 != 0)
    return fail(c, GPBO_E_INVALID_ARG, "training sample count must be a positive multiple of 64 (got %d)", n);
  return GPBO_OK;
}

gpbo_status gpbo_mlp_grads(gpbo_ctx c, gpbo_mlp mlp, int32_t n, const float* X, const float* y,
                           float* grad, float* loss) {
  if (!c) return GPBO_E_INVALID_ARG;
  gpbo_status st = check_train_args(c, mlp, n, X, y);
  if (st != GPBO_OK) return st;
  if (!grad || !loss) return fail(c, GPBO_E_INVALID_ARG, "grad and loss are required");
  DeviceGuard g(c->device);
  if (!mlp_grads(mlp->st, n, X, y, grad, loss, c->stream))
    return fail(c, GPBO_E_OOM, "MLP workspace allocation failed");
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_mlp_train(gpbo_ctx c, gpbo_mlp mlp, int32_t n, const float* X, const float* y,
                           int32_t steps, double lr, float* loss_hist) {
  if (!c) return GPBO_E_INVALID_ARG;
  gpbo_status st = check_train_args(c, mlp, n, X, y);
  if (st != GPBO_OK) return st;
  if (steps < 0 || !(lr > 0.0)) return fail(c, GPBO_E_INVALID_ARG, "steps >= 0 and lr > 0 required");
  DeviceGuard g(c->device);
  if (!mlp_train(mlp->st, n, X, y, steps, lr, loss_hist, !c->no_graph, c->stream))
    return fail(c, GPBO_E_HIP, "MLP training launch failed");
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_mlp_train_model(gpbo_ctx c, gpbo_mlp mlp, gpbo_model M, int32_t steps, double lr,
                                 float* loss_hist) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!mlp || !M) return fail(c, GPBO_E_INVALID_ARG, "mlp and model are required");
  if (M->d != mlp->D)
    return fail(c, GPBO_E_INVALID_ARG, "model has d=%d, the network d_in=%d", M->d, mlp->D);
  if (M->n % 64 != 0)
    return fail(c, GPBO_E_INVALID_ARG,
                "training sample count must be a positive multiple of 64 (the model has n=%d)", M->n);
  if (steps < 0 || !(lr > 0.0)) return fail(c, GPBO_E_INVALID_ARG, "steps >= 0 and lr > 0 required");
  DeviceGuard g(c->device);
  if (M->alloc_stream != c->stream) M->alloc_mixed = true;
  if (!mlp_train_model(mlp->st, M, steps, lr, loss_hist, !c->no_graph, c->stream))
    return fail(c, GPBO_E_OOM, "MLP training data or launch failed");
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_mlp_set_occupancy(gpbo_ctx c, gpbo_mlp mlp, int32_t workgroups_per_cu) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!mlp || workgroups_per_cu < 0)
    return fail(c, GPBO_E_INVALID_ARG, "invalid occupancy arguments");
  mlp_set_occupancy(mlp->st, workgroups_per_cu);
  return GPBO_OK;
}

gpbo_status gpbo_mlp_forward(gpbo_ctx c, gpbo_mlp mlp, int64_t m, const float* Xc, float* out) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (!mlp || m < 0 || (m > 0 && (!Xc || !out))) return fail(c, GPBO_E_INVALID_ARG, "invalid forward arguments");
  if (m == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  timed_mlp_forward(c, mlp->st, m, Xc, out);
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

// Shared body of the two prescreen rules: member outputs, per-candidate score
// (EI against f_best, or the negated lower confidence bound), top k.
static gpbo_status prescreen(Ctx* c, gpbo_mlp mlp, int64_t m, const float* Xc, bool lcb,
                             double arg, int64_t k, int64_t* topk_idx, float* score_out) {
  if (!mlp || m < 0 || k < 0 || k > m || (m > 0 && !Xc) || (k > 0 && !topk_idx))
    return fail(c, GPBO_E_INVALID_ARG, "invalid prescreen arguments");
  if (lcb && !(arg >= 0.0)) return fail(c, GPBO_E_INVALID_ARG, "kappa must be >= 0");
  if (m > 0xffffffffLL) return fail(c, GPBO_E_UNSUPPORTED, "m >= 2^32 is not supported");
  if (m == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  // up to the sort's limit the k indices come sorted by score; beyond it, as
  // the same set in ascending index order
  const bool sorted = k <= topk_max_k();
  Carve cv;
  const size_t o_outs = cv.take((size_t)mlp->E * m * sizeof(float));
  const size_t o_sc = score_out ? 0 : cv.take((size_t)m * sizeof(float));
  const size_t o_scr =
      k > 0 ? cv.take(sorted ? topk_scratch_bytes(m, k) : topk_set_scratch_bytes(m)) : 0;
  // on the network's own context the workspace persists (stream order makes
  // the next call's reuse safe); another context allocates for the call
  const bool own = c == mlp->ctx;
  if (own && mlp->ws_bytes < cv.bytes) {
    if (mlp->ws) dfree(c, mlp->ws);
    mlp->ws = dmalloc(c, cv.bytes);
    mlp->ws_bytes = mlp->ws ? cv.bytes : 0;
  }
  char* wsb = own ? (char*)mlp->ws : (char*)dmalloc(c, cv.bytes);
  if (!wsb) return fail(c, GPBO_E_OOM, "prescreen workspace allocation of %zu bytes failed", cv.bytes);
  float* outs = (float*)(wsb + o_outs);
  float* sc = score_out ? score_out : (float*)(wsb + o_sc);
  void* scratch = k > 0 ? (void*)(wsb + o_scr) : nullptr;
  timed_mlp_forward(c, mlp->st, m, Xc, outs);
  if (lcb)
    mlp_ens_lcb(mlp->st, m, outs, arg, sc, s);
  else
    mlp_ens_ei(mlp->st, m, outs, arg, sc, s);
  if (k > 0) {
    if (sorted) launch_topk_into(m, sc, k, topk_idx, scratch, s);
    else launch_topk_set_into(m, sc, k, topk_idx, scratch, s);
  }
  HIP_TRY(c, hipGetLastError());
  if (!own) dfree(c, wsb);
  return GPBO_OK;
}

gpbo_status gpbo_ens_select(gpbo_ctx c, int32_t E, int64_t m, const float* outs, int32_t rule,
                            double arg, int64_t k, int64_t* topk_idx, float* score_out) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (E < 1 || m < 0 || k < 0 || k > m || (m > 0 && !outs) || (k > 0 && !topk_idx) ||
      (rule != GPBO_SELECT_EI && rule != GPBO_SELECT_LCB))
    return fail(c, GPBO_E_INVALID_ARG, "invalid selection arguments");
  if (rule == GPBO_SELECT_LCB && !(arg >= 0.0))
    return fail(c, GPBO_E_INVALID_ARG, "kappa must be >= 0");
  if (m > 0xffffffffLL) return fail(c, GPBO_E_UNSUPPORTED, "m >= 2^32 is not supported");
  if (m == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  hipStream_t s = c->stream;
  const bool sorted = k <= topk_max_k();
  Carve cv;
  const size_t o_sc = score_out ? 0 : cv.take((size_t)m * sizeof(float));
  const size_t o_scr =
      k > 0 ? cv.take(sorted ? topk_scratch_bytes(m, k) : topk_set_scratch_bytes(m)) : 0;
  {
    const gpbo_status st = ensure_red(c, std::max<size_t>(cv.bytes, 256));
    if (st != GPBO_OK) return st;
  }
  char* wsb = (char*)c->red;
  float* sc = score_out ? score_out : (float*)(wsb + o_sc);
  ens_score(E, m, outs, rule == GPBO_SELECT_LCB, arg, sc, s);
  if (k > 0) {
    if (sorted) launch_topk_into(m, sc, k, topk_idx, wsb + o_scr, s);
    else launch_topk_set_into(m, sc, k, topk_idx, wsb + o_scr, s);
  }
  HIP_TRY(c, hipGetLastError());
  return GPBO_OK;
}

gpbo_status gpbo_mlp_prescreen(gpbo_ctx c, gpbo_mlp mlp, int64_t m, const float* Xc, double f_best,
                               int64_t k, int64_t* topk_idx, float* ei_out) {
  if (!c) return GPBO_E_INVALID_ARG;
  return prescreen(c, mlp, m, Xc, false, f_best, k, topk_idx, ei_out);
}

gpbo_status gpbo_mlp_prescreen_lcb(gpbo_ctx c, gpbo_mlp mlp, int64_t m, const float* Xc,
                                   double kappa, int64_t k, int64_t* topk_idx, float* score_out) {
  if (!c) return GPBO_E_INVALID_ARG;
  return prescreen(c, mlp, m, Xc, true, kappa, k, topk_idx, score_out);
}

gpbo_status gpbo_lml_grad_batched(gpbo_ctx c, int32_t B, const gpbo_model* models, int32_t ldg,
                                  double* grad, double* lml) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!models || !grad)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  if (!device_writable(grad) || (lml && !device_writable(lml)))
    return fail(c, GPBO_E_INVALID_ARG, "grad and lml must be device memory");
  std::vector<FitDesc> hd(B);
  for (int b = 0; b < B; ++b) {
    Model* M = models[b];
    if (!M) return fail(c, GPBO_E_INVALID_ARG, "model %d is NULL", b);
    if (M->ctx != c) return fail(c, GPBO_E_INVALID_ARG, "model %d belongs to another context", b);
    if (ldg < M->d + 2)
      return fail(c, GPBO_E_INVALID_ARG, "ldg %d is smaller than model %d's d + 2", ldg, b);
    hd[b] = make_fit_desc(M, M->X64, M->il64, M->y64, M->normalize, M->refine);
  }
  {
    const gpbo_status st = ensure_desc(c, hd.size() * sizeof(FitDesc));
    if (st != GPBO_OK) return st;
  }
  int ldp = 0;
  int64_t ts = 0;
  const size_t nd = lml_grad_part_doubles(hd.data(), B, &ldp, &ts);
  {
    const gpbo_status st = ensure_red(c, nd * sizeof(double));
    if (st != GPBO_OK) return st;
  }
  HIP_TRY(c, hipMemcpyAsync(c->desc_buf, hd.data(), hd.size() * sizeof(FitDesc),
                            hipMemcpyHostToDevice, c->stream));
  launch_lml_grad(hd.data(), (const FitDesc*)c->desc_buf, B, (double*)c->red, ldg, grad, lml,
                  c->stream);
  HIP_TRY(c, hipGetLastError());
  for (int b = 0; b < B; ++b) note_stream(models[b], c->stream);
  return GPBO_OK;
}

gpbo_status gpbo_fit_hyper_batched(gpbo_ctx c, int32_t B, const gpbo_problem* probs,
                                   const gpbo_hyper_opts* o, const double* theta0, const double* lo,
                                   const double* hi, int32_t ldt, double* theta, double* lml,
                                   double* jitter, gpbo_model* out, int32_t* status) {
  if (!c) return GPBO_E_INVALID_ARG;
  if (B < 0 || (B > 0 && (!probs || !o || !theta0 || !lo || !hi || !theta || !lml || !status)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid batch arguments");
  if (o && (o->starts < 1 || o->steps < 0 || !(o->lr > 0.0) || o->retries < 0 ||
            !(o->jitter0 > 0.0)))
    return fail(c, GPBO_E_INVALID_ARG, "invalid optimiser options");
  if (B == 0) return GPBO_OK;
  DeviceGuard g(c->device);
  const int S = o->starts, N = B * S;
  for (int b = 0; b < B; ++b) {
    const gpbo_problem& p = probs[b];
    if (out) out[b] = nullptr;
    if (p.n <= 0 || p.d <= 0 || p.d > 64 || p.n > 65536 || !p.X || !p.y ||
        (p.kernel != GPBO_KERNEL_SE && p.kernel != GPBO_KERNEL_MATERN52))
      return fail(c, GPBO_E_INVALID_ARG, "problem %d is invalid", b);
    if (ldt < p.d + 2) return fail(c, GPBO_E_INVALID_ARG, "ldt %d is smaller than d + 2", ldt);
    for (int j = 0; j < p.d + 2; ++j)
      if (!(lo[(size_t)b * ldt + j] <= hi[(size_t)b * ldt + j]) ||
          !std::isfinite(lo[(size_t)b * ldt + j]) || !std::isfinite(hi[(size_t)b * ldt + j]))
        return fail(c, GPBO_E_INVALID_ARG, "bounds of problem %d are invalid", b);
  }
  // run r = b * S + s: start s of problem b
  std::vector<std::vector<double>> th(N), mo(N), ve(N);
  std::vector<char> alive(N, 1);
  std::vector<double> fin_lml(N, -INFINITY), fin_jit(N, NAN);
  for (int r = 0; r < N; ++r) {
    const int b = r / S, d = probs[b].d;
    th[r].resize(d + 2);
    mo[r].assign(d + 2, 0.0);
    ve[r].assign(d + 2, 0.0);
    for (int j = 0; j < d + 2; ++j) {
      const double v = theta0[((size_t)b * S + (r % S)) * ldt + j];
      th[r][j] = std::min(std::max(v, lo[(size_t)b * ldt + j]), hi[(size_t)b * ldt + j]);
    }
  }
  int ldg = 2;
  for (int b = 0; b < B; ++b) ldg = std::max(ldg, probs[b].d + 2);
  std::shared_ptr<void> gbuf = dshared(c, (size_t)N * (ldg + 1) * sizeof(double));
  if (!gbuf) return fail(c, GPBO_E_OOM, "gradient buffer allocation failed");
  double* g_dev = (double*)gbuf.get();
  double* l_dev = g_dev + (size_t)N * ldg;
  std::vector<double> g_h((size_t)N * ldg), l_h(N);
  // Gradient and LML of the runs in `rs` at their theta, with the jitter
  // policy: a fit that is not positive definite is repeated with
  // sf2 * jitter0 * 10^(k-1) added to the noise, k = 1 .. retries.  Returns
  // per run OK (grad in g_h row r, lml, jitter) or the last failure.
  std::vector<double> jit_r(N, 0.0);
  std::vector<int32_t> st_r(N, GPBO_OK);
  auto evaluate = [&](const std::vector<int>& rs) -> gpbo_status {
    std::vector<int> pend = rs;
    std::vector<Model*> ok_m;
    std::vector<int> ok_r;
    for (int k = 0; k <= o->retries && !pend.empty(); ++k) {
      const int np = (int)pend.size();
      std::vector<gpbo_problem> pp(np);
      std::vector<std::vector<double>> ls(np);
      std::vector<Model*> ms(np);
      std::vector<int32_t> st(np, GPBO_OK);
      for (int q = 0; q < np; ++q) {
        const int r = pend[q], b = r / S, d = probs[b].d;
        ls[q].resize(d);
        for (int j = 0; j < d; ++j) ls[q][j] = std::exp(th[r][j]);
        const double sf2 = std::exp(th[r][d]), sn2 = std::exp(th[r][d + 1]);
        jit_r[r] = k == 0 ? 0.0 : sf2 * o->jitter0 * std::pow(10.0, k - 1);
        pp[q] = probs[b];
        pp[q].lengthscale = ls[q].data();
        pp[q].signal_var = sf2;
        pp[q].noise_var = sn2 + jit_r[r];
        ms[q] = new (std::nothrow) gpbo_model_s();
        if (!ms[q]) st[q] = GPBO_E_OOM;
      }
      const gpbo_status gst = fit_group(c, np, pp.data(), ms.data(), st.data(), true);
      std::vector<int> next;
      for (int q = 0; q < np; ++q) {
        const int r = pend[q];
        gpbo_status s = gst != GPBO_OK && st[q] == GPBO_OK ? gst : (gpbo_status)st[q];
        if (s == GPBO_OK && ms[q]) s = fit_status(c, ms[q], nullptr);
        st_r[r] = s;
        if (s == GPBO_OK) {
          ok_m.push_back(ms[q]);
          ok_r.push_back(r);
          continue;
        }
        if (ms[q]) {
          free_model_buffers(ms[q]);
          delete ms[q];
        }
        if (s == GPBO_E_NOT_PD) next.push_back(r);
      }
      pend.swap(next);
    }
    gpbo_status res = GPBO_OK;
    if (!ok_m.empty()) {
      const int nk = (int)ok_m.size();
      res = gpbo_lml_grad_batched(c, nk, (const gpbo_model*)ok_m.data(), ldg, g_dev, l_dev);
      if (res == GPBO_OK) {
        HIP_TRY(c, hipMemcpyAsync(g_h.data(), g_dev, (size_t)nk * ldg * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(l_h.data(), l_dev, (size_t)nk * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
      }
      // rows of g_h / l_h in ok order move to the runs' slots below
      std::vector<double> gg((size_t)nk * ldg), ll(nk);
      std::copy(g_h.begin(), g_h.begin() + (size_t)nk * ldg, gg.begin());
      std::copy(l_h.begin(), l_h.begin() + nk, ll.begin());
      for (int q = 0; q < nk; ++q) {
        const int r = ok_r[q], d = probs[r / S].d;
        const double sn2 = std::exp(th[r][d + 1]);
        for (int j = 0; j < ldg; ++j) g_h[(size_t)r * ldg + j] = gg[(size_t)q * ldg + j];
        // the derivative with respect to log sn2, not the jittered variance
        g_h[(size_t)r * ldg + d + 1] *= sn2 / (sn2 + jit_r[r]);
        l_h[r] = ll[q];
        free_model_buffers(ok_m[q]);
        delete ok_m[q];
      }
    }
    return res;
  };
  // g_h / l_h are indexed by run after evaluate (it needs N rows)
  g_h.resize((size_t)std::max(N, 1) * ldg);
  l_h.resize(std::max(N, 1));
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int t = 1; t <= o->steps; ++t) {
    std::vector<int> rs;
    for (int r = 0; r < N; ++r)
      if (alive[r]) rs.push_back(r);
    if (rs.empty()) break;
    {
      const gpbo_status st = evaluate(rs);
      if (st != GPBO_OK) return st;
    }
    for (int r : rs) {
      if (st_r[r] != GPBO_OK) {
        alive[r] = 0;
        continue;
      }
      const int b = r / S, d = probs[b].d;
      const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
      for (int j = 0; j < d + 2; ++j) {
        const double gj = g_h[(size_t)r * ldg + j];
        mo[r][j] = b1 * mo[r][j] + (1.0 - b1) * gj;
        ve[r][j] = b2 * ve[r][j] + (1.0 - b2) * gj * gj;
        const double mh = mo[r][j] / c1, vh = ve[r][j] / c2;
        const double v = th[r][j] + o->lr * mh / (std::sqrt(vh) + eps);
        th[r][j] = std::min(std::max(v, lo[(size_t)b * ldt + j]), hi[(size_t)b * ldt + j]);
      }
    }
  }
  {
    std::vector<int> rs;
    for (int r = 0; r < N; ++r)
      if (alive[r]) rs.push_back(r);
    if (!rs.empty()) {
      const gpbo_status st = evaluate(rs);
      if (st != GPBO_OK) return st;
    }
    for (int r : rs)
      if (st_r[r] == GPBO_OK) {
        fin_lml[r] = l_h[r];
        fin_jit[r] = jit_r[r];
      }
  }
  gpbo_status first = GPBO_OK;
  std::vector<int> best_r(B);
  for (int b = 0; b < B; ++b) {
    int best = b * S;
    for (int s = 1; s < S; ++s)
      if (fin_lml[b * S + s] > fin_lml[best]) best = b * S + s;
    best_r[b] = best;
    const int d = probs[b].d;
    for (int j = 0; j < ldt; ++j) theta[(size_t)b * ldt + j] = j < d + 2 ? th[best][j] : 0.0;
    lml[b] = fin_lml[best];
    if (jitter) jitter[b] = fin_jit[best];
    status[b] = std::isfinite(fin_lml[best]) ? GPBO_OK : GPBO_E_NOT_PD;
    if (status[b] != GPBO_OK && first == GPBO_OK) first = (gpbo_status)status[b];
  }
  if (out) {  // the models at the chosen hyperparameters (with their jitter)
    std::vector<gpbo_problem> pp;
    std::vector<std::vector<double>> ls;
    std::vector<int> idx;
    for (int b = 0; b < B; ++b)
      if (status[b] == GPBO_OK) idx.push_back(b);
    ls.resize(idx.size());
    for (size_t q = 0; q < idx.size(); ++q) {
      const int b = idx[q], d = probs[b].d;
      ls[q].resize(d);
      for (int j = 0; j < d; ++j) ls[q][j] = std::exp(theta[(size_t)b * ldt + j]);
      gpbo_problem p = probs[b];
      p.lengthscale = ls[q].data();
      p.signal_var = std::exp(theta[(size_t)b * ldt + d]);
      p.noise_var = std::exp(theta[(size_t)b * ldt + d + 1]) + fin_jit[best_r[b]];
      pp.push_back(p);
    }
    if (!pp.empty()) {
      std::vector<gpbo_model> om(pp.size(), nullptr);
      std::vector<int32_t> os(pp.size(), GPBO_OK);
      const gpbo_status st = gpbo_fit_batched(c, (int32_t)pp.size(), pp.data(), om.data(), nullptr,
                                              os.data());
      for (size_t q = 0; q < idx.size(); ++q) {
        out[idx[q]] = om[q];
        if (os[q] != GPBO_OK) status[idx[q]] = os[q];
      }
      if (st != GPBO_OK && first == GPBO_OK) first = st;
    }
  }
  return first;
}

}  // extern "C"
