// Top-k selection and row gather on the GPU.
//
// top-k of m float scores by (value descending, index ascending):
//   1. radix select on the order-preserving 32-bit keys of the scores, eight
//      bits per pass from the most significant: a histogram of the current
//      digit among the keys that match the prefix found so far, then a
//      single-workgroup scan that fixes the digit and the count still needed;
//   2. compaction: every key above the threshold, and the lowest-index keys
//      equal to it (an ordered prefix over per-block counts), into k slots;
//   3. one workgroup sorts the k (key, index) pairs in LDS (bitonic).
// NaN scores map to the lowest key and never rank ahead of a number.
#include <climits>
#include <mutex>

#include "gpbo_internal.h"

namespace gpbo {

// Scratch of the allocation-free top-k (gpbo_topk_noalloc): a static device
// array, one copy per GPU, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host the name is a stand-in,
// not a device address): the address comes from hipGetSymbolAddress, once
// per device, with that device current (topk_noalloc_init).
constexpr size_t kTopkNoallocBytes = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[kTopkNoallocBytes];
static_assert(kTopkNoallocBytes == GPBO_TOPK_NOALLOC_SCRATCH, "size stated in the header");

namespace {

constexpr int SEL_BLOCK = 256;
constexpr int SEL_MAXK = 8192;  // LDS of the final sort: 8192 x 12 bytes

// Order-preserving key: larger float -> larger unsigned; NaN -> 0.
__device__ __forceinline__ unsigned fkey(float f) {
  if (f != f) return 0u;
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Workgroups of a histogram pass: each adds its nonzero bins to the global
// histogram with one atomic each, so on concentrated keys every workgroup
// hits the same bin; about one per CU keeps that serialisation short.
constexpr int kHistBlocks = 256;

// state[0] = prefix, state[1] = prefix mask, state[2] = k still needed
__global__ void __launch_bounds__(SEL_BLOCK) k_radix_hist(const float* __restrict__ v, int64_t m,
                                                          const unsigned* __restrict__ state,
                                                          int shift, unsigned* __restrict__ hist) {
  __shared__ unsigned h[256];
  for (int i = threadIdx.x; i < 256; i += SEL_BLOCK) h[i] = 0;
  __syncthreads();
  const unsigned prefix = state[0], mask = state[1];
  const int lane = threadIdx.x % 64;
  for (int64_t i = blockIdx.x * (int64_t)SEL_BLOCK + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * SEL_BLOCK) {
    const unsigned key = fkey(v[i]);
    const bool mine = (key & mask) == prefix;
    const unsigned dg = (key >> shift) & 255u;
    // keys concentrated on one digit (the later passes, or a narrow range of
    // values): when every counted lane of the wave has the first one's
    // digit, one LDS atomic adds them all
    const unsigned long long act = __ballot(mine);
    if (act == 0ull) continue;
    const int leader = __ffsll((long long)act) - 1;
    const unsigned dl = __shfl(dg, leader);
    const unsigned long long same = __ballot(mine && dg == dl);
    if (same == act) {
      if (lane == leader) atomicAdd(&h[dl], (unsigned)__popcll(same));
    } else if (mine) {
      atomicAdd(&h[dg], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += SEL_BLOCK)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Fix this pass's digit: the largest digit whose suffix count reaches the k
// still needed.  Clears the histogram for the next pass.
__global__ void k_radix_scan(unsigned* __restrict__ hist, unsigned* __restrict__ state, int shift) {
  if (threadIdx.x == 0) {
    unsigned need = state[2];
    unsigned above = 0;
    int digit = 0;
    for (int b = 255; b >= 0; --b) {
      if (above + hist[b] >= need) {
        digit = b;
        break;
      }
      above += hist[b];
    }
    state[0] |= (unsigned)digit << shift;
    state[1] |= 255u << shift;
    state[2] = need - above;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

__global__ void k_sel_init(unsigned* __restrict__ state, unsigned* __restrict__ hist,
                           unsigned k) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) {
    state[0] = 0;
    state[1] = 0;
    state[2] = k;
    state[3] = 0;  // slots used by keys above the threshold
  }
}

// Per-block count of keys equal to the threshold.
__global__ void __launch_bounds__(SEL_BLOCK) k_eq_count(const float* __restrict__ v, int64_t m,
                                                        const unsigned* __restrict__ state,
                                                        int64_t per_block,
                                                        unsigned* __restrict__ counts) {
  __shared__ unsigned c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const unsigned thr = state[0];
  const int64_t beg = blockIdx.x * per_block, end = min(m, beg + per_block);
  unsigned local = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += SEL_BLOCK) local += fkey(v[i]) == thr;
  if (local) atomicAdd(&c, local);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// Exclusive scan of the per-block equal counts (one workgroup).
// (Exclusive prefix sum of the per-block counts, in place, by one workgroup:
// each thread owns a run of consecutive blocks, the run totals are scanned
// across the wave by shuffles and across the waves through LDS.)
constexpr int SCAN_THREADS = 1024;
__global__ void __launch_bounds__(SCAN_THREADS) k_eq_scan(unsigned* __restrict__ counts,
                                                          int nblocks) {
  __shared__ unsigned wsum[SCAN_THREADS / 64];
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int per = (nblocks + SCAN_THREADS - 1) / SCAN_THREADS;
  const int b0 = min(nblocks, t * per), b1 = min(nblocks, b0 + per);
  unsigned own = 0;
  for (int b = b0; b < b1; ++b) own += counts[b];
  unsigned x = own;  // inclusive scan within the wave
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  unsigned before = 0;
  for (int q = 0; q < w; ++q) before += wsum[q];
  unsigned run = before + x - own;
  for (int b = b0; b < b1; ++b) {
    const unsigned c = counts[b];
    counts[b] = run;
    run += c;
  }
}

// Write the selected (key, index) pairs: keys above the threshold take slots
// from a counter (any order); equal keys take the slots after them in index
// order, as long as the k still needed allows.
__global__ void __launch_bounds__(SEL_BLOCK) k_sel_write(const float* __restrict__ v, int64_t m,
                                                         unsigned* __restrict__ state,
                                                         int64_t per_block,
                                                         const unsigned* __restrict__ eq_before,
                                                         unsigned k, unsigned* __restrict__ okey,
                                                         int64_t* __restrict__ oidx) {
  __shared__ unsigned wave_base[SEL_BLOCK / 64];
  const unsigned thr = state[0], need_eq = state[2];
  const unsigned n_above = k - need_eq;
  const int64_t beg = blockIdx.x * per_block, end = min(m, beg + per_block);
  unsigned eq_run = eq_before[blockIdx.x];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  for (int64_t base = beg; base < end; base += SEL_BLOCK) {
    const int64_t i = base + threadIdx.x;
    const unsigned key = i < end ? fkey(v[i]) : 0u;
    const bool valid = i < end;
    if (valid && key > thr) {
      const unsigned slot = atomicAdd(&state[3], 1u);
      if (slot < n_above) {
        okey[slot] = key;
        oidx[slot] = i;
      }
    }
    // ordered rank among the equal keys of this chunk
    const bool eq = valid && key == thr;
    const unsigned long long bal = __ballot(eq);
    const unsigned below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_base[w] = __popcll(bal);
    __syncthreads();
    unsigned off = eq_run;
    for (int q = 0; q < w; ++q) off += wave_base[q];
    unsigned chunk_total = 0;
    for (int q = 0; q < SEL_BLOCK / 64; ++q) chunk_total += wave_base[q];
    if (eq) {
      const unsigned r = off + below;
      if (r < need_eq) {
        okey[n_above + r] = key;
        oidx[n_above + r] = i;
      }
    }
    eq_run += chunk_total;
    __syncthreads();
  }
}

// Top-k as a set in ascending index order (k beyond the sort's limit): per
// block, the number of selected entries -- keys above the threshold, and
// keys equal to it whose rank among the equal keys (in index order) is below
// the count still needed -- then an exclusive scan over the blocks, then an
// ordered write.  eq_before: exclusive prefix of the per-block equal counts.
__device__ __forceinline__ void set_flags(const float* __restrict__ v, int64_t i, int64_t end,
                                          unsigned thr, unsigned need_eq, unsigned eq_run,
                                          unsigned* wave_eq, bool& sel, unsigned& chunk_eq) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const bool valid = i < end;
  const unsigned key = valid ? fkey(v[i]) : 0u;
  const bool eq = valid && key == thr;
  const unsigned long long bal = __ballot(eq);
  if (lane == 0) wave_eq[w] = __popcll(bal);
  __syncthreads();
  unsigned off = eq_run;
  for (int q = 0; q < w; ++q) off += wave_eq[q];
  chunk_eq = 0;
  for (int q = 0; q < SEL_BLOCK / 64; ++q) chunk_eq += wave_eq[q];
  __syncthreads();
  const unsigned r = off + __popcll(bal & ((1ull << lane) - 1ull));
  sel = valid && (key > thr || (eq && r < need_eq));
}

__global__ void __launch_bounds__(SEL_BLOCK) k_set_count(const float* __restrict__ v, int64_t m,
                                                         const unsigned* __restrict__ state,
                                                         int64_t per_block,
                                                         const unsigned* __restrict__ eq_before,
                                                         unsigned* __restrict__ sel_counts) {
  __shared__ unsigned wave_eq[SEL_BLOCK / 64];
  __shared__ unsigned c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const unsigned thr = state[0], need_eq = state[2];
  const int64_t beg = blockIdx.x * per_block, end = min(m, beg + per_block);
  unsigned eq_run = eq_before[blockIdx.x];
  unsigned local = 0;
  for (int64_t base = beg; base < end; base += SEL_BLOCK) {
    bool sel;
    unsigned chunk_eq;
    set_flags(v, base + threadIdx.x, end, thr, need_eq, eq_run, wave_eq, sel, chunk_eq);
    local += sel;
    eq_run += chunk_eq;
  }
  if (local) atomicAdd(&c, local);
  __syncthreads();
  if (threadIdx.x == 0) sel_counts[blockIdx.x] = c;
}

__global__ void __launch_bounds__(SEL_BLOCK) k_set_write(const float* __restrict__ v, int64_t m,
                                                         const unsigned* __restrict__ state,
                                                         int64_t per_block,
                                                         const unsigned* __restrict__ eq_before,
                                                         const unsigned* __restrict__ sel_before,
                                                         int64_t* __restrict__ out) {
  __shared__ unsigned wave_eq[SEL_BLOCK / 64], wave_sel[SEL_BLOCK / 64];
  const unsigned thr = state[0], need_eq = state[2];
  const int64_t beg = blockIdx.x * per_block, end = min(m, beg + per_block);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  unsigned eq_run = eq_before[blockIdx.x];
  unsigned sel_run = sel_before[blockIdx.x];
  for (int64_t base = beg; base < end; base += SEL_BLOCK) {
    const int64_t i = base + threadIdx.x;
    bool sel;
    unsigned chunk_eq;
    set_flags(v, i, end, thr, need_eq, eq_run, wave_eq, sel, chunk_eq);
    const unsigned long long bal = __ballot(sel);
    if (lane == 0) wave_sel[w] = __popcll(bal);
    __syncthreads();
    unsigned off = sel_run, chunk_sel = 0;
    for (int q = 0; q < SEL_BLOCK / 64; ++q) {
      if (q < w) off += wave_sel[q];
      chunk_sel += wave_sel[q];
    }
    if (sel) out[off + __popcll(bal & ((1ull << lane) - 1ull))] = i;
    eq_run += chunk_eq;
    sel_run += chunk_sel;
    __syncthreads();
  }
}

// Bitonic sort of k pairs by (key descending, index ascending), one
// workgroup, in LDS; writes the indices.
__global__ void __launch_bounds__(1024) k_sel_sort(const unsigned* __restrict__ key,
                                                   const int64_t* __restrict__ idx, int k,
                                                   int64_t* __restrict__ out) {
  __shared__ unsigned sk[SEL_MAXK];
  __shared__ int64_t si[SEL_MAXK];
  int p2 = 1;
  while (p2 < k) p2 <<= 1;
  for (int i = threadIdx.x; i < p2; i += blockDim.x) {
    sk[i] = i < k ? key[i] : 0u;
    si[i] = i < k ? idx[i] : INT64_MAX;
  }
  __syncthreads();
  // "a before b" when a.key > b.key, or equal keys and a.idx < b.idx
  for (int size = 2; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const bool i_first = sk[i] > sk[j] || (sk[i] == sk[j] && si[i] < si[j]);
          if (up != i_first) {
            const unsigned tk = sk[i];
            sk[i] = sk[j];
            sk[j] = tk;
            const int64_t ti = si[i];
            si[i] = si[j];
            si[j] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) out[i] = si[i];
}

__global__ void k_gather_rows(int64_t k, const int64_t* __restrict__ idx, int d,
                              const float* __restrict__ X, float* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < k * d;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d;
    const int c = (int)(e % d);
    out[e] = X[idx[r] * d + c];
  }
}

// The chosen configuration of each of up to NEXT_MAX searches: row argmax[b]
// of search b's pool, widened to float64, into row b of out (ldx columns,
// zero beyond the search's d; a row of NaN for an index outside the pool,
// such as the -1 of an empty pool).
struct NextArgs {
  const void* X[NEXT_MAX];
  int64_t m[NEXT_MAX];
  int d[NEXT_MAX];
};
__global__ void __launch_bounds__(64) k_next_rows(NextArgs A, int dbl, const int64_t* __restrict__ am,
                                                  int ldx, double* __restrict__ out) {
  const int b = blockIdx.x, k = threadIdx.x;
  const int d = A.d[b];
  const int64_t i = am[b];
  for (int c = k; c < ldx; c += 64) {
    double v = 0.0;
    if (c < d)
      v = (i < 0 || i >= A.m[b]) ? __builtin_nan("")
                : dbl ? ((const double*)A.X[b])[i * d + c] : (double)((const float*)A.X[b])[i * d + c];
    out[(int64_t)b * ldx + c] = v;
  }
}

}  // namespace

int topk_max_k() { return SEL_MAXK; }

// Scratch (device, from the context): state (4 u32), histogram (256 u32),
// per-block counts, k keys, k indices.
size_t topk_scratch_bytes(int64_t m, int64_t k) {
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  return 4096 + round_up(nb * 4, 256) + round_up(k * 4, 256) + k * 8;
}

// Scratch of the set selection: state, histogram, two per-block count arrays.
size_t topk_set_scratch_bytes(int64_t m) {
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  return 4096 + 2 * round_up(nb * 4, 256);
}

const unsigned* topk_set_threshold(const void* ws) { return (const unsigned*)ws; }

void launch_topk_set_into(int64_t m, const float* v, int64_t k, int64_t* idx, void* ws,
                          hipStream_t s) {
  unsigned* state = (unsigned*)ws;
  unsigned* hist = state + 64;
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  unsigned* eq_counts = (unsigned*)((unsigned char*)ws + 4096);
  unsigned* sel_counts = (unsigned*)((unsigned char*)eq_counts + round_up(nb * 4, 256));
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, state, hist, (unsigned)k);
  const int g = (int)std::min<int64_t>(kHistBlocks, ceil_div(m, SEL_BLOCK));
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(g), dim3(SEL_BLOCK), 0, s, v, m, state, shift, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(256), 0, s, hist, state, shift);
  }
  const int64_t per_block = round_up(ceil_div(m, nb), SEL_BLOCK);
  const int nblocks = (int)ceil_div(m, per_block);
  hipLaunchKernelGGL(k_eq_count, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     eq_counts);
  hipLaunchKernelGGL(k_eq_scan, dim3(1), dim3(SCAN_THREADS), 0, s, eq_counts, nblocks);
  hipLaunchKernelGGL(k_set_count, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     eq_counts, sel_counts);
  hipLaunchKernelGGL(k_eq_scan, dim3(1), dim3(SCAN_THREADS), 0, s, sel_counts, nblocks);
  hipLaunchKernelGGL(k_set_write, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     eq_counts, sel_counts, idx);
}

void launch_topk_into(int64_t m, const float* v, int64_t k, int64_t* idx, void* ws,
                      hipStream_t s) {
  unsigned* state = (unsigned*)ws;
  unsigned* hist = state + 64;
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  unsigned* counts = (unsigned*)((unsigned char*)ws + 4096);
  unsigned* okey = (unsigned*)((unsigned char*)counts + round_up(nb * 4, 256));
  int64_t* oidx = (int64_t*)((unsigned char*)okey + round_up(k * 4, 256));
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, state, hist, (unsigned)k);
  const int g = (int)std::min<int64_t>(kHistBlocks, ceil_div(m, SEL_BLOCK));
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(g), dim3(SEL_BLOCK), 0, s, v, m, state, shift, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(256), 0, s, hist, state, shift);
  }
  const int64_t per_block = round_up(ceil_div(m, nb), SEL_BLOCK);
  const int nblocks = (int)ceil_div(m, per_block);
  hipLaunchKernelGGL(k_eq_count, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     counts);
  hipLaunchKernelGGL(k_eq_scan, dim3(1), dim3(SCAN_THREADS), 0, s, counts, nblocks);
  hipLaunchKernelGGL(k_sel_write, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     counts, (unsigned)k, okey, oidx);
  hipLaunchKernelGGL(k_sel_sort, dim3(1), dim3(1024), 0, s, okey, oidx, (int)k, idx);
}

__global__ void k_compose_idx(int64_t k, const int64_t* __restrict__ outer,
                              const int64_t* __restrict__ inner, int64_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = outer[inner[i]];
}

void launch_compose_idx(int64_t k, const int64_t* outer, const int64_t* inner, int64_t* out,
                        hipStream_t s) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(k, 256)));
  hipLaunchKernelGGL(k_compose_idx, dim3(g), dim3(256), 0, s, k, outer, inner, out);
}

// The float whose order-preserving key is `key` (inverse of fkey).
__device__ __forceinline__ float key_float(unsigned key) {
  return __uint_as_float((key & 0x80000000u) ? (key & 0x7fffffffu) : ~key);
}

// Result of an exact re-score of a subset: the pool index of the argmax and
// whether no unscored candidate of the subset can beat it.  thr_key: the
// order-preserving key of the smallest EI bound that was scored (the
// selection threshold; NULL when every candidate was scored): every
// unscored candidate's bound is at most that value.  tol: allowance in
// units of s_y (stats[1], the model's scale of y).
__global__ void k_subset_finish(const int64_t* __restrict__ am, const double* __restrict__ em,
                                const int64_t* __restrict__ pool_idx,
                                const unsigned* __restrict__ thr_key, double tol,
                                const double* __restrict__ stats, int64_t* __restrict__ next,
                                double* __restrict__ ei_max, int* __restrict__ certified) {
  if (threadIdx.x != 0) return;
  const int64_t a = *am;
  next[0] = a >= 0 ? pool_idx[a] : -1;
  ei_max[0] = *em;
  int cert = a >= 0;
  if (thr_key) cert = cert && *em >= (double)key_float(*thr_key) + tol * stats[S_YSTD];
  certified[0] = cert;
}

void launch_subset_finish(const int64_t* am, const double* em, const int64_t* pool_idx,
                          const unsigned* thr_key, double tol, const double* stats, int64_t* next,
                          double* ei_max, int* certified, hipStream_t s) {
  hipLaunchKernelGGL(k_subset_finish, dim3(1), dim3(64), 0, s, am, em, pool_idx, thr_key, tol,
                     stats, next, ei_max, certified);
}

namespace {
std::mutex g_noalloc_mu;
constexpr int kMaxDevices = 64;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

bool topk_noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return true;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) {
    (void)hipGetLastError();
    return false;  // the caller makes `device` current first
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return false;
  }
  g_noalloc_ptr[device] = p;
  return true;
}

void* topk_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

size_t topk_noalloc_bytes() { return kTopkNoallocBytes; }

void launch_next_rows(int B, const void* const* X, const int64_t* m, const int* d, int dbl,
                      const int64_t* am, int ldx, double* out, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += NEXT_MAX) {
    const int nb = std::min(NEXT_MAX, B - b0);
    NextArgs A{};
    for (int q = 0; q < nb; ++q) {
      A.X[q] = X[b0 + q];
      A.m[q] = m[b0 + q];
      A.d[q] = d[b0 + q];
    }
    hipLaunchKernelGGL(k_next_rows, dim3(nb), dim3(64), 0, s, A, dbl, am + b0, ldx,
                       out + (int64_t)b0 * ldx);
  }
}

void launch_gather_rows(int64_t k, const int64_t* idx, int d, const float* Xc, float* out,
                        hipStream_t s) {
  const int g = (int)std::min<int64_t>(4096, ceil_div(k * d, 256));
  hipLaunchKernelGGL(k_gather_rows, dim3(std::max(g, 1)), dim3(256), 0, s, k, idx, d, Xc, out);
}

}  // namespace gpbo
