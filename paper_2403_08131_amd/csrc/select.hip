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

#include "gpbo_internal.h"

namespace gpbo {

namespace {

constexpr int SEL_BLOCK = 256;
constexpr int SEL_MAXK = 8192;  // LDS of the final sort: 8192 x 12 bytes

// Order-preserving key: larger float -> larger unsigned; NaN -> 0.
__device__ __forceinline__ unsigned fkey(float f) {
  if (f != f) return 0u;
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// state[0] = prefix, state[1] = prefix mask, state[2] = k still needed
__global__ void __launch_bounds__(SEL_BLOCK) k_radix_hist(const float* __restrict__ v, int64_t m,
                                                          const unsigned* __restrict__ state,
                                                          int shift, unsigned* __restrict__ hist) {
  __shared__ unsigned h[256];
  for (int i = threadIdx.x; i < 256; i += SEL_BLOCK) h[i] = 0;
  __syncthreads();
  const unsigned prefix = state[0], mask = state[1];
  for (int64_t i = blockIdx.x * (int64_t)SEL_BLOCK + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * SEL_BLOCK) {
    const unsigned key = fkey(v[i]);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
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
__global__ void k_eq_scan(unsigned* __restrict__ counts, int nblocks) {
  if (threadIdx.x == 0) {
    unsigned run = 0;
    for (int b = 0; b < nblocks; ++b) {
      const unsigned c = counts[b];
      counts[b] = run;
      run += c;
    }
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

}  // namespace

int topk_max_k() { return SEL_MAXK; }

// Scratch (device, from the context): state (4 u32), histogram (256 u32),
// per-block counts, k keys, k indices.
size_t topk_scratch_bytes(int64_t m, int64_t k) {
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  return 4096 + round_up(nb * 4, 256) + round_up(k * 4, 256) + k * 8;
}

void launch_topk_into(int64_t m, const float* v, int64_t k, int64_t* idx, void* scratch,
                      hipStream_t s) {
  unsigned* state = (unsigned*)scratch;
  unsigned* hist = state + 64;
  const int64_t nb = std::min<int64_t>(1024, ceil_div(m, SEL_BLOCK));
  unsigned* counts = (unsigned*)((unsigned char*)scratch + 4096);
  unsigned* okey = (unsigned*)((unsigned char*)counts + round_up(nb * 4, 256));
  int64_t* oidx = (int64_t*)((unsigned char*)okey + round_up(k * 4, 256));
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, state, hist, (unsigned)k);
  const int g = (int)std::min<int64_t>(2048, ceil_div(m, SEL_BLOCK));
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(g), dim3(SEL_BLOCK), 0, s, v, m, state, shift, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(256), 0, s, hist, state, shift);
  }
  const int64_t per_block = round_up(ceil_div(m, nb), SEL_BLOCK);
  const int nblocks = (int)ceil_div(m, per_block);
  hipLaunchKernelGGL(k_eq_count, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     counts);
  hipLaunchKernelGGL(k_eq_scan, dim3(1), dim3(64), 0, s, counts, nblocks);
  hipLaunchKernelGGL(k_sel_write, dim3(nblocks), dim3(SEL_BLOCK), 0, s, v, m, state, per_block,
                     counts, (unsigned)k, okey, oidx);
  hipLaunchKernelGGL(k_sel_sort, dim3(1), dim3(1024), 0, s, okey, oidx, (int)k, idx);
}

void launch_gather_rows(int64_t k, const int64_t* idx, int d, const float* Xc, float* out,
                        hipStream_t s) {
  const int g = (int)std::min<int64_t>(4096, ceil_div(k * d, 256));
  hipLaunchKernelGGL(k_gather_rows, dim3(std::max(g, 1)), dim3(256), 0, s, k, idx, d, Xc, out);
}

}  // namespace gpbo
