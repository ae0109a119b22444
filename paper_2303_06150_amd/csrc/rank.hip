// Global ranking of a library (Sec. 2: rank the input chemical library by the
// docked ligands' scores): the top m of n groups by each group's best value,
// equal values ordered by lower group index.
//
// Keys.  Group i with best value v gets one 64-bit key: the upper word orders
// the values (larger value, larger key; -0 counts as +0), the lower word is
// 0xFFFFFFFF - i, so equal values rank the lower index first.  Keys are
// distinct, so "the top m" is a set and no sort stability is needed.
//
// Steps.  (1) keys and best members; (2) radix select of the m-th largest key,
// one byte per pass from the top (histogram of the keys that still match the
// selected prefix, then one thread walks the 256 bins from the top), stopping as
// soon as the selected bin holds exactly the keys still needed; (3) compaction
// of the m keys >= that threshold (wave-aggregated counter); (4) a descending
// bitonic sort of the m keys, in LDS for m <= 4096, else tile sorts in LDS plus
// global merge steps; (5) ids, values and members of the sorted keys.
#include "lg.h"
#include "lg_internal.h"

#include <algorithm>
#include <mutex>

namespace lg {

namespace {

constexpr int kTile = 4096;          // keys sorted in LDS by one block (32 KB)
constexpr int kSortThreads = 1024;

__device__ __forceinline__ uint64_t rank_key(float v, int i) {
  const uint32_t hi = (uint32_t)orderable(v + 0.0f) ^ 0x80000000u;
  return ((uint64_t)hi << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
}

__device__ __forceinline__ float key_value(uint64_t k) {
  const int o = (int)((uint32_t)(k >> 32) ^ 0x80000000u);
  return __int_as_float(o ^ ((o >> 31) & 0x7FFFFFFF));   // orderable() is its own inverse
}

__device__ __forceinline__ int key_index(uint64_t k) { return (int)(0xFFFFFFFFu - (uint32_t)k); }

// Per group: best value (first member on equal values) and its key.
__global__ void rank_keys_kernel(const float* score, int n, int group, uint64_t* keys, int32_t* member) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    const float* s = score + i * group;
    float best = s[0];
    int bm = 0;
    for (int q = 1; q < group; ++q)
      if (s[q] > best) { best = s[q]; bm = q; }
    keys[i] = rank_key(best, (int)i);
    member[i] = bm;
  }
}

__global__ void rank_init_kernel(RankState* st, uint32_t* hist, int m) {
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->mask = 0;
    st->need = (uint32_t)m;
    st->done = 0;
    st->count = 0;
  }
  hist[threadIdx.x] = 0;
}

// Histogram of byte `shift` of the keys that match the selected prefix.
__global__ __launch_bounds__(256) void rank_hist_kernel(const uint64_t* keys, int n, const RankState* st,
                                                        uint32_t* hist, int shift) {
  if (st->done) return;
  __shared__ uint32_t lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t prefix = st->prefix, mask = st->mask;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t k = keys[i];
    if ((k & mask) == prefix) atomicAdd(&lh[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

// The bin of the key of rank `need` (counting from the largest) among the keys
// matching the prefix; extends the prefix by it.  Done once that bin holds
// exactly the keys still needed: then the threshold is the prefix with zero
// lower bits, and the keys >= it are the top m.
__global__ __launch_bounds__(256) void rank_pick_kernel(RankState* st, uint32_t* hist, int shift) {
  if (threadIdx.x == 0 && !st->done) {
    uint32_t above = 0;
    int b = 255;
    for (; b > 0; --b) {
      if (above + hist[b] >= st->need) break;
      above += hist[b];
    }
    st->need -= above;
    st->prefix |= (uint64_t)b << shift;
    st->mask |= (uint64_t)255u << shift;
    if (hist[b] == st->need) st->done = 1;
  }
  __syncthreads();
  hist[threadIdx.x] = 0;
}

// The keys >= threshold (exactly m of them), in any order; [m, padded) set to 0.
__global__ __launch_bounds__(256) void rank_compact_kernel(const uint64_t* keys, int n, RankState* st, uint64_t* cand,
                                                           int m, long long padded) {
  const uint64_t t = st->prefix;
  const int lane = lane_id();
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long base = blockIdx.x * (long long)blockDim.x + threadIdx.x - lane; base < n; base += stride) {
    const long long i = base + lane;
    const uint64_t k = i < n ? keys[i] : 0;
    const bool sel = i < n && k >= t;
    const uint64_t bal = __ballot(sel);
    if (bal == 0) continue;
    uint32_t first = 0;
    if (lane == 0) first = atomicAdd(&st->count, (uint32_t)__popcll(bal));
    first = __builtin_amdgcn_readfirstlane(first);
    const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (sel && first + pre < (uint32_t)m) cand[first + pre] = k;
  }
  for (long long i = m + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < padded; i += stride) cand[i] = 0;
}

// One compare-exchange of the descending bitonic network: stage k, distance j.
__device__ __forceinline__ void bitonic_cx(uint64_t& a, uint64_t& b, long long i, long long k) {
  const bool desc = (i & k) == 0;
  if (desc ? a < b : a > b) {
    const uint64_t t = a;
    a = b;
    b = t;
  }
}

// Sort of `len` (power of two, <= kTile) keys in LDS, stages k0 (first) to
// kmax, then writes them back.  With k0 = 2 a whole tile is sorted; with
// k0 = kmax > kTile only the steps j < kTile of stage kmax run (the merge tail).
__global__ __launch_bounds__(kSortThreads) void rank_tile_kernel(uint64_t* a, int len, long long k0, long long kmax) {
  __shared__ uint64_t s[kTile];
  const long long base = (long long)blockIdx.x * len;
  for (int t = threadIdx.x; t < len; t += blockDim.x) s[t] = a[base + t];
  __syncthreads();
  for (long long k = k0; k <= kmax; k *= 2) {
    for (long long j = (k > len ? len : k) / 2; j >= 1; j /= 2) {
      for (int p = threadIdx.x; p < len / 2; p += blockDim.x) {
        const int i = (int)(2 * j * (p / j) + (p % j));
        bitonic_cx(s[i], s[i + j], base + i, k);
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < len; t += blockDim.x) a[base + t] = s[t];
}

// One global step (stage k, distance j >= kTile) of the bitonic network.
__global__ __launch_bounds__(256) void rank_merge_kernel(uint64_t* a, long long padded, long long k, long long j) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < padded / 2; p += stride) {
    const long long i = 2 * j * (p / j) + (p % j);
    bitonic_cx(a[i], a[i + j], i, k);
  }
}

__global__ void rank_out_kernel(const uint64_t* sorted, const int32_t* member, int n, int m, int32_t* top_idx,
                                float* top_score, int32_t* top_member) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const uint64_t k = sorted[q];
  const int i = key_index(k);
  top_idx[q] = i;
  top_score[q] = key_value(k);
  if (top_member) top_member[q] = (i >= 0 && i < n) ? member[i] : -1;
}

long long pow2_at_least(long long m) {
  long long p = 1;
  while (p < m) p *= 2;
  return p;
}

constexpr size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr size_t scratch_bytes(size_t n, size_t pow2_m) {
  return up256(sizeof(RankState)) + up256(256 * sizeof(uint32_t)) + up256(n * 8) + up256(n * 4) +
         up256(pow2_m * 8);
}

// Fixed device scratch of lg_rank_static, sized for its largest accepted call
// (LG_RANK_STATIC_MAX_TOP is a power of two).  Every device the library runs on
// holds one copy until the process ends.  Host code must not pass this name to
// a kernel: its device address comes from hipGetSymbolAddress.
static_assert((LG_RANK_STATIC_MAX_TOP & (LG_RANK_STATIC_MAX_TOP - 1)) == 0, "power of two");
constexpr size_t kStaticScratchBytes = scratch_bytes(LG_RANK_STATIC_MAX_GROUPS, LG_RANK_STATIC_MAX_TOP);
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;

}  // namespace

size_t rank_scratch_bytes(int n, int m) { return scratch_bytes((size_t)n, (size_t)pow2_at_least(m < 1 ? 1 : m)); }

// Device address of the current device's copy of the fixed scratch, looked up
// once per device (with that device current) and kept.
hipError_t rank_static_scratch(void** out, size_t* bytes) {
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

hipError_t launch_rank(const float* score, int n, int group, int m, void* work, int32_t* top_idx,
                       float* top_score, int32_t* top_member, hipStream_t st) {
  if (n <= 0 || m <= 0) return hipSuccess;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* w = (char*)work;
  RankState* state = (RankState*)w;
  w += up(sizeof(RankState));
  uint32_t* hist = (uint32_t*)w;
  w += up(256 * sizeof(uint32_t));
  uint64_t* keys = (uint64_t*)w;
  w += up((size_t)n * 8);
  int32_t* member = (int32_t*)w;
  w += up((size_t)n * 4);
  uint64_t* cand = (uint64_t*)w;
  const long long padded = pow2_at_least(m);
  const int blocks = (int)std::min<long long>(((long long)n + 255) / 256, 2048);
  hipLaunchKernelGGL(rank_keys_kernel, dim3(blocks), dim3(256), 0, st, score, n, group, keys, member);
  hipLaunchKernelGGL(rank_init_kernel, dim3(1), dim3(256), 0, st, state, hist, m);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(rank_hist_kernel, dim3(blocks), dim3(256), 0, st, keys, n, state, hist, shift);
    hipLaunchKernelGGL(rank_pick_kernel, dim3(1), dim3(256), 0, st, state, hist, shift);
  }
  hipLaunchKernelGGL(rank_compact_kernel, dim3(blocks), dim3(256), 0, st, keys, n, state, cand, m, padded);
  if (padded <= kTile) {
    hipLaunchKernelGGL(rank_tile_kernel, dim3(1), dim3(kSortThreads), 0, st, cand, (int)padded, 2LL, padded);
  } else {
    const int tiles = (int)(padded / kTile);
    const int mblocks = (int)std::min<long long>(padded / 2 / 256, 4096);
    hipLaunchKernelGGL(rank_tile_kernel, dim3(tiles), dim3(kSortThreads), 0, st, cand, kTile, 2LL, (long long)kTile);
    for (long long k = 2LL * kTile; k <= padded; k *= 2) {
      for (long long j = k / 2; j >= kTile; j /= 2)
        hipLaunchKernelGGL(rank_merge_kernel, dim3(mblocks), dim3(256), 0, st, cand, padded, k, j);
      hipLaunchKernelGGL(rank_tile_kernel, dim3(tiles), dim3(kSortThreads), 0, st, cand, kTile, k, k);
    }
  }
  hipLaunchKernelGGL(rank_out_kernel, dim3((m + 255) / 256), dim3(256), 0, st, cand, member, n, m, top_idx,
                     top_score, top_member);
  return hipGetLastError();
}

}  // namespace lg
