// scan_sort.hip -- device-wide exclusive scans and a stable LSD radix sort
// (4-bit digits), the integer building blocks of the partition tree and of
// the pair lists.  Stability of the sort is what makes the point order and
// the sorted pair lists bit-exact and reproducible.
#include <map>
#include <mutex>

#include "common.cuh"

namespace smash {

// Process-wide cache of idle device chunks (per device, best fit within
// twice the request), so repeated builds reuse memory without allocator
// calls.  Holds at most CACHE_CAP bytes; the rest is freed.
namespace {
constexpr size_t CACHE_CAP = (size_t)48 << 30;
struct ChunkCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<int, void *>> idle;  // size -> (device, base)
  size_t held = 0;
};
ChunkCache &chunk_cache() {
  static ChunkCache c;
  return c;
}
bool take_cached(int dev, size_t n, void **p, size_t *sz) {
  ChunkCache &c = chunk_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto it = c.idle.lower_bound(n); it != c.idle.end() && it->first <= 2 * n; ++it) {
    if (it->second.first != dev) continue;
    *p = it->second.second;
    *sz = it->first;
    c.held -= it->first;
    c.idle.erase(it);
    return true;
  }
  return false;
}
}  // namespace

void trim_chunk_cache(int dev) {
  ChunkCache &c = chunk_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto it = c.idle.begin(); it != c.idle.end();) {
    if (it->second.first == dev) {
      (void)hipFree(it->second.second);
      c.held -= it->first;
      it = c.idle.erase(it);
    } else {
      ++it;
    }
  }
}

namespace {
thread_local const AllocHooks *tl_hooks = nullptr;
thread_local MemAcct *tl_acct = nullptr;
}
const AllocHooks *current_hooks() { return tl_hooks; }
HooksScope::HooksScope(const AllocHooks *h) : prev(tl_hooks) {
  tl_hooks = (h && h->alloc && h->free) ? h : nullptr;
}
HooksScope::~HooksScope() { tl_hooks = prev; }
MemAcct *current_acct() { return tl_acct; }
AcctScope::AcctScope(MemAcct *a) : prev(tl_acct) { tl_acct = a; }
AcctScope::~AcctScope() { tl_acct = prev; }

void *DeviceArena::alloc(size_t n) {
  n = (n + 255) & ~(size_t)255;
  if (!bound) {
    hooks = current_hooks();
    acct = current_acct();
    bound = true;
  }
  if (n > left) {
    size_t sz = n > chunk ? n : chunk;
    void *p = nullptr;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hooks) {
      p = hooks->alloc(hooks->ctx, sz, (void *)stream);
      if (!p) throw Error{SMASH_E_OOM, "allocator hook returned NULL for " + std::to_string(sz) +
                                           " bytes"};
      if ((uintptr_t)p & 255) {
        hooks->free(hooks->ctx, p, sz, (void *)stream);
        throw Error{SMASH_E_INVALID_ARG, "allocator hook returned memory not aligned to 256 bytes"};
      }
    } else if (!take_cached(dev, sz, &p, &sz)) {
      hipError_t e = hipMallocAsync(&p, sz, stream);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw Error{SMASH_E_OOM, "device allocation of " + std::to_string(sz) + " bytes failed"};
      }
    }
    blocks.emplace_back(p, sz);
    if (acct) acct->add((int64_t)sz);
    cur = (char *)p;
    left = sz;
  }
  void *r = cur;
  cur += n;
  left -= n;
  bytes += (int64_t)n;
  return r;
}

void DeviceArena::release(bool idle) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  ChunkCache &c = chunk_cache();
  for (auto &b : blocks) {
    if (acct) acct->add(-(int64_t)b.second);
    if (hooks) {
      hooks->free(hooks->ctx, b.first, b.second, (void *)stream);
      continue;
    }
    bool kept = false;
    if (idle) {
      std::lock_guard<std::mutex> lk(c.mu);
      if (c.held + b.second <= CACHE_CAP) {
        c.idle.emplace(b.second, std::make_pair(dev, b.first));
        c.held += b.second;
        kept = true;
      }
    }
    if (!kept) (void)hipFreeAsync(b.first, stream);
  }
  blocks.clear();
  cur = nullptr;
  left = 0;
  bytes = 0;
}

void stream_wait(hipStream_t s) {
  int dev = 0;
  SMASH_HIP(hipGetDevice(&dev));
  thread_local std::vector<hipEvent_t> evs;
  if ((int)evs.size() <= dev) evs.resize(dev + 1, nullptr);
  if (!evs[dev]) SMASH_HIP(hipEventCreateWithFlags(&evs[dev], hipEventDisableTiming));
  SMASH_HIP(hipEventRecord(evs[dev], s));
  for (;;) {
    const hipError_t e = hipEventQuery(evs[dev]);
    if (e == hipSuccess) return;
    if (e != hipErrorNotReady) SMASH_HIP(e);
  }
}

struct PickArgs {
  const void *src[16];
  int bytes[16];
  int n;
  int64_t *dst;  // pinned host memory, written from the device
};

__global__ void k_pick(PickArgs A) {
  const int t = threadIdx.x;
  if (t < A.n)
    A.dst[t] = A.bytes[t] == 8 ? *(const int64_t *)A.src[t] : (int64_t)*(const int *)A.src[t];
  __threadfence_system();
}

int64_t *pick_words(hipStream_t s, std::initializer_list<std::pair<const void *, int>> items) {
  if (items.size() > 16) throw Error{SMASH_E_INVALID_ARG, "pick_words: at most 16 items"};
  int64_t *pin = pinned_words();
  PickArgs A{};
  A.n = 0;
  for (const auto &it : items) {
    A.src[A.n] = it.first;
    A.bytes[A.n] = it.second;
    A.n++;
  }
  A.dst = pin;
  k_pick<<<1, 64, 0, s>>>(A);
  SMASH_CHECK_LAUNCH();
  stream_wait(s);
  return pin;
}

int64_t *pinned_words() {
  thread_local int64_t *buf = nullptr;
  if (!buf) {
    void *p = nullptr;
    if (hipHostMalloc(&p, 64 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error{SMASH_E_OOM, "pinned host buffer allocation failed"};
    }
    buf = (int64_t *)p;
  }
  return buf;
}

__global__ void k_set_i64(int64_t *dev, int64_t v) { *dev = v; }

void set_i64(int64_t *dev, int64_t v, hipStream_t s) {
  k_set_i64<<<1, 1, 0, s>>>(dev, v);
  SMASH_CHECK_LAUNCH();
}

__global__ void k_copy_i64(int64_t *dst, const int64_t *src) { *dst = *src; }

void copy_i64(int64_t *dst, const int64_t *src, hipStream_t s) {
  k_copy_i64<<<1, 1, 0, s>>>(dst, src);
  SMASH_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ scan
constexpr int SC_NT = 256, SC_IT = 8, SC_TILE = SC_NT * SC_IT;

__global__ void __launch_bounds__(SC_NT) k_scan_reduce(const int64_t *in, int64_t n,
                                                       int64_t *bsum) {
  __shared__ int64_t lds[SC_NT / 64 + 1];
  int64_t b0 = (int64_t)blockIdx.x * SC_TILE;
  int64_t s = 0;
  for (int u = 0; u < SC_IT; u++) {
    int64_t i = b0 + (int64_t)threadIdx.x * SC_IT + u;
    if (i < n) s += in[i];
  }
  int64_t tot;
  block_excl_scan_i64(s, &tot, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of the block sums in one workgroup; writes out[n] = total
__global__ void __launch_bounds__(1024) k_scan_top(int64_t *bsum, int nb, const int64_t *base_dev,
                                                   int64_t *out, int64_t n) {
  __shared__ int64_t lds[1024 / 64 + 1];
  int per = (nb + 1023) / 1024;
  int b0 = threadIdx.x * per;
  int64_t s = 0;
  for (int u = 0; u < per; u++)
    if (b0 + u < nb) s += bsum[b0 + u];
  int64_t tot;
  int64_t ex = block_excl_scan_i64(s, &tot, lds);
  int64_t base = base_dev ? *base_dev : 0;
  ex += base;
  for (int u = 0; u < per; u++)
    if (b0 + u < nb) {
      int64_t v = bsum[b0 + u];
      bsum[b0 + u] = ex;
      ex += v;
    }
  if (threadIdx.x == 0) out[n] = base + tot;
}

__global__ void __launch_bounds__(SC_NT) k_scan_down(const int64_t *in, int64_t n,
                                                     const int64_t *bsum, int64_t *out) {
  __shared__ int64_t lds[SC_NT / 64 + 1];
  int64_t b0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_IT;
  int64_t v[SC_IT];
  int64_t s = 0;
  for (int u = 0; u < SC_IT; u++) {
    int64_t i = b0 + u;
    v[u] = i < n ? in[i] : 0;
    s += v[u];
  }
  int64_t tot;
  int64_t ex = block_excl_scan_i64(s, &tot, lds) + bsum[blockIdx.x];
  for (int u = 0; u < SC_IT; u++) {
    int64_t i = b0 + u;
    if (i < n) out[i] = ex;
    ex += v[u];
  }
}

// one workgroup for short arrays (most per-level scans): a single launch
constexpr int SC1_NT = 1024, SC1_IT = 8;
__global__ void __launch_bounds__(SC1_NT) k_scan_one(const int64_t *in, int64_t n,
                                                     const int64_t *base_dev, int64_t *out) {
  __shared__ int64_t lds[SC1_NT / 64 + 1];
  const int64_t b0 = (int64_t)threadIdx.x * SC1_IT;
  int64_t v[SC1_IT];
  int64_t sum = 0;
  for (int u = 0; u < SC1_IT; u++) {
    v[u] = b0 + u < n ? in[b0 + u] : 0;
    sum += v[u];
  }
  int64_t tot;
  int64_t ex = block_excl_scan_i64(sum, &tot, lds);
  const int64_t base = base_dev ? *base_dev : 0;
  ex += base;
  for (int u = 0; u < SC1_IT; u++) {
    if (b0 + u < n) out[b0 + u] = ex;
    ex += v[u];
  }
  if (threadIdx.x == 0) out[n] = base + tot;
}

void scan_i64(const int64_t *in, int64_t *out, int64_t n, const int64_t *base_dev,
              hipStream_t s, DeviceArena &tmp) {
  if (n <= (int64_t)SC1_NT * SC1_IT) {
    k_scan_one<<<1, SC1_NT, 0, s>>>(in, n, base_dev, out);
    SMASH_CHECK_LAUNCH();
    return;
  }
  int nb = n > 0 ? ceil_div(n, SC_TILE) : 0;
  int64_t *bsum = tmp.alloc_n<int64_t>(nb + 1);
  if (nb > 0) {
    k_scan_reduce<<<nb, SC_NT, 0, s>>>(in, n, bsum);
    SMASH_CHECK_LAUNCH();
  }
  k_scan_top<<<1, 1024, 0, s>>>(bsum, nb, base_dev, out, n);
  SMASH_CHECK_LAUNCH();
  if (nb > 0) {
    k_scan_down<<<nb, SC_NT, 0, s>>>(in, n, bsum, out);
    SMASH_CHECK_LAUNCH();
  }
}

// ------------------------------------------------------------------ radix sort
constexpr int RS_NT = 256, RS_IT = 8, RS_TILE = RS_NT * RS_IT, RS_R = 16;

__global__ void __launch_bounds__(RS_NT) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                   int ntiles, int *hist) {
  __shared__ int cnt[RS_R];
  if (threadIdx.x < RS_R) cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t b0 = (int64_t)blockIdx.x * RS_TILE;
  for (int u = 0; u < RS_IT; u++) {
    int64_t i = b0 + (int64_t)u * RS_NT + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (RS_R - 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x < RS_R) hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of the digit-major histogram (RS_R x ntiles), one workgroup
__global__ void __launch_bounds__(1024) k_rs_scan(int *hist, int total) {
  __shared__ int64_t lds[1024 / 64 + 1];
  int per = (total + 1023) / 1024;
  int b0 = threadIdx.x * per;
  int64_t s = 0;
  for (int u = 0; u < per; u++)
    if (b0 + u < total) s += hist[b0 + u];
  int64_t tot;
  int64_t ex = block_excl_scan_i64(s, &tot, lds);
  for (int u = 0; u < per; u++)
    if (b0 + u < total) {
      int v = hist[b0 + u];
      hist[b0 + u] = (int)ex;
      ex += v;
    }
}

// Each thread owns RS_IT consecutive elements of the tile, so tile order is
// (thread, item); ranks are (digit, thread, item)-ordered: stable.
__global__ void __launch_bounds__(RS_NT) k_rs_scatter(const uint64_t *kin, const int32_t *vin,
                                                      uint64_t *kout, int32_t *vout, int64_t n,
                                                      int shift, int ntiles, const int *hist) {
  __shared__ int cnt[RS_R * RS_NT];
  __shared__ int64_t lds[RS_NT / 64 + 1];
  __shared__ int dbase[RS_R];
  const int t = threadIdx.x;
  for (int r = 0; r < RS_R; r++) cnt[r * RS_NT + t] = 0;
  int64_t b0 = (int64_t)blockIdx.x * RS_TILE + (int64_t)t * RS_IT;
  uint64_t kk[RS_IT];
  int32_t vv[RS_IT];
  for (int u = 0; u < RS_IT; u++) {
    int64_t i = b0 + u;
    if (i < n) {
      kk[u] = kin[i];
      vv[u] = vin[i];
      cnt[((kk[u] >> shift) & (RS_R - 1)) * RS_NT + t]++;
    }
  }
  __syncthreads();
  // exclusive scan over cnt in (digit, thread) order; thread t owns entries
  // [t*RS_R, t*RS_R + RS_R) of the flattened array
  int loc[RS_R];
  int s = 0;
  for (int r = 0; r < RS_R; r++) {
    loc[r] = cnt[t * RS_R + r];
    s += loc[r];
  }
  int64_t tot;
  int64_t ex = block_excl_scan_i64(s, &tot, lds);
  __syncthreads();
  for (int r = 0; r < RS_R; r++) {
    cnt[t * RS_R + r] = (int)ex;
    ex += loc[r];
  }
  __syncthreads();
  // tile-local start of every digit: entry (digit, thread 0)
  if (t < RS_R) dbase[t] = hist[t * ntiles + blockIdx.x] - cnt[t * RS_NT];
  __syncthreads();
  for (int u = 0; u < RS_IT; u++) {
    int64_t i = b0 + u;
    if (i < n) {
      int dg = (int)((kk[u] >> shift) & (RS_R - 1));
      int pos = dbase[dg] + cnt[dg * RS_NT + t]++;
      kout[pos] = kk[u];
      vout[pos] = vv[u];
    }
  }
}

void radix_sort_u64(uint64_t *keys, int32_t *vals, uint64_t *keys_alt, int32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s, DeviceArena &tmp, int lo_bit) {
  if (n <= 1 || nbits <= lo_bit) return;
  int ntiles = ceil_div(n, RS_TILE);
  int *hist = tmp.alloc_n<int>((size_t)RS_R * ntiles);
  int passes = (nbits - lo_bit + 3) / 4;
  uint64_t *ka = keys, *kb = keys_alt;
  int32_t *va = vals, *vb = vals_alt;
  for (int ps = 0; ps < passes; ps++) {
    int shift = lo_bit + 4 * ps;
    k_rs_hist<<<ntiles, RS_NT, 0, s>>>(ka, n, shift, ntiles, hist);
    SMASH_CHECK_LAUNCH();
    k_rs_scan<<<1, 1024, 0, s>>>(hist, RS_R * ntiles);
    SMASH_CHECK_LAUNCH();
    k_rs_scatter<<<ntiles, RS_NT, 0, s>>>(ka, va, kb, vb, n, shift, ntiles, hist);
    SMASH_CHECK_LAUNCH();
    uint64_t *tk = ka;
    ka = kb;
    kb = tk;
    int32_t *tv = va;
    va = vb;
    vb = tv;
  }
  if (ka != keys) {
    SMASH_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
    SMASH_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace smash
