// HIP kernels of the DBL index for gfx950 (wave64) and their launch wrappers.
//
// Label record: every vertex owns 32 bytes {DL_in, BL_in, DL_out, BL_out} (Definitions 1 and
// 2, 64 bits each). Forward propagation reads and ORs the first 16 bytes along Suc; backward
// propagation the last 16 bytes along Pre, so one 16-byte access carries both labels of a
// direction and a query reads two 32-byte records.
//
// Propagation is the bit-parallel form of Algorithms 1 and 3: instead of one BFS per landmark
// or leaf bucket, every frontier vertex ORs its whole 128-bit direction label into each
// neighbour, and a neighbour whose label grew joins the next frontier. The labels reach the
// least fixpoint of "label(x) contains label(p) for every edge (p, x)" over the seeds, which is
// exactly what one BFS per bit computes; Algorithm 3's pruning (stop at a vertex that already
// holds the added bits) is the "did the OR change anything" test.
#include "dbl_internal.hpp"

namespace dbl {

using u64 = unsigned long long;

// ---------------------------------------------------------------- wave / block helpers

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ __forceinline__ u64 wave_incl_scan64(u64 x) {
  const uint32_t lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u64 y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint32_t lanemask_lt_popc(u64 mask) {
  const uint32_t lane = __lane_id();
  return (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

// Append `val` for every active lane with `pred` to q, reserving space with one atomic per wave.
__device__ __forceinline__ void wave_push(uint32_t *q, uint32_t *cnt, bool pred, uint32_t val) {
  const u64 mask = __ballot(pred);
  if (mask == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(mask);
  uint32_t base = 0;
  if (__lane_id() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
  base = __shfl(base, (int)leader, 64);
  if (pred) q[base + lanemask_lt_popc(mask)] = val;
}

// Neighbouring active lanes with the same target form a run; an active lane receives the first
// and last lane of its run. Counting into LDS with one atomic per run (by its last lane) keeps
// input sorted by key, where the lanes of a wave share a few counters, from serialising on
// them.
__device__ __forceinline__ void lane_run(uint32_t tgt, bool active, uint32_t &first,
                                         uint32_t &last) {
  const uint32_t lane = __lane_id();
  const uint32_t up = __shfl_up(tgt, 1, 64), dn = __shfl_down(tgt, 1, 64);
  const u64 act = __ballot(active);
  const bool head = active && (lane == 0 || !((act >> (lane - 1)) & 1ull) || up != tgt);
  const bool tail = active && (lane == 63 || !((act >> (lane + 1)) & 1ull) || dn != tgt);
  const u64 heads = __ballot(head) & (~0ull >> (63 - lane));
  const u64 tails = __ballot(tail) & (~0ull << lane);
  first = heads ? 63u - (uint32_t)__builtin_clzll(heads) : lane;
  last = tails ? (uint32_t)__builtin_ctzll(tails) : lane;
}

// ctr[idx] += 1 for every active lane, returning the old value plus the lane's place among the
// active lanes. When every active lane of the wave targets the same counter (sorted input) one
// atomic serves them all; otherwise each lane adds its own (the test costs two ballots and a
// lane read, less than forming runs when targets are scattered).
__device__ __forceinline__ uint32_t wave_add(uint32_t *ctr, uint32_t idx, bool active) {
  const u64 act = __ballot(active);
  if (act == 0) return 0;
  const uint32_t leader = (uint32_t)__builtin_ctzll(act);
  const uint32_t lead = __builtin_amdgcn_readlane(idx, leader);
  if (__ballot(active && idx != lead) == 0) {
    uint32_t old = 0;
    if (__lane_id() == leader) old = atomicAdd(&ctr[lead], (uint32_t)__popcll(act));
    return __builtin_amdgcn_readlane(old, leader) + lanemask_lt_popc(act);
  }
  return active ? atomicAdd(&ctr[idx], 1u) : 0u;
}

// Exclusive scan over a block of NT threads; *total receives the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *s_wsum,
                                                    uint32_t &total) {
  const uint32_t incl = wave_incl_scan(x);
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  if (lane == 63u) s_wsum[w] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; i++) {
    const uint32_t t = s_wsum[i];
    if ((uint32_t)i < w) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + incl - x;
}

// Queue appends staged in LDS: a block collects the appends of many tiles in s_buf (CAP
// entries, CAP >= NT) and writes them out with one atomic on the queue counter per flush
// instead of one per tile (atomics on one address are served one at a time, ~10 ns each).
// Every thread of the block must call both; *s_n starts at 0.
template <int NT>
__device__ __forceinline__ void stage_flush(uint32_t *q, uint32_t *cnt, uint32_t *s_buf,
                                            uint32_t *s_n, uint32_t *s_base) {
  const uint32_t k = *s_n;
  if (k == 0) return;
  if (threadIdx.x == 0) *s_base = atomicAdd(cnt, k);
  __syncthreads();
  const uint32_t base = *s_base;
  for (uint32_t i = threadIdx.x; i < k; i += NT) q[base + i] = s_buf[i];
  __syncthreads();
  if (threadIdx.x == 0) *s_n = 0;
  __syncthreads();
}

template <int NT, uint32_t CAP>
__device__ __forceinline__ void stage_push(uint32_t *q, uint32_t *cnt, bool pred, uint32_t val,
                                           uint32_t *s_buf, uint32_t *s_n, uint32_t *s_base,
                                           uint32_t *s_wsum) {
  static_assert(CAP >= (uint32_t)NT, "a tile must fit the stage");
  uint32_t total;
  const uint32_t ex = block_excl_scan<NT>(pred ? 1u : 0u, s_wsum, total);
  if (total == 0) return;
  if (*s_n + total > CAP) stage_flush<NT>(q, cnt, s_buf, s_n, s_base);
  if (pred) s_buf[*s_n + ex] = val;
  __syncthreads();
  if (threadIdx.x == 0) *s_n += total;
  __syncthreads();
}

__device__ __forceinline__ u64 ld_agent(const u64 *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One direction half of a vertex's label record: W words of DL, then W words of BL.
template <int W>
struct alignas(16) Half {
  u64 w[2 * W];
};

template <int W>
__device__ __forceinline__ const u64 *half_ptr(const u64 *lab, uint32_t x, uint32_t dir) {
  return lab + 4ull * W * x + 2u * W * dir;
}
template <int W>
__device__ __forceinline__ u64 *half_ptr(u64 *lab, uint32_t x, uint32_t dir) {
  return lab + 4ull * W * x + 2u * W * dir;
}

template <int W>
__device__ __forceinline__ Half<W> ld_half(const u64 *p) {
  Half<W> h;
#pragma unroll
  for (int i = 0; i < W; i++) {
    const ulonglong2 t = reinterpret_cast<const ulonglong2 *>(p)[i];
    h.w[2 * i] = t.x;
    h.w[2 * i + 1] = t.y;
  }
  return h;
}

// Device-coherent read of a half (past the L1 cache), for labels other waves of the same kernel
// may have grown.
template <int W>
__device__ __forceinline__ Half<W> ld_half_agent(const u64 *p) {
  Half<W> h;
#pragma unroll
  for (int i = 0; i < 2 * W; i++) h.w[i] = ld_agent(p + i);
  return h;
}

template <int W>
__device__ __forceinline__ bool any_bits(const Half<W> &h) {
  u64 a = 0;
#pragma unroll
  for (int i = 0; i < 2 * W; i++) a |= h.w[i];
  return a != 0ull;
}

// OR the half `a` into the half at w, given `cur`, an earlier plain read of w. Returns true if
// the call added a bit. The pre-read only avoids atomics on words that already hold the bits; a
// stale pre-read costs an extra atomic, never a missed change, because the decision uses the
// atomic's old value.
template <int W>
__device__ __forceinline__ bool or_half(u64 *__restrict__ w, const Half<W> &a, const Half<W> &cur) {
  bool changed = false;
#pragma unroll
  for (int i = 0; i < 2 * W; i++)
    if (a.w[i] & ~cur.w[i]) changed |= (a.w[i] & ~atomicOr(w + i, a.w[i])) != 0ull;
  return changed;
}

template <int W>
__device__ __forceinline__ bool relax(u64 *__restrict__ w, const Half<W> &a) {
  return or_half<W>(w, a, ld_half<W>(w));
}

// Launch kernel template `kern` instantiated for the label width `words` (1, 2 or 4).
#define DBL_LAUNCH_W(words, kern, grid, block, stream, ...)                                    \
  do {                                                                                         \
    switch (words) {                                                                           \
      case 1: hipLaunchKernelGGL(kern<1>, grid, block, 0, stream, __VA_ARGS__); break;         \
      case 2: hipLaunchKernelGGL(kern<2>, grid, block, 0, stream, __VA_ARGS__); break;         \
      case 4: hipLaunchKernelGGL(kern<4>, grid, block, 0, stream, __VA_ARGS__); break;         \
      default: return hipErrorInvalidValue;                                                    \
    }                                                                                          \
  } while (0)

// Claim the right to queue (vertex, direction) in the frontier stamped `stamp`. Stamps only
// grow, so a stale read can never equal `stamp` by accident.
__device__ __forceinline__ bool claim(uint32_t *slot, uint32_t stamp) {
  if (*slot == stamp) return false;
  return atomicExch(slot, stamp) != stamp;
}

// A pointer that is the same in every lane, held in scalar registers.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// r when sel is set, else f, chosen field by field from scalar copies of the (uniform)
// kernel-argument pointers, so a per-lane `sel` costs a select instead of per-lane loads of the
// pointers from argument memory.
__device__ __forceinline__ Csr pick_csr(const Csr &f, const Csr &r, bool sel) {
  Csr g;
  g.off = sel ? uniform_ptr(r.off) : uniform_ptr(f.off);
  g.deg = sel ? uniform_ptr(r.deg) : uniform_ptr(f.deg);
  g.cap = sel ? uniform_ptr(r.cap) : uniform_ptr(f.cap);
  g.col = sel ? uniform_ptr(r.col) : uniform_ptr(f.col);
  return g;
}

__device__ __forceinline__ uint32_t fib_bucket(uint32_t x, uint32_t bits) {
  return bits == 0 ? 0u : (uint32_t)(((u64)x * 0x9E3779B97F4A7C15ull) >> (64u - bits));
}

// ---------------------------------------------------------------- small utility kernels

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t count) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(u64 *p, u64 v, uint64_t count) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static uint32_t grid_for(uint64_t items, uint32_t per_block, uint32_t cap) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g == 0) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, value,
                     count);
  return hipGetLastError();
}

// *out += sum of a[0..count): per-block partial sums, one atomic per block.
__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t *a, uint64_t count, u64 *out) {
  __shared__ u64 s_w[4];
  u64 v = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * 256u)
    v += a[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (__lane_id() == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const u64 t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    if (t) atomicAdd(out, t);
  }
}

hipError_t launch_sum_u32(const uint32_t *a, uint64_t count, u64 *out, hipStream_t s) {
  hipError_t e = launch_fill_u64(out, 0ull, 1, s);
  if (e != hipSuccess || count == 0) return e;
  hipLaunchKernelGGL(k_sum_u32, dim3(grid_for(count, 256, 2048)), dim3(256), 0, s, a, count, out);
  return hipGetLastError();
}

// Read `bytes` of a buffer once (16-byte loads), so that it sits in the memory-side cache for
// the latency-bound work that follows; the OR of what was read goes to *sink so the loads stay.
__global__ __launch_bounds__(256) void k_touch(const ulonglong2 *p, uint64_t count, u64 *sink) {
  u64 acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * 256u) {
    const ulonglong2 v = p[i];
    acc |= v.x | v.y;
  }
  if (acc == 0x5DEECE66Dull) *sink = acc;  // practically never taken; keeps the loads
}

hipError_t launch_touch(const void *p, uint64_t bytes, u64 *sink, hipStream_t s) {
  const uint64_t count = bytes / 16;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_touch, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s,
                     (const ulonglong2 *)p, count, sink);
  return hipGetLastError();
}

hipError_t launch_fill_u64(u64 *p, u64 value, uint64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s, p, value,
                     count);
  return hipGetLastError();
}

__global__ void k_ctl_reset_query(Ctl *ctl) {
  ctl->und_count = 0;
  ctl->bfs_next = 0;
  ctl->bfs_heavy = 0;
}

hipError_t launch_ctl_reset_query(Ctl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_reset_query, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

__device__ __forceinline__ void st_sys32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// One thread copies the fields the host needs into the host mirror, then releases `seq`.
__device__ void publish_status(Ctl *ctl, Mirror *m, uint32_t seq) {
  st_sys32(&m->err, ld_agent32(&ctl->err));
  st_sys32(&m->cur, ld_agent32(&ctl->cur));
  st_sys32(&m->stamp, ld_agent32(&ctl->stamp));
  for (int i = 0; i < 3; i++) st_sys32(&m->fsize[i], ld_agent32(&ctl->fsize[i]));
  st_sys32(&m->ovf_count, ld_agent32(&ctl->ovf_count));
  st_sys32(&m->und_count, ld_agent32(&ctl->und_count));
  st_sys32(&m->bfs_heavy, ld_agent32(&ctl->bfs_heavy));
  st_sys32(&m->found, ld_agent32(&ctl->found));
  for (int i = 0; i < 4; i++)
    __hip_atomic_store(&m->dstat[i], ld_agent(&ctl->ctr[kCtrFrontEntries + i]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&m->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_publish(Ctl *ctl, Mirror *m, uint32_t seq) { publish_status(ctl, m, seq); }

hipError_t launch_publish(Ctl *ctl, Mirror *m, uint32_t seq, hipStream_t s) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, s, ctl, m, seq);
  return hipGetLastError();
}

// ---------------------------------------------------------------- ingest

__global__ void k_validate(const uint32_t *a, const uint32_t *b, uint64_t count, uint32_t n,
                           Ctl *ctl) {
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    bad |= (a[i] >= n) | (b[i] >= n);
  if (__ballot(bad) && __lane_id() == 0) atomicOr(&ctl->err, kErrRange);
}

hipError_t launch_validate_pairs(const uint32_t *a, const uint32_t *b, uint64_t count, uint32_t n,
                                 Ctl *ctl, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, a, b, count,
                     n, ctl);
  return hipGetLastError();
}

__device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// keep[e] = 1 for the first copy of each distinct non-loop edge (open-addressing hash set).
__global__ void k_dedup_mark(const uint32_t *src, const uint32_t *dst, uint64_t m, u64 *table,
                             uint64_t mask, uint8_t *keep, int assume_unique) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t a = src[e], b = dst[e];
    uint8_t k = 0;
    if (a != b) {
      if (assume_unique) {
        k = 1;
      } else {
        const u64 key = ((u64)a << 32) | b;
        uint64_t h = mix64(key) & mask;
        for (;;) {
          const u64 prev = atomicCAS(&table[h], ~0ull, key);
          if (prev == ~0ull) { k = 1; break; }
          if (prev == key) break;
          h = (h + 1) & mask;
        }
      }
    }
    keep[e] = k;
  }
}

hipError_t launch_dedup_mark(const uint32_t *src, const uint32_t *dst, uint64_t m, u64 *table,
                             uint64_t mask, uint8_t *keep, int assume_unique, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dedup_mark, dim3(grid_for(m, 256, 16384)), dim3(256), 0, s, src, dst, m,
                     table, mask, keep, assume_unique);
  return hipGetLastError();
}


__global__ void k_slack_cap(const uint32_t *deg, uint32_t *cap, uint32_t n, float frac,
                            uint32_t smin) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    const uint32_t d = deg[x];
    uint32_t sl = (uint32_t)ceilf(frac * (float)d);
    if (sl < smin) sl = smin;
    cap[x] = d + sl;
  }
}

hipError_t launch_slack_cap(const uint32_t *deg, uint32_t *cap, uint32_t n, float frac,
                            uint32_t smin, hipStream_t s) {
  hipLaunchKernelGGL(k_slack_cap, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, deg, cap, n,
                     frac, smin);
  return hipGetLastError();
}

// ---- exclusive scan (uint32 -> uint64), three phases
constexpr uint32_t kScanNT = 256, kScanIT = 8, kScanTile = kScanNT * kScanIT;

uint64_t scan_tmp_words(uint32_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ __launch_bounds__(kScanNT) void k_scan_local(const uint32_t *in, u64 *out, uint32_t n,
                                                        u64 *block_sums) {
  __shared__ u64 s_w[kScanNT / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanIT;
  uint32_t v[kScanIT];
  u64 sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanIT; j++) {
    v[j] = (base + j < n) ? in[base + j] : 0u;
    sum += v[j];
  }
  const u64 incl = wave_incl_scan64(sum);
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  if (lane == 63u) s_w[w] = incl;
  __syncthreads();
  u64 off = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanNT / 64; i++) {
    if (i < w) off += s_w[i];
    tot += s_w[i];
  }
  u64 run = off + incl - sum;
#pragma unroll
  for (uint32_t j = 0; j < kScanIT; j++) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(u64 *sums, uint32_t nb, u64 *total) {
  __shared__ u64 s_w[16];
  __shared__ u64 s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const u64 x = i < nb ? sums[i] : 0ull;
    const u64 incl = wave_incl_scan64(x);
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    if (lane == 63u) s_w[w] = incl;
    __syncthreads();
    u64 off = 0, tot = 0;
    for (uint32_t j = 0; j < 16; j++) {
      if (j < w) off += s_w[j];
      tot += s_w[j];
    }
    const u64 carry = s_carry;
    if (i < nb) sums[i] = carry + off + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s_carry;
}

__global__ __launch_bounds__(kScanNT) void k_scan_add(u64 *out, uint32_t n, const u64 *sums) {
  const u64 add = sums[blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  for (uint32_t j = threadIdx.x; j < kScanTile; j += kScanNT)
    if (base + j < n) out[base + j] += add;
}

hipError_t scan_exclusive(const uint32_t *in, u64 *out, uint32_t n, u64 *tmp, u64 *total,
                          hipStream_t s) {
  const uint32_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanNT), 0, s, in, out, n, tmp);
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, nb, total);
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanNT), 0, s, out, n, tmp);
  }
  return hipGetLastError();
}

// ---- binned ingest
// Scattering edges straight into rows costs one random atomic and one random store per edge
// and direction, spread over the whole graph. Instead the kept edges of one direction are first
// partitioned by key range (bin = key >> shift, at most kMaxBins bins, each bin's edges
// contiguous and bins in increasing key order); degree counts and row fills then walk the
// partitioned edges in order, so the atomics and stores of neighbouring threads fall into the
// rows of one or two bins at a time, a window that stays in cache.
constexpr uint32_t kMaxBins = 4096;
// One workgroup per bin counts degrees and fills rows in LDS while a bin spans at most kBinVerts
// vertices (see k_bin_deg).
constexpr uint32_t kBinVerts = 16384, kBinNT = 1024;
static_assert(kBinVerts == kBinVertsMax, "bin width of the LDS kernels");

// The fewest bins of at most kMaxBins: narrow bins keep the row writes of k_bin_fill within a
// small window of the rows.
uint32_t bin_shift(uint32_t n) {
  uint32_t sh = 0;
  while (((uint64_t)(n - 1) >> sh) >= kMaxBins) sh++;
  return sh;
}

// counts[bin * nblk + b]: kept edges of block b's chunk whose key falls in `bin` (bin-major, so
// one exclusive scan over the array gives every (bin, block) its output offset)
// Every thread walks its part of the chunk kBinUnroll edges at a time: all their loads are
// issued before the first LDS update, so a wave keeps that many reads in flight.
// runs[0..1] (zero on entry) sample how far the input is grouped by key: over the first edge
// of every thread's group of kBinUnroll (lanes 1..63), runs[1] counts the kept ones and runs[0]
// those whose key equals the key of the input edge before them.
constexpr uint32_t kBinUnroll = 8;

__global__ __launch_bounds__(256) void k_bin_hist(const uint32_t *__restrict__ key,
                                                  const uint8_t *__restrict__ keep, uint64_t m,
                                                  uint32_t shift, uint32_t nbins, uint64_t chunk,
                                                  uint32_t *__restrict__ counts,
                                                  u64 *__restrict__ runs) {
  __shared__ uint32_t hist[kMaxBins];
  __shared__ uint32_t s_runs[2];
  for (uint32_t i = threadIdx.x; i < nbins; i += 256u) hist[i] = 0;
  if (threadIdx.x < 2) s_runs[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lo = blockIdx.x * chunk, hi = min(m, lo + chunk);
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t same = 0, sampled = 0;
  for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += 256u * kBinUnroll) {
    uint32_t k[kBinUnroll];
    bool ok[kBinUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kBinUnroll; j++) {
      const uint64_t e = e0 + 256u * j;
      ok[j] = e < hi;
      k[j] = ok[j] ? key[e] : 0u;
      ok[j] = ok[j] && keep[e];
    }
    {
      const uint32_t prev = __shfl_up(k[0], 1);  // the input edge before, for lanes 1..63
      if (lane && ok[0]) {
        sampled++;
        same += prev == k[0];
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kBinUnroll; j++) (void)wave_add(hist, k[j] >> shift, ok[j]);
  }
  for (uint32_t o = 32; o; o >>= 1) {
    same += __shfl_xor(same, o);
    sampled += __shfl_xor(sampled, o);
  }
  if (lane == 0 && sampled) {
    atomicAdd(&s_runs[0], same);
    atomicAdd(&s_runs[1], sampled);
  }
  __syncthreads();
  if (threadIdx.x < 2 && s_runs[threadIdx.x])
    atomicAdd(&runs[threadIdx.x], (u64)s_runs[threadIdx.x]);
  for (uint32_t i = threadIdx.x; i < nbins; i += 256u)
    counts[(uint64_t)i * gridDim.x + blockIdx.x] = hist[i];
}

// out[pos] = key << 32 | val for every kept edge, grouped by bin (order inside a bin is
// arbitrary). Each block sorts its chunk by bin one tile of kScatTile edges at a time in LDS
// (rank by LDS atomic, exclusive scan of the tile's bin counts) and writes the tile out in
// sorted order: consecutive threads write consecutive slots of one bin's run, so the output is
// written in runs instead of one scattered 8-byte store per edge.
constexpr uint32_t kScatNT = 512, kScatPer = 24, kScatTile = kScatNT * kScatPer;

__global__ __launch_bounds__(kScatNT) void k_bin_scatter(const uint32_t *__restrict__ key,
                                                         const uint32_t *__restrict__ val,
                                                         const uint8_t *__restrict__ keep,
                                                         uint64_t m, uint32_t shift,
                                                         uint32_t nbins, uint64_t chunk,
                                                         const u64 *__restrict__ offs,
                                                         u64 *__restrict__ out) {
  __shared__ u64 s_item[kScatTile];
  __shared__ u64 s_cur[kMaxBins];      // next output slot of each bin for this block
  __shared__ uint32_t s_pos[kMaxBins];  // tile counts, then their exclusive scan
  __shared__ uint32_t s_wsum[kScatNT / 64];
  const uint32_t t = threadIdx.x;
  constexpr uint32_t kPerT = (kMaxBins + kScatNT - 1) / kScatNT;  // bins per thread in the scan
  for (uint32_t i = t; i < nbins; i += kScatNT) {
    s_cur[i] = offs[(uint64_t)i * gridDim.x + blockIdx.x];
    s_pos[i] = 0;
  }
  __syncthreads();
  const uint64_t lo = blockIdx.x * chunk, hi = min(m, lo + chunk);
  for (uint64_t base = lo; base < hi; base += kScatTile) {
    u64 item[kScatPer];
    uint32_t rank[kScatPer];
    bool ok[kScatPer];
#pragma unroll
    for (uint32_t j = 0; j < kScatPer; j++) {
      const uint64_t e = base + kScatNT * j + t;
      ok[j] = e < hi;
      item[j] = ok[j] ? ((u64)__builtin_nontemporal_load(&key[e]) << 32) |
                            __builtin_nontemporal_load(&val[e])
                      : 0ull;
      ok[j] = ok[j] && __builtin_nontemporal_load(&keep[e]);
    }
#pragma unroll
    for (uint32_t j = 0; j < kScatPer; j++)
      rank[j] = wave_add(s_pos, (uint32_t)(item[j] >> 32) >> shift, ok[j]);
    __syncthreads();
    // exclusive scan of the tile's counts over the bins (thread t owns bins [t*kPerT, ...))
    uint32_t c[kPerT], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPerT; k++) {
      const uint32_t b = t * kPerT + k;
      c[k] = b < nbins ? s_pos[b] : 0u;
      sum += c[k];
    }
    uint32_t total;
    uint32_t run = block_excl_scan<kScatNT>(sum, s_wsum, total);
#pragma unroll
    for (uint32_t k = 0; k < kPerT; k++) {
      const uint32_t b = t * kPerT + k;
      if (b < nbins) s_pos[b] = run;
      run += c[k];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kScatPer; j++)
      if (ok[j]) s_item[s_pos[(uint32_t)(item[j] >> 32) >> shift] + rank[j]] = item[j];
    __syncthreads();
    for (uint32_t p = t; p < total; p += kScatNT) {
      const u64 x = s_item[p];
      const uint32_t b = (uint32_t)(x >> 32) >> shift;
      out[s_cur[b] + (p - s_pos[b])] = x;
    }
    __syncthreads();
    for (uint32_t b = t; b < nbins; b += kScatNT) {
      const uint32_t end = b + 1 < nbins ? s_pos[b + 1] : total;
      s_cur[b] += end - s_pos[b];
    }
    __syncthreads();
    for (uint32_t b = t; b < nbins; b += kScatNT) s_pos[b] = 0;
    __syncthreads();
  }
}

hipError_t launch_bin_edges(const uint32_t *key, const uint32_t *val, const uint8_t *keep,
                            uint64_t m, uint32_t n, uint32_t nblk, uint32_t *counts, u64 *offs,
                            u64 *scan_tmp, u64 *kept, u64 *runs, u64 *out, hipStream_t s) {
  if (m == 0 || nblk == 0) return hipErrorInvalidValue;
  const uint32_t shift = bin_shift(n), nbins = ((n - 1) >> shift) + 1;
  const uint64_t chunk = (m + nblk - 1) / nblk;
  hipError_t e = launch_fill_u64(runs, 0ull, 2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_hist, dim3(nblk), dim3(256), 0, s, key, keep, m, shift, nbins, chunk,
                     counts, runs);
  e = scan_exclusive(counts, offs, nbins * nblk, scan_tmp, kept, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_scatter, dim3(nblk), dim3(kScatNT), 0, s, key, val, keep, m, shift,
                     nbins, chunk, offs, out);
  return hipGetLastError();
}

// One workgroup per bin (while a bin spans at most kBinVerts vertices): the bin's edges are
// contiguous, so degrees and row cursors are counted in LDS, degrees are written in order and
// row writes stay within the bin's rows; no global atomics.

__device__ __forceinline__ void bin_range(const u64 *offs, uint32_t nblk, uint32_t nbins,
                                          u64 kept, uint32_t bin, u64 &lo, u64 &hi) {
  lo = offs[(uint64_t)bin * nblk];
  hi = bin + 1 < nbins ? offs[(uint64_t)(bin + 1) * nblk] : kept;
}

__global__ __launch_bounds__(kBinNT) void k_bin_deg(const u64 *__restrict__ edges,
                                                    const u64 *__restrict__ offs, uint32_t nblk,
                                                    uint32_t nbins, uint32_t shift,
                                                    const u64 *__restrict__ kept, uint32_t n,
                                                    uint32_t *__restrict__ deg, u64 long_min) {
  __shared__ uint32_t cnt[kBinVerts];
  for (uint32_t bin = blockIdx.x; bin < nbins; bin += gridDim.x) {
    const uint32_t first = bin << shift, nv = min(1u << shift, n - first);
    u64 lo, hi;
    bin_range(offs, nblk, nbins, *kept, bin, lo, hi);
    if (hi - lo >= long_min) continue;  // a long bin: k_bin_deg_long
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT) cnt[i] = 0;
    __syncthreads();
    for (u64 e0 = lo + threadIdx.x; e0 < hi; e0 += kBinNT * 4u) {
      uint32_t k[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        const u64 e = e0 + kBinNT * j;
        k[j] = e < hi ? (uint32_t)(edges[e] >> 32) : ~0u;
      }
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        const bool ok = k[j] != ~0u;
        uint32_t f, l;
        lane_run(k[j], ok, f, l);
        if (ok && __lane_id() == l) atomicAdd(&cnt[k[j] - first], l - f + 1u);
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT) deg[first + i] = cnt[i];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBinNT) void k_bin_fill(const u64 *__restrict__ edges,
                                                     const u64 *__restrict__ offs, uint32_t nblk,
                                                     uint32_t nbins, uint32_t shift,
                                                     const u64 *__restrict__ kept, uint32_t n,
                                                     Csr g, u64 long_min) {
  __shared__ uint32_t cur[kBinVerts];
  for (uint32_t bin = blockIdx.x; bin < nbins; bin += gridDim.x) {
    const uint32_t first = bin << shift, nv = min(1u << shift, n - first);
    u64 lo, hi;
    bin_range(offs, nblk, nbins, *kept, bin, lo, hi);
    if (hi - lo >= long_min) continue;  // a long bin: k_bin_fill_long
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT) cur[i] = 0;
    __syncthreads();
    for (u64 e0 = lo + threadIdx.x; e0 < hi; e0 += kBinNT * 4u) {
      u64 kv[4];
      u64 o[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        const u64 e = e0 + kBinNT * j;
        kv[j] = e < hi ? __builtin_nontemporal_load(&edges[e]) : ~0ull;
      }
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        o[j] = kv[j] != ~0ull ? g.off[(uint32_t)(kv[j] >> 32)] : 0ull;
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        if (kv[j] != ~0ull) {
          const uint32_t k = (uint32_t)(kv[j] >> 32);
          const uint32_t p = atomicAdd(&cur[k - first], 1u);
          g.col[o[j] + p] = (uint32_t)kv[j];
        }
    }
    __syncthreads();
  }
}

// Row fill through LDS, for bins of at most kFillVerts vertices. A bin's rows are cut into
// sub-bins by where each row starts (a new sub-bin every kFillSub column slots); the bin's edges
// are first regrouped by sub-bin into tmp (same index range as the bin), then each sub-bin's rows
// are assembled in LDS and written out as one contiguous run of columns, slack included (slack
// slots are never read, so they carry whatever the stage held). Row cursors start at the row's offset from the bin's first column, so
// the fill itself reads no offsets. A sub-bin whose rows span more than kFillStage slots (a long
// row) is filled directly. Whatever order the bin's edges arrive in, the columns reach memory in
// whole runs.
constexpr uint32_t kFillVerts = 8192, kFillSub = 4096, kFillStage = 8192, kFillMaxSub = 256;
constexpr uint32_t kFillTile = kBinNT * 4;  // edges regrouped at a time (fills the stage as u64)
static_assert(kFillTile * sizeof(u64) <= kFillStage * sizeof(uint32_t), "tile exceeds the stage");
static_assert(kFillTile <= 65536 && kFillMaxSub <= 65536, "packed sub-bin and rank");

// two workgroups per compute unit (8 waves per SIMD): at most 64 VGPRs
__global__ __launch_bounds__(kBinNT, 8) void k_bin_fill_staged(const u64 *__restrict__ edges,
                                                            const u64 *__restrict__ offs,
                                                            uint32_t nblk, uint32_t nbins,
                                                            uint32_t shift,
                                                            const u64 *__restrict__ kept,
                                                            uint32_t n, Csr g,
                                                            u64 *__restrict__ tmp,
                                                            u64 long_min) {
  __shared__ uint32_t cur[kFillVerts];
  __shared__ uint32_t stage[kFillStage];
  __shared__ uint8_t sbid[kFillVerts];
  __shared__ uint32_t sbcnt[kFillMaxSub], sbstart[kFillMaxSub], sbcur[kFillMaxSub];
  __shared__ uint32_t sbfirst[kFillMaxSub + 1];
  __shared__ uint32_t sbrow[kFillMaxSub + 1];  // column (from the bin's first) of sbfirst's row
  __shared__ uint32_t tcnt[kFillMaxSub], tpos[kFillMaxSub];  // per tile of the regrouping
  __shared__ uint32_t s_wsum[kBinNT / 64];
  const uint32_t t = threadIdx.x;
  for (uint32_t bin = blockIdx.x; bin < nbins; bin += gridDim.x) {
    const uint32_t first = bin << shift, nv = min(1u << shift, n - first);
    {
      u64 lo, hi;
      bin_range(offs, nblk, nbins, *kept, bin, lo, hi);
      if (hi - lo >= long_min) continue;  // a long bin: k_bin_fill_long
    }
    const u64 base = g.off[first];
    const u64 span = g.off[first + nv - 1] + g.cap[first + nv - 1] - base;
    const uint32_t nsb =
        (uint32_t)max<u64>(1, min<u64>(kFillMaxSub, (span + kFillSub - 1) / kFillSub));
    for (uint32_t i = t; i <= kFillMaxSub; i += kBinNT) {
      if (i < kFillMaxSub) {
        sbcnt[i] = 0;
        sbcur[i] = 0;
        tcnt[i] = 0;
      }
      sbfirst[i] = nv;
    }
    __syncthreads();
    // per row: cursor, sub-bin; per sub-bin: edge count and first row
    for (uint32_t v = t; v < nv; v += kBinNT) {
      const uint32_t rel = (uint32_t)(g.off[first + v] - base);
      cur[v] = rel;
      const uint32_t sb = min(nsb - 1u, rel / kFillSub);
      sbid[v] = (uint8_t)sb;
      const uint32_t d = g.deg[first + v];
      if (d) atomicAdd(&sbcnt[sb], d);
      atomicMin(&sbfirst[sb], v);
    }
    __syncthreads();
    if (t == 0) {
      // exclusive scan of the counts; a sub-bin where no row starts takes the next one's first
      // row, so every sub-bin's rows are [sbfirst[sb], sbfirst[sb + 1])
      uint32_t acc = 0;
      for (uint32_t sb = 0; sb < nsb; sb++) {
        sbstart[sb] = acc;
        acc += sbcnt[sb];
      }
      for (uint32_t sb = nsb; sb-- > 1;)
        sbfirst[sb - 1] = min(sbfirst[sb - 1], sbfirst[sb]);
      for (uint32_t sb = 0; sb <= nsb; sb++)
        sbrow[sb] = sbfirst[sb] < nv ? cur[sbfirst[sb]] : (uint32_t)span;
    }
    __syncthreads();
    u64 lo, hi;
    bin_range(offs, nblk, nbins, *kept, bin, lo, hi);
    // regroup by sub-bin one tile of kFillTile edges at a time: rank each edge within its
    // sub-bin by LDS atomic, scan the tile's sub-bin counts, sort the tile in the (still idle)
    // stage and write it out, so that each sub-bin's edges of the tile leave as one run
    u64 *const s_tile = reinterpret_cast<u64 *>(stage);
    uint32_t run = 0;  // thread sb < nsb: edges of sub-bin sb written so far
    for (u64 e0 = lo; e0 < hi; e0 += kFillTile) {
      u64 kv[4];
      uint32_t sr[4];  // sub-bin << 16 | rank within the tile (rank < kFillTile <= 2^16)
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        const u64 e = e0 + t + kBinNT * j;
        kv[j] = e < hi ? __builtin_nontemporal_load(&edges[e]) : ~0ull;
      }
#pragma unroll
      for (uint32_t j = 0; j < 4; j++) {
        sr[j] = 0;
        if (kv[j] != ~0ull) {
          const uint32_t s = sbid[(uint32_t)(kv[j] >> 32) - first];
          sr[j] = s << 16 | atomicAdd(&tcnt[s], 1u);
        }
      }
      __syncthreads();
      const uint32_t c = t < nsb ? tcnt[t] : 0u;
      uint32_t n_tile;
      const uint32_t ex = block_excl_scan<kBinNT>(c, s_wsum, n_tile);
      if (t < nsb) {
        tcnt[t] = 0;
        tpos[t] = ex;
        sbcur[t] = run;
        run += c;
      }
      __syncthreads();
#pragma unroll
      for (uint32_t j = 0; j < 4; j++)
        if (kv[j] != ~0ull) s_tile[tpos[sr[j] >> 16] + (sr[j] & 0xFFFFu)] = kv[j];
      __syncthreads();
      for (uint32_t p = t; p < n_tile; p += kBinNT) {
        const u64 x = s_tile[p];
        const uint32_t s = sbid[(uint32_t)(x >> 32) - first];
        tmp[lo + sbstart[s] + sbcur[s] + (p - tpos[s])] = x;
      }
      __syncthreads();
    }
    for (uint32_t sb = 0; sb < nsb; sb++) {
      if (sbfirst[sb] >= sbfirst[sb + 1]) continue;  // no row starts here (same for every thread)
      const uint32_t r0 = sbrow[sb], r1 = sbrow[sb + 1];
      const u64 e_lo = lo + sbstart[sb], e_hi = e_lo + sbcnt[sb];
      if (r1 - r0 <= kFillStage) {
        for (u64 e0 = e_lo + t; e0 < e_hi; e0 += kBinNT * 4u) {
          u64 kv[4];
#pragma unroll
          for (uint32_t j = 0; j < 4; j++) {
            const u64 e = e0 + kBinNT * j;
            kv[j] = e < e_hi ? tmp[e] : ~0ull;
          }
#pragma unroll
          for (uint32_t j = 0; j < 4; j++)
            if (kv[j] != ~0ull)
              stage[atomicAdd(&cur[(uint32_t)(kv[j] >> 32) - first], 1u) - r0] = (uint32_t)kv[j];
        }
        __syncthreads();
        for (uint32_t i = t; i < r1 - r0; i += kBinNT) g.col[base + r0 + i] = stage[i];
      } else {
        for (u64 e = e_lo + t; e < e_hi; e += kBinNT) {
          const u64 kv = tmp[e];
          g.col[base + atomicAdd(&cur[(uint32_t)(kv >> 32) - first], 1u)] = (uint32_t)kv;
        }
      }
      __syncthreads();
    }
    // the sub-bin table is rebuilt for the next bin only once every thread has walked it to the
    // end (trailing sub-bins where no row starts pass no barrier)
    __syncthreads();
  }
}

// out[b] = offs[b * nblk]: where each bin's edges start (for the host's long-bin test)
__global__ void k_bin_starts(const u64 *offs, uint32_t nblk, uint32_t nbins, u64 *out) {
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nbins; b += gridDim.x * blockDim.x)
    out[b] = offs[(uint64_t)b * nblk];
}

hipError_t launch_bin_starts(const u64 *offs, uint32_t nblk, uint32_t nbins, u64 *out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_bin_starts, dim3(grid_for(nbins, 256, 64)), dim3(256), 0, s, offs, nblk,
                     nbins, out);
  return hipGetLastError();
}

// Long bins. One workgroup per bin serialises a bin that holds far more than its share of the
// edges (ids numbered so that the high-degree vertices share a few ranges). Such a bin is cut
// into chunks of its edges, each taken by a workgroup of its own: a chunk counts its keys in LDS
// and adds the counts to the (zeroed) global degrees; for the fill, it counts again, reserves
// each row's share with one global atomic per row on the bin's cursor table (zeroed), and writes
// its edges from those bases with LDS cursors.

__global__ __launch_bounds__(kBinNT) void k_bin_deg_long(const u64 *__restrict__ edges,
                                                         const LongChunk *__restrict__ chunks,
                                                         uint32_t nchunks, uint32_t shift,
                                                         uint32_t n, uint32_t *__restrict__ deg) {
  __shared__ uint32_t cnt[kBinVerts];
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const LongChunk ch = chunks[c];
    const uint32_t first = ch.bin << shift, nv = min(1u << shift, n - first);
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT) cnt[i] = 0;
    __syncthreads();
    for (u64 e = ch.lo + threadIdx.x; e < ch.hi; e += kBinNT) {
      const uint32_t k = (uint32_t)(__builtin_nontemporal_load(&edges[e]) >> 32);
      uint32_t f, l;
      lane_run(k, true, f, l);
      if (__lane_id() == l) atomicAdd(&cnt[k - first], l - f + 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT)
      if (cnt[i]) atomicAdd(&deg[first + i], cnt[i]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBinNT) void k_bin_fill_long(const u64 *__restrict__ edges,
                                                          const LongChunk *__restrict__ chunks,
                                                          uint32_t nchunks, uint32_t shift,
                                                          uint32_t n, Csr g,
                                                          uint32_t *__restrict__ cursors) {
  __shared__ uint32_t cur[kBinVerts];
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const LongChunk ch = chunks[c];
    const uint32_t first = ch.bin << shift, nv = min(1u << shift, n - first);
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT) cur[i] = 0;
    __syncthreads();
    for (u64 e = ch.lo + threadIdx.x; e < ch.hi; e += kBinNT) {
      const uint32_t k = (uint32_t)(edges[e] >> 32);
      uint32_t f, l;
      lane_run(k, true, f, l);
      if (__lane_id() == l) atomicAdd(&cur[k - first], l - f + 1u);
    }
    __syncthreads();
    // this chunk's part of each row starts where the chunks before it (in any order) ended
    uint32_t *bc = cursors + (uint64_t)ch.slot * kBinVerts;
    for (uint32_t i = threadIdx.x; i < nv; i += kBinNT)
      if (cur[i]) cur[i] = atomicAdd(&bc[i], cur[i]);
    __syncthreads();
    for (u64 e = ch.lo + threadIdx.x; e < ch.hi; e += kBinNT) {
      const u64 kv = __builtin_nontemporal_load(&edges[e]);
      const uint32_t k = (uint32_t)(kv >> 32);
      // neighbouring lanes with the same row (long rows fill whole waves) take their slots
      // with one LDS atomic per run, made by the run's last lane
      uint32_t f, l;
      lane_run(k, true, f, l);
      uint32_t old = 0;
      if (__lane_id() == l) old = atomicAdd(&cur[k - first], l - f + 1u);
      const uint32_t base = __shfl(old, (int)l, 64);
      g.col[g.off[k] + base + (__lane_id() - f)] = (uint32_t)kv;
    }
    __syncthreads();
  }
}

// Degrees (deg[key] = edges of key) and row fill of partitioned edges. Rows are filled from
// position 0; deg is left as the degree. With fill_tmp (kept_host entries, and every row of the
// CSR within 2^32 column slots of its bin's first row) the fill goes through LDS. Bins of at
// least long_min edges are skipped by the per-bin kernels and handled in the chunks of `chunks`
// (nchunks entries, device memory): for the degrees, deg must then be zero on entry; for the
// fill, `cursors` holds kBinVerts zeroed words per long bin.
hipError_t launch_bin_rows(const u64 *edges, const u64 *offs, uint32_t nblk, uint32_t n,
                           const u64 *kept, uint64_t kept_host, uint32_t *deg, const Csr *g,
                           u64 *fill_tmp, u64 long_min, const LongChunk *chunks,
                           uint32_t nchunks, uint32_t *cursors, hipStream_t s) {
  const uint32_t shift = bin_shift(n), nbins = ((n - 1) >> shift) + 1;
  if ((1u << shift) <= kBinVerts) {
    const uint32_t grid = min(nbins, 8192u);
    const uint32_t cgrid = min(nchunks, 8192u);
    if (!g) {
      hipLaunchKernelGGL(k_bin_deg, dim3(grid), dim3(kBinNT), 0, s, edges, offs, nblk, nbins,
                         shift, kept, n, deg, long_min);
      if (nchunks)
        hipLaunchKernelGGL(k_bin_deg_long, dim3(cgrid), dim3(kBinNT), 0, s, edges, chunks,
                           nchunks, shift, n, deg);
    } else {
      if (fill_tmp && (1u << shift) <= kFillVerts) {
        hipLaunchKernelGGL(k_bin_fill_staged, dim3(grid), dim3(kBinNT), 0, s, edges, offs, nblk,
                           nbins, shift, kept, n, *g, fill_tmp, long_min);
      } else {
        hipLaunchKernelGGL(k_bin_fill, dim3(grid), dim3(kBinNT), 0, s, edges, offs, nblk, nbins,
                           shift, kept, n, *g, long_min);
      }
      if (nchunks)
        hipLaunchKernelGGL(k_bin_fill_long, dim3(cgrid), dim3(kBinNT), 0, s, edges, chunks,
                           nchunks, shift, n, *g, cursors);
    }
    return hipGetLastError();
  }
  // very large vertex counts: bins too wide for LDS counters, count with global atomics
  hipError_t e;
  if (!g) {
    e = launch_fill_u32(deg, 0u, n, s);
    if (e == hipSuccess) e = launch_deg_binned(edges, kept_host, deg, s);
    return e;
  }
  e = launch_fill_u32(g->deg, 0u, n, s);
  if (e == hipSuccess) e = launch_fill_binned(edges, kept_host, *g, s);
  return e;
}

__global__ __launch_bounds__(256) void k_deg_binned(const u64 *edges, uint64_t cnt,
                                                    uint32_t *deg) {
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < cnt; e += gridDim.x * 256ull)
    atomicAdd(&deg[(uint32_t)(edges[e] >> 32)], 1u);
}

hipError_t launch_deg_binned(const u64 *edges, uint64_t cnt, uint32_t *deg, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_deg_binned, dim3(grid_for(cnt, 256, 4096)), dim3(256), 0, s, edges, cnt,
                     deg);
  return hipGetLastError();
}

// g.deg must be zero: it is counted up again while the rows fill
__global__ __launch_bounds__(256) void k_fill_binned(const u64 *edges, uint64_t cnt, Csr g) {
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < cnt; e += gridDim.x * 256ull) {
    const u64 kv = edges[e];
    const uint32_t k = (uint32_t)(kv >> 32);
    const uint32_t p = atomicAdd(&g.deg[k], 1u);
    g.col[g.off[k] + p] = (uint32_t)kv;
  }
}

hipError_t launch_fill_binned(const u64 *edges, uint64_t cnt, Csr g, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_binned, dim3(grid_for(cnt, 256, 4096)), dim3(256), 0, s, edges, cnt,
                     g);
  return hipGetLastError();
}

// ---------------------------------------------------------------- landmark selection
// Tiles of 2048 candidates are bitonic-sorted in LDS by (M descending, id ascending); the best
// `keep` (64, or 256 when k > 64) of each tile survive to the next pass until one tile remains.
constexpr uint32_t kTkTile = 2048, kTkNT = 256, kTkKeepMax = kMaxLabelBits;

uint64_t topk_tmp_entries(uint32_t n) {
  const uint64_t tiles = ((uint64_t)n + kTkTile - 1) / kTkTile;
  return 2 * (tiles * kTkKeepMax + kTkKeepMax);
}

__global__ __launch_bounds__(kTkNT) void k_topk(const uint32_t *indeg, const uint32_t *outdeg,
                                                const u64 *in_m, const uint32_t *in_id,
                                                uint64_t count, uint32_t rank, uint32_t keep,
                                                u64 *out_m, uint32_t *out_id) {
  __shared__ u64 sm[kTkTile];
  __shared__ uint32_t sid[kTkTile];
  const uint64_t base = (uint64_t)blockIdx.x * kTkTile;
  for (uint32_t j = threadIdx.x; j < kTkTile; j += kTkNT) {
    const uint64_t idx = base + j;
    u64 m = 0;
    uint32_t id = 0xFFFFFFFFu;
    if (idx < count) {
      if (in_m) {
        m = in_m[idx];
        id = in_id[idx];
      } else {
        const u64 p = indeg[idx], q = outdeg[idx];
        m = rank == 1 ? (p > q ? p : q) : rank == 2 ? (p < q ? p : q) : rank == 3 ? p + q : p * q;
        id = (uint32_t)idx;
      }
    }
    sm[j] = m;
    sid[j] = id;
  }
  for (uint32_t size = 2; size <= kTkTile; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t p = threadIdx.x; p < kTkTile / 2; p += kTkNT) {
        const uint32_t i = 2 * p - (p & (stride - 1));
        const uint32_t j = i + stride;
        const bool best_first = (i & size) == 0;
        const u64 mi = sm[i], mj = sm[j];
        const uint32_t ii = sid[i], ij = sid[j];
        const bool j_before_i = (mj > mi) || (mj == mi && ij < ii);
        if (j_before_i == best_first) {
          sm[i] = mj; sm[j] = mi;
          sid[i] = ij; sid[j] = ii;
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < keep; j += kTkNT) {
    out_m[(uint64_t)blockIdx.x * keep + j] = sm[j];
    out_id[(uint64_t)blockIdx.x * keep + j] = sid[j];
  }
}

hipError_t select_topk(const uint32_t *indeg, const uint32_t *outdeg, uint32_t n, uint32_t k,
                       uint32_t rank, u64 *tmp_m, uint32_t *tmp_id, uint32_t *out,
                       hipStream_t s) {
  if (k == 0) return hipSuccess;
  if (k > kTkKeepMax) return hipErrorInvalidValue;
  const uint32_t keep = k <= 64u ? 64u : kTkKeepMax;
  const uint64_t half = topk_tmp_entries(n) / 2;
  uint64_t count = n;
  const u64 *in_m = nullptr;
  const uint32_t *in_id = nullptr;
  int side = 0;
  for (;;) {
    const uint64_t tiles = (count + kTkTile - 1) / kTkTile;
    u64 *om = tmp_m + side * half;
    uint32_t *oi = tmp_id + side * half;
    hipLaunchKernelGGL(k_topk, dim3((uint32_t)tiles), dim3(kTkNT), 0, s, indeg, outdeg, in_m,
                       in_id, count, rank, keep, om, oi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tiles == 1) return hipMemcpyAsync(out, oi, sizeof(uint32_t) * k, hipMemcpyDeviceToDevice, s);
    in_m = om;
    in_id = oi;
    count = tiles * keep;
    side ^= 1;
  }
}

// ---------------------------------------------------------------- seeds

// Landmark i sets bit i of its own DL_in and DL_out (a landmark reaches itself).
__global__ void k_mark_landmarks(u64 *lab, uint32_t words, const uint32_t *landmarks, uint32_t k,
                                 uint8_t *is_landmark) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const uint32_t x = landmarks[i];
  is_landmark[x] = 1;
  u64 *rec = lab + 4ull * words * x;
  atomicOr(&rec[i >> 6], 1ull << (i & 63u));              // DL_in
  atomicOr(&rec[2u * words + (i >> 6)], 1ull << (i & 63u));  // DL_out
}

// A leaf of S_in (S_out) sets bit h(x) of its own BL_in (BL_out). One thread per vertex, so the
// plain read-modify-write is race-free.
__global__ void k_seed_leaves(u64 *lab, uint32_t words, uint32_t n, const uint32_t *indeg,
                              const uint32_t *outdeg, const uint8_t *is_landmark,
                              const uint8_t *flags_in, const uint8_t *bucket_in, uint32_t kp_bits,
                              u64 leaf_threshold, uint8_t *flags_out, uint8_t *bucket_out) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    uint32_t fl;
    if (flags_in) {
      fl = flags_in[x] & 3u;
    } else if (leaf_threshold) {
      const bool lm = is_landmark[x] != 0;
      fl = (!lm && (u64)indeg[x] * (u64)outdeg[x] <= leaf_threshold) ? 3u : 0u;
    } else {
      const bool lm = is_landmark[x] != 0;
      fl = (uint32_t)(!lm && indeg[x] == 0) | ((uint32_t)(!lm && outdeg[x] == 0) << 1);
    }
    const uint32_t b = bucket_in ? bucket_in[x] : fib_bucket(x, kp_bits);
    u64 *rec = lab + 4ull * words * x;
    if (fl & 1u) rec[words + (b >> 6)] |= 1ull << (b & 63u);       // BL_in
    if (fl & 2u) rec[3u * words + (b >> 6)] |= 1ull << (b & 63u);  // BL_out
    flags_out[x] = (uint8_t)fl;
    bucket_out[x] = (uint8_t)b;
  }
}

hipError_t launch_seed(LabelsView L, uint32_t n, const uint32_t *landmarks, uint32_t k,
                       const uint32_t *indeg, const uint32_t *outdeg,
                       const uint8_t *leaf_flags_in, const uint8_t *bucket_in, uint32_t kp_bits,
                       u64 leaf_threshold, uint8_t *leaf_flags_out, uint8_t *bucket_out,
                       uint8_t *is_landmark, hipStream_t s) {
  if (k > kMaxLabelBits || k > 64u * L.words || (1u << kp_bits) > 64u * L.words)
    return hipErrorInvalidValue;
  if (k) {
    hipLaunchKernelGGL(k_mark_landmarks, dim3(1), dim3(kMaxLabelBits), 0, s, L.lab, L.words,
                       landmarks, k, is_landmark);
  }
  hipLaunchKernelGGL(k_seed_leaves, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, L.lab,
                     L.words, n, indeg, outdeg, is_landmark, leaf_flags_in, bucket_in, kp_bits,
                     leaf_threshold, leaf_flags_out, bucket_out);
  return hipGetLastError();
}

constexpr uint32_t kInitStage = 4096;

template <int W>
__global__ __launch_bounds__(256) void k_init_frontier(const u64 *lab, uint32_t n, Csr f, Csr r,
                                                       uint32_t *frontier, Ctl *ctl,
                                                       uint32_t ring, uint32_t *inq,
                                                       uint32_t stamp) {
  __shared__ uint32_t s_wsum[4], s_base, s_n;
  __shared__ uint32_t s_stage[kInitStage];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->heavy[0] = 0;
    ctl->heavy[1] = 0;
  }
  if (threadIdx.x == 0) s_n = 0;
  for (uint32_t x0 = blockIdx.x * blockDim.x; x0 < n; x0 += gridDim.x * blockDim.x) {
    const uint32_t x = x0 + threadIdx.x;
    bool pf = false, pb = false;
    if (x < n) {
      pf = any_bits<W>(ld_half<W>(half_ptr<W>(lab, x, 0))) && min(f.deg[x], f.cap[x]) > 0u;
      pb = any_bits<W>(ld_half<W>(half_ptr<W>(lab, x, 1))) && min(r.deg[x], r.cap[x]) > 0u;
      if (pf) inq[2ull * x] = stamp;
      if (pb) inq[2ull * x + 1] = stamp;
    }
    stage_push<256, kInitStage>(frontier, &ctl->fsize[ring], pf, x, s_stage, &s_n, &s_base,
                                s_wsum);
    stage_push<256, kInitStage>(frontier, &ctl->fsize[ring], pb, x | kDirBit, s_stage, &s_n,
                                &s_base, s_wsum);
  }
  stage_flush<256>(frontier, &ctl->fsize[ring], s_stage, &s_n, &s_base);
}

hipError_t launch_init_frontier(LabelsView L, uint32_t n, Csr f, Csr r, uint32_t *frontier,
                                Ctl *ctl, uint32_t *inq, uint32_t stamp, hipStream_t s) {
  // the pending frontier is ring 0 at build time
  DBL_LAUNCH_W(L.words, k_init_frontier, dim3(grid_for(n, 256, 1024)), dim3(256), s, L.lab, n, f,
               r, frontier, ctl, 0u, inq, stamp);
  return hipGetLastError();
}

// ---------------------------------------------------------------- propagation

constexpr uint32_t kExpandUnroll = 4;

// Expand frontier entries [beg, end) (at most NT, one per thread): every edge of every entry
// relaxes its target; targets whose label grew are queued in nq with stamp nstamp. With a heavy
// list, rows longer than kHeavyDeg are split into chunks for k_heavy instead.
// `coherent` reads the frontier vertices' labels past the L1 cache (needed when earlier rounds
// of the same kernel changed them).
template <int NT, int W>
__device__ __forceinline__ void expand_tile(const PropArgs &a, const uint32_t *fq, uint32_t beg,
                                            uint32_t end, uint32_t *nq, uint32_t *ncnt,
                                            uint32_t nstamp, u64 *heavy_list,
                                            uint32_t *heavy_cnt, bool coherent,
                                            uint32_t *s_start, u64 *s_off, Half<W> *s_lab,
                                            uint32_t *s_ent, uint32_t *s_wsum, u64 &relaxed,
                                            u64 &expanded, uint32_t skip_mask) {
  const uint32_t t = threadIdx.x;
  const uint32_t i = beg + t;
  uint32_t d = 0;
  bool mine = false;
  if (i < end) {
    const uint32_t ent = fq[i];
    const uint32_t dir = ent >> 31, x = ent & kIdMask;
    mine = !((skip_mask >> dir) & 1u);
    const u64 *offp = dir ? a.r.off : a.f.off;
    const uint32_t* degp = dir ? a.r.deg : a.f.deg;
    const uint32_t* capp = dir ? a.r.cap : a.f.cap;
    uint32_t dg = mine ? min(degp[x], capp[x]) : 0u;
    const u64 *lp = half_ptr<W>(a.L.lab, x, dir);
    Half<W> lv = {};
    if (mine) lv = coherent ? ld_half_agent<W>(lp) : ld_half<W>(lp);
    if (heavy_list && dg > kHeavyDeg) {
      const uint32_t nch = (dg + kChunk - 1) / kChunk;
      const uint32_t hb = atomicAdd(heavy_cnt, nch);
      for (uint32_t c = 0; c < nch; c++)
        if (hb + c < a.heavy_cap) heavy_list[hb + c] = ((u64)ent << 32) | c;
      dg = 0;
    }
    s_ent[t] = ent;
    s_off[t] = offp[x];
    s_lab[t] = lv;
    d = dg;
  }
  uint32_t total;
  const uint32_t ex = block_excl_scan<NT>(d, s_wsum, total);
  s_start[t] = ex;
  const uint32_t nexp = (uint32_t)__syncthreads_count(mine);
  const uint32_t last = min((uint32_t)NT, end - beg) - 1u;
  // kExpandUnroll / W edges per thread at a time: their column reads, then their target-label
  // reads are each issued together before the first update
  constexpr uint32_t U = kExpandUnroll / W;
  for (uint32_t e0 = t; e0 < total; e0 += NT * U) {
    uint32_t lo[U], y[U];
    Half<W> cur[U];
#pragma unroll
    for (uint32_t j = 0; j < U; j++) {
      const uint32_t e = e0 + NT * j;
      lo[j] = 0;
      y[j] = 0;
      if (e < total) {
        uint32_t hi = last;
        while (lo[j] < hi) {
          const uint32_t mid = (lo[j] + hi + 1) >> 1;
          if (s_start[mid] <= e) lo[j] = mid; else hi = mid - 1;
        }
        const uint32_t *col = (s_ent[lo[j]] >> 31) ? a.r.col : a.f.col;
        y[j] = col[s_off[lo[j]] + (e - s_start[lo[j]])];
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < U; j++) {
      cur[j] = {};
      if (e0 + NT * j < total) cur[j] = ld_half<W>(half_ptr<W>(a.L.lab, y[j], s_ent[lo[j]] >> 31));
    }
#pragma unroll
    for (uint32_t j = 0; j < U; j++) {
      const bool ea = e0 + NT * j < total;
      const uint32_t ent = s_ent[lo[j]];
      const uint32_t dir = ent >> 31;
      const bool ch = ea && or_half<W>(half_ptr<W>(a.L.lab, y[j], dir), s_lab[lo[j]], cur[j]);
      const bool push = ch && claim(&a.inq[2ull * y[j] + dir], nstamp);
      wave_push(nq, ncnt, push, y[j] | (ent & kDirBit));
    }
  }
  if (t == 0) {
    relaxed += total;
    expanded += nexp;
  }
  __syncthreads();
}

template <int W>
__global__ __launch_bounds__(256) void k_round(PropArgs a, uint32_t ring, uint32_t stamp,
                                               uint32_t skip_mask, uint32_t bookkeep) {
  __shared__ uint32_t s_start[256];
  __shared__ u64 s_off[256];
  __shared__ Half<W> s_lab[256];
  __shared__ uint32_t s_ent[256];
  __shared__ uint32_t s_wsum[4];
  Ctl *ctl = a.ctl;
  const uint32_t nring = ring == 2u ? 0u : ring + 1u;
  const uint32_t fsz = ctl->fsize[ring];
  if (bookkeep && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->fsize[nring == 2u ? 0u : nring + 1u] = 0;
    ctl->heavy[(stamp + 1u) & 1u] = 0;
    ctl->cur = nring;
    ctl->stamp = stamp + 1u;
  }
  u64 relaxed = 0, expanded = 0;
  for (uint32_t beg = blockIdx.x * 256u; beg < fsz; beg += gridDim.x * 256u) {
    const uint32_t end = min(beg + 256u, fsz);
    expand_tile<256, W>(a, a.fq[ring], beg, end, a.fq[nring], &ctl->fsize[nring], stamp + 1u,
                     a.heavy_list, &ctl->heavy[stamp & 1u], false, s_start, s_off, s_lab, s_ent,
                     s_wsum, relaxed, expanded, skip_mask);
  }
  if (threadIdx.x == 0 && (expanded | relaxed)) {
    a.pcnt[2 * blockIdx.x] += expanded;
    a.pcnt[2 * blockIdx.x + 1] += relaxed;
  }
}

// Chunks of high-degree frontier rows: one block per chunk of kChunk entries.
template <int W>
__global__ __launch_bounds__(256) void k_heavy(PropArgs a, uint32_t hidx, uint32_t nring,
                                               uint32_t nstamp) {
  Ctl *ctl = a.ctl;
  uint32_t cnt = ctl->heavy[hidx];
  if (cnt > a.heavy_cap) cnt = (uint32_t)a.heavy_cap;
  u64 relaxed = 0;
  for (uint32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const u64 h = a.heavy_list[item];
    const uint32_t ent = (uint32_t)(h >> 32), c = (uint32_t)h;
    const uint32_t dir = ent >> 31, x = ent & kIdMask;
    const Csr g = dir ? a.r : a.f;
    const uint32_t dg = min(g.deg[x], g.cap[x]);
    const uint32_t b = c * kChunk, e_end = min(dg, b + kChunk);
    const Half<W> lv = ld_half<W>(half_ptr<W>(a.L.lab, x, dir));
    const u64 o = g.off[x];
    for (uint32_t e0 = b; e0 < e_end; e0 += 256u) {
      const uint32_t e = e0 + threadIdx.x;
      bool push = false;
      uint32_t y = 0;
      if (e < e_end) {
        y = g.col[o + e];
        push = relax<W>(half_ptr<W>(a.L.lab, y, dir), lv) &&
               claim(&a.inq[2ull * y + dir], nstamp);
      }
      wave_push(a.fq[nring], &ctl->fsize[nring], push, y | (ent & kDirBit));
    }
    relaxed += e_end > b ? e_end - b : 0;
  }
  if (threadIdx.x == 0 && relaxed) a.pcnt[2 * (kRoundGridMax + blockIdx.x) + 1] += relaxed;
}

hipError_t launch_round(const PropArgs &a, uint32_t ring, uint32_t stamp, uint32_t grid,
                        hipStream_t s, uint32_t skip_mask, bool bookkeep) {
  if (grid > kRoundGridMax) grid = kRoundGridMax;
  DBL_LAUNCH_W(a.L.words, k_round, dim3(grid), dim3(256), s, a, ring, stamp, skip_mask,
               bookkeep ? 1u : 0u);
  const uint32_t nring = ring == 2u ? 0u : ring + 1u;
  DBL_LAUNCH_W(a.L.words, k_heavy, dim3(kHeavyGrid), dim3(256), s, a, stamp & 1u, nring,
               stamp + 1u);
  return hipGetLastError();
}

// ---- direction-optimised rounds
// A round whose frontier covers a large share of a direction's edges can run as a pull: every
// vertex y ORs in the labels of its neighbours p that are in the frontier (Pre(y) for the
// forward labels, Suc(y) for the backward ones). The result equals the push round's: each
// frontier edge is relaxed once either way, and labels only grow. A pull reads the target
// rows in order, reads source labels only for frontier edges, and writes each grown label once
// without atomics (a row has one owner thread), so it moves far less memory per relaxation than
// scattered pushes with their atomics and queue claims.

// One bitmap per direction (a pull of one direction tests only its own, half the footprint of
// an interleaved layout, which matters for staying in L2): bit x of fbm[dir * wpd ...].
__device__ __forceinline__ bool in_frontier(const u64 *fbm, uint64_t wpd, uint32_t x,
                                            uint32_t dir) {
  return (fbm[dir * wpd + (x >> 6)] >> (x & 63u)) & 1ull;
}

template <int W>
__global__ __launch_bounds__(256) void k_frontier_scan(PropArgs a, uint32_t ring,
                                                       uint32_t stamp) {
  __shared__ u64 s_red[4][4];
  __shared__ u64 s_or[4][2][2 * W];
  Ctl *ctl = a.ctl;
  const uint32_t fsz = ctl->fsize[ring];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // what k_round does at its start: the pending frontier moves on to the next ring
    const uint32_t nring = ring == 2u ? 0u : ring + 1u;
    ctl->fsize[nring == 2u ? 0u : nring + 1u] = 0;
    ctl->heavy[(stamp + 1u) & 1u] = 0;
    ctl->pheavy = 0;
    ctl->cur = nring;
    ctl->stamp = stamp + 1u;
  }
  u64 v[4] = {0, 0, 0, 0};  // entries fwd, bwd, push edges fwd, bwd
  Half<W> un[2] = {};       // OR of the entries' labels, per direction
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < fsz; i += gridDim.x * 256u) {
    const uint32_t e = a.fq[ring][i];
    const uint32_t d = e >> 31, x = e & kIdMask;
    const uint32_t dg = d ? min(a.r.deg[x], a.r.cap[x]) : min(a.f.deg[x], a.f.cap[x]);
    atomicOr(&a.fbm[d * a.fbm_wpd + (x >> 6)], 1ull << (x & 63u));
    const Half<W> l = ld_half<W>(half_ptr<W>(a.L.lab, x, d));
    if (d) {
      v[1] += 1;
      v[3] += dg;
#pragma unroll
      for (int j = 0; j < 2 * W; j++) un[1].w[j] |= l.w[j];
    } else {
      v[0] += 1;
      v[2] += dg;
#pragma unroll
      for (int j = 0; j < 2 * W; j++) un[0].w[j] |= l.w[j];
    }
  }
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; k++) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if (lane == 0) s_red[w][k] = v[k];
  }
#pragma unroll
  for (int d = 0; d < 2; d++)
#pragma unroll
    for (int j = 0; j < 2 * W; j++) {
      u64 x = un[d].w[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
      if (lane == 0) s_or[w][d][j] = x;
    }
  __syncthreads();
  u64 *stripe = a.fu + kFuStride * (1u + (blockIdx.x & (kFuStripes - 1u)));
  if (threadIdx.x < 4) {
    const u64 sum = s_red[0][threadIdx.x] + s_red[1][threadIdx.x] + s_red[2][threadIdx.x] +
                    s_red[3][threadIdx.x];
    if (sum) atomicAdd(&stripe[16 + threadIdx.x], sum);
  }
  if (threadIdx.x < 4 * W) {
    const uint32_t d = threadIdx.x / (2 * W), j = threadIdx.x % (2 * W);
    const u64 x = s_or[0][d][j] | s_or[1][d][j] | s_or[2][d][j] | s_or[3][d][j];
    if (x) atomicOr(&stripe[d * 8 + j], x);
  }
}

// One wave: reduce the scan's stripes into fu[0, 16) and the four frontier counts, and zero
// the stripes for the next scan.
__global__ __launch_bounds__(64) void k_frontier_reduce(u64 *fu, Ctl *ctl) {
  u64 *st = fu + kFuStride * (1u + threadIdx.x);
  for (uint32_t k = 0; k < 20; k++) {
    u64 x = st[k];
    st[k] = 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const u64 y = __shfl_xor(x, o, 64);
      x = k < 16 ? (x | y) : (x + y);
    }
    if (threadIdx.x == 0) {
      if (k < 16) fu[k] = x;
      else ctl->ctr[kCtrFrontEntries + (k - 16)] = x;
    }
  }
}

hipError_t launch_frontier_scan(const PropArgs &a, uint32_t ring, uint32_t stamp,
                                uint64_t fbm_words, hipStream_t s) {
  hipError_t e = launch_fill_u64(a.fbm, 0ull, fbm_words, s);
  if (e != hipSuccess) return e;
  DBL_LAUNCH_W(a.L.words, k_frontier_scan, dim3(kRoundGridMax), dim3(256), s, a, ring, stamp);
  hipLaunchKernelGGL(k_frontier_reduce, dim3(1), dim3(kFuStripes), 0, s, a.fu, a.ctl);
  return hipGetLastError();
}

// Sum of a per-thread 64-bit count over a block of 256 threads; the result is valid in thread 0.
__device__ __forceinline__ u64 block_sum256(u64 v, u64 *s_tmp) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (__lane_id() == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  const u64 r = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
  __syncthreads();
  return r;
}

// OR `v` (2W words) into the LDS accumulator of row `row` for every lane that holds a value.
// When the whole wave works on one row (long rows) the wave reduces first and one lane adds.
template <int W>
__device__ __forceinline__ void acc_or(u64 (*s_acc)[2 * W], uint32_t row, bool act, bool hit,
                                       Half<W> v) {
  const uint32_t lane = __lane_id();
  const uint32_t row0 = __shfl(row, 0, 64);
  const bool uniform = __ballot(act && row != row0) == 0ull && __shfl(act ? 1u : 0u, 0, 64);
  if (uniform) {
#pragma unroll
    for (int i = 0; i < 2 * W; i++) {
      u64 x = hit ? v.w[i] : 0ull;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
      if (lane == 0 && x) atomicOr(&s_acc[row0][i], x);
    }
  } else if (hit) {
#pragma unroll
    for (int i = 0; i < 2 * W; i++)
      if (v.w[i]) atomicOr(&s_acc[row][i], v.w[i]);
  }
}

// Pull rows: 256 rows per tile, the rows' edges laid end to end and taken one per thread (as
// in expand_tile). Rows longer than kHeavyDeg go to k_pull_heavy in chunks. For a direction in
// allmask (a frontier that holds most of the direction's edges) every neighbour's label is
// read without the frontier-bitmap test: a neighbour outside the frontier adds nothing, and at
// 2^25 vertices the bitmap lookups and the label reads evict each other from L2 (measured: the
// first pull of the build takes 39 ms with the test, 27 ms without, 12 ms with either the
// label reads or the bitmap misses alone).
constexpr uint32_t kPullUnroll = 4, kPullStage = 2048;

template <int W>
__global__ __launch_bounds__(256) void k_pull(PropArgs a, uint32_t n, uint32_t dmask,
                                              uint32_t allmask, uint32_t nring, uint32_t nstamp) {
  __shared__ uint32_t s_start[256];
  __shared__ u64 s_off[256];
  __shared__ uint32_t s_row[256];
  __shared__ uint32_t s_wsum[4];
  __shared__ u64 s_acc[256][2 * W];
  __shared__ uint32_t s_base, s_n;
  __shared__ uint32_t s_stage[kPullStage];
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x;
  if (t == 0) s_n = 0;
  const uint32_t ndir = __popc(dmask);
  const uint32_t d_only = (dmask & 1u) ? 0u : 1u;
  const uint64_t rows = (uint64_t)n * ndir;
  u64 relaxed = 0;
  for (uint64_t beg = (uint64_t)blockIdx.x * 256u; beg < rows;
       beg += (uint64_t)gridDim.x * 256u) {
    const uint64_t r = beg + t;
    const bool act = r < rows;
    uint32_t y = 0, d = 0, dg = 0;
    Half<W> cur = {};
    if (act) {
      d = ndir == 2 ? (r >= n ? 1u : 0u) : d_only;
      y = (uint32_t)(r - (ndir == 2 && r >= n ? (uint64_t)n : 0ull));
      const Csr g = pick_csr(a.r, a.f, d);  // neighbours the labels come from
      dg = min(g.deg[y], g.cap[y]);
      // a row already holding every bit of this direction's frontier cannot grow this round
      // (a source that grows later in the round is queued again and delivers next round)
      cur = ld_half<W>(half_ptr<W>(a.L.lab, y, d));
      u64 miss = 0;
#pragma unroll
      for (int i = 0; i < 2 * W; i++) miss |= a.fu[d * 8 + i] & ~cur.w[i];
      if (!miss) dg = 0;
      if (dg > kHeavyDeg) {
        const uint32_t nch = (dg + kChunk - 1) / kChunk;
        const uint32_t hb = atomicAdd(&ctl->pheavy, nch);
        for (uint32_t c = 0; c < nch; c++)
          if (hb + c < a.heavy_cap)
            a.pheavy_list[hb + c] = ((u64)(y | (d << 31)) << 32) | c;
        dg = 0;
      }
      s_off[t] = g.off[y];
    }
    s_row[t] = y | (d << 31);
#pragma unroll
    for (int i = 0; i < 2 * W; i++) s_acc[t][i] = 0ull;
    uint32_t total;
    const uint32_t ex = block_excl_scan<256>(dg, s_wsum, total);
    s_start[t] = ex;
    __syncthreads();
    const uint32_t last = (uint32_t)min<uint64_t>(256u, rows - beg) - 1u;
    // kPullUnroll edges per thread at a time: their column reads, then their frontier-bit
    // reads, then their label reads are each issued together
    constexpr uint32_t U = kPullUnroll / W;
    for (uint32_t e0 = 0; e0 < total; e0 += 256u * U) {
      uint32_t lo[U], p[U], rd[U];
      bool eact[U], hit[U];
      Half<W> lv[U];
#pragma unroll
      for (uint32_t j = 0; j < U; j++) {
        const uint32_t e = e0 + 256u * j + t;
        eact[j] = e < total;
        lo[j] = 0;
        p[j] = 0;
        rd[j] = 0;
        if (eact[j]) {
          uint32_t hi = last;
          while (lo[j] < hi) {
            const uint32_t mid = (lo[j] + hi + 1) >> 1;
            if (s_start[mid] <= e) lo[j] = mid; else hi = mid - 1;
          }
          rd[j] = s_row[lo[j]] >> 31;
          const uint32_t *col = rd[j] ? a.f.col : a.r.col;
          p[j] = col[s_off[lo[j]] + (e - s_start[lo[j]])];
        }
      }
#pragma unroll
      for (uint32_t j = 0; j < U; j++)
        hit[j] = eact[j] && (((allmask >> rd[j]) & 1u) || in_frontier(a.fbm, a.fbm_wpd, p[j], rd[j]));
#pragma unroll
      for (uint32_t j = 0; j < U; j++) {
        lv[j] = {};
        if (hit[j]) {
          lv[j] = ld_half<W>(half_ptr<W>(a.L.lab, p[j], rd[j]));
          relaxed++;
        }
      }
#pragma unroll
      for (uint32_t j = 0; j < U; j++) acc_or<W>(s_acc, lo[j], eact[j], hit[j], lv[j]);
    }
    __syncthreads();
    bool push = false;
    if (act && dg) {
      u64 *wl = half_ptr<W>(a.L.lab, y, d);
      bool grew = false;
#pragma unroll
      for (int i = 0; i < 2 * W; i++) {
        const u64 add = s_acc[t][i] & ~cur.w[i];
        if (add) {
          wl[i] = cur.w[i] | add;  // this thread is the row's only writer in this kernel
          grew = true;
        }
      }
      push = grew && claim(&a.inq[2ull * y + d], nstamp);
    }
    stage_push<256, kPullStage>(a.fq[nring], &ctl->fsize[nring], push, y | (d << 31), s_stage,
                                &s_n, &s_base, s_wsum);
    __syncthreads();
  }
  stage_flush<256>(a.fq[nring], &ctl->fsize[nring], s_stage, &s_n, &s_base);
  __shared__ u64 s_tmp[4];
  relaxed = block_sum256(relaxed, s_tmp);
  if (t == 0 && relaxed) a.pcnt[2 * blockIdx.x + 1] += relaxed;
}

template <int W>
__global__ __launch_bounds__(256) void k_pull_heavy(PropArgs a, uint32_t nring,
                                                    uint32_t nstamp) {
  __shared__ u64 s_acc[1][2 * W];
  Ctl *ctl = a.ctl;
  uint32_t cnt = ctl->pheavy;
  if (cnt > a.heavy_cap) cnt = (uint32_t)a.heavy_cap;
  u64 relaxed = 0;
  for (uint32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const u64 h = a.pheavy_list[item];
    const uint32_t row = (uint32_t)(h >> 32), c = (uint32_t)h;
    const uint32_t d = row >> 31, y = row & kIdMask;
    const Csr g = pick_csr(a.r, a.f, d);
    const uint32_t dg = min(g.deg[y], g.cap[y]);
    uint32_t b = c * kChunk, e_end = min(dg, b + kChunk);
    {
      // as in k_pull: a row holding every bit of the frontier cannot grow this round
      const Half<W> cur = ld_half<W>(half_ptr<W>(a.L.lab, y, d));
      u64 miss = 0;
#pragma unroll
      for (int i = 0; i < 2 * W; i++) miss |= a.fu[d * 8 + i] & ~cur.w[i];
      if (!miss) e_end = b;
    }
    const u64 o = g.off[y];
    if (threadIdx.x < 2 * W) s_acc[0][threadIdx.x] = 0ull;
    __syncthreads();
    for (uint32_t e0 = b; e0 < e_end; e0 += 256u) {
      const uint32_t e = e0 + threadIdx.x;
      bool hit = false;
      Half<W> lv = {};
      if (e < e_end) {
        const uint32_t p = g.col[o + e];
        if (in_frontier(a.fbm, a.fbm_wpd, p, d)) {
          hit = true;
          lv = ld_half<W>(half_ptr<W>(a.L.lab, p, d));
          relaxed++;
        }
      }
      acc_or<W>(s_acc, 0u, e < e_end, hit, lv);
    }
    __syncthreads();
    bool push = false;
    if (threadIdx.x == 0) {
      Half<W> acc;
#pragma unroll
      for (int i = 0; i < 2 * W; i++) acc.w[i] = s_acc[0][i];
      // chunks of one row run in different blocks: OR with atomics
      push = relax<W>(half_ptr<W>(a.L.lab, y, d), acc) && claim(&a.inq[2ull * y + d], nstamp);
    }
    if (threadIdx.x < 64) wave_push(a.fq[nring], &ctl->fsize[nring], push, row);
    __syncthreads();
  }
  __shared__ u64 s_tmp[4];
  relaxed = block_sum256(relaxed, s_tmp);
  if (threadIdx.x == 0 && relaxed) a.pcnt[2 * (kRoundGridMax + blockIdx.x) + 1] += relaxed;
}

hipError_t launch_pull(const PropArgs &a, uint32_t n, uint32_t dmask, uint32_t allmask,
                       uint32_t ring, uint32_t stamp, uint32_t grid, hipStream_t s) {
  if (!dmask) return hipSuccess;
  if (grid > kRoundGridMax) grid = kRoundGridMax;
  const uint32_t nring = ring == 2u ? 0u : ring + 1u;
  allmask &= dmask;
  DBL_LAUNCH_W(a.L.words, k_pull, dim3(grid), dim3(256), s, a, n, dmask, allmask, nring,
               stamp + 1u);
  DBL_LAUNCH_W(a.L.words, k_pull_heavy, dim3(kHeavyGrid), dim3(256), s, a, nring, stamp + 1u);
  return hipGetLastError();
}

// Rounds inside one workgroup while the frontier is small (no kernel launch per round). Reads
// the pending frontier from ctl->cur / ctl->stamp and writes back where it stopped: either the
// frontier is empty, or it outgrew the local bounds and grid rounds take over.
// LDS of one kLocalThreads-wide workgroup expanding frontier tiles.
template <int W>
struct TileLds {
  uint32_t start[kLocalThreads];
  u64 off[kLocalThreads];
  Half<W> lab[kLocalThreads];
  uint32_t ent[kLocalThreads];
  uint32_t wsum[kLocalThreads / 64];
  uint32_t edges;
};

template <int W>
__device__ void local_rounds_core(const PropArgs &a, TileLds<W> &sm) {
  uint32_t *s_start = sm.start, *s_ent = sm.ent, *s_wsum = sm.wsum;
  u64 *s_off = sm.off;
  Half<W> *s_lab = sm.lab;
  uint32_t &s_edges = sm.edges;
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x;
  uint32_t ring = ld_agent32(&ctl->cur), stamp = ld_agent32(&ctl->stamp);
  u64 relaxed = 0, expanded = 0;
  uint32_t rounds = 0;
  for (;;) {
    const uint32_t fsz = ld_agent32(&ctl->fsize[ring]);
    if (fsz == 0 || fsz > a.local_max_frontier) break;
    uint32_t my = 0;
    const uint32_t *fq = a.fq[ring];
    for (uint32_t i = t; i < fsz; i += kLocalThreads) {
      const uint32_t ent = fq[i];
      const uint32_t x = ent & kIdMask;
      my += (ent >> 31) ? min(a.r.deg[x], a.r.cap[x]) : min(a.f.deg[x], a.f.cap[x]);
    }
    if (t == 0) s_edges = 0;
    __syncthreads();
    if (my) atomicAdd(&s_edges, my);
    __syncthreads();
    const uint32_t edges = s_edges;
    __syncthreads();
    if (edges > a.local_max_edges) break;
    const uint32_t nring = ring == 2u ? 0u : ring + 1u;
    if (t == 0) st_agent32(&ctl->fsize[nring], 0u);
    __syncthreads();
    for (uint32_t beg = 0; beg < fsz; beg += kLocalThreads) {
      const uint32_t end = min(beg + kLocalThreads, fsz);
      expand_tile<kLocalThreads, W>(a, fq, beg, end, a.fq[nring], &ctl->fsize[nring], stamp + 1u,
                                 nullptr, nullptr, true, s_start, s_off, s_lab, s_ent, s_wsum,
                                 relaxed, expanded, 0u);
    }
    __syncthreads();
    ring = nring;
    stamp++;
    rounds++;
  }
  __syncthreads();
  if (t == 0) {
    const uint32_t nring = ring == 2u ? 0u : ring + 1u;
    st_agent32(&ctl->fsize[nring], 0u);
    st_agent32(&ctl->cur, ring);
    st_agent32(&ctl->stamp, stamp);
    ctl->local_rounds += rounds;
    if (expanded) {
      a.pcnt[2 * (kRoundGridMax + kHeavyGrid)] += expanded;
      a.pcnt[2 * (kRoundGridMax + kHeavyGrid) + 1] += relaxed;
    }
  }
}

template <int W>
__device__ void local_rounds_body(const PropArgs &a) {
  __shared__ TileLds<W> sm;
  local_rounds_core<W>(a, sm);
}

template <int W>
__global__ __launch_bounds__(kLocalThreads) void k_local_rounds(PropArgs a, Mirror *m,
                                                                uint32_t seq) {
  local_rounds_body<W>(a);
  if (m && threadIdx.x == 0) publish_status(a.ctl, m, seq);
}

hipError_t launch_local_rounds(const PropArgs &a, Mirror *m, uint32_t seq, hipStream_t s) {
  DBL_LAUNCH_W(a.L.words, k_local_rounds, dim3(1), dim3(kLocalThreads), s, a, m, seq);
  return hipGetLastError();
}

// ---------------------------------------------------------------- insertion

// Append y to row x; returns false when the row is full and the entry went to the overflow list.
__device__ __forceinline__ bool append_edge(const Csr &g, uint32_t x, uint32_t y,
                                            uint32_t dirbit, Ovf *ovf, uint64_t ovf_cap,
                                            Ctl *ctl) {
  // the row's capacity and offset do not depend on the append: read them first
  const uint32_t cap = g.cap[x];
  const u64 off = g.off[x];
  const uint32_t pos = atomicAdd(&g.deg[x], 1u);
  if (pos < cap) {
    g.col[off + pos] = y;
    return true;
  }
  const uint32_t k = atomicAdd(&ctl->ovf_count, 1u);
  if (k < ovf_cap) {
    Ovf o;
    o.x = x | dirbit;
    o.pos = pos;
    o.y = y;
    o.pad = 0;
    ovf[k] = o;
  }
  return false;
}

// Half of an insertion (u,v) for one direction. Forward: append v to Suc(u) and OR
// (DL_in(u), BL_in(u)) into v (Algorithm 3 starts from v). Backward: append u to Pre(v) and OR
// (DL_out(v), BL_out(v)) into u. A changed endpoint joins the pending frontier. Returns whether
// it was queued. `coherent_tail` reads the tail's label past the L1 cache (the request server,
// whose earlier requests may have grown it through L2 atomics); the head's label is only a
// pre-read, where an older value merely costs an extra atomic.
template <int W>
__device__ __forceinline__ bool apply_half(const PropArgs &a, uint32_t u, uint32_t v, uint32_t dir,
                                           uint32_t ring, uint32_t stamp, Ovf *ovf,
                                           uint64_t ovf_cap, bool active, bool *overflowed,
                                           bool coherent_tail = false) {
  bool p = false;
  const uint32_t tail = dir ? v : u, head = dir ? u : v;
  if (active && u != v) {
    // the label reads do not depend on the append: issue them first
    const u64 *tp = half_ptr<W>(a.L.lab, tail, dir);
    const Half<W> lt = coherent_tail ? ld_half_agent<W>(tp) : ld_half<W>(tp);
    u64 *wh = half_ptr<W>(a.L.lab, head, dir);
    const Half<W> lh = ld_half<W>(wh);
    if (!append_edge(pick_csr(a.f, a.r, dir), tail, head, dir ? kDirBit : 0u, ovf, ovf_cap, a.ctl))
      *overflowed = true;
    p = or_half<W>(wh, lt, lh) && claim(&a.inq[2ull * head + dir], stamp);
  }
  wave_push(a.fq[ring], &a.ctl->fsize[ring], p, head | (dir ? kDirBit : 0u));
  return p;
}

// A small batch in one workgroup: thread 2i handles the forward half of edge i and thread
// 2i+1 the backward half. Every id is checked before anything changes (a block-wide vote);
// then the halves are applied and the propagation rounds run here when something changed.
// Returns the flags of the host status word (kFastErr, kFastOvf, kFastPending), the same in
// every thread. Control-block fields are read past the caches: the request server runs this
// body many times in one launch.
template <int W>
__device__ uint32_t insert_small_body(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                                      uint32_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap) {
  __shared__ uint32_t s_pushed, s_ovf, s_flags;
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x;
  const uint32_t halves = 2 * count;  // half j: edge j / 2, direction j % 2
  if (t == 0) {
    s_pushed = 0;
    s_ovf = 0;
  }
  bool bad = false;
  for (uint32_t j = t; j < halves; j += kLocalThreads) {
    const uint32_t i = j >> 1;
    bad |= (src[i] >= n) | (dst[i] >= n);
  }
  if (__syncthreads_or(bad)) {
    if (t == 0) atomicOr(&ctl->err, kErrRange);
    return kFastErr;
  }
  const uint32_t ring = ld_agent32(&ctl->cur), stamp = ld_agent32(&ctl->stamp);
  if (t == 0) {
    st_agent32(&ctl->heavy[0], 0u);
    st_agent32(&ctl->heavy[1], 0u);
  }
  bool pushed = false, ovfl = false;
  for (uint32_t j0 = 0; j0 < halves; j0 += kLocalThreads) {
    const uint32_t j = j0 + t;
    const bool act = j < halves;
    const uint32_t i = act ? j >> 1 : 0u;
    pushed |= apply_half<W>(a, act ? src[i] : 0u, act ? dst[i] : 0u, j & 1u, ring, stamp, ovf,
                            ovf_cap, act, &ovfl);
  }
  if (pushed) s_pushed = 1;
  if (ovfl) s_ovf = 1;
  __syncthreads();
  // nothing changed: the pending frontier is still empty and no round is needed
  if (s_pushed) local_rounds_body<W>(a);
  __syncthreads();
  if (t == 0) {
    uint32_t flags = 0;
    if (s_ovf) flags |= kFastOvf;
    if (s_pushed && ld_agent32(&ctl->fsize[ld_agent32(&ctl->cur)])) flags |= kFastPending;
    s_flags = flags;
  }
  __syncthreads();
  return s_flags;
}

__device__ __forceinline__ void publish_fast(Mirror *m, uint32_t flags, uint32_t seq) {
  __hip_atomic_store(&m->fast, ((u64)flags << 32) | seq, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// One small batch, then one 64-bit word {seq, flags} to the host mirror.
template <int W>
__global__ __launch_bounds__(kLocalThreads) void k_insert_small(PropArgs a, const uint32_t *src,
                                                                const uint32_t *dst,
                                                                uint32_t count, uint32_t n,
                                                                Ovf *ovf, uint64_t ovf_cap,
                                                                Mirror *m, uint32_t seq) {
  const uint32_t flags = insert_small_body<W>(a, src, dst, count, n, ovf, ovf_cap);
  if (threadIdx.x == 0) publish_fast(m, flags, seq);
}

hipError_t launch_insert_small(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint32_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap, Mirror *m,
                               uint32_t seq, hipStream_t s) {
  DBL_LAUNCH_W(a.L.words, k_insert_small, dim3(1), dim3(kLocalThreads), s, a, src, dst, count, n,
               ovf, ovf_cap, m, seq);
  return hipGetLastError();
}

// Request server: the one-request-at-a-time form without a launch per request. Request i is
// released by the host writing its edge into doorbell slot i & 1 (pinned host memory), so its
// ids arrive with the release itself. Lane 0 of wave 1 watches the doorbell and hands each
// request to wave 0 through LDS; wave 0 inserts it with lanes 0 and 1 (the two halves) and
// publishes {seq0 + i - first + 1, flags}. The watching and the serving sit in different waves
// because a wave's memory counter covers all its reads in issue order: host-memory polls still
// in flight in the serving wave would hold up the label reads of the request just released.
// Requests that change no label need nothing else, so the other waves stay parked at a
// barrier. A request whose halves queue a vertex wakes the workgroup, which runs the
// propagation rounds and publishes. The launch returns after the last request, after a request
// that needs the host (nonzero flags: a bad id, a full row, a frontier too large for one
// workgroup), on kDoorStop, or when no request arrives for idle_ticks of the device wall clock.
constexpr uint32_t kServerMaxSpins = 1u << 23;
constexpr uint32_t kCmdExit = 0u, kCmdPropagate = 1u;
constexpr u64 kDoorHalt = ~0ull - 2ull;  // internal: the serving wave asked the watcher to stop

// Wait for a doorbell slot to leave kDoorEmpty and return what it holds (an edge, or
// kDoorStop); kDoorStop also after idle_ticks of the device wall clock, kDoorHalt once *halt is
// set. D reads of the (host-memory) slot are kept in flight, first issued a fraction of a round
// trip apart, so a release is seen sooner than with one read at a time. The iteration bound is
// a backstop that ends the wait even if the clock stood still (each iteration waits for a
// host-memory read).
template <int D>
__device__ __forceinline__ u64 wait_door(const u64 *slot, u64 idle_ticks, const uint32_t *halt) {
  const u64 t0 = wall_clock64();
  u64 d[D];
#pragma unroll
  for (int k = 0; k < D; k++) {
    d[k] = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (k + 1 < D) __builtin_amdgcn_s_sleep(8);
  }
  // branch-free body in which read k is checked and reissued before read k + 1 is looked at
  // (scheduling barriers keep the compiler from hoisting the later checks, which would wait for
  // every read in flight and bunch the reissues), so the reads stay spread out
  for (uint32_t spin = 0; spin < kServerMaxSpins; spin++) {
    u64 got = kDoorEmpty;
#pragma unroll
    for (int k = 0; k < D; k++) {
      __builtin_amdgcn_sched_barrier(0);
      const bool h = d[k] != kDoorEmpty;
      got = h ? d[k] : got;
      d[k] = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (got != kDoorEmpty) return got;
    if (__hip_atomic_load(halt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return kDoorHalt;
    if (wall_clock64() - t0 > idle_ticks) return kDoorStop;
    if (D == 1) __builtin_amdgcn_s_sleep(2);
  }
  return kDoorStop;
}

template <int W>
__global__ __launch_bounds__(kLocalThreads) void k_insert_server(
    PropArgs a, uint32_t first, uint32_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap,
    Mirror *m, const u64 *door, uint32_t seq0, u64 idle_ticks, uint32_t polls) {
  __shared__ uint32_t s_cmd, s_flags;
  __shared__ u64 s_req;        // request handed from the watching wave to the serving wave
  __shared__ uint32_t s_req_i;  // ... and its index (~0u: none yet)
  __shared__ uint32_t s_halt;   // serving wave -> watching wave: stop watching
  __shared__ uint32_t s_next;   // first request index of the next serving pass
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x, lane = t & 63u;
  uint32_t i = first;   // meaningful in wave 0
  bool any_ovf = false;  // ditto
  u64 t_go = 0, busy = 0, served = 0;  // meaningful in thread 0
  if (t == 0) {
    s_req_i = ~0u;
    s_halt = 0;
    s_next = first;
  }
  __syncthreads();
  for (;;) {
    if (t < 64u) {
      uint32_t cmd = kCmdExit;
      // the frontier ring and the queue stamp change only in propagation rounds
      const uint32_t ring = ld_agent32(&ctl->cur), stamp = ld_agent32(&ctl->stamp);
      for (; i < count; i++) {
        u64 req = kDoorStop;
        if (lane == 0) {
          // the watcher hands over request i (or a stop) within idle_ticks, or within its
          // iteration bound; twice the idle limit is a backstop for this wait
          const u64 w0 = wall_clock64();
          for (uint32_t spin = 0;; spin++) {
            if (__hip_atomic_load(&s_req_i, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == i) {
              req = s_req;
              break;
            }
            if ((spin & 255u) == 255u && wall_clock64() - w0 > 2 * idle_ticks + 1000000ull) break;
          }
          t_go = wall_clock64();
        }
        req = __shfl(req, 0, 64);
        if (req == kDoorStop) break;
        // No cache invalidation here: this path reads row bounds (fixed during the launch), the
        // tail label past L1, and pre-reads where an older value only costs an atomic (head
        // label, queue stamp).
        const bool act = lane < 2u;
        const uint32_t u = (uint32_t)(req >> 32), v = (uint32_t)req;
        if (u >= n || v >= n) {  // the host releases no such request; kept as a guard
          if (lane == 0) {
            atomicOr(&ctl->err, kErrRange);
            publish_fast(m, kFastErr, seq0 + (i - first) + 1u);
          }
          break;
        }
        bool ovfl = false;
        const bool pushed = apply_half<W>(a, u, v, lane & 1u, ring, stamp, ovf, ovf_cap, act,
                                          &ovfl, true);
        any_ovf = __ballot(ovfl) != 0ull;
        if (__ballot(pushed)) {
          if (lane == 0) {
            st_agent32(&ctl->heavy[0], 0u);
            st_agent32(&ctl->heavy[1], 0u);
          }
          cmd = kCmdPropagate;
          break;
        }
        if (lane == 0) {
          publish_fast(m, any_ovf ? kFastOvf : 0u, seq0 + (i - first) + 1u);
          busy += wall_clock64() - t_go;
          served++;
        }
        if (any_ovf) break;
      }
      if (t == 0) {
        s_cmd = cmd;
        __hip_atomic_store(&s_halt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cmd == kCmdExit) {
          ctl->ctr[kCtrServerTicks] += busy;
          ctl->ctr[kCtrServerReqs] += served;
        }
      }
    } else if (t == 64u) {
      // the watcher: hand over requests in order until a stop, the last one, or a halt
      for (uint32_t j = s_next; j < count; j++) {
        const u64 r = polls > 1 ? wait_door<4>(door + (j & 1u), idle_ticks, &s_halt)
                                : wait_door<1>(door + (j & 1u), idle_ticks, &s_halt);
        if (r == kDoorHalt) break;
        // Keep the hand-over the first thing after the doorbell read, and keep the loop lean:
        // doorbell reads are still in flight here, and code that makes the compiler wait for
        // them (s_waitcnt vmcnt(0)) ahead of these stores delays every request by up to a host
        // round trip (a clock read added after the hand-over did: +1.7 us per request).
        s_req = r;
        __hip_atomic_store(&s_req_i, j, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (r == kDoorStop) break;
      }
    }
    __syncthreads();
    if (s_cmd == kCmdExit) return;
    // request i queued vertices: the whole workgroup propagates. Earlier requests changed
    // labels and queues through L2: drop this CU's cached lines first.
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    local_rounds_body<W>(a);
    __syncthreads();
    if (t == 0) {
      uint32_t flags = any_ovf ? kFastOvf : 0u;
      if (ld_agent32(&ctl->fsize[ld_agent32(&ctl->cur)])) flags |= kFastPending;
      publish_fast(m, flags, seq0 + (i - first) + 1u);
      busy += wall_clock64() - t_go;
      served++;
      s_flags = flags;
      s_halt = 0;
      s_next = i + 1;
      if (flags) {
        ctl->ctr[kCtrServerTicks] += busy;
        ctl->ctr[kCtrServerReqs] += served;
      }
    }
    __syncthreads();
    if (s_flags) return;
    i++;
  }
}

hipError_t launch_insert_server(const PropArgs &a, uint32_t first, uint32_t count, uint32_t n,
                                Ovf *ovf, uint64_t ovf_cap, Mirror *m, const u64 *door,
                                uint32_t seq0, u64 idle_ticks, uint32_t polls, hipStream_t s) {
  if (first >= count) return hipSuccess;
  DBL_LAUNCH_W(a.L.words, k_insert_server, dim3(1), dim3(kLocalThreads), s, a, first, count, n,
               ovf, ovf_cap, m, door, seq0, idle_ticks, polls);
  return hipGetLastError();
}

// Device-fed form of the one-request-at-a-time insertion: request i is the edge (src[i],
// dst[i]) read from device memory, and each request is applied, and propagated to its fixpoint
// when it changed a label, before the next one takes effect (Algorithm 3 edge by edge). Wave 0
// serves the requests in windows of up to 32: lanes 2j and 2j+1 hold request i+j's forward and
// backward halves and issue all of the window's reads at once (both label halves past the L1
// cache, the tail row's capacity, offset and degree, and the next window's ids: a window's own
// ids were read during the window before); the requests are then applied one after another. While the launch lasts this wave is the only writer of the degrees, so a row's
// degree is read once per window, and a request's slot in its row is that degree plus the
// number of earlier requests of the window on the same row (counted once per window); each
// request then only stores. A request that changes a label ends its window (the later requests'
// label reads may be stale): this wave runs the propagation rounds while the frontier stays
// small (stream_rounds), the workgroup's rounds take over beyond that, and the next window
// starts after that request. The launch returns after
// the last request, after a request whose flags need the host (a full row, a frontier too large
// for one workgroup), or before a request with an id out of range, publishing {seq0 + requests
// applied, flags}. ticks (may be null): ticks[i] = device clock ticks from the end of request
// i - 1 (or the launch's start) to the end of request i.
constexpr uint32_t kStreamWindow = 32;

// One direction's row arrays for each lane of the stream (lane parity = direction), as global
// pointers chosen once per launch from scalar copies of the arguments: selecting the argument
// fields per lane inside the loop reads the pointers back from argument memory per lane, and
// the window then waits for those reads.
typedef __attribute__((address_space(1))) uint32_t gu32_t;
typedef __attribute__((address_space(1))) u64 gu64_t;
struct LaneRows {
  gu32_t *col, *deg, *cap;
  gu64_t *off;
};

__device__ __forceinline__ u64 scalar_addr(const void *p) {
  const u64 v = reinterpret_cast<u64>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ LaneRows lane_rows(const PropArgs &a, uint32_t d) {
  LaneRows r;
  r.col = (gu32_t *)(d ? scalar_addr(a.r.col) : scalar_addr(a.f.col));
  r.deg = (gu32_t *)(d ? scalar_addr(a.r.deg) : scalar_addr(a.f.deg));
  r.cap = (gu32_t *)(d ? scalar_addr(a.r.cap) : scalar_addr(a.f.cap));
  r.off = (gu64_t *)(d ? scalar_addr(a.r.off) : scalar_addr(a.f.off));
  return r;
}

// Lane `l`'s 64-bit value (two 32-bit lane reads; each half widened as unsigned: the builtin
// returns a signed int, which would spread bit 31 of the low half over the high half).
__device__ __forceinline__ u64 readlane_u64(u64 x, uint32_t l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)l);
  return ((u64)hi << 32) | lo;
}

// Both directions' row arrays as scalar global pointers (chosen per lane by a frontier entry's
// direction bit).
struct BothRows {
  LaneRows f, r;
};

__device__ __forceinline__ BothRows both_rows(const PropArgs &a) {
  BothRows b;
  b.f.col = (gu32_t *)scalar_addr(a.f.col);
  b.f.deg = (gu32_t *)scalar_addr(a.f.deg);
  b.f.cap = (gu32_t *)scalar_addr(a.f.cap);
  b.f.off = (gu64_t *)scalar_addr(a.f.off);
  b.r.col = (gu32_t *)scalar_addr(a.r.col);
  b.r.deg = (gu32_t *)scalar_addr(a.r.deg);
  b.r.cap = (gu32_t *)scalar_addr(a.r.cap);
  b.r.off = (gu64_t *)scalar_addr(a.r.off);
  return b;
}

// The propagation rounds of a small frontier by one wave (the stream's label-changing requests,
// which mostly reach a vertex or two): the frontier holds at most one entry per lane (vertex |
// direction bit where `fin` is set), all claimed with `stamp`. A round reads every entry's row
// and label half past L1, lays the rows end to end over the lanes (one edge per lane, at most 64
// edges), ORs the entry's label half into each target and claims a target that gained bits with
// the next stamp; the claimed targets are the next frontier (the rounds of Algorithm 3, as the
// workgroup's rounds run them). Returns true once a frontier is empty. A round that would scan
// more than 64 edges is not started: its frontier goes to the pending ring (ctl->cur, fsize,
// stamp) for the workgroup's rounds, and false is returned. Either way ctl->stamp and `stamp`
// end at the stamp of the last frontier, and the round counters are added to the statistics.
template <int W>
__device__ bool stream_rounds(const PropArgs &a, const BothRows &b, uint32_t fent, bool fin,
                              uint32_t ring, uint32_t fbase, uint32_t &stamp) {
  Ctl *ctl = a.ctl;
  const uint32_t lane = __lane_id();
  u64 relaxed = 0, expanded = 0;
  uint32_t rounds = 0;
  bool done = false;
  for (;;) {
    const u64 fm = __ballot(fin);
    if (!fm) {
      done = true;
      break;
    }
    const uint32_t x = fent & kIdMask, dir = fent >> 31;
    uint32_t dg = 0;
    u64 off = 0;
    Half<W> lv = {};
    if (fin) {
      const LaneRows &c = dir ? b.r : b.f;
      dg = min(c.deg[x], c.cap[x]);
      off = c.off[x];
      lv = ld_half_agent<W>(half_ptr<W>(a.L.lab, x, dir));
    }
    // all of the round's reads are waited for here (they arrive with the degrees): a read left
    // in flight where the frontier is handed on would be waited for, with every memory
    // operation after it, at the start of the stream's next window
    asm volatile("" ::"v"(off));
#pragma unroll
    for (int k = 0; k < 2 * W; k++) asm volatile("" ::"v"(lv.w[k]));
    // exclusive prefix of the row lengths over the lanes
    uint32_t incl = dg;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= (uint32_t)o) incl += y;
    }
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    if (total > 64u) {
      // too many edges for one wave: the workgroup's rounds take this frontier
      if (fin) a.fq[ring][fbase + lanemask_lt_popc(fm)] = fent;
      if (lane == 0) st_agent32(&ctl->fsize[ring], fbase + (uint32_t)__popcll(fm));
      break;
    }
    const uint32_t start = incl - dg;
    // every lane below `total` takes one edge: its owner entry is found by a scalar walk over
    // the entries that have edges (usually one or two)
    uint32_t e_dir = 0;
    u64 e_addr = 0;
    Half<W> src = {};
    bool has = false;
    for (u64 em = __ballot(fin && dg > 0); em; em &= em - 1) {
      const uint32_t f = (uint32_t)__builtin_ctzll(em);
      const uint32_t sf = __builtin_amdgcn_readlane(start, f);
      const uint32_t df = __builtin_amdgcn_readlane(dg, f);
      if (lane >= sf && lane < sf + df) {
        has = true;
        e_dir = __builtin_amdgcn_readlane(dir, f);
        e_addr = readlane_u64(off, f) + (lane - sf);
#pragma unroll
        for (int k = 0; k < 2 * W; k++) src.w[k] = readlane_u64(lv.w[k], f);
      }
    }
    const uint32_t nstamp = stamp + 1u;
    bool push = false;
    uint32_t y = 0;
    if (has) {
      y = (e_dir ? b.r.col : b.f.col)[e_addr];
      u64 *wy = half_ptr<W>(a.L.lab, y, e_dir);
      u64 gained = 0;
#pragma unroll
      for (int k = 0; k < 2 * W; k++)
        if (src.w[k]) gained |= src.w[k] & ~atomicOr(wy + k, src.w[k]);
      push = gained && atomicExch(&a.inq[2ull * y + e_dir], nstamp) != nstamp;
    }
    relaxed += total;
    expanded += (uint32_t)__popcll(fm);
    rounds++;
    stamp = nstamp;
    fin = push;
    fent = y | (e_dir ? kDirBit : 0u);
  }
  if (lane == 0) {
    st_agent32(&ctl->stamp, stamp);
    ctl->local_rounds += rounds;
    if (expanded) {
      a.pcnt[2 * (kRoundGridMax + kHeavyGrid)] += expanded;
      a.pcnt[2 * (kRoundGridMax + kHeavyGrid) + 1] += relaxed;
    }
  }
  return done;
}

template <int W>
__global__ __launch_bounds__(kLocalThreads) void k_insert_stream(
    PropArgs a, const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst,
    uint32_t first, uint32_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap, Mirror *m,
    uint32_t seq0, uint32_t *ticks) {
  __shared__ uint32_t s_cmd, s_i, s_flags;
  __shared__ uint32_t s_rowkey[2 * kStreamWindow];  // wave 0: each lane's row in the window
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x, lane = t & 63u, slot = lane >> 1, d = lane & 1u;
  uint32_t i = first;  // next request (wave 0)
  uint32_t flags = 0;  // wave 0
  u64 t_prev = 0, t_start = 0;
  if (t == 0) t_start = t_prev = wall_clock64();
  const LaneRows g = lane_rows(a, d);
  const BothRows rows = both_rows(a);
  for (;;) {
    if (t < 64u) {
      uint32_t cmd = kCmdExit;
      // values the whole wave shares are taken into scalar registers, so the compiler keeps
      // the request loops uniform (no per-lane exit masks)
      const uint32_t ring = __builtin_amdgcn_readfirstlane(ld_agent32(&ctl->cur));
      uint32_t stamp = __builtin_amdgcn_readfirstlane(ld_agent32(&ctl->stamp));
      // the pending frontier (empty)
      const uint32_t fbase = __builtin_amdgcn_readfirstlane(ld_agent32(&ctl->fsize[ring]));
      i = __builtin_amdgcn_readfirstlane(i);
      // The ids are read one window ahead: a window starts with its requests' ids in registers
      // (cu, cv: request i + slot) and reads the next window's (nu, nv: request i + 32 + slot)
      // with its labels, so it waits for one memory round trip instead of two. Only the first
      // window after the workgroup's rounds reads its own ids first.
      uint32_t cu, cv;
      {
        const uint32_t r = min(i + slot, count - 1u);
        cu = src[r];
        cv = dst[r];
        // waited for here: a read still in flight on the way into the loop would make every
        // window wait for all memory operations before its first instruction
        asm volatile("" ::"v"(cu), "v"(cv));
      }
      for (;;) {
        // the window's first request, as a scalar (the loop stays uniform)
        i = __builtin_amdgcn_readfirstlane(i);
        if (i >= count) break;
        const uint32_t nwin = min(kStreamWindow, count - i);
        const bool in_win = slot < nwin;
        const uint32_t r2 = min(i + kStreamWindow + slot, count - 1u);
        const uint32_t nu = src[r2], nv = dst[r2];
        const uint32_t u = cu, v = cv;
        const u64 badm = __ballot(in_win && (u >= n || v >= n));
        // requests up to the first one with a bad id
        const uint32_t nok =
            __builtin_amdgcn_readfirstlane(badm ? (uint32_t)__builtin_ctzll(badm) >> 1 : nwin);
        if (nok == 0) {  // request i has an id out of range: refused, nothing of it applied
          flags = kFastErr;
          break;
        }
        const bool act = slot < nok && u != v;
        const uint32_t tail = d ? v : u, head = d ? u : v;
        // Every lane reads (a lane without a request reads vertex 0's entries, which exist since
        // request i's ids are in range, and ignores them): reads under a lane mask would first
        // clear their registers, and the compiler holds that clear until the memory operations
        // before it, the previous window's stores among them, are done.
        const uint32_t rt = act ? tail : 0u, rh = act ? head : 0u;
        Half<W> lt = ld_half_agent<W>(half_ptr<W>(a.L.lab, rt, d));
        Half<W> lh = ld_half_agent<W>(half_ptr<W>(a.L.lab, rh, d));
        const uint32_t cap = g.cap[rt];
        const u64 off = g.off[rt];
        // past L1: this wave's earlier stores
        uint32_t deg = __hip_atomic_load(&g.deg[rt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // A lane's slot in its row: the row's degree at the window start plus the number of
        // earlier requests of the window that append to the same row (same direction), counted
        // once per window, so that the request loop below hands nothing between lanes. Each
        // lane publishes its row in LDS and reads the 32 rows of its direction, all reads
        // issued before the first compare (the empty asm needs every key at once); bit k of
        // `same` is set when the window's request k appends to this lane's row, and the
        // requests before this one are the bits below `slot`. A compare against `slot` per k
        // instead is a lane mask the compiler keeps for the whole launch, 64 scalar registers
        // that spill. The count needs only the ids, so it runs while the window's reads (and
        // the previous window's stores) are in flight.
        s_rowkey[lane] = act ? tail : 0xFFFFFFFFu;  // no vertex id is all ones
        // the wave's LDS operations run in order; this keeps the compiler from moving the reads
        // of the other lanes' entries above the write
        __builtin_amdgcn_wave_barrier();
        uint32_t key[kStreamWindow];
#pragma unroll
        for (uint32_t k = 0; k < kStreamWindow; k++) key[k] = s_rowkey[2 * k + d];
#pragma unroll
        for (uint32_t k = 0; k < kStreamWindow; k++) asm volatile("" ::"v"(key[k]));
        // shifted in from the last request down (no per-bit constants held in registers)
        uint32_t same = 0;
#pragma unroll
        for (int k = (int)kStreamWindow - 1; k >= 0; k--)
          same = 2u * same + (key[k] == tail ? 1u : 0u);
        const uint32_t rank = (uint32_t)__popc(same & ((1u << slot) - 1u));
        // Every read of the window is taken here, before its first request (an empty asm that
        // reads the registers, on every path): the wait for them then falls outside the request
        // loop. A wait inside it would also cover the stores of the request before (vector
        // stores count with the loads): one memory round trip per request.
        asm volatile("" ::"v"(deg), "v"(cap), "v"(off), "v"(nu), "v"(nv), "v"(rank));
#pragma unroll
        for (int k = 0; k < 2 * W; k++) asm volatile("" ::"v"(lt.w[k]), "v"(lh.w[k]));
        bool lane_newbits = false;
        if (act) {
          u64 nb = 0;
#pragma unroll
          for (int k = 0; k < 2 * W; k++) nb |= lt.w[k] & ~lh.w[k];
          lane_newbits = nb != 0ull;
          deg += rank;
        }
        // Whether a request is rare (a full row, or new label bits for its head) is known now:
        // the requests before the first rare one are the common ones, which only store, so
        // nothing in the window waits for memory. The rare request ends the window.
        const u64 rarem = __ballot(act && (lane_newbits || deg >= cap));
        const uint32_t stop =
            __builtin_amdgcn_readfirstlane(rarem ? (uint32_t)__builtin_ctzll(rarem) >> 1 : nok);
        uint32_t jj = 0;
        for (; jj < stop; jj++) {
          if (act && slot == jj) {
            g.col[off + deg] = head;
            g.deg[tail] = deg + 1u;
          }
          if (ticks && lane == 0) {
            const u64 now = wall_clock64();
            ticks[i + jj] = (uint32_t)(now - t_prev);
            t_prev = now;
          }
        }
        if (jj < nok) {
          // request i + jj, the rare one: its appends (the lane's own degree holds its slot)
          const bool mine = act && slot == jj;
          if (mine) {
            if (deg < cap) g.col[off + deg] = head;
            g.deg[tail] = deg + 1u;
          }
          const bool of = mine && deg >= cap;
          if (of) {
            const uint32_t k = atomicAdd(&ctl->ovf_count, 1u);
            if (k < ovf_cap) {
              Ovf o;
              o.x = tail | (d ? kDirBit : 0u);
              o.pos = deg;
              o.y = head;
              o.pad = 0;
              ovf[k] = o;
            }
          }
          // While the window runs no other wave writes labels and the head's half was read
          // past L1, so the head changes exactly when it gets new bits, and every propagation
          // left the frontier empty and advanced the stamp (no vertex holds this one): the
          // head's OR, its stamp and its frontier entry need no answer from memory.
          const bool p = mine && lane_newbits;
          if (p) {
            u64 *wh = half_ptr<W>(a.L.lab, head, d);
#pragma unroll
            for (int k = 0; k < 2 * W; k++)
              if (lt.w[k] & ~lh.w[k]) (void)atomicOr(wh + k, lt.w[k]);
            a.inq[2ull * head + d] = stamp;
          }
          // the head(s) that changed start the rounds: this wave alone while the frontier stays
          // small, else the workgroup's rounds from the pending ring
          if (__ballot(p) &&
              !stream_rounds<W>(a, rows, head | (d ? kDirBit : 0u), p, ring, fbase, stamp))
            cmd = kCmdPropagate;
          if (__ballot(of)) flags |= kFastOvf;
          if (ticks && lane == 0) {
            const u64 now = wall_clock64();
            ticks[i + jj] = (uint32_t)(now - t_prev);
            t_prev = now;
          }
          // the request that ended the window: done unless the workgroup's rounds still have to
          // finish it; a full row also ends the launch, for the host. Otherwise this wave's
          // rounds finished it and the next window starts after it (the later requests' label
          // reads may be stale).
          i += jj;
          if (cmd == kCmdExit) i++;
          if (cmd == kCmdPropagate || (flags & kFastOvf)) break;
          // the next window starts jj + 1 requests on: its ids are the rest of this window's
          // and the first of the next one's, moved down by jj + 1 slots
          const uint32_t s2 = slot + jj + 1u;
          const uint32_t from = 2u * (s2 & (kStreamWindow - 1u)) + d;
          const uint32_t au = __shfl(u, from), av = __shfl(v, from);
          const uint32_t bu = __shfl(nu, from), bv = __shfl(nv, from);
          cu = s2 < kStreamWindow ? au : bu;
          cv = s2 < kStreamWindow ? av : bv;
          continue;
        }
        i += nok;
        if (nok < nwin) {  // request i has an id out of range: refused, nothing of it applied
          flags = kFastErr;
          break;
        }
        cu = nu;
        cv = nv;
      }
      if (t == 0) {
        s_cmd = cmd;
        s_i = i;
        if (cmd == kCmdExit) {
          publish_fast(m, flags, seq0 + (i - first));
          ctl->ctr[kCtrServerTicks] += wall_clock64() - t_start;
          ctl->ctr[kCtrServerReqs] += i - first;
        } else {
          st_agent32(&ctl->heavy[0], 0u);
          st_agent32(&ctl->heavy[1], 0u);
        }
      }
      // the appends and label changes so far become visible to the other waves' rounds
      if (cmd == kCmdPropagate) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (s_cmd == kCmdExit) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    local_rounds_body<W>(a);
    __syncthreads();
    if (t == 0) {
      uint32_t fl = flags;
      if (ld_agent32(&ctl->fsize[ld_agent32(&ctl->cur)])) fl |= kFastPending;
      s_flags = fl;
      if (ticks) {
        const u64 now = wall_clock64();
        ticks[s_i] += (uint32_t)(now - t_prev);
        t_prev = now;
      }
      if (fl) {
        publish_fast(m, fl, seq0 + (s_i - first) + 1u);
        ctl->ctr[kCtrServerTicks] += wall_clock64() - t_start;
        ctl->ctr[kCtrServerReqs] += s_i - first + 1u;
      }
    }
    __syncthreads();
    if (s_flags) return;
    if (t < 64u) i = s_i + 1u;
  }
}

hipError_t launch_insert_stream(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                                uint32_t first, uint32_t count, uint32_t n, Ovf *ovf,
                                uint64_t ovf_cap, Mirror *m, uint32_t seq0, uint32_t *ticks,
                                hipStream_t s) {
  if (first >= count) return hipSuccess;
  DBL_LAUNCH_W(a.L.words, k_insert_stream, dim3(1), dim3(kLocalThreads), s, a, src, dst, first,
               count, n, ovf, ovf_cap, m, seq0, ticks);
  return hipGetLastError();
}

template <int W>
__global__ __launch_bounds__(256) void k_insert_apply(PropArgs a, const uint32_t *src,
                                                      const uint32_t *dst, uint64_t count,
                                                      Ovf *ovf, uint64_t ovf_cap) {
  Ctl *ctl = a.ctl;
  if (ctl->err) return;  // validation failed: leave the index untouched
  const uint32_t ring = ctl->cur, stamp = ctl->stamp;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->heavy[0] = 0;
    ctl->heavy[1] = 0;
  }
  // one half per thread (thread 2i: edge i forward, 2i + 1: backward), so the two halves'
  // dependent memory chains run side by side
  const uint64_t halves = 2 * count;
  for (uint64_t j0 = (uint64_t)blockIdx.x * blockDim.x; j0 < halves;
       j0 += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j = j0 + threadIdx.x;
    const bool act = j < halves;
    const uint64_t i = act ? j >> 1 : 0;
    bool ovfl = false;
    apply_half<W>(a, act ? src[i] : 0u, act ? dst[i] : 0u, (uint32_t)(j & 1u), ring, stamp, ovf,
                  ovf_cap, act, &ovfl);
  }
}

hipError_t launch_insert_apply(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint64_t count, Ovf *ovf, uint64_t ovf_cap, hipStream_t s) {
  DBL_LAUNCH_W(a.L.words, k_insert_apply, dim3(grid_for(2 * count, 256, 4096)), dim3(256), s, a,
               src, dst, count, ovf, ovf_cap);
  return hipGetLastError();
}

// ---- one insertion batch in one persistent launch
//
// The phases of Algorithm 3 for a whole batch follow each other inside one launch: validation of
// every id, the appends and seeds of every edge (both halves), then propagation. While the
// frontier is larger than one workgroup handles, every block expands it (grid rounds, with
// high-degree rows split into chunks handled after a barrier); once it is small, block 0
// finishes the rounds alone and the other blocks leave. A frontier above max_frontier, or one
// that block 0 cannot take on (it would scan more than local_max_edges), is left pending for the
// host's direction-optimised rounds.
//
// Before anything is modified, every block validates its share of the ids and then waits,
// bounded, until every block of the launch is resident (grid_gather). That wait ends the same
// way for every block: either all arrived, or one block, having waited too long, cancels the
// gathering before the last arrival, and then no block modifies anything (kErrStallEarly: the
// host runs the batch without this kernel). Once gathered, the blocks stay resident until they
// leave, so the later grid barriers (grid_barrier) only wait for the slowest block's share of a
// phase; their waits are bounded too, and a wait that runs out (kErrStallLate; it would take a
// share of seconds) leaves every block to finish its current phase and leave at its next
// barrier, after which the host re-propagates from every vertex. No wait is unbounded,
// whatever the occupancy.
//
// Every decision the blocks take after a barrier (where the frontier is and how large it is)
// comes from a snapshot that the last block to arrive takes while every other block still
// waits, so all blocks decide alike even when block 0 has already moved on and changed those
// fields again. Waiting blocks poll with plain device-scope loads and fence once when the wait
// is over: a polling load that also invalidated the cache would slow every other block.
//
// Synchronisation words, each on a 128-byte line of its own so that polling one does not slow
// the atomics on another: bar[kBarGather] blocks gathered (kGatherCancel once cancelled),
// bar[kBarCount] arrivals at the current barrier, bar[kBarGen] its generation followed by the
// snapshot {cur, stamp, fsize[cur]}, bar[kBarDone] blocks that have left (the last one resets the
// words and publishes).

constexpr uint32_t kGatherCancel = 0x80000000u;

__device__ bool grid_gather(uint32_t *bar, Ctl *ctl, uint32_t nblocks, u64 limit) {
  __shared__ uint32_t s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t *g = bar + kBarGather;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    uint32_t c = __hip_atomic_fetch_add(g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    const u64 t0 = wall_clock64();
    u64 spins = 0;
    while (c < nblocks) {  // c has the cancel bit once cancelled, which ends the loop too
      // past the time limit (or, should the clock stand still, as many polls as ticks)
      if (wall_clock64() - t0 > limit || ++spins > limit) {
        // cancel, unless the last block arrives first
        const uint32_t seen = atomicCAS(g, c, c | kGatherCancel);
        if (seen == c) {
          atomicOr(&ctl->err, kErrStallEarly);
          c |= kGatherCancel;
        } else {
          c = seen;
        }
        continue;
      }
      __builtin_amdgcn_s_sleep(2);
      c = __hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // every block's range check was made visible before its arrival
    s_ok = c == nblocks && !(ld_agent32(&ctl->err) & kErrRange);
  }
  __syncthreads();
  return s_ok != 0u;
}

struct Snap {
  uint32_t cur, stamp, fsz;
};

__device__ bool grid_barrier(uint32_t *bar, Ctl *ctl, uint32_t nblocks, u64 limit,
                             uint32_t stall_bit, Snap *snap) {
  __shared__ uint32_t s_ok;
  __shared__ Snap s_snap;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    uint32_t *gen = bar + kBarGen;
    const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t arrived = __hip_atomic_fetch_add(bar + kBarCount, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1u) {
      // every block has finished the phase: its results are final until the next barrier
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t cur = ld_agent32(&ctl->cur);
      st_agent32(gen + 1, cur);
      st_agent32(gen + 2, ld_agent32(&ctl->stamp));
      st_agent32(gen + 3, ld_agent32(&ctl->fsize[cur]));
      st_agent32(bar + kBarCount, 0u);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const u64 t0 = wall_clock64();
      u64 spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        ++spins;
        if ((spins & 63u) == 0u && (ld_agent32(&ctl->err) & (kErrStallEarly | kErrStallLate))) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > limit || spins > limit) {
          atomicOr(&ctl->err, stall_bit);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok && (ld_agent32(&ctl->err) & (kErrStallEarly | kErrStallLate))) ok = 0;
    // the snapshot stays as it is until this block has arrived at the next barrier
    if (ok) {
      s_snap.cur = ld_agent32(gen + 1);
      s_snap.stamp = ld_agent32(gen + 2);
      s_snap.fsz = ld_agent32(gen + 3);
    }
    s_ok = ok;
  }
  __syncthreads();
  *snap = s_snap;
  return s_ok != 0u;
}

template <int W>
__global__ __launch_bounds__(kLocalThreads) void k_insert_batch(
    PropArgs a, const uint32_t *src, const uint32_t *dst, uint64_t count, uint32_t n, Ovf *ovf,
    uint64_t ovf_cap, Mirror *m, uint32_t seq, uint32_t max_frontier, u64 start_ticks,
    u64 wait_ticks, uint32_t *bar) {
  __shared__ TileLds<W> sm;
  __shared__ uint32_t s_bad;
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x, nb = gridDim.x;
  const uint64_t halves = 2 * count;
  u64 relaxed = 0, expanded = 0;
  // state of the pending frontier as of the launch (the same in every block: every block reads
  // it before the gathering, and nothing changes it before)
  uint32_t ring = ld_agent32(&ctl->cur), stamp = ld_agent32(&ctl->stamp);
  Snap sn;
  {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * kLocalThreads + t; i < count;
         i += (uint64_t)nb * kLocalThreads)
      bad |= (src[i] >= n) | (dst[i] >= n);
    if (t == 0) s_bad = 0;
    __syncthreads();
    if (bad) s_bad = 1;
    __syncthreads();
    if (t == 0 && s_bad) atomicOr(&ctl->err, kErrRange);
  }
  // every block resident and every id checked; nothing is modified before this point
  bool go = grid_gather(bar, ctl, nb, start_ticks);
  if (go) {
    // Algorithm 3's first step for every edge: append, seed the head, queue it if it grew
    if (blockIdx.x == 0 && t == 0) {
      st_agent32(&ctl->heavy[0], 0u);
      st_agent32(&ctl->heavy[1], 0u);
      const uint32_t r1 = ring == 2u ? 0u : ring + 1u;
      st_agent32(&ctl->fsize[r1], 0u);
      st_agent32(&ctl->fsize[r1 == 2u ? 0u : r1 + 1u], 0u);
    }
    for (uint64_t j0 = (uint64_t)blockIdx.x * kLocalThreads; j0 < halves;
         j0 += (uint64_t)nb * kLocalThreads) {
      const uint64_t j = j0 + t;
      const bool act = j < halves;
      const uint64_t i = act ? j >> 1 : 0;
      bool ovfl = false;
      apply_half<W>(a, act ? src[i] : 0u, act ? dst[i] : 0u, (uint32_t)(j & 1u), ring, stamp,
                    ovf, ovf_cap, act, &ovfl);
    }
    go = grid_barrier(bar, ctl, nb, wait_ticks, kErrStallLate, &sn);
  }
  while (go) {
    ring = sn.cur;
    stamp = sn.stamp;
    const uint32_t fsz = sn.fsz;
    if (fsz == 0 || fsz > max_frontier) break;
    if (fsz <= a.local_max_frontier) {
      // small frontier: block 0 runs the remaining rounds alone and the other blocks leave; a
      // frontier that outgrows one workgroup again is left pending for the host
      if (blockIdx.x == 0) local_rounds_core<W>(a, sm);
      break;
    }
    // one round over every block: frontier tiles of kLocalThreads entries, long rows deferred.
    // Block 0 records the round's bookkeeping.
    const uint32_t nring = ring == 2u ? 0u : ring + 1u;
    if (blockIdx.x == 0 && t == 0) {
      st_agent32(&ctl->fsize[nring == 2u ? 0u : nring + 1u], 0u);
      st_agent32(&ctl->heavy[(stamp + 1u) & 1u], 0u);
      st_agent32(&ctl->cur, nring);
      st_agent32(&ctl->stamp, stamp + 1u);
    }
    for (uint32_t beg = blockIdx.x * kLocalThreads; beg < fsz; beg += nb * kLocalThreads) {
      const uint32_t end = min(beg + kLocalThreads, fsz);
      expand_tile<kLocalThreads, W>(a, a.fq[ring], beg, end, a.fq[nring], &ctl->fsize[nring],
                                    stamp + 1u, a.heavy_list, &ctl->heavy[stamp & 1u], true,
                                    sm.start, sm.off, sm.lab, sm.ent, sm.wsum, relaxed, expanded,
                                    0u);
    }
    go = grid_barrier(bar, ctl, nb, wait_ticks, kErrStallLate, &sn);
    if (!go) break;
    // the deferred chunks of long rows, one chunk per block at a time (the count is final: the
    // phase that adds to it ended at the barrier, and it is cleared only after the next one)
    uint32_t hcnt = ld_agent32(&ctl->heavy[stamp & 1u]);
    if (hcnt > a.heavy_cap) hcnt = (uint32_t)a.heavy_cap;
    for (uint32_t item = blockIdx.x; item < hcnt; item += nb) {
      const u64 h = a.heavy_list[item];
      const uint32_t ent = (uint32_t)(h >> 32), c = (uint32_t)h;
      const uint32_t dir = ent >> 31, x = ent & kIdMask;
      const Csr g = dir ? a.r : a.f;
      const uint32_t dg = min(g.deg[x], g.cap[x]);
      const uint32_t b = c * kChunk, e_end = min(dg, b + kChunk);
      const Half<W> lv = ld_half_agent<W>(half_ptr<W>(a.L.lab, x, dir));
      const u64 o = g.off[x];
      for (uint32_t e0 = b; e0 < e_end; e0 += kLocalThreads) {
        const uint32_t e = e0 + t;
        bool push = false;
        uint32_t y = 0;
        if (e < e_end) {
          y = g.col[o + e];
          push = relax<W>(half_ptr<W>(a.L.lab, y, dir), lv) &&
                 claim(&a.inq[2ull * y + dir], stamp + 1u);
        }
        wave_push(a.fq[nring], &ctl->fsize[nring], push, y | (ent & kDirBit));
      }
      if (t == 0) relaxed += e_end > b ? e_end - b : 0;
    }
    go = grid_barrier(bar, ctl, nb, wait_ticks, kErrStallLate, &sn);
  }
  if (t == 0 && (expanded | relaxed)) {
    a.pcnt[2 * blockIdx.x] += expanded;
    a.pcnt[2 * blockIdx.x + 1] += relaxed;
  }
  // ctl->cur / ctl->stamp already say where the frontier stands (kept by block 0). The last
  // block to leave resets the synchronisation words and publishes.
  __syncthreads();
  if (t == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t done = __hip_atomic_fetch_add(bar + kBarDone, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done == nb - 1u) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      st_agent32(bar + kBarDone, 0u);
      st_agent32(bar + kBarGather, 0u);
      st_agent32(bar + kBarCount, 0u);
      const uint32_t err = ld_agent32(&ctl->err);
      uint32_t flags = 0;
      if (err) flags |= kFastErr;
      if (ld_agent32(&ctl->ovf_count)) flags |= kFastOvf;
      if (ld_agent32(&ctl->fsize[ld_agent32(&ctl->cur)])) flags |= kFastPending;
      publish_fast(m, flags, seq);
    }
  }
}

hipError_t insert_batch_grid(uint32_t words, BatchLaunch *out) {
  const void *f = nullptr;
  switch (words) {
    case 1: f = (const void *)k_insert_batch<1>; break;
    case 2: f = (const void *)k_insert_batch<2>; break;
    case 4: f = (const void *)k_insert_batch<4>; break;
    default: return hipErrorInvalidValue;
  }
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, (int)kLocalThreads, 0);
  if (e != hipSuccess) return e;
  if (cus <= 0 || per_cu <= 0) return hipErrorInvalidValue;
  out->func = f;
  // one block per compute unit (blocks of 16 waves; more per unit only lengthen the barriers)
  out->grid = (uint32_t)std::min<int>(cus, (int)kRoundGridMax);
  return hipSuccess;
}

hipError_t launch_insert_batch(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint64_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap, Mirror *m,
                               uint32_t seq, uint32_t max_frontier, u64 start_ticks,
                               u64 wait_ticks, uint32_t *bar, uint32_t grid, hipStream_t s) {
  DBL_LAUNCH_W(a.L.words, k_insert_batch, dim3(grid), dim3(kLocalThreads), s, a, src, dst, count,
               n, ovf, ovf_cap, m, seq, max_frontier, start_ticks, wait_ticks, bar);
  return hipGetLastError();
}

hipError_t insert_batch_node_params(uint32_t words, uint32_t grid, void **args,
                                    hipKernelNodeParams *p) {
  const void *f = nullptr;
  switch (words) {
    case 1: f = (const void *)k_insert_batch<1>; break;
    case 2: f = (const void *)k_insert_batch<2>; break;
    case 4: f = (const void *)k_insert_batch<4>; break;
    default: return hipErrorInvalidValue;
  }
  *p = hipKernelNodeParams{};
  p->func = const_cast<void *>(f);
  p->gridDim = dim3(grid);
  p->blockDim = dim3(kLocalThreads);
  p->kernelParams = args;
  return hipSuccess;
}

// Copy every row of old_g into new_g (same deg array; new offsets and capacities). A block takes
// 256 consecutive rows at a time, lays their entries end to end (prefix sum of the degrees in
// LDS) and copies them one entry per thread, so reads and writes both run along the rows
// however short or long they are.
constexpr uint32_t kCopyUnroll = 4;

__global__ __launch_bounds__(256) void k_regrow_copy(Csr old_g, Csr new_g, uint32_t n) {
  __shared__ uint32_t s_start[256];
  __shared__ u64 s_src[256], s_dst[256];
  __shared__ uint32_t s_wsum[4];
  const uint32_t t = threadIdx.x;
  for (uint32_t beg = blockIdx.x * 256u; beg < n; beg += gridDim.x * 256u) {
    const uint32_t x = beg + t;
    uint32_t d = 0;
    if (x < n) {
      d = min(old_g.deg[x], old_g.cap[x]);
      s_src[t] = old_g.off[x];
      s_dst[t] = new_g.off[x];
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan<256>(d, s_wsum, total);
    s_start[t] = ex;
    __syncthreads();
    const uint32_t last = min(256u, n - beg) - 1u;
    // kCopyUnroll entries per thread at a time, all their reads in flight together; a thread's
    // entries only move forward, so each row search starts from the row found before
    uint32_t lo = 0;
    for (uint32_t e0 = t; e0 < total; e0 += 256u * kCopyUnroll) {
      uint32_t v[kCopyUnroll];
      u64 to[kCopyUnroll];
#pragma unroll
      for (uint32_t j = 0; j < kCopyUnroll; j++) {
        const uint32_t e = e0 + 256u * j;
        if (e < total) {
          uint32_t hi = last;
          while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
          }
          const uint32_t k = e - s_start[lo];
          to[j] = s_dst[lo] + k;
          v[j] = old_g.col[s_src[lo] + k];
        }
      }
#pragma unroll
      for (uint32_t j = 0; j < kCopyUnroll; j++)
        if (e0 + 256u * j < total) new_g.col[to[j]] = v[j];
    }
    __syncthreads();
  }
}

hipError_t launch_regrow_copy(Csr old_g, Csr new_g, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_regrow_copy, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, old_g, new_g,
                     n);
  return hipGetLastError();
}

__global__ void k_place_overflow(const Ovf *ovf, uint32_t count, uint32_t dir, Csr g) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const Ovf o = ovf[i];
    if ((o.x >> 31) != dir) continue;
    const uint32_t x = o.x & kIdMask;
    g.col[g.off[x] + o.pos] = o.y;
  }
}

hipError_t launch_place_overflow(const Ovf *ovf, uint32_t count, uint32_t dir, Csr new_g,
                                 hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_place_overflow, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, ovf,
                     count, dir, new_g);
  return hipGetLastError();
}

// After a regrow, the tail of each overflowed edge re-enters the pending frontier so that its
// label flows over the edge that was missing from the CSR during the first propagation.
__global__ void k_push_overflow(PropArgs a, const Ovf *ovf, uint32_t count) {
  Ctl *ctl = a.ctl;
  const uint32_t ring = ctl->cur, stamp = ctl->stamp;
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < count; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    bool p = false;
    uint32_t ent = 0;
    if (i < count) {
      ent = ovf[i].x;
      const uint32_t x = ent & kIdMask, dir = ent >> 31;
      p = claim(&a.inq[2ull * x + dir], stamp);
    }
    wave_push(a.fq[ring], &ctl->fsize[ring], p, ent);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->heavy[0] = 0;
    ctl->heavy[1] = 0;
  }
}

hipError_t launch_push_overflow(const PropArgs &a, const Ovf *ovf, uint32_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  // one block: the pending frontier's ring and stamp are read once per thread from ctl
  hipLaunchKernelGGL(k_push_overflow, dim3(1), dim3(256), 0, s, a, ovf, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------- queries

// Label phase of Algorithm 2: one lane per pair. Decided pairs get their answer byte now.
// A pair the rules leave open whose source has no out-edge is answered here too: the BFS from u
// would scan nothing, so the answer is "BFS false". The remaining pairs are compacted per block
// into und[block * kQueryNT ...] with their number in seg[block] (no shared counter).
template <int W>
__global__ __launch_bounds__(kQueryNT) void k_query_label(const u64 *lab, const uint32_t *qu,
                                                          const uint32_t *qv, uint64_t count,
                                                          uint32_t n, const uint32_t *fdeg,
                                                          uint8_t *out, uint32_t *und,
                                                          uint32_t *seg, Ctl *ctl, u64 *qcls,
                                                          uint32_t rules) {
  __shared__ uint32_t s_cls[kQueryNT / 64][8];
  __shared__ uint32_t s_und[kQueryNT / 64];
  const uint64_t i = (uint64_t)blockIdx.x * kQueryNT + threadIdx.x;
  const bool act = i < count;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // per-call counters of the BFS kernel that follows on the stream
    ctl->bfs_heavy = 0;
    ctl->bfs_done = 0;
  }
  int cls = -1;
  bool undecided = false, bad = false;
  if (act) {
    const uint32_t u = qu[i], v = qv[i];
    if (u >= n || v >= n) {
      bad = true;
      out[i] = 0xFF;
    } else if (u == v) {
      cls = 0;
    } else {
      // fu = {DL_in(u), BL_in(u)}, bu = {DL_out(u), BL_out(u)}, likewise for v
      const Half<W> fu = ld_half<W>(half_ptr<W>(lab, u, 0)), bu = ld_half<W>(half_ptr<W>(lab, u, 1));
      const Half<W> fv = ld_half<W>(half_ptr<W>(lab, v, 0)), bv = ld_half<W>(half_ptr<W>(lab, v, 1));
      u64 l1 = 0, l2 = 0, t1 = 0, t2 = 0;
#pragma unroll
      for (int j = 0; j < W; j++) {
        l1 |= bu.w[j] & fv.w[j];
        l2 |= (fu.w[W + j] & ~fv.w[W + j]) | (bv.w[W + j] & ~bu.w[W + j]);
        t1 |= bv.w[j] & fu.w[j];
        t2 |= (bu.w[j] & fu.w[j]) | (bv.w[j] & fv.w[j]);
      }
      // a disabled label reads as 0 for the rules that use it (the ablations of Table 4)
      const bool dl = rules & 1u, bl = (rules & 2u) != 0;
      if (dl && l1) cls = 1;                   // Lemma 1
      else if (bl && l2) cls = 2;              // Lemma 2
      else if (dl && t1) cls = 3;              // Theorem 1
      else if (dl && t2) cls = 4;              // Theorem 2
      else if (fdeg[u] == 0) cls = 6;          // empty BFS
      else undecided = true;
    }
    if (cls >= 0) out[i] = (uint8_t)((cls <= 1 ? 1u : 0u) | ((uint32_t)cls << 1));
  }
  const uint32_t lane = __lane_id(), w = threadIdx.x >> 6;
  const u64 um = __ballot(undecided);
  // every lane takes part in the ballots (a ballot only sees the lanes that execute it)
  uint32_t ccount[7];
#pragma unroll
  for (int c = 0; c < 7; c++) ccount[c] = (uint32_t)__popcll(__ballot(cls == c));
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 7; c++) s_cls[w][c] = ccount[c];
    s_und[w] = (uint32_t)__popcll(um);
  }
  if (__ballot(bad) && lane == 0) atomicOr(&ctl->err, kErrRange);
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (uint32_t j = 0; j < kQueryNT / 64; j++) {
    if (j < w) base += s_und[j];
    tot += s_und[j];
  }
  if (undecided)
    und[(uint64_t)blockIdx.x * kQueryNT + base + lanemask_lt_popc(um)] = (uint32_t)i;
  if (threadIdx.x == 0) seg[blockIdx.x] = tot;
  if (threadIdx.x < 7) {
    const uint32_t c = threadIdx.x;
    uint32_t sum = 0;
    for (uint32_t j = 0; j < kQueryNT / 64; j++) sum += s_cls[j][c];
    if (sum) atomicAdd(&qcls[(blockIdx.x % kQueryGrid) * kQClsStride + c], (u64)sum);
  }
}

hipError_t launch_query_label(LabelsView L, const uint32_t *u, const uint32_t *v, uint64_t count,
                              uint32_t n, const uint32_t *fdeg, uint8_t *out, uint32_t *und,
                              uint32_t *seg, Ctl *ctl, u64 *qcls, uint32_t rules, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint64_t blocks = (count + kQueryNT - 1) / kQueryNT;
  DBL_LAUNCH_W(L.words, k_query_label, dim3((uint32_t)blocks), dim3(kQueryNT), s, L.lab, u, v,
               count, n, fdeg, out, und, seg, ctl, qcls, rules);
  return hipGetLastError();
}

// Pruned BFS of Algorithm 2, one wavefront per undecided pair. A search runs first in the wave's
// LDS: a queue of up to kBfsLdsQ vertices and an open-addressing visited set, so that no step
// of a small search waits for a global queue write to come back or for a global atomic. A
// search that outgrows the LDS queue starts again over the slot's global queue and visited
// bitmap (up to the context's queue capacity); one that outgrows that goes to the whole-device
// BFS. The queue is processed 64 entries at a time: their rows are laid end to end and every
// lane takes one edge (a prefix sum over the lanes' degrees maps edge slots to rows), so short
// and long rows both keep the lanes busy. Prunes: a target x is skipped when a landmark of u
// reaches it (DL_out(u) & DL_in(x)) or when it cannot reach v (BL_Contain(x, v) fails).
constexpr uint32_t kBfsNT = 256;
constexpr uint32_t kBfsLdsQ = 1024, kBfsHashBits = 11, kBfsHash = 1u << kBfsHashBits;
constexpr uint32_t kBfsEmpty = 0xFFFFFFFFu;

// The prune of Algorithm 2 for a target x with record rx, against the query's wave-uniform
// label words: skip x when DL_out(u) & DL_in(x) != 0 or when BL_in(x) is not inside BL_in(v) or
// BL_out(v) is not inside BL_out(x).
template <int W>
__device__ __forceinline__ bool bfs_prune(const u64 *rx, const u64 *dlo_u, const u64 *bli_v,
                                          const u64 *blo_v) {
  const Half<W> fx = ld_half<W>(rx);
  u64 hit = 0;
#pragma unroll
  for (int j = 0; j < W; j++)
    hit |= (dlo_u[j] & fx.w[j]) | (fx.w[W + j] & ~bli_v[j]) | (blo_v[j] & ~rx[3 * W + j]);
  return hit != 0ull;
}

// The query's side of the prune; a disabled label prunes nothing: DL_out(u) = 0, BL_in(v) =
// all, BL_out(v) = none.
template <int W>
__device__ __forceinline__ void bfs_prune_words(const u64 *lab, uint32_t u, uint32_t v,
                                                uint32_t rules, u64 *dlo_u, u64 *bli_v,
                                                u64 *blo_v) {
  const u64 *ru = lab + 4ull * W * u, *rv = lab + 4ull * W * v;
#pragma unroll
  for (int j = 0; j < W; j++) {
    dlo_u[j] = (rules & 1u) ? ru[2 * W + j] : 0ull;
    bli_v[j] = (rules & 2u) ? rv[W + j] : ~0ull;
    blo_v[j] = (rules & 2u) ? rv[3 * W + j] : 0ull;
  }
}

// Insert x into a wave's LDS visited set (linear probing); true when x was not in it. The set
// never holds more than kBfsLdsQ + 64 ids (inserts stop once the queue is full), so a probe
// always reaches a free slot.
__device__ __forceinline__ bool lds_visit(uint32_t *h, uint32_t x) {
  uint32_t i = (x * 2654435761u) >> (32 - kBfsHashBits);
  for (;;) {
    const uint32_t old = atomicCAS(&h[i], kBfsEmpty, x);
    if (old == kBfsEmpty) return true;
    if (old == x) return false;
    i = (i + 1u) & (kBfsHash - 1u);
  }
}

// One pruned BFS from u toward v over the forward rows, with the queue at qp (capacity cap)
// and the visited set in LDS (LOCAL, hs) or in the bitmap vis. Returns 1 when v is reached, 0
// when the search is exhausted, 2 when the queue would exceed cap (then, in the bitmap form,
// every set bit is listed in the queue). *tail_out: the queue length at the end.
template <int W, bool LOCAL>
__device__ uint32_t bfs_run(const BfsArgs &a, uint32_t u, uint32_t v, const u64 *dlo_u,
                            const u64 *bli_v, const u64 *blo_v, uint32_t *qp, u64 *vis,
                            uint32_t *hs, uint32_t cap, uint32_t *tail_out, u64 &n_vert,
                            u64 &n_edge) {
  const uint32_t lane = __lane_id();
  const u64 *lab = a.L.lab;
  if (lane == 0) {
    if (LOCAL) lds_visit(hs, u);
    else atomicOr(&vis[u >> 6], 1ull << (u & 63u));
    qp[0] = u;
  }
  uint32_t head = 0, tail = 1, st = 0;
  while (head < tail) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint32_t chunk = min(64u, tail - head);
    uint32_t d = 0;
    u64 o = 0;
    if (lane < chunk) {
      const uint32_t w = qp[head + lane];
      d = min(a.f.deg[w], a.f.cap[w]);
      o = a.f.off[w];
    }
    const uint32_t incl = wave_incl_scan(d);
    const uint32_t ex = incl - d;
    const uint32_t total = __shfl(incl, 63, 64);
    n_vert += chunk;
    n_edge += total;
    for (uint32_t base = 0; base < total; base += 64u) {
      const uint32_t e = base + lane;
      // owner row of edge slot e: the last lane whose exclusive prefix is <= e
      uint32_t lo = 0;
#pragma unroll
      for (uint32_t step = 32; step > 0; step >>= 1) {
        const uint32_t cand = lo + step;
        const uint32_t stt = __shfl(ex, (int)cand, 64);
        if (cand < 64u && stt <= e) lo = cand;
      }
      const u64 ow_off = __shfl(o, (int)lo, 64);
      const uint32_t ow_ex = __shfl(ex, (int)lo, 64);
      const bool act = e < total;
      uint32_t x = 0;
      if (act) x = a.f.col[ow_off + (e - ow_ex)];
      if (__ballot(act && x == v)) {
        st = 1;
        break;
      }
      bool keep = false;
      u64 bit = 0;
      if (act) {
        keep = !bfs_prune<W>(lab + 4ull * W * x, dlo_u, bli_v, blo_v);
        if (keep) {
          if (LOCAL) {
            keep = lds_visit(hs, x);
          } else {
            bit = 1ull << (x & 63u);
            keep = !(atomicOr(&vis[x >> 6], bit) & bit);
          }
        }
      }
      const u64 km = __ballot(keep);
      const uint32_t cnt = (uint32_t)__popcll(km);
      if (tail + cnt > cap) {
        if (!LOCAL && keep) atomicAnd(&vis[x >> 6], ~bit);  // every set bit stays listed
        st = 2;
        break;
      }
      if (keep) qp[tail + lanemask_lt_popc(km)] = x;
      tail += cnt;
    }
    if (st) break;
    head += chunk;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  *tail_out = tail;
  return st;
}

// Undecided pairs sit in per-block segments of the label kernel; wave `slot` takes segments
// slot, slot + waves, ..., reading 64 segment counts at a time (one per lane).
template <int W>
__global__ __launch_bounds__(kBfsNT) void k_query_bfs(BfsArgs a, Mirror *m, uint32_t seq) {
  __shared__ uint32_t s_q[kBfsNT / 64][kBfsLdsQ];
  __shared__ uint32_t s_h[kBfsNT / 64][kBfsHash];
  Ctl *ctl = a.ctl;
  const uint32_t lane = __lane_id(), wv = threadIdx.x >> 6;
  const uint32_t slot = blockIdx.x * (kBfsNT / 64u) + wv;
  u64 *vis = a.vis + (uint64_t)slot * a.vis_words;
  uint32_t *q = a.queue + (uint64_t)slot * a.qcap;
  uint32_t *sq = s_q[wv], *hs = s_h[wv];
  const uint32_t waves = gridDim.x * (kBfsNT / 64u);
  const uint32_t lcap = min(kBfsLdsQ, a.qcap);
  const u64 *lab = a.L.lab;
  u64 n_vert = 0, n_edge = 0, cls_t = 0, cls_f = 0;
  for (uint32_t i = lane; i < kBfsHash; i += 64u) hs[i] = kBfsEmpty;
  // one undecided pair: the search in LDS, then over the slot's global queue, else handed on
  auto search = [&](uint32_t qi) {
    const uint32_t u = a.u[qi], v = a.v[qi];
    u64 dlo_u[W], bli_v[W], blo_v[W];
    bfs_prune_words<W>(lab, u, v, a.rules, dlo_u, bli_v, blo_v);
    uint32_t tail = 0;
    uint32_t st = bfs_run<W, true>(a, u, v, dlo_u, bli_v, blo_v, sq, vis, hs, lcap, &tail,
                                   n_vert, n_edge);
    for (uint32_t i = lane; i < kBfsHash; i += 64u) hs[i] = kBfsEmpty;
    if (st == 2 && a.qcap > lcap) {
      // too large for LDS: again over the slot's global queue and bitmap
      st = bfs_run<W, false>(a, u, v, dlo_u, bli_v, blo_v, q, vis, hs, a.qcap, &tail, n_vert,
                             n_edge);
      for (uint32_t i = lane; i < tail; i += 64u) atomicExch(&vis[q[i] >> 6], 0ull);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane == 0) {
      if (st == 2) {
        const uint32_t h = atomicAdd(&ctl->bfs_heavy, 1u);
        a.heavy_q[h] = qi;
      } else {
        a.out[qi] = st == 1 ? (uint8_t)(1u | (5u << 1)) : (uint8_t)(6u << 1);
        if (st == 1) cls_t++; else cls_f++;
      }
    }
  };
  if (a.nseg >= waves) {
    for (uint64_t sb = slot; sb < a.nseg; sb += 64ull * waves) {
      const uint64_t my = sb + (uint64_t)lane * waves;
      const uint32_t mycnt = my < a.nseg ? a.seg[my] : 0u;
      u64 busy = __ballot(mycnt != 0u);
      while (busy) {
        const uint32_t k = (uint32_t)__builtin_ctzll(busy);
        busy &= busy - 1ull;
        const uint64_t sg = sb + (uint64_t)k * waves;
        const uint32_t scnt = __shfl(mycnt, (int)k, 64);
        for (uint32_t sj = 0; sj < scnt; sj++) search(a.und[sg * kQueryNT + sj]);
      }
    }
  } else if (a.nseg > 0) {
    // fewer segments than waves (a small batch): the pairs of each segment are dealt round
    // robin to waves / nseg waves, so that many searches of one segment run side by side
    const uint32_t wps = waves / a.nseg, sg = slot / wps, sub = slot - sg * wps;
    if (sg < a.nseg) {
      const uint32_t scnt = a.seg[sg];
      for (uint32_t sj = sub; sj < scnt; sj += wps) search(a.und[(uint64_t)sg * kQueryNT + sj]);
    }
  }
  if (lane == 0 && (n_vert | cls_t | cls_f)) {
    u64 *c = a.cnt + (uint64_t)slot * kBfsCtrStride;  // this wave's own counters
    c[0] += n_vert;
    c[1] += n_edge;
    c[2] += cls_t;
    c[3] += cls_f;
  }
  // The last block to finish publishes; one done count per block, not per wave (atomics on one
  // address are served one at a time, ~10 ns each). No device-wide fence: on a multi-XCD device
  // each one writes back and invalidates the XCD's L2 under the waves still searching. The
  // answers are only read through work ordered after this kernel on its stream, and the status
  // fields are device-scope atomics that every wave has seen performed (it waited for their
  // results) before the block's done count.
  __syncthreads();
  if (threadIdx.x == 0 && atomicAdd(&ctl->bfs_done, 1u) == gridDim.x - 1u)
    publish_status(ctl, m, seq);
}

hipError_t launch_query_bfs(const BfsArgs &a, uint32_t slots, Mirror *m, uint32_t seq,
                            hipStream_t s) {
  DBL_LAUNCH_W(a.L.words, k_query_bfs, dim3(slots / (kBfsNT / 64u)), dim3(kBfsNT), s, a, m, seq);
  return hipGetLastError();
}

// Graph-node form of a query batch: the two kernels of launch_query_label and
// launch_query_bfs with their launch shapes and arguments (pointed to, in kernel order).
hipError_t query_node_params(LabelsView L, uint64_t count, uint32_t slots, void **label_args,
                             void **bfs_args, hipKernelNodeParams *label,
                             hipKernelNodeParams *bfs) {
  const void *fl = nullptr, *fb = nullptr;
  switch (L.words) {
    case 1: fl = (const void *)k_query_label<1>; fb = (const void *)k_query_bfs<1>; break;
    case 2: fl = (const void *)k_query_label<2>; fb = (const void *)k_query_bfs<2>; break;
    case 4: fl = (const void *)k_query_label<4>; fb = (const void *)k_query_bfs<4>; break;
    default: return hipErrorInvalidValue;
  }
  *label = hipKernelNodeParams{};
  label->func = const_cast<void *>(fl);
  label->gridDim = dim3((uint32_t)((count + kQueryNT - 1) / kQueryNT));
  label->blockDim = dim3(kQueryNT);
  label->kernelParams = label_args;
  *bfs = hipKernelNodeParams{};
  bfs->func = const_cast<void *>(fb);
  bfs->gridDim = dim3(slots / (kBfsNT / 64u));
  bfs->blockDim = dim3(kBfsNT);
  bfs->kernelParams = bfs_args;
  return hipSuccess;
}

// ---- whole-device BFS for one pair whose slot queue overflowed (rare)
//
// The pair is searched from both ends: side 0 follows out-edges from u, side 1 in-edges from v,
// one side per launch (the host picks the side whose pending level has fewer edges). Each side
// has a visited bitmap and one queue whose levels are consecutive segments. A side that reaches
// a vertex the other side has visited has found a path. A vertex on a path from u to v passes
// both sides' prunes (the prunes only drop vertices that cannot be on such a path while the
// labels left the pair undecided), so every path is found, and a side whose level comes out
// empty has shown that none exists.

__global__ void k_gbfs_start(GbfsArgs a, uint32_t u, uint32_t v) {
  Ctl *ctl = a.ctl;
  a.vis[0][u >> 6] |= 1ull << (u & 63u);
  a.vis[1][v >> 6] |= 1ull << (v & 63u);
  a.q[0][0] = u;
  a.q[1][0] = v;
  ctl->fsize[0] = 1;
  ctl->fsize[1] = 1;
  ctl->fsize[2] = 0;
  ctl->found = u == v ? 1u : 0u;
  ctl->ctr[kCtrFrontEdges] = min(a.g[0].deg[u], a.g[0].cap[u]);
  ctl->ctr[kCtrFrontEdges + 1] = min(a.g[1].deg[v], a.g[1].cap[v]);
}

hipError_t launch_gbfs_start(const GbfsArgs &a, uint64_t vis_words, uint32_t u, uint32_t v,
                             hipStream_t s) {
  hipError_t e = launch_fill_u64(a.vis[0], 0ull, vis_words, s);
  if (e == hipSuccess) e = launch_fill_u64(a.vis[1], 0ull, vis_words, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gbfs_start, dim3(1), dim3(1), 0, s, a, u, v);
  return hipGetLastError();
}

// The query's words of one side's prune (a disabled label prunes nothing). Side 0 skips a target
// x when DL_out(u) & DL_in(x) != 0 (u reaches x through a landmark, so x reaching v would have
// decided the pair by Theorem 1), when BL_in(x) is not inside BL_in(v) or when BL_out(v) is not
// inside BL_out(x) (x cannot reach v, Lemma 2). Side 1 mirrors it for a source y of v: DL_out(y)
// & DL_in(v) != 0, BL_in(u) not inside BL_in(y), or BL_out(y) not inside BL_out(u) (u cannot
// reach y).
template <int W>
__device__ __forceinline__ void gbfs_prune_words(const u64 *lab, uint32_t u, uint32_t v,
                                                 uint32_t side, uint32_t rules, u64 *dl, u64 *bi,
                                                 u64 *bo) {
  const u64 *ru = lab + 4ull * W * u, *rv = lab + 4ull * W * v;
  const bool use_dl = rules & 1u, use_bl = rules & 2u;
#pragma unroll
  for (int j = 0; j < W; j++) {
    if (side == 0) {
      dl[j] = use_dl ? ru[2 * W + j] : 0ull;
      bi[j] = use_bl ? rv[W + j] : ~0ull;
      bo[j] = use_bl ? rv[3 * W + j] : 0ull;
    } else {
      dl[j] = use_dl ? rv[j] : 0ull;
      bi[j] = use_bl ? ru[W + j] : 0ull;
      bo[j] = use_bl ? ru[3 * W + j] : ~0ull;
    }
  }
}

template <int W>
__device__ __forceinline__ bool gbfs_prune(const u64 *rx, uint32_t side, const u64 *dl,
                                           const u64 *bi, const u64 *bo) {
  u64 hit = 0;
  if (side == 0) {
#pragma unroll
    for (int j = 0; j < W; j++)
      hit |= (dl[j] & rx[j]) | (rx[W + j] & ~bi[j]) | (bo[j] & ~rx[3 * W + j]);
  } else {
#pragma unroll
    for (int j = 0; j < W; j++)
      hit |= (dl[j] & rx[2 * W + j]) | (bi[j] & ~rx[W + j]) | (rx[3 * W + j] & ~bo[j]);
  }
  return hit != 0ull;
}

// One level of one side: the level's queue segment [lo, hi) in tiles of 256 vertices, their rows
// laid end to end (prefix sum of the degrees in LDS) and one edge per thread, so a long row is
// spread over the block instead of being walked by one thread. A target already visited on this
// side is dropped on a plain load of its bitmap word before its labels are read; the atomic OR
// that claims it comes after the prune. Every claimed vertex adds its degree to the side's
// summed degrees (the next level's edges).
template <int W>
__global__ __launch_bounds__(256) void k_gbfs_round(GbfsArgs a, uint32_t side, uint32_t lo,
                                                    uint32_t hi, uint32_t u, uint32_t v,
                                                    uint32_t rules) {
  __shared__ uint32_t s_start[256];
  __shared__ u64 s_off[256];
  __shared__ uint32_t s_wsum[4];
  Ctl *ctl = a.ctl;
  const uint32_t t = threadIdx.x;
  const Csr g = a.g[side];
  u64 *vs = a.vis[side];
  const u64 *vo = a.vis[side ^ 1u];
  uint32_t *qs = a.q[side];
  const u64 *lab = a.L.lab;
  u64 dl[W], bi[W], bo[W];
  gbfs_prune_words<W>(lab, u, v, side, rules, dl, bi, bo);
  bool found = false;
  const uint32_t fsz = hi - lo;
  for (uint32_t beg = blockIdx.x * 256u; beg < fsz; beg += gridDim.x * 256u) {
    const uint32_t i = beg + t;
    uint32_t d = 0;
    if (i < fsz) {
      const uint32_t w = qs[lo + i];
      d = min(g.deg[w], g.cap[w]);
      s_off[t] = g.off[w];
    }
    uint32_t total;
    const uint32_t ex = block_excl_scan<256>(d, s_wsum, total);
    s_start[t] = ex;
    __syncthreads();
    const uint32_t last = min(256u, fsz - beg) - 1u;
    uint32_t r = 0;  // a thread's edges only move forward: each row search starts from the last
    for (uint32_t e0 = 0; e0 < total; e0 += 256u) {
      const uint32_t e = e0 + t;
      bool keep = false;
      uint32_t x = 0, dx = 0;
      if (e < total) {
        uint32_t top = last;
        while (r < top) {
          const uint32_t mid = (r + top + 1) >> 1;
          if (s_start[mid] <= e) r = mid; else top = mid - 1;
        }
        x = g.col[s_off[r] + (e - s_start[r])];
        const u64 bit = 1ull << (x & 63u);
        if (vo[x >> 6] & bit) {
          found = true;
        } else if (!(vs[x >> 6] & bit) && !gbfs_prune<W>(lab + 4ull * W * x, side, dl, bi, bo)) {
          keep = !(atomicOr(&vs[x >> 6], bit) & bit);
          if (keep) dx = min(g.deg[x], g.cap[x]);
        }
      }
      wave_push(qs, &ctl->fsize[side], keep, x);
      if (__ballot(keep)) {
        u64 sum = dx;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (__lane_id() == 0) atomicAdd(&ctl->ctr[kCtrFrontEdges + side], sum);
      }
    }
    __syncthreads();
  }
  if (__ballot(found) && __lane_id() == 0) ctl->found = 1;
}

hipError_t launch_gbfs_round(const GbfsArgs &a, uint32_t side, uint32_t lo, uint32_t hi,
                             uint32_t u, uint32_t v, uint32_t rules, hipStream_t s) {
  if (hi <= lo) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(2048, ((uint64_t)hi - lo + 255) / 256);
  DBL_LAUNCH_W(a.L.words, k_gbfs_round, dim3(grid), dim3(256), s, a, side, lo, hi, u, v, rules);
  return hipGetLastError();
}

__global__ void k_gbfs_finish(GbfsArgs a, uint32_t qi, uint8_t *out, u64 *qcls) {
  Ctl *ctl = a.ctl;
  const bool found = ctl->found != 0;
  out[qi] = found ? (uint8_t)(1u | (5u << 1)) : (uint8_t)(6u << 1);
  qcls[found ? 5 : 6] += 1ull;  // block 0's class slots; this kernel runs alone
  ctl->fsize[0] = 0;
  ctl->fsize[1] = 0;
  ctl->fsize[2] = 0;
  ctl->found = 0;
  ctl->ctr[kCtrFrontEdges] = 0;
  ctl->ctr[kCtrFrontEdges + 1] = 0;
}

hipError_t launch_gbfs_finish(const GbfsArgs &a, uint32_t qi, uint8_t *out, u64 *qcls,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_gbfs_finish, dim3(1), dim3(1), 0, s, a, qi, out, qcls);
  return hipGetLastError();
}

__global__ void k_init_buckets(uint8_t *bucket, uint32_t n0, uint32_t n1, uint32_t kp_bits) {
  for (uint32_t x = n0 + blockIdx.x * blockDim.x + threadIdx.x; x < n1; x += gridDim.x * blockDim.x)
    bucket[x] = (uint8_t)fib_bucket(x, kp_bits);
}

hipError_t launch_init_buckets(uint8_t *bucket, uint32_t n0, uint32_t n1, uint32_t kp_bits,
                               hipStream_t s) {
  if (n1 <= n0) return hipSuccess;
  hipLaunchKernelGGL(k_init_buckets, dim3(grid_for(n1 - n0, 256, 4096)), dim3(256), 0, s, bucket,
                     n0, n1, kp_bits);
  return hipGetLastError();
}

// ---------------------------------------------------------------- label read-out

// Label i of vertex x goes to out[x * W + i / 64] bit i % 64.
__global__ void k_unpack_labels(const u64 *lab, uint32_t words, uint32_t n, u64 *dl_in,
                                u64 *dl_out, u64 *bl_in, u64 *bl_out) {
  const uint64_t total = (uint64_t)n * words;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = e / words, j = e - x * words;
    const u64 *rec = lab + 4ull * words * x;
    if (dl_in) dl_in[e] = rec[j];
    if (bl_in) bl_in[e] = rec[words + j];
    if (dl_out) dl_out[e] = rec[2 * words + j];
    if (bl_out) bl_out[e] = rec[3 * words + j];
  }
}

hipError_t launch_unpack_labels(LabelsView L, uint32_t n, u64 *dl_in, u64 *dl_out, u64 *bl_in,
                                u64 *bl_out, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_labels, dim3(grid_for((uint64_t)n * L.words, 256, 8192)), dim3(256),
                     0, s, L.lab, L.words, n, dl_in, dl_out, bl_in, bl_out);
  return hipGetLastError();
}

}  // namespace dbl
