// C ABI of the DBL index (declared in include/dbl.h): device memory, call orchestration and
// status reporting. Every step of the method runs in the kernels of dbl_kernels.hip; this file
// only allocates, launches and reads back the small control block.
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "dbl.h"
#include "dbl_internal.hpp"

using dbl::Csr;
using dbl::Ctl;
using dbl::Ovf;
using u64 = unsigned long long;

// Scratch of one in-flight query batch. The index owns a default one (used by dbl_query_batch);
// callers create more to run query batches concurrently on several streams.
struct dbl_query_ctx {
  dbl_index *ix = nullptr;
  bool is_default = false;
  Ctl *ctl = nullptr;
  dbl::Mirror *mirror = nullptr;
  dbl::Mirror hs{};
  uint32_t seq = 0;
  uint32_t *und = nullptr, *heavy_q = nullptr, *seg = nullptr;
  uint64_t und_cap = 0;
  u64 *vis = nullptr;
  uint64_t vis_words = 0;
  uint32_t *bfs_queue = nullptr;
  uint32_t slots = 0, qcap = 0;
  u64 *bfs_cnt = nullptr;  // per-slot BFS counters
  u64 *qcls = nullptr;     // per-block query class counters
  u64 *gvis = nullptr;     // whole-device BFS: both sides' visited bitmaps and queues
  uint32_t *gq[2] = {nullptr, nullptr};
  uint64_t bfs_heavy = 0;
  // graph form of a batch (label kernel -> BFS kernel), instantiated on first use and
  // replayed with new node arguments
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraphNode_t gn_label = nullptr, gn_bfs = nullptr;
  uint32_t g_words = 0;
};

struct dbl_index {
  int device = 0;
  uint32_t n = 0, k = 0, kp = 0, kp_bits = 0;
  uint32_t lw = 1;  // 64-bit words per label (1, 2 or 4)
  uint32_t n_cap = 0;  // vertices the per-vertex arrays have room for
  float slack_frac = 0.25f;
  uint32_t slack_min = 4;
  Csr f{}, r{};
  uint64_t f_total = 0, r_total = 0;  // entries reserved in f.col / r.col
  u64 *lab = nullptr;
  uint32_t *fq[3] = {nullptr, nullptr, nullptr};
  uint32_t *inq = nullptr;
  u64 *heavy_list = nullptr;  // two lists of heavy_cap entries: push chunks, pull chunks
  uint64_t heavy_cap = 0;
  u64 *fbm = nullptr;         // frontier bitmaps of pull rounds (one bit per vertex per direction)
  uint64_t fbm_words = 0;
  u64 *fu = nullptr;          // OR of the frontier's labels per direction (2 x 8 words)
  uint64_t pull_expanded = 0;  // frontier entries expanded by pull rounds
  uint64_t pull_rounds = 0;    // (round, direction) pairs pulled
  Ctl *ctl = nullptr;
  dbl::Mirror *mirror = nullptr;  // pinned, device-mapped host memory written by the device
  u64 *door = nullptr;            // request server doorbell slots (pinned host memory, 2 words)
  u64 clock_khz = 100000;         // device wall-clock rate
  uint32_t server_idle_us = 200000;  // request-server idle limit
  uint32_t server_polls = 4;         // doorbell reads in flight (1 or 4)
  dbl::Mirror hs{};               // host copy of the last published status
  uint32_t seq = 0;
  u64 *pcnt = nullptr;  // per-block propagation counters
  Ovf *ovf = nullptr;
  uint64_t ovf_cap = 0;
  uint32_t *landmarks_d = nullptr;
  uint32_t landmarks_h[dbl::kMaxLabelBits] = {};
  uint8_t *leaf_flags = nullptr, *bucket = nullptr;
  u64 *scan_tmp = nullptr, *scan_total = nullptr;
  uint64_t scan_tmp_words = 0;
  // runtime tuning (never changes a result)
  uint32_t small_batch = dbl::kSmallBatch;
  uint32_t local_max_frontier = dbl::kLocalMaxFrontier, local_max_edges = dbl::kLocalMaxEdges;
  uint32_t round_grid = dbl::kRoundGridMax;
  uint32_t insert_server = 2;  // dbl_insert_edges_each: 0 launches, 1 request server, 2 stream
  uint32_t pull_threshold = 128;  // pull a direction when its push edges >= this/1024 of its edges
  uint32_t pull_all_threshold = 512;  // ... and skip the frontier test above this/1024
  uint32_t query_graph = 0;       // query batches as one graph launch
  uint32_t server_warm = 0;       // read the labels and row descriptors before serving
  uint32_t insert_persistent = 1;  // batches above small_batch in one persistent launch
  uint32_t insert_graph = 0;       // ... launched as a replayed one-node graph
  uint32_t batch_max_frontier = 1u << 17;  // larger frontiers go to the host's rounds
  uint32_t gather_wait_us = 20000;        // persistent launch: longest wait for all blocks
  uint32_t barrier_wait_us = 2000000;     // ... and at one later grid barrier
  uint32_t batch_grid_opt = 0;            // its blocks (0 = one per compute unit)
  // persistent insertion kernel: blocks per launch at most (0 = not yet queried), its
  // synchronisation words and its graph
  uint32_t batch_grid = 0, batch_grid_words = 0;
  uint32_t *bar = nullptr;
  hipGraph_t igraph = nullptr;
  hipGraphExec_t igexec = nullptr;
  hipGraphNode_t ig_node = nullptr;
  uint32_t ig_words = 0, ig_grid = 0;
  uint64_t batch_stalls_early = 0, batch_stalls_late = 0;
  uint64_t build_long_bins = 0;  // bins of the last build split over several workgroups
  // query contexts: the default one and those created by callers (guarded by ctx_mu)
  uint32_t slots_opt = 0, qcap_opt = 0;
  dbl_query_ctx *qctx = nullptr;
  std::vector<dbl_query_ctx *> ctxs;
  std::mutex ctx_mu;
  uint64_t retired_class[7] = {}, retired_bfs_v = 0, retired_bfs_e = 0, retired_heavy = 0;
  // statistics kept on the host
  uint64_t build_rounds = 0, insert_calls = 0, insert_rounds = 0, regrows = 0;
  // kernel timing (HIP events around selected launches)
  uint32_t time_mask = 0;
  struct Pending {
    uint32_t kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> spare;
  uint32_t time_period = 1;  // time one launch in every `time_period` of a selected kind
  uint64_t t_seen[16] = {};
  uint64_t t_launches[16] = {};
  double t_total[16] = {}, t_max[16] = {};
};

namespace {

enum TimedKind : uint32_t {
  kTInsertSmall = 0,
  kTInsertApply,
  kTLocalRounds,
  kTInsertServer,
  kTRound,
  kTQueryLabel,
  kTQueryBfs,
  kTQueryGraph,
  kTInsertBatch,
  kTInsertStream,
  kTKinds
};
const char *const kKindNames[kTKinds] = {"insert_small", "insert_apply", "local_rounds",
                                         "insert_server", "round",
                                         "query_label", "query_bfs", "query_graph",
                                         "insert_batch", "insert_stream"};

hipEvent_t take_event(dbl_index *ix) {
  if (!ix->spare.empty()) {
    hipEvent_t e = ix->spare.back();
    ix->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when its kind is selected; otherwise does nothing.
struct Timed {
  dbl_index *ix;
  uint32_t kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timed(dbl_index *ix_, uint32_t kind_, hipStream_t s_) : ix(ix_), kind(kind_), s(s_) {
    if (kind >= kTKinds || !(ix->time_mask & (1u << kind))) return;
    if (ix->t_seen[kind]++ % ix->time_period) return;
    a = take_event(ix);
    if (a && hipEventRecord(a, s) != hipSuccess) {
      ix->spare.push_back(a);
      a = nullptr;
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(ix);
    if (b && hipEventRecord(b, s) == hipSuccess) {
      ix->pending.push_back({kind, a, b});
    } else {
      ix->spare.push_back(a);
      if (b) ix->spare.push_back(b);
    }
  }
};

// Fold finished timed launches into the per-kind totals (the stream has been synchronised).
void resolve_times(dbl_index *ix) {
  for (const auto &p : ix->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ix->t_launches[p.kind]++;
      ix->t_total[p.kind] += ms;
      ix->t_max[p.kind] = std::max<double>(ix->t_max[p.kind], ms);
    }
    ix->spare.push_back(p.a);
    ix->spare.push_back(p.b);
  }
  ix->pending.clear();
}

dbl_status from_hip(hipError_t e) {
  if (e == hipSuccess) return DBL_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DBL_ERR_OUT_OF_MEMORY;
  return DBL_ERR_DEVICE;
}

#define CK(expr)                                   \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return from_hip(e_);     \
  } while (0)

#define CKS(expr)                                  \
  do {                                             \
    dbl_status s_ = (expr);                        \
    if (s_ != DBL_OK) return s_;                   \
  } while (0)

// ---------------------------------------------------------------- memory cache
// Freed device and pinned host blocks are kept, keyed by (kind, device, size), and handed out
// again, so repeated builds of one workload and each index's query scratch cost no driver
// allocation (and no hipFree, which waits for the whole device). Block sizes are rounded up to
// 64 KiB (4 KiB below that). Cached bytes are capped (dbl_set_cache_limit); everything cached
// goes back to the driver on dbl_release_cache and when an allocation fails. A block is put
// back only after the work that used it has finished (every call synchronises its stream before
// returning, and dbl_destroy waits for the device first).
struct Block {
  void *p;
  size_t size;
  int dev;
  bool host;
};

struct MemCache {
  std::mutex mu;
  std::unordered_map<void *, Block> live;
  std::vector<Block> spare;
  uint64_t cached = 0;
  uint64_t limit = 64ull << 30;
  uint64_t live_device = 0;    // bytes of device blocks in use
  uint64_t device_limit = 0;   // refuse device blocks beyond this many live bytes (0 = no cap)
};

MemCache &mem_cache() {
  static MemCache *c = new MemCache();  // never destroyed: usable until the process ends
  return *c;
}

size_t granule(size_t bytes) {
  return bytes <= 4096 ? 4096 : (bytes + 65535) & ~(size_t)65535;
}

void release_block(const Block &b) {
  if (b.host) (void)hipHostFree(b.p);
  else (void)hipFree(b.p);
}

// Return cached blocks to the driver (of one device, or all with dev < 0) until at most `keep`
// bytes stay cached. Caller holds the lock.
void trim_locked(MemCache &c, int dev, uint64_t keep) {
  for (size_t i = 0; i < c.spare.size() && c.cached > keep;) {
    if (dev >= 0 && c.spare[i].dev != dev) {
      i++;
      continue;
    }
    release_block(c.spare[i]);
    c.cached -= c.spare[i].size;
    c.spare[i] = c.spare.back();
    c.spare.pop_back();
  }
}

void *take_block(size_t size, bool host) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (!host && c.device_limit && c.live_device + size > c.device_limit) return nullptr;
  for (size_t i = 0; i < c.spare.size(); i++) {
    const Block b = c.spare[i];
    if (b.size == size && b.dev == dev && b.host == host) {
      c.spare[i] = c.spare.back();
      c.spare.pop_back();
      c.cached -= b.size;
      c.live[b.p] = b;
      if (!host) c.live_device += b.size;
      return b.p;
    }
  }
  for (int attempt = 0; attempt < 2; attempt++) {
    void *p = nullptr;
    const hipError_t e = host ? hipHostMalloc(&p, size, hipHostMallocMapped | hipHostMallocCoherent)
                              : hipMalloc(&p, size);
    if (e == hipSuccess) {
      c.live[p] = Block{p, size, dev, host};
      if (!host) c.live_device += size;
      return p;
    }
    (void)hipGetLastError();
    trim_locked(c, -1, 0);  // out of memory: give the cache back and try once more
  }
  return nullptr;
}

void put_block(void *p) {
  if (!p) return;
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) return;
  const Block b = it->second;
  c.live.erase(it);
  if (!b.host) c.live_device -= b.size;
  c.spare.push_back(b);
  c.cached += b.size;
  if (c.cached > c.limit) trim_locked(c, -1, c.limit);
}

template <typename T>
dbl_status dalloc(T **p, uint64_t count) {
  if (count == 0) count = 1;
  *p = (T *)take_block(granule(sizeof(T) * count), false);
  return *p ? DBL_OK : DBL_ERR_OUT_OF_MEMORY;
}

template <typename T>
void dfree(T *&p) {
  put_block((void *)p);
  p = nullptr;
}

// pinned, device-mapped, coherent host memory (status mirrors, doorbells)
template <typename T>
dbl_status halloc(T **p, size_t bytes) {
  *p = (T *)take_block(granule(bytes), true);
  return *p ? DBL_OK : DBL_ERR_OUT_OF_MEMORY;
}

template <typename T>
void hfree(T *&p) {
  put_block((void *)p);
  p = nullptr;
}

// Device scratch local to one call. The normal path frees it explicitly once the work using it
// has finished; on an early (error) return the destructor waits for the stream first, so no
// path leaks it or hands it out again while a kernel may still use it.
template <typename T>
struct Scoped {
  T *p = nullptr;
  hipStream_t s;
  explicit Scoped(hipStream_t st) : s(st) {}
  Scoped(const Scoped &) = delete;
  Scoped &operator=(const Scoped &) = delete;
  ~Scoped() {
    if (p) {
      (void)hipStreamSynchronize(s);
      dfree(p);
    }
  }
  void release() { dfree(p); }
};

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

dbl::PropArgs prop_args(const dbl_index *ix) {
  dbl::PropArgs a;
  a.L = {ix->lab, ix->lw};
  a.f = ix->f;
  a.r = ix->r;
  for (int i = 0; i < 3; i++) a.fq[i] = ix->fq[i];
  a.inq = ix->inq;
  a.heavy_list = ix->heavy_list;
  a.pheavy_list = ix->heavy_list ? ix->heavy_list + ix->heavy_cap : nullptr;
  a.heavy_cap = ix->heavy_cap;
  a.fbm = ix->fbm;
  a.fbm_wpd = ix->fbm_words / 2;
  a.fu = ix->fu;
  a.pcnt = ix->pcnt;
  a.local_max_frontier = ix->local_max_frontier;
  a.local_max_edges = ix->local_max_edges;
  a.ctl = ix->ctl;
  return a;
}

// Wait until the device has published status `seq` into the host mirror `m` and copy it to
// `h`. The host spins on the mirror; every few thousand polls it asks the stream whether it
// failed or went idle without publishing, so a fault can never leave the host spinning.
dbl_status wait_mirror(dbl::Mirror *m, dbl::Mirror &h, hipStream_t s, uint32_t seq) {
  for (uint64_t spin = 1;; spin++) {
    if (__atomic_load_n(&m->seq, __ATOMIC_ACQUIRE) == seq) break;
    if ((spin & 4095) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        if (__atomic_load_n(&m->seq, __ATOMIC_ACQUIRE) == seq) break;
        return DBL_ERR_DEVICE;  // the stream drained without publishing
      }
      if (q != hipErrorNotReady) return from_hip(q);
    }
  }
  volatile dbl::Mirror *vm = m;
  h.seq = seq;
  h.err = vm->err;
  h.cur = vm->cur;
  h.stamp = vm->stamp;
  for (int i = 0; i < 3; i++) h.fsize[i] = vm->fsize[i];
  h.ovf_count = vm->ovf_count;
  h.und_count = vm->und_count;
  h.bfs_heavy = vm->bfs_heavy;
  h.found = vm->found;
  for (int i = 0; i < 4; i++) h.dstat[i] = vm->dstat[i];
  return DBL_OK;
}

// Publish a control block after the work queued so far and wait for it.
dbl_status sync_chan(Ctl *ctl, dbl::Mirror *m, dbl::Mirror &h, uint32_t &seq, hipStream_t s) {
  const uint32_t sq = ++seq;
  CK(dbl::launch_publish(ctl, m, sq, s));
  return wait_mirror(m, h, s, sq);
}

dbl_status wait_status(dbl_index *ix, hipStream_t s, uint32_t seq) {
  CKS(wait_mirror(ix->mirror, ix->hs, s, seq));
  if (!ix->pending.empty()) resolve_times(ix);
  return DBL_OK;
}

// Wait for the fast status word of a small insertion. With no flag set the call is complete and
// nothing else needs reading; otherwise the whole status is published and read.
dbl_status wait_fast(dbl_index *ix, hipStream_t s, uint32_t seq, uint32_t *flags);

dbl_status sync_ctl(dbl_index *ix, hipStream_t s) {
  CKS(sync_chan(ix->ctl, ix->mirror, ix->hs, ix->seq, s));
  if (!ix->pending.empty()) resolve_times(ix);
  return DBL_OK;
}

// Write one 32-bit field of the device control block (host value, stream ordered).
dbl_status set_ctl_u32(dbl_index *ix, size_t offset, uint32_t value, hipStream_t s) {
  CK(dbl::launch_fill_u32((uint32_t *)((char *)ix->ctl + offset), value, 1, s));
  return DBL_OK;
}

dbl_status wait_fast(dbl_index *ix, hipStream_t s, uint32_t seq, uint32_t *flags) {
  for (uint64_t spin = 1;; spin++) {
    const u64 w = __atomic_load_n(&ix->mirror->fast, __ATOMIC_ACQUIRE);
    if ((uint32_t)w == seq) {
      *flags = (uint32_t)(w >> 32);
      break;
    }
    if ((spin & 4095) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        const u64 w2 = __atomic_load_n(&ix->mirror->fast, __ATOMIC_ACQUIRE);
        if ((uint32_t)w2 == seq) {
          *flags = (uint32_t)(w2 >> 32);
          break;
        }
        return DBL_ERR_DEVICE;
      }
      if (q != hipErrorNotReady) return from_hip(q);
    }
  }
  if (!ix->pending.empty()) resolve_times(ix);
  if (*flags) return sync_ctl(ix, s);
  // fast path: the pending frontier is empty and nothing overflowed
  ix->hs.err = 0;
  ix->hs.ovf_count = 0;
  ix->hs.fsize[ix->hs.cur] = 0;
  return DBL_OK;
}

dbl_status ensure_heavy_cap(dbl_index *ix) {
  const uint64_t need = (ix->f_total + ix->r_total) / 2048 + 1024;
  if (need <= ix->heavy_cap) return DBL_OK;
  dfree(ix->heavy_list);
  CKS(dalloc(&ix->heavy_list, 2 * need));
  ix->heavy_cap = need;
  return DBL_OK;
}

// Grid rounds until the pending frontier is empty.
// With pulls enabled, every round starts with a frontier scan; after reading its counts the
// host pulls each direction whose frontier would push at least pull_threshold / 1024 of the
// direction's edges and pushes the rest (one control-block read per round). Without pulls,
// `group` push rounds are enqueued between reads of the control block; a round that finds an
// empty frontier does nothing.
// `fresh`: ix->hs already holds the status after the last queued work.
dbl_status grid_propagate(dbl_index *ix, hipStream_t s, uint32_t group, uint64_t *rounds,
                          bool fresh) {
  for (;;) {
    if (!fresh) CKS(sync_ctl(ix, s));
    fresh = false;
    const uint32_t cur = ix->hs.cur;
    const uint32_t fsz = ix->hs.fsize[cur];
    if (fsz == 0) return DBL_OK;
    uint32_t stamp = ix->hs.stamp;
    if (stamp > 0xF0000000u) {
      // restart the stamp sequence before it wraps; the pending frontier is already closed, so
      // only later frontiers use the cleared marks
      CK(dbl::launch_fill_u32(ix->inq, 0u, 2ull * ix->n, s));
      CKS(set_ctl_u32(ix, offsetof(Ctl, stamp), 1u, s));
      stamp = 1;
    }
    const uint32_t gmax = ix->round_grid;
    uint32_t grid = (uint32_t)std::min<uint64_t>(gmax, std::max<uint64_t>(std::min(64u, gmax),
                                                                          (fsz + 255) / 256));
    if (ix->pull_threshold) {
      const uint64_t words = 2 * (((uint64_t)ix->n + 63) / 64);
      if (words > ix->fbm_words) {
        dfree(ix->fbm);
        ix->fbm = nullptr;
        ix->fbm_words = 0;
        CKS(dalloc(&ix->fbm, words));
        ix->fbm_words = words;
        if (!ix->fu) {
          CKS(dalloc(&ix->fu, dbl::kFuWords));
          CK(dbl::launch_fill_u64(ix->fu, 0ull, dbl::kFuWords, s));  // stripes start at zero
        }
      }
      dbl::PropArgs a = prop_args(ix);
      CK(dbl::launch_frontier_scan(a, cur, stamp, ix->fbm_words, s));
      CKS(sync_ctl(ix, s));
      uint32_t pull = 0, pull_all = 0;
      // the scan counted every entry of the frontier once; anything else: push them all
      const bool counted = ix->hs.dstat[0] + ix->hs.dstat[1] == fsz;
      for (uint32_t d = 0; d < 2 && counted; d++) {
        const uint64_t edges = d ? ix->r_total : ix->f_total;
        if (ix->hs.dstat[2 + d] && ix->hs.dstat[2 + d] * 1024 >= (u64)ix->pull_threshold * edges) {
          pull |= 1u << d;
          ix->pull_expanded += ix->hs.dstat[d];
          ix->pull_rounds++;
          if (ix->pull_all_threshold &&
              ix->hs.dstat[2 + d] * 1024 >= (u64)ix->pull_all_threshold * edges)
            pull_all |= 1u << d;
        }
      }
      const uint64_t pushed = !counted ? fsz
                              : (pull & 1 ? 0 : ix->hs.dstat[0]) + (pull & 2 ? 0 : ix->hs.dstat[1]);
      {
        Timed tm(ix, kTRound, s);
        if (pull) {
          const uint64_t rows = (uint64_t)ix->n * (uint32_t)__builtin_popcount(pull);
          CK(dbl::launch_pull(a, ix->n, pull, pull_all, cur, stamp,
                              (uint32_t)std::min<uint64_t>(gmax, (rows + 255) / 256), s));
        }
        if (pushed) CK(dbl::launch_round(a, cur, stamp, grid, s, pull, false));
      }
      *rounds += 1;
      continue;
    }
    dbl::PropArgs a = prop_args(ix);
    uint32_t ring = cur;
    for (uint32_t g = 0; g < group; g++) {
      Timed tm(ix, kTRound, s);
      CK(dbl::launch_round(a, ring, stamp, grid, s));
      ring = ring == 2 ? 0 : ring + 1;
      stamp++;
      grid = gmax;
    }
    *rounds += group;
  }
}

dbl_status regrow(dbl_index *ix, uint32_t dir, uint32_t novf, hipStream_t s) {
  Csr &g = dir ? ix->r : ix->f;
  uint64_t &total_ref = dir ? ix->r_total : ix->f_total;
  Csr ng{};
  ng.deg = g.deg;
  CKS(dalloc(&ng.cap, ix->n));
  dbl_status st = dalloc(&ng.off, ix->n);
  if (st != DBL_OK) { dfree(ng.cap); return st; }
  CK(dbl::launch_slack_cap(g.deg, ng.cap, ix->n, ix->slack_frac, ix->slack_min, s));
  CK(dbl::scan_exclusive(ng.cap, ng.off, ix->n, ix->scan_tmp, ix->scan_total, s));
  u64 total = 0;
  CK(hipMemcpyAsync(&total, ix->scan_total, sizeof(u64), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  st = dalloc(&ng.col, total);
  if (st != DBL_OK) { dfree(ng.cap); dfree(ng.off); return st; }
  CK(dbl::launch_regrow_copy(g, ng, ix->n, s));
  CK(dbl::launch_place_overflow(ix->ovf, novf, dir, ng, s));
  CK(hipStreamSynchronize(s));
  dfree(g.col);
  dfree(g.cap);
  dfree(g.off);
  g.col = ng.col;
  g.cap = ng.cap;
  g.off = ng.off;
  total_ref = total;
  ix->regrows++;
  return ensure_heavy_cap(ix);
}

// After the appends (ix->hs holds the status they published): regrow rows that ran out of
// slack, then finish propagation.
dbl_status finish_insert(dbl_index *ix, hipStream_t s, uint64_t *rounds) {
  const uint32_t novf = ix->hs.ovf_count;
  if (novf) {
    if (novf > ix->ovf_cap) return DBL_ERR_DEVICE;  // cannot happen: capacity is 2 per edge
    // which directions overflowed
    std::vector<Ovf> rec(novf);
    CK(hipMemcpyAsync(rec.data(), ix->ovf, sizeof(Ovf) * novf, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    bool any_f = false, any_r = false;
    for (const Ovf &o : rec) ((o.x >> 31) ? any_r : any_f) = true;
    if (any_f) CKS(regrow(ix, 0, novf, s));
    if (any_r) CKS(regrow(ix, 1, novf, s));
    dbl::PropArgs a = prop_args(ix);
    CK(dbl::launch_push_overflow(a, ix->ovf, novf, s));
    CKS(set_ctl_u32(ix, offsetof(Ctl, ovf_count), 0u, s));
    const uint32_t seq = ++ix->seq;
    CK(dbl::launch_local_rounds(a, ix->mirror, seq, s));
    CKS(wait_status(ix, s, seq));
  }
  return grid_propagate(ix, s, 2, rounds, true);
}

// One batch in one persistent launch (k_insert_batch), directly or as the replay of a one-node
// graph instantiated on first use and given each batch's arguments. Waits for its status.
dbl_status insert_persistent(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                             const uint32_t *d_dst, hipStream_t s, uint32_t seq) {
  if (ix->batch_grid_words != ix->lw) {
    dbl::BatchLaunch bl;
    CK(dbl::insert_batch_grid(ix->lw, &bl));
    ix->batch_grid = bl.grid;
    ix->batch_grid_words = ix->lw;
  }
  if (!ix->bar) {
    CKS(dalloc(&ix->bar, dbl::kBarWords));
    CK(dbl::launch_fill_u32(ix->bar, 0u, dbl::kBarWords, s));
  }
  // As many blocks as the batch's halves fill, one per compute unit at most: the appends queue at
  // most one frontier entry per half, so the first grid round has at most one tile per block,
  // and a grid barrier's cost grows with the blocks that arrive at it.
  const uint64_t halves = 2 * count;
  const uint32_t grid =
      ix->batch_grid_opt
          ? ix->batch_grid_opt
          : (uint32_t)std::min<uint64_t>(ix->batch_grid,
                                         (halves + dbl::kLocalThreads - 1) / dbl::kLocalThreads);
  dbl::PropArgs a = prop_args(ix);
  uint32_t n = ix->n, maxf = ix->batch_max_frontier, sq = seq;
  Ovf *ovf = ix->ovf;
  uint64_t ovf_cap = ix->ovf_cap;
  dbl::Mirror *m = ix->mirror;
  u64 start_ticks = ix->clock_khz * ix->gather_wait_us / 1000;
  u64 wait_ticks = ix->clock_khz * ix->barrier_wait_us / 1000;
  if (ix->insert_graph) {
    uint32_t *bar = ix->bar;
    void *args[13] = {(void *)&a, (void *)&d_src, (void *)&d_dst, (void *)&count, (void *)&n,
                      (void *)&ovf, (void *)&ovf_cap, (void *)&m, (void *)&sq, (void *)&maxf,
                      (void *)&start_ticks, (void *)&wait_ticks, (void *)&bar};
    hipKernelNodeParams p;
    CK(dbl::insert_batch_node_params(ix->lw, grid, args, &p));
    if (!ix->igexec || ix->ig_words != ix->lw || ix->ig_grid != grid) {
      if (ix->igexec) (void)hipGraphExecDestroy(ix->igexec);
      if (ix->igraph) (void)hipGraphDestroy(ix->igraph);
      ix->igexec = nullptr;
      ix->igraph = nullptr;
      CK(hipGraphCreate(&ix->igraph, 0));
      CK(hipGraphAddKernelNode(&ix->ig_node, ix->igraph, nullptr, 0, &p));
      CK(hipGraphInstantiate(&ix->igexec, ix->igraph, nullptr, nullptr, 0));
      ix->ig_words = ix->lw;
      ix->ig_grid = grid;
    } else {
      CK(hipGraphExecKernelNodeSetParams(ix->igexec, ix->ig_node, &p));
    }
    Timed tm(ix, kTInsertBatch, s);
    CK(hipGraphLaunch(ix->igexec, s));
  } else {
    Timed tm(ix, kTInsertBatch, s);
    CK(dbl::launch_insert_batch(a, d_src, d_dst, count, n, ovf, ovf_cap, m, seq, maxf,
                                start_ticks, wait_ticks, ix->bar, grid, s));
  }
  uint32_t flags = 0;
  return wait_fast(ix, s, seq, &flags);
}

// The multi-launch form of a batch above small_batch: validation, the appends and seeds, then
// single-workgroup rounds; waits for the status.
dbl_status insert_launches(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                           const uint32_t *d_dst, hipStream_t s, uint32_t seq) {
  dbl::PropArgs a = prop_args(ix);
  CK(dbl::launch_validate_pairs(d_src, d_dst, count, ix->n, ix->ctl, s));
  {
    Timed tm(ix, kTInsertApply, s);
    CK(dbl::launch_insert_apply(a, d_src, d_dst, count, ix->ovf, ix->ovf_cap, s));
  }
  {
    Timed tm(ix, kTLocalRounds, s);
    CK(dbl::launch_local_rounds(a, ix->mirror, seq, s));
  }
  return wait_status(ix, s, seq);
}

// After a persistent launch stalled past its gathering (every append and seed is done, the
// rounds stopped somewhere): restart propagation from every vertex that has a label bit and an
// edge. The labels only grow toward the least fixpoint, so rounds from there reach it.
dbl_status repropagate_all(dbl_index *ix, hipStream_t s) {
  // fresh claim stamps: whatever the stopped rounds claimed is forgotten
  const uint32_t stamp = 1u;
  CK(dbl::launch_fill_u32(ix->inq, 0u, 2ull * ix->n, s));
  CKS(set_ctl_u32(ix, offsetof(Ctl, cur), 0u, s));
  CKS(set_ctl_u32(ix, offsetof(Ctl, stamp), stamp, s));
  for (int i = 0; i < 3; i++) CKS(set_ctl_u32(ix, offsetof(Ctl, fsize) + 4 * i, 0u, s));
  CK(dbl::launch_init_frontier({ix->lab, ix->lw}, ix->n, ix->f, ix->r, ix->fq[0], ix->ctl,
                               ix->inq, stamp, s));
  return sync_ctl(ix, s);
}

uint32_t bits_of(uint32_t kp) {
  uint32_t b = 0;
  while ((1u << b) < kp) b++;
  return b;
}

uint64_t ctx_bytes(const dbl_index *ix, uint32_t slots, uint32_t qcap, uint64_t batch) {
  const uint64_t words = (ix->n + 63) / 64;
  return sizeof(Ctl) + words * 8 * slots + (uint64_t)qcap * 4 * slots +
         (uint64_t)slots * dbl::kBfsCtrStride * 8 + (uint64_t)dbl::kQueryGrid * dbl::kQClsStride * 8 +
         batch * 8;
}

void ctx_free(dbl_query_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  dfree(c->ctl);
  hfree(c->mirror);
  c->mirror = nullptr;
  dfree(c->und);
  dfree(c->heavy_q);
  dfree(c->seg);
  dfree(c->vis);
  dfree(c->bfs_queue);
  dfree(c->bfs_cnt);
  dfree(c->qcls);
  dfree(c->gvis);
  for (int i = 0; i < 2; i++) dfree(c->gq[i]);
}

// (Re)allocate the parts of a context sized by the vertex count: visited bitmaps and queues.
dbl_status ctx_size_bfs(dbl_index *ix, dbl_query_ctx *c, uint32_t slots, uint32_t qcap) {
  dfree(c->vis);
  dfree(c->bfs_queue);
  dfree(c->gvis);
  for (int i = 0; i < 2; i++) dfree(c->gq[i]);
  const uint64_t words = (ix->n + 63) / 64;
  hipStream_t s0 = nullptr;
  CKS(dalloc(&c->vis, words * slots));
  CKS(dalloc(&c->bfs_queue, (uint64_t)qcap * slots));
  CK(dbl::launch_fill_u64(c->vis, 0ull, words * slots, s0));
  CK(hipStreamSynchronize(s0));
  c->slots = slots;
  c->vis_words = words;
  c->qcap = qcap;
  return DBL_OK;
}

uint32_t ctx_qcap(const dbl_index *ix, uint32_t qcap) {
  return qcap ? std::min<uint32_t>(qcap, ix->n)
              : (ix->qcap_opt ? std::min<uint32_t>(ix->qcap_opt, ix->n)
                              : (uint32_t)std::min<uint64_t>(ix->n, 1u << 18));
}

// Allocate a context's fixed scratch: control block, mirror, counters, BFS slots.
dbl_status ctx_init(dbl_index *ix, dbl_query_ctx *c, uint32_t slots, uint32_t qcap) {
  c->ix = ix;
  slots = slots ? slots : (ix->slots_opt ? ix->slots_opt : 1024);
  slots = std::max<uint32_t>(4, (slots + 3) / 4 * 4);
  qcap = ctx_qcap(ix, qcap);
  hipStream_t s0 = nullptr;
  CKS(dalloc(&c->ctl, 1));
  CKS(halloc(&c->mirror, sizeof(dbl::Mirror)));
  memset((void *)c->mirror, 0, sizeof(dbl::Mirror));
  {
    Ctl init;
    memset(&init, 0, sizeof(init));
    CK(hipMemcpy(c->ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice));
  }
  CKS(dalloc(&c->bfs_cnt, (uint64_t)slots * dbl::kBfsCtrStride));
  CKS(dalloc(&c->qcls, (uint64_t)dbl::kQueryGrid * dbl::kQClsStride));
  CK(dbl::launch_fill_u64(c->bfs_cnt, 0ull, (uint64_t)slots * dbl::kBfsCtrStride, s0));
  CK(dbl::launch_fill_u64(c->qcls, 0ull, (uint64_t)dbl::kQueryGrid * dbl::kQClsStride, s0));
  CK(hipStreamSynchronize(s0));
  return ctx_size_bfs(ix, c, slots, qcap);
}

dbl_status ctx_reserve(dbl_query_ctx *c, uint64_t count) {
  if (count <= c->und_cap) return DBL_OK;
  dfree(c->und);
  dfree(c->heavy_q);
  dfree(c->seg);
  const uint64_t blocks = (std::max<uint64_t>(count, 1024) + dbl::kQueryNT - 1) / dbl::kQueryNT;
  const uint64_t cap = blocks * dbl::kQueryNT;
  CKS(dalloc(&c->und, cap));
  CKS(dalloc(&c->heavy_q, cap));
  CKS(dalloc(&c->seg, blocks));
  c->und_cap = cap;
  return DBL_OK;
}

// Host copy of a context's counters, added into `out`.
dbl_status ctx_add_counts(const dbl_query_ctx *c, uint64_t cls[7], uint64_t *bv, uint64_t *be) {
  std::vector<u64> qc((uint64_t)dbl::kQueryGrid * dbl::kQClsStride), bc((uint64_t)c->slots * dbl::kBfsCtrStride);
  CK(hipMemcpy(qc.data(), c->qcls, sizeof(u64) * qc.size(), hipMemcpyDeviceToHost));
  CK(hipMemcpy(bc.data(), c->bfs_cnt, sizeof(u64) * bc.size(), hipMemcpyDeviceToHost));
  for (uint32_t b = 0; b < dbl::kQueryGrid; b++)
    for (uint32_t k = 0; k < 7; k++) cls[k] += qc[b * dbl::kQClsStride + k];
  for (uint32_t sl = 0; sl < c->slots; sl++) {
    *bv += bc[sl * dbl::kBfsCtrStride + 0];
    *be += bc[sl * dbl::kBfsCtrStride + 1];
    cls[5] += bc[sl * dbl::kBfsCtrStride + 2];
    cls[6] += bc[sl * dbl::kBfsCtrStride + 3];
  }
  return DBL_OK;
}

// The index's own query context, created on first use.
dbl_status ensure_default_ctx(dbl_index *ix) {
  if (ix->qctx) return DBL_OK;
  dbl_query_ctx *c = new (std::nothrow) dbl_query_ctx();
  if (!c) return DBL_ERR_OUT_OF_MEMORY;
  c->is_default = true;
  const dbl_status st = ctx_init(ix, c, 0, 0);
  if (st != DBL_OK) {
    ctx_free(c);
    delete c;
    return st;
  }
  ix->qctx = c;
  return DBL_OK;
}

dbl::GbfsArgs gbfs_args(const dbl_index *ix, u64 *vis, uint64_t vis_words, uint32_t *const q[2],
                        Ctl *ctl) {
  dbl::GbfsArgs g;
  g.L = {ix->lab, ix->lw};
  g.g[0] = ix->f;
  g.g[1] = ix->r;
  g.vis[0] = vis;
  g.vis[1] = vis + vis_words;
  g.q[0] = q[0];
  g.q[1] = q[1];
  g.ctl = ctl;
  return g;
}

// Whole-device BFS of pair qi = (u, v) from both ends (Algorithm 2's BFS, with each side's
// prunes): each step expands the level of the side whose level has fewer edges; the search
// ends when a side reaches the other's visited set (a path) or a side's next level is empty (no
// path). sync() publishes the control block into h.
template <class Sync>
dbl_status gbfs_pair(const dbl::GbfsArgs &g, uint64_t vis_words, uint32_t u, uint32_t v,
                     uint32_t qi, uint32_t rules, uint8_t *d_out, u64 *qcls, hipStream_t s,
                     const dbl::Mirror &h, Sync sync) {
  CK(dbl::launch_gbfs_start(g, vis_words, u, v, s));
  CKS(sync());
  uint32_t lo[2] = {0, 0}, hi[2] = {1, 1};
  u64 seen[2] = {h.dstat[2], h.dstat[3]};  // summed degrees up to each side's level end
  u64 pend[2] = {seen[0], seen[1]};        // edges of each side's pending level
  while (!h.found) {
    const uint32_t side = pend[1] < pend[0] ? 1u : 0u;
    CK(dbl::launch_gbfs_round(g, side, lo[side], hi[side], u, v, rules, s));
    CKS(sync());
    lo[side] = hi[side];
    hi[side] = h.fsize[side];
    pend[side] = h.dstat[2 + side] - seen[side];
    seen[side] = h.dstat[2 + side];
    if (hi[side] == lo[side]) break;
  }
  CK(dbl::launch_gbfs_finish(g, qi, d_out, qcls, s));
  return DBL_OK;
}

// Algorithm 2 over a batch with the scratch of context c (see dbl_query_batch).
dbl_status run_queries(dbl_index *ix, dbl_query_ctx *c, uint64_t count, const uint32_t *d_u,
                       const uint32_t *d_v, uint8_t *d_out, hipStream_t s,
                       uint32_t rules = DBL_RULES_ALL) {
  CKS(ctx_reserve(c, count));
  dbl::BfsArgs b;
  b.L = {ix->lab, ix->lw};
  b.f = ix->f;
  b.u = d_u;
  b.v = d_v;
  b.und = c->und;
  b.seg = c->seg;
  b.nseg = (uint32_t)((count + dbl::kQueryNT - 1) / dbl::kQueryNT);
  b.out = d_out;
  b.vis = c->vis;
  b.vis_words = c->vis_words;
  b.queue = c->bfs_queue;
  b.qcap = c->qcap;
  b.heavy_q = c->heavy_q;
  b.cnt = c->bfs_cnt;
  b.rules = rules;
  b.ctl = c->ctl;
  const uint32_t seq = ++c->seq;
  if (ix->query_graph) {
    // one graph launch per batch: instantiate once, then replay with this batch's arguments
    const u64 *lab = ix->lab;
    uint32_t n = ix->n;
    const uint32_t *fdeg = ix->f.deg;
    void *la[12] = {(void *)&lab, (void *)&d_u, (void *)&d_v, (void *)&count, (void *)&n,
                    (void *)&fdeg, (void *)&d_out, (void *)&c->und, (void *)&c->seg,
                    (void *)&c->ctl, (void *)&c->qcls, (void *)&rules};
    dbl::Mirror *mirror = c->mirror;
    uint32_t sq = seq;
    void *ba[3] = {(void *)&b, (void *)&mirror, (void *)&sq};
    hipKernelNodeParams lp, bp;
    CK(dbl::query_node_params({ix->lab, ix->lw}, count, c->slots, la, ba, &lp, &bp));
    if (!c->gexec || c->g_words != ix->lw) {
      if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
      if (c->graph) (void)hipGraphDestroy(c->graph);
      c->gexec = nullptr;
      c->graph = nullptr;
      CK(hipGraphCreate(&c->graph, 0));
      CK(hipGraphAddKernelNode(&c->gn_label, c->graph, nullptr, 0, &lp));
      CK(hipGraphAddKernelNode(&c->gn_bfs, c->graph, &c->gn_label, 1, &bp));
      CK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
      c->g_words = ix->lw;
    } else {
      CK(hipGraphExecKernelNodeSetParams(c->gexec, c->gn_label, &lp));
      CK(hipGraphExecKernelNodeSetParams(c->gexec, c->gn_bfs, &bp));
    }
    Timed tm(ix, c->is_default ? (uint32_t)kTQueryGraph : (uint32_t)kTKinds, s);
    CK(hipGraphLaunch(c->gexec, s));
  } else {
    {
      Timed tm(ix, c->is_default ? (uint32_t)kTQueryLabel : (uint32_t)kTKinds, s);
      CK(dbl::launch_query_label({ix->lab, ix->lw}, d_u, d_v, count, ix->n, ix->f.deg, d_out,
                                 c->und, c->seg, c->ctl, c->qcls, rules, s));
    }
    Timed tm(ix, c->is_default ? (uint32_t)kTQueryBfs : (uint32_t)kTKinds, s);
    CK(dbl::launch_query_bfs(b, c->slots, c->mirror, seq, s));
  }
  CKS(wait_mirror(c->mirror, c->hs, s, seq));
  if (c->is_default && !ix->pending.empty()) resolve_times(ix);
  if (c->hs.err) {
    CK(dbl::launch_fill_u32((uint32_t *)((char *)c->ctl + offsetof(Ctl, err)), 0u, 1, s));
    CK(hipStreamSynchronize(s));
    return DBL_ERR_VERTEX_RANGE;
  }
  const uint32_t nheavy = c->hs.bfs_heavy;
  if (nheavy) {
    // pairs whose pruned BFS outgrew a slot: one whole-device BFS each (rare)
    std::vector<uint32_t> hq(nheavy);
    CK(hipMemcpyAsync(hq.data(), c->heavy_q, sizeof(uint32_t) * nheavy, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (!c->gvis) {
      CKS(dalloc(&c->gvis, 2 * c->vis_words));
      for (int i = 0; i < 2; i++) CKS(dalloc(&c->gq[i], ix->n));
    }
    const dbl::GbfsArgs g = gbfs_args(ix, c->gvis, c->vis_words, c->gq, c->ctl);
    for (uint32_t i = 0; i < nheavy; i++) {
      uint32_t u = 0, v = 0;
      CK(hipMemcpyAsync(&u, d_u + hq[i], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      CK(hipMemcpyAsync(&v, d_v + hq[i], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
      CKS(gbfs_pair(g, c->vis_words, u, v, hq[i], rules, d_out, c->qcls, s, c->hs,
                    [&] { return sync_chan(c->ctl, c->mirror, c->hs, c->seq, s); }));
    }
    CK(hipStreamSynchronize(s));
    c->bfs_heavy += nheavy;
  }
  return DBL_OK;
}

// Row fill choice for one direction (dbl_options.row_fill). The direct fill writes each edge
// straight into its row; its scattered writes combine in cache while the rows of the bins in
// flight (two fill workgroups per compute unit, 256 units) fit in the 256 MiB last-level cache,
// or while edges arrive grouped by row (a partition tile then covers a few whole rows). Past
// that, assembling rows in LDS first costs an extra pass over the edges but writes every column
// once, in runs.
// same / sampled: the grouping sample of launch_bin_edges.
bool use_staged_fill(uint32_t mode, u64 same, u64 sampled, u64 total, uint32_t n) {
  if (mode != 0) return mode == 2;
  const u64 nbins = dbl::bin_count(n);
  const u64 in_flight = std::min<u64>(nbins, 512);
  const u64 window_bytes = total * sizeof(uint32_t) / nbins * in_flight;
  return same * 2 < sampled && window_bytes > (256ull << 20);
}

dbl_status do_build(dbl_index *ix, uint64_t m, const uint32_t *src, const uint32_t *dst,
                    const dbl_options &o, hipStream_t s) {
  const uint32_t n = ix->n;
  CKS(dalloc(&ix->ctl, 1));
  CKS(halloc(&ix->mirror, sizeof(dbl::Mirror)));
  memset((void *)ix->mirror, 0, sizeof(dbl::Mirror));
  CKS(halloc(&ix->door, 64));
  ix->door[0] = ix->door[1] = dbl::kDoorStop;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ix->device) == hipSuccess &&
        khz > 0)
      ix->clock_khz = (u64)khz;
  }
  CKS(dalloc(&ix->pcnt, 2ull * dbl::kPropCtrSlots));
  CK(dbl::launch_fill_u64(ix->pcnt, 0ull, 2ull * dbl::kPropCtrSlots, s));
  {
    Ctl init;
    memset(&init, 0, sizeof(init));
    init.cur = 0;
    init.stamp = 1;
    CK(hipMemcpyAsync(ix->ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
  }
  // ---- a1: validate, de-duplicate, count degrees, reserve slack, scatter into both CSRs
  CK(dbl::launch_validate_pairs(src, dst, m, n, ix->ctl, s));
  CKS(sync_ctl(ix, s));
  if (ix->hs.err) return DBL_ERR_VERTEX_RANGE;
  Scoped<uint8_t> keep(s);
  Scoped<u64> table(s);
  CKS(dalloc(&keep.p, m));
  uint64_t mask = 0;
  if (!o.edges_unique && m) {
    uint64_t cap = 1024;
    while (cap < 2 * m) cap <<= 1;
    CKS(dalloc(&table.p, cap));
    CK(dbl::launch_fill_u64(table.p, ~0ull, cap, s));
    mask = cap - 1;
  }
  CK(dbl::launch_dedup_mark(src, dst, m, table.p, mask, keep.p, o.edges_unique ? 1 : 0, s));
  CKS(dalloc(&ix->f.deg, n));
  CKS(dalloc(&ix->r.deg, n));
  CKS(dalloc(&ix->f.cap, n));
  CKS(dalloc(&ix->r.cap, n));
  CKS(dalloc(&ix->f.off, n));
  CKS(dalloc(&ix->r.off, n));
  ix->scan_tmp_words = dbl::scan_tmp_words(n);
  CKS(dalloc(&ix->scan_tmp, ix->scan_tmp_words));
  CKS(dalloc(&ix->scan_total, 2));
  // in/out degrees are needed by selection and seeding; the row fill recounts deg
  Scoped<uint32_t> indeg_s(s), outdeg_s(s);
  CKS(dalloc(&indeg_s.p, n));
  CKS(dalloc(&outdeg_s.p, n));
  uint32_t *const indeg = indeg_s.p, *const outdeg = outdeg_s.p;
  {
    // per direction: partition the kept edges by vertex range, count degrees, reserve slack,
    // lay out the rows, fill them in partition order
    const uint32_t nbins = dbl::bin_count(n);
    const uint32_t nblk = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(dbl::kBinBlocks, (m + 65535) / 65536));
    uint32_t *counts = nullptr;
    u64 *offs = nullptr, *btmp = nullptr, *bkept = nullptr, *edges = nullptr;
    dbl_status st = dalloc(&counts, (uint64_t)nblk * nbins);
    if (st == DBL_OK) st = dalloc(&offs, (uint64_t)nblk * nbins);
    if (st == DBL_OK) st = dalloc(&btmp, dbl::scan_tmp_words(nblk * nbins));
    if (st == DBL_OK) st = dalloc(&bkept, 3);  // kept edges, then the grouping sample
    u64 *bstarts = nullptr;                    // first edge of each bin (long-bin test)
    if (st == DBL_OK) st = dalloc(&bstarts, nbins);
    if (st == DBL_OK) st = dalloc(&edges, m);
    // staging for the row fill, taken when a direction wants it: the dedup table (at least 2m
    // entries) is free by then; without one, a buffer of its own, and without that the rows
    // fill directly
    u64 *own_tmp = nullptr;
    // long bins of the current direction: chunk table and per-bin row cursors
    dbl::LongChunk *chunks_d = nullptr;
    uint32_t *cursors_d = nullptr;
    for (uint32_t d = 0; d < 2 && st == DBL_OK; d++) {
      Csr &g = d ? ix->r : ix->f;
      uint64_t &total = d ? ix->r_total : ix->f_total;
      hipError_t e = hipSuccess;
      u64 kept = 0, same = 0, sampled = 0;
      if (m) {
        e = dbl::launch_bin_edges(d ? dst : src, d ? src : dst, keep.p, m, n, nblk, counts, offs,
                                  btmp, bkept, bkept + 1, edges, s);
        u64 kr[3] = {0, 0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(kr, bkept, sizeof(kr), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        kept = kr[0];
        same = kr[1];
        sampled = kr[2];
      }
      // A bin with far more than its share of the edges (ids that put the high-degree vertices
      // in a few ranges) would hold up the one workgroup it gets: such bins are cut into chunks
      // of about one workgroup's share (kept / 512: two workgroups on each of 256 units), each
      // taken by a workgroup of its own.
      u64 long_min = ~0ull;
      std::vector<dbl::LongChunk> chunks;
      uint32_t nlong = 0;
      dfree(chunks_d);
      dfree(cursors_d);
      if (e == hipSuccess && m && (1u << dbl::bin_shift(n)) <= dbl::kBinVertsMax) {
        std::vector<u64> starts(nbins);
        e = dbl::launch_bin_starts(offs, nblk, nbins, bstarts, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(starts.data(), bstarts, sizeof(u64) * nbins, hipMemcpyDeviceToHost,
                             s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        const u64 share = (kept + 511) / 512;
        long_min = std::max<u64>(4 * share, 1ull << 16);
        const u64 chunk = std::max<u64>(share, 1ull << 16);
        for (uint32_t b = 0; e == hipSuccess && b < nbins; b++) {
          const u64 lo = starts[b], hi = b + 1 < nbins ? starts[b + 1] : kept;
          if (hi - lo < long_min) continue;
          for (u64 c = lo; c < hi; c += chunk) chunks.push_back({b, nlong, c, std::min(c + chunk, hi)});
          nlong++;
        }
        ix->build_long_bins += nlong;
        if (!chunks.empty() && e == hipSuccess) {
          st = dalloc(&chunks_d, chunks.size());
          if (st == DBL_OK) st = dalloc(&cursors_d, (uint64_t)nlong * dbl::kBinVertsMax);
          if (st != DBL_OK) break;
          e = hipMemcpyAsync(chunks_d, chunks.data(), sizeof(dbl::LongChunk) * chunks.size(),
                             hipMemcpyHostToDevice, s);
          if (e == hipSuccess)
            e = dbl::launch_fill_u32(cursors_d, 0u, (uint64_t)nlong * dbl::kBinVertsMax, s);
          if (e == hipSuccess) e = dbl::launch_fill_u32(g.deg, 0u, n, s);  // long bins add up
        }
      }
      const uint32_t nchunks = (uint32_t)chunks.size();
      if (e == hipSuccess && m)
        e = dbl::launch_bin_rows(edges, offs, nblk, n, bkept, kept, g.deg, nullptr, nullptr,
                                 long_min, chunks_d, nchunks, cursors_d, s);
      else if (e == hipSuccess)
        e = dbl::launch_fill_u32(g.deg, 0u, n, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d ? indeg : outdeg, g.deg, sizeof(uint32_t) * n,
                           hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = dbl::launch_slack_cap(g.deg, g.cap, n, ix->slack_frac, ix->slack_min, s);
      if (e == hipSuccess)
        e = dbl::scan_exclusive(g.cap, g.off, n, ix->scan_tmp, ix->scan_total + d, s);
      u64 t = 0;
      if (e == hipSuccess)
        e = hipMemcpyAsync(&t, ix->scan_total + d, sizeof(u64), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        st = from_hip(e);
        break;
      }
      total = t;
      st = dalloc(&g.col, total);
      if (st != DBL_OK) break;
      u64 *fill_tmp = nullptr;
      if (m && total < (1ull << 32) && use_staged_fill(o.row_fill, same, sampled, total, n)) {
        if (!table.p && !own_tmp && dalloc(&own_tmp, m) != DBL_OK) own_tmp = nullptr;
        fill_tmp = table.p ? table.p : own_tmp;
      }
      if (m)
        e = dbl::launch_bin_rows(edges, offs, nblk, n, bkept, kept, g.deg, &g, fill_tmp,
                                 long_min, chunks_d, nchunks, cursors_d, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = from_hip(e);
    }
    if (st != DBL_OK) (void)hipStreamSynchronize(s);
    dfree(chunks_d);
    dfree(cursors_d);
    dfree(bstarts);
    dfree(counts);
    dfree(offs);
    dfree(btmp);
    dfree(bkept);
    dfree(edges);
    if (own_tmp) dfree(own_tmp);
    if (st != DBL_OK) return st;
  }
  CK(hipStreamSynchronize(s));
  table.release();
  keep.release();

  // ---- a2: landmarks (top-k by |Pre|*|Suc|), leaves and their hash buckets
  CKS(dalloc(&ix->landmarks_d, dbl::kMaxLabelBits));
  if (ix->k) {
    if (o.landmarks) {
      CK(hipMemcpyAsync(ix->landmarks_d, o.landmarks, sizeof(uint32_t) * ix->k,
                        hipMemcpyHostToDevice, s));
    } else {
      const uint64_t te = dbl::topk_tmp_entries(n);
      Scoped<u64> tm(s);
      Scoped<uint32_t> tid(s);
      CKS(dalloc(&tm.p, te));
      CKS(dalloc(&tid.p, te));
      CK(dbl::select_topk(indeg, outdeg, n, ix->k, o.landmark_rank, tm.p, tid.p, ix->landmarks_d,
                          s));
      CK(hipStreamSynchronize(s));
      tm.release();
      tid.release();
    }
    CK(hipMemcpyAsync(ix->landmarks_h, ix->landmarks_d, sizeof(uint32_t) * ix->k,
                      hipMemcpyDeviceToHost, s));
  }
  CKS(dalloc(&ix->lab, 4ull * ix->lw * n));
  CK(dbl::launch_fill_u64(ix->lab, 0ull, 4ull * ix->lw * n, s));
  Scoped<uint8_t> is_lm(s), flags_in(s), bucket_in(s);
  CKS(dalloc(&is_lm.p, n));
  CK(hipMemsetAsync(is_lm.p, 0, n, s));
  if (o.leaf_flags) {
    CKS(dalloc(&flags_in.p, n));
    CK(hipMemcpyAsync(flags_in.p, o.leaf_flags, n, hipMemcpyHostToDevice, s));
  }
  if (o.leaf_bucket) {
    CKS(dalloc(&bucket_in.p, n));
    CK(hipMemcpyAsync(bucket_in.p, o.leaf_bucket, n, hipMemcpyHostToDevice, s));
  }
  CKS(dalloc(&ix->leaf_flags, n));
  CKS(dalloc(&ix->bucket, n));
  CK(dbl::launch_seed({ix->lab, ix->lw}, n, ix->landmarks_d, ix->k, indeg, outdeg, flags_in.p,
                      bucket_in.p, ix->kp_bits, o.leaf_threshold, ix->leaf_flags, ix->bucket,
                      is_lm.p, s));
  CK(hipStreamSynchronize(s));
  is_lm.release();
  flags_in.release();
  bucket_in.release();
  indeg_s.release();
  outdeg_s.release();

  // ---- a3: bit-parallel propagation of the seeds to the least fixpoint
  for (int i = 0; i < 3; i++) CKS(dalloc(&ix->fq[i], 2ull * n));
  CKS(dalloc(&ix->inq, 2ull * n));
  CK(dbl::launch_fill_u32(ix->inq, 0u, 2ull * n, s));
  CKS(ensure_heavy_cap(ix));
  CK(dbl::launch_init_frontier({ix->lab, ix->lw}, n, ix->f, ix->r, ix->fq[0], ix->ctl, ix->inq, 1u, s));
  uint64_t rounds = 0;
  CKS(grid_propagate(ix, s, 4, &rounds, false));
  ix->build_rounds = rounds;
  return DBL_OK;
}

// The one-request-at-a-time form through the request server (k_insert_server). The host holds
// the request stream (a copy of the ids, as a server receives them) and releases request i by
// writing its edge into doorbell slot i & 1; the request is done when the device publishes its
// sequence number, and its slot is emptied before the next release. An id out of range is
// refused before its release. A request whose flags need the host (a full row, a large
// frontier) ends the launch; the host finishes it exactly as dbl_insert_edges does and starts a
// new launch for the rest. A launch that timed out waiting (the host was slow) is started again.
dbl_status insert_each_served(dbl_index *ix, uint32_t count, const uint32_t *d_src,
                              const uint32_t *d_dst, float *h_latency_us, hipStream_t s) {
  u64 *door = ix->door;
  // release stores: x86 makes stores visible in program order, so an emptied slot is seen
  // empty before the next release becomes visible, with no fence on the request path
  auto put = [](u64 *slot, u64 v) { __atomic_store_n(slot, v, __ATOMIC_RELEASE); };
  // whatever way this returns, a launch still waiting for a request ends at once, and the
  // staging copy of the ids goes back to the cache
  struct OnExit {
    u64 *door;
    uint32_t *ids;
    ~OnExit() {
      __atomic_store_n(door, dbl::kDoorStop, __ATOMIC_SEQ_CST);
      __atomic_store_n(door + 1, dbl::kDoorStop, __ATOMIC_SEQ_CST);
      hfree(ids);
    }
  } on_exit{door, nullptr};
  CKS(halloc(&on_exit.ids, 8ull * count));
  const uint32_t *h_src = on_exit.ids, *h_dst = on_exit.ids + count;
  CK(hipMemcpyAsync(on_exit.ids, d_src, 4ull * count, hipMemcpyDeviceToHost, s));
  CK(hipMemcpyAsync(on_exit.ids + count, d_dst, 4ull * count, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (ix->ovf_cap < 2) {
    dfree(ix->ovf);
    CKS(dalloc(&ix->ovf, 1024));
    ix->ovf_cap = 1024;
  }
  if (ix->server_warm) {
    // every request reads two labels and two rows' descriptors at random: read them all once
    // so that they come from the memory-side cache instead of HBM (about 200 MB at 2^22
    // vertices, well inside MI355X's 256 MB Infinity Cache)
    const uint64_t n = ix->n;
    CK(dbl::launch_touch(ix->lab, 32ull * ix->lw * n, ix->scan_total, s));
    for (const Csr *g : {&ix->f, &ix->r}) {
      CK(dbl::launch_touch(g->off, 8 * n, ix->scan_total, s));
      CK(dbl::launch_touch(g->deg, 4 * (n & ~3ull), ix->scan_total, s));
      CK(dbl::launch_touch(g->cap, 4 * (n & ~3ull), ix->scan_total, s));
    }
  }
  uint32_t i = 0;
  while (i < count) {
    put(door, dbl::kDoorEmpty);
    put(door + 1, dbl::kDoorEmpty);
    const dbl::PropArgs a = prop_args(ix);
    const uint32_t first = i, seq0 = ix->seq;
    {
      Timed tm(ix, kTInsertServer, s);
      CK(dbl::launch_insert_server(a, first, count, ix->n, ix->ovf, ix->ovf_cap, ix->mirror,
                                   door, seq0, ix->clock_khz * ix->server_idle_us / 1000,
                                   ix->server_polls, s));
    }
    bool relaunch = false;
    for (; i < count && !relaunch; i++) {
      const uint32_t seq = seq0 + (i - first) + 1;
      const auto t0 = std::chrono::steady_clock::now();
      if (h_src[i] >= ix->n || h_dst[i] >= ix->n) {
        // refused before release: the index stays as the earlier requests left it
        put(door, dbl::kDoorStop);
        put(door + 1, dbl::kDoorStop);
        CK(hipStreamSynchronize(s));
        if (h_latency_us)
          h_latency_us[i] = std::chrono::duration<float, std::micro>(
                                std::chrono::steady_clock::now() - t0).count();
        return DBL_ERR_VERTEX_RANGE;
      }
      put(door + (i & 1u), ((u64)h_src[i] << 32) | h_dst[i]);
      uint32_t flags = 0;
      bool gone = false;
      for (uint64_t spin = 1;; spin++) {
        const u64 w = __atomic_load_n(&ix->mirror->fast, __ATOMIC_ACQUIRE);
        if ((uint32_t)w == seq) {
          flags = (uint32_t)(w >> 32);
          break;
        }
        if ((spin & 4095) == 0) {
          const hipError_t q = hipStreamQuery(s);
          if (q == hipSuccess) {
            const u64 w2 = __atomic_load_n(&ix->mirror->fast, __ATOMIC_ACQUIRE);
            if ((uint32_t)w2 == seq) {
              flags = (uint32_t)(w2 >> 32);
              break;
            }
            gone = true;  // the launch ended before taking request i
            break;
          }
          if (q != hipErrorNotReady) return from_hip(q);
        }
      }
      if (gone) {
        relaunch = true;
        i--;  // request i again, in a new launch
        ix->seq = seq - 1;
        continue;
      }
      put(door + (i & 1u), dbl::kDoorEmpty);
      ix->seq = seq;
      if (flags) {
        // the launch has ended after this request; finish it on the host
        CK(hipStreamSynchronize(s));
        CKS(sync_ctl(ix, s));
        if (ix->hs.err) {
          CKS(set_ctl_u32(ix, offsetof(Ctl, err), 0u, s));
          CK(hipStreamSynchronize(s));
          if (h_latency_us)
            h_latency_us[i] = std::chrono::duration<float, std::micro>(
                                  std::chrono::steady_clock::now() - t0).count();
          return DBL_ERR_VERTEX_RANGE;
        }
        uint64_t rounds = 0;
        CKS(finish_insert(ix, s, &rounds));
        ix->insert_calls++;
        ix->insert_rounds += rounds;
        relaunch = true;
      } else {
        ix->insert_calls++;
        ix->hs.err = 0;
        ix->hs.ovf_count = 0;
        ix->hs.fsize[ix->hs.cur] = 0;
      }
      if (h_latency_us)
        h_latency_us[i] = std::chrono::duration<float, std::micro>(
                              std::chrono::steady_clock::now() - t0).count();
    }
    if (!relaunch) break;
  }
  put(door, dbl::kDoorStop);
  put(door + 1, dbl::kDoorStop);
  CK(hipStreamSynchronize(s));
  if (!ix->pending.empty()) resolve_times(ix);
  return DBL_OK;
}

// The device-fed one-request-at-a-time form (k_insert_stream): the requests stay in device
// memory and one resident workgroup applies them in order. A request whose flags need the host
// (a full row, a large frontier) ends the launch; the host finishes it exactly as
// dbl_insert_edges does and starts a new launch for the rest. A request with an id out of range
// ends the call with its status; the requests before it stay applied. Latencies are the device
// clock's time per request, plus the host's part for a request the host finished.
dbl_status insert_each_streamed(dbl_index *ix, uint32_t count, const uint32_t *d_src,
                                const uint32_t *d_dst, float *h_latency_us, hipStream_t s) {
  if (ix->ovf_cap < 2) {
    dfree(ix->ovf);
    CKS(dalloc(&ix->ovf, 1024));
    ix->ovf_cap = 1024;
  }
  Scoped<uint32_t> ticks(s);
  if (h_latency_us) CKS(dalloc(&ticks.p, count));
  std::vector<float> host_us;
  if (h_latency_us) host_us.assign(count, 0.0f);
  dbl_status result = DBL_OK;
  uint32_t i = 0;
  while (i < count) {
    const dbl::PropArgs a = prop_args(ix);
    const uint32_t seq0 = ix->seq;
    {
      Timed tm(ix, kTInsertStream, s);
      CK(dbl::launch_insert_stream(a, d_src, d_dst, i, count, ix->n, ix->ovf, ix->ovf_cap,
                                   ix->mirror, seq0, ticks.p, s));
    }
    CK(hipStreamSynchronize(s));
    const u64 w = __atomic_load_n(&ix->mirror->fast, __ATOMIC_ACQUIRE);
    const uint32_t done = (uint32_t)w - seq0, flags = (uint32_t)(w >> 32);
    if (done > count - i) return DBL_ERR_DEVICE;
    ix->seq = (uint32_t)w;
    ix->insert_calls += done;
    i += done;
    if (flags & dbl::kFastErr) {
      result = DBL_ERR_VERTEX_RANGE;  // request i was refused; nothing of it applied
      break;
    }
    if (flags) {
      // request i - 1 ended the launch: finish it on the host
      const auto t0 = std::chrono::steady_clock::now();
      CKS(sync_ctl(ix, s));
      uint64_t rounds = 0;
      CKS(finish_insert(ix, s, &rounds));
      ix->insert_rounds += rounds;
      if (h_latency_us)
        host_us[i - 1] = std::chrono::duration<float, std::micro>(
                             std::chrono::steady_clock::now() - t0).count();
    } else if (i < count) {
      return DBL_ERR_DEVICE;  // a launch without flags serves every request
    }
  }
  ix->hs.err = 0;
  ix->hs.ovf_count = 0;
  if (h_latency_us) {
    std::vector<uint32_t> tk(count);
    CK(hipMemcpyAsync(tk.data(), ticks.p, 4ull * count, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const double us_per_tick = 1000.0 / (double)ix->clock_khz;
    for (uint32_t k = 0; k < count; k++)
      h_latency_us[k] = k < i ? (float)(tk[k] * us_per_tick) + host_us[k] : 0.0f;
  }
  if (!ix->pending.empty()) resolve_times(ix);
  return result;
}

// Move p to a new allocation of new_count entries, keeping the first old_count.
template <typename T>
dbl_status grow(T *&p, uint64_t old_count, uint64_t new_count, hipStream_t s) {
  T *q = nullptr;
  CKS(dalloc(&q, new_count));
  if (old_count) {
    const hipError_t e = hipMemcpyAsync(q, p, sizeof(T) * old_count, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      dfree(q);
      return from_hip(e);
    }
  }
  const hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dfree(q);
    return from_hip(e);
  }
  dfree(p);
  p = q;
  return DBL_OK;
}

// ---------------------------------------------------------------- allocation-free queries
// dbl_query_batch_noalloc keeps all of a batch's scratch in one static device array: every GPU
// the library runs on holds its own copy from the moment the code object is loaded until the
// process ends. In host code `scratch` only names a host-side stand-in; the device address of
// each GPU's copy comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is ever handed to kernels.
constexpr uint64_t kScratchBytes = 128ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
constexpr uint32_t kScratchMaxSlots = 256;
constexpr uint32_t kScratchMaxQueue = 1u << 16;

struct ScratchDev {
  std::mutex mu;                 // held by a call for as long as its work uses the array
  unsigned char *ptr = nullptr;  // device address of this GPU's `scratch`
  uint64_t zero_bytes = 0;       // leading bytes of the visited-bitmap area known to be zero
};
ScratchDev g_scratch[kScratchDevices];

// Fixed header: control block, device-side status, class counters, per-slot BFS counters.
constexpr uint64_t kScrCtl = 0, kScrMirror = 256, kScrQcls = 512;
constexpr uint64_t kScrBfsCnt = kScrQcls + (uint64_t)dbl::kQueryGrid * dbl::kQClsStride * 8;
constexpr uint64_t kScrVis = 16384;  // visited bitmaps start here (the zero-tracked area)
static_assert(sizeof(Ctl) <= 256 && sizeof(dbl::Mirror) <= 256, "header fields");
static_assert(kScrBfsCnt + (uint64_t)kScratchMaxSlots * dbl::kBfsCtrStride * 8 <= kScrVis,
              "header size");

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Where each part of one batch goes in the scratch array.
struct ScratchLayout {
  uint32_t slots = 0, qcap = 0;
  uint64_t vis_words = 0, vis = 0, queue = 0, und = 0, heavy_q = 0, seg = 0, gvis = 0;
  uint64_t gq[2] = {0, 0};
  uint64_t end = 0;
};

// Lay out a batch of `count` pairs on an index of ix->n vertices: as many BFS slots (a multiple
// of four, at most the index's bfs_slots option or 256) as fit beside the rest. False when not
// even four slots fit.
bool scratch_layout(const dbl_index *ix, uint64_t count, ScratchLayout *L) {
  const uint64_t n = ix->n;
  L->vis_words = (n + 63) / 64;
  L->qcap = (uint32_t)std::min<uint64_t>(n, ix->qcap_opt ? std::min(ix->qcap_opt, kScratchMaxQueue)
                                                           : kScratchMaxQueue);
  const uint64_t blocks = (count + dbl::kQueryNT - 1) / dbl::kQueryNT;
  const uint64_t fixed = align256(blocks * dbl::kQueryNT * 4) * 2 + align256(blocks * 4) +
                         align256(2 * L->vis_words * 8) + 2 * align256(n * 4);
  const uint64_t per_slot = L->vis_words * 8 + (uint64_t)L->qcap * 4;
  const uint64_t room = kScratchBytes - kScrVis;
  if (fixed + 4 * per_slot + 512 > room) return false;
  uint64_t slots = (room - fixed - 512) / per_slot;
  const uint32_t want = ix->slots_opt ? std::min(ix->slots_opt, kScratchMaxSlots) : kScratchMaxSlots;
  slots = std::min<uint64_t>(slots, std::max<uint32_t>(4, want)) / 4 * 4;
  L->slots = (uint32_t)slots;
  uint64_t at = kScrVis;
  L->vis = at;
  at = align256(at + slots * L->vis_words * 8);
  L->queue = at;
  at = align256(at + slots * (uint64_t)L->qcap * 4);
  L->und = at;
  at += align256(blocks * dbl::kQueryNT * 4);
  L->heavy_q = at;
  at += align256(blocks * dbl::kQueryNT * 4);
  L->seg = at;
  at += align256(blocks * 4);
  L->gvis = at;
  at += align256(2 * L->vis_words * 8);
  for (int i = 0; i < 2; i++) {
    L->gq[i] = at;
    at += align256(n * 4);
  }
  L->end = at;
  return at <= kScratchBytes;
}

// Device address of the current device's `scratch`, resolved on the first call per device
// (the caller holds that device's lock and has made the device current).
dbl_status scratch_ptr(ScratchDev &d) {
  if (!d.ptr) {
    void *p = nullptr;
    CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return DBL_ERR_DEVICE;
    d.ptr = (unsigned char *)p;
    d.zero_bytes = 0;
  }
  return DBL_OK;
}

// Algorithm 2 over a batch (as run_queries) with every piece of scratch in the static array.
dbl_status run_queries_noalloc(const dbl_index *ix, ScratchDev *sd, uint64_t count, const uint32_t *d_u,
                               const uint32_t *d_v, uint8_t *d_out, hipStream_t s) {
  ScratchLayout L;
  if (!scratch_layout(ix, count, &L)) return DBL_ERR_INVALID_ARG;
  unsigned char *base = sd->ptr;
  Ctl *ctl = (Ctl *)(base + kScrCtl);
  dbl::Mirror *mirror = (dbl::Mirror *)(base + kScrMirror);
  u64 *qcls = (u64 *)(base + kScrQcls);
  u64 *bfs_cnt = (u64 *)(base + kScrBfsCnt);
  // The array keeps whatever the last call left: the header starts at zero on every call; the
  // visited bitmaps must be zero where this batch's slots lie (searches clear what they set, so
  // after a completed call the bitmap area it used is zero again).
  CK(dbl::launch_fill_u64((u64 *)base, 0ull, kScrVis / 8, s));
  const uint64_t vis_bytes = L.queue - L.vis;
  if (sd->zero_bytes < vis_bytes)
    CK(dbl::launch_fill_u64((u64 *)(base + L.vis + sd->zero_bytes), 0ull,
                            (vis_bytes - sd->zero_bytes) / 8, s));
  sd->zero_bytes = 0;  // until this call completes
  dbl::BfsArgs b;
  b.L = {ix->lab, ix->lw};
  b.f = ix->f;
  b.u = d_u;
  b.v = d_v;
  b.und = (uint32_t *)(base + L.und);
  b.seg = (uint32_t *)(base + L.seg);
  b.nseg = (uint32_t)((count + dbl::kQueryNT - 1) / dbl::kQueryNT);
  b.out = d_out;
  b.vis = (u64 *)(base + L.vis);
  b.vis_words = L.vis_words;
  b.queue = (uint32_t *)(base + L.queue);
  b.qcap = L.qcap;
  b.heavy_q = (uint32_t *)(base + L.heavy_q);
  b.cnt = bfs_cnt;
  b.rules = DBL_RULES_ALL;
  b.ctl = ctl;
  CK(dbl::launch_query_label({ix->lab, ix->lw}, d_u, d_v, count, ix->n, ix->f.deg, d_out,
                             (uint32_t *)(base + L.und), (uint32_t *)(base + L.seg), ctl, qcls,
                             DBL_RULES_ALL, s));
  CK(dbl::launch_query_bfs(b, L.slots, mirror, 1u, s));
  dbl::Mirror h;
  CK(hipMemcpyAsync(&h, mirror, sizeof(h), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (h.seq != 1u) return DBL_ERR_DEVICE;
  if (h.err) {
    sd->zero_bytes = vis_bytes;
    return DBL_ERR_VERTEX_RANGE;
  }
  if (h.bfs_heavy) {
    // pairs whose pruned BFS outgrew a slot: one whole-device BFS each (rare), over the
    // scratch's own bitmaps and queues
    uint32_t *gq[2] = {(uint32_t *)(base + L.gq[0]), (uint32_t *)(base + L.gq[1])};
    const dbl::GbfsArgs g = gbfs_args(ix, (u64 *)(base + L.gvis), L.vis_words, gq, ctl);
    const uint32_t *heavy_q = (const uint32_t *)(base + L.heavy_q);
    uint32_t seq = 1;
    auto sync = [&]() -> dbl_status {
      CK(dbl::launch_publish(ctl, mirror, ++seq, s));
      CK(hipMemcpyAsync(&h, mirror, sizeof(h), hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
      return h.seq == seq ? DBL_OK : DBL_ERR_DEVICE;
    };
    const uint32_t nheavy = h.bfs_heavy;  // h is rewritten by every sync
    uint32_t qi[64];
    for (uint32_t i0 = 0; i0 < nheavy; i0 += 64) {
      const uint32_t nb = std::min<uint32_t>(64, nheavy - i0);
      CK(hipMemcpyAsync(qi, heavy_q + i0, sizeof(uint32_t) * nb, hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
      for (uint32_t i = 0; i < nb; i++) {
        uint32_t uv[2] = {0, 0};
        CK(hipMemcpyAsync(&uv[0], d_u + qi[i], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(&uv[1], d_v + qi[i], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        CKS(gbfs_pair(g, L.vis_words, uv[0], uv[1], qi[i], DBL_RULES_ALL, d_out, qcls, s, h,
                      sync));
      }
    }
    CK(hipStreamSynchronize(s));
  }
  sd->zero_bytes = vis_bytes;
  return DBL_OK;
}

}  // namespace

extern "C" {

void dbl_default_options(dbl_options *opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->num_landmarks = 64;
  opt->bl_bits = 64;
  opt->slack_fraction = 0.25f;
  opt->slack_min = 4;
  opt->pull_threshold = 128;
  opt->pull_all_threshold = 512;
}

const char *dbl_status_str(dbl_status s) {
  switch (s) {
    case DBL_OK: return "ok";
    case DBL_ERR_INVALID_ARG: return "invalid argument";
    case DBL_ERR_VERTEX_RANGE: return "vertex id out of range";
    case DBL_ERR_OUT_OF_MEMORY: return "out of device memory";
    case DBL_ERR_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

dbl_status dbl_build(uint32_t n, uint64_t m, const uint32_t *d_src, const uint32_t *d_dst,
                     const dbl_options *opt, void *stream, dbl_index **out) {
  if (!out) return DBL_ERR_INVALID_ARG;
  *out = nullptr;
  if (n == 0 || n > 0x7FFFFFFFu) return DBL_ERR_INVALID_ARG;
  if (m && (!d_src || !d_dst)) return DBL_ERR_INVALID_ARG;
  dbl_options o;
  if (opt) o = *opt; else dbl_default_options(&o);
  if (o.num_landmarks > dbl::kMaxLabelBits) return DBL_ERR_INVALID_ARG;
  if (o.bl_bits == 0 || o.bl_bits > dbl::kMaxLabelBits || (o.bl_bits & (o.bl_bits - 1)))
    return DBL_ERR_INVALID_ARG;
  if (!(o.slack_fraction >= 0.0f) || o.slack_fraction > 16.0f) return DBL_ERR_INVALID_ARG;
  if (o.landmark_rank > 3 || o.row_fill > 2) return DBL_ERR_INVALID_ARG;
  if (o.pull_threshold > 1u << 20 || o.pull_all_threshold > 1u << 20) return DBL_ERR_INVALID_ARG;
  const uint32_t k = std::min<uint32_t>(o.num_landmarks, n);
  if (o.landmarks) {
    std::vector<uint32_t> seen(o.landmarks, o.landmarks + k);
    for (uint32_t x : seen)
      if (x >= n) return DBL_ERR_INVALID_ARG;
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return DBL_ERR_INVALID_ARG;
  }
  if (o.leaf_bucket)
    for (uint32_t x = 0; x < n; x++)
      if (o.leaf_bucket[x] >= o.bl_bits) return DBL_ERR_INVALID_ARG;
  dbl_index *ix = new (std::nothrow) dbl_index();
  if (!ix) return DBL_ERR_OUT_OF_MEMORY;
  if (hipGetDevice(&ix->device) != hipSuccess) {
    delete ix;
    return DBL_ERR_DEVICE;
  }
  ix->n = n;
  ix->n_cap = n;
  ix->k = k;
  ix->kp = o.bl_bits;
  ix->kp_bits = bits_of(o.bl_bits);
  {
    const uint32_t bits = std::max<uint32_t>(o.num_landmarks, o.bl_bits);
    ix->lw = bits <= 64 ? 1 : bits <= 128 ? 2 : 4;
  }
  ix->slack_frac = o.slack_fraction;
  ix->slack_min = o.slack_min;
  ix->slots_opt = o.bfs_slots;
  ix->pull_threshold = o.pull_threshold;
  ix->pull_all_threshold = o.pull_all_threshold;
  ix->qcap_opt = o.bfs_queue_cap;
  hipStream_t s = (hipStream_t)stream;
  if (o.time_kernels) {
    const dbl_status ts = dbl_time_kernels(ix, o.time_kernels);
    if (ts != DBL_OK) {
      delete ix;
      return ts;
    }
  }
  dbl_status st = do_build(ix, m, d_src, d_dst, o, s);
  if (st != DBL_OK) {
    (void)hipStreamSynchronize(s);
    dbl_destroy(ix);
    return st;
  }
  *out = ix;
  return DBL_OK;
}

dbl_status dbl_insert_edges(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                            const uint32_t *d_dst, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_src || !d_dst || count > 0xFFFFFFFFull / 2) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  hipStream_t s = (hipStream_t)stream;
  if (2 * count > ix->ovf_cap) {
    dfree(ix->ovf);
    const uint64_t cap = std::max<uint64_t>(2 * count, 1024);
    CKS(dalloc(&ix->ovf, cap));
    ix->ovf_cap = cap;
  }
  dbl::PropArgs a = prop_args(ix);
  const uint32_t seq = ++ix->seq;
  bool late_stall = false;
  if (count <= ix->small_batch) {
    {
      Timed tm(ix, kTInsertSmall, s);
      CK(dbl::launch_insert_small(a, d_src, d_dst, (uint32_t)count, ix->n, ix->ovf, ix->ovf_cap,
                                  ix->mirror, seq, s));
    }
    uint32_t flags = 0;
    CKS(wait_fast(ix, s, seq, &flags));
  } else if (ix->insert_persistent) {
    CKS(insert_persistent(ix, count, d_src, d_dst, s, seq));
    if (ix->hs.err & dbl::kErrStallEarly) {
      // not every block became resident in time, and nothing was changed: the same batch in
      // several launches instead
      ix->batch_stalls_early++;
      CKS(set_ctl_u32(ix, offsetof(Ctl, err), 0u, s));
      CKS(insert_launches(ix, count, d_src, d_dst, s, ++ix->seq));
    } else if (ix->hs.err & dbl::kErrStallLate) {
      ix->batch_stalls_late++;
      CKS(set_ctl_u32(ix, offsetof(Ctl, err), 0u, s));
      ix->hs.err = 0;
      late_stall = true;
    }
  } else {
    CKS(insert_launches(ix, count, d_src, d_dst, s, seq));
  }
  if (late_stall) CKS(repropagate_all(ix, s));
  if (ix->hs.err) {
    CKS(set_ctl_u32(ix, offsetof(Ctl, err), 0u, s));
    CK(hipStreamSynchronize(s));
    return DBL_ERR_VERTEX_RANGE;
  }
  uint64_t rounds = 0;
  dbl_status st = finish_insert(ix, s, &rounds);
  ix->insert_calls++;
  ix->insert_rounds += rounds;
  return st;
}

dbl_status dbl_insert_edges_each(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                                 const uint32_t *d_dst, float *h_latency_us, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_src || !d_dst || count > 0xFFFFFFFFull) return DBL_ERR_INVALID_ARG;
  if (!ix->insert_server) {
    for (uint64_t i = 0; i < count; i++) {
      const auto t0 = std::chrono::steady_clock::now();
      const dbl_status st = dbl_insert_edges(ix, 1, d_src + i, d_dst + i, stream);
      if (h_latency_us)
        h_latency_us[i] = std::chrono::duration<float, std::micro>(
                              std::chrono::steady_clock::now() - t0).count();
      if (st != DBL_OK) return st;
    }
    return DBL_OK;
  }
  DeviceGuard dg(ix->device);
  if (ix->insert_server == 2)
    return insert_each_streamed(ix, (uint32_t)count, d_src, d_dst, h_latency_us,
                                (hipStream_t)stream);
  return insert_each_served(ix, (uint32_t)count, d_src, d_dst, h_latency_us,
                            (hipStream_t)stream);
}

dbl_status dbl_query_batch_noalloc(dbl_index *ix, uint64_t count, const uint32_t *d_u,
                                   const uint32_t *d_v, uint8_t *d_out, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_u || !d_v || !d_out || count > 0xFFFFFFFFull) return DBL_ERR_INVALID_ARG;
  if (ix->device < 0 || ix->device >= kScratchDevices) return DBL_ERR_DEVICE;
  ScratchLayout L;
  if (!scratch_layout(ix, count, &L)) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  ScratchDev &sd = g_scratch[ix->device];
  std::lock_guard<std::mutex> lk(sd.mu);
  CKS(scratch_ptr(sd));
  return run_queries_noalloc(ix, &sd, count, d_u, d_v, d_out, (hipStream_t)stream);
}

dbl_status dbl_query_batch(dbl_index *ix, uint64_t count, const uint32_t *d_u,
                           const uint32_t *d_v, uint8_t *d_out, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_u || !d_v || !d_out || count > 0xFFFFFFFFull) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  CKS(ensure_default_ctx(ix));
  return run_queries(ix, ix->qctx, count, d_u, d_v, d_out, (hipStream_t)stream);
}

uint64_t dbl_query_ctx_bytes(const dbl_index *ix, uint32_t bfs_slots, uint32_t queue_cap,
                             uint64_t batch) {
  if (!ix) return 0;
  uint32_t slots = bfs_slots ? bfs_slots : (ix->slots_opt ? ix->slots_opt : 1024);
  slots = std::max<uint32_t>(4, (slots + 3) / 4 * 4);
  const uint32_t qcap = queue_cap ? std::min<uint32_t>(queue_cap, ix->n)
                                  : (uint32_t)std::min<uint64_t>(ix->n, 1u << 18);
  return ctx_bytes(ix, slots, qcap, batch);
}

dbl_status dbl_query_ctx_create(dbl_index *ix, uint32_t bfs_slots, uint32_t queue_cap,
                                dbl_query_ctx **out) {
  if (!ix || !out) return DBL_ERR_INVALID_ARG;
  *out = nullptr;
  DeviceGuard dg(ix->device);
  dbl_query_ctx *c = new (std::nothrow) dbl_query_ctx();
  if (!c) return DBL_ERR_OUT_OF_MEMORY;
  const dbl_status st = ctx_init(ix, c, bfs_slots, queue_cap);
  if (st != DBL_OK) {
    ctx_free(c);
    delete c;
    return st;
  }
  std::lock_guard<std::mutex> lk(ix->ctx_mu);
  ix->ctxs.push_back(c);
  *out = c;
  return DBL_OK;
}

dbl_status dbl_query_batch_ctx(dbl_index *ix, dbl_query_ctx *ctx, uint64_t count,
                               const uint32_t *d_u, const uint32_t *d_v, uint8_t *d_out,
                               void *stream) {
  if (!ix || !ctx || ctx->ix != ix) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_u || !d_v || !d_out || count > 0xFFFFFFFFull) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  return run_queries(ix, ctx, count, d_u, d_v, d_out, (hipStream_t)stream);
}

dbl_status dbl_query_batch_rules(dbl_index *ix, dbl_query_ctx *ctx, uint64_t count,
                                 const uint32_t *d_u, const uint32_t *d_v, uint8_t *d_out,
                                 uint32_t rules, void *stream) {
  if (!ix || (ctx && ctx->ix != ix) || rules > DBL_RULES_ALL) return DBL_ERR_INVALID_ARG;
  if (count == 0) return DBL_OK;
  if (!d_u || !d_v || !d_out || count > 0xFFFFFFFFull) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  if (!ctx) {
    CKS(ensure_default_ctx(ix));
    ctx = ix->qctx;
  }
  return run_queries(ix, ctx, count, d_u, d_v, d_out, (hipStream_t)stream, rules);
}

void dbl_query_ctx_destroy(dbl_query_ctx *ctx) {
  if (!ctx) return;
  dbl_index *ix = ctx->ix;
  DeviceGuard dg(ix->device);
  {
    std::lock_guard<std::mutex> lk(ix->ctx_mu);
    uint64_t cls[7] = {}, bv = 0, be = 0;
    if (ctx_add_counts(ctx, cls, &bv, &be) == DBL_OK) {
      for (int k = 0; k < 7; k++) ix->retired_class[k] += cls[k];
      ix->retired_bfs_v += bv;
      ix->retired_bfs_e += be;
    }
    ix->retired_heavy += ctx->bfs_heavy;
    ix->ctxs.erase(std::remove(ix->ctxs.begin(), ix->ctxs.end(), ctx), ix->ctxs.end());
  }
  ctx_free(ctx);
  delete ctx;
}

dbl_status dbl_read_labels(const dbl_index *ix, uint64_t *d_dl_in, uint64_t *d_dl_out,
                           uint64_t *d_bl_in, uint64_t *d_bl_out, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  hipStream_t s = (hipStream_t)stream;
  CK(dbl::launch_unpack_labels({ix->lab, ix->lw}, ix->n, (u64 *)d_dl_in, (u64 *)d_dl_out, (u64 *)d_bl_in,
                               (u64 *)d_bl_out, s));
  CK(hipStreamSynchronize(s));
  return DBL_OK;
}

dbl_status dbl_get_landmarks(const dbl_index *ix, uint32_t *h_out, uint32_t *k) {
  if (!ix || !h_out || !k) return DBL_ERR_INVALID_ARG;
  memcpy(h_out, ix->landmarks_h, sizeof(uint32_t) * ix->k);
  *k = ix->k;
  return DBL_OK;
}

dbl_status dbl_get_leaves(const dbl_index *ix, uint8_t *h_flags, uint8_t *h_bucket) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  if (h_flags) CK(hipMemcpy(h_flags, ix->leaf_flags, ix->n, hipMemcpyDeviceToHost));
  if (h_bucket) CK(hipMemcpy(h_bucket, ix->bucket, ix->n, hipMemcpyDeviceToHost));
  return DBL_OK;
}

dbl_status dbl_get_stats(const dbl_index *ix_c, dbl_stats *out) {
  if (!ix_c || !out) return DBL_ERR_INVALID_ARG;
  dbl_index *ix = const_cast<dbl_index *>(ix_c);
  DeviceGuard dg(ix->device);
  std::vector<u64> pc(2ull * dbl::kPropCtrSlots);
  CK(hipMemcpy(pc.data(), ix->pcnt, sizeof(u64) * pc.size(), hipMemcpyDeviceToHost));
  // stored forward entries: summed on the device (scan_total is free outside build and regrow)
  uint64_t stored = 0;
  CK(dbl::launch_sum_u32(ix->f.deg, ix->n, ix->scan_total, nullptr));
  CK(hipMemcpy(&stored, ix->scan_total, sizeof(stored), hipMemcpyDeviceToHost));
  memset(out, 0, sizeof(*out));
  out->num_edges = stored;
  out->build_rounds = ix->build_rounds;
  out->insert_calls = ix->insert_calls;
  out->insert_rounds = ix->insert_rounds;
  out->vertices_expanded = ix->pull_expanded;
  for (uint32_t b = 0; b < dbl::kPropCtrSlots; b++) {
    out->vertices_expanded += pc[2 * b];
    out->edges_relaxed += pc[2 * b + 1];
  }
  out->csr_regrows = ix->regrows;
  std::lock_guard<std::mutex> lk(ix->ctx_mu);
  uint64_t cls[7] = {}, bv = ix->retired_bfs_v, be = ix->retired_bfs_e;
  for (int k = 0; k < 7; k++) cls[k] = ix->retired_class[k];
  uint64_t heavy = ix->retired_heavy;
  std::vector<dbl_query_ctx *> all(ix->ctxs);
  if (ix->qctx) all.push_back(ix->qctx);
  for (dbl_query_ctx *c : all) {
    CKS(ctx_add_counts(c, cls, &bv, &be));
    heavy += c->bfs_heavy;
  }
  for (int k = 0; k < 7; k++) {
    out->query_class[k] = cls[k];
    out->queries += cls[k];
  }
  out->bfs_vertices = bv;
  out->bfs_edges = be;
  out->bfs_heavy = heavy;
  u64 sc[2] = {0, 0};
  CK(hipMemcpy(sc, ix->ctl->ctr + dbl::kCtrServerTicks, sizeof(sc), hipMemcpyDeviceToHost));
  out->server_requests = sc[1];
  out->pull_rounds = ix->pull_rounds;
  out->server_busy_us = (double)sc[0] * 1000.0 / (double)ix->clock_khz;
  out->batch_stalls = ix->batch_stalls_early + ix->batch_stalls_late;
  out->build_long_bins = ix->build_long_bins;
  return DBL_OK;
}

dbl_status dbl_time_kernels(dbl_index *ix, const char *kinds) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  uint32_t mask = 0, period = 1;
  if (kinds && *kinds) {
    std::string all(kinds);
    const size_t colon = all.find(':');
    if (colon != std::string::npos) {
      const long p = strtol(all.c_str() + colon + 1, nullptr, 10);
      if (p < 1 || p > 1000000) return DBL_ERR_INVALID_ARG;
      period = (uint32_t)p;
      all.resize(colon);
    }
    size_t pos = 0;
    while (pos <= all.size()) {
      size_t end = all.find(',', pos);
      if (end == std::string::npos) end = all.size();
      const std::string tok = all.substr(pos, end - pos);
      if (tok == "all") {
        mask = (1u << kTKinds) - 1u;
      } else if (!tok.empty()) {
        uint32_t k = 0;
        while (k < kTKinds && tok != kKindNames[k]) k++;
        if (k == kTKinds) return DBL_ERR_INVALID_ARG;
        mask |= 1u << k;
      }
      pos = end + 1;
    }
  }
  DeviceGuard dg(ix->device);
  resolve_times(ix);
  ix->time_mask = mask;
  ix->time_period = period;
  for (uint32_t k = 0; k < kTKinds; k++) {
    ix->t_seen[k] = 0;
    ix->t_launches[k] = 0;
    ix->t_total[k] = 0.0;
    ix->t_max[k] = 0.0;
  }
  return DBL_OK;
}

dbl_status dbl_read_kernel_times(dbl_index *ix, dbl_kernel_time *h_out, uint32_t cap,
                                 uint32_t *count) {
  if (!ix || !count || (cap && !h_out)) return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  resolve_times(ix);
  uint32_t w = 0;
  for (uint32_t k = 0; k < kTKinds && w < cap; k++) {
    if (!ix->t_launches[k]) continue;
    dbl_kernel_time &o = h_out[w++];
    memset(&o, 0, sizeof(o));
    strncpy(o.name, kKindNames[k], sizeof(o.name) - 1);
    o.launches = ix->t_launches[k];
    o.total_ms = ix->t_total[k];
    o.max_ms = ix->t_max[k];
  }
  *count = w;
  return DBL_OK;
}


dbl_status dbl_add_vertices(dbl_index *ix, uint32_t count, uint32_t *first, void *stream) {
  if (!ix) return DBL_ERR_INVALID_ARG;
  const uint64_t n0 = ix->n, n1 = n0 + count;
  if (n1 > 0x7FFFFFFFull) return DBL_ERR_INVALID_ARG;
  if (first) *first = (uint32_t)n0;
  if (count == 0) return DBL_OK;
  DeviceGuard dg(ix->device);
  hipStream_t s = (hipStream_t)stream;
  CK(hipStreamSynchronize(s));
  if (n1 > ix->n_cap) {
    const uint64_t cap = std::min<uint64_t>(0x7FFFFFFFull, std::max<uint64_t>(n1, ix->n_cap + ix->n_cap / 2));
    for (Csr *g : {&ix->f, &ix->r}) {
      CKS(grow(g->off, n0, cap, s));
      CKS(grow(g->deg, n0, cap, s));
      CKS(grow(g->cap, n0, cap, s));
    }
    CKS(grow(ix->lab, 4ull * ix->lw * n0, 4ull * ix->lw * cap, s));
    for (int i = 0; i < 3; i++) CKS(grow(ix->fq[i], 0, 2 * cap, s));
    CKS(grow(ix->inq, 2 * n0, 2 * cap, s));
    CKS(grow(ix->leaf_flags, n0, cap, s));
    CKS(grow(ix->bucket, n0, cap, s));
    dfree(ix->scan_tmp);
    ix->scan_tmp_words = dbl::scan_tmp_words((uint32_t)cap);
    CKS(dalloc(&ix->scan_tmp, ix->scan_tmp_words));
    ix->n_cap = (uint32_t)cap;
  }
  // new vertices: no edges (empty rows; the first append overflows and regrows the CSR),
  // empty labels, not leaves, never queued
  for (Csr *g : {&ix->f, &ix->r}) {
    CK(dbl::launch_fill_u32(g->deg + n0, 0u, count, s));
    CK(dbl::launch_fill_u32(g->cap + n0, 0u, count, s));
    CK(dbl::launch_fill_u64(g->off + n0, 0ull, count, s));
  }
  CK(dbl::launch_fill_u64(ix->lab + 4ull * ix->lw * n0, 0ull, 4ull * ix->lw * count, s));
  CK(dbl::launch_fill_u32(ix->inq + 2 * n0, 0u, 2ull * count, s));
  CK(hipMemsetAsync(ix->leaf_flags + n0, 0, count, s));
  CK(dbl::launch_init_buckets(ix->bucket, (uint32_t)n0, (uint32_t)n1, ix->kp_bits, s));
  CK(hipStreamSynchronize(s));
  ix->n = (uint32_t)n1;
  // query scratch is sized by the vertex count
  std::lock_guard<std::mutex> lk(ix->ctx_mu);
  std::vector<dbl_query_ctx *> all(ix->ctxs);
  if (ix->qctx) all.push_back(ix->qctx);
  for (dbl_query_ctx *c : all) CKS(ctx_size_bfs(ix, c, c->slots, ctx_qcap(ix, c->qcap == n0 ? 0 : c->qcap)));
  return DBL_OK;
}

dbl_status dbl_get_tuning(const dbl_index *ix, dbl_tuning *out) {
  if (!ix || !out) return DBL_ERR_INVALID_ARG;
  out->small_batch = ix->small_batch;
  out->local_max_frontier = ix->local_max_frontier;
  out->local_max_edges = ix->local_max_edges;
  out->round_grid = ix->round_grid;
  out->insert_server = ix->insert_server;
  out->server_idle_us = ix->server_idle_us;
  out->pull_threshold = ix->pull_threshold;
  out->pull_all_threshold = ix->pull_all_threshold;
  out->server_polls = ix->server_polls;
  out->query_graph = ix->query_graph;
  out->server_warm = ix->server_warm;
  out->insert_persistent = ix->insert_persistent;
  out->insert_graph = ix->insert_graph;
  out->batch_max_frontier = ix->batch_max_frontier;
  out->gather_wait_us = ix->gather_wait_us;
  out->barrier_wait_us = ix->barrier_wait_us;
  out->batch_grid = ix->batch_grid_opt;
  out->bfs_slots = ix->qctx ? ix->qctx->slots : (ix->slots_opt ? ix->slots_opt : 1024);
  return DBL_OK;
}

dbl_status dbl_set_tuning(dbl_index *ix, const dbl_tuning *t) {
  if (!ix || !t) return DBL_ERR_INVALID_ARG;
  if (t->small_batch > dbl::kSmallBatchMax || t->round_grid == 0 ||
      t->round_grid > dbl::kRoundGridMax || t->bfs_slots > (1u << 16) || t->insert_server > 2 ||
      t->server_idle_us > 10000000 || t->pull_threshold > 1u << 20 ||
      t->pull_all_threshold > 1u << 20 ||
      (t->server_polls != 1 && t->server_polls != 4) || t->query_graph > 1 ||
      t->server_warm > 1 || t->insert_persistent > 1 || t->insert_graph > 1 ||
      t->batch_max_frontier == 0 || t->gather_wait_us > 10000000 ||
      t->barrier_wait_us > 100000000 || t->batch_grid > dbl::kRoundGridMax)
    return DBL_ERR_INVALID_ARG;
  DeviceGuard dg(ix->device);
  ix->small_batch = t->small_batch;
  ix->local_max_frontier = t->local_max_frontier;
  ix->local_max_edges = t->local_max_edges;
  ix->round_grid = t->round_grid;
  ix->insert_server = t->insert_server;
  ix->server_idle_us = t->server_idle_us;
  ix->pull_threshold = t->pull_threshold;
  ix->pull_all_threshold = t->pull_all_threshold;
  ix->server_polls = t->server_polls;
  ix->query_graph = t->query_graph;
  ix->server_warm = t->server_warm;
  ix->insert_persistent = t->insert_persistent;
  ix->insert_graph = t->insert_graph;
  ix->batch_max_frontier = t->batch_max_frontier;
  ix->gather_wait_us = t->gather_wait_us;
  ix->barrier_wait_us = t->barrier_wait_us;
  ix->batch_grid_opt = t->batch_grid;
  const uint32_t slots = t->bfs_slots ? std::max<uint32_t>(4, (t->bfs_slots + 3) / 4 * 4) : 0;
  if (slots && (!ix->qctx || ix->qctx->slots != slots)) {
    // rebuild the index's own query context with the new slot count (its counters are kept)
    ix->slots_opt = slots;
    if (ix->qctx) {
      std::lock_guard<std::mutex> lk(ix->ctx_mu);
      uint64_t cls[7] = {}, bv = 0, be = 0;
      CKS(ctx_add_counts(ix->qctx, cls, &bv, &be));
      for (int k = 0; k < 7; k++) ix->retired_class[k] += cls[k];
      ix->retired_bfs_v += bv;
      ix->retired_bfs_e += be;
      ix->retired_heavy += ix->qctx->bfs_heavy;
      ctx_free(ix->qctx);
      delete ix->qctx;
      ix->qctx = nullptr;
    }
    CKS(ensure_default_ctx(ix));
  }
  return DBL_OK;
}

uint32_t dbl_num_vertices(const dbl_index *ix) { return ix ? ix->n : 0; }

void dbl_release_cache(void) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  trim_locked(c, -1, 0);
}

void dbl_set_cache_limit(uint64_t bytes) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.limit = bytes;
  trim_locked(c, -1, c.limit);
}

uint64_t dbl_live_bytes(void) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return c.live_device;
}

void dbl_set_device_limit(uint64_t bytes) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.device_limit = bytes;
}

uint64_t dbl_cached_bytes(void) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return c.cached;
}

uint32_t dbl_label_words(const dbl_index *ix) { return ix ? ix->lw : 0; }

void dbl_destroy(dbl_index *ix) {
  if (!ix) return;
  DeviceGuard dg(ix->device);
  // the blocks go back to the cache for reuse: nothing may still be using them
  (void)hipDeviceSynchronize();
  dfree(ix->f.off); dfree(ix->f.deg); dfree(ix->f.cap); dfree(ix->f.col);
  dfree(ix->r.off); dfree(ix->r.deg); dfree(ix->r.cap); dfree(ix->r.col);
  dfree(ix->lab);
  for (int i = 0; i < 3; i++) dfree(ix->fq[i]);
  dfree(ix->inq);
  dfree(ix->heavy_list);
  dfree(ix->fbm);
  dfree(ix->fu);
  dfree(ix->ctl);
  hfree(ix->mirror);
  hfree(ix->door);
  if (ix->igexec) (void)hipGraphExecDestroy(ix->igexec);
  if (ix->igraph) (void)hipGraphDestroy(ix->igraph);
  dfree(ix->bar);
  dfree(ix->pcnt);
  dfree(ix->ovf);
  dfree(ix->landmarks_d);
  dfree(ix->leaf_flags);
  dfree(ix->bucket);
  dfree(ix->scan_tmp);
  dfree(ix->scan_total);
  for (dbl_query_ctx *c : ix->ctxs) {
    ctx_free(c);
    delete c;
  }
  ix->ctxs.clear();
  if (ix->qctx) {
    ctx_free(ix->qctx);
    delete ix->qctx;
  }
  for (const auto &p : ix->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ix->spare) (void)hipEventDestroy(e);
  delete ix;
}

}  // extern "C"
