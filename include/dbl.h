/*
 * dbl.h — C ABI of the DBL reachability index on one MI355X (gfx950).
 *
 * DBL (Lyu, Li, He, Gong, arXiv 2101.09441) answers reachability queries q(u,v) on a directed
 * graph that only grows by edge insertion. Every vertex carries four bitset labels:
 *   DL_in(v)  - the landmarks that reach v           (Definition 1)
 *   DL_out(v) - the landmarks v reaches              (Definition 1)
 *   BL_in(v)  - hashed zero-in-degree leaves reaching v   (Definition 2, hashed into k' bits)
 *   BL_out(v) - hashed zero-out-degree leaves v reaches   (Definition 2, hashed into k' bits)
 * Reachability includes the vertex itself (Table 1: Des(u) and Anc(u) contain u).
 * A label takes W 64-bit words, W = 1, 2 or 4, the smallest that holds max(k, k') bits
 * (dbl_label_words); bit i of a label is bit i % 64 of its word i / 64.
 *
 * Conventions for every entry point:
 *   - Array arguments named d_* are DEVICE pointers (for example the data pointer of a torch
 *     tensor on the same GPU); arguments named h_* or documented as host arrays are host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is ordered on that stream; the
 *     call returns after its own work has finished (each call synchronises the stream once at
 *     its end to report its status), unless stated otherwise.
 *   - The caller owns every array it passes; the index owns all device memory it allocates.
 *   - Vertex ids are uint32 in [0, n). No exception crosses this boundary; every call returns a
 *     dbl_status. An index is used by one host thread at a time.
 *   - The index lives on the device that is current when dbl_build is called; later calls make
 *     that device current themselves.
 */
#ifndef DBL_H
#define DBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dbl_index dbl_index;
typedef struct dbl_query_ctx dbl_query_ctx;

typedef enum {
  DBL_OK = 0,
  DBL_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad option */
  DBL_ERR_VERTEX_RANGE = 2,  /* some vertex id >= n; nothing was changed */
  DBL_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed */
  DBL_ERR_DEVICE = 4         /* a HIP runtime error */
} dbl_status;

/* Decision class of a query, stored in bits 1-3 of each output byte of dbl_query_batch. */
typedef enum {
  DBL_CLASS_SELF = 0,      /* u == v: true (Table 1, Des(u) contains u) */
  DBL_CLASS_DL_HIT = 1,    /* DL_out(u) & DL_in(v) != 0: true (Lemma 1) */
  DBL_CLASS_BL_MISS = 2,   /* BL containment fails: false (Lemma 2) */
  DBL_CLASS_THM1 = 3,      /* DL_out(v) & DL_in(u) != 0: false (Theorem 1) */
  DBL_CLASS_THM2 = 4,      /* u or v shares an SCC with a landmark: false (Theorem 2) */
  DBL_CLASS_BFS_TRUE = 5,  /* label-pruned BFS of Algorithm 2 found v */
  DBL_CLASS_BFS_FALSE = 6  /* label-pruned BFS of Algorithm 2 did not find v */
} dbl_class;

typedef struct {
  /* k: number of landmarks, 0..256 (default 64). Landmarks are the top-k vertices by
     M(u) = |Pre(u)| * |Suc(u)| (Section 3.1), ties broken by smaller id; DL bit i stands for
     the i-th landmark. Bits >= k stay zero. */
  uint32_t num_landmarks;
  /* k': number of BL hash buckets, a power of two in 1..256 (default 64). */
  uint32_t bl_bits;
  /* Optional HOST array [num_landmarks]: explicit ordered landmark list (distinct ids < n). */
  const uint32_t *landmarks;
  /* Optional HOST array [n]: the leaf hash h(x) for every vertex, each < bl_bits. Default:
     h(x) = (x * 0x9E3779B97F4A7C15 mod 2^64) >> (64 - log2 k') (Fibonacci hashing). */
  const uint8_t *leaf_bucket;
  /* Optional HOST array [n]: explicit leaf sets, bit 0 = x in S_in, bit 1 = x in S_out.
     Default: S_in / S_out = vertices of zero in- / out-degree that are not landmarks. */
  const uint8_t *leaf_flags;
  /* Per-vertex spare adjacency capacity: cap = deg + max(ceil(slack_fraction*deg), slack_min),
     in both the forward and the reverse CSR. Defaults 0.25 and 4. */
  float slack_fraction;
  uint32_t slack_min;
  /* Concurrent BFS slots (one wavefront each) for queries the labels cannot decide; 0 = auto. */
  uint32_t bfs_slots;
  /* Queue entries per BFS slot (0 = auto: min(n, 2^18)). A query whose pruned BFS needs more
     runs on the whole device instead; the answer is the same. */
  uint32_t bfs_queue_cap;
  /* Nonzero: the build edges are known to hold no duplicate (the hash de-duplication pass is
     skipped). Self-loops are always dropped. */
  uint32_t edges_unique;
  /* Landmark ranking (Table 3): 0 = |Pre|*|Suc| (the paper's choice, default), 1 = max,
     2 = min, 3 = sum of |Pre| and |Suc|. Ties go to the smaller id. */
  uint32_t landmark_rank;
  /* Leaf threshold r (the leaf-selection paragraph of the experiments): 0 = leaves are the
     zero-in / zero-out-degree vertices (default); r > 0 = every non-landmark vertex with
     |Pre|*|Suc| <= r is a source of both BL labels. */
  uint64_t leaf_threshold;
  /* Kernel kinds to time from the build on, as the argument of dbl_time_kernels (NULL = none);
     lets the build's own propagation rounds be timed. */
  const char *time_kernels;
  /* Initial dbl_tuning.pull_threshold, so that the build's own rounds follow it (default 128;
     0 = push only). */
  uint32_t pull_threshold;
  /* Initial dbl_tuning.pull_all_threshold (default 512; 0 = always test the frontier). */
  uint32_t pull_all_threshold;
  /* Row fill of the build's CSRs (layout only; the labels never depend on it): 0 = auto
     (default; rows are assembled in on-chip memory when a direction's edges are not grouped by
     source row and the rows being filled at once span more than the last-level cache),
     1 = always direct, 2 = always assembled when possible. Values above 2 are rejected. */
  uint32_t row_fill;
} dbl_options;

/* Which labels a query may use (the ablations of Table 4). */
enum { DBL_RULES_DL = 1, DBL_RULES_BL = 2, DBL_RULES_ALL = 3 };

typedef struct {
  uint64_t num_edges;         /* stored forward adjacency entries (build edges + insertions) */
  uint64_t build_rounds;      /* propagation rounds of the last build */
  uint64_t insert_calls;      /* dbl_insert_edges calls that changed the graph */
  uint64_t insert_rounds;     /* propagation rounds over all insertion calls */
  uint64_t vertices_expanded; /* frontier entries expanded (build + insertions) */
  uint64_t edges_relaxed;     /* adjacency entries scanned by propagation */
  uint64_t csr_regrows;       /* times the CSR was rebuilt because a row ran out of slack */
  uint64_t queries;           /* pairs answered */
  uint64_t query_class[7];    /* pairs per dbl_class */
  uint64_t bfs_vertices;      /* vertices dequeued by query BFS */
  uint64_t bfs_edges;         /* adjacency entries scanned by query BFS */
  uint64_t bfs_heavy;         /* BFS that outgrew a slot and ran on the whole device */
  uint64_t pull_rounds;       /* (round, direction) pairs propagated by pulling */
  uint64_t server_requests;   /* requests served by a resident workgroup (dbl_insert_edges_each
                                 with insert_server 1 or 2) */
  double server_busy_us;      /* device time it spent on them (device wall clock): from seeing a
                                 request to publishing its status (1); the launches' whole
                                 time (2) */
  uint64_t batch_stalls;      /* persistent insertion launches that ran out of time at a grid
                                 barrier and were finished another way (dbl_tuning) */
  uint64_t build_long_bins;   /* vertex-range bins of the last build (both directions) that held
                                 so many edges that they were split over several workgroups */
} dbl_stats;

/* Fill *opt with the defaults listed above. */
void dbl_default_options(dbl_options *opt);

/*
 * Build the index for G = (V = [0,n), E = {(d_src[i], d_dst[i])}) (Algorithm 1 and the
 * construction paragraph of Section 3.1).
 *   n: vertex count, 1 <= n < 2^31.  m: edge count (0 allowed).
 *   d_src, d_dst: device arrays [m]. Self-loops are dropped; duplicate edges are dropped.
 *   opt: NULL = defaults.  *out receives the new index (NULL on error).
 * Device memory: besides the index, the build holds scratch until it returns: 9 bytes per
 * edge for the partitioned edges and keep flags, the de-duplication table (16-32 bytes per
 * edge) unless edges_unique, and, once a direction's rows are assembled in LDS (row_fill), 8
 * bytes per edge of staging, which lives in that table when there is one. If the staging
 * buffer cannot be had, rows are filled directly instead. A vertex range holding far more than
 * its share of the edges (ids numbered by degree) is split over several workgroups, with a few
 * MB of cursors.
 * Errors: INVALID_ARG (bad options or sizes), VERTEX_RANGE (an id >= n), OUT_OF_MEMORY,
 * DEVICE. On error no index is returned and nothing is leaked.
 */
dbl_status dbl_build(uint32_t n, uint64_t m, const uint32_t *d_src, const uint32_t *d_dst,
                     const dbl_options *opt, void *stream, dbl_index **out);

/*
 * Insert edges (d_src[i], d_dst[i]), i < count, and bring all four labels to the values they
 * have on the grown graph (Algorithm 3 and Section 4, for DL_in / DL_out / BL_in / BL_out).
 * The landmarks, the leaf sets and h stay those fixed at build time. A batch is a set: the
 * result equals inserting its edges one at a time in any order. Self-loops are ignored;
 * duplicates are accepted and change no label.
 *   d_src, d_dst: device arrays [count]; count == 0 is a no-op.
 * Errors: VERTEX_RANGE if any id >= n — then the index is left exactly as it was.
 */
dbl_status dbl_insert_edges(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                            const uint32_t *d_dst, void *stream);

/*
 * Add `count` vertices (Section 1: the graph grows by new edges and vertices). The new ids are
 * n .. n+count-1 (*first receives n; may be NULL). A new vertex has no edges and empty labels,
 * and it is not a BL source: the leaf sets stay those fixed at build time. Edges to and from
 * new vertices are then inserted with dbl_insert_edges. Any pending work on `stream` finishes
 * first. Errors: INVALID_ARG if the vertex count would reach 2^31; OUT_OF_MEMORY.
 */
dbl_status dbl_add_vertices(dbl_index *ix, uint32_t count, uint32_t *first, void *stream);

/*
 * The one-request-at-a-time form of dbl_insert_edges: edge i is inserted as its own request
 * (validate, append, seed, propagate to the fixpoint, report), in order, exactly as `count`
 * calls of dbl_insert_edges with one edge each. By default (dbl_tuning.insert_server = 2) one
 * resident workgroup reads the requests from d_src/d_dst and applies them in that order, with
 * no host step per request. With insert_server = 1 the ids are first copied to the host (the
 * stream is synchronised), and the host then hands each edge to a resident workgroup with its
 * release, after the previous request was reported. h_latency_us: optional HOST array [count]
 * that receives each request's time in microseconds (insert_server 2: device time from the end
 * of the previous request, plus the host's part when the host finished the request; 1 and 0:
 * wall time from release to report).
 * Stops at the first failing request and returns its status (earlier requests stay applied).
 */
dbl_status dbl_insert_edges_each(dbl_index *ix, uint64_t count, const uint32_t *d_src,
                                 const uint32_t *d_dst, float *h_latency_us, void *stream);

/*
 * Answer q(d_u[i], d_v[i]) for i < count (Algorithm 2 with Theorems 1 and 2).
 *   d_out: device array [count]; d_out[i] = answer | (dbl_class << 1), answer 1 = u reaches v.
 * Answers are exact reachability on the current graph. Errors: VERTEX_RANGE if any id >= n
 * (d_out is then unspecified); the index is never modified by a query.
 */
dbl_status dbl_query_batch(dbl_index *ix, uint64_t count, const uint32_t *d_u,
                           const uint32_t *d_v, uint8_t *d_out, void *stream);

/*
 * Query contexts: the scratch of one in-flight query batch (control block, status word, BFS
 * slots, undecided-pair list). dbl_query_batch uses a context owned by the index; a caller that
 * wants several query batches in flight at once (on different streams, from different host
 * threads) gives each its own context. Queries never modify the index, so batches on different
 * contexts may overlap each other; they must not overlap an insertion on the same index.
 *   bfs_slots, queue_cap: as in dbl_options (0 = the index's setting).
 *   dbl_query_ctx_bytes: device memory a context needs for batches of `batch` pairs (for
 *   admission decisions).
 * A context belongs to one index, is used by one host thread at a time, and is released by
 * dbl_query_ctx_destroy (or with its index). Its counters stay in the index's statistics.
 */
uint64_t dbl_query_ctx_bytes(const dbl_index *ix, uint32_t bfs_slots, uint32_t queue_cap,
                             uint64_t batch);
dbl_status dbl_query_ctx_create(dbl_index *ix, uint32_t bfs_slots, uint32_t queue_cap,
                                dbl_query_ctx **out);
/* dbl_query_batch with the scratch of `ctx`; same semantics and errors. */
dbl_status dbl_query_batch_ctx(dbl_index *ix, dbl_query_ctx *ctx, uint64_t count,
                               const uint32_t *d_u, const uint32_t *d_v, uint8_t *d_out,
                               void *stream);
void dbl_query_ctx_destroy(dbl_query_ctx *ctx);

/* dbl_query_batch using only the labels in `rules` (DBL_RULES_*): without DL the rules of
   Lemma 1 and Theorems 1-2 and the BFS's DL prune are skipped; without BL the rule of Lemma 2
   and the BL prune. Answers stay exact; only the decision classes and the BFS work change.
   ctx may be NULL (the index's own context). */
dbl_status dbl_query_batch_rules(dbl_index *ix, dbl_query_ctx *ctx, uint64_t count,
                                 const uint32_t *d_u, const uint32_t *d_v, uint8_t *d_out,
                                 uint32_t rules, void *stream);

/*
 * dbl_query_batch for callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation). Same arguments, answers
 * and errors as dbl_query_batch; it calls no allocator at all. Its scratch (control block,
 * undecided-pair list, BFS slots, the whole-device BFS's bitmaps and queues) lives in one
 * static device array of 128 MiB that every GPU the library runs on holds from the loading of
 * the library's code until the process ends. Limits: with n the index's vertex count and
 * B = ceil(count / 256), 8.25 n + 2 KiB * B + 4 (n / 8 + 4 q) bytes (q = min(n, 65536, the
 * index's bfs_queue_cap if set), each part rounded up to 256 bytes) must fit in the 128 MiB
 * less a 16 KiB header, i.e. at least four BFS slots must fit; a larger n or count returns
 * DBL_ERR_INVALID_ARG and does nothing. Up to 256 BFS slots (at most the index's bfs_slots
 * option) are used, as many as fit. The array keeps what the last call left; each call clears
 * what must start at zero. All calls on one GPU share its array, so two calls that overlapped
 * on one GPU would race; the library serialises them instead (a call holds the GPU's array
 * until its work has finished). The stream is synchronised before the call returns. These
 * batches are not counted in dbl_get_stats.
 */
dbl_status dbl_query_batch_noalloc(dbl_index *ix, uint64_t count, const uint32_t *d_u,
                                   const uint32_t *d_v, uint8_t *d_out, void *stream);

/* Copy the labels out: each argument is a device array [n * W] of uint64, W =
   dbl_label_words(ix), vertex x's label in words [x * W, x * W + W) (any may be NULL). */
dbl_status dbl_read_labels(const dbl_index *ix, uint64_t *d_dl_in, uint64_t *d_dl_out,
                           uint64_t *d_bl_in, uint64_t *d_bl_out, void *stream);

/* Copy the ordered landmark list to HOST array h_out (room for num_landmarks entries, at most
   256); *k receives the landmark count. */
dbl_status dbl_get_landmarks(const dbl_index *ix, uint32_t *h_out, uint32_t *k);

/* Copy the leaf sets fixed at build time to HOST array h_flags [n] (bit 0 S_in, bit 1 S_out)
   and the leaf hash table to HOST array h_bucket [n]; either may be NULL. */
dbl_status dbl_get_leaves(const dbl_index *ix, uint8_t *h_flags, uint8_t *h_bucket);

/* Counters since build (host struct). */
dbl_status dbl_get_stats(const dbl_index *ix, dbl_stats *out);

/* Launch timing of the library's own kernels, measured with HIP events recorded on the
   caller's stream around each launch of the selected kinds (for roofline measurements). */
typedef struct {
  char name[32];      /* kernel kind, e.g. "query_label", "query_bfs", "insert_small" */
  uint64_t launches;  /* timed launches since timing was enabled */
  double total_ms;    /* summed event-to-event time */
  double max_ms;
} dbl_kernel_time;

/* Enable timing for a comma-separated list of kernel kinds ("all" = every kind; NULL or "" =
   off), optionally followed by ":N" to time one launch in every N of each kind (the first, the
   N+1-th, ...). Enabling clears the accumulated times. Kinds: insert_small, insert_apply, local_rounds,
   insert_server (one request-server launch), round (one grid propagation round), query_label,
   query_bfs, query_graph (one graph launch of a query batch), insert_batch (one persistent
   launch of an insertion batch, or its graph launch), insert_stream (one launch of the
   device-fed request stream). */
dbl_status dbl_time_kernels(dbl_index *ix, const char *kinds);

/* Copy up to `cap` per-kind records (kinds with at least one launch) to HOST array h_out;
   *count receives the number written. Waits for outstanding timed launches. */
dbl_status dbl_read_kernel_times(dbl_index *ix, dbl_kernel_time *h_out, uint32_t cap,
                                 uint32_t *count);

/* Runtime tuning. None of these changes a label or an answer (the labels are the unique least
   fixpoint whatever the schedule); they change how work is split into launches. */
typedef struct {
  uint32_t small_batch;        /* insertion batches up to this size run in one workgroup
                                  (0..65536; default 2048) */
  uint32_t local_max_frontier; /* single-workgroup propagation rounds while the frontier has at
                                  most this many entries (default 8192) */
  uint32_t local_max_edges;    /* ... and would scan at most this many edges (default 65536) */
  uint32_t round_grid;         /* blocks of a grid propagation round (1..2048; default 2048) */
  uint32_t bfs_slots;          /* BFS slots of the index's own query context (default 1024) */
  uint32_t insert_server;      /* how dbl_insert_edges_each delivers its requests. 2 (default):
                                  one resident workgroup reads them from the device arrays and
                                  applies them one after another (no host step per request;
                                  latencies are device time); 1: one resident workgroup takes
                                  them one after another from pinned host memory, the host
                                  releasing each after the previous one was reported (a host
                                  round trip per request); 0: one launch per request */
  uint32_t server_idle_us;     /* a server launch ends after this long without a request and is
                                  started again by the next one (0..10^7; default 200000) */
  uint32_t pull_threshold;     /* a grid propagation round pulls a direction (every vertex ORs in
                                  its frontier neighbours' labels) when the frontier would push at
                                  least pull_threshold / 1024 of that direction's edges, and
                                  pushes otherwise; 0 = always push (default 128) */
  uint32_t server_polls;       /* reads of the doorbell the request server keeps in flight: 1 or
                                  4 (default 4) */
  uint32_t query_graph;        /* 1: each query batch is one HIP graph launch (label kernel, then
                                  the BFS kernel), instantiated once per query context and replayed
                                  with the batch's arguments; 0 (default): two kernel launches */
  uint32_t server_warm;        /* 1: before serving, dbl_insert_edges_each reads the labels and
                                  row descriptors once so that the requests find them in the
                                  memory-side cache; 0 (default): it does not (measured: the same
                                  per-request latency either way) */
  uint32_t pull_all_threshold; /* a pulled direction whose frontier would push at least
                                  pull_all_threshold / 1024 of its edges reads the label of every
                                  neighbour instead of testing which ones are in the frontier (a
                                  neighbour outside it adds no bit); 0 = always test (default
                                  512) */
  uint32_t insert_persistent;  /* 1 (default): an insertion batch above small_batch runs in one
                                  persistent launch (one workgroup per compute unit): validation,
                                  appends and seeds, and the propagation rounds separated by grid
                                  barriers; 0: several launches, rounds driven by the host */
  uint32_t insert_graph;       /* 1: that launch is the replay of a one-node HIP graph
                                  instantiated once per index and given each batch's arguments;
                                  0 (default): a plain launch */
  uint32_t batch_max_frontier; /* the persistent launch leaves a frontier of more entries than
                                  this to the host's direction-optimised rounds (default 131072;
                                  at least 1) */
  uint32_t gather_wait_us;     /* the persistent launch first waits until all its workgroups are
                                  resident, at most this long (default 20000, at most 10^7); if
                                  they are not, nothing has changed and the batch runs in several
                                  launches instead */
  uint32_t barrier_wait_us;    /* longest wait at one of its later grid barriers (default
                                  2000000, at most 10^8); past it the launch stops and the host
                                  re-propagates from every vertex (the result is the same) */
  uint32_t batch_grid;         /* workgroups of the persistent launch (0 = one per compute unit,
                                  the default; at most 2048). More than fit on the device at once
                                  never gather: such a launch gives up after gather_wait_us */
} dbl_tuning;

dbl_status dbl_get_tuning(const dbl_index *ix, dbl_tuning *out);
dbl_status dbl_set_tuning(dbl_index *ix, const dbl_tuning *t);

/* Vertex count of the index. */
uint32_t dbl_num_vertices(const dbl_index *ix);

/* Words per label W (1, 2 or 4; 0 for NULL): the smallest W with 64 W >= max(k, k') as
   requested in dbl_options. */
uint32_t dbl_label_words(const dbl_index *ix);

/* Release every device buffer of the index (NULL is ignored). Waits for the device first. */
void dbl_destroy(dbl_index *ix);

/* Memory cache. Device and pinned host blocks the library frees (dbl_destroy, internal resizes)
   are kept for reuse by later allocations of the same size on the same device, so repeated
   builds and query contexts do not go back to the driver. Up to the limit (default 64 GiB) of
   cached bytes is kept; everything cached is returned when an allocation fails.
     dbl_release_cache: return every cached block to the driver.
     dbl_set_cache_limit: change the limit (0 = cache nothing), trimming at once.
     dbl_cached_bytes: bytes currently cached (not in use by any index). */
void dbl_release_cache(void);
void dbl_set_cache_limit(uint64_t bytes);
uint64_t dbl_cached_bytes(void);

/* Device memory the library holds in use (every index, query context and scratch block, over
   all devices; cached blocks not included), and a cap on it: a device allocation that would
   take the bytes in use above `bytes` fails as DBL_ERR_OUT_OF_MEMORY, exactly as if the device
   were full (0 = no cap, the default). For admission decisions, and to force the out-of-memory
   paths. */
uint64_t dbl_live_bytes(void);
void dbl_set_device_limit(uint64_t bytes);

/* Static text for a status code. */
const char *dbl_status_str(dbl_status s);

#ifdef __cplusplus
}
#endif

#endif /* DBL_H */
