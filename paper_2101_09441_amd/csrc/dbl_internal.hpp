// Internal types and launch wrappers shared by the two translation units of libdbl
// (dbl_kernels.hip: device code + launch wrappers; dbl_api.cpp: the C ABI and orchestration).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbl {

// A frontier entry is a vertex id with the propagation direction in bit 31: forward entries
// carry (DL_in, BL_in) along Suc, backward entries carry (DL_out, BL_out) along Pre.
constexpr uint32_t kDirBit = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;

// Frontier vertices whose row is longer than kHeavyDeg are split into chunks of kChunk entries
// and expanded by a separate kernel so that one hub does not serialise a whole round.
constexpr uint32_t kHeavyDeg = 4096;
constexpr uint32_t kChunk = 4096;

// Single-workgroup propagation handles a round itself while the frontier and the edges it
// would scan stay below runtime bounds (defaults below); above them it hands the frontier to
// grid rounds.
constexpr uint32_t kLocalMaxFrontier = 8192;
constexpr uint32_t kLocalMaxEdges = 1u << 16;
constexpr uint32_t kLocalThreads = 1024;

// Insert batches up to this size (runtime, default below, at most kSmallBatchMax) are
// validated, applied and propagated by one workgroup.
constexpr uint32_t kSmallBatch = 2048;
constexpr uint32_t kSmallBatchMax = 1u << 16;

constexpr uint32_t kErrRange = 1u;
// A grid barrier of the persistent insertion kernel ran out of time: before anything was
// changed (the host runs the batch another way) or after (the host re-propagates every label).
constexpr uint32_t kErrStallEarly = 2u, kErrStallLate = 4u;

// One direction of the adjacency: row x holds entries col[off[x] .. off[x] + min(deg, cap)).
// deg may exceed cap after an append found the row full; the overflowing entries wait in the
// overflow list until the CSR is regrown.
struct Csr {
  unsigned long long *off;
  uint32_t *deg;
  uint32_t *cap;
  uint32_t *col;
};

// Counters in the control block (written by one thread at a time).
enum CtrIdx : uint32_t {
  kCtrServerTicks = 0,  // device wall-clock ticks the request server spent on requests
  kCtrServerReqs = 1,   // requests it published
  kCtrFrontEntries = 2, // 2, 3: frontier entries per direction (frontier scan)
  kCtrFrontEdges = 4,   // 4, 5: edges a push of those entries would scan, per direction
  kCtrCount = 16
};

// Device-side control block; the host reads it back in one transfer at each synchronisation.
struct Ctl {
  uint32_t err;
  uint32_t cur;         // ring index (0..2) of the pending frontier
  uint32_t stamp;       // stamp of the pending frontier's entries
  uint32_t fsize[3];    // frontier sizes (ring of three)
  uint32_t heavy[2];    // chunk counts of high-degree frontier vertices (ring of two)
  uint32_t ovf_count;   // adjacency appends that found their row full
  uint32_t und_count;   // queries the labels left undecided
  uint32_t bfs_next;    // work counter of the BFS kernel
  uint32_t bfs_heavy;   // queries whose BFS outgrew a slot
  uint32_t found;       // grid BFS: target reached
  uint32_t local_rounds;
  uint32_t bfs_done;    // BFS blocks finished (the last one publishes the status)
  uint32_t pheavy;      // chunks of high-degree rows queued for the pull round
  unsigned long long ctr[kCtrCount];
};

// Status published by the device into pinned, device-mapped host memory at the end of a call's
// work; the host waits for `seq` to change instead of copying the control block and
// synchronising the stream.
struct Mirror {
  uint32_t seq;
  uint32_t err, cur, stamp;
  uint32_t fsize[3];
  uint32_t ovf_count, und_count, bfs_heavy, found;
  uint32_t pad[5];
  unsigned long long dstat[4];  // frontier scan: entries and push edges per direction
  // Fast path of one small insertion: sequence number (low 32 bits) and flags (high 32 bits)
  // in one store; the host reads the other fields only when a flag is set.
  unsigned long long fast;
};
constexpr uint32_t kFastErr = 1u, kFastOvf = 2u, kFastPending = 4u;
// Doorbell of the request server: two 64-bit slots in pinned host memory written by the host.
// Request i is released by writing its edge ((u << 32) | v) into slot i & 1; the host empties
// that slot again once request i is done (before it releases request i + 2). kDoorStop in a
// slot ends the server. Neither marker is an edge: their u is 0xFFFFFFFF, never a vertex id.
constexpr unsigned long long kDoorEmpty = ~0ull;
constexpr unsigned long long kDoorStop = ~0ull - 1ull;

// Per-block / per-slot statistics (plain read-modify-write by the owning block, no atomics).
constexpr uint32_t kQueryGrid = 64;    // class-counter stripes (label-kernel block % 64)
constexpr uint32_t kQClsStride = 8;    // class counters per stripe
constexpr uint32_t kQueryNT = 256;     // pairs per label-kernel block (one per thread)
constexpr uint32_t kBfsCtrStride = 4;  // vertices, edges, true, false per BFS slot
// propagation counters: grid rounds use slots [0, 2048), heavy chunks [2048, 3072), the
// single-workgroup rounds slot 3072
constexpr uint32_t kRoundGridMax = 2048, kHeavyGrid = 1024;
// Stripes of the frontier scan's block reductions (atomics on one address are served one at a
// time); stripe s holds 16 label words and 4 counts at fu + kFuStride * (1 + s).
constexpr uint32_t kFuStripes = 64, kFuStride = 32, kFuWords = kFuStride * (1 + kFuStripes);
constexpr uint32_t kPropCtrSlots = kRoundGridMax + kHeavyGrid + 1;

// Overflowing append: row `x` (bit 31 = reverse CSR) wanted entry `y` at position `pos`.
struct Ovf {
  uint32_t x, pos, y, pad;
};

// Labels of k (DL) and k' (BL) bits take W = words 64-bit words each, W in {1, 2, 4} (the
// smallest power of two with 64 W >= max(k, k')); bit i of a label sits in word i / 64, bit
// i % 64. Vertex x owns the record lab[4 W x .. 4 W x + 4 W) = {DL_in, BL_in, DL_out, BL_out},
// so each propagation direction reads and ORs one contiguous half {DL, BL} of 2 W words.
constexpr uint32_t kMaxLabelBits = 256;
struct LabelsView {
  unsigned long long *lab;
  uint32_t words;
};

// ---------------------------------------------------------------- launch wrappers
// Every wrapper enqueues on `s` and returns the launch status.

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, uint64_t count,
                           hipStream_t s);
hipError_t launch_ctl_reset_query(Ctl *ctl, hipStream_t s);
// read `bytes` at p once (16-byte aligned) so they are cached for what follows
hipError_t launch_touch(const void *p, uint64_t bytes, unsigned long long *sink, hipStream_t s);
// *out = sum of a[0..count)
hipError_t launch_sum_u32(const uint32_t *a, uint64_t count, unsigned long long *out,
                          hipStream_t s);
hipError_t launch_publish(Ctl *ctl, Mirror *m, uint32_t seq, hipStream_t s);

// build: ingest
hipError_t launch_validate_pairs(const uint32_t *a, const uint32_t *b, uint64_t count, uint32_t n,
                                 Ctl *ctl, hipStream_t s);
hipError_t launch_dedup_mark(const uint32_t *src, const uint32_t *dst, uint64_t m,
                             unsigned long long *table, uint64_t mask, uint8_t *keep,
                             int assume_unique, hipStream_t s);
hipError_t launch_slack_cap(const uint32_t *deg, uint32_t *cap, uint32_t n, float frac,
                            uint32_t smin, hipStream_t s);
// exclusive scan of cap[n] into off[n]; *total receives the sum. tmp: scan_tmp_words(n) words.
uint64_t scan_tmp_words(uint32_t n);
hipError_t scan_exclusive(const uint32_t *in, unsigned long long *out, uint32_t n, unsigned long long *tmp,
                          unsigned long long *total, hipStream_t s);
// Binned ingest of one direction: partition the kept (key, val) edges by key range into
// out[cnt] = key << 32 | val (*kept receives cnt; runs[1] counts a sample of the kept edges and
// runs[0] those of the sample whose key repeats the key of the input edge before them); nblk
// chunks (<= kBinBlocks);
// counts/offs: nblk * bin_count(n) entries; scan_tmp: scan_tmp_words(nblk * bin_count(n)).
constexpr uint32_t kBinBlocks = 2048;
uint32_t bin_shift(uint32_t n);
inline uint32_t bin_count(uint32_t n) { return ((n - 1) >> bin_shift(n)) + 1; }
hipError_t launch_bin_edges(const uint32_t *key, const uint32_t *val, const uint8_t *keep,
                            uint64_t m, uint32_t n, uint32_t nblk, uint32_t *counts,
                            unsigned long long *offs, unsigned long long *scan_tmp,
                            unsigned long long *kept, unsigned long long *runs,
                            unsigned long long *out, hipStream_t s);
// From partitioned edges (offs, nblk, kept as left by launch_bin_edges; kept_host = *kept):
// g == nullptr: deg[v] = degree of v; else fill g's rows (g.off set; g.deg is the degree and
// stays so). fill_tmp (optional; kept_host entries, allowed only while the CSR holds fewer than
// 2^32 column slots) lets the fill assemble runs of rows in LDS.
// Bins of at least long_min edges are cut into chunks (LongChunk entries in device memory,
// nchunks of them; slot = the bin's index among the long bins) handled by one workgroup each;
// deg must be zero on entry when there are any, and the fill needs `cursors`, kBinVerts zeroed
// words per long bin. long_min = ~0 and nchunks = 0: every bin in one workgroup.
struct LongChunk {
  uint32_t bin, slot;
  unsigned long long lo, hi;
};
constexpr uint32_t kBinVertsMax = 16384;  // vertices of a bin handled in LDS (kBinVerts)
// out[b] = offs[b * nblk] for b < nbins: the first partitioned edge of each bin
hipError_t launch_bin_starts(const unsigned long long *offs, uint32_t nblk, uint32_t nbins,
                             unsigned long long *out, hipStream_t s);
hipError_t launch_bin_rows(const unsigned long long *edges, const unsigned long long *offs,
                           uint32_t nblk, uint32_t n, const unsigned long long *kept,
                           uint64_t kept_host, uint32_t *deg, const Csr *g,
                           unsigned long long *fill_tmp, unsigned long long long_min,
                           const LongChunk *chunks, uint32_t nchunks, uint32_t *cursors,
                           hipStream_t s);
// deg[key] += 1 per partitioned edge; rows filled from partitioned edges (g.deg zero on entry)
hipError_t launch_deg_binned(const unsigned long long *edges, uint64_t cnt, uint32_t *deg,
                             hipStream_t s);
hipError_t launch_fill_binned(const unsigned long long *edges, uint64_t cnt, Csr g,
                              hipStream_t s);

// build: landmark selection. Writes the top-k vertex ids by (M desc, id asc) into out[k].
// tmp_m / tmp_id: topk_tmp_entries(n) entries each.
uint64_t topk_tmp_entries(uint32_t n);
// rank: 0 product, 1 max, 2 min, 3 sum of in- and out-degree
hipError_t select_topk(const uint32_t *indeg, const uint32_t *outdeg, uint32_t n, uint32_t k,
                       uint32_t rank, unsigned long long *tmp_m, uint32_t *tmp_id, uint32_t *out,
                       hipStream_t s);

// build: seeds
hipError_t launch_seed(LabelsView L, uint32_t n, const uint32_t *landmarks, uint32_t k,
                       const uint32_t *indeg, const uint32_t *outdeg,
                       const uint8_t *leaf_flags_in, const uint8_t *bucket_in, uint32_t kp_bits,
                       unsigned long long leaf_threshold, uint8_t *leaf_flags_out,
                       uint8_t *bucket_out, uint8_t *is_landmark, hipStream_t s);
hipError_t launch_init_frontier(LabelsView L, uint32_t n, Csr f, Csr r, uint32_t *frontier,
                                Ctl *ctl, uint32_t *inq, uint32_t stamp, hipStream_t s);

// propagation
struct PropArgs {
  LabelsView L;
  Csr f, r;
  uint32_t *fq[3];  // frontier ring
  uint32_t *inq;    // [2n] stamp of the frontier each (vertex, direction) is queued in
  unsigned long long *heavy_list;
  unsigned long long *pheavy_list;  // chunks of the pull round (same capacity)
  uint64_t heavy_cap;
  unsigned long long *fbm;          // frontier bitmaps of the pull round, one per direction:
  uint64_t fbm_wpd;                 // bit x of fbm[dir * fbm_wpd + x / 64]
  // OR of the frontier's labels, per direction, in fu[dir * 8 ...]; the frontier scan adds
  // into kFuStripes stripes (each kFuStride words, from word kFuStride on) that a one-block
  // kernel then reduces
  unsigned long long *fu;
  unsigned long long *pcnt;  // [kPropCtrSlots * 2] per-block (expanded, relaxed) counters
  uint32_t local_max_frontier, local_max_edges;
  Ctl *ctl;
};
// one grid round: expand the frontier at ring `ring` (entries stamped `stamp`). skip_mask: the
// directions (bit d) another kernel handles this round; bookkeep: advance ctl->cur / stamp (off
// when the frontier scan has done it)
hipError_t launch_round(const PropArgs &a, uint32_t ring, uint32_t stamp, uint32_t grid,
                        hipStream_t s, uint32_t skip_mask = 0, bool bookkeep = true);
// Direction-optimised rounds. frontier_scan: clear the bitmap (fbm_words words) and the
// per-direction counters, mark the frontier, count entries and push edges per direction and
// advance ctl->cur / stamp. pull: for the directions in dmask, every vertex ORs in the labels
// of its frontier neighbours (Pre for forward, Suc for backward) and joins the next frontier
// if it grew; for the directions in allmask it ORs in every neighbour's label without the
// frontier test (a neighbour outside the frontier has no bit its out-neighbours lack), except
// on rows long enough for k_pull_heavy.
hipError_t launch_frontier_scan(const PropArgs &a, uint32_t ring, uint32_t stamp,
                                uint64_t fbm_words, hipStream_t s);
hipError_t launch_pull(const PropArgs &a, uint32_t n, uint32_t dmask, uint32_t allmask,
                       uint32_t ring, uint32_t stamp, uint32_t grid, hipStream_t s);
// single-workgroup rounds starting from ctl->cur / ctl->stamp; publishes the status to m (if
// not null) with sequence number seq when done
hipError_t launch_local_rounds(const PropArgs &a, Mirror *m, uint32_t seq, hipStream_t s);

// insertion
hipError_t launch_insert_small(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint32_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap, Mirror *m,
                               uint32_t seq, hipStream_t s);
// request server for requests [first, count); see k_insert_server
hipError_t launch_insert_server(const PropArgs &a, uint32_t first, uint32_t count, uint32_t n,
                                Ovf *ovf, uint64_t ovf_cap, Mirror *m,
                                const unsigned long long *door, uint32_t seq0,
                                unsigned long long idle_ticks, uint32_t polls, hipStream_t s);
// the device-fed one-request-at-a-time form: requests [first, count) of src/dst, one after
// another; publishes {seq0 + requests applied, flags}; ticks (may be null): per-request device
// clock ticks
hipError_t launch_insert_stream(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                                uint32_t first, uint32_t count, uint32_t n, Ovf *ovf,
                                uint64_t ovf_cap, Mirror *m, uint32_t seq0, uint32_t *ticks,
                                hipStream_t s);
hipError_t launch_insert_apply(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint64_t count, Ovf *ovf, uint64_t ovf_cap, hipStream_t s);
// One insertion batch in one persistent launch (see k_insert_batch): validation, the appends and
// seeds, and the propagation rounds, separated by grid barriers; publishes the fast status word
// {seq, flags} to m. grid: blocks of kLocalThreads threads, all of which must fit on the device
// at once (insert_batch_grid gives one per compute unit). max_frontier: a frontier larger than
// this is left pending for the host's rounds. start_ticks / wait_ticks: the longest wait at the
// start gathering / at a later barrier, in device wall-clock ticks. bar: kBarWords words, zero
// before the first launch (every launch leaves them zero).
struct BatchLaunch {
  const void *func;   // kernel for the label width
  uint32_t grid;
};
hipError_t insert_batch_grid(uint32_t words, BatchLaunch *out);
constexpr uint32_t kBarLine = 32;  // 32-bit words per 128-byte line
constexpr uint32_t kBarGather = 0, kBarCount = kBarLine, kBarGen = 2 * kBarLine,
                   kBarDone = 3 * kBarLine, kBarWords = 4 * kBarLine;
hipError_t launch_insert_batch(const PropArgs &a, const uint32_t *src, const uint32_t *dst,
                               uint64_t count, uint32_t n, Ovf *ovf, uint64_t ovf_cap, Mirror *m,
                               uint32_t seq, uint32_t max_frontier,
                               unsigned long long start_ticks, unsigned long long wait_ticks,
                               uint32_t *bar, uint32_t grid, hipStream_t s);
// Kernel-node parameters of the same launch, for a graph; args points to its 13 arguments in
// order (a, src, dst, count, n, ovf, ovf_cap, m, seq, max_frontier, start_ticks, wait_ticks,
// bar).
hipError_t insert_batch_node_params(uint32_t words, uint32_t grid, void **args,
                                    hipKernelNodeParams *p);
hipError_t launch_regrow_copy(Csr old_g, Csr new_g, uint32_t n, hipStream_t s);
hipError_t launch_place_overflow(const Ovf *ovf, uint32_t count, uint32_t dir, Csr new_g,
                                 hipStream_t s);
hipError_t launch_push_overflow(const PropArgs &a, const Ovf *ovf, uint32_t count,
                                hipStream_t s);

// queries
// Undecided pairs of label-kernel block b go to und[b * kQueryNT ...], their number to seg[b].
hipError_t launch_query_label(LabelsView L, const uint32_t *u, const uint32_t *v, uint64_t count,
                              uint32_t n, const uint32_t *fdeg, uint8_t *out, uint32_t *und,
                              uint32_t *seg, Ctl *ctl, unsigned long long *qcls, uint32_t rules,
                              hipStream_t s);
struct BfsArgs {
  LabelsView L;
  Csr f;
  const uint32_t *u, *v;
  const uint32_t *und;
  const uint32_t *seg;      // undecided count per label-kernel block
  uint32_t nseg;            // label-kernel blocks
  uint8_t *out;
  unsigned long long *vis;  // [slots * vis_words]
  uint64_t vis_words;
  uint32_t *queue;          // [slots * qcap]
  uint32_t qcap;
  uint32_t *heavy_q;        // queries handed to the grid BFS
  unsigned long long *cnt;  // [slots * kBfsCtrStride]
  uint32_t rules;           // bit 0: DL prune, bit 1: BL prune
  Ctl *ctl;
};
// The last wave to finish publishes the context's status (mirror m, sequence seq).
hipError_t launch_query_bfs(const BfsArgs &a, uint32_t slots, Mirror *m, uint32_t seq,
                            hipStream_t s);
// Kernel-node parameters of the two query kernels (for a graph). label_args points to the 12
// arguments of the label kernel in order (lab, u, v, count, n, fdeg, out, und, seg, ctl, qcls,
// rules); bfs_args to the 3 of the BFS kernel (BfsArgs, mirror, seq).
hipError_t query_node_params(LabelsView L, uint64_t count, uint32_t slots, void **label_args,
                             void **bfs_args, hipKernelNodeParams *label,
                             hipKernelNodeParams *bfs);
// Whole-device BFS of one query (u, v) whose slot overflowed, searched from both ends. Side 0
// follows out-edges from u, side 1 in-edges from v; each side has a visited bitmap and a queue
// of n entries whose levels are consecutive segments. In the control block fsize[side] is the
// side's queue tail, ctr[kCtrFrontEdges + side] the summed degrees of its queued vertices, and
// found is set once a side reaches a vertex the other has visited.
struct GbfsArgs {
  LabelsView L;
  Csr g[2];                         // out-edges (f) and in-edges (r)
  unsigned long long *vis[2];
  uint32_t *q[2];
  Ctl *ctl;
};
// clear both bitmaps (vis_words each) and queue u on side 0, v on side 1
hipError_t launch_gbfs_start(const GbfsArgs &a, uint64_t vis_words, uint32_t u, uint32_t v,
                             hipStream_t s);
// expand the level q[side][lo, hi)
hipError_t launch_gbfs_round(const GbfsArgs &a, uint32_t side, uint32_t lo, uint32_t hi,
                             uint32_t u, uint32_t v, uint32_t rules, hipStream_t s);
// write the answer of query qi and reset the control block's search fields
hipError_t launch_gbfs_finish(const GbfsArgs &a, uint32_t qi, uint8_t *out,
                              unsigned long long *qcls, hipStream_t s);

// bucket[x] = h(x) for x in [n0, n1) (vertices added after the build; never BL sources)
hipError_t launch_init_buckets(uint8_t *bucket, uint32_t n0, uint32_t n1, uint32_t kp_bits,
                               hipStream_t s);

hipError_t launch_unpack_labels(LabelsView L, uint32_t n, unsigned long long *dl_in,
                                unsigned long long *dl_out, unsigned long long *bl_in,
                                unsigned long long *bl_out, hipStream_t s);

}  // namespace dbl
