/*
 * DBL oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately unoptimised CPU implementation of the DBL reachability
 * index (Lyu, Li, He, Gong, "DBL: Efficient Reachability Queries on Dynamic Graphs",
 * arXiv 2101.09441). It exists to check the GPU library against, and only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes (section numbers are the paper's):
 *   - Graph model, Section 2 / Table 1: G and its reverse G'; Des(u) and Anc(u) include u.
 *   - DL label, Definition 1: DL_in(v) = landmarks that reach v, DL_out(v) = landmarks v reaches.
 *     Landmarks: top-k vertices by M(u) = |Pre(u)| * |Suc(u)| (Section 3.1).
 *   - BL label, Definition 2: BL_in(v) = hashed zero-in-degree vertices reaching v, BL_out(v) =
 *     hashed zero-out-degree vertices reached by v; leaves exclude landmarks (Section 1); a hash h
 *     maps each leaf to one of k' bits (Section 3.1, the paragraph on hash sets).
 *   - Construction, Algorithm 1: one BFS per landmark (forward for DL_in, on G' for DL_out); BL
 *     replaces the landmark by all leaves hashed to bucket i.
 *   - Query, Algorithm 2 with Theorems 1 and 2: label rules, then a pruned BFS.
 *   - Insertion, Algorithm 3 and Section 4: pruned BFS from v over Suc adding DL_in(u); the
 *     symmetric DL_out update over Pre from u adding DL_out(v); BL likewise.
 *
 * Readings where the paper is silent or its listings are incomplete (each one is listed in the
 * design notes of the repository):
 *   R1  Algorithm 1 keeps no visited set and does not label the landmark itself. Here each BFS
 *       keeps a visited set and the source receives its own bit (Des/Anc include the vertex;
 *       the Figure 1 labels give v8 its own bit although v8 is on no cycle).
 *   R2  Algorithm 3 starts from Suc(v) and never updates v. Here v is seeded first: if DL_in(u) is
 *       not contained in DL_in(v), DL_in(v) gains it and v is enqueued (the worked example of
 *       Section 4 copies DL_in(v9) into DL_in(v2)).
 *   R3  Algorithm 2's BFS keeps a visited set (marked when a vertex is enqueued).
 *   R4  q(u,u) is true (Des(u) includes u) and is decided before the label rules, class SELF.
 *   R5  Landmark order: M descending, then vertex id ascending; M is computed in 64 bits; exactly
 *       min(k, n) landmarks are taken; bit i of a DL label stands for the i-th landmark.
 *   R6  The leaf sets and h are fixed when the index is built; later insertions never add or
 *       remove BL sources.
 *   R7  Leaves are the zero-in-degree (S_in) / zero-out-degree (S_out) vertices that are not
 *       landmarks; an isolated vertex is in both. Self-loops and duplicate edges are dropped when
 *       the graph is ingested, so degrees count distinct neighbours other than the vertex itself.
 *   R8  h(x) = (x * 0x9E3779B97F4A7C15 mod 2^64) >> (64 - log2 k') (Fibonacci hashing), unless
 *       the caller supplies a bucket table (the worked example of the paper gives one).
 *   R9  Algorithm 3's skip test (Lemma 1: u already reaches v) skips all four label updates.
 *   R10 Inserted self-loops are no-ops; inserted duplicates change no label.
 *   R11 The ablations of Table 4 ("the other label disabled"): with DL disabled the rules of
 *       Lemma 1 and Theorems 1-2 and the DL prune of the BFS are skipped; with BL disabled the
 *       rule of Lemma 2 and the BL prune are skipped. Answers stay exact.
 *   R14 Labels longer than 64 bits (Table 5 uses k and k' up to 256): a label of k bits is
 *       ceil(k / 64) 64-bit words per vertex; bit i lives in word i / 64 at position i % 64.
 *   R13 Vertex insertion (Section 1: "new edges and vertices"): a new vertex arrives without
 *       edges; its labels are empty and it is not a BL source (the leaf sets stay fixed).
 *   R12 Selection variants of Table 3: the landmark rank may be max, min or sum of |Pre| and
 *       |Suc| instead of their product (ties by smaller id). Leaf threshold r (the leaf-
 *       selection paragraph of the experiments): r = 0 is the main body's rule (R7); r > 0
 *       makes every non-landmark vertex with |Pre|*|Suc| <= r a source of both BL labels.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONE 0xFFFFFFFFu

enum {
  ORC_CLASS_SELF = 0,
  ORC_CLASS_R1_DL_HIT = 1,   /* Lemma 1 */
  ORC_CLASS_R2_BL_MISS = 2,  /* Lemma 2 */
  ORC_CLASS_R3_THM1 = 3,     /* Theorem 1 */
  ORC_CLASS_R4_THM2 = 4,     /* Theorem 2 */
  ORC_CLASS_BFS_TRUE = 5,
  ORC_CLASS_BFS_FALSE = 6
};

/* growable per-vertex neighbour list */
typedef struct {
  uint32_t *v;
  uint32_t len, cap;
} orc_list;

typedef struct {
  uint32_t n;
  orc_list *suc; /* Suc(x) */
  orc_list *pre; /* Pre(x) */
  uint32_t k, kp;
  uint32_t wd, wb;          /* 64-bit words per DL / BL label (reading R14) */
  uint32_t rank_mode;       /* 0 product, 1 max, 2 min, 3 sum */
  uint64_t leaf_threshold;  /* r */
  uint32_t landmark[256];
  uint8_t *in_leaf, *out_leaf; /* membership in S_in / S_out, fixed at build */
  uint8_t *bucket;             /* h(x) for every x */
  uint64_t *dl_in, *dl_out, *bl_in, *bl_out;
} orc_index;

static int list_push(orc_list *l, uint32_t x) {
  if (l->len == l->cap) {
    uint32_t nc = l->cap ? 2 * l->cap : 4;
    uint32_t *nv = (uint32_t *)realloc(l->v, sizeof(uint32_t) * nc);
    if (!nv) return -1;
    l->v = nv;
    l->cap = nc;
  }
  l->v[l->len++] = x;
  return 0;
}

static int list_has(const orc_list *l, uint32_t x) {
  for (uint32_t i = 0; i < l->len; i++)
    if (l->v[i] == x) return 1;
  return 0;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

/* sort and drop repeated neighbours */
static void list_unique(orc_list *l) {
  if (l->len < 2) return;
  qsort(l->v, l->len, sizeof(uint32_t), cmp_u32);
  uint32_t w = 1;
  for (uint32_t i = 1; i < l->len; i++)
    if (l->v[i] != l->v[w - 1]) l->v[w++] = l->v[i];
  l->len = w;
}

void orc_free(orc_index *ix) {
  if (!ix) return;
  if (ix->suc)
    for (uint32_t x = 0; x < ix->n; x++) free(ix->suc[x].v);
  if (ix->pre)
    for (uint32_t x = 0; x < ix->n; x++) free(ix->pre[x].v);
  free(ix->suc); free(ix->pre);
  free(ix->in_leaf); free(ix->out_leaf); free(ix->bucket);
  free(ix->dl_in); free(ix->dl_out); free(ix->bl_in); free(ix->bl_out);
  free(ix);
}

/* Graph model: ingest edges (self-loops and duplicates dropped). */
orc_index *orc_new(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst) {
  orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
  if (!ix) return NULL;
  ix->n = n;
  size_t nn = n ? n : 1;
  ix->suc = (orc_list *)calloc(nn, sizeof(orc_list));
  ix->pre = (orc_list *)calloc(nn, sizeof(orc_list));
  ix->in_leaf = (uint8_t *)calloc(nn, 1);
  ix->out_leaf = (uint8_t *)calloc(nn, 1);
  ix->bucket = (uint8_t *)calloc(nn, 1);
  ix->dl_in = (uint64_t *)calloc(nn, 8);
  ix->dl_out = (uint64_t *)calloc(nn, 8);
  ix->bl_in = (uint64_t *)calloc(nn, 8);
  ix->bl_out = (uint64_t *)calloc(nn, 8);
  ix->wd = ix->wb = 1;
  if (!ix->suc || !ix->pre || !ix->in_leaf || !ix->out_leaf || !ix->bucket || !ix->dl_in ||
      !ix->dl_out || !ix->bl_in || !ix->bl_out) {
    orc_free(ix);
    return NULL;
  }
  for (uint64_t e = 0; e < m; e++) {
    uint32_t a = src[e], b = dst[e];
    if (a >= n || b >= n) { orc_free(ix); return NULL; }
    if (a == b) continue;
    if (list_push(&ix->suc[a], b) || list_push(&ix->pre[b], a)) { orc_free(ix); return NULL; }
  }
  for (uint32_t x = 0; x < n; x++) {
    list_unique(&ix->suc[x]);
    list_unique(&ix->pre[x]);
  }
  return ix;
}

uint32_t orc_out_degree(const orc_index *ix, uint32_t x) { return ix->suc[x].len; }
uint32_t orc_in_degree(const orc_index *ix, uint32_t x) { return ix->pre[x].len; }

/* Landmark rank (Section 3.1: M(u) = |Pre(u)| * |Suc(u)|; Table 3's variants: max, min, sum). */
static uint64_t rank_of(const orc_index *ix, uint32_t x) {
  uint64_t p = ix->pre[x].len, s = ix->suc[x].len;
  switch (ix->rank_mode) {
    case 1: return p > s ? p : s;
    case 2: return p < s ? p : s;
    case 3: return p + s;
    default: return p * s;
  }
}

/* Landmark selection: top-k by rank; ties by smaller id. */
static int ranks_before(const orc_index *ix, uint32_t a, uint32_t b) {
  uint64_t ma = rank_of(ix, a), mb = rank_of(ix, b);
  if (ma != mb) return ma > mb;
  return a < b;
}

void orc_set_selection(orc_index *ix, uint32_t rank_mode, uint64_t leaf_threshold) {
  ix->rank_mode = rank_mode;
  ix->leaf_threshold = leaf_threshold;
}

uint32_t orc_select_landmarks(const orc_index *ix, uint32_t k, uint32_t *out) {
  /* keep the best k seen so far in `out`, ordered best first (insertion into a sorted list) */
  uint32_t have = 0;
  for (uint32_t x = 0; x < ix->n; x++) {
    if (have < k) {
      uint32_t p = have++;
      while (p > 0 && ranks_before(ix, x, out[p - 1])) { out[p] = out[p - 1]; p--; }
      out[p] = x;
    } else if (k > 0 && ranks_before(ix, x, out[k - 1])) {
      uint32_t p = k - 1;
      while (p > 0 && ranks_before(ix, x, out[p - 1])) { out[p] = out[p - 1]; p--; }
      out[p] = x;
    }
  }
  return have;
}

/* Fibonacci hashing of a vertex id into [0, kp), kp a power of two in [1, 64]. */
uint32_t orc_hash(uint32_t x, uint32_t kp) {
  if (kp <= 1) return 0;
  uint32_t bits = 0;
  while ((1u << bits) < kp) bits++;
  return (uint32_t)(((uint64_t)x * 0x9E3779B97F4A7C15ULL) >> (64 - bits));
}

/* ---------------------------------------------------------------- construction (Algorithm 1) */

typedef struct {
  uint32_t *queue;
  uint32_t *seen; /* seen[x] == stamp means visited in the current BFS */
  uint32_t stamp;
} orc_bfs_ws;

static int ws_init(orc_bfs_ws *w, uint32_t n) {
  size_t nn = n ? n : 1;
  w->queue = (uint32_t *)malloc(sizeof(uint32_t) * nn);
  w->seen = (uint32_t *)calloc(nn, sizeof(uint32_t));
  w->stamp = 0;
  return (w->queue && w->seen) ? 0 : -1;
}

static void ws_free(orc_bfs_ws *w) { free(w->queue); free(w->seen); }

static void ws_next_stamp(orc_bfs_ws *w, uint32_t n) {
  if (++w->stamp == 0) {
    memset(w->seen, 0, sizeof(uint32_t) * (n ? n : 1));
    w->stamp = 1;
  }
}

/*
 * One BFS of Algorithm 1 from a set of sources, over Suc (forward) or Pre (backward), setting
 * `bit` in `label` of every vertex reached, sources included (reading R1).
 */
static void bfs_set_bit(const orc_index *ix, orc_bfs_ws *w, const uint32_t *sources, uint32_t ns,
                        int forward, uint64_t *label, uint32_t words, uint32_t bit, int atomic) {
  const orc_list *adj = forward ? ix->suc : ix->pre;
  const uint64_t mask = 1ULL << (bit % 64);
  label += bit / 64;
  ws_next_stamp(w, ix->n);
  uint64_t head = 0, tail = 0;
  for (uint32_t i = 0; i < ns; i++) {
    uint32_t s = sources[i];
    if (w->seen[s] == w->stamp) continue;
    w->seen[s] = w->stamp;
    w->queue[tail++] = s;
  }
  while (head < tail) {
    uint32_t p = w->queue[head++];
    if (atomic) __atomic_fetch_or(&label[(size_t)p * words], mask, __ATOMIC_RELAXED);
    else label[(size_t)p * words] |= mask;
    for (uint32_t j = 0; j < adj[p].len; j++) {
      uint32_t x = adj[p].v[j];
      if (w->seen[x] == w->stamp) continue;
      w->seen[x] = w->stamp;
      w->queue[tail++] = x;
    }
  }
}

/* One unit of construction work: a (label, bit) pair and its source set. */
typedef struct {
  int forward;
  uint64_t *label;
  uint32_t words;
  uint32_t bit;
  uint32_t *sources;
  uint32_t ns;
} orc_task;

typedef struct {
  const orc_index *ix;
  orc_task *tasks;
  uint32_t ntasks;
  uint32_t next; /* shared task counter */
  int atomic;
  int failed;
} orc_pool;

static void *pool_worker(void *arg) {
  orc_pool *p = (orc_pool *)arg;
  orc_bfs_ws w;
  if (ws_init(&w, p->ix->n)) {
    __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
    ws_free(&w);
    return NULL;
  }
  for (;;) {
    uint32_t t = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
    if (t >= p->ntasks) break;
    orc_task *tk = &p->tasks[t];
    bfs_set_bit(p->ix, &w, tk->sources, tk->ns, tk->forward, tk->label, tk->words, tk->bit,
                p->atomic);
  }
  ws_free(&w);
  return NULL;
}

/*
 * Build all four labels. landmarks: explicit ordered list (NULL = select top-k by M).
 * bucket_table: explicit h(x) for every x (NULL = Fibonacci hashing). leaf_flags: explicit leaf
 * sets, bit 0 = x in S_in, bit 1 = x in S_out (NULL = from the degrees, reading R7); it lets a
 * rebuild use the leaf sets fixed by an earlier build (reading R6). k in [0,64], kp a power of
 * two in [1,64]. threads <= 1 runs sequentially. Returns 0 on success.
 */
int orc_build(orc_index *ix, uint32_t k, uint32_t kp, const uint32_t *landmarks,
              const uint8_t *bucket_table, const uint8_t *leaf_flags, uint32_t threads) {
  if (k > 256 || kp == 0 || kp > 256 || (kp & (kp - 1))) return -1;
  uint32_t n = ix->n;
  {
    /* label widths (reading R14), from the requested k before it is capped at n */
    const uint32_t wd = k > 64 ? (k + 63) / 64 : 1, wb = kp > 64 ? kp / 64 : 1;
    const size_t nn = n ? n : 1;
    uint64_t **ld[2] = {&ix->dl_in, &ix->dl_out}, **lb[2] = {&ix->bl_in, &ix->bl_out};
    for (int i = 0; i < 2; i++) {
      uint64_t *p = (uint64_t *)realloc(*ld[i], 8 * nn * wd);
      if (!p) return -1;
      *ld[i] = p;
      p = (uint64_t *)realloc(*lb[i], 8 * nn * wb);
      if (!p) return -1;
      *lb[i] = p;
    }
    ix->wd = wd;
    ix->wb = wb;
  }
  if (k > n) k = n;
  ix->k = k;
  ix->kp = kp;
  if (landmarks) {
    for (uint32_t i = 0; i < k; i++) {
      if (landmarks[i] >= n) return -1;
      ix->landmark[i] = landmarks[i];
    }
  } else {
    orc_select_landmarks(ix, k, ix->landmark);
  }
  uint8_t *is_landmark = (uint8_t *)calloc(n ? n : 1, 1);
  if (!is_landmark) return -1;
  for (uint32_t i = 0; i < k; i++) is_landmark[ix->landmark[i]] = 1;
  for (uint32_t x = 0; x < n; x++) {
    if (leaf_flags) {
      ix->in_leaf[x] = leaf_flags[x] & 1;
      ix->out_leaf[x] = (leaf_flags[x] >> 1) & 1;
    } else if (ix->leaf_threshold) {
      const uint64_t m = (uint64_t)ix->pre[x].len * ix->suc[x].len;
      ix->in_leaf[x] = ix->out_leaf[x] = !is_landmark[x] && m <= ix->leaf_threshold;
    } else {
      ix->in_leaf[x] = !is_landmark[x] && ix->pre[x].len == 0;
      ix->out_leaf[x] = !is_landmark[x] && ix->suc[x].len == 0;
    }
    ix->bucket[x] = (uint8_t)(bucket_table ? bucket_table[x] : orc_hash(x, kp));
    if (ix->bucket[x] >= kp) { free(is_landmark); return -1; }
  }
  free(is_landmark);
  memset(ix->dl_in, 0, 8 * (size_t)(n ? n : 1) * ix->wd);
  memset(ix->dl_out, 0, 8 * (size_t)(n ? n : 1) * ix->wd);
  memset(ix->bl_in, 0, 8 * (size_t)(n ? n : 1) * ix->wb);
  memset(ix->bl_out, 0, 8 * (size_t)(n ? n : 1) * ix->wb);

  /* task list: DL forward/backward per landmark, BL forward/backward per bucket */
  uint32_t ntasks = 2 * k + 2 * kp;
  orc_task *tasks = (orc_task *)calloc(ntasks ? ntasks : 1, sizeof(orc_task));
  uint32_t *src_in = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
  uint32_t *src_out = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
  uint32_t *cnt_in = (uint32_t *)calloc(kp + 1, sizeof(uint32_t));
  uint32_t *cnt_out = (uint32_t *)calloc(kp + 1, sizeof(uint32_t));
  if (!tasks || !src_in || !src_out || !cnt_in || !cnt_out) {
    free(tasks); free(src_in); free(src_out); free(cnt_in); free(cnt_out);
    return -1;
  }
  /* group leaves by bucket (counting sort) so each bucket's sources are contiguous */
  for (uint32_t x = 0; x < n; x++) {
    if (ix->in_leaf[x]) cnt_in[ix->bucket[x] + 1]++;
    if (ix->out_leaf[x]) cnt_out[ix->bucket[x] + 1]++;
  }
  for (uint32_t j = 0; j < kp; j++) { cnt_in[j + 1] += cnt_in[j]; cnt_out[j + 1] += cnt_out[j]; }
  {
    uint32_t *fi = (uint32_t *)malloc(sizeof(uint32_t) * (kp + 1));
    uint32_t *fo = (uint32_t *)malloc(sizeof(uint32_t) * (kp + 1));
    if (!fi || !fo) {
      free(fi); free(fo); free(tasks); free(src_in); free(src_out); free(cnt_in); free(cnt_out);
      return -1;
    }
    memcpy(fi, cnt_in, sizeof(uint32_t) * (kp + 1));
    memcpy(fo, cnt_out, sizeof(uint32_t) * (kp + 1));
    for (uint32_t x = 0; x < n; x++) {
      if (ix->in_leaf[x]) src_in[fi[ix->bucket[x]]++] = x;
      if (ix->out_leaf[x]) src_out[fo[ix->bucket[x]]++] = x;
    }
    free(fi); free(fo);
  }
  uint32_t t = 0;
  for (uint32_t i = 0; i < k; i++) {
    tasks[t++] = (orc_task){1, ix->dl_in, ix->wd, i, &ix->landmark[i], 1};
    tasks[t++] = (orc_task){0, ix->dl_out, ix->wd, i, &ix->landmark[i], 1};
  }
  for (uint32_t j = 0; j < kp; j++) {
    tasks[t++] = (orc_task){1, ix->bl_in, ix->wb, j, src_in + cnt_in[j],
                            cnt_in[j + 1] - cnt_in[j]};
    tasks[t++] = (orc_task){0, ix->bl_out, ix->wb, j, src_out + cnt_out[j],
                            cnt_out[j + 1] - cnt_out[j]};
  }
  orc_pool pool = {ix, tasks, ntasks, 0, threads > 1, 0};
  if (threads <= 1) {
    pool_worker(&pool);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    uint32_t started = 0;
    if (th)
      for (; started < threads; started++)
        if (pthread_create(&th[started], NULL, pool_worker, &pool)) break;
    if (started == 0) pool_worker(&pool);
    for (uint32_t i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
  }
  free(tasks); free(src_in); free(src_out); free(cnt_in); free(cnt_out);
  return pool.failed ? -1 : 0;
}

/* ---------------------------------------------------------------- queries (Algorithm 2) */

/* DL_Intersec(x, y) of Algorithm 2: DL_out(x) and DL_in(y) share a landmark. */
static int dl_intersec(const orc_index *ix, uint32_t x, uint32_t y) {
  const uint64_t *a = ix->dl_out + (size_t)x * ix->wd, *b = ix->dl_in + (size_t)y * ix->wd;
  for (uint32_t i = 0; i < ix->wd; i++)
    if (a[i] & b[i]) return 1;
  return 0;
}

/* BL_Contain(x, y) of Algorithm 2: BL_in(x) within BL_in(y) and BL_out(y) within BL_out(x). */
static int bl_contain(const orc_index *ix, uint32_t x, uint32_t y) {
  const size_t wb = ix->wb;
  for (uint32_t i = 0; i < wb; i++) {
    if (ix->bl_in[x * wb + i] & ~ix->bl_in[y * wb + i]) return 0;
    if (ix->bl_out[y * wb + i] & ~ix->bl_out[x * wb + i]) return 0;
  }
  return 1;
}

#define ORC_RULES_DL 1u
#define ORC_RULES_BL 2u

/* The label-only part of Algorithm 2; returns a class, or -1 if the labels cannot decide.
   rules: which labels may be used (reading R11). */
static int label_rules(const orc_index *ix, uint32_t u, uint32_t v, uint32_t rules) {
  const int dl = (rules & ORC_RULES_DL) != 0, bl = (rules & ORC_RULES_BL) != 0;
  if (u == v) return ORC_CLASS_SELF;
  if (dl && dl_intersec(ix, u, v)) return ORC_CLASS_R1_DL_HIT;
  if (bl && !bl_contain(ix, u, v)) return ORC_CLASS_R2_BL_MISS;
  if (dl && dl_intersec(ix, v, u)) return ORC_CLASS_R3_THM1;
  if (dl && (dl_intersec(ix, u, u) || dl_intersec(ix, v, v))) return ORC_CLASS_R4_THM2;
  return -1;
}

/* Algorithm 2's pruned BFS from u looking for v (reading R3: visited marks on enqueue). */
static int pruned_bfs(const orc_index *ix, orc_bfs_ws *w, uint32_t u, uint32_t v, uint32_t rules) {
  ws_next_stamp(w, ix->n);
  uint64_t head = 0, tail = 0;
  w->seen[u] = w->stamp;
  w->queue[tail++] = u;
  while (head < tail) {
    uint32_t p = w->queue[head++];
    const orc_list *s = &ix->suc[p];
    for (uint32_t j = 0; j < s->len; j++) {
      uint32_t x = s->v[j];
      if (x == v) return 1;
      if ((rules & ORC_RULES_DL) && dl_intersec(ix, u, x)) continue; /* a landmark of u reaches x */
      if ((rules & ORC_RULES_BL) && !bl_contain(ix, x, v)) continue; /* x cannot reach v */
      if (w->seen[x] == w->stamp) continue;
      w->seen[x] = w->stamp;
      w->queue[tail++] = x;
    }
  }
  return 0;
}

/* Plain BFS reachability with no labels at all (the truth the index must reproduce). */
static int plain_reach(const orc_index *ix, orc_bfs_ws *w, uint32_t u, uint32_t v) {
  if (u == v) return 1;
  ws_next_stamp(w, ix->n);
  uint64_t head = 0, tail = 0;
  w->seen[u] = w->stamp;
  w->queue[tail++] = u;
  while (head < tail) {
    uint32_t p = w->queue[head++];
    const orc_list *s = &ix->suc[p];
    for (uint32_t j = 0; j < s->len; j++) {
      uint32_t x = s->v[j];
      if (x == v) return 1;
      if (w->seen[x] == w->stamp) continue;
      w->seen[x] = w->stamp;
      w->queue[tail++] = x;
    }
  }
  return 0;
}

typedef struct {
  const orc_index *ix;
  const uint32_t *u, *v;
  uint8_t *out;
  uint64_t count;
  uint64_t next;
  int mode; /* 0 = Algorithm 2 (answer | class << 1), 1 = plain BFS truth (answer only) */
  uint32_t rules;
  int failed;
} orc_qpool;

#define ORC_QCHUNK 256

static void *query_worker(void *arg) {
  orc_qpool *p = (orc_qpool *)arg;
  orc_bfs_ws w;
  if (ws_init(&w, p->ix->n)) {
    __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
    ws_free(&w);
    return NULL;
  }
  for (;;) {
    uint64_t b = __atomic_fetch_add(&p->next, ORC_QCHUNK, __ATOMIC_RELAXED);
    if (b >= p->count) break;
    uint64_t e = b + ORC_QCHUNK < p->count ? b + ORC_QCHUNK : p->count;
    for (uint64_t i = b; i < e; i++) {
      uint32_t u = p->u[i], v = p->v[i];
      if (p->mode == 1) {
        p->out[i] = (uint8_t)plain_reach(p->ix, &w, u, v);
        continue;
      }
      int c = label_rules(p->ix, u, v, p->rules);
      int ans;
      if (c < 0) {
        ans = pruned_bfs(p->ix, &w, u, v, p->rules);
        c = ans ? ORC_CLASS_BFS_TRUE : ORC_CLASS_BFS_FALSE;
      } else {
        ans = (c == ORC_CLASS_SELF || c == ORC_CLASS_R1_DL_HIT);
      }
      p->out[i] = (uint8_t)(ans | (c << 1));
    }
  }
  ws_free(&w);
  return NULL;
}

static int run_queries(const orc_index *ix, uint64_t count, const uint32_t *u, const uint32_t *v,
                       uint8_t *out, int mode, uint32_t rules, uint32_t threads) {
  for (uint64_t i = 0; i < count; i++)
    if (u[i] >= ix->n || v[i] >= ix->n) return -1;
  orc_qpool pool = {ix, u, v, out, count, 0, mode, rules, 0};
  if (threads <= 1) {
    query_worker(&pool);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    uint32_t started = 0;
    if (th)
      for (; started < threads; started++)
        if (pthread_create(&th[started], NULL, query_worker, &pool)) break;
    if (started == 0) query_worker(&pool);
    for (uint32_t i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
  }
  return pool.failed ? -1 : 0;
}

/* Algorithm 2 per pair: out[i] = answer | (class << 1). */
int orc_query_dbl(const orc_index *ix, uint64_t count, const uint32_t *u, const uint32_t *v,
                  uint8_t *out, uint32_t threads) {
  return run_queries(ix, count, u, v, out, 0, ORC_RULES_DL | ORC_RULES_BL, threads);
}

/* Algorithm 2 with only some labels (reading R11): rules bit 0 = DL, bit 1 = BL. */
int orc_query_dbl_rules(const orc_index *ix, uint64_t count, const uint32_t *u, const uint32_t *v,
                        uint8_t *out, uint32_t rules, uint32_t threads) {
  return run_queries(ix, count, u, v, out, 0, rules, threads);
}

/* Plain BFS reachability per pair: out[i] = 1 if u reaches v (u reaches u). */
int orc_query_truth(const orc_index *ix, uint64_t count, const uint32_t *u, const uint32_t *v,
                    uint8_t *out, uint32_t threads) {
  return run_queries(ix, count, u, v, out, 1, 0, threads);
}

/* ---------------------------------------------------------------- insertion (Algorithm 3) */

/*
 * Algorithm 3 for one label: add `add` (the inserted edge's endpoint label, read before the
 * update) to every vertex of Des(start) (forward) or Anc(start) (backward), pruning a vertex as
 * soon as it already contains `add`. Reading R2: start itself is checked and updated first.
 */
static int misses(const uint64_t *add, const uint64_t *lab, uint32_t words) {
  for (uint32_t i = 0; i < words; i++)
    if (add[i] & ~lab[i]) return 1;
  return 0;
}

static void absorb(const uint64_t *add, uint64_t *lab, uint32_t words) {
  for (uint32_t i = 0; i < words; i++) lab[i] |= add[i];
}

static void alg3_propagate(const orc_index *ix, orc_bfs_ws *w, uint64_t *label, uint32_t words,
                           const uint64_t *add, uint32_t start, int forward) {
  const orc_list *adj = forward ? ix->suc : ix->pre;
  if (!misses(add, label + (size_t)start * words, words)) return;
  absorb(add, label + (size_t)start * words, words);
  uint64_t head = 0, tail = 0;
  w->queue[tail++] = start;
  while (head < tail) {
    uint32_t p = w->queue[head++];
    for (uint32_t j = 0; j < adj[p].len; j++) {
      uint32_t x = adj[p].v[j];
      if (misses(add, label + (size_t)x * words, words)) {
        absorb(add, label + (size_t)x * words, words);
        w->queue[tail++] = x; /* each vertex is enqueued at most once: it now contains `add` */
      }
    }
  }
}

/* Insert edges one at a time in the given order, each by Algorithm 3 on all four labels. */
int orc_insert(orc_index *ix, uint64_t count, const uint32_t *src, const uint32_t *dst) {
  for (uint64_t e = 0; e < count; e++)
    if (src[e] >= ix->n || dst[e] >= ix->n) return -1;
  orc_bfs_ws w;
  if (ws_init(&w, ix->n)) { ws_free(&w); return -1; }
  for (uint64_t e = 0; e < count; e++) {
    uint32_t u = src[e], v = dst[e];
    if (u == v) continue;                 /* reading R10 */
    if (list_has(&ix->suc[u], v)) continue; /* duplicate: reachability unchanged */
    if (list_push(&ix->suc[u], v) || list_push(&ix->pre[v], u)) { ws_free(&w); return -1; }
    if (dl_intersec(ix, u, v)) continue;  /* reading R9: u already reaches v (Lemma 1) */
    uint64_t dl_in_u[4], bl_in_u[4], dl_out_v[4], bl_out_v[4];
    memcpy(dl_in_u, ix->dl_in + (size_t)u * ix->wd, 8 * ix->wd);
    memcpy(bl_in_u, ix->bl_in + (size_t)u * ix->wb, 8 * ix->wb);
    memcpy(dl_out_v, ix->dl_out + (size_t)v * ix->wd, 8 * ix->wd);
    memcpy(bl_out_v, ix->bl_out + (size_t)v * ix->wb, 8 * ix->wb);
    alg3_propagate(ix, &w, ix->dl_in, ix->wd, dl_in_u, v, 1);
    alg3_propagate(ix, &w, ix->bl_in, ix->wb, bl_in_u, v, 1);
    alg3_propagate(ix, &w, ix->dl_out, ix->wd, dl_out_v, u, 0);
    alg3_propagate(ix, &w, ix->bl_out, ix->wb, bl_out_v, u, 0);
  }
  ws_free(&w);
  return 0;
}

/* Append `count` new vertices (reading R13); returns the first new id, or UINT32_MAX on
   allocation failure. */
uint32_t orc_add_vertices(orc_index *ix, uint32_t count) {
  const uint32_t n0 = ix->n, n1 = n0 + count;
  if (n1 < n0) return ORC_NONE;
  orc_list *suc = (orc_list *)realloc(ix->suc, sizeof(orc_list) * (size_t)n1);
  if (!suc) return ORC_NONE;
  ix->suc = suc;
  orc_list *pre = (orc_list *)realloc(ix->pre, sizeof(orc_list) * (size_t)n1);
  if (!pre) return ORC_NONE;
  ix->pre = pre;
  uint8_t **u8s[3] = {&ix->in_leaf, &ix->out_leaf, &ix->bucket};
  for (int i = 0; i < 3; i++) {
    uint8_t *p = (uint8_t *)realloc(*u8s[i], (size_t)n1);
    if (!p) return ORC_NONE;
    *u8s[i] = p;
  }
  uint64_t **labs[4] = {&ix->dl_in, &ix->dl_out, &ix->bl_in, &ix->bl_out};
  const uint32_t wds[4] = {ix->wd, ix->wd, ix->wb, ix->wb};
  for (int i = 0; i < 4; i++) {
    uint64_t *p = (uint64_t *)realloc(*labs[i], 8 * (size_t)n1 * wds[i]);
    if (!p) return ORC_NONE;
    memset(p + (size_t)n0 * wds[i], 0, 8 * (size_t)count * wds[i]);
    *labs[i] = p;
  }
  for (uint32_t x = n0; x < n1; x++) {
    memset(&ix->suc[x], 0, sizeof(orc_list));
    memset(&ix->pre[x], 0, sizeof(orc_list));
    ix->in_leaf[x] = ix->out_leaf[x] = 0;
    ix->bucket[x] = (uint8_t)orc_hash(x, ix->kp ? ix->kp : 1);
  }
  ix->n = n1;
  return n0;
}

/* ---------------------------------------------------------------- accessors */

void orc_label_words(const orc_index *ix, uint32_t *wd, uint32_t *wb) {
  *wd = ix->wd;
  *wb = ix->wb;
}

/* Copy the labels out: DL arrays hold n * wd words, BL arrays n * wb (vertex-major). */
void orc_read_labels(const orc_index *ix, uint64_t *dl_in, uint64_t *dl_out, uint64_t *bl_in,
                     uint64_t *bl_out) {
  const size_t bd = 8 * (size_t)ix->n * ix->wd, bb = 8 * (size_t)ix->n * ix->wb;
  memcpy(dl_in, ix->dl_in, bd);
  memcpy(dl_out, ix->dl_out, bd);
  memcpy(bl_in, ix->bl_in, bb);
  memcpy(bl_out, ix->bl_out, bb);
}

uint32_t orc_landmarks(const orc_index *ix, uint32_t *out) {
  memcpy(out, ix->landmark, sizeof(uint32_t) * ix->k);
  return ix->k;
}

void orc_leaves(const orc_index *ix, uint8_t *in_leaf, uint8_t *out_leaf, uint8_t *bucket) {
  memcpy(in_leaf, ix->in_leaf, ix->n);
  memcpy(out_leaf, ix->out_leaf, ix->n);
  memcpy(bucket, ix->bucket, ix->n);
}

uint64_t orc_num_edges(const orc_index *ix) {
  uint64_t m = 0;
  for (uint32_t x = 0; x < ix->n; x++) m += ix->suc[x].len;
  return m;
}

/* Bitset transitive closure for small n (Warshall): row u holds every v that u reaches. */
int orc_closure(const orc_index *ix, uint64_t *rows) {
  uint32_t n = ix->n, words = (n + 63) / 64;
  memset(rows, 0, 8 * (size_t)n * words);
  for (uint32_t u = 0; u < n; u++) {
    rows[(size_t)u * words + u / 64] |= 1ULL << (u % 64);
    for (uint32_t j = 0; j < ix->suc[u].len; j++) {
      uint32_t v = ix->suc[u].v[j];
      rows[(size_t)u * words + v / 64] |= 1ULL << (v % 64);
    }
  }
  for (uint32_t k = 0; k < n; k++)
    for (uint32_t i = 0; i < n; i++)
      if (rows[(size_t)i * words + k / 64] >> (k % 64) & 1)
        for (uint32_t w = 0; w < words; w++) rows[(size_t)i * words + w] |= rows[(size_t)k * words + w];
  return 0;
}

/* ---------------------------------------------------------------- large graphs (sampled checks) */
/*
 * For graphs too large for the per-vertex lists above: forward and reverse CSR built by a
 * counting sort (self-loops dropped; the edges are expected to be distinct), with
 *   - the landmark selection of Section 3.1 and the leaf rule (readings R5, R7, R8),
 *   - the reachable set of a source set (one BFS of Algorithm 1: the vertices whose label has
 *     the source set's bit),
 *   - plain BFS reachability per pair.
 * A label column of the full index can then be checked one bit at a time.
 */
typedef struct {
  uint32_t n;
  uint64_t *fo, *ro; /* [n + 1] */
  uint32_t *fc, *rc;
} orc_big;

void orc_big_free(orc_big *g) {
  if (!g) return;
  free(g->fo); free(g->ro); free(g->fc); free(g->rc);
  free(g);
}

orc_big *orc_big_new(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst) {
  orc_big *g = (orc_big *)calloc(1, sizeof(orc_big));
  if (!g) return NULL;
  g->n = n;
  g->fo = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  g->ro = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  if (!g->fo || !g->ro) { orc_big_free(g); return NULL; }
  uint64_t kept = 0;
  for (uint64_t e = 0; e < m; e++) {
    if (src[e] >= n || dst[e] >= n) { orc_big_free(g); return NULL; }
    if (src[e] == dst[e]) continue;
    g->fo[src[e] + 1]++;
    g->ro[dst[e] + 1]++;
    kept++;
  }
  for (uint32_t x = 0; x < n; x++) { g->fo[x + 1] += g->fo[x]; g->ro[x + 1] += g->ro[x]; }
  g->fc = (uint32_t *)malloc(sizeof(uint32_t) * (kept ? kept : 1));
  g->rc = (uint32_t *)malloc(sizeof(uint32_t) * (kept ? kept : 1));
  uint64_t *ff = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  uint64_t *rf = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  if (!g->fc || !g->rc || !ff || !rf) { free(ff); free(rf); orc_big_free(g); return NULL; }
  memcpy(ff, g->fo, sizeof(uint64_t) * ((size_t)n + 1));
  memcpy(rf, g->ro, sizeof(uint64_t) * ((size_t)n + 1));
  for (uint64_t e = 0; e < m; e++) {
    if (src[e] == dst[e]) continue;
    g->fc[ff[src[e]]++] = dst[e];
    g->rc[rf[dst[e]]++] = src[e];
  }
  free(ff); free(rf);
  return g;
}

/* top-k by |Pre|*|Suc| (ties by smaller id), as orc_select_landmarks */
uint32_t orc_big_landmarks(const orc_big *g, uint32_t k, uint32_t *out) {
  uint32_t have = 0;
  for (uint32_t x = 0; x < g->n; x++) {
    const uint64_t mx = (g->ro[x + 1] - g->ro[x]) * (g->fo[x + 1] - g->fo[x]);
    uint32_t p;
    if (have < k) {
      p = have++;
    } else if (k > 0) {
      const uint32_t y = out[k - 1];
      const uint64_t my = (g->ro[y + 1] - g->ro[y]) * (g->fo[y + 1] - g->fo[y]);
      if (!(mx > my || (mx == my && x < y))) continue;
      p = k - 1;
    } else {
      continue;
    }
    while (p > 0) {
      const uint32_t y = out[p - 1];
      const uint64_t my = (g->ro[y + 1] - g->ro[y]) * (g->fo[y + 1] - g->fo[y]);
      if (!(mx > my || (mx == my && x < y))) break;
      out[p] = out[p - 1];
      p--;
    }
    out[p] = x;
  }
  return have;
}

/* in-degree and out-degree per vertex */
void orc_big_degrees(const orc_big *g, uint32_t *indeg, uint32_t *outdeg) {
  for (uint32_t x = 0; x < g->n; x++) {
    indeg[x] = (uint32_t)(g->ro[x + 1] - g->ro[x]);
    outdeg[x] = (uint32_t)(g->fo[x + 1] - g->fo[x]);
  }
}

/* Reachable set (bitmap, n bits) of a source set, forward over Suc or backward over Pre;
   sources included. Returns the number of vertices reached, or -1 on allocation failure. */
int64_t orc_big_reach(const orc_big *g, uint64_t ns, const uint32_t *sources, int forward,
                      uint64_t *bitmap) {
  const uint64_t *off = forward ? g->fo : g->ro;
  const uint32_t *col = forward ? g->fc : g->rc;
  uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->n ? g->n : 1));
  if (!queue) return -1;
  memset(bitmap, 0, 8 * (size_t)((g->n + 63) / 64));
  uint64_t head = 0, tail = 0;
  for (uint64_t i = 0; i < ns; i++) {
    const uint32_t s = sources[i];
    if (bitmap[s >> 6] >> (s & 63) & 1) continue;
    bitmap[s >> 6] |= 1ULL << (s & 63);
    queue[tail++] = s;
  }
  while (head < tail) {
    const uint32_t p = queue[head++];
    for (uint64_t j = off[p]; j < off[p + 1]; j++) {
      const uint32_t x = col[j];
      if (bitmap[x >> 6] >> (x & 63) & 1) continue;
      bitmap[x >> 6] |= 1ULL << (x & 63);
      queue[tail++] = x;
    }
  }
  free(queue);
  return (int64_t)tail;
}

typedef struct {
  const orc_big *g;
  const uint32_t *u, *v;
  uint8_t *out;
  uint64_t count, next;
  int failed;
} orc_big_qpool;

static void *big_query_worker(void *arg) {
  orc_big_qpool *p = (orc_big_qpool *)arg;
  const orc_big *g = p->g;
  uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->n ? g->n : 1));
  uint64_t *seen = (uint64_t *)calloc((g->n + 63) / 64 + 1, sizeof(uint64_t));
  if (!queue || !seen) {
    __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
    free(queue); free(seen);
    return NULL;
  }
  for (;;) {
    const uint64_t i = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
    if (i >= p->count) break;
    const uint32_t u = p->u[i], v = p->v[i];
    int found = u == v;
    uint64_t head = 0, tail = 0;
    if (!found) {
      seen[u >> 6] |= 1ULL << (u & 63);
      queue[tail++] = u;
    }
    while (!found && head < tail) {
      const uint32_t w = queue[head++];
      for (uint64_t j = g->fo[w]; j < g->fo[w + 1]; j++) {
        const uint32_t x = g->fc[j];
        if (x == v) { found = 1; break; }
        if (seen[x >> 6] >> (x & 63) & 1) continue;
        seen[x >> 6] |= 1ULL << (x & 63);
        queue[tail++] = x;
      }
    }
    for (uint64_t j = 0; j < tail; j++) seen[queue[j] >> 6] = 0;
    p->out[i] = (uint8_t)found;
  }
  free(queue);
  free(seen);
  return NULL;
}

/* Plain BFS reachability per pair (u reaches u), on `threads` threads. */
int orc_big_query_truth(const orc_big *g, uint64_t count, const uint32_t *u, const uint32_t *v,
                        uint8_t *out, uint32_t threads) {
  for (uint64_t i = 0; i < count; i++)
    if (u[i] >= g->n || v[i] >= g->n) return -1;
  orc_big_qpool pool = {g, u, v, out, count, 0, 0};
  if (threads <= 1) {
    big_query_worker(&pool);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    uint32_t started = 0;
    if (th)
      for (; started < threads; started++)
        if (pthread_create(&th[started], NULL, big_query_worker, &pool)) break;
    if (started == 0) big_query_worker(&pool);
    for (uint32_t i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
  }
  return pool.failed ? -1 : 0;
}

/*
 * All four labels of the large graph at k, k' <= 64 (one 64-bit word per label), straight from
 * Definitions 1 and 2: bit i of DL_in(x) is set when x is in the reachable set of landmark
 * landmarks[i] (forward), bit i of DL_out(x) when x reaches it (backward); bit j of BL_in(x) when
 * x is reachable from some vertex of S_in hashed to j (forward from that source set), bit j of
 * BL_out(x) when x reaches some vertex of S_out hashed to j (backward). Every bit column is one
 * orc_big_reach of its source set (Algorithm 1 with the visited set of reading R1); the columns
 * are spread over `threads` threads and OR-ed into the labels atomically (different bits of one
 * word belong to different columns). s_in / s_out: uint8[n] masks; bucket: uint8[n], h(x) < kp.
 * kinds: which labels to compute (bit 0 DL_in, 1 DL_out, 2 BL_in, 3 BL_out); each of those is
 * zeroed first, the others are left as they are. Returns 0, or -1 on bad sizes or allocation
 * failure.
 */
typedef struct {
  const orc_big *g;
  uint32_t k, kp;
  const uint32_t *landmarks;
  const uint8_t *s_in, *s_out, *bucket;
  uint64_t *lab[4]; /* DL_in, DL_out, BL_in, BL_out */
  uint32_t kinds;   /* labels to compute (bit i = lab[i]) */
  uint32_t next;    /* shared column counter: column c is (label c / 64, bit c % 64) */
  int failed;
} orc_big_colpool;

static void *big_column_worker(void *arg) {
  orc_big_colpool *p = (orc_big_colpool *)arg;
  const orc_big *g = p->g;
  const size_t words = (size_t)(g->n + 63) / 64;
  uint64_t *bm = (uint64_t *)malloc(8 * (words ? words : 1));
  uint32_t *src = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->n ? g->n : 1));
  if (!bm || !src) {
    __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
    free(bm); free(src);
    return NULL;
  }
  for (;;) {
    const uint32_t c = __atomic_fetch_add(&p->next, 1, __ATOMIC_RELAXED);
    if (c >= 4 * 64) break;
    const uint32_t which = c / 64, bit = c % 64;
    uint64_t ns = 0;
    if (!(p->kinds >> which & 1)) continue;
    if (which < 2) {
      if (bit >= p->k) continue;
      src[ns++] = p->landmarks[bit];
    } else {
      if (bit >= p->kp) continue;
      const uint8_t *leaf = which == 2 ? p->s_in : p->s_out;
      for (uint32_t x = 0; x < g->n; x++)
        if (leaf[x] && p->bucket[x] == bit) src[ns++] = x;
    }
    const int forward = which == 0 || which == 2;
    if (orc_big_reach(g, ns, src, forward, bm) < 0) {
      __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
      break;
    }
    uint64_t *lab = p->lab[which];
    const uint64_t mask = 1ULL << bit;
    for (size_t w = 0; w < words; w++)
      for (uint64_t b = bm[w]; b; b &= b - 1)
        __atomic_fetch_or(&lab[w * 64 + (uint64_t)__builtin_ctzll(b)], mask, __ATOMIC_RELAXED);
  }
  free(bm);
  free(src);
  return NULL;
}

int orc_big_labels(const orc_big *g, uint32_t k, const uint32_t *landmarks, uint32_t kp,
                   const uint8_t *s_in, const uint8_t *s_out, const uint8_t *bucket,
                   uint32_t kinds, uint32_t threads, uint64_t *dl_in, uint64_t *dl_out,
                   uint64_t *bl_in, uint64_t *bl_out) {
  if (k > 64 || kp == 0 || kp > 64 || (kp & (kp - 1))) return -1;
  for (uint32_t i = 0; i < k; i++)
    if (landmarks[i] >= g->n) return -1;
  for (uint32_t x = 0; x < g->n; x++)
    if (bucket[x] >= kp) return -1;
  uint64_t *labs[4] = {dl_in, dl_out, bl_in, bl_out};
  for (int i = 0; i < 4; i++)
    if (kinds >> i & 1) memset(labs[i], 0, 8 * (size_t)g->n);
  orc_big_colpool pool = {g, k, kp, landmarks, s_in, s_out, bucket,
                          {dl_in, dl_out, bl_in, bl_out}, kinds & 15u, 0, 0};
  if (threads <= 1) {
    big_column_worker(&pool);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    uint32_t started = 0;
    if (th)
      for (; started < threads; started++)
        if (pthread_create(&th[started], NULL, big_column_worker, &pool)) break;
    if (started == 0) big_column_worker(&pool);
    for (uint32_t i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
  }
  return pool.failed ? -1 : 0;
}

/*
 * Algorithm 2 on the large graph with given labels (one word each, e.g. from orc_big_labels):
 * self, then Lemma 1, Lemma 2, Theorem 1, Theorem 2 on the labels, else the pruned BFS from u
 * over Suc (prune x when DL_out(u) and DL_in(x) share a landmark, or when BL_Contain(x, v)
 * fails; visited marks on enqueue, reading R3). out[i] = answer | (class << 1), the class codes
 * of orc_query_dbl.
 */
typedef struct {
  const orc_big *g;
  const uint64_t *dl_in, *dl_out, *bl_in, *bl_out;
  const uint32_t *u, *v;
  uint8_t *out;
  uint64_t count, next;
  int mode; /* 0: Algorithm 2; 1: bidirectional plain BFS (answer only) */
  int failed;
} orc_big_apool;

static int big_label_rules(const orc_big_apool *p, uint32_t u, uint32_t v) {
  if (u == v) return ORC_CLASS_SELF;
  if (p->dl_out[u] & p->dl_in[v]) return ORC_CLASS_R1_DL_HIT;
  if ((p->bl_in[u] & ~p->bl_in[v]) || (p->bl_out[v] & ~p->bl_out[u])) return ORC_CLASS_R2_BL_MISS;
  if (p->dl_out[v] & p->dl_in[u]) return ORC_CLASS_R3_THM1;
  if ((p->dl_out[u] & p->dl_in[u]) || (p->dl_out[v] & p->dl_in[v])) return ORC_CLASS_R4_THM2;
  return -1;
}

static int big_pruned_bfs(const orc_big_apool *p, uint32_t *queue, uint64_t *seen, uint32_t u,
                          uint32_t v) {
  const orc_big *g = p->g;
  uint64_t head = 0, tail = 0;
  int found = 0;
  seen[u >> 6] |= 1ULL << (u & 63);
  queue[tail++] = u;
  while (!found && head < tail) {
    const uint32_t w = queue[head++];
    for (uint64_t j = g->fo[w]; j < g->fo[w + 1]; j++) {
      const uint32_t x = g->fc[j];
      if (x == v) { found = 1; break; }
      if (p->dl_out[u] & p->dl_in[x]) continue;                      /* a landmark of u reaches x */
      if ((p->bl_in[x] & ~p->bl_in[v]) || (p->bl_out[v] & ~p->bl_out[x])) continue; /* x misses v */
      if (seen[x >> 6] >> (x & 63) & 1) continue;
      seen[x >> 6] |= 1ULL << (x & 63);
      queue[tail++] = x;
    }
  }
  for (uint64_t j = 0; j < tail; j++) seen[queue[j] >> 6] = 0;
  return found;
}

/*
 * Textbook bidirectional BFS with no labels: a forward search from u over Suc and a backward
 * search from v over Pre, each step expanding one whole level of the side whose frontier has
 * fewer vertices; u reaches v exactly when the two visited sets meet, and not when either
 * search runs out first.
 */
static int big_bibfs(const orc_big *g, uint32_t *qf, uint32_t *qb, uint64_t *sf, uint64_t *sb,
                     uint32_t u, uint32_t v) {
  if (u == v) return 1;
  uint64_t fh = 0, ft = 0, bh = 0, bt = 0;
  int met = 0;
  sf[u >> 6] |= 1ULL << (u & 63);
  qf[ft++] = u;
  sb[v >> 6] |= 1ULL << (v & 63);
  qb[bt++] = v;
  while (!met && fh < ft && bh < bt) {
    const int fwd = (ft - fh) <= (bt - bh);
    const uint64_t *off = fwd ? g->fo : g->ro;
    const uint32_t *col = fwd ? g->fc : g->rc;
    uint32_t *q = fwd ? qf : qb;
    uint64_t *mine = fwd ? sf : sb, *other = fwd ? sb : sf;
    uint64_t *head = fwd ? &fh : &bh, *tail = fwd ? &ft : &bt;
    const uint64_t level_end = *tail;
    while (!met && *head < level_end) {
      const uint32_t w = q[(*head)++];
      for (uint64_t j = off[w]; j < off[w + 1]; j++) {
        const uint32_t x = col[j];
        if (other[x >> 6] >> (x & 63) & 1) { met = 1; break; }
        if (mine[x >> 6] >> (x & 63) & 1) continue;
        mine[x >> 6] |= 1ULL << (x & 63);
        q[(*tail)++] = x;
      }
    }
  }
  for (uint64_t j = 0; j < ft; j++) sf[qf[j] >> 6] = 0;
  for (uint64_t j = 0; j < bt; j++) sb[qb[j] >> 6] = 0;
  return met;
}

static void *big_answer_worker(void *arg) {
  orc_big_apool *p = (orc_big_apool *)arg;
  const orc_big *g = p->g;
  const size_t nn = g->n ? g->n : 1, words = (size_t)(g->n + 63) / 64 + 1;
  uint32_t *qa = (uint32_t *)malloc(sizeof(uint32_t) * nn);
  uint32_t *qb = (uint32_t *)malloc(sizeof(uint32_t) * nn);
  uint64_t *sa = (uint64_t *)calloc(words, sizeof(uint64_t));
  uint64_t *sb = (uint64_t *)calloc(words, sizeof(uint64_t));
  if (!qa || !qb || !sa || !sb) {
    __atomic_store_n(&p->failed, 1, __ATOMIC_RELAXED);
    free(qa); free(qb); free(sa); free(sb);
    return NULL;
  }
  for (;;) {
    const uint64_t b = __atomic_fetch_add(&p->next, ORC_QCHUNK, __ATOMIC_RELAXED);
    if (b >= p->count) break;
    const uint64_t e = b + ORC_QCHUNK < p->count ? b + ORC_QCHUNK : p->count;
    for (uint64_t i = b; i < e; i++) {
      const uint32_t u = p->u[i], v = p->v[i];
      if (p->mode == 1) {
        p->out[i] = (uint8_t)big_bibfs(g, qa, qb, sa, sb, u, v);
        continue;
      }
      int c = big_label_rules(p, u, v), ans;
      if (c < 0) {
        ans = big_pruned_bfs(p, qa, sa, u, v);
        c = ans ? ORC_CLASS_BFS_TRUE : ORC_CLASS_BFS_FALSE;
      } else {
        ans = (c == ORC_CLASS_SELF || c == ORC_CLASS_R1_DL_HIT);
      }
      p->out[i] = (uint8_t)(ans | (c << 1));
    }
  }
  free(qa); free(qb); free(sa); free(sb);
  return NULL;
}

static int big_answers(orc_big_apool *pool, uint32_t threads) {
  for (uint64_t i = 0; i < pool->count; i++)
    if (pool->u[i] >= pool->g->n || pool->v[i] >= pool->g->n) return -1;
  if (threads <= 1) {
    big_answer_worker(pool);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    uint32_t started = 0;
    if (th)
      for (; started < threads; started++)
        if (pthread_create(&th[started], NULL, big_answer_worker, pool)) break;
    if (started == 0) big_answer_worker(pool);
    for (uint32_t i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
  }
  return pool->failed ? -1 : 0;
}

int orc_big_query_dbl(const orc_big *g, const uint64_t *dl_in, const uint64_t *dl_out,
                      const uint64_t *bl_in, const uint64_t *bl_out, uint64_t count,
                      const uint32_t *u, const uint32_t *v, uint8_t *out, uint32_t threads) {
  orc_big_apool pool = {g, dl_in, dl_out, bl_in, bl_out, u, v, out, count, 0, 0, 0};
  return big_answers(&pool, threads);
}

/* Reachability per pair by bidirectional BFS (no labels): out[i] = 1 if u reaches v. */
int orc_big_query_bibfs(const orc_big *g, uint64_t count, const uint32_t *u, const uint32_t *v,
                        uint8_t *out, uint32_t threads) {
  orc_big_apool pool = {g, NULL, NULL, NULL, NULL, u, v, out, count, 0, 1, 0};
  return big_answers(&pool, threads);
}
