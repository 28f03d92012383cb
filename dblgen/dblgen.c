/*
 * dblgen: seeded synthetic inputs for the DBL reachability index.
 *
 * This module produces graphs, insertion streams and query streams. It holds none of the
 * index's arithmetic (no labels, no landmark selection, no reachability): it is input only,
 * and both the CPU oracle and the GPU path read what it writes.
 *
 * Random numbers: xoshiro256** (Blackman & Vigna, "Scrambled linear pseudorandom number
 * generators", 2018), seeded by expanding the user seed with splitmix64 (Steele, Lea & Flood,
 * 2014). A uniform double takes the top 53 bits of one 64-bit output.
 *
 * Graphs: R-MAT (Chakrabarti, Zhan & Faloutsos, 2004). Each edge descends `scale` levels, most
 * significant bit first; at each level one uniform double picks a quadrant with probabilities
 * a, b, c, d = 1-a-b-c. Quadrant b sets the destination bit, c the source bit, d both. The edge
 * set is the first unique, non-self-loop edges of the draw stream, in stream order. Vertex ids
 * are then relabelled by a seeded Fisher-Yates shuffle so that ids carry no degree information.
 * The same stream continues after the build edges to give insertion edges (loops and edges
 * already present are skipped), so insertions have the same power-law shape as the graph.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- RNG */
typedef struct { uint64_t s[4]; } xoshiro256;

static uint64_t splitmix64_next(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xoshiro256 *r, uint64_t seed) {
  uint64_t x = seed;
  for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&x);
}

static uint64_t xo_next(xoshiro256 *r) {
  uint64_t *s = r->s;
  const uint64_t result = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return result;
}

static double xo_double(xoshiro256 *r) { return (double)(xo_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, bound), bound >= 1, by rejection (no modulo bias) */
static uint64_t xo_below(xoshiro256 *r, uint64_t bound) {
  uint64_t limit = UINT64_MAX - (UINT64_MAX % bound);
  uint64_t x;
  do { x = xo_next(r); } while (x >= limit);
  return x % bound;
}

/* ---------------------------------------------------------------- edge set (hash set of keys) */
typedef struct {
  uint64_t *slot; /* key+1, 0 = empty */
  uint64_t mask;
  uint64_t count;
} edge_set;

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* zeroed table, touched up front (pages are faulted in once, in order, not at random) */
static uint64_t *table_alloc(uint64_t cap) {
  uint64_t *p = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
  if (p) memset(p, 0, (size_t)cap * sizeof(uint64_t));
  return p;
}

static int set_init(edge_set *s, uint64_t expected) {
  uint64_t cap = 1024;
  while (cap < expected + expected / 3 + 16) cap <<= 1; /* load factor at most 3/4 */
  s->slot = table_alloc(cap);
  s->mask = cap - 1;
  s->count = 0;
  return s->slot ? 0 : -1;
}

static int set_grow(edge_set *s) {
  uint64_t old_cap = s->mask + 1, cap = old_cap * 2;
  uint64_t *ns = table_alloc(cap);
  if (!ns) return -1;
  for (uint64_t i = 0; i < old_cap; i++) {
    uint64_t k = s->slot[i];
    if (!k) continue;
    uint64_t h = mix64(k) & (cap - 1);
    while (ns[h]) h = (h + 1) & (cap - 1);
    ns[h] = k;
  }
  free(s->slot);
  s->slot = ns;
  s->mask = cap - 1;
  return 0;
}

/* returns 1 if inserted (new), 0 if present, -1 on allocation failure */
static int set_insert(edge_set *s, uint64_t key) {
  if (4 * (s->count + 1) > 3 * (s->mask + 1) && set_grow(s)) return -1;
  uint64_t k = key + 1;
  uint64_t h = mix64(k) & s->mask;
  while (s->slot[h]) {
    if (s->slot[h] == k) return 0;
    h = (h + 1) & s->mask;
  }
  s->slot[h] = k;
  s->count++;
  return 1;
}

static int set_contains(const edge_set *s, uint64_t key) {
  uint64_t k = key + 1;
  uint64_t h = mix64(k) & s->mask;
  while (s->slot[h]) {
    if (s->slot[h] == k) return 1;
    h = (h + 1) & s->mask;
  }
  return 0;
}

/* ---------------------------------------------------------------- R-MAT stream */
typedef struct {
  uint32_t scale, n;
  double a, b, c;
  xoshiro256 rng;
  xoshiro256 rng_mark; /* generator state at the start of the current batch of draws */
  uint32_t *perm; /* raw id -> output id */
  edge_set set;   /* keys over output ids: (src << 32) | dst */
  uint64_t draws;
} dblgen_rmat;

dblgen_rmat *dblgen_rmat_new(uint32_t scale, uint64_t seed, double a, double b, double c,
                             uint64_t expected_edges) {
  if (scale == 0 || scale > 31) return NULL;
  dblgen_rmat *g = (dblgen_rmat *)calloc(1, sizeof(dblgen_rmat));
  if (!g) return NULL;
  g->scale = scale;
  g->n = 1u << scale;
  g->a = a; g->b = b; g->c = c;
  xo_seed(&g->rng, seed);
  g->rng_mark = g->rng;
  g->perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)g->n);
  if (!g->perm || set_init(&g->set, expected_edges)) {
    free(g->perm); free(g->set.slot); free(g);
    return NULL;
  }
  /* Fisher-Yates relabelling, seeded with seed + 1 */
  xoshiro256 pr;
  xo_seed(&pr, seed + 1);
  for (uint32_t i = 0; i < g->n; i++) g->perm[i] = i;
  for (uint32_t i = g->n - 1; i > 0; i--) {
    uint32_t j = (uint32_t)xo_below(&pr, (uint64_t)i + 1);
    uint32_t t = g->perm[i]; g->perm[i] = g->perm[j]; g->perm[j] = t;
  }
  return g;
}

void dblgen_rmat_free(dblgen_rmat *g) {
  if (!g) return;
  free(g->perm);
  free(g->set.slot);
  free(g);
}

uint32_t dblgen_rmat_n(const dblgen_rmat *g) { return g->n; }
uint64_t dblgen_rmat_draws(const dblgen_rmat *g) { return g->draws; }
uint64_t dblgen_rmat_count(const dblgen_rmat *g) { return g->set.count; }

static void rmat_draw_raw(dblgen_rmat *g, uint32_t *src, uint32_t *dst) {
  uint32_t s = 0, d = 0;
  const double ab = g->a + g->b, abc = g->a + g->b + g->c;
  for (int lvl = (int)g->scale - 1; lvl >= 0; lvl--) {
    double r = xo_double(&g->rng);
    if (r < g->a) {
    } else if (r < ab) {
      d |= 1u << lvl;
    } else if (r < abc) {
      s |= 1u << lvl;
    } else {
      s |= 1u << lvl;
      d |= 1u << lvl;
    }
  }
  *src = s; *dst = d;
}

/*
 * Draw from the stream until `max_unique` new edges were produced or `max_draws` draws were
 * made (0 = no draw limit). Self-loops and edges already produced are skipped. Returns the
 * number of edges written, or -1 on allocation failure.
 */
int64_t dblgen_rmat_next(dblgen_rmat *g, uint64_t max_unique, uint64_t max_draws, uint32_t *src,
                         uint32_t *dst) {
  /* Draws are made in small batches so that the hash-set slots of a batch can be prefetched
     before the keys are inserted one by one, in stream order. */
  enum { B = 64 };
  uint64_t got = 0, drawn = 0;
  uint64_t key[B];
  while (got < max_unique && (max_draws == 0 || drawn < max_draws)) {
    uint64_t nb = B;
    if (max_draws && max_draws - drawn < nb) nb = max_draws - drawn;
    for (uint64_t i = 0; i < nb; i++) {
      uint32_t s, d;
      rmat_draw_raw(g, &s, &d);
      key[i] = s == d ? UINT64_MAX : (((uint64_t)g->perm[s] << 32) | g->perm[d]);
      if (key[i] != UINT64_MAX) __builtin_prefetch(&g->set.slot[mix64(key[i] + 1) & g->set.mask]);
    }
    uint64_t i = 0;
    for (; i < nb && got < max_unique; i++) {
      if (key[i] == UINT64_MAX) continue;
      int r = set_insert(&g->set, key[i]);
      if (r < 0) return -1;
      if (r == 0) continue;
      src[got] = (uint32_t)(key[i] >> 32);
      dst[got] = (uint32_t)key[i];
      got++;
    }
    drawn += i;
    if (i < nb) {
      /* the unique target was reached inside the batch: rewind the stream so that the draws
         after the last one consumed are drawn again by the next call */
      g->rng = g->rng_mark;
      g->draws += drawn;
      for (uint64_t j = 0; j < i; j++) { uint32_t s, d; rmat_draw_raw(g, &s, &d); }
      g->rng_mark = g->rng;
      return (int64_t)got;
    }
    g->rng_mark = g->rng;
  }
  g->draws += drawn;
  return (int64_t)got;
}

/* Uniform new edges (u != v, not already in the stream's edge set), added to the set. */
int64_t dblgen_rmat_uniform_new(dblgen_rmat *g, uint64_t seed, uint64_t count, uint32_t *src,
                                uint32_t *dst) {
  xoshiro256 r;
  xo_seed(&r, seed);
  uint64_t got = 0;
  while (got < count) {
    uint32_t u = (uint32_t)xo_below(&r, g->n), v = (uint32_t)xo_below(&r, g->n);
    if (u == v) continue;
    int ins = set_insert(&g->set, ((uint64_t)u << 32) | v);
    if (ins < 0) return -1;
    if (ins == 0) continue;
    src[got] = u; dst[got] = v;
    got++;
  }
  return (int64_t)got;
}

int dblgen_rmat_contains(const dblgen_rmat *g, uint32_t u, uint32_t v) {
  return set_contains(&g->set, ((uint64_t)u << 32) | v);
}

/* ---------------------------------------------------------------- query streams */

/* count uniform pairs over [0, n); u == v is allowed */
void dblgen_queries_uniform(uint32_t n, uint64_t seed, uint64_t count, uint32_t *u, uint32_t *v) {
  xoshiro256 r;
  xo_seed(&r, seed);
  for (uint64_t i = 0; i < count; i++) {
    u[i] = (uint32_t)xo_below(&r, n);
    v[i] = (uint32_t)xo_below(&r, n);
  }
}

/*
 * Mixed pairs: with probability p_walk, v is the end of a forward random walk of uniform length
 * in [1, max_len] started at u (u is redrawn until it has an out-edge; the walk stops early at a
 * vertex with no out-edge), so the pair is reachable by construction; otherwise v is uniform.
 * The walk runs over the given edge list. Returns 0, or -1 on allocation failure.
 */
int dblgen_queries_mixed(uint32_t n, uint64_t m, const uint32_t *esrc, const uint32_t *edst,
                         uint64_t seed, uint64_t count, double p_walk, uint32_t max_len, uint32_t *u,
                         uint32_t *v) {
  uint64_t *start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  uint32_t *adj = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
  uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  if (!start || !adj || !fill) { free(start); free(adj); free(fill); return -1; }
  for (uint64_t e = 0; e < m; e++) start[esrc[e] + 1]++;
  for (uint32_t x = 0; x < n; x++) start[x + 1] += start[x];
  memcpy(fill, start, sizeof(uint64_t) * ((size_t)n + 1));
  for (uint64_t e = 0; e < m; e++) adj[fill[esrc[e]]++] = edst[e];
  free(fill);
  int any_out = 0;
  for (uint32_t x = 0; x < n && !any_out; x++) any_out = start[x + 1] > start[x];
  xoshiro256 r;
  xo_seed(&r, seed);
  for (uint64_t i = 0; i < count; i++) {
    if (any_out && xo_double(&r) < p_walk) {
      uint32_t a;
      do { a = (uint32_t)xo_below(&r, n); } while (start[a + 1] == start[a]);
      uint32_t len = 1 + (uint32_t)xo_below(&r, max_len), x = a;
      for (uint32_t s = 0; s < len; s++) {
        uint64_t deg = start[x + 1] - start[x];
        if (deg == 0) break;
        x = adj[start[x] + xo_below(&r, deg)];
      }
      u[i] = a; v[i] = x;
    } else {
      u[i] = (uint32_t)xo_below(&r, n);
      v[i] = (uint32_t)xo_below(&r, n);
    }
  }
  free(start);
  free(adj);
  return 0;
}

/*
 * Zipf-skewed sources: rank r in [1, n] has probability proportional to r^-s; ranks map to
 * vertices through a seeded random permutation. Destinations are uniform. Sampling inverts the
 * cumulative distribution by binary search over a table of n doubles.
 */
int dblgen_queries_zipf(uint32_t n, uint64_t seed, uint64_t count, double s, uint32_t *u,
                        uint32_t *v) {
  double *cdf = (double *)malloc(sizeof(double) * (size_t)n);
  uint32_t *rank_to_v = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  if (!cdf || !rank_to_v) { free(cdf); free(rank_to_v); return -1; }
  double acc = 0.0;
  for (uint32_t r = 0; r < n; r++) {
    double w = exp(-s * log((double)(r + 1)));
    acc += w;
    cdf[r] = acc;
  }
  xoshiro256 pr;
  xo_seed(&pr, seed + 7);
  for (uint32_t i = 0; i < n; i++) rank_to_v[i] = i;
  for (uint32_t i = n - 1; i > 0; i--) {
    uint32_t j = (uint32_t)xo_below(&pr, (uint64_t)i + 1);
    uint32_t t = rank_to_v[i]; rank_to_v[i] = rank_to_v[j]; rank_to_v[j] = t;
  }
  xoshiro256 r;
  xo_seed(&r, seed);
  for (uint64_t i = 0; i < count; i++) {
    double x = xo_double(&r) * acc;
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      uint32_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    u[i] = rank_to_v[lo];
    v[i] = (uint32_t)xo_below(&r, n);
  }
  free(cdf);
  free(rank_to_v);
  return 0;
}

/* raw access to the generator for tests of its published definition */
void dblgen_xoshiro_outputs(uint64_t seed, uint64_t count, uint64_t *out) {
  xoshiro256 r;
  xo_seed(&r, seed);
  for (uint64_t i = 0; i < count; i++) out[i] = xo_next(&r);
}

/* ---------------------------------------------------------------- large graphs, in parallel */
/*
 * The large workload uses a chunked stream so that draws can be made by several threads:
 * chunk c (c = 0, 1, ...) holds `chunk` consecutive draws from its own xoshiro256** state,
 * seeded with seed + 0x9E3779B97F4A7C15 * (c + 1) through splitmix64. The edge set is the set of
 * distinct non-loop edges among the first `draws` draws (after the same Fisher-Yates relabelling
 * as above), returned sorted by (src, dst). Insertion edges continue with the chunks after
 * `draws`, skipping loops, edges of the set and repeats.
 */
#include <pthread.h>

typedef struct {
  uint32_t scale;
  double a, b, c;
  const uint32_t *perm;
  uint64_t seed, chunk, draws;
  uint64_t *keys; /* [draws] */
  uint32_t nthreads, tid;
} par_draw_job;

static void draw_chunk_keys(const par_draw_job *j, uint64_t c, uint64_t *out, uint64_t count) {
  xoshiro256 r;
  xo_seed(&r, j->seed + 0x9E3779B97F4A7C15ULL * (c + 1));
  dblgen_rmat g;
  memset(&g, 0, sizeof(g));
  g.scale = j->scale;
  g.a = j->a; g.b = j->b; g.c = j->c;
  g.rng = r;
  for (uint64_t i = 0; i < count; i++) {
    uint32_t s, d;
    rmat_draw_raw(&g, &s, &d);
    out[i] = s == d ? UINT64_MAX : (((uint64_t)j->perm[s] << 32) | j->perm[d]);
  }
}

static void *par_draw_worker(void *arg) {
  par_draw_job *j = (par_draw_job *)arg;
  const uint64_t nchunks = (j->draws + j->chunk - 1) / j->chunk;
  for (uint64_t c = j->tid; c < nchunks; c += j->nthreads) {
    const uint64_t beg = c * j->chunk;
    const uint64_t cnt = beg + j->chunk <= j->draws ? j->chunk : j->draws - beg;
    draw_chunk_keys(j, c, j->keys + beg, cnt);
  }
  return NULL;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

typedef struct {
  uint64_t *keys;       /* bucketed keys */
  const uint64_t *bstart; /* [nb + 1] */
  uint64_t *bunique;    /* [nb] unique count per bucket */
  uint32_t nb, nthreads, tid;
} par_sort_job;

static void *par_sort_worker(void *arg) {
  par_sort_job *j = (par_sort_job *)arg;
  for (uint32_t b = j->tid; b < j->nb; b += j->nthreads) {
    uint64_t *k = j->keys + j->bstart[b];
    const uint64_t n = j->bstart[b + 1] - j->bstart[b];
    qsort(k, n, sizeof(uint64_t), cmp_u64);
    uint64_t w = 0;
    for (uint64_t i = 0; i < n; i++)
      if (k[i] != UINT64_MAX && (w == 0 || k[i] != k[w - 1])) k[w++] = k[i];
    j->bunique[b] = w;
  }
  return NULL;
}

static int has_key(const uint64_t *sorted, uint64_t n, uint64_t key) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (sorted[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo < n && sorted[lo] == key;
}

/*
 * Build edges of the large workload. On success *m receives the edge count and src/dst (each
 * with room for `draws` entries) hold the sorted edge set; ins_src/ins_dst receive n_ins new
 * edges. Returns 0, or -1 on allocation failure.
 */
int dblgen_rmat_large(uint32_t scale, uint64_t seed, double a, double b, double c, uint64_t draws,
                      uint64_t chunk, uint32_t threads, uint32_t *src, uint32_t *dst, uint64_t *m,
                      uint64_t n_ins, uint32_t *ins_src, uint32_t *ins_dst) {
  if (scale == 0 || scale > 31 || threads == 0 || chunk == 0) return -1;
  const uint32_t n = 1u << scale;
  uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(draws ? draws : 1));
  uint64_t *bkeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(draws ? draws : 1));
  const uint32_t bbits = 12, nb = 1u << bbits;
  uint64_t *cnt = (uint64_t *)calloc((size_t)nb * threads + 1, sizeof(uint64_t));
  uint64_t *bstart = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
  uint64_t *bunique = (uint64_t *)calloc(nb, sizeof(uint64_t));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
  if (!perm || !keys || !bkeys || !cnt || !bstart || !bunique || !th) {
    free(perm); free(keys); free(bkeys); free(cnt); free(bstart); free(bunique); free(th);
    return -1;
  }
  xoshiro256 pr;
  xo_seed(&pr, seed + 1);
  for (uint32_t i = 0; i < n; i++) perm[i] = i;
  for (uint32_t i = n - 1; i > 0; i--) {
    uint32_t j = (uint32_t)xo_below(&pr, (uint64_t)i + 1);
    uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  par_draw_job *jobs = (par_draw_job *)calloc(threads, sizeof(par_draw_job));
  for (uint32_t t = 0; t < threads; t++) {
    jobs[t] = (par_draw_job){scale, a, b, c, perm, seed, chunk, draws, keys, threads, t};
    pthread_create(&th[t], NULL, par_draw_worker, &jobs[t]);
  }
  for (uint32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
  fprintf(stderr, "[dblgen] %llu draws done\n", (unsigned long long)draws);
  fflush(stderr);
  /* bucket by the top bits of the source id (ids are relabelled at random, so buckets are
     balanced) and sort each bucket */
  const uint32_t shift = 32 + scale - bbits;
  for (uint64_t i = 0; i < draws; i++)
    if (keys[i] != UINT64_MAX) bstart[(keys[i] >> shift) + 1]++;
  for (uint32_t k = 0; k < nb; k++) bstart[k + 1] += bstart[k];
  {
    uint64_t *fill = cnt; /* reuse as fill pointers */
    memcpy(fill, bstart, sizeof(uint64_t) * nb);
    for (uint64_t i = 0; i < draws; i++)
      if (keys[i] != UINT64_MAX) bkeys[fill[keys[i] >> shift]++] = keys[i];
  }
  par_sort_job *sj = (par_sort_job *)calloc(threads, sizeof(par_sort_job));
  for (uint32_t t = 0; t < threads; t++) {
    sj[t] = (par_sort_job){bkeys, bstart, bunique, nb, threads, t};
    pthread_create(&th[t], NULL, par_sort_worker, &sj[t]);
  }
  for (uint32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
  fprintf(stderr, "[dblgen] buckets sorted\n");
  fflush(stderr);
  uint64_t w = 0;
  for (uint32_t k = 0; k < nb; k++) {
    const uint64_t *kb = bkeys + bstart[k];
    for (uint64_t i = 0; i < bunique[k]; i++) {
      keys[w] = kb[i];
      src[w] = (uint32_t)(kb[i] >> 32);
      dst[w] = (uint32_t)kb[i];
      w++;
    }
  }
  *m = w;
  fprintf(stderr, "[dblgen] %llu distinct edges\n", (unsigned long long)w);
  fflush(stderr);
  /* insertion edges: later chunks, skipping loops, existing edges and repeats */
  int rc = 0;
  if (n_ins) {
    edge_set seen;
    if (set_init(&seen, n_ins)) rc = -1;
    uint64_t got = 0, cidx = (draws + chunk - 1) / chunk;
    uint64_t *buf = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)chunk);
    if (!buf) rc = -1;
    while (rc == 0 && got < n_ins) {
      draw_chunk_keys(&jobs[0], cidx++, buf, chunk);
      for (uint64_t i = 0; i < chunk && got < n_ins; i++) {
        const uint64_t k = buf[i];
        if (k == UINT64_MAX || has_key(keys, w, k)) continue;
        const int r = set_insert(&seen, k);
        if (r < 0) { rc = -1; break; }
        if (r == 0) continue;
        ins_src[got] = (uint32_t)(k >> 32);
        ins_dst[got] = (uint32_t)k;
        got++;
      }
    }
    free(buf);
    free(seen.slot);
  }
  free(perm); free(keys); free(bkeys); free(cnt); free(bstart); free(bunique); free(th);
  free(jobs); free(sj);
  return rc;
}
