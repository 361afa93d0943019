/*
 * Seeded synthetic graph generators.
 *
 * This module only produces inputs: it holds none of the BFS/SSSP arithmetic.
 * Both the GPU library's tests/benchmark and the CPU oracle consume its
 * output.  Everything is deterministic for a given seed, independent of the
 * number of worker threads.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used counter-style: the i-th
 * value of stream s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), which equals the
 * i-th output of a SplitMix64 generator seeded with s.  Bounded integers use
 * Lemire's multiply-shift map (Lemire, "Fast random integer generation in an
 * interval", TOMACS 2019) without the rejection step; the bias is below
 * range / 2^32 and is irrelevant for test inputs.
 *
 * Families (all CSR, int32 ids, rows sorted unless stated otherwise):
 *   uniform: every node gets k out-arcs to uniform targets, self-loops dropped,
 *            duplicates kept, rows in generation order, one weight per arc.
 *   rmat:    recursive-matrix (R-MAT) pairs with quadrant probabilities
 *            a, b, c, d; seeded relabelling permutation; self-loops dropped;
 *            symmetrised; duplicates removed; one weight per undirected edge.
 *   grid:    W x H 4-neighbour lattice, each undirected edge dropped with a
 *            given probability, plus uniformly random long-range shortcuts;
 *            symmetrised; duplicates removed; one weight per undirected edge.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* i-th output of the SplitMix64 stream seeded with s */
static inline uint64_t sm_at(uint64_t s, uint64_t i) { return sm_mix(s + (i + 1) * GOLDEN); }
static inline uint32_t bounded32(uint32_t x, uint32_t range) {
  return (uint32_t)(((uint64_t)x * (uint64_t)range) >> 32);
}
static inline uint64_t bounded64(uint64_t x, uint64_t range) {
  return (uint64_t)(((unsigned __int128)x * range) >> 64);
}

uint64_t gg_splitmix_at(uint64_t s, uint64_t i) { return sm_at(s, i); }

/* ------------------------------------------------------------- threads -- */
static int g_threads = 0;
void gg_set_threads(int t) { g_threads = t; }
static int nthreads(void) {
  if (g_threads > 0) return g_threads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  if (c < 1) c = 1;
  if (c > 16) c = 16;
  return (int)c;
}

typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi);
typedef struct {
  range_fn fn;
  void* ctx;
  int64_t lo, hi;
} job_t;
static void* job_run(void* p) {
  job_t* j = (job_t*)p;
  j->fn(j->ctx, j->lo, j->hi);
  return NULL;
}
static void parallel_for(int64_t n, range_fn fn, void* ctx) {
  int t = nthreads();
  if (n < 4096 || t == 1) {
    fn(ctx, 0, n);
    return;
  }
  pthread_t th[64];
  job_t jobs[64];
  if (t > 64) t = 64;
  for (int i = 0; i < t; ++i) {
    jobs[i].fn = fn;
    jobs[i].ctx = ctx;
    jobs[i].lo = n * i / t;
    jobs[i].hi = n * (i + 1) / t;
    pthread_create(&th[i], NULL, job_run, &jobs[i]);
  }
  for (int i = 0; i < t; ++i) pthread_join(th[i], NULL);
}

/* ----------------------------------------------------------- graph obj -- */
typedef struct {
  int64_t n, m;
  int32_t* offsets; /* n+1 (m must fit in int32) */
  int32_t* cols;
  uint32_t* weights;
} gg_graph;

int64_t gg_n(const gg_graph* g) { return g->n; }
int64_t gg_m(const gg_graph* g) { return g->m; }
void gg_copy(const gg_graph* g, int32_t* offsets, int32_t* cols, uint32_t* weights) {
  memcpy(offsets, g->offsets, sizeof(int32_t) * (size_t)(g->n + 1));
  if (g->m) {
    memcpy(cols, g->cols, sizeof(int32_t) * (size_t)g->m);
    memcpy(weights, g->weights, sizeof(uint32_t) * (size_t)g->m);
  }
}
void gg_free(gg_graph* g) {
  if (!g) return;
  free(g->offsets);
  free(g->cols);
  free(g->weights);
  free(g);
}

/* ------------------------------------------------------------- uniform -- */
gg_graph* gg_uniform(int64_t n, int32_t k, uint64_t seed_struct, uint64_t seed_w,
                     uint32_t wlo, uint32_t whi) {
  if (n <= 0 || k < 0 || whi < wlo || n * (int64_t)k > INT32_MAX) return NULL;
  gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph));
  g->n = n;
  g->offsets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  g->cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n * k + 1));
  g->weights = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n * k + 1));
  uint32_t range = whi - wlo + 1;
  int64_t m = 0;
  g->offsets[0] = 0;
  for (int64_t u = 0; u < n; ++u) {
    for (int32_t j = 0; j < k; ++j) {
      uint64_t idx = (uint64_t)u * (uint64_t)k + (uint64_t)j;
      int64_t v = (int64_t)bounded64(sm_at(seed_struct, idx), (uint64_t)n);
      if (v == u) continue; /* self-loop dropped; duplicates kept */
      g->cols[m] = (int32_t)v;
      g->weights[m] = wlo + bounded32((uint32_t)(sm_at(seed_w, idx) >> 32), range);
      ++m;
    }
    g->offsets[u + 1] = (int32_t)m;
  }
  g->m = m;
  return g;
}

/* ------------------------------------------- symmetric edge-list to CSR -- */
typedef struct {
  int64_t n;
  int64_t npairs;
  const int32_t* pu;
  const int32_t* pv;
  int32_t* cnt;   /* n, atomically incremented */
  int32_t* cur;   /* n, scatter cursors */
  int32_t* cols;  /* 2*npairs */
  const int64_t* start;
  int32_t* newdeg;
} sym_ctx;

static void sym_count(void* c, int64_t lo, int64_t hi) {
  sym_ctx* s = (sym_ctx*)c;
  for (int64_t i = lo; i < hi; ++i) {
    int32_t u = s->pu[i], v = s->pv[i];
    if (u == v) continue;
    __atomic_fetch_add(&s->cnt[u], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&s->cnt[v], 1, __ATOMIC_RELAXED);
  }
}
static void sym_scatter(void* c, int64_t lo, int64_t hi) {
  sym_ctx* s = (sym_ctx*)c;
  for (int64_t i = lo; i < hi; ++i) {
    int32_t u = s->pu[i], v = s->pv[i];
    if (u == v) continue;
    int32_t a = __atomic_fetch_add(&s->cur[u], 1, __ATOMIC_RELAXED);
    s->cols[s->start[u] + a] = v;
    int32_t b = __atomic_fetch_add(&s->cur[v], 1, __ATOMIC_RELAXED);
    s->cols[s->start[v] + b] = u;
  }
}
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}
static void sort_small(int32_t* a, int64_t len) {
  if (len > 32) {
    qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    return;
  }
  for (int64_t i = 1; i < len; ++i) {
    int32_t x = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}
static void sym_sort_dedupe(void* c, int64_t lo, int64_t hi) {
  sym_ctx* s = (sym_ctx*)c;
  for (int64_t u = lo; u < hi; ++u) {
    int32_t* row = s->cols + s->start[u];
    int64_t len = s->cnt[u];
    sort_small(row, len);
    int64_t w = 0;
    for (int64_t i = 0; i < len; ++i)
      if (w == 0 || row[i] != row[w - 1]) row[w++] = row[i];
    s->newdeg[u] = (int32_t)w;
  }
}

typedef struct {
  gg_graph* g;
  const int64_t* start;
  const int32_t* tmp;
  uint64_t seed_w;
  uint32_t wlo, range;
} fill_ctx;
static void fill_rows(void* c, int64_t lo, int64_t hi) {
  fill_ctx* f = (fill_ctx*)c;
  for (int64_t u = lo; u < hi; ++u) {
    int64_t a = f->g->offsets[u], b = f->g->offsets[u + 1];
    memcpy(f->g->cols + a, f->tmp + f->start[u], sizeof(int32_t) * (size_t)(b - a));
    for (int64_t e = a; e < b; ++e) {
      uint64_t x = (uint64_t)u, y = (uint64_t)(uint32_t)f->g->cols[e];
      uint64_t lo2 = x < y ? x : y, hi2 = x < y ? y : x;
      uint64_t h = sm_at(f->seed_w, (lo2 << 32) | hi2); /* one weight per undirected edge */
      f->g->weights[e] = f->wlo + bounded32((uint32_t)(h >> 32), f->range);
    }
  }
}

/* Builds a symmetric, duplicate-free, self-loop-free CSR from undirected pairs. */
static gg_graph* symmetric_csr(int64_t n, int64_t npairs, const int32_t* pu, const int32_t* pv,
                               uint64_t seed_w, uint32_t wlo, uint32_t whi) {
  sym_ctx s;
  memset(&s, 0, sizeof(s));
  s.n = n;
  s.npairs = npairs;
  s.pu = pu;
  s.pv = pv;
  s.cnt = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  s.cur = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  parallel_for(npairs, sym_count, &s);
  start[0] = 0;
  for (int64_t u = 0; u < n; ++u) start[u + 1] = start[u] + s.cnt[u];
  s.start = start;
  s.cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(start[n] + 1));
  parallel_for(npairs, sym_scatter, &s);
  free(s.cur);
  s.newdeg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  parallel_for(n, sym_sort_dedupe, &s);
  gg_graph* g = (gg_graph*)calloc(1, sizeof(gg_graph));
  g->n = n;
  g->offsets = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int64_t m = 0;
  g->offsets[0] = 0;
  for (int64_t u = 0; u < n; ++u) {
    m += s.newdeg[u];
    if (m > INT32_MAX) {
      free(s.cnt);
      free(s.cols);
      free(s.newdeg);
      free(start);
      free(g->offsets);
      free(g);
      return NULL;
    }
    g->offsets[u + 1] = (int32_t)m;
  }
  g->m = m;
  g->cols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->weights = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m + 1));
  fill_ctx f = {g, start, s.cols, seed_w, wlo, whi - wlo + 1};
  parallel_for(n, fill_rows, &f);
  free(s.cnt);
  free(s.cols);
  free(s.newdeg);
  free(start);
  return g;
}

/* ---------------------------------------------------------------- rmat -- */
typedef struct {
  int scale;
  uint64_t seed;
  uint32_t ta, tab, tabc; /* cumulative quadrant thresholds scaled to 2^32 */
  const int32_t* perm;
  int32_t* pu;
  int32_t* pv;
} rmat_ctx;

static void rmat_pairs(void* c, int64_t lo, int64_t hi) {
  rmat_ctx* r = (rmat_ctx*)c;
  for (int64_t p = lo; p < hi; ++p) {
    uint32_t u = 0, v = 0;
    for (int lev = 0; lev < r->scale; ++lev) {
      uint32_t x = (uint32_t)(sm_at(r->seed, (uint64_t)p * (uint64_t)r->scale + (uint64_t)lev) >> 32);
      uint32_t bu, bv;
      if (x < r->ta) { bu = 0; bv = 0; }
      else if (x < r->tab) { bu = 0; bv = 1; }
      else if (x < r->tabc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    r->pu[p] = r->perm[u];
    r->pv[p] = r->perm[v];
  }
}

static int32_t* permutation(int64_t n, uint64_t seed) {
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) { /* Fisher-Yates */
    int64_t j = (int64_t)bounded64(sm_at(seed, (uint64_t)(n - 1 - i)), (uint64_t)(i + 1));
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  return perm;
}

gg_graph* gg_rmat(int scale, int32_t edge_factor, double a, double b, double c,
                  uint64_t seed_struct, uint64_t seed_perm, uint64_t seed_w, uint32_t wlo,
                  uint32_t whi) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || whi < wlo) return NULL;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return NULL;
  int64_t n = (int64_t)1 << scale;
  int64_t npairs = n * edge_factor;
  rmat_ctx r;
  r.scale = scale;
  r.seed = seed_struct;
  r.ta = (uint32_t)(a * 4294967296.0 > 4294967295.0 ? 4294967295.0 : a * 4294967296.0);
  double ab = (a + b) * 4294967296.0, abc = (a + b + c) * 4294967296.0;
  r.tab = (uint32_t)(ab > 4294967295.0 ? 4294967295.0 : ab);
  r.tabc = (uint32_t)(abc > 4294967295.0 ? 4294967295.0 : abc);
  r.perm = permutation(n, seed_perm);
  r.pu = (int32_t*)malloc(sizeof(int32_t) * (size_t)npairs);
  r.pv = (int32_t*)malloc(sizeof(int32_t) * (size_t)npairs);
  parallel_for(npairs, rmat_pairs, &r);
  free((void*)r.perm);
  gg_graph* g = symmetric_csr(n, npairs, r.pu, r.pv, seed_w, wlo, whi);
  free(r.pu);
  free(r.pv);
  return g;
}

/* ---------------------------------------------------------------- grid -- */
gg_graph* gg_grid(int64_t width, int64_t height, double drop_prob, double shortcut_frac,
                  uint64_t seed_struct, uint64_t seed_short, uint64_t seed_w, uint32_t wlo,
                  uint32_t whi) {
  if (width < 1 || height < 1 || whi < wlo || drop_prob < 0 || drop_prob > 1 || shortcut_frac < 0)
    return NULL;
  int64_t n = width * height;
  if (n > INT32_MAX) return NULL;
  int64_t nh = (width - 1) * height, nv = width * (height - 1);
  int64_t cap = nh + nv;
  uint32_t tdrop = (uint32_t)(drop_prob * 4294967296.0 > 4294967295.0 ? 4294967295.0
                                                                       : drop_prob * 4294967296.0);
  int64_t nshort_cap = (int64_t)(shortcut_frac * (double)cap) + 1;
  int32_t* pu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap + nshort_cap));
  int32_t* pv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap + nshort_cap));
  int64_t k = 0;
  for (int64_t id = 0; id < cap; ++id) {
    uint32_t x = (uint32_t)(sm_at(seed_struct, (uint64_t)id) >> 32);
    if (drop_prob >= 1.0 || x < tdrop) continue; /* dropped */
    int64_t u, v;
    if (id < nh) { /* horizontal edge (r, c)-(r, c+1) */
      int64_t rr = id / (width - 1), cc = id % (width - 1);
      u = rr * width + cc;
      v = u + 1;
    } else { /* vertical edge (r, c)-(r+1, c) */
      int64_t j = id - nh;
      int64_t rr = j / width, cc = j % width;
      u = rr * width + cc;
      v = u + width;
    }
    pu[k] = (int32_t)u;
    pv[k] = (int32_t)v;
    ++k;
  }
  int64_t nshort = (int64_t)(shortcut_frac * (double)k + 0.5);
  for (int64_t i = 0; i < nshort; ++i) {
    pu[k + i] = (int32_t)bounded64(sm_at(seed_short, 2 * (uint64_t)i), (uint64_t)n);
    pv[k + i] = (int32_t)bounded64(sm_at(seed_short, 2 * (uint64_t)i + 1), (uint64_t)n);
  }
  gg_graph* g = symmetric_csr(n, k + nshort, pu, pv, seed_w, wlo, whi);
  free(pu);
  free(pv);
  return g;
}

/* ------------------------------------------------------------- sources -- */
/* Up to `count` distinct nodes with out-degree > 0, drawn uniformly from
 * stream `seed`.  Returns how many were found. */
int64_t gg_sources(const int32_t* offsets, int64_t n, int64_t count, uint64_t seed,
                   int32_t* out) {
  int64_t found = 0;
  for (uint64_t i = 0; found < count && i < (uint64_t)(64 * n + 1024); ++i) {
    int64_t v = (int64_t)bounded64(sm_at(seed, i), (uint64_t)n);
    if (offsets[v + 1] == offsets[v]) continue;
    int dup = 0;
    for (int64_t j = 0; j < found; ++j)
      if (out[j] == v) { dup = 1; break; }
    if (!dup) out[found++] = (int32_t)v;
  }
  return found;
}
