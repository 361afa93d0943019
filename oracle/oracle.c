/*
 * Oracle for level-synchronous BFS and SSSP -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this.  It shares nothing with the HIP library.  Each function states the
 * passage of the paper it follows.  Where the paper's method reaches a result
 * with a plain definition (hop distance, shortest path weight), the oracle is
 * that definition computed by a textbook algorithm, not the paper's GPU
 * procedure: the data-driven Bellman-Ford of the paper converges to the unique
 * least fixed point d[v] = min(d[v], d[u] + w(u,v)), which is exactly the
 * shortest-path distance.
 *
 * ORACLE_MUTANT (compile-time, default 0) plants one deliberate mistake per
 * value.  The CPU test suite builds each mutant and checks that the pins catch
 * it; production builds never define it.
 */
#include "oracle.h"

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

#define U64_INF UINT64_MAX

static int check_graph(int64_t n, const int64_t* offsets, const int32_t* cols) {
  if (n <= 0 || offsets == NULL) return -1;
  if (offsets[0] != 0) return -2;
  for (int64_t u = 0; u < n; ++u)
    if (offsets[u + 1] < offsets[u]) return -2;
  int64_t m = offsets[n];
  if (m > 0 && cols == NULL) return -1;
  for (int64_t e = 0; e < m; ++e)
    if (cols[e] < 0 || (int64_t)cols[e] >= n) return -2;
  return 0;
}

/* ------------------------------------------------------------------ BFS --
 * Hop distance along out-edges (BFS is the paper's level-propagation
 * application, Section IV; its edge form is justified by the distributivity
 * remark of Section II-B).  Textbook FIFO queue. */
int oracle_bfs(int64_t n, const int64_t* offsets, const int32_t* cols,
               int64_t src, int32_t* level_out) {
  int rc = check_graph(n, offsets, cols);
  if (rc) return rc;
  if (src < 0 || src >= n || level_out == NULL) return -1;
  int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!queue) return -4;
  for (int64_t v = 0; v < n; ++v) level_out[v] = ORACLE_BFS_INF;
  level_out[src] = 0;
  int64_t head = 0, tail = 0;
  queue[tail++] = src;
  while (head < tail) {
    int64_t u = queue[head++];
    for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
      int64_t v = cols[e];
      if (level_out[v] == ORACLE_BFS_INF) {
#if ORACLE_MUTANT == 1
        level_out[v] = level_out[u]; /* planted: dropped "+1" */
#else
        level_out[v] = level_out[u] + 1;
#endif
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return 0;
}

/* ------------------------------------------------------------- Dijkstra --
 * Minimum path weight from src (the quantity the EP and WD SSSP algorithms of
 * Sections II-B and III-A converge to).  Binary min-heap of (dist, node) with
 * lazy deletion; distances accumulate in 64 bits and are narrowed at the end. */
typedef struct {
  uint64_t d;
  int64_t v;
} heap_item;

static void heap_push(heap_item* h, int64_t* size, heap_item it) {
  int64_t i = (*size)++;
  h[i] = it;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= h[i].d) break;
    heap_item t = h[p];
    h[p] = h[i];
    h[i] = t;
    i = p;
  }
}

static heap_item heap_pop(heap_item* h, int64_t* size) {
  heap_item top = h[0];
  h[0] = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, s = i;
    if (l < *size && h[l].d < h[s].d) s = l;
    if (r < *size && h[r].d < h[s].d) s = r;
    if (s == i) break;
    heap_item t = h[s];
    h[s] = h[i];
    h[i] = t;
    i = s;
  }
  return top;
}

static int narrow(int64_t n, const uint64_t* d64, uint32_t* out) {
  for (int64_t v = 0; v < n; ++v) {
    if (d64[v] == U64_INF) {
      out[v] = ORACLE_SSSP_INF;
    } else {
      if (d64[v] >= (uint64_t)ORACLE_SSSP_INF) return -3;
      out[v] = (uint32_t)d64[v];
    }
  }
  return 0;
}

int oracle_dijkstra(int64_t n, const int64_t* offsets, const int32_t* cols,
                    const uint32_t* weights, int64_t src, uint32_t* dist_out) {
  int rc = check_graph(n, offsets, cols);
  if (rc) return rc;
  if (src < 0 || src >= n || dist_out == NULL) return -1;
  if (offsets[n] > 0 && weights == NULL) return -1;
  int64_t m = offsets[n];
  uint64_t* dist = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  heap_item* heap = (heap_item*)malloc(sizeof(heap_item) * (size_t)(m + 1));
  if (!dist || !heap) {
    free(dist);
    free(heap);
    return -4;
  }
  for (int64_t v = 0; v < n; ++v) dist[v] = U64_INF;
  dist[src] = 0;
  int64_t hs = 0;
  heap_push(heap, &hs, (heap_item){0, src});
  while (hs > 0) {
    heap_item it = heap_pop(heap, &hs);
    int64_t u = it.v;
    if (it.d > dist[u]) continue; /* stale entry */
#if ORACLE_MUTANT == 2
    int64_t end = offsets[u + 1] - (offsets[u + 1] > offsets[u] ? 1 : 0); /* planted: last arc skipped */
#else
    int64_t end = offsets[u + 1];
#endif
    for (int64_t e = offsets[u]; e < end; ++e) {
      int64_t v = cols[e];
#if ORACLE_MUTANT == 3
      uint64_t nd = it.d + (uint64_t)weights[offsets[u]]; /* planted: first arc's weight for all */
#else
      uint64_t nd = it.d + (uint64_t)weights[e];
#endif
      if (nd < dist[v]) {
        dist[v] = nd;
        heap_push(heap, &hs, (heap_item){nd, v});
      }
    }
  }
  rc = narrow(n, dist, dist_out);
  free(dist);
  free(heap);
  return rc;
}

/* -------------------------------------------------------- Bellman-Ford --
 * Textbook: n-1 rounds, each relaxing every arc in CSR order. */
int oracle_bellman_ford(int64_t n, const int64_t* offsets, const int32_t* cols,
                        const uint32_t* weights, int64_t src, uint32_t* dist_out) {
  int rc = check_graph(n, offsets, cols);
  if (rc) return rc;
  if (src < 0 || src >= n || dist_out == NULL) return -1;
  if (offsets[n] > 0 && weights == NULL) return -1;
  uint64_t* dist = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  if (!dist) return -4;
  for (int64_t v = 0; v < n; ++v) dist[v] = U64_INF;
  dist[src] = 0;
  for (int64_t round = 0; round + 1 < n; ++round) {
    int changed = 0;
    for (int64_t u = 0; u < n; ++u) {
      if (dist[u] == U64_INF) continue;
      for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
        uint64_t nd = dist[u] + (uint64_t)weights[e];
        if (nd < dist[cols[e]]) {
          dist[cols[e]] = nd;
          changed = 1;
        }
      }
    }
    if (!changed) break;
  }
  rc = narrow(n, dist, dist_out);
  free(dist);
  return rc;
}

/* ------------------------------------------------------ Floyd-Warshall --
 * Textbook all-pairs closure over the min-plus semiring (min distributes over
 * +, the property Section II-B requires of edge-based processing). */
int oracle_floyd_warshall(int64_t n, const int64_t* offsets, const int32_t* cols,
                          const uint32_t* weights, uint32_t* dist_out) {
  int rc = check_graph(n, offsets, cols);
  if (rc) return rc;
  if (n > 512 || dist_out == NULL) return -1;
  if (offsets[n] > 0 && weights == NULL) return -1;
  uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n * n));
  if (!D) return -4;
  for (int64_t i = 0; i < n * n; ++i) D[i] = U64_INF;
  for (int64_t i = 0; i < n; ++i) D[i * n + i] = 0;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
      uint64_t w = weights[e];
      if (w < D[u * n + cols[e]]) D[u * n + cols[e]] = w;
    }
  for (int64_t k = 0; k < n; ++k)
    for (int64_t i = 0; i < n; ++i) {
      if (D[i * n + k] == U64_INF) continue;
      for (int64_t j = 0; j < n; ++j) {
        if (D[k * n + j] == U64_INF) continue;
        uint64_t c = D[i * n + k] + D[k * n + j];
        if (c < D[i * n + j]) D[i * n + j] = c;
      }
    }
  rc = narrow(n * n, D, dist_out);
  free(D);
  return rc;
}

/* --------------------------------------------------------- certificate --
 * (i) d[src] = 0; (ii) no arc can still be relaxed; (iii) every finite node is
 * reached from src over tight arcs and no infinite node is.  (ii) gives
 * d <= true distance by induction along any path; (iii) exhibits a path of
 * weight d[v], so d >= true distance.  Together: d is exact. */
int oracle_certificate(int64_t n, const int64_t* offsets, const int32_t* cols,
                       const uint32_t* weights, int64_t src, const void* d,
                       int64_t* bad_index) {
  int rc = check_graph(n, offsets, cols);
  if (rc) return rc;
  if (src < 0 || src >= n || d == NULL) return -1;
  const int32_t* di = (const int32_t*)d;
  const uint32_t* du = (const uint32_t*)d;
  int bfs = (weights == NULL);
  uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
  if (!D || !stack || !seen) {
    free(D);
    free(stack);
    free(seen);
    return -4;
  }
  int result = 0;
  int64_t bad = -1;
  for (int64_t v = 0; v < n; ++v) {
    if (bfs) {
      D[v] = (di[v] == ORACLE_BFS_INF) ? U64_INF : (uint64_t)(int64_t)di[v];
      if (di[v] < 0 && di[v] != ORACLE_BFS_INF) { result = 1; bad = v; }
    } else {
      D[v] = (du[v] == ORACLE_SSSP_INF) ? U64_INF : (uint64_t)du[v];
    }
  }
  if (!result && D[src] != 0) {
    result = 1;
    bad = src;
  }
#if ORACLE_MUTANT != 4
  if (!result) {
    for (int64_t u = 0; u < n && !result; ++u) {
      if (D[u] == U64_INF) continue;
      for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
        uint64_t w = bfs ? 1 : (uint64_t)weights[e];
        if (D[cols[e]] > D[u] + w) {
          result = 2;
          bad = e;
          break;
        }
      }
    }
  }
#endif
#if ORACLE_MUTANT != 5
  if (!result) {
    int64_t top = 0;
    stack[top++] = src;
    seen[src] = 1;
    while (top > 0) {
      int64_t u = stack[--top];
      for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
        int64_t v = cols[e];
        uint64_t w = bfs ? 1 : (uint64_t)weights[e];
        if (!seen[v] && D[v] != U64_INF && D[u] + w == D[v]) {
          seen[v] = 1;
          stack[top++] = v;
        }
      }
    }
    for (int64_t v = 0; v < n; ++v) {
      if ((D[v] != U64_INF) != (seen[v] != 0)) {
        result = 3;
        bad = v;
        break;
      }
    }
  }
#endif
  if (bad_index) *bad_index = bad;
  free(D);
  free(stack);
  free(seen);
  return result;
}

/* ------------------------------------------------------------------ MDT --
 * Section III-B: HistogramBinCount bins over the out-degree range; binIndex is
 * the tallest bin; MDT = (binIndex / HistogramBinCount) * maxDegree.
 * Reading of what the paper leaves open: bins have width maxDegree/bins and
 * are numbered from 1 (a degree d falls in bin max(1, ceil(d*bins/maxDegree)),
 * so degree 0 counts in bin 1); ties go to the smaller bin; the product is
 * rounded down and clamped to at least 1.  With 0-based numbering every
 * power-law graph would get MDT = 0, which the paper's rmat20 value (118 for
 * maxDegree 1181) rules out. */
int oracle_mdt(int64_t n, const int64_t* offsets, int32_t bins,
               int64_t* mdt_out, int64_t* hist_out) {
  if (n <= 0 || offsets == NULL || bins <= 0 || mdt_out == NULL) return -1;
  int64_t maxdeg = 0;
  for (int64_t u = 0; u < n; ++u) {
    int64_t dg = offsets[u + 1] - offsets[u];
    if (dg < 0) return -2;
    if (dg > maxdeg) maxdeg = dg;
  }
  int64_t* hist = (int64_t*)calloc((size_t)bins + 1, sizeof(int64_t));
  if (!hist) return -4;
  if (maxdeg == 0) {
    hist[1] = n;
  } else {
    for (int64_t u = 0; u < n; ++u) {
      int64_t dg = offsets[u + 1] - offsets[u];
      int64_t k = (dg * bins + maxdeg - 1) / maxdeg; /* ceil(d*bins/maxdeg) */
      if (k < 1) k = 1;
      hist[k]++;
    }
  }
  int64_t best = 1;
  for (int64_t k = 2; k <= bins; ++k)
    if (hist[k] > hist[best]) best = k;
#if ORACLE_MUTANT == 6
  best -= 1; /* planted: 0-based bin index */
#endif
  int64_t mdt = best * maxdeg / bins;
  if (mdt < 1) mdt = 1;
  *mdt_out = mdt;
  if (hist_out)
    for (int64_t k = 1; k <= bins; ++k) hist_out[k - 1] = hist[k];
  free(hist);
  return 0;
}

/* ------------------------------------------------------------ WD split --
 * Section III-A: the worklist's edges, in worklist order, are cut into
 * contiguous chunks of edgesPerThread = ceil(total / threads); thread t
 * starts at global edge t*edgesPerThread, i.e. at the worklist node whose
 * edge range holds it and at the matching offset inside that node (the
 * NodeOffset/EdgeOffset pair of the WD algorithm's offsets array). */
int oracle_wd_offsets(int64_t count, const int64_t* deg, int64_t num_threads,
                      int64_t* edges_per_thread, int64_t* node_offset,
                      int64_t* edge_offset) {
  if (count < 0 || num_threads <= 0 || edges_per_thread == NULL) return -1;
  if (count > 0 && deg == NULL) return -1;
  int64_t total = 0;
  for (int64_t k = 0; k < count; ++k) {
    if (deg[k] < 0) return -2;
    total += deg[k];
  }
#if ORACLE_MUTANT == 7
  int64_t ept = total / num_threads; /* planted: floor instead of ceil */
  if (ept == 0) ept = 1;
#else
  int64_t ept = (total + num_threads - 1) / num_threads;
#endif
  *edges_per_thread = ept;
  if (node_offset == NULL || edge_offset == NULL) return 0;
  int64_t k = 0, begin = 0; /* begin = first global edge of node k */
  for (int64_t t = 0; t < num_threads; ++t) {
    int64_t g = t * ept;
    while (k < count && begin + deg[k] <= g) {
      begin += deg[k];
      ++k;
    }
    if (k >= count || g >= total) {
      node_offset[t] = count;
      edge_offset[t] = 0;
    } else {
      node_offset[t] = k;
      edge_offset[t] = g - begin;
    }
  }
  return 0;
}

/* ---------------------------------------------------------- HP schedule --
 * Section III-C: sub-iteration s gives every node of the current sublist its
 * next MDT unprocessed edges; a node whose edges are not exhausted enters the
 * next sublist.  The first sublist is the whole (super) worklist. */
int oracle_hp_schedule(int64_t count, const int64_t* deg, int64_t mdt,
                       int64_t max_sub, int64_t* sizes_out, int64_t* num_sub) {
  if (count < 0 || mdt <= 0 || num_sub == NULL) return -1;
  if (count > 0 && deg == NULL) return -1;
  int64_t s = 0;
  for (;;) {
    /* sublist of sub-iteration s: every node at s = 0, afterwards the nodes
       whose edges were not exhausted by the first s windows */
    int64_t size = 0;
    for (int64_t k = 0; k < count; ++k)
#if ORACLE_MUTANT == 8
      if (s == 0 || deg[k] >= s * mdt) size++; /* planted: a node whose edges end exactly on a window boundary stays one sub-iteration too long */
#else
      if (s == 0 || deg[k] > s * mdt) size++;
#endif
    if (size == 0) break;
    if (sizes_out && s < max_sub) sizes_out[s] = size;
    ++s;
  }
  *num_sub = s;
  return 0;
}

/* ------------------------------------------------------------ NS pieces --
 * Section III-B: a node with out-degree above MDT becomes ceil(deg/MDT)
 * nodes (the parent and its children) whose out-edges are spread evenly;
 * a node at or below MDT is one piece. */
int oracle_ns_pieces(int64_t deg, int64_t mdt, int64_t max_pieces,
                     int64_t* sizes_out, int64_t* num_pieces) {
  if (deg < 0 || mdt <= 0 || num_pieces == NULL) return -1;
  int64_t p = (deg > mdt) ? (deg + mdt - 1) / mdt : 1;
  *num_pieces = p;
  if (sizes_out) {
    int64_t base = deg / p, extra = deg % p;
    for (int64_t i = 0; i < p && i < max_pieces; ++i)
      sizes_out[i] = base + (i < extra ? 1 : 0);
  }
  return 0;
}
