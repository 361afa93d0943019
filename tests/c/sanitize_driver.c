/* Host sanitizer run of the CPU oracle and the input generators: builds with
 * -fsanitize=address,undefined (see tests/test_sanitize_cpu.py), generates
 * graphs of every family, runs every oracle routine on them and checks the
 * answers against each other.  Exit status 0 = all checks passed; any
 * sanitizer report aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

typedef struct gg_graph gg_graph;
gg_graph* gg_uniform(int64_t n, int32_t k, uint64_t seed_struct, uint64_t seed_w, uint32_t wlo,
                     uint32_t whi);
gg_graph* gg_rmat(int scale, int32_t edge_factor, double a, double b, double c, uint64_t seed_struct,
                  uint64_t seed_perm, uint64_t seed_w, uint32_t wlo, uint32_t whi);
gg_graph* gg_grid(int64_t width, int64_t height, double drop_prob, double shortcut_frac,
                  uint64_t seed_struct, uint64_t seed_short, uint64_t seed_w, uint32_t wlo, uint32_t whi);
int64_t gg_n(const gg_graph* g);
int64_t gg_m(const gg_graph* g);
void gg_copy(const gg_graph* g, int32_t* offsets, int32_t* cols, uint32_t* weights);
void gg_free(gg_graph* g);
int64_t gg_sources(const int32_t* offsets, int64_t n, int64_t count, uint64_t seed, int32_t* out);
void gg_set_threads(int t);

static int failures = 0;
#define CHECK(cond, ...)              \
  do {                                \
    if (!(cond)) {                    \
      fprintf(stderr, __VA_ARGS__);   \
      fprintf(stderr, "\n");          \
      ++failures;                     \
    }                                 \
  } while (0)

static void run(const char* name, gg_graph* g, int brute) {
  CHECK(g != NULL, "%s: generator failed", name);
  if (!g) return;
  const int64_t n = gg_n(g), m = gg_m(g);
  int32_t* off32 = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* cols = malloc(sizeof(int32_t) * (size_t)(m + 1));
  uint32_t* w = malloc(sizeof(uint32_t) * (size_t)(m + 1));
  int64_t* off = malloc(sizeof(int64_t) * (size_t)(n + 1));
  gg_copy(g, off32, cols, w);
  for (int64_t i = 0; i <= n; ++i) off[i] = off32[i];
  int32_t srcs[3];
  const int64_t ns = gg_sources(off32, n, 3, 12345, srcs);
  int32_t* lv = malloc(sizeof(int32_t) * (size_t)n);
  uint32_t* d = malloc(sizeof(uint32_t) * (size_t)n);
  uint32_t* bf = malloc(sizeof(uint32_t) * (size_t)n);
  for (int64_t k = 0; k < ns; ++k) {
    int64_t bad = -1;
    CHECK(oracle_bfs(n, off, cols, srcs[k], lv) == 0, "%s: bfs failed", name);
    CHECK(oracle_certificate(n, off, cols, NULL, srcs[k], lv, &bad) == 0, "%s: bfs certificate (%lld)", name,
          (long long)bad);
    CHECK(oracle_dijkstra(n, off, cols, w, srcs[k], d) == 0, "%s: dijkstra failed", name);
    CHECK(oracle_certificate(n, off, cols, w, srcs[k], d, &bad) == 0, "%s: sssp certificate (%lld)", name,
          (long long)bad);
    if (brute) {
      CHECK(oracle_bellman_ford(n, off, cols, w, srcs[k], bf) == 0, "%s: bellman-ford failed", name);
      CHECK(memcmp(bf, d, sizeof(uint32_t) * (size_t)n) == 0, "%s: bellman-ford != dijkstra", name);
    }
  }
  if (brute && n <= 512) {
    uint32_t* fw = malloc(sizeof(uint32_t) * (size_t)(n * n));
    CHECK(oracle_floyd_warshall(n, off, cols, w, fw) == 0, "%s: floyd-warshall failed", name);
    for (int64_t k = 0; k < ns; ++k) {
      oracle_dijkstra(n, off, cols, w, srcs[k], d);
      CHECK(memcmp(fw + (size_t)srcs[k] * (size_t)n, d, sizeof(uint32_t) * (size_t)n) == 0,
            "%s: floyd-warshall != dijkstra", name);
    }
    free(fw);
  }
  int64_t mdt = 0, hist[10];
  CHECK(oracle_mdt(n, off, 10, &mdt, hist) == 0 && mdt >= 1, "%s: mdt", name);
  /* decomposition helpers on the first 100 degrees */
  const int64_t cnt = n < 100 ? n : 100;
  int64_t* deg = malloc(sizeof(int64_t) * (size_t)(cnt + 1));
  for (int64_t i = 0; i < cnt; ++i) deg[i] = off[i + 1] - off[i];
  int64_t ept = 0, node_off[16], edge_off[16], sizes[4096], nsub = 0, npc = 0;
  CHECK(oracle_wd_offsets(cnt, deg, 16, &ept, node_off, edge_off) == 0, "%s: wd", name);
  CHECK(oracle_hp_schedule(cnt, deg, mdt, 4096, sizes, &nsub) == 0, "%s: hp", name);
  for (int64_t i = 0; i < cnt; ++i)
    CHECK(oracle_ns_pieces(deg[i], mdt, 4096, sizes, &npc) == 0 && npc >= 1, "%s: ns", name);
  free(deg);
  free(lv);
  free(d);
  free(bf);
  free(off);
  free(off32);
  free(cols);
  free(w);
  gg_free(g);
}

int main(void) {
  gg_set_threads(2);
  run("uniform-n300", gg_uniform(300, 4, 1, 2, 1, 9), 1);
  run("uniform-n5000", gg_uniform(5000, 8, 3, 4, 1, 100), 0);
  run("rmat-9", gg_rmat(9, 16, 0.57, 0.19, 0.19, 5, 6, 7, 1, 255), 1);
  run("rmat-12", gg_rmat(12, 16, 0.57, 0.19, 0.19, 8, 9, 10, 1, 255), 0);
  run("grid-20", gg_grid(20, 20, 0.1, 0.01, 11, 12, 13, 1, 1000), 1);
  run("grid-60-noshortcut", gg_grid(60, 40, 0.1, 0.0, 14, 15, 16, 1, 1000), 0);
  run("uniform-n1", gg_uniform(1, 3, 17, 18, 0, 0), 1);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("sanitized oracle and generators: all checks passed\n");
  return 0;
}
