/*
 * Oracle for level-synchronous BFS and SSSP -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct CPU reference of what the GPU library
 * computes.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper with
 * the HIP library, and the library never calls it.
 *
 * Graph format (Section I, CSR description): offsets[n+1] (int64 here, so the
 * oracle has no size limit of its own), cols[m], optional weights[m] (uint32).
 * Edges are out-edges; BFS and SSSP follow them.
 *
 * Infinity: BFS levels use INT32_MAX, SSSP distances use UINT32_MAX.  The
 * paper only writes "infinity" for unreached nodes (EP and WD pseudocode
 * initialisation); these are the values the library returns too.
 *
 * Every function returns 0 on success and a negative code on bad input.
 */
#ifndef LBG_ORACLE_H
#define LBG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_BFS_INF INT32_MAX
#define ORACLE_SSSP_INF UINT32_MAX

/* Hop distance from src along out-edges: FIFO-queue breadth-first search. */
int oracle_bfs(int64_t n, const int64_t* offsets, const int32_t* cols,
               int64_t src, int32_t* level_out);

/* Minimum total weight over directed paths from src: Dijkstra with a binary
 * min-heap and lazy deletion, 64-bit accumulation.  Returns -3 if a finite
 * distance does not fit below UINT32_MAX. */
int oracle_dijkstra(int64_t n, const int64_t* offsets, const int32_t* cols,
                    const uint32_t* weights, int64_t src, uint32_t* dist_out);

/* Brute force references for tiny graphs. */
int oracle_bellman_ford(int64_t n, const int64_t* offsets, const int32_t* cols,
                        const uint32_t* weights, int64_t src, uint32_t* dist_out);
/* All-pairs Floyd-Warshall; dist_out is n*n row-major (row = source). n <= 512. */
int oracle_floyd_warshall(int64_t n, const int64_t* offsets, const int32_t* cols,
                          const uint32_t* weights, uint32_t* dist_out);

/* Optimality certificate.  weights == NULL means unit weights (BFS) and d is
 * read as int32 with INT32_MAX infinity; otherwise d is uint32 with UINT32_MAX
 * infinity.  Checks (i) d[src]==0, (ii) d[v] <= d[u]+w for every arc with
 * finite d[u], (iii) the nodes reachable from src over tight arcs
 * (d[u]+w == d[v]) are exactly the nodes with finite d.  Returns 0 if all
 * hold (then d is the exact distance vector), 1/2/3 for the first failed
 * condition, negative for bad input.  *bad_index receives the offending node
 * (conditions 1 and 3) or arc (condition 2). */
int oracle_certificate(int64_t n, const int64_t* offsets, const int32_t* cols,
                       const uint32_t* weights, int64_t src, const void* d,
                       int64_t* bad_index);

/* Histogram-based maximum-degree threshold (Section III-B, automatic
 * determination of the node splitting threshold).  Writes the bin counts
 * (length bins) if hist_out is not NULL. */
int oracle_mdt(int64_t n, const int64_t* offsets, int32_t bins,
               int64_t* mdt_out, int64_t* hist_out);

/* Workload decomposition split (Section III-A and Algorithm "SSSP Pseudocode
 * illustrating Workload Decomposition"): the worklist's edges (degrees deg[k])
 * are block-distributed over num_threads threads, edgesPerThread =
 * ceil(total/num_threads) each.  For thread t writes the worklist index of the
 * node it starts in and the edge offset inside that node; threads whose chunk
 * starts past the end get node_offset = count.  Writes edges_per_thread. */
int oracle_wd_offsets(int64_t count, const int64_t* deg, int64_t num_threads,
                      int64_t* edges_per_thread, int64_t* node_offset,
                      int64_t* edge_offset);

/* Hierarchical processing schedule (Section III-C): in sub-iteration s a node
 * relaxes its edges [s*MDT, (s+1)*MDT); nodes with edges left form the next
 * sublist.  Writes the sublist size of every sub-iteration (at most
 * max_sub entries) and their number. */
int oracle_hp_schedule(int64_t count, const int64_t* deg, int64_t mdt,
                       int64_t max_sub, int64_t* sizes_out, int64_t* num_sub);

/* Node splitting (Section III-B): pieces = ceil(deg/MDT) for deg > MDT, edges
 * spread evenly, parent keeps the first (largest) piece.  Writes piece sizes
 * of one node (at most max_pieces) and their number. */
int oracle_ns_pieces(int64_t deg, int64_t mdt, int64_t max_pieces,
                     int64_t* sizes_out, int64_t* num_pieces);

#ifdef __cplusplus
}
#endif
#endif
