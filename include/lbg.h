/*
 * lbg -- level-synchronous BFS and SSSP with load-balanced frontier expansion
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: "Dynamic Load Balancing Strategies for Graph Applications on GPUs"
 * (Raval, Nasre, Kumar, R, Vadhiyar, Pingali; arXiv 1711.00231).
 *   - BFS: each level expands the current frontier along out-edges; a newly
 *     discovered node gets level+1 (Section IV; the distributivity remark of
 *     Section II-B makes the per-edge form legal).
 *   - SSSP: data-driven Bellman-Ford: every frontier node u relaxes its
 *     out-arcs, dist[v] = min(dist[v], dist[u] + w(u,v)) with an atomic
 *     minimum, and every improved v joins the next worklist; the loop ends
 *     when the worklist is empty (Algorithm "SSSP Pseudocode illustrating
 *     Edge-Based Parallelism", Section II-B, and its workload-decomposition
 *     variant, Section III-A).
 * Work assignment strategies (Section II and III-A):
 *   LBG_NODE      one thread per frontier node (the node-based baseline, BS)
 *   LBG_EDGE      one thread per worklist edge over a COO source array (the
 *                 edge-based baseline, EP, with work-chunked pushes)
 *   LBG_BALANCED  workload decomposition: the frontier's edges are cut into
 *                 equal contiguous tiles that ignore node boundaries, so hubs
 *                 are shared by many workgroups (WD)
 *   LBG_BINNED    degree bins: a node with more than `mdt` out-arcs enters
 *                 the worklist as pieces of at most mdt arcs (the node
 *                 splitting of Section III-B, applied to worklist entries),
 *                 and each entry is expanded by one lane, one wavefront or one
 *                 workgroup according to its length (lbg_set_bins)
 *   LBG_HIER      hierarchical processing (Section III-C): sub-iteration s
 *                 of a level relaxes arcs [s*MDT, (s+1)*MDT) of each frontier
 *                 node still active, one thread per node, MDT by the
 *                 histogram rule (lbg_degree_mdt); once fewer than 1024
 *                 nodes remain active their remaining arcs are expanded
 *                 edge-balanced
 *   LBG_EDGE_NOCHUNK  LBG_EDGE without work chunking: every arc of an
 *                 improved node is reserved with its own atomic on the tail
 *                 (the ablation of Section IV-D; slow by design)
 *   LBG_SLICED    workload decomposition per destination slice: node ids are
 *                 cut into 8 slices (one per XCD of the MI355X), every
 *                 adjacency list is grouped by destination slice once
 *                 (lbg_slice_graph); a frontier node with at least
 *                 lbg_set_slice_min() arcs is split into its per-slice
 *                 segments (the node splitting of Section III-B, pieces by
 *                 destination), each slice's segments are tiled as in
 *                 LBG_BALANCED and expanded by the workgroups of one XCD, so
 *                 their random node-state accesses stay within that XCD's L2;
 *                 smaller nodes are tiled together by all workgroups
 *                 (lbg_bfs_sliced, lbg_sssp_sliced)
 *   LBG_SPLIT     node splitting with child nodes (Section III-B): a node
 *                 with more than MDT out-arcs is cut into ceil(deg / MDT)
 *                 pieces; it keeps the first, and child nodes of a split
 *                 graph built once (lbg_split_graph) hold the others.  A
 *                 pushed node queues its own piece and its children's, which
 *                 carry its distance (the parent-to-child propagation), and
 *                 the pieces are tiled as in LBG_BALANCED (lbg_bfs_split,
 *                 lbg_sssp_split)
 *   LBG_AUTO      currently LBG_BALANCED
 *
 * Conventions for every entry point
 *   - Graph in CSR (Section I): offsets[n+1] int32 (offsets[0] = 0,
 *     non-decreasing, offsets[n] = m), cols[m] int32 in [0, n), weights[m]
 *     uint32.  Duplicate arcs and self-loops are allowed.
 *   - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors), except `stats` and the batched query table (host).  The
 *     caller owns every buffer; the library allocates no device memory.  It
 *     keeps, between calls: process-wide profiling counters and degree-bin
 *     parameters, per-device launch sizes, and per host thread one pinned
 *     control-block copy, its event pool and the last batch graph.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *     work is ordered on it.  The call returns after the solve has finished
 *     on the stream (the level loop reads the frontier size back to decide
 *     when to stop), so outputs are ready when it returns LBG_OK.
 *   - Argument errors are detected on the host before any launch; the call
 *     then returns a negative lbg_status, outputs are untouched and
 *     lbg_last_error() describes the problem.  A full structural check of the
 *     CSR is O(n + m) and therefore opt-in: lbg_validate_csr().
 *   - Thread safety: concurrent calls are safe on distinct workspaces (and
 *     output buffers); lbg_set_bins affects binned solves that start later.
 */
#ifndef LBG_H
#define LBG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBG_OK = 0,
  LBG_EINVAL = -1,     /* bad argument (null pointer, n <= 0, bad strategy) */
  LBG_ERANGE = -2,     /* src out of [0, n), m > INT32_MAX, m < 0 */
  LBG_ENOMEM = -3,     /* workspace smaller than lbg_workspace_bytes() */
  LBG_EHIP = -4,       /* a HIP runtime call or kernel launch failed */
  LBG_EOVERFLOW = -5,  /* device-side capacity guard tripped (library bug) */
  LBG_EINTERNAL = -6,  /* level count exceeded n + 1 (library bug or bad CSR) */
  LBG_EBUSY = -7       /* engine: no free query slot */
} lbg_status;

typedef enum {
  LBG_AUTO = 0,
  LBG_NODE = 1,
  LBG_EDGE = 2,
  LBG_BALANCED = 3,
  LBG_BINNED = 4,
  LBG_EDGE_NOCHUNK = 5,
  LBG_HIER = 6,
  LBG_SLICED = 7,
  LBG_SPLIT = 8
} lbg_strategy;

/* Counters of one solve (host struct, filled when `stats` is not NULL).
 * levels: number of frontiers holding at least one out-arc (BFS: 1 + the
 *         largest level of a reached node with out-arcs, which is the
 *         eccentricity of src + 1 unless every farthest node is a sink;
 *         SSSP: Bellman-Ford iterations).
 * frontier_entries: total worklist entries processed (nodes; LBG_EDGE: edges;
 *         LBG_SLICED: (node, slice) pairs; LBG_SPLIT: pieces).
 * edges_scanned: total arcs of the worklist entries processed (BFS: the
 *         arcs leaving reached nodes; SSSP: at least that, re-relaxations
 *         included).
 * updates: successful distance improvements (SSSP) or discoveries (BFS).
 * atomics: device-scope atomics issued on node state (claims / atomicMin).
 * edges_skipped: the part of edges_scanned that was never loaded: the arcs
 *         of SSSP worklist entries whose node improved again during the
 *         iteration that expands them (the node is queued for the next
 *         iteration, where its arcs are relaxed with the better distance).
 *         edges_scanned - edges_skipped arcs were read and relaxed.  0 for
 *         BFS and for strategies that relax every queued arc. */
typedef struct {
  int32_t levels;
  int32_t reserved;
  int64_t frontier_entries;
  int64_t edges_scanned;
  int64_t updates;
  int64_t atomics;
  int64_t edges_skipped;
} lbg_stats;

/* Bytes of device workspace a bfs (is_sssp = 0) or sssp (is_sssp = 1) call
 * with this strategy needs for a graph of n nodes and m arcs.  Returns 0 for
 * invalid arguments.  Node-based and balanced strategies need O(n + m/tile)
 * (CSR only, the space argument of Section III-A); the edge-based one needs
 * two edge worklists of m entries (the COO cost of Section II-B). */
size_t lbg_workspace_bytes(int32_t n, int64_t m, int32_t strategy, int32_t is_sssp);

/* BFS levels from src.  levels_out[v] = hop distance of v from src along
 * out-arcs, INT32_MAX if v is unreachable.  workspace: device buffer of at
 * least lbg_workspace_bytes(n, m, strategy, 0) bytes, 256-byte aligned, that
 * the call overwrites.  coo_src: device int32[m], the source node of every
 * arc in CSR order; required for LBG_EDGE and LBG_EDGE_NOCHUNK, ignored
 * otherwise (may be NULL). */
int lbg_bfs(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m, int32_t src,
            int32_t* levels_out, void* workspace, size_t workspace_bytes, int32_t strategy,
            const int32_t* coo_src, lbg_stats* stats, void* stream);

/* Scan levels of balanced BFS (Section II-B's worklist, built by a scan).
 * A level of lbg_bfs with LBG_BALANCED (or LBG_AUTO) whose frontier has at
 * least `arcs` out-arcs is expanded without claim atomics or pushes: each
 * newly reached node gets its level by a plain store, then one pass over the
 * levels array builds the next worklist from the nodes of the new level, in
 * node order.  Smaller levels claim and push as before.  Results are the
 * same either way.  arcs < 0 (the default): n / 4 for a graph of n nodes;
 * 0: every level; >= 2^32: never.  Process-wide, read when a solve starts;
 * lbg_get_bfs_scan_min returns the setting (-1 for the default).  Always
 * LBG_OK. */
int lbg_set_bfs_scan_min(int64_t arcs);
int64_t lbg_get_bfs_scan_min(void);

/* Element addressing of the kernels of single and batched solves that start
 * later and of engines created later (an engine keeps the form it was
 * created with).  mode 0 (the default): 32-bit element offsets from a
 * scalar base whenever every array the solve touches stays below 4 GiB
 * (n < 2^29 nodes, m < 2^30 arcs), 64-bit addresses otherwise; mode 1:
 * 64-bit addresses always (the form graphs above those bounds take; results
 * are the same, this exists so that form can be checked on small graphs).
 * Process-wide.  LBG_EINVAL for any other mode.  lbg_get_addressing returns
 * the setting. */
int lbg_set_addressing(int32_t mode);
int32_t lbg_get_addressing(void);

/* SSSP distances from src.  dist_out[v] = minimum total weight of a directed
 * path from src to v, UINT32_MAX if unreachable.  Precondition: every finite
 * shortest-path weight is below UINT32_MAX (e.g. (n-1) * max weight <
 * UINT32_MAX); distances are exact integers, so the result is bit-identical
 * whatever the order in which relaxations happen.  Other arguments as for
 * lbg_bfs, with lbg_workspace_bytes(n, m, strategy, 1). */
int lbg_sssp(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
             int64_t m, int32_t src, uint32_t* dist_out, void* workspace, size_t workspace_bytes,
             int32_t strategy, const int32_t* coo_src, lbg_stats* stats, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbg_sssp without a
 * workspace argument.  The call makes no device or host allocation of any
 * kind (no hipMalloc, hipFree, hipHostMalloc, event creation or library
 * allocator); its workspace is a file-scope device array of
 * LBG_NOALLOC_SCRATCH_BYTES bytes that every GPU the library runs on holds
 * from the library's first use on it until the process ends.
 *   - Sizes: lbg_workspace_bytes(n, m, strategy, 1) must not exceed
 *     LBG_NOALLOC_SCRATCH_BYTES (64 MiB: e.g. R-MAT scale 20, n = 2^20 with
 *     31 M arcs, fits; scale 22 does not); larger problems return
 *     LBG_ENOMEM before any launch, with dist_out untouched.
 *   - strategy: LBG_AUTO, LBG_BALANCED, LBG_NODE, LBG_BINNED or LBG_HIER
 *     (the ones that need no other input); others return LBG_EINVAL.
 *   - Results are identical to lbg_sssp's.  The solve is stream-ordered on
 *     `stream` and returns when dist_out is written, as lbg_sssp does; the
 *     control block is read back through pageable host memory.  Launch
 *     timing (lbg_profile_enable) does not apply to these calls, and an
 *     LBG_HIER call leaves lbg_hier_last_schedule untouched.
 *   - Every call on one GPU uses that GPU's one array, and each call
 *     re-initialises everything it reads there: calls that overlap on one
 *     GPU (other host threads, other streams) race and must be serialised
 *     by the caller.
 * Other arguments and errors as for lbg_sssp. */
#define LBG_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbg_sssp_noalloc(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                     int64_t m, int32_t src, uint32_t* dist_out, int32_t strategy, lbg_stats* stats,
                     void* stream);

/* COO source array of a CSR graph (what LBG_EDGE and LBG_EDGE_NOCHUNK
 * read beside the CSR; Section II-B): coo_out[e] = the node u with
 * offsets[u] <= e < offsets[u + 1], for every arc e in [0, m).  coo_out is a
 * device int32[m] the caller allocates (may be NULL when m = 0).  Offsets
 * outside [0, m] are clamped (lbg_validate_csr first on untrusted input).
 * Returns after coo_out is written; LBG_EINVAL / LBG_ERANGE on bad
 * arguments. */
int lbg_coo_sources(const int32_t* offsets, int32_t n, int64_t m, int32_t* coo_out, void* stream);

/* ------------------------------------------------------------------------
 * Packed arcs for SSSP (the balanced strategy of Section III-A on a denser
 * arc encoding).
 *
 * lbg_pack_arcs: arcs_out[e] = (cols[e] << wbits) | weights[e], with wbits
 * the bit length of the largest weight (0 if all weights are 0), written to
 * *wbits_out.  Needs bitlength(n - 1) + wbits <= 32, else LBG_ERANGE (e.g.
 * n = 2^22 nodes with weights below 256, or n = 2^24 with weights below
 * 256).  workspace: device scratch of at least 1152 bytes (the control
 * block; any solve workspace will do), 256-byte aligned, overwritten.  cols must lie in [0, n)
 * (lbg_validate_csr).  Returns when arcs_out is written.
 *
 * lbg_sssp_packed: lbg_sssp with strategy LBG_BALANCED reading arc e as one
 * 32-bit word of arcs[] instead of cols[e] and weights[e] (one load per arc
 * instead of two, half the arc bytes); same offsets, same workspace
 * (lbg_workspace_bytes(n, m, LBG_BALANCED, 1)), identical results.
 * LBG_ERANGE if wbits is outside [0, 31] or the node ids of n do not fit
 * beside wbits weight bits. */
int lbg_pack_arcs(const int32_t* cols, const uint32_t* weights, int32_t n, int64_t m, uint32_t* arcs_out,
                  int32_t* wbits_out, void* workspace, size_t workspace_bytes, void* stream);
int lbg_sssp_packed(const int32_t* offsets, const uint32_t* arcs, int32_t wbits, int32_t n, int64_t m,
                    int32_t src, uint32_t* dist_out, void* workspace, size_t workspace_bytes,
                    lbg_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Destination-sliced graphs (LBG_SLICED; the workload decomposition of
 * Section III-A, cut per destination slice).
 *
 * Slices: node v belongs to slice v / S, S = lbg_slice_nodes(n) =
 * ceil(n / 8) rounded up to a multiple of 64; there are at most 8 slices.
 *
 * lbg_slice_graph: from a CSR graph (offsets[n+1], cols[m], optional
 * weights[m]; conventions above) writes
 *   slice_offsets[8n + 1] int32: the arcs of node u into slice x are
 *     positions slice_offsets[8u + x] .. slice_offsets[8u + x + 1] - 1 of
 *     cols_out (so slice_offsets[8u] = offsets[u], slice_offsets[8n] = m);
 *   cols_out[m], weights_out[m]: each adjacency list regrouped by destination
 *     slice, arcs of one slice in their input order.
 * (offsets, cols_out, weights_out) is a CSR of the same graph, valid for
 * every other strategy.  weights and weights_out are both NULL (BFS only) or
 * both given (when m > 0).  All outputs are device buffers the caller allocates; they
 * must not overlap the inputs.  Offsets outside [0, m] are clamped (run
 * lbg_validate_csr first on untrusted input).  Returns when the outputs are
 * written; LBG_EINVAL / LBG_ERANGE on bad arguments.
 *
 * lbg_bfs_sliced / lbg_sssp_sliced: as lbg_bfs / lbg_sssp with strategy
 * LBG_SLICED, on the output of lbg_slice_graph: offsets = the CSR offsets
 * (unchanged by the grouping), slice_offsets, cols = cols_out, weights =
 * weights_out; workspace of at least
 * lbg_workspace_bytes(n, m, LBG_SLICED, is_sssp) bytes (for each of the 8
 * slice lists and the mixed list: two worklists of min(n, m) entries and
 * their tile marks).  Results are identical to every other strategy's.
 * lbg_bfs / lbg_sssp reject LBG_SLICED with LBG_EINVAL.
 *
 * lbg_set_slice_min: process-wide degree from which a frontier node is split
 * by destination slice (default 512; 0 = every node, INT32_MAX = none, which
 * leaves one list tiled by every workgroup).  LBG_EINVAL if negative; affects
 * sliced solves that start later.  lbg_get_slice_min returns it. */
int32_t lbg_slice_nodes(int32_t n);
int lbg_set_slice_min(int32_t min_degree);
int32_t lbg_get_slice_min(void);
int lbg_slice_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t* slice_offsets, int32_t* cols_out, uint32_t* weights_out,
                    void* stream);
int lbg_bfs_sliced(const int32_t* offsets, const int32_t* slice_offsets, const int32_t* cols, int32_t n,
                   int64_t m, int32_t src, int32_t* levels_out, void* workspace, size_t workspace_bytes,
                   lbg_stats* stats, void* stream);
int lbg_sssp_sliced(const int32_t* offsets, const int32_t* slice_offsets, const int32_t* cols,
                    const uint32_t* weights, int32_t n, int64_t m, int32_t src, uint32_t* dist_out,
                    void* workspace, size_t workspace_bytes, lbg_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Split graphs (LBG_SPLIT; node splitting with child nodes, Section III-B).
 *
 * Under split size mdt (>= 1; 0 = no splitting) a node v with d > mdt
 * out-arcs has p = ceil(d / mdt) pieces, the first d % p of them one arc
 * longer (piece k starts at arc k * floor(d / p) + min(k, d % p)); v keeps
 * piece 0 and pieces 1 .. p - 1 go to p - 1 child nodes.  The split graph
 * has n + C nodes (C = total child count): node v < n holds v's piece 0,
 * node n + child_base[v] + k - 1 holds v's piece k.  Arcs still point at
 * original nodes only.  The histogram rule of Section III-B for mdt is
 * lbg_degree_mdt.
 *
 * lbg_split_scratch_bytes(n): device scratch the next two calls need
 * (12 bytes per 4096 nodes, rounded up to 256).
 * lbg_split_count: *children_out = C.  Returns after a read-back.
 * lbg_split_graph: writes
 *   split_offsets[n + C + 1] int32: CSR offsets of the split graph; the
 *     parents' pieces come first in the arc array (in node order), then the
 *     children's (in child order), so split_offsets[n] is the number of arcs
 *     in parents' pieces and split_offsets[n + C] = m;
 *   child_base[n + 1] int32: exclusive prefix sum of the child counts;
 *   cols_out[m], weights_out[m]: the arcs regrouped in that order.
 * children must equal lbg_split_count's result (LBG_EINVAL otherwise).
 * weights and weights_out are both NULL (BFS only) or both given (m > 0).
 * Outputs are device buffers the caller allocates, not overlapping the
 * inputs; offsets outside [0, m] are clamped (lbg_validate_csr first on
 * untrusted input).  LBG_ERANGE if n + C does not fit in int32.
 *
 * lbg_bfs_split / lbg_sssp_split: as lbg_bfs / lbg_sssp on the split graph:
 * split_offsets, child_base, cols = cols_out, weights = weights_out, the
 * original n, the child count C; workspace of at least
 * lbg_split_workspace_bytes(n, m, C, is_sssp) bytes (two worklists of n + C
 * entries and their tile marks; lbg_workspace_bytes(n, m, LBG_SPLIT, .)
 * gives the bound for C = m).  levels_out / dist_out have n entries; results
 * are identical to every other strategy's.  lbg_bfs / lbg_sssp reject
 * LBG_SPLIT with LBG_EINVAL. */
size_t lbg_split_scratch_bytes(int32_t n);
int lbg_split_count(const int32_t* offsets, int32_t n, int64_t m, int32_t mdt, int64_t* children_out,
                    void* scratch, size_t scratch_bytes, void* stream);
int lbg_split_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t mdt, int64_t children, int32_t* split_offsets, int32_t* child_base,
                    int32_t* cols_out, uint32_t* weights_out, void* scratch, size_t scratch_bytes,
                    void* stream);
size_t lbg_split_workspace_bytes(int32_t n, int64_t m, int64_t children, int32_t is_sssp);
int lbg_bfs_split(const int32_t* split_offsets, const int32_t* child_base, const int32_t* cols, int32_t n,
                  int64_t children, int64_t m, int32_t src, int32_t* levels_out, void* workspace,
                  size_t workspace_bytes, lbg_stats* stats, void* stream);
int lbg_sssp_split(const int32_t* split_offsets, const int32_t* child_base, const int32_t* cols,
                   const uint32_t* weights, int32_t n, int64_t children, int64_t m, int32_t src,
                   uint32_t* dist_out, void* workspace, size_t workspace_bytes, lbg_stats* stats,
                   void* stream);

/* ------------------------------------------------------------------------
 * Degree-class ordered copy for SSSP (the balanced strategy of Section III-A
 * on a renumbered copy of the graph; a memory layout, the arithmetic is
 * unchanged).
 *
 * lbg_order_graph: renumbers the nodes by degree class, largest first (the
 * class of out-degree d is its bit length: 0 for d = 0, 1 for d = 1, 2 for
 * 2..3, ...; original order within a class) and writes
 *   new_id[n] int32: the new id of original node v;
 *   order_offsets[n+1], order_cols[m], order_weights[m]: the same graph in
 *     new ids; the arcs of new node k are those of the original node, with
 *     destinations renamed, ordered by destination class (largest first) and
 *     by input position within a class (ascending new id when the input
 *     adjacency lists are sorted).
 * weights and order_weights are both NULL or both given (when m > 0).
 * scratch: device buffer of lbg_order_scratch_bytes(n) bytes (4n plus 132
 * bytes per 4096 nodes, each part rounded up to 256), 256-byte aligned,
 * overwritten.  Outputs are device
 * buffers the caller allocates, not overlapping the inputs; offsets outside
 * [0, m] are clamped and destinations outside [0, n) are copied unchanged
 * (lbg_validate_csr first on untrusted input).  Returns when the outputs are
 * written.
 *
 * lbg_sssp_ordered: lbg_sssp with strategy LBG_BALANCED on the ordered copy:
 * src and dist_out are in ORIGINAL ids (the source is renamed and the
 * distances gathered back through new_id on the device), so results equal
 * lbg_sssp's on the original graph.  Workspace:
 * lbg_workspace_bytes(n, m, LBG_BALANCED, 1). */
size_t lbg_order_scratch_bytes(int32_t n);
int lbg_order_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t* order_offsets, int32_t* order_cols, uint32_t* order_weights,
                    int32_t* new_id, void* scratch, size_t scratch_bytes, void* stream);
int lbg_sssp_ordered(const int32_t* order_offsets, const int32_t* order_cols, const uint32_t* order_weights,
                     const int32_t* new_id, int32_t n, int64_t m, int32_t src, uint32_t* dist_out,
                     void* workspace, size_t workspace_bytes, lbg_stats* stats, void* stream);

/* Structural check of a CSR graph on the device: offsets[0] == 0,
 * non-decreasing offsets, offsets[n] == m, every col in [0, n).  Needs
 * lbg_workspace_bytes(n, m, LBG_NODE, 0) bytes of workspace.  Returns LBG_OK
 * or LBG_EINVAL (with a message naming the first kind of defect found). */
int lbg_validate_csr(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m,
                     void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Hierarchical processing (LBG_HIER, Section III-C).
 *
 * lbg_set_hier_mdt: process-wide MDT of LBG_HIER solves that start later; 0
 * (the default) = the histogram rule of Section III-B per solve (as
 * lbg_degree_mdt), > 0 = that window length.  LBG_EINVAL if negative.
 * lbg_get_hier_mdt returns the setting.
 *
 * lbg_hier_last_schedule: the sub-iteration schedule of the calling thread's
 * last LBG_HIER solve: sizes[l * max_subs + s] (host array of max_levels *
 * max_subs int32) = the number of worklist entries active in sub-iteration s
 * of level l (sub-iteration 0 holds the whole worklist; an entry stays active
 * while it has arcs beyond the windows already processed), 0 past the last
 * sub-iteration.  The sub-iteration whose sublist holds fewer than 1024
 * entries expands all of their remaining arcs (the hand-over to workload
 * decomposition), so it is the level's last.  Recorded for levels < 64 and
 * sub-iterations < 256.  Returns the number of levels written (at most
 * max_levels; 0 before any LBG_HIER solve); *mdt_out (nullable) receives the
 * MDT that solve used. */
int lbg_set_hier_mdt(int32_t mdt);
int32_t lbg_get_hier_mdt(void);
int32_t lbg_hier_last_schedule(int32_t* sizes, int32_t max_levels, int32_t max_subs, int32_t* mdt_out);

/* ------------------------------------------------------------------------
 * Degree-bin parameters of LBG_BINNED solves (process-wide).
 *   mdt      split size: a node with more out-arcs is queued as ceil(deg/mdt)
 *            pieces, the first deg % pieces of them one arc longer (0 = no
 *            splitting; otherwise at least 64)
 *   t_wave   pieces longer than this are expanded by one wavefront
 *   t_block  pieces longer than this are expanded by one workgroup
 * lbg_set_bins returns LBG_EINVAL (and changes nothing) for mdt in [1, 63]
 * or t_wave > t_block; it applies to solves that start afterwards.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t mdt, t_wave, t_block;
} lbg_bins;

int lbg_set_bins(const lbg_bins* bins);
void lbg_get_bins(lbg_bins* bins);

/* The MDT of Section III-B computed on the device from the CSR offsets: the
 * out-degrees are histogrammed into 10 bins of width maxDegree/10 numbered
 * from 1 (bin of degree d: max(1, ceil(10 d / maxDegree))), k = the fullest
 * bin (ties to the smaller), MDT = max(1, floor(k * maxDegree / 10)).
 * workspace: lbg_workspace_bytes(n, m, LBG_NODE, 0) bytes.  *mdt_out is a
 * host int32; *max_degree_out (nullable) receives maxDegree. */
int lbg_degree_mdt(const int32_t* offsets, int32_t n, int64_t m, void* workspace,
                   size_t workspace_bytes, int32_t* mdt_out, int32_t* max_degree_out, void* stream);

/* Autotuner of the degree bins on the caller's graph: times LBG_BINNED BFS
 * (and SSSP when weights is not NULL) from the given host array of sources
 * for split sizes seeded by lbg_degree_mdt and a small grid of t_wave /
 * t_block values, keeps the fastest set (lbg_set_bins) and returns it in
 * *best.  out: device int32[n] scratch; workspace: at least
 * lbg_workspace_bytes(n, m, LBG_BINNED, 1) bytes.  Results of the timed
 * solves are discarded; the call synchronises `stream`. */
int lbg_autotune_bins(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                      int32_t n, int64_t m, const int32_t* sources, int32_t num_sources,
                      int32_t* out, void* workspace, size_t workspace_bytes, lbg_bins* best,
                      void* stream);

/* Human-readable message for the last non-OK return on the calling thread. */
const char* lbg_last_error(void);

/* Per-kernel timing of the frontier-expansion kernels, for roofline
 * reporting.  While enabled, HIP events on the caller's stream time every
 * expansion launch of single solves (one event when a batch of launches
 * starts, then one after each launch, so a launch's duration runs from the
 * event before it to the event after it; the events skip the system-scope
 * cache fence, which the read-out does not need) and its duration is
 * accumulated process-wide,
 * together with the work it did, separately for BFS and SSSP solves (they run
 * different kernels).  enable = 0 stops collection; reset = 1 clears the
 * totals. */
void lbg_profile_enable(int32_t enable, int32_t reset);

typedef struct {
  int64_t launches;          /* expansion kernel launches that had work */
  int64_t empty_launches;    /* launches that found an empty frontier */
  double kernel_ms;          /* summed duration of the launches with work */
  double empty_ms;           /* summed duration of the empty launches */
  int64_t frontier_entries;  /* worklist entries they consumed */
  int64_t edges_scanned;     /* arcs they relaxed */
  int64_t updates;           /* successful distance improvements/discoveries */
  int64_t atomics;           /* device-scope atomics issued on node state */
  int64_t edges_skipped;     /* arcs of edges_scanned never loaded (lbg_stats) */
} lbg_profile;

/* Totals since the last reset of the one-level launches of BFS solves
 * (which = 0), SSSP solves (1) or batched solves (2), and of the
 * small-frontier launches of BFS (3) and SSSP (4) solves (the
 * single-workgroup level loop that balanced solves switch to while a level
 * has at most 4000 entries and 16384 edges; `launches` counts launches, the
 * work counters cover every level they ran, empty_* stay 0). */
void lbg_profile_read(int32_t which, lbg_profile* out);

/* ------------------------------------------------------------------------
 * Batched solves.  Many independent BFS/SSSP queries advance level by level
 * through ONE shared worklist whose entries carry their query, so a batch
 * costs one launch per level however many queries it holds, and the work of
 * small and large queries is balanced together (the edge-tile split of the
 * balanced strategy, over the union of all queries' frontiers).
 *
 * The graph is a disjoint union of instances in one CSR with global node
 * ids: instance k owns the node range [lo, hi) and every arc leaving a node
 * of that range lands in it (pack instances by offsetting their ids).  BFS
 * and SSSP queries mix freely in one batch: a BFS query claims each node of
 * its row once, with a bit in a per-row bitmap, and an SSSP query relaxes
 * with the atomic minimum of the single-query path.
 * ------------------------------------------------------------------------ */
#define LBG_KIND_BFS 0
#define LBG_KIND_SSSP 1

typedef struct {
  int32_t src;     /* global source node, lo <= src < hi */
  int32_t lo, hi;  /* node range of the query's instance */
  int32_t kind;    /* LBG_KIND_BFS or LBG_KIND_SSSP */
  int64_t out_off; /* first element of the query's result row in `out` */
} lbg_query;

/* Device workspace for lbg_batch_solve (0 for invalid arguments). */
size_t lbg_batch_workspace_bytes(int32_t num_queries, int64_t total_rows, int64_t total_arcs);

/* Solves num_queries queries (a HOST array) over the packed graph.  Query q
 * writes hi - lo results to out[out_off .. out_off + hi - lo): int32 levels
 * (INT32_MAX = unreachable) for BFS, uint32 distances (UINT32_MAX) for SSSP,
 * element j for node lo + j.  Rows must not overlap; total_rows (< 2^31) is
 * the length of `out` (device uint32, int32 bit patterns for BFS rows).
 * total_arcs bounds the edge space of one level: the sum over queries of the
 * arcs leaving their instance (< 2^32).  weights are required (BFS queries
 * ignore them).  Errors as for lbg_bfs; an arc leaving its instance makes the
 * call return LBG_EOVERFLOW instead of touching another row.  The call is
 * stream-ordered and returns when all queries have finished. */
int lbg_batch_solve(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, const lbg_query* queries, int32_t num_queries, uint32_t* out,
                    int64_t total_rows, int64_t total_arcs, void* workspace, size_t workspace_bytes,
                    lbg_stats* stats, void* stream);

/* lbg_batch_solve with the level loop as a HIP graph: one instantiated graph
 * runs 64 levels (the expansion reads its level from the control block; a
 * level whose worklist is empty returns at once), moves
 * the level base on, writes the rows out once the worklist is empty and reads
 * the control block back; the host replays it until the batch is done.  The
 * executable graph is cached per host thread and reused while every argument
 * stays the same (same buffers, sizes and queries' workspace layout); a call
 * with other arguments rebuilds it.  Same arguments, results and errors as
 * lbg_batch_solve.  For callers that launch many batches: the host issues one
 * graph launch per 64 levels instead of 64 kernel launches, so a batch of at
 * most 64 levels (every query's BFS depth and SSSP iteration count) is one
 * graph launch and one read-back. */
int lbg_batch_solve_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                          int32_t n, int64_t m, const lbg_query* queries, int32_t num_queries,
                          uint32_t* out, int64_t total_rows, int64_t total_arcs, void* workspace,
                          size_t workspace_bytes, lbg_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Engine: continuous batching for serving.  An engine keeps one packed graph
 * (as for lbg_batch_solve) and a pool of query slots; queries submitted
 * while others are in flight join the shared worklist at the next level
 * boundary, finished queries leave, and their slots and rows can be reused.
 * A query's result is the same whatever else runs with it: the relaxation
 * reaches the same least fixed point in any order.
 *
 * The caller owns the graph, the result rows (`rows_out`, device uint32[max_rows],
 * one row per query at the query's out_off) and the workspace; it chooses
 * each query's row (admission by memory footprint is the caller's policy).
 * All calls on one engine must come from one thread; work is ordered on the
 * engine's stream and every call returns with its work finished.
 * ------------------------------------------------------------------------ */
typedef struct lbg_engine lbg_engine;

/* Device workspace for an engine with these capacities (0 if invalid).
 * max_rows: total result elements of concurrently admitted queries (< 2^31);
 * max_level_arcs: bound on the arcs one level can hold (< 2^32), e.g. the sum
 * of the arc counts of the instances that may be queried concurrently. */
size_t lbg_engine_workspace_bytes(int32_t max_queries, int64_t max_rows, int64_t max_level_arcs);

/* Create an engine over the packed graph (device offsets/cols/weights as for
 * lbg_batch_solve) with the given capacities, result rows `rows_out` and a
 * workspace of at least lbg_engine_workspace_bytes (256-byte aligned); all
 * stay the caller's and must outlive the engine.  *engine receives a host
 * handle (the library's pinned host buffers for the slot table and
 * read-backs) that lbg_engine_destroy frees.  LBG_EINVAL for a null
 * pointer, n <= 0 or a misaligned workspace, LBG_ERANGE for m outside
 * [0, INT32_MAX] or invalid capacities, LBG_ENOMEM for a small workspace,
 * LBG_EHIP if the pinned host buffers cannot be allocated. */
int lbg_engine_create(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                      int32_t n, int64_t m, int32_t max_queries, int64_t max_rows,
                      int64_t max_level_arcs, uint32_t* rows_out, void* workspace,
                      size_t workspace_bytes, void* stream, lbg_engine** engine);

/* Queue a query (host struct; out_off = its row in rows_out).  It joins the
 * batch at the next lbg_engine_step.  *slot receives its slot; LBG_EBUSY if
 * every slot is in use. */
int lbg_engine_submit(lbg_engine* e, const lbg_query* q, int32_t* slot);

/* Inject queued queries, expand `levels` levels, then detect queries whose
 * worklist emptied and write their rows.  *finished (nullable) receives how
 * many finished in this step; lbg_engine_finished lists them. */
int lbg_engine_step(lbg_engine* e, int32_t levels, int32_t* finished);

/* Slots that finished in the last step (their rows in rows_out are final).
 * Returns how many were written to `slots`. */
int32_t lbg_engine_finished(const lbg_engine* e, int32_t* slots, int32_t max_slots);

/* Return a finished slot to the pool (its row may then be reused). */
int lbg_engine_release(lbg_engine* e, int32_t slot);

/* Cumulative stats, number of queued + running queries, next level index. */
int lbg_engine_info(const lbg_engine* e, lbg_stats* stats, int32_t* running, uint32_t* level);

/* Wait for the engine's stream and free the handle and its pinned host
 * buffers (not the caller's graph, rows or workspace).  NULL is a no-op. */
void lbg_engine_destroy(lbg_engine* e);

/* Tile of edges one workgroup of the balanced expansion processes (the
 * granularity of the workload decomposition), and the persistent grid size
 * used on the current device.  For reporting and tests. */
int32_t lbg_tile_edges(void);
int32_t lbg_grid_blocks(void);

#ifdef __cplusplus
}
#endif
#endif
