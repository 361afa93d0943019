// Device-side building blocks shared by the frontier-expansion kernels:
// wave64 scans, the per-wave LDS push queue and the argument block.
//
// Target: gfx950 (CDNA4), 64-lane wavefronts, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbg {

constexpr int kBlock = 256;              // threads per workgroup (4 waves)
constexpr int kWaves = kBlock / 64;
constexpr int kQueue = 256;              // per-wave LDS push-queue entries (node/edge kernels)
constexpr int kWQ = 256;                 // per-wave LDS push-queue entries (balanced kernel)

// Balanced kernel: a tile is the run of consecutive edges one wavefront
// expands at a time, 64 lanes x kItems edges.  BFS carries 16 items per lane,
// SSSP (more state per arc) 8.
template <bool kSssp, bool kMulti = false>
struct TileCfg {
  static constexpr int kItems = kMulti ? 4 : (kSssp ? 8 : 16);
  static constexpr uint32_t kEdges = 64u * kItems;
};
constexpr uint32_t kMinTile = TileCfg<true>::kEdges;          // sizes single-query tile marks
constexpr uint32_t kMultiTile = TileCfg<true, true>::kEdges;  // sizes batched tile marks

// Batched solves: one row of node state per query.  row(q, v) = v + delta.
struct QInfo {
  int32_t delta;      // row_start - lo
  int32_t kind;       // 0 = BFS (unit weights, int32 levels out), 1 = SSSP
  int32_t row_start;  // first element of the query's result row
  int32_t row_len;    // hi - lo
  int32_t src;        // global source node
  uint32_t level0;    // level whose worklist received the source (engine admissions)
  int32_t pad[2];
};
constexpr int kXcds = 8;                 // MI355X: 8 XCDs, workgroups dealt round-robin

// Control block at the start of the workspace.  ctr[] are the worklist tail
// counters of three consecutive levels, packed as (nodes << 32) | edges so a
// single 64-bit atomic reserves node slots and the matching range of the
// next level's edge space at once (the edge prefix of Section III-A built at
// push time, with no separate scan).
//
// Counters that many workgroups bump are striped per XCD (one 128-byte line
// each): a single device-wide address serialises atomics (about 12 ns each
// on MI355X), eight independent lines do not.
struct Ctl {
  unsigned long long ctr[3];
  unsigned int error;         // capacity/bounds guards, kErr* below
  unsigned int levels;        // number of non-empty frontiers so far
  unsigned long long frontier_entries;
  unsigned long long edges_scanned;
  unsigned int csr_flags;     // lbg_validate_csr findings
  unsigned int pad0;
  unsigned long long p_frontier_entries;  // the part of the two totals above
  unsigned long long p_edges_scanned;     // done by the small-frontier kernel
  unsigned int deg_max;       // lbg_degree_mdt
  unsigned int level_base;    // graph-launched batches: first level of the next replay
  unsigned int sub_cnt[3];    // hierarchical strategy: sublist sizes of three sub-iterations
  unsigned int pad3;
  unsigned long long scan_levels;  // BFS: bit L set when level L (< 64) ran in scan mode
  unsigned long long pad1[3];
  // [x][0] updates, [x][1] global atomics issued; [x][2], [x][3] the same for
  // levels run by the small-frontier kernel; [x][4 + L % 3] the packed tail
  // (nodes << 32 | edges) of slice x's worklist of level L (destination-
  // sliced strategy); [x][8 + L % 3] the balanced kernel's tile counter of
  // XCD x for level L (single solves)
  unsigned long long xstat[kXcds][16];
};
static_assert(sizeof(Ctl) == 128 + kXcds * 128, "Ctl layout");

// One worklist (frontier) buffer.  For node worklists entry i holds the node,
// the position of its first edge in this level's edge space (strictly
// increasing in i because every stored node has out-degree >= 1) and the CSR
// offset of its first arc.  tile_node[t] is the entry whose edge range holds
// edge t * T (T = the tile size of the kernel that consumes the worklist):
// the per-tile NodeOffset of the workload decomposition.
// Edge worklists (edge-based strategy) use `node` as the list of arc ids.
struct Frontier {
  int32_t* node;
  uint32_t* eprefix;
  int32_t* estart;
  int32_t* tile_node;
  int32_t* qid;  // batched solves: the query an entry belongs to
  uint32_t level;  // index of the level this worklist feeds (set per launch)
};

struct KArgs {
  const int32_t* offsets;
  const int32_t* cols;
  const uint32_t* weights;
  const int32_t* coo_src;
  int32_t* levels;       // BFS output
  uint32_t* dist;        // SSSP output
  uint32_t* visited;     // BFS: one bit per node (set by claim atomics, or by k_bfs_compact for scan levels)
  uint32_t* seen[2];     // BFS: read-only-per-level snapshots of `visited` (double-buffered)
  uint32_t* xfilter;     // BFS: per-XCD advisory copy of `visited`, kXcds x words
  unsigned long long* dstate;  // SSSP: (distance << 32) | iteration of last improvement
  uint16_t* d16;         // SSSP filter per node (batched: per row), min(an upper bound of the distance, 0xffff)
  // Packed arcs (SSSP, balanced): arc e = (cols[e] << wbits) | weights[e],
  // one 32-bit load per arc instead of two.
  const uint32_t* arcs;
  uint32_t wbits;
  Frontier fr[2];
  int32_t* sub[2];       // hierarchical strategy: sublists (worklist indices) of two sub-iterations
  Ctl* ctl;
  uint32_t n;
  uint32_t m;
  uint32_t words;        // (n + 31) / 32
  uint32_t node_cap;     // entries per node worklist
  uint32_t tile_cap;     // entries per tile_node array
  uint32_t edge_cap;     // entries per edge worklist
  uint32_t count_stats;
  // BFS single solves on the balanced strategy: a level of at least scan_min
  // arcs runs in scan mode (no claim atomics, no pushes; k_bfs_compact
  // builds the next worklist from the levels array).  UINT32_MAX: never.
  uint32_t scan_min;
  const QInfo* qtab;     // batched solves
  uint32_t num_queries;
  uint32_t rows;         // batched solves: total elements of node state
  uint32_t* qlast;       // engine: per query, the last level that holds one of its entries
  // Degree-binned strategy: a node with more than `mdt` out-arcs is queued as
  // ceil(deg / mdt) pieces (0 = no splitting); a piece longer than t_block
  // is expanded by a workgroup, longer than t_wave by a wavefront, else by
  // one lane.
  uint32_t mdt, t_wave, t_block;
  // Destination-sliced strategy: the arcs of node u into slice x (nodes
  // [x * slice_nodes, (x + 1) * slice_nodes)) are soff[8u + x] ..
  // soff[8u + x + 1] - 1; nodes with at least slice_min arcs are queued per
  // slice, the others in one mixed list (list 8).  Worklist entries and tile
  // marks of list x sit at x * scap / x * stcap of each frontier array.
  const int32_t* soff;
  uint32_t sliced;
  uint32_t scap, stcap;
  uint32_t slice_nodes;
  uint32_t slice_min;
  // Split graph (node splitting with child nodes): offsets covers n parents
  // then the children; the children of parent v are nodes
  // n + child_base[v] .. n + child_base[v + 1] - 1, each holding one piece
  // of v's arcs (null: no split graph).
  const int32_t* child_base;
  // Degree-class ordered copy: the graph's ids are new ids, node_map[v] is
  // the new id of original node v; the source is given and the distances
  // are written in original ids (null: no renaming).
  const int32_t* node_map;
  // Hierarchical strategy: sublist size of sub-iteration s of level L at
  // [L * kHierTraceSubs + s] for L < kHierTraceLevels, s < kHierTraceSubs
  // (null: not recorded).
  uint32_t* hier_trace;
};
constexpr uint32_t kHierTraceLevels = 64, kHierTraceSubs = 256;

// Pieces of a node with d out-arcs under split size mdt, and piece k's
// offset within the node's arcs and length: the first d % p pieces carry one
// arc more (node splitting, Section III-B).
__device__ __forceinline__ uint32_t split_count(uint32_t d, uint32_t mdt) {
  return (mdt != 0u && d > mdt) ? (d + mdt - 1u) / mdt : 1u;
}
__device__ __forceinline__ void split_piece(uint32_t d, uint32_t p, uint32_t k, uint32_t* off,
                                            uint32_t* len) {
  const uint32_t q = d / p, r = d % p;
  *off = k * q + (k < r ? k : r);
  *len = q + (k < r ? 1u : 0u);
}

// Ctl::error bits.  None can trip for a well-formed CSR; they turn what
// would otherwise be an out-of-bounds access into an LBG_EOVERFLOW return.
// kErrBadSrc: the source, after renaming through node_map, is outside
// [0, n) (a new-id table that does not belong to the graph); kErrBadSplit: a
// split graph's child table names a child outside the graph or a child piece
// without arcs (tables that did not come from lbg_split_graph).
constexpr unsigned kErrNodeCap = 1u, kErrTileCap = 2u, kErrEdgeCap = 4u, kErrBadArc = 8u,
                   kErrBadTile = 16u, kErrBadSrc = 32u, kErrBadSplit = 64u;

// Address of element idx of an array.  With kNarrow the byte offset is
// formed in 32 bits, so the access is a uniform (SGPR) base plus a 32-bit
// VGPR offset: one VGPR per address instead of two and no 64-bit address
// arithmetic, which matters with 16 loads in flight per lane.  Valid when
// every array the kernel touches is below 4 GiB (n < 2^29, m < 2^30); the
// host picks the wide form otherwise.
// 16-bit distance filter: any value stored is at least the node's current
// distance (values only decrease); 0xffff carries no information.
constexpr uint32_t kF16None = 0xffffu;
__device__ __forceinline__ uint32_t f16_bound(uint16_t f) { return f < kF16None ? f : 0xffffffffu; }
__device__ __forceinline__ uint16_t f16_of(uint32_t d) { return static_cast<uint16_t>(d < kF16None ? d : kF16None); }

template <bool kNarrow, typename T>
__device__ __forceinline__ T* at(T* base, uint32_t idx) {
  if constexpr (kNarrow)
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) +
                                static_cast<uint32_t>(idx * static_cast<uint32_t>(sizeof(T))));
  else
    return base + idx;
}
template <bool kNarrow, typename T>
__device__ __forceinline__ const T* at(const T* base, uint32_t idx) {
  if constexpr (kNarrow)
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                      static_cast<uint32_t>(idx * static_cast<uint32_t>(sizeof(T))));
  else
    return base + idx;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= static_cast<uint32_t>(d)) x += y;
  }
  return x;
}

__device__ __forceinline__ int32_t wave_max(int32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int32_t y = __shfl_xor(x, d, 64);
    x = x > y ? x : y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int src_lane) {
  const uint32_t lo = __shfl(static_cast<uint32_t>(v), src_lane, 64);
  const uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src_lane, 64);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// Per-wave push queue in LDS.  push() and flush() must be reached by all 64
// lanes (convergent); `count` is wave-uniform.  Entries are (first arc,
// out-degree, node).  A flush reserves node slots and edge space for the
// whole batch with one 64-bit atomic (the work-chunked push of Section II-B,
// aggregated over a wave), so worklist tails see one atomic per up to
// kQueue pushes instead of one per push.
template <bool kWithNode>
struct WaveQueue {
  int32_t* qs;
  int32_t* qd;
  int32_t* qv;
  uint32_t count;

  // Node worklist flush: writes node / eprefix / estart and, if kMarks, the
  // tile_node marks of every tile whose first edge falls in an entry.
  template <bool kMarks, uint32_t kTileE = kMinTile>
  __device__ __forceinline__ void flush_nodes(const KArgs& a, Frontier out, int ctr_idx) {
    if (count == 0) return;
    const uint32_t lane = lane_id();
    uint32_t pre[kQueue / 64];
    uint32_t carry = 0;
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      const uint32_t d = k < count ? static_cast<uint32_t>(qd[k]) : 0u;
      const uint32_t inc = wave_incl_scan(d);
      pre[r] = carry + inc - d;
      carry += __shfl(inc, 63, 64);
    }
    unsigned long long base = 0;
    if (lane == 0)
      base = atomicAdd(&a.ctl->ctr[ctr_idx],
                       (static_cast<unsigned long long>(count) << 32) | carry);
    base = bcast64(base, 0);
    const uint32_t nb = static_cast<uint32_t>(base >> 32);
    const uint32_t eb = static_cast<uint32_t>(base);
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      if (k < count) {
        const uint32_t i = nb + k;
        const uint32_t p = eb + pre[r];
        const int32_t d = qd[k];
        if (i < a.node_cap) {
          if (kWithNode) out.node[i] = qv[k];
          out.eprefix[i] = p;
          out.estart[i] = qs[k];
          if (kMarks) {
            uint32_t t = (p + kTileE - 1) / kTileE;
            const uint32_t end = p + static_cast<uint32_t>(d);
            for (; t * static_cast<unsigned long long>(kTileE) < end; ++t) {
              if (t < a.tile_cap) out.tile_node[t] = static_cast<int32_t>(i);
              else atomicOr(&a.ctl->error, kErrTileCap);
            }
          }
        } else {
          atomicOr(&a.ctl->error, kErrNodeCap);
        }
      }
    }
    count = 0;
  }

  // Node worklist flush with node splitting: a queued node of degree d is
  // written as split_count(d, a.mdt) entries (node, first arc of the piece,
  // edge prefix), reserved with the same single packed atomic.
  __device__ __forceinline__ void flush_split(const KArgs& a, Frontier out, int ctr_idx) {
    if (count == 0) return;
    const uint32_t lane = lane_id();
    uint32_t pre_n[kQueue / 64], pre_e[kQueue / 64];
    uint32_t cn = 0, ce = 0;
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      const uint32_t d = k < count ? static_cast<uint32_t>(qd[k]) : 0u;
      const uint32_t pc = k < count ? split_count(d, a.mdt) : 0u;
      const uint32_t in = wave_incl_scan(pc), ie = wave_incl_scan(d);
      pre_n[r] = cn + in - pc;
      pre_e[r] = ce + ie - d;
      cn += __shfl(in, 63, 64);
      ce += __shfl(ie, 63, 64);
    }
    unsigned long long base = 0;
    if (lane == 0)
      base = atomicAdd(&a.ctl->ctr[ctr_idx], (static_cast<unsigned long long>(cn) << 32) | ce);
    base = bcast64(base, 0);
    const uint32_t nb = static_cast<uint32_t>(base >> 32);
    const uint32_t eb = static_cast<uint32_t>(base);
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      if (k < count) {
        const uint32_t d = static_cast<uint32_t>(qd[k]);
        const uint32_t pc = split_count(d, a.mdt);
        for (uint32_t j = 0; j < pc; ++j) {
          const uint32_t i = nb + pre_n[r] + j;
          uint32_t off, len;
          split_piece(d, pc, j, &off, &len);
          if (i < a.node_cap) {
            if (kWithNode) out.node[i] = qv[k];
            out.eprefix[i] = eb + pre_e[r] + off;
            out.estart[i] = qs[k] + static_cast<int32_t>(off);
          } else {
            atomicOr(&a.ctl->error, kErrNodeCap);
          }
        }
      }
    }
    count = 0;
  }

  // Edge worklist flush: every queued node contributes all of its arc ids
  // (one reservation for the whole batch; Section II-B work chunking).
  __device__ __forceinline__ void flush_edges(const KArgs& a, int32_t* out, int ctr_idx) {
    if (count == 0) return;
    const uint32_t lane = lane_id();
    uint32_t pre[kQueue / 64];
    uint32_t carry = 0;
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      const uint32_t d = k < count ? static_cast<uint32_t>(qd[k]) : 0u;
      const uint32_t inc = wave_incl_scan(d);
      pre[r] = carry + inc - d;
      carry += __shfl(inc, 63, 64);
    }
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&a.ctl->ctr[ctr_idx], static_cast<unsigned long long>(carry));
    base = bcast64(base, 0);
    const uint32_t eb = static_cast<uint32_t>(base);
#pragma unroll
    for (int r = 0; r < kQueue / 64; ++r) {
      const uint32_t k = r * 64 + lane;
      if (k < count) {
        const uint32_t p = eb + pre[r];
        const int32_t s = qs[k], d = qd[k];
        if (static_cast<unsigned long long>(p) + static_cast<uint32_t>(d) <= a.edge_cap) {
          for (int32_t t = 0; t < d; ++t) out[p + t] = s + t;
        } else {
          atomicOr(&a.ctl->error, kErrEdgeCap);
        }
      }
    }
    count = 0;
  }

  template <typename Flush>
  __device__ __forceinline__ void push(bool want, int32_t s, int32_t d, int32_t v, Flush&& flush) {
    const uint64_t mask = __ballot(want);
    if (mask == 0) return;
    const uint32_t c = static_cast<uint32_t>(__popcll(mask));
    if (count + c > kQueue) flush();
    if (want) {
      const uint32_t k = count + lane_rank(mask);
      qs[k] = s;
      qd[k] = d;
      if (kWithNode) qv[k] = v;
    }
    count += c;
    __builtin_amdgcn_wave_barrier();
  }
};

// ---------------------------------------------------------------------------
// Push path of the balanced kernel.  Each wavefront appends discovered node
// ids to its own LDS queue (no atomic at all: the count is wave-uniform);
// between tiles a queue that is half full is flushed by its wavefront with
// bulk degree reads, a wave scan and ONE packed 64-bit atomic on the worklist
// tail.  At the end of the launch the four queues of a workgroup are merged
// into one reservation, so the tail sees about one atomic per workgroup
// rather than one per wavefront (same-address atomics serialise at ~12 ns).

// Writes worklist entry i (node v of query q, first edge p of the level's
// edge space, first arc s, out-degree d) and marks the tiles whose first edge
// it holds.  kPay: 0 = no node id stored (BFS), 1 = node, 2 = node + query.
template <int kPay, uint32_t kTileE, bool kNarrow>
__device__ __forceinline__ void write_entry(const KArgs& a, const Frontier& out, uint32_t i,
                                            uint32_t p, int32_t v, int32_t q, int32_t s, int32_t d) {
  if (i >= a.node_cap) {
    atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  if (kPay >= 1) *at<kNarrow>(out.node, i) = v;
  if (kPay == 2) {
    *at<kNarrow>(out.qid, i) = q;
    if (a.qlast) a.qlast[q] = out.level;  // same value from every writer: no atomic needed
  }
  *at<kNarrow>(out.eprefix, i) = p;
  *at<kNarrow>(out.estart, i) = s;
  const uint32_t end = p + static_cast<uint32_t>(d);
  for (uint32_t t = (p + kTileE - 1) / kTileE; static_cast<unsigned long long>(t) * kTileE < end; ++t) {
    if (t < a.tile_cap) *at<kNarrow>(out.tile_node, t) = static_cast<int32_t>(i);
    else atomicOr(&a.ctl->error, kErrTileCap);
  }
}

// Split graph: the children of parent v and the arcs they hold in total.  A
// child range that is decreasing or leaves the graph's n + C nodes (node_cap
// = n + C) is flagged and treated as empty.
__device__ __forceinline__ void split_children(const KArgs& a, int32_t v, int32_t* cb, int32_t* ce,
                                               int32_t* arcs) {
  *cb = a.child_base[v];
  *ce = a.child_base[v + 1];
  if (*cb < 0 || *ce < *cb || static_cast<uint32_t>(*ce) > a.node_cap - a.n) {
    atomicOr(&a.ctl->error, kErrBadSplit);
    *ce = *cb = 0;
  }
  *arcs = *ce > *cb ? a.offsets[a.n + *ce] - a.offsets[a.n + *cb] : 0;
}

// Split graph: entries i, i + 1, ... for parent v's own piece (first arc s,
// d arcs; skipped when empty) and then each of its children's pieces, edge
// prefixes from p on.  Every piece carries the parent's id, so a child is
// relaxed with its parent's distance (the parent-to-child propagation).
template <int kPay, uint32_t kTileE, bool kNarrow>
__device__ __forceinline__ void write_split_entries(const KArgs& a, const Frontier& out, uint32_t i,
                                                    uint32_t p, int32_t v, int32_t q, int32_t s,
                                                    int32_t d, int32_t cb, int32_t ce) {
  if (d > 0) {
    write_entry<kPay, kTileE, kNarrow>(a, out, i, p, v, q, s, d);
    ++i;
    p += static_cast<uint32_t>(d);
  }
  for (int32_t c = cb; c < ce; ++c) {
    const int32_t cs = a.offsets[a.n + c];
    const int32_t cl = a.offsets[a.n + c + 1] - cs;
    if (cl <= 0) {
      // the reservation counted this piece: its slot stays unwritten, so the
      // solve must not be trusted (lbg_split_graph never writes such pieces)
      atomicOr(&a.ctl->error, kErrBadSplit);
      continue;
    }
    write_entry<kPay, kTileE, kNarrow>(a, out, i, p, v, q, cs, cl);
    ++i;
    p += static_cast<uint32_t>(cl);
  }
}

// Wave-direct append of the lanes with `act` set (convergent); used when a
// wave queue cannot take a whole push, and to seed batched worklists.
template <int kPay, uint32_t kTileE, bool kNarrow, bool kSplit = false>
__device__ __forceinline__ void wave_append(const KArgs& a, bool act, int32_t v, int32_t q,
                                            const Frontier& out, int ctr_idx) {
  int32_t s = 0, d = 0, cb = 0, ce = 0, ca = 0;
  if (act) {
    s = *at<kNarrow>(a.offsets, v);
    d = *at<kNarrow>(a.offsets, v + 1) - s;
    if (kSplit) split_children(a, v, &cb, &ce, &ca);
  }
  const bool ok = act && (d > 0 || ca > 0);
  const uint64_t mask = __ballot(ok);
  if (mask == 0) return;
  const uint32_t dd = ok ? static_cast<uint32_t>(d + ca) : 0u;
  const uint32_t nn = ok ? static_cast<uint32_t>((d > 0 ? 1 : 0) + (ce - cb)) : 0u;
  const uint32_t inc = wave_incl_scan(dd);
  const uint32_t tot = __shfl(inc, 63, 64);
  const uint32_t inn = kSplit ? wave_incl_scan(nn) : lane_rank(mask) + 1u;
  const uint32_t totn = kSplit ? __shfl(inn, 63, 64) : static_cast<uint32_t>(__popcll(mask));
  unsigned long long base = 0;
  if (lane_id() == 0)
    base = atomicAdd(&a.ctl->ctr[ctr_idx], (static_cast<unsigned long long>(totn) << 32) | tot);
  base = bcast64(base, 0);
  if (ok) {
    const uint32_t i = static_cast<uint32_t>(base >> 32) + (kSplit ? inn - nn : lane_rank(mask));
    const uint32_t p = static_cast<uint32_t>(base) + inc - dd;
    if (kSplit) write_split_entries<kPay, kTileE, kNarrow>(a, out, i, p, v, q, s, d, cb, ce);
    else write_entry<kPay, kTileE, kNarrow>(a, out, i, p, v, q, s, d);
  }
}

// Queue (v, q) if `want` (convergent per wave).  `count` is wave-uniform.
template <int kPay, uint32_t kTileE, bool kNarrow, bool kSplit = false>
__device__ __forceinline__ void wq_push(const KArgs& a, int32_t* qv, int32_t* qq, uint32_t& count,
                                        bool want, int32_t v, int32_t q, const Frontier& out,
                                        int ctr_idx) {
  const uint64_t mask = __ballot(want);
  if (mask == 0) return;
  const uint32_t k = count + lane_rank(mask);
  const bool fits = want && k < static_cast<uint32_t>(kWQ);
  if (fits) {
    qv[k] = v;
    if (kPay == 2) qq[k] = q;
  }
  const uint32_t c = static_cast<uint32_t>(__popcll(mask));
  count = min(count + c, static_cast<uint32_t>(kWQ));
  const bool over = want && !fits;
  if (__ballot(over)) wave_append<kPay, kTileE, kNarrow, kSplit>(a, over, v, q, out, ctr_idx);
  __builtin_amdgcn_wave_barrier();
}

// Split graph: each queued parent's child range and the arcs its children
// hold (empty without a split graph, so the plain flush keeps its layout).
template <bool kOn, int R>
struct SplitKids {
  int32_t cb[R], ce[R], ca[R];
};
template <int R>
struct SplitKids<false, R> {};

// A wave queue's flush, split so a workgroup can merge the reservations of
// its four queues: prepare() reads degrees and scans within the wave,
// write() stores the entries once the base of the reservation is known.
template <int kPay, uint32_t kTileE, bool kNarrow, bool kSplit = false>
struct WaveFlush : SplitKids<kSplit, kWQ / 64> {
  static constexpr int R = kWQ / 64;
  int32_t vs[R], ss[R], ds[R], qs[kPay == 2 ? R : 1];
  uint32_t pn[R], pe[R];
  uint32_t tot_n, tot_e;

  __device__ __forceinline__ void prepare(const KArgs& a, const int32_t* qv, const int32_t* qq,
                                          uint32_t count) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = r * 64 + lane;
      vs[r] = 0;
      ss[r] = 0;
      ds[r] = 0;
      if (kPay == 2) qs[r] = 0;
      if (k < count) {
        vs[r] = qv[k];
        if (kPay == 2) qs[r] = qq[k];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * 64 + lane < count) {
        ss[r] = *at<kNarrow>(a.offsets, vs[r]);
        ds[r] = *at<kNarrow>(a.offsets, vs[r] + 1);
      }
    }
    if constexpr (kSplit) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        this->cb[r] = 0;
        this->ce[r] = 0;
        this->ca[r] = 0;
        if (r * 64 + lane < count) split_children(a, vs[r], &this->cb[r], &this->ce[r], &this->ca[r]);
      }
    }
    uint32_t cn = 0, ce = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ds[r] -= ss[r];
      uint32_t n1 = ds[r] > 0 ? 1u : 0u;
      uint32_t e1 = ds[r] > 0 ? static_cast<uint32_t>(ds[r]) : 0u;
      if constexpr (kSplit) {
        n1 += static_cast<uint32_t>(this->ce[r] - this->cb[r]);
        e1 += static_cast<uint32_t>(this->ca[r]);
      }
      const uint32_t in = wave_incl_scan(n1), ie = wave_incl_scan(e1);
      pn[r] = cn + in - n1;
      pe[r] = ce + ie - e1;
      cn += __shfl(in, 63, 64);
      ce += __shfl(ie, 63, 64);
    }
    tot_n = cn;
    tot_e = ce;
  }

  __device__ __forceinline__ void write(const KArgs& a, const Frontier& out, uint32_t nb,
                                        uint32_t eb) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (kSplit) {
        if (ds[r] > 0 || this->ce[r] > this->cb[r])
          write_split_entries<kPay, kTileE, kNarrow>(a, out, nb + pn[r], eb + pe[r], vs[r],
                                                     kPay == 2 ? qs[kPay == 2 ? r : 0] : 0, ss[r], ds[r],
                                                     this->cb[r], this->ce[r]);
      } else {
        if (ds[r] > 0)
          write_entry<kPay, kTileE, kNarrow>(a, out, nb + pn[r], eb + pe[r], vs[r],
                                             kPay == 2 ? qs[kPay == 2 ? r : 0] : 0, ss[r], ds[r]);
      }
    }
  }

  // Standalone flush by one wavefront.
  __device__ __forceinline__ void flush(const KArgs& a, const int32_t* qv, const int32_t* qq,
                                        uint32_t count, const Frontier& out, int ctr_idx) {
    prepare(a, qv, qq, count);
    if (tot_n == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0)
      base = atomicAdd(&a.ctl->ctr[ctr_idx], (static_cast<unsigned long long>(tot_n) << 32) | tot_e);
    base = bcast64(base, 0);
    write(a, out, static_cast<uint32_t>(base >> 32), static_cast<uint32_t>(base));
  }
};

}  // namespace lbg
