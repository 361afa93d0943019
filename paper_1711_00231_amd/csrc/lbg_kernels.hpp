// Frontier-expansion kernels for level-synchronous BFS and SSSP on gfx950.
//
// One launch processes one level (BFS) or one Bellman-Ford iteration (SSSP):
// it consumes worklist L (buffer L & 1, tail counter ctr[L % 3]), appends to
// worklist L+1 (buffer (L+1) & 1, counter ctr[(L+1) % 3]) and clears
// ctr[(L+2) % 3] for the launch after it.  Launches read their work size
// from device memory, so the host can enqueue many levels without waiting;
// a launch that finds an empty worklist returns at once.
//
// Relaxation (Section II-B).  Device atomics are the scarce resource on
// MI355X (about 27 G/s chip-wide, any scope, against ~250 G/s random L2
// reads), so each path filters with plain reads before it issues one:
//  * BFS claims an undiscovered node with an atomic OR on a visited bitmap.
//    An atomic on a line invalidates that line in every XCD's L2, so the hot
//    path never reads the bitmap it claims through.  It reads one per-XCD
//    advisory filter (n/8 bytes, resident in the XCD's L2) that holds `seen`
//    (a copy of the bitmap frozen for the level, merged in when the level
//    starts) plus the claims of the XCD's own blocks (plain stores), so a
//    visited node costs one L2 read and an XCD issues about one atomic per
//    new node.  The winner writes level L+1 and sets the bit in next level's
//    `seen`, which this launch also refreshes from the current one (plain
//    stores; a bit lost to a racing store only costs one more atomic later).
//  * SSSP keeps (distance << 32 | iteration of last improvement) per node and
//    relaxes with a single 64-bit atomicMin: the returned old value says both
//    whether the arc improved the node and whether the node is already queued
//    for this iteration (the worklist condensing concern of Section II-B is
//    handled at push time, with no second atomic).  The per-arc filter reads
//    a 2-byte copy, min(distance, 0xffff), instead of the 8-byte state (a
//    quarter of the random-read footprint: 8 MiB at scale 22, half of what an
//    XCD's L2 holds); winners refresh it with plain stores, so it may lag the
//    state but never undercuts it, and 0xffff (too large, or unknown) never
//    filters.  Batched SSSP rows keep the same 2-byte copy per row: their
//    state is far larger than the last-level cache, and the copy halves the
//    random-read footprint of filtering on the 4-byte output row (measured:
//    3.5 % faster on 2,048 solves over 322 M arcs).  A frontier node's own
//    distance is always read from the state, and the epilogue writes the
//    output from the state.
// Plain reads may be stale inside a launch; values only move one way (bits
// set, distances decrease), so a stale read can only cost an extra atomic,
// never a missed update.
#pragma once

#include "lbg_device.hpp"

namespace lbg {

constexpr uint32_t kBfsInf = 0x7fffffffu;
constexpr uint32_t kSsspInf = 0xffffffffu;

// Arc e of a single SSSP solve: destination and weight, from the CSR arrays
// or from one packed word.
template <bool kPacked, bool kNarrow>
__device__ __forceinline__ void load_arc(const KArgs& a, uint32_t e, int32_t* v, uint32_t* w) {
  if (kPacked) {
    const uint32_t pa = *at<kNarrow>(a.arcs, e);
    *v = static_cast<int32_t>(pa >> a.wbits);
    *w = pa & ((1u << a.wbits) - 1u);
  } else {
    *v = *at<kNarrow>(a.cols, e);
    *w = *at<kNarrow>(a.weights, e);
  }
}


// Level bookkeeping, by one thread of the grid: clear the counter two levels
// ahead (the one level L+1 appends to) and account level L.  kSmall: the
// level runs in the small-frontier kernel, whose work is also counted apart.
template <bool kSmall = false>
__device__ __forceinline__ void level_account(const KArgs& a, uint32_t L, unsigned long long c) {
  __hip_atomic_store(&a.ctl->ctr[(L + 2) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (static_cast<uint32_t>(c) != 0u) {
    const unsigned long long fe = (c >> 32) ? (c >> 32) : static_cast<uint32_t>(c);
    a.ctl->levels = L + 1;
    a.ctl->frontier_entries += fe;
    a.ctl->edges_scanned += static_cast<uint32_t>(c);
    if (kSmall) {
      a.ctl->p_frontier_entries += fe;
      a.ctl->p_edges_scanned += static_cast<uint32_t>(c);
    }
  }
}

// Shared prologue of the one-level kernels: read this level's worklist size
// and account the level.  Returns the packed (nodes, edges) tail.
__device__ __forceinline__ unsigned long long level_begin(const KArgs& a, uint32_t L) {
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && threadIdx.x == 0) level_account(a, L, c);
  return c;
}

// BFS, at the start of level L: the next level's `seen` snapshot starts as
// this level's (whole grid), and each XCD's advisory filter absorbs this
// level's snapshot (by the XCD's own blocks), so one read of the filter
// answers both "visited before this level" and "claimed by this XCD".
// Plain read-modify-writes: a bit lost to a racing store costs one atomic.
__device__ __forceinline__ void refresh_seen(const KArgs& a, uint32_t L) {
  const uint32_t* cur = a.seen[L & 1];
  uint32_t* nxt = a.seen[(L + 1) & 1];
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < a.words; k += gridDim.x * kBlock)
    nxt[k] = cur[k];
  uint32_t* fx = a.xfilter + static_cast<size_t>(blockIdx.x % kXcds) * a.words;
  const uint32_t xb = blockIdx.x / kXcds, nxb = (gridDim.x - blockIdx.x % kXcds + kXcds - 1) / kXcds;
  for (uint32_t k = xb * kBlock + threadIdx.x; k < a.words; k += nxb * kBlock) {
    const uint32_t sw = cur[k];
    if (sw) fx[k] |= sw;
  }
}

// Block-level reduction of the per-thread counters, then one atomic per
// block on this XCD's stats line.  Must be reached by the whole block.
// skip: arcs of worklist entries passed over without loading them (an SSSP
// node that improved again in the iteration that expands it; its arcs are
// relaxed in the next one), kept in slot 7.
__device__ __forceinline__ void add_stats(const KArgs& a, uint32_t upd, uint32_t atom, uint32_t skip = 0u) {
  if (!a.count_stats) return;  // kernel-argument uniform
  __shared__ uint32_t red[3][kWaves];
  const uint32_t su = wave_sum(upd), sa = wave_sum(atom), sk = wave_sum(skip);
  const uint32_t wid = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[0][wid] = su;
    red[1][wid] = sa;
    red[2][wid] = sk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tu = 0, ta = 0, tk = 0;
    for (int w = 0; w < kWaves; ++w) {
      tu += red[0][w];
      ta += red[1][w];
      tk += red[2][w];
    }
    const int x = blockIdx.x % kXcds;
    if (tu) atomicAdd(&a.ctl->xstat[x][0], tu);
    if (ta) atomicAdd(&a.ctl->xstat[x][1], ta);
    if (tk) atomicAdd(&a.ctl->xstat[x][7], tk);
  }
}

// Relax one arc u -> v.  Returns true if v must be queued for the next
// level; then *s / *d receive v's first arc and out-degree.  *upd counts
// successful improvements/discoveries, *atom the global atomics issued.
template <bool kSssp>
__device__ __forceinline__ bool relax(const KArgs& a, uint32_t L, int32_t v, uint32_t du,
                                      uint32_t w, uint32_t* upd, uint32_t* atom, int32_t* s,
                                      int32_t* d) {
  if (static_cast<uint32_t>(v) >= a.n) {  // malformed cols (see lbg_validate_csr)
    atomicOr(&a.ctl->error, kErrBadArc);
    return false;
  }
  if (!kSssp) {
    const uint32_t word = static_cast<uint32_t>(v) >> 5;
    const uint32_t bit = 1u << (v & 31);
    uint32_t* f = a.xfilter + static_cast<size_t>(blockIdx.x % kXcds) * a.words;  // holds `seen`
    const uint32_t fw = f[word];
    if (fw & bit) return false;  // this XCD already claimed (or is claiming) v
    f[word] = fw | bit;          // plain store; a lost bit only costs one more atomic
    ++*atom;
    if (atomicOr(&a.visited[word], bit) & bit) return false;  // another XCD won
    a.levels[v] = static_cast<int32_t>(L + 1);
    uint32_t* sn = a.seen[(L + 1) & 1];
    sn[word] |= bit;  // plain read-modify-write: a lost bit only costs an atomic later
    ++*upd;
  } else {
    const uint32_t alt = du + w;
    if (alt >= f16_bound(a.d16[v])) return false;
    const unsigned long long mine = (static_cast<unsigned long long>(alt) << 32) | (L + 1);
    ++*atom;
    const unsigned long long old = atomicMin(&a.dstate[v], mine);
    if (alt >= static_cast<uint32_t>(old >> 32)) return false;
    a.d16[v] = f16_of(alt);  // filter; may lag the state, never undercuts it
    ++*upd;
    if (static_cast<uint32_t>(old) == L + 1) return false;  // already queued this iteration
  }
  const int32_t s0 = a.offsets[v];
  *s = s0;
  *d = a.offsets[v + 1] - s0;
  return *d > 0;  // a node without out-arcs has nothing to expand
}

// relax() for kB arcs of one lane at once: each step (filter reads, claims
// or atomic minima, the winners' offsets) is issued for all kB arcs before
// any result is used, so a lane keeps kB requests in flight instead of one.
// v[b] < 0: no arc.  On return want[b] says whether v[b] joins the next
// worklist, with its first arc s[b] and out-degree d[b].
template <bool kSssp, int kB>
__device__ __forceinline__ void relax_batch(const KArgs& a, uint32_t L, int32_t (&v)[kB], const uint32_t (&du)[kB],
                                            const uint32_t (&w)[kB], uint32_t* upd, uint32_t* atom,
                                            int32_t (&s)[kB], int32_t (&d)[kB], bool (&want)[kB]) {
  bool bad = false;
#pragma unroll
  for (int b = 0; b < kB; ++b)
    if (v[b] >= 0 && static_cast<uint32_t>(v[b]) >= a.n) {  // malformed cols (see lbg_validate_csr)
      bad = true;
      v[b] = -1;
    }
  if (bad) atomicOr(&a.ctl->error, kErrBadArc);
  uint32_t x[kB];
  bool win[kB];
  if (!kSssp) {
    uint32_t* f = a.xfilter + static_cast<size_t>(blockIdx.x % kXcds) * a.words;  // holds `seen`
#pragma unroll
    for (int b = 0; b < kB; ++b) x[b] = v[b] >= 0 ? f[static_cast<uint32_t>(v[b]) >> 5] : ~0u;
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t word = static_cast<uint32_t>(v[b]) >> 5, bit = 1u << (v[b] & 31);
      if (v[b] >= 0 && !(x[b] & bit)) {
        f[word] = x[b] | bit;  // plain store; a lost bit only costs one more atomic
        ++*atom;
        x[b] = atomicOr(&a.visited[word], bit);
      } else {
        x[b] = ~0u;
      }
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t word = static_cast<uint32_t>(v[b]) >> 5, bit = 1u << (v[b] & 31);
      win[b] = v[b] >= 0 && !(x[b] & bit);
      if (win[b]) {
        a.levels[v[b]] = static_cast<int32_t>(L + 1);
        a.seen[(L + 1) & 1][word] |= bit;  // plain read-modify-write: a lost bit only costs an atomic later
        ++*upd;
      }
    }
  } else {
#pragma unroll
    for (int b = 0; b < kB; ++b) x[b] = v[b] >= 0 ? f16_bound(a.d16[v[b]]) : 0u;
    unsigned long long old[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t alt = du[b] + w[b];
      old[b] = 0ull;
      if (v[b] >= 0 && alt < x[b]) {
        ++*atom;
        old[b] = atomicMin(&a.dstate[v[b]], (static_cast<unsigned long long>(alt) << 32) | (L + 1));
      }
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t alt = du[b] + w[b];
      const bool better = v[b] >= 0 && alt < x[b] && alt < static_cast<uint32_t>(old[b] >> 32);
      if (better) {
        a.d16[v[b]] = f16_of(alt);  // filter; may lag the state, never undercuts it
        ++*upd;
      }
      win[b] = better && static_cast<uint32_t>(old[b]) != L + 1;  // not yet queued this iteration
    }
  }
#pragma unroll
  for (int b = 0; b < kB; ++b) {
    s[b] = 0;
    d[b] = 0;
    if (win[b]) {
      s[b] = a.offsets[v[b]];
      d[b] = a.offsets[v[b] + 1];
    }
  }
#pragma unroll
  for (int b = 0; b < kB; ++b) {
    d[b] -= s[b];
    want[b] = win[b] && d[b] > 0;  // a node without out-arcs has nothing to expand
  }
}

// ------------------------------------------------------------------ init --
// Output = infinity, source = 0, visited/stamp cleared, worklist 0 = {src}
// (node strategies) or src's arcs (edge strategy).
template <bool kSssp>
__device__ __forceinline__ void init_state(const KArgs& a, int32_t src, uint32_t gid, uint32_t stride) {
  for (uint32_t v = gid; v < a.n; v += stride) {
    if (kSssp) {
      a.dstate[v] = (v == static_cast<uint32_t>(src)) ? 0ull
                                                      : (static_cast<unsigned long long>(kSsspInf) << 32);
      a.dist[v] = (v == static_cast<uint32_t>(src)) ? 0u : kSsspInf;
      a.d16[v] = (v == static_cast<uint32_t>(src)) ? 0 : static_cast<uint16_t>(kF16None);
    } else {
      a.levels[v] = (v == static_cast<uint32_t>(src)) ? 0 : static_cast<int32_t>(kBfsInf);
    }
  }
  if (!kSssp) {
    const uint32_t sw = static_cast<uint32_t>(src) >> 5;
    for (uint32_t w = gid; w < a.words; w += stride) {
      const uint32_t bits = (w == sw) ? (1u << (src & 31)) : 0u;
      a.visited[w] = bits;
      a.seen[0][w] = bits;
      // seen[1] must not carry another solve's bits: level 0 may OR into a
      // word of it before refreshing that word
      a.seen[1][w] = 0u;
    }
    const uint32_t fwords = a.words * kXcds;
    for (uint32_t w = gid; w < fwords; w += stride) a.xfilter[w] = 0u;
  }
  if (gid == 0) {
    a.ctl->error = 0u;
    a.ctl->levels = 0u;
    a.ctl->frontier_entries = 0ull;
    a.ctl->edges_scanned = 0ull;
    a.ctl->p_frontier_entries = 0ull;
    a.ctl->p_edges_scanned = 0ull;
    a.ctl->scan_levels = 0ull;
  }
}

template <bool kSssp, bool kEdgeWl>
__global__ __launch_bounds__(kBlock) void k_init(KArgs a, int32_t src) {
  const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  // the host checked 0 <= src < n; a renaming table is the caller's array
  if (a.node_map) src = a.node_map[src];
  if (static_cast<uint32_t>(src) >= a.n) {
    if (gid == 0) {
      a.ctl->error = kErrBadSrc;
      a.ctl->levels = 0u;
      a.ctl->ctr[0] = a.ctl->ctr[1] = a.ctl->ctr[2] = 0ull;  // every level finds no work
    }
    return;
  }
  init_state<kSssp>(a, src, gid, stride);
  if (a.hier_trace)
    for (uint32_t k = gid; k < kHierTraceLevels * kHierTraceSubs; k += stride) a.hier_trace[k] = 0u;
  const int32_t s0 = a.offsets[src];
  int32_t d0 = a.offsets[src + 1] - s0;
  if (s0 < 0 || d0 < 0 || static_cast<uint32_t>(s0) + static_cast<unsigned long long>(d0) > a.m) {
    if (gid == 0) atomicOr(&a.ctl->error, kErrBadArc);  // malformed offsets: start with no work
    d0 = 0;
  }
  if (kEdgeWl) {
    for (uint32_t k = gid; k < static_cast<uint32_t>(d0); k += stride) a.fr[0].node[k] = s0 + k;
  } else {
    constexpr uint32_t T = TileCfg<kSssp>::kEdges;
    const uint32_t tiles = (static_cast<uint32_t>(d0) + T - 1) / T;
    for (uint32_t t = gid; t < tiles && t < a.tile_cap; t += stride) a.fr[0].tile_node[t] = 0;
  }
  if (!kEdgeWl && a.child_base) {
    // split graph: the source's own piece, then its children's pieces (one
    // thread; tile marks by the thread that owns each tile)
    int32_t cb = a.child_base[src], ce = a.child_base[src + 1];
    if (cb < 0 || ce < cb || static_cast<uint32_t>(ce) > a.node_cap - a.n) {
      if (gid == 0) atomicOr(&a.ctl->error, kErrBadSplit);
      cb = ce = 0;
    }
    if (gid == 0) {
      uint32_t i = 0, p = 0;
      if (d0 > 0) {
        a.fr[0].node[0] = src;
        a.fr[0].eprefix[0] = 0u;
        a.fr[0].estart[0] = s0;
        i = 1;
        p = static_cast<uint32_t>(d0);
      }
      for (int32_t c = cb; c < ce && i < a.node_cap; ++c) {
        const int32_t cs = a.offsets[a.n + c], cl = a.offsets[a.n + c + 1] - cs;
        if (cl <= 0) {  // not a table lbg_split_graph wrote
          atomicOr(&a.ctl->error, kErrBadSplit);
          continue;
        }
        a.fr[0].node[i] = src;
        a.fr[0].eprefix[i] = p;
        a.fr[0].estart[i] = cs;
        ++i;
        p += static_cast<uint32_t>(cl);
      }
      a.ctl->ctr[0] = p > 0 ? ((static_cast<unsigned long long>(i) << 32) | p) : 0ull;
      a.ctl->ctr[1] = 0ull;
      a.ctl->ctr[2] = 0ull;
    }
    // tile t starts in the piece holding edge t * T
    constexpr uint32_t T = TileCfg<kSssp>::kEdges;
    const int32_t tot = d0 + (ce > cb ? a.offsets[a.n + ce] - a.offsets[a.n + cb] : 0);
    const uint32_t tiles = tot > 0 ? (static_cast<uint32_t>(tot) + T - 1) / T : 0u;
    for (uint32_t t = gid; t < tiles && t < a.tile_cap; t += stride) {
      const uint32_t e = t * T;
      uint32_t i = 0, p = 0;
      if (d0 > 0) {
        if (e < static_cast<uint32_t>(d0)) {
          a.fr[0].tile_node[t] = 0;
          continue;
        }
        i = 1;
        p = static_cast<uint32_t>(d0);
      }
      for (int32_t c = cb; c < ce; ++c) {
        const int32_t cl = a.offsets[a.n + c + 1] - a.offsets[a.n + c];
        if (cl <= 0) continue;
        if (e < p + static_cast<uint32_t>(cl)) break;
        ++i;
        p += static_cast<uint32_t>(cl);
      }
      a.fr[0].tile_node[t] = static_cast<int32_t>(i);
    }
    if (gid < kXcds * 16) a.ctl->xstat[gid / 16][gid % 16] = 0ull;
    return;
  }
  // the source's entry (pieces of at most a.mdt arcs for the binned strategy)
  const uint32_t pc = kEdgeWl ? 0u : split_count(static_cast<uint32_t>(d0 > 0 ? d0 : 0), a.mdt);
  for (uint32_t k = gid; k < pc; k += stride) {
    uint32_t off, len;
    split_piece(static_cast<uint32_t>(d0), pc, k, &off, &len);
    a.fr[0].node[k] = src;
    a.fr[0].eprefix[k] = off;
    a.fr[0].estart[k] = s0 + static_cast<int32_t>(off);
  }
  if (gid == 0) {
    const unsigned long long nodes = kEdgeWl ? 0ull : pc;
    a.ctl->ctr[0] = d0 > 0 ? ((nodes << 32) | static_cast<uint32_t>(d0)) : 0ull;
    a.ctl->ctr[1] = 0ull;
    a.ctl->ctr[2] = 0ull;
  }
  if (gid < kXcds * 16) a.ctl->xstat[gid / 16][gid % 16] = 0ull;
}

// SSSP epilogue: once the worklist of the next level to expand (ctl->levels:
// the last non-empty level + 1) is empty, copy the distances out of the
// packed state.  Launched after every step of the level loop; exits at once
// while work remains, so the host needs no extra synchronisation.
__global__ __launch_bounds__(kBlock) void k_sssp_finish(KArgs a) {
  const uint32_t L = __hip_atomic_load(&a.ctl->levels, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  if (static_cast<uint32_t>(c) != 0u) return;
  if (a.sliced) {  // and the 8 slice lists
    for (int x = 0; x < kXcds; ++x)
      if (static_cast<uint32_t>(__hip_atomic_load(&a.ctl->xstat[x][4 + L % 3], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)) != 0u)
        return;
  }
  const uint32_t stride = gridDim.x * kBlock;
  if (a.node_map) {  // distances in original ids
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += stride) {
      const uint32_t u = static_cast<uint32_t>(a.node_map[v]);
      a.dist[v] = u < a.n ? static_cast<uint32_t>(a.dstate[u] >> 32) : kSsspInf;
    }
    return;
  }
  for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += stride)
    a.dist[v] = static_cast<uint32_t>(a.dstate[v] >> 32);
}

// ------------------------------------------------------ balanced (WD) ----
// Workload decomposition (Section III-A): the E_f edges of worklist L are cut
// into tiles of T = 64 x kItems consecutive edges, and global wavefront g
// (of W) takes tiles g, g + W, ...  Within a tile, the worklist entries that
// overlap it are staged in the wavefront's LDS (one word per entry: the arc
// index of the tile's first slot if the entry covered it, plus the entry's
// current distance for SSSP); a bitmask of entry starts with per-word
// popcount prefixes maps each edge slot to its entry in O(1).  Lane l handles
// slots l, l + 64, ..., so the lanes read consecutive arcs of the same node
// (coalesced) whatever the degree distribution; hubs simply span many tiles
// and are expanded by many wavefronts at once.
//
// The kernel is latency-bound unless each round trip carries many
// independent requests, and a workgroup-wide barrier per tile would make
// every tile wait for its slowest wavefront.  So wavefronts run their tiles
// independently (no barrier inside the loop), every phase issues all of a
// lane's kItems loads (or atomics) before consuming any, the next tile's
// start entry is fetched one tile ahead, and discoveries go to per-wave LDS
// queues whose degree reads happen in bulk at flush time.
template <bool kSssp, bool kMulti>
struct WaveLds {
  static constexpr uint32_t T = TileCfg<kSssp, kMulti>::kEdges;
  uint32_t base[T];
  uint32_t du[kSssp ? T : 1];
  int32_t delta[kMulti ? T : 1];
  int32_t lo[kMulti ? T : 1];        // first node of the query's instance
  uint32_t lenkind[kMulti ? T : 1];  // instance size | (kind << 31)
  int32_t qid[kMulti ? T : 1];
  uint32_t flag[T / 32];
  uint32_t wpre[T / 32];
  int32_t qv[kWQ];
  int32_t qq[kMulti ? kWQ : 1];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// kMulti: batched solves (always the SSSP relaxation; BFS queries use unit
// weights).  Entry (q, u) relaxes arc u -> v into row(q, v) = v + delta(q).
// Capacity check of a level's packed (nodes, edges) tail; block-uniform.
template <bool kSssp, bool kMulti>
__device__ __forceinline__ bool level_fits(const KArgs& a, unsigned long long c) {
  constexpr uint32_t T = TileCfg<kSssp, kMulti>::kEdges;
  const uint32_t Ef = static_cast<uint32_t>(c);
  const uint32_t nf = static_cast<uint32_t>(c >> 32);
  return nf <= a.node_cap &&
         Ef <= (kMulti ? static_cast<unsigned long long>(a.tile_cap) * T : static_cast<unsigned long long>(a.m));
}

// One level of the balanced expansion by the whole grid (all threads of
// every block must call it).  c = the level's packed tail, non-empty and
// within capacity.
template <bool kSssp, bool kNarrow, bool kMulti, bool kPacked = false, bool kSplit = false>
__device__ __forceinline__ void expand_level(const KArgs& a, uint32_t L, unsigned long long c) {
  static_assert(!kMulti || kSssp, "batched solves use the SSSP relaxation");
  static_assert(!kPacked || (kSssp && !kMulti), "packed arcs: single SSSP solves");
  constexpr int kItems = TileCfg<kSssp, kMulti>::kItems;
  constexpr uint32_t T = TileCfg<kSssp, kMulti>::kEdges;
  constexpr int kPay = kMulti ? 2 : (kSssp ? 1 : 0);
  __shared__ WaveLds<kSssp, kMulti> lds[kWaves];
  __shared__ uint32_t merge[2 * kWaves];
  __shared__ unsigned long long merge_base;

  const uint32_t Ef = static_cast<uint32_t>(c);
  const uint32_t nf = static_cast<uint32_t>(c >> 32);
  const Frontier cur = a.fr[L & 1];
  Frontier nxt = a.fr[(L + 1) & 1];
  nxt.level = L + 1;
  const int nctr = (L + 1) % 3;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wid = threadIdx.x >> 6;
  WaveLds<kSssp, kMulti>& w = lds[wid];
  uint32_t* fx = a.xfilter + static_cast<size_t>(blockIdx.x % kXcds) * a.words;
  uint32_t* seen_nxt = a.seen[(L + 1) & 1];
  // A frontier node's own distance comes from the packed state
  // (authoritative); the per-arc filter reads the 2-byte copy.
  const uint32_t state_len = kMulti ? a.rows : a.n;
  uint32_t upd = 0, atom = 0, qcount = 0, skip = 0;
  // BFS scan mode (see k_bfs_compact): grid-uniform.  A scan level needs no
  // snapshot refresh: k_bfs_prep already merged `visited` into every XCD's
  // filter, and the compaction rewrites the next snapshot from the levels.
  const bool scan = !kSssp && !kMulti && !kSplit && Ef >= a.scan_min;
  if (!kSssp && !scan) refresh_seen(a, L);

  const uint32_t ntiles = (Ef + T - 1) / T;
  const uint32_t W = gridDim.x * kWaves;
  // Tile deal.  Tiles [0, S) go round-robin to the W wavefronts (tile g,
  // g + W, ...); single solves take the last eighth from per-XCD counters
  // (XCD x hands out S + x, S + x + 8, ...), so a wavefront that drew cheap
  // tiles (skipped entries, few winners) takes more at the end instead of
  // waiting at the workgroup's final barrier for its slowest sibling.  A
  // larger dynamic share loses: hundreds of wavefronts then queue on each
  // counter (measured on R-MAT 22: an eighth dynamic, BFS 2 % and SSSP 2.4 %
  // faster than all round-robin; a quarter 1 %; half or all, SSSP 4-11 %
  // slower).  The first round is always round-robin, so levels of at most
  // W tiles take no atomic.  The counters of level L are
  // ctl->xstat[x][8 + L % 3], cleared by launch L - 1 (or by the
  // small-frontier kernel that ran level L - 1, or by k_init).
  const bool dyn = !kMulti && gridDim.x >= static_cast<uint32_t>(kXcds);
  const uint32_t S = (dyn && ntiles > W) ? max(W, (ntiles - ntiles / 8) / W * W) : ntiles;
  const uint32_t xcd = blockIdx.x % kXcds;
  unsigned long long* const dctr = &a.ctl->xstat[xcd][8 + L % 3];
  if (dyn && blockIdx.x < static_cast<uint32_t>(kXcds) && threadIdx.x == 0)
    a.ctl->xstat[blockIdx.x][8 + (L + 1) % 3] = 0ull;
  auto take = [&]() -> uint32_t {  // wave-uniform
    uint32_t k = 0;
    if (lane == 0) k = static_cast<uint32_t>(atomicAdd(dctr, 1ull));
    k = __shfl(k, 0, 64);
    return S + xcd + static_cast<uint32_t>(kXcds) * k;
  };
  uint32_t tile = blockIdx.x * kWaves + wid;
  if (tile >= S) tile = S < ntiles ? take() : ntiles;
  uint32_t i0_next = tile < ntiles ? static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tile)) : 0u;
  uint32_t tnext = ntiles;
  for (; tile < ntiles; tile = tnext) {
    const uint32_t i0 = i0_next;
    // next tile: its mark is fetched now (round-robin) or once the counter
    // has answered, after staging (dynamic)
    const bool rr = tile + W < S;
    tnext = rr ? tile + W : (S < ntiles ? take() : ntiles);
    if (rr) i0_next = static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tnext));
    const uint32_t t0 = tile * T;
    const uint32_t t1 = min(t0 + T, Ef);
    if (i0 >= nf) {  // wave-uniform; cannot happen when every tile was marked
      if (lane == 0) atomicOr(&a.ctl->error, kErrBadTile);
      if (!rr && tnext < ntiles) i0_next = static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tnext));
      continue;
    }
    if (lane < T / 32) w.flag[lane] = 0u;
    wave_sync();
    // Stage the entries overlapping [t0, t1): a contiguous run starting at i0
    // of at most T entries (each holds >= 1 edge).  An entry's reads are
    // issued together.
    bool bad = false;  // malformed input (see lbg_validate_csr): flagged, arc skipped
    bool live = false;  // SSSP: this lane staged an entry that is not skipped
    for (uint32_t j = lane; j < T; j += 64) {
      const uint32_t i = i0 + j;
      bool valid = false;
      if (i < nf) {
        const uint32_t p = *at<kNarrow>(cur.eprefix, i);
        const uint32_t st = static_cast<uint32_t>(*at<kNarrow>(cur.estart, i));
        const int32_t node = kSssp ? *at<kNarrow>(cur.node, i) : 0;
        const int32_t q = kMulti ? *at<kNarrow>(cur.qid, i) : 0;
        if (p < t1) {
          valid = true;
          w.base[j] = st + t0 - p;  // arc of slot s is base + s (mod 2^32)
          int32_t delta = 0;
          uint32_t level0 = 0;
          if (kMulti) {
            const QInfo qi = a.qtab[q];
            delta = qi.delta;
            level0 = qi.level0;
            w.delta[j] = qi.delta;
            w.lo[j] = qi.row_start - qi.delta;
            w.lenkind[j] = static_cast<uint32_t>(qi.row_len) | (qi.kind ? 0x80000000u : 0u);
            w.qid[j] = q;
          }
          if (kSssp) {
            const uint32_t row = static_cast<uint32_t>(node + delta);
            if (kMulti && !(w.lenkind[j] >> 31)) {
              // BFS query: its frontier nodes are exactly its nodes at hop
              // distance L - level0
              w.du[j] = L - level0;
              live = true;
              if (row >= state_len) {
                w.du[j] = kSsspInf;
                bad = true;
              }
            } else if (row < state_len) {
              // A node that already improved during this launch is queued
              // for the next iteration with a distance at least as good, and
              // its arcs are relaxed there: skip them here (du = infinity
              // marks the entry as skipped).  The state never moves back, so
              // a stale read can only miss a skip, never invent one.
              const unsigned long long sv = *at<kNarrow>(static_cast<const unsigned long long*>(a.dstate), row);
              w.du[j] = static_cast<uint32_t>(sv) == L + 1 ? kSsspInf : static_cast<uint32_t>(sv >> 32);
              live = live || static_cast<uint32_t>(sv) != L + 1;
            } else {
              w.du[j] = kSsspInf;
              bad = true;
            }
          }
          const uint32_t s = (p > t0 ? p : t0) - t0;
          atomicOr(&w.flag[s >> 5], 1u << (s & 31));
        }
      }
      if (!__any(valid)) break;
    }
    if (!rr && tnext < ntiles) i0_next = static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tnext));
    wave_sync();
    if (kSssp && !__any(live) && !__any(bad)) {
      // every entry of the tile improved again this iteration (a hub queued
      // for the next one, typically): nothing to load, the tile ends here
      skip += (t1 - t0 + 63u - lane) / 64u;  // this lane's share of the tile's slots
      wave_sync();
      continue;
    }
    uint32_t nent;  // entries staged for this tile (wave-uniform)
    {
      const uint32_t x = lane < T / 32 ? __popc(w.flag[lane]) : 0u;
      const uint32_t inc = wave_incl_scan(x);
      if (lane < T / 32) w.wpre[lane] = inc - x;
      nent = __shfl(inc, T / 32 - 1, 64);
    }
    wave_sync();
    // a tile inside one entry (a hub's arcs): every slot maps to entry 0,
    // with no per-slot lookups (measured: SSSP 11 % faster on R-MAT 22;
    // batched solves 1 % faster with this and the skipped-tile exit)
    const bool single = nent == 1u;
    uint32_t b0 = 0, d0 = 0;
    if (single) {
      b0 = w.base[0];
      if (kSssp) d0 = w.du[0];
    }

    // Phase A: the arcs of this lane's kItems slots.
    int32_t vv[kItems];
    uint32_t ww[kItems];
    uint32_t du[kItems];
    int32_t dl[kMulti ? kItems : 1];
    int32_t qd[kMulti ? kItems : 1];
    bool inside[kMulti ? kItems : 1];
    bool bfsq[kMulti ? kItems : 1];  // batched: the slot belongs to a BFS query
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t s = r * 64 + lane;
      vv[r] = -1;
      ww[r] = 0;
      du[r] = 0;
      if (kMulti) {
        dl[kMulti ? r : 0] = 0;
        qd[kMulti ? r : 0] = 0;
        inside[kMulti ? r : 0] = true;
        bfsq[kMulti ? r : 0] = false;
      }
      if (t0 + s < t1) {
        int slot = 0;
        uint32_t e, dslot = d0;
        if (single) {
          e = b0 + s;
        } else {
          const uint32_t k = s >> 5;
          const uint32_t msk = static_cast<uint32_t>((2ull << (s & 31)) - 1ull);
          slot = static_cast<int>(w.wpre[k] + __popc(w.flag[k] & msk)) - 1;
          e = slot >= 0 ? w.base[slot] + s : a.m;
          if (kSssp && slot >= 0) dslot = w.du[slot];
        }
        if (kSssp && slot >= 0 && dslot == kSsspInf) {
          ++skip;  // skipped entry (see staging)
        } else if (e < a.m) {
          if (kPacked) {
            load_arc<true, kNarrow>(a, e, &vv[r], &ww[r]);
          } else {
            vv[r] = *at<kNarrow>(a.cols, e);
          }
          if (kSssp) {
            du[r] = dslot;
            if (kMulti) {
              dl[kMulti ? r : 0] = w.delta[slot];
              qd[kMulti ? r : 0] = w.qid[slot];
              const uint32_t lk = w.lenkind[slot];
              inside[kMulti ? r : 0] =
                  static_cast<uint32_t>(vv[r] - w.lo[slot]) < (lk & 0x7fffffffu);
              bfsq[kMulti ? r : 0] = !(lk >> 31);
              ww[r] = (lk >> 31) ? *at<kNarrow>(a.weights, e) : 1u;
            } else if (!kPacked) {
              ww[r] = *at<kNarrow>(a.weights, e);
            }
          }
        } else {
          bad = true;
        }
      }
    }
    uint32_t row[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      row[r] = static_cast<uint32_t>(vv[r] + (kMulti ? dl[kMulti ? r : 0] : 0));
      if (vv[r] >= 0 && (static_cast<uint32_t>(vv[r]) >= a.n || row[r] >= state_len ||
                         (kMulti && !inside[kMulti ? r : 0]))) {
        bad = true;  // malformed cols, or an arc leaving its query's instance
        vv[r] = -1;
      }
    }
    bool push[kItems];
    if (!kSssp) {
      // Phase B: this XCD's advisory filter, which holds the frozen visited
      // snapshot (merged in at level start) and the XCD's own claims: one
      // random read per arc; phase C: one atomic per surviving candidate.
      uint32_t x[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r) x[r] = vv[r] >= 0 ? *at<kNarrow>(fx, static_cast<uint32_t>(vv[r]) >> 5) : ~0u;
      if (scan) {
        // Scan mode: the filter holds every node reached before this level
        // (k_bfs_prep merged the exact `visited` bitmap into it before the
        // launch), so a clear bit proves the node unreached until now and
        // it gets level L + 1 by a plain store.  Several writers of one
        // node store the same value.  No claim, no push.
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t bit = 1u << (vv[r] & 31);
          if (vv[r] >= 0 && !(x[r] & bit)) {
            *at<kNarrow>(fx, static_cast<uint32_t>(vv[r]) >> 5) = x[r] | bit;  // fewer repeat stores
            *at<kNarrow>(a.levels, vv[r]) = static_cast<int32_t>(L + 1);
          }
          x[r] = ~0u;  // nothing to push
        }
      } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t bit = 1u << (vv[r] & 31);
          const bool cand = vv[r] >= 0 && !(x[r] & bit);
          if (cand) {
            *at<kNarrow>(fx, static_cast<uint32_t>(vv[r]) >> 5) = x[r] | bit;  // a lost bit costs one more atomic
            ++atom;
            x[r] = atomicOr(at<kNarrow>(a.visited, static_cast<uint32_t>(vv[r]) >> 5), bit);
          } else {
            x[r] = ~0u;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        push[r] = vv[r] >= 0 && !(x[r] & (1u << (vv[r] & 31)));
        if (push[r]) {
          *at<kNarrow>(a.levels, vv[r]) = static_cast<int32_t>(L + 1);
          uint32_t* sw = at<kNarrow>(seen_nxt, static_cast<uint32_t>(vv[r]) >> 5);
          *sw |= 1u << (vv[r] & 31);  // a lost bit only costs an atomic later
          ++upd;
        }
      }
    } else {
      // Phase B: filter distances; phase C: one 64-bit atomicMin per
      // improving arc, returning both the old distance and whether the node
      // is already queued for this iteration.  Batched BFS queries instead
      // read and claim their bit in the per-row bitmap (a BFS node is final
      // when first reached), and write the level straight to their row.
      uint32_t cd[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        cd[r] = 0u;
        if (vv[r] >= 0) {
          if (kMulti && bfsq[kMulti ? r : 0]) cd[r] = *at<kNarrow>(static_cast<const uint32_t*>(a.visited), row[r] >> 5);
          else cd[r] = f16_bound(*at<kNarrow>(static_cast<const uint16_t*>(a.d16), row[r]));
        }
      }
      unsigned long long old[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t alt = du[r] + ww[r];
        old[r] = 0ull;
        if (kMulti && bfsq[kMulti ? r : 0]) {
          const uint32_t bit = 1u << (row[r] & 31);
          if (vv[r] >= 0 && !(cd[r] & bit)) {
            ++atom;
            old[r] = atomicOr(at<kNarrow>(a.visited, row[r] >> 5), bit);
          } else {
            old[r] = bit;
          }
        } else if (vv[r] >= 0 && alt < cd[r]) {
          if (kMulti) {
            ++atom;
            old[r] = atomicMin(at<kNarrow>(a.dstate, row[r]),
                               (static_cast<unsigned long long>(alt) << 32) | (L + 1));
          } else {
            // single solves read the state coherently first (the filter is
            // a plain read and may lag other XCDs' improvements) and issue
            // the atomic only when it can still win: contended atomics on
            // popular nodes cost more than the read (measured on R-MAT 22:
            // 37 % fewer atomics, SSSP 2 % faster)
            old[r] = __hip_atomic_load(at<kNarrow>(a.dstate, row[r]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      if (!kMulti) {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t alt = du[r] + ww[r];
          if (vv[r] >= 0 && alt < cd[r] && alt < static_cast<uint32_t>(old[r] >> 32)) {
            ++atom;
            old[r] = atomicMin(at<kNarrow>(a.dstate, row[r]),
                               (static_cast<unsigned long long>(alt) << 32) | (L + 1));
          }
        }
      }
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t alt = du[r] + ww[r];
        if (kMulti && bfsq[kMulti ? r : 0]) {
          const bool won = vv[r] >= 0 && !(static_cast<uint32_t>(old[r]) & (1u << (row[r] & 31)));
          if (won) *at<kNarrow>(a.dist, row[r]) = alt;  // = L + 1, final
          upd += won ? 1u : 0u;
          push[r] = won;
        } else {
          const bool better = vv[r] >= 0 && alt < static_cast<uint32_t>(old[r] >> 32);
          if (better) *at<kNarrow>(a.d16, row[r]) = f16_of(alt);  // filter (see top of file)
          upd += better ? 1u : 0u;
          push[r] = better && static_cast<uint32_t>(old[r]) != L + 1;
        }
      }
    }
    if (__any(bad) && lane == 0) atomicOr(&a.ctl->error, kErrBadArc);
    // Single solves push in groups of four rounds (at most 256 nodes, the
    // wave queue's size); a group that would not fit flushes the queue
    // first, so a push-heavy tile pays one reservation per 256 nodes.
    // Batched tiles (four rounds in all) push directly.
    constexpr int kGroup = kMulti ? kItems : 4;
    static_assert(kItems % kGroup == 0 && 64 * kGroup <= kWQ, "push group must fit the wave queue");
#pragma unroll
    for (int r0 = 0; r0 < kItems; r0 += kGroup) {
      if constexpr (!kMulti) {
        uint32_t P = 0;
#pragma unroll
        for (int r = r0; r < r0 + kGroup; ++r) P += static_cast<uint32_t>(__popcll(__ballot(push[r])));
        if (qcount + P > static_cast<uint32_t>(kWQ)) {
          WaveFlush<kPay, T, kNarrow, kSplit> f;
          f.flush(a, w.qv, w.qq, qcount, nxt, nctr);
          qcount = 0;
          wave_sync();
        }
      }
#pragma unroll
      for (int r = r0; r < r0 + kGroup; ++r)
        wq_push<kPay, T, kNarrow, kSplit>(a, w.qv, w.qq, qcount, push[r], vv[r], kMulti ? qd[kMulti ? r : 0] : 0,
                                          nxt, nctr);
    }
    // (single solves flush only when the next group would not fit)
    if (kMulti && qcount >= kWQ / 2) {
      WaveFlush<kPay, T, kNarrow, kSplit> f;
      f.flush(a, w.qv, w.qq, qcount, nxt, nctr);
      qcount = 0;
    }
    wave_sync();
  }

  // Final flush: one reservation for the whole workgroup.
  WaveFlush<kPay, T, kNarrow, kSplit> f;
  f.prepare(a, w.qv, w.qq, qcount);
  if (lane == 0) {
    merge[wid] = f.tot_n;
    merge[kWaves + wid] = f.tot_e;
  }
  __syncthreads();
  uint32_t pn = 0, pe = 0, tn = 0, te = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    if (static_cast<uint32_t>(k) < wid) {
      pn += merge[k];
      pe += merge[kWaves + k];
    }
    tn += merge[k];
    te += merge[kWaves + k];
  }
  if (threadIdx.x == 0)
    merge_base = tn ? atomicAdd(&a.ctl->ctr[nctr], (static_cast<unsigned long long>(tn) << 32) | te) : 0ull;
  __syncthreads();
  f.write(a, nxt, static_cast<uint32_t>(merge_base >> 32) + pn, static_cast<uint32_t>(merge_base) + pe);
  add_stats(a, upd, atom, skip);
}

template <bool kSssp, bool kNarrow, bool kMulti, bool kPacked = false, bool kSplit = false>
__device__ __forceinline__ void balanced_level(const KArgs& a, uint32_t L) {
  const unsigned long long c = level_begin(a, L);
  if (static_cast<uint32_t>(c) == 0u) return;
  if (!level_fits<kSssp, kMulti>(a, c)) {
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  expand_level<kSssp, kNarrow, kMulti, kPacked, kSplit>(a, L, c);
}

template <bool kSssp, bool kNarrow, bool kMulti = false, bool kPacked = false, bool kSplit = false>
__global__ __launch_bounds__(kBlock) void k_expand_balanced(KArgs a, uint32_t L) {
  balanced_level<kSssp, kNarrow, kMulti, kPacked, kSplit>(a, L);
}

// BFS scan levels.  A level of at least a.scan_min arcs is expanded without
// claims or pushes (expand_level, scan mode): every newly reached node gets
// level L + 1 in the levels array.  This kernel, launched after each
// balanced BFS level, then builds worklist L + 1 from the nodes whose level
// is L + 1 (the worklist of Section II-B, made by a scan of the node states
// instead of by atomic claims; at R-MAT scale 22 a big level issues ~8 M
// claim atomics, at a memory-side rate of ~25 G/s).  Each workgroup takes
// 4096-node chunks: coalesced loads of the chunk's levels and offsets into
// LDS, then thread t handles nodes 16t .. 16t + 15 of the chunk, so a block
// scan gives every new node with out-arcs its place in node order and one
// packed atomic reserves the chunk's entries: the next level reads the CSR
// in order.  `visited` and next level's `seen` snapshot are rewritten from
// the levels (each 32-node word by one thread, plain stores).
// Returns at once after a push-mode level, whose pushes already built
// worklist L + 1.  The host launches it only after levels it allows to scan
// (it passes scan_min = UINT32_MAX to the expansion of any other level), so
// a scan level is always followed by its compaction.
// Before a level that may scan: every XCD's filter absorbs `visited`, which
// is exact (push levels set it with claim atomics, the small-frontier kernel
// too, scan levels by k_bfs_compact's whole-word stores), so in scan mode a
// clear filter bit proves the node unreached before the level and the
// expansion needs no read of the node's level (measured: BFS 2.6 % faster
// on R-MAT 22 than reading it).  Returns at once unless level L scans.
template <bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_bfs_prep(KArgs a, uint32_t L) {
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t Ef = static_cast<uint32_t>(c);
  if (Ef == 0u || Ef < a.scan_min) return;
  const uint32_t total = a.words * kXcds;
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < total; k += gridDim.x * kBlock) {
    const uint32_t v = *at<kNarrow>(a.visited, k % a.words);
    if (v) a.xfilter[k] |= v;
  }
}

constexpr uint32_t kCompactPer = 16;                      // nodes per thread
constexpr uint32_t kCompactChunk = kBlock * kCompactPer;  // nodes per workgroup step
__device__ __forceinline__ uint32_t compact_slot(uint32_t j) { return j + (j >> 4); }  // one pad word per 16

template <bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_bfs_compact(KArgs a, uint32_t L) {
  constexpr uint32_t T = TileCfg<false>::kEdges;
  constexpr uint32_t kSlots = kCompactChunk + kCompactChunk / 16 + 1;
  __shared__ int32_t lvs[kSlots];
  __shared__ int32_t offs[kSlots];
  __shared__ uint32_t wsum[2][kWaves];
  __shared__ unsigned long long base_sh;
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t Ef = static_cast<uint32_t>(c);
  if (Ef == 0u || Ef < a.scan_min || !level_fits<false, false>(a, c)) return;  // push-mode level
  if (blockIdx.x == 0 && threadIdx.x == 0 && L < 64u) atomicOr(&a.ctl->scan_levels, 1ull << L);
  Frontier nxt = a.fr[(L + 1) & 1];
  nxt.level = L + 1;
  const int nctr = (L + 1) % 3;
  uint32_t* seen_nxt = a.seen[(L + 1) & 1];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int32_t want = static_cast<int32_t>(L + 1);
  uint32_t upd = 0;
  for (uint32_t c0 = blockIdx.x * kCompactChunk; c0 < a.n; c0 += gridDim.x * kCompactChunk) {
    // the chunk's levels and offsets (offsets of nodes c0 .. c0 + 4096)
#pragma unroll
    for (uint32_t k = 0; k < kCompactPer; ++k) {
      const uint32_t j = k * kBlock + tid, v = c0 + j;
      lvs[compact_slot(j)] = v < a.n ? *at<kNarrow>(a.levels, v) : 0;
      offs[compact_slot(j)] = v <= a.n ? *at<kNarrow>(a.offsets, v) : 0;
    }
    if (tid == 0) {
      const uint32_t v = c0 + kCompactChunk;
      offs[compact_slot(kCompactChunk)] = v <= a.n ? *at<kNarrow>(a.offsets, v) : 0;
    }
    __syncthreads();
    // this thread's 16 nodes: which are new, their degrees
    const uint32_t j0 = tid * kCompactPer;
    uint32_t newm = 0, reached = 0, cnt = 0, deg = 0;
#pragma unroll
    for (uint32_t k = 0; k < kCompactPer; ++k) {
      const uint32_t j = j0 + k;
      const int32_t lv = lvs[compact_slot(j)];
      if (c0 + j < a.n && lv != static_cast<int32_t>(kBfsInf)) reached |= 1u << k;
      if (c0 + j < a.n && lv == want) {
        newm |= 1u << k;
        const uint32_t d = static_cast<uint32_t>(offs[compact_slot(j + 1)] - offs[compact_slot(j)]);
        cnt += d > 0u ? 1u : 0u;
        deg += d;
      }
    }
    upd += __popc(newm);
    // The chunk's 32-node words of `visited` and of next level's `seen`:
    // every node of level <= L + 1, which is exactly what the levels say
    // now, so the even thread of a pair stores whole words, no read needed.
    const uint32_t pair = static_cast<uint32_t>(__shfl_xor(static_cast<int>(reached), 1, 64));
    if (!(tid & 1u) && c0 + j0 < a.n) {
      const uint32_t word = reached | (pair << 16);
      const uint32_t w = (c0 + j0) >> 5;
      *at<kNarrow>(a.visited, w) = word;
      *at<kNarrow>(seen_nxt, w) = word;
    }
    // block exclusive scan of (entries, arcs) in node order, one reservation
    const uint32_t ic = wave_incl_scan(cnt), ie = wave_incl_scan(deg);
    if (lane == 63) {
      wsum[0][wid] = ic;
      wsum[1][wid] = ie;
    }
    __syncthreads();
    uint32_t pc = ic - cnt, pe = ie - deg, tc = 0, te = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      if (static_cast<uint32_t>(k) < wid) {
        pc += wsum[0][k];
        pe += wsum[1][k];
      }
      tc += wsum[0][k];
      te += wsum[1][k];
    }
    if (tid == 0) base_sh = tc ? atomicAdd(&a.ctl->ctr[nctr], (static_cast<unsigned long long>(tc) << 32) | te) : 0ull;
    __syncthreads();
    const uint32_t nb = static_cast<uint32_t>(base_sh >> 32) + pc;
    uint32_t eb = static_cast<uint32_t>(base_sh) + pe;
    uint32_t i = 0;
#pragma unroll
    for (uint32_t k = 0; k < kCompactPer; ++k) {
      const uint32_t j = j0 + k;
      if (newm & (1u << k)) {
        const int32_t s = offs[compact_slot(j)];
        const int32_t d = offs[compact_slot(j + 1)] - s;
        if (d > 0) {
          write_entry<0, T, kNarrow>(a, nxt, nb + i, eb, static_cast<int32_t>(c0 + j), 0, s, d);
          ++i;
          eb += static_cast<uint32_t>(d);
        }
      }
    }
    __syncthreads();  // LDS reused by the next chunk
  }
  add_stats(a, upd, 0u);
}

// Graph-launched batches: one replay of a graph runs levels level_base + k
// for k = 0 .. K-1, then k_level_advance moves level_base on by K, so the
// same graph, its arguments fixed, serves every replay.
template <bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_expand_batched_graph(KArgs a, uint32_t k) {
  const uint32_t L = __hip_atomic_load(&a.ctl->level_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + k;
  balanced_level<true, kNarrow, true>(a, L);
}

__global__ void k_level_advance(Ctl* ctl, uint32_t K) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->level_base += K;
}

// ------------------------------------------------ small frontiers (a8) ----
// Level loop inside ONE workgroup for small frontiers.  High-diameter graphs
// spend thousands of levels with a few thousand edges each; there a level's
// cost is its chain of dependent memory round trips, not its bandwidth, and
// a one-level launch adds several (tile marks, worklist staging, per-XCD
// filters, the tail reservation, the kernel boundary).  Here the frontier
// stays in LDS and a level is three round trips: the arcs of the frontier,
// one atomic per arc (OR on the visited bitmap / 64-bit min on the packed
// state), then the offsets of the arcs' winners, so a discovered node is
// pushed with its first arc and degree (SSSP adds a coherent read of each
// pushed node's distance).  Slots of the
// level's edge space map to entries through an LDS bitmask of entry starts
// with per-word popcount prefixes.  Pushes also go to the global node list
// of the next worklist, for the case that they outgrow LDS.
//
// The kernel runs levels L0, L0+1, ... and returns when a level is empty,
// after max_levels levels, or when the next level has more than kSmallF
// entries or kSmallE edges; then it writes that level in the one-level
// kernels' worklist format (entries, edge prefix, tile marks, tail counter)
// and the host continues from ctl->levels.  Entry condition (host): level
// L0 has at most kSmallF entries and kSmallE edges.
constexpr int kSmallBlock = 1024;
constexpr int kSmallWaves = kSmallBlock / 64;
constexpr uint32_t kSmallF = 4000;   // frontier entries held in LDS
constexpr uint32_t kSmallE = 16384;  // edges of a level run in this kernel
constexpr uint32_t kSmallW = kSmallE / 32;
constexpr int kSmallU = 4;           // edge slots per thread issued together
constexpr int kSmallC = 4;           // entries per thread per scan chunk

template <bool kSssp>
struct SmallLds {
  uint32_t s[kSmallF];      // current level: first arc of entry i
  uint32_t p[kSmallF];      //   exclusive prefix of the entries' degrees
  uint32_t du[kSssp ? kSmallF : 1];  //   distance of entry i's node
  int32_t nv[kSmallF];      // pushes of this level: node,
  int32_t ns[kSmallF];      //   first arc,
  int32_t nd[kSmallF];      //   out-degree (> 0)
  uint32_t flag[kSmallW];   // bit e: an entry starts at edge slot e
  uint32_t wpre[kSmallW];   // set bits in the words before
  uint32_t wsum[2][kSmallWaves];
  uint32_t ncount;          // pushes so far this level
};

// Exclusive block scan of two counters (kSmallBlock threads).  Returns the
// thread's prefixes; *tn, *te receive the block totals.
template <bool kSssp>
__device__ __forceinline__ void small_scan2(SmallLds<kSssp>& sm, uint32_t xn, uint32_t xe,
                                            uint32_t* pn, uint32_t* pe, uint32_t* tn, uint32_t* te) {
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t in = wave_incl_scan(xn), ie = wave_incl_scan(xe);
  __syncthreads();  // wsum may still be read by a previous scan
  if (lane == 63) {
    sm.wsum[0][wid] = in;
    sm.wsum[1][wid] = ie;
  }
  __syncthreads();
  uint32_t bn = 0, be = 0, an = 0, ae = 0;
  for (int k = 0; k < kSmallWaves; ++k) {
    const uint32_t wn = sm.wsum[0][k], we = sm.wsum[1][k];
    if (static_cast<uint32_t>(k) < wid) {
      bn += wn;
      be += we;
    }
    an += wn;
    ae += we;
  }
  *pn = bn + in - xn;
  *pe = be + ie - xe;
  *tn = an;
  *te = ae;
}

// The `cnt` (> kSmallF) nodes pushed for level L, all with out-arcs, from
// the global list out.node to the one-level worklist format.  Returns the
// level's packed tail.
template <bool kSssp, bool kNarrow>
__device__ __forceinline__ unsigned long long small_overflow(const KArgs& a, SmallLds<kSssp>& sm,
                                                             const Frontier& out, uint32_t cnt) {
  constexpr uint32_t T = TileCfg<kSssp>::kEdges;
  constexpr int kPay = kSssp ? 1 : 0;
  uint32_t base_e = 0;
  for (uint32_t c0 = 0; c0 < cnt; c0 += kSmallBlock * kSmallC) {
    int32_t v[kSmallC], st[kSmallC], dg[kSmallC];
    uint32_t xe = 0;
#pragma unroll
    for (int r = 0; r < kSmallC; ++r) {
      const uint32_t i = c0 + threadIdx.x * kSmallC + r;
      v[r] = i < cnt ? *at<kNarrow>(out.node, i) : -1;
    }
#pragma unroll
    for (int r = 0; r < kSmallC; ++r) {
      st[r] = 0;
      dg[r] = 0;
      if (v[r] >= 0) {
        st[r] = *at<kNarrow>(a.offsets, v[r]);
        dg[r] = *at<kNarrow>(a.offsets, v[r] + 1) - st[r];
        xe += static_cast<uint32_t>(dg[r]);
      }
    }
    uint32_t pn, pe, tn, te;
    small_scan2(sm, 0u, xe, &pn, &pe, &tn, &te);
#pragma unroll
    for (int r = 0; r < kSmallC; ++r) {
      if (v[r] >= 0) {
        write_entry<kPay, T, kNarrow>(a, out, c0 + threadIdx.x * kSmallC + r, base_e + pe, v[r], 0,
                                      st[r], dg[r]);
        pe += static_cast<uint32_t>(dg[r]);
      }
    }
    base_e += te;
  }
  return (static_cast<unsigned long long>(cnt) << 32) | base_e;
}

template <bool kSssp, bool kNarrow, bool kPacked = false>
__global__ __launch_bounds__(kSmallBlock) void k_expand_small(KArgs a, uint32_t L0, uint32_t max_levels) {
  static_assert(!kPacked || kSssp, "packed arcs: SSSP");
  constexpr uint32_t T = TileCfg<kSssp>::kEdges;
  constexpr int kPay = kSssp ? 1 : 0;
  __shared__ SmallLds<kSssp> sm;
  __shared__ uint32_t red[2][kSmallWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63;

  // Level L0 from the one-level worklist format.
  unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L0 % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t nf = static_cast<uint32_t>(c >> 32), E = static_cast<uint32_t>(c);
  if (E == 0u || nf == 0u || nf > kSmallF || E > kSmallE) return;  // the host checked; uniform
  {
    const Frontier f0 = a.fr[L0 & 1];
    for (uint32_t i = tid; i < nf; i += kSmallBlock) {
      sm.s[i] = static_cast<uint32_t>(*at<kNarrow>(f0.estart, i));
      sm.p[i] = *at<kNarrow>(f0.eprefix, i);
      if (kSssp) {
        const int32_t u = *at<kNarrow>(f0.node, i);
        sm.du[i] = static_cast<uint32_t>(__hip_atomic_load(at<kNarrow>(a.dstate, static_cast<uint32_t>(u)),
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32);
      }
    }
  }
  uint32_t upd = 0, atom = 0;
  unsigned long long tot_f = 0, tot_e = 0;  // this launch's levels (thread 0)
  bool bad = false;
  uint32_t L = L0;
  for (;; ++L) {
    if (tid == 0) {
      tot_f += nf;
      tot_e += E;
      sm.ncount = 0u;
    }
    // Entry starts -> bitmask -> per-word prefixes.
    const uint32_t words = (E + 31) / 32;
    for (uint32_t k = tid; k < words; k += kSmallBlock) sm.flag[k] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < nf; i += kSmallBlock) atomicOr(&sm.flag[sm.p[i] >> 5], 1u << (sm.p[i] & 31));
    __syncthreads();
    if (tid < 64) {
      constexpr uint32_t kPer = kSmallW / 64;
      uint32_t x[kPer], t = 0;
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t k = tid * kPer + r;
        x[r] = k < words ? __popc(sm.flag[k]) : 0u;
        t += x[r];
      }
      uint32_t pre = wave_incl_scan(t) - t;
#pragma unroll
      for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t k = tid * kPer + r;
        if (k < words) sm.wpre[k] = pre;
        pre += x[r];
      }
    }
    __syncthreads();

    const Frontier nxt = a.fr[(L + 1) & 1];
    for (uint32_t b0 = 0; b0 < E; b0 += kSmallBlock * kSmallU) {
      int32_t vv[kSmallU];
      uint32_t ww[kSmallU], du[kSmallU];
#pragma unroll
      for (int r = 0; r < kSmallU; ++r) {
        const uint32_t e = b0 + r * kSmallBlock + tid;
        vv[r] = -1;
        ww[r] = 0;
        du[r] = 0;
        if (e < E) {
          const uint32_t k = e >> 5;
          const uint32_t msk = static_cast<uint32_t>((2ull << (e & 31)) - 1ull);
          const uint32_t i = sm.wpre[k] + __popc(sm.flag[k] & msk) - 1;  // entry 0 starts at slot 0
          const uint32_t arc = sm.s[i] + (e - sm.p[i]);
          if (i < nf && arc < a.m) {
            if (kPacked) {
              load_arc<true, kNarrow>(a, arc, &vv[r], &ww[r]);
            } else {
              vv[r] = *at<kNarrow>(a.cols, arc);
              if (kSssp) ww[r] = *at<kNarrow>(a.weights, arc);
            }
            if (kSssp) du[r] = sm.du[i];
          } else {
            bad = true;
          }
        }
      }
      // One atomic per arc.
      bool win[kSmallU];
      int32_t s0[kSmallU], s1[kSmallU];
#pragma unroll
      for (int r = 0; r < kSmallU; ++r) {
        if (vv[r] >= 0 && static_cast<uint32_t>(vv[r]) >= a.n) {
          bad = true;
          vv[r] = -1;
        }
        s0[r] = 0;
        s1[r] = 0;
      }
#pragma unroll
      for (int r = 0; r < kSmallU; ++r) {
        win[r] = false;
        if (vv[r] < 0) continue;
        ++atom;
        if (!kSssp) {
          const uint32_t bit = 1u << (vv[r] & 31);
          const uint32_t old = atomicOr(at<kNarrow>(a.visited, static_cast<uint32_t>(vv[r]) >> 5), bit);
          win[r] = !(old & bit);
        } else {
          const uint32_t alt = du[r] + ww[r];
          const unsigned long long old =
              atomicMin(at<kNarrow>(a.dstate, static_cast<uint32_t>(vv[r])),
                        (static_cast<unsigned long long>(alt) << 32) | (L + 1));
          if (alt < static_cast<uint32_t>(old >> 32)) {
            *at<kNarrow>(a.d16, vv[r]) = f16_of(alt);  // filter of the one-level launches
            ++upd;
            win[r] = static_cast<uint32_t>(old) != L + 1;  // not yet queued this level
          }
        }
      }
      // Offsets of the winners only: the workgroup's CU issues about one
      // random lane access per cycle, and most arcs do not win (measured on
      // the 2048 x 2048 grid without shortcuts: BFS 11 % faster than loading
      // every target's offsets alongside its atomic).
#pragma unroll
      for (int r = 0; r < kSmallU; ++r) {
        if (win[r]) {
          s0[r] = *at<kNarrow>(a.offsets, vv[r]);
          s1[r] = *at<kNarrow>(a.offsets, vv[r] + 1);
        }
      }
#pragma unroll
      for (int r = 0; r < kSmallU; ++r) {
        if (!kSssp && win[r]) {
          *at<kNarrow>(a.levels, vv[r]) = static_cast<int32_t>(L + 1);
          ++upd;
        }
        const int32_t d = s1[r] - s0[r];
        if (win[r] && d > 0) {  // a node without out-arcs has nothing to expand
          const uint32_t k = atomicAdd(&sm.ncount, 1u);  // LDS
          if (k < kSmallF) {
            sm.nv[k] = vv[r];
            sm.ns[k] = s0[r];
            sm.nd[k] = d;
          }
          if (k < a.node_cap) *at<kNarrow>(nxt.node, k) = vv[r];
          else bad = true;
        }
      }
    }
    if (__any(bad) && lane == 0) atomicOr(&a.ctl->error, kErrBadArc);
    __syncthreads();
    // at most one push per node per level, so never above node_cap
    const uint32_t cnt = min(sm.ncount, a.node_cap);
    const uint32_t Ln = L + 1;
    bool stop = false;
    if (cnt == 0u) {
      c = 0ull;
      stop = true;
    } else if (cnt > kSmallF) {
      c = small_overflow<kSssp, kNarrow>(a, sm, nxt, cnt);
      stop = true;
    } else {
      // pushes -> the next level's entries: scan the degrees
      uint32_t d[kSmallC], xe = 0;
#pragma unroll
      for (int r = 0; r < kSmallC; ++r) {
        const uint32_t i = tid * kSmallC + r;
        d[r] = i < cnt ? static_cast<uint32_t>(sm.nd[i]) : 0u;
        xe += d[r];
      }
      uint32_t pn, pe, tn, te;
      small_scan2(sm, 0u, xe, &pn, &pe, &tn, &te);
#pragma unroll
      for (int r = 0; r < kSmallC; ++r) {
        const uint32_t i = tid * kSmallC + r;
        if (i < cnt) {
          sm.s[i] = static_cast<uint32_t>(sm.ns[i]);
          sm.p[i] = pe;
          if (kSssp)
            sm.du[i] = static_cast<uint32_t>(__hip_atomic_load(at<kNarrow>(a.dstate, static_cast<uint32_t>(sm.nv[i])),
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32);
          pe += d[r];
        }
      }
      nf = cnt;
      E = te;
      c = (static_cast<unsigned long long>(nf) << 32) | E;
      if (E > kSmallE || Ln - L0 >= max_levels) {
        __syncthreads();
        for (uint32_t i = tid; i < nf; i += kSmallBlock)
          write_entry<kPay, T, kNarrow>(a, nxt, i, sm.p[i], sm.nv[i], 0, sm.ns[i], sm.nd[i]);
        stop = true;
      }
    }
    if (stop) break;
    __syncthreads();
  }
  // Bookkeeping of every level run here, then the tail of level L + 1 (the
  // next to expand) and a cleared counter for the level after it.
  if (tid == 0) {
    const uint32_t Ln = L + 1;
    a.ctl->levels = Ln;
    a.ctl->frontier_entries += tot_f;
    a.ctl->edges_scanned += tot_e;
    a.ctl->p_frontier_entries += tot_f;
    a.ctl->p_edges_scanned += tot_e;
    __hip_atomic_store(&a.ctl->ctr[Ln % 3], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&a.ctl->ctr[(Ln + 1) % 3], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // the balanced kernel's tile counters of level L + 1 (see expand_level)
  if (tid < static_cast<uint32_t>(kXcds)) a.ctl->xstat[tid][8 + (L + 1) % 3] = 0ull;
  if (a.count_stats) {
    const uint32_t su = wave_sum(upd), sa = wave_sum(atom);
    if (lane == 0) {
      red[0][tid >> 6] = su;
      red[1][tid >> 6] = sa;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long tu = 0, ta = 0;
      for (int w = 0; w < kSmallWaves; ++w) {
        tu += red[0][w];
        ta += red[1][w];
      }
      const int x = blockIdx.x % kXcds;
      atomicAdd(&a.ctl->xstat[x][2], tu);
      atomicAdd(&a.ctl->xstat[x][3], ta);
    }
  }
}

// ---------------------------------------------------------- node (BS) ----
// Node-based baseline (Section II-A): thread i of the grid-stride loop owns
// worklist entry i and walks all of its arcs; a wave runs for as long as its
// highest-degree node, which is the load imbalance the paper measures.
template <bool kSssp>
__global__ __launch_bounds__(kBlock) void k_expand_node(KArgs a, uint32_t L) {
  __shared__ int32_t qS[kWaves][kQueue];
  __shared__ int32_t qD[kWaves][kQueue];
  __shared__ int32_t qV[kSssp ? kWaves : 1][kQueue];

  const unsigned long long c = level_begin(a, L);
  const uint32_t Ef = static_cast<uint32_t>(c);
  const uint32_t nf = static_cast<uint32_t>(c >> 32);
  if (Ef == 0) return;
  if (nf > a.node_cap || Ef > a.m) {
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  if (!kSssp) refresh_seen(a, L);
  const Frontier cur = a.fr[L & 1];
  const Frontier nxt = a.fr[(L + 1) & 1];
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x;
  const uint32_t wid = tid >> 6;
  WaveQueue<kSssp> q{qS[wid], qD[wid], qV[kSssp ? wid : 0], 0u};
  auto flush = [&]() { q.template flush_nodes<false>(a, nxt, nctr); };
  uint32_t upd = 0, atom = 0;

  for (uint32_t base = blockIdx.x * kBlock; base < nf; base += gridDim.x * kBlock) {
    const uint32_t i = base + tid;
    int32_t s0 = 0, deg = 0;
    uint32_t du = 0;
    if (i < nf) {
      const uint32_t p = cur.eprefix[i];
      const uint32_t pn = (i + 1 < nf) ? cur.eprefix[i + 1] : Ef;
      s0 = cur.estart[i];
      deg = static_cast<int32_t>(pn - p);
      if (static_cast<uint64_t>(static_cast<uint32_t>(s0)) + static_cast<uint32_t>(deg) > a.m) {
        atomicOr(&a.ctl->error, kErrBadArc);
        deg = 0;
      }
      if (kSssp) du = static_cast<uint32_t>(a.dstate[cur.node[i]] >> 32);
    }
    const int32_t dmax = wave_max(deg);
    for (int32_t k = 0; k < dmax; ++k) {
      int32_t v = -1, s = 0, d = 0;
      bool want = false;
      if (k < deg) {
        const int32_t e = s0 + k;
        v = a.cols[e];
        want = relax<kSssp>(a, L, v, du, kSssp ? a.weights[e] : 0u, &upd, &atom, &s, &d);
      }
      q.push(want, s, d, v, flush);
    }
  }
  flush();
  add_stats(a, upd, atom);
}

// ------------------------------------------------------ degree bins ----
// Degree-binned expansion: worklist entries are nodes, or pieces of at most
// a.mdt arcs of a hub (split when pushed; Section III-B's node splitting
// applied to worklist entries instead of the graph).  Each workgroup takes
// 256 consecutive entries at a time and bins them by length: pieces longer
// than t_block are expanded one after another by the whole workgroup,
// longer than t_wave by one wavefront each, the rest by their own lane
// (the thread / wavefront / workgroup cooperation of degree-binned
// load balancing).  Lanes of a cooperating group read consecutive arcs.
constexpr uint32_t kMinMdt = 64;  // smallest split size (bounds entries per level)

template <bool kSssp>
__global__ __launch_bounds__(kBlock) void k_expand_binned(KArgs a, uint32_t L) {
  __shared__ int32_t qS[kWaves][kQueue];
  __shared__ int32_t qD[kWaves][kQueue];
  __shared__ int32_t qV[kSssp ? kWaves : 1][kQueue];
  __shared__ uint32_t bs[2][kBlock], bl[2][kBlock], bdu[2][kSssp ? kBlock : 1];
  __shared__ uint32_t bcount[2];

  const unsigned long long c = level_begin(a, L);
  const uint32_t Ef = static_cast<uint32_t>(c);
  const uint32_t nf = static_cast<uint32_t>(c >> 32);
  if (Ef == 0) return;
  if (nf > a.node_cap || Ef > a.m) {
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  if (!kSssp) refresh_seen(a, L);
  const Frontier cur = a.fr[L & 1];
  const Frontier nxt = a.fr[(L + 1) & 1];
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  WaveQueue<kSssp> q{qS[wid], qD[wid], qV[kSssp ? wid : 0], 0u};
  auto flush = [&]() { q.flush_split(a, nxt, nctr); };
  uint32_t upd = 0, atom = 0;

  // relax the arcs [s + k0, s + len) of one entry, k0 + stride*j per lane,
  // kBinB of a lane's arcs at a time (relax_batch); `rounds` is uniform over
  // the lanes that share the entry (wave or workgroup)
  constexpr int kBinB = kSssp ? 4 : 8;  // SSSP: fewer registers per arc in flight (measured)
  auto expand = [&](bool act, uint32_t s, uint32_t len, uint32_t du, uint32_t k0, uint32_t stride,
                    uint32_t rounds) {
    for (uint32_t j0 = 0; j0 < rounds; j0 += kBinB) {
      int32_t v[kBinB], ns[kBinB], nd[kBinB];
      uint32_t w[kBinB], dd[kBinB];
      bool want[kBinB];
#pragma unroll
      for (int b = 0; b < kBinB; ++b) {
        const uint32_t k = k0 + (j0 + b) * stride;
        v[b] = -1;
        w[b] = 0;
        dd[b] = du;
        if (act && j0 + b < rounds && k < len) {
          const uint32_t e = s + k;
          if (e < a.m) {
            v[b] = a.cols[e];
            if (kSssp) w[b] = a.weights[e];
          } else {
            atomicOr(&a.ctl->error, kErrBadArc);
          }
        }
      }
      relax_batch<kSssp, kBinB>(a, L, v, dd, w, &upd, &atom, ns, nd, want);
#pragma unroll
      for (int b = 0; b < kBinB; ++b) q.push(want[b], ns[b], nd[b], v[b], flush);
    }
  };

  for (uint32_t base = blockIdx.x * kBlock; base < nf; base += gridDim.x * kBlock) {
    if (tid < 2) bcount[tid] = 0u;
    __syncthreads();
    const uint32_t i = base + tid;
    uint32_t s = 0, len = 0, du = 0;
    if (i < nf) {
      const uint32_t p = cur.eprefix[i];
      const uint32_t pn = (i + 1 < nf) ? cur.eprefix[i + 1] : Ef;
      s = static_cast<uint32_t>(cur.estart[i]);
      len = pn - p;
      if (static_cast<unsigned long long>(s) + len > a.m) {
        atomicOr(&a.ctl->error, kErrBadArc);
        len = 0;
      }
      if (kSssp) {
        const unsigned long long sv = a.dstate[cur.node[i]];
        // already improved this iteration: relaxed with its better distance next time
        if (static_cast<uint32_t>(sv) == L + 1) len = 0;
        du = static_cast<uint32_t>(sv >> 32);
      }
    }
    // bins: 0 = workgroup, 1 = wavefront, lane otherwise
    const int bin = len > a.t_block ? 0 : (len > a.t_wave ? 1 : 2);
    if (bin < 2) {
      const uint32_t k = atomicAdd(&bcount[bin], 1u);
      bs[bin][k] = s;
      bl[bin][k] = len;
      if (kSssp) bdu[bin][k] = du;
    }
    __syncthreads();
    const uint32_t nb0 = bcount[0], nb1 = bcount[1];
    for (uint32_t k = 0; k < nb0; ++k) {  // workgroup bin, one piece at a time
      const uint32_t l = bl[0][k];
      expand(true, bs[0][k], l, kSssp ? bdu[0][k] : 0u, tid, kBlock, (l + kBlock - 1) / kBlock);
    }
    for (uint32_t k0 = 0; k0 < nb1; k0 += kWaves) {  // wavefront bin
      const uint32_t k = k0 + wid;
      const bool act = k < nb1;
      const uint32_t l = act ? bl[1][k] : 0u;
      const uint32_t r = static_cast<uint32_t>(wave_max(static_cast<int32_t>((l + 63) / 64)));
      expand(act, act ? bs[1][k] : 0u, l, (kSssp && act) ? bdu[1][k] : 0u, lane, 64, r);
    }
    {  // lane bin
      const bool act = bin == 2;
      const uint32_t r = static_cast<uint32_t>(wave_max(static_cast<int32_t>(act ? len : 0u)));
      expand(act, s, len, du, 0, 1, r);
    }
    __syncthreads();
  }
  flush();
  add_stats(a, upd, atom);
}

// -------------------------------------------------- hierarchical (HP) ----
// Hierarchical processing (Section III-C).  Sub-iteration s of a level
// relaxes window [s * mdt, (s + 1) * mdt) of the arcs of every frontier
// node still active, one thread per node; nodes with arcs beyond the window
// form the sublist of sub-iteration s + 1 (appended with one atomic per
// wavefront).  Once a sublist holds fewer than kHierWd nodes, its remaining
// arcs are expanded edge-balanced instead (the hand-over to workload
// decomposition): every block stages the sublist's remaining ranges and
// their prefix in LDS and takes a grid-strided share of the arcs.  The host
// enqueues ceil(maxDegree / mdt) sub-iterations per level; later ones find
// an empty sublist and return.  Sublist counters rotate over three slots:
// sub-iteration s reads sub_cnt[s % 3], appends to sub_cnt[(s + 1) % 3] and
// clears sub_cnt[(s + 2) % 3]; k_hier_reset clears slot 1 before a level.
constexpr uint32_t kHierWd = 1024;

__global__ void k_hier_reset(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->sub_cnt[1] = 0u;
}

template <bool kSssp>
__global__ __launch_bounds__(kBlock) void k_expand_hier(KArgs a, uint32_t L, uint32_t sub, uint32_t mdt) {
  __shared__ int32_t qS[kWaves][kQueue];
  __shared__ int32_t qD[kWaves][kQueue];
  __shared__ int32_t qV[kSssp ? kWaves : 1][kQueue];
  __shared__ uint32_t ws_start[kHierWd], ws_pre[kHierWd], ws_du[kSssp ? kHierWd : 1];
  __shared__ uint32_t wsum[kWaves];

  unsigned long long c;
  if (sub == 0) {
    c = level_begin(a, L);
  } else {
    c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const uint32_t Ef = static_cast<uint32_t>(c);
  const uint32_t nf = static_cast<uint32_t>(c >> 32);
  if (Ef == 0) return;
  if (nf > a.node_cap || Ef > a.m) {
    if (threadIdx.x == 0 && sub == 0) atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  const uint32_t cnt = sub == 0 ? nf
                                : __hip_atomic_load(&a.ctl->sub_cnt[sub % 3], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl->sub_cnt[(sub + 2) % 3] = 0u;
    if (a.hier_trace && cnt && L < kHierTraceLevels && sub < kHierTraceSubs)
      a.hier_trace[L * kHierTraceSubs + sub] = cnt;
  }
  if (cnt == 0) return;
  if (!kSssp && sub == 0) refresh_seen(a, L);
  const Frontier cur = a.fr[L & 1];
  const Frontier nxt = a.fr[(L + 1) & 1];
  const int32_t* in = sub == 0 ? nullptr : a.sub[(sub - 1) & 1];
  int32_t* out = a.sub[sub & 1];
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  WaveQueue<kSssp> q{qS[wid], qD[wid], qV[kSssp ? wid : 0], 0u};
  auto flush = [&]() { q.template flush_nodes<false>(a, nxt, nctr); };
  uint32_t upd = 0, atom = 0, skip = 0;
  const unsigned long long w0 = static_cast<unsigned long long>(sub) * mdt;

  // entry e of the level: first arc, degree and (SSSP) current distance;
  // deg = 0 when it was improved again this iteration (relaxed next time:
  // its arcs from this sub-iteration's window on count as skipped, by the
  // one thread that stages the entry for the grid: count_skip)
  auto entry = [&](uint32_t e, uint32_t* st, uint32_t* deg, uint32_t* du, bool count_skip) {
    const uint32_t p = cur.eprefix[e];
    const uint32_t pn = (e + 1 < nf) ? cur.eprefix[e + 1] : Ef;
    *st = static_cast<uint32_t>(cur.estart[e]);
    *deg = pn - p;
    if (static_cast<unsigned long long>(*st) + *deg > a.m) {
      atomicOr(&a.ctl->error, kErrBadArc);
      *deg = 0;
    }
    *du = 0;
    if (kSssp) {
      const unsigned long long sv = a.dstate[cur.node[e]];
      if (static_cast<uint32_t>(sv) == L + 1) {
        if (count_skip) skip += *deg > w0 ? static_cast<uint32_t>(*deg - w0) : 0u;
        *deg = 0;
      }
      *du = static_cast<uint32_t>(sv >> 32);
    }
  };
  auto relax_push = [&](bool act, uint32_t arc, uint32_t du) {
    int32_t v = -1, ns = 0, nd = 0;
    bool want = false;
    if (act) {
      v = a.cols[arc];
      want = relax<kSssp>(a, L, v, du, kSssp ? a.weights[arc] : 0u, &upd, &atom, &ns, &nd);
    }
    q.push(want, ns, nd, v, flush);
  };

  if (cnt >= kHierWd) {
    // one thread per active node: this sub-iteration's window of its arcs
    for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += gridDim.x * kBlock) {
      const uint32_t i = base + tid;
      uint32_t st = 0, deg = 0, du = 0;
      if (i < cnt) entry(sub == 0 ? i : static_cast<uint32_t>(in[i]), &st, &deg, &du, true);
      const unsigned long long lo = w0 < deg ? w0 : deg;
      const unsigned long long hi = (w0 + mdt) < deg ? (w0 + mdt) : deg;
      const uint32_t len = static_cast<uint32_t>(hi - lo);
      const uint32_t rounds = static_cast<uint32_t>(wave_max(static_cast<int32_t>(len)));
      // the window's arcs, kHierB of this thread's at a time (relax_batch)
      constexpr int kHierB = kSssp ? 4 : 8;
      for (uint32_t k0 = 0; k0 < rounds; k0 += kHierB) {
        int32_t v[kHierB], ns[kHierB], nd[kHierB];
        uint32_t w[kHierB], dd[kHierB];
        bool want[kHierB];
#pragma unroll
        for (int b = 0; b < kHierB; ++b) {
          v[b] = -1;
          w[b] = 0;
          dd[b] = du;
          if (k0 + b < len) {
            const uint32_t arc = st + static_cast<uint32_t>(lo) + k0 + b;
            v[b] = a.cols[arc];
            if (kSssp) w[b] = a.weights[arc];
          }
        }
        relax_batch<kSssp, kHierB>(a, L, v, dd, w, &upd, &atom, ns, nd, want);
#pragma unroll
        for (int b = 0; b < kHierB; ++b) q.push(want[b], ns[b], nd[b], v[b], flush);
      }
      // arcs beyond the window: the node stays active
      const bool more = i < cnt && deg > w0 + mdt;
      const uint64_t mask = __ballot(more);
      if (mask) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(&a.ctl->sub_cnt[(sub + 1) % 3], static_cast<uint32_t>(__popcll(mask)));
        b = __shfl(b, 0, 64);
        if (more) {
          const uint32_t k = b + lane_rank(mask);
          if (k < a.node_cap) out[k] = static_cast<int32_t>(sub == 0 ? i : static_cast<uint32_t>(in[i]));
          else atomicOr(&a.ctl->error, kErrNodeCap);
        }
      }
    }
  } else {
    // hand-over: all remaining arcs of the (< kHierWd) active nodes, balanced
    // (every workgroup stages every entry; workgroup 0 counts the skips)
    uint32_t st = 0, deg = 0, du = 0;
    for (uint32_t j = tid; j < kHierWd; j += kBlock) {
      uint32_t rem = 0, s0 = 0, d0 = 0;
      if (j < cnt) {
        entry(sub == 0 ? j : static_cast<uint32_t>(in[j]), &st, &deg, &du, blockIdx.x == 0);
        rem = deg > w0 ? static_cast<uint32_t>(deg - w0) : 0u;
        s0 = st + static_cast<uint32_t>(deg > w0 ? w0 : deg);
        d0 = du;
      }
      ws_start[j] = s0;
      ws_pre[j] = rem;  // lengths for now, prefix below
      if (kSssp) ws_du[j] = d0;
    }
    __syncthreads();
    // exclusive prefix of the kHierWd lengths (4 per thread)
    uint32_t v[kHierWd / kBlock], tsum = 0;
#pragma unroll
    for (uint32_t r = 0; r < kHierWd / kBlock; ++r) {
      v[r] = ws_pre[tid * (kHierWd / kBlock) + r];
      tsum += v[r];
    }
    const uint32_t inc = wave_incl_scan(tsum);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t before = inc - tsum, total = 0;
    for (uint32_t w = 0; w < kWaves; ++w) {
      if (w < wid) before += wsum[w];
      total += wsum[w];
    }
#pragma unroll
    for (uint32_t r = 0; r < kHierWd / kBlock; ++r) {
      ws_pre[tid * (kHierWd / kBlock) + r] = before;
      before += v[r];
    }
    __syncthreads();
    const uint32_t ne = cnt;  // entries with a range (zero lengths are skipped by the search)
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t rounds = (total + stride - 1) / stride;
    for (uint32_t r = 0; r < rounds; ++r) {
      const uint32_t e = r * stride + blockIdx.x * kBlock + tid;
      bool act = e < total;
      uint32_t arc = 0, d = 0;
      if (act) {
        uint32_t lo = 0, hi = ne;  // last entry with prefix <= e
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (ws_pre[mid] <= e) lo = mid;
          else hi = mid;
        }
        arc = ws_start[lo] + (e - ws_pre[lo]);
        d = kSssp ? ws_du[lo] : 0u;
      }
      relax_push(act, arc, d);
    }
  }
  flush();
  add_stats(a, upd, atom, skip);
}

// ---------------------------------------------------------- edge (EP) ----
// Edge-based baseline (Section II-B): the worklist holds arc ids; thread i of
// the grid-stride loop relaxes arc wl[i] (SSSP reads its source from the COO
// array); a node whose value improved pushes all of its arcs, reserved with
// one atomic per wave batch (work chunking).
//
// kChunk = false is the ablation without work chunking (Section IV-D): an
// improved node reserves each of its arcs with its own atomic on the tail.
template <bool kSssp, bool kChunk>
__global__ __launch_bounds__(kBlock) void k_expand_edge(KArgs a, uint32_t L) {
  __shared__ int32_t qS[kWaves][kQueue];
  __shared__ int32_t qD[kWaves][kQueue];

  const unsigned long long c = level_begin(a, L);
  const uint32_t cnt = static_cast<uint32_t>(c);
  if (cnt == 0) return;
  if (cnt > a.edge_cap) {
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrEdgeCap);
    return;
  }
  if (!kSssp) refresh_seen(a, L);
  const int32_t* wl = a.fr[L & 1].node;
  int32_t* nwl = a.fr[(L + 1) & 1].node;
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x;
  const uint32_t wid = tid >> 6;
  WaveQueue<false> q{qS[wid], qD[wid], nullptr, 0u};
  auto flush = [&]() { q.flush_edges(a, nwl, nctr); };
  uint32_t upd = 0, atom = 0;

  for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += gridDim.x * kBlock) {
    const uint32_t i = base + tid;
    int32_t s = 0, d = 0;
    bool want = false;
    if (i < cnt) {
      const int32_t e = wl[i];
      const int32_t v = static_cast<uint32_t>(e) < a.m ? a.cols[e] : -1;
      uint32_t du = 0, w = 0;
      if (kSssp) {
        du = static_cast<uint32_t>(a.dstate[a.coo_src[e]] >> 32);
        w = a.weights[e];
      }
      want = relax<kSssp>(a, L, v, du, w, &upd, &atom, &s, &d);
    }
    if (kChunk) {
      q.push(want, s, d, 0, flush);
    } else if (want) {
      for (int32_t t = 0; t < d; ++t) {
        const uint32_t p = static_cast<uint32_t>(atomicAdd(&a.ctl->ctr[nctr], 1ull));
        if (p < a.edge_cap) nwl[p] = s + t;
        else atomicOr(&a.ctl->error, kErrEdgeCap);
      }
    }
  }
  flush();
  add_stats(a, upd, atom);
}

// Batched rows.  SSSP rows keep the packed state; BFS rows keep one bit per
// row in the row bitmap (`visited`) and their level in the output row.  Fill
// and finish kernels run a 2-D grid: y walks the queries, x the kRowChunk
// element chunks of a query's row, so a large instance is spread over many
// workgroups.  Bitmap words that a chunk shares with a neighbouring chunk or
// row range are cleared with an atomic AND.
constexpr uint32_t kRowChunk = 4096;

__device__ __forceinline__ void fill_chunk(const KArgs& a, const QInfo& qi, uint32_t c0) {
  const uint32_t r0 = static_cast<uint32_t>(qi.row_start) + c0;
  const uint32_t r1 = static_cast<uint32_t>(qi.row_start) + min(static_cast<uint32_t>(qi.row_len), c0 + kRowChunk);
  for (uint32_t idx = r0 + threadIdx.x; idx < r1; idx += kBlock) {
    if (qi.kind) {
      a.dstate[idx] = static_cast<unsigned long long>(kSsspInf) << 32;
      a.d16[idx] = static_cast<uint16_t>(kF16None);
    }
    a.dist[idx] = kSsspInf;
  }
  if (!qi.kind) {
    const uint32_t w0 = r0 >> 5, w1 = (r1 - 1) >> 5;
    for (uint32_t w = w0 + threadIdx.x; w <= w1; w += kBlock) {
      const uint32_t lo = w == w0 ? (r0 & 31) : 0u;
      const uint32_t hi = w == w1 ? ((r1 - 1) & 31) : 31u;
      const uint32_t m = (hi == 31u ? ~0u : ((2u << hi) - 1u)) & ~((1u << lo) - 1u);
      if (m == ~0u) a.visited[w] = 0u;
      else atomicAnd(&a.visited[w], ~m);
    }
  }
}

__device__ __forceinline__ void finish_chunk(const KArgs& a, const QInfo& qi, uint32_t c0) {
  const uint32_t r0 = static_cast<uint32_t>(qi.row_start) + c0;
  const uint32_t r1 = static_cast<uint32_t>(qi.row_start) + min(static_cast<uint32_t>(qi.row_len), c0 + kRowChunk);
  for (uint32_t idx = r0 + threadIdx.x; idx < r1; idx += kBlock) {
    if (qi.kind) a.dist[idx] = static_cast<uint32_t>(a.dstate[idx] >> 32);
    else if (a.dist[idx] == kSsspInf) a.dist[idx] = kBfsInf;
  }
}

__device__ __forceinline__ void seed_row(const KArgs& a, const QInfo& qi) {
  const uint32_t row = static_cast<uint32_t>(qi.src + qi.delta);
  if (qi.kind) {
    a.dstate[row] = 0ull;
    a.d16[row] = 0;
  } else atomicOr(&a.visited[row >> 5], 1u << (row & 31));
  a.dist[row] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_batch_fill(KArgs a) {
  for (uint32_t q = blockIdx.y; q < a.num_queries; q += gridDim.y) {
    const QInfo qi = a.qtab[q];
    for (uint32_t c0 = blockIdx.x * kRowChunk; c0 < static_cast<uint32_t>(qi.row_len); c0 += gridDim.x * kRowChunk)
      fill_chunk(a, qi, c0);
  }
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    if (threadIdx.x == 0) {
      a.ctl->ctr[0] = a.ctl->ctr[1] = a.ctl->ctr[2] = 0ull;
      a.ctl->error = 0u;
      a.ctl->levels = 0u;
      a.ctl->level_base = 0u;
      a.ctl->frontier_entries = 0ull;
      a.ctl->edges_scanned = 0ull;
    }
    for (uint32_t k = threadIdx.x; k < kXcds * 16; k += kBlock) a.ctl->xstat[k / 16][k % 16] = 0ull;
  }
}

// Each query's source gets distance 0 and (query, source) enters worklist 0.
template <bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_batch_seed(KArgs a) {
  const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
  const bool act = q < a.num_queries;
  int32_t v = 0;
  if (act) {
    const QInfo qi = a.qtab[q];
    v = qi.src;
    seed_row(a, qi);
  }
  Frontier f0 = a.fr[0];
  f0.level = 0;
  wave_append<2, kMultiTile, kNarrow>(a, act, v, static_cast<int32_t>(q), f0, 0);
}

// ------------------------------------------------------------------ engine --
// Continuous batching: queries join a running batch between levels.  Rows of
// the listed slots start at infinity ...
__global__ __launch_bounds__(kBlock) void k_engine_fill(KArgs a, const int32_t* slots, const QInfo* stage,
                                                        QInfo* qtab, int count) {
  for (int k = blockIdx.y; k < count; k += gridDim.y) {
    const QInfo qi = stage[k];
    if (blockIdx.x == 0 && threadIdx.x == 0) qtab[slots[k]] = qi;  // read there by later kernels
    for (uint32_t c0 = blockIdx.x * kRowChunk; c0 < static_cast<uint32_t>(qi.row_len); c0 += gridDim.x * kRowChunk)
      fill_chunk(a, qi, c0);
  }
}

// ... then each source gets distance 0 and joins worklist L, the next one to
// be expanded (appending to it exactly like a push of the previous level).
template <bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_engine_seed(KArgs a, const int32_t* slots, int count,
                                                        uint32_t L) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const bool act = k < count;
  int32_t v = 0, q = 0;
  if (act) {
    q = slots[k];
    const QInfo qi = a.qtab[q];
    v = qi.src;
    seed_row(a, qi);
    a.qlast[q] = L;  // even a source without out-arcs is live until level L ends
  }
  Frontier f = a.fr[L & 1];
  f.level = L;
  wave_append<2, kMultiTile, kNarrow>(a, act, v, q, f, static_cast<int>(L % 3));
}

// Rows of finished slots are written out (as k_batch_finish).
__global__ __launch_bounds__(kBlock) void k_engine_finish(KArgs a, const int32_t* slots, int count) {
  for (int k = blockIdx.y; k < count; k += gridDim.y) {
    const QInfo qi = a.qtab[slots[k]];
    for (uint32_t c0 = blockIdx.x * kRowChunk; c0 < static_cast<uint32_t>(qi.row_len); c0 += gridDim.x * kRowChunk)
      finish_chunk(a, qi, c0);
  }
}

// Once worklist L is empty, each row is written out: SSSP rows as distances,
// BFS rows as int32 levels (INT32_MAX for unreached).  L = UINT32_MAX: the
// level is ctl->level_base (graph-launched batches).
__global__ __launch_bounds__(kBlock) void k_batch_finish(KArgs a, uint32_t L) {
  if (L == 0xffffffffu) L = __hip_atomic_load(&a.ctl->level_base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  if (static_cast<uint32_t>(c) != 0u) return;
  for (uint32_t q = blockIdx.y; q < a.num_queries; q += gridDim.y) {
    const QInfo qi = a.qtab[q];
    for (uint32_t c0 = blockIdx.x * kRowChunk; c0 < static_cast<uint32_t>(qi.row_len); c0 += gridDim.x * kRowChunk)
      finish_chunk(a, qi, c0);
  }
}

// ------------------------------------------------------ MDT histogram --
// Out-degree histogram for the MDT rule of Section III-B: maximum degree,
// then counts of 10 bins of width maxDegree/10 numbered from 1 (bin of
// degree d: max(1, ceil(10 d / maxDegree))), summed per workgroup in LDS and
// added to per-XCD lines (xstat[x][bin - 1]).
constexpr int kMdtBins = 10;

__global__ __launch_bounds__(kBlock) void k_deg_clear(Ctl* ctl) {
  if (threadIdx.x == 0) ctl->deg_max = 0u;
  for (int k = threadIdx.x; k < kXcds * 16; k += kBlock) ctl->xstat[k / 16][k % 16] = 0ull;
}

__global__ __launch_bounds__(kBlock) void k_deg_max(const int32_t* offsets, uint32_t n, Ctl* ctl) {
  uint32_t mx = 0;
  for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
    mx = max(mx, static_cast<uint32_t>(offsets[v + 1] - offsets[v]));
  mx = static_cast<uint32_t>(wave_max(static_cast<int32_t>(mx)));
  if (lane_id() == 0 && mx) atomicMax(&ctl->deg_max, mx);
}

__global__ __launch_bounds__(kBlock) void k_deg_hist(const int32_t* offsets, uint32_t n, Ctl* ctl) {
  __shared__ uint32_t h[kMdtBins];
  if (threadIdx.x < kMdtBins) h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long mx = ctl->deg_max;
  for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
    const unsigned long long d = static_cast<uint32_t>(offsets[v + 1] - offsets[v]);
    unsigned long long b = mx ? (d * kMdtBins + mx - 1) / mx : 1ull;
    if (b < 1) b = 1;
    if (b > kMdtBins) b = kMdtBins;
    atomicAdd(&h[b - 1], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kMdtBins && h[threadIdx.x])
    atomicAdd(&ctl->xstat[blockIdx.x % kXcds][threadIdx.x], static_cast<unsigned long long>(h[threadIdx.x]));
}

// ------------------------------------------------------- CSR validation --
__global__ __launch_bounds__(kBlock) void k_validate(const int32_t* offsets, const int32_t* cols,
                                                     uint32_t n, uint32_t m, Ctl* ctl) {
  const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  uint32_t flags = 0;
  if (gid == 0) {
    if (offsets[0] != 0) flags |= 1u;
    if (offsets[n] != static_cast<int32_t>(m)) flags |= 4u;
  }
  for (uint32_t u = gid; u < n; u += stride)
    if (offsets[u + 1] < offsets[u]) flags |= 2u;
  for (uint32_t e = gid; e < m; e += stride)
    if (cols[e] < 0 || static_cast<uint32_t>(cols[e]) >= n) flags |= 8u;
  if (flags) atomicOr(&ctl->csr_flags, flags);
}

// ------------------------------------------------------- packed arcs --
// Largest weight (into ctl->deg_max), then the packed words
// (cols[e] << wbits) | weights[e].
__global__ __launch_bounds__(kBlock) void k_weight_max(const uint32_t* weights, uint32_t m, Ctl* ctl) {
  uint32_t mx = 0u;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < m; e += gridDim.x * kBlock) mx = max(mx, weights[e]);
  mx = static_cast<uint32_t>(wave_max(static_cast<int32_t>(mx ^ 0x80000000u))) ^ 0x80000000u;  // unsigned max
  if (lane_id() == 0 && mx) atomicMax(&ctl->deg_max, mx);
}

// Source node of every arc (the COO array the edge-based strategy reads,
// Section II-B): wavefront w of the grid writes the arcs of nodes w, w + W,
// ..., 64 consecutive positions per store, so hubs cost many stores of one
// wavefront but every store is coalesced.  Offsets outside [0, m] are
// clamped (lbg_validate_csr first on untrusted input).
__global__ __launch_bounds__(kBlock) void k_coo_sources(const int32_t* offsets, uint32_t n, uint32_t m,
                                                        int32_t* coo) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t W = gridDim.x * kWaves;
  for (uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6); u < n; u += W) {
    const int32_t s0 = offsets[u], s1 = offsets[u + 1];
    const uint32_t b = static_cast<uint32_t>(s0 < 0 ? 0 : s0), e = min(static_cast<uint32_t>(s1 < 0 ? 0 : s1), m);
    for (uint32_t k = b + lane; k < e; k += 64) coo[k] = static_cast<int32_t>(u);
  }
}

__global__ __launch_bounds__(kBlock) void k_pack_arcs(const int32_t* cols, const uint32_t* weights, uint32_t m,
                                                      uint32_t wbits, uint32_t* arcs) {
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < m; e += gridDim.x * kBlock)
    arcs[e] = (static_cast<uint32_t>(cols[e]) << wbits) | weights[e];
}

}  // namespace lbg
