// Frontier-expansion kernels for level-synchronous BFS and SSSP on gfx950.
//
// One launch processes one level (BFS) or one Bellman-Ford iteration (SSSP):
// it consumes worklist L (buffer L & 1, tail counter ctr[L % 3]), appends to
// worklist L+1 (buffer (L+1) & 1, counter ctr[(L+1) % 3]) and clears
// ctr[(L+2) % 3] for the launch after it.  Launches read their work size
// from device memory, so the host can enqueue many levels without waiting;
// a launch that finds an empty worklist returns at once.
//
// Relaxation (Section II-B): BFS claims an undiscovered node with an atomic
// OR on a visited bitmap (n/8 bytes, small enough to stay in each XCD's L2)
// and the winner writes level L+1; SSSP does alt = dist[u] + w, a plain read
// to skip hopeless arcs, then atomicMin, and queues an improved node once
// per iteration through an atomicExch on its stamp (the worklist condensing
// concern of Section II-B handled at push time).  Plain reads may be stale
// inside a launch; values only move one way (bits set, distances decrease),
// so a stale read can only cause an extra atomic, never a missed update.
#pragma once

#include "lbg_device.hpp"

namespace lbg {

constexpr uint32_t kBfsInf = 0x7fffffffu;
constexpr uint32_t kSsspInf = 0xffffffffu;

// Ctl::error bits.  None can trip for a well-formed CSR; they turn what
// would otherwise be an out-of-bounds access into an LBG_EOVERFLOW return.
constexpr unsigned kErrNodeCap = 1u, kErrTileCap = 2u, kErrEdgeCap = 4u, kErrBadArc = 8u,
                   kErrBadTile = 16u;

// Shared prologue: read this level's worklist size, clear the counter two
// levels ahead, account the level.  Returns the packed (nodes, edges) tail.
__device__ __forceinline__ unsigned long long level_begin(const KArgs& a, uint32_t L) {
  const unsigned long long c = __hip_atomic_load(&a.ctl->ctr[L % 3], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl->ctr[(L + 2) % 3] = 0ull;
    if (static_cast<uint32_t>(c) != 0u) {
      a.ctl->levels = L + 1;
      a.ctl->frontier_entries += (c >> 32) ? (c >> 32) : static_cast<uint32_t>(c);
      a.ctl->edges_scanned += static_cast<uint32_t>(c);
    }
  }
  return c;
}

__device__ __forceinline__ void add_updates(const KArgs& a, uint32_t upd) {
  if (!a.count_updates) return;
  const uint32_t s = wave_sum(upd);
  if (lane_id() == 0 && s) atomicAdd(&a.ctl->updates, static_cast<unsigned long long>(s));
}

// Relax one arc u -> v.  Returns true if v must be queued for the next
// level; then *s / *d receive v's first arc and out-degree.
template <bool kSssp>
__device__ __forceinline__ bool relax(const KArgs& a, uint32_t L, int32_t v, uint32_t du,
                                      uint32_t w, uint32_t* upd, int32_t* s, int32_t* d) {
  if (static_cast<uint32_t>(v) >= a.n) {  // malformed cols (see lbg_validate_csr)
    atomicOr(&a.ctl->error, kErrBadArc);
    return false;
  }
  if (!kSssp) {
    const uint32_t word = static_cast<uint32_t>(v) >> 5;
    const uint32_t bit = 1u << (v & 31);
    if (a.visited[word] & bit) return false;
    if (atomicOr(&a.visited[word], bit) & bit) return false;  // another lane won
    a.levels[v] = static_cast<int32_t>(L + 1);
    ++*upd;
  } else {
    const uint32_t alt = du + w;
    if (alt >= a.dist[v]) return false;
    const uint32_t old = atomicMin(&a.dist[v], alt);
    if (alt >= old) return false;
    ++*upd;
    if (atomicExch(&a.stamp[v], L + 1) == L + 1) return false;  // already queued
  }
  const int32_t s0 = a.offsets[v];
  *s = s0;
  *d = a.offsets[v + 1] - s0;
  return *d > 0;  // a node without out-arcs has nothing to expand
}

// ------------------------------------------------------------------ init --
// Output = infinity, source = 0, visited/stamp cleared, worklist 0 = {src}
// (node strategies) or src's arcs (edge strategy).
template <bool kSssp, bool kEdgeWl>
__global__ __launch_bounds__(kBlock) void k_init(KArgs a, int32_t src) {
  const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t v = gid; v < a.n; v += stride) {
    if (kSssp) {
      a.dist[v] = (v == static_cast<uint32_t>(src)) ? 0u : kSsspInf;
      a.stamp[v] = 0u;
    } else {
      a.levels[v] = (v == static_cast<uint32_t>(src)) ? 0 : static_cast<int32_t>(kBfsInf);
    }
  }
  if (!kSssp) {
    const uint32_t words = (a.n + 31) / 32;
    const uint32_t sw = static_cast<uint32_t>(src) >> 5;
    for (uint32_t w = gid; w < words; w += stride) a.visited[w] = (w == sw) ? (1u << (src & 31)) : 0u;
  }
  const int32_t s0 = a.offsets[src];
  const int32_t d0 = a.offsets[src + 1] - s0;
  if (kEdgeWl) {
    for (uint32_t k = gid; k < static_cast<uint32_t>(d0); k += stride) a.fr[0].node[k] = s0 + k;
  } else {
    const uint32_t tiles = (static_cast<uint32_t>(d0) + kTile - 1) / kTile;
    for (uint32_t t = gid; t < tiles; t += stride) a.fr[0].tile_node[t] = 0;
  }
  if (gid == 0) {
    if (!kEdgeWl) {
      a.fr[0].node[0] = src;
      a.fr[0].eprefix[0] = 0u;
      a.fr[0].estart[0] = s0;
    }
    const unsigned long long nodes = kEdgeWl ? 0ull : 1ull;
    a.ctl->ctr[0] = d0 > 0 ? ((nodes << 32) | static_cast<uint32_t>(d0)) : 0ull;
    a.ctl->ctr[1] = 0ull;
    a.ctl->ctr[2] = 0ull;
    a.ctl->error = 0u;
    a.ctl->levels = 0u;
    a.ctl->frontier_entries = 0ull;
    a.ctl->edges_scanned = 0ull;
    a.ctl->updates = 0ull;
  }
}

// ------------------------------------------------------ balanced (WD) ----
// Workload decomposition (Section III-A): the E_f edges of worklist L are cut
// into tiles of kTile consecutive edges; workgroup b takes tiles b, b + G, ...
// Within a tile, the worklist entries that overlap it are staged in LDS
// (their edge-space start, first arc and, for SSSP, current distance); a
// bitmask of entry starts plus per-word popcount prefixes maps each edge slot
// to its entry in O(1), so lane t of the block handles slots t, t + 256, ...
// and consecutive lanes read consecutive arcs of the same node (coalesced),
// however the degrees are distributed.  Hubs simply span many tiles and are
// expanded by many workgroups at once.
template <bool kSssp>
__global__ __launch_bounds__(kBlock) void k_expand_balanced(KArgs a, uint32_t L) {
  __shared__ uint32_t sP[kTile];
  __shared__ int32_t sS[kTile];
  __shared__ uint32_t sD[kSssp ? kTile : 1];
  __shared__ uint32_t sFlag[kTile / 32];
  __shared__ uint32_t sWpre[kTile / 32];
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
  const Frontier cur = a.fr[L & 1];
  const Frontier nxt = a.fr[(L + 1) & 1];
  const int nctr = (L + 1) % 3;

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63;
  const uint32_t wid = tid >> 6;
  WaveQueue<kSssp> q{qS[wid], qD[wid], qV[kSssp ? wid : 0], 0u};
  auto flush = [&]() { q.template flush_nodes<true>(a, nxt, nctr); };
  uint32_t upd = 0;

  const uint32_t ntiles = (Ef + kTile - 1) / kTile;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t t0 = tile * kTile;
    const uint32_t t1 = min(t0 + static_cast<uint32_t>(kTile), Ef);
    const uint32_t i0 = static_cast<uint32_t>(cur.tile_node[tile]);
    if (i0 >= nf) {  // block-uniform; cannot happen when every tile was marked
      if (tid == 0) atomicOr(&a.ctl->error, kErrBadTile);
      continue;
    }
    for (uint32_t k = tid; k < kTile / 32; k += kBlock) sFlag[k] = 0u;
    __syncthreads();
    // Stage the entries overlapping [t0, t1): a contiguous run starting at i0
    // of at most kTile entries (each holds >= 1 edge).
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = r * kBlock + tid;
      const uint32_t i = i0 + j;
      int valid = 0;
      if (i < nf) {
        const uint32_t p = cur.eprefix[i];
        if (p < t1) {
          valid = 1;
          sP[j] = p;
          sS[j] = cur.estart[i];
          if (kSssp) sD[j] = a.dist[cur.node[i]];
          const uint32_t s = (p > t0 ? p : t0) - t0;
          atomicOr(&sFlag[s >> 5], 1u << (s & 31));
        }
      }
      if (!__syncthreads_or(valid)) break;
    }
    if (wid == 0) {
      const uint32_t x = lane < kTile / 32 ? __popc(sFlag[lane]) : 0u;
      const uint32_t inc = wave_incl_scan(x);
      if (lane < kTile / 32) sWpre[lane] = inc - x;
    }
    __syncthreads();

    int32_t vv[kItems];
    uint32_t ww[kItems];
    uint32_t du[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = t0 + r * kBlock + tid;
      vv[r] = -1;
      if (j < t1) {
        const uint32_t s = j - t0;
        const uint32_t w = s >> 5;
        const uint32_t msk = static_cast<uint32_t>((2ull << (s & 31)) - 1ull);
        const int slot = static_cast<int>(sWpre[w] + __popc(sFlag[w] & msk)) - 1;
        const uint32_t e = slot >= 0 ? static_cast<uint32_t>(sS[slot]) + (j - sP[slot]) : a.m;
        if (e < a.m) {
          vv[r] = a.cols[e];
          if (kSssp) {
            ww[r] = a.weights[e];
            du[r] = sD[slot];
          }
        } else {
          atomicOr(&a.ctl->error, kErrBadArc);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      int32_t s = 0, d = 0;
      const bool want = vv[r] >= 0 && relax<kSssp>(a, L, vv[r], kSssp ? du[r] : 0u,
                                                   kSssp ? ww[r] : 0u, &upd, &s, &d);
      q.push(want, s, d, vv[r], flush);
    }
    __syncthreads();  // LDS descriptors are rewritten by the next tile
  }
  flush();
  add_updates(a, upd);
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
  const Frontier cur = a.fr[L & 1];
  const Frontier nxt = a.fr[(L + 1) & 1];
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x;
  const uint32_t wid = tid >> 6;
  WaveQueue<kSssp> q{qS[wid], qD[wid], qV[kSssp ? wid : 0], 0u};
  auto flush = [&]() { q.template flush_nodes<false>(a, nxt, nctr); };
  uint32_t upd = 0;

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
      if (kSssp) du = a.dist[cur.node[i]];
    }
    const int32_t dmax = wave_max(deg);
    for (int32_t k = 0; k < dmax; ++k) {
      int32_t v = -1, s = 0, d = 0;
      bool want = false;
      if (k < deg) {
        const int32_t e = s0 + k;
        v = a.cols[e];
        want = relax<kSssp>(a, L, v, du, kSssp ? a.weights[e] : 0u, &upd, &s, &d);
      }
      q.push(want, s, d, v, flush);
    }
  }
  flush();
  add_updates(a, upd);
}

// ---------------------------------------------------------- edge (EP) ----
// Edge-based baseline (Section II-B): the worklist holds arc ids; thread i of
// the grid-stride loop relaxes arc wl[i] (SSSP reads its source from the COO
// array); a node whose value improved pushes all of its arcs, reserved with
// one atomic per wave batch (work chunking).
template <bool kSssp>
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
  const int32_t* wl = a.fr[L & 1].node;
  int32_t* nwl = a.fr[(L + 1) & 1].node;
  const int nctr = (L + 1) % 3;
  const uint32_t tid = threadIdx.x;
  const uint32_t wid = tid >> 6;
  WaveQueue<false> q{qS[wid], qD[wid], nullptr, 0u};
  auto flush = [&]() { q.flush_edges(a, nwl, nctr); };
  uint32_t upd = 0;

  for (uint32_t base = blockIdx.x * kBlock; base < cnt; base += gridDim.x * kBlock) {
    const uint32_t i = base + tid;
    int32_t s = 0, d = 0;
    bool want = false;
    if (i < cnt) {
      const int32_t e = wl[i];
      const int32_t v = static_cast<uint32_t>(e) < a.m ? a.cols[e] : -1;
      uint32_t du = 0, w = 0;
      if (kSssp) {
        du = a.dist[a.coo_src[e]];
        w = a.weights[e];
      }
      want = relax<kSssp>(a, L, v, du, w, &upd, &s, &d);
    }
    q.push(want, s, d, 0, flush);
  }
  flush();
  add_updates(a, upd);
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

}  // namespace lbg
