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
constexpr int kItems = 4;                // edges per thread per tile (balanced)
constexpr int kTile = kBlock * kItems;   // edges per tile
constexpr int kQueue = 256;              // per-wave LDS push-queue entries

// Control block at the start of the workspace.  ctr[] are the worklist tail
// counters of three consecutive levels, packed as (nodes << 32) | edges so a
// single 64-bit atomic reserves node slots and the matching range of the
// next level's edge space at once (the edge prefix of Section III-A built at
// push time, with no separate scan).
struct Ctl {
  unsigned long long ctr[3];
  unsigned int error;         // capacity/bounds guards, see kErr* in lbg_kernels.hpp
  unsigned int levels;        // number of non-empty frontiers so far
  unsigned long long frontier_entries;
  unsigned long long edges_scanned;
  unsigned long long updates;
  unsigned int csr_flags;     // lbg_validate_csr findings
  unsigned int pad[5];
};

// One worklist (frontier) buffer.  For node worklists entry i holds the node,
// the position of its first edge in this level's edge space (strictly
// increasing in i because every stored node has out-degree >= 1) and the CSR
// offset of its first arc.  tile_node[t] is the entry whose edge range holds
// edge t * kTile: the per-tile NodeOffset of the workload decomposition.
// Edge worklists (edge-based strategy) use `node` as the list of arc ids.
struct Frontier {
  int32_t* node;
  uint32_t* eprefix;
  int32_t* estart;
  int32_t* tile_node;
};

struct KArgs {
  const int32_t* offsets;
  const int32_t* cols;
  const uint32_t* weights;
  const int32_t* coo_src;
  int32_t* levels;       // BFS output
  uint32_t* dist;        // SSSP output
  uint32_t* visited;     // BFS: one bit per node
  uint32_t* stamp;       // SSSP: last level a node was queued for
  Frontier fr[2];
  Ctl* ctl;
  uint32_t n;
  uint32_t m;
  uint32_t node_cap;     // entries per node worklist
  uint32_t tile_cap;     // entries per tile_node array
  uint32_t edge_cap;     // entries per edge worklist
  uint32_t count_updates;
};

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
  template <bool kMarks>
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
            uint32_t t = (p + kTile - 1) / kTile;
            const uint32_t end = p + static_cast<uint32_t>(d);
            for (; t * static_cast<unsigned long long>(kTile) < end; ++t) {
              if (t < a.tile_cap) out.tile_node[t] = static_cast<int32_t>(i);
              else atomicOr(&a.ctl->error, 2u);  // tile capacity
            }
          }
        } else {
          atomicOr(&a.ctl->error, 1u);  // node capacity
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
          atomicOr(&a.ctl->error, 4u);  // edge capacity
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

}  // namespace lbg
