// Node splitting with child nodes (strategy LBG_SPLIT; Section III-B).
//
// A node with more than MDT out-arcs keeps the first of its ceil(deg / MDT)
// pieces and hands the others to child nodes appended after the n original
// ids (the first deg % pieces pieces one arc longer, the parent's first).
// The split graph is a CSR over n + C nodes: parents 0 .. n-1 with their
// own piece, then the children of parent 0, of parent 1, ... in order, so
// the arc array is regrouped once.  Arcs still point at parents only (a
// child is never a destination), and child_base[v] .. child_base[v+1] - 1
// numbers v's children.  During a solve a pushed parent queues its own piece
// and its children's pieces, each entry carrying the parent's id, so the
// children take the parent's distance: the parent-to-child propagation of
// node splitting, done at push time instead of by a separate pass.
//
// Building the split graph: k_split_sums (per-workgroup totals of children,
// own-piece arcs and children's arcs), k_split_scan (exclusive scan of those
// totals, one workgroup), k_split_build (child numbering and split offsets),
// k_split_copy (one wavefront per node copies its arcs into place).
#pragma once

#include "lbg_kernels.hpp"

namespace lbg {

constexpr int kSplitPer = 16;                                   // nodes per thread
constexpr uint32_t kSplitChunk = static_cast<uint32_t>(kBlock) * kSplitPer;  // nodes per workgroup

// Shape of node v under split size mdt: children c, own-piece arcs len0,
// children's arcs rest.  Offsets are clamped to [0, m] so a malformed CSR
// cannot produce negative sizes.
__device__ __forceinline__ void split_shape(const int32_t* offsets, uint32_t v, uint32_t m, uint32_t mdt,
                                            uint32_t* c, uint32_t* len0, uint32_t* rest) {
  int64_t s = offsets[v], e = offsets[v + 1];
  s = s < 0 ? 0 : (s > m ? m : s);
  e = e < s ? s : (e > m ? m : e);
  const uint32_t d = static_cast<uint32_t>(e - s);
  const uint32_t p = split_count(d, mdt);
  uint32_t off, len;
  split_piece(d, p, 0, &off, &len);
  *c = p - 1u;
  *len0 = d ? len : 0u;
  *rest = d - *len0;
}

// Block-wide exclusive scan of three counters (kBlock threads, convergent).
__device__ __forceinline__ void block_scan3(uint32_t x[3], uint32_t pre[3], uint32_t tot[3]) {
  __shared__ uint32_t wsum[3][kWaves];
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  uint32_t inc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    inc[k] = wave_incl_scan(x[k]);
    if (lane == 63) wsum[k][wid] = inc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (static_cast<uint32_t>(w) < wid) before += wsum[k][w];
      all += wsum[k][w];
    }
    pre[k] = before + inc[k] - x[k];
    tot[k] = all;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_split_sums(const int32_t* offsets, uint32_t n, uint32_t m,
                                                       uint32_t mdt, uint32_t* sums) {
  const uint32_t v0 = blockIdx.x * kSplitChunk + threadIdx.x * kSplitPer;
  uint32_t x[3] = {0u, 0u, 0u};
  for (int k = 0; k < kSplitPer; ++k) {
    const uint32_t v = v0 + k;
    if (v < n) {
      uint32_t c, l0, r;
      split_shape(offsets, v, m, mdt, &c, &l0, &r);
      x[0] += c;
      x[1] += l0;
      x[2] += r;
    }
  }
  uint32_t pre[3], tot[3];
  block_scan3(x, pre, tot);
  if (threadIdx.x == 0) {
    sums[3 * blockIdx.x + 0] = tot[0];
    sums[3 * blockIdx.x + 1] = tot[1];
    sums[3 * blockIdx.x + 2] = tot[2];
  }
}

// One workgroup: sums[3b + k] becomes the exclusive prefix of counter k over
// blocks 0 .. b-1, and sums[3 nb + k] the total.
__global__ __launch_bounds__(kBlock) void k_split_scan(uint32_t* sums, uint32_t nb) {
  uint32_t carry[3] = {0u, 0u, 0u};
  for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
    const uint32_t b = b0 + threadIdx.x;
    uint32_t x[3] = {0u, 0u, 0u};
    if (b < nb) {
      x[0] = sums[3 * b + 0];
      x[1] = sums[3 * b + 1];
      x[2] = sums[3 * b + 2];
    }
    uint32_t pre[3], tot[3];
    block_scan3(x, pre, tot);
    if (b < nb) {
      sums[3 * b + 0] = carry[0] + pre[0];
      sums[3 * b + 1] = carry[1] + pre[1];
      sums[3 * b + 2] = carry[2] + pre[2];
    }
    carry[0] += tot[0];
    carry[1] += tot[1];
    carry[2] += tot[2];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[3 * nb + 0] = carry[0];
    sums[3 * nb + 1] = carry[1];
    sums[3 * nb + 2] = carry[2];
  }
}

// Child numbering and split offsets.  soffs has n + C + 1 entries and
// child_base n + 1 (C = the children total).  Parents' pieces come first in
// the arc array (P arcs), then the children's.
__global__ __launch_bounds__(kBlock) void k_split_build(const int32_t* offsets, uint32_t n, uint32_t m,
                                                        uint32_t mdt, const uint32_t* sums, uint32_t nb,
                                                        int32_t* soffs, int32_t* child_base) {
  const uint32_t v0 = blockIdx.x * kSplitChunk + threadIdx.x * kSplitPer;
  uint32_t c[kSplitPer], l0[kSplitPer], r[kSplitPer];
  uint32_t x[3] = {0u, 0u, 0u};
#pragma unroll
  for (int k = 0; k < kSplitPer; ++k) {
    c[k] = l0[k] = r[k] = 0u;
    if (v0 + k < n) split_shape(offsets, v0 + k, m, mdt, &c[k], &l0[k], &r[k]);
    x[0] += c[k];
    x[1] += l0[k];
    x[2] += r[k];
  }
  uint32_t pre[3], tot[3];
  block_scan3(x, pre, tot);
  const uint32_t P = sums[3 * nb + 1];  // arcs in parents' own pieces
  uint32_t cb = sums[3 * blockIdx.x + 0] + pre[0];
  uint32_t s0 = sums[3 * blockIdx.x + 1] + pre[1];
  uint32_t s1 = sums[3 * blockIdx.x + 2] + pre[2];
#pragma unroll
  for (int k = 0; k < kSplitPer; ++k) {
    const uint32_t v = v0 + k;
    if (v >= n) break;
    child_base[v] = static_cast<int32_t>(cb);
    soffs[v] = static_cast<int32_t>(s0);
    if (c[k]) {
      const uint32_t d = l0[k] + r[k], p = c[k] + 1u;
      for (uint32_t j = 1; j < p; ++j) {
        uint32_t off, len;
        split_piece(d, p, j, &off, &len);
        soffs[n + cb + j - 1] = static_cast<int32_t>(P + s1 + (off - l0[k]));
      }
    }
    cb += c[k];
    s0 += l0[k];
    s1 += r[k];
    if (v == n - 1) {
      child_base[n] = static_cast<int32_t>(cb);
      soffs[n + cb] = static_cast<int32_t>(P + s1);
    }
  }
}

// One wavefront per node: the node's own piece to soffs[v], its children's
// arcs (contiguous, in piece order) to soffs[n + child_base[v]].  Every store
// is bounded by m.
__global__ __launch_bounds__(kBlock) void k_split_copy(const int32_t* offsets, const int32_t* cols,
                                                       const uint32_t* weights, uint32_t n, uint32_t m,
                                                       const int32_t* soffs, const int32_t* child_base,
                                                       int32_t* cols_out, uint32_t* w_out) {
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWaves;
  for (uint32_t v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < n; v += nwaves) {
    int64_t s = offsets[v], e = offsets[v + 1];
    s = s < 0 ? 0 : (s > m ? m : s);
    e = e < s ? s : (e > m ? m : e);
    const int64_t d = e - s;
    const int64_t len0 = static_cast<int64_t>(soffs[v + 1]) - soffs[v];
    const int32_t cb = child_base[v], ce = child_base[v + 1];
    const int64_t dst1 = ce > cb ? soffs[n + cb] : 0;
    for (int64_t k = lane; k < d; k += 64) {
      const int64_t dst = k < len0 ? soffs[v] + k : dst1 + (k - len0);
      if (dst >= 0 && dst < m) {
        cols_out[dst] = cols[s + k];
        if (w_out) w_out[dst] = weights[s + k];
      }
    }
  }
}

}  // namespace lbg
