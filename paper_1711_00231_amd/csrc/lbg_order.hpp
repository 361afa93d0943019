// Degree-class ordered copy of a graph (an MI355X layout for SSSP, beyond
// the paper).
//
// Nodes are renumbered by degree class, largest first: the class of a node
// of out-degree d is its bit length (0 for d = 0, 1 for d = 1, 2 for 2..3,
// ...), and within a class nodes keep their original order.  Every
// adjacency list is then rewritten with the new ids, ordered by class of the
// destination (largest first) and by original id within a class, which is
// ascending new id whenever the input lists are sorted.  On a skewed graph
// the nodes most arcs point at end up in a short id range, so the random
// reads and atomics of the relaxation land on fewer cache lines and stay in
// L2 more often; results are mapped back through new_id on output.
//
// Build: k_ord_count (per-workgroup class counts), k_ord_scan (exclusive scan
// of the class-major counts, one workgroup), k_ord_scatter (stable placement:
// order[new] = old, new_id[old] = new), k_ord_deg_sums + k_ord_scan +
// k_ord_offsets (new CSR offsets), k_ord_copy (one wavefront per node: a
// stable partition of its list by destination class, ids renamed).
#pragma once

#include "lbg_kernels.hpp"

namespace lbg {

constexpr int kOrdClasses = 32;
constexpr int kOrdRounds = 16;                                                   // rounds of kBlock nodes
constexpr uint32_t kOrdChunk = static_cast<uint32_t>(kBlock) * kOrdRounds;      // nodes per workgroup

// Out-degree of v from offsets clamped to [0, m].
__device__ __forceinline__ uint32_t ord_degree(const int32_t* offsets, uint32_t v, uint32_t m) {
  int64_t s = offsets[v], e = offsets[v + 1];
  s = s < 0 ? 0 : (s > m ? m : s);
  e = e < s ? s : (e > m ? m : e);
  return static_cast<uint32_t>(e - s);
}

// Sort key of a degree: 0 for the largest class, 31 for degree 0.
__device__ __forceinline__ uint32_t ord_key(uint32_t d) {
  return static_cast<uint32_t>(31 - (d ? 32 - __clz(d) : 0));
}

__global__ __launch_bounds__(kBlock) void k_ord_count(const int32_t* offsets, uint32_t n, uint32_t m,
                                                      uint32_t* cnt, uint32_t nb) {
  __shared__ uint32_t c[kOrdClasses];
  if (threadIdx.x < kOrdClasses) c[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t v0 = blockIdx.x * kOrdChunk;
  for (int r = 0; r < kOrdRounds; ++r) {
    const uint32_t v = v0 + r * kBlock + threadIdx.x;
    if (v < n) atomicAdd(&c[ord_key(ord_degree(offsets, v, m))], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrdClasses) cnt[threadIdx.x * nb + blockIdx.x] = c[threadIdx.x];
}

// One workgroup: x[0 .. len) becomes its exclusive prefix sum and x[len]
// the total.
__global__ __launch_bounds__(kBlock) void k_ord_scan(uint32_t* x, uint32_t len) {
  __shared__ uint32_t wsum[kWaves];
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < len; b0 += kBlock) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < len ? x[i] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kWaves; ++w) {
      if (static_cast<uint32_t>(w) < wid) before += wsum[w];
      all += wsum[w];
    }
    if (i < len) x[i] = carry + before + inc - v;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) x[len] = carry;
}

// Stable placement.  cnt holds the scanned class-major counts: the first new
// id of workgroup b's nodes of class k is cnt[k * nb + b].  Each round ranks
// kBlock consecutive nodes: within a wavefront by ballot, across the four
// wavefronts through LDS.
__global__ __launch_bounds__(kBlock) void k_ord_scatter(const int32_t* offsets, uint32_t n, uint32_t m,
                                                        const uint32_t* cnt, uint32_t nb, int32_t* order,
                                                        int32_t* new_id) {
  __shared__ uint32_t base[kOrdClasses];
  __shared__ uint32_t wcnt[kWaves][kOrdClasses];
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  if (threadIdx.x < kOrdClasses) base[threadIdx.x] = cnt[threadIdx.x * nb + blockIdx.x];
  const uint32_t v0 = blockIdx.x * kOrdChunk;
  for (int r = 0; r < kOrdRounds; ++r) {
    const uint32_t v = v0 + r * kBlock + threadIdx.x;
    const bool valid = v < n;
    const uint32_t key = valid ? ord_key(ord_degree(offsets, v, m)) : 0u;
    if (lane < kOrdClasses) wcnt[wid][lane] = 0u;
    uint32_t rank = 0;
    uint64_t left = __ballot(valid);
    while (left) {
      const uint32_t kk = __shfl(key, __ffsll(static_cast<long long>(left)) - 1, 64);
      const uint64_t mk = __ballot(valid && key == kk);
      if (valid && key == kk) rank = lane_rank(mk);
      if (lane == 0) wcnt[wid][kk] = static_cast<uint32_t>(__popcll(mk));
      left &= ~mk;
    }
    __syncthreads();
    if (valid) {
      uint32_t pos = base[key] + rank;
      for (uint32_t w = 0; w < wid; ++w) pos += wcnt[w][key];
      if (pos < n) {
        order[pos] = static_cast<int32_t>(v);
        new_id[v] = static_cast<int32_t>(pos);
      }
    }
    __syncthreads();
    if (threadIdx.x < kOrdClasses) {
      uint32_t t = 0;
      for (int w = 0; w < kWaves; ++w) t += wcnt[w][threadIdx.x];
      base[threadIdx.x] += t;
    }
    __syncthreads();
  }
}

// Per-workgroup sums of the degrees in new order (kOrdChunk new ids each).
__global__ __launch_bounds__(kBlock) void k_ord_deg_sums(const int32_t* offsets, uint32_t n, uint32_t m,
                                                         const int32_t* order, uint32_t* sums) {
  __shared__ uint32_t wsum[kWaves];
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  uint32_t t = 0;
  const uint32_t k0 = blockIdx.x * kOrdChunk + threadIdx.x * kOrdRounds;
  for (int r = 0; r < kOrdRounds; ++r) {
    const uint32_t k = k0 + r;
    if (k < n) {
      const uint32_t v = static_cast<uint32_t>(order[k]);
      if (v < n) t += ord_degree(offsets, v, m);
    }
  }
  const uint32_t inc = wave_incl_scan(t);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t all = 0;
    for (int w = 0; w < kWaves; ++w) all += wsum[w];
    sums[blockIdx.x] = all;
  }
}

// New offsets: noff[k] = the arcs of new ids 0 .. k-1; noff[n] = the total.
__global__ __launch_bounds__(kBlock) void k_ord_offsets(const int32_t* offsets, uint32_t n, uint32_t m,
                                                        const int32_t* order, const uint32_t* sums,
                                                        uint32_t nb, int32_t* noff) {
  __shared__ uint32_t wsum[kWaves];
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  const uint32_t k0 = blockIdx.x * kOrdChunk + threadIdx.x * kOrdRounds;
  uint32_t d[kOrdRounds];
  uint32_t t = 0;
#pragma unroll
  for (int r = 0; r < kOrdRounds; ++r) {
    d[r] = 0u;
    const uint32_t k = k0 + r;
    if (k < n) {
      const uint32_t v = static_cast<uint32_t>(order[k]);
      if (v < n) d[r] = ord_degree(offsets, v, m);
    }
    t += d[r];
  }
  const uint32_t inc = wave_incl_scan(t);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t w = 0; w < wid; ++w) before += wsum[w];
  uint32_t p = sums[blockIdx.x] + before + inc - t;
#pragma unroll
  for (int r = 0; r < kOrdRounds; ++r) {
    const uint32_t k = k0 + r;
    if (k < n) noff[k] = static_cast<int32_t>(p);
    p += d[r];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) noff[n] = static_cast<int32_t>(sums[nb]);
}

// One wavefront per new id k: the arcs of old node order[k] go to
// noff[k] .. noff[k+1] - 1, partitioned stably by the class of their
// destination (largest first), destinations renamed through new_id.  A
// destination outside [0, n) is copied unchanged (the solve reports it).
__global__ __launch_bounds__(kBlock) void k_ord_copy(const int32_t* offsets, const int32_t* cols,
                                                     const uint32_t* weights, uint32_t n, uint32_t m,
                                                     const int32_t* order, const int32_t* new_id,
                                                     const int32_t* noff, int32_t* cols_out, uint32_t* w_out) {
  const uint32_t lane = lane_id();
  const uint32_t nwaves = gridDim.x * kWaves;
  for (uint32_t k = blockIdx.x * kWaves + (threadIdx.x >> 6); k < n; k += nwaves) {
    const uint32_t v = static_cast<uint32_t>(order[k]);
    if (v >= n) continue;
    int64_t s = offsets[v], e = offsets[v + 1];
    s = s < 0 ? 0 : (s > m ? m : s);
    e = e < s ? s : (e > m ? m : e);
    const int64_t d = e - s, dst = noff[k];
    // pass 1: lane c counts the arcs of destination class c
    uint32_t cnt = 0;
    for (int64_t j0 = 0; j0 < d; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool valid = j < d;
      uint32_t key = 31u;
      if (valid) {
        const int32_t t = cols[s + j];
        if (t >= 0 && static_cast<uint32_t>(t) < n) key = ord_key(ord_degree(offsets, static_cast<uint32_t>(t), m));
      }
      uint64_t left = __ballot(valid);
      while (left) {
        const uint32_t kk = __shfl(key, __ffsll(static_cast<long long>(left)) - 1, 64);
        const uint64_t mk = __ballot(valid && key == kk);
        if (lane == kk) cnt += static_cast<uint32_t>(__popcll(mk));
        left &= ~mk;
      }
    }
    uint32_t base = wave_incl_scan(lane < kOrdClasses ? cnt : 0u) - (lane < kOrdClasses ? cnt : 0u);
    // pass 2: place
    for (int64_t j0 = 0; j0 < d; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool valid = j < d;
      uint32_t key = 31u;
      int32_t t = 0;
      uint32_t w = 0;
      if (valid) {
        t = cols[s + j];
        if (w_out) w = weights[s + j];
        if (t >= 0 && static_cast<uint32_t>(t) < n) key = ord_key(ord_degree(offsets, static_cast<uint32_t>(t), m));
      }
      uint64_t left = __ballot(valid);
      while (left) {
        const uint32_t kk = __shfl(key, __ffsll(static_cast<long long>(left)) - 1, 64);
        const uint64_t mk = __ballot(valid && key == kk);
        const uint32_t b = __shfl(base, kk, 64);
        if (valid && key == kk) {
          const int64_t at_ = dst + b + lane_rank(mk);
          if (at_ >= 0 && at_ < m) {
            cols_out[at_] = (t >= 0 && static_cast<uint32_t>(t) < n) ? new_id[t] : t;
            if (w_out) w_out[at_] = w;
          }
        }
        if (lane == kk) base += static_cast<uint32_t>(__popcll(mk));
        left &= ~mk;
      }
    }
  }
}

}  // namespace lbg
