// Destination-sliced workload decomposition (strategy LBG_SLICED).
//
// The balanced expansion (Section III-A tiles) relaxes every arc of a tile
// on whatever XCD runs the tile, so the per-arc filter read (SSSP: the
// 16-bit distance copy, 8 MiB at R-MAT scale 22; BFS: the claim filter) is a
// random read into an array larger than one XCD's 4 MiB L2, and on gfx950
// each miss moves a whole 128-byte line across the fabric for 2 useful
// bytes.  Here the node ids are cut into 8 slices of S consecutive nodes,
// one per XCD, and the arcs of every adjacency list are grouped by the slice
// of their destination (k_slice_group, once per graph).  A node with at
// least slice_min out-arcs is queued with one entry per slice it has arcs
// into (first arc of its segment, own edge prefix and tile marks in that
// slice's list), and the workgroups with blockIdx % 8 == x (dealt to XCD x
// by the dispatcher) tile only slice x's list, so their filter reads and
// state atomics fall in a 1/8 slice of the node state that can stay in that
// XCD's L2.  Smaller nodes would pay more for up to 8 entries than they gain,
// so they are queued once in a mixed list (list 8) whose tiles every
// workgroup takes after its slice's, as in the balanced kernel.  The node
// splitting of Section III-B by a degree threshold, with destination slices
// as the pieces.
//
// The XCD mapping only buys locality: every atomic is device-scope and the
// filters are advisory exactly as in the balanced kernel, so results do not
// depend on which XCD runs which workgroup.  Pushed nodes are looked up in
// the slice offsets in bulk when a wave queue is flushed, and each non-empty
// list gets one packed reservation on its tail counter (slice x:
// Ctl::xstat[x][4 + level % 3]; mixed list: Ctl::ctr[level % 3]).
#pragma once

#include "lbg_kernels.hpp"

namespace lbg {

// Nodes per slice: ceil(n / 8) rounded up to 64 nodes, so slices start on a
// 128-byte line of the 16-bit filter and on a 32-bit word of the bitmaps.
__host__ __device__ inline uint32_t slice_size(uint32_t n) {
  return ((n + kXcds - 1) / kXcds + 63u) / 64u * 64u;
}

constexpr int kLists = kXcds + 1;  // 8 slice lists + the mixed list

__device__ __forceinline__ unsigned long long* slice_ctr(const KArgs& a, int x, uint32_t L) {
  return x < kXcds ? &a.ctl->xstat[x][4 + L % 3] : &a.ctl->ctr[L % 3];
}

// List x's part of a worklist buffer (x = kXcds: the mixed list).
__device__ __forceinline__ Frontier slice_of(const Frontier& f, const KArgs& a, int x) {
  Frontier g = f;
  const size_t eo = static_cast<size_t>(x) * a.scap, to = static_cast<size_t>(x) * a.stcap;
  g.node = f.node + eo;
  g.eprefix = f.eprefix + eo;
  g.estart = f.estart + eo;
  g.tile_node = f.tile_node + to;
  return g;
}

// ------------------------------------------------------------- grouping --
// One wavefront per node: count the node's arcs per destination slice, write
// the slice offsets soff[8u .. 8u + 7], then scatter the arcs slice by slice,
// each slice keeping the input order.  Offsets outside [0, m] are clamped, so
// a malformed CSR cannot make the kernel write out of bounds (its arcs then
// fail the solve's own bounds checks).
__global__ __launch_bounds__(kBlock) void k_slice_group(const int32_t* offsets, const int32_t* cols,
                                                        const uint32_t* weights, uint32_t n, uint32_t m,
                                                        uint32_t S, int32_t* soff, int32_t* cols_out,
                                                        uint32_t* w_out) {
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t nwaves = gridDim.x * kWaves;
  auto clampm = [m](int64_t v) -> int64_t { return v < 0 ? 0 : (v > m ? m : v); };
  for (uint32_t u = blockIdx.x * kWaves + (threadIdx.x >> 6); u < n; u += nwaves) {
    const int64_t s = clampm(offsets[u]);
    int64_t e = clampm(offsets[u + 1]);
    if (e < s) e = s;
    uint32_t cnt[kXcds];
#pragma unroll
    for (int x = 0; x < kXcds; ++x) cnt[x] = 0u;
    for (int64_t k0 = s; k0 < e; k0 += 64) {
      const int64_t k = k0 + lane;
      uint32_t sl = kXcds;  // no arc
      if (k < e) sl = min(static_cast<uint32_t>(cols[k]) / S, static_cast<uint32_t>(kXcds - 1));
#pragma unroll
      for (int x = 0; x < kXcds; ++x) cnt[x] += static_cast<uint32_t>(__popcll(__ballot(sl == static_cast<uint32_t>(x))));
    }
    uint32_t pos[kXcds];
    uint32_t run = static_cast<uint32_t>(s), mine = 0u;
#pragma unroll
    for (int x = 0; x < kXcds; ++x) {
      pos[x] = run;
      if (lane == static_cast<uint32_t>(x)) mine = run;
      run += cnt[x];
    }
    if (lane < static_cast<uint32_t>(kXcds)) soff[static_cast<size_t>(u) * kXcds + lane] = static_cast<int32_t>(mine);
    for (int64_t k0 = s; k0 < e; k0 += 64) {
      const int64_t k = k0 + lane;
      uint32_t sl = kXcds, v = 0u, w = 0u;
      if (k < e) {
        v = static_cast<uint32_t>(cols[k]);
        sl = min(v / S, static_cast<uint32_t>(kXcds - 1));
        if (w_out) w = weights[k];
      }
#pragma unroll
      for (int x = 0; x < kXcds; ++x) {
        const uint64_t msk = __ballot(sl == static_cast<uint32_t>(x));
        if (sl == static_cast<uint32_t>(x)) {
          const uint32_t d = pos[x] + static_cast<uint32_t>(__popcll(msk & below));
          cols_out[d] = static_cast<int32_t>(v);
          if (w_out) w_out[d] = w;
        }
        pos[x] += static_cast<uint32_t>(__popcll(msk));
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t e = clampm(offsets[n]);
    soff[static_cast<size_t>(n) * kXcds] = static_cast<int32_t>(e);
  }
}

// ----------------------------------------------------------------- init --
// Node state as for the other strategies; worklist 0 = the source, per slice
// or in the mixed list by its degree.
template <bool kSssp>
__global__ __launch_bounds__(kBlock) void k_init_sliced(KArgs a, int32_t src) {
  const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  init_state<kSssp>(a, src, gid, stride);
  constexpr uint32_t T = TileCfg<kSssp>::kEdges;
  const int32_t* so = a.soff + static_cast<size_t>(src) * kXcds;
  const int32_t deg = so[kXcds] - so[0];
  const bool split = deg >= static_cast<int32_t>(a.slice_min);
  // list x of the source: first arc and length
  auto seg = [&](int x, int32_t* s, int32_t* d) {
    if (x < kXcds) {
      *s = so[x];
      *d = split ? so[x + 1] - so[x] : 0;
    } else {
      *s = so[0];
      *d = split ? 0 : deg;
    }
  };
#pragma unroll 1
  for (int x = 0; x < kLists; ++x) {
    int32_t s, d;
    seg(x, &s, &d);
    const Frontier f = slice_of(a.fr[0], a, x);
    const uint32_t tiles = d > 0 ? (static_cast<uint32_t>(d) + T - 1) / T : 0u;
    for (uint32_t t = gid; t < tiles && t < a.stcap; t += stride) f.tile_node[t] = 0;
    if (gid == 0 && d > 0) {
      f.node[0] = src;
      f.eprefix[0] = 0u;
      f.estart[0] = s;
    }
  }
  if (gid < kXcds * 16) {
    const int x = static_cast<int>(gid / 16), k = static_cast<int>(gid % 16);
    unsigned long long v = 0ull;
    if (k == 4) {
      int32_t s, d;
      seg(x, &s, &d);
      if (d > 0) v = (1ull << 32) | static_cast<uint32_t>(d);
    }
    a.ctl->xstat[x][k] = v;
  }
  if (gid == 0) {
    int32_t s, d;
    seg(kXcds, &s, &d);
    a.ctl->ctr[0] = d > 0 ? ((1ull << 32) | static_cast<uint32_t>(d)) : 0ull;
    a.ctl->ctr[1] = 0ull;
    a.ctl->ctr[2] = 0ull;
  }
}

// --------------------------------------------------------------- flushes --
// A wave queue's flush into the 9 lists of the next level.  A queued node of
// degree >= slice_min goes to slice x with its arcs soff[8v + x] ..
// soff[8v + x + 1] (if any), a smaller one to the mixed list with all its
// arcs; each non-empty list gets one packed reservation (nodes << 32 | edges).
template <int kPay, uint32_t kTileE, bool kNarrow>
struct SliceFlush {
  static constexpr int R = kWQ / 64;
  int32_t vs[R], s0[R], dg[R];
  bool any_split;  // wave-uniform: some queued node goes to the slice lists

  // Reads the degrees from the CSR offsets (adjacent words); the slice
  // offsets are read only for nodes that are split.
  __device__ __forceinline__ void load(const KArgs& a, const int32_t* qv, uint32_t count) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t k = r * 64 + lane;
      vs[r] = k < count ? qv[k] : -1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      s0[r] = 0;
      dg[r] = 0;
      if (vs[r] >= 0) {
        const int32_t* p = at<kNarrow>(a.offsets, static_cast<uint32_t>(vs[r]));
        s0[r] = p[0];
        dg[r] = p[1];
      }
    }
    bool sp = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      dg[r] -= s0[r];
      sp = sp || (dg[r] > 0 && dg[r] >= static_cast<int32_t>(a.slice_min));
    }
    any_split = __any(sp);
  }

  // Whether list x can get an entry from this wave's batch (wave-uniform).
  __device__ __forceinline__ bool feeds(int x) const { return x == kXcds || any_split; }

  // List x's segment of each of the lane's nodes and its prefix within the
  // wave's batch; tn / te = the wave's totals (wave-uniform).
  __device__ __forceinline__ void scan(const KArgs& a, int x, int32_t* ss, int32_t* ds, uint32_t* pn,
                                       uint32_t* pe, uint32_t& tn, uint32_t& te) const {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool split = dg[r] >= static_cast<int32_t>(a.slice_min);
      ss[r] = s0[r];
      ds[r] = 0;
      if (x == kXcds) {
        if (!split) ds[r] = dg[r];
      } else if (split && dg[r] > 0) {
        const int32_t* p = at<kNarrow>(a.soff, static_cast<uint32_t>(vs[r]) * kXcds + static_cast<uint32_t>(x));
        ss[r] = p[0];
        ds[r] = p[1] - p[0];
      }
    }
    uint32_t cn = 0, ce = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t n1 = ds[r] > 0 ? 1u : 0u;
      const uint32_t e1 = ds[r] > 0 ? static_cast<uint32_t>(ds[r]) : 0u;
      const uint32_t in = wave_incl_scan(n1), ie = wave_incl_scan(e1);
      pn[r] = cn + in - n1;
      pe[r] = ce + ie - e1;
      cn += __shfl(in, 63, 64);
      ce += __shfl(ie, 63, 64);
    }
    tn = cn;
    te = ce;
  }

  __device__ __forceinline__ void write(const KArgs& a, const Frontier& nxt, int x, uint32_t nb,
                                        uint32_t eb, const int32_t* ss, const int32_t* ds,
                                        const uint32_t* pn, const uint32_t* pe) const {
    const Frontier f = slice_of(nxt, a, x);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (ds[r] > 0) write_entry<kPay, kTileE, kNarrow>(a, f, nb + pn[r], eb + pe[r], vs[r], 0, ss[r], ds[r]);
  }

  // Standalone flush by one wavefront (convergent).
  __device__ __forceinline__ void flush(const KArgs& a, const int32_t* qv, uint32_t count,
                                        const Frontier& nxt) {
    load(a, qv, count);
#pragma unroll 1
    for (int x = 0; x < kLists; ++x) {
      if (!feeds(x)) continue;
      int32_t ss[R], ds[R];
      uint32_t pn[R], pe[R], tn, te;
      scan(a, x, ss, ds, pn, pe, tn, te);
      if (tn == 0u) continue;
      unsigned long long base = 0;
      if (lane_id() == 0)
        base = atomicAdd(slice_ctr(a, x, nxt.level), (static_cast<unsigned long long>(tn) << 32) | te);
      base = bcast64(base, 0);
      write(a, nxt, x, static_cast<uint32_t>(base >> 32), static_cast<uint32_t>(base), ss, ds, pn, pe);
    }
  }
};

// Queue v if `want` (convergent per wave; `count` is wave-uniform).  A queue
// that cannot take the whole push is flushed first.
template <int kPay, uint32_t kTileE, bool kNarrow>
__device__ __forceinline__ void wq_push_sliced(const KArgs& a, int32_t* qv, uint32_t& count, bool want,
                                               int32_t v, const Frontier& nxt) {
  const uint64_t mask = __ballot(want);
  if (mask == 0) return;
  const uint32_t c = static_cast<uint32_t>(__popcll(mask));
  if (count + c > static_cast<uint32_t>(kWQ)) {
    SliceFlush<kPay, kTileE, kNarrow> f;
    f.flush(a, qv, count, nxt);
    count = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  if (want) qv[count + lane_rank(mask)] = v;
  count += c;
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ expansion --
// The tiles first, first + W, ... of one list (cur: nf entries, Ef edges) by
// one wavefront.  The loop body is the balanced kernel's: the entries
// overlapping the tile are staged through the LDS start bitmask, each lane
// issues its kItems arc loads, then its filter reads, then one atomic per
// surviving arc; pushes go to the wave queue, which flushes into the 9 lists
// of level L + 1.
template <bool kSssp, bool kNarrow>
__device__ __forceinline__ void sliced_tiles(const KArgs& a, uint32_t L, const Frontier& cur, uint32_t nf,
                                             uint32_t Ef, uint32_t first, uint32_t W,
                                             WaveLds<kSssp, false>& w, const Frontier& nxt,
                                             uint32_t& upd, uint32_t& atom, uint32_t& skip,
                                             uint32_t& qcount) {
  constexpr int kItems = TileCfg<kSssp>::kItems;
  constexpr uint32_t T = TileCfg<kSssp>::kEdges;
  constexpr int kPay = kSssp ? 1 : 0;
  const uint32_t lane = threadIdx.x & 63;
  uint32_t* fx = a.xfilter + static_cast<size_t>(blockIdx.x % kXcds) * a.words;
  uint32_t* seen_nxt = a.seen[(L + 1) & 1];
  const uint32_t ntiles = (Ef + T - 1) / T;
  uint32_t tile = first;
  uint32_t i0_next = tile < ntiles ? static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tile)) : 0u;
  for (; tile < ntiles; tile += W) {
    const uint32_t i0 = i0_next;
    if (tile + W < ntiles) i0_next = static_cast<uint32_t>(*at<kNarrow>(cur.tile_node, tile + W));
    const uint32_t t0 = tile * T;
    const uint32_t t1 = min(t0 + T, Ef);
    if (i0 >= nf) {  // wave-uniform; cannot happen when every tile was marked
      if (lane == 0) atomicOr(&a.ctl->error, kErrBadTile);
      continue;
    }
    if (lane < T / 32) w.flag[lane] = 0u;
    wave_sync();
    bool bad = false;
    for (uint32_t j = lane; j < T; j += 64) {
      const uint32_t i = i0 + j;
      bool valid = false;
      if (i < nf) {
        const uint32_t p = *at<kNarrow>(cur.eprefix, i);
        const uint32_t st = static_cast<uint32_t>(*at<kNarrow>(cur.estart, i));
        const int32_t node = kSssp ? *at<kNarrow>(cur.node, i) : 0;
        if (p < t1) {
          valid = true;
          w.base[j] = st + t0 - p;
          if (kSssp) {
            if (static_cast<uint32_t>(node) < a.n) {
              // improved again during this launch: relaxed next iteration
              const unsigned long long sv = *at<kNarrow>(static_cast<const unsigned long long*>(a.dstate),
                                                         static_cast<uint32_t>(node));
              w.du[j] = static_cast<uint32_t>(sv) == L + 1 ? kSsspInf : static_cast<uint32_t>(sv >> 32);
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
    wave_sync();
    {
      const uint32_t xx = lane < T / 32 ? __popc(w.flag[lane]) : 0u;
      const uint32_t inc = wave_incl_scan(xx);
      if (lane < T / 32) w.wpre[lane] = inc - xx;
    }
    wave_sync();

    int32_t vv[kItems];
    uint32_t ww[kItems];
    uint32_t du[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t s = r * 64 + lane;
      vv[r] = -1;
      ww[r] = 0;
      du[r] = 0;
      if (t0 + s < t1) {
        const uint32_t k = s >> 5;
        const uint32_t msk = static_cast<uint32_t>((2ull << (s & 31)) - 1ull);
        const int slot = static_cast<int>(w.wpre[k] + __popc(w.flag[k] & msk)) - 1;
        const uint32_t e = slot >= 0 ? w.base[slot] + s : a.m;
        if (kSssp && slot >= 0 && w.du[slot] == kSsspInf) {
          ++skip;  // skipped entry
        } else if (e < a.m) {
          vv[r] = *at<kNarrow>(a.cols, e);
          if (kSssp) {
            du[r] = w.du[slot];
            ww[r] = *at<kNarrow>(a.weights, e);
          }
        } else {
          bad = true;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      if (vv[r] >= 0 && static_cast<uint32_t>(vv[r]) >= a.n) {
        bad = true;
        vv[r] = -1;
      }
    }
    bool push[kItems];
    if (!kSssp) {
      uint32_t xw[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r) xw[r] = vv[r] >= 0 ? *at<kNarrow>(fx, static_cast<uint32_t>(vv[r]) >> 5) : ~0u;
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t bit = 1u << (vv[r] & 31);
        const bool cand = vv[r] >= 0 && !(xw[r] & bit);
        if (cand) {
          *at<kNarrow>(fx, static_cast<uint32_t>(vv[r]) >> 5) = xw[r] | bit;
          ++atom;
          xw[r] = atomicOr(at<kNarrow>(a.visited, static_cast<uint32_t>(vv[r]) >> 5), bit);
        } else {
          xw[r] = ~0u;
        }
      }
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        push[r] = vv[r] >= 0 && !(xw[r] & (1u << (vv[r] & 31)));
        if (push[r]) {
          *at<kNarrow>(a.levels, vv[r]) = static_cast<int32_t>(L + 1);
          uint32_t* sw = at<kNarrow>(seen_nxt, static_cast<uint32_t>(vv[r]) >> 5);
          *sw |= 1u << (vv[r] & 31);
          ++upd;
        }
      }
    } else {
      uint32_t cd[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r)
        cd[r] = vv[r] >= 0 ? f16_bound(*at<kNarrow>(static_cast<const uint16_t*>(a.d16), static_cast<uint32_t>(vv[r]))) : 0u;
      unsigned long long old[kItems];
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t alt = du[r] + ww[r];
        old[r] = 0ull;
        if (vv[r] >= 0 && alt < cd[r]) {
          ++atom;
          old[r] = atomicMin(at<kNarrow>(a.dstate, static_cast<uint32_t>(vv[r])),
                             (static_cast<unsigned long long>(alt) << 32) | (L + 1));
        }
      }
#pragma unroll
      for (int r = 0; r < kItems; ++r) {
        const uint32_t alt = du[r] + ww[r];
        const bool better = vv[r] >= 0 && alt < static_cast<uint32_t>(old[r] >> 32);
        if (better) *at<kNarrow>(a.d16, static_cast<uint32_t>(vv[r])) = f16_of(alt);
        upd += better ? 1u : 0u;
        push[r] = better && static_cast<uint32_t>(old[r]) != L + 1;
      }
    }
    if (__any(bad) && lane == 0) atomicOr(&a.ctl->error, kErrBadArc);
#pragma unroll
    for (int r = 0; r < kItems; ++r) wq_push_sliced<kPay, T, kNarrow>(a, w.qv, qcount, push[r], vv[r], nxt);
    if (qcount >= kWQ / 2) {
      SliceFlush<kPay, T, kNarrow> f;
      f.flush(a, w.qv, qcount, nxt);
      qcount = 0;
    }
    wave_sync();
  }
}

// One level (BFS) or iteration (SSSP): the workgroups of slice x take slice
// x's tiles, then every workgroup takes its share of the mixed list's tiles.
// Every block reads all 9 tails (a level is empty only when all are); block
// 0 accounts the level and clears the tails two levels ahead.
template <bool kSssp, bool kNarrow>
__global__ __launch_bounds__(kBlock) void k_expand_sliced(KArgs a, uint32_t L) {
  constexpr uint32_t T = TileCfg<kSssp>::kEdges;
  constexpr int kPay = kSssp ? 1 : 0;
  using Flush = SliceFlush<kPay, T, kNarrow>;
  __shared__ WaveLds<kSssp, false> lds[kWaves];
  __shared__ uint32_t merge[kLists][2 * kWaves];
  __shared__ unsigned long long merge_base[kLists];

  const int x = static_cast<int>(blockIdx.x % kXcds);
  unsigned long long cx = 0ull, cm = 0ull, tn = 0ull, te = 0ull;
#pragma unroll
  for (int y = 0; y < kLists; ++y) {
    const unsigned long long cy = __hip_atomic_load(slice_ctr(a, y, L), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (y == x) cx = cy;
    if (y == kXcds) cm = cy;
    tn += cy >> 32;
    te += static_cast<uint32_t>(cy);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int y = 0; y < kLists; ++y)
      __hip_atomic_store(slice_ctr(a, y, L + 2), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (te) {
      a.ctl->levels = L + 1;
      a.ctl->frontier_entries += tn;
      a.ctl->edges_scanned += te;
    }
  }
  if (te == 0ull) return;
  if (static_cast<uint32_t>(cx >> 32) > a.scap || static_cast<uint32_t>(cx) > a.m ||
      static_cast<uint32_t>(cm >> 32) > a.scap || static_cast<uint32_t>(cm) > a.m) {
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrNodeCap);
    return;
  }
  if (!kSssp) refresh_seen(a, L);  // whole-bitmap filter: the mixed list reaches every slice

  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t lane = threadIdx.x & 63;
  WaveLds<kSssp, false>& w = lds[wid];
  Frontier nxt = a.fr[(L + 1) & 1];
  nxt.level = L + 1;
  uint32_t upd = 0, atom = 0, skip = 0, qcount = 0;
  if (static_cast<uint32_t>(cx) != 0u)
    sliced_tiles<kSssp, kNarrow>(a, L, slice_of(a.fr[L & 1], a, x), static_cast<uint32_t>(cx >> 32),
                                 static_cast<uint32_t>(cx), (blockIdx.x / kXcds) * kWaves + wid,
                                 ((gridDim.x - x + kXcds - 1) / kXcds) * kWaves, w, nxt, upd, atom, skip, qcount);
  if (static_cast<uint32_t>(cm) != 0u)
    sliced_tiles<kSssp, kNarrow>(a, L, slice_of(a.fr[L & 1], a, kXcds), static_cast<uint32_t>(cm >> 32),
                                 static_cast<uint32_t>(cm), blockIdx.x * kWaves + wid, gridDim.x * kWaves, w,
                                 nxt, upd, atom, skip, qcount);

  // Final flush: per list, one reservation for the whole workgroup.
  Flush f;
  f.load(a, w.qv, qcount);
#pragma unroll 1
  for (int y = 0; y < kLists; ++y) {
    int32_t ss[Flush::R], ds[Flush::R];
    uint32_t pn[Flush::R], pe[Flush::R], yn = 0, ye = 0;
    if (f.feeds(y)) f.scan(a, y, ss, ds, pn, pe, yn, ye);
    if (lane == 0) {
      merge[y][wid] = yn;
      merge[y][kWaves + wid] = ye;
    }
  }
  __syncthreads();
  if (threadIdx.x < static_cast<uint32_t>(kLists)) {
    const int y = static_cast<int>(threadIdx.x);
    uint32_t yn = 0, ye = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      yn += merge[y][k];
      ye += merge[y][kWaves + k];
    }
    merge_base[y] = yn ? atomicAdd(slice_ctr(a, y, L + 1), (static_cast<unsigned long long>(yn) << 32) | ye) : 0ull;
  }
  __syncthreads();
#pragma unroll 1
  for (int y = 0; y < kLists; ++y) {
    if (!f.feeds(y)) continue;
    int32_t ss[Flush::R], ds[Flush::R];
    uint32_t pn[Flush::R], pe[Flush::R], yn, ye;
    f.scan(a, y, ss, ds, pn, pe, yn, ye);
    uint32_t bn = 0, be = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      if (static_cast<uint32_t>(k) < wid) {
        bn += merge[y][k];
        be += merge[y][kWaves + k];
      }
    }
    if (yn) f.write(a, nxt, y, static_cast<uint32_t>(merge_base[y] >> 32) + bn, static_cast<uint32_t>(merge_base[y]) + be,
                    ss, ds, pn, pe);
  }
  add_stats(a, upd, atom, skip);
}

}  // namespace lbg
