// Host emulation of the index arithmetic of the balanced (workload-
// decomposition, Section III-A) one-level kernel for single BFS and SSSP
// solves: the source's worklist, the per-level tile walk with its look-ahead
// of the next tile mark, the staging of a tile's entries into the wave's
// LDS arrays, the slot-to-entry map (start bitmask + popcount prefixes), the
// per-XCD filter words, the push path (per-wave queue, queue overflow
// append, group flush, the workgroup's merged final reservation) and the
// tile marks written with each worklist entry.  Every global and LDS array
// access goes through a bounds check against the size the host allocates
// for it (node_cap, tile_cap, n, m, words, kWQ, T), and every LDS read of a
// staged entry is checked to come from the current tile.
//
// It mirrors the GPU code's arithmetic with the tile size as a parameter
// (64 lanes x kItems arcs per tile) so tile sizes the library does not ship
// can be checked on the CPU.  Lanes of a wavefront are run one after
// another inside each phase, wavefronts and workgroups one after another
// (any such order is one of the interleavings the GPU may produce), and a
// grid of G workgroups of 4 wavefronts is dealt tiles exactly as on the
// device (the per-XCD counters of the last eighth answered in that order),
// and every tile of a level must be dealt exactly once (flag 0x100).  The small-frontier single-workgroup kernel is not emulated: every
// level runs the one-level path.
//
// Test infrastructure only (tests/test_index_emulation_cpu.py).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int kWaves = 4;
constexpr int kXcds = 8;
constexpr uint32_t kWQ = 256;
constexpr uint32_t kBfsInf = 0x7fffffffu;
constexpr uint32_t kSsspInf = 0xffffffffu;
constexpr uint32_t kF16None = 0xffffu;

struct Report {
  long violations = 0;
  long stale_lds = 0;
  long guards = 0;  // device guard flags that would be raised
  char first[512] = "";
  void oob(const char* arr, uint64_t idx, uint64_t size) {
    if (violations++ == 0)
      snprintf(first, sizeof(first), "%s[%llu] outside [0, %llu)", arr, static_cast<unsigned long long>(idx),
               static_cast<unsigned long long>(size));
  }
};
Report* R = nullptr;

template <typename T>
struct Arr {
  std::vector<T> v;
  const char* name;
  T sink{};
  Arr(const char* nm, size_t n, T init = T()) : v(n, init), name(nm) {}
  T& operator[](uint64_t i) {
    if (i >= v.size()) {
      R->oob(name, i, v.size());
      sink = T();
      return sink;
    }
    return v[i];
  }
};

uint32_t popc(uint32_t x) { return static_cast<uint32_t>(__builtin_popcount(x)); }
uint32_t f16_bound(uint16_t f) { return f < kF16None ? f : 0xffffffffu; }
uint16_t f16_of(uint32_t d) { return static_cast<uint16_t>(d < kF16None ? d : kF16None); }

struct Graph {
  Arr<int32_t>* offsets;
  Arr<int32_t>* cols;
  Arr<uint32_t>* weights;
  uint32_t n, m;
};

struct Frontier {
  Arr<int32_t> node;
  Arr<uint32_t> eprefix;
  Arr<int32_t> estart;
  Arr<int32_t> tile_node;
  Frontier(uint32_t node_cap, uint32_t tile_cap, int b)
      : node(b ? "node[1]" : "node[0]", node_cap),
        eprefix(b ? "eprefix[1]" : "eprefix[0]", node_cap),
        estart(b ? "estart[1]" : "estart[0]", node_cap),
        tile_node(b ? "tile_node[1]" : "tile_node[0]", tile_cap) {}
};

struct Lane64 {
  uint32_t v[64];
};

template <bool kSssp>
struct Solver {
  Graph g;
  uint32_t T, kItems, node_cap, tile_cap, words, grid;
  Frontier* fr[2];
  unsigned long long ctr[3] = {0, 0, 0};
  unsigned long long dctr[3][kXcds] = {};  // per-XCD tile counters (ctl->xstat[x][8 + L % 3])
  unsigned error = 0;
  uint32_t max_nf = 0, max_ef = 0;
  uint32_t scan_min = 0xffffffffu;  // BFS: levels of at least this many arcs run in scan mode
  long scan_levels = 0;
  Arr<int32_t> levels;
  Arr<uint32_t> visited, seen0, seen1, xfilter;
  Arr<unsigned long long> dstate;
  Arr<uint16_t> d16;
  // the wave's LDS
  Arr<uint32_t> base, du, flag, wpre;
  Arr<int32_t> qv;
  std::vector<uint32_t> base_tile;  // tile that wrote base[j] / du[j] (stale-read check)
  uint32_t cur_tile_id = 0;

  Solver(Graph gr, uint32_t items, uint32_t min_tile, uint32_t grid_blocks)
      : g(gr),
        T(64 * items),
        kItems(items),
        node_cap(std::max<uint32_t>(gr.n, 1)),
        tile_cap((gr.m + min_tile - 1) / min_tile + 2),
        words((gr.n + 31) / 32),
        grid(grid_blocks),
        levels("levels", kSssp ? 0 : gr.n),
        visited("visited", kSssp ? 0 : (gr.n + 31) / 32),
        seen0("seen[0]", kSssp ? 0 : (gr.n + 31) / 32),
        seen1("seen[1]", kSssp ? 0 : (gr.n + 31) / 32),
        xfilter("xfilter", kSssp ? 0 : static_cast<size_t>(kXcds) * ((gr.n + 31) / 32)),
        dstate("dstate", kSssp ? gr.n : 0),
        d16("d16", kSssp ? gr.n : 0),
        base("lds.base", 64 * items),
        du("lds.du", kSssp ? 64 * items : 1),
        flag("lds.flag", 64 * items / 32),
        wpre("lds.wpre", 64 * items / 32),
        qv("lds.qv", kWQ),
        base_tile(64 * items, 0xffffffffu) {
    fr[0] = new Frontier(node_cap, tile_cap, 0);
    fr[1] = new Frontier(node_cap, tile_cap, 1);
  }
  ~Solver() {
    delete fr[0];
    delete fr[1];
  }
  Arr<uint32_t>& seen(int b) { return b ? seen1 : seen0; }

  // k_init (balanced strategy, no split size, no renaming)
  void init(int32_t src) {
    for (uint32_t v = 0; v < g.n; ++v) {
      if (kSssp) {
        dstate[v] = v == static_cast<uint32_t>(src) ? 0ull : (static_cast<unsigned long long>(kSsspInf) << 32);
        d16[v] = v == static_cast<uint32_t>(src) ? 0 : static_cast<uint16_t>(kF16None);
      } else {
        levels[v] = v == static_cast<uint32_t>(src) ? 0 : static_cast<int32_t>(kBfsInf);
      }
    }
    if (!kSssp) {
      for (uint32_t w = 0; w < words; ++w) {
        const uint32_t bits = w == static_cast<uint32_t>(src) >> 5 ? 1u << (src & 31) : 0u;
        visited[w] = bits;
        seen0[w] = bits;
        seen1[w] = 0u;
      }
      for (uint32_t w = 0; w < words * kXcds; ++w) xfilter[w] = 0u;
    }
    const int32_t s0 = (*g.offsets)[src];
    int32_t d0 = (*g.offsets)[src + 1] - s0;
    if (s0 < 0 || d0 < 0 || static_cast<uint64_t>(s0) + d0 > g.m) d0 = 0;
    const uint32_t tiles = (static_cast<uint32_t>(d0) + T - 1) / T;
    for (uint32_t t = 0; t < tiles && t < tile_cap; ++t) fr[0]->tile_node[t] = 0;
    fr[0]->node[0] = src;
    fr[0]->eprefix[0] = 0;
    fr[0]->estart[0] = s0;
    ctr[0] = d0 > 0 ? ((1ull << 32) | static_cast<uint32_t>(d0)) : 0ull;
    ctr[1] = ctr[2] = 0;
  }

  void write_entry(Frontier& out, uint32_t i, uint32_t p, int32_t v, int32_t s, int32_t d) {
    if (i >= node_cap) {
      error |= 1u;
      return;
    }
    if (kSssp) out.node[i] = v;
    out.eprefix[i] = p;
    out.estart[i] = s;
    const uint32_t end = p + static_cast<uint32_t>(d);
    for (uint32_t t = (p + T - 1) / T; static_cast<unsigned long long>(t) * T < end; ++t) {
      if (t < tile_cap) out.tile_node[t] = static_cast<int32_t>(i);
      else error |= 2u;
    }
  }

  // WaveFlush::prepare for one wave's queue: per queued node its first arc
  // and degree, and the wave's exclusive prefixes (entries, edges).
  struct Prep {
    std::vector<int32_t> vs, ss, ds;
    std::vector<uint32_t> pn, pe;
    uint32_t tot_n = 0, tot_e = 0;
  };
  Prep prepare(uint32_t count) {
    Prep P;
    const uint32_t R = kWQ / 64;
    P.vs.assign(kWQ, 0);
    P.ss.assign(kWQ, 0);
    P.ds.assign(kWQ, 0);
    P.pn.assign(kWQ, 0);
    P.pe.assign(kWQ, 0);
    for (uint32_t k = 0; k < count; ++k) P.vs[k] = qv[k];
    for (uint32_t k = 0; k < count; ++k) {
      P.ss[k] = (*g.offsets)[static_cast<uint32_t>(P.vs[k])];
      P.ds[k] = (*g.offsets)[static_cast<uint32_t>(P.vs[k]) + 1] - P.ss[k];
    }
    // the wave scans row r = k / 64 over its 64 lanes, rows in order
    uint32_t cn = 0, ce = 0;
    for (uint32_t r = 0; r < R; ++r)
      for (uint32_t l = 0; l < 64; ++l) {
        const uint32_t k = r * 64 + l;
        const uint32_t n1 = P.ds[k] > 0 ? 1u : 0u, e1 = P.ds[k] > 0 ? static_cast<uint32_t>(P.ds[k]) : 0u;
        P.pn[k] = cn;
        P.pe[k] = ce;
        cn += n1;
        ce += e1;
      }
    P.tot_n = cn;
    P.tot_e = ce;
    return P;
  }
  void write_prep(const Prep& P, Frontier& out, uint32_t nb, uint32_t eb) {
    for (uint32_t k = 0; k < kWQ; ++k)
      if (P.ds[k] > 0) write_entry(out, nb + P.pn[k], eb + P.pe[k], P.vs[k], P.ss[k], P.ds[k]);
  }
  void flush(uint32_t count, Frontier& out, int nctr) {
    Prep P = prepare(count);
    if (P.tot_n == 0) return;
    const unsigned long long b = ctr[nctr];
    ctr[nctr] += (static_cast<unsigned long long>(P.tot_n) << 32) | P.tot_e;
    write_prep(P, out, static_cast<uint32_t>(b >> 32), static_cast<uint32_t>(b));
  }
  // wave_append: lanes whose push did not fit the queue go straight to the
  // worklist with their own reservation
  void wave_append(const bool* over, const int32_t* v, Frontier& out, int nctr) {
    uint32_t tot = 0, cnt = 0;
    int32_t s[64], d[64];
    uint32_t pre[64], rank[64];
    for (int l = 0; l < 64; ++l) {
      s[l] = d[l] = 0;
      if (over[l]) {
        s[l] = (*g.offsets)[static_cast<uint32_t>(v[l])];
        d[l] = (*g.offsets)[static_cast<uint32_t>(v[l]) + 1] - s[l];
      }
    }
    for (int l = 0; l < 64; ++l) {
      const bool ok = over[l] && d[l] > 0;
      pre[l] = tot;
      rank[l] = cnt;
      if (ok) {
        tot += static_cast<uint32_t>(d[l]);
        ++cnt;
      }
    }
    if (!cnt) return;
    const unsigned long long b = ctr[nctr];
    ctr[nctr] += (static_cast<unsigned long long>(cnt) << 32) | tot;
    for (int l = 0; l < 64; ++l)
      if (over[l] && d[l] > 0)
        write_entry(out, static_cast<uint32_t>(b >> 32) + rank[l], static_cast<uint32_t>(b) + pre[l], v[l], s[l],
                    d[l]);
  }
  void wq_push(uint32_t& count, const bool* want, const int32_t* v, Frontier& out, int nctr) {
    uint32_t c = 0;
    bool over[64];
    for (int l = 0; l < 64; ++l) {
      over[l] = false;
      if (!want[l]) continue;
      const uint32_t k = count + c++;
      if (k < kWQ) qv[k] = v[l];
      else over[l] = true;
    }
    if (!c) return;
    count = std::min(count + c, kWQ);
    bool any = false;
    for (int l = 0; l < 64; ++l) any = any || over[l];
    if (any) wave_append(over, v, out, nctr);
  }

  // One level (launch L) of the balanced kernel over the whole grid.
  void level(uint32_t L) {
    const unsigned long long c = ctr[L % 3];
    ctr[(L + 2) % 3] = 0;
    const uint32_t Ef = static_cast<uint32_t>(c), nf = static_cast<uint32_t>(c >> 32);
    if (Ef == 0) return;
    max_nf = std::max(max_nf, nf);
    max_ef = std::max(max_ef, Ef);
    if (!(nf <= node_cap && Ef <= g.m)) {
      error |= 1u;
      return;
    }
    Frontier& cur = *fr[L & 1];
    Frontier& nxt = *fr[(L + 1) & 1];
    const int nctr = (L + 1) % 3;
    const bool scan = !kSssp && Ef >= scan_min;
    if (scan) {  // k_bfs_prep: every XCD's filter absorbs `visited`
      for (uint32_t x = 0; x < kXcds; ++x)
        for (uint32_t k = 0; k < words; ++k) xfilter[static_cast<uint64_t>(x) * words + k] |= visited[k];
    }
    if (!kSssp && !scan) {  // refresh_seen by the whole grid
      for (uint32_t k = 0; k < words; ++k) seen((L + 1) & 1)[k] = seen(L & 1)[k];
      for (uint32_t x = 0; x < kXcds; ++x)
        for (uint32_t k = 0; k < words; ++k) {
          const uint32_t sw = seen(L & 1)[k];
          if (sw) xfilter[static_cast<uint64_t>(x) * words + k] |= sw;
        }
    }
    const uint32_t ntiles = (Ef + T - 1) / T;
    const uint32_t W = grid * kWaves;
    // tile deal: round-robin below S, then per-XCD counters (slot L % 3,
    // cleared by the previous level; every level here is a one-level launch)
    const bool dyn = grid >= static_cast<uint32_t>(kXcds);
    const uint32_t S = (dyn && ntiles > W) ? std::max(W, (ntiles - ntiles / 8) / W * W) : ntiles;
    for (int x = 0; x < kXcds; ++x) dctr[(L + 1) % 3][x] = 0;
    std::vector<uint8_t> dealt(ntiles, 0);
    for (uint32_t blk = 0; blk < grid; ++blk) {
      Prep preps[kWaves];
      const uint32_t xcd = blk % kXcds;
      auto take = [&]() { return S + xcd + static_cast<uint32_t>(kXcds) * static_cast<uint32_t>(dctr[L % 3][xcd]++); };
      for (int wid = 0; wid < kWaves; ++wid) {
        uint32_t qcount = 0;
        const uint64_t fx = static_cast<uint64_t>(blk % kXcds) * words;
        uint32_t tile = blk * kWaves + wid;
        if (tile >= S) tile = S < ntiles ? take() : ntiles;
        uint32_t i0_next = tile < ntiles ? static_cast<uint32_t>(cur.tile_node[tile]) : 0u;
        uint32_t tnext = ntiles;
        for (; tile < ntiles; tile = tnext) {
          ++cur_tile_id;
          if (dealt[tile]++) error |= 0x100u;  // a tile dealt twice
          const uint32_t i0 = i0_next;
          const bool rr = tile + W < S;
          tnext = rr ? tile + W : (S < ntiles ? take() : ntiles);
          if (tnext < ntiles) i0_next = static_cast<uint32_t>(cur.tile_node[tnext]);
          const uint32_t t0 = tile * T, t1 = std::min(t0 + T, Ef);
          if (i0 >= nf) {
            error |= 16u;
            continue;
          }
          for (uint32_t l = 0; l < T / 32; ++l) flag[l] = 0u;
          // staging
          bool live = false;
          for (uint32_t j0 = 0; j0 < T; j0 += 64) {
            bool anyv = false;
            for (uint32_t lane = 0; lane < 64; ++lane) {
              const uint32_t j = j0 + lane, i = i0 + j;
              if (i >= nf) continue;
              const uint32_t p = cur.eprefix[i];
              const uint32_t st = static_cast<uint32_t>(cur.estart[i]);
              const int32_t node = kSssp ? cur.node[i] : 0;
              if (p < t1) {
                anyv = true;
                base[j] = st + t0 - p;
                base_tile[j] = cur_tile_id;
                if (kSssp) {
                  const uint32_t row = static_cast<uint32_t>(node);
                  if (row < g.n) {
                    const unsigned long long sv = dstate[row];
                    du[j] = static_cast<uint32_t>(sv) == L + 1 ? kSsspInf : static_cast<uint32_t>(sv >> 32);
                    live = live || static_cast<uint32_t>(sv) != L + 1;
                  } else {
                    du[j] = kSsspInf;
                    error |= 8u;
                  }
                }
                const uint32_t s = (p > t0 ? p : t0) - t0;
                flag[s >> 5] |= 1u << (s & 31);
              }
            }
            if (!anyv) break;
          }
          // SSSP: a tile whose staged entries were all improved again ends here
          if (kSssp && !live && !(error & 8u)) continue;
          uint32_t nent = 0;
          {
            uint32_t acc = 0;
            for (uint32_t l = 0; l < T / 32; ++l) {
              wpre[l] = acc;
              acc += popc(flag[l]);
            }
            nent = acc;
          }
          // a tile inside one entry maps every slot to entry 0
          const bool single = nent == 1u;
          if (single && base_tile[0] != cur_tile_id) ++R->stale_lds;
          const uint32_t b0 = single ? base[0] : 0u, d0 = (single && kSssp) ? du[0] : 0u;
          // phase A
          std::vector<int32_t> vv(kItems * 64, -1);
          std::vector<uint32_t> ww(kItems * 64, 0), dd(kItems * 64, 0);
          for (uint32_t r = 0; r < kItems; ++r)
            for (uint32_t lane = 0; lane < 64; ++lane) {
              const uint32_t s = r * 64 + lane, q = r * 64 + lane;
              if (t0 + s >= t1) continue;
              int slot = 0;
              uint32_t e, dslot = d0;
              if (single) {
                e = b0 + s;
              } else {
                const uint32_t k = s >> 5;
                const uint32_t msk = static_cast<uint32_t>((2ull << (s & 31)) - 1ull);
                slot = static_cast<int>(wpre[k] + popc(flag[k] & msk)) - 1;
                if (slot >= 0 && base_tile[static_cast<uint32_t>(slot) % T] != cur_tile_id) ++R->stale_lds;
                e = slot >= 0 ? base[static_cast<uint32_t>(slot)] + s : g.m;
                if (kSssp && slot >= 0) dslot = du[static_cast<uint32_t>(slot)];
              }
              if (kSssp && slot >= 0 && dslot == kSsspInf) {
                // skipped entry
              } else if (e < g.m) {
                vv[q] = (*g.cols)[e];
                if (kSssp) {
                  dd[q] = dslot;
                  ww[q] = (*g.weights)[e];
                }
              } else {
                error |= 8u;
              }
            }
          for (auto& x : vv)
            if (x >= 0 && static_cast<uint32_t>(x) >= g.n) {
              error |= 8u;
              x = -1;
            }
          std::vector<char> push(kItems * 64, 0);
          if (!kSssp && scan) {
            // scan mode: an unvisited node gets level L + 1, nothing is pushed
            for (uint32_t q = 0; q < kItems * 64; ++q) {
              if (vv[q] < 0) continue;
              const uint32_t v = static_cast<uint32_t>(vv[q]), bit = 1u << (v & 31);
              const uint32_t x = xfilter[fx + (v >> 5)];
              if (x & bit) continue;
              xfilter[fx + (v >> 5)] = x | bit;
              // the filter holds every node reached before this level
              if (levels[v] != static_cast<int32_t>(kBfsInf) && levels[v] != static_cast<int32_t>(L + 1))
                error |= 0x400u;  // would overwrite an earlier level
              levels[v] = static_cast<int32_t>(L + 1);
            }
          } else if (!kSssp) {
            for (uint32_t q = 0; q < kItems * 64; ++q) {
              if (vv[q] < 0) continue;
              const uint32_t v = static_cast<uint32_t>(vv[q]), bit = 1u << (v & 31);
              const uint32_t x = xfilter[fx + (v >> 5)];
              if (x & bit) continue;
              xfilter[fx + (v >> 5)] = x | bit;
              const uint32_t old = visited[v >> 5];
              visited[v >> 5] = old | bit;
              if (!(old & bit)) {
                push[q] = 1;
                levels[v] = static_cast<int32_t>(L + 1);
                seen((L + 1) & 1)[v >> 5] |= bit;
              }
            }
          } else {
            for (uint32_t q = 0; q < kItems * 64; ++q) {
              if (vv[q] < 0) continue;
              const uint32_t v = static_cast<uint32_t>(vv[q]);
              const uint32_t alt = dd[q] + ww[q];
              if (alt >= f16_bound(d16[v])) continue;
              const unsigned long long old = dstate[v];
              const unsigned long long mine = (static_cast<unsigned long long>(alt) << 32) | (L + 1);
              if (mine < old) dstate[v] = mine;
              if (alt < static_cast<uint32_t>(old >> 32)) {
                d16[v] = f16_of(alt);
                push[q] = static_cast<uint32_t>(old) != L + 1;
              }
            }
          }
          // push in groups of four rounds
          for (uint32_t r0 = 0; r0 < kItems; r0 += 4) {
            uint32_t P = 0;
            for (uint32_t r = r0; r < r0 + 4; ++r)
              for (uint32_t lane = 0; lane < 64; ++lane) P += push[r * 64 + lane] ? 1u : 0u;
            if (qcount + P > kWQ) {
              flush(qcount, nxt, nctr);
              qcount = 0;
            }
            for (uint32_t r = r0; r < r0 + 4; ++r) {
              bool want[64];
              int32_t v[64];
              for (uint32_t lane = 0; lane < 64; ++lane) {
                want[lane] = push[r * 64 + lane] != 0;
                v[lane] = vv[r * 64 + lane];
              }
              wq_push(qcount, want, v, nxt, nctr);
            }
          }
        }
        preps[wid] = prepare(qcount);
      }
      // the workgroup's merged reservation
      uint32_t tn = 0, te = 0, pn[kWaves], pe[kWaves];
      for (int k = 0; k < kWaves; ++k) {
        pn[k] = tn;
        pe[k] = te;
        tn += preps[k].tot_n;
        te += preps[k].tot_e;
      }
      unsigned long long mb = 0;
      if (tn) {
        mb = ctr[nctr];
        ctr[nctr] += (static_cast<unsigned long long>(tn) << 32) | te;
      }
      for (int k = 0; k < kWaves; ++k)
        write_prep(preps[k], nxt, static_cast<uint32_t>(mb >> 32) + pn[k], static_cast<uint32_t>(mb) + pe[k]);
    }
    for (uint32_t t = 0; t < ntiles; ++t)
      if (!dealt[t]) error |= 0x100u;  // a tile nobody took
    if (scan) compact(L);
  }

  // k_bfs_compact after a scan-mode level: worklist L + 1 from the nodes of
  // level L + 1, 4096-node chunks per workgroup (grid: one per chunk, at most
  // the expansion's grid), 16 consecutive nodes per thread, LDS slots padded
  // one word per 16, one reservation per chunk, entries in node order.
  void compact(uint32_t L) {
    ++scan_levels;
    constexpr uint32_t kBlock = 256, kPer = 16, kChunk = kBlock * kPer;
    constexpr uint32_t kSlots = kChunk + kChunk / 16 + 1;
    auto slot = [](uint32_t j) { return j + (j >> 4); };
    Arr<int32_t> lvs("lds.compact.levels", kSlots), offs("lds.compact.offsets", kSlots);
    Frontier& nxt = *fr[(L + 1) & 1];
    const int nctr = (L + 1) % 3;
    const int32_t want = static_cast<int32_t>(L + 1);
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>((g.n + kChunk - 1) / kChunk, grid));
    for (uint32_t b = 0; b < blocks; ++b) {
      for (uint32_t c0 = b * kChunk; c0 < g.n; c0 += blocks * kChunk) {
        for (uint32_t k = 0; k < kPer; ++k)
          for (uint32_t tid = 0; tid < kBlock; ++tid) {
            const uint32_t j = k * kBlock + tid, v = c0 + j;
            lvs[slot(j)] = v < g.n ? levels[v] : 0;
            offs[slot(j)] = v <= g.n ? (*g.offsets)[v] : 0;
          }
        {
          const uint32_t v = c0 + kChunk;
          offs[slot(kChunk)] = v <= g.n ? (*g.offsets)[v] : 0;
        }
        uint32_t newm[kBlock], reached[kBlock], cnt[kBlock], deg[kBlock];
        for (uint32_t tid = 0; tid < kBlock; ++tid) {
          newm[tid] = reached[tid] = cnt[tid] = deg[tid] = 0;
          for (uint32_t k = 0; k < kPer; ++k) {
            const uint32_t j = tid * kPer + k;
            if (c0 + j < g.n && lvs[slot(j)] != static_cast<int32_t>(kBfsInf)) reached[tid] |= 1u << k;
            if (c0 + j < g.n && lvs[slot(j)] == want) {
              newm[tid] |= 1u << k;
              const uint32_t d = static_cast<uint32_t>(offs[slot(j + 1)] - offs[slot(j)]);
              cnt[tid] += d > 0u ? 1u : 0u;
              deg[tid] += d;
            }
          }
        }
        for (uint32_t tid = 0; tid < kBlock; tid += 2) {
          if (c0 + tid * kPer >= g.n) continue;
          const uint32_t word = reached[tid] | (reached[tid + 1] << 16);
          const uint32_t w = (c0 + tid * kPer) >> 5;
          // the words must equal what the claims of push levels left
          // (every reached node, no other bit): checked before storing
          if ((visited[w] | (newm[tid] | (newm[tid + 1] << 16))) != word) error |= 0x200u;
          visited[w] = word;
          seen((L + 1) & 1)[w] = word;
        }
        uint32_t tc = 0, te = 0;
        for (uint32_t tid = 0; tid < kBlock; ++tid) {
          tc += cnt[tid];
          te += deg[tid];
        }
        const unsigned long long mb = ctr[nctr];
        if (tc) ctr[nctr] += (static_cast<unsigned long long>(tc) << 32) | te;
        uint32_t nb = static_cast<uint32_t>(mb >> 32), eb = static_cast<uint32_t>(mb);
        for (uint32_t tid = 0; tid < kBlock; ++tid)
          for (uint32_t k = 0; k < kPer; ++k) {
            const uint32_t j = tid * kPer + k;
            if (!(newm[tid] & (1u << k))) continue;
            const int32_t s = offs[slot(j)];
            const int32_t d = offs[slot(j + 1)] - s;
            if (d > 0) {
              write_entry(nxt, nb++, eb, static_cast<int32_t>(c0 + j), s, d);
              eb += static_cast<uint32_t>(d);
            }
          }
      }
    }
  }

  uint32_t run(int32_t src, uint32_t max_levels) {
    init(src);
    uint32_t L = 0;
    for (; L < max_levels; ++L) {
      if (static_cast<uint32_t>(ctr[L % 3]) == 0u) break;
      level(L);
      if (error & 1u) break;
    }
    return L;
  }
};

}  // namespace

extern "C" {

// BFS (is_sssp = 0) or SSSP (1) from src with tiles of 64 x items arcs,
// tile marks sized by min_tile (the smallest tile any single-solve kernel
// uses), a grid of grid_blocks workgroups.  out: int32 levels or uint32
// distances, n entries.  BFS levels of at least scan_min arcs run in scan
// mode (UINT32_MAX: never).  stats[0..6]: out-of-bounds accesses, stale LDS
// reads, device guard flags raised, levels run, entries and edges of the
// largest level, levels run in scan mode.
// msg: the first out-of-bounds access (empty when none).
int emu_solve(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, uint32_t n, uint32_t m,
              int32_t src, int is_sssp, uint32_t items, uint32_t min_tile, uint32_t grid_blocks,
              uint32_t scan_min, void* out, long* stats, char* msg, int msg_len) {
  Report rep;
  R = &rep;
  Arr<int32_t> off("offsets", n + 1), cl("cols", m);
  Arr<uint32_t> wt("weights", is_sssp ? m : 0);
  memcpy(off.v.data(), offsets, sizeof(int32_t) * (n + 1));
  if (m) memcpy(cl.v.data(), cols, sizeof(int32_t) * m);
  if (is_sssp && m) memcpy(wt.v.data(), weights, sizeof(uint32_t) * m);
  Graph g{&off, &cl, &wt, n, m};
  uint32_t levels = 0, mnf = 0, mef = 0;
  long scans = 0;
  unsigned err = 0;
  if (is_sssp) {
    Solver<true> s(g, items, min_tile, grid_blocks);
    levels = s.run(src, n + 2);
    err = s.error;
    mnf = s.max_nf;
    mef = s.max_ef;
    uint32_t* d = static_cast<uint32_t*>(out);
    for (uint32_t v = 0; v < n; ++v) d[v] = static_cast<uint32_t>(s.dstate.v[v] >> 32);
  } else {
    Solver<false> s(g, items, min_tile, grid_blocks);
    s.scan_min = scan_min;
    levels = s.run(src, n + 2);
    err = s.error;
    mnf = s.max_nf;
    mef = s.max_ef;
    scans = s.scan_levels;
    memcpy(out, s.levels.v.data(), sizeof(int32_t) * n);
  }
  stats[0] = rep.violations;
  stats[1] = rep.stale_lds;
  stats[2] = static_cast<long>(err);
  stats[3] = static_cast<long>(levels);
  stats[4] = static_cast<long>(mnf);
  stats[5] = static_cast<long>(mef);
  stats[6] = scans;
  snprintf(msg, static_cast<size_t>(msg_len), "%s", rep.first);
  R = nullptr;
  return 0;
}

}  // extern "C"
