// C ABI of the lbg library: argument checks, workspace carving, the level
// loop and kernel launches.  Declarations and contracts: include/lbg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/lbg.h"
#include "lbg_kernels.hpp"
#include "lbg_sliced.hpp"
#include "lbg_split.hpp"
#include "lbg_order.hpp"

namespace {

using lbg::Ctl;
using lbg::Frontier;
using lbg::KArgs;

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(LBG_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Names of the device guard flags set in Ctl::error.
const char* guard_names(unsigned flags) {
  thread_local char buf[160];
  buf[0] = 0;
  static const char* names[] = {"worklist capacity", "tile-mark capacity", "edge-worklist capacity",
                                "arc outside the graph", "tile without an entry", "source outside [0, n)",
                                "malformed split table"};
  for (int b = 0; b < 7; ++b)
    if (flags & (1u << b)) {
      if (buf[0]) strncat(buf, ", ", sizeof(buf) - strlen(buf) - 1);
      strncat(buf, names[b], sizeof(buf) - strlen(buf) - 1);
    }
  return buf;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool strategy_ok(int32_t s) { return s >= LBG_AUTO && s <= LBG_SPLIT; }
bool edge_wl(int32_t s) { return s == LBG_EDGE || s == LBG_EDGE_NOCHUNK; }
int32_t resolve(int32_t s) { return s == LBG_AUTO ? LBG_BALANCED : s; }

// Workspace layout.  All offsets 256-byte aligned.
struct Layout {
  size_t ctl, visited, seen[2], xfilter, dstate, d16, node[2], eprefix[2], estart[2], tile[2], sub[2],
      hier_trace, total;
  uint32_t node_cap, tile_cap, edge_cap;
};

// children: child nodes of the split graph (LBG_SPLIT; negative: the bound
// m, which holds for every split size).
Layout layout(int32_t n, int64_t m, int32_t strategy, int is_sssp, int64_t children = -1) {
  Layout L{};
  const int32_t s = resolve(strategy);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.ctl = take(sizeof(Ctl));
  const size_t words = (static_cast<size_t>(n) + 31) / 32;
  if (is_sssp) {
    L.dstate = take(sizeof(unsigned long long) * static_cast<size_t>(n));
    L.d16 = take(sizeof(uint16_t) * static_cast<size_t>(n));
  } else {
    L.visited = take(sizeof(uint32_t) * words);
    L.seen[0] = take(sizeof(uint32_t) * words);
    L.seen[1] = take(sizeof(uint32_t) * words);
    L.xfilter = take(sizeof(uint32_t) * words * lbg::kXcds);
  }
  if (edge_wl(s)) {
    L.edge_cap = static_cast<uint32_t>(m);
    for (int b = 0; b < 2; ++b) L.node[b] = take(sizeof(int32_t) * static_cast<size_t>(m > 0 ? m : 1));
  } else if (s == LBG_SLICED) {
    // per list (8 slices + the mixed one): a node has at most one entry per
    // level (and only if it has arcs there), and the list's edge space is at
    // most m
    L.node_cap = static_cast<uint32_t>(std::max<int64_t>(1, std::min<int64_t>(n, m)));
    L.tile_cap = static_cast<uint32_t>((m + lbg::kMinTile - 1) / lbg::kMinTile + 2);
    const size_t ns = static_cast<size_t>(lbg::kLists) * L.node_cap;
    for (int b = 0; b < 2; ++b) {
      L.node[b] = take(sizeof(int32_t) * ns);
      L.eprefix[b] = take(sizeof(uint32_t) * ns);
      L.estart[b] = take(sizeof(int32_t) * ns);
      L.tile[b] = take(sizeof(int32_t) * static_cast<size_t>(lbg::kLists) * L.tile_cap);
    }
  } else {
    // split hubs add at most m / kMinMdt entries per level; a split graph at
    // most one entry per child node
    int64_t extra = 0;
    if (s == LBG_BINNED) extra = m / lbg::kMinMdt + 1;
    if (s == LBG_SPLIT) extra = children < 0 ? m : children;
    L.node_cap = static_cast<uint32_t>(n + extra);
    L.tile_cap = static_cast<uint32_t>((m + lbg::kMinTile - 1) / lbg::kMinTile + 2);
    for (int b = 0; b < 2; ++b) {
      L.node[b] = take(sizeof(int32_t) * static_cast<size_t>(L.node_cap));
      L.eprefix[b] = take(sizeof(uint32_t) * static_cast<size_t>(L.node_cap));
      L.estart[b] = take(sizeof(int32_t) * static_cast<size_t>(L.node_cap));
      L.tile[b] = take(sizeof(int32_t) * static_cast<size_t>(L.tile_cap));
      if (s == LBG_HIER) L.sub[b] = take(sizeof(int32_t) * static_cast<size_t>(n));
    }
    if (s == LBG_HIER) L.hier_trace = take(sizeof(uint32_t) * lbg::kHierTraceLevels * lbg::kHierTraceSubs);
  }
  L.total = off;
  return L;
}

// Persistent grids: exactly as many workgroups as can be resident at once
// (occupancy x CUs), so tiles dealt round-robin to workgroups all start
// immediately; workgroups are dealt to the 8 XCDs round-robin by the
// dispatcher, which the per-XCD filter and stats lines rely on for locality
// only (never for correctness).
int cu_count() {
  static std::mutex mu;
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

template <typename K>
int resident_grid(K kernel) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, lbg::kBlock, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  return per_cu * cu_count();
}

struct Grids {
  int bal[2][2], node[2], edge[2], edge_nc[2], multi[2], binned[2], hier[2];  // bal[is_sssp][narrow], multi[narrow]
  int sliced[2][2];                                      // [is_sssp][narrow], a multiple of 8 (>= 8)
  int bal_p[2];                                          // SSSP with packed arcs [narrow]
  int bal_s[2][2];                                       // split graph [is_sssp][narrow]
  bool small_p[2];
  bool small[2][2];                                      // small-frontier kernel fits the device
};

// The small-frontier kernel holds its frontier in LDS (about 100 KiB for
// SSSP); use it only where the device grants a workgroup that much.
template <typename K>
bool fits_lds(K kernel) {
  int dev = 0, max_lds = 0;
  hipFuncAttributes fa{};
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) != hipSuccess)
    return false;
  return fa.sharedSizeBytes <= static_cast<size_t>(max_lds) && fa.maxThreadsPerBlock >= lbg::kSmallBlock;
}

// Sliced expansion: every slice needs at least one workgroup; equal counts
// per slice keep the XCDs evenly loaded.
int slice_grid(int g) { return std::max(lbg::kXcds, g - g % lbg::kXcds); }

const Grids& grids() {
  static std::mutex mu;
  static Grids g[64];
  static bool done[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!done[dev]) {
    g[dev].bal[0][0] = resident_grid(lbg::k_expand_balanced<false, false>);
    g[dev].bal[0][1] = resident_grid(lbg::k_expand_balanced<false, true>);
    g[dev].bal[1][0] = resident_grid(lbg::k_expand_balanced<true, false>);
    g[dev].bal[1][1] = resident_grid(lbg::k_expand_balanced<true, true>);
    g[dev].node[0] = resident_grid(lbg::k_expand_node<false>);
    g[dev].node[1] = resident_grid(lbg::k_expand_node<true>);
    g[dev].edge[0] = resident_grid(lbg::k_expand_edge<false, true>);
    g[dev].edge[1] = resident_grid(lbg::k_expand_edge<true, true>);
    g[dev].edge_nc[0] = resident_grid(lbg::k_expand_edge<false, false>);
    g[dev].edge_nc[1] = resident_grid(lbg::k_expand_edge<true, false>);
    g[dev].hier[0] = resident_grid(lbg::k_expand_hier<false>);
    g[dev].hier[1] = resident_grid(lbg::k_expand_hier<true>);
    g[dev].binned[0] = resident_grid(lbg::k_expand_binned<false>);
    g[dev].binned[1] = resident_grid(lbg::k_expand_binned<true>);
    g[dev].multi[0] = resident_grid(lbg::k_expand_balanced<true, false, true>);
    g[dev].multi[1] = resident_grid(lbg::k_expand_balanced<true, true, true>);
    g[dev].bal_p[0] = resident_grid(lbg::k_expand_balanced<true, false, false, true>);
    g[dev].bal_p[1] = resident_grid(lbg::k_expand_balanced<true, true, false, true>);
    g[dev].bal_s[0][0] = resident_grid(lbg::k_expand_balanced<false, false, false, false, true>);
    g[dev].bal_s[0][1] = resident_grid(lbg::k_expand_balanced<false, true, false, false, true>);
    g[dev].bal_s[1][0] = resident_grid(lbg::k_expand_balanced<true, false, false, false, true>);
    g[dev].bal_s[1][1] = resident_grid(lbg::k_expand_balanced<true, true, false, false, true>);
    g[dev].small_p[0] = fits_lds(lbg::k_expand_small<true, false, true>);
    g[dev].small_p[1] = fits_lds(lbg::k_expand_small<true, true, true>);
    g[dev].sliced[0][0] = slice_grid(resident_grid(lbg::k_expand_sliced<false, false>));
    g[dev].sliced[0][1] = slice_grid(resident_grid(lbg::k_expand_sliced<false, true>));
    g[dev].sliced[1][0] = slice_grid(resident_grid(lbg::k_expand_sliced<true, false>));
    g[dev].sliced[1][1] = slice_grid(resident_grid(lbg::k_expand_sliced<true, true>));
    g[dev].small[0][0] = fits_lds(lbg::k_expand_small<false, false>);
    g[dev].small[0][1] = fits_lds(lbg::k_expand_small<false, true>);
    g[dev].small[1][0] = fits_lds(lbg::k_expand_small<true, false>);
    g[dev].small[1][1] = fits_lds(lbg::k_expand_small<true, true>);
    done[dev] = true;
  }
  return g[dev];
}

int grid_blocks() { return grids().bal[0][1]; }

// Degree-bin parameters of LBG_BINNED solves (process-wide; lbg_set_bins).
std::mutex g_bins_mu;
lbg_bins g_bins{256, 16, 1024};  // what the autotuner picks on R-MAT scale 22
int32_t g_slice_min = 512;       // LBG_SLICED: degree from which a node is split by slice
int64_t g_bfs_scan_min = -1;     // balanced BFS: arcs from which a level runs in scan mode (< 0: n / 4)
std::atomic<int32_t> g_addressing{0};  // 0: 32-bit element offsets when every array fits, 1: always 64-bit
int32_t g_hier_mdt = 0;          // LBG_HIER: fixed MDT (0 = the histogram rule per solve)

// Sub-iteration schedule of this thread's last LBG_HIER solve (read back
// from the workspace after the solve): sublist sizes, kHierTraceSubs per level.
thread_local std::vector<uint32_t> g_hier_sched;
thread_local int32_t g_hier_sched_levels = 0, g_hier_sched_mdt = 0;

// Host side of the profiling counters (see lbg_profile_enable).
std::mutex g_prof_mu;
bool g_prof_on = false;
// [0] BFS, [1] SSSP, [2] batched solves (one-level launches); [3] BFS,
// [4] SSSP levels run by the small-frontier kernel
lbg_profile g_prof[5]{};

struct PinnedCtl {
  Ctl* p = nullptr;
  ~PinnedCtl() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local PinnedCtl g_pinned;
// Level count of this thread's previous single solve, per kind (BFS, SSSP),
// or 0 when it used the small-frontier kernel: repeated solves on one graph
// enqueue that many levels in the first batch, so a typical solve needs one
// read-back and few empty launches.
thread_local uint32_t g_level_hint[2] = {0u, 0u};

// Balanced BFS: the levels that ran in scan mode in this thread's solves of
// a graph (keyed by offsets pointer, n, m), accumulated since the last
// re-check.  A later solve lets only those levels and their neighbours scan,
// and launches the compaction kernel only after them, so graphs whose levels
// never reach the threshold stop paying for compaction launches that would
// find nothing to do (~2 us each).  A graph not in the table, and every 16th
// solve of one that is (the re-check, which restarts the record), may scan
// at any level.  Sources whose big levels lie elsewhere only lose speed: a
// level that may not scan claims and pushes.
struct ScanHint {
  const void* off = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  uint64_t mask = 0;
  uint32_t uses = 0;
};
thread_local ScanHint g_scan_hint[4];
thread_local uint32_t g_scan_hint_next = 0;
thread_local std::vector<hipEvent_t> g_events;
// Profiling mode: per timed launch, its level (-1 = small-frontier launch)
// and the index of the event recorded right after it; the launch's interval
// starts at the event before that one (one event per batch start, then one
// after each launch).
thread_local std::vector<int64_t> g_event_level;
thread_local std::vector<size_t> g_event_end;

Ctl* pinned_ctl() {
  if (!g_pinned.p) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return nullptr;
    g_pinned.p = static_cast<Ctl*>(p);
  }
  return g_pinned.p;
}

// Timing events of profiling mode.  They are read only after the solve has
// synchronised its stream, so they need no system-scope fence when
// recorded; without one a record does not write back and invalidate the
// caches between two levels, which would slow the level after it.
hipEvent_t event_at(size_t i) {
  while (g_events.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    g_events.push_back(e);
  }
  return g_events[i];
}

// Sum of one per-XCD stats slot.
int64_t xsum(const Ctl* c, int k) {
  int64_t t = 0;
  for (int x = 0; x < lbg::kXcds; ++x) t += static_cast<int64_t>(c->xstat[x][k]);
  return t;
}

// MDT of Section III-B from the degree histogram the k_deg_* kernels left in
// the control block: k = the fullest bin (ties to the smaller, bins numbered
// from 1), MDT = max(1, floor(k * maxDegree / bins)).
uint32_t mdt_rule(const Ctl* c) {
  int best = 1;
  int64_t best_count = -1;
  for (int b = 1; b <= lbg::kMdtBins; ++b) {
    const int64_t cnt = xsum(c, b - 1);
    if (cnt > best_count) {
      best_count = cnt;
      best = b;
    }
  }
  return static_cast<uint32_t>(std::max<int64_t>(1, best * static_cast<int64_t>(c->deg_max) / lbg::kMdtBins));
}

struct Problem {
  const int32_t* offsets;
  const int32_t* cols;
  const uint32_t* weights;
  const int32_t* coo_src;
  int32_t n;
  int64_t m;
  int32_t src;
  void* out;
  void* ws;
  size_t ws_bytes;
  int32_t strategy;
  int is_sssp;
  lbg_stats* stats;
  hipStream_t stream;
  bool sliced = false;           // called through lbg_bfs_sliced / lbg_sssp_sliced
  const int32_t* soff = nullptr;  // their slice offsets
  const uint32_t* arcs = nullptr; // lbg_sssp_packed: packed arcs (cols/weights unused)
  int32_t wbits = 0;
  const int32_t* child_base = nullptr;  // lbg_bfs_split / lbg_sssp_split: the split graph's
  int64_t children = 0;                 // child table and child count
  const int32_t* node_map = nullptr;    // lbg_sssp_ordered: new id of every original node
  bool no_alloc = false;                // lbg_sssp_noalloc: no allocating call of any kind
};

int check_common(const Problem& P) {
  if (!strategy_ok(P.strategy)) return fail(LBG_EINVAL, "unknown strategy %d", P.strategy);
  if (P.n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", P.n);
  if (P.m < 0 || P.m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(P.m));
  if (P.src < 0 || P.src >= P.n) return fail(LBG_ERANGE, "src %d outside [0, %d)", P.src, P.n);
  if (!P.offsets || !P.out || !P.ws) return fail(LBG_EINVAL, "null offsets/output/workspace pointer");
  if (P.m > 0 && !P.cols) return fail(LBG_EINVAL, "null cols (or packed arcs) pointer with m > 0");
  if (P.is_sssp && P.m > 0 && !P.weights) return fail(LBG_EINVAL, "null weights (or packed arcs) pointer with m > 0");
  if (edge_wl(resolve(P.strategy)) && !P.coo_src)
    return fail(LBG_EINVAL, "LBG_EDGE needs the coo_src array");
  if ((resolve(P.strategy) == LBG_SLICED) != P.sliced)
    return fail(LBG_EINVAL, "LBG_SLICED runs through lbg_bfs_sliced / lbg_sssp_sliced only");
  if (P.sliced && !P.soff) return fail(LBG_EINVAL, "null slice_offsets pointer");
  if ((resolve(P.strategy) == LBG_SPLIT) != (P.child_base != nullptr))
    return fail(LBG_EINVAL, "LBG_SPLIT runs through lbg_bfs_split / lbg_sssp_split only");
  if (P.child_base && (P.children < 0 || P.children > P.m || P.n + P.children >= INT32_MAX))
    return fail(LBG_ERANGE, "children must be in [0, m] with n + children < INT32_MAX (got %lld)",
                static_cast<long long>(P.children));
  if (P.arcs) {
    if (P.wbits < 0 || P.wbits > 31)
      return fail(LBG_ERANGE, "wbits must be in [0, 31] (got %d)", P.wbits);
    if (P.wbits > 0 && (static_cast<uint64_t>(P.n - 1) >> (32 - P.wbits)) != 0)
      return fail(LBG_ERANGE, "node ids of n = %d do not fit beside %d weight bits", P.n, P.wbits);
  }
  if (reinterpret_cast<uintptr_t>(P.ws) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  const size_t need = layout(P.n, P.m, P.strategy, P.is_sssp, P.children).total;
  if (P.ws_bytes < need)
    return fail(LBG_ENOMEM, "workspace has %zu bytes, needs %zu", P.ws_bytes, need);
  return LBG_OK;
}

int solve(const Problem& P) {
  int rc = check_common(P);
  if (rc) return rc;
  const int32_t strat = resolve(P.strategy);
  const Layout Lay = layout(P.n, P.m, P.strategy, P.is_sssp, P.children);
  char* ws = static_cast<char*>(P.ws);

  KArgs a{};
  a.offsets = P.offsets;
  a.cols = P.cols;
  a.weights = P.weights;
  a.coo_src = P.coo_src;
  a.arcs = P.arcs;
  a.wbits = static_cast<uint32_t>(P.wbits);
  const bool packed = P.arcs != nullptr;
  if (P.is_sssp) {
    a.dist = static_cast<uint32_t*>(P.out);
    a.dstate = reinterpret_cast<unsigned long long*>(ws + Lay.dstate);
    a.d16 = reinterpret_cast<uint16_t*>(ws + Lay.d16);
  } else {
    a.levels = static_cast<int32_t*>(P.out);
    a.visited = reinterpret_cast<uint32_t*>(ws + Lay.visited);
    a.seen[0] = reinterpret_cast<uint32_t*>(ws + Lay.seen[0]);
    a.seen[1] = reinterpret_cast<uint32_t*>(ws + Lay.seen[1]);
    a.xfilter = reinterpret_cast<uint32_t*>(ws + Lay.xfilter);
  }
  for (int b = 0; b < 2; ++b) {
    a.fr[b].node = reinterpret_cast<int32_t*>(ws + Lay.node[b]);
    if (!edge_wl(strat)) {
      a.fr[b].eprefix = reinterpret_cast<uint32_t*>(ws + Lay.eprefix[b]);
      a.fr[b].estart = reinterpret_cast<int32_t*>(ws + Lay.estart[b]);
      a.fr[b].tile_node = reinterpret_cast<int32_t*>(ws + Lay.tile[b]);
    }
    if (strat == LBG_HIER) a.sub[b] = reinterpret_cast<int32_t*>(ws + Lay.sub[b]);
  }
  if (strat == LBG_HIER) a.hier_trace = reinterpret_cast<uint32_t*>(ws + Lay.hier_trace);
  a.ctl = reinterpret_cast<Ctl*>(ws + Lay.ctl);
  a.n = static_cast<uint32_t>(P.n);
  a.m = static_cast<uint32_t>(P.m);
  a.words = static_cast<uint32_t>((static_cast<size_t>(P.n) + 31) / 32);
  a.node_cap = Lay.node_cap;
  a.tile_cap = Lay.tile_cap;
  a.edge_cap = Lay.edge_cap;
  a.scan_min = 0xffffffffu;
  if (!P.is_sssp && strat == LBG_BALANCED) {
    int64_t smin;
    {
      std::lock_guard<std::mutex> lk(g_bins_mu);
      smin = g_bfs_scan_min;
    }
    // default n / 4, measured: R-MAT 22 BFS 10 % faster than never scanning
    // (n / 2: 0.5 % faster still), the 2048 x 2048 grid with shortcuts 8.5 %
    // (n / 2: its levels never reach it)
    if (smin < 0) smin = std::max<int64_t>(1, P.n / 4);
    a.scan_min = static_cast<uint32_t>(std::min<int64_t>(smin, 0xffffffffll));
  }
  // a level can only run in scan mode if the graph has that many arcs
  const bool scan_possible = static_cast<int64_t>(a.scan_min) <= P.m;
  ScanHint* shint = nullptr;
  if (scan_possible) {
    for (ScanHint& h : g_scan_hint)
      if (h.off == P.offsets && h.n == P.n && h.m == P.m) shint = &h;
    if (!shint) {
      shint = &g_scan_hint[g_scan_hint_next++ % 4];
      *shint = ScanHint{P.offsets, P.n, P.m, 0ull, 0u};
    }
  }
  const bool scan_any = scan_possible && shint->uses % 16u == 0u;  // unknown, or a periodic re-check
  const uint64_t scan_near = scan_possible ? (shint->mask | (shint->mask << 1) | (shint->mask >> 1)) : 0ull;
  auto scan_at = [&](uint32_t L) {
    return scan_possible && (scan_any || (L < 64u && ((scan_near >> L) & 1ull)));
  };
  const int compact_blocks = static_cast<int>(
      std::max<int64_t>(1, std::min<int64_t>((static_cast<int64_t>(P.n) + lbg::kCompactChunk - 1) / lbg::kCompactChunk,
                                            grids().bal[0][1])));
  const bool sl = strat == LBG_SLICED;
  const bool split = strat == LBG_SPLIT;
  a.child_base = P.child_base;
  a.node_map = P.node_map;
  if (sl) {
    a.soff = P.soff;
    a.sliced = 1u;
    a.scap = Lay.node_cap;
    a.stcap = Lay.tile_cap;
    a.slice_nodes = lbg::slice_size(a.n);
    std::lock_guard<std::mutex> lk(g_bins_mu);
    a.slice_min = static_cast<uint32_t>(g_slice_min);
  }
  if (strat == LBG_BINNED) {
    std::lock_guard<std::mutex> lk(g_bins_mu);
    a.mdt = static_cast<uint32_t>(g_bins.mdt);
    a.t_wave = static_cast<uint32_t>(g_bins.t_wave);
    a.t_block = static_cast<uint32_t>(g_bins.t_block);
  }
  bool profiling;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    profiling = g_prof_on && !P.no_alloc;  // launch timing creates events
  }
  a.count_stats = (P.stats || profiling) ? 1u : 0u;

  // the control block is read back into pinned memory allocated on first
  // use, or, for callers that cannot allocate, into this thread's pageable copy
  thread_local Ctl pageable_ctl;
  Ctl* host = P.no_alloc ? &pageable_ctl : pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");

  const hipStream_t st = P.stream;
  const Grids& GR = grids();
  const int sv = P.is_sssp ? 1 : 0;
  // 32-bit element offsets are enough when every array stays below 4 GiB
  // (the slice offsets have 8n + 1 entries, the split offsets n + children + 1)
  const bool narrow = g_addressing.load() == 0 &&
                      (split ? P.n + P.children : P.n) < (sl ? (1 << 26) : (1 << 29)) &&
                      P.m < (int64_t{1} << 30);
  const int nw = narrow ? 1 : 0;
  const int init_blocks = static_cast<int>(
      std::min<int64_t>(std::max<int64_t>((static_cast<int64_t>(P.n) + lbg::kBlock - 1) / lbg::kBlock, 1), 4096));

  // hierarchical strategy: MDT and the number of sub-iterations per level
  // from the degree histogram (one read-back per solve)
  uint32_t hier_mdt = 1, hier_subs = 1;
  if (strat == LBG_HIER) {
    hipLaunchKernelGGL(lbg::k_deg_clear, dim3(1), dim3(lbg::kBlock), 0, st, a.ctl);
    hipLaunchKernelGGL(lbg::k_deg_max, dim3(init_blocks), dim3(lbg::kBlock), 0, st, P.offsets, a.n, a.ctl);
    hipLaunchKernelGGL(lbg::k_deg_hist, dim3(init_blocks), dim3(lbg::kBlock), 0, st, P.offsets, a.n, a.ctl);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(host, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const uint32_t mx = host->deg_max;
    int32_t fixed;
    {
      std::lock_guard<std::mutex> lk(g_bins_mu);
      fixed = g_hier_mdt;
    }
    hier_mdt = fixed > 0 ? static_cast<uint32_t>(fixed) : mdt_rule(host);
    hier_subs = std::max<uint32_t>(1, (mx + hier_mdt - 1) / hier_mdt);
  }

  if (sl) {
    if (P.is_sssp) hipLaunchKernelGGL((lbg::k_init_sliced<true>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
    else hipLaunchKernelGGL((lbg::k_init_sliced<false>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
  } else if (P.is_sssp) {
    if (edge_wl(strat)) hipLaunchKernelGGL((lbg::k_init<true, true>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
    else hipLaunchKernelGGL((lbg::k_init<true, false>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
  } else {
    if (edge_wl(strat)) hipLaunchKernelGGL((lbg::k_init<false, true>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
    else hipLaunchKernelGGL((lbg::k_init<false, false>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
  }
  HIP_TRY(hipGetLastError());

  auto launch = [&](uint32_t L) {
    if (P.is_sssp) {
      switch (strat) {
        case LBG_NODE: hipLaunchKernelGGL((lbg::k_expand_node<true>), dim3(GR.node[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE: hipLaunchKernelGGL((lbg::k_expand_edge<true, true>), dim3(GR.edge[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE_NOCHUNK: hipLaunchKernelGGL((lbg::k_expand_edge<true, false>), dim3(GR.edge_nc[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_BINNED: hipLaunchKernelGGL((lbg::k_expand_binned<true>), dim3(GR.binned[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_SLICED:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_sliced<true, true>), dim3(GR.sliced[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_sliced<true, false>), dim3(GR.sliced[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
        case LBG_HIER:
          hipLaunchKernelGGL(lbg::k_hier_reset, dim3(1), dim3(64), 0, st, a.ctl);
          for (uint32_t k = 0; k < hier_subs; ++k)
            hipLaunchKernelGGL((lbg::k_expand_hier<true>), dim3(GR.hier[sv]), dim3(lbg::kBlock), 0, st, a, L, k, hier_mdt);
          break;
        case LBG_SPLIT:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<true, true, false, false, true>), dim3(GR.bal_s[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_balanced<true, false, false, false, true>), dim3(GR.bal_s[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
        default:
          if (packed) {
            if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<true, true, false, true>), dim3(GR.bal_p[nw]), dim3(lbg::kBlock), 0, st, a, L);
            else hipLaunchKernelGGL((lbg::k_expand_balanced<true, false, false, true>), dim3(GR.bal_p[nw]), dim3(lbg::kBlock), 0, st, a, L);
          } else if (narrow) {
            hipLaunchKernelGGL((lbg::k_expand_balanced<true, true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          } else {
            hipLaunchKernelGGL((lbg::k_expand_balanced<true, false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          }
          break;
      }
    } else {
      switch (strat) {
        case LBG_NODE: hipLaunchKernelGGL((lbg::k_expand_node<false>), dim3(GR.node[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE: hipLaunchKernelGGL((lbg::k_expand_edge<false, true>), dim3(GR.edge[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE_NOCHUNK: hipLaunchKernelGGL((lbg::k_expand_edge<false, false>), dim3(GR.edge_nc[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_BINNED: hipLaunchKernelGGL((lbg::k_expand_binned<false>), dim3(GR.binned[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_SLICED:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_sliced<false, true>), dim3(GR.sliced[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_sliced<false, false>), dim3(GR.sliced[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
        case LBG_HIER:
          hipLaunchKernelGGL(lbg::k_hier_reset, dim3(1), dim3(64), 0, st, a.ctl);
          for (uint32_t k = 0; k < hier_subs; ++k)
            hipLaunchKernelGGL((lbg::k_expand_hier<false>), dim3(GR.hier[sv]), dim3(lbg::kBlock), 0, st, a, L, k, hier_mdt);
          break;
        case LBG_SPLIT:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<false, true, false, false, true>), dim3(GR.bal_s[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_balanced<false, false, false, false, true>), dim3(GR.bal_s[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
        default:
          if (scan_at(L)) {  // may scan: the filter merge precedes, the compaction follows
            if (narrow) hipLaunchKernelGGL((lbg::k_bfs_prep<true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
            else hipLaunchKernelGGL((lbg::k_bfs_prep<false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
            if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<false, true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
            else hipLaunchKernelGGL((lbg::k_expand_balanced<false, false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
            if (narrow) hipLaunchKernelGGL((lbg::k_bfs_compact<true>), dim3(compact_blocks), dim3(lbg::kBlock), 0, st, a, L);
            else hipLaunchKernelGGL((lbg::k_bfs_compact<false>), dim3(compact_blocks), dim3(lbg::kBlock), 0, st, a, L);
          } else {
            KArgs ap = a;
            ap.scan_min = 0xffffffffu;  // push mode
            if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<false, true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, ap, L);
            else hipLaunchKernelGGL((lbg::k_expand_balanced<false, false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, ap, L);
          }
          break;
      }
    }
  };

  // Level loop.  One-level launches are enqueued in batches (each launch
  // reads its own work size on the device) and the host reads the control
  // block once per batch.  When the next level is small (at most kSmallF
  // entries and kSmallE edges) the balanced strategy hands the following
  // levels to the single-workgroup kernel, which keeps going on the device
  // until a level outgrows those limits or the worklist empties; the host
  // then resumes from ctl->levels, the next level to expand.
  const bool small_ok = strat == LBG_BALANCED && (packed ? GR.small_p[nw] : GR.small[sv][nw]);
  uint32_t L = 0, L_prev = 0;
  const uint32_t hint = g_level_hint[P.is_sssp ? 1 : 0];
  uint32_t batch = hint ? std::min<uint32_t>(std::max<uint32_t>(hint + 1, 8), 64) : 8;
  bool small = false, used_small = false;
  size_t nev = 0;
  g_event_level.clear();
  g_event_end.clear();
  const uint64_t level_cap = static_cast<uint64_t>(P.n) + 2;
  auto mark = [&]() -> int {
    hipEvent_t e = event_at(nev++);
    if (!e) return fail(LBG_EHIP, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(e, st));
    return LBG_OK;
  };
  for (;;) {
    if (profiling && (rc = mark()) != LBG_OK) return rc;  // the batch's first interval starts here
    if (small) {
      const uint32_t max_levels = static_cast<uint32_t>(level_cap + 1 - L);
      if (P.is_sssp && packed) {
        if (narrow) hipLaunchKernelGGL((lbg::k_expand_small<true, true, true>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
        else hipLaunchKernelGGL((lbg::k_expand_small<true, false, true>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
      } else if (P.is_sssp) {
        if (narrow) hipLaunchKernelGGL((lbg::k_expand_small<true, true>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
        else hipLaunchKernelGGL((lbg::k_expand_small<true, false>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
      } else {
        if (narrow) hipLaunchKernelGGL((lbg::k_expand_small<false, true>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
        else hipLaunchKernelGGL((lbg::k_expand_small<false, false>), dim3(1), dim3(lbg::kSmallBlock), 0, st, a, L, max_levels);
      }
      HIP_TRY(hipGetLastError());
      if (profiling) {
        if ((rc = mark()) != LBG_OK) return rc;
        g_event_level.push_back(-1);
        g_event_end.push_back(nev - 1);
      }
    } else {
      for (uint32_t k = 0; k < batch; ++k, ++L) {
        launch(L);
        HIP_TRY(hipGetLastError());
        if (profiling) {  // ends this launch's interval and starts the next one's
          if ((rc = mark()) != LBG_OK) return rc;
          g_event_level.push_back(L);
          g_event_end.push_back(nev - 1);
        }
      }
      batch = std::min<uint32_t>(batch * 2, 64);
    }
    if (P.is_sssp) {
      hipLaunchKernelGGL(lbg::k_sssp_finish, dim3(init_blocks), dim3(lbg::kBlock), 0, st, a);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(host, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host->error)
      return fail(LBG_EOVERFLOW, "device guard tripped (flags 0x%x: %s)", host->error, guard_names(host->error));
    L = host->levels;
    uint64_t ef = static_cast<uint32_t>(host->ctr[L % 3]), nfr = host->ctr[L % 3] >> 32;
    if (sl) {  // the mixed list's tail (ctr) plus the 8 slice tails
      for (int x = 0; x < lbg::kXcds; ++x) {
        ef += static_cast<uint32_t>(host->xstat[x][4 + L % 3]);
        nfr += host->xstat[x][4 + L % 3] >> 32;
      }
    }
    if (ef == 0u) break;
    if (L > level_cap)
      return fail(LBG_EINTERNAL, "more than n + 1 levels; the CSR is probably malformed");
    const bool was_small = small;
    small = small_ok && ef <= lbg::kSmallE && nfr <= lbg::kSmallF &&
            !(was_small && L == L_prev);  // a small step always advances; never spin
    if (was_small && !small) batch = 8;
    used_small = used_small || small;
    L_prev = L;
  }

  g_level_hint[P.is_sssp ? 1 : 0] = used_small ? 0u : host->levels;
  if (shint) {
    shint->mask = scan_any ? host->scan_levels : (shint->mask | host->scan_levels);
    ++shint->uses;
  }
  if (strat == LBG_HIER && !P.no_alloc) {
    g_hier_sched.assign(static_cast<size_t>(lbg::kHierTraceLevels) * lbg::kHierTraceSubs, 0u);
    HIP_TRY(hipMemcpyAsync(g_hier_sched.data(), a.hier_trace, sizeof(uint32_t) * g_hier_sched.size(),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    g_hier_sched_levels = static_cast<int32_t>(std::min<uint32_t>(host->levels, lbg::kHierTraceLevels));
    g_hier_sched_mdt = static_cast<int32_t>(hier_mdt);
  }
  const int64_t p_upd = xsum(host, 2), p_atom = xsum(host, 3);
  if (profiling) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    lbg_profile& gp = g_prof[P.is_sssp ? 1 : 0];
    lbg_profile& pp = g_prof[P.is_sssp ? 4 : 3];
    for (size_t j = 0; j < g_event_end.size(); ++j) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, g_events[g_event_end[j] - 1], g_events[g_event_end[j]]));
      const int64_t lv = g_event_level[j];
      if (lv < 0) {
        pp.launches += 1;
        pp.kernel_ms += ms;
      } else if (lv < static_cast<int64_t>(host->levels)) {
        gp.launches += 1;
        gp.kernel_ms += ms;
      } else {
        gp.empty_launches += 1;
        gp.empty_ms += ms;
      }
    }
    const int64_t pfe = static_cast<int64_t>(host->p_frontier_entries);
    const int64_t pes = static_cast<int64_t>(host->p_edges_scanned);
    gp.frontier_entries += static_cast<int64_t>(host->frontier_entries) - pfe;
    gp.edges_scanned += static_cast<int64_t>(host->edges_scanned) - pes;
    gp.updates += xsum(host, 0);
    gp.atomics += xsum(host, 1);
    gp.edges_skipped += xsum(host, 7);
    pp.frontier_entries += pfe;
    pp.edges_scanned += pes;
    pp.updates += p_upd;
    pp.atomics += p_atom;
  }
  if (P.stats) {
    P.stats->levels = static_cast<int32_t>(host->levels);
    P.stats->reserved = 0;
    P.stats->frontier_entries = static_cast<int64_t>(host->frontier_entries);
    P.stats->edges_scanned = static_cast<int64_t>(host->edges_scanned);
    P.stats->updates = xsum(host, 0) + p_upd;
    P.stats->atomics = xsum(host, 1) + p_atom;
    P.stats->edges_skipped = xsum(host, 7);
  }
  return LBG_OK;
}


// 2-D grid of the row fill/finish kernels: y over the queries, x over the
// kRowChunk chunks of the longest row.
dim3 row_grid(int64_t queries, int64_t max_len) {
  const int64_t chunks = (max_len + lbg::kRowChunk - 1) / lbg::kRowChunk;
  return dim3(static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(chunks, 256))),
              static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(queries, 65535))));
}

// ----------------------------------------------------------------- batch --
struct BatchLayout {
  size_t ctl, qtab, dstate, rbits, d16, node[2], qid[2], eprefix[2], estart[2], tile[2], total;
  uint32_t node_cap, tile_cap;
};

BatchLayout batch_layout(int32_t num_queries, int64_t rows, int64_t total_arcs) {
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  L.ctl = take(sizeof(Ctl));
  L.qtab = take(sizeof(lbg::QInfo) * static_cast<size_t>(num_queries));
  L.dstate = take(sizeof(unsigned long long) * static_cast<size_t>(rows));
  L.rbits = take(sizeof(uint32_t) * ((static_cast<size_t>(rows) + 31) / 32));  // BFS rows
  L.d16 = take(sizeof(uint16_t) * static_cast<size_t>(rows));  // filter of SSSP rows
  L.node_cap = static_cast<uint32_t>(rows);
  L.tile_cap = static_cast<uint32_t>((total_arcs + lbg::kMultiTile - 1) / lbg::kMultiTile + 2);
  for (int b = 0; b < 2; ++b) {
    L.node[b] = take(sizeof(int32_t) * static_cast<size_t>(rows));
    L.qid[b] = take(sizeof(int32_t) * static_cast<size_t>(rows));
    L.eprefix[b] = take(sizeof(uint32_t) * static_cast<size_t>(rows));
    L.estart[b] = take(sizeof(int32_t) * static_cast<size_t>(rows));
    L.tile[b] = take(sizeof(int32_t) * static_cast<size_t>(L.tile_cap));
  }
  L.total = off;
  return L;
}

// An instantiated graph of one replay of a graph-launched batch: kGraphLevels
// expansion launches, the level advance, the conditional write-out and the
// read-back of the control block.  Cached per thread and reused while the
// launch arguments stay the same (they are copied into the graph).
constexpr uint32_t kGraphLevels = 64;

struct GraphCache {
  std::vector<char> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
};
thread_local GraphCache g_graph;  // not destroyed at exit: the runtime may be gone

int batch_graph(const KArgs& a, bool narrow, int expand_blocks, dim3 rgrid, Ctl* host,
                hipGraphExec_t* exec_out) {
  std::vector<char> key(sizeof(KArgs) + 4 * sizeof(int64_t));
  std::memcpy(key.data(), &a, sizeof(KArgs));
  const int64_t extra[4] = {narrow ? 1 : 0, expand_blocks, static_cast<int64_t>(rgrid.x) << 32 | rgrid.y,
                            static_cast<int64_t>(reinterpret_cast<uintptr_t>(host))};
  std::memcpy(key.data() + sizeof(KArgs), extra, sizeof(extra));
  if (g_graph.exec && g_graph.key == key) {
    *exec_out = g_graph.exec;
    return LBG_OK;
  }
  g_graph.drop();
  hipGraph_t g = nullptr;
  HIP_TRY(hipGraphCreate(&g, 0));
  g_graph.graph = g;
  hipGraphNode_t prev = nullptr;
  KArgs args = a;
  auto add_kernel = [&](const void* fn, dim3 grid, void** params) -> int {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(fn);
    p.gridDim = grid;
    p.blockDim = dim3(lbg::kBlock);
    p.sharedMemBytes = 0;
    p.kernelParams = params;
    p.extra = nullptr;
    hipGraphNode_t node = nullptr;
    HIP_TRY(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p));
    prev = node;
    return LBG_OK;
  };
  int rc;
  const void* expand = narrow ? reinterpret_cast<const void*>(lbg::k_expand_batched_graph<true>)
                              : reinterpret_cast<const void*>(lbg::k_expand_batched_graph<false>);
  for (uint32_t k = 0; k < kGraphLevels; ++k) {
    uint32_t kk = k;
    void* params[] = {&args, &kk};
    if ((rc = add_kernel(expand, dim3(expand_blocks), params)) != LBG_OK) return rc;
  }
  {
    Ctl* ctl = args.ctl;
    uint32_t K = kGraphLevels;
    void* params[] = {&ctl, &K};
    if ((rc = add_kernel(reinterpret_cast<const void*>(lbg::k_level_advance), dim3(1), params)) != LBG_OK)
      return rc;
  }
  {
    uint32_t L = 0xffffffffu;
    void* params[] = {&args, &L};
    if ((rc = add_kernel(reinterpret_cast<const void*>(lbg::k_batch_finish), rgrid, params)) != LBG_OK)
      return rc;
  }
  hipGraphNode_t cp = nullptr;
  HIP_TRY(hipGraphAddMemcpyNode1D(&cp, g, &prev, 1, host, args.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  hipGraphExec_t exec = nullptr;
  HIP_TRY(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
  g_graph.exec = exec;
  g_graph.key = key;
  *exec_out = exec;
  return LBG_OK;
}

int batch_solve(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                int64_t m, const lbg_query* queries, int32_t num_queries, uint32_t* out,
                int64_t rows, int64_t total_arcs, void* workspace, size_t workspace_bytes,
                lbg_stats* stats, hipStream_t st, bool use_graph) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (num_queries <= 0 || !queries) return fail(LBG_EINVAL, "need at least one query");
  if (rows <= 0 || rows > INT32_MAX)
    return fail(LBG_ERANGE, "total_rows must be in [1, INT32_MAX] (got %lld)", static_cast<long long>(rows));
  if (total_arcs < 0 || total_arcs > UINT32_MAX)
    return fail(LBG_ERANGE, "total_arcs must be in [0, 2^32)");
  if (!offsets || !out || !workspace || (m > 0 && (!cols || !weights)))
    return fail(LBG_EINVAL, "null offsets/cols/weights/output/workspace pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  const BatchLayout Lay = batch_layout(num_queries, rows, total_arcs);
  if (workspace_bytes < Lay.total)
    return fail(LBG_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, Lay.total);
  std::vector<lbg::QInfo> qt(static_cast<size_t>(num_queries));
  for (int32_t q = 0; q < num_queries; ++q) {
    const lbg_query& Q = queries[q];
    if (Q.lo < 0 || Q.hi > n || Q.lo >= Q.hi || Q.src < Q.lo || Q.src >= Q.hi)
      return fail(LBG_ERANGE, "query %d: need 0 <= lo <= src < hi <= n", q);
    if (Q.kind != LBG_KIND_BFS && Q.kind != LBG_KIND_SSSP)
      return fail(LBG_EINVAL, "query %d: unknown kind %d", q, Q.kind);
    if (Q.out_off < 0 || Q.out_off + (Q.hi - Q.lo) > rows)
      return fail(LBG_ERANGE, "query %d: result row outside [0, total_rows)", q);
    lbg::QInfo& I = qt[static_cast<size_t>(q)];
    I.row_start = static_cast<int32_t>(Q.out_off);
    I.row_len = Q.hi - Q.lo;
    I.delta = I.row_start - Q.lo;
    I.kind = Q.kind;
    I.src = Q.src;
    I.level0 = 0;
    I.pad[0] = I.pad[1] = 0;
  }

  char* ws = static_cast<char*>(workspace);
  KArgs a{};
  a.offsets = offsets;
  a.cols = cols;
  a.weights = weights;
  a.dist = out;
  a.dstate = reinterpret_cast<unsigned long long*>(ws + Lay.dstate);
  a.visited = reinterpret_cast<uint32_t*>(ws + Lay.rbits);
  a.d16 = reinterpret_cast<uint16_t*>(ws + Lay.d16);
  for (int b = 0; b < 2; ++b) {
    a.fr[b].node = reinterpret_cast<int32_t*>(ws + Lay.node[b]);
    a.fr[b].qid = reinterpret_cast<int32_t*>(ws + Lay.qid[b]);
    a.fr[b].eprefix = reinterpret_cast<uint32_t*>(ws + Lay.eprefix[b]);
    a.fr[b].estart = reinterpret_cast<int32_t*>(ws + Lay.estart[b]);
    a.fr[b].tile_node = reinterpret_cast<int32_t*>(ws + Lay.tile[b]);
  }
  a.ctl = reinterpret_cast<Ctl*>(ws + Lay.ctl);
  a.qtab = reinterpret_cast<const lbg::QInfo*>(ws + Lay.qtab);
  a.n = static_cast<uint32_t>(n);
  a.m = static_cast<uint32_t>(m);
  a.node_cap = Lay.node_cap;
  a.tile_cap = Lay.tile_cap;
  a.num_queries = static_cast<uint32_t>(num_queries);
  a.rows = static_cast<uint32_t>(rows);
  bool profiling;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    profiling = g_prof_on;
  }
  a.count_stats = (stats || profiling) ? 1u : 0u;
  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");

  HIP_TRY(hipMemcpyAsync(ws + Lay.qtab, qt.data(), sizeof(lbg::QInfo) * qt.size(),
                         hipMemcpyHostToDevice, st));
  const bool narrow = g_addressing.load() == 0 && n < (1 << 29) && m < (int64_t{1} << 30) &&
                      rows < (int64_t{1} << 29);
  const Grids& GR = grids();
  int64_t max_len = 1;
  for (const lbg::QInfo& I : qt) max_len = std::max<int64_t>(max_len, I.row_len);
  const dim3 rgrid = row_grid(num_queries, max_len);
  const int seed_blocks = (num_queries + lbg::kBlock - 1) / lbg::kBlock;
  hipLaunchKernelGGL(lbg::k_batch_fill, rgrid, dim3(lbg::kBlock), 0, st, a);
  if (narrow) hipLaunchKernelGGL(lbg::k_batch_seed<true>, dim3(seed_blocks), dim3(lbg::kBlock), 0, st, a);
  else hipLaunchKernelGGL(lbg::k_batch_seed<false>, dim3(seed_blocks), dim3(lbg::kBlock), 0, st, a);
  HIP_TRY(hipGetLastError());

  uint32_t L = 0, batch = 8;
  size_t nev = 0;
  const uint64_t level_cap = static_cast<uint64_t>(rows) + 2;
  if (use_graph) {
    hipGraphExec_t exec = nullptr;
    int rc = batch_graph(a, narrow, GR.multi[narrow ? 1 : 0], rgrid, host, &exec);
    if (rc) return rc;
    for (;;) {
      HIP_TRY(hipGraphLaunch(exec, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (host->error)
        return fail(LBG_EOVERFLOW, "device guard tripped (flags 0x%x: %s)", host->error, guard_names(host->error));
      L = host->level_base;
      if (static_cast<uint32_t>(host->ctr[L % 3]) == 0u) break;
      if (L > level_cap) return fail(LBG_EINTERNAL, "more levels than rows; malformed input?");
    }
  }
  for (; !use_graph;) {
    for (uint32_t k = 0; k < batch; ++k, ++L) {
      if (profiling) {
        hipEvent_t e = event_at(nev++);
        if (!e) return fail(LBG_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, st));
      }
      if (narrow)
        hipLaunchKernelGGL((lbg::k_expand_balanced<true, true, true>), dim3(GR.multi[1]), dim3(lbg::kBlock), 0, st, a, L);
      else
        hipLaunchKernelGGL((lbg::k_expand_balanced<true, false, true>), dim3(GR.multi[0]), dim3(lbg::kBlock), 0, st, a, L);
      HIP_TRY(hipGetLastError());
      if (profiling) {
        hipEvent_t e = event_at(nev++);
        if (!e) return fail(LBG_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, st));
      }
    }
    hipLaunchKernelGGL(lbg::k_batch_finish, rgrid, dim3(lbg::kBlock), 0, st, a, L);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(host, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host->error)
      return fail(LBG_EOVERFLOW, "device guard tripped (flags 0x%x: %s)", host->error, guard_names(host->error));
    if (static_cast<uint32_t>(host->ctr[L % 3]) == 0u) break;
    if (L > level_cap) return fail(LBG_EINTERNAL, "more levels than rows; malformed input?");
    batch = std::min<uint32_t>(batch * 2, 64);
  }
  if (profiling) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    lbg_profile& gp = g_prof[2];
    for (size_t k = 0; k + 1 < nev; k += 2) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, g_events[k], g_events[k + 1]));
      if (k / 2 < host->levels) {
        gp.launches += 1;
        gp.kernel_ms += ms;
      } else {
        gp.empty_launches += 1;
        gp.empty_ms += ms;
      }
    }
    gp.frontier_entries += static_cast<int64_t>(host->frontier_entries);
    gp.edges_scanned += static_cast<int64_t>(host->edges_scanned);
    gp.updates += xsum(host, 0);
    gp.atomics += xsum(host, 1);
    gp.edges_skipped += xsum(host, 7);
  }
  if (stats) {
    stats->levels = static_cast<int32_t>(host->levels);
    stats->reserved = 0;
    stats->frontier_entries = static_cast<int64_t>(host->frontier_entries);
    stats->edges_scanned = static_cast<int64_t>(host->edges_scanned);
    stats->updates = xsum(host, 0);
    stats->atomics = xsum(host, 1);
    stats->edges_skipped = xsum(host, 7);
  }
  return LBG_OK;
}


// ---------------------------------------------------------------- engine --
struct EngineLayout {
  BatchLayout b;
  size_t qlast, slots, qstage, total;
};

EngineLayout engine_layout(int32_t max_queries, int64_t max_rows, int64_t max_level_arcs) {
  EngineLayout E{};
  E.b = batch_layout(max_queries, max_rows, max_level_arcs);
  size_t off = E.b.total;
  E.qlast = off;
  off += align_up(sizeof(uint32_t) * static_cast<size_t>(max_queries));
  E.slots = off;
  off += align_up(sizeof(int32_t) * static_cast<size_t>(max_queries));
  E.qstage = off;  // descriptors of the queries being admitted
  off += align_up(sizeof(lbg::QInfo) * static_cast<size_t>(max_queries));
  E.total = off;
  return E;
}

}  // namespace

struct lbg_engine {
  KArgs a{};
  hipStream_t st = nullptr;
  int32_t max_q = 0;
  int64_t max_rows = 0;
  uint32_t L = 0;  // next level to expand
  bool narrow = false;
  char* ws = nullptr;
  EngineLayout lay{};
  std::vector<lbg::QInfo> qt;
  std::vector<uint8_t> state;  // 0 free, 1 pending seed, 2 running, 3 finished (row written)
  std::vector<int32_t> pending, done;
  uint32_t* host_qlast = nullptr;  // pinned
  int32_t* host_slots = nullptr;   // pinned
  lbg::QInfo* host_qstage = nullptr;  // pinned
  Ctl* host_ctl = nullptr;         // pinned
  int64_t steps = 0;
};

namespace {

int engine_sync_state(lbg_engine* e) {
  HIP_TRY(hipMemcpyAsync(e->host_ctl, e->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, e->st));
  HIP_TRY(hipMemcpyAsync(e->host_qlast, e->ws + e->lay.qlast, sizeof(uint32_t) * e->max_q,
                         hipMemcpyDeviceToHost, e->st));
  HIP_TRY(hipStreamSynchronize(e->st));
  if (e->host_ctl->error)
    return fail(LBG_EOVERFLOW, "device guard tripped (flags 0x%x: %s)", e->host_ctl->error,
                guard_names(e->host_ctl->error));
  return LBG_OK;
}

}  // namespace

extern "C" {

size_t lbg_engine_workspace_bytes(int32_t max_queries, int64_t max_rows, int64_t max_level_arcs) {
  if (max_queries <= 0 || max_rows <= 0 || max_rows > INT32_MAX || max_level_arcs < 0 ||
      max_level_arcs > UINT32_MAX)
    return 0;
  return engine_layout(max_queries, max_rows, max_level_arcs).total;
}

int lbg_engine_create(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                      int32_t n, int64_t m, int32_t max_queries, int64_t max_rows,
                      int64_t max_level_arcs, uint32_t* rows_out, void* workspace,
                      size_t workspace_bytes, void* stream, lbg_engine** engine) {
  if (!engine) return fail(LBG_EINVAL, "null engine handle");
  *engine = nullptr;
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX) return fail(LBG_ERANGE, "m must be in [0, INT32_MAX]");
  if (!offsets || !rows_out || !workspace || (m > 0 && (!cols || !weights)))
    return fail(LBG_EINVAL, "null offsets/cols/weights/rows/workspace pointer");
  const size_t need = lbg_engine_workspace_bytes(max_queries, max_rows, max_level_arcs);
  if (need == 0) return fail(LBG_ERANGE, "invalid engine capacities");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < need)
    return fail(LBG_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  lbg_engine* e = new lbg_engine();
  e->st = static_cast<hipStream_t>(stream);
  e->max_q = max_queries;
  e->max_rows = max_rows;
  e->lay = engine_layout(max_queries, max_rows, max_level_arcs);
  e->ws = static_cast<char*>(workspace);
  e->narrow = g_addressing.load() == 0 && n < (1 << 29) && m < (int64_t{1} << 30) &&
              max_rows < (int64_t{1} << 29);
  e->qt.assign(static_cast<size_t>(max_queries), lbg::QInfo{});
  e->state.assign(static_cast<size_t>(max_queries), 0);
  void* p1 = nullptr;
  void* p2 = nullptr;
  void* p3 = nullptr;
  void* p4 = nullptr;
  if (hipHostMalloc(&p1, sizeof(uint32_t) * max_queries, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&p2, sizeof(int32_t) * max_queries, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&p3, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&p4, sizeof(lbg::QInfo) * max_queries, hipHostMallocDefault) != hipSuccess) {
    for (void* p : {p1, p2, p3, p4})
      if (p) (void)hipHostFree(p);
    delete e;
    return fail(LBG_EHIP, "hipHostMalloc failed");
  }
  e->host_qlast = static_cast<uint32_t*>(p1);
  e->host_slots = static_cast<int32_t*>(p2);
  e->host_ctl = static_cast<Ctl*>(p3);
  e->host_qstage = static_cast<lbg::QInfo*>(p4);
  const BatchLayout& Lay = e->lay.b;
  KArgs& a = e->a;
  a.offsets = offsets;
  a.cols = cols;
  a.weights = weights;
  a.dist = rows_out;
  a.dstate = reinterpret_cast<unsigned long long*>(e->ws + Lay.dstate);
  a.visited = reinterpret_cast<uint32_t*>(e->ws + Lay.rbits);
  a.d16 = reinterpret_cast<uint16_t*>(e->ws + Lay.d16);
  for (int b = 0; b < 2; ++b) {
    a.fr[b].node = reinterpret_cast<int32_t*>(e->ws + Lay.node[b]);
    a.fr[b].qid = reinterpret_cast<int32_t*>(e->ws + Lay.qid[b]);
    a.fr[b].eprefix = reinterpret_cast<uint32_t*>(e->ws + Lay.eprefix[b]);
    a.fr[b].estart = reinterpret_cast<int32_t*>(e->ws + Lay.estart[b]);
    a.fr[b].tile_node = reinterpret_cast<int32_t*>(e->ws + Lay.tile[b]);
  }
  a.ctl = reinterpret_cast<Ctl*>(e->ws + Lay.ctl);
  a.qtab = reinterpret_cast<const lbg::QInfo*>(e->ws + Lay.qtab);
  a.qlast = reinterpret_cast<uint32_t*>(e->ws + e->lay.qlast);
  a.n = static_cast<uint32_t>(n);
  a.m = static_cast<uint32_t>(m);
  a.node_cap = Lay.node_cap;
  a.tile_cap = Lay.tile_cap;
  a.num_queries = static_cast<uint32_t>(max_queries);
  a.rows = static_cast<uint32_t>(max_rows);
  a.count_stats = 1u;
  // clear the control block (counters of levels 0..2, stats) and qlast
  if (hipMemsetAsync(a.ctl, 0, sizeof(Ctl), e->st) != hipSuccess ||
      hipMemsetAsync(a.qlast, 0, sizeof(uint32_t) * max_queries, e->st) != hipSuccess ||
      hipStreamSynchronize(e->st) != hipSuccess) {
    lbg_engine_destroy(e);
    return fail(LBG_EHIP, "engine initialisation failed");
  }
  *engine = e;
  return LBG_OK;
}

int lbg_engine_submit(lbg_engine* e, const lbg_query* q, int32_t* slot) {
  if (!e || !q || !slot) return fail(LBG_EINVAL, "null argument");
  if (q->lo < 0 || q->hi > static_cast<int32_t>(e->a.n) || q->lo >= q->hi || q->src < q->lo ||
      q->src >= q->hi)
    return fail(LBG_ERANGE, "need 0 <= lo <= src < hi <= n");
  if (q->kind != LBG_KIND_BFS && q->kind != LBG_KIND_SSSP)
    return fail(LBG_EINVAL, "unknown kind %d", q->kind);
  if (q->out_off < 0 || q->out_off + (q->hi - q->lo) > e->max_rows)
    return fail(LBG_ERANGE, "result row outside [0, max_rows)");
  int32_t s = -1;
  for (int32_t k = 0; k < e->max_q; ++k)
    if (e->state[static_cast<size_t>(k)] == 0) {
      s = k;
      break;
    }
  if (s < 0) return fail(LBG_EBUSY, "all %d query slots are in use", e->max_q);
  lbg::QInfo& I = e->qt[static_cast<size_t>(s)];
  I.row_start = static_cast<int32_t>(q->out_off);
  I.row_len = q->hi - q->lo;
  I.delta = I.row_start - q->lo;
  I.kind = q->kind;
  I.src = q->src;
  I.level0 = 0;
  I.pad[0] = I.pad[1] = 0;
  e->state[static_cast<size_t>(s)] = 1;
  e->pending.push_back(s);
  *slot = s;
  return LBG_OK;
}

int lbg_engine_step(lbg_engine* e, int32_t levels, int32_t* finished) {
  if (!e || levels < 0) return fail(LBG_EINVAL, "bad arguments");
  KArgs& a = e->a;
  const hipStream_t st = e->st;
  const Grids& GR = grids();
  if (!e->pending.empty()) {
    // Admissions: descriptors and slots go up in one copy each (pinned
    // staging; the previous step's copies finished before it returned).
    const int cnt = static_cast<int>(e->pending.size());
    for (int k = 0; k < cnt; ++k) {
      const int32_t s = e->pending[static_cast<size_t>(k)];
      e->host_slots[k] = s;
      e->qt[static_cast<size_t>(s)].level0 = e->L;  // its source joins worklist L
      e->host_qstage[k] = e->qt[static_cast<size_t>(s)];
    }
    int32_t* dslots = reinterpret_cast<int32_t*>(e->ws + e->lay.slots);
    lbg::QInfo* dstage = reinterpret_cast<lbg::QInfo*>(e->ws + e->lay.qstage);
    HIP_TRY(hipMemcpyAsync(dstage, e->host_qstage, sizeof(lbg::QInfo) * cnt, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dslots, e->host_slots, sizeof(int32_t) * cnt, hipMemcpyHostToDevice, st));
    int64_t max_len = 1;
    for (int k = 0; k < cnt; ++k) max_len = std::max<int64_t>(max_len, e->host_qstage[k].row_len);
    hipLaunchKernelGGL(lbg::k_engine_fill, row_grid(cnt, max_len), dim3(lbg::kBlock), 0, st, a,
                       static_cast<const int32_t*>(dslots), static_cast<const lbg::QInfo*>(dstage),
                       reinterpret_cast<lbg::QInfo*>(e->ws + e->lay.b.qtab), cnt);
    const int sb = (cnt + lbg::kBlock - 1) / lbg::kBlock;
    if (e->narrow) hipLaunchKernelGGL(lbg::k_engine_seed<true>, dim3(sb), dim3(lbg::kBlock), 0, st, a, static_cast<const int32_t*>(dslots), cnt, e->L);
    else hipLaunchKernelGGL(lbg::k_engine_seed<false>, dim3(sb), dim3(lbg::kBlock), 0, st, a, static_cast<const int32_t*>(dslots), cnt, e->L);
    HIP_TRY(hipGetLastError());
    for (int32_t s : e->pending) e->state[static_cast<size_t>(s)] = 2;
    e->pending.clear();
  }
  for (int32_t k = 0; k < levels; ++k, ++e->L) {
    if (e->narrow)
      hipLaunchKernelGGL((lbg::k_expand_balanced<true, true, true>), dim3(GR.multi[1]), dim3(lbg::kBlock), 0, st, a, e->L);
    else
      hipLaunchKernelGGL((lbg::k_expand_balanced<true, false, true>), dim3(GR.multi[0]), dim3(lbg::kBlock), 0, st, a, e->L);
    HIP_TRY(hipGetLastError());
  }
  int rc = engine_sync_state(e);
  if (rc) return rc;
  // a running query is finished once no worklist from level L on holds it
  e->done.clear();
  int cnt = 0;
  for (int32_t s = 0; s < e->max_q; ++s)
    if (e->state[static_cast<size_t>(s)] == 2 && e->host_qlast[s] < e->L) {
      e->done.push_back(s);
      e->host_slots[cnt++] = s;
    }
  if (cnt) {
    int32_t* dslots = reinterpret_cast<int32_t*>(e->ws + e->lay.slots);
    HIP_TRY(hipMemcpyAsync(dslots, e->host_slots, sizeof(int32_t) * cnt, hipMemcpyHostToDevice, st));
    int64_t max_len = 1;
    for (int32_t s : e->done) max_len = std::max<int64_t>(max_len, e->qt[static_cast<size_t>(s)].row_len);
    hipLaunchKernelGGL(lbg::k_engine_finish, row_grid(cnt, max_len), dim3(lbg::kBlock), 0, st, a,
                       static_cast<const int32_t*>(dslots), cnt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t s : e->done) e->state[static_cast<size_t>(s)] = 3;
  }
  ++e->steps;
  if (finished) *finished = cnt;
  return LBG_OK;
}

int32_t lbg_engine_finished(const lbg_engine* e, int32_t* slots, int32_t max_slots) {
  if (!e || !slots) return 0;
  const int32_t k = std::min<int32_t>(max_slots, static_cast<int32_t>(e->done.size()));
  for (int32_t i = 0; i < k; ++i) slots[i] = e->done[static_cast<size_t>(i)];
  return k;
}

int lbg_engine_release(lbg_engine* e, int32_t slot) {
  if (!e || slot < 0 || slot >= e->max_q) return fail(LBG_EINVAL, "bad slot");
  if (e->state[static_cast<size_t>(slot)] != 3) return fail(LBG_EINVAL, "slot %d has not finished", slot);
  e->state[static_cast<size_t>(slot)] = 0;
  return LBG_OK;
}

int lbg_engine_info(const lbg_engine* e, lbg_stats* stats, int32_t* running, uint32_t* level) {
  if (!e) return fail(LBG_EINVAL, "null engine");
  if (running) {
    int32_t r = 0;
    for (uint8_t s : e->state) r += (s == 1 || s == 2) ? 1 : 0;
    *running = r;
  }
  if (level) *level = e->L;
  if (stats) {
    stats->levels = static_cast<int32_t>(e->host_ctl->levels);
    stats->reserved = 0;
    stats->frontier_entries = static_cast<int64_t>(e->host_ctl->frontier_entries);
    stats->edges_scanned = static_cast<int64_t>(e->host_ctl->edges_scanned);
    stats->updates = xsum(e->host_ctl, 0);
    stats->atomics = xsum(e->host_ctl, 1);
    stats->edges_skipped = xsum(e->host_ctl, 7);
  }
  return LBG_OK;
}

void lbg_engine_destroy(lbg_engine* e) {
  if (!e) return;
  if (e->st) (void)hipStreamSynchronize(e->st);
  if (e->host_qlast) (void)hipHostFree(e->host_qlast);
  if (e->host_slots) (void)hipHostFree(e->host_slots);
  if (e->host_ctl) (void)hipHostFree(e->host_ctl);
  if (e->host_qstage) (void)hipHostFree(e->host_qstage);
  delete e;
}

}  // extern "C"

namespace {
}  // namespace

// Scratch of lbg_sssp_noalloc: the workspace of one solve, in a file-scope
// device array that every GPU the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it only stands in for the symbol); it uses the device address
// hipGetSymbolAddress gives, looked up once per device.
static __device__ __align__(256) unsigned char scratch[LBG_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of this device's copy of `scratch` (the current device's).
int noalloc_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(LBG_EINVAL, "device %d outside the 64 the library tracks", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBG_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBG_OK;
}

}  // namespace

extern "C" {

size_t lbg_workspace_bytes(int32_t n, int64_t m, int32_t strategy, int32_t is_sssp) {
  if (n <= 0 || m < 0 || m > INT32_MAX || !strategy_ok(strategy)) return 0;
  return layout(n, m, strategy, is_sssp ? 1 : 0).total;
}

int lbg_bfs(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m, int32_t src,
            int32_t* levels_out, void* workspace, size_t workspace_bytes, int32_t strategy,
            const int32_t* coo_src, lbg_stats* stats, void* stream) {
  Problem P{offsets, cols, nullptr, coo_src, n, m, src, levels_out, workspace, workspace_bytes,
            strategy, 0, stats, static_cast<hipStream_t>(stream)};
  return solve(P);
}

int lbg_sssp(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
             int64_t m, int32_t src, uint32_t* dist_out, void* workspace, size_t workspace_bytes,
             int32_t strategy, const int32_t* coo_src, lbg_stats* stats, void* stream) {
  Problem P{offsets, cols, weights, coo_src, n, m, src, dist_out, workspace, workspace_bytes,
            strategy, 1, stats, static_cast<hipStream_t>(stream)};
  return solve(P);
}

int lbg_sssp_noalloc(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                     int64_t m, int32_t src, uint32_t* dist_out, int32_t strategy, lbg_stats* stats,
                     void* stream) {
  const int32_t s = strategy_ok(strategy) ? resolve(strategy) : strategy;
  if (s != LBG_BALANCED && s != LBG_NODE && s != LBG_BINNED && s != LBG_HIER)
    return fail(LBG_EINVAL, "lbg_sssp_noalloc runs LBG_AUTO, LBG_BALANCED, LBG_NODE, LBG_BINNED or LBG_HIER "
                            "(got %d)", strategy);
  if (n > 0 && m >= 0 && m <= INT32_MAX) {
    const size_t need = layout(n, m, strategy, 1).total;
    if (need > LBG_NOALLOC_SCRATCH_BYTES)
      return fail(LBG_ENOMEM, "lbg_sssp_noalloc: n = %d, m = %lld need %zu bytes of scratch, above its "
                  "maximum of %zu", n, static_cast<long long>(m), need,
                  static_cast<size_t>(LBG_NOALLOC_SCRATCH_BYTES));
  }
  void* ws = nullptr;
  const int rc = noalloc_scratch(&ws);
  if (rc) return rc;
  Problem P{offsets, cols, weights, nullptr, n, m, src, dist_out, ws, LBG_NOALLOC_SCRATCH_BYTES,
            strategy, 1, stats, static_cast<hipStream_t>(stream)};
  P.no_alloc = true;
  return solve(P);
}

int lbg_slice_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t* slice_offsets, int32_t* cols_out, uint32_t* weights_out,
                    void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!offsets || !slice_offsets || (m > 0 && (!cols || !cols_out)))
    return fail(LBG_EINVAL, "null offsets/slice_offsets/cols/cols_out pointer");
  if (m > 0 && (weights == nullptr) != (weights_out == nullptr))
    return fail(LBG_EINVAL, "weights and weights_out must both be given or both be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int blocks = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(n) + lbg::kWaves - 1) / lbg::kWaves, 16384));
  hipLaunchKernelGGL(lbg::k_slice_group, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, cols, weights,
                     static_cast<uint32_t>(n), static_cast<uint32_t>(m), lbg::slice_size(static_cast<uint32_t>(n)),
                     slice_offsets, cols_out, weights_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return LBG_OK;
}

int lbg_coo_sources(const int32_t* offsets, int32_t n, int64_t m, int32_t* coo_out, void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!offsets || (m > 0 && !coo_out)) return fail(LBG_EINVAL, "null offsets or output pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (m > 0) {
    const int blocks = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(n) + lbg::kWaves - 1) / lbg::kWaves, 4096));
    hipLaunchKernelGGL(lbg::k_coo_sources, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets,
                       static_cast<uint32_t>(n), static_cast<uint32_t>(m), coo_out);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  return LBG_OK;
}

int lbg_pack_arcs(const int32_t* cols, const uint32_t* weights, int32_t n, int64_t m, uint32_t* arcs_out,
                  int32_t* wbits_out, void* workspace, size_t workspace_bytes, void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!wbits_out || !workspace || (m > 0 && (!cols || !weights || !arcs_out)))
    return fail(LBG_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < sizeof(Ctl)) return fail(LBG_ENOMEM, "workspace smaller than %zu bytes", sizeof(Ctl));
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctl* ctl = static_cast<Ctl*>(workspace);
  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");
  const int blocks = static_cast<int>(
      std::min<int64_t>(std::max<int64_t>((m + lbg::kBlock - 1) / lbg::kBlock, 1), 4096));
  hipLaunchKernelGGL(lbg::k_deg_clear, dim3(1), dim3(lbg::kBlock), 0, st, ctl);
  if (m > 0)
    hipLaunchKernelGGL(lbg::k_weight_max, dim3(blocks), dim3(lbg::kBlock), 0, st, weights, static_cast<uint32_t>(m), ctl);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const uint32_t wmax = host->deg_max;
  int32_t wbits = 0;
  while (wbits < 32 && (wmax >> wbits) != 0u) ++wbits;
  if (wbits > 31 || (wbits > 0 && (static_cast<uint64_t>(n - 1) >> (32 - wbits)) != 0))
    return fail(LBG_ERANGE, "n = %d node ids and weights up to %u do not fit in 32 bits", n, wmax);
  if (m > 0)
    hipLaunchKernelGGL(lbg::k_pack_arcs, dim3(blocks), dim3(lbg::kBlock), 0, st, cols, weights,
                       static_cast<uint32_t>(m), static_cast<uint32_t>(wbits), arcs_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  *wbits_out = wbits;
  return LBG_OK;
}

int lbg_sssp_packed(const int32_t* offsets, const uint32_t* arcs, int32_t wbits, int32_t n, int64_t m,
                    int32_t src, uint32_t* dist_out, void* workspace, size_t workspace_bytes,
                    lbg_stats* stats, void* stream) {
  // any stray read of cols/weights stays inside the arc array
  Problem P{offsets, reinterpret_cast<const int32_t*>(arcs), arcs, nullptr, n, m, src, dist_out, workspace,
            workspace_bytes, LBG_BALANCED, 1, stats, static_cast<hipStream_t>(stream)};
  P.arcs = arcs;
  P.wbits = wbits;
  if (m > 0 && !arcs) return fail(LBG_EINVAL, "null arcs pointer with m > 0");
  return solve(P);
}

int lbg_set_hier_mdt(int32_t mdt) {
  if (mdt < 0) return fail(LBG_EINVAL, "MDT must be >= 0 (got %d)", mdt);
  std::lock_guard<std::mutex> lk(g_bins_mu);
  g_hier_mdt = mdt;
  return LBG_OK;
}

int32_t lbg_get_hier_mdt(void) {
  std::lock_guard<std::mutex> lk(g_bins_mu);
  return g_hier_mdt;
}

int32_t lbg_hier_last_schedule(int32_t* sizes, int32_t max_levels, int32_t max_subs, int32_t* mdt_out) {
  if (mdt_out) *mdt_out = g_hier_sched_mdt;
  const int32_t nl = std::min(g_hier_sched_levels, std::max(max_levels, 0));
  const int32_t ns = std::min<int32_t>(static_cast<int32_t>(lbg::kHierTraceSubs), std::max(max_subs, 0));
  if (sizes) {
    for (int64_t k = 0; k < static_cast<int64_t>(std::max(max_levels, 0)) * std::max(max_subs, 0); ++k) sizes[k] = 0;
    for (int32_t l = 0; l < nl; ++l)
      for (int32_t k = 0; k < ns; ++k)
        sizes[static_cast<size_t>(l) * max_subs + k] =
            static_cast<int32_t>(g_hier_sched[static_cast<size_t>(l) * lbg::kHierTraceSubs + k]);
  }
  return nl;
}

int lbg_set_slice_min(int32_t min_degree) {
  if (min_degree < 0) return fail(LBG_EINVAL, "slice_min must be >= 0 (got %d)", min_degree);
  std::lock_guard<std::mutex> lk(g_bins_mu);
  g_slice_min = min_degree;
  return LBG_OK;
}

int32_t lbg_get_slice_min(void) {
  std::lock_guard<std::mutex> lk(g_bins_mu);
  return g_slice_min;
}

int lbg_set_addressing(int32_t mode) {
  if (mode != 0 && mode != 1) return fail(LBG_EINVAL, "addressing mode must be 0 or 1 (got %d)", mode);
  g_addressing.store(mode);
  return LBG_OK;
}

int32_t lbg_get_addressing(void) { return g_addressing.load(); }

int lbg_set_bfs_scan_min(int64_t arcs) {
  std::lock_guard<std::mutex> lk(g_bins_mu);
  g_bfs_scan_min = arcs < 0 ? -1 : arcs;
  return LBG_OK;
}

int64_t lbg_get_bfs_scan_min(void) {
  std::lock_guard<std::mutex> lk(g_bins_mu);
  return g_bfs_scan_min;
}

int32_t lbg_slice_nodes(int32_t n) {
  return n > 0 ? static_cast<int32_t>(lbg::slice_size(static_cast<uint32_t>(n))) : 0;
}

int lbg_bfs_sliced(const int32_t* offsets, const int32_t* slice_offsets, const int32_t* cols, int32_t n,
                   int64_t m, int32_t src, int32_t* levels_out, void* workspace, size_t workspace_bytes,
                   lbg_stats* stats, void* stream) {
  Problem P{offsets, cols, nullptr, nullptr, n, m, src, levels_out, workspace, workspace_bytes,
            LBG_SLICED, 0, stats, static_cast<hipStream_t>(stream), true, slice_offsets};
  return solve(P);
}

int lbg_sssp_sliced(const int32_t* offsets, const int32_t* slice_offsets, const int32_t* cols,
                    const uint32_t* weights, int32_t n, int64_t m, int32_t src, uint32_t* dist_out,
                    void* workspace, size_t workspace_bytes, lbg_stats* stats, void* stream) {
  Problem P{offsets, cols, weights, nullptr, n, m, src, dist_out, workspace, workspace_bytes,
            LBG_SLICED, 1, stats, static_cast<hipStream_t>(stream), true, slice_offsets};
  return solve(P);
}

size_t lbg_split_scratch_bytes(int32_t n) {
  if (n <= 0) return 0;
  const size_t nb = (static_cast<size_t>(n) + lbg::kSplitChunk - 1) / lbg::kSplitChunk;
  return align_up(sizeof(uint32_t) * 3 * (nb + 1));
}

namespace {

// Per-workgroup sums and their scan (k_split_sums, k_split_scan); leaves the
// three totals (children, own-piece arcs, children's arcs) in totals.
int split_scan(const int32_t* offsets, int32_t n, int64_t m, int32_t mdt, void* scratch,
               size_t scratch_bytes, hipStream_t st, uint32_t totals[3]) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (mdt < 0) return fail(LBG_EINVAL, "mdt must be >= 0 (got %d)", mdt);
  if (!offsets || !scratch) return fail(LBG_EINVAL, "null offsets/scratch pointer");
  if (reinterpret_cast<uintptr_t>(scratch) % kAlign)
    return fail(LBG_EINVAL, "scratch must be %zu-byte aligned", kAlign);
  if (scratch_bytes < lbg_split_scratch_bytes(n))
    return fail(LBG_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, lbg_split_scratch_bytes(n));
  const uint32_t nb = static_cast<uint32_t>((static_cast<int64_t>(n) + lbg::kSplitChunk - 1) / lbg::kSplitChunk);
  uint32_t* sums = static_cast<uint32_t*>(scratch);
  hipLaunchKernelGGL(lbg::k_split_sums, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, static_cast<uint32_t>(n),
                     static_cast<uint32_t>(m), static_cast<uint32_t>(mdt), sums);
  hipLaunchKernelGGL(lbg::k_split_scan, dim3(1), dim3(lbg::kBlock), 0, st, sums, nb);
  HIP_TRY(hipGetLastError());
  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");
  HIP_TRY(hipMemcpyAsync(host, sums + 3 * static_cast<size_t>(nb), 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(totals, host, 3 * sizeof(uint32_t));
  return LBG_OK;
}

}  // namespace

int lbg_split_count(const int32_t* offsets, int32_t n, int64_t m, int32_t mdt, int64_t* children_out,
                    void* scratch, size_t scratch_bytes, void* stream) {
  if (!children_out) return fail(LBG_EINVAL, "null children_out pointer");
  uint32_t tot[3];
  const int rc = split_scan(offsets, n, m, mdt, scratch, scratch_bytes, static_cast<hipStream_t>(stream), tot);
  if (rc) return rc;
  *children_out = tot[0];
  return LBG_OK;
}

int lbg_split_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t mdt, int64_t children, int32_t* split_offsets, int32_t* child_base,
                    int32_t* cols_out, uint32_t* weights_out, void* scratch, size_t scratch_bytes,
                    void* stream) {
  if (!split_offsets || !child_base || (m > 0 && (!cols || !cols_out)))
    return fail(LBG_EINVAL, "null split_offsets/child_base/cols/cols_out pointer");
  if (m > 0 && (weights == nullptr) != (weights_out == nullptr))
    return fail(LBG_EINVAL, "weights and weights_out must both be given or both be NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t tot[3];
  int rc = split_scan(offsets, n, m, mdt, scratch, scratch_bytes, st, tot);
  if (rc) return rc;
  if (static_cast<int64_t>(tot[0]) != children)
    return fail(LBG_EINVAL, "children = %lld, but mdt = %d gives %u child nodes",
                static_cast<long long>(children), mdt, tot[0]);
  if (static_cast<int64_t>(n) + children >= INT32_MAX)
    return fail(LBG_ERANGE, "n + children = %lld does not fit in int32", static_cast<long long>(n + children));
  const uint32_t nb = static_cast<uint32_t>((static_cast<int64_t>(n) + lbg::kSplitChunk - 1) / lbg::kSplitChunk);
  hipLaunchKernelGGL(lbg::k_split_build, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, static_cast<uint32_t>(n),
                     static_cast<uint32_t>(m), static_cast<uint32_t>(mdt), static_cast<const uint32_t*>(scratch), nb,
                     split_offsets, child_base);
  if (m > 0) {
    const int blocks = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(n) + lbg::kWaves - 1) / lbg::kWaves, 16384));
    hipLaunchKernelGGL(lbg::k_split_copy, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, cols, weights,
                       static_cast<uint32_t>(n), static_cast<uint32_t>(m), split_offsets, child_base, cols_out,
                       weights_out);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return LBG_OK;
}

size_t lbg_split_workspace_bytes(int32_t n, int64_t m, int64_t children, int32_t is_sssp) {
  if (n <= 0 || m < 0 || m > INT32_MAX || children < 0 || children > m) return 0;
  return layout(n, m, LBG_SPLIT, is_sssp ? 1 : 0, children).total;
}

int lbg_bfs_split(const int32_t* split_offsets, const int32_t* child_base, const int32_t* cols, int32_t n,
                  int64_t children, int64_t m, int32_t src, int32_t* levels_out, void* workspace,
                  size_t workspace_bytes, lbg_stats* stats, void* stream) {
  if (!child_base) return fail(LBG_EINVAL, "null child_base pointer");
  Problem P{split_offsets, cols, nullptr, nullptr, n, m, src, levels_out, workspace, workspace_bytes,
            LBG_SPLIT, 0, stats, static_cast<hipStream_t>(stream)};
  P.child_base = child_base;
  P.children = children;
  return solve(P);
}

int lbg_sssp_split(const int32_t* split_offsets, const int32_t* child_base, const int32_t* cols,
                   const uint32_t* weights, int32_t n, int64_t children, int64_t m, int32_t src,
                   uint32_t* dist_out, void* workspace, size_t workspace_bytes, lbg_stats* stats,
                   void* stream) {
  if (!child_base) return fail(LBG_EINVAL, "null child_base pointer");
  Problem P{split_offsets, cols, weights, nullptr, n, m, src, dist_out, workspace, workspace_bytes,
            LBG_SPLIT, 1, stats, static_cast<hipStream_t>(stream)};
  P.child_base = child_base;
  P.children = children;
  return solve(P);
}

size_t lbg_order_scratch_bytes(int32_t n) {
  if (n <= 0) return 0;
  const size_t nb = (static_cast<size_t>(n) + lbg::kOrdChunk - 1) / lbg::kOrdChunk;
  return align_up(sizeof(uint32_t) * (lbg::kOrdClasses * nb + 1)) + align_up(sizeof(uint32_t) * (nb + 1)) +
         align_up(sizeof(int32_t) * static_cast<size_t>(n));
}

int lbg_order_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, int32_t* order_offsets, int32_t* order_cols, uint32_t* order_weights,
                    int32_t* new_id, void* scratch, size_t scratch_bytes, void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!offsets || !order_offsets || !new_id || !scratch || (m > 0 && (!cols || !order_cols)))
    return fail(LBG_EINVAL, "null offsets/order_offsets/new_id/scratch/cols/order_cols pointer");
  if (m > 0 && (weights == nullptr) != (order_weights == nullptr))
    return fail(LBG_EINVAL, "weights and order_weights must both be given or both be NULL");
  if (reinterpret_cast<uintptr_t>(scratch) % kAlign)
    return fail(LBG_EINVAL, "scratch must be %zu-byte aligned", kAlign);
  if (scratch_bytes < lbg_order_scratch_bytes(n))
    return fail(LBG_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, lbg_order_scratch_bytes(n));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t un = static_cast<uint32_t>(n), um = static_cast<uint32_t>(m);
  const uint32_t nb = static_cast<uint32_t>((static_cast<int64_t>(n) + lbg::kOrdChunk - 1) / lbg::kOrdChunk);
  char* sc = static_cast<char*>(scratch);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(sc);
  sc += align_up(sizeof(uint32_t) * (lbg::kOrdClasses * static_cast<size_t>(nb) + 1));
  uint32_t* sums = reinterpret_cast<uint32_t*>(sc);
  sc += align_up(sizeof(uint32_t) * (static_cast<size_t>(nb) + 1));
  int32_t* order = reinterpret_cast<int32_t*>(sc);
  hipLaunchKernelGGL(lbg::k_ord_count, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, un, um, cnt, nb);
  hipLaunchKernelGGL(lbg::k_ord_scan, dim3(1), dim3(lbg::kBlock), 0, st, cnt, lbg::kOrdClasses * nb);
  hipLaunchKernelGGL(lbg::k_ord_scatter, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, un, um,
                     static_cast<const uint32_t*>(cnt), nb, order, new_id);
  hipLaunchKernelGGL(lbg::k_ord_deg_sums, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, un, um,
                     static_cast<const int32_t*>(order), sums);
  hipLaunchKernelGGL(lbg::k_ord_scan, dim3(1), dim3(lbg::kBlock), 0, st, sums, nb);
  hipLaunchKernelGGL(lbg::k_ord_offsets, dim3(nb), dim3(lbg::kBlock), 0, st, offsets, un, um,
                     static_cast<const int32_t*>(order), static_cast<const uint32_t*>(sums), nb, order_offsets);
  if (m > 0) {
    const int blocks = static_cast<int>(std::min<int64_t>((static_cast<int64_t>(n) + lbg::kWaves - 1) / lbg::kWaves, 16384));
    hipLaunchKernelGGL(lbg::k_ord_copy, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, cols, weights, un, um,
                       static_cast<const int32_t*>(order), static_cast<const int32_t*>(new_id),
                       static_cast<const int32_t*>(order_offsets), order_cols, order_weights);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return LBG_OK;
}

int lbg_sssp_ordered(const int32_t* order_offsets, const int32_t* order_cols, const uint32_t* order_weights,
                     const int32_t* new_id, int32_t n, int64_t m, int32_t src, uint32_t* dist_out,
                     void* workspace, size_t workspace_bytes, lbg_stats* stats, void* stream) {
  if (!new_id) return fail(LBG_EINVAL, "null new_id pointer");
  Problem P{order_offsets, order_cols, order_weights, nullptr, n, m, src, dist_out, workspace, workspace_bytes,
            LBG_BALANCED, 1, stats, static_cast<hipStream_t>(stream)};
  P.node_map = new_id;
  return solve(P);
}

int lbg_validate_csr(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m,
                     void* workspace, size_t workspace_bytes, void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!offsets || (m > 0 && !cols) || !workspace)
    return fail(LBG_EINVAL, "null offsets/cols/workspace pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < layout(n, m, LBG_NODE, 0).total)
    return fail(LBG_ENOMEM, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctl* ctl = static_cast<Ctl*>(workspace);
  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");
  HIP_TRY(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
  const int blocks = static_cast<int>(std::min<int64_t>(
      std::max<int64_t>((std::max<int64_t>(n, m) + lbg::kBlock - 1) / lbg::kBlock, 1), 4096));
  hipLaunchKernelGGL(lbg::k_validate, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, cols,
                     static_cast<uint32_t>(n), static_cast<uint32_t>(m), ctl);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const unsigned f = host->csr_flags;
  if (f & 1u) return fail(LBG_EINVAL, "offsets[0] != 0");
  if (f & 2u) return fail(LBG_EINVAL, "offsets decrease somewhere");
  if (f & 4u) return fail(LBG_EINVAL, "offsets[n] != m");
  if (f & 8u) return fail(LBG_EINVAL, "a column index is outside [0, n)");
  return LBG_OK;
}

const char* lbg_last_error(void) { return g_err; }

int lbg_set_bins(const lbg_bins* bins) {
  if (!bins) return fail(LBG_EINVAL, "null bins");
  if (bins->mdt < 0 || (bins->mdt > 0 && bins->mdt < static_cast<int32_t>(lbg::kMinMdt)) ||
      bins->t_wave < 0 || bins->t_block < 0 || bins->t_wave > bins->t_block)
    return fail(LBG_EINVAL, "need mdt = 0 or mdt >= %u, and 0 <= t_wave <= t_block", lbg::kMinMdt);
  std::lock_guard<std::mutex> lk(g_bins_mu);
  g_bins = *bins;
  return LBG_OK;
}

void lbg_get_bins(lbg_bins* bins) {
  if (!bins) return;
  std::lock_guard<std::mutex> lk(g_bins_mu);
  *bins = g_bins;
}

int lbg_degree_mdt(const int32_t* offsets, int32_t n, int64_t m, void* workspace,
                   size_t workspace_bytes, int32_t* mdt_out, int32_t* max_degree_out, void* stream) {
  if (n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", n);
  if (m < 0 || m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(m));
  if (!offsets || !workspace || !mdt_out) return fail(LBG_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < layout(n, m, LBG_NODE, 0).total) return fail(LBG_ENOMEM, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctl* ctl = static_cast<Ctl*>(workspace);
  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");
  const int blocks = static_cast<int>(
      std::min<int64_t>(std::max<int64_t>((static_cast<int64_t>(n) + lbg::kBlock - 1) / lbg::kBlock, 1), 4096));
  hipLaunchKernelGGL(lbg::k_deg_clear, dim3(1), dim3(lbg::kBlock), 0, st, ctl);
  hipLaunchKernelGGL(lbg::k_deg_max, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, static_cast<uint32_t>(n), ctl);
  hipLaunchKernelGGL(lbg::k_deg_hist, dim3(blocks), dim3(lbg::kBlock), 0, st, offsets, static_cast<uint32_t>(n), ctl);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *mdt_out = static_cast<int32_t>(mdt_rule(host));
  if (max_degree_out) *max_degree_out = static_cast<int32_t>(host->deg_max);
  return LBG_OK;
}

int lbg_autotune_bins(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                      int32_t n, int64_t m, const int32_t* sources, int32_t num_sources,
                      int32_t* out, void* workspace, size_t workspace_bytes, lbg_bins* best,
                      void* stream) {
  if (!sources || num_sources <= 0 || !out || !best) return fail(LBG_EINVAL, "null or empty argument");
  if (n <= 0 || m < 0 || m > INT32_MAX) return fail(LBG_EINVAL, "bad graph size");
  if (workspace_bytes < layout(n, m, LBG_BINNED, 1).total || workspace_bytes < layout(n, m, LBG_BINNED, 0).total)
    return fail(LBG_ENOMEM, "workspace too small");
  int32_t seed = 0;
  int rc = lbg_degree_mdt(offsets, n, m, workspace, workspace_bytes, &seed, nullptr, stream);
  if (rc) return rc;
  std::vector<int32_t> mdts = {std::max<int32_t>(seed, static_cast<int32_t>(lbg::kMinMdt)), 256, 1024, 4096, 16384};
  std::sort(mdts.begin(), mdts.end());
  mdts.erase(std::unique(mdts.begin(), mdts.end()), mdts.end());
  lbg_bins saved;
  lbg_get_bins(&saved);
  auto run_all = [&]() -> int {
    for (int32_t k = 0; k < num_sources; ++k) {
      int r = lbg_bfs(offsets, cols, n, m, sources[k], out, workspace, workspace_bytes, LBG_BINNED,
                      nullptr, nullptr, stream);
      if (r) return r;
      if (weights) {
        r = lbg_sssp(offsets, cols, weights, n, m, sources[k], reinterpret_cast<uint32_t*>(out), workspace,
                     workspace_bytes, LBG_BINNED, nullptr, nullptr, stream);
        if (r) return r;
      }
    }
    return LBG_OK;
  };
  if ((rc = run_all()) != LBG_OK) return rc;  // warm-up
  double best_s = -1.0;
  lbg_bins pick = saved;
  for (int32_t mdt : mdts)
    for (int32_t tw : {16, 32, 64})
      for (int32_t tb : {256, 1024}) {
        const lbg_bins b{mdt, tw, tb};
        if ((rc = lbg_set_bins(&b)) != LBG_OK) return rc;
        const auto t0 = std::chrono::steady_clock::now();
        if ((rc = run_all()) != LBG_OK) {
          (void)lbg_set_bins(&saved);
          return rc;
        }
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (best_s < 0 || t < best_s) {
          best_s = t;
          pick = b;
        }
      }
  (void)lbg_set_bins(&pick);
  *best = pick;
  return LBG_OK;
}

void lbg_profile_enable(int32_t enable, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  if (reset)
    for (lbg_profile& p : g_prof) p = lbg_profile{};
}

void lbg_profile_read(int32_t which, lbg_profile* out) {
  if (!out || which < 0 || which > 4) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  *out = g_prof[which];
}

size_t lbg_batch_workspace_bytes(int32_t num_queries, int64_t total_rows, int64_t total_arcs) {
  if (num_queries <= 0 || total_rows <= 0 || total_rows > INT32_MAX || total_arcs < 0 ||
      total_arcs > UINT32_MAX)
    return 0;
  return batch_layout(num_queries, total_rows, total_arcs).total;
}

int lbg_batch_solve(const int32_t* offsets, const int32_t* cols, const uint32_t* weights, int32_t n,
                    int64_t m, const lbg_query* queries, int32_t num_queries, uint32_t* out,
                    int64_t total_rows, int64_t total_arcs, void* workspace, size_t workspace_bytes,
                    lbg_stats* stats, void* stream) {
  return batch_solve(offsets, cols, weights, n, m, queries, num_queries, out, total_rows,
                     total_arcs, workspace, workspace_bytes, stats, static_cast<hipStream_t>(stream),
                     false);
}

int lbg_batch_solve_graph(const int32_t* offsets, const int32_t* cols, const uint32_t* weights,
                          int32_t n, int64_t m, const lbg_query* queries, int32_t num_queries,
                          uint32_t* out, int64_t total_rows, int64_t total_arcs, void* workspace,
                          size_t workspace_bytes, lbg_stats* stats, void* stream) {
  return batch_solve(offsets, cols, weights, n, m, queries, num_queries, out, total_rows,
                     total_arcs, workspace, workspace_bytes, stats, static_cast<hipStream_t>(stream),
                     true);
}

int32_t lbg_tile_edges(void) { return static_cast<int32_t>(lbg::kMinTile); }

int32_t lbg_grid_blocks(void) { return grid_blocks(); }

}  // extern "C"
