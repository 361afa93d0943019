// C ABI of the lbg library: argument checks, workspace carving, the level
// loop and kernel launches.  Declarations and contracts: include/lbg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lbg.h"
#include "lbg_kernels.hpp"

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

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool strategy_ok(int32_t s) { return s >= LBG_AUTO && s <= LBG_BALANCED; }
int32_t resolve(int32_t s) { return s == LBG_AUTO ? LBG_BALANCED : s; }

// Workspace layout.  All offsets 256-byte aligned.
struct Layout {
  size_t ctl, visited, seen[2], xfilter, dstate, node[2], eprefix[2], estart[2], tile[2], total;
  uint32_t node_cap, tile_cap, edge_cap;
};

Layout layout(int32_t n, int64_t m, int32_t strategy, int is_sssp) {
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
  } else {
    L.visited = take(sizeof(uint32_t) * words);
    L.seen[0] = take(sizeof(uint32_t) * words);
    L.seen[1] = take(sizeof(uint32_t) * words);
    L.xfilter = take(sizeof(uint32_t) * words * lbg::kXcds);
  }
  if (s == LBG_EDGE) {
    L.edge_cap = static_cast<uint32_t>(m);
    for (int b = 0; b < 2; ++b) L.node[b] = take(sizeof(int32_t) * static_cast<size_t>(m > 0 ? m : 1));
  } else {
    L.node_cap = static_cast<uint32_t>(n);
    L.tile_cap = static_cast<uint32_t>((m + lbg::kMinTile - 1) / lbg::kMinTile + 2);
    for (int b = 0; b < 2; ++b) {
      L.node[b] = take(sizeof(int32_t) * static_cast<size_t>(n));
      L.eprefix[b] = take(sizeof(uint32_t) * static_cast<size_t>(n));
      L.estart[b] = take(sizeof(int32_t) * static_cast<size_t>(n));
      L.tile[b] = take(sizeof(int32_t) * static_cast<size_t>(L.tile_cap));
    }
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
  int bal[2][2], node[2], edge[2];  // bal[is_sssp][narrow]
};

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
    g[dev].edge[0] = resident_grid(lbg::k_expand_edge<false>);
    g[dev].edge[1] = resident_grid(lbg::k_expand_edge<true>);
    done[dev] = true;
  }
  return g[dev];
}

int grid_blocks() { return grids().bal[0][1]; }

// Host side of the profiling counters (see lbg_profile_enable).
std::mutex g_prof_mu;
bool g_prof_on = false;
lbg_profile g_prof[2]{};  // [is_sssp]

struct PinnedCtl {
  Ctl* p = nullptr;
  ~PinnedCtl() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local PinnedCtl g_pinned;
thread_local std::vector<hipEvent_t> g_events;

Ctl* pinned_ctl() {
  if (!g_pinned.p) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return nullptr;
    g_pinned.p = static_cast<Ctl*>(p);
  }
  return g_pinned.p;
}

hipEvent_t event_at(size_t i) {
  while (g_events.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_events.push_back(e);
  }
  return g_events[i];
}

int64_t xsum(const Ctl* c, int k) {
  int64_t t = 0;
  for (int x = 0; x < lbg::kXcds; ++x) t += static_cast<int64_t>(c->xstat[x][k]);
  return t;
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
};

int check_common(const Problem& P) {
  if (!strategy_ok(P.strategy)) return fail(LBG_EINVAL, "unknown strategy %d", P.strategy);
  if (P.n <= 0) return fail(LBG_EINVAL, "n must be positive (got %d)", P.n);
  if (P.m < 0 || P.m > INT32_MAX)
    return fail(LBG_ERANGE, "m must be in [0, INT32_MAX] (got %lld)", static_cast<long long>(P.m));
  if (P.src < 0 || P.src >= P.n) return fail(LBG_ERANGE, "src %d outside [0, %d)", P.src, P.n);
  if (!P.offsets || !P.out || !P.ws) return fail(LBG_EINVAL, "null offsets/output/workspace pointer");
  if (P.m > 0 && !P.cols) return fail(LBG_EINVAL, "null cols pointer with m > 0");
  if (P.is_sssp && P.m > 0 && !P.weights) return fail(LBG_EINVAL, "null weights pointer with m > 0");
  if (resolve(P.strategy) == LBG_EDGE && !P.coo_src)
    return fail(LBG_EINVAL, "LBG_EDGE needs the coo_src array");
  if (reinterpret_cast<uintptr_t>(P.ws) % kAlign)
    return fail(LBG_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  const size_t need = layout(P.n, P.m, P.strategy, P.is_sssp).total;
  if (P.ws_bytes < need)
    return fail(LBG_ENOMEM, "workspace has %zu bytes, needs %zu", P.ws_bytes, need);
  return LBG_OK;
}

int solve(const Problem& P) {
  int rc = check_common(P);
  if (rc) return rc;
  const int32_t strat = resolve(P.strategy);
  const Layout Lay = layout(P.n, P.m, P.strategy, P.is_sssp);
  char* ws = static_cast<char*>(P.ws);

  KArgs a{};
  a.offsets = P.offsets;
  a.cols = P.cols;
  a.weights = P.weights;
  a.coo_src = P.coo_src;
  if (P.is_sssp) {
    a.dist = static_cast<uint32_t*>(P.out);
    a.dstate = reinterpret_cast<unsigned long long*>(ws + Lay.dstate);
  } else {
    a.levels = static_cast<int32_t*>(P.out);
    a.visited = reinterpret_cast<uint32_t*>(ws + Lay.visited);
    a.seen[0] = reinterpret_cast<uint32_t*>(ws + Lay.seen[0]);
    a.seen[1] = reinterpret_cast<uint32_t*>(ws + Lay.seen[1]);
    a.xfilter = reinterpret_cast<uint32_t*>(ws + Lay.xfilter);
  }
  for (int b = 0; b < 2; ++b) {
    a.fr[b].node = reinterpret_cast<int32_t*>(ws + Lay.node[b]);
    if (strat != LBG_EDGE) {
      a.fr[b].eprefix = reinterpret_cast<uint32_t*>(ws + Lay.eprefix[b]);
      a.fr[b].estart = reinterpret_cast<int32_t*>(ws + Lay.estart[b]);
      a.fr[b].tile_node = reinterpret_cast<int32_t*>(ws + Lay.tile[b]);
    }
  }
  a.ctl = reinterpret_cast<Ctl*>(ws + Lay.ctl);
  a.n = static_cast<uint32_t>(P.n);
  a.m = static_cast<uint32_t>(P.m);
  a.words = static_cast<uint32_t>((static_cast<size_t>(P.n) + 31) / 32);
  a.node_cap = Lay.node_cap;
  a.tile_cap = Lay.tile_cap;
  a.edge_cap = Lay.edge_cap;
  bool profiling;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    profiling = g_prof_on;
  }
  a.count_stats = (P.stats || profiling) ? 1u : 0u;

  Ctl* host = pinned_ctl();
  if (!host) return fail(LBG_EHIP, "hipHostMalloc of the readback word failed");

  const hipStream_t st = P.stream;
  const Grids& GR = grids();
  const int sv = P.is_sssp ? 1 : 0;
  // 32-bit element offsets are enough when every array stays below 4 GiB
  const bool narrow = P.n < (1 << 29) && P.m < (int64_t{1} << 30);
  const int nw = narrow ? 1 : 0;
  const int init_blocks = static_cast<int>(
      std::min<int64_t>(std::max<int64_t>((static_cast<int64_t>(P.n) + lbg::kBlock - 1) / lbg::kBlock, 1), 4096));

  if (P.is_sssp) {
    if (strat == LBG_EDGE) hipLaunchKernelGGL((lbg::k_init<true, true>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
    else hipLaunchKernelGGL((lbg::k_init<true, false>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
  } else {
    if (strat == LBG_EDGE) hipLaunchKernelGGL((lbg::k_init<false, true>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
    else hipLaunchKernelGGL((lbg::k_init<false, false>), dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, P.src);
  }
  HIP_TRY(hipGetLastError());

  auto launch = [&](uint32_t L) {
    if (P.is_sssp) {
      switch (strat) {
        case LBG_NODE: hipLaunchKernelGGL((lbg::k_expand_node<true>), dim3(GR.node[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE: hipLaunchKernelGGL((lbg::k_expand_edge<true>), dim3(GR.edge[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        default:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<true, true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_balanced<true, false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
      }
    } else {
      switch (strat) {
        case LBG_NODE: hipLaunchKernelGGL((lbg::k_expand_node<false>), dim3(GR.node[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        case LBG_EDGE: hipLaunchKernelGGL((lbg::k_expand_edge<false>), dim3(GR.edge[sv]), dim3(lbg::kBlock), 0, st, a, L); break;
        default:
          if (narrow) hipLaunchKernelGGL((lbg::k_expand_balanced<false, true>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          else hipLaunchKernelGGL((lbg::k_expand_balanced<false, false>), dim3(GR.bal[sv][nw]), dim3(lbg::kBlock), 0, st, a, L);
          break;
      }
    }
  };

  // Level loop: enqueue a batch of levels back to back (each launch reads its
  // own work size on the device), then read the tail of the next level once.
  uint32_t L = 0;
  uint32_t batch = 8;
  size_t nev = 0;
  const uint64_t level_cap = static_cast<uint64_t>(P.n) + 2;
  for (;;) {
    for (uint32_t k = 0; k < batch; ++k, ++L) {
      if (profiling) {
        hipEvent_t e = event_at(nev++);
        if (!e) return fail(LBG_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, st));
      }
      launch(L);
      HIP_TRY(hipGetLastError());
      if (profiling) {
        hipEvent_t e = event_at(nev++);
        if (!e) return fail(LBG_EHIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e, st));
      }
    }
    if (P.is_sssp) {
      hipLaunchKernelGGL(lbg::k_sssp_finish, dim3(init_blocks), dim3(lbg::kBlock), 0, st, a, L);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(host, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (host->error)
      return fail(LBG_EOVERFLOW, "device capacity guard tripped (flags 0x%x)", host->error);
    if (static_cast<uint32_t>(host->ctr[L % 3]) == 0u) break;
    if (L > level_cap)
      return fail(LBG_EINTERNAL, "more than n + 1 levels; the CSR is probably malformed");
    batch = std::min<uint32_t>(batch * 2, 64);
  }

  if (profiling) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    lbg_profile& gp = g_prof[P.is_sssp ? 1 : 0];
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
  }
  if (P.stats) {
    P.stats->levels = static_cast<int32_t>(host->levels);
    P.stats->reserved = 0;
    P.stats->frontier_entries = static_cast<int64_t>(host->frontier_entries);
    P.stats->edges_scanned = static_cast<int64_t>(host->edges_scanned);
    P.stats->updates = xsum(host, 0);
    P.stats->atomics = xsum(host, 1);
  }
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

void lbg_profile_enable(int32_t enable, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  if (reset) g_prof[0] = g_prof[1] = lbg_profile{};
}

void lbg_profile_read(int32_t is_sssp, lbg_profile* out) {
  if (!out) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  *out = g_prof[is_sssp ? 1 : 0];
}

int32_t lbg_tile_edges(void) { return static_cast<int32_t>(lbg::kMinTile); }

int32_t lbg_grid_blocks(void) { return grid_blocks(); }

}  // extern "C"
