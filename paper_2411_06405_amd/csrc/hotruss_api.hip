// hotruss_api.hip -- host side of libhotruss: argument checks, workspace
// planning and the launch sequence of the peeling method (paper, Section 3).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>
#include <map>
#include <new>
#include <functional>
#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "../../include/hotruss.h"
#include "hotruss_dev.h"
#include "hotruss_kernels.hip"
#include "hotruss_hindex.hip"

// status words per engine slot: {done, halt, live edges, unused}
#define HO_STATUS_WORDS 4

namespace hotruss {

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t MAX_LDS_ROW = 64 * 1024;  // one bitset row per workgroup in LDS
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Plan {
  uint32_t n = 0, h = 0, W = 0, evcap = 0, itcap = 0;
  uint64_t m = 0;
  bool full = true;  // decomposition (false: support only)
  size_t off_ctl, off_eid, off_eu, off_ev, off_s1, off_s2, off_srem, off_upcnt, off_upoff,
      off_scan, off_minpart, off_sup, off_rho, off_R0, off_R1, off_L[HMAX + 1],
      off_Dm[HMAX + 1], off_evl[HMAX + 1][2], off_itl[HMAX + 2], off_cix, off_len, off_tci,
      off_teid, off_acct, off_ce;
  size_t total = 0;
};

uint32_t words_per_row(uint32_t n) {
  uint32_t w = (n + 63) / 64;
  return (w + 7) / 8 * 8;  // 64-byte rows
}

uint32_t clamp_cap(uint64_t want, uint64_t lo, uint64_t hi) {
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, lo), hi);
}

bool make_plan(uint32_t n, uint64_t m, uint32_t h, const hoTuning* tune, bool full, Plan* P,
               uint64_t cap_factor = 128) {
  if (h == 0 || m >= (1ull << 31) || n == 0xffffffffu) return false;
  if (n > 1 && h > n - 1) h = n - 1;  // any h beyond n-1 is the same as n-1
  if (h == 0) h = 1;
  if (h > HMAX) return false;
  Plan p;
  p.n = n; p.m = m; p.h = h; p.full = full;
  p.W = words_per_row(n);
  // Lists are sized so that a round rarely overflows them (a round that does
  // re-runs the overflowed step from the host in windows that fit).
  p.evcap = tune && tune->event_capacity ? tune->event_capacity
                                         : clamp_cap(cap_factor * m, 1u << 16, 1u << 28);
  p.itcap = tune && tune->item_capacity ? tune->item_capacity
                                        : clamp_cap(cap_factor * m, 1u << 16, 1u << 28);
  // room for the items of any single source (two rows' worth, or a ball row's
  // words), so that a round can always be re-run one source at a time
  p.itcap = std::max<uint32_t>(p.itcap, 2 * ((n + CHUNK - 1) / CHUNK) + 4);
  const size_t rowbytes = (size_t)p.W * 8;
  if (rowbytes > MAX_LDS_ROW) return false;  // rows are built in LDS
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  p.off_ctl = take(sizeof(Ctl));
  p.off_eid = take(8 * m + 4);
  p.off_eu = take(4 * m + 4);
  p.off_ev = take(4 * m + 4);
  p.off_s1 = take(4 * m + 4);
  p.off_s2 = take(4 * m + 4);
  p.off_srem = take(8 * m + 4);
  p.off_upcnt = take(4 * (size_t)n + 4);
  p.off_upoff = take(4 * (size_t)n + 4);
  p.off_scan = take(4 * ((size_t)n / 1024 + 2));
  p.off_minpart = take(4 * MIN_PART);
  p.off_sup = take(4 * m + 4);
  p.off_rho = take(full ? 4 * m + 4 : 0);
  p.off_cix = take(full ? 8 * m + 4 : 0);
  p.off_len = take(full ? 4 * (size_t)n + 4 : 0);
  p.off_tci = take(full ? 8 * m + 4 : 0);
  p.off_teid = take(full ? 8 * m + 4 : 0);
  p.off_R0 = take(full ? 4 * m + 4 : 0);
  p.off_R1 = take(full ? 4 * m + 4 : 0);
  p.off_acct = take(full ? 6 * (4 * (size_t)n + 4) : 0);  // stats-mode work count
  p.off_ce = take(full ? 16 * m + 8 : 0);
  for (uint32_t j = 0; j <= HMAX; ++j) {
    p.off_L[j] = p.off_Dm[j] = 0;
    p.off_evl[j][0] = p.off_evl[j][1] = 0;
  }
  for (uint32_t j = 0; j <= HMAX + 1; ++j) p.off_itl[j] = 0;
  for (uint32_t j = 1; j <= h; ++j) p.off_L[j] = take(rowbytes * n);
  if (full) {
    for (uint32_t j = 1; j <= h; ++j) {
      // level-1 change marks are read only when level 1 is the top level
      if (j >= 2 || h == 1) p.off_Dm[j] = take(rowbytes * n);
      const size_t c = (j == 1) ? 2 * m + 2 : p.evcap;
      p.off_evl[j][0] = take(8 * c);
      p.off_evl[j][1] = take(8 * c);
    }
    for (uint32_t j = 2; j <= h + 1; ++j) p.off_itl[j] = take(sizeof(Item) * (size_t)p.itcap);
  }
  p.total = o + ALIGN;  // slack for aligning the caller's base pointer
  *P = p;
  return true;
}

// Workspace of the truss extraction: validation state, edge ids, and the
// union-find arrays (parent, touched) plus a counter, after the plan.
bool make_topo_plan(uint32_t n, uint64_t m, Plan* P, size_t* off_cc) {
  if (m >= (1ull << 31) || n == 0xffffffffu) return false;
  Plan p;
  p.n = n; p.m = m; p.h = 0; p.full = false;
  p.W = words_per_row(n);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  p.off_ctl = take(sizeof(Ctl));
  p.off_eid = take(8 * m + 4);
  p.off_eu = take(4 * m + 4);
  p.off_ev = take(4 * m + 4);
  p.off_s1 = take(4 * m + 4);
  p.off_s2 = take(4 * m + 4);
  p.off_srem = take(8 * m + 4);
  p.off_upcnt = take(4 * (size_t)n + 4);
  p.off_upoff = take(4 * (size_t)n + 4);
  p.off_scan = take(4 * ((size_t)n / 1024 + 2));
  p.off_minpart = take(4 * MIN_PART);
  p.off_sup = take(4 * m + 4);
  p.off_rho = p.off_R0 = p.off_R1 = p.off_cix = p.off_len = p.off_tci = p.off_teid = 0;
  p.off_acct = 0;
  p.off_ce = 0;
  for (uint32_t j = 0; j <= HMAX; ++j) {
    p.off_L[j] = p.off_Dm[j] = 0;
    p.off_evl[j][0] = p.off_evl[j][1] = 0;
  }
  for (uint32_t j = 0; j <= HMAX + 1; ++j) p.off_itl[j] = 0;
  *off_cc = take(8 * (size_t)n + 64);  // parent [n], touched [n], counter
  p.total = o + ALIGN;
  *P = p;
  return true;
}

int g_num_cu = 0;
std::once_flag g_once;

int num_cu() {
  std::call_once(g_once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess)
      g_num_cu = 256;
  });
  return g_num_cu > 0 ? g_num_cu : 256;
}

unsigned grid_for(size_t items, unsigned per_block, unsigned cap_mult = 16) {
  size_t g = (items + per_block - 1) / per_block;
  size_t cap = (size_t)num_cu() * cap_mult;
  if (g > cap) g = cap;
  if (g == 0) g = 1;
  return (unsigned)g;
}

Dev carve(const Plan& p, void* ws, const uint32_t* rp, const uint32_t* ci, uint32_t* t,
          uint32_t* rho) {
  uintptr_t base = ((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN;
  auto at = [&](size_t off) { return (void*)(base + off); };
  Dev d;
  memset(&d, 0, sizeof d);
  d.rp = rp; d.ci = ci;
  d.n = p.n; d.m = (uint32_t)p.m; d.h = p.h; d.W = p.W;
  d.nnz = (uint32_t)(2 * p.m);
  d.evcap = p.evcap;
  d.itcap = p.itcap;
  d.nminpart = 1;  // set by the engine to the grid width of its minimum kernels
  d.ctl = (Ctl*)at(p.off_ctl);
  d.eid = (uint32_t*)at(p.off_eid);
  d.eu = (uint32_t*)at(p.off_eu);
  d.ev = (uint32_t*)at(p.off_ev);
  d.s1 = (uint32_t*)at(p.off_s1);
  d.s2 = (uint32_t*)at(p.off_s2);
  d.srem = (uint32_t*)at(p.off_srem);
  d.up_cnt = (uint32_t*)at(p.off_upcnt);
  d.up_off = (uint32_t*)at(p.off_upoff);
  d.scan_tmp = (uint32_t*)at(p.off_scan);
  d.minpart = (uint32_t*)at(p.off_minpart);
  d.self = nullptr;   // the engine's device-resident copy
  d.serial = 0;
  d.spart = nullptr;  // set in stats mode
  d.status = nullptr;
  d.sup = (uint32_t*)at(p.off_sup);
  d.t = t;
  d.rho = rho ? rho : (p.full ? (uint32_t*)at(p.off_rho) : nullptr);
  if (p.full) {
    d.R[0] = (uint32_t*)at(p.off_R0);
    d.R[1] = (uint32_t*)at(p.off_R1);
    d.cix = (uint32_t*)at(p.off_cix);
    d.len = (uint32_t*)at(p.off_len);
    d.tci = (uint32_t*)at(p.off_tci);
    d.teid = (uint32_t*)at(p.off_teid);
    d.ce = (uint64_t*)at(p.off_ce);
    uint32_t* acct = (uint32_t*)at(p.off_acct);
    const size_t na = (size_t)p.n + 1;
    d.acct_ball = acct;
    d.acct_deg = acct + na;
    d.acct_stamp = acct + 2 * na;
    d.acct_vstamp = acct + 3 * na;
    d.acct_list = acct + 4 * na;
    d.acct_vlist = acct + 5 * na;
  }
  for (uint32_t j = 1; j <= p.h; ++j) {
    d.L[j] = (uint64_t*)at(p.off_L[j]);
    if (p.full) {
      d.Dm[j] = p.off_Dm[j] ? (uint64_t*)at(p.off_Dm[j]) : nullptr;
      d.evl[j][0] = (uint64_t*)at(p.off_evl[j][0]);
      d.evl[j][1] = (uint64_t*)at(p.off_evl[j][1]);
    }
  }
  if (p.full)
    for (uint32_t j = 2; j <= p.h + 1; ++j) d.itl[j] = (Item*)at(p.off_itl[j]);
  return d;
}

thread_local hoStats t_stats;

// A HIP event destroyed with its scope.
struct EventGuard {
  hipEvent_t e = nullptr;
  EventGuard() = default;
  EventGuard(const EventGuard&) = delete;
  EventGuard& operator=(const EventGuard&) = delete;
  ~EventGuard() {
    if (e) (void)hipEventDestroy(e);
  }
};

#define HIPCHK(x)                             \
  do {                                        \
    if ((x) != hipSuccess) return HO_ERR_HIP; \
  } while (0)

#define HOCHK(x)                      \
  do {                                \
    const hoStatus st_ = (x);         \
    if (st_ != HO_OK) return st_;     \
  } while (0)

// Canonical edge ids, ball build and initial h-support into out_sup.
// CSR validation and canonical edge ids (slot <-> edge maps).
void run_topology(const Dev& d, hipStream_t s) {
  const unsigned T = 256;
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, d.ctl, d.m);
  hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(d.n + 1, T)), dim3(T), 0, s, d);
  hipLaunchKernelGGL(k_row_upper, dim3(grid_for(d.n, T / WAVE)), dim3(T), 0, s, d);
  const uint32_t nb = (d.n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan1, dim3(nb ? nb : 1), dim3(256), 0, s, d.up_cnt, d.up_off,
                     d.scan_tmp, d.n);
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(64), 0, s, d.scan_tmp, nb);
  hipLaunchKernelGGL(k_scan3, dim3(grid_for(d.n, T)), dim3(T), 0, s, d.up_off, d.scan_tmp, d.n);
  hipLaunchKernelGGL(k_edge_ids, dim3(grid_for(d.n, T / WAVE)), dim3(T), 0, s, d);
}

hoStatus run_init(const Dev& d, uint32_t* out_sup, const hoTuning* tune, hipStream_t s,
                  hipEvent_t sup0 = nullptr, hipEvent_t sup1 = nullptr) {
  const unsigned T = 256;
  run_topology(d, s);
  const size_t lds = (size_t)d.W * 8;
  const unsigned rows_grid = grid_for(d.n, 1, 64);
  hipLaunchKernelGGL(k_build_L1, dim3(rows_grid), dim3(T), lds, s, d);
  const uint32_t dthr = tune && tune->dense_threshold ? tune->dense_threshold : 32;
  if (d.h >= 2) hipLaunchKernelGGL(k_build_L2, dim3(rows_grid), dim3(T), lds, s, d, dthr);
  for (uint32_t j = 3; j <= d.h; ++j)
    hipLaunchKernelGGL(k_build_Lj, dim3(rows_grid), dim3(T), 0, s, d, j);
  uint32_t epw = tune && tune->edges_per_wave ? tune->edges_per_wave : 0;
  if (!epw) epw = d.W <= 8 ? 16 : d.W <= 32 ? 4 : 1;
  if (sup0) HIPCHK(hipEventRecord(sup0, s));
  const bool wide = tune && tune->word_bits == 128;
#define HO_SUPINIT(G)                                                                       \
  do {                                                                                      \
    if (wide)                                                                               \
      hipLaunchKernelGGL((k_support_init<G, 2>), dim3(grid_for(d.m, T / G)), dim3(T), 0, s, \
                         d, out_sup);                                                       \
    else                                                                                    \
      hipLaunchKernelGGL((k_support_init<G, 1>), dim3(grid_for(d.m, T / G)), dim3(T), 0, s, \
                         d, out_sup);                                                       \
  } while (0)
  if (epw >= 16) HO_SUPINIT(4);
  else if (epw >= 8) HO_SUPINIT(8);
  else if (epw >= 4) HO_SUPINIT(16);
  else if (epw >= 2) HO_SUPINIT(32);
  else HO_SUPINIT(64);
#undef HO_SUPINIT
  if (sup1) HIPCHK(hipEventRecord(sup1, s));
  HIPCHK(hipGetLastError());
  return HO_OK;
}

// Launch geometry of the round kernels (x: workgroups per slot).
struct RoundGrid {
  unsigned jump, mark, level, support;
  unsigned lv_threads;  // k_level's workgroup shape: LV_WIDE_THREADS or LV_NARROW_THREADS
};

RoundGrid plain_grid(uint64_t m, const hoTuning* tune) {
  RoundGrid g;
  const unsigned wide = tune && tune->grid_blocks ? tune->grid_blocks : (unsigned)num_cu() * 8;
  g.jump = std::min<unsigned>(MIN_PART, grid_for(m, 256, 4));
  g.mark = std::max(1u, std::min(wide, grid_for(m, 256)));
  // k_level's register use leaves room for one of its 1,024-thread
  // workgroups per CU: an eighth of the wide grid (one per CU by default)
  // runs in a single pass, where more would queue behind the first batch
  g.level = std::max(1u, std::min<unsigned>(wide, STAT_GRID) * 128 / LV_WIDE_THREADS);
  g.lv_threads = LV_WIDE_THREADS;
  g.support = std::min<unsigned>(wide, STAT_GRID);
  return g;
}

RoundGrid batch_grid(uint32_t slots, const hoTuning* tune) {
  // Up to 256 workgroups per slot (64 per CU across all slots): a slot in a
  // large round gets a wide grid while the workgroups of slots with little or
  // no work in this step return at once.  Narrower per-slot grids make every
  // step wait on the slot with the largest round.
  const unsigned total = tune && tune->grid_blocks ? tune->grid_blocks : (unsigned)num_cu() * 64;
  const unsigned per = std::max(4u, std::min(256u, total / std::max(1u, slots)));
  RoundGrid g{std::min<unsigned>(MIN_PART, per), per, std::max(1u, per * 256 / LV_NARROW_THREADS),
              per, LV_NARROW_THREADS};
  return g;
}

// Kernel kinds timed in stats mode.
enum { KT_SUPINIT = 0, KT_JUMP, KT_MARK, KT_LEVEL, KT_SUPPORT, KT_ADVANCE, KT_N };

void launch_level(const Dev* devs, uint32_t S, const RoundGrid& g, hipStream_t s, uint32_t j) {
  if (g.lv_threads == LV_WIDE_THREADS)
    hipLaunchKernelGGL((k_level<LV_WIDE_THREADS, LV_WIDE_CAP>), dim3(g.level, S),
                       dim3(LV_WIDE_THREADS), 0, s, devs, j);
  else
    hipLaunchKernelGGL((k_level<LV_NARROW_THREADS, LV_NARROW_CAP>), dim3(g.level, S),
                       dim3(LV_NARROW_THREADS), 0, s, devs, j);
}

void launch_step(const Dev* devs, uint32_t S, uint32_t hmax, const RoundGrid& g, hipStream_t s) {
  const unsigned T = 256;
  hipLaunchKernelGGL(k_mark, dim3(g.mark, S), dim3(T), 0, s, devs);
  for (uint32_t j = 2; j <= hmax; ++j)
    launch_level(devs, S, g, s, j);
  hipLaunchKernelGGL(k_support, dim3(g.support, S), dim3(T), 0, s, devs);
  hipLaunchKernelGGL(k_end, dim3(g.jump, S), dim3(T), 0, s, devs);
}

// Compact again once a tenth of the live edges have been peeled since the
// last compaction (a compaction reads and writes the active slots once).
uint32_t compact_next(uint32_t live) { return live - live / 10; }

void launch_compact(const Dev& d, hipStream_t s) {
  const unsigned T = 256;
  const unsigned g = grid_for(d.n, T / WAVE);
  hipLaunchKernelGGL(k_compact_rows, dim3(g), dim3(T), 0, s, d);
  hipLaunchKernelGGL(k_compact_commit, dim3(g), dim3(T), 0, s, d);
}

hoStatus read_ctl(const Dev& d, Ctl* host, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HO_OK;
}

// Timing of host-driven round steps (stats mode).
struct StepTimer {
  bool on = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double* kms = nullptr;
  uint64_t* kl = nullptr;
  hoStatus begin(hipStream_t s) {
    if (on) HIPCHK(hipEventRecord(e0, s));
    return HO_OK;
  }
  hoStatus end(hipStream_t s, int kind) {
    if (!on) return HO_OK;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    kms[kind] += ms;
    kl[kind] += 1;
    return HO_OK;
  }
};

// Recovery sources of a step (see k_fill_level / k_fill_support).
uint64_t recovery_sources(const Dev& d, const Ctl& c, uint32_t step) {
  const uint32_t p = c.r & 1;
  const uint64_t nA = 2ull * c.nR;
  if (step <= d.h) {
    if (step == 2) return nA;
    const uint64_t nB = c.ovf[step - 1][p] ? (uint64_t)d.n * d.W * 64
                                           : std::min<uint64_t>(c.nev[step - 1][p], d.evcap);
    return nA + nB;
  }
  if (c.ovf[d.h][p]) return (uint64_t)d.n * d.W * 64;
  if (d.h == 1) return nA;
  return std::min<uint64_t>(c.nev[d.h][p], d.evcap);
}

// Re-run one step (2..h: level, h+1: support update) of the current round
// whose work list overflowed: its work items are re-created from their
// sources a window at a time (halving the window whenever the list would
// overflow again) and the ordinary step kernel runs on each window.
hoStatus recover_step(const Dev& d, const RoundGrid& g, hipStream_t s, uint32_t step,
                      StepTimer& tm) {
  const unsigned T = 256;
  const Dev* dp = d.self;
  const uint32_t list = step;  // level j uses list j, the support update list h+1
  Ctl c;
  HOCHK(read_ctl(d, &c, s));
  const uint64_t total = recovery_sources(d, c, step);
  uint64_t lo = 0, win = std::max<uint64_t>(total, 1);
  const unsigned fill_grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + T - 1) / T, (uint64_t)num_cu() * 16));
  // at least one window, also when the step has no sources: the window start
  // is what clears the halt
  do {
    const uint64_t hi = std::min(total, lo + win);
    HOCHK(tm.begin(s));
    hipLaunchKernelGGL(k_window_begin, dim3(1), dim3(64), 0, s, dp, list);
    if (step <= d.h) hipLaunchKernelGGL(k_fill_level, dim3(fill_grid), dim3(T), 0, s, dp, step, lo, hi);
    else hipLaunchKernelGGL(k_fill_support, dim3(fill_grid), dim3(T), 0, s, dp, lo, hi);
    HOCHK(tm.end(s, step <= d.h ? KT_LEVEL : KT_SUPPORT));
    HOCHK(read_ctl(d, &c, s));
    if (c.iovf[list]) {
      if (hi - lo == 1) return HO_ERR_INTERNAL;  // one source's items exceed the list
      win = std::max<uint64_t>(1, (hi - lo) / 2);
      continue;
    }
    HOCHK(tm.begin(s));
    if (step <= d.h) launch_level(dp, 1, g, s, step);
    else hipLaunchKernelGGL(k_support, dim3(g.support), dim3(T), 0, s, dp);
    HOCHK(tm.end(s, step <= d.h ? KT_LEVEL : KT_SUPPORT));
    if (d.spart) {
      if (step <= d.h) hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 0u, 5u, g.level);
      else hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 5u, 3u, g.support);
    }
    lo = hi;
    win = std::min<uint64_t>(std::max<uint64_t>(total, 1), win * 2);
  } while (lo < total);
  hipLaunchKernelGGL(k_recovery_end, dim3(1), dim3(64), 0, s, dp);
  HIPCHK(hipGetLastError());
  return HO_OK;
}

// Run one slot's round steps from `from` on (2..h: level j, h+1: support
// update) and end the round, from the host; a step whose list kernel halts on
// an overflowed work list (or every step from `from` when recover_first) is
// re-run in windows by recover_step.
hoStatus steps_host(const Dev& d, const RoundGrid& g, hipStream_t s, uint32_t from,
                    bool recover_first, StepTimer& tm) {
  const unsigned T = 256;
  const Dev* dp = d.self;
  Ctl c;
  for (uint32_t step = from; step <= d.h + 1; ++step) {
    bool recover = recover_first && step == from;
    if (!recover) {
      HOCHK(tm.begin(s));
      if (step <= d.h) launch_level(dp, 1, g, s, step);
      else hipLaunchKernelGGL(k_support, dim3(g.support), dim3(T), 0, s, dp);
      HOCHK(tm.end(s, step <= d.h ? KT_LEVEL : KT_SUPPORT));
      if (d.spart) {
        if (step <= d.h) hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 0u, 5u, g.level);
        else hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 5u, 3u, g.support);
      }
      HOCHK(read_ctl(d, &c, s));
      recover = c.halt != 0;
    }
    if (recover) HOCHK(recover_step(d, g, s, step, tm));
  }
  if (d.spart) {
    // stats mode: the method-level work count of this round (not timed)
    const unsigned ag = (unsigned)num_cu() * 4;
    hipLaunchKernelGGL(k_acct_round1, dim3(ag), dim3(T), 0, s, dp);
    hipLaunchKernelGGL(k_acct_round2, dim3(ag), dim3(T), 0, s, dp);
    hipLaunchKernelGGL(k_acct_round3, dim3(ag), dim3(T), 0, s, dp);
    hipLaunchKernelGGL(k_acct_reset, dim3(1), dim3(64), 0, s, dp);
  }
  HOCHK(tm.begin(s));
  hipLaunchKernelGGL(k_end, dim3(g.jump), dim3(T), 0, s, dp);
  HOCHK(tm.end(s, KT_ADVANCE));
  HIPCHK(hipGetLastError());
  return HO_OK;
}

// ----------------------------------------------------------------- engine
// A pool of device memory, S slots and a queue of decompositions.  Every
// replay of the captured step graph advances each active slot by one of its
// own peel rounds; finished slots are retired and queued graphs admitted
// between graph launches (continuous batching).  The plain entry point is the
// same engine with one slot and a full-GPU grid.

struct Request {
  const uint32_t* rp = nullptr;
  const uint32_t* ci = nullptr;
  uint32_t n = 0, h = 0;
  uint64_t m = 0;
  uint32_t* t = nullptr;
  uint32_t* rho = nullptr;
  hoTuning tune{};
  bool has_tune = false;
  int state = 0;  // 0 queued, 1 running, 2 finished, 3 cancelled
  hoStatus result = HO_OK;
  Plan plan;
  int slot = -1;
  size_t off = 0;
};

class Pool {  // first-fit allocator over [lo, hi), 256-byte granules
 public:
  void reset(size_t lo, size_t hi) {
    free_.clear();
    if (hi > lo) free_[lo] = hi - lo;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t b = 0;
    for (auto& kv : free_) b = std::max(b, kv.second);
    return b;
  }

 private:
  std::map<size_t, size_t> free_;
};

// Instantiated step graphs, kept for the life of the process: a graph's
// kernel nodes hold the descriptor array's address and the grid, so the key
// is those plus the device.  Beyond GRAPH_CACHE keys an engine owns its graphs.
struct GraphKey {
  int dev;
  const void* devs;
  uint32_t S, hmax, jump, mark, level, support;
  bool operator==(const GraphKey& o) const {
    return dev == o.dev && devs == o.devs && S == o.S && hmax == o.hmax && jump == o.jump &&
           mark == o.mark && level == o.level && support == o.support;
  }
};
struct GraphCacheEntry {
  GraphKey key;
  hipGraphExec_t exec[3];
};
constexpr size_t GRAPH_CACHE = 64;
std::mutex g_graph_mu;
std::vector<GraphCacheEntry> g_graph_cache;

// Engine header: S slot descriptors, S {done, halt} status pairs, the stats
// counters and the control block of an idle slot (finished, so every round
// kernel returns at once).
size_t engine_header_bytes(uint32_t S) {
  return up(sizeof(Dev) * S) + up(4ull * HO_STATUS_WORDS * S) + up(4ull * NSTAT * STAT_GRID) +
         up(sizeof(Ctl));
}

// Pinned host buffers and events of the plain entry point, kept per host
// thread and reused by its later calls (calls on one thread never overlap).
// They live until the process ends: freeing them from a thread-exit
// destructor could run after the HIP runtime has shut down.
struct HostCache {
  void* pinned = nullptr;
  size_t bytes = 0;
  int dev = -1;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // two polling, two timing
  hoStatus ensure(size_t need) {
    int d = 0;
    HIPCHK(hipGetDevice(&d));
    if (d != dev) {  // events belong to the device current at creation
      for (auto& e : ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
      }
      HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
      HIPCHK(hipEventCreate(&ev[2]));
      HIPCHK(hipEventCreate(&ev[3]));
      dev = d;
    }
    if (need > bytes) {
      if (pinned) (void)hipHostFree(pinned);
      pinned = nullptr;
      bytes = 0;
      HIPCHK(hipHostMalloc(&pinned, need, hipHostMallocDefault));
      bytes = need;
    }
    return HO_OK;
  }
};

HostCache& host_cache() {
  static thread_local HostCache* c = new HostCache();
  return *c;
}

// Pinned bytes an engine of S slots polls and stages through.
size_t host_bytes(uint32_t S) {
  return up(8ull * HO_STATUS_WORDS * S + sizeof(Ctl)) + 2 * sizeof(Dev) * (size_t)S;
}

class Engine {
 public:
  hipStream_t s = nullptr;
  uintptr_t base = 0;
  size_t bytes = 0;
  uint32_t S = 1, hmax = 1;
  uint64_t cap_factor = 128;
  RoundGrid g{};
  bool plain = false;
  Dev* devs_d = nullptr;
  uint32_t* status_d = nullptr;
  uint32_t* spart_d = nullptr;
  std::vector<int> slot_req;
  std::vector<Dev> slot_dev;
  std::vector<uint64_t> slot_since;  // first graph launch that can report on the slot
  std::vector<uint32_t> live_seen;   // live edges in the slot's latest status snapshot
  std::vector<uint32_t> compact_at;  // compact the slot's rows once live falls to this
  std::vector<uint8_t> compact_each; // testing: compact at every opportunity
  Pool pool;
  std::vector<Request> reqs;
  std::vector<size_t> queue;
  Ctl* idle_ctl_d = nullptr;
  uint32_t* hstat = nullptr;  // pinned: 2 buffers x S x status words, then a Ctl
  Dev* idle_h = nullptr;      // pinned: descriptor of each idle slot
  Dev* dev_h = nullptr;       // pinned: staging of each admitted slot's descriptor
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool borrowed_host = false;  // pinned buffers and events belong to the thread's cache
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  bool owns_graphs = false;
  bool copy_failed = false;
  uint64_t steps = 0;

  ~Engine() {
    if (s) (void)hipStreamSynchronize(s);  // nothing in flight may target freed host buffers
    if (owns_graphs)
      for (auto& e : exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (borrowed_host) return;
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (hstat) (void)hipHostFree(hstat);
    if (idle_h) (void)hipHostFree(idle_h);
    if (dev_h) (void)hipHostFree(dev_h);
  }

  hoStatus init(void* ws, size_t ws_bytes, uint32_t slots, uint32_t hmax_, const RoundGrid& grid,
                hipStream_t stream, bool plain_, bool borrow_host = false) {
    s = stream;
    base = ((uintptr_t)ws + ALIGN - 1) / ALIGN * ALIGN;
    if (ws_bytes < ALIGN + engine_header_bytes(slots)) return HO_ERR_WORKSPACE;
    bytes = ws_bytes - (base - (uintptr_t)ws);
    S = slots;
    hmax = hmax_;
    g = grid;
    plain = plain_;
    devs_d = (Dev*)base;
    status_d = (uint32_t*)(base + up(sizeof(Dev) * S));
    spart_d = (uint32_t*)(base + up(sizeof(Dev) * S) + up(4ull * HO_STATUS_WORDS * S));
    idle_ctl_d = (Ctl*)(base + up(sizeof(Dev) * S) + up(4ull * HO_STATUS_WORDS * S) +
                        up(4ull * NSTAT * STAT_GRID));
    pool.reset(engine_header_bytes(S), bytes);
    slot_req.assign(S, -1);
    slot_dev.assign(S, Dev{});
    slot_since.assign(S, 0);
    live_seen.assign(S, 0);
    compact_at.assign(S, 0);
    compact_each.assign(S, 0);
    if (borrow_host) {
      HostCache& hc = host_cache();
      HOCHK(hc.ensure(host_bytes(S)));
      hstat = (uint32_t*)hc.pinned;
      idle_h = (Dev*)((char*)hc.pinned + up(8ull * HO_STATUS_WORDS * S + sizeof(Ctl)));
      dev_h = idle_h + S;
      ev[0] = hc.ev[0];
      ev[1] = hc.ev[1];
      borrowed_host = true;
    } else {
      HIPCHK(hipHostMalloc((void**)&hstat, 8ull * HO_STATUS_WORDS * S + sizeof(Ctl),
                           hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&idle_h, sizeof(Dev) * S, hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&dev_h, sizeof(Dev) * S, hipHostMallocDefault));
      HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    }
    // every slot starts idle: finished status, a descriptor with no levels
    // whose control block says finished, so every round kernel returns at once
    for (uint32_t i = 0; i < HO_STATUS_WORDS * S; ++i) hstat[i] = (i % HO_STATUS_WORDS == 0) ? 1u : 0u;
    Ctl* hc = (Ctl*)(hstat + 2ull * HO_STATUS_WORDS * S);
    memset(hc, 0, sizeof(Ctl));
    hc->done = 1;
    for (uint32_t i = 0; i < S; ++i) {
      memset(&idle_h[i], 0, sizeof(Dev));
      idle_h[i].ctl = idle_ctl_d;
      idle_h[i].status = status_d + HO_STATUS_WORDS * i;
      idle_h[i].self = devs_d + i;
    }
    HIPCHK(hipMemcpyAsync(idle_ctl_d, hc, sizeof(Ctl), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(status_d, hstat, 4ull * HO_STATUS_WORDS * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(devs_d, idle_h, sizeof(Dev) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return HO_OK;
  }

  size_t need_bytes(uint32_t n, uint64_t m, uint32_t h, const hoTuning* tune, Plan* p) const {
    if (!make_plan(n, m, h, tune, true, p, cap_factor)) return 0;
    return p->total;
  }

  hoStatus submit(const Request& r0, size_t* id) {
    Request r = r0;
    if (!need_bytes(r.n, r.m, r.h, r.has_tune ? &r.tune : nullptr, &r.plan)) return HO_ERR_INVALID_ARG;
    if (r.plan.h > hmax) return HO_ERR_INVALID_ARG;
    if (r.plan.total > bytes - engine_header_bytes(S)) return HO_ERR_BUDGET;
    reqs.push_back(r);
    *id = reqs.size() - 1;
    queue.push_back(*id);
    return HO_OK;
  }

  // Admit queued requests (in queue order) while a slot and memory are free.
  hoStatus admit(hipEvent_t sup0 = nullptr, hipEvent_t sup1 = nullptr) {
    for (size_t qi = 0; qi < queue.size();) {
      Request& r = reqs[queue[qi]];
      int slot = -1;
      for (uint32_t i = 0; i < S; ++i)
        if (slot_req[i] < 0) { slot = (int)i; break; }
      if (slot < 0) return HO_OK;
      size_t off;
      if (!pool.alloc(r.plan.total, &off)) {
        ++qi;  // a later, smaller request may still fit
        continue;
      }
      r.slot = slot;
      r.off = off;
      r.state = 1;
      slot_req[slot] = (int)queue[qi];
      queue.erase(queue.begin() + qi);
      Dev d = carve(r.plan, (void*)(base + off), r.rp, r.ci, r.t, r.rho);
      d.self = devs_d + slot;
      d.status = status_d + HO_STATUS_WORDS * slot;
      d.nminpart = g.jump;
      if (r.has_tune)
        d.serial = r.tune.flags & (HO_FLAG_SERIAL_LEVELS | HO_FLAG_SERIAL_SUPPORT | HO_FLAG_COMPACT_EACH);
      slot_dev[slot] = d;
      slot_since[slot] = steps;
      live_seen[slot] = 0;
      compact_at[slot] = compact_next((uint32_t)r.m);
      compact_each[slot] = r.has_tune && (r.tune.flags & HO_FLAG_COMPACT_EACH) ? 1 : 0;
      HOCHK(start_slot(d, r.has_tune ? &r.tune : nullptr, sup0, sup1));
    }
    return HO_OK;
  }

  hoStatus start_slot(const Dev& d, const hoTuning* tune, hipEvent_t sup0 = nullptr,
                      hipEvent_t sup1 = nullptr) {
    const unsigned T = 256;
    hipLaunchKernelGGL(k_fill32, dim3(grid_for(d.m, T)), dim3(T), 0, s, d.t, (size_t)d.m, 0u);
    for (uint32_t j = 1; j <= d.h; ++j)
      if (d.Dm[j])
        hipLaunchKernelGGL(k_fill64, dim3(grid_for((size_t)d.n * d.W, T)), dim3(T), 0, s, d.Dm[j],
                           (size_t)d.n * d.W, 0ull);
    HOCHK(run_init(d, d.sup, tune, s, sup0, sup1));
    hipLaunchKernelGGL(k_init_rows, dim3(grid_for(d.nnz, T)), dim3(T), 0, s, d);
    const size_t i = (size_t)(d.self - devs_d);
    dev_h[i] = d;
    HIPCHK(hipMemcpyAsync(d.self, &dev_h[i], sizeof(Dev), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_post_init, dim3(1), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_first_min, dim3(g.jump), dim3(T), 0, s, d.self);
    HIPCHK(hipGetLastError());
    return HO_OK;
  }

  hoStatus ensure_graphs() {
    if (exec[0]) return HO_OK;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const GraphKey key{dev, devs_d, S, hmax, g.jump, g.mark, g.level, g.support};
    {
      std::lock_guard<std::mutex> lk(g_graph_mu);
      for (auto& e : g_graph_cache)
        if (e.key == key) {
          for (int i = 0; i < 3; ++i) exec[i] = e.exec[i];
          return HO_OK;
        }
    }
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    const uint32_t sizes[3] = {4, 32, 128};
    hoStatus st = HO_OK;
    for (int i = 0; i < 3 && st == HO_OK; ++i) {
      hipGraph_t graph;
      if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = HO_ERR_HIP;
        break;
      }
      for (uint32_t k = 0; k < sizes[i]; ++k) launch_step(devs_d, S, hmax, g, cap);
      if (hipStreamEndCapture(cap, &graph) != hipSuccess) {
        st = HO_ERR_HIP;
        break;
      }
      if (hipGraphInstantiate(&exec[i], graph, nullptr, nullptr, 0) != hipSuccess) st = HO_ERR_HIP;
      (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cap);
    if (st != HO_OK) return st;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (g_graph_cache.size() < GRAPH_CACHE) {
      GraphCacheEntry e{key, {exec[0], exec[1], exec[2]}};
      g_graph_cache.push_back(e);
    } else {
      owns_graphs = true;
    }
    return HO_OK;
  }

  bool busy() const {
    for (int r : slot_req)
      if (r >= 0) return true;
    return false;
  }

  // Retire finished slots seen in the status snapshot taken after graph
  // launch `at`; returns whether an active slot halted.  A slot admitted
  // after that launch was enqueued is not described by the snapshot.
  bool retire(const uint32_t* st, uint64_t at) {
    bool halted = false;
    for (uint32_t i = 0; i < S; ++i) {
      const int ri = slot_req[i];
      if (ri < 0 || at < slot_since[i]) continue;
      const uint32_t* sw = st + HO_STATUS_WORDS * i;
      if (sw[1]) halted = true;
      if (!sw[0]) {
        live_seen[i] = sw[2];
        continue;
      }
      Request& r = reqs[ri];
      r.state = 2;
      r.result = sw[0] == 2 ? HO_ERR_BAD_CSR : HO_OK;
      // park the slot before its memory can be handed to another request:
      // replays already in flight still read the old, finished control block
      if (hipMemcpyAsync(devs_d + i, &idle_h[i], sizeof(Dev), hipMemcpyHostToDevice, s) !=
          hipSuccess)
        copy_failed = true;
      pool.release(r.off, r.plan.total);
      slot_req[i] = -1;
    }
    return halted;
  }

  // Compact the adjacency rows of running slots whose live edge count halved
  // since the last compaction (enqueued after the launches in flight, so it
  // runs at a round boundary; the kernels do nothing for a slot that has
  // finished or halted meanwhile).
  hoStatus maybe_compact() {
    for (uint32_t i = 0; i < S; ++i) {
      if (slot_req[i] < 0 || live_seen[i] == 0) continue;
      if (!compact_each[i] && live_seen[i] > compact_at[i]) continue;
      launch_compact(slot_dev[i], s);
      compact_at[i] = compact_next(live_seen[i]);
      live_seen[i] = 0;
    }
    HIPCHK(hipGetLastError());
    return HO_OK;
  }

  // Finish the current round of every halted slot from the host.
  hoStatus recover_halts() {
    HIPCHK(hipStreamSynchronize(s));
    StepTimer tm;
    for (uint32_t i = 0; i < S; ++i) {
      if (slot_req[i] < 0) continue;
      Ctl c;
      HOCHK(read_ctl(slot_dev[i], &c, s));
      if (!c.halt) continue;
      if (c.halt_step < 2 || c.halt_step > slot_dev[i].h + 1) return HO_ERR_INTERNAL;
      HOCHK(steps_host(slot_dev[i], g, s, c.halt_step, true, tm));
      HOCHK(read_ctl(slot_dev[i], &c, s));
      if (c.halt) return HO_ERR_INTERNAL;  // the round must have ended
    }
    return HO_OK;
  }

  // Replay the step graph until no slot is active and the queue is empty
  // (or max_launches replays have been launched), two replays in flight, the
  // slots' status words copied to pinned memory after each.
  // Progress on stderr for long calls (environment HOTRUSS_PROGRESS set): at
  // most every 10 s, from the host loop that drives the work.
  void report_progress(std::chrono::steady_clock::time_point& last) {
    static const bool on = std::getenv("HOTRUSS_PROGRESS") != nullptr;
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    if (now - last < std::chrono::seconds(10)) return;
    last = now;
    uint32_t active = 0;
    uint64_t live = 0;
    for (uint32_t i = 0; i < S; ++i)
      if (slot_req[i] >= 0) {
        ++active;
        live += live_seen[i];
      }
    size_t finished = 0;
    for (const Request& r : reqs) finished += r.state >= 2;
    std::fprintf(stderr, "[hotruss] %llu graph launches: %zu finished, %u running (%llu live edges), %zu queued\n",
                 (unsigned long long)steps, finished, active, (unsigned long long)live, queue.size());
    std::fflush(stderr);
  }

  hoStatus run(uint64_t max_launches = UINT64_MAX) {
    HOCHK(admit());
    if (!busy()) return HO_OK;
    HOCHK(ensure_graphs());
    auto last_report = std::chrono::steady_clock::now();
    uint64_t launched = 0;
    uint64_t buf_at[2] = {0, 0};
    int head = 0, inflight = 0;
    int calm = 2;  // graph launches since the last halt (saturating)
    while (true) {
      while (inflight < 2 && busy() && launched < max_launches) {
        const int buf = (head + inflight) & 1;
        // short graphs right after a halt (overflowing rounds tend to come in
        // runs, and every round after a halt in the same graph is skipped)
        const int which = calm < 2 ? 0
                          : plain ? (steps == 0 ? 0 : steps < 4 ? 1 : 2) : (queue.empty() ? 2 : 1);
        HIPCHK(hipGraphLaunch(exec[which], s));
        HIPCHK(hipMemcpyAsync(hstat + HO_STATUS_WORDS * S * buf, status_d,
                              4ull * HO_STATUS_WORDS * S, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ev[buf], s));
        buf_at[buf] = steps++;
        ++launched;
        ++inflight;
      }
      if (inflight == 0) break;
      HIPCHK(hipEventSynchronize(ev[head]));
      const bool halted = retire(hstat + HO_STATUS_WORDS * S * head, buf_at[head]);
      if (copy_failed) return HO_ERR_HIP;
      head ^= 1;
      --inflight;
      if (halted) {
        HIPCHK(hipStreamSynchronize(s));
        inflight = 0;
        head = 0;
        HOCHK(recover_halts());
        calm = 0;
      } else if (calm < 2) {
        ++calm;
      }
      HOCHK(admit());
      report_progress(last_report);
      HOCHK(maybe_compact());
    }
    HIPCHK(hipStreamSynchronize(s));
    return HO_OK;
  }
};

// Debug / stats form of the plain path: every round driven from the host.
hoStatus run_rounds_host(const Dev& d, const RoundGrid& g, hipStream_t s, bool timed, double* kms,
                         uint64_t* klaunch) {
  const unsigned T = 256;
  const Dev* dp = d.self;
  StepTimer tm;
  tm.on = timed;
  tm.kms = kms;
  tm.kl = klaunch;
  EventGuard g0, g1;
  if (timed) {
    HIPCHK(hipEventCreate(&g0.e));
    HIPCHK(hipEventCreate(&g1.e));
    tm.e0 = g0.e;
    tm.e1 = g1.e;
  }
  Ctl c;
  hoStatus st = read_ctl(d, &c, s);
  uint64_t rounds = 0;
  uint32_t compact_at = compact_next(d.m);
  // Stats mode, environment HOTRUSS_ROUND_LOG = path: one line per round
  // (level, jump, peel-set size, work items, events, work counters, kernel
  // times) for studying how the work is spread over rounds.
  FILE* rlog = nullptr;
  if (timed) {
    if (const char* path = std::getenv("HOTRUSS_ROUND_LOG")) {
      rlog = std::fopen(path, "w");
      if (rlog)
        std::fprintf(rlog, "r k jump nR items2 live ev_top lv_items lv_slots lv_cand lv_probes "
                           "lv_drops su_items su_slots su_hits us_jump us_mark us_level us_support "
                           "us_advance\n");
    }
  }
  while (st == HO_OK && !c.done) {
    if (c.live <= compact_at || (d.serial & HO_FLAG_COMPACT_EACH)) {
      launch_compact(d, s);
      compact_at = compact_next(c.live);
    }
    double kms0[KT_N];
    for (int i = 0; i < KT_N; ++i) kms0[i] = timed ? kms[i] : 0.0;
    const Ctl before = c;
    if ((st = tm.begin(s)) != HO_OK) break;
    hipLaunchKernelGGL(k_mark, dim3(g.mark), dim3(T), 0, s, dp);
    if ((st = tm.end(s, KT_MARK)) != HO_OK) break;
    Ctl mid;
    if (rlog && (st = read_ctl(d, &mid, s)) != HO_OK) break;
    st = steps_host(d, g, s, 2, false, tm);
    if (st == HO_OK) st = read_ctl(d, &c, s);
    if (rlog && st == HO_OK) {
      std::fprintf(rlog, "%u %u %u %u %u %u %llu", mid.r, mid.k, mid.jump, mid.nR, mid.nit[2],
                   c.live, (unsigned long long)(c.events - before.events));
      for (uint32_t i = 0; i < NSTAT; ++i)
        std::fprintf(rlog, " %llu", (unsigned long long)(c.stat[i] - before.stat[i]));
      for (int i = KT_JUMP; i <= KT_ADVANCE; ++i) std::fprintf(rlog, " %.1f", (kms[i] - kms0[i]) * 1e3);
      std::fputc('\n', rlog);
    }
    if (++rounds > (uint64_t)d.m + 2) st = HO_ERR_INTERNAL;
  }
  if (rlog) std::fclose(rlog);
  return st;
}

// ------------------------------------------- allocation-free decomposition
// The library's own device scratch for hoTrussDecomposeNoAlloc: the slot
// descriptor, its status words and the whole workspace of one decomposition
// are carved from this array, so that the call allocates nothing.  Each GPU
// the library runs on holds its own copy until the process ends.  In host
// code the array's name is not a device address: the address comes from
// hipGetSymbolAddress, taken once per device (scratch_base), and only that
// address is used.
constexpr size_t SCRATCH_BYTES = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu[SCRATCH_MAX_DEVICES];  // one call at a time per device
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
std::once_flag g_scratch_once[SCRATCH_MAX_DEVICES];
hipError_t g_scratch_err[SCRATCH_MAX_DEVICES] = {};

// Device address of this device's scratch array (the current device must be
// `dev`); null if the runtime could not resolve it.
void* scratch_base(int dev) {
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
  });
  return g_scratch_ptr[dev];
}

// Bytes of scratch a decomposition of (n, m, h) takes (0: invalid arguments).
size_t noalloc_bytes(uint32_t n, uint64_t m, uint32_t h, Plan* p) {
  if (!make_plan(n, m, h, nullptr, true, p, 16)) return 0;
  return up(sizeof(Dev)) + up(4ull * HO_STATUS_WORDS) + p->total;
}

hoStatus check_common(const uint32_t* rp, const uint32_t* ci, uint32_t n, uint64_t m, uint32_t h,
                      const void* out, void* ws) {
  if (h == 0) return HO_ERR_INVALID_ARG;
  if (m >= (1ull << 31)) return HO_ERR_INVALID_ARG;
  if (m == 0) return HO_OK;
  if (!rp || !ci || !out || !ws || n == 0) return HO_ERR_INVALID_ARG;
  return HO_OK;
}

// ---------------------------------------------------- H-index fixpoint
constexpr uint32_t HX_CHUNKS = 8;  // vertex chunks of an asynchronous sweep

// Workspace of the H-index method: the support-only plan (balls of G, edge
// ids, H in `sup`), then the method's own arrays; the path keys follow at
// `base` and take one (h <= 2) or two (h >= 3) u32 per ball member.
struct HxPlan {
  Plan p;
  size_t off_wp, off_cnt, off_boff, off_dirty, off_touched, off_tbits, off_tlist, off_ord,
      off_cbound, off_ctr, off_stat, off_dmask, off_tmin, off_bigctr, off_bigu, off_bigoff,
      off_cmask, base;
};

bool make_hx_plan(uint32_t n, uint64_t m, uint32_t h, HxPlan* out) {
  HxPlan q;
  if (!make_plan(n, m, h, nullptr, false, &q.p)) return false;
  size_t o = q.p.total - ALIGN;
  auto take = [&](size_t bytes) { size_t r = o; o += up(bytes); return r; };
  const size_t W = q.p.W;
  q.off_wp = take(4 * W * n);
  q.off_cnt = take(4 * (size_t)n + 4);
  q.off_boff = take(8 * ((size_t)n + 1));
  q.off_dirty = take(4 * (size_t)n + 4);
  q.off_touched = take(4 * (size_t)n + 4);
  q.off_tbits = take(8 * W);
  q.off_tlist = take(4 * W);
  q.off_ord = take(4 * m + 4);
  q.off_cbound = take(4 * (HX_CHUNKS + 1));
  q.off_ctr = take(64);
  q.off_stat = take(64);
  q.off_dmask = take(8 * (size_t)n + 8);
  q.off_tmin = take(4 * (size_t)n + 4);
  q.off_bigctr = take(8);
  q.off_bigu = take(4 * (size_t)n + 4);
  q.off_bigoff = take(4 * (size_t)n + 4);
  q.off_cmask = take(8 * (size_t)n + 8);
  q.base = o;
  *out = q;
  return true;
}

size_t hx_key_bytes(uint64_t members) { return up(4 * members + 4); }

}  // namespace
}  // namespace hotruss

using namespace hotruss;

struct hoSession {
  Engine eng;
  std::mutex mu;
};

extern "C" {

const char* hoStatusString(hoStatus s) {
  switch (s) {
    case HO_OK: return "ok";
    case HO_ERR_INVALID_ARG: return "invalid argument";
    case HO_ERR_BAD_CSR: return "malformed CSR";
    case HO_ERR_WORKSPACE: return "workspace too small";
    case HO_ERR_HIP: return "HIP runtime error";
    case HO_ERR_BUDGET: return "request exceeds the memory budget";
    case HO_ERR_CANCELLED: return "cancelled";
    case HO_ERR_BUSY: return "no free slot";
    case HO_ERR_NOT_FOUND: return "unknown ticket";
    case HO_ERR_INTERNAL: return "internal invariant violated";
  }
  return "unknown status";
}

size_t hoTrussWorkspaceBytes(uint32_t n, uint64_t m, uint32_t h, const hoTuning* tune) {
  Plan p;
  if (!make_plan(n, m, h, tune, true, &p)) return 0;
  return p.total + engine_header_bytes(1) + ALIGN;
}

hoStatus hoTrussHSupport(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n, uint64_t m,
                         uint32_t h, uint32_t* out_support, void* workspace,
                         size_t workspace_bytes, const hoTuning* tune, hipStream_t stream) {
  hoStatus st = check_common(row_ptr, col_idx, n, m, h, out_support, workspace);
  if (st != HO_OK || m == 0) return st;
  Plan p;
  if (!make_plan(n, m, h, tune, false, &p)) return HO_ERR_INVALID_ARG;
  if (workspace_bytes < p.total) return HO_ERR_WORKSPACE;
  Dev d = carve(p, workspace, row_ptr, col_idx, nullptr, nullptr);
  st = run_init(d, out_support, tune, stream);
  if (st != HO_OK) return st;
  Ctl c;
  st = read_ctl(d, &c, stream);
  if (st != HO_OK) return st;
  return c.err ? HO_ERR_BAD_CSR : HO_OK;
}

hoStatus hoTrussDecompose(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n,
                          uint64_t m, uint32_t h, uint32_t* out_trussness, uint32_t* out_round,
                          void* workspace, size_t workspace_bytes, const hoTuning* tune,
                          hipStream_t stream) {
  hoStatus st = check_common(row_ptr, col_idx, n, m, h, out_trussness, workspace);
  if (st != HO_OK) return st;
  if (m == 0) {
    t_stats = hoStats{};
    return HO_OK;
  }
  Plan p;
  if (!make_plan(n, m, h, tune, true, &p)) return HO_ERR_INVALID_ARG;
  if (workspace_bytes < p.total + engine_header_bytes(1) + ALIGN) return HO_ERR_WORKSPACE;
  const bool stats = tune && (tune->flags & HO_FLAG_STATS);
  const bool host_loop = stats || (tune && (tune->flags & HO_FLAG_HOST_LOOP));
  const RoundGrid g = plain_grid(m, tune);
  Engine eng;
  HOCHK(eng.init(workspace, workspace_bytes, 1, p.h, g, stream, true, true));
  Request r;
  r.rp = row_ptr; r.ci = col_idx; r.n = n; r.m = m; r.h = h;
  r.t = out_trussness; r.rho = out_round;
  if (tune) { r.tune = *tune; r.has_tune = true; }
  size_t id;
  st = eng.submit(r, &id);
  if (st == HO_ERR_BUDGET) return HO_ERR_WORKSPACE;
  HOCHK(st);
  hoStats out{};
  EventGuard es0, es1;  // destroyed on every return path
  struct { hipEvent_t e; } ev0{host_cache().ev[2]}, ev1{host_cache().ev[3]};
  if (stats) {
    HIPCHK(hipEventCreate(&es0.e));
    HIPCHK(hipEventCreate(&es1.e));
  }
  HIPCHK(hipEventRecord(ev0.e, stream));
  if (host_loop) {
    HOCHK(eng.admit(es0.e, es1.e));
    Dev d = eng.slot_dev[0];
    Ctl c;
    HOCHK(read_ctl(d, &c, stream));
    if (c.err) return HO_ERR_BAD_CSR;
    if (stats) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, es0.e, es1.e));
      out.kernel_ms[KT_SUPINIT] = ms;
      out.kernel_launches[KT_SUPINIT] = 1;
      d.spart = eng.spart_d;
      HIPCHK(hipMemsetAsync(d.spart, 0, 4ull * NSTAT * STAT_GRID, stream));
      HIPCHK(hipMemcpyAsync(d.self, &d, sizeof(Dev), hipMemcpyHostToDevice, stream));
      // method-level work count: ball sizes and degrees in G, the initial pass
      const unsigned ag = (unsigned)num_cu() * 4;
      hipLaunchKernelGGL(k_acct_init, dim3(grid_for(d.n, 4)), dim3(256), 0, stream, d.self);
      hipLaunchKernelGGL(k_acct_start, dim3(ag), dim3(256), 0, stream, d.self);
      HIPCHK(hipGetLastError());
    }
    HOCHK(run_rounds_host(d, g, stream, stats, out.kernel_ms, out.kernel_launches));
  } else {
    HOCHK(eng.run());
    if (eng.reqs[id].state != 2) return HO_ERR_INTERNAL;
    HOCHK(eng.reqs[id].result);
  }
  HIPCHK(hipEventRecord(ev1.e, stream));
  HIPCHK(hipEventSynchronize(ev1.e));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0.e, ev1.e));
  Ctl c;
  HOCHK(read_ctl(eng.slot_dev[0], &c, stream));
  if (c.err) return HO_ERR_BAD_CSR;
  if (!c.done) return HO_ERR_INTERNAL;
  out.rounds = c.r;
  out.levels = c.levels;
  out.events = c.events;
  out.overflows = c.overflows;
  out.compactions = c.compactions;
  out.device_ms = ms;
  for (uint32_t i = 0; i < NSTAT; ++i) out.work[i] = c.stat[i];
  if (stats && !c.acct_incomplete) {
    out.evaluations = c.acct_evals;
    out.alg_bytes = c.acct_bytes;
  }
  for (uint32_t j = 1; j <= std::min<uint32_t>(p.h, 16); ++j) out.level_events[j - 1] = c.levents[j];
  t_stats = out;
  return HO_OK;
}

hoStatus hoTrussDecomposeNoAlloc(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n,
                                 uint64_t m, uint32_t h, uint32_t* out_trussness,
                                 uint32_t* out_round, hipStream_t stream) {
  hoStatus st = check_common(row_ptr, col_idx, n, m, h, out_trussness, (void*)1);
  if (st != HO_OK) return st;
  if (m == 0) {
    t_stats = hoStats{};
    return HO_OK;
  }
  Plan p;
  const size_t need = noalloc_bytes(n, m, h, &p);
  if (need == 0) return HO_ERR_INVALID_ARG;
  if (need > SCRATCH_BYTES) return HO_ERR_WORKSPACE;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return HO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
  void* base = scratch_base(dev);
  if (!base) return HO_ERR_HIP;
  const unsigned T = 256;
  const uintptr_t b = (uintptr_t)base;
  Dev* dself = (Dev*)b;
  uint32_t* status = (uint32_t*)(b + up(sizeof(Dev)));
  Dev d = carve(p, (void*)(b + up(sizeof(Dev)) + up(4ull * HO_STATUS_WORDS)), row_ptr, col_idx,
                out_trussness, out_round);
  const RoundGrid g = plain_grid(m, nullptr);
  d.self = dself;
  d.status = status;
  d.nminpart = g.jump;
  // the array keeps the previous call's contents: every buffer that must
  // start at a known value is written before it is read
  hipLaunchKernelGGL(k_fill32, dim3(1), dim3(64), 0, stream, status, (size_t)HO_STATUS_WORDS, 0u);
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(d.m, T)), dim3(T), 0, stream, d.t, (size_t)d.m, 0u);
  for (uint32_t j = 1; j <= d.h; ++j)
    if (d.Dm[j])
      hipLaunchKernelGGL(k_fill64, dim3(grid_for((size_t)d.n * d.W, T)), dim3(T), 0, stream,
                         d.Dm[j], (size_t)d.n * d.W, 0ull);
  HOCHK(run_init(d, d.sup, nullptr, stream));
  hipLaunchKernelGGL(k_init_rows, dim3(grid_for(d.nnz, T)), dim3(T), 0, stream, d);
  // the descriptor goes to the device from a host stack copy (staged by the
  // runtime, so the copy is complete when the call returns)
  HIPCHK(hipMemcpyAsync(dself, &d, sizeof(Dev), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_post_init, dim3(1), dim3(64), 0, stream, d);
  hipLaunchKernelGGL(k_first_min, dim3(g.jump), dim3(T), 0, stream, dself);
  HIPCHK(hipGetLastError());
  Ctl c;
  HOCHK(read_ctl(d, &c, stream));
  if (c.err) return HO_ERR_BAD_CSR;
  hoStats out{};
  HOCHK(run_rounds_host(d, g, stream, false, out.kernel_ms, out.kernel_launches));
  HOCHK(read_ctl(d, &c, stream));
  if (c.err) return HO_ERR_BAD_CSR;
  if (!c.done) return HO_ERR_INTERNAL;
  out.rounds = c.r;
  out.levels = c.levels;
  out.events = c.events;
  out.overflows = c.overflows;
  out.compactions = c.compactions;
  t_stats = out;
  return HO_OK;
}

hoStatus hoTrussLastStats(hoStats* out) {
  if (!out) return HO_ERR_INVALID_ARG;
  *out = t_stats;
  return HO_OK;
}

// ----------------------------------------------------------------- batched
static uint32_t batch_slots(uint32_t B, const hoTuning* tune) {
  (void)tune;
  return std::max(1u, std::min(B, 256u));
}

size_t hoTrussBatchedWorkspaceBytes(const uint64_t* vtx_off, const uint64_t* edge_off,
                                    const uint32_t* h, uint32_t B, const hoTuning* tune) {
  if (!vtx_off || !edge_off || !h || B == 0) return 0;
  // every graph resident at once, capped at what the widest graphs need
  // when 64 run together; any workspace that holds the largest graph works
  std::vector<size_t> need(B);
  size_t sum = 0, mx = 0;
  for (uint32_t g = 0; g < B; ++g) {
    Plan p;
    const uint32_t n = (uint32_t)(vtx_off[g + 1] - vtx_off[g]);
    const uint64_t m = edge_off[g + 1] - edge_off[g];
    if (m == 0) continue;
    if (!make_plan(n, m, h[g], tune, true, &p, 16)) return 0;
    need[g] = up(p.total);
    sum += need[g];
    mx = std::max(mx, need[g]);
  }
  std::sort(need.begin(), need.end(), std::greater<size_t>());
  size_t top = 0;
  for (uint32_t g = 0; g < B && g < 64; ++g) top += need[g];
  return std::min(sum, top) + engine_header_bytes(batch_slots(B, tune)) + 2 * ALIGN;
}

hoStatus hoTrussDecomposeBatched(const uint32_t* row_ptr_cat, const uint32_t* col_idx_cat,
                                 const uint64_t* vtx_off, const uint64_t* adj_off,
                                 const uint64_t* edge_off, const uint32_t* h, uint32_t B,
                                 uint32_t* out_t_cat, uint32_t* out_round_cat, void* workspace,
                                 size_t workspace_bytes, const hoTuning* tune,
                                 hipStream_t stream) {
  if (!vtx_off || !adj_off || !edge_off || !h) return HO_ERR_INVALID_ARG;
  if (B == 0) return HO_OK;
  if (!row_ptr_cat || !col_idx_cat || !out_t_cat || !workspace) return HO_ERR_INVALID_ARG;
  uint32_t hmax = 1;
  for (uint32_t g = 0; g < B; ++g) {
    if (h[g] == 0) return HO_ERR_INVALID_ARG;
    const uint64_t n = vtx_off[g + 1] - vtx_off[g];
    if (adj_off[g + 1] - adj_off[g] != 2 * (edge_off[g + 1] - edge_off[g])) return HO_ERR_INVALID_ARG;
    hmax = std::max<uint32_t>(hmax, std::min<uint64_t>(h[g], n > 1 ? n - 1 : 1));
  }
  if (hmax > HMAX) return HO_ERR_INVALID_ARG;
  // longest first: graphs ordered by workspace (the ball store grows as n^2 h)
  uint32_t S = batch_slots(B, tune);
  std::vector<std::pair<size_t, uint32_t>> order;
  size_t largest = 0;
  for (uint32_t g = 0; g < B; ++g) {
    const uint64_t m = edge_off[g + 1] - edge_off[g];
    if (m == 0) continue;
    Plan p;
    const uint32_t n = (uint32_t)(vtx_off[g + 1] - vtx_off[g]);
    if (!make_plan(n, m, h[g], tune, true, &p, 16)) return HO_ERR_INVALID_ARG;
    order.push_back({p.total, g});
    largest = std::max(largest, up(p.total));
  }
  if (order.empty()) return HO_OK;
  // fewer slots (a smaller header) when the workspace holds little more than
  // the largest graph
  while (S > 1 && workspace_bytes < largest + engine_header_bytes(S) + ALIGN) S = S / 2;
  if (workspace_bytes < largest + engine_header_bytes(S) + ALIGN) return HO_ERR_WORKSPACE;
  Engine eng;
  eng.cap_factor = 16;
  HOCHK(eng.init(workspace, workspace_bytes, S, hmax, batch_grid(S, tune), stream, false));
  std::sort(order.begin(), order.end(), std::greater<std::pair<size_t, uint32_t>>());
  std::vector<size_t> ids;
  for (auto& og : order) {
    const uint32_t g = og.second;
    Request r;
    r.rp = row_ptr_cat + vtx_off[g] + g;
    r.ci = col_idx_cat + adj_off[g];
    r.n = (uint32_t)(vtx_off[g + 1] - vtx_off[g]);
    r.m = edge_off[g + 1] - edge_off[g];
    r.h = h[g];
    r.t = out_t_cat + edge_off[g];
    r.rho = out_round_cat ? out_round_cat + edge_off[g] : nullptr;
    if (tune) { r.tune = *tune; r.has_tune = true; }
    size_t id;
    const hoStatus st = eng.submit(r, &id);
    if (st == HO_ERR_BUDGET) return HO_ERR_WORKSPACE;  // a graph that can never fit
    HOCHK(st);
    ids.push_back(id);
  }
  while (!eng.queue.empty() || eng.busy()) {
    HOCHK(eng.run());
    if (!eng.busy() && !eng.queue.empty()) return HO_ERR_WORKSPACE;
  }
  for (size_t id : ids)
    if (eng.reqs[id].result != HO_OK) return eng.reqs[id].result;
  return HO_OK;
}

// ----------------------------------------------------------------- sessions
hoStatus hoSessionCreate(void* pool, size_t pool_bytes, uint32_t max_slots, uint32_t max_h,
                         hipStream_t stream, hoSession** out) {
  if (!pool || !out || max_slots == 0 || max_slots > 4096 || max_h == 0 || max_h > HMAX)
    return HO_ERR_INVALID_ARG;
  hoSession* ss = new (std::nothrow) hoSession();
  if (!ss) return HO_ERR_INVALID_ARG;
  ss->eng.cap_factor = 16;
  hoStatus st = ss->eng.init(pool, pool_bytes, max_slots, max_h, batch_grid(max_slots, nullptr),
                             stream, false);
  if (st != HO_OK) {
    delete ss;
    return st;
  }
  *out = ss;
  return HO_OK;
}

hoStatus hoSubmit(hoSession* ss, const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n,
                  uint64_t m, uint32_t h, uint32_t* out_trussness, uint32_t* out_round,
                  uint64_t* out_ticket) {
  if (!ss || !out_ticket) return HO_ERR_INVALID_ARG;
  hoStatus st = check_common(row_ptr, col_idx, n, m, h, out_trussness, (void*)1);
  if (st != HO_OK) return st;
  std::lock_guard<std::mutex> lk(ss->mu);
  Request r;
  r.rp = row_ptr; r.ci = col_idx; r.n = n; r.m = m; r.h = h;
  r.t = out_trussness; r.rho = out_round;
  size_t id;
  if (m == 0) {  // nothing to compute: finished at once
    r.state = 2;
    ss->eng.reqs.push_back(r);
    *out_ticket = ss->eng.reqs.size() - 1;
    return HO_OK;
  }
  st = ss->eng.submit(r, &id);
  if (st != HO_OK) return st;
  *out_ticket = id;
  return HO_OK;
}

hoStatus hoSessionProgress(hoSession* ss, uint32_t max_graph_launches, uint32_t* active,
                           uint32_t* queued) {
  if (!ss) return HO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ss->mu);
  hoStatus st = ss->eng.run(max_graph_launches ? max_graph_launches : UINT64_MAX);
  if (active) {
    uint32_t a = 0;
    for (int r : ss->eng.slot_req) a += r >= 0;
    *active = a;
  }
  if (queued) *queued = (uint32_t)ss->eng.queue.size();
  return st;
}

hoStatus hoPoll(hoSession* ss, uint64_t ticket, int* done) {
  if (!ss || !done) return HO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ss->mu);
  if (ticket >= ss->eng.reqs.size()) return HO_ERR_NOT_FOUND;
  const Request& r = ss->eng.reqs[ticket];
  *done = r.state >= 2;
  if (r.state == 3) return HO_ERR_CANCELLED;
  return r.state == 2 ? r.result : HO_OK;
}

hoStatus hoCancel(hoSession* ss, uint64_t ticket) {
  if (!ss) return HO_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(ss->mu);
  if (ticket >= ss->eng.reqs.size()) return HO_ERR_NOT_FOUND;
  Request& r = ss->eng.reqs[ticket];
  if (r.state != 0) return HO_ERR_BUSY;  // only queued requests can be cancelled
  r.state = 3;
  auto& q = ss->eng.queue;
  q.erase(std::remove(q.begin(), q.end(), (size_t)ticket), q.end());
  return HO_OK;
}

hoStatus hoSessionDestroy(hoSession* ss) {
  if (!ss) return HO_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(ss->mu);
    (void)hipStreamSynchronize(ss->eng.s);
  }
  delete ss;
  return HO_OK;
}

// ------------------------------------------------------ truss extraction
size_t hoTrussComponentsWorkspaceBytes(uint32_t n, uint64_t m) {
  Plan p;
  size_t off_cc;
  if (!make_topo_plan(n, m, &p, &off_cc)) return 0;
  return p.total;
}

hoStatus hoTrussComponents(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n, uint64_t m,
                           const uint32_t* trussness, uint32_t k, uint32_t* out_component,
                           uint32_t* out_count, void* workspace, size_t workspace_bytes,
                           hipStream_t stream) {
  if (!out_count) return HO_ERR_INVALID_ARG;
  if (m >= (1ull << 31)) return HO_ERR_INVALID_ARG;
  if (m == 0) {
    *out_count = 0;
    return HO_OK;
  }
  if (!row_ptr || !col_idx || !trussness || !out_component || !workspace || n == 0)
    return HO_ERR_INVALID_ARG;
  Plan p;
  size_t off_cc;
  if (!make_topo_plan(n, m, &p, &off_cc)) return HO_ERR_INVALID_ARG;
  if (workspace_bytes < p.total) return HO_ERR_WORKSPACE;
  Dev d = carve(p, workspace, row_ptr, col_idx, nullptr, nullptr);
  const uintptr_t base = ((uintptr_t)workspace + ALIGN - 1) / ALIGN * ALIGN;
  uint32_t* parent = (uint32_t*)(base + off_cc);
  uint32_t* touched = parent + n;
  uint32_t* counter = touched + n;
  const unsigned T = 256;
  run_topology(d, stream);
  hipLaunchKernelGGL(k_cc_init, dim3(grid_for(n, T)), dim3(T), 0, stream, parent, touched, n);
  HIPCHK(hipMemsetAsync(counter, 0, sizeof(uint32_t), stream));
  hipLaunchKernelGGL(k_cc_hook, dim3(grid_for(m, T)), dim3(T), 0, stream, d, trussness, k, parent,
                     touched);
  hipLaunchKernelGGL(k_cc_label, dim3(grid_for(std::max<uint64_t>(m, n), T)), dim3(T), 0, stream, d,
                     trussness, k, parent, touched, out_component, counter);
  HIPCHK(hipGetLastError());
  Ctl c;
  HOCHK(read_ctl(d, &c, stream));
  if (c.err) return HO_ERR_BAD_CSR;
  uint32_t cnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, counter, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  *out_count = cnt;
  return HO_OK;
}


// ------------------------------------------------------ H-index fixpoint
size_t hoTrussHIndexWorkspaceBytes(uint32_t n, uint64_t m, uint32_t h) {
  HxPlan q;
  if (!make_hx_plan(n, m, h, &q)) return 0;
  return q.base + ALIGN;
}

hoStatus hoTrussHIndex(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n, uint64_t m,
                       uint32_t h, uint32_t flags, uint32_t max_sweeps, uint32_t* out_trussness,
                       uint32_t* out_sweeps, void* workspace, size_t workspace_bytes,
                       size_t* needed_bytes, hipStream_t stream) {
  if (!out_sweeps ||
      (flags & ~(HO_HINDEX_ASYNC | HO_HINDEX_ALL | HO_HINDEX_STATS | HO_HINDEX_KEYS)))
    return HO_ERR_INVALID_ARG;
  hoStatus st = check_common(row_ptr, col_idx, n, m, h, out_trussness, workspace);
  if (st != HO_OK) return st;
  t_stats = hoStats{};
  if (m == 0) {
    *out_sweeps = 0;
    if (needed_bytes) *needed_bytes = 0;
    return HO_OK;
  }
  HxPlan q;
  if (!make_hx_plan(n, m, h, &q)) return HO_ERR_INVALID_ARG;
  if (needed_bytes) *needed_bytes = q.base + ALIGN;
  if (workspace_bytes < q.base + ALIGN) return HO_ERR_WORKSPACE;
  Dev d = carve(q.p, workspace, row_ptr, col_idx, nullptr, nullptr);
  const uintptr_t wsb = ((uintptr_t)workspace + ALIGN - 1) / ALIGN * ALIGN;
  auto at = [&](size_t off) { return (void*)(wsb + off); };
  EventGuard ev0, ev1, ka, kb;
  HIPCHK(hipEventCreate(&ev0.e));
  HIPCHK(hipEventCreate(&ev1.e));
  const bool stats = flags & HO_HINDEX_STATS;
  if (stats) {
    HIPCHK(hipEventCreate(&ka.e));
    HIPCHK(hipEventCreate(&kb.e));
  }
  // stats mode: every launch group timed on its own (0 balls, H^(0) and
  // ranks, 1 path-key rows, 2 edge updates, 3 change tracking)
  auto timed = [&](int kind, const std::function<void()>& launch) -> hoStatus {
    if (!stats) {
      launch();
      return HO_OK;
    }
    HIPCHK(hipEventRecord(ka.e, stream));
    launch();
    HIPCHK(hipEventRecord(kb.e, stream));
    HIPCHK(hipEventSynchronize(kb.e));
    float kms = 0.f;
    HIPCHK(hipEventElapsedTime(&kms, ka.e, kb.e));
    t_stats.kernel_ms[kind] += kms;
    t_stats.kernel_launches[kind] += 1;
    return HO_OK;
  };
  HIPCHK(hipEventRecord(ev0.e, stream));
  // G's balls and H^(0) = sup_G(e, h)
  hoStatus init_st = HO_OK;
  HOCHK(timed(0, [&] { init_st = run_init(d, d.sup, nullptr, stream); }));
  HOCHK(init_st);
  Ctl c;
  HOCHK(read_ctl(d, &c, stream));
  if (c.err) return HO_ERR_BAD_CSR;
  Hx x;
  memset(&x, 0, sizeof x);
  x.rp = d.rp; x.ci = d.ci; x.eid = d.eid; x.eu = d.eu; x.ev = d.ev;
  x.up_cnt = d.up_cnt; x.up_off = d.up_off;
  for (uint32_t j = 1; j <= d.h; ++j) x.L[j] = d.L[j];
  x.n = d.n; x.m = d.m; x.h = d.h; x.W = d.W;
  x.wp = (uint32_t*)at(q.off_wp);
  x.cnt = (uint32_t*)at(q.off_cnt);
  x.boff = (uint64_t*)at(q.off_boff);
  x.H = d.sup;
  x.dirty = (uint32_t*)at(q.off_dirty);
  x.touched = (uint32_t*)at(q.off_touched);
  x.tbits = (uint64_t*)at(q.off_tbits);
  x.tlist = (uint32_t*)at(q.off_tlist);
  x.ord = (uint32_t*)at(q.off_ord);
  x.cbound = (uint32_t*)at(q.off_cbound);
  x.ctr = (uint32_t*)at(q.off_ctr);
  x.stat = stats ? (unsigned long long*)at(q.off_stat) : nullptr;
  const unsigned T = 256;
  if (stats)
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(64), 0, stream, (uint64_t*)x.stat, (size_t)8,
                       (uint64_t)0);
  HOCHK(timed(0, [&] {
    hipLaunchKernelGGL(k_hx_rank, dim3(grid_for(n, T / WAVE)), dim3(T), 0, stream, x);
    hipLaunchKernelGGL(k_hx_scan, dim3(1), dim3(1024), 0, stream, x.cnt, x.boff, n);
  }));
  uint64_t members = 0;
  HIPCHK(hipMemcpyAsync(&members, x.boff + n, sizeof members, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  // P[0], P[1] (h >= 3), previous keys (path-key pruning only)
  const bool keys = !(flags & HO_HINDEX_ALL) && (flags & HO_HINDEX_KEYS);
  // plus the member lists
  const uint32_t nbuf = (d.h >= 3 ? 2 : 1) + (keys ? 1 : 0) + 1;
  const size_t need = q.base + nbuf * hx_key_bytes(members) + ALIGN;
  if (needed_bytes) *needed_bytes = need;
  if (workspace_bytes < need) return HO_ERR_WORKSPACE;
  x.P[0] = (uint32_t*)at(q.base);
  x.P[1] = d.h >= 3 ? (uint32_t*)at(q.base + hx_key_bytes(members)) : nullptr;
  x.Pold = keys ? (uint32_t*)at(q.base + (nbuf - 2) * hx_key_bytes(members)) : nullptr;
  x.mem = (uint32_t*)at(q.base + (nbuf - 1) * hx_key_bytes(members));
  HOCHK(timed(0, [&] {
    hipLaunchKernelGGL(k_hx_members, dim3(grid_for(n, T / WAVE)), dim3(T), 0, stream, x);
  }));
  x.dmask = (uint64_t*)at(q.off_dmask);
  x.tmin = (uint32_t*)at(q.off_tmin);
  x.bigctr = (unsigned long long*)at(q.off_bigctr);
  x.bigu = (uint32_t*)at(q.off_bigu);
  x.bigoff = (uint32_t*)at(q.off_bigoff);
  x.cmask = (uint32_t*)at(q.off_cmask);
  const bool async = flags & HO_HINDEX_ASYNC;
  x.track = (flags & HO_HINDEX_ALL) ? 0u : 1u;
  x.lemma4 = (x.track && !(flags & HO_HINDEX_KEYS)) ? 1u : 0u;
  const uint32_t chunks = async ? HX_CHUNKS : 1;
  if (async) {
    hipLaunchKernelGGL(k_hx_order, dim3(grid_for(n, T / WAVE)), dim3(T), 0, stream, x);
    hipLaunchKernelGGL(k_hx_bounds, dim3(1), dim3(64), 0, stream, x, chunks);
  }
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(n, T)), dim3(T), 0, stream, x.dirty, (size_t)n, 1u);
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(n, T)), dim3(T), 0, stream, x.touched, (size_t)n, 0u);
  HIPCHK(hipGetLastError());
  uint32_t sweeps = 0;
  uint64_t evals = 0, rows = 0, changes = 0;
  // environment HOTRUSS_SWEEPS set: one line per sweep on stderr
  const bool trace = std::getenv("HOTRUSS_SWEEPS") != nullptr;
  auto sweep_t0 = std::chrono::steady_clock::now();
  uint32_t prev_changed = 0, prev_evals = 0;
  while (true) {
    x.first = sweeps == 0 ? 1u : 0u;
    // fold the first histogram into the counting pass while more than a
    // quarter of the evaluated edges change
    x.hist1 = (sweeps == 0 || (uint64_t)prev_changed * 4 > prev_evals) ? 1u : 0u;
    hipLaunchKernelGGL(k_fill32, dim3(1), dim3(64), 0, stream, x.ctr, (size_t)4, 0u);
    if (x.track) {
      // Lemma 4 mode: the masks the previous sweep's changes left are read
      // now, and this sweep's crossings start empty
      if (x.lemma4)
        hipLaunchKernelGGL(k_fill32, dim3(grid_for(2 * (size_t)n, T)), dim3(T), 0, stream,
                           x.cmask, 2 * (size_t)n, 0u);
      else
        hipLaunchKernelGGL(k_fill64, dim3(grid_for(n, T)), dim3(T), 0, stream, x.dmask,
                           (size_t)n, (uint64_t)0);
      hipLaunchKernelGGL(k_fill32, dim3(grid_for(n, T)), dim3(T), 0, stream, x.tmin, (size_t)n,
                         0xffffffffu);
    }
    for (uint32_t cc = 0; cc < chunks; ++cc) {
      const uint32_t vlo = (uint32_t)((uint64_t)cc * n / chunks);
      const uint32_t vhi = (uint32_t)((uint64_t)(cc + 1) * n / chunks);
      if (vhi > vlo)
        HOCHK(timed(1, [&] {
          hipLaunchKernelGGL(k_fill64, dim3(1), dim3(64), 0, stream, (uint64_t*)x.bigctr,
                             (size_t)1, (uint64_t)0);
          hipLaunchKernelGGL(k_hx_paths, dim3(grid_for(vhi - vlo, 1)), dim3(T), 0, stream, x,
                             vlo, vhi);
          if (x.h == 2) {
            hipLaunchKernelGGL(k_hx_split, dim3(num_cu() * 8), dim3(T), 0, stream, x);
            if (x.track && !x.lemma4)
              hipLaunchKernelGGL(k_hx_split_mask, dim3(num_cu() * 2), dim3(T), 0, stream, x);
          }
        }));
      HOCHK(timed(2, [&] {
        hipLaunchKernelGGL(k_hx_edges, dim3(grid_for((m + chunks - 1) / chunks, T / WAVE)),
                           dim3(T), 0, stream, x, cc, async ? 1u : 0u);
      }));
    }
    if (x.track)
      HOCHK(timed(3, [&] {
        hipLaunchKernelGGL(k_hx_tbits, dim3(grid_for(x.W, T)), dim3(T), 0, stream, x);
        hipLaunchKernelGGL(k_hx_dirty, dim3(grid_for(n, T / WAVE)), dim3(T), 0, stream, x);
      }));
    HIPCHK(hipGetLastError());
    uint32_t hc[4];
    HIPCHK(hipMemcpyAsync(hc, x.ctr, sizeof hc, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    ++sweeps;
    if (trace) {
      const auto now = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[hotruss] sweep %u: %u changed, %u evaluated, %u rows, %.3f ms\n",
                   sweeps, hc[HX_CTR_CHANGED], hc[HX_CTR_EVALS], hc[HX_CTR_ROWS],
                   std::chrono::duration<double, std::milli>(now - sweep_t0).count());
      std::fflush(stderr);
      sweep_t0 = now;
    }
    changes += hc[HX_CTR_CHANGED];
    prev_changed = hc[HX_CTR_CHANGED];
    prev_evals = hc[HX_CTR_EVALS];
    evals += hc[HX_CTR_EVALS];
    rows += hc[HX_CTR_ROWS];
    if (hc[HX_CTR_CHANGED] == 0 || (max_sweeps && sweeps >= max_sweeps)) break;
    // every sweep but the last lowers the sum of H, which starts below m*n
    if (sweeps > m * (uint64_t)n + 1) return HO_ERR_INTERNAL;
  }
  hipLaunchKernelGGL(k_hx_finish, dim3(grid_for(m, T)), dim3(T), 0, stream, x.H, out_trussness,
                     d.m);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ev1.e, stream));
  HIPCHK(hipEventSynchronize(ev1.e));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ev0.e, ev1.e));
  t_stats.rounds = sweeps;
  t_stats.events = changes;
  t_stats.device_ms = ms;
  t_stats.work[0] = evals;
  t_stats.work[1] = rows;
  if (stats) {
    unsigned long long st8[8];
    HIPCHK(hipMemcpyAsync(st8, x.stat, sizeof st8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    t_stats.work[2] = st8[HX_ST_RELAX];
    t_stats.work[3] = st8[HX_ST_DIRECT];
    t_stats.work[4] = st8[HX_ST_ENTRIES];
    t_stats.work[5] = st8[HX_ST_PASSES];
    t_stats.work[6] = st8[HX_ST_SCAN];
    t_stats.work[7] = st8[HX_ST_MEMBERS];
  }
  *out_sweeps = sweeps;
  return HO_OK;
}

}  // extern "C"
