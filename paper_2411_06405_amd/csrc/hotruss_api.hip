// hotruss_api.hip -- host side of libhotruss: argument checks, workspace
// planning and the launch sequence of the peeling method (paper, Section 3).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/hotruss.h"
#include "hotruss_dev.h"
#include "hotruss_kernels.hip"

namespace hotruss {
// serial forms (hotruss_serial.hip, a separate translation unit)
__global__ void k_level_serial(const Dev* __restrict__ dp, uint32_t j);
__global__ void k_support_serial(const Dev* __restrict__ dp);
}  // namespace hotruss

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
      off_scan, off_minpart, off_dev, off_spart, off_sup, off_rho, off_R0, off_R1, off_L[HMAX + 1],
      off_Dm[HMAX + 1], off_evl[HMAX + 1][2], off_itl[HMAX + 2];
  size_t total = 0;
};

uint32_t words_per_row(uint32_t n) {
  uint32_t w = (n + 63) / 64;
  return (w + 7) / 8 * 8;  // 64-byte rows
}

uint32_t clamp_cap(uint64_t want, uint64_t lo, uint64_t hi) {
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, lo), hi);
}

bool make_plan(uint32_t n, uint64_t m, uint32_t h, const hoTuning* tune, bool full, Plan* P) {
  if (h == 0 || m >= (1ull << 31) || n == 0xffffffffu) return false;
  if (n > 1 && h > n - 1) h = n - 1;  // any h beyond n-1 is the same as n-1
  if (h == 0) h = 1;
  if (h > HMAX) return false;
  Plan p;
  p.n = n; p.m = m; p.h = h; p.full = full;
  p.W = words_per_row(n);
  // Lists are sized so that a round rarely overflows them (a round that does
  // runs its level or support step through the serial kernels, far slower).
  p.evcap = tune && tune->event_capacity ? tune->event_capacity
                                         : clamp_cap(128 * m, 1u << 20, 1u << 27);
  p.itcap = tune && tune->item_capacity ? tune->item_capacity
                                        : clamp_cap(128 * m, 1u << 20, 1u << 27);
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
  p.off_dev = take(sizeof(Dev));
  p.off_spart = take(4ull * NSTAT * STAT_GRID);
  p.off_sup = take(4 * m + 4);
  p.off_rho = take(full ? 4 * m + 4 : 0);
  p.off_R0 = take(full ? 4 * m + 4 : 0);
  p.off_R1 = take(full ? 4 * m + 4 : 0);
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

thread_local uint32_t* stats_part_base = nullptr;  // workspace slot of the stats counters

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
  d.nminpart = std::min<uint32_t>(MIN_PART, grid_for(p.m, 256, 4));
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
  d.self = (Dev*)at(p.off_dev);
  d.serial = 0;
  d.spart = nullptr;  // set in stats mode
  stats_part_base = (uint32_t*)at(p.off_spart);
  d.sup = (uint32_t*)at(p.off_sup);
  d.t = t;
  d.rho = rho ? rho : (p.full ? (uint32_t*)at(p.off_rho) : nullptr);
  if (p.full) {
    d.R[0] = (uint32_t*)at(p.off_R0);
    d.R[1] = (uint32_t*)at(p.off_R1);
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
hoStatus run_init(const Dev& d, uint32_t* out_sup, const hoTuning* tune, hipStream_t s,
                  hipEvent_t sup0 = nullptr, hipEvent_t sup1 = nullptr) {
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
  const size_t lds = (size_t)d.W * 8;
  const unsigned rows_grid = grid_for(d.n, 1, 64);
  hipLaunchKernelGGL(k_build_L1, dim3(rows_grid), dim3(T), lds, s, d);
  if (d.h >= 2) hipLaunchKernelGGL(k_build_L2, dim3(rows_grid), dim3(T), lds, s, d);
  for (uint32_t j = 3; j <= d.h; ++j)
    hipLaunchKernelGGL(k_build_Lj, dim3(rows_grid), dim3(T), 0, s, d, j);
  uint32_t epw = tune && tune->edges_per_wave ? tune->edges_per_wave : 0;
  if (!epw) epw = d.W <= 8 ? 16 : d.W <= 32 ? 4 : 1;
  if (sup0) HIPCHK(hipEventRecord(sup0, s));
  if (epw >= 16) hipLaunchKernelGGL(k_support_init<4>, dim3(grid_for(d.m, T / 4)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 8) hipLaunchKernelGGL(k_support_init<8>, dim3(grid_for(d.m, T / 8)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 4) hipLaunchKernelGGL(k_support_init<16>, dim3(grid_for(d.m, T / 16)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 2) hipLaunchKernelGGL(k_support_init<32>, dim3(grid_for(d.m, T / 32)), dim3(T), 0, s, d, out_sup);
  else hipLaunchKernelGGL(k_support_init<64>, dim3(grid_for(d.m, T / 64)), dim3(T), 0, s, d, out_sup);
  if (sup1) HIPCHK(hipEventRecord(sup1, s));
  HIPCHK(hipGetLastError());
  return HO_OK;
}

// Launch geometry of the round kernels.
struct RoundGrid {
  unsigned jump, mark, level, support;
};

RoundGrid round_grid(const Dev& d, const hoTuning* tune) {
  RoundGrid g;
  const unsigned wide = tune && tune->grid_blocks ? tune->grid_blocks : (unsigned)num_cu() * 8;
  g.jump = d.nminpart;
  g.mark = std::max(1u, std::min(wide, grid_for(d.m, 256)));
  g.level = wide;
  g.support = wide;
  return g;
}

// Kernel kinds timed in stats mode.
enum { KT_SUPINIT = 0, KT_JUMP, KT_MARK, KT_LEVEL, KT_SUPPORT, KT_ADVANCE, KT_N };

void launch_round(const Dev& d, const RoundGrid& g, hipStream_t s) {
  const unsigned T = 256;
  const Dev* dp = d.self;
  hipLaunchKernelGGL(k_jump_min, dim3(g.jump), dim3(T), 0, s, dp);
  hipLaunchKernelGGL(k_mark, dim3(g.mark), dim3(T), 0, s, dp);
  for (uint32_t j = 2; j <= d.h; ++j)
    hipLaunchKernelGGL(k_level, dim3(g.level), dim3(LV_THREADS), 0, s, dp, j);
  hipLaunchKernelGGL(k_support, dim3(g.support), dim3(T), 0, s, dp);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, dp);
}

// Captured round sequences, cached per device state (workspace, buffers).
struct GraphEntry {
  Dev key;
  uint32_t rounds;
  unsigned level_grid;
  hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
hipStream_t g_capture_stream = nullptr;

hoStatus get_graph(const Dev& d, const RoundGrid& g, uint32_t rounds, hipGraphExec_t* out) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& e : g_graphs)
    if (e.rounds == rounds && e.key.self == d.self && e.key.h == d.h && e.key.m == d.m &&
        e.key.nminpart == d.nminpart && e.level_grid == g.level) {
      *out = e.exec;
      return HO_OK;
    }
  if (!g_capture_stream) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
  hipGraph_t graph;
  HIPCHK(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
  for (uint32_t i = 0; i < rounds; ++i) launch_round(d, g, g_capture_stream);
  HIPCHK(hipStreamEndCapture(g_capture_stream, &graph));
  hipGraphExec_t exec;
  hipError_t err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (err != hipSuccess) return HO_ERR_HIP;
  if (g_graphs.size() >= 64) {  // bounded cache: drop the oldest
    (void)hipGraphExecDestroy(g_graphs.front().exec);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back(GraphEntry{d, rounds, g.level, exec});
  *out = exec;
  return HO_OK;
}

uint32_t* g_done_host = nullptr;  // pinned {done, halt} words, one pair per graph in flight

hoStatus read_ctl(const Dev& d, Ctl* host, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HO_OK;
}

// Timing of the host-driven round steps (stats mode).
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

// Run the round steps from `from` on (2..h: level j, h+1: support update,
// h+2: end of round) from the host, taking the serial kernel for any step
// whose chunked kernel halts on an overflowed work list.
hoStatus steps_host(const Dev& d, const RoundGrid& g, hipStream_t s, uint32_t from, bool serial_first,
                    StepTimer& tm) {
  const unsigned T = 256;
  const Dev* dp = d.self;
  Ctl c;
  for (uint32_t step = from; step <= d.h + 1; ++step) {
    bool serial = serial_first && step == from;
    if (!serial) {
      HOCHK(tm.begin(s));
      if (step <= d.h) hipLaunchKernelGGL(k_level, dim3(g.level), dim3(LV_THREADS), 0, s, dp, step);
      else hipLaunchKernelGGL(k_support, dim3(g.support), dim3(T), 0, s, dp);
      HOCHK(tm.end(s, step <= d.h ? KT_LEVEL : KT_SUPPORT));
      if (d.spart) {
        if (step <= d.h) hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 0u, 5u, g.level);
        else hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, dp, 5u, 3u, g.support);
      }
      hoStatus st = read_ctl(d, &c, s);
      if (st != HO_OK) return st;
      serial = c.halt != 0;
    }
    if (serial) {
      HIPCHK(hipMemsetAsync(&d.ctl->halt, 0, sizeof(uint32_t), s));
      HOCHK(tm.begin(s));
      if (step <= d.h) hipLaunchKernelGGL(k_level_serial, dim3(g.level), dim3(T), 0, s, dp, step);
      else hipLaunchKernelGGL(k_support_serial, dim3(g.support), dim3(T), 0, s, dp);
      HOCHK(tm.end(s, step <= d.h ? KT_LEVEL : KT_SUPPORT));
    }
  }
  HOCHK(tm.begin(s));
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, dp);
  HOCHK(tm.end(s, KT_ADVANCE));
  HIPCHK(hipGetLastError());
  return HO_OK;
}

// A graph stopped on a halted step: finish that round from the host.
hoStatus finish_halted_round(const Dev& d, const RoundGrid& g, hipStream_t s, StepTimer& tm) {
  Ctl c;
  hoStatus st = read_ctl(d, &c, s);
  if (st != HO_OK) return st;
  if (!c.halt) return HO_OK;
  return steps_host(d, g, s, c.halt_step, true, tm);
}

// Peel rounds until the device reports completion: graphs of G rounds are
// replayed with two in flight; the host only polls the {done, halt} words.
hoStatus run_rounds_graph(const Dev& d, const hoTuning* tune, hipStream_t s) {
  const RoundGrid g = round_grid(d, tune);
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (!g_done_host) HIPCHK(hipHostMalloc((void**)&g_done_host, 64, hipHostMallocDefault));
  }
  hipEvent_t ev[2];
  HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  const uint32_t sizes[3] = {4, 32, 128};
  hipGraphExec_t ex[3];
  for (int i = 0; i < 3; ++i) {
    hoStatus st = get_graph(d, g, sizes[i], &ex[i]);
    if (st != HO_OK) return st;
  }
  volatile uint32_t* flag = g_done_host;
  StepTimer tm;
  uint64_t launched = 0, maxlaunch = 8 + 2 * (uint64_t)d.m;  // every round peels >= 1 edge
  auto launch = [&](int slot) -> hoStatus {
    const int which = launched == 0 ? 0 : launched == 1 ? 1 : 2;
    HIPCHK(hipGraphLaunch(ex[which], s));
    HIPCHK(hipMemcpyAsync((void*)&flag[2 * slot], &d.ctl->done, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(ev[slot], s));
    ++launched;
    return HO_OK;
  };
  hoStatus st = launch(0);
  if (st == HO_OK) st = launch(1);
  int cur = 0;
  while (st == HO_OK) {
    HIPCHK(hipEventSynchronize(ev[cur]));
    if (flag[2 * cur]) break;  // done
    if (launched > maxlaunch) { st = HO_ERR_INTERNAL; break; }
    if (flag[2 * cur + 1]) {  // halted: drain, finish the round here, restart
      HIPCHK(hipStreamSynchronize(s));
      st = finish_halted_round(d, g, s, tm);
      if (st != HO_OK) break;
      st = launch(0);
      if (st == HO_OK) st = launch(1);
      cur = 0;
      continue;
    }
    st = launch(cur);
    cur ^= 1;
  }
  HIPCHK(hipStreamSynchronize(s));
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return st;
}

// Debug / stats form: every round driven from the host, optional timing.
hoStatus run_rounds_host(const Dev& d, const hoTuning* tune, hipStream_t s, bool timed,
                         double* kms, uint64_t* klaunch) {
  const RoundGrid g = round_grid(d, tune);
  const unsigned T = 256;
  const Dev* dp = d.self;
  StepTimer tm;
  tm.on = timed;
  tm.kms = kms;
  tm.kl = klaunch;
  if (timed) {
    HIPCHK(hipEventCreate(&tm.e0));
    HIPCHK(hipEventCreate(&tm.e1));
  }
  Ctl c;
  hoStatus st = read_ctl(d, &c, s);
  uint64_t rounds = 0;
  while (st == HO_OK && !c.done) {
    if ((st = tm.begin(s)) != HO_OK) break;
    hipLaunchKernelGGL(k_jump_min, dim3(g.jump), dim3(T), 0, s, dp);
    if ((st = tm.end(s, KT_JUMP)) != HO_OK) break;
    if ((st = tm.begin(s)) != HO_OK) break;
    hipLaunchKernelGGL(k_mark, dim3(g.mark), dim3(T), 0, s, dp);
    if ((st = tm.end(s, KT_MARK)) != HO_OK) break;
    st = steps_host(d, g, s, 2, false, tm);
    if (st == HO_OK) st = read_ctl(d, &c, s);
    if (++rounds > (uint64_t)d.m + 2) st = HO_ERR_INTERNAL;
  }
  if (timed) {
    (void)hipEventDestroy(tm.e0);
    (void)hipEventDestroy(tm.e1);
  }
  return st;
}

hoStatus check_common(const uint32_t* rp, const uint32_t* ci, uint32_t n, uint64_t m, uint32_t h,
                      const void* out, void* ws) {
  if (h == 0) return HO_ERR_INVALID_ARG;
  if (m >= (1ull << 31)) return HO_ERR_INVALID_ARG;
  if (m == 0) return HO_OK;
  if (!rp || !ci || !out || !ws || n == 0) return HO_ERR_INVALID_ARG;
  return HO_OK;
}

}  // namespace
}  // namespace hotruss

using namespace hotruss;

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
  return p.total;
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
  if (workspace_bytes < p.total) return HO_ERR_WORKSPACE;
  Dev d = carve(p, workspace, row_ptr, col_idx, out_trussness, out_round);
  if (tune) d.serial = tune->flags & (HO_FLAG_SERIAL_LEVELS | HO_FLAG_SERIAL_SUPPORT);
  const bool stats = tune && (tune->flags & HO_FLAG_STATS);
  if (stats) {
    d.spart = stats_part_base;
    HIPCHK(hipMemsetAsync(d.spart, 0, 4ull * NSTAT * STAT_GRID, stream));
  }
  const bool host_loop = stats || (tune && (tune->flags & HO_FLAG_HOST_LOOP));
  hoStats out{};
  hipEvent_t ev0, ev1, es0 = nullptr, es1 = nullptr;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  if (stats) {
    HIPCHK(hipEventCreate(&es0));
    HIPCHK(hipEventCreate(&es1));
  }
  HIPCHK(hipEventRecord(ev0, stream));
  const unsigned T = 256;
  // outputs and change marks start at zero
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(d.m, T)), dim3(T), 0, stream, d.t, (size_t)d.m, 0u);
  for (uint32_t j = 1; j <= d.h; ++j)
    if (d.Dm[j])
      hipLaunchKernelGGL(k_fill64, dim3(grid_for((size_t)d.n * d.W, T)), dim3(T), 0, stream,
                         d.Dm[j], (size_t)d.n * d.W, 0ull);
  st = run_init(d, d.sup, tune, stream, es0, es1);
  if (st != HO_OK) return st;
  Ctl c;
  st = read_ctl(d, &c, stream);
  if (st != HO_OK) return st;
  if (c.err) return HO_ERR_BAD_CSR;
  if (stats) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, es0, es1));
    out.kernel_ms[KT_SUPINIT] = ms;
    out.kernel_launches[KT_SUPINIT] = 1;
    (void)hipEventDestroy(es0);
    (void)hipEventDestroy(es1);
  }
  HIPCHK(hipMemcpyAsync(d.self, &d, sizeof(Dev), hipMemcpyHostToDevice, stream));
  st = host_loop ? run_rounds_host(d, tune, stream, stats, out.kernel_ms, out.kernel_launches)
                 : run_rounds_graph(d, tune, stream);
  if (st != HO_OK) return st;
  HIPCHK(hipEventRecord(ev1, stream));
  HIPCHK(hipEventSynchronize(ev1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  st = read_ctl(d, &c, stream);
  if (st != HO_OK) return st;
  if (c.err) return HO_ERR_INTERNAL;
  out.rounds = c.r;
  out.levels = c.levels;
  out.events = c.events;
  out.overflows = c.overflows;
  out.device_ms = ms;
  for (uint32_t i = 0; i < NSTAT; ++i) out.work[i] = c.stat[i];
  t_stats = out;
  return HO_OK;
}

hoStatus hoTrussLastStats(hoStats* out) {
  if (!out) return HO_ERR_INVALID_ARG;
  *out = t_stats;
  return HO_OK;
}

size_t hoTrussBatchedWorkspaceBytes(const uint64_t* vtx_off, const uint64_t* edge_off,
                                    const uint32_t* h, uint32_t B, const hoTuning* tune) {
  (void)vtx_off; (void)edge_off; (void)h; (void)B; (void)tune;
  return 0;
}

hoStatus hoTrussDecomposeBatched(const uint32_t*, const uint32_t*, const uint64_t*,
                                 const uint64_t*, const uint64_t*, const uint32_t*, uint32_t,
                                 uint32_t*, uint32_t*, void*, size_t, const hoTuning*,
                                 hipStream_t) {
  return HO_ERR_INVALID_ARG;
}

}  // extern "C"
