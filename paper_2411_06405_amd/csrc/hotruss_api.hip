// hotruss_api.hip -- host side of libhotruss: argument checks, workspace
// planning and the launch sequence of the peeling method (paper, Section 3).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/hotruss.h"
#include "hotruss_dev.h"
#include "hotruss_kernels.hip"

namespace hotruss {

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t MAX_LDS_ROW = 64 * 1024;  // one bitset row per workgroup in LDS
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Plan {
  uint32_t n = 0, h = 0, W = 0, evcap = 0;
  uint64_t m = 0;
  bool full = true;  // decomposition (false: support only)
  size_t off_ctl, off_eid, off_eu, off_ev, off_s1, off_s2, off_srem, off_upcnt, off_upoff,
      off_scan, off_sup, off_rho, off_R0, off_R1, off_L[HMAX + 1], off_Dm[HMAX + 1],
      off_evl[HMAX + 1][2];
  size_t total = 0;
};

uint32_t words_per_row(uint32_t n) {
  uint32_t w = (n + 63) / 64;
  return (w + 7) / 8 * 8;  // 64-byte rows
}

bool make_plan(uint32_t n, uint64_t m, uint32_t h, const hoTuning* tune, bool full, Plan* P) {
  if (h == 0 || m >= (1ull << 31) || n == 0xffffffffu) return false;
  if (n > 1 && h > n - 1) h = n - 1;  // any h beyond n-1 is the same as n-1
  if (h == 0) h = 1;
  if (h > HMAX) return false;
  Plan p;
  p.n = n; p.m = m; p.h = h; p.full = full;
  p.W = words_per_row(n);
  uint64_t cap = tune && tune->event_capacity ? tune->event_capacity
                                              : std::max<uint64_t>(1u << 20, 8 * m);
  cap = std::min<uint64_t>(cap, 1u << 28);
  p.evcap = (uint32_t)cap;
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
  p.off_sup = take(4 * m + 4);
  p.off_rho = take(full ? 4 * m + 4 : 0);
  p.off_R0 = take(full ? 4 * m + 4 : 0);
  p.off_R1 = take(full ? 4 * m + 4 : 0);
  for (uint32_t j = 0; j <= HMAX; ++j) {
    p.off_L[j] = p.off_Dm[j] = 0;
    p.off_evl[j][0] = p.off_evl[j][1] = 0;
  }
  for (uint32_t j = 1; j <= h; ++j) p.off_L[j] = take(rowbytes * n);
  if (full) {
    for (uint32_t j = 1; j <= h; ++j) {
      // level-1 marks are needed only when level 1 is the top level
      if (j >= 2 || h == 1) p.off_Dm[j] = take(rowbytes * n);
      const size_t c = (j == 1) ? 2 * m + 2 : p.evcap;
      p.off_evl[j][0] = take(8 * c);
      p.off_evl[j][1] = take(8 * c);
    }
  }
  p.total = o + ALIGN;  // slack for aligning the caller's base pointer
  *P = p;
  return true;
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
  return d;
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

thread_local hoStats t_stats;

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return HO_ERR_HIP; \
  } while (0)

// A1 + ball build + initial h-support into out_sup.
hoStatus run_init(const Dev& d, uint32_t* out_sup, const hoTuning* tune, hipStream_t s) {
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
  if (epw >= 16) hipLaunchKernelGGL(k_support_init<4>, dim3(grid_for(d.m, T / 4)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 8) hipLaunchKernelGGL(k_support_init<8>, dim3(grid_for(d.m, T / 8)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 4) hipLaunchKernelGGL(k_support_init<16>, dim3(grid_for(d.m, T / 16)), dim3(T), 0, s, d, out_sup);
  else if (epw >= 2) hipLaunchKernelGGL(k_support_init<32>, dim3(grid_for(d.m, T / 32)), dim3(T), 0, s, d, out_sup);
  else hipLaunchKernelGGL(k_support_init<64>, dim3(grid_for(d.m, T / 64)), dim3(T), 0, s, d, out_sup);
  HIPCHK(hipGetLastError());
  return HO_OK;
}

hoStatus read_ctl(const Dev& d, Ctl* host, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HO_OK;
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
  hipEvent_t ev0, ev1;
  HIPCHK(hipEventCreate(&ev0));
  HIPCHK(hipEventCreate(&ev1));
  HIPCHK(hipEventRecord(ev0, stream));
  const unsigned T = 256;
  // outputs and marks start at zero
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(d.m, T)), dim3(T), 0, stream, d.t, (size_t)d.m, 0u);
  for (uint32_t j = 1; j <= d.h; ++j)
    if (d.Dm[j])
      hipLaunchKernelGGL(k_fill64, dim3(grid_for((size_t)d.n * d.W, T)), dim3(T), 0, stream,
                         d.Dm[j], (size_t)d.n * d.W, 0ull);
  st = run_init(d, d.sup, tune, stream);
  if (st != HO_OK) return st;
  Ctl c;
  st = read_ctl(d, &c, stream);
  if (st != HO_OK) return st;
  if (c.err) return HO_ERR_BAD_CSR;
  const unsigned gmark = grid_for(d.m, T);
  const unsigned gwave = grid_for(1u << 30, T / WAVE);
  uint64_t iters = 0;
  while (!c.done) {
    if (c.nR == 0) {
      hipLaunchKernelGGL(k_level_min, dim3(gmark), dim3(T), 0, stream, d);
      hipLaunchKernelGGL(k_level_collect, dim3(gmark), dim3(T), 0, stream, d);
      st = read_ctl(d, &c, stream);
      if (st != HO_OK) return st;
      if (c.nR == 0) return HO_ERR_INTERNAL;  // a level jump always peels something
    }
    if (++iters > 2 * (uint64_t)d.m + 2) return HO_ERR_INTERNAL;
    hipLaunchKernelGGL(k_mark, dim3(gmark), dim3(T), 0, stream, d);
    for (uint32_t j = 2; j <= d.h; ++j)
      hipLaunchKernelGGL(k_level_events, dim3(gwave), dim3(T), 0, stream, d, j);
    hipLaunchKernelGGL(k_support_update, dim3(gwave), dim3(T), 0, stream, d);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, d);
    HIPCHK(hipGetLastError());
    st = read_ctl(d, &c, stream);
    if (st != HO_OK) return st;
  }
  HIPCHK(hipEventRecord(ev1, stream));
  HIPCHK(hipEventSynchronize(ev1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  t_stats.rounds = c.r;
  t_stats.levels = c.levels;
  t_stats.events = c.events;
  t_stats.overflows = c.overflows;
  t_stats.device_ms = ms;
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
