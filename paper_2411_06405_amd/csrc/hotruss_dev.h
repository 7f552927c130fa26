// hotruss_dev.h -- device-side state and helpers shared by the libhotruss
// kernels (gfx950, wave64).  Internal header of the GPU library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hotruss {

constexpr uint32_t HMAX = 16;            // largest hop threshold with its own ball level
constexpr uint32_t ALIVE = 0xffffffffu;  // srem value of a slot whose edge is still in S
constexpr uint32_t SLOT_GONE = 0x80000000u;  // in the low word of ce: the slot's edge is peeled
constexpr int WAVE = 64;
constexpr uint32_t CHUNK = 64;           // slots (or bitset words) per work item
constexpr uint32_t MIN_PART = 1024;      // partial-minimum slots of the level-jump reduction
constexpr uint32_t NSTAT = 8;            // work counters kept in stats mode
constexpr uint32_t STAT_GRID = 8192;     // most workgroups a counted kernel may use

// error bits in Ctl::err (set by the validation kernels)
constexpr uint32_t ERR_ROWPTR = 1u, ERR_COL = 2u, ERR_ORDER = 4u, ERR_LOOP = 8u,
                   ERR_ASYM = 16u, ERR_COUNT = 32u;

// Work item kinds.  A work item covers at most CHUNK consecutive CSR slots
// (or bitset words) of one vertex, so that a wavefront handles it in one step.
//   KIND_A_SLOTS  level j = 2, x lost its neighbour z:   candidates (x, y), y in the
//                 old neighbourhood of z (slots with srem >= r); extra: (x, z)
//   KIND_A_WORDS  level j >= 3, x lost its neighbour z:  candidates (x, w), w in z's
//                 old (j-1)-ball (bitset words [base, base+len))
//   KIND_B_SLOTS  w left z's (j-1)-ball: candidates (y, w), y a live neighbour of z
//                 (slots with srem > r); extra: (z, w)
// Item = {x, y, base, meta}: meta = kind << 30 | extra << 29 | len << 22 | vstart.
constexpr uint32_t KIND_A_SLOTS = 0, KIND_A_WORDS = 1, KIND_B_SLOTS = 2;

struct Item {
  uint32_t x, y, base, meta;
};

__host__ __device__ inline uint32_t item_meta(uint32_t kind, uint32_t extra, uint32_t len,
                                              uint32_t vstart) {
  return (kind << 30) | (extra << 29) | (len << 22) | vstart;
}
__device__ inline uint32_t meta_kind(uint32_t m) { return m >> 30; }
__device__ inline uint32_t meta_extra(uint32_t m) { return (m >> 29) & 1u; }
__device__ inline uint32_t meta_len(uint32_t m) { return (m >> 22) & 127u; }
__device__ inline uint32_t meta_vstart(uint32_t m) { return m & ((1u << 22) - 1); }

// Device control block: the whole round state lives on the device so that
// the round driver never needs the host between rounds.
struct Ctl {
  uint32_t err;
  uint32_t k;        // current level: edges with sup <= k-2 are peeled
  uint32_t r;        // index of the current peel round
  uint32_t nR;       // |R_r|, edges peeled in the current round
  uint32_t nPush;    // edges whose support crossed k-2 during this round
  uint32_t live;     // edges still in S
  uint32_t levels;   // levels visited
  uint32_t done;     // decomposition finished (read by the host with halt)
  uint32_t halt;     // a work list overflowed: the host re-runs the step in windows
  uint32_t halt_step;  // step that halted: level j (2..h), or h+1 for the support update
  uint32_t jump;     // this round starts with a level jump
  uint64_t events;   // top-level ball-change events (statistics)
  uint64_t overflows;
  uint32_t nev[HMAX + 1][2];  // events per level and round parity
  uint32_t ovf[HMAX + 1][2];  // event list overflowed
  uint32_t nit[HMAX + 2];     // work items per level (index h+1: support items)
  uint32_t iovf[HMAX + 2];    // work item list overflowed
  uint32_t compactions;  // adjacency compactions done (statistics)
  uint32_t recovering;   // the host is re-running an overflowed step in windows
  // stats mode: method-level work count (support evaluations and bytes of the
  // re-evaluating peeling method on the same round schedule)
  uint32_t acct_nch;     // vertices whose h-ball changed this round (listed)
  uint32_t acct_nv;      // ball builds of this round (listed)
  uint32_t acct_incomplete;  // an event list overflowed: the count is a lower bound
  uint32_t pad[2];
  uint64_t acct_evals;
  uint64_t acct_bytes;
  uint64_t levents[HMAX + 1];  // ball-change events per level, all rounds
  // stats mode: work counters, level kernel [0..5), support kernel [5..8)
  uint64_t stat[NSTAT];
};

// Everything a kernel needs, passed by value.
struct Dev {
  const uint32_t* rp;   // row_ptr [n+1]
  const uint32_t* ci;   // col_idx [2m]
  uint32_t n, m, h, W;  // W: 64-bit words per bitset row (padded)
  uint32_t nnz;
  uint32_t evcap;       // capacity of each level>=2 event list
  uint32_t itcap;       // capacity of each work item list
  uint32_t nminpart;    // blocks of the level-jump minimum kernel
  uint32_t serial;      // testing: bit 2 forces the windowed re-run of every level step,
                        // bit 3 of every support step, bit 4 compacts rows at every chance
  uint32_t* eid;        // slot -> edge id           [2m]
  uint32_t* eu;         // edge id -> lower endpoint  [m]
  uint32_t* ev;         // edge id -> upper endpoint  [m]
  uint32_t* s1;         // edge id -> slot in row eu  [m]
  uint32_t* s2;         // edge id -> slot in row ev  [m]
  uint32_t* srem;       // slot -> round its edge was peeled, ALIVE if in S [2m]
  // Round kernels read the adjacency through a private copy whose rows are
  // compacted now and then (live slots first, in order): row x's active
  // slots are [rp[x], rp[x] + len[x]); slots past len[x] are dead.
  uint32_t* cix;        // private column ids [2m]
  uint32_t* len;        // active slots per row [n]
  uint32_t* tci;        // compaction staging: column ids [2m]
  uint32_t* teid;       // compaction staging: edge ids [2m]
  // The support update's view of a slot, one 8-byte load: low word the
  // neighbour id with SLOT_GONE set once the edge is peeled, high word the
  // edge id [2m] (same row layout as cix)
  uint64_t* ce;
  uint32_t* up_cnt;     // per row: neighbours above the row vertex [n]
  uint32_t* up_off;     // exclusive prefix sum of up_cnt [n]
  uint32_t* scan_tmp;   // block sums for the scan
  uint32_t* minpart;    // per-block minima of the level-jump reduction
  uint32_t* sup;        // current h-support of every edge [m]
  uint32_t* t;          // output trussness (0 while live) [m]
  uint32_t* rho;        // output peel round [m]
  uint32_t* R[2];       // peel lists by round parity [m]
  uint64_t* L[HMAX + 1];   // L[j]: closed j-hop balls, n rows of W words
  uint64_t* Dm[HMAX + 1];  // Dm[j]: pairs that left the j-ball this round
  uint64_t* evl[HMAX + 1][2];  // event lists (x<<32|w) per level and parity
  Item* itl[HMAX + 2];     // work items per level; index h+1: support items
  Ctl* ctl;
  Dev* self;               // device-resident copy of this struct (round kernels read it)
  uint32_t* spart;         // stats mode: per-workgroup counters [NSTAT][STAT_GRID], else null
  uint32_t* status;        // this slot's {done, halt, live, -} words in the engine's status
                           // array (done: 1 finished, 2 malformed CSR; live: edges left)
  // stats mode, method-level work count: per vertex |N(x,h)|, live degree,
  // round stamps (h-ball changed, ball build counted) and this round's lists
  uint32_t* acct_ball;
  uint32_t* acct_deg;
  uint32_t* acct_stamp;
  uint32_t* acct_vstamp;
  uint32_t* acct_list;
  uint32_t* acct_vlist;
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t slot_word(uint32_t e, uint32_t y, bool gone) {
  return ((uint64_t)e << 32) | y | (gone ? SLOT_GONE : 0u);
}

// End of row x's active slots (round kernels).
__device__ __forceinline__ uint32_t row_end(const Dev& d, uint32_t x) { return d.rp[x] + d.len[x]; }

__device__ __forceinline__ uint64_t* row(uint64_t* base, uint32_t W, uint32_t x) {
  return base + (size_t)x * W;
}
__device__ __forceinline__ const uint64_t* row(const uint64_t* base, uint32_t W, uint32_t x) {
  return base + (size_t)x * W;
}

__device__ __forceinline__ bool getbit(const uint64_t* base, uint32_t W, uint32_t x, uint32_t w) {
  return (base[(size_t)x * W + (w >> 6)] >> (w & 63)) & 1ull;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o, WAVE));
  return v;
}

// Exclusive prefix sum across the wave (all 64 lanes must call).
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
  uint32_t incl = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, WAVE);
    if ((int)lane_id() >= o) incl += t;
  }
  *total = __shfl(incl, WAVE - 1, WAVE);
  return incl - v;
}

// Wave-aggregated reservation of `cnt` slots of a counter (all lanes call).
// Returns this lane's first slot.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* counter, uint32_t cnt) {
  uint32_t total;
  const uint32_t off = wave_excl_scan(cnt, &total);
  uint32_t base = 0;
  if (lane_id() == 0 && total) base = atomicAdd(counter, total);
  base = __shfl(base, 0, WAVE);
  return base + off;
}

}  // namespace hotruss
