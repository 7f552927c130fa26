// hotruss_dev.h -- device-side state and helpers shared by the libhotruss
// kernels (gfx950, wave64).  Internal header of the GPU library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hotruss {

constexpr uint32_t HMAX = 16;            // largest hop threshold with its own ball level
constexpr uint32_t ALIVE = 0xffffffffu;  // srem value of a slot whose edge is still in S
constexpr int WAVE = 64;

// error bits in Ctl::err (set by the validation kernels)
constexpr uint32_t ERR_ROWPTR = 1u, ERR_COL = 2u, ERR_ORDER = 4u, ERR_LOOP = 8u,
                   ERR_ASYM = 16u, ERR_COUNT = 32u;

// Device control block: the whole round state lives on the device so that
// the round driver never needs the host between rounds.
struct Ctl {
  uint32_t err;
  uint32_t k;        // current level: edges with sup <= k-2 are peeled
  uint32_t r;        // index of the current peel round
  uint32_t nR;       // |R_r|, edges peeled in the current round
  uint32_t nPush;    // edges whose support crossed k-2 during this round
  uint32_t live;     // edges still in S
  uint32_t minsup;   // level jump: min support over live edges
  uint32_t levels;   // levels visited
  uint32_t done;
  uint32_t phase;    // persistent driver: next phase to run
  uint64_t events;   // top-level ball-change events (statistics)
  uint64_t overflows;
  uint32_t nev[HMAX + 1][2];  // events per level and round parity
  uint32_t ovf[HMAX + 1][2];  // event list overflowed
  uint32_t bar_count;         // grid barrier arrival counter
  uint32_t bar_gen;           // grid barrier generation
  uint32_t pad[14];
};

// Everything a kernel needs, passed by value.
struct Dev {
  const uint32_t* rp;   // row_ptr [n+1]
  const uint32_t* ci;   // col_idx [2m]
  uint32_t n, m, h, W;  // W: 64-bit words per bitset row (padded)
  uint32_t nnz;
  uint32_t evcap;       // capacity of each level>=2 event list
  uint32_t* eid;        // slot -> edge id           [2m]
  uint32_t* eu;         // edge id -> lower endpoint  [m]
  uint32_t* ev;         // edge id -> upper endpoint  [m]
  uint32_t* s1;         // edge id -> slot in row eu  [m]
  uint32_t* s2;         // edge id -> slot in row ev  [m]
  uint32_t* srem;       // slot -> round its edge was peeled, ALIVE if in S [2m]
  uint32_t* up_cnt;     // per row: neighbours above the row vertex [n]
  uint32_t* up_off;     // exclusive prefix sum of up_cnt [n]
  uint32_t* scan_tmp;   // block sums for the scan
  uint32_t* sup;        // current h-support of every edge [m]
  uint32_t* t;          // output trussness (0 while live) [m]
  uint32_t* rho;        // output peel round [m]
  uint32_t* R[2];       // peel lists by round parity [m]
  uint64_t* L[HMAX + 1];   // L[j]: closed j-hop balls, n rows of W words
  uint64_t* Dm[HMAX + 1];  // Dm[j]: pairs that left the j-ball this round
  uint64_t* evl[HMAX + 1][2];  // event lists (x<<32|w) per level and parity
  Ctl* ctl;
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ uint64_t* row(uint64_t* base, uint32_t W, uint32_t x) {
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

}  // namespace hotruss
