// hotruss_kernels.hip -- CDNA4 (gfx950) kernels of the peeling method for
// higher-order truss decomposition (paper, Section 3, Algorithm 1), executed
// as bulk-synchronous rounds with exact incremental h-support maintenance.
//
// State per vertex x and level j = 1..h: L[j](x), the closed j-hop ball
// {y : dist_S(x,y) <= j} as a dense bitset row (x included).  The h-support
// of a live edge (u,v) is |L[h](u) & L[h](v)| - 2: u and v lie in both closed
// balls and are exactly the two members that the definition excludes.
//
// A peel round removes R (all live edges with sup <= k-2).  Ball members only
// ever leave.  A pair {x,w} leaves level j exactly when every path of length
// <= j between them in the old edge set used a removed edge, and its shortest
// such path starts either with a removed edge (x,z), with w in z's old
// (j-1)-ball, or with a surviving edge (x,z) (or x itself), where w left z's
// (j-1)-ball this round.  Those two families are the candidates tested at
// level j ("ball-change events" are the pairs that really left).  For the top
// level h, the support of a live edge (a,b) drops by
//     |D(a) & Bold(b)| + |D(b) & Bnew(a)|,
// D = pairs that left, Bold = Bnew + D; each top-level event (a -> w) is
// charged to every live edge (a,b) with w in Bold(b) when a < b and w in
// Bnew(b) when a > b, which counts every lost common neighbour exactly once.
// Edges whose support crosses k-2 form the next round's R.
#include "hotruss_dev.h"

namespace hotruss {

// ---------------------------------------------------------------- fills
__global__ void k_fill64(uint64_t* __restrict__ p, size_t cnt, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill32(uint32_t* __restrict__ p, size_t cnt, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_init_ctl(Ctl* ctl, uint32_t m) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(ctl);
    for (uint32_t i = 0; i < sizeof(Ctl) / 4; ++i) w[i] = 0;
    ctl->k = 2;
    ctl->live = m;
    ctl->minsup = 0xffffffffu;
    ctl->levels = 0;
  }
}

// ---------------------------------------------------- CSR check, edge ids
// row_ptr must start at 0, never decrease and end at 2m.
__global__ void k_check_rowptr(Dev d) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x <= d.n;
       x += gridDim.x * blockDim.x) {
    uint32_t bad = 0;
    if (x == 0 && d.rp[0] != 0) bad |= ERR_ROWPTR;
    if (x == d.n && d.rp[d.n] != d.nnz) bad |= ERR_COUNT;
    if (x < d.n && d.rp[x] > d.rp[x + 1]) bad |= ERR_ROWPTR;
    if (bad) atomicOr(&d.ctl->err, bad);
  }
}

// Per row: ids in range, no self-loop, strictly ascending; count of
// neighbours above the row vertex.
__global__ void k_row_upper(Dev d) {
  if (d.ctl->err) return;
  const uint32_t lane = lane_id();
  const uint32_t wpb = blockDim.x / WAVE;
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb) {
    const uint32_t beg = d.rp[x], end = d.rp[x + 1];
    uint32_t cnt = 0, bad = 0;
    for (uint32_t j = beg + lane; j < end; j += WAVE) {
      const uint32_t y = d.ci[j];
      if (y >= d.n) bad |= ERR_COL;
      if (y == x) bad |= ERR_LOOP;
      if (j > beg && d.ci[j - 1] >= y) bad |= ERR_ORDER;
      cnt += (y > x && y < d.n);
    }
    cnt = wave_sum(cnt);
    for (int o = WAVE / 2; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, WAVE);
    if (lane == 0) {
      d.up_cnt[x] = cnt;
      if (bad) atomicOr(&d.ctl->err, bad);
    }
  }
}

// Exclusive scan of up_cnt into up_off: 1024 entries per block.
__global__ void __launch_bounds__(256) k_scan1(const uint32_t* __restrict__ in,
                                               uint32_t* __restrict__ out,
                                               uint32_t* __restrict__ bsum, uint32_t cnt) {
  __shared__ uint32_t ws[4];
  const uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4;
  uint32_t v[4], s = 0;
  for (int i = 0; i < 4; ++i) {
    v[i] = (base + i < cnt) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t incl = s;
  for (int o = 1; o < WAVE; o <<= 1) {
    uint32_t t = __shfl_up(incl, o, WAVE);
    if ((int)lane_id() >= o) incl += t;
  }
  if (lane_id() == WAVE - 1) ws[threadIdx.x / WAVE] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (uint32_t w = 0; w < threadIdx.x / WAVE; ++w) woff += ws[w];
  uint32_t run = woff + incl - s;
  for (int i = 0; i < 4; ++i) {
    if (base + i < cnt) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = woff + incl;
}

__global__ void __launch_bounds__(64) k_scan2(uint32_t* bsum, uint32_t nb) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (uint32_t i = 0; i < nb; ++i) {
    uint32_t t = bsum[i];
    bsum[i] = run;
    run += t;
  }
}

__global__ void k_scan3(uint32_t* __restrict__ out, const uint32_t* __restrict__ bsum,
                        uint32_t cnt) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    out[i] += bsum[i / 1024];
}

// Canonical edge ids (upper-triangle CSR order), endpoints and slots; every
// lower slot (x,y), y < x, finds its partner (y,x) by binary search.
__global__ void k_edge_ids(Dev d) {
  if (d.ctl->err) return;
  const uint32_t lane = lane_id();
  const uint32_t wpb = blockDim.x / WAVE;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t tot = d.n ? d.up_off[d.n - 1] + d.up_cnt[d.n - 1] : 0;
    if (tot != d.m) atomicOr(&d.ctl->err, ERR_COUNT);
  }
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb) {
    const uint32_t beg = d.rp[x], end = d.rp[x + 1];
    const uint32_t fu = end - d.up_cnt[x];
    for (uint32_t j = beg + lane; j < end; j += WAVE) {
      const uint32_t y = d.ci[j];
      d.srem[j] = ALIVE;
      if (y > x) {
        const uint32_t e = d.up_off[x] + (j - fu);
        if (e >= d.m) { atomicOr(&d.ctl->err, ERR_COUNT); continue; }
        d.eid[j] = e; d.eu[e] = x; d.ev[e] = y; d.s1[e] = j;
      } else {
        uint32_t lo = d.rp[y + 1] - d.up_cnt[y], hi = d.rp[y + 1];
        const uint32_t first = lo;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (d.ci[mid] < x) lo = mid + 1; else hi = mid;
        }
        if (lo == d.rp[y + 1] || d.ci[lo] != x) { atomicOr(&d.ctl->err, ERR_ASYM); continue; }
        const uint32_t e = d.up_off[y] + (lo - first);
        if (e >= d.m) { atomicOr(&d.ctl->err, ERR_COUNT); continue; }
        d.eid[j] = e; d.s2[e] = j;
      }
    }
  }
}

// ------------------------------------------------------------ ball build
// Level 1: closed neighbourhood N[x].  One workgroup per row, built in LDS
// and written out once (coalesced).
__global__ void __launch_bounds__(256) k_build_L1(Dev d) {
  extern __shared__ uint64_t srow[];
  if (d.ctl->err) return;
  uint64_t* L1 = d.L[1];
  for (uint32_t x = blockIdx.x; x < d.n; x += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) srow[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) atomicOr(&srow[x >> 6], 1ull << (x & 63));
    for (uint32_t j = d.rp[x] + threadIdx.x; j < d.rp[x + 1]; j += blockDim.x) {
      const uint32_t y = d.ci[j];
      atomicOr(&srow[y >> 6], 1ull << (y & 63));
    }
    __syncthreads();
    uint64_t* out = row(L1, d.W, x);
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) out[i] = srow[i];
    __syncthreads();
  }
}

// Level 2 by top-down expansion: scatter the adjacency of every z in N[x]
// into an LDS row.
__global__ void __launch_bounds__(256) k_build_L2(Dev d) {
  extern __shared__ uint64_t srow[];
  if (d.ctl->err) return;
  const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  for (uint32_t x = blockIdx.x; x < d.n; x += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) srow[i] = 0;
    __syncthreads();
    const uint32_t beg = d.rp[x], end = d.rp[x + 1];
    // z = x (index beg-1) and every neighbour z = ci[q]
    for (uint32_t q = beg + wv; q < end + 1; q += nw) {
      const uint32_t z = (q == end) ? x : d.ci[q];
      if (lane == 0) atomicOr(&srow[z >> 6], 1ull << (z & 63));
      for (uint32_t j = d.rp[z] + lane; j < d.rp[z + 1]; j += WAVE) {
        const uint32_t y = d.ci[j];
        atomicOr(&srow[y >> 6], 1ull << (y & 63));
      }
    }
    __syncthreads();
    uint64_t* out = row(d.L[2], d.W, x);
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) out[i] = srow[i];
    __syncthreads();
  }
}

// Level j >= 3 by OR-ing the (j-1)-balls of x and its neighbours
// (B(x,j) = union over z in N[x] of B(z,j-1)); each thread owns a set of words.
__global__ void __launch_bounds__(256) k_build_Lj(Dev d, uint32_t j) {
  if (d.ctl->err) return;
  const uint64_t* P = d.L[j - 1];
  uint64_t* O = d.L[j];
  for (uint32_t x = blockIdx.x; x < d.n; x += gridDim.x) {
    const uint32_t beg = d.rp[x], end = d.rp[x + 1];
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) {
      uint64_t acc = P[(size_t)x * d.W + i];
      for (uint32_t q = beg; q < end; ++q) acc |= P[(size_t)d.ci[q] * d.W + i];
      O[(size_t)x * d.W + i] = acc;
    }
  }
}

// Initial h-support of every edge: |L[h](u) & L[h](v)| - 2 (Def. 3).
// G lanes cooperate on one edge.
template <int G>
__global__ void __launch_bounds__(256) k_support_init(Dev d, uint32_t* __restrict__ out) {
  if (d.ctl->err) return;
  const uint64_t* Lh = d.L[d.h];
  const uint32_t sub = threadIdx.x & (G - 1);
  const uint32_t gpb = blockDim.x / G;
  for (uint32_t e = blockIdx.x * gpb + threadIdx.x / G; e < d.m; e += gridDim.x * gpb) {
    const uint64_t* a = Lh + (size_t)d.eu[e] * d.W;
    const uint64_t* b = Lh + (size_t)d.ev[e] * d.W;
    uint32_t c = 0;
    for (uint32_t i = sub; i < d.W; i += G) c += __popcll(a[i] & b[i]);
    for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, WAVE);
    if (sub == 0) out[e] = c - 2;
  }
}

// ------------------------------------------------------------ level jump
__global__ void k_level_min(Dev d) {
  uint32_t mn = 0xffffffffu;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < d.m; e += gridDim.x * blockDim.x)
    if (d.t[e] == 0) mn = min(mn, d.sup[e]);
  mn = wave_min(mn);
  if (lane_id() == 0 && mn != 0xffffffffu) atomicMin(&d.ctl->minsup, mn);
}

// k <- min sup + 2; R <- live edges with sup <= k-2 (Algorithm 1 moving on
// to the next non-empty bin).
__global__ void k_level_collect(Dev d) {
  const uint32_t k = d.ctl->minsup + 2;
  const uint32_t p = d.ctl->r & 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.ctl->k = k;
    d.ctl->levels += 1;
  }
  uint32_t* R = d.R[p];
  const uint32_t lane = lane_id();
  const uint32_t nthreads = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1)); base < d.m;
       base += nthreads) {
    const uint32_t e = base + lane;
    const bool take = e < d.m && d.t[e] == 0 && d.sup[e] + 2 <= k;
    const uint64_t bal = __ballot(take);
    if (!bal) continue;
    uint32_t off = 0;
    if (lane == 0) off = atomicAdd(&d.ctl->nR, (uint32_t)__popcll(bal));
    off = __shfl(off, 0, WAVE);
    if (take) R[off + __popcll(bal & ((1ull << lane) - 1))] = e;
  }
}

// ------------------------------------------------------------ peel round
// Peel R: record t = k and the round, take the edges out of S, record the
// level-1 events, and clear the previous round's change marks.
__global__ void k_mark(Dev d) {
  Ctl* c = d.ctl;
  const uint32_t r = c->r, k = c->k, nR = c->nR, p = r & 1, q = p ^ 1;
  const uint32_t* R = d.R[p];
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  uint64_t* E1 = d.evl[1][p];
  for (size_t i = tid; i < nR; i += nth) {
    const uint32_t e = R[i];
    d.t[e] = k;
    d.rho[e] = r;
    d.srem[d.s1[e]] = r;
    d.srem[d.s2[e]] = r;
    const uint32_t a = d.eu[e], b = d.ev[e];
    atomicAnd(&row(d.L[1], d.W, a)[b >> 6], ~(1ull << (b & 63)));
    atomicAnd(&row(d.L[1], d.W, b)[a >> 6], ~(1ull << (a & 63)));
    if (d.Dm[1]) {
      atomicOr(&row(d.Dm[1], d.W, a)[b >> 6], 1ull << (b & 63));
      atomicOr(&row(d.Dm[1], d.W, b)[a >> 6], 1ull << (a & 63));
    }
    E1[2 * i] = ((uint64_t)a << 32) | b;
    E1[2 * i + 1] = ((uint64_t)b << 32) | a;
  }
  if (tid == 0) c->nev[1][p] = 2 * nR;
  // clear the marks of the previous round (distinct bits from this round's)
  for (uint32_t j = 1; j <= d.h; ++j) {
    uint64_t* D = d.Dm[j];
    if (!D) continue;
    if (c->ovf[j][q]) {
      const size_t cnt = (size_t)d.n * d.W;
      for (size_t i = tid; i < cnt; i += nth) D[i] = 0;
    } else {
      const uint32_t ne = c->nev[j][q];
      const uint64_t* E = d.evl[j][q];
      for (size_t i = tid; i < ne; i += nth) {
        const uint64_t xw = E[i];
        const uint32_t x = (uint32_t)(xw >> 32), w = (uint32_t)xw;
        atomicAnd(&row(D, d.W, x)[w >> 6], ~(1ull << (w & 63)));
      }
    }
  }
}

struct RoundCtx {
  uint32_t r, k, p;
};

// Record that w left x's level-j ball (exactly once, by the thread whose
// atomic clear found the bit set).
__device__ __forceinline__ void drop_pair(const Dev& d, uint32_t j, uint32_t p, uint32_t x,
                                          uint32_t w) {
  const uint64_t bit = 1ull << (w & 63);
  const uint64_t old = atomicAnd(&row(d.L[j], d.W, x)[w >> 6], ~bit);
  if (!(old & bit)) return;
  atomicOr(&row(d.Dm[j], d.W, x)[w >> 6], bit);
  const uint32_t idx = atomicAdd(&d.ctl->nev[j][p], 1u);
  if (idx < d.evcap) d.evl[j][p][idx] = ((uint64_t)x << 32) | w;
  else d.ctl->ovf[j][p] = 1;
}

// Candidate pair (x,w) at level j: if w is still in x's j-ball but no longer
// within j hops in S_{r+1}, drop the pair in both directions.
__device__ void test_pair(const Dev& d, uint32_t j, const RoundCtx& rc, uint32_t x, uint32_t w) {
  if (x == w) return;
  const uint32_t lo = min(x, w), hi = max(x, w);
  if (!getbit(d.L[j], d.W, lo, hi)) return;
  uint32_t a = x, b = w;
  if (d.rp[a + 1] - d.rp[a] > d.rp[b + 1] - d.rp[b]) { a = w; b = x; }
  const uint64_t* P = d.L[j - 1];
  if (getbit(P, d.W, a, b)) return;
  for (uint32_t q = d.rp[a]; q < d.rp[a + 1]; ++q)
    if (d.srem[q] > rc.r && getbit(P, d.W, d.ci[q], b)) return;
  drop_pair(d, j, rc.p, x, w);
  drop_pair(d, j, rc.p, w, x);
}

// The wave handles the candidates generated by event (z -> w) at level j-1:
// (z,w) and (y,w) for every live neighbour y of z.
__device__ void wave_event_candidates(const Dev& d, uint32_t j, const RoundCtx& rc, uint32_t z,
                                      uint32_t w) {
  const uint32_t lane = lane_id();
  if (lane == 0) test_pair(d, j, rc, z, w);
  for (uint32_t q = d.rp[z] + lane; q < d.rp[z + 1]; q += WAVE)
    if (d.srem[q] > rc.r) test_pair(d, j, rc, d.ci[q], w);
}

// Level-j events of this round (j >= 2).
__global__ void __launch_bounds__(256) k_level_events(Dev d, uint32_t j) {
  Ctl* c = d.ctl;
  RoundCtx rc{c->r, c->k, c->r & 1};
  const uint32_t nR = c->nR;
  const uint32_t A = 2 * nR;
  const bool scan = c->ovf[j - 1][rc.p] != 0;
  // level-1 lists always hold every event (2|R| entries); deeper lists may overflow
  const uint32_t Bn = scan ? d.n : (j - 1 == 1 ? c->nev[1][rc.p] : min(c->nev[j - 1][rc.p], d.evcap));
  const uint32_t lane = lane_id();
  const uint32_t wpb = blockDim.x / WAVE;
  const uint64_t total = (uint64_t)A + Bn;
  for (uint64_t it = blockIdx.x * wpb + threadIdx.x / WAVE; it < total;
       it += (uint64_t)gridDim.x * wpb) {
    if (it < A) {
      // x lost its neighbour z: candidates w in z's old (j-1)-ball
      const uint32_t e = d.R[rc.p][it >> 1];
      const bool o = it & 1;
      const uint32_t x = o ? d.ev[e] : d.eu[e];
      const uint32_t z = o ? d.eu[e] : d.ev[e];
      if (j == 2) {
        if (lane == 0) test_pair(d, j, rc, x, z);
        for (uint32_t q = d.rp[z] + lane; q < d.rp[z + 1]; q += WAVE)
          if (d.srem[q] >= rc.r) test_pair(d, j, rc, x, d.ci[q]);
      } else {
        const uint64_t* Lp = row(d.L[j - 1], d.W, z);
        const uint64_t* Dp = row(d.Dm[j - 1], d.W, z);
        for (uint32_t i = lane; i < d.W; i += WAVE) {
          uint64_t wd = Lp[i] | Dp[i];
          while (wd) {
            const uint32_t b = __ffsll((unsigned long long)wd) - 1;
            wd &= wd - 1;
            test_pair(d, j, rc, x, i * 64 + b);
          }
        }
      }
    } else if (!scan) {
      const uint64_t zw = d.evl[j - 1][rc.p][it - A];
      wave_event_candidates(d, j, rc, (uint32_t)(zw >> 32), (uint32_t)zw);
    } else {
      // event list overflowed: enumerate row z of the change marks
      const uint32_t z = (uint32_t)(it - A);
      const uint64_t* Dp = row(d.Dm[j - 1], d.W, z);
      for (uint32_t i0 = 0; i0 < d.W; i0 += WAVE) {
        const uint64_t wd = (i0 + lane < d.W) ? Dp[i0 + lane] : 0ull;
        uint64_t nz = __ballot(wd != 0);
        while (nz) {
          const uint32_t src = __ffsll((unsigned long long)nz) - 1;
          nz &= nz - 1;
          uint64_t bits = __shfl(wd, src, WAVE);
          while (bits) {
            const uint32_t b = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            wave_event_candidates(d, j, rc, z, (i0 + src) * 64 + b);
          }
        }
      }
    }
  }
}

// Top-level event (a -> w): charge every live edge (a,b) that had w as a
// common h-neighbour (see the header comment for the old/new rule).
__device__ void wave_support_event(const Dev& d, const RoundCtx& rc, uint32_t a, uint32_t w,
                                   uint32_t* Rn) {
  const uint32_t lane = lane_id();
  const uint64_t* Lw = row(d.L[d.h], d.W, w);
  const uint64_t* Dw = row(d.Dm[d.h], d.W, w);
  for (uint32_t q = d.rp[a] + lane; q < d.rp[a + 1]; q += WAVE) {
    if (d.srem[q] <= rc.r) continue;
    const uint32_t b = d.ci[q];
    uint64_t word = Lw[b >> 6];
    if (a < b) word |= Dw[b >> 6];
    if (!((word >> (b & 63)) & 1ull)) continue;
    const uint32_t e = d.eid[q];
    const uint32_t old = atomicSub(&d.sup[e], 1u);
    if (old == rc.k - 1) {
      const uint32_t idx = atomicAdd(&d.ctl->nPush, 1u);
      Rn[idx] = e;
    }
  }
}

__global__ void __launch_bounds__(256) k_support_update(Dev d) {
  Ctl* c = d.ctl;
  RoundCtx rc{c->r, c->k, c->r & 1};
  const uint32_t h = d.h;
  const bool scan = c->ovf[h][rc.p] != 0;
  const uint32_t total = scan ? d.n : min(c->nev[h][rc.p], h == 1 ? 2 * d.m : d.evcap);
  uint32_t* Rn = d.R[rc.p ^ 1];
  const uint32_t lane = lane_id();
  const uint32_t wpb = blockDim.x / WAVE;
  for (uint32_t it = blockIdx.x * wpb + threadIdx.x / WAVE; it < total; it += gridDim.x * wpb) {
    if (!scan) {
      const uint64_t aw = d.evl[h][rc.p][it];
      wave_support_event(d, rc, (uint32_t)(aw >> 32), (uint32_t)aw, Rn);
    } else {
      const uint32_t a = it;
      const uint64_t* Dp = row(d.Dm[h], d.W, a);
      for (uint32_t i0 = 0; i0 < d.W; i0 += WAVE) {
        const uint64_t wd = (i0 + lane < d.W) ? Dp[i0 + lane] : 0ull;
        uint64_t nz = __ballot(wd != 0);
        while (nz) {
          const uint32_t src = __ffsll((unsigned long long)nz) - 1;
          nz &= nz - 1;
          uint64_t bits = __shfl(wd, src, WAVE);
          while (bits) {
            const uint32_t b = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            wave_support_event(d, rc, a, (i0 + src) * 64 + b, Rn);
          }
        }
      }
    }
  }
}

// End of round: bookkeeping by one thread.
__global__ void k_advance(Dev d) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctl* c = d.ctl;
  const uint32_t p = c->r & 1, q = p ^ 1;
  c->events += c->nev[d.h][p];
  uint32_t any = 0;
  for (uint32_t j = 1; j <= d.h; ++j) {
    any |= c->ovf[j][p];
    c->nev[j][q] = 0;
    c->ovf[j][q] = 0;
  }
  c->overflows += any ? 1 : 0;
  c->live -= c->nR;
  c->r += 1;
  c->nR = c->nPush;
  c->nPush = 0;
  c->minsup = 0xffffffffu;
  if (c->live == 0) c->done = 1;
}

}  // namespace hotruss
