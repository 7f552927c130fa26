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
    ctl->jump = 1;  // nothing pushed yet: the first round jumps to min sup + 2
    ctl->live = m;
    ctl->levels = 0;
    ctl->done = (m == 0);
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

// Level 2.  Each row is built in LDS, by whichever of two frontier
// expansions reads less: top-down (sparse) scatters the adjacency of every
// z in N[x]; bottom-up (dense) ORs the level-1 rows of every z in N[x]
// (B(x,2) = union of N[z] over z in N[x]).  The dense form is taken when the
// frontier's adjacency entries exceed dthr/16 times the bitset words it
// would read, (deg(x)+1)·W.
__global__ void __launch_bounds__(256) k_build_L2(Dev d, uint32_t dthr) {
  extern __shared__ uint64_t srow[];
  __shared__ uint32_t s_fsum;
  if (d.ctl->err) return;
  const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  const uint64_t* L1 = d.L[1];
  for (uint32_t x = blockIdx.x; x < d.n; x += gridDim.x) {
    const uint32_t beg = d.rp[x], end = d.rp[x + 1];
    if (threadIdx.x == 0) s_fsum = 0;
    for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) srow[i] = 0;
    __syncthreads();
    uint32_t fs = 0;
    for (uint32_t q = beg + threadIdx.x; q < end; q += blockDim.x) {
      const uint32_t z = d.ci[q];
      fs += d.rp[z + 1] - d.rp[z];
    }
    fs = wave_sum(fs);
    if (lane == 0 && fs) atomicAdd(&s_fsum, fs);
    __syncthreads();
    const bool dense = (uint64_t)s_fsum * 16 > (uint64_t)dthr * (end - beg + 1) * d.W;
    if (dense) {
      for (uint32_t i = threadIdx.x; i < d.W; i += blockDim.x) {
        uint64_t acc = L1[(size_t)x * d.W + i];
        for (uint32_t q = beg; q < end; ++q) acc |= L1[(size_t)d.ci[q] * d.W + i];
        srow[i] = acc;
      }
    } else {
      // z = x (index end) and every neighbour z = ci[q]
      for (uint32_t q = beg + wv; q < end + 1; q += nw) {
        const uint32_t z = (q == end) ? x : d.ci[q];
        if (lane == 0) atomicOr(&srow[z >> 6], 1ull << (z & 63));
        for (uint32_t k = d.rp[z] + lane; k < d.rp[z + 1]; k += WAVE) {
          const uint32_t y = d.ci[k];
          atomicOr(&srow[y >> 6], 1ull << (y & 63));
        }
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
// G lanes cooperate on one edge; each lane loads V 64-bit words at a time
// (V = 1: 64-bit loads, V = 2: 128-bit loads; rows are 64-byte aligned).
template <int G, int V>
__global__ void __launch_bounds__(256) k_support_init(Dev d, uint32_t* __restrict__ out) {
  if (d.ctl->err) return;
  const uint64_t* Lh = d.L[d.h];
  const uint32_t sub = threadIdx.x & (G - 1);
  const uint32_t gpb = blockDim.x / G;
  const uint32_t nv = d.W / V;  // W is a multiple of 8
  for (uint32_t e = blockIdx.x * gpb + threadIdx.x / G; e < d.m; e += gridDim.x * gpb) {
    const uint64_t* a = Lh + (size_t)d.eu[e] * d.W;
    const uint64_t* b = Lh + (size_t)d.ev[e] * d.W;
    uint32_t c = 0;
    if constexpr (V == 2) {
      const ulonglong2* a2 = reinterpret_cast<const ulonglong2*>(a);
      const ulonglong2* b2 = reinterpret_cast<const ulonglong2*>(b);
      for (uint32_t i = sub; i < nv; i += G) {
        const ulonglong2 x = a2[i], y = b2[i];
        c += __popcll(x.x & y.x) + __popcll(x.y & y.y);
      }
    } else {
      for (uint32_t i = sub; i < nv; i += G) c += __popcll(a[i] & b[i]);
    }
    for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, WAVE);
    if (sub == 0) out[e] = c - 2;
  }
}

// ============================================================ peel rounds
// A round runs as a fixed kernel sequence (captured once into a HIP graph and
// replayed): k_mark, k_level(j) for j = 2..h, k_support, k_end.  Every kernel reads the control block and returns at once when
// the decomposition is finished, so a graph may run past the last round.

struct RoundCtx {
  uint32_t r, k, p;
};

__device__ __forceinline__ RoundCtx round_ctx(const Ctl* c) { return RoundCtx{c->r, c->k, c->r & 1}; }

// ---- work item emission (all 64 lanes call; per-lane counts may be 0) ----
// A lane's group of items covers one CSR row (or one ball row's words), CHUNK
// entries per item.  The wave reserves the items of all its lanes with one
// atomic and writes them cooperatively, consecutive lanes on consecutive list
// entries, so a lane whose row belongs to a hub (hundreds of items) does not
// write them alone.
//   ITEM_ROW    Item{x, y, base, meta(kind, extra, len, vstart)}: nv virtual
//               entries (the row's slots, plus the extra candidate at virtual
//               index 0 when extra = 1)
//   ITEM_SLOTS  Item{x, y, base + vstart, meta(0, 0, len, 0)}: support items
//   ITEM_WORDS  Item{x, y, vstart, meta(KIND_A_WORDS, 0, len, 0)}: ball words
enum { ITEM_ROW = 0, ITEM_SLOTS = 1, ITEM_WORDS = 2 };

__device__ __forceinline__ uint32_t chunks_of(uint32_t nv) { return (nv + CHUNK - 1) / CHUNK; }

// Lane 0 reserves `total` entries of a counter for the whole wave.
__device__ __forceinline__ uint32_t reserve_wave(uint32_t* counter, uint32_t total) {
  uint32_t b = 0;
  if (lane_id() == 0 && total) b = atomicAdd(counter, total);
  return __shfl(b, 0, WAVE);
}

// Write the wave's groups: this lane's items are entries [first + excl,
// first + excl + cnt) of list `list` (excl: exclusive prefix of cnt over the
// wave, total: the wave's sum; both from wave_excl_scan).
template <int MODE>
__device__ void emit_items_wave(const Dev& d, uint32_t list, uint32_t first, uint32_t total,
                                uint32_t excl, uint32_t cnt, uint32_t kind, uint32_t extra,
                                uint32_t x, uint32_t y, uint32_t base, uint32_t nv) {
  const uint32_t incl = excl + cnt;
  bool over = false;
  for (uint32_t t0 = 0; t0 < total; t0 += WAVE) {
    const uint32_t t = t0 + lane_id();
    // owner of entry t: the number of lanes whose groups end at or before t
    uint32_t own = 0;
#pragma unroll
    for (uint32_t step = 32; step > 0; step >>= 1) {
      const uint32_t v = (uint32_t)__shfl(incl, (int)(own + step - 1), WAVE);
      if (v <= t) own += step;
    }
    const uint32_t ox = __shfl(x, own, WAVE), oy = __shfl(y, own, WAVE);
    const uint32_t ob = __shfl(base, own, WAVE), onv = __shfl(nv, own, WAVE);
    const uint32_t oex = __shfl(excl, own, WAVE);
    if (t < total) {
      const uint32_t vs = (t - oex) * CHUNK;
      const uint32_t len = min(CHUNK, onv - vs);
      Item it;
      if (MODE == ITEM_ROW) it = Item{ox, oy, ob, item_meta(kind, extra, len, vs)};
      else if (MODE == ITEM_SLOTS) it = Item{ox, oy, ob + vs, item_meta(0, 0, len, 0)};
      else it = Item{ox, oy, vs, item_meta(KIND_A_WORDS, 0, len, 0)};
      const uint32_t idx = first + t;
      if (idx < d.itcap) d.itl[list][idx] = it;
      else over = true;
    }
  }
  if (over) d.ctl->iovf[list] = 1;
}

// One group per lane with its own reservation.
template <int MODE>
__device__ void emit_group(const Dev& d, uint32_t list, uint32_t kind, uint32_t extra, uint32_t x,
                           uint32_t y, uint32_t base, uint32_t nv) {
  const uint32_t cnt = chunks_of(nv);
  uint32_t total;
  const uint32_t excl = wave_excl_scan(cnt, &total);
  if (!total) return;
  const uint32_t first = reserve_wave(&d.ctl->nit[list], total);
  emit_items_wave<MODE>(d, list, first, total, excl, cnt, kind, extra, x, y, base, nv);
}

// Support items of event (a -> w): the live edges (a,b), CHUNK slots per item.
__device__ void emit_support_items(const Dev& d, bool active, uint32_t a, uint32_t w) {
  uint32_t base = 0, deg = 0;
  if (active) {
    base = d.rp[a];
    deg = row_end(d, a) - base;
  }
  emit_group<ITEM_SLOTS>(d, d.h + 1, 0, 0, a, w, base, deg);
}

// Items over z's old (j-1)-ball words for candidates (x, w), j >= 3.
__device__ void emit_word_items(const Dev& d, uint32_t j, bool active, uint32_t x, uint32_t z) {
  emit_group<ITEM_WORDS>(d, j, 0, 0, x, z, 0, active ? d.W : 0u);
}

// ---- level-jump minimum ----------------------------------------------------
// Per-workgroup minima of the live edges' supports (read by k_mark of a round
// that starts with a level jump).  Computed by the end-of-round kernel of the
// previous round, when every support of that round is final, and once after
// the initial pass.
__device__ void jump_partials(const Dev& d) {
  __shared__ uint32_t smin[4];
  // four edges per thread in flight: both loads unconditional
  uint32_t mn = 0xffffffffu;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  for (; e + 3 * stride < d.m; e += 4 * stride) {
    uint32_t tv[4], sv[4];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
      tv[u] = d.t[e + u * stride];
      sv[u] = d.sup[e + u * stride];
    }
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u)
      if (tv[u] == 0) mn = min(mn, sv[u]);
  }
  for (; e < d.m; e += stride) {
    const uint32_t tv = d.t[e], sv = d.sup[e];
    if (tv == 0) mn = min(mn, sv);
  }
  mn = wave_min(mn);
  if (lane_id() == 0) smin[threadIdx.x / WAVE] = mn;
  __syncthreads();
  if (threadIdx.x == 0)
    d.minpart[blockIdx.x] = min(min(smin[0], smin[1]), min(smin[2], smin[3]));
}

// After the initial pass: the first round starts with a level jump.
__global__ void __launch_bounds__(256) k_first_min(const Dev* __restrict__ devs) {
  const Dev& d = devs[blockIdx.y];
  if (d.ctl->done || d.ctl->err) return;
  jump_partials(d);
}

// ---- K2: peel R (level jump: collect it first), level-1 events, items ----
__device__ void mark_edge(const Dev& d, const RoundCtx& rc, bool valid, uint32_t e, uint32_t i) {
  uint32_t a = 0, b = 0;
  if (valid) {
    d.t[e] = rc.k;
    d.rho[e] = rc.r;
    const uint32_t q1 = d.s1[e], q2 = d.s2[e];
    d.srem[q1] = rc.r;
    d.srem[q2] = rc.r;
    a = d.eu[e];
    b = d.ev[e];
    d.ce[q1] = slot_word(e, b, true);
    d.ce[q2] = slot_word(e, a, true);
    atomicAnd(&row(d.L[1], d.W, a)[b >> 6], ~(1ull << (b & 63)));
    atomicAnd(&row(d.L[1], d.W, b)[a >> 6], ~(1ull << (a & 63)));
    if (d.h == 1) {
      atomicOr(&row(d.Dm[1], d.W, a)[b >> 6], 1ull << (b & 63));
      atomicOr(&row(d.Dm[1], d.W, b)[a >> 6], 1ull << (a & 63));
    }
    d.evl[1][rc.p][2 * i] = ((uint64_t)a << 32) | b;
    d.evl[1][rc.p][2 * i + 1] = ((uint64_t)b << 32) | a;
  }
  if (d.h == 1) {
    emit_support_items(d, valid, a, b);
    emit_support_items(d, valid, b, a);
    return;
  }
  // level 2: a lost neighbour b (candidates (a, y), y in b's old neighbourhood,
  // plus (a, b) itself) and symmetrically; level-1 events (a->b), (b->a):
  // candidates (y, b), y a live neighbour of a, and symmetrically.
  // (one reservation for the four item groups)
  uint32_t ba = 0, da = 0, bb = 0, db = 0;
  if (valid) {
    ba = d.rp[a];
    da = row_end(d, a) - ba;
    bb = d.rp[b];
    db = row_end(d, b) - bb;
  }
  // virtual entries per group: (a, y), y in N(b), plus (a, b); (b, y), y in
  // N(a), plus (b, a); (y, b), y in N(a); (y, a), y in N(b)
  const uint32_t v0 = valid ? db + 1 : 0, v1 = valid ? da + 1 : 0, v2 = valid ? da : 0,
                 v3 = valid ? db : 0;
  const uint32_t n0 = chunks_of(v0), n1 = chunks_of(v1), n2 = chunks_of(v2), n3 = chunks_of(v3);
  uint32_t t0, t1, t2, t3;
  const uint32_t e0 = wave_excl_scan(n0, &t0), e1 = wave_excl_scan(n1, &t1);
  const uint32_t e2 = wave_excl_scan(n2, &t2), e3 = wave_excl_scan(n3, &t3);
  const uint32_t first = reserve_wave(&d.ctl->nit[2], t0 + t1 + t2 + t3);
  emit_items_wave<ITEM_ROW>(d, 2, first, t0, e0, n0, KIND_A_SLOTS, 1, a, b, bb, v0);
  emit_items_wave<ITEM_ROW>(d, 2, first + t0, t1, e1, n1, KIND_A_SLOTS, 1, b, a, ba, v1);
  emit_items_wave<ITEM_ROW>(d, 2, first + t0 + t1, t2, e2, n2, KIND_B_SLOTS, 0, a, b, ba, v2);
  emit_items_wave<ITEM_ROW>(d, 2, first + t0 + t1 + t2, t3, e3, n3, KIND_B_SLOTS, 0, b, a, bb,
                            v3);
  for (uint32_t j = 3; j <= d.h; ++j) {
    emit_word_items(d, j, valid, a, b);
    emit_word_items(d, j, valid, b, a);
  }
}

// At most 64 registers per lane (eight waves per SIMD): the launch's 2,048
// workgroups of 256 threads are then all resident at once on 256 CUs, so a
// level-jump scan runs in one pass instead of leaving a second batch waiting.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_mark(const Dev* __restrict__ devs) {
  const Dev& d = devs[blockIdx.y];
  Ctl* c = d.ctl;
  if (c->done || c->halt) return;
  RoundCtx rc = round_ctx(c);
  const uint32_t q = rc.p ^ 1;
  const uint32_t lane = lane_id();
  const uint32_t wstride = gridDim.x * blockDim.x;
  const uint32_t wbase = blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1));
  if (c->jump) {
    // level jump: k <- min live sup + 2 (Algorithm 1 moving to the next
    // non-empty bin); R <- every live edge with sup <= k-2
    uint32_t mn = 0xffffffffu;
    for (uint32_t i = lane; i < d.nminpart; i += WAVE) mn = min(mn, d.minpart[i]);
    mn = wave_min(mn);
    rc.k = mn + 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->k = rc.k;
      c->levels += 1;
    }
    for (uint32_t base = wbase; base < d.m; base += wstride) {
      const uint32_t e = base + lane;
      const uint32_t tv = e < d.m ? d.t[e] : 1u, sv = e < d.m ? d.sup[e] : 0xffffffffu;
      const bool take = tv == 0 && sv <= rc.k - 2;
      if (!__ballot(take)) continue;  // nothing to peel in these 64 edges
      const uint32_t i = wave_reserve(&c->nR, take ? 1u : 0u);
      if (take) d.R[rc.p][i] = e;
      mark_edge(d, rc, take, e, i);
    }
  } else {
    const uint32_t nR = c->nR;
    if (nR <= wstride / WAVE) {
      // no more peeled edges than wavefronts: one edge per wavefront (lane 0
      // holds it), so the 64 lanes share the writing of its work items --
      // the rows of a hub endpoint are hundreds of items
      const uint32_t i = wbase / WAVE;
      if (i < nR) mark_edge(d, rc, lane == 0, lane == 0 ? d.R[rc.p][i] : 0, i);
    } else {
      for (uint32_t base = wbase; base < nR; base += wstride) {
        const uint32_t i = base + lane;
        const bool valid = i < nR;
        mark_edge(d, rc, valid, valid ? d.R[rc.p][i] : 0, i);
      }
    }
  }
  // clear the change marks of the previous round: the whole array of a level
  // whose event list overflowed, else the listed events.  At levels j >= 2 every bit set now is from
  // the previous round (this round sets its own in k_level, later), so whole
  // words are zeroed with plain stores; level 1 (h = 1 only) gets this
  // round's marks in this launch, so its old bits are cleared one by one.
  for (uint32_t j = 2; j <= d.h; ++j) {
    if (!c->ovf[j][q]) continue;
    uint64_t* D = d.Dm[j];
    const size_t cnt = (size_t)d.n * d.W;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt;
         i += (size_t)gridDim.x * blockDim.x)
      D[i] = 0;
  }
  for (uint32_t j = 1; j <= d.h; ++j) {
    uint64_t* D = d.Dm[j];
    if (!D || c->ovf[j][q]) continue;
    const uint32_t ne = c->nev[j][q];
    const uint64_t* E = d.evl[j][q];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += wstride) {
      const uint64_t xw = E[i];
      const uint32_t x = (uint32_t)(xw >> 32), w = (uint32_t)xw;
      if (j >= 2) row(D, d.W, x)[w >> 6] = 0;
      else atomicAnd(&row(D, d.W, x)[w >> 6], ~(1ull << (w & 63)));
    }
  }
}

// ---- K3: ball-change events at level j >= 2 ----------------------------
// Two workgroup shapes.  A single graph runs 16 wavefronts per workgroup,
// one workgroup per CU (its registers allow no second): the drop phase
// reserves list space once per workgroup on device-wide counters
// (same-address atomics serialise at about 11 ns each), so fewer, larger
// workgroups mean fewer of them, and a hub pair's witness probes spread over
// 1,024 threads.  Batched and served steps give every slot its own small
// grid, most of whose workgroups find nothing to do and return at once:
// there 256-thread workgroups pass through the CUs several at a time, where
// 1,024-thread ones would queue one per CU.
// The buffer holds the candidate pairs of a workgroup: a flush comes once
// another emission step (one candidate per thread at most) might not fit, so
// it holds at least two steps' worth -- bitset-word items at j >= 3 yield few
// candidates per step, and a flush per step would dominate their time.
constexpr uint32_t LV_WIDE_THREADS = 1024, LV_WIDE_CAP = 2048;    // single graph
constexpr uint32_t LV_NARROW_THREADS = 256, LV_NARROW_CAP = 1024; // batched slots
constexpr uint32_t LV_DENSE = 256; // of those, most tested on bitset rows per flush

// Block-wide exclusive scan of v[0..n) (n <= LV_CAP) into out; returns the total.
template <uint32_t LV_THREADS, uint32_t LV_CAP>
__device__ uint32_t block_scan_cap(const uint32_t* v, uint32_t* out, uint32_t n, uint32_t* wsum) {
  constexpr uint32_t LV_WAVES = LV_THREADS / WAVE;
  const uint32_t per = LV_CAP / LV_THREADS;  // entries per thread
  const uint32_t b0 = threadIdx.x * per;
  uint32_t loc[per];
  uint32_t s = 0;
  for (uint32_t i = 0; i < per; ++i) {
    loc[i] = (b0 + i < n) ? v[b0 + i] : 0u;
    s += loc[i];
  }
  uint32_t wtot;
  const uint32_t wex = wave_excl_scan(s, &wtot);
  if (lane_id() == 0) wsum[threadIdx.x / WAVE] = wtot;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (uint32_t w = 0; w < LV_WAVES; ++w) {
    if (w < threadIdx.x / WAVE) off += wsum[w];
    tot += wsum[w];
  }
  uint32_t run = off + wex;
  for (uint32_t i = 0; i < per; ++i) {
    if (b0 + i < n) out[b0 + i] = run;
    run += loc[i];
  }
  __syncthreads();
  return tot;
}

// Level-j events.  Each workgroup turns its share of work items into
// candidate pairs (quick filters: still in the j-ball, not directly
// reachable), buffers them in LDS, then tests every buffered pair at once:
// the pair's probes (the live neighbours y of its lower-degree endpoint a,
// each checked against the other endpoint's (j-1)-ball) are laid out flat
// over all threads of the workgroup.  Pairs with no witness leave the ball.
template <uint32_t LV_THREADS, uint32_t LV_CAP>
__global__ void __launch_bounds__(LV_THREADS) k_level(const Dev* __restrict__ devs, uint32_t j) {
  static_assert(LV_CAP >= 2 * LV_THREADS && LV_CAP % LV_THREADS == 0, "two emission steps fit");
  constexpr uint32_t LV_WAVES = LV_THREADS / WAVE;
  const Dev& d = devs[blockIdx.y];
  if (j > d.h) return;  // this slot's graph has fewer levels
  __shared__ uint32_t cx[LV_CAP], cw[LV_CAP], cb[LV_CAP], cbeg[LV_CAP], cdeg[LV_CAP],
      coff[LV_CAP];
  __shared__ uint32_t cflag[LV_CAP];
  __shared__ uint32_t cdense[LV_DENSE];  // candidates tested by bitset rows (see the flush)
  __shared__ uint32_t s_count, s_busy[2], s_wsum[LV_WAVES], s_ndense;
  __shared__ uint32_t s_wres[LV_WAVES][2], s_bres[2];  // per-wave and workgroup reservations
  __shared__ uint32_t s_stat[5];  // stats mode: items, slots, candidates, probes, drops
  Ctl* c = d.ctl;
  if (c->done) return;
  if (c->halt) return;
  // a round that peels every remaining edge leaves no ball or support that
  // could matter: the decomposition ends with it
  if (c->nR == c->live) return;
  if (!c->recovering && (c->iovf[j] || (d.serial & 4u))) {
    // work list overflowed (or forced): halt; the host re-runs this level in windows
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->halt = 1;
      c->halt_step = j;
      d.status[1] = 1;
    }
    return;
  }
  const RoundCtx rc = round_ctx(c);
  const uint32_t nit = min(c->nit[j], d.itcap);
  const uint32_t wave = threadIdx.x / WAVE, lane = lane_id();
  // items are dealt to workgroups first, then to their waves, so a round
  // with few items still spreads its candidates (and their probes) over as
  // many CUs as it has items
  const uint32_t stride = gridDim.x * LV_WAVES;
  uint32_t it = wave * gridDim.x + blockIdx.x;
  const bool counting = d.spart != nullptr;
  if (counting && threadIdx.x < 5) s_stat[threadIdx.x] = 0;
  if (blockIdx.x >= nit) {  // whole workgroup idle
    if (counting && threadIdx.x < 5) d.spart[threadIdx.x * STAT_GRID + blockIdx.x] = 0;
    return;
  }
  const uint64_t* Lj = d.L[j];
  const uint64_t* Lp = d.L[j - 1];
  const Item* items = d.itl[j];
  if (threadIdx.x == 0) {
    s_count = 0;
    s_busy[0] = s_busy[1] = 0;
  }
  for (uint32_t i = threadIdx.x; i < LV_CAP; i += LV_THREADS) cflag[i] = 0;
  uint32_t par = 0;
  uint64_t wd = 0;       // KIND_A_WORDS: this lane's remaining ball word
  bool inword = false;   // KIND_A_WORDS item in progress
  __syncthreads();
  while (true) {
    // ---- one emission step per wave: at most one candidate per lane ----
    bool have = false, examined = false, it_taken = false;
    uint32_t X = 0, Wv = 0;
    if (it < nit) {
      const Item I = items[it];
      const uint32_t kind = meta_kind(I.meta), len = meta_len(I.meta);
      if (kind == KIND_A_WORDS) {
        if (!inword) {
          wd = 0;
          if (lane < len) {
            const size_t o = (size_t)I.y * d.W + I.base + lane;
            wd = d.L[j - 1][o] | d.Dm[j - 1][o];
          }
          inword = true;
        }
        if (wd) {
          const uint32_t b = __ffsll((unsigned long long)wd) - 1;
          wd &= wd - 1;
          have = true;
          X = I.x;
          Wv = (I.base + lane) * 64 + b;
        }
        examined = have;
        if (!__ballot(wd != 0)) {
          inword = false;
          it += stride;
          it_taken = true;
        }
      } else {
        const uint32_t extra = meta_extra(I.meta);
        const uint32_t v = meta_vstart(I.meta) + lane;
        examined = lane < len;
        if (lane < len) {
          if (extra && v == 0) {
            have = true;
            X = I.x;
            Wv = I.y;
          } else {
            const uint32_t q = I.base + v - extra;
            const uint32_t sr = d.srem[q];
            if (kind == KIND_A_SLOTS ? sr >= rc.r : sr > rc.r) {
              have = true;
              const uint32_t y2 = d.cix[q];
              X = (kind == KIND_A_SLOTS) ? I.x : y2;
              Wv = (kind == KIND_A_SLOTS) ? y2 : I.y;
            }
          }
        }
        it += stride;
        it_taken = true;
      }
    }
    // quick filters: a real pair, still in the j-ball, not within j-1 hops
    // (both balls are symmetric, so both bits are read from the row of the
    // smaller vertex, together with the two row extents)
    // the witness probes run over the endpoint with fewer active slots
    uint32_t b = 0, beg = 0, deg = 0;
    if (have) {
      have = X != Wv;
      if (have) {
        const size_t o = (size_t)min(X, Wv) * d.W + (max(X, Wv) >> 6);
        const uint64_t sh = max(X, Wv) & 63;
        const uint64_t wj = Lj[o], wp = Lp[o];
        const uint32_t bx = d.rp[X], dx = d.len[X];
        const uint32_t bw = d.rp[Wv], dw = d.len[Wv];
        b = dx <= dw ? Wv : X;
        beg = dx <= dw ? bx : bw;
        deg = dx <= dw ? dx : dw;
        have = ((wj >> sh) & 1ull) && !((wp >> sh) & 1ull);
      }
    }
    const uint64_t bal = __ballot(have);
    if (counting) {
      const uint32_t nex = (uint32_t)__popcll(__ballot(examined));  // every lane votes
      if (lane == 0) {
        if (it_taken) atomicAdd(&s_stat[0], 1u);
        atomicAdd(&s_stat[1], nex);
        atomicAdd(&s_stat[2], (uint32_t)__popcll(bal));
      }
    }
    uint32_t slot = 0;
    if (lane == 0 && bal) slot = atomicAdd(&s_count, (uint32_t)__popcll(bal));
    slot = __shfl(slot, 0, WAVE) + (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (have) {
      cx[slot] = X;
      cw[slot] = Wv;
      cb[slot] = b;
      cbeg[slot] = beg;
      cdeg[slot] = deg;
    }
    __syncthreads();  // appends visible
    if (lane == 0 && (it < nit || inword)) atomicOr(&s_busy[par], 1u);
    __syncthreads();  // flags visible
    const bool busy = s_busy[par] != 0;
    const uint32_t n = s_count;
    __syncthreads();  // everyone has read both before anyone changes them
    if (threadIdx.x == 0) s_busy[par ^ 1] = 0;
    par ^= 1;
    if (n == 0 && !busy) break;
    if (n + LV_THREADS <= LV_CAP && busy) continue;
    // ---- flush: look for a witness of every buffered pair ----
    // A pair whose lower-degree endpoint has more active slots than a ball
    // row has words is tested on the bitset rows instead: the witnesses are
    // exactly the members of L[1](low) & L[j-1](other) (L[1] holds the live
    // closed neighbourhood, and low itself is not within j-1 hops of the
    // other endpoint), so one wave ANDs the two rows and stops at the first
    // non-zero word.  The other pairs' probes (a live neighbour y of the
    // lower-degree endpoint, checked against the other's (j-1)-ball) are laid
    // out flat over all threads of the workgroup.
    if (threadIdx.x == 0) s_ndense = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += LV_THREADS) {
      const uint32_t i = base + threadIdx.x;
      const bool dense = i < n && cdeg[i] > d.W;
      const uint64_t bd = __ballot(dense);  // one LDS reservation per wave
      uint32_t at = 0;
      if (lane == 0 && bd) at = atomicAdd(&s_ndense, (uint32_t)__popcll(bd));
      at = __shfl(at, 0, WAVE) + (uint32_t)__popcll(bd & ((1ull << lane) - 1));
      if (dense && at < LV_DENSE) {  // the rest keep their neighbour probes
        cdense[at] = i;
        cdeg[i] = 0;
      }
    }
    __syncthreads();
    const uint32_t total = block_scan_cap<LV_THREADS, LV_CAP>(cdeg, coff, n, s_wsum);
    const uint32_t ndense = min(s_ndense, LV_DENSE);
    if (counting && threadIdx.x == 0) s_stat[3] += total;
    // four probes per thread in flight: owners found in LDS first, then all
    // slot loads, then all ball-word loads
    constexpr uint32_t PU = 4;
    for (uint32_t p0 = threadIdx.x; p0 < total; p0 += PU * LV_THREADS) {
      uint32_t own[PU], q[PU], sr[PU], y[PU];
      bool act[PU];
#pragma unroll
      for (uint32_t u = 0; u < PU; ++u) {
        const uint32_t pidx = p0 + u * LV_THREADS;
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (coff[mid] <= pidx) lo = mid; else hi = mid;
        }
        own[u] = lo;
        act[u] = pidx < total && !cflag[lo];
        q[u] = cbeg[lo] + (pidx - coff[lo]);
      }
#pragma unroll
      for (uint32_t u = 0; u < PU; ++u) {
        sr[u] = act[u] ? d.srem[q[u]] : 0u;
        y[u] = act[u] ? d.cix[q[u]] : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < PU; ++u)
        if (act[u] && sr[u] > rc.r && getbit(Lp, d.W, cb[own[u]], y[u])) cflag[own[u]] = 1;
    }
    for (uint32_t k = wave; k < ndense; k += LV_WAVES) {
      const uint32_t i = cdense[k];
      const uint32_t hi = cb[i], lo = (hi == cx[i]) ? cw[i] : cx[i];
      const uint64_t* ra = row(d.L[1], d.W, lo);
      const uint64_t* rb = row(Lp, d.W, hi);
      uint32_t words = 0;
      bool found = false;
      for (uint32_t w0 = 0; w0 < d.W && !found; w0 += 4 * WAVE) {
        uint64_t any = 0;
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
          const uint32_t wi = w0 + u * WAVE + lane;
          if (wi < d.W) any |= ra[wi] & rb[wi];
        }
        words += min(4 * WAVE, d.W - w0);
        found = __ballot(any != 0) != 0;
      }
      if (lane == 0) {
        if (found) cflag[i] = 1;
        if (counting) atomicAdd(&s_stat[3], words);  // a word pair counts as one probe
      }
    }
    __syncthreads();
    // ---- pairs without a witness leave the j-ball (both directions) ----
    for (uint32_t base = 0; base < n; base += LV_THREADS) {
      const uint32_t i = base + threadIdx.x;
      const bool drop = i < n && !cflag[i];
      uint32_t x = 0, w = 0;
      bool w1 = false, w2 = false;
      if (drop) {
        x = cx[i];
        w = cw[i];
        const uint64_t bx = 1ull << (w & 63), bw = 1ull << (x & 63);
        w1 = atomicAnd(&row(d.L[j], d.W, x)[w >> 6], ~bx) & bx;
        w2 = atomicAnd(&row(d.L[j], d.W, w)[x >> 6], ~bw) & bw;
        if (w1) atomicOr(&row(d.Dm[j], d.W, x)[w >> 6], bx);
        if (w2) atomicOr(&row(d.Dm[j], d.W, w)[x >> 6], bw);
      }
      if (counting && (w1 || w2)) atomicAdd(&s_stat[4], (uint32_t)w1 + (uint32_t)w2);
      // Follow-up work of both events: the events themselves, and items over
      // the row of each event's source -- the support update (j == h), else
      // the next level's candidates (y, w) over that row plus (x, w) itself.
      // Both lists are reserved once per workgroup: device-scope atomics on
      // one address serialise, and a large round has thousands of wavefronts
      // with drops.
      const uint32_t extra = j == d.h ? 0u : 1u;
      const uint32_t list = j == d.h ? d.h + 1 : j + 1;
      uint32_t bx = 0, nx = 0, bw = 0, nw = 0;
      if (w1) {
        bx = d.rp[x];
        nx = row_end(d, x) - bx + extra;
      }
      if (w2) {
        bw = d.rp[w];
        nw = row_end(d, w) - bw + extra;
      }
      const uint32_t c1 = chunks_of(nx), c2 = chunks_of(nw);
      const uint32_t ne = (uint32_t)w1 + (uint32_t)w2;
      uint32_t t1, t2, te;
      const uint32_t e1 = wave_excl_scan(c1, &t1), e2 = wave_excl_scan(c2, &t2);
      const uint32_t ee = wave_excl_scan(ne, &te);
      if (lane == 0) {
        s_wres[wave][0] = t1 + t2;
        s_wres[wave][1] = te;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t ti = 0, tv = 0;
        for (uint32_t v = 0; v < LV_WAVES; ++v) {
          ti += s_wres[v][0];
          tv += s_wres[v][1];
        }
        s_bres[0] = ti ? atomicAdd(&d.ctl->nit[list], ti) : 0u;
        s_bres[1] = tv ? atomicAdd(&d.ctl->nev[j][rc.p], tv) : 0u;
      }
      __syncthreads();
      uint32_t ifirst = s_bres[0], efirst = s_bres[1];
      for (uint32_t v = 0; v < wave; ++v) {
        ifirst += s_wres[v][0];
        efirst += s_wres[v][1];
      }
      {
        const uint64_t exw = ((uint64_t)x << 32) | w, ewx = ((uint64_t)w << 32) | x;
        const uint32_t slot = efirst + ee;
        bool over = false;
        for (uint32_t k = 0; k < ne; ++k) {
          if (slot + k < d.evcap) d.evl[j][rc.p][slot + k] = (k || !w1) ? ewx : exw;
          else over = true;
        }
        if (over) d.ctl->ovf[j][rc.p] = 1;
      }
      if (j == d.h) {
        // support items carry the slot base of their chunk
        emit_items_wave<ITEM_SLOTS>(d, list, ifirst, t1, e1, c1, 0, 0, x, w, bx, nx);
        emit_items_wave<ITEM_SLOTS>(d, list, ifirst + t1, t2, e2, c2, 0, 0, w, x, bw, nw);
      } else {
        emit_items_wave<ITEM_ROW>(d, list, ifirst, t1, e1, c1, KIND_B_SLOTS, 1, x, w, bx, nx);
        emit_items_wave<ITEM_ROW>(d, list, ifirst + t1, t2, e2, c2, KIND_B_SLOTS, 1, w, x, bw,
                                  nw);
      }
      __syncthreads();  // s_wres and s_bres are reused by the next pass
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += LV_THREADS) cflag[i] = 0;
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    if (!busy) break;
  }
  if (counting) {
    __syncthreads();
    if (threadIdx.x < 5) d.spart[threadIdx.x * STAT_GRID + blockIdx.x] = s_stat[threadIdx.x];
  }
}

// ---- K4: support update --------------------------------------------------
// Top-level event (a -> w): every live edge (a,b) that had w as a common
// h-neighbour loses it.  Old/new rule: w counts against (a,b) if it was in
// b's old ball when a < b, and in b's new ball when a > b (see the header).
__global__ void __launch_bounds__(256) k_support(const Dev* __restrict__ devs) {
  const Dev& d = devs[blockIdx.y];
  Ctl* c = d.ctl;
  if (c->done) return;
  const uint32_t list = d.h + 1;
  if (c->halt) return;
  if (c->nR == c->live) return;  // the last round: nothing left to update
  if (!c->recovering && (c->iovf[list] || (d.serial & 8u))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->halt = 1;
      c->halt_step = list;
      d.status[1] = 1;
    }
    return;
  }
  const RoundCtx rc = round_ctx(c);
  const uint32_t nit = min(c->nit[list], d.itcap);
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  __shared__ uint32_t s_stat[3];  // stats mode: items, slots, hits
  const bool counting = d.spart != nullptr;
  if (counting) {
    if (threadIdx.x < 3) s_stat[threadIdx.x] = 0;
    __syncthreads();
  }
  const uint64_t* Lh = d.L[d.h];
  const uint64_t* Dh = d.Dm[d.h];
  uint32_t* Rn = d.R[rc.p ^ 1];
  const Item* items = d.itl[list];
  const uint32_t stride = gridDim.x * wpb;
  // Items are dealt to workgroups first, then to their waves.  Each wave
  // takes two items per step (its items it and it + stride), and the step's
  // successors and their slots (state, neighbour, edge id) load while the
  // current pair's ball words and support atomics are in flight: more memory
  // operations outstanding per wave than one item's dependent chain.
  // a slot is one 8-byte word: neighbour b (with SLOT_GONE once the edge is
  // peeled, i.e. not alive after this round) and edge id e
  struct Slot {
    Item I;
    uint32_t b, e;
  };
  auto fetch = [&](uint32_t i, Slot& S) {
    S.I = Item{0, 0, 0, 0};
    S.b = SLOT_GONE;
    S.e = 0;
    if (i < nit) {
      S.I = items[i];
      if (lane < meta_len(S.I.meta)) {
        const uint64_t w = d.ce[S.I.base + lane];
        S.b = (uint32_t)w;
        S.e = (uint32_t)(w >> 32);
      }
    }
  };
  // w in b's old ball when the event's source a < b, in its new ball when a > b
  auto hit_of = [&](const Slot& S) -> bool {
    if (S.b & SLOT_GONE) return false;
    const size_t o = (size_t)S.I.y * d.W + (S.b >> 6);
    uint64_t word = Lh[o];
    if (S.I.x < S.b) word |= Dh[o];
    return (word >> (S.b & 63)) & 1ull;
  };
  uint32_t it = (threadIdx.x / WAVE) * gridDim.x + blockIdx.x;
  Slot A, B;
  fetch(it, A);
  fetch(it + stride, B);
  while (it < nit) {
    const bool ha = hit_of(A), hb = hit_of(B);
    Slot A2, B2;
    fetch(it + 2 * stride, A2);
    fetch(it + 3 * stride, B2);
    const bool pa = ha && atomicSub(&d.sup[A.e], 1u) == rc.k - 1;
    const bool pb = hb && atomicSub(&d.sup[B.e], 1u) == rc.k - 1;
    const uint32_t slot = wave_reserve(&c->nPush, (uint32_t)pa + (uint32_t)pb);
    if (pa) Rn[slot] = A.e;
    if (pb) Rn[slot + (uint32_t)pa] = B.e;
    if (counting) {
      const uint32_t hits = (uint32_t)__popcll(__ballot(ha)) + (uint32_t)__popcll(__ballot(hb));
      if (lane == 0) {
        atomicAdd(&s_stat[0], 1u + (it + stride < nit ? 1u : 0u));
        atomicAdd(&s_stat[1], meta_len(A.I.meta) + meta_len(B.I.meta));
        atomicAdd(&s_stat[2], hits);
      }
    }
    A = A2;
    B = B2;
    it += 2 * stride;
  }
  if (counting) {
    __syncthreads();
    if (threadIdx.x < 3) d.spart[(5 + threadIdx.x) * STAT_GRID + blockIdx.x] = s_stat[threadIdx.x];
  }
}

// Stats mode: fold the per-workgroup counters of one launch into Ctl::stat.
__global__ void k_stats_fold(const Dev* __restrict__ dp, uint32_t first, uint32_t count,
                             uint32_t grid) {
  const Dev& d = *dp;
  __shared__ uint64_t acc[NSTAT];
  if (threadIdx.x < NSTAT) acc[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t c = first; c < first + count; ++c) {
    uint64_t s = 0;
    for (uint32_t b = threadIdx.x; b < grid; b += blockDim.x) {
      s += d.spart[c * STAT_GRID + b];
      d.spart[c * STAT_GRID + b] = 0;  // a launch that returns early leaves zeros
    }
    atomicAdd((unsigned long long*)&acc[c], (unsigned long long)s);
  }
  __syncthreads();
  if (threadIdx.x < NSTAT && threadIdx.x >= first && threadIdx.x < first + count)
    d.ctl->stat[threadIdx.x] += acc[threadIdx.x];
}

// ---- K5: end of round ------------------------------------------------------
// One thread closes the round (counters, next round's peel set and level-jump
// flag).  When the round pushed no edge, the next round starts with a level
// jump, and every workgroup computes its share of the live minimum now.  A
// workgroup may read the push count after the closing thread reset it: it
// then computes a minimum that nobody reads, which is harmless, and it never
// skips one that is needed (the count is only ever reset to zero).
__global__ void __launch_bounds__(256) k_end(const Dev* __restrict__ devs) {
  const Dev& d = devs[blockIdx.y];
  Ctl* c = d.ctl;
  // one decision per workgroup, taken before its closing thread (workgroup 0)
  // changes anything, so that every thread of it takes the same branch
  __shared__ uint32_t s_mode;  // 0 close only, 1 minimum and close, 2 nothing
  if (threadIdx.x == 0) s_mode = (c->done || c->halt) ? 2u : (c->nPush == 0 ? 1u : 0u);
  __syncthreads();
  const uint32_t mode = s_mode;
  if (mode == 2) return;
  if (mode == 1) jump_partials(d);
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint32_t p = c->r & 1, q = p ^ 1;
  c->nev[1][p] = 2 * c->nR;  // level-1 events: both directions of every peeled edge
  c->events += c->nev[d.h][p];
  for (uint32_t j = 1; j <= d.h; ++j) c->levents[j] += c->nev[j][p];
  c->jump = c->nPush == 0;
  uint32_t any = 0;
  for (uint32_t j = 1; j <= d.h; ++j) {
    any |= c->ovf[j][p];
    c->nev[j][q] = 0;
    c->ovf[j][q] = 0;
  }
  for (uint32_t j = 0; j <= d.h + 1; ++j) {
    any |= c->iovf[j];
    c->nit[j] = 0;
    c->iovf[j] = 0;
  }
  c->overflows += any ? 1 : 0;
  c->live -= c->nR;
  c->r += 1;
  c->nR = c->nPush;
  c->nPush = 0;
  d.status[2] = c->live;
  if (c->live == 0) {
    c->done = 1;
    d.status[0] = 1;
  }
}

// After the initial pass of a newly admitted graph: publish its state
// (malformed CSR: finished with error).
__global__ void k_post_init(Dev d) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctl* c = d.ctl;
  if (c->err) c->done = 1;
  d.status[0] = c->err ? 2u : (c->done ? 1u : 0u);
  d.status[1] = 0;
  d.status[2] = c->err ? 0u : c->live;
}

// ---- recovery of a round whose work list overflowed ----------------------
// The host re-creates the work items of the overflowed step from their
// sources, a window of sources at a time small enough for the list, and
// runs the ordinary step kernel on each window.  Re-testing a pair is
// harmless: pairs that already left fail the ball-bit filter.  Sources of
// level j: the directed removals x-lost-z of the round (index < 2|R|), then
// the level-(j-1) events from their list, or, when that list overflowed,
// the bits of the level-(j-1) change marks (row-major, 64 per word).

// Follow-up items of the event (x -> w) at list `list` (all lanes call).
__device__ __forceinline__ void fill_event_items(const Dev& d, uint32_t list, bool support,
                                                 bool has, uint32_t x, uint32_t w) {
  uint32_t bx = 0, nx = 0;
  if (has) {
    bx = d.rp[x];
    nx = d.len[x] + (support ? 0u : 1u);
  }
  if (support) emit_group<ITEM_SLOTS>(d, list, 0, 0, x, w, bx, nx);
  else emit_group<ITEM_ROW>(d, list, KIND_B_SLOTS, 1, x, w, bx, nx);
}

// Change-mark bits [blo, bhi) of level jm as events (x -> w): follow-up
// items at `list` (support items when `support`).
__device__ void fill_from_marks(const Dev& d, uint32_t jm, uint32_t list, bool support,
                                uint64_t blo, uint64_t bhi) {
  if (blo >= bhi) return;
  const uint64_t wlo = blo / 64, whi = (bhi + 63) / 64;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t wb = wlo + blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~(WAVE - 1)); wb < whi;
       wb += stride) {
    const uint64_t kw = wb + lane_id();
    uint64_t wd = 0;
    uint32_t x = 0, word = 0;
    if (kw < whi) {
      x = (uint32_t)(kw / d.W);
      word = (uint32_t)(kw % d.W);
      wd = row(d.Dm[jm], d.W, x)[word];
      if (kw == wlo && (blo & 63)) wd &= ~0ull << (blo & 63);
      if (kw == whi - 1 && (bhi & 63)) wd &= (1ull << (bhi & 63)) - 1;
    }
    while (__ballot(wd != 0)) {
      const bool has = wd != 0;
      uint32_t w = 0;
      if (has) {
        w = word * 64 + (uint32_t)(__ffsll((unsigned long long)wd) - 1);
        wd &= wd - 1;
      }
      fill_event_items(d, list, support, has, x, w);
    }
  }
}

// Listed events [elo, ehi) of level je (or the directed removals when
// `removals`): follow-up items at `list`.
__device__ void fill_from_list(const Dev& d, uint32_t je, bool removals, uint32_t p,
                               uint32_t list, bool support, uint64_t elo, uint64_t ehi) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = elo + blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~(WAVE - 1)); b < ehi;
       b += stride) {
    const uint64_t i = b + lane_id();
    const bool has = i < ehi;
    uint32_t x = 0, w = 0;
    if (has) {
      if (removals) {
        const uint32_t e = d.R[p][i >> 1];
        x = (i & 1) ? d.ev[e] : d.eu[e];
        w = (i & 1) ? d.eu[e] : d.ev[e];
      } else {
        const uint64_t xw = d.evl[je][p][i];
        x = (uint32_t)(xw >> 32);
        w = (uint32_t)xw;
      }
    }
    fill_event_items(d, list, support, has, x, w);
  }
}

__global__ void __launch_bounds__(256) k_fill_level(const Dev* __restrict__ dp, uint32_t j,
                                                    uint64_t lo, uint64_t hi) {
  const Dev& d = *dp;
  const Ctl* c = d.ctl;
  const RoundCtx rc = round_ctx(c);
  const uint64_t nA = 2ull * c->nR;
  // the directed removals x-lost-z
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t ahi = min(hi, nA);
  for (uint64_t b = lo + blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~(WAVE - 1)); b < ahi;
       b += stride) {
    const uint64_t src = b + lane_id();
    const bool a = src < ahi;
    uint32_t x = 0, z = 0;
    if (a) {
      const uint32_t e = d.R[rc.p][src >> 1];
      x = (src & 1) ? d.ev[e] : d.eu[e];
      z = (src & 1) ? d.eu[e] : d.ev[e];
    }
    if (j == 2) {
      // (x, y), y an old neighbour of z, and (x, z); (y, z), y a live neighbour of x
      uint32_t bz = 0, dz = 0, bx = 0, dx = 0;
      if (a) {
        bz = d.rp[z];
        dz = d.len[z];
        bx = d.rp[x];
        dx = d.len[x];
      }
      const uint32_t v0 = a ? dz + 1 : 0, v1 = a ? dx : 0;
      const uint32_t n0 = chunks_of(v0), n1 = chunks_of(v1);
      uint32_t t0, t1;
      const uint32_t e0 = wave_excl_scan(n0, &t0), e1 = wave_excl_scan(n1, &t1);
      const uint32_t first = reserve_wave(&d.ctl->nit[2], t0 + t1);
      emit_items_wave<ITEM_ROW>(d, 2, first, t0, e0, n0, KIND_A_SLOTS, 1, x, z, bz, v0);
      emit_items_wave<ITEM_ROW>(d, 2, first + t0, t1, e1, n1, KIND_B_SLOTS, 0, x, z, bx, v1);
    } else {
      emit_word_items(d, j, a, x, z);  // (x, w), w in z's old (j-1)-ball
    }
  }
  // the level-(j-1) events (x -> w): (y, w), y a live neighbour of x, and (x, w)
  if (j == 2 || hi <= nA) return;
  const uint64_t blo = lo > nA ? lo - nA : 0, bhi = hi - nA;
  if (c->ovf[j - 1][rc.p]) fill_from_marks(d, j - 1, j, false, blo, bhi);
  else fill_from_list(d, j - 1, false, rc.p, j, false, blo, bhi);
}

// Support items of the top-level events (listed, or the bits of the
// top-level change marks); for h = 1 the events are the directed removals.
__global__ void __launch_bounds__(256) k_fill_support(const Dev* __restrict__ dp, uint64_t lo,
                                                      uint64_t hi) {
  const Dev& d = *dp;
  const Ctl* c = d.ctl;
  const RoundCtx rc = round_ctx(c);
  if (c->ovf[d.h][rc.p]) fill_from_marks(d, d.h, d.h + 1, true, lo, hi);
  else fill_from_list(d, d.h, d.h == 1, rc.p, d.h + 1, true, lo, hi);
}

// Start of a recovery window: the step's work list is empty again.
__global__ void k_window_begin(const Dev* __restrict__ dp, uint32_t list) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  Ctl* c = dp->ctl;
  c->nit[list] = 0;
  c->iovf[list] = 0;
  c->halt = 0;
  c->recovering = 1;
  dp->status[1] = 0;
}

__global__ void k_recovery_end(const Dev* __restrict__ dp) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  dp->ctl->recovering = 0;
}

// ---- adjacency compaction (between rounds, host-triggered) --------------
// Keep each row's live slots at its front, in order, so that later rounds
// scan only live ones.  Runs only at a round boundary of a running slot:
// both kernels see the same (finished / halted) state and do nothing then.
__global__ void __launch_bounds__(256) k_compact_rows(Dev d) {
  const Ctl* c = d.ctl;
  if (c->done || c->halt) return;
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb) {
    const uint32_t beg = d.rp[x], n = d.len[x];
    uint32_t kept = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += WAVE) {
      const uint32_t i = i0 + lane;
      const bool live = i < n && d.srem[beg + i] == ALIVE;
      const uint64_t bal = __ballot(live);
      if (live) {
        const uint32_t pos = kept + (uint32_t)__popcll(bal & ((1ull << lane) - 1));
        d.tci[beg + pos] = d.cix[beg + i];
        d.teid[beg + pos] = d.eid[beg + i];
      }
      kept += (uint32_t)__popcll(bal);
    }
    if (lane == 0) d.len[x] = kept;
  }
}

__global__ void __launch_bounds__(256) k_compact_commit(Dev d) {
  Ctl* c = d.ctl;
  if (c->done || c->halt) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) c->compactions += 1;
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb) {
    const uint32_t beg = d.rp[x], n = d.len[x];
    for (uint32_t i = lane; i < n; i += WAVE) {
      const uint32_t q = beg + i, y = d.tci[q], e = d.teid[q];
      d.cix[q] = y;
      d.eid[q] = e;
      d.srem[q] = ALIVE;
      d.ce[q] = slot_word(e, y, false);
      if (y > x) d.s1[e] = q;
      else d.s2[e] = q;
    }
  }
}

// Private adjacency copy and full rows, before the first round.
__global__ void k_init_rows(Dev d) {
  if (d.ctl->err) return;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < d.nnz;
       i += (size_t)gridDim.x * blockDim.x) {
    d.cix[i] = d.ci[i];
    d.ce[i] = slot_word(d.eid[i], d.ci[i], false);
  }
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < d.n; x += gridDim.x * blockDim.x)
    d.len[x] = d.rp[x + 1] - d.rp[x];
}

// ============================================ method-level work count
// Stats mode only.  On the bulk round schedule the kernels follow, count what
// the re-evaluating form of the peeling method (Section 3) would do:
//   evaluations  every edge once at the start, then in each round the live
//                edges with an endpoint whose h-ball changed (an endpoint with
//                a top-level ball-change event: h-support depends only on the
//                two endpoint balls, Def. 3);
//   bytes        per evaluation (u,v): s(u) + s(v) + 4, s(x) = min(4 |N(x,h)|,
//                ceil(n/8)) (the smaller exact encoding of a ball); per ball
//                build: min(frontier reads of a bounded BFS to depth h-1,
//                8 + 4 deg per vertex reached; h full scans of the CSR and a
//                bitset); builds: every non-isolated vertex at the start, then
//                in each round the vertices within h-1 hops (before the round)
//                of an endpoint of a removed edge.  A round that removes every
//                remaining edge evaluates and builds nothing.
// Per-vertex ball sizes and live degrees are kept from the round's top-level
// events and removals.

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ uint64_t acct_s(const Dev& d, uint32_t x) {
  return min((uint64_t)4 * d.acct_ball[x], (uint64_t)((d.n + 7) / 8));
}

// Cost of building x's ball in the live edge set after round r (all lanes
// call with the same x; every lane gets the wave total).  live_m: |S|.
__device__ uint64_t acct_build(const Dev& d, uint32_t x, uint32_t r, uint64_t live_m) {
  uint64_t f = 0;
  const uint32_t lane = lane_id();
  if (lane == 0) f = 8 + 4ull * d.acct_deg[x];
  if (d.h == 2) {
    for (uint32_t q = d.rp[x] + lane; q < row_end(d, x); q += WAVE)
      if (d.srem[q] > r) f += 8 + 4ull * d.acct_deg[d.cix[q]];
  } else if (d.h >= 3) {
    const uint64_t* B = row(d.L[d.h - 1], d.W, x);
    for (uint32_t i = lane; i < d.W; i += WAVE) {
      uint64_t wd = B[i];
      if (i == (x >> 6)) wd &= ~(1ull << (x & 63));  // x itself is counted above
      while (wd) {
        const uint32_t y = i * 64 + (uint32_t)(__ffsll((unsigned long long)wd) - 1);
        wd &= wd - 1;
        f += 8 + 4ull * d.acct_deg[y];
      }
    }
  }
  f = wave_sum64(f);
  const uint64_t scans = (uint64_t)d.h * (4ull * (d.n + 1) + 8 * live_m + (d.n + 7) / 8);
  return min(f, scans);
}

// Start: ball sizes and degrees in G (one wave per vertex), stamps cleared.
__global__ void __launch_bounds__(256) k_acct_init(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  if (d.ctl->err) return;
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb) {
    const uint64_t* B = row(d.L[d.h], d.W, x);
    uint32_t c = 0;
    for (uint32_t i = lane; i < d.W; i += WAVE) c += (uint32_t)__popcll(B[i]);
    c = wave_sum(c);
    if (lane == 0) {
      d.acct_ball[x] = c - 1;
      d.acct_deg[x] = d.rp[x + 1] - d.rp[x];
      d.acct_stamp[x] = 0;
      d.acct_vstamp[x] = 0;
    }
  }
}

// Start: the initial pass (every edge evaluated, every non-isolated vertex's
// ball built in G).
__global__ void __launch_bounds__(256) k_acct_start(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  if (d.ctl->err) return;
  uint64_t bytes = 0;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < d.m; e += gridDim.x * blockDim.x)
    bytes += acct_s(d, d.eu[e]) + acct_s(d, d.ev[e]) + 4;
  bytes = wave_sum64(bytes);
  const uint32_t wpb = blockDim.x / WAVE;
  uint64_t builds = 0;
  for (uint32_t x = blockIdx.x * wpb + threadIdx.x / WAVE; x < d.n; x += gridDim.x * wpb)
    if (d.acct_deg[x]) builds += acct_build(d, x, 0, d.m);
  if (lane_id() == 0) {
    atomicAdd((unsigned long long*)&d.ctl->acct_bytes, (unsigned long long)(bytes + builds));
    if (blockIdx.x == 0 && threadIdx.x == 0)
      atomicAdd((unsigned long long*)&d.ctl->acct_evals, (unsigned long long)d.m);
  }
}

// True when this round leaves edges for the count (not finished, not the
// round that removes everything).
__device__ __forceinline__ bool acct_round_counts(const Ctl* c) {
  return !c->done && !c->halt && !c->err && c->nR < c->live;
}

// Round, step 1: degrees after the removals; vertices whose h-ball changed
// (sources of top-level events; at h = 1 the events are the removals), their
// ball sizes after the round, listed once each.
__global__ void __launch_bounds__(256) k_acct_round1(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  Ctl* c = d.ctl;
  if (!acct_round_counts(c)) return;
  const RoundCtx rc = round_ctx(c);
  const uint32_t stride = gridDim.x * blockDim.x, tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nR = c->nR;
  for (uint32_t i = tid; i < 2 * nR; i += stride) {
    const uint32_t e = d.R[rc.p][i >> 1];
    atomicSub(&d.acct_deg[(i & 1) ? d.ev[e] : d.eu[e]], 1u);
  }
  const bool from_removals = d.h == 1;
  if (!from_removals && c->ovf[d.h][rc.p]) {
    if (tid == 0) c->acct_incomplete = 1;
    return;
  }
  const uint32_t ne = from_removals ? 2 * nR : min(c->nev[d.h][rc.p], d.evcap);
  for (uint32_t i = tid; i < ne; i += stride) {
    uint32_t x;
    if (from_removals) {
      const uint32_t e = d.R[rc.p][i >> 1];
      x = (i & 1) ? d.ev[e] : d.eu[e];
    } else {
      x = (uint32_t)(d.evl[d.h][rc.p][i] >> 32);
    }
    atomicSub(&d.acct_ball[x], 1u);
    if (atomicExch(&d.acct_stamp[x], rc.r + 1) != rc.r + 1)
      d.acct_list[atomicAdd(&c->acct_nch, 1u)] = x;
  }
}

// Round, step 2: the evaluations (each live edge at a changed vertex once: by
// its smaller endpoint when both changed) and the ball builds, listed once
// each: the vertices within h-1 hops, before the round, of a removed edge's
// endpoint (at h-1 = 1 the endpoint and its neighbours then; above, the old
// (h-1)-ball = L[h-1] plus the pairs that left it this round).
__global__ void __launch_bounds__(256) k_acct_round2(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  Ctl* c = d.ctl;
  if (!acct_round_counts(c) || c->acct_incomplete) return;
  const RoundCtx rc = round_ctx(c);
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  const uint32_t wid = blockIdx.x * wpb + threadIdx.x / WAVE, nw = gridDim.x * wpb;
  uint64_t evals = 0, bytes = 0;
  const uint32_t nch = c->acct_nch;
  for (uint32_t k = wid; k < nch; k += nw) {
    const uint32_t x = d.acct_list[k];
    const uint64_t sx = acct_s(d, x);
    for (uint32_t q = d.rp[x] + lane; q < row_end(d, x); q += WAVE) {
      if (d.srem[q] <= rc.r) continue;
      const uint32_t b = d.cix[q];
      if (d.acct_stamp[b] == rc.r + 1 && b < x) continue;  // counted from b
      evals += 1;
      bytes += sx + acct_s(d, b) + 4;
    }
  }
  const uint32_t nR = c->nR;
  for (uint32_t k = wid; k < 2 * nR; k += nw) {
    const uint32_t e = d.R[rc.p][k >> 1];
    const uint32_t z = (k & 1) ? d.ev[e] : d.eu[e];
    auto claim = [&](uint32_t x) {
      if (atomicExch(&d.acct_vstamp[x], rc.r + 1) != rc.r + 1)
        d.acct_vlist[atomicAdd(&c->acct_nv, 1u)] = x;
    };
    if (lane == 0) claim(z);
    if (d.h == 2) {
      for (uint32_t q = d.rp[z] + lane; q < row_end(d, z); q += WAVE)
        if (d.srem[q] >= rc.r) claim(d.cix[q]);
    } else if (d.h >= 3) {
      const uint64_t* B = row(d.L[d.h - 1], d.W, z);
      const uint64_t* D = row(d.Dm[d.h - 1], d.W, z);
      for (uint32_t i = lane; i < d.W; i += WAVE) {
        uint64_t wd = B[i] | D[i];
        while (wd) {
          claim(i * 64 + (uint32_t)(__ffsll((unsigned long long)wd) - 1));
          wd &= wd - 1;
        }
      }
    }
  }
  evals = wave_sum64(evals);
  bytes = wave_sum64(bytes);
  if (lane == 0) {
    if (evals) atomicAdd((unsigned long long*)&c->acct_evals, (unsigned long long)evals);
    if (bytes) atomicAdd((unsigned long long*)&c->acct_bytes, (unsigned long long)bytes);
  }
}

// Round, step 3: the listed ball builds, in the edge set after the round;
// the round's lists are emptied for the next round.
__global__ void __launch_bounds__(256) k_acct_round3(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  Ctl* c = d.ctl;
  if (!acct_round_counts(c) || c->acct_incomplete) return;
  const RoundCtx rc = round_ctx(c);
  const uint32_t wpb = blockDim.x / WAVE;
  const uint64_t live_m = c->live - c->nR;
  uint64_t bytes = 0;
  const uint32_t nv = c->acct_nv;
  for (uint32_t k = blockIdx.x * wpb + threadIdx.x / WAVE; k < nv; k += gridDim.x * wpb)
    bytes += acct_build(d, d.acct_vlist[k], rc.r, live_m);
  if (lane_id() == 0 && bytes)
    atomicAdd((unsigned long long*)&c->acct_bytes, (unsigned long long)bytes);
}

// After step 3 (one thread): the round's lists are empty again.
__global__ void k_acct_reset(const Dev* __restrict__ dp) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  dp->ctl->acct_nch = 0;
  dp->ctl->acct_nv = 0;
}

// ============================================ (k,h)-truss extraction
// The (k,h)-truss is the edge set {e : t(e,h) >= k} (Def. 4: t(e,h) is the
// largest k whose truss holds e, and trusses are nested).  Its connected
// components come from a lock-free union-find over the vertices: a root is
// only ever linked below a smaller root, so parent[x] <= x throughout and
// every component's root is its smallest vertex.

__device__ __forceinline__ uint32_t cc_find(uint32_t* parent, uint32_t x) {
  uint32_t p = parent[x];
  while (p != x) {
    const uint32_t g = parent[p];
    if (g != p) parent[x] = g;  // path halving (any ancestor is a valid parent)
    x = p;
    p = g;
  }
  return x;
}

__global__ void k_cc_init(uint32_t* __restrict__ parent, uint32_t* __restrict__ touched,
                          uint32_t n) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    parent[x] = x;
    touched[x] = 0;
  }
}

__global__ void k_cc_hook(Dev d, const uint32_t* __restrict__ t, uint32_t k,
                          uint32_t* parent, uint32_t* __restrict__ touched) {
  if (d.ctl->err) return;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < d.m; e += gridDim.x * blockDim.x) {
    if (t[e] < k) continue;
    const uint32_t u = d.eu[e], v = d.ev[e];
    touched[u] = 1;
    touched[v] = 1;
    while (true) {
      uint32_t ru = cc_find(parent, u), rv = cc_find(parent, v);
      if (ru == rv) break;
      if (ru > rv) {
        const uint32_t tmp = ru;
        ru = rv;
        rv = tmp;
      }
      // link the larger root below the smaller one, if it is still a root
      if (atomicCAS(&parent[rv], rv, ru) == rv) break;
    }
  }
}

// Every vertex points at its root; edges of the truss take their component's
// root, the others UINT32_MAX; roots of touched vertices are counted.
__global__ void k_cc_label(Dev d, const uint32_t* __restrict__ t, uint32_t k, uint32_t* parent,
                           const uint32_t* __restrict__ touched, uint32_t* __restrict__ out,
                           uint32_t* __restrict__ count) {
  if (d.ctl->err) return;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~(WAVE - 1)); base < d.n;
       base += stride) {
    const uint32_t x = base + lane_id();
    const bool root = x < d.n && touched[x] && parent[x] == x;
    const uint32_t c = (uint32_t)__popcll(__ballot(root));
    if (lane_id() == 0 && c) atomicAdd(count, c);
  }
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < d.m; e += stride)
    out[e] = t[e] >= k ? cc_find(parent, d.eu[e]) : 0xffffffffu;
}

}  // namespace hotruss
