// hotruss_hindex.hip -- CDNA4 (gfx950) kernels of the H-index fixpoint
// method for higher-order truss decomposition (paper, Section 4.1: the h-hop
// reachable path key and the higher-order H-index; Section 4.2, Algorithm 2:
// the parallel update loop; Section 4.1: asynchronous updating).
//
// Every sweep recomputes, for each edge e = (u,v),
//     H(e) <- H({ min(P(u,w), P(v,w)) : w in the common h-hop neighbourhood }),
// where P(x,w) is the largest smallest-key over paths of at most h edges
// from x to w, keys being the current H values.  The values never rise
// (Theorem 1) and settle at t(e,h) - 2 (Theorem 2).
//
// Path keys depend on the source vertex only, so a sweep first builds the
// path-key row of every vertex that needs one (k_hx_paths) and then updates
// the edges (k_hx_edges), instead of the paper's per-edge searches.
//
// Layout.  L[h](x) is the closed h-hop ball of x in G as a dense bitset row
// (built once by the peeling method's ball kernels; G never changes here).
// Row x of the path keys holds one u32 per member of L[h](x), in increasing
// vertex order: the key of w is at P[boff[x] + rank_x(w)], with
//     rank_x(w) = wp[x*W + w/64] + popcount(L[h](x) word w/64 below bit w),
// wp holding, per row and word, the members in the row's earlier words.
// The members themselves are listed in the same order (mem), so the key of
// the i-th member of x's ball is P[boff[x] + i].
// A key of 0 also stands for "not reached yet": a path key is never below
// 0, so the placeholder can only lose a maximum.
//
// Change tracking (exact; the same answer as recomputing everything): an edge
// whose H changed marks both endpoints "touched".  P(x,.) reads only keys of
// edges with an endpoint within h-1 hops of x, so a row needs rebuilding only
// if L[h-1](x) (for h = 1: x itself) holds a touched vertex.  A rebuilt row
// records in a 64-bucket mask the value ranges its keys fell through: a key
// that went from a to b < a marks the buckets of b+1 .. a.  An edge with
// value c keeps it unless some key of its endpoints' rows fell from >= c to
// < c: otherwise at least c common members still have both keys >= c, and
// values never rise.  So after the first sweep an edge is re-evaluated only if
// the bucket of c is marked in either endpoint's mask.
//
// The default rule is the paper's pruning (Section 4.3, Lemma 4): the same
// crossing test on edge values instead of path keys.  A changed edge (a -> b)
// marks the buckets of b+1 .. a at both endpoints; a vertex's mask for the
// next sweep is the OR over its closed (h-1)-ball, i.e. over every edge its
// path keys read; an edge is skipped unless c's bucket is marked (cases i-iii
// of the lemma all leave the bucket of c unmarked).  It re-evaluates a few
// more edges than the path-key rule but needs no previous keys.
//
// Asynchronous sweeps split the vertices into consecutive chunks processed in
// order; chunk c rebuilds its rows from the keys as they stand (including the
// ones earlier chunks of the same sweep changed) and then updates the edges
// whose upper endpoint lies in c, so both endpoint rows are from this sweep.
#include "hotruss_dev.h"

namespace hotruss {

constexpr uint32_t HX_SRC = 1024;   // relaxation sources staged per batch
constexpr uint32_t HX_BIG = 16384;  // h = 2: rows with more relaxations are split
constexpr uint32_t HX_SLICE = 16;   // sources per slice of a split row
constexpr uint32_t HX_BINS = 4 * 64;  // histogram bins per wave (4 per lane)
constexpr uint32_t HX_STAGE_WORDS = HX_SRC / 64;
constexpr uint32_t HX_CTR_CHANGED = 0, HX_CTR_EVALS = 1, HX_CTR_ROWS = 2, HX_CTR_TLIST = 3;
// work counters of the stats mode
constexpr uint32_t HX_ST_PASSES = 0, HX_ST_SCAN = 1, HX_ST_MEMBERS = 2, HX_ST_ROWS = 3,
                   HX_ST_DIRECT = 4, HX_ST_RELAX = 5, HX_ST_ENTRIES = 6, HX_ST_EVALS = 7;

struct Hx {
  const uint32_t* rp;      // row_ptr [n+1]
  const uint32_t* ci;      // col_idx [2m]
  const uint32_t* eid;     // slot -> edge id [2m]
  const uint32_t* eu;      // edge -> lower endpoint [m]
  const uint32_t* ev;      // edge -> upper endpoint [m]
  const uint32_t* up_cnt;  // per row: neighbours above the row vertex [n]
  const uint32_t* up_off;  // exclusive prefix sum of up_cnt [n]
  const uint64_t* L[HMAX + 1];  // closed balls of G, n rows of W words
  uint32_t n, m, h, W;
  uint32_t* wp;        // per row and word: members of L[h] in earlier words [n*W]
  uint32_t* mem;       // the members of L[h](x) in increasing order, row x at boff[x] [S]
  uint32_t* cnt;       // |L[h](x)| [n]
  uint64_t* boff;      // start of row x's path keys [n+1]
  uint32_t* H;         // current H-index of every edge [m]
  uint32_t* P[2];      // path keys; P[0] holds the finished rows (P[1]: h >= 3 only)
  uint32_t* Pold;      // tracking: a rebuilt row's previous keys [S]
  uint64_t* dmask;     // tracking: value buckets the keys of row x fell through [n]
  uint32_t* dirty;     // row x is rebuilt (and its edges re-evaluated) this sweep [n]
  uint32_t* touched;   // x is an endpoint of an edge changed this sweep [n]
  uint64_t* tbits;     // touched as a bitset [W]
  uint32_t* tlist;     // nonzero words of tbits [W]
  uint32_t* ord;       // edge ids ordered by upper endpoint [m]
  uint32_t* cbound;    // chunk c's edges are ord[cbound[c] .. cbound[c+1]) [chunks+1]
  uint32_t* ctr;       // counters: changed, evaluated, rows built, tlist length
  uint32_t track;      // change tracking on: skip clean rows and edges
  uint32_t first;      // first sweep: every edge is evaluated
  uint32_t lemma4;     // edge masks from changed edge values (Lemma 4), not from path keys
  uint32_t* cmask;     // Lemma 4: value buckets crossed by changed edges at x, as 2 u32 [2n]
  uint32_t hist1;      // the counting pass also fills the first histogram
  uint32_t* tmin;      // smallest new value among the changed edges at x this sweep [n]
  // h = 2: rows whose relaxations are split over workgroups, {rows, slices} in
  // one counter; row i is bigu[i], its slices start at bigoff[i] [n each]
  unsigned long long* bigctr;
  uint32_t* bigu;
  uint32_t* bigoff;
  unsigned long long* stat;  // stats mode: work counters HX_ST_* [8], else null
};

// Bucket of a value for the drop masks: 0..31 exact, then two buckets per
// octave up to 2^20, the rest in bucket 63.  Non-decreasing in v.
__device__ __forceinline__ uint32_t hx_bucket(uint32_t v) {
  if (v < 32) return v;
  const uint32_t e = 31u - (uint32_t)__clz(v);
  return min(63u, 32u + (e - 5) * 2 + ((v >> (e - 1)) & 1u));
}

// Buckets of the thresholds c with b < c <= a (a value that fell from a to b).
__device__ __forceinline__ unsigned long long hx_range_mask(uint32_t b, uint32_t a) {
  const uint32_t lo = hx_bucket(b + 1), hi = hx_bucket(a);
  return (~0ull >> (63 - hi)) & ~((1ull << lo) - 1);
}

__device__ __forceinline__ uint32_t hx_rank(const Hx& x, uint32_t u, uint32_t w) {
  const size_t i = (size_t)u * x.W + (w >> 6);
  const uint64_t below = (1ull << (w & 63)) - 1;
  return x.wp[i] + (uint32_t)__popcll(x.L[x.h][i] & below);
}

// Ball sizes and per-word member counts of every row (one wave per row).
__global__ void __launch_bounds__(256) k_hx_rank(Hx x) {
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  const uint64_t* Lh = x.L[x.h];
  for (uint32_t r = blockIdx.x * wpb + threadIdx.x / WAVE; r < x.n; r += gridDim.x * wpb) {
    uint32_t run = 0;
    for (uint32_t i0 = 0; i0 < x.W; i0 += WAVE) {
      const uint32_t i = i0 + lane;
      const uint32_t c = i < x.W ? (uint32_t)__popcll(Lh[(size_t)r * x.W + i]) : 0;
      uint32_t tot;
      const uint32_t ex = wave_excl_scan(c, &tot);
      if (i < x.W) x.wp[(size_t)r * x.W + i] = run + ex;
      run += tot;
    }
    if (lane == 0) x.cnt[r] = run;
  }
}

// 64-bit exclusive prefix sum of cnt[0..n) into off[0..n]; one workgroup of
// 1024 threads, each summing a contiguous segment.
__global__ void __launch_bounds__(1024) k_hx_scan(const uint32_t* __restrict__ cnt,
                                                   uint64_t* __restrict__ off, uint32_t n) {
  __shared__ uint64_t s[1024];
  const uint32_t t = threadIdx.x, per = (n + 1023) / 1024;
  const uint32_t b = min(n, t * per), e = min(n, b + per);
  uint64_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += cnt[i];
  s[t] = sum;
  __syncthreads();
  for (uint32_t o = 1; o < 1024; o <<= 1) {
    const uint64_t v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  uint64_t run = s[t] - sum;
  for (uint32_t i = b; i < e; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[n] = s[1023];
}

// Member lists of every ball, in vertex order (one wave per row).
__global__ void __launch_bounds__(256) k_hx_members(Hx x) {
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  const uint64_t* Lh = x.L[x.h];
  for (uint32_t r = blockIdx.x * wpb + threadIdx.x / WAVE; r < x.n; r += gridDim.x * wpb) {
    uint32_t* out = x.mem + x.boff[r];
    uint32_t run = 0;
    for (uint32_t i0 = 0; i0 < x.W; i0 += WAVE) {
      const uint32_t i = i0 + lane;
      uint64_t b = i < x.W ? Lh[(size_t)r * x.W + i] : 0;
      uint32_t tot;
      uint32_t at = run + wave_excl_scan((uint32_t)__popcll(b), &tot);
      while (b) {
        out[at++] = i * 64 + (uint32_t)__ffsll((long long)b) - 1;
        b &= b - 1;
      }
      run += tot;
    }
  }
}

// Edge ids in order of their upper endpoint: row x's lower slots (its first
// deg(x) - up_cnt(x) slots) list the edges whose upper endpoint is x, and the
// lower slots of rows before x number rp[x] - up_off[x].
__global__ void __launch_bounds__(256) k_hx_order(Hx x) {
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t r = blockIdx.x * wpb + threadIdx.x / WAVE; r < x.n; r += gridDim.x * wpb) {
    const uint32_t beg = x.rp[r], nlow = x.rp[r + 1] - beg - x.up_cnt[r];
    const uint32_t at = beg - x.up_off[r];
    for (uint32_t j = lane; j < nlow; j += WAVE) x.ord[at + j] = x.eid[beg + j];
  }
}

// Chunk c covers vertices [c*n/chunks, (c+1)*n/chunks).
__global__ void k_hx_bounds(Hx x, uint32_t chunks) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > chunks) return;
  const uint32_t v = (uint32_t)((uint64_t)c * x.n / chunks);
  x.cbound[c] = v < x.n ? x.rp[v] - x.up_off[v] : x.m;
}

// Relax the staged sources s_y[0..nb) with path keys s_k into row `dst` of
// vertex u: for every edge (y, w), w != u, key(u,w) >= min(s_k, H(y,w)).
// Work is spread over the whole workgroup by a prefix sum of the sources'
// degrees (sources with key 0 contribute nothing and get degree 0).
// Returns the number of relaxations.
__device__ uint32_t hx_relax(const Hx& x, uint32_t u, uint32_t nb, uint32_t* __restrict__ dst,
                             const uint32_t* s_y, const uint32_t* s_k, uint32_t* s_pre) {
  if (threadIdx.x < WAVE) {
    uint32_t run = 0;
    for (uint32_t i0 = 0; i0 < nb; i0 += WAVE) {
      const uint32_t i = i0 + threadIdx.x;
      uint32_t d = 0;
      if (i < nb && s_k[i]) d = x.rp[s_y[i] + 1] - x.rp[s_y[i]];
      uint32_t tot;
      const uint32_t ex = wave_excl_scan(d, &tot);
      if (i < nb) s_pre[i] = run + ex;
      run += tot;
    }
    if (threadIdx.x == 0) s_pre[nb] = run;
  }
  __syncthreads();
  const uint32_t total = s_pre[nb];
  for (uint32_t k = threadIdx.x; k < total; k += blockDim.x) {
    // the last source whose range starts at or before k
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_pre[mid] <= k) lo = mid; else hi = mid;
    }
    const uint32_t y = s_y[lo];
    const uint32_t r = x.rp[y] + (k - s_pre[lo]);
    const uint32_t w = x.ci[r];
    if (w == u) continue;
    const uint32_t val = min(s_k[lo], x.H[x.eid[r]]);
    if (val) atomicMax(&dst[hx_rank(x, u, w)], val);
  }
  return total;
}

// Drop mask of row u (all threads of the workgroup call; s_mask is LDS).
__device__ void hx_row_mask(const Hx& x, uint32_t u, const uint32_t* old, const uint32_t* fin,
                            uint32_t len, uint32_t* s_mask) {
  if (threadIdx.x < 2) s_mask[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long mk = 0;
  for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
    const uint32_t a = old[i], b = fin[i];
    if (b < a) mk |= hx_range_mask(b, a);
  }
  if ((uint32_t)mk) atomicOr(&s_mask[0], (uint32_t)mk);
  if (mk >> 32) atomicOr(&s_mask[1], (uint32_t)(mk >> 32));
  __syncthreads();
  if (threadIdx.x == 0) x.dmask[u] = (uint64_t)s_mask[1] << 32 | s_mask[0];
  __syncthreads();
}

// Path-key rows of the vertices in [vlo, vhi) (one workgroup per vertex):
// one hop from u's own edges, a second hop relaxed in place (its sources read
// the direct keys from H, never the row), further hops double-buffered so a
// pass extends paths by exactly one edge.
__global__ void __launch_bounds__(256) k_hx_paths(Hx x, uint32_t vlo, uint32_t vhi) {
  __shared__ uint32_t s_y[HX_SRC], s_k[HX_SRC], s_pre[HX_SRC + 1];
  __shared__ uint32_t s_cnt[HX_STAGE_WORDS];
  __shared__ uint32_t s_mask[2], s_rs;
  uint32_t built = 0;
  unsigned long long direct = 0, relax = 0, entries = 0;
  for (uint32_t u = vlo + blockIdx.x; u < vhi; u += gridDim.x) {
    if (x.track && !x.dirty[u]) continue;
    ++built;
    const uint64_t base = x.boff[u];
    const uint32_t len = (uint32_t)(x.boff[u + 1] - base);
    uint32_t cur = x.h >= 2 ? ((x.h - 2) & 1u) : 0u;  // so that the last hop lands in P[0]
    uint32_t* row = x.P[cur] + base;
    uint32_t* fin = x.P[0] + base;
    uint32_t* old = x.Pold + base;
    if (threadIdx.x == 0) s_rs = 0;
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
      if (x.track && !x.lemma4) old[i] = fin[i];
      row[i] = 0;
    }
    __syncthreads();
    const uint32_t beg = x.rp[u], end = x.rp[u + 1];
    direct += end - beg;
    entries += (unsigned long long)len * (x.h >= 3 ? x.h - 1 : 1);
    uint32_t rs = 0;  // relaxations of the second hop
    for (uint32_t q = beg + threadIdx.x; q < end; q += blockDim.x) {
      const uint32_t y = x.ci[q];
      row[hx_rank(x, u, y)] = x.H[x.eid[q]];
      rs += x.rp[y + 1] - x.rp[y];
    }
    rs = wave_sum(rs);
    if (lane_id() == 0 && rs) atomicAdd(&s_rs, rs);
    __syncthreads();
    if (x.h == 2 && (end - beg > HX_SRC || s_rs > HX_BIG)) {
      // a heavy row: its second hop is relaxed in slices by k_hx_split
      if (threadIdx.x == 0) {
        const uint32_t slices = (end - beg + HX_SLICE - 1) / HX_SLICE;
        const unsigned long long at = atomicAdd(x.bigctr, (1ull << 32) | slices);
        x.bigu[at >> 32] = u;
        x.bigoff[at >> 32] = (uint32_t)at;
      }
      __syncthreads();
      continue;
    }
    if (x.h >= 2) {
      for (uint32_t q0 = beg; q0 < end; q0 += HX_SRC) {
        const uint32_t nb = min(HX_SRC, end - q0);
        for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
          s_y[i] = x.ci[q0 + i];
          s_k[i] = x.H[x.eid[q0 + i]];
        }
        __syncthreads();
        relax += hx_relax(x, u, nb, row, s_y, s_k, s_pre);
        __syncthreads();
      }
    }
    for (uint32_t j = 3; j <= x.h; ++j) {
      const uint32_t* src = x.P[cur] + base;
      uint32_t* dst = x.P[cur ^ 1u] + base;
      for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) dst[i] = src[i];
      __syncthreads();
      // sources: members y != u of L[j-1](u), HX_STAGE_WORDS words at a time
      const uint64_t* Lp = x.L[j - 1] + (size_t)u * x.W;
      const uint64_t* Lh = x.L[x.h] + (size_t)u * x.W;
      for (uint32_t i0 = 0; i0 < x.W; i0 += HX_STAGE_WORDS) {
        const uint32_t i = i0 + threadIdx.x;
        uint64_t bits = 0;
        if (threadIdx.x < HX_STAGE_WORDS && i < x.W) {
          bits = Lp[i];
          if (i == (u >> 6)) bits &= ~(1ull << (u & 63));
        }
        if (threadIdx.x < HX_STAGE_WORDS) s_cnt[threadIdx.x] = (uint32_t)__popcll(bits);
        __syncthreads();
        uint32_t at = 0, nb = 0;
        for (uint32_t t = 0; t < HX_STAGE_WORDS; ++t) {
          if (t == threadIdx.x) at = nb;
          nb += s_cnt[t];
        }
        if (threadIdx.x < HX_STAGE_WORDS && bits) {
          const uint64_t hw = Lh[i];
          const uint32_t rb = x.wp[(size_t)u * x.W + i];
          uint64_t b = bits;
          do {
            const uint32_t bit = (uint32_t)__ffsll((long long)b) - 1;
            const uint32_t y = i * 64 + bit;
            s_y[at] = y;
            s_k[at] = src[rb + (uint32_t)__popcll(hw & ((1ull << bit) - 1))];
            ++at;
            b &= b - 1;
          } while (b);
        }
        __syncthreads();
        if (nb) relax += hx_relax(x, u, nb, dst, s_y, s_k, s_pre);
        __syncthreads();
      }
      cur ^= 1u;
    }
    if (x.track && !x.lemma4) hx_row_mask(x, u, old, fin, len, s_mask);
  }
  if (threadIdx.x == 0 && built) {
    atomicAdd(&x.ctr[HX_CTR_ROWS], built);
    if (x.stat) {
      atomicAdd(&x.stat[HX_ST_ROWS], (unsigned long long)built);
      atomicAdd(&x.stat[HX_ST_DIRECT], direct);
      atomicAdd(&x.stat[HX_ST_RELAX], relax);
      atomicAdd(&x.stat[HX_ST_ENTRIES], entries);
    }
  }
}

// Second hop of the heavy rows k_hx_paths set aside (h = 2): one workgroup
// per slice of HX_SLICE sources; the maxima are atomic, so slices of one row
// may run in any order on any workgroups.
__global__ void __launch_bounds__(256) k_hx_split(Hx x) {
  __shared__ uint32_t s_y[HX_SLICE], s_k[HX_SLICE], s_pre[HX_SLICE + 1];
  const unsigned long long ctr = *x.bigctr;
  const uint32_t nbig = (uint32_t)(ctr >> 32), total = (uint32_t)ctr;
  unsigned long long relax = 0;
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    uint32_t lo = 0, hi = nbig;  // the last row whose slices start at or before t
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (x.bigoff[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t u = x.bigu[lo];
    const uint32_t q0 = x.rp[u] + (t - x.bigoff[lo]) * HX_SLICE;
    const uint32_t nb = min(HX_SLICE, x.rp[u + 1] - q0);
    if (threadIdx.x < nb) {
      s_y[threadIdx.x] = x.ci[q0 + threadIdx.x];
      s_k[threadIdx.x] = x.H[x.eid[q0 + threadIdx.x]];
    }
    __syncthreads();
    relax += hx_relax(x, u, nb, x.P[0] + x.boff[u], s_y, s_k, s_pre);
    __syncthreads();
  }
  if (x.stat && threadIdx.x == 0 && relax) atomicAdd(&x.stat[HX_ST_RELAX], relax);
}

// Drop masks of the heavy rows, once all their slices are done.
__global__ void __launch_bounds__(256) k_hx_split_mask(Hx x) {
  __shared__ uint32_t s_mask[2];
  const uint32_t nbig = (uint32_t)(*x.bigctr >> 32);
  for (uint32_t i = blockIdx.x; i < nbig; i += gridDim.x) {
    const uint32_t u = x.bigu[i];
    const uint64_t base = x.boff[u];
    hx_row_mask(x, u, x.Pold + base, x.P[0] + base, (uint32_t)(x.boff[u + 1] - base), s_mask);
  }
}

// f(min(P(u,w), P(v,w))) for every common member w != u, v of the two balls
// (all 64 lanes call).  Two ways, chosen per edge:
//   list:   walk the member list of the smaller ball (its keys are aligned
//           with it) and test each member in the other ball's bitset row,
//           taking that key through the rank words.  Lanes share the work
//           evenly, and consecutive edges share an endpoint whose rows stay
//           cached, so little more than the list and its keys come from HBM.
//   bitset: AND the two rows word by word, lanes on consecutive words (used
//           when both balls are large, where the rows are cheaper than lists).
// Every HX_STOP_EVERY steps, at a point all lanes reach together, stop() may
// end the scan.  Returns the algorithmic bytes this lane read, keys excluded.
constexpr uint32_t HX_STOP_EVERY = 4;
constexpr uint32_t HX_UNROLL = 2;   // list members per lane per step of the walk

template <class F, class S>
__device__ __forceinline__ unsigned long long hx_common(const Hx& x, uint32_t u, uint32_t v,
                                                        F&& f, S&& stop) {
  const uint32_t cu = x.cnt[u], cv = x.cnt[v];
  unsigned long long bytes = 0;
  uint32_t it = 0;
  if (min(cu, cv) < 2 * x.W) {
    const uint32_t a = cu <= cv ? u : v, b = cu <= cv ? v : u;  // walk a, probe b
    const uint32_t na = min(cu, cv);
    const uint32_t* Ma = x.mem + x.boff[a];
    const uint32_t* Pa = x.P[0] + x.boff[a];
    const uint32_t* Pb = x.P[0] + x.boff[b];
    const uint64_t* Lb = x.L[x.h] + (size_t)b * x.W;
    const uint32_t* Wb = x.wp + (size_t)b * x.W;
    // HX_UNROLL members per lane per step, each level of the dependent
    // chain (member, probed ball word, rank word, the two keys) issued for
    // all of them before the next: more loads in flight per wave
    for (uint32_t i0 = 0; i0 < na; i0 += HX_UNROLL * WAVE) {
      uint32_t w[HX_UNROLL], rb[HX_UNROLL], ka[HX_UNROLL], kb[HX_UNROLL];
      uint64_t word[HX_UNROLL];
      bool hit[HX_UNROLL];
#pragma unroll
      for (uint32_t q = 0; q < HX_UNROLL; ++q) {
        const uint32_t i = i0 + q * WAVE + lane_id();
        w[q] = i < na ? Ma[i] : u;
      }
#pragma unroll
      for (uint32_t q = 0; q < HX_UNROLL; ++q) {
        const bool probe = w[q] != u && w[q] != v;
        word[q] = probe ? Lb[w[q] >> 6] : 0ull;
      }
#pragma unroll
      for (uint32_t q = 0; q < HX_UNROLL; ++q) {
        const uint32_t i = i0 + q * WAVE + lane_id();
        if (i < na) bytes += 12;
        hit[q] = (word[q] >> (w[q] & 63)) & 1ull;
        rb[q] = hit[q] ? Wb[w[q] >> 6] : 0u;
        ka[q] = hit[q] ? Pa[i] : 0u;
      }
#pragma unroll
      for (uint32_t q = 0; q < HX_UNROLL; ++q) {
        rb[q] += (uint32_t)__popcll(word[q] & ((1ull << (w[q] & 63)) - 1));
        kb[q] = hit[q] ? Pb[rb[q]] : 0u;
      }
#pragma unroll
      for (uint32_t q = 0; q < HX_UNROLL; ++q)
        if (hit[q]) {
          bytes += 4;
          f(min(ka[q], kb[q]));
        }
      it += HX_UNROLL;
      if (it >= HX_STOP_EVERY) {
        it = 0;
        if (stop()) break;
      }
    }
    return bytes;
  }
  const uint64_t* Lu = x.L[x.h] + (size_t)u * x.W;
  const uint64_t* Lv = x.L[x.h] + (size_t)v * x.W;
  const uint32_t* Wu = x.wp + (size_t)u * x.W;
  const uint32_t* Wv = x.wp + (size_t)v * x.W;
  const uint32_t* Pu = x.P[0] + x.boff[u];
  const uint32_t* Pv = x.P[0] + x.boff[v];
  for (uint32_t i0 = 0; i0 < x.W; i0 += WAVE) {
    const uint32_t i = i0 + lane_id();
    if (i < x.W) {
      const uint64_t a = Lu[i], b = Lv[i];
      bytes += 16;
      uint64_t c = a & b;
      if (i == (u >> 6)) c &= ~(1ull << (u & 63));
      if (i == (v >> 6)) c &= ~(1ull << (v & 63));
      if (c) {
        bytes += 8;
        const uint32_t ra = Wu[i], rb = Wv[i];
        do {
          const uint64_t below = (c & (~c + 1)) - 1;  // bits under the lowest set bit
          f(min(Pu[ra + (uint32_t)__popcll(a & below)], Pv[rb + (uint32_t)__popcll(b & below)]));
          c &= c - 1;
        } while (c);
      }
    }
    if (++it == HX_STOP_EVERY) {
      it = 0;
      if (stop()) break;
    }
  }
  return bytes;
}

// Update the edges of chunk `chunk` (ord[cbound[chunk] .. cbound[chunk+1]))
// or, when ord is not used, every edge; one wave per edge.  The new value is the largest y <= H(e)
// with at least y common members keyed >= y: one pass counts the members
// keyed >= H(e) (enough when H(e) stands); otherwise passes with a 256-bin
// histogram narrow [lo, hi) by 256x each until one value is left.  When most
// edges are expected to change (hist1), the counting pass fills the first
// histogram as well.
__global__ void __launch_bounds__(256, 5) k_hx_edges(Hx x, uint32_t chunk, uint32_t use_ord) {
  __shared__ uint32_t s_hist[256 / WAVE][HX_BINS];
  const uint32_t lane = lane_id(), wv = threadIdx.x / WAVE, wpb = blockDim.x / WAVE;
  uint32_t* hist = s_hist[wv];
  uint32_t evals = 0, changes = 0;
  unsigned long long passes = 0, scan = 0, members = 0;  // stats mode (per lane)
  const uint32_t klo = use_ord ? x.cbound[chunk] : 0, khi = use_ord ? x.cbound[chunk + 1] : x.m;
  for (uint32_t k = klo + blockIdx.x * wpb + wv; k < khi; k += gridDim.x * wpb) {
    const uint32_t e = use_ord ? x.ord[k] : k;
    const uint32_t u = x.eu[e], v = x.ev[e];
    const uint32_t c = x.H[e];
    if (c == 0) continue;
    if (x.track && !x.first && !(((x.dmask[u] | x.dmask[v]) >> hx_bucket(c)) & 1ull)) continue;
    ++evals;
    // invariant once counted: lo is feasible, hi is not, above = members keyed >= hi
    uint32_t lo = 0, hi = c, above = 0, y = c;
    bool counted = false;
    while (true) {
      const bool histo = counted || x.hist1;
      const uint32_t s = (hi - lo + HX_BINS - 1) / HX_BINS;
      if (histo) {
        for (uint32_t k = 0; k < 4; ++k) hist[4 * lane + k] = 0;
        __threadfence_block();
      }
      uint32_t ge = 0, seen = 0;
      ++passes;
      // the counting pass may stop as soon as c members are keyed >= c
      scan += hx_common(
          x, u, v,
          [&](uint32_t val) {
            ++seen;
            if (val >= hi) ++ge;
            else if (histo && val >= lo) atomicAdd(&hist[(val - lo) / s], 1u);
          },
          [&]() { return !counted && wave_sum(ge) >= c; });
      members += seen;
      if (!counted) {
        above = wave_sum(ge);
        counted = true;
        if (above >= c) break;  // H(e) stands
        if (!histo) continue;
      }
      __threadfence_block();
      // lane l holds bins 4l .. 4l+3; bin j starts at lo + j*s
      uint32_t hk[4], tot = 0;
      for (uint32_t k = 0; k < 4; ++k) {
        hk[k] = hist[4 * lane + k];
        tot += hk[k];
      }
      uint32_t suf = tot;  // members in bins 4*lane .. 255
      for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t t = __shfl_down(suf, o, WAVE);
        if (lane + o < WAVE) suf += t;
      }
      // the highest bin whose start is feasible: count(>= start) >= start
      int best = -1;
      uint32_t best_cum = 0, best_h = 0, under = 0;
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t bnd = lo + (4 * lane + k) * s, cum = above + suf - under;
        if (bnd < hi && cum >= bnd) {
          best = (int)k;
          best_cum = cum;
          best_h = hk[k];
        }
        under += hk[k];
      }
      const uint64_t mask = __ballot(best >= 0);  // lane 0's first bin (start lo) holds
      const uint32_t bl = 63u - (uint32_t)__clzll(mask);
      const uint32_t j = 4 * bl + (uint32_t)__shfl(best, bl, WAVE);
      const uint32_t nlo = lo + j * s;
      if (s == 1) {
        y = nlo;
        break;
      }
      above = __shfl(best_cum, bl, WAVE) - __shfl(best_h, bl, WAVE);
      hi = min(nlo + s, hi);
      lo = nlo;
      __threadfence_block();
    }
    if (y == c) continue;
    if (lane == 0) {
      x.H[e] = y;
      x.touched[u] = 1;
      x.touched[v] = 1;
      atomicMin(&x.tmin[u], y);
      atomicMin(&x.tmin[v], y);
      if (x.lemma4) {
        const unsigned long long mk = hx_range_mask(y, c);
        for (uint32_t z : {u, v}) {
          if ((uint32_t)mk) atomicOr(&x.cmask[2 * z], (uint32_t)mk);
          if (mk >> 32) atomicOr(&x.cmask[2 * z + 1], (uint32_t)(mk >> 32));
        }
      }
    }
    ++changes;
  }
  if (lane == 0) {
    if (evals) atomicAdd(&x.ctr[HX_CTR_EVALS], evals);
    if (changes) atomicAdd(&x.ctr[HX_CTR_CHANGED], changes);
  }
  if (x.stat) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      scan += __shfl_xor(scan, o, WAVE);
      members += __shfl_xor(members, o, WAVE);
    }
    if (lane == 0 && evals) {
      atomicAdd(&x.stat[HX_ST_EVALS], (unsigned long long)evals);
      atomicAdd(&x.stat[HX_ST_PASSES], passes);
      atomicAdd(&x.stat[HX_ST_SCAN], scan);
      atomicAdd(&x.stat[HX_ST_MEMBERS], members);
    }
  }
}

// touched -> bitset (clearing touched) and the list of its nonzero words.
__global__ void __launch_bounds__(256) k_hx_tbits(Hx x) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < x.W; i += gridDim.x * blockDim.x) {
    uint64_t bits = 0;
    const uint32_t v0 = i * 64;
    for (uint32_t b = 0; b < 64 && v0 + b < x.n; ++b) {
      if (x.touched[v0 + b]) {
        bits |= 1ull << b;
        x.touched[v0 + b] = 0;
      }
    }
    x.tbits[i] = bits;
    if (bits) x.tlist[atomicAdd(&x.ctr[HX_CTR_TLIST], 1u)] = i;
  }
}

// dirty(x) for the next sweep: L[h-1](x) (x alone when h = 1) meets a
// touched vertex.  For h = 2 the test is sharper: a changed edge (y,w), y a
// neighbour of x, now valued b, moves a two-hop key of x only if
// H(x,y) > b, so x is dirty if it is touched itself or some neighbour y has
// tmin(y) < H(x,y).  One wave per vertex, scanning either the listed words or,
// when many are listed, the whole row.
__global__ void __launch_bounds__(256) k_hx_dirty(Hx x) {
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  const uint32_t nt = x.ctr[HX_CTR_TLIST];
  for (uint32_t r = blockIdx.x * wpb + threadIdx.x / WAVE; r < x.n; r += gridDim.x * wpb) {
    bool hit = false;
    if (x.h == 1) {
      hit = (x.tbits[r >> 6] >> (r & 63)) & 1ull;
    } else if (x.h == 2 && nt) {
      hit = (x.tbits[r >> 6] >> (r & 63)) & 1ull;
      for (uint32_t q = x.rp[r] + lane; q < x.rp[r + 1] && !hit; q += WAVE)
        hit = x.tmin[x.ci[q]] < x.H[x.eid[q]];
      hit = __ballot(hit) != 0;
    } else if (nt) {
      const uint64_t* Lr = x.L[x.h - 1] + (size_t)r * x.W;
      if ((uint64_t)nt * 8 > x.W) {
        for (uint32_t i = lane; i < x.W && !hit; i += WAVE) hit = (Lr[i] & x.tbits[i]) != 0;
      } else {
        for (uint32_t t = lane; t < nt && !hit; t += WAVE) {
          const uint32_t i = x.tlist[t];
          hit = (Lr[i] & x.tbits[i]) != 0;
        }
      }
      hit = __ballot(hit) != 0;
    }
    if (lane == 0) x.dirty[r] = hit ? 1u : 0u;
    if (x.lemma4) {
      // OR of the crossing masks over the closed (h-1)-ball of r
      const uint32_t* cm = x.cmask;
      uint32_t lo = 0, hi = 0;
      if (lane == 0) {
        lo = cm[2 * r];
        hi = cm[2 * r + 1];
      }
      if (x.h == 2) {
        for (uint32_t q = x.rp[r] + lane; q < x.rp[r + 1]; q += WAVE) {
          const uint32_t y = x.ci[q];
          lo |= cm[2 * y];
          hi |= cm[2 * y + 1];
        }
      } else if (x.h >= 3 && nt) {
        const uint64_t* Lr = x.L[x.h - 1] + (size_t)r * x.W;
        for (uint32_t t = lane; t < nt; t += WAVE) {
          const uint32_t i = x.tlist[t];
          uint64_t b = Lr[i] & x.tbits[i];
          while (b) {
            const uint32_t y = i * 64 + (uint32_t)__ffsll((long long)b) - 1;
            lo |= cm[2 * y];
            hi |= cm[2 * y + 1];
            b &= b - 1;
          }
        }
      }
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        lo |= (uint32_t)__shfl_xor(lo, o, WAVE);
        hi |= (uint32_t)__shfl_xor(hi, o, WAVE);
      }
      if (lane == 0) x.dmask[r] = (uint64_t)hi << 32 | lo;
    }
  }
}

__global__ void k_hx_finish(const uint32_t* __restrict__ H, uint32_t* __restrict__ out, uint32_t m) {
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x)
    out[e] = H[e] + 2;
}

}  // namespace hotruss
