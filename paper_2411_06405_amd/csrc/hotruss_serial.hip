// hotruss_serial.hip -- serial forms of the ball-change and support-update
// steps, used for the rare peel rounds whose work lists overflow.  They read
// the per-level event lists (or, when those overflowed too, the change-mark
// bitsets row by row) instead of the chunked work items, and they give the
// same results as the chunked kernels.  This translation unit is built at -O1:
// at -O3 the compiler's schedule of these nested data-dependent loops gave
// results that changed from run to run on gfx950, while -O1 is exact.
#include "hotruss_dev.h"

namespace hotruss {

struct RoundCtx {
  uint32_t r, k, p;
};

__device__ __forceinline__ RoundCtx round_ctx(const Ctl* c) { return RoundCtx{c->r, c->k, c->r & 1}; }


// Is w still within j hops of x in S_{r+1}?  Probe x's or w's live
// neighbourhood (the smaller) against the other's (j-1)-ball.
__device__ bool reach_serial(const Dev& d, uint32_t j, uint32_t r, uint32_t x, uint32_t w) {
  uint32_t a = x, b = w;
  if (row_end(d, a) - d.rp[a] > row_end(d, b) - d.rp[b]) { a = w; b = x; }
  const uint64_t* P = d.L[j - 1];
  if (getbit(P, d.W, a, b)) return true;
  for (uint32_t q = d.rp[a]; q < row_end(d, a); ++q)
    if (d.srem[q] > r && getbit(P, d.W, b, d.cix[q])) return true;
  return false;
}

// Per-thread drop of the directed pair (x -> w) at level j (serial form).
__device__ void drop_serial(const Dev& d, uint32_t j, const RoundCtx& rc, uint32_t x, uint32_t w) {
  const uint64_t bit = 1ull << (w & 63);
  const uint64_t old = atomicAnd(&row(d.L[j], d.W, x)[w >> 6], ~bit);
  if (!(old & bit)) return;
  atomicOr(&row(d.Dm[j], d.W, x)[w >> 6], bit);
  const uint32_t idx = atomicAdd(&d.ctl->nev[j][rc.p], 1u);
  if (idx < d.evcap) d.evl[j][rc.p][idx] = ((uint64_t)x << 32) | w;
  else d.ctl->ovf[j][rc.p] = 1;
  // follow-up work for the next level (or the support update)
  const uint32_t list = (j == d.h) ? d.h + 1 : j + 1;
  const uint32_t base = d.rp[x];
  const uint32_t deg = row_end(d, x) - base;
  const uint32_t extra = (j == d.h) ? 0 : 1;
  const uint32_t nv = deg + extra;
  const uint32_t nch = (nv + CHUNK - 1) / CHUNK;
  if (!nch) return;
  const uint32_t slot = atomicAdd(&d.ctl->nit[list], nch);
  for (uint32_t c = 0; c < nch; ++c) {
    if (slot + c >= d.itcap) { d.ctl->iovf[list] = 1; break; }
    const uint32_t vs = c * CHUNK;
    d.itl[list][slot + c] = (j == d.h)
        ? Item{x, w, base + vs, item_meta(0, 0, min(CHUNK, deg - vs), 0)}
        : Item{x, w, base, item_meta(KIND_B_SLOTS, 1, min(CHUNK, nv - vs), vs)};
  }
}

__device__ void test_serial(const Dev& d, uint32_t j, const RoundCtx& rc, uint32_t x, uint32_t w) {
  if (x == w) return;
  if (!getbit(d.L[j], d.W, min(x, w), max(x, w))) return;
  if (reach_serial(d, j, rc.r, x, w)) return;
  drop_serial(d, j, rc, x, w);
  drop_serial(d, j, rc, w, x);
}

__global__ void __launch_bounds__(256) k_level_serial(const Dev* __restrict__ dp, uint32_t j) {
  const Dev& d = *dp;
  const Ctl* c = d.ctl;
  const RoundCtx rc = round_ctx(c);
  const uint32_t nR = c->nR;
  const bool scan = c->ovf[j - 1][rc.p] != 0;
  // the level-1 events of a round are exactly both directions of every peeled edge
  const uint32_t nB = scan ? d.n : (j - 1 == 1 ? 2 * nR : min(c->nev[j - 1][rc.p], d.evcap));
  const uint32_t A = 2 * nR;
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t it = blockIdx.x * wpb + threadIdx.x / WAVE; it < A + nB; it += gridDim.x * wpb) {
    if (it < A) {
      const uint32_t e = d.R[rc.p][it >> 1];
      const uint32_t x = (it & 1) ? d.ev[e] : d.eu[e];
      const uint32_t z = (it & 1) ? d.eu[e] : d.ev[e];
      if (j == 2) {
        if (lane == 0) test_serial(d, j, rc, x, z);
        for (uint32_t q = d.rp[z] + lane; q < row_end(d, z); q += WAVE)
          if (d.srem[q] >= rc.r) test_serial(d, j, rc, x, d.cix[q]);
      } else {
        for (uint32_t i = lane; i < d.W; i += WAVE) {
          uint64_t wd = row(d.L[j - 1], d.W, z)[i] | row(d.Dm[j - 1], d.W, z)[i];
          while (wd) {
            const uint32_t b = __ffsll((unsigned long long)wd) - 1;
            wd &= wd - 1;
            test_serial(d, j, rc, x, i * 64 + b);
          }
        }
      }
    } else if (!scan) {
      const uint64_t zw = d.evl[j - 1][rc.p][it - A];
      const uint32_t z = (uint32_t)(zw >> 32), w = (uint32_t)zw;
      if (lane == 0) test_serial(d, j, rc, z, w);
      for (uint32_t q = d.rp[z] + lane; q < row_end(d, z); q += WAVE)
        if (d.srem[q] > rc.r) test_serial(d, j, rc, d.cix[q], w);
    } else {
      // row z of the change marks, one word at a time (wave-uniform loop)
      const uint32_t z = it - A;
      for (uint32_t i = 0; i < d.W; ++i) {
        uint64_t wd = row(d.Dm[j - 1], d.W, z)[i];
        while (wd) {
          const uint32_t b = __ffsll((unsigned long long)wd) - 1;
          wd &= wd - 1;
          const uint32_t w = i * 64 + b;
          if (lane == 0) test_serial(d, j, rc, z, w);
          for (uint32_t q = d.rp[z] + lane; q < row_end(d, z); q += WAVE)
            if (d.srem[q] > rc.r) test_serial(d, j, rc, d.cix[q], w);
        }
      }
    }
  }
}


// Top-level events from the event list (or the change marks): every live
// edge (a,b) that had w as a common h-neighbour loses it (same old/new rule
// as the chunked support kernel).
__global__ void __launch_bounds__(256) k_support_serial(const Dev* __restrict__ dp) {
  const Dev& d = *dp;
  const Ctl* c = d.ctl;
  const RoundCtx rc = round_ctx(c);
  const uint32_t h = d.h;
  const bool scan = c->ovf[h][rc.p] != 0;
  const uint32_t ne = scan ? d.n : (h == 1 ? 2 * c->nR : min(c->nev[h][rc.p], d.evcap));
  uint32_t* Rn = d.R[rc.p ^ 1];
  const uint32_t lane = lane_id(), wpb = blockDim.x / WAVE;
  for (uint32_t it = blockIdx.x * wpb + threadIdx.x / WAVE; it < ne; it += gridDim.x * wpb) {
    const uint32_t a0 = scan ? it : (uint32_t)(d.evl[h][rc.p][it] >> 32);
    const uint32_t wcount = scan ? d.W : 1;
    for (uint32_t i = 0; i < wcount; ++i) {
      uint64_t wd = scan ? row(d.Dm[h], d.W, a0)[i] : 1ull;
      while (wd) {
        const uint32_t bpos = __ffsll((unsigned long long)wd) - 1;
        wd &= wd - 1;
        const uint32_t a = a0;
        const uint32_t w = scan ? i * 64 + bpos : (uint32_t)d.evl[h][rc.p][it];
        const uint64_t* Lw = row(d.L[h], d.W, w);
        const uint64_t* Dw = row(d.Dm[h], d.W, w);
        for (uint32_t q = d.rp[a] + lane; q < row_end(d, a); q += WAVE) {
          if (d.srem[q] <= rc.r) continue;
          const uint32_t bb = d.cix[q];
          uint64_t word = Lw[bb >> 6];
          if (a < bb) word |= Dw[bb >> 6];
          if (!((word >> (bb & 63)) & 1ull)) continue;
          const uint32_t e = d.eid[q];
          if (atomicSub(&d.sup[e], 1u) == rc.k - 1) Rn[atomicAdd(&d.ctl->nPush, 1u)] = e;
        }
      }
    }
  }
}

}  // namespace hotruss
