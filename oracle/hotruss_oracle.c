/*
 * hotruss_oracle.c -- plain CPU oracle for higher-order (k,h)-truss
 * decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library; it reads the same
 * CSR input layout and writes the same canonical edge order, nothing more.
 *
 * Definitions followed (paper, Section 2):
 *   N_S(x,h)      vertices y != x with dist_S(x,y) <= h, distances measured
 *                 with the edges of the current edge set S only;
 *   sup_S(e,h)    |N_S(u,h) intersect N_S(v,h)| for e = (u,v)   (Def. 3);
 *   (k,h)-truss   the maximal S with sup_S(e,h) >= k-2 for all e in S (Def. 4);
 *   t(e,h)        the largest k whose (k,h)-truss contains e.
 *
 * Readings taken where the paper is silent (listed in the design notes):
 *   - N_S(x,h) excludes x itself, so neither endpoint of e is ever counted
 *     (at h = 1 this is the triangle support of Section 2);
 *   - paths may run through either endpoint and through e itself;
 *   - S is an edge subset (peeling removes single edges), not induced.
 *
 * Peeling (Section 3, Algorithm 1), bulk-synchronous form: every round
 * recomputes sup_S for every live edge from scratch with a fresh bounded BFS,
 * removes at once every live edge with sup <= k-2, giving them t = k, and
 * when no edge qualifies raises k to min sup + 2 (Algorithm 1 skipping empty
 * bins).  Removing all qualifying edges together gives the same t as the
 * one-at-a-time order of Algorithm 1, because removals only lower supports
 * (Lemma 1 and monotonicity of sup in S).  The round index rho(e) counts only
 * rounds that removed at least one edge, from 0.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC hotruss_oracle.c -o libhotruss_oracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_CSR (-2)
#define OR_ERR_MEM (-3)
#define OR_CERT_FAIL (-10)

typedef struct {
    uint32_t n;
    uint64_t m;
    const uint32_t *rp;   /* row_ptr [n+1] */
    const uint32_t *ci;   /* col_idx [2m]  */
    uint32_t *slot_eid;   /* CSR slot -> canonical edge id */
    uint32_t *eu, *ev;    /* endpoints of edge id, eu < ev */
} og_t;

/* Canonical edge ids: rank of (x,y), y > x, in row-major upper-triangle order;
 * the lower slot (y,x) finds its partner by binary search in row y. */
static int og_build(og_t *g, uint32_t n, const uint32_t *rp, const uint32_t *ci)
{
    memset(g, 0, sizeof *g);
    g->n = n; g->rp = rp; g->ci = ci;
    uint64_t nnz = rp[n];
    if (nnz % 2) return OR_ERR_CSR;
    g->m = nnz / 2;
    g->slot_eid = (uint32_t *)malloc((nnz ? nnz : 1) * sizeof(uint32_t));
    g->eu = (uint32_t *)malloc((g->m ? g->m : 1) * sizeof(uint32_t));
    g->ev = (uint32_t *)malloc((g->m ? g->m : 1) * sizeof(uint32_t));
    if (!g->slot_eid || !g->eu || !g->ev) return OR_ERR_MEM;
    uint64_t next = 0;
    for (uint32_t x = 0; x < n; ++x) {
        for (uint64_t j = rp[x]; j < rp[x + 1]; ++j) {
            uint32_t y = ci[j];
            if (y >= n || y == x) return OR_ERR_CSR;
            if (j > rp[x] && ci[j - 1] >= y) return OR_ERR_CSR;
            if (y > x) {
                if (next >= g->m) return OR_ERR_CSR;
                g->slot_eid[j] = (uint32_t)next;
                g->eu[next] = x; g->ev[next] = y;
                ++next;
            }
        }
    }
    if (next != g->m) return OR_ERR_CSR;
    for (uint32_t x = 0; x < n; ++x) {
        for (uint64_t j = rp[x]; j < rp[x + 1]; ++j) {
            uint32_t y = ci[j];
            if (y > x) continue;
            uint64_t lo = rp[y], hi = rp[y + 1];
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                if (ci[mid] < x) lo = mid + 1; else hi = mid;
            }
            if (lo == rp[y + 1] || ci[lo] != x) return OR_ERR_CSR; /* not symmetric */
            g->slot_eid[j] = g->slot_eid[lo];
        }
    }
    return OR_OK;
}

static void og_free(og_t *g)
{
    free(g->slot_eid); free(g->eu); free(g->ev);
}

/* Per-thread BFS scratch: stamp arrays avoid clearing between searches. */
typedef struct {
    uint32_t *seen;    /* BFS visited stamp */
    uint32_t *dist;
    uint32_t *inball;  /* stamp: vertex belongs to N_S(src,h) of the first endpoint */
    uint32_t *queue;
    uint32_t stamp;
} bfs_ws;

static int ws_init(bfs_ws *w, uint32_t n)
{
    size_t b = (size_t)(n ? n : 1) * sizeof(uint32_t);
    w->seen = (uint32_t *)calloc(1, b);
    w->dist = (uint32_t *)calloc(1, b);
    w->inball = (uint32_t *)calloc(1, b);
    w->queue = (uint32_t *)malloc(b);
    w->stamp = 0;
    return (w->seen && w->dist && w->inball && w->queue) ? OR_OK : OR_ERR_MEM;
}

static void ws_free(bfs_ws *w)
{
    free(w->seen); free(w->dist); free(w->inball); free(w->queue);
}

/* Edge filter: edge f is in S iff key[f] >= thr (key == NULL: every edge). */
typedef struct { const uint32_t *key; uint32_t thr; } filt_t;

static inline int in_S(const filt_t *f, uint32_t e)
{
    return f->key == NULL || f->key[e] >= f->thr;
}

/* Bounded BFS from src to depth h in S.  Calls visit(w) for every w in
 * N_S(src,h), i.e. every vertex other than src at distance 1..h (Section 2,
 * h-hop neighbours).  Implemented as a macro-free two-mode routine: mode 0
 * stamps inball[w], mode 1 counts w with inball[w] == mark and w != skip. */
static uint64_t bounded_bfs(const og_t *g, const filt_t *f, uint32_t src, uint32_t h,
                            bfs_ws *w, int mode, uint32_t mark, uint32_t skip)
{
    uint32_t s = ++w->stamp;
    if (s == 0) { /* stamp wrap: clear and restart */
        memset(w->seen, 0, (size_t)g->n * sizeof(uint32_t));
        s = w->stamp = 1;
    }
    uint64_t head = 0, tail = 0, count = 0;
    w->seen[src] = s; w->dist[src] = 0; w->queue[tail++] = src;
    while (head < tail) {
        uint32_t x = w->queue[head++];
        if (w->dist[x] == h) continue;
        for (uint64_t j = g->rp[x]; j < g->rp[x + 1]; ++j) {
            if (!in_S(f, g->slot_eid[j])) continue;
            uint32_t y = g->ci[j];
            if (w->seen[y] == s) continue;
            w->seen[y] = s; w->dist[y] = w->dist[x] + 1; w->queue[tail++] = y;
            if (mode == 0) w->inball[y] = mark;
            else if (w->inball[y] == mark && y != skip) ++count;
        }
    }
    return count;
}

/* sup_S(e,h) = |N_S(u,h) intersect N_S(v,h)| (Def. 3), from two fresh BFS. */
static uint64_t h_support(const og_t *g, const filt_t *f, uint32_t e, uint32_t h,
                          bfs_ws *w, uint32_t *mark_ctr)
{
    uint32_t u = g->eu[e], v = g->ev[e];
    uint32_t mark = ++(*mark_ctr);
    if (mark == 0) {
        memset(w->inball, 0, (size_t)g->n * sizeof(uint32_t));
        mark = *mark_ctr = 1;
    }
    bounded_bfs(g, f, u, h, w, 0, mark, 0);
    /* count w in N_S(v,h) that were marked as members of N_S(u,h); u itself
     * was never marked (the BFS does not mark its source), so skip only
     * needs to exclude nothing further: pass u anyway for clarity. */
    return bounded_bfs(g, f, v, h, w, 1, mark, u);
}

static int nthreads_or_default(int threads)
{
    return threads > 0 ? threads : omp_get_max_threads();
}

/* ---------------------------------------------------------------------------
 * Public entry points (C ABI, host pointers; caller owns every buffer).
 * ------------------------------------------------------------------------- */

uint64_t oracle_num_edges(uint32_t n, const uint32_t *row_ptr)
{
    return row_ptr[n] / 2;
}

/* sup_S(e,h) for every edge e (Def. 3).  S = { f : key[f] >= thr }, or all
 * edges when key is NULL.  Edges outside S get sup 0. */
int oracle_h_support(uint32_t n, const uint32_t *row_ptr, const uint32_t *col_idx,
                     uint32_t h, const uint32_t *key, uint32_t thr,
                     uint32_t *sup_out, int threads)
{
    if (!row_ptr || !col_idx || !sup_out || h == 0) return OR_ERR_ARG;
    og_t g;
    int rc = og_build(&g, n, row_ptr, col_idx);
    if (rc) { og_free(&g); return rc; }
    filt_t f = { key, thr };
    int nt = nthreads_or_default(threads);
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        bfs_ws w; uint32_t mk = 0;
        if (ws_init(&w, n)) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t e = 0; e < (int64_t)g.m; ++e)
                sup_out[e] = in_S(&f, (uint32_t)e)
                           ? (uint32_t)h_support(&g, &f, (uint32_t)e, h, &w, &mk) : 0u;
        }
        ws_free(&w);
    }
    og_free(&g);
    return err ? OR_ERR_MEM : OR_OK;
}

/* sup_S(e,h) for the listed edges only (same evaluation as above), for
 * graphs too large to evaluate every edge: sup_out[i] = sup_S(edges[i],h). */
int oracle_h_support_edges(uint32_t n, const uint32_t *row_ptr, const uint32_t *col_idx,
                           uint32_t h, const uint32_t *key, uint32_t thr,
                           const uint32_t *edges, uint64_t num_edges,
                           uint32_t *sup_out, int threads)
{
    if (!row_ptr || !col_idx || !edges || !sup_out || h == 0) return OR_ERR_ARG;
    og_t g;
    int rc = og_build(&g, n, row_ptr, col_idx);
    if (rc) { og_free(&g); return rc; }
    filt_t f = { key, thr };
    int nt = nthreads_or_default(threads);
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        bfs_ws w; uint32_t mk = 0;
        if (ws_init(&w, n)) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t i = 0; i < (int64_t)num_edges; ++i) {
                uint32_t e = edges[i];
                if (e >= g.m) {
#pragma omp atomic write
                    err = 2;
                    continue;
                }
                sup_out[i] = in_S(&f, e) ? (uint32_t)h_support(&g, &f, e, h, &w, &mk) : 0u;
            }
        }
        ws_free(&w);
    }
    og_free(&g);
    return err == 1 ? OR_ERR_MEM : (err == 2 ? OR_ERR_ARG : OR_OK);
}

/* Peeling decomposition (Algorithm 1, bulk-synchronous rounds).
 *
 * t_out[m]   h-trussness of every edge (always >= 2);
 * rho_out[m] round in which the edge was removed (may be NULL);
 * round_k[cap], round_size[cap]  level k_r and |R_r| per round (may be NULL);
 * stats[4]   {rounds, levels visited, support evaluations, cap overflow}.
 */
int oracle_decompose(uint32_t n, const uint32_t *row_ptr, const uint32_t *col_idx,
                     uint32_t h, uint32_t *t_out, uint32_t *rho_out,
                     uint32_t *round_k, uint32_t *round_size, uint64_t round_cap,
                     uint64_t *stats, int threads)
{
    if (!row_ptr || !col_idx || !t_out || h == 0) return OR_ERR_ARG;
    og_t g;
    int rc = og_build(&g, n, row_ptr, col_idx);
    if (rc) { og_free(&g); return rc; }
    const uint64_t m = g.m;
    /* key[e] = 1 while e is in S, 0 once peeled: S = { f : key[f] >= 1 } */
    uint32_t *key = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *sup = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *R = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!key || !sup || !R) { free(key); free(sup); free(R); og_free(&g); return OR_ERR_MEM; }
    for (uint64_t e = 0; e < m; ++e) { key[e] = 1; t_out[e] = 0; if (rho_out) rho_out[e] = 0; }
    filt_t f = { key, 1 };
    int nt = nthreads_or_default(threads);
    uint64_t live = m, r = 0, levels = 1, evals = 0, overflow = 0;
    uint32_t k = 2;
    int err = 0;
#pragma omp parallel num_threads(nt)
    {
        bfs_ws w; uint32_t mk = 0;
        int bad = ws_init(&w, n);
        if (bad) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp barrier
        while (!err && live > 0) {
            /* every live edge: fresh h-support in the current S */
#pragma omp for schedule(dynamic, 16)
            for (int64_t e = 0; e < (int64_t)m; ++e)
                if (key[e]) sup[e] = (uint32_t)h_support(&g, &f, (uint32_t)e, h, &w, &mk);
#pragma omp single
            {
                evals += live;
                uint64_t nr = 0;
                uint32_t mn = UINT32_MAX;
                for (uint64_t e = 0; e < m; ++e) {
                    if (!key[e]) continue;
                    if (sup[e] < mn) mn = sup[e];
                    if ((uint64_t)sup[e] + 2 <= k) R[nr++] = (uint32_t)e;
                }
                if (nr == 0) {
                    /* empty bin: jump to the next non-empty level */
                    k = mn + 2;
                    ++levels;
                    for (uint64_t e = 0; e < m; ++e)
                        if (key[e] && (uint64_t)sup[e] + 2 <= k) R[nr++] = (uint32_t)e;
                }
                for (uint64_t i = 0; i < nr; ++i) {
                    uint32_t e = R[i];
                    t_out[e] = k;
                    if (rho_out) rho_out[e] = (uint32_t)r;
                    key[e] = 0;
                }
                if (r < round_cap) {
                    if (round_k) round_k[r] = k;
                    if (round_size) round_size[r] = (uint32_t)nr;
                } else {
                    overflow = 1;
                }
                live -= nr;
                ++r;
            }
        }
        ws_free(&w);
    }
    if (stats) { stats[0] = r; stats[1] = levels; stats[2] = evals; stats[3] = overflow; }
    free(key); free(sup); free(R); og_free(&g);
    return err ? OR_ERR_MEM : OR_OK;
}

/* Exactness certificate for a claimed (t, rho):
 *  C0  every edge has t >= 2; the rounds 0..R-1 are all non-empty; all edges
 *      of round r share one level k_r, and k_r never decreases with r;
 *  C1  e removed in round r has sup_{S_r}(e,h) <= k_r - 2,
 *      S_r = { f : rho(f) >= r };
 *  C2  e has sup_{S^t}(e,h) >= t(e) - 2, S^t = { f : t(f) >= t(e) }.
 * C2 makes every S^k a (k,h)-valid set (so t is not too high); C0 and C1,
 * with containment (Lemma 1), keep the (k_r+1,h)-truss inside S_r round by
 * round (so t is not too low).  C0 is checked on all edges; C1 and C2 on the
 * listed sample (all edges when sample is NULL).
 * fail[3] = {check (0,1,2), edge id, observed support} on failure. */
int oracle_certify(uint32_t n, const uint32_t *row_ptr, const uint32_t *col_idx,
                   uint32_t h, const uint32_t *t, const uint32_t *rho,
                   const uint32_t *sample, uint64_t num_sample,
                   uint64_t *fail, int threads)
{
    if (!row_ptr || !col_idx || !t || !rho || h == 0) return OR_ERR_ARG;
    og_t g;
    int rc = og_build(&g, n, row_ptr, col_idx);
    if (rc) { og_free(&g); return rc; }
    const uint64_t m = g.m;
    if (fail) { fail[0] = fail[1] = fail[2] = UINT64_MAX; }
    /* C0 */
    uint32_t R = 0;
    for (uint64_t e = 0; e < m; ++e) if (rho[e] + 1 > R) R = rho[e] + 1;
    uint32_t *kr = (uint32_t *)calloc(R ? R : 1, sizeof(uint32_t));
    /* rho and t, reversed so that S_r and S^t are "key >= threshold" sets */
    uint32_t *rkey = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!kr || !rkey) { free(kr); free(rkey); og_free(&g); return OR_ERR_MEM; }
    int bad = 0;
    for (uint64_t e = 0; e < m && !bad; ++e) {
        if (t[e] < 2) { bad = 1; if (fail) { fail[0] = 0; fail[1] = e; fail[2] = t[e]; } break; }
        if (kr[rho[e]] == 0) kr[rho[e]] = t[e];
        else if (kr[rho[e]] != t[e]) { bad = 1; if (fail) { fail[0] = 0; fail[1] = e; fail[2] = t[e]; } }
        rkey[e] = rho[e];
    }
    for (uint32_t r = 0; r < R && !bad; ++r) {
        if (kr[r] == 0 || (r > 0 && kr[r] < kr[r - 1])) {
            bad = 1; if (fail) { fail[0] = 0; fail[1] = UINT64_MAX; fail[2] = r; }
        }
    }
    if (bad) { free(kr); free(rkey); og_free(&g); return OR_CERT_FAIL; }
    uint64_t ns = sample ? num_sample : m;
    int nt = nthreads_or_default(threads);
    int err = 0;
    volatile int failed = 0;
#pragma omp parallel num_threads(nt)
    {
        bfs_ws w; uint32_t mk = 0;
        if (ws_init(&w, n)) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 8)
            for (int64_t i = 0; i < (int64_t)ns; ++i) {
                if (failed) continue;
                uint32_t e = sample ? sample[i] : (uint32_t)i;
                if (e >= m) {
#pragma omp critical
                    { failed = 1; err = 2; }
                    continue;
                }
                filt_t f1 = { rkey, rho[e] };       /* S_r */
                uint64_t s1 = h_support(&g, &f1, e, h, &w, &mk);
                filt_t f2 = { t, t[e] };            /* S^t(e) */
                uint64_t s2 = h_support(&g, &f2, e, h, &w, &mk);
                int c1 = (s1 + 2 > t[e]);
                int c2 = (s2 + 2 < t[e]);
                if (c1 || c2) {
#pragma omp critical
                    {
                        if (!failed && fail) {
                            fail[0] = c1 ? 1 : 2; fail[1] = e; fail[2] = c1 ? s1 : s2;
                        }
                        failed = 1;
                    }
                }
            }
        }
        ws_free(&w);
    }
    free(kr); free(rkey); og_free(&g);
    if (err == 1) return OR_ERR_MEM;
    if (err == 2) return OR_ERR_ARG;
    return failed ? OR_CERT_FAIL : OR_OK;
}
