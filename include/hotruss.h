/*
 * hotruss.h -- C ABI of libhotruss, higher-order (k,h)-truss decomposition on
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (paper, Section 2, problem statement): given an undirected simple
 * graph G = (V, E) and a hop threshold h >= 1, compute the h-trussness
 * t(e,h) of every edge, the largest k such that the (k,h)-truss contains e.
 *   N_S(x,h)    vertices other than x within h hops of x, hops counted over
 *               the edges of the current edge set S;
 *   sup_S(e,h)  |N_S(u,h) intersect N_S(v,h)| for e = (u,v)        (Def. 3);
 *   (k,h)-truss the maximal S with sup_S(e,h) >= k-2 on all of S   (Def. 4).
 * Neither endpoint of e is ever one of its common h-neighbours; paths may pass
 * through either endpoint; S is an edge subset.
 *
 * Conventions shared by every entry point:
 *   Graph     symmetric CSR: row_ptr[n+1] and col_idx[2m] (uint32), both
 *             directions of each edge stored, rows strictly ascending, no
 *             self-loops, no duplicates; isolated vertices allowed.
 *   m         number of undirected edges = row_ptr[n] / 2, below 2^31.
 *   Edge ids  canonical upper-triangle order: for x = 0..n-1 ascending, each
 *             neighbour y > x ascending; edge (x,y) has the rank of that pair.
 *             Every per-edge output is laid out in this order.
 *   Memory    unless a comment says "host", pointers are DEVICE pointers on
 *             the current HIP device, owned by the caller; the library never
 *             allocates device memory, it carves everything from the caller's
 *             workspace and keeps no pointer after the call returns (sessions
 *             excepted, see below; hoTrussDecomposeNoAlloc uses a fixed device
 *             array inside the library instead of a workspace).
 *   Streams   work is enqueued on `stream`.  Calls return after the work has
 *             completed on that stream unless stated otherwise (hoSubmit is
 *             host-only).  This is deliberate: the number of peel rounds is
 *             decided on the device as the rounds run (Algorithm 1 stops when
 *             S is empty), so the host keeps replaying captured round graphs
 *             until the device reports that the decomposition has finished,
 *             and it can only stop once it has seen that report.  Callers that
 *             need asynchrony use a session (hoSubmit / hoSessionProgress /
 *             hoPoll) or a host thread per stream.
 *   Sizes     n <= 524,288 for every entry point that keeps h-hop balls
 *             (hoTrussHSupport, hoTrussDecompose and its batched and session
 *             forms, hoTrussHIndex): a ball is a bitset row of ceil(n/64)
 *             64-bit words, rounded up to a multiple of 8, and each row is
 *             built in the 64 KiB of LDS one workgroup may use, so at most
 *             8,192 words.  Larger n gives HO_ERR_INVALID_ARG (and a
 *             workspace query of 0).  The ball store itself is about
 *             (2h-1) * n^2 / 8 bytes (h = 2, n = 524,288: 103 GB).
 *   Errors    argument errors return at once, before any device work.  The
 *             CSR is always validated on the device (row_ptr monotone and
 *             row_ptr[n] == 2m, ids < n, rows strictly ascending, no loops,
 *             symmetric); a malformed CSR returns HO_ERR_BAD_CSR and leaves
 *             the outputs unspecified.  m == 0 returns HO_OK with no work.
 */
#ifndef HOTRUSS_H
#define HOTRUSS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HO_OK = 0,
    HO_ERR_INVALID_ARG = -1, /* NULL pointer, h == 0, m too large, ...        */
    HO_ERR_BAD_CSR = -2,     /* device-side CSR validation failed             */
    HO_ERR_WORKSPACE = -3,   /* workspace smaller than the query returned     */
    HO_ERR_HIP = -4,         /* a HIP runtime call failed                     */
    HO_ERR_BUDGET = -5,      /* session: request does not fit the pool now    */
    HO_ERR_CANCELLED = -6,   /* session: ticket was cancelled                 */
    HO_ERR_BUSY = -7,        /* session: no free slot                         */
    HO_ERR_NOT_FOUND = -8,   /* session: unknown ticket                       */
    HO_ERR_INTERNAL = -9     /* an internal invariant failed (a bug)          */
} hoStatus;

/* Optional knobs; pass NULL for defaults.  Every setting gives the same
 * results; they only change speed and workspace size.  The first three tune
 * the initial pass (edge ids, ball build, initial h-support); the autotuner
 * in the Python package picks them per graph shape by measurement. */
typedef struct {
    uint32_t word_bits;       /* initial h-support: bitset load width per lane, 64 or 128
                                 (0 = 64)                                                 */
    uint32_t dense_threshold; /* level-2 ball build: a row is built bottom-up (OR of the
                                 neighbours' level-1 rows, dense frontier) instead of
                                 top-down (scatter of their adjacency lists, sparse
                                 frontier) when those lists hold more than
                                 dense_threshold/16 entries per bitset word the bottom-up
                                 build reads, i.e. (deg(x)+1)*W words; 0 = 32            */
    uint32_t edges_per_wave;  /* initial h-support: edges sharing one wavefront, 1..16
                                 (0 = by row width)                                      */
    uint32_t flags;           /* HO_FLAG_*                                               */
    uint32_t event_capacity;  /* per-level ball-change event list entries; a round that
                                 overflows it re-creates the next step's work from the
                                 change-mark bitsets (0 = auto)                          */
    uint32_t grid_blocks;     /* workgroups of the round driver (0 = auto)               */
    uint32_t item_capacity;   /* per-level work item list entries; a round that overflows
                                 it re-runs that step in windows that fit (0 = auto)      */
} hoTuning;

#define HO_FLAG_HOST_LOOP 0x1u  /* drive peel rounds from the host, one round per
                                   launch sequence (debugging; slower)                */
#define HO_FLAG_STATS 0x2u      /* time every kernel with HIP events (implies host loop) */
#define HO_FLAG_SERIAL_LEVELS 0x4u   /* testing: run every ball-change step the way a round
                                        whose work list overflowed runs it (work items
                                        re-created from their sources in windows, host-driven) */
#define HO_FLAG_SERIAL_SUPPORT 0x8u  /* testing: the same for the support update step       */
#define HO_FLAG_COMPACT_EACH 0x10u   /* testing: compact the adjacency rows at every chance  */

/* Work counters of the last decomposition on this host thread. */
typedef struct {
    uint64_t rounds;        /* peel rounds that removed at least one edge          */
    uint64_t levels;        /* distinct levels k visited (level jumps)             */
    uint64_t events;        /* ball-change events at the top level h               */
    uint64_t overflows;     /* rounds in which a list overflowed (windowed re-run)    */
    uint64_t compactions;   /* adjacency compactions (live slots moved to the row fronts) */
    double   device_ms;     /* device time of the whole call (HIP events)          */
    /* HO_FLAG_STATS only: summed HIP-event time and launch count per kernel kind:
     * 0 initial h-support, 1 unused (the level-jump minimum is computed by the
     * end-of-round kernel), 2 peel/mark, 3 ball-change events (all levels),
     * 4 support update, 5 end of round with the next round's level-jump
     * minimum.  Stats mode drives the rounds from the host, so device_ms is
     * then not the production time. */
    double   kernel_ms[6];
    uint64_t kernel_launches[6];
    /* HO_FLAG_STATS only: work done by the chunked kernels.  Ball-change
     * events: [0] work items, [1] candidate slots examined, [2] candidate pairs
     * tested, [3] witness probes, [4] pairs dropped (directed events).  Support
     * update: [5] work items, [6] adjacency slots, [7] common h-neighbours lost.
     * Witness tests done on bitset rows count one probe per word pair. */
    uint64_t work[8];
    /* HO_FLAG_STATS only (0 otherwise, and 0 if an event list overflowed):
     * the method-level work of the same round schedule done the re-evaluating
     * way (Section 3): evaluations = m + the live edges, summed over rounds,
     * that have an endpoint whose h-ball changed in the round; alg_bytes = per
     * evaluation (u,v) s(u) + s(v) + 4 with s(x) = min(4|N(x,h)|, ceil(n/8)),
     * plus per ball build min(frontier reads of a bounded BFS to depth h-1 at
     * 8 + 4 deg per vertex reached, h full scans 4(n+1) + 8|S| + ceil(n/8)),
     * builds being every non-isolated vertex at the start and, in each round,
     * the vertices within h-1 hops (before the round) of a removed edge's
     * endpoint.  A round that removes every remaining edge counts nothing. */
    uint64_t evaluations;
    uint64_t alg_bytes;
    /* Ball-change events per level j = 1..h (index j-1): pairs {x, w}, counted
     * once per direction, that left the j-hop ball in some round; level 1
     * counts both directions of every removed edge.  The round that removes
     * every remaining edge updates no ball above level 1, so for j >= 2 this
     * is sum_x |N_G(x,j)| - sum_x |N_S(x,j)|, S the edges of that last round. */
    uint64_t level_events[16];
} hoStats;

/* Bytes of device workspace hoTrussDecompose / hoTrussHSupport need for a
 * graph with n vertices, m undirected edges and hop threshold h.  Dominated by
 * 2h bitset arrays of n x ceil(n/64) words (the h-hop balls at every level and
 * the per-round change marks).  Returns 0 on invalid arguments. */
size_t hoTrussWorkspaceBytes(uint32_t n, uint64_t m, uint32_t h, const hoTuning *tune);

/* h-support of every edge in the whole graph, sup_G(e,h) (Def. 3).
 * out_support[m] (device, uint32) receives the counts in edge-id order. */
hoStatus hoTrussHSupport(const uint32_t *row_ptr, const uint32_t *col_idx,
                         uint32_t n, uint64_t m, uint32_t h,
                         uint32_t *out_support,
                         void *workspace, size_t workspace_bytes,
                         const hoTuning *tune, hipStream_t stream);

/* Full decomposition (Section 3, the peeling method): t(e,h) of every edge.
 * out_trussness[m] (device, uint32) receives t(e,h) >= 2.
 * out_round[m] (device, uint32, may be NULL) receives the 0-based peel round
 * of each edge under the bulk schedule: round r removes at once every live
 * edge with sup <= k-2 at the current level k; rounds that remove nothing
 * are not counted; k rises to min sup + 2 when nothing qualifies. */
hoStatus hoTrussDecompose(const uint32_t *row_ptr, const uint32_t *col_idx,
                          uint32_t n, uint64_t m, uint32_t h,
                          uint32_t *out_trussness, uint32_t *out_round,
                          void *workspace, size_t workspace_bytes,
                          const hoTuning *tune, hipStream_t stream);

/* hoTrussDecompose for callers that cannot allocate memory (serving loops
 * and harnesses that forbid allocation): the same computation and outputs,
 * with no workspace argument and no allocation of any kind (no device or
 * pinned host memory, no events, no graphs).  The workspace, slot descriptor
 * and status words live in a fixed 256 MiB device array inside the library
 * (one per GPU, held until the process ends); a graph whose workspace does
 * not fit it returns HO_ERR_WORKSPACE before any device work (h = 2 fits up
 * to about n = 20,000 with m = 10^5).  Rounds are driven from the host, one
 * synchronisation per step, so it is slower per round than hoTrussDecompose.
 * Inputs and outputs as for hoTrussDecompose (device pointers); returns after
 * the work has completed on `stream`.  The array keeps the last call's
 * contents; each call initialises what it reads.  Calls on one GPU share
 * the array: the library serialises calls made from this process, and the
 * caller must not let two processes' calls, or a call and a stream still
 * running an earlier call's work, overlap on one GPU.  hoTrussLastStats
 * reports its counters (device_ms 0). */
hoStatus hoTrussDecomposeNoAlloc(const uint32_t *row_ptr, const uint32_t *col_idx,
                                 uint32_t n, uint64_t m, uint32_t h,
                                 uint32_t *out_trussness, uint32_t *out_round,
                                 hipStream_t stream);

/* Counters of the last hoTrussDecompose on this host thread (host pointer). */
hoStatus hoTrussLastStats(hoStats *out);

/* Many independent graphs in one call (batched decomposition: the same
 * per-graph computation as hoTrussDecompose, graphs sharing the GPU).
 * row_ptr_cat holds graph g's local (n_g+1)-entry row_ptr at offset
 * vtx_off[g] + g; col_idx_cat holds its local ids at offset adj_off[g]; its
 * outputs start at edge_off[g] of out_trussness_cat / out_round_cat (the
 * latter may be NULL).  vtx_off, adj_off and edge_off are HOST arrays of B+1
 * entries (prefix sums of n_g, 2m_g and m_g); h is a HOST array of B hop
 * thresholds (each 1..16 after clamping at n_g - 1).  Results are identical to
 * B separate hoTrussDecompose calls (components never interact).
 *
 * Execution: graphs are admitted largest workspace first into up to 256
 * concurrent slots carved from the workspace; one replay of a captured step
 * graph advances every active slot by one of its own peel rounds, and finished
 * slots are refilled between replays.  Any workspace at least as large as the
 * largest single graph's share works; more lets more graphs run together.
 * hoTrussBatchedWorkspaceBytes returns the size that lets the 64 largest
 * graphs run at once (or all of them, if smaller); 0 on invalid arguments.
 * A graph that cannot fit the workspace at all returns HO_ERR_WORKSPACE; a
 * malformed CSR in any graph returns HO_ERR_BAD_CSR (the other graphs'
 * outputs are still written).  tune->grid_blocks, if set, is the total
 * workgroup count shared by the slots. */
size_t hoTrussBatchedWorkspaceBytes(const uint64_t *vtx_off, const uint64_t *edge_off,
                                    const uint32_t *h, uint32_t B, const hoTuning *tune);
hoStatus hoTrussDecomposeBatched(const uint32_t *row_ptr_cat, const uint32_t *col_idx_cat,
                                 const uint64_t *vtx_off, const uint64_t *adj_off,
                                 const uint64_t *edge_off, const uint32_t *h, uint32_t B,
                                 uint32_t *out_trussness_cat, uint32_t *out_round_cat,
                                 void *workspace, size_t workspace_bytes,
                                 const hoTuning *tune, hipStream_t stream);

/* Sessions: continuous batching of decomposition requests that arrive over
 * time (a serving loop).  A session owns a caller-provided device memory pool
 * and up to max_slots concurrent decompositions, all on one stream.
 *
 *   hoSessionCreate   pool (device, pool_bytes) and stream are borrowed until
 *                     hoSessionDestroy; max_h (1..16) bounds the requests' h.
 *                     Writes the session handle to *out (host).
 *   hoSubmit          queues one graph (same CSR conventions and outputs as
 *                     hoTrussDecompose); CSR and output buffers must stay valid
 *                     until the ticket is done.  Host-only: no device work.
 *                     HO_ERR_BUDGET if the graph's share can never fit the
 *                     pool; HO_ERR_INVALID_ARG if h exceeds max_h.  Writes a
 *                     ticket (host).  An empty graph (m == 0) is done at once.
 *   hoSessionProgress admits queued requests first-come first-served while a
 *                     slot and pool memory are free (a request too large for
 *                     the memory free now waits, and later smaller ones may
 *                     pass it), then replays the step graph up to
 *                     max_graph_launches times (0: until nothing is queued or
 *                     running), retiring finished requests.  Blocks on
 *                     `stream`.  Reports active and queued counts (host, may
 *                     be NULL).
 *   hoPoll            *done (host) = 1 once the ticket's outputs are final;
 *                     returns that request's status (HO_ERR_BAD_CSR for a
 *                     malformed graph, HO_ERR_CANCELLED if cancelled).
 *   hoCancel          removes a request that is still queued; HO_ERR_BUSY if
 *                     it already started or finished.
 *   hoSessionDestroy  waits for the stream and frees the host-side state; the
 *                     pool is the caller's to free.
 * Calls on one session may come from several host threads: each takes the
 * session's lock, so they serialize. */
typedef struct hoSession hoSession;
hoStatus hoSessionCreate(void *pool, size_t pool_bytes, uint32_t max_slots, uint32_t max_h,
                         hipStream_t stream, hoSession **out);
hoStatus hoSubmit(hoSession *s, const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                  uint64_t m, uint32_t h, uint32_t *out_trussness, uint32_t *out_round,
                  uint64_t *out_ticket);
hoStatus hoSessionProgress(hoSession *s, uint32_t max_graph_launches, uint32_t *active,
                           uint32_t *queued);
hoStatus hoPoll(hoSession *s, uint64_t ticket, int *done);
hoStatus hoCancel(hoSession *s, uint64_t ticket);
hoStatus hoSessionDestroy(hoSession *s);

/* (k,h)-truss extraction: the (k,h)-truss is the edge set {e : t(e,h) >= k}
 * (Def. 4; trusses are nested, so one decomposition answers every k).
 * Given the trussness of every edge (device, uint32 [m], as written by
 * hoTrussDecompose) and k, writes for each edge of the truss the smallest
 * vertex id of its connected component in the truss, and UINT32_MAX for the
 * edges below k (out_component, device, uint32 [m]); *out_count (host)
 * receives the number of components.  Validates the CSR like the other
 * entry points; returns after the work has completed.  The workspace
 * (hoTrussComponentsWorkspaceBytes, about 32m + 8n bytes) is the caller's. */
size_t hoTrussComponentsWorkspaceBytes(uint32_t n, uint64_t m);
hoStatus hoTrussComponents(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                           const uint32_t *trussness, uint32_t k, uint32_t *out_component,
                           uint32_t *out_count, void *workspace, size_t workspace_bytes,
                           hipStream_t stream);

/* ------------------------------------------------------------------------
 * H-index fixpoint method (Section 4: the h-hop reachable path key, the
 * higher-order H-index, Theorems 1-2; Section 4.2, Algorithm 2, the parallel
 * update loop, and the asynchronous updating of Section 4.1).  A second exact
 * algorithm for the same trussness: starting from H(e) = sup_G(e, h), every
 * sweep sets
 *     H(u,v) = H-index of { min(P(u,w), P(v,w)) : w a common h-hop neighbour }
 * where P(x,w) is the largest smallest-H over paths of at most h edges from x
 * to w; the values never rise and stop at t(e, h) - 2.
 *
 *   row_ptr, col_idx, n, m, h  as for hoTrussDecompose (device CSR of a simple
 *               undirected graph, symmetric, rows sorted; h >= 1).
 *   flags       0: synchronous sweeps (every update reads the previous
 *               sweep's values; the sequence of the paper's definition).
 *               HO_HINDEX_ASYNC: asynchronous sweeps (vertices in 8 chunks
 *               taken in order; a chunk reads the values earlier chunks of
 *               the same sweep wrote).  HO_HINDEX_ALL: recompute every path-key
 *               row and edge in every sweep instead of only those whose inputs
 *               changed (same values; for measurement).  By default an edge
 *               is re-evaluated only as the paper's pruning rule allows
 *               (Section 4.3, Lemma 4: skipped unless some edge its update
 *               reads fell from >= its value to below it).  HO_HINDEX_KEYS:
 *               apply that test to the path keys of its endpoints instead
 *               (finer, but each rebuilt row is compared with its previous
 *               keys; same values).  HO_HINDEX_STATS: time every launch
 *               group with HIP events and count work (slower).
 *   max_sweeps  0: run until a sweep changes nothing (that sweep is counted);
 *               else stop after that many sweeps.  out_trussness then holds
 *               H + 2 of the last sweep (synchronous: H^(max_sweeps) + 2).
 *   out_trussness  device [m]: H + 2 per canonical edge id.
 *   out_sweeps  host: sweeps run.  The call waits on `stream` once per sweep
 *               (to read how many values changed) and returns when done.
 *   workspace   device, caller-owned.  Its size depends on the total size of
 *               the h-hop balls, known only on the device: pass at least
 *               hoTrussHIndexWorkspaceBytes(n, m, h) bytes; when the balls
 *               need more, the call returns HO_ERR_WORKSPACE with
 *               *needed_bytes set (8 bytes per ball member, 12 for h >= 3, and
 *               4 more with HO_HINDEX_KEYS, on top of the minimum); call again
 *               with that much.
 *   needed_bytes  host, may be NULL: the workspace size this graph and these
 *               flags need (set on success and on HO_ERR_WORKSPACE).
 *   Errors as for hoTrussDecompose; flags outside the four bits give
 *   HO_ERR_INVALID_ARG.  hoTrussLastStats afterwards: rounds = sweeps, events =
 *   value changes, work[0] = edge evaluations, work[1] = path-key rows built,
 *   device_ms = the whole call.  HO_HINDEX_STATS adds kernel_ms/kernel_launches
 *   [0] balls, H^(0) and ranks, [1] path-key rows, [2] edge updates, [3] change
 *   tracking, and work [2] relaxations, [3] direct keys, [4] row entries
 *   written, [5] passes over a common neighbourhood, [6] bytes those passes
 *   read (ball rows, rank words, member lists; keys excluded), [7] common
 *   members visited. */
#define HO_HINDEX_ASYNC 0x1u
#define HO_HINDEX_ALL 0x2u
#define HO_HINDEX_STATS 0x4u
#define HO_HINDEX_KEYS 0x8u
size_t hoTrussHIndexWorkspaceBytes(uint32_t n, uint64_t m, uint32_t h);
hoStatus hoTrussHIndex(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                       uint32_t h, uint32_t flags, uint32_t max_sweeps, uint32_t *out_trussness,
                       uint32_t *out_sweeps, void *workspace, size_t workspace_bytes,
                       size_t *needed_bytes, hipStream_t stream);

const char *hoStatusString(hoStatus s);

#ifdef __cplusplus
}
#endif

#endif /* HOTRUSS_H */
