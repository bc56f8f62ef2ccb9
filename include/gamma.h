/*
 * gamma.h - C ABI of the MI355X (gfx950) batch-dynamic subgraph matching
 * library.
 *
 * Problem (paper Sec. II-A, Def. 1, Def. 2 and the problem statement): a
 * data graph G = (V, E, L) is undirected, simple and vertex-labelled; a query
 * Q is a small connected labelled graph; a batch is a set of edge insertions
 * and deletions.  A match is an injective map f: V(Q) -> V with L(f(u)) =
 * L(u) for every query vertex and {f(u), f(w)} in E for every query edge (not
 * induced; automorphic images are distinct matches).  For every batch the
 * library reports the incremental matches: the matches of the updated graph
 * G' that are not matches of G (insertion results, sign +) and the matches
 * of G that are not matches of G' (deletion results, sign -).
 *
 * Method (Sec. IV): the batch is applied to a dynamic CSR; a neighbourhood
 * label frequency filter (Sec. IV-B) marks candidate vertices per query
 * vertex; for every batch edge and every query edge it can map to, a
 * depth-first search extends partial matches by intersecting sorted
 * neighbour lists (Algorithm 1), and a total order over the batch edges
 * makes each match come from exactly one of them (the rule stated after
 * Algorithm 1).  Everything after the input copy runs in HIP kernels on the
 * device; there is no CPU fallback.
 *
 * Conventions
 *   - Vertex ids are uint32 in [0, n), n < 2^31.  Labels are uint32 < 65536.
 *   - All functions return gamma_status.  0 (GAMMA_OK) and 1
 *     (GAMMA_TRUNCATED) are successes; negative values are failures.  Every
 *     failure other than GAMMA_EDEVICE leaves the graph and the registered
 *     queries unchanged (inputs are validated before anything is mutated).
 *     GAMMA_EDEVICE poisons the context: every later call returns it.
 *   - Callers own every input array; the library reads it during the call
 *     and keeps its own copy.  `where` tells whether a pointer is host
 *     memory or device memory on the context's device (device inputs are
 *     read on the context stream, ordered after work the caller queued on
 *     that stream).
 *   - The library owns the graph, the queries, all scratch memory and the
 *     result buffers.  Result pointers stay valid until the next
 *     gamma_apply_batch on the context, gamma_result_release or
 *     gamma_destroy.
 *   - One host thread at a time per context.
 */
#ifndef GAMMA_H
#define GAMMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Edge labels are < GAMMA_MAX_EDGE_LABELS. */
#define GAMMA_MAX_EDGE_LABELS 256u

typedef enum gamma_status {
  GAMMA_OK = 0,
  GAMMA_TRUNCATED = 1,      /* success; tuple capacity reached, counts/hashes still exact */
  GAMMA_EINVAL = -1,        /* malformed argument (ids out of range, self loop, bad CSR, ...) */
  GAMMA_ECONFLICT = -2,     /* the batch inserts and deletes the same edge */
  GAMMA_ENOMEM = -3,        /* device or host allocation failed (nothing mutated) */
  GAMMA_EUNSUPPORTED = -4,  /* outside the supported envelope (k > 16, disconnected query, ...) */
  GAMMA_ESTATE = -5,        /* call order (e.g. apply_batch before load_graph) */
  GAMMA_ETIMEDOUT = -6,     /* search deadline exceeded; batch not committed (graph unchanged) */
  GAMMA_EDEVICE = -7        /* HIP runtime error; the context is poisoned */
} gamma_status;

typedef enum gamma_mem { GAMMA_MEM_HOST = 0, GAMMA_MEM_DEVICE = 1 } gamma_mem;

/* Context options.  Zero-initialise and set what you need. */
typedef struct gamma_options {
  int32_t device;            /* HIP device ordinal */
  void* stream;              /* hipStream_t to run on; NULL = library-created stream */
  uint64_t tuple_capacity;   /* max tuple records stored per batch (0 = no tuple buffer) */
  uint32_t waves_per_cu;     /* persistent DFS waves per CU (0 = default: as many as stay
                                resident with the lean search build's register use, 16 on
                                gfx950; more than can reside add nothing) */
  uint32_t steal;            /* 0 = no work stealing, 1 = on (default when unset: see below) */
  uint32_t steal_set;        /* nonzero: honour `steal`; zero: library default (on) */
  uint32_t deadline_ms;      /* search deadline (0 = none), counted from the start of each
                                search launch: the batch's one launch, or with
                                query_launch = 2 each query's own launch (a time limit
                                per query, Sec. VI-A).  A query whose search passes it is
                                unsolved (open_seeds > 0); the batch then returns
                                GAMMA_ETIMEDOUT and is not committed */
  uint32_t reserved[7];
} gamma_options;

/* Flags of gamma_apply_batch. */
enum {
  GAMMA_F_COUNT = 1u << 0,          /* counts per query and sign (always on) */
  GAMMA_F_HASH = 1u << 1,           /* order-independent multiset hash per query and sign */
  GAMMA_F_TUPLES = 1u << 2,         /* store match tuples (up to tuple_capacity records) */
  GAMMA_F_SEED_ATTR = 1u << 3,      /* store the seed ord of each tuple record */
  GAMMA_F_PER_UPDATE = 1u << 4,     /* count / hash per canonical batch edge (attribution) */
  GAMMA_F_CANONICAL = 1u << 5,      /* return the canonical batch on the host */
  GAMMA_F_DRY_RUN = 1u << 6         /* search the batch but do not commit it: results and
                                       statistics as for a normal call, graph unchanged */
};

/* Search tunables.  They change how the work is spread over the chip, never
 * the result.  In gamma_set_tuning a zero field keeps the current value. */
typedef struct gamma_tuning {
  uint32_t waves_per_cu;  /* persistent search waves per CU, 1..32 */
  uint32_t steal;         /* 1 = chip-wide work hand-over (Sec. V-A), 2 = none */
  uint32_t poll_cycles;   /* shader cycles between a busy wave's hand-over polls, 500..10^6 */
  uint32_t split_inner;   /* smallest inner-level candidate range handed over, 2..2^20 */
  uint32_t split_leaf;    /* smallest last-level candidate range handed over, 2..2^20 */
  uint32_t query_launch;  /* 1 = every query's seeds in one search launch, 2 = one launch per query */
  uint32_t handover_gate; /* with c idle waves a busy wave tries a hand-over per poll with
                             probability min(1, c * handover_gate / 1024), 1..1024 */
  uint32_t coalesced_search; /* 2 = on (default): directed query edges that a label-preserving
                                automorphism of the query maps onto each other are searched
                                once and the other matches are produced by permuting the
                                found ones (Sec. V-B); 3 = also over the k-degenerated
                                automorphic subgraph left by removing the degree-1 query
                                vertices, for queries with no automorphism of their own: the
                                core edges of one orbit are searched once, each core match is
                                permuted by the core's automorphisms and the removed vertices
                                are matched anew for each permutation; 1 = off.  Results are
                                identical in every mode */
  uint32_t group_seeds;   /* update-edge grouping (Alg. 1's loop over update edges).  3 = seeds
                             grouped by (query, directed query edge (x, y), data vertex a of x);
                             a group of two or more whose level 2 has a list from a gets that
                             list built once, filtered by the candidate table, and its seeds
                             search level 2 from it.  2 = seeds only sorted (stably) by a, so
                             that waves starting together share rows.  1 = generation order
                             (default).  With query_launch = 2 seeds stay in generation order.
                             Results are identical in every mode. */
  uint32_t shared_leaf;   /* set-ups shared between partial matches that differ only in the
                             vertex matched last.  3 = the last level: when none of the last
                             query vertex's lists comes from the vertex matched just before
                             it, its candidates are read and filtered once per chunk of 64
                             partial matches and paired with each of them.  2 (default) = that,
                             and an inner level whose lists do not come from the vertex
                             matched just before it keeps its set-up from one such partial
                             match to the next.  1 = neither.  Results are identical in every
                             mode. */
} gamma_tuning;

/* Per query results of one batch.  Index 1 = insertion results (+),
 * index 0 = deletion results (-). */
typedef struct gamma_query_result {
  uint32_t qid;
  uint32_t k;
  uint64_t count[2];
  uint64_t hash_sum[2];  /* sum mod 2^64 of the per-tuple hash (GAMMA_F_HASH) */
  uint64_t hash_xor[2];  /* xor of the per-tuple hash (GAMMA_F_HASH) */
  /* seeds of this query whose search did not finish before the deadline
   * (tracked when a deadline is set or with GAMMA_F_PER_UPDATE): 0 = the
   * figures above are exact, > 0 = the query is unsolved and they are a
   * lower bound of what the search found */
  uint64_t open_seeds;
} gamma_query_result;

typedef struct gamma_batch_stats {
  uint32_t n_input;        /* updates passed in */
  uint32_t n_canonical;    /* |I| + |D| */
  uint32_t n_insert;       /* |I| */
  uint32_t n_delete;       /* |D| */
  uint32_t n_noop;         /* +e with e in E, or -e with e not in E (skipped) */
  uint32_t n_duplicate;    /* repeated updates collapsed */
  uint32_t n_touched;      /* vertices whose neighbour list changed */
  uint32_t n_groups;       /* update-edge grouping (group_seeds = 3): groups of seeds by
                              (query, directed query edge, a); 0 when not grouped */
  uint64_t n_seeds;        /* (batch edge x directed query edge) pairs that pass the filter */
  uint64_t dfs_nodes;      /* partial matches extended (levels >= 2) */
  uint64_t steals;         /* successful work steals */
  uint64_t cand_scanned;   /* candidate-list entries examined */
  uint64_t bytes_alg_dfs;  /* algorithmic bytes of the search by a fixed model (Sec. IV-C's
                              GenCandidates): per candidate examined 4 B id + 1 B label +
                              1 bit of the candidate table; per lower-bound search in a list
                              of length n, (ceil(log2 n) + 1) x 4 B; 16 B per batch-hash
                              probe; 4 B per tuple element written */
  uint64_t bytes_alg_update; /* algorithmic bytes of the graph update (merge + commit) */
  float ms_canon, ms_merge, ms_filter, ms_seed, ms_dfs, ms_commit, ms_total;
  float reserved1;
  /* search-kernel time split, summed over waves, in shader clock cycles */
  uint64_t cyc_idle;       /* waiting for work */
  uint64_t cyc_init;       /* setting up a level (neighbour-list subranges) */
  uint64_t cyc_inner;      /* evaluating candidate chunks above the last level */
  uint64_t cyc_leaf;       /* evaluating and emitting last-level chunks */
  uint64_t cyc_handover;   /* handing work to idle waves */
  uint64_t tasks_received; /* work items received from other waves */
  uint64_t seeds_started;  /* seeds taken by the search (all of n_seeds unless timed out) */
} gamma_batch_stats;

typedef struct gamma_batch_result {
  uint32_t n_queries;
  uint32_t tuple_width;           /* words per tuple row = max k over registered queries */
  gamma_query_result* queries;    /* host array [n_queries], library-owned */
  /* tuple records (GAMMA_F_TUPLES): device pointers, library-owned.
   * tuples  [n_tuples * tuple_width] external vertex ids in query-vertex order,
   *         unused trailing words are 0xFFFFFFFF;
   * meta    [n_tuples] = qid << 1 | sign;
   * ord     [n_tuples] seed ord (GAMMA_F_SEED_ATTR), else NULL. */
  uint64_t n_tuples;              /* records stored */
  uint64_t n_tuples_found;        /* records found (> n_tuples when truncated) */
  uint32_t* tuples;
  uint32_t* meta;
  uint32_t* ord;
  /* canonical batch on the host (GAMMA_F_CANONICAL), ascending (lo, hi),
   * entry i has ord i; external ids. */
  uint32_t n_canonical;
  uint32_t reserved0;
  uint32_t* canon_lo;
  uint32_t* canon_hi;
  uint8_t* canon_sign;
  /* per canonical batch edge, indexed by ord (GAMMA_F_PER_UPDATE): totals
   * over every registered query of the matches attributed to that edge. */
  uint64_t* upd_count;
  uint64_t* upd_hash_sum;
  uint64_t* upd_hash_xor;
  gamma_batch_stats stats;
  /* with GAMMA_F_PER_UPDATE, per ord: 1 = some search work seeded from this
   * update did not finish, so its figures above are partial.  All 0 after a
   * completed search; after a deadline (GAMMA_ETIMEDOUT) the updates marked
   * 0 still carry exact figures. */
  uint8_t* upd_open;
} gamma_batch_result;

typedef struct gamma_ctx gamma_ctx;

/* Create a context on opt->device (all fields of opt may be zero).
 * Errors: EINVAL (null out), EDEVICE (no such device / HIP failure). */
gamma_status gamma_create(const gamma_options* opt, gamma_ctx** out);

/* Free every library allocation of the context.  NULL is accepted. */
gamma_status gamma_destroy(gamma_ctx* ctx);

/* Load (replace) the data graph: symmetric CSR with ascending rows.
 *   n        number of vertices (1 <= n < 2^31)
 *   nnz      row_ptr[n] = number of directed entries (= 2|E|)
 *   row_ptr  [n+1] uint64, non-decreasing, row_ptr[0] = 0
 *   col      [nnz] uint32, each row strictly ascending, no self loops,
 *            every entry (v, w) has its mirror (w, v)
 *   labels   [n] uint32 < 65536
 * The paper's data model (Sec. II-A).  Registered queries are kept and their
 * candidate filters are rebuilt.  Errors: EINVAL (malformed CSR, leaves the
 * previous graph in place), ENOMEM, EDEVICE. */
gamma_status gamma_load_graph(gamma_ctx* ctx, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                              const uint32_t* col, const uint32_t* labels, gamma_mem where);

/* Load an edge-labelled graph (Sec. II-A: the labelling function covers
 * edges too).  As gamma_load_graph, plus
 *   elabels    [nnz] uint32 < n_elabels, the label of each CSR entry (the
 *              mirror entry carries the same label)
 *   n_elabels  1 .. GAMMA_MAX_EDGE_LABELS
 * The graph stays simple (one edge, with one label, per pair; rows ascend
 * strictly as for gamma_load_graph).  A query edge with label e maps only
 * onto data edges with label e.  Storage: one
 * row per (vertex, label) (row id v << ceil(log2 n_elabels) | e), so device
 * memory for row offsets and the label index grows with n * n_elabels; n
 * times the power of two above n_elabels must stay below 2^31 (else
 * EUNSUPPORTED).  gamma_load_graph is this call with one label. */
gamma_status gamma_load_graph_el(gamma_ctx* ctx, uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                                 const uint32_t* col, const uint32_t* labels, const uint32_t* elabels,
                                 uint32_t n_elabels, gamma_mem where);

/* Register a standing query (host arrays).
 *   k        vertices, 2 <= k <= 16
 *   qlabels  [k] labels < 65536
 *   m        edges, k-1 <= m <= k(k-1)/2
 *   qedges   [2m] pairs (a, b), a != b, < k, no repeated pair
 * The query must be connected.  A matching order is planned for each
 * directed query edge (Sec. IV-C: more selective query vertices first) and
 * the candidate filter (Sec. IV-B) is built over the whole graph.
 * Errors: EINVAL, EUNSUPPORTED (disconnected, k > 16, too many queries),
 * ENOMEM, EDEVICE.  *out_qid receives the query id (0, 1, ...). */
gamma_status gamma_register_query(gamma_ctx* ctx, uint32_t k, const uint32_t* qlabels, uint32_t m,
                                  const uint32_t* qedges, uint32_t* out_qid);

/* As gamma_register_query with qelabels [m] < GAMMA_MAX_EDGE_LABELS, the
 * label of each query edge (NULL: all 0).  A query with an edge label the
 * loaded graph does not have (>= its n_elabels) matches nothing. */
gamma_status gamma_register_query_el(gamma_ctx* ctx, uint32_t k, const uint32_t* qlabels, uint32_t m,
                                     const uint32_t* qedges, const uint32_t* qelabels, uint32_t* out_qid);

/* Apply one batch and report its incremental matches for every registered
 * query (the problem statement of Sec. II-A; Algorithm 1 of Sec. IV-C).
 *   n_upd    updates, <= 2^20 per call
 *   src,dst  [n_upd] endpoints (either orientation)
 *   op       [n_upd] 1 = insert, 0 = delete
 *   where    memory kind of src/dst/op
 *   flags    GAMMA_F_* (COUNT is implied)
 *   out      filled on success (library-owned buffers, see above)
 * Canonical semantics: duplicates collapse; +e with e in E and -e with e not
 * in E are skipped as no-ops; a self loop or an id >= n gives EINVAL; +e
 * together with -e gives ECONFLICT.  Either error leaves the graph unchanged.
 * Returns OK or TRUNCATED (tuple capacity reached; counts and hashes exact).
 * With a deadline (gamma_options.deadline_ms, gamma_set_deadline) a search
 * launch stops cooperatively once it passes; the call then returns
 * GAMMA_ETIMEDOUT, the graph keeps its state from before the batch, and
 * `out` holds the partial statistics (stats.seeds_started tells how far the
 * search got) and every query's figures: those with open_seeds = 0 finished
 * and are exact (with query_launch = 2 every query gets its own time). */
gamma_status gamma_apply_batch(gamma_ctx* ctx, uint32_t n_upd, const uint32_t* src,
                               const uint32_t* dst, const uint8_t* op, gamma_mem where,
                               uint32_t flags, gamma_batch_result* out);

/* gamma_apply_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same batch semantics and results, with every per-batch
 * device buffer taken from a static 64 MiB array in the library (one per
 * GPU, held until the process ends) instead of the context's buffers.  It
 * calls no hipMalloc, hipFree or hipHostMalloc (results are staged through
 * the context's pinned buffer when it is large enough, else through
 * pageable host memory).
 *   Same arguments as gamma_apply_batch.  TUPLES and SEED_ATTR are not
 *   available (EUNSUPPORTED); grouping of seeds (group_seeds = 2) is skipped.
 * Errors: ENOMEM, with the graph unchanged, when the batch's buffers exceed
 * the array (about 270 bytes per update plus 16 per update and directed
 * query edge: roughly 120,000 updates for one 8-vertex, 8-edge query) or
 * when the graph's arena has no
 * room for the batch's rows (a gamma_apply_batch call compacts it);
 * EDEVICE when the array's address could not be found on this device.
 * The array is shared by every context on a GPU and keeps the last call's
 * contents (each call clears what it needs): calls that overlap on one GPU,
 * from several threads or contexts, race and must be serialised by the
 * caller. */
gamma_status gamma_apply_batch_noalloc(gamma_ctx* ctx, uint32_t n_upd, const uint32_t* src,
                                       const uint32_t* dst, const uint8_t* op, gamma_mem where,
                                       uint32_t flags, gamma_batch_result* out);

/* As gamma_apply_batch on an edge-labelled graph: update i names the
 * triple {src[i], dst[i], elab[i]} (elab NULL: all 0; a label >= n_elabels
 * gives EINVAL).  Two updates of one pair in a batch must name the same
 * triple with the same op (a duplicate), else ECONFLICT; so a pair occurs
 * at most once in the canonical batch and ord is its rank by (lo, hi).
 * Inserting a present triple or deleting an absent one (also a present pair
 * under another label) is a no-op; inserting a pair that is present under
 * another label gives EINVAL (relabelling takes a deletion and a later
 * insertion). */
gamma_status gamma_apply_batch_el(gamma_ctx* ctx, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                  const uint8_t* op, const uint32_t* elab, gamma_mem where, uint32_t flags,
                                  gamma_batch_result* out);

/* Vertex updates (Sec. II-A, the batch-dynamic setting): a vertex deletion
 * is the deletion of all of its incident edges; a vertex insertion adds the
 * vertex first, its edges then come as edge insertions.
 *
 * gamma_apply_batch_vertices applies one batch of edge updates plus vertex
 * deletions.  Each deleted vertex (external id in vdel[n_vdel], duplicates
 * allowed) is expanded on the device into deletions of every edge it has in
 * the current graph, appended after the explicit updates; the merged batch
 * is then applied exactly as by gamma_apply_batch (same flags, result and
 * per-update attribution, whose canonical order covers the expanded edges
 * too).  The vertex keeps its id and label and is isolated afterwards.
 *   src,dst,op,n_upd  explicit edge updates as for gamma_apply_batch
 *   elab              their edge labels as for gamma_apply_batch_el (may be
 *                     NULL); expanded deletions carry each edge's own label
 *   vdel,n_vdel       vertices to delete, n_vdel <= 2^20
 *   where             memory kind of all six arrays
 * Errors: EINVAL (an id >= n, null arrays, more than 2^20 updates after the
 * expansion), ECONFLICT (an explicit insertion touches a deleted vertex, or
 * the rules of gamma_apply_batch), and those of gamma_apply_batch.  Any
 * error leaves the graph unchanged. */
gamma_status gamma_apply_batch_vertices(gamma_ctx* ctx, uint32_t n_upd, const uint32_t* src,
                                        const uint32_t* dst, const uint8_t* op, const uint32_t* elab,
                                        uint32_t n_vdel, const uint32_t* vdel, gamma_mem where,
                                        uint32_t flags, gamma_batch_result* out);

/* Append `count` isolated vertices with host labels[count] (< 2^16); they
 * get the external ids n, n+1, ... (*first_id = n, may be NULL).  The graph
 * is rebuilt on the device and registered queries are re-planned, as by
 * gamma_load_graph.  Errors: EINVAL (count 0, null labels, n + count >=
 * 2^31), ESTATE (no graph), ENOMEM, EDEVICE; on error the graph is as before
 * except after EDEVICE. */
gamma_status gamma_add_vertices(gamma_ctx* ctx, uint32_t count, const uint32_t* labels, uint32_t* first_id);

/* Current search tunables (every field filled).  Errors: EINVAL (NULL). */
gamma_status gamma_get_tuning(const gamma_ctx* ctx, gamma_tuning* out);

/* Set search tunables; zero fields keep their value.  Errors: EINVAL (a
 * value outside the ranges in gamma_tuning; nothing changed). */
gamma_status gamma_set_tuning(gamma_ctx* ctx, const gamma_tuning* in);

/* Pause (active = 0) or resume a standing query.  A paused query's
 * candidate table is kept current with every batch, but it gets no seeds:
 * its results are 0 until it is resumed, and later batches report it again
 * (matches of the batches it missed are not replayed).  Errors: EINVAL
 * (NULL ctx, no such qid), EDEVICE. */
gamma_status gamma_set_query_active(gamma_ctx* ctx, uint32_t qid, uint32_t active);

/* Set the search deadline of later batches, as gamma_options.deadline_ms
 * (0 = none; with query_launch = 2 it is a time limit per query, after
 * which the query is reported unsolved, Sec. VI-A).  Errors: EINVAL (NULL). */
gamma_status gamma_set_deadline(gamma_ctx* ctx, uint32_t deadline_ms);

/* Tune the search for the current graph and queries on a calibration batch.
 * Every evaluation is a dry run (GAMMA_F_DRY_RUN with `flags`) of the batch,
 * timed as the median device time of `reps` runs (1..9).  Coordinate
 * search from the current tunables over query_launch, coalesced_search, steal, waves_per_cu,
 * handover_gate, poll_cycles, split_leaf and split_inner, at most max_points evaluations
 * (1..64).  The fastest point is applied and written to *best; *best_ms and
 * *base_ms (may be NULL) receive its time and the starting point's.  The
 * graph is unchanged.  Errors: those of gamma_apply_batch (ETIMEDOUT from a
 * deadline ends the search early and keeps the best point so far), EINVAL. */
gamma_status gamma_autotune(gamma_ctx* ctx, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                            const uint8_t* op, gamma_mem where, uint32_t flags, uint32_t max_points,
                            uint32_t reps, gamma_tuning* best, double* best_ms, double* base_ms);

/* ------------------------------------------------------------------ serving
 * A served update stream with continuous batching (the paper's asynchronous
 * pipeline keeps batch preparation off the search's critical path,
 * Sec. IV-A).  A server owns a worker thread that applies queued update
 * requests to the context's graph.  Each device batch takes queued requests
 * in submission order while their updates fit max_batch_updates, and closes
 * before a request that inserts an edge another request of the batch
 * deletes (or the reverse): such pairs are applied in order.  After each
 * batch the graph equals the one that applying its requests one at a time
 * would give, and the batch's net result per query (|+| - |-|) equals the
 * sum of theirs; the batch reports M(G_after) \ M(G_before) and the reverse.
 * Batches commit in submission order.  While a server exists, the context
 * may only be used through the server (the worker calls gamma_apply_batch
 * on it). */
typedef struct gamma_server gamma_server;

typedef struct gamma_serve_options {
  uint32_t max_batch_updates; /* admission limit per device batch, 1..2^20 (0 = 2^17); a single
                                 request may not exceed it */
  uint32_t flags;             /* GAMMA_F_HASH / GAMMA_F_PER_UPDATE / GAMMA_F_TUPLES (+ SEED_ATTR)
                                 for every batch (no DRY_RUN or CANONICAL) */
  uint32_t coalesce;          /* 1 = continuous batching (default), 2 = one request per batch */
  uint32_t tuple_fill_pct;    /* with TUPLES: admission keeps a batch's estimated tuples within
                                 this share of the context's tuple_capacity, 1..100 (0 = 50) */
  uint32_t max_batch_ms;      /* admission by estimated work, in every mode: keeps a batch's
                                 estimated device time (a moving estimate of device ms per
                                 update over the batches so far) within this budget; the first
                                 request of a batch is always admitted (0 = no limit) */
  uint32_t reserved[3];
} gamma_serve_options;

/* A committed request. */
typedef struct gamma_request_result {
  uint64_t ticket;       /* submission order, from 0 */
  uint64_t batch;        /* device batch that committed it */
  double t_submit_ms;    /* server clock (ms since gamma_serve_create) at submission */
  double t_done_ms;      /* at commit of its batch */
  uint32_t n_updates;
  int32_t status;        /* the batch's gamma_status */
} gamma_request_result;

/* A device batch of the server. */
typedef struct gamma_serve_batch {
  uint64_t batch;
  uint64_t first_ticket; /* its requests are first_ticket .. first_ticket + n_requests - 1 */
  uint32_t n_requests;
  uint32_t n_updates;    /* before canonicalisation */
  uint32_t n_canonical;
  uint32_t n_queries;
  int32_t status;
  float ms_device;       /* stats.ms_total of the batch */
  double t_start_ms, t_done_ms;
  uint64_t n_tuples;       /* with TUPLES: tuple records kept for the batch */
  uint64_t n_tuples_found; /* matches found (> n_tuples when the buffer overflowed: TRUNCATED) */
} gamma_serve_batch;

/* Start a server on a context with a loaded graph.  Errors: EINVAL (bad
 * options), ESTATE (no graph), ENOMEM. */
gamma_status gamma_serve_create(gamma_ctx* ctx, const gamma_serve_options* opt, gamma_server** out);

/* Queue one request (host arrays, copied; thread-safe).  The request is
 * validated like a batch (ids < n, no self loop, no +e with -e inside it):
 * EINVAL / ECONFLICT reject it and nothing is queued.  *ticket (may be
 * NULL) receives its ticket. */
gamma_status gamma_serve_submit(gamma_server* srv, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                const uint8_t* op, uint64_t* ticket);

/* As gamma_serve_submit on an edge-labelled graph: update i names the
 * triple (src[i], dst[i], elab[i]) (elab NULL: all 0), labels < the
 * graph's n_elabels (else EINVAL); one pair twice in a request must be the
 * same triple with the same op (else ECONFLICT).  A request naming a pair
 * of the forming batch under another label or op starts the next batch. */
gamma_status gamma_serve_submit_el(gamma_server* srv, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                   const uint8_t* op, const uint32_t* elab, uint64_t* ticket);

/* Move up to `max` committed requests (ticket order) into out[]; *n_out
 * receives how many.  Each is returned once. */
gamma_status gamma_serve_poll(gamma_server* srv, gamma_request_result* out, uint32_t max, uint32_t* n_out);

/* Block until every submitted request is committed. */
gamma_status gamma_serve_drain(gamma_server* srv);

/* Requests submitted and committed, and device batches applied (any may be NULL). */
gamma_status gamma_serve_counts(gamma_server* srv, uint64_t* submitted, uint64_t* committed, uint64_t* batches);

/* Information and per-query results (up to max_queries entries, may be
 * NULL) of device batch `batch`.  Errors: EINVAL (no such batch). */
gamma_status gamma_serve_get_batch(gamma_server* srv, uint64_t batch, gamma_serve_batch* info,
                                   gamma_query_result* queries, uint32_t max_queries);

/* Match buffer of a served batch (servers created with GAMMA_F_TUPLES).
 * Admission by estimated match-buffer memory: the server keeps a moving
 * estimate of tuple records per update from the batches it has committed
 * and admits requests into a batch while the estimate for the batch stays
 * within tuple_fill_pct of the context's tuple_capacity (one request per
 * batch until a batch has been seen).  After each commit the batch's
 * records (layout as in gamma_batch_result) are copied to host memory and
 * kept with the batch until the server is destroyed.  This copies up to
 * max_records of them into caller host buffers (any may be NULL; ord only
 * with SEED_ATTR); *n_records and *width receive the batch's totals.
 * Errors: EINVAL (no such batch), ESTATE (the server keeps no tuples). */
gamma_status gamma_serve_get_tuples(gamma_server* srv, uint64_t batch, uint32_t* tuples, uint32_t* meta,
                                    uint32_t* ord, uint64_t max_records, uint64_t* n_records, uint32_t* width);

/* Apply what is queued, stop the worker and free the server.  NULL is accepted. */
gamma_status gamma_serve_destroy(gamma_server* srv);

/* Copy up to max_records tuple records of the last batch into caller
 * buffers (any may be NULL) on the context stream; `where` is the memory
 * kind of the destinations.  Layout as in gamma_batch_result.  Errors:
 * ESTATE (no batch result), EDEVICE. */
gamma_status gamma_copy_tuples(gamma_ctx* ctx, uint32_t* tuples, uint32_t* meta, uint32_t* ord,
                               uint64_t max_records, gamma_mem where);

/* Release the result buffers of the last batch early (optional). */
gamma_status gamma_result_release(gamma_ctx* ctx, gamma_batch_result* res);

/* Snapshot the current graph into caller host buffers: row_ptr [n+1],
 * col [nnz] (ascending rows, external ids), labels [n].  Query sizes first
 * with col == NULL: *n_out and *nnz_out are always written. */
gamma_status gamma_export_graph(gamma_ctx* ctx, uint32_t* n_out, uint64_t* nnz_out,
                                uint64_t* row_ptr, uint32_t* col, uint32_t* labels);

/* As gamma_export_graph, plus *n_elabels_out and elabels [nnz] (each row
 * ascending by (neighbour, label)); any output may be NULL. */
gamma_status gamma_export_graph_el(gamma_ctx* ctx, uint32_t* n_out, uint64_t* nnz_out, uint32_t* n_elabels_out,
                                   uint64_t* row_ptr, uint32_t* col, uint32_t* labels, uint32_t* elabels);

/* Host-only validators (no device needed); same rules as the calls above. */
gamma_status gamma_validate_graph(uint32_t n, uint64_t nnz, const uint64_t* row_ptr,
                                  const uint32_t* col, const uint32_t* labels);
gamma_status gamma_validate_query(uint32_t k, const uint32_t* qlabels, uint32_t m,
                                  const uint32_t* qedges);

/* The matching plans of a query as registration builds them (Algorithm 1
 * runs one per directed query edge; Sec. V-B groups them), for inspection
 * and tests.  Host only: no context, no GPU.  Without a graph the label
 * frequencies are unknown, so ties in the matching order are broken by
 * query degree and vertex id only (registration after load_graph also
 * prefers rarer labels); the groups do not depend on the order.
 *
 * plans[i], i < 2m, describes directed query edge (x, y):
 *   order[0 .. k-1]  the order query vertices are matched in (x, y first)
 *   n_perm           whole-query coalescing (coalesced_search >= 2): >= 1 on a
 *                    group's representative, whose matches f stand for f o pi
 *                    for each of its n_perm permutations
 *                    perms[perm_first .. perm_first + n_perm); 0 on a plan a
 *                    representative stands for
 *   n_core, n_cperm  core coalescing (coalesced_search = 3): a representative
 *                    (n_cperm >= 2) matches its n_core core vertices first, and
 *                    each core match f is continued as f o pi for each
 *                    pi in perms[cperm_first .. cperm_first + n_cperm);
 *                    n_cperm = 0: stood for; 1: ordinary (n_core = k)
 *   omask[u]         bit w set: a representative's core search admits at query
 *                    vertex u a data vertex that passes the filter of w
 * perms[16 * j + v] = pi_j(v): the forward map of permutation j (a match g
 * derived from f is g(v) = f(pi_j(v))).
 * Errors: the query rules of gamma_validate_query (and edge labels < 256);
 * EINVAL for null outputs or when 2m > max_plans or the permutations exceed
 * max_perms (n_plans and n_perms are still set to the sizes needed). */
typedef struct gamma_plan_info {
  uint32_t x, y;
  uint32_t n_perm, perm_first;
  uint32_t n_core, n_cperm, cperm_first;
  uint32_t reserved;
  uint32_t order[16];
  uint32_t omask[16];
} gamma_plan_info;
gamma_status gamma_describe_query(uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges,
                                  const uint32_t* qelabels, uint32_t max_plans, gamma_plan_info* plans,
                                  uint32_t* n_plans, uint32_t max_perms, uint32_t* perms, uint32_t* n_perms);
gamma_status gamma_validate_batch(uint32_t n, uint32_t n_upd, const uint32_t* src,
                                  const uint32_t* dst, const uint8_t* op);
/* Edge-labelled forms, the rules of gamma_load_graph_el and
 * gamma_apply_batch_el: labels < n_elabels, a mirror entry carries its
 * entry's label (validate_graph_el); one pair twice in a batch must be
 * the same triple with the same op, else ECONFLICT (validate_batch_el).
 * NULL labels: the unlabelled rules. */
gamma_status gamma_validate_graph_el(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col,
                                     const uint32_t* labels, const uint32_t* elabels, uint32_t n_elabels);
gamma_status gamma_validate_batch_el(uint32_t n, uint32_t n_elabels, uint32_t n_upd, const uint32_t* src,
                                     const uint32_t* dst, const uint8_t* op, const uint32_t* elab);

/* Text of a status code, and of the last error on a context. */
const char* gamma_status_string(gamma_status s);
const char* gamma_last_error(const gamma_ctx* ctx);

/* Library version: major * 10000 + minor * 100 + patch. */
uint32_t gamma_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GAMMA_H */
