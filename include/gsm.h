/*
 * gsm.h — C ABI of an MI355X (gfx950) subgraph matcher.
 *
 * The library enumerates or counts every embedding of a small connected query
 * graph Q in a large undirected data graph G stored as CSR: injective maps f
 * from query vertices to data vertices that keep vertex labels and map every
 * query edge onto a data edge (non-induced).  Automorphic images are distinct
 * embeddings.  This is the matching problem of the GSM paper (Wang and Owens,
 * "Fast Gunrock Subgraph Matching (GSM) on GPUs", arXiv 2003.01527), Sec. 3.2
 * and Alg. 1: inputs Q and G, outputs the count and the listing.
 *
 * The method is the paper's breadth-first filtering-and-verification:
 *   - a host pre-computation orders the query vertices (Alg. 1
 *     PreCompute_on_CPUs);
 *   - candidates are filtered on the GPU by label, degree and neighbourhood
 *     encoding, with refinement rounds (Alg. 1 Filter_candidate_set);
 *   - partial matches are expanded level by level: gather the neighbours of
 *     an already-matched vertex, verify every edge back to the matched
 *     vertices plus injectivity, and compact the survivors (Alg. 1
 *     Verify_Constraints: Advance, Compute, Write_to_Partial);
 *   - each expansion is cut into chunks that fit a device memory budget, so
 *     memory stays bounded however many partial matches there are (the
 *     paper's stated memory goal, Sec. 1 and Sec. 5).
 *
 * Conventions shared by every entry point:
 *   - Every call returns a gsm_status.  On an error the out-parameters are
 *     left untouched (except as noted for GSM_E_TRUNCATED) and
 *     gsm_last_error() gives a message for the calling thread.
 *   - Create calls deep-copy their inputs; the caller may free them on
 *     return.  The library owns the handles it returns; destroy(NULL) is a
 *     no-op.
 *   - Pointers are host pointers unless a flag or option says "device".
 *   - Calls on one graph handle are serialised internally (one workspace per
 *     handle); distinct handles may be used from distinct threads.
 *   - Rows are q int32 columns in query-vertex-id order.  Row order is
 *     unspecified (work is distributed with atomics).
 */
#ifndef GSM_H
#define GSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsm_graph *gsm_graph_t;
typedef struct gsm_query *gsm_query_t;
typedef struct gsm_server *gsm_server_t;

typedef enum gsm_status {
  GSM_OK = 0,
  GSM_E_INVALID_ARG = 1, /* NULL handle or pointer, size out of range */
  GSM_E_BAD_GRAPH = 2,   /* CSR fails validation */
  GSM_E_BAD_QUERY = 3,   /* query disconnected, not simple, or too large */
  GSM_E_OOM = 4,         /* device or host allocation failed */
  GSM_E_BUDGET = 5,      /* memory budget below one row of some level */
  GSM_E_DEVICE = 6,      /* a HIP call failed */
  GSM_E_TRUNCATED = 7,   /* output buffer smaller than the count */
  GSM_E_CANCELLED = 8,   /* the emit callback asked to stop */
  GSM_E_UNSUPPORTED = 9, /* option not available in this build */
  GSM_E_TIMEOUT = 10     /* server wait timed out */
} gsm_status;

#define GSM_MAX_QUERY_VERTICES 16

/* ------------------------------------------------------------------ graph -- */

#define GSM_GRAPH_VALIDATE 1u    /* check the CSR (see gsm_graph_create) */
#define GSM_GRAPH_DEVICE_PTRS 2u /* row_ptr, col, labels are device pointers */
#define GSM_GRAPH_STRIP 4u       /* make the adjacency simple and undirected first */
#define GSM_GRAPH_NO_HUB_BITMAPS 8u /* no adjacency bitmaps for high-degree vertices */
#define GSM_GRAPH_DEGREE_ORDER 16u  /* store the graph renumbered by degree (see below) */

/*
 * Uploads a data graph.  The graph must be simple and undirected: each edge
 * stored in both rows, rows strictly ascending, no self-loops (the paper takes
 * undirected CSR input with no preprocessing, Sec. 2 and Sec. 3.3).
 *   n        number of vertices, 0 <= n < 2^31
 *   row_ptr  n+1 offsets, row_ptr[0] = 0, non-decreasing
 *   col      row_ptr[n] neighbour ids in [0, n)
 *   labels   n vertex labels >= 0, or NULL for an unlabelled graph (all 0)
 *   flags    GSM_GRAPH_VALIDATE checks every property above (O(m log d) on
 *            the host) and returns GSM_E_BAD_GRAPH on a violation;
 *            GSM_GRAPH_DEVICE_PTRS takes device pointers (copied device-side;
 *            validation then copies them to the host first);
 *            GSM_GRAPH_STRIP accepts any adjacency with valid offsets and ids
 *            in [0, n): self-loops are dropped, each entry v->w also adds
 *            w->v, rows are sorted and duplicates removed, on the host, before
 *            the upload (GSM_E_BAD_GRAPH only for bad offsets or ids).
 * Also computes per-vertex degree and neighbourhood encoding on the device,
 * and, unless GSM_GRAPH_NO_HUB_BITMAPS, an adjacency bitmap (n bits) for each
 * vertex of degree >= 512, highest degree first, while they fit 8 GiB and a
 * quarter of the free device memory:
 * an edge check against such a vertex is then one load instead of a search
 * of its sorted list (results are the same).
 * GSM_GRAPH_DEGREE_ORDER stores the graph with its vertices renumbered by
 * ascending degree (ties by id), on the host at creation (O(m log d), host
 * threads; offsets and ids are range-checked, GSM_E_BAD_GRAPH otherwise).
 * On skewed graphs whose ids carry no order (e.g. randomly permuted R-MAT)
 * the vertices that edge checks test most often then sit together, so the
 * words of adjacency bitmaps and the list entries those checks read share
 * cache lines.  Every result is in the caller's ids: rows (translated back
 * before they reach any sink or the row sort), candidate masks, and root
 * slices (which hash the caller's ids).  One exception: in the
 * unique-subgraph mode the embedding kept for each subgraph satisfies the
 * ordering constraints in the internal order (degree, then id), so it can be
 * another embedding of the same subgraph than without the flag; the count
 * is the same.
 */
gsm_status gsm_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const int32_t *labels, uint32_t flags, gsm_graph_t *out);

/*
 * gsm_graph_create with edge labels (the labelled graphs of Sec. 3.1 carry
 * node and edge labels).
 *   edge_labels  row_ptr[n] labels >= 0, one per CSR entry, aligned with col;
 *                both entries of an edge carry its label (checked under
 *                GSM_GRAPH_VALIDATE); device memory with GSM_GRAPH_DEVICE_PTRS;
 *                NULL = no edge labels (every edge then has label 0 for
 *                edge-labelled queries)
 * GSM_E_UNSUPPORTED with GSM_GRAPH_STRIP (cleaning reorders the entries).
 */
gsm_status gsm_graph_create_ex(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels,
                               const int32_t *edge_labels, uint32_t flags, gsm_graph_t *out);
void gsm_graph_destroy(gsm_graph_t g);

/* n, CSR entries (2m), largest label, largest degree. Any out pointer may be NULL. */
gsm_status gsm_graph_info(gsm_graph_t g, int64_t *n, int64_t *nnz, int32_t *max_label,
                          int64_t *max_degree);

/* ------------------------------------------------------------------ query -- */

/*
 * A connected, simple query graph with 1 <= q <= 16 vertices (Sec. 3.2).
 *   edges   ne pairs (a, b), 0 <= a, b < q, a != b, no duplicates
 *   labels  q labels >= 0, or NULL (all 0)
 * GSM_E_BAD_QUERY when disconnected, not simple, or q out of range.
 */
gsm_status gsm_query_create(int32_t q, int32_t ne, const int32_t *edges, const int32_t *labels,
                            gsm_query_t *out);
void gsm_query_destroy(gsm_query_t qh);

/*
 * Symmetry of a query for the unique-subgraph mode (producing each node
 * combination once, Sec. 3.3; host only, computed at gsm_query_create): aut gets
 * |Aut(Q)|, the number of automorphisms (label- and edge-preserving
 * permutations of the query vertices); pairs gets up to pairs_cap constraints
 * as (a, b) query-id pairs meaning f(a) < f(b), npairs their number (at most
 * q*(q-1)/2).  Stabilizer chain: the smallest vertex with a non-trivial orbit
 * under the automorphisms fixing the vertices chosen before is required below
 * every other vertex of its orbit, then fixed.  Any pointer may be NULL when
 * its cap is 0.
 */
gsm_status gsm_query_symmetry(gsm_query_t qh, uint64_t *aut, int32_t *pairs, int32_t pairs_cap,
                              int32_t *npairs);

/*
 * Gives every query edge a label >= 0 (edge_labels[e] for the e-th edge
 * passed to gsm_query_create; the node- and edge-labelled graphs of Sec. 3.1):
 * an embedding must then map each query edge onto a data edge with the same
 * label.  The labels are copied; GSM_E_BAD_QUERY for a negative label.  Recomputes the query's symmetry
 * (automorphisms must keep edge labels).  Edge-labelled queries are matched
 * by gsm_match only: gsm_match_batch and gsm_server_submit return
 * GSM_E_UNSUPPORTED.  Call it before the query is first used: a query that
 * another thread is matching must not change.
 */
gsm_status gsm_query_set_edge_labels(gsm_query_t qh, const int32_t *edge_labels);

/*
 * The host pre-computation of Alg. 1 (PreCompute_on_CPUs, Sec. 3.2): query
 * vertices in visiting order, greedily by larger d_M (edges to vertices
 * already ordered), smaller P_f (label frequency times the fraction of data
 * vertices of at least the query vertex's degree), larger degree, smaller id.
 *   order[i]     query vertex at position i
 *   parent[i]    position of its spanning-tree parent (earliest earlier
 *                neighbour), -1 at position 0
 *   backmask[i]  bit j set when position j < i is adjacent to position i
 */
typedef struct gsm_plan_info {
  int32_t q;
  int32_t order[GSM_MAX_QUERY_VERTICES];
  int32_t parent[GSM_MAX_QUERY_VERTICES];
  uint32_t backmask[GSM_MAX_QUERY_VERTICES];
} gsm_plan_info;

gsm_status gsm_query_plan(gsm_graph_t g, gsm_query_t qh, gsm_plan_info *out);

/* ------------------------------------------------------------------ match -- */

/* Per-call counters.  Level i is the expansion from i matched vertices to i+1. */
typedef struct gsm_stats {
  uint32_t struct_size;
  int32_t q;
  uint64_t candidates_root;             /* rows of the first frontier */
  uint64_t rows[GSM_MAX_QUERY_VERTICES];  /* rows[i]: partial matches with i+1 vertices */
  uint64_t pairs[GSM_MAX_QUERY_VERTICES]; /* pairs[i]: (row, neighbour) pairs tested at level i */
  uint64_t chunks[GSM_MAX_QUERY_VERTICES];
  uint64_t probes;                      /* binary-search steps of the back-edge checks */
  uint64_t alg_bytes;                   /* algorithmic bytes of the expansion launches */
  uint64_t filter_bytes;                /* algorithmic bytes of the filter */
  uint64_t expand_launches;             /* expansion kernel launches */
  double ms_expand;                     /* summed expansion kernel time (HIP events; needs profile) */
  double ms_total;                      /* host wall time of the call */
  uint64_t frontier_bytes;              /* bytes of intermediate rows written (packed or not) */
} gsm_stats;

/* Emit callback: receives nrows rows, valid only during the call: host memory,
 * or device memory written on the match's stream when rows_on_device is also
 * set (the stream is synchronised before the call).  Return 0 to continue,
 * non-zero to stop (gsm_match then returns GSM_E_CANCELLED). */
typedef int (*gsm_emit_fn)(void *ctx, const int32_t *rows, uint64_t nrows, int32_t q);

typedef struct gsm_match_opts {
  uint32_t struct_size;         /* sizeof(gsm_match_opts) */
  uint64_t memory_budget_bytes; /* device bytes for frontiers; 0 = 4 GiB */
  int32_t filter_rounds;        /* refinement rounds (Alg. 1 Filter+Compute), default 1 */
  int32_t use_degree;           /* degree test, default 1 */
  int32_t use_ne;               /* neighbourhood-encoding test, default 1 */
  int32_t rows_on_device;       /* the rows argument of gsm_match is device memory */
  void *hip_stream;             /* hipStream_t to run on; NULL = the null stream */
  int32_t root_qvertex;         /* -1 = no slice; else keep f(root) with */
  uint32_t root_mod, root_rem;  /*   splitmix64(f(root)) % root_mod == root_rem */
  gsm_emit_fn emit;             /* optional row sink, called once per output chunk */
  void *emit_ctx;
  gsm_stats *stats;             /* optional */
  int32_t tile_items;           /* pairs per thread per tile: 1, 2, 4, 8 (0 = 4) */
  int32_t wg_size;              /* threads per workgroup: 128, 256, 512 (0 = 512) */
  int32_t profile;              /* time each expansion launch with HIP events into stats */
  uint32_t flags;               /* GSM_MATCH_* tuning flags */
  uint64_t batch_heavy_pairs;   /* gsm_match_batch: a query whose first level has more
                                   (row, neighbour) pairs runs on launches of its own
                                   (0 = 2^18; UINT64_MAX = never) */
  uint32_t stage_bytes;         /* LDS bytes an expansion launch may use to stage its tile's
                                   input and output rows (0 = 48 KiB; at most 64 KiB): a launch
                                   shape, results unchanged */
} gsm_match_opts;

/* Write output rows straight from registers instead of staging them in LDS. */
#define GSM_MATCH_NO_OUTPUT_STAGING 1u
/* Leave the rows written to gsm_match's rows buffer in ascending
 * lexicographic order (the order of the oracle's result set); with
 * GSM_E_TRUNCATED the rows_cap rows kept are sorted among themselves.  Costs
 * device memory beyond the frontier budget, see gsm_sort_rows.  Not valid
 * with an emit callback (GSM_E_UNSUPPORTED). */
#define GSM_MATCH_SORT_ROWS 2u
/* One-step look-ahead (Sec. 3.3, k-look-ahead, k = 1) in the verification of
 * every level that writes rows: a new row is dropped when some later query
 * neighbour of the vertex just placed can no longer find an image among that
 * data vertex's neighbours (too few of its label, or none that is a candidate
 * outside the row).  Pure pruning: the result is unchanged. */
#define GSM_MATCH_LOOKAHEAD 4u
/* Two-step look-ahead (Sec. 3.3, k-look-ahead, k = 2; implies
 * GSM_MATCH_LOOKAHEAD): the neighbour found for a later query neighbour must
 * itself have, for each label among that query vertex's own neighbours, at
 * least as many neighbours of that label (the four labels with most such
 * neighbours are tested; labelled graphs with the label table only).  Pure
 * pruning: the result is unchanged. */
#define GSM_MATCH_LOOKAHEAD2 64u
/* gsm_match_batch: run every level of a group of queries with sizes read back
 * to the host between levels (the chunked path) instead of device-driven. */
#define GSM_MATCH_HOST_LEVELS 128u
/* gsm_match_batch: enqueue the device-driven levels directly instead of
 * capturing them once in a HIP graph and replaying it. */
#define GSM_MATCH_NO_GRAPH 256u
/* Unique-subgraph mode: one embedding per subgraph of the data graph that
 * the query maps onto (the paper's way of producing each node combination
 * once by visiting equivalent query nodes in increasing id order, Sec. 3.3).
 * Embeddings f and f o s, s an automorphism of the query, are one subgraph;
 * the one kept satisfies the ordering constraints that gsm_query_symmetry
 * returns (compared in the graph's internal order on a graph created with
 * GSM_GRAPH_DEGREE_ORDER).  count = (count without the flag) / |Aut(Q)|.  Single-query
 * matching only (gsm_match_batch returns GSM_E_UNSUPPORTED). */
#define GSM_MATCH_UNIQUE 8u
/* Induced semantics (the other reading of subgraph isomorphism, Sec. 1):
 * query vertices that are not adjacent must map to data vertices that are
 * not adjacent either.  Every earlier non-neighbour of a new query vertex
 * costs one more membership search per surviving pair.  Combines with the
 * other flags; single-query matching only. */
#define GSM_MATCH_INDUCED 16u
/* Packed frontier (the paper's compact storage of partial results, Sec. 3.2
 * and 3.3, read as a reversible encoding): rows of the intermediate levels
 * are stored as b-bit ids laid end to end in 32-bit words, b = bit width of
 * n - 1, at every level where that takes fewer words than ids (e.g. 4 ids of
 * a 2^21-vertex graph in 12 bytes instead of 16) and the level's rows can be
 * staged whole in LDS.  Rows are decoded exactly, so the
 * result is unchanged; more rows fit a memory budget.  Single-query matching
 * only. */
#define GSM_MATCH_PACK_FRONTIER 32u

/* Fills defaults (struct_size set, budget 0, rounds 1, degree and NE on, no slice). */
void gsm_match_opts_init(gsm_match_opts *o);

/*
 * Candidate sets of the filtering stage (Alg. 1 Filter_candidate_set):
 * cmask[v] bit u is set when data vertex v is a candidate of query vertex u:
 * labels equal, deg(v) >= deg(u), NE(v) >= NE(u) where NE(x) sums (label+1)
 * over x's neighbours, then filter_rounds refinement rounds recomputing deg
 * and NE over neighbours that are still candidates of some query vertex.
 *   cmask  host array of n uint16 (query-vertex-id bits)
 */
gsm_status gsm_filter(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint16_t *cmask);

/*
 * Counts, and optionally lists, the embeddings of qh in g.
 *   opts          NULL = defaults
 *   count         out: exact number of embeddings (also on GSM_E_TRUNCATED)
 *   rows          NULL = count only; else rows_cap rows of q int32 (host,
 *                 or device when opts->rows_on_device)
 *   rows_written  out, may be NULL: rows stored = min(count, rows_cap)
 * Returns GSM_E_TRUNCATED (count still exact) when count > rows_cap.
 * With opts->emit set, rows are handed to the callback chunk by chunk
 * instead (rows may be NULL).
 */
gsm_status gsm_match(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint64_t *count,
                     int32_t *rows, uint64_t rows_cap, uint64_t *rows_written);

/*
 * gsm_match for callers that cannot allocate device memory: code that must
 * not call hipMalloc (tight serving loops, harnesses that forbid it, work
 * recorded around HIP graph capture).  Same arguments, results and errors as
 * gsm_match; no device memory is allocated or freed by the call, nor by any
 * library routine it calls.
 * Every buffer of the call (candidate masks, level frontiers, scans, output
 * staging, counters) lives in one device array of
 * GSM_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends.  Limits:
 *   - the graph's candidate masks and first frontier must fit:
 *     29 n + 4 KiB bytes plus 28 KiB of fixed overhead, so n up to about
 *     2.2 million vertices; a larger graph returns GSM_E_BUDGET with the sizes
 *     in gsm_last_error();
 *   - opts->memory_budget_bytes is capped at what the array holds (frontier
 *     chunks are smaller than with gsm_match, so large outputs take more
 *     launches; results are identical);
 *   - GSM_MATCH_SORT_ROWS returns GSM_E_UNSUPPORTED (sort with gsm_sort_rows,
 *     which allocates), opts->profile is ignored.
 * Calls on one device share its array and are serialised inside the library
 * (a call waits for the previous one); the array keeps the last call's
 * contents, and every call clears its counters before use.  Two processes
 * each have their own array.  Rows handed to an emit callback point into the
 * array and are valid only during the callback.
 */
#define GSM_NOALLOC_SCRATCH_BYTES (64ull << 20)
gsm_status gsm_match_noalloc(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint64_t *count,
                             int32_t *rows, uint64_t rows_cap, uint64_t *rows_written);

/*
 * Sorts nrows rows of q int32 ids (row-major) into ascending lexicographic
 * order in place, on the device, on the graph's stream-ordered workspace
 * (the embedding list of Alg. 1 output M, as a sorted set).
 *   rows            host memory, or device memory when rows_on_device
 *   q               1..16 columns
 *   ids must lie in [0, n) of g; other values give an unspecified order but
 *   never an access outside the buffers.
 * Device memory used: 16 * ceil(q*b/64) bytes per row, b = bit width of n-1,
 * plus 4*q bytes per row when rows are on the host; it stays with the graph
 * for reuse.  Waits for the sort before returning.  GSM_E_OOM when the
 * buffers cannot be allocated.
 */
gsm_status gsm_sort_rows(gsm_graph_t g, int32_t *rows, uint64_t nrows, int32_t q, int32_t rows_on_device,
                         void *hip_stream);

/*
 * The smallest memory_budget_bytes gsm_match accepts for qh on g: the first
 * frontier (up to n rows), the candidate masks, and one row of every further
 * level (and of the output staging buffer when rows go to the host).
 *   host_rows  non-zero when rows will be delivered through host memory
 */
gsm_status gsm_match_min_budget(gsm_graph_t g, gsm_query_t qh, int32_t host_rows, uint64_t *bytes);

/*
 * Counts the embeddings of nq queries on one graph.  Queries whose first level
 * is small share launches, grouped by size: their rows, tagged by query, form
 * one frontier per level, so one first-frontier launch and, per level, one
 * scan and one expansion launch serve a whole group (chunked by the budget
 * like one query).
 * Queries above opts->batch_heavy_pairs first-level pairs run on launches of
 * their own, where a query-uniform kernel is faster.  counts[k] equals
 * gsm_match's count for qs[k].
 * A group runs device-driven: every level's launches are enqueued at once and
 * read the level's row count and pair total from device memory, each level
 * expanded in one chunk at its capacity from the budget, and queries whose
 * pairs at some level pass batch_heavy_pairs are taken out of the shared
 * launches on the device (and counted alone afterwards).  The launch sequence
 * is captured once in a HIP graph and replayed by later calls that ask for
 * the same work on the same buffers (GSM_MATCH_NO_GRAPH: enqueue directly).
 * When some level's pairs pass its capacity the group is redone level by
 * level with sizes read back and chunks (GSM_MATCH_HOST_LEVELS: always).  A root slice in opts (root_qvertex,
 * root_mod, root_rem) applies to every query (root_qvertex must be below
 * every query's size).  No rows or emit callback.
 */
gsm_status gsm_match_batch(gsm_graph_t g, int32_t nq, const gsm_query_t *qs,
                           const gsm_match_opts *opts, uint64_t *counts);

/* ---------------------------------------------------------------- serving -- */

/*
 * A serving engine over one resident graph (continuous batching): queries are
 * submitted as they arrive and counted by worker threads, each with its own
 * HIP stream.  A worker keeps several batched runs in flight and advances
 * them in turn one step at a time (a level's scan or one chunk's expansion);
 * between any two steps it admits the oldest waiting queries that fit the
 * device memory still free (each query reserves its frontier estimate: its
 * first level's neighbour total for its second vertex's label times the row
 * size, clamped to [what it needs alone, per_query_budget]) and starts them
 * as a new run, queries of one size sharing launches (a run of one query
 * uses the faster query-uniform kernels of gsm_match).  A query whose level
 * pairs pass batch_heavy_pairs leaves its shared run and continues in a run
 * of its own, so one exploding query does not hold back the others.  Runs of
 * different workers overlap on the device.  The memory-bounded expansion
 * keeps every run within its reservation.
 */
typedef struct gsm_server_opts {
  uint32_t struct_size;
  uint64_t arena_bytes;       /* device memory shared by in-flight queries (0 = 16 GiB) */
  uint64_t per_query_budget;  /* largest reservation of one query (0 = 4 GiB) */
  int32_t workers;            /* worker threads / streams (0 = 2) */
  int32_t max_batch;          /* queries per batch (0 = 64) */
  int32_t max_active;         /* queries admitted at once (0 = 1024) */
  int32_t wg_size, tile_items;
  uint64_t batch_heavy_pairs; /* as in gsm_match_opts */
} gsm_server_opts;

typedef struct gsm_result {
  gsm_status status;
  uint64_t count;
  uint64_t t_submit_ns, t_admit_ns, t_done_ns; /* steady-clock nanoseconds */
  int32_t batch_size;                          /* queries in the run that finished it */
  int32_t worker;                              /* worker (stream) that ran it */
  double dev_start_ms, dev_end_ms;             /* device time of its run's first and last work, in ms
                                                  since gsm_server_create (HIP events on the worker's
                                                  stream; runs of different workers that overlap in
                                                  these times ran on the device at the same time) */
} gsm_result;

void gsm_server_opts_init(gsm_server_opts *o);
/* The graph must outlive the server. */
gsm_status gsm_server_create(gsm_graph_t g, const gsm_server_opts *opts, gsm_server_t *out);
/* Copies the query (the caller may destroy it on return); *ticket identifies the request. */
gsm_status gsm_server_submit(gsm_server_t srv, gsm_query_t qh, uint64_t *ticket);
/* gsm_server_submit restricted to a root slice (the gsm_match_opts
 * convention): only embeddings with splitmix64(f(root_qvertex)) % root_mod ==
 * root_rem are counted; root_qvertex < 0 = no slice.  Slices of one query
 * over all residues partition its embeddings, so a large query can be served
 * as root_mod independent requests.  GSM_E_INVALID_ARG unless
 * root_qvertex < q and root_rem < root_mod. */
gsm_status gsm_server_submit_slice(gsm_server_t srv, gsm_query_t qh, int32_t root_qvertex, uint32_t root_mod,
                                   uint32_t root_rem, uint64_t *ticket);
/* Waits for a ticket (timeout_ms < 0: forever) and releases it.  GSM_E_TIMEOUT if not done. */
gsm_status gsm_server_wait(gsm_server_t srv, uint64_t ticket, int32_t timeout_ms, gsm_result *out);
/* Finishes the admitted work, stops the workers, frees everything. */
void gsm_server_destroy(gsm_server_t srv);
/* Steady-clock time in nanoseconds (the clock of gsm_result's timestamps). */
uint64_t gsm_now_ns(void);

/* ----------------------------------------------------------------- errors -- */

const char *gsm_status_str(gsm_status s);

/* ---------------------------------------------------------------- testing -- */

/* Failure injection for tests of the error paths: after `after` more device
 * allocations by the library, every further one fails (the call then returns
 * GSM_E_OOM) until this is called again with after < 0.  Process-wide. */
void gsm_testing_fail_allocations(int64_t after);
const char *gsm_last_error(void); /* thread-local; "" when none */

#ifdef __cplusplus
}
#endif

#endif /* GSM_H */
