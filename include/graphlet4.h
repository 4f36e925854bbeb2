/*
 * graphlet4 -- batch fully dynamic counting of all induced 4-vertex
 * graphlets on one AMD MI355X (gfx950).
 *
 * What is computed.  For a simple undirected graph G = (V, E) on a fixed
 * vertex set V = {0..n-1}, the eleven counts
 *     I_c = |{ S subset of V : |S| = 4, G[S] isomorphic to class c }|
 * indexed by gc_class below: the six connected induced 4-graphlets of Fig. 1
 * of the paper (3-path g1, 3-star g2, 4-cycle g3, tailed triangle g4,
 * diamond g5, 4-clique g6) and the five disconnected graphs on four vertices.
 * Problem 1 asks to maintain these under batches B = A u D of edge
 * insertions A and deletions D, giving the counts of (V, E + A - D).
 *
 * How.  Alg. 2 (FDGC): per batch the library marks the region of change
 * around the changed pairs, counts its graphlets before (G_b) and after
 * (G_a) the batch with a per-edge static counter (triangles, 4-cliques,
 * 4-cycles and combinatorics) in one fused pass on the GPU, adds C_a - C_b
 * to the maintained connected counts (Lemma 2) and then applies the batch to
 * the resident graph.  The five disconnected classes are not local; they
 * follow from the connected counts and the global totals n, m,
 * W = sum_v C(deg v, 2) and the triangle count, which are maintained too.
 *
 * Batch semantics (stream model of Sec. 3, batch protocol of Sec. 6):
 *   - (u, v) and (v, u) name the same edge; self loops are ignored;
 *   - repeated pairs inside the insertions (or the deletions) collapse;
 *   - a pair that is both inserted and deleted by one batch is dropped and
 *     leaves the graph unchanged;
 *   - inserting an existing edge or deleting a missing one has no effect;
 *   - an id outside [0, n) rejects the whole batch (GC_EINVAL) and leaves
 *     the graph and its counts unchanged (after gc_add_vertices /
 *     gc_remove_vertices: an id not issued, or of a removed vertex).
 *
 * Conventions.  Every function returns GC_OK (0) or a negative gc_status,
 * and gc_last_error() describes the cause (thread-local string).  On error
 * the graph is unchanged, with one exception: a device failure (GC_EDEVICE,
 * or GC_ENOMEM while growing scratch) once a call has started to merge a
 * batch into the resident graph, or a static recount has started to mark it,
 * leaves the handle unusable, and every later call on it returns GC_ESTATE.  Input arrays are borrowed for the duration of the
 * call only: host arrays are copied before the call returns; device arrays
 * (the _dev variants) must stay valid until the call returns.  A handle owns
 * all of its device memory; it is not re-entrant (one call at a time per
 * handle), distinct handles may be used from distinct threads.
 *
 * Counts are int64.  For n > 121977 the empty class exceeds 2^63 - 1: its
 * int64 value is then the low 64 bits (two's complement) and bit c of the
 * overflow mask is set; gc_get_counts_exact returns every class exactly as a
 * 128-bit (hi, lo) pair.
 */
#ifndef GRAPHLET4_H
#define GRAPHLET4_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gc_graph gc_graph;

typedef enum {
  GC_OK = 0,
  GC_EINVAL = -1,   /* bad argument or vertex id out of range */
  GC_ENOMEM = -2,   /* device or host allocation failed */
  GC_EDEVICE = -3,  /* HIP runtime error, or no usable gfx950 device */
  GC_EBUSY = -4,    /* server queue full */
  GC_ESTATE = -5    /* handle unusable after an earlier device failure */
} gc_status;

typedef enum {
  GC_P4 = 0,       /* 3-path (g1) */
  GC_STAR = 1,     /* 3-star (g2) */
  GC_C4 = 2,       /* 4-cycle (g3) */
  GC_PAW = 3,      /* tailed triangle (g4) */
  GC_DIAMOND = 4,  /* diamond (g5) */
  GC_K4 = 5,       /* 4-clique (g6) */
  GC_TRI_ISO = 6,  /* triangle + isolated vertex */
  GC_P3_ISO = 7,   /* 2-path + isolated vertex */
  GC_2K2 = 8,      /* two disjoint edges */
  GC_K2_2ISO = 9,  /* one edge + two isolated vertices */
  GC_EMPTY = 10,   /* no edge */
  GC_NUM_CLASSES = 11
} gc_class;

typedef struct {
  /* Region of change: vertices within `radius` hops of a changed pair,
   * counted on the subgraph they induce.  Alg. 2 uses 3-hop balls; 2 hops
   * already contain every 4-vertex set that holds a changed pair and is
   * connected in either version, so 2 is exact and the default.  0 counts
   * the whole graph (also exact).  1 is NOT exact and exists only so that
   * tests can show that the region matters. */
  int32_t radius;
  /* Free space left in every adjacency row when it is (re)built, as a
   * fraction of its length (default 0.25). */
  float slack;
  /* HIP device ordinal (default 0). */
  int32_t device;
  /* hipStream_t to run on (NULL = the library's own stream). */
  void* stream;
  /* 1 (default): online autotuning of speed knobs; results never change.
   * The first five passes that count a region (rather than edge-locally)
   * each try one density threshold of the hub windows of the 4-cycle count
   * and the fastest per wedge is kept; the next five try the tier
   * thresholds (tri_small_max below).  Per
   * batch-size decade, once the region of change covers >= 90% of the graph,
   * later batches of that size count the whole graph (same result, no
   * marking): this measured switch takes the place of a fixed "whole graph
   * above this percentage" option.  Per half-decade of batch size, the
   * edge-local and the region kinds of pass are chosen by their measured
   * times (the delta option).  0: the defaults, nothing measured. */
  int32_t autotune;
  /* 1 (default): a host-array pass without statistics runs as one HIP graph:
   * the whole pass (upload, ingest, merge, region, counting, purge, result
   * download) is captured the first time a pass of its shape is enqueued and
   * replayed afterwards.  The shape is the number of batches, the capacity
   * classes of the batch sizes (powers of two), the region mode, the tuned
   * knobs and the scratch buffers; a pass whose scratch has to grow runs
   * directly and is captured anew.  0: every pass launches its kernels one
   * by one.  Results are identical either way. */
  int32_t graphs;
  /* Edge-local passes (one batch per graph of a pass only): instead of
   * counting the region of change before and after, enumerate only the
   * structures that contain a changed pair (triangles, 4-cliques and
   * 4-cycles through each changed edge, the edges whose triangle count
   * changed), each once from its changed pair of smallest key, with the
   * triangles at every vertex kept on the device.  Same counts; far less
   * work for small batches, more for very large ones.  0 (default): per
   * batch-size decade the faster kind as measured (with autotune), 1:
   * always, -1: never. */
  int32_t delta;
  /* Vertex ids reserved for gc_add_vertices (single-graph handles): the
   * resident rows and per-vertex arrays are sized for this many ids, so
   * that adding vertices up to it costs no device work.  0 (default) or
   * any value <= n: n.  Beyond it, gc_add_vertices rebuilds the graph over
   * a larger id space. */
  int64_t vertex_capacity;
  /* Tier thresholds of the counting kernels (speed only; results never
   * depend on them): the largest out-degree counted by the one-wave
   * triangle tier (at most 64, the slots of its bit matrices), and the
   * largest wedge bound counted by the one-wave and by the one-workgroup
   * 4-cycle tiers (at most 256 and 4096, half their hash tables).  Vertices
   * above a threshold go to the next tier up.  0 (default): with autotune,
   * five passes that count a region anyway try (64, 256, 4096), a triangle
   * threshold of 32, a one-wave 4-cycle threshold of 128 and one-workgroup
   * thresholds of 2048 and 1024 (after the hub-window trials), and keep the
   * fastest per unit of work
   * (triangle entries read, wedges); without, the maxima.  Nonzero: fixed
   * (an unset one takes its maximum); GC_EINVAL outside [1, max], or with
   * c4_mid_max below c4_small_max. */
  int32_t tri_small_max, c4_small_max, c4_mid_max;
} gc_options;

typedef struct {
  int64_t offered_ins, offered_del;  /* as submitted */
  int64_t eff_ins, eff_del;          /* effective insertions / deletions */
  int64_t loops, dups, cancelled, ins_existing, del_missing;
  int64_t touched_vertices;          /* endpoints of effective changes */
  int64_t region_vertices, region_entries;  /* region size (entries = 2 x edges) */
  int64_t wedges;                    /* 4-cycle wedges enumerated */
  int64_t c4_entries_small, c4_entries_mid, c4_entries_large;  /* adjacency entries read per 4-cycle tier */
  int64_t c4_tail_wedges;            /* wedges of the large tier counted in the global tail (below the windows) */
  int64_t max_out_degree;
  int64_t tier_tri_small, tier_tri_large, tier_c4_small, tier_c4_mid, tier_c4_large;  /* vertices per tier */
  int64_t c4_dense_min;              /* hub-window density threshold used */
  int32_t whole_graph;               /* 1: counted the whole graph instead of the region */
  uint32_t overflow_mask;            /* classes whose count left int64 */
  int32_t pass_batches;              /* batches that shared the counting pass (1: one batch per graph) */
  float ms_total;                    /* wall time of the call */
  float ms_prepare;                  /* ingest, merge, region, per-vertex pass (device): one figure, as they
                                        run back to back with no event between them */
  float ms_tri, ms_edge;             /* triangle/4-clique kernels, edge pass (device) */
  float ms_c4_small, ms_c4_mid, ms_c4_large;  /* 4-cycle tiers (device) */
  float ms_finish;                   /* combine + purge (device) */
  int64_t c4_windows;                /* dense LDS windows of the large 4-cycle tier */
  int64_t c4_searches;               /* cursor visits of that tier (lower neighbours x window passes) */
  int64_t tri_global_vertices;       /* vertices whose out-degree exceeds the LDS triangle tiers (global scratch) */
  int64_t tri_exc_rebuilds;          /* triangle-tier vertices counted once per version (too many version-specific edges) */
  int32_t retries;                   /* counting stages run again after growing scratch for a larger vertex */
  int32_t delta;                     /* 1: the pass was edge-local (gc_options.delta) */
  int64_t tri_entries;               /* adjacency entries read by the triangle tiers (N+(u) and each N+(v) probed) */
  int32_t tri_small_max, c4_small_max, c4_mid_max;  /* tier thresholds of the pass (gc_options) */
  int64_t k4_split_edges;            /* edge-local: changed edges whose 4-cliques were spread over workgroups */
} gc_batch_stats;

/* One batch for one graph of a pool (host pointers). */
typedef struct {
  const int32_t* ins_src; const int32_t* ins_dst; int64_t n_ins;
  const int32_t* del_src; const int32_t* del_dst; int64_t n_del;
} gc_batch_desc;

/* Fills *opt with the defaults (radius 2, slack 0.25, device 0, own stream). */
int gc_options_default(gc_options* opt);

/* Builds the resident graph on n vertices from m edge pairs (src[i],
 * dst[i]) (host arrays; loops ignored, repeats collapse) and returns its
 * counts.  Following Alg. 2's initialisation (F = 0), this is one batch
 * inserting every edge into the empty graph on n vertices.
 * n must be in [1, 2^28); opt may be NULL; counts may be NULL. */
int gc_graph_init(int64_t n, const int32_t* src, const int32_t* dst, int64_t m,
                  const gc_options* opt, gc_graph** out, int64_t counts[11]);

/* Several independent graphs in one handle ("pool"; a batched interface of
 * this library: the paper maintains one graph): graph g has n[g]
 * vertices and m[g] edges.  Batches for all of them are then applied
 * together by gc_apply_batches (one pass of device work for all graphs).
 * counts (k x 11) may be NULL. */
int gc_pool_init(int32_t k, const int64_t* n, const int32_t* const* src, const int32_t* const* dst,
                 const int64_t* m, const gc_options* opt, gc_graph** out, int64_t (*counts)[11]);

/* Applies one batch (host arrays) to a single-graph handle and returns the
 * counts after it (Problem 1).  stats may be NULL. */
int gc_apply_batch(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins,
                   const int32_t* del_src, const int32_t* del_dst, int64_t n_del,
                   int64_t counts[11], gc_batch_stats* stats);

/* Same with device arrays (int32, on the handle's device): the batch of
 * Problem 1 already resident in HBM.  An interface of this library, not of
 * the paper; the ids are checked on the device, before anything changes. */
int gc_apply_batch_dev(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins,
                       const int32_t* del_src, const int32_t* del_dst, int64_t n_del,
                       int64_t counts[11], gc_batch_stats* stats);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture of the caller's own work, tight serving loops, harnesses that
 * forbid hipMalloc): gc_apply_batch_dev with no allocation in the call: no
 * hipMalloc, hipFree or pinned memory, and on success no host heap memory
 * either (only an error path allocates its message).  The batch's
 * staging (keys, merge lists, per-row work arrays; at most 64 MiB) lives in
 * one static device array per GPU, which the library holds until the process
 * ends; every other buffer is the handle's own and must already be large
 * enough.  Limits: the staging, 72 (c_i + c_d) + 32 c_i + 64 c_d bytes with
 * c_i, c_d the numbers of insertions and deletions rounded up to powers of
 * two (at least 64), must fit the 64 MiB array -- every batch of at most
 * 262144 insertions and 262144 deletions does (GC_EINVAL beyond, nothing
 * changed); a graph whose resident rows, region
 * view or counting scratch would have to grow for this batch is refused with
 * GC_ENOMEM and left unchanged, and so is a batch after which a vertex
 * outgrows the counting scratch (its merge is undone on the device) -- one
 * gc_apply_batch_dev call of that size grows the handle's buffers.  Results
 * are those of gc_apply_batch_dev.  Single-graph handles only.  The static
 * array is shared by every handle on a device: calls that overlap in time on
 * one GPU (from several host threads) race and must not be made. */
int gc_apply_batch_dev_noalloc(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins,
                               const int32_t* del_src, const int32_t* del_dst, int64_t n_del,
                               int64_t counts[11], gc_batch_stats* stats);

/* Applies batch[g] to graph g of a pool, for all k graphs at once; counts
 * is k x 11 (may be NULL).  The batches are independent; the result for
 * each graph equals k separate gc_apply_batch calls. */
int gc_apply_batches(gc_graph* pool, const gc_batch_desc* batch, int64_t (*counts)[11],
                     gc_batch_stats* stats);

/* Applies nb batches (host arrays) to a single-graph handle in order, each
 * to the graph the previous one left, exactly as nb gc_apply_batch calls
 * would; counts[j] (nb x 11, may be NULL) receives the counts after batch
 * j, stats[j] (nb entries, may be NULL) its statistics.  Up to three
 * batches share one counting pass: Lemma 2 applied to G_0 and each G_j,
 * with the region of change taken in the union of G_0 .. G_j (a superset of
 * each version's region, so exact) and every adjacency entry marking the
 * versions its edge belongs to.  Whether they do: with autotune and
 * automatic pass kinds (gc_options.delta = 0), when the measured cost of
 * such a pass is below that of the batches one by one (each then
 * edge-local where that is faster; while nothing is measured, batches of at
 * most 1000 updates run alone); always with delta = -1 or without autotune;
 * never with delta = 1.  Results are the same either way.  The arrays of
 * all nb batches are checked first: one id outside [0, n) rejects the
 * whole call with GC_EINVAL and leaves the graph unchanged. */
int gc_apply_batch_seq(gc_graph* g, const gc_batch_desc* batches, int32_t nb, int64_t (*counts)[11],
                       gc_batch_stats* stats);

/* Current counts of graph `graph` (0 for a single-graph handle): the
 * frequencies Problem 1 maintains, for the six connected classes of Fig. 1,
 * and the five disconnected classes derived from them and n, m, W, T. */
int gc_get_counts(const gc_graph* g, int32_t graph, int64_t counts[11], uint32_t* overflow_mask);
int gc_get_counts_exact(const gc_graph* g, int32_t graph, int64_t hi[11], uint64_t lo[11]);

/* The four induced 3-vertex counts of graph `graph`, exactly (128-bit
 * hi/lo pairs), in the order gc_class3: Sec. 3 notes that the static
 * per-edge counter finds the size-3 graphlets along with the size-4 ones.
 * They follow from the totals maintained for the disconnected 4-vertex
 * classes: triangles T, 2-paths W = sum_v C(deg v, 2) (a triangle holds
 * three), edges m and n.  No device work. */
typedef enum { GC3_TRIANGLE = 0, GC3_PATH = 1, GC3_EDGE_ISO = 2, GC3_EMPTY = 3 } gc_class3;
int gc_get_counts3(const gc_graph* g, int32_t graph, int64_t hi[4], uint64_t lo[4]);

/* Static recount of graph `graph` from scratch on the GPU (the baseline of
 * Sec. 4.1); does not change the maintained counts.  For checking. */
int gc_recount_exact(gc_graph* g, int32_t graph, int64_t hi[11], uint64_t lo[11]);

/* Vertex insertion and deletion (Sec. 3: vertex operations reduce to edge
 * operations, a vertex losing its incident edges before it leaves V).
 * Single-graph handles only; the vertex count n of the disconnected
 * classes is that of the live vertices.
 *
 * gc_add_vertices adds `count` isolated vertices with the next unused ids
 * first_id .. first_id + count - 1 (ids are never reused; the first call
 * after gc_graph_init on n vertices returns first_id = n) and returns the
 * counts (they change through n only).  Within gc_options.vertex_capacity
 * this is host bookkeeping; beyond it the edges are read back and the graph
 * is built again over max(needed, 2 x capacity) ids (external ids and
 * counts kept; a failure there leaves the handle unusable).  count = 0 only
 * reports first_id.  GC_EINVAL if ids would reach 2^28.
 *
 * gc_remove_vertices deletes every edge at the `count` listed vertices as
 * one batch (the rules, statistics and failure behaviour of gc_apply_batch;
 * stats may be NULL) and then takes the vertices out of V: n falls by
 * count, and their ids are rejected by every later batch (GC_EINVAL, as
 * for ids out of range; the device-array variants report them like other
 * invalid ids).  GC_EINVAL, with nothing changed, for an id not yet issued,
 * already removed or listed twice. */
int gc_add_vertices(gc_graph* g, int64_t count, int64_t* first_id, int64_t counts[11]);
int gc_remove_vertices(gc_graph* g, const int32_t* ids, int64_t count, int64_t counts[11], gc_batch_stats* stats);

/* Number of graphs, vertices (live ones) and edges. */
int gc_graph_info(const gc_graph* g, int32_t* num_graphs, int32_t graph, int64_t* n, int64_t* m);

/* Copies the edges of graph `graph` (each once, external ids) into host
 * arrays of capacity cap; *m_out = edge count (GC_EINVAL if cap < m).
 * Library interface (for checking and persistence), not in the paper. */
int gc_export_edges(gc_graph* g, int32_t graph, int32_t* src, int32_t* dst, int64_t cap, int64_t* m_out);

/* Estimated device bytes a single-graph handle built from this edge list
 * reaches (resident rows with slack, region view, per-edge triangle counts,
 * hub counters, multi-version passes, the transient arrays of the build),
 * from the same sizing rules the library allocates by; batch staging is not
 * included.  Host arrays; needs no device.  The server's admission uses it.
 * Library interface, not in the paper. */
int gc_graph_footprint(int64_t n, const int32_t* src, const int32_t* dst, int64_t m, const gc_options* opt,
                       int64_t* bytes);

/* Diagnostics of the graphs option: passes captured as HIP graphs and
 * passes launched from a captured graph (replays included) so far
 * (library interface). */
int gc_graph_replays(const gc_graph* g, int64_t* captures, int64_t* launches);

/* Copies what the online autotuner of src has learned into dst: the
 * hub-window threshold and the tier thresholds with their trials (the tier
 * thresholds only when dst's are not fixed by gc_options.tiers), the
 * whole-graph switch per batch-size decade, the measured costs of region,
 * edge-local and multi-version passes, and the edge-local list demand per
 * update.  A new handle on the same or a similar graph then skips the trials
 * and starts from those measurements.  Speed knobs only: counts do not
 * change, whatever the two graphs.  Host state only (no device work); call
 * it while neither handle is in use by another thread.  GC_EINVAL for a
 * NULL handle (library interface, not in the paper). */
int gc_copy_tuning(gc_graph* dst, const gc_graph* src);

/* Frees the handle and its device memory (library interface). */
int gc_graph_free(gc_graph* g);

/* ------------------------------------------------------------- serving
 * (A serving interface of this library; no passage of the paper defines
 * it.  Each batch is still applied by Alg. 2 as gc_apply_batch does.)
 * A server keeps graphs resident on one device, each with its own stream and
 * worker thread, and answers asynchronously submitted update batches through
 * tickets.  Batches for different graphs run at the same time (their kernels
 * overlap on the device); batches for one graph are applied in submission
 * order, and each ticket's result is the counts right after its batch, the
 * same as gc_apply_batch would return in that order.  Continuous batching:
 * when a graph's worker becomes free it takes up to three queued batches of
 * that graph into one gc_apply_batch_seq call, which folds them into one
 * counting pass when that is measured to be faster; a batch that fails
 * the host-side id check fails alone.  Admission by memory:
 * a graph is admitted only if its footprint (gc_graph_footprint) fits the
 * free HBM (hipMemGetInfo, or, when hbm_budget_bytes > 0, that budget minus
 * the footprints of the graphs already admitted) minus hbm_reserve_bytes,
 * else GC_ENOMEM; a batch starts only while the estimated bytes of batches in
 * flight stay within batch_budget_bytes (one batch always runs).  A server
 * may be used from several host threads. */
typedef struct gc_server gc_server;

typedef struct {
  int32_t device;              /* HIP device (default 0) */
  int32_t max_graphs;          /* resident graphs (default 64) */
  int64_t hbm_reserve_bytes;   /* kept free when admitting a graph (default 8 GiB) */
  int64_t hbm_budget_bytes;    /* > 0: use this instead of the device's free memory */
  int64_t batch_budget_bytes;  /* bytes of batches in flight (default 4 GiB) */
} gc_server_opts;

int gc_server_opts_default(gc_server_opts* opts);
int gc_server_create(const gc_server_opts* opts /* NULL = defaults */, gc_server** out);

/* Builds a resident graph (as gc_graph_init; opt->stream is ignored) and
 * returns its id.  GC_ENOMEM: refused by memory admission; GC_EBUSY: full. */
int gc_server_add_graph(gc_server* s, int64_t n, const int32_t* src, const int32_t* dst, int64_t m,
                        const gc_options* opt, int32_t* graph_id);

/* Queues one batch (host arrays, copied before return) for a graph. */
int gc_server_submit(gc_server* s, int32_t graph_id, const gc_batch_desc* batch, uint64_t* ticket);

/* Blocks until the ticket's batch is applied; returns its status and, when
 * the pointers are non-NULL, the counts after it, its statistics, and
 * latency_ms[0] = submit -> result, latency_ms[1] = submit -> start.
 * A ticket can be waited on once. */
int gc_server_wait(gc_server* s, uint64_t ticket, int64_t counts[11], gc_batch_stats* stats,
                   double latency_ms[2]);

/* Exact counts of a graph once every batch submitted for it is applied. */
int gc_server_counts(gc_server* s, int32_t graph_id, int64_t hi[11], uint64_t lo[11]);

/* Finishes the queued batches, stops the workers and frees every graph. */
int gc_server_destroy(gc_server* s);

const char* gc_strerror(int code);
const char* gc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GRAPHLET4_H */
