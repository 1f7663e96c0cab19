/* dbbc.h -- exact counting of balanced and unbalanced butterflies in signed
 * bipartite graphs on AMD Instinct MI355X (gfx950).
 *
 * A butterfly (Definition 1) is a 2x2 biclique {u, u'} x {v, v'} of a
 * bipartite graph G = (U, V, E).  With edge signs s: E -> {+1, -1} it is
 * balanced (Definition 2) when its number of negative edges is even, i.e.
 * when the product of its four signs is +1, and unbalanced otherwise.  The
 * library computes, exactly, the number of balanced butterflies (the
 * problem statement of Section III), the number of unbalanced ones, their sum
 * (the unsigned butterfly count) and the number of vertex-priority wedges the
 * method walks (Algorithm 1, Phase 5, with the vertex priority of
 * Definition 3), optionally per vertex.
 *
 * Conventions shared by every entry point:
 *   - Vertex ids: u in [0, n_u) on side U and v in [0, n_v) on side V, two
 *     separate id spaces.  For the tie-break of Definition 3 (equal degrees:
 *     the larger id has the higher priority) vertex v of V has id n_u + v.
 *     Counts do not depend on the tie-break (Theorem 1).  n_u + n_v < 2^30
 *     and every per-side edge count below 2^31 - 1.
 *   - Signs: int8 values +1 (positive) or -1 (negative).  The paper's edge
 *     records use 1 for positive and 0 for negative; callers map 0 to -1.
 *   - Duplicate (u, v) pairs: the last occurrence in input order wins (the
 *     paper keeps the latest interaction, Section V); the number dropped is
 *     reported.  DBBC_DUP_REJECT turns any duplicate into DBBC_E_DUPLICATE.
 *   - Errors: every int-returning call returns DBBC_OK (0) or a negative
 *     status; on error no output is written and dbbc_last_error() holds a
 *     message for the calling thread.
 *   - Streams: hip_stream is a hipStream_t (NULL = the null stream).  Device
 *     work is ordered on it; calls that return host results synchronise it.
 *   - Threads: distinct handles may be used from different threads at once.
 *     One handle owns its scratch memory, so calls on the same handle must
 *     not overlap (the caller serialises them).
 */
#ifndef DBBC_H
#define DBBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define DBBC_OK 0
#define DBBC_E_INVALID_ARG (-1) /* NULL pointer, negative size, bad flag */
#define DBBC_E_ID_RANGE (-2)    /* u not in [0, n_u) or v not in [0, n_v) */
#define DBBC_E_SIGN (-3)        /* sign not +1 or -1 */
#define DBBC_E_DUPLICATE (-4)   /* duplicate pair under DBBC_DUP_REJECT */
#define DBBC_E_OOM (-5)         /* host or device allocation failed */
#define DBBC_E_DEVICE (-6)      /* a HIP call or kernel launch failed, or a kernel or the planner
                                   reported a broken internal bound (dbbc_last_error says which) */
#define DBBC_E_TOO_LARGE (-7)   /* sizes beyond the limits stated above */
#define DBBC_E_NO_DEVICE (-8)   /* no gfx950 device visible */
#define DBBC_E_PARSE (-9)       /* malformed record in an edge-list text */

/* ---- flags for dbbc_graph_create ---------------------------------------- */
#define DBBC_INPUT_DEVICE 0x1u /* u, v, sign point to device memory */
#define DBBC_DUP_REJECT 0x2u   /* fail on duplicate pairs instead of dropping */

typedef struct dbbc_graph dbbc_graph; /* opaque; owns its device memory */

/* Exact results of one count. */
typedef struct {
  int64_t balanced;   /* butterflies with an even number of negative edges */
  int64_t unbalanced; /* butterflies with an odd number of negative edges */
  int64_t total;      /* all butterflies (= balanced + unbalanced) */
  int64_t wedges;     /* vertex-priority wedges of the graph (W_VP): wedges
                         u-v-w with v and w both of lower priority than u */
} dbbc_counts;

/* Facts about a built graph (host memory, filled by dbbc_graph_stats). */
typedef struct {
  int64_t n_u, n_v, m;      /* vertices per side, distinct edges kept */
  int64_t dups_dropped;     /* input records dropped as duplicates */
  int64_t max_deg_u, max_deg_v;
  int64_t device_bytes;     /* device memory held by the handle */
  int64_t wedges_vp;        /* W_VP, computed in closed form at build time */
  int64_t pivots_active;    /* pivots that walk at least one wedge */
} dbbc_stats;

/* Tuning knobs for a count.  Pass NULL for the library's defaults (chosen
 * from the graph's statistics).  Every setting gives the same exact counts;
 * only the work split and speed change. */
typedef struct {
  int32_t hub_T;    /* side of the dense hub block counted with int8 MFMA:
                       the T highest-priority vertices of each side (a
                       multiple of 128, at most window_L); 0 turns
                       the dense path off; -1 = default */
  int32_t window_L; /* per side, the L highest-priority vertices whose pair
                       counts are kept in on-chip direct arrays; a multiple
                       of 256 in [256, 32768]; -1 = default */
  int32_t reverse_L; /* per side, the R highest-priority vertices counted
                        from the low-priority end of their pairs; a multiple
                        of 64 in [64, 4096], at most window_L; -1 = default */
  int32_t small_work; /* work items with at most this many wedges (at most
                         512) are packed into groups counted with
                         per-wavefront hash counters; -1 = default */
  int32_t part_work;  /* wedge budget per work part of a high-priority
                         pivot; -1 = default */
  int32_t long_len;   /* CSR runs of at least this many entries are streamed
                         by a whole wavefront with 16-byte loads; shorter
                         runs are packed end to end across the wavefront's
                         lanes; in [16, 65536]; -1 = default */
  uint32_t flags;     /* DBBC_OPT_* bits */
} dbbc_options;

/* dbbc_options.flags: record HIP events around every kernel of a count on
 * the count's stream; read them back with dbbc_last_kernel_times. */
#define DBBC_OPT_TIME_KERNELS 0x1u
/* dbbc_options.flags, per-edge pass: keep every edge's credits in two 64-bit
 * words (the form the pass uses for edges that may lie in 2^32 or more
 * butterflies) instead of one packed word; for testing the two forms. */
#define DBBC_OPT_WIDE_EDGES 0x2u
/* dbbc_options.flags, counts and the per-vertex and per-edge passes: make
 * the plan with the host planner (a copy of the graph's arrays to host
 * memory, then loops over its pivots) instead of the device planner's
 * kernels; both split the same wedges into work items (Algorithm 1, Eq. 1),
 * so the results are the same; for testing the two planners against each
 * other. */
#define DBBC_OPT_HOST_PLAN 0x4u

/* One kernel launch of the last timed count and the work it was given. */
typedef struct {
  char name[24];     /* "direct", "reverse", "small", "hash", "reduce", "hub" */
  float ms;          /* launch duration between its two HIP events */
  int64_t wedges;    /* vertex-priority wedges tallied by the launch */
  int64_t segments;  /* CSR runs (one per expanded edge) it walked */
  int64_t items;     /* work items (pivots, endpoints or pivot parts) */
  int64_t macs;      /* int8 multiply-accumulates (dense hub block only) */
} dbbc_kernel_time;

/* Where a handle's device memory comes from.  Every device allocation the
 * library makes for a handle (its CSR, plans, scratch and per-vertex / per-
 * edge buffers, and the temporary arrays of its build) goes through alloc,
 * and each such block is returned through free when the library no longer
 * needs it (at the latest in dbbc_graph_destroy).
 *   alloc(bytes, hip_stream, ctx): a block of at least bytes bytes of
 *       device memory, aligned to 256 bytes, usable on hip_stream (the
 *       stream of the call that allocates); NULL when none is available
 *       (the call then fails with DBBC_E_OOM)
 *   free(ptr, hip_stream, ctx): give back a block from alloc; hip_stream is
 *       the stream it was allocated for.  The library has waited for its own
 *       work on the block, except work enqueued on that stream.
 *   ctx: passed through.
 * Both functions are called on the thread of the library call that needs
 * them.  A NULL dbbc_allocator means hipMalloc / hipFree.  Pinned host memory
 * (a few words per handle or batch for results) does not go through it. */
typedef struct {
  void *(*alloc)(size_t bytes, void *hip_stream, void *ctx);
  void (*free)(void *ptr, void *hip_stream, void *ctx);
  void *ctx;
} dbbc_allocator;

/* Build a graph handle from an edge list.
 *   n_u, n_v  : vertices per side (> 0 each, n_u + n_v < 2^30)
 *   m         : number of input records (>= 0)
 *   u, v, sign: m int32 / int32 / int8 values each, host memory unless
 *               DBBC_INPUT_DEVICE; borrowed for the duration of the call
 *   flags     : DBBC_INPUT_DEVICE | DBBC_DUP_REJECT
 *   alloc     : the handle's device allocator for its whole life (copied;
 *               NULL = hipMalloc / hipFree); both functions must be set
 *   hip_stream: stream for the uploads
 *   out       : receives the handle (unchanged on error)
 * The degree-priority relabelling (Definition 3) and the rank-ordered CSR of
 * both sides are built here and kept on the device until destroy. */
int dbbc_graph_create(int32_t n_u, int32_t n_v, int64_t m, const int32_t *u, const int32_t *v,
                      const int8_t *sign, uint32_t flags, const dbbc_allocator *alloc, void *hip_stream,
                      dbbc_graph **out);

/* Build a graph handle from an edge list in text form, parsed on the device
 * (the paper's Phase 1 loading aligned to whole records and Phase 2 compact
 * identifiers, Section IV-A, on one GPU).
 *   text, len: the bytes (host memory, or device memory with
 *              DBBC_INPUT_DEVICE); len < 2^31 - 1.  One record per line:
 *              "u v s", fields separated by spaces, tabs or commas, "\n" or
 *              "\r\n" line ends; u and v decimal ids below 2^63 (the two
 *              sides are separate id spaces); s = 1 or +1 (positive), 0 or -1
 *              (negative), the paper's record format (Section III) with
 *              either sign convention; fields after the third are ignored;
 *              blank lines and lines starting with '#' or '%' are skipped.
 *   flags    : DBBC_INPUT_DEVICE | DBBC_DUP_REJECT (duplicates: as in
 *              dbbc_graph_create, in line order)
 *   alloc    : as for dbbc_graph_create
 *   info     : optional (host memory): lines and records read, n_u, n_v
 * Each side's distinct ids become the compact ids 0 .. n - 1 in increasing
 * raw id order; dbbc_graph_raw_ids returns the map.  Per-vertex outputs of
 * such a graph are in compact id order; per-edge outputs in record order
 * (the records being the non-skipped lines).  A malformed line fails with
 * DBBC_E_PARSE, its line number in dbbc_last_error(); a text without
 * records fails with DBBC_E_INVALID_ARG. */
typedef struct {
  int64_t lines, records; /* lines in the text, edge records among them */
  int64_t n_u, n_v;       /* distinct ids per side */
} dbbc_text_info;
int dbbc_graph_create_text(const char *text, int64_t len, uint32_t flags, const dbbc_allocator *alloc,
                           void *hip_stream, dbbc_graph **out, dbbc_text_info *info);

/* The raw id of every compact id of one side (side 0 = U, 1 = V) of a graph
 * made by dbbc_graph_create_text: n_side int64 values written to out
 * (caller-owned device memory), ascending.  DBBC_E_INVALID_ARG for a graph
 * made from id arrays (its ids are the compact ids). */
int dbbc_graph_raw_ids(const dbbc_graph *g, int32_t side, int64_t *out, void *hip_stream);

/* Copy the handle's statistics into *out (host memory). */
int dbbc_graph_stats(const dbbc_graph *g, dbbc_stats *out);

/* Count balanced and unbalanced butterflies (Algorithm 1 Phases 5 and 6,
 * Lemma 1; see the file comment).  opt may be NULL.  out_host: host memory,
 * written after the stream has drained. */
int dbbc_count(dbbc_graph *g, const dbbc_options *opt, dbbc_counts *out_host, void *hip_stream);

/* Per-vertex counts (Section I, Applications: the butterflies a vertex
 * participates in): for every vertex, the number of balanced and of
 * unbalanced butterflies that contain it.  A second pass walks each
 * priority-owned pair's wedges again once the pair's symmetric and
 * asymmetric counts p and n are known: the pair's two same-side vertices
 * each lie in C(p,2) + C(n,2) balanced and p n unbalanced of its
 * butterflies, a mid of a symmetric wedge in p - 1 balanced and n
 * unbalanced ones, a mid of an asymmetric wedge in n - 1 and p.  Every
 * vertex of U (and of V) is in 2 of each butterfly's 4 places, so the U
 * entries (and the V entries) sum to twice the global counts.
 *   opt      : window_L, reverse_L, small_work and long_len apply (NULL =
 *              defaults); there is no dense block in this pass
 *   bal_u, unb_u: n_u int64 values, bal_v, unb_v: n_v int64 values, in input
 *              id order, caller-owned device memory; any may be NULL; they
 *              are overwritten
 *   out_host : the global counts of the same pass (host memory, may be NULL)
 * The pass keeps a plan and four n-sized int64 arrays of its own on the
 * handle, beside those of dbbc_count. */
int dbbc_count_per_vertex(dbbc_graph *g, const dbbc_options *opt, int64_t *bal_u, int64_t *bal_v,
                          int64_t *unb_u, int64_t *unb_v, dbbc_counts *out_host, void *hip_stream);

/* Per-edge counts (Section I, Applications: the butterflies an edge takes
 * part in, the measure of the wing decomposition): for every input record i,
 * the number of balanced and of unbalanced butterflies that contain the
 * edge (u[i], v[i]).  The same pass as dbbc_count_per_vertex: a butterfly
 * of a pair is the union of two of the pair's wedges, so each edge of a
 * symmetric wedge lies in p - 1 balanced and n unbalanced butterflies of the
 * pair, each edge of an asymmetric wedge in n - 1 and p.  Each butterfly has
 * four edges, so the entries sum to four times the global counts.
 *   opt      : as for dbbc_count_per_vertex
 *   bal_e, unb_e: m int64 values each (m = the records passed to
 *              dbbc_graph_create, duplicates included), in input record
 *              order, caller-owned device memory; either may be NULL; they
 *              are overwritten.  A record dropped as a duplicate reads 0
 *              (the last record of the pair carries the edge's counts).
 *   out_host : the global counts of the same pass (host memory, may be NULL)
 * Besides the per-vertex pass's state, the handle keeps four int64 arrays
 * and two int32 maps of the edge count on the device. */
int dbbc_count_per_edge(dbbc_graph *g, const dbbc_options *opt, int64_t *bal_e, int64_t *unb_e,
                        dbbc_counts *out_host, void *hip_stream);

/* The baseline of the paper's symmetric / asymmetric wedge separation study
 * (Section V, Table IV), for measuring what Lemma 1's two buckets save: the
 * same vertex-priority wedges, but every pair of wedges of a vertex pair is
 * checked on its four signs one by one (work proportional to the
 * butterflies rather than the wedges).  Same results as dbbc_count (wedges =
 * W_VP); on graphs with many butterflies it is slow by design.  Keeps the
 * reverse positions and cuts of the CSR and per-workgroup scratch on the
 * handle's device memory while it runs. */
int dbbc_count_explicit(dbbc_graph *g, dbbc_counts *out_host, void *hip_stream);

/* For callers that cannot allocate (tight serving loops, harnesses that
 * forbid device allocation): the count of dbbc_count with no device or host
 * allocation of any kind.  g must already be planned for opt (by
 * dbbc_graph_plan, or by a dbbc_count with the same options); otherwise the
 * call fails with DBBC_E_INVALID_ARG and does nothing.  The buffers the
 * kernels write -- control words, side table, multi-part accumulators and
 * the dense block's hub-pair partials -- live in a file-scope device array of
 * DBBC_NOALLOC_SCRATCH_BYTES bytes of which each GPU the library runs on
 * holds one copy until the process ends; a count that needs more fails with
 * DBBC_E_TOO_LARGE (a smaller hub_T or window_L needs less).  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams or threads) race and must be serialised by the caller.  The
 * current device must be the graph's.  Results go to out_host (host memory)
 * once hip_stream has drained, as for dbbc_count; kernel timing is not
 * available.  Same counts as dbbc_count. */
#define DBBC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int dbbc_count_noalloc(dbbc_graph *g, const dbbc_options *opt, dbbc_counts *out_host, void *hip_stream);

/* Build the handle's counting plan for opt now (NULL = defaults), so that
 * the next count with the same options starts at once; returns when the plan
 * is on the device.  Counts re-plan by themselves when the options change. */
int dbbc_graph_plan(dbbc_graph *g, const dbbc_options *opt, void *hip_stream);

/* Asynchronous count: enqueue the same work as dbbc_count on hip_stream,
 * with the results copied to host memory owned by the handle, and return
 * without waiting.  Once the stream has passed this point (an event or a
 * stream synchronisation of the caller), dbbc_count_read(g, out_host) checks
 * and returns the results.  Until then no other call may use g.  Kernel
 * timing (DBBC_OPT_TIME_KERNELS) is not available here. */
int dbbc_count_async(dbbc_graph *g, const dbbc_options *opt, void *hip_stream);
int dbbc_count_read(dbbc_graph *g, dbbc_counts *out_host);

/* ---- batches: many graphs counted by one launch sequence ------------------ */

/* A batch counts k distinct graphs with one launch of each kernel: the
 * graphs' work lists are concatenated on the device and every item knows its
 * graph, so the kernels' persistent workgroups drain the work of all graphs
 * together and each graph's sums land in its own result slot.  Counts are
 * exactly those of dbbc_count on each graph alone (same plans, same
 * arithmetic).  With DBBC_BATCH_CAPTURE the launch sequence is captured once
 * into a HIP graph and each dbbc_batch_launch replays it.  A batch's own
 * device buffers come from the allocator of its first graph at creation
 * (hipMalloc for an empty batch); each graph's plan from the graph's. */
typedef struct dbbc_batch dbbc_batch;

#define DBBC_BATCH_CAPTURE 0x1u

/* Make a batch of the k graphs gs[0..k) (k >= 0, no handle twice).  opt
 * applies to every graph (NULL = defaults; kernel timing not allowed) and
 * plans each graph like dbbc_count would.  The batch borrows the handles:
 * they must outlive it, and a graph must not be counted or re-planned
 * elsewhere while the batch is in use (dbbc_batch_launch fails with
 * DBBC_E_INVALID_ARG if a graph was re-planned since).  hip_stream orders the
 * set-up copies; the call returns once they are done. */
int dbbc_batch_create(dbbc_graph *const *gs, int32_t k, const dbbc_options *opt, uint32_t flags,
                      void *hip_stream, dbbc_batch **out);

/* Re-target batch b at the graphs gs[0..k) (same rules as
 * dbbc_batch_create), reusing b's device and pinned buffers when they are
 * large enough: for request loops that form a new batch for every launch.
 * The previous launch of b must have completed.  On error b is left empty. */
int dbbc_batch_reset(dbbc_batch *b, dbbc_graph *const *gs, int32_t k, const dbbc_options *opt,
                     uint32_t flags, void *hip_stream);

/* Enqueue one count of every graph of the batch on hip_stream (replaying the
 * captured HIP graph if there is one) and the copy of the k results to host
 * memory owned by the batch; returns without waiting.  After the stream has
 * passed this point, dbbc_batch_read writes the k results (host memory, in
 * batch order) to out_host.  Launches of one batch must not overlap. */
int dbbc_batch_launch(dbbc_batch *b, void *hip_stream);
int dbbc_batch_read(const dbbc_batch *b, dbbc_counts *out_host);

/* dbbc_batch_launch, a synchronisation of hip_stream and dbbc_batch_read. */
int dbbc_batch_count(dbbc_batch *b, dbbc_counts *out_host, void *hip_stream);

/* Number of graphs in the batch (0 for NULL). */
int32_t dbbc_batch_size(const dbbc_batch *b);

/* Free the batch (NULL is a no-op); the graphs stay. */
void dbbc_batch_destroy(dbbc_batch *b);

/* One-shot batch: make an uncaptured batch of gs[0..k), count it into
 * out_host (k results, host memory) and free it. */
int dbbc_count_batch(dbbc_graph *const *gs, int32_t k, const dbbc_options *opt,
                     dbbc_counts *out_host, void *hip_stream);

/* Autotuner: picks the knobs of dbbc_options for the graphs gs[0..k)
 * counted together as a batch (k = 1 tunes one graph).  Starting from
 * *start (NULL = all defaults), a coordinate search visits the knobs in the
 * order long_len, small_work (hash versus direct counters), window_L (direct
 * array window, with reverse_L = min(window_L, 4096)), hub_T (the
 * high-degree block counted with int8 MFMA) and part_work, tries each value
 * of the knob's list with the others fixed, and keeps the fastest.  Every
 * try captures the batch into a HIP graph, replays it once to warm up and
 * times reps replays with HIP events on hip_stream.  Writes the winner to
 * *best and its time per batch in ms to *best_ms (may be NULL).  Every
 * candidate gives the same counts; only speed differs.  On return the
 * graphs are planned with *best (batches made before are invalidated). */
int dbbc_autotune(dbbc_graph *const *gs, int32_t k, const dbbc_options *start, int32_t reps,
                  void *hip_stream, dbbc_options *best, float *best_ms);

/* ---- request server: continuous batching over resident graphs ------------ */

/* A server keeps graphs resident on the device and answers count requests
 * on them from a scheduler thread of its own.  Whenever one of its launch
 * slots (a HIP stream each) is free, it takes the oldest waiting requests: a
 * graph with at least solo_wedges vertex-priority wedges is counted alone;
 * smaller graphs are packed, oldest request first, into one batch of at most
 * max_batch graphs and batch_wedges wedges.  Requests arriving while
 * launches run join the next free slot, so several launches overlap on the
 * device; requests for a graph already being counted wait for the next
 * launch, and requests for one graph waiting together share one count
 * (unless DBBC_SERVER_NO_MERGE: then every request is counted by a launch of
 * its own graph, one request per graph and launch).
 * Uploaded graphs are built by a worker thread and admitted against
 * hbm_budget (device bytes of all resident graphs): idle uploaded graphs are
 * evicted least recently used first; an upload that still does not fit is
 * rejected with DBBC_E_OOM.  Counts equal those of dbbc_count on each graph
 * alone. */
typedef struct dbbc_server dbbc_server;

typedef struct {
  int64_t hbm_budget;   /* device bytes for resident graphs; <= 0: 85% of the
                           free device memory at creation */
  int32_t slots;        /* launches in flight at once, 1..16; <= 0: 4 */
  int32_t max_batch;    /* graphs per batch; <= 0: 512 */
  int64_t solo_wedges;  /* graphs with at least this many wedges are counted
                           alone; <= 0: 2^26 */
  int64_t batch_wedges; /* a batch stops growing at this many wedges; <= 0:
                           2^28 */
  uint32_t flags;       /* DBBC_SERVER_* bits */
  int32_t reserved;     /* 0 */
} dbbc_server_config;

/* dbbc_server_config.flags: never let waiting requests for one graph share a
 * count (every request costs one count; for measuring served throughput on
 * equal work). */
#define DBBC_SERVER_NO_MERGE 0x1u

/* What happened to one request (times from dbbc_now_ns). */
typedef struct {
  int32_t status;       /* DBBC_OK or the request's error */
  int32_t graph_id;     /* graph counted (-1 for a rejected upload) */
  int32_t batch_size;   /* graphs in the launch that counted it (1 = alone) */
  int32_t queued_ahead; /* requests waiting when it arrived */
  int64_t t_submit_ns, t_launch_ns, t_done_ns;
} dbbc_request_info;

typedef struct {
  int64_t submitted, completed, failed, rejected, uploads, evicted;
  int64_t launches, batched_graphs; /* launches made and graphs they held */
  int64_t max_queue, queued;        /* waiting requests: peak and now */
  int64_t resident_graphs, resident_bytes;
} dbbc_server_stats;

/* Steady-clock time in ns (the clock of dbbc_request_info). */
int64_t dbbc_now_ns(void);

/* Start a server on the current device.  cfg and opt may be NULL (defaults;
 * opt applies to every count, kernel timing not allowed). */
int dbbc_server_create(const dbbc_server_config *cfg, const dbbc_options *opt, dbbc_server **out);

/* Build and plan a resident graph (host edge arrays, rules of
 * dbbc_graph_create); it is never evicted.  Writes its id.  May be called
 * from several threads at once. */
int dbbc_server_add_graph(dbbc_server *s, int32_t n_u, int32_t n_v, int64_t m, const int32_t *u,
                          const int32_t *v, const int8_t *sign, int32_t *graph_id);

/* Request a count of resident graph graph_id; writes a ticket. */
int dbbc_server_submit(dbbc_server *s, int32_t graph_id, int64_t *ticket);

/* Upload a new graph (host arrays, copied before return) and request its
 * count; writes a ticket.  The graph stays resident (evictable) afterwards. */
int dbbc_server_submit_upload(dbbc_server *s, int32_t n_u, int32_t n_v, int64_t m, const int32_t *u,
                              const int32_t *v, const int8_t *sign, int64_t *ticket);

/* Wait for a request; writes its counts and info (either may be NULL) and
 * forgets the ticket.  Returns the request's status. */
int dbbc_server_wait(dbbc_server *s, int64_t ticket, dbbc_counts *out, dbbc_request_info *info);

int dbbc_server_get_stats(dbbc_server *s, dbbc_server_stats *out);

/* Detail of the calling thread's last server error ("" if none). */
const char *dbbc_server_last_error(void);

/* Finish every accepted request, stop the threads, free all graphs. */
void dbbc_server_destroy(dbbc_server *s);

/* Kernel timings of the handle's last dbbc_count made with
 * DBBC_OPT_TIME_KERNELS.  Writes at most cap entries to out (host memory)
 * and the number available to *n_out.  Returns DBBC_E_INVALID_ARG if no timed
 * count has run on the handle. */
int dbbc_last_kernel_times(const dbbc_graph *g, dbbc_kernel_time *out, int32_t cap,
                           int32_t *n_out);

/* Free the handle and its device memory (NULL is a no-op). */
void dbbc_graph_destroy(dbbc_graph *g);

/* Static text for a status code. */
const char *dbbc_status_string(int status);

/* Detail of the calling thread's last error ("" if none). */
const char *dbbc_last_error(void);

/* Library version, e.g. "0.1.0". */
const char *dbbc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBBC_H */
