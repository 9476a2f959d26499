/*
 * tg.h — C ABI of the MI355X graph library (libtg.so).
 *
 * The library runs the data-parallel hot path of a hybrid bulk-synchronous
 * (BSP) graph engine — Gharaibeh et al., "Efficient Large-Scale Graph
 * Processing on Hybrid CPU and GPU Systems" (TOTEM):
 *   - CSR partitions (section 4.3.1) built by degree centrality (section 6.2),
 *   - per-partition superstep kernels: BFS frontier expansion (section 6.3.2,
 *     Figure 11), SSSP relaxation (section 7.3, Figure 20), the PageRank pull
 *     gather (section 7.1, Figure 14) and Brandes betweenness built from the
 *     same superstep (section 7.2, Figure 18),
 *   - boundary messages reduced at the source partition (section 3.4,
 *     section 4.3.2) and exchanged with a host-thread partition over PCIe
 *     once per superstep (section 4.1).
 *
 * Conventions for every call:
 *   - Vertex ids at the ABI are the caller's original int32 ids in [0, V).
 *     V <= INT32_MAX; edge counts and offsets are int64.
 *   - Every function returns TG_OK (0) or a negative tg_status and, on error,
 *     sets a thread-local message readable with tg_last_error().  Output
 *     buffers are undefined after an error.  No C++ exception crosses the ABI.
 *   - Graphs and partitions are library-owned (opaque handles, freed with
 *     graph_free / partition_free).  Output buffers are caller-owned device
 *     memory (for example a torch tensor's data pointer).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Algorithm calls
 *     enqueue their kernels on it, so they are ordered after the caller's
 *     earlier work on that stream, and return only when the results are in
 *     the output buffer (host-blocking).
 *   - A partition holds per-call scratch memory; calls on one partition must
 *     not overlap (one host thread at a time per partition).
 */
#ifndef TG_H
#define TG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tg_graph tg_graph;         /* host-resident validated CSR     */
typedef struct tg_partition tg_partition; /* device (+host) partitions       */

typedef enum {
  TG_OK = 0,
  TG_EINVAL = -1,        /* malformed argument or graph                   */
  TG_ENOMEM = -2,        /* host or device allocation failed              */
  TG_EDEVICE = -3,       /* a HIP runtime call failed                     */
  TG_ERANGE = -4,        /* a result does not fit its output type         */
  TG_EUNSUPPORTED = -5,  /* the request needs data the graph does not have */
  TG_ETIMEOUT = -6       /* a wait ran out of time                        */
} tg_status;

/* Partitioning strategies of section 6.3.1: HIGH puts the highest-degree
 * vertices on the host, LOW the lowest-degree ones, RAND a random subset. */
enum { TG_PART_HIGH = 0, TG_PART_LOW = 1, TG_PART_RAND = 2 };

/* PageRank treatment of out-degree-0 vertices: UNIFORM spreads their rank
 * over all vertices (mass is conserved); DROP discards it. */
enum { TG_PR_DANGLING_UNIFORM = 0, TG_PR_DANGLING_DROP = 1 };

/* graph_load_csr flags */
#define TG_PTRS_DEVICE 0x1u /* the three arrays are device pointers          */
#define TG_VALIDATE 0x2u    /* check offsets, ids and weights (O(V + E))      */
#define TG_SYMMETRIC 0x4u   /* caller asserts u->v in E iff v->u in E (with
                               equal weights); checked when TG_VALIDATE     */

/* Level / distance value of an unreachable vertex. */
#define TG_INF INT32_MAX

/* Load a CSR graph (section 4.3.1: offsets array V and destination array E).
 *   row_offsets  [V+1] int64, row_offsets[0] == 0, non-decreasing,
 *                row_offsets[V] == num_edges.
 *   col_indices  [E] int32 destination ids in [0, V).
 *   weights      [E] int32 edge weights >= 1, or NULL (then sssp() returns
 *                TG_EUNSUPPORTED).
 * The arrays are copied; the caller keeps ownership.  Self-loops and
 * duplicate edges are kept as given.  With TG_PTRS_DEVICE the copy is a
 * device-to-host transfer enqueued on `stream`.
 * Errors: TG_EINVAL for a malformed graph (only detected with TG_VALIDATE,
 * except sizes and NULL pointers, which are always checked), TG_ENOMEM. */
int graph_load_csr(int64_t num_vertices, int64_t num_edges,
                   const int64_t *row_offsets, const int32_t *col_indices,
                   const int32_t *weights, uint32_t flags, void *stream,
                   tg_graph **out);

/* Partition a loaded graph by degree centrality (section 6.2) and place it
 * on the device.  Vertices are relabelled in order of decreasing out-degree
 * so that each degree bin (thread / wavefront / block / multi-block per
 * vertex) is a contiguous id range.
 *   strategy        TG_PART_HIGH, TG_PART_LOW or TG_PART_RAND.
 *   cpu_edge_share  alpha in [0, 1): share of the edges kept on host threads.
 *                   0 places the whole graph on the GPU.  For alpha > 0 the
 *                   host partition takes whole vertices, in strategy order,
 *                   until it holds at least alpha * E edges (section 6.3.1).
 *   seed            drives TG_PART_RAND only.
 *   tuning_json     a JSON object with any of "hub_min_deg", "block_min_deg",
 *                   "wave_min_deg", "g16_min_deg", "g4_min_deg", "hub_chunk"
 *                   and the launch-shape keys of partition_retune; keys it
 *                   leaves out take their built-in values ("{}" = all
 *                   built-in).  NULL: the autotuner's cached entry for this
 *                   device and graph, if there is one, else the built-in
 *                   values.  The cache is the file named by the environment
 *                   variable TG_TUNING_CACHE, else tuning_cache.json in the
 *                   directory of this library: a JSON object keyed
 *                   "<arch>:V2^<round(log2 V)>:deg<round(E/V)>:<sym|dir>"
 *                   (round to nearest, ties to even; sym when loaded with
 *                   TG_SYMMETRIC) whose values hold the tuning object under
 *                   "config".  partition_info reports the choice as
 *                   "tuning_source".
 * The graph must outlive the partition (the partition reads its host CSR).
 * Errors: TG_EINVAL, TG_ENOMEM, TG_EDEVICE. */
int partition_by_degree(const tg_graph *g, int strategy, double cpu_edge_share,
                        uint64_t seed, const char *tuning_json,
                        tg_partition **out);

/* Re-derive the degree bins and launch shapes of an existing partition from
 * a tuning object without rebuilding it (NULL restores the built-in values).
 * This is the autotuner's hook.  Keys (all optional, integers):
 *   degree bins  "hub_min_deg", "block_min_deg", "wave_min_deg",
 *                "g16_min_deg", "g4_min_deg" (decreasing), "hub_chunk"
 *                (edges per block of a hub);
 *   BFS          "bfs_do" (1: direction-optimizing steps), "bfs_alpha",
 *                "bfs_beta" (the switch thresholds), "bfs_lanes" (searches
 *                in flight, 1..4), "bfs_td_grid", "bfs_bu_grid" (blocks of
 *                the top-down and bottom-up steps), "bfs_graph" (1: chunks of
 *                supersteps captured once as HIP graphs and replayed; kernel
 *                timing off only); "bfs_lds_words",
 *                "bfs_grid", "bfs_lds_min_vblocks" for the top-down steps of
 *                betweenness and hybrid searches;
 *   SSSP         "sssp_delta" (0: plain frontier; > 0: near/far step),
 *                "sssp_lanes" (roots in flight, 1..8), "sssp_pull" (a
 *                superstep whose frontier holds more than this percentage
 *                of the edges pulls over in-edges; 0: never), "sssp_grid",
 *                "sssp_lds_verts", "sssp_xcd" (per-XCD destination classes),
 *                "sssp_packed" (1: relax from one 32-bit word per edge,
 *                id | weight << 24, which the partition keeps when every
 *                local id fits in 24 bits and every weight in 8),
 *                "sssp_ring" (1: the near/far step keeps active vertices
 *                in a ring of bucket bitmaps by distance and filters only
 *                the current bucket, when at most 16 buckets of width
 *                sssp_delta span the largest weight; 0: one far pile,
 *                rescanned every superstep), "sssp_split" (1, with the ring
 *                and packed rows: a bucket's vertices relax their edges
 *                lighter than sssp_delta while it is processed and their
 *                heavier edges once when it is done), "sssp_hpull" (100,
 *                with the split on a TG_SYMMETRIC graph: that heavy pass
 *                is pulled by the vertices whose distance is not yet final
 *                when their out-degree sum times sssp_hpull / 100 is below
 *                the bucket's; 0: always pushed);
 *   layout       "mapped_edges" (1: the edge arrays -- neighbour ids, weights,
 *                in-edge ids -- stay in pinned host memory mapped into the
 *                GPU and kernels read them over the host link, for graphs
 *                beyond device memory; honoured by partition_by_degree only,
 *                and it keeps the per-XCD class layouts off);
 *   PageRank     "pr_xcd" (per-XCD source classes), "pr_rows" (256 or 512
 *                edges per row block), "pr_lds_verts" (hot-table entries,
 *                <= 40960), "pr_grid" (workgroups).
 * Results do not depend on the tuning.  Waits for the device to be idle
 * first.  Errors: TG_EINVAL (bad tuning), TG_ENOMEM, TG_EDEVICE. */
int partition_retune(tg_partition *p, const char *tuning_json);

/* Level-synchronous breadth-first search (section 6.3.2, Figure 11).  With
 * "bfs_do" (the default) a superstep whose frontier holds many edges runs
 * bottom-up instead: every unvisited vertex looks for an in-neighbour on the
 * frontier.  Levels are the same either way.
 *   roots     host array of num_roots original vertex ids.
 *   levels    device int32 [num_roots * V]; row r holds each vertex's hop
 *             count from roots[r] (TG_INF when unreachable).
 *   parents   NULL, or device int32 [num_roots * V]: parent[root] = root,
 *             -1 when unreachable, otherwise an in-neighbour one level up
 *             (the lowest such id in the partition's internal order).
 * Errors: TG_EINVAL (root out of range, NULL output), TG_ENOMEM, TG_EDEVICE. */
int bfs(const tg_partition *p, const int32_t *roots, int32_t num_roots,
        int32_t *levels, int32_t *parents, void *stream);

/* Batched BFS: the same result as bfs() (levels only), computed for up to 64
 * roots at a time in one chain of supersteps; every vertex carries one bit
 * per root in its visited / frontier masks, so an edge is streamed once per
 * superstep for all roots that have its source on their frontier.
 * GPU-only partitions (cpu_edge_share 0).  Same buffers and errors as bfs(),
 * plus TG_EUNSUPPORTED on a hybrid partition. */
int bfs_batched(const tg_partition *p, const int32_t *roots, int32_t num_roots,
                int32_t *levels, void *stream);

/* Single-source shortest paths (section 7.3, Figure 20: the superstep
 * relaxation of active vertices' out-edges) over the int32 weights given to
 * graph_load_csr.  The schedule is the tuning's: by default delta-stepping
 * with buckets of width "sssp_delta" kept in a ring of bitmaps
 * ("sssp_ring"), edges lighter than the width relaxed per pass and heavier
 * ones once per bucket ("sssp_split"), pulled instead of pushed on
 * TG_SYMMETRIC graphs when that touches fewer edges ("sssp_hpull");
 * "sssp_ring": 0 and "sssp_delta": 0 give the paper's frontier
 * Bellman-Ford.  Up to "sssp_lanes" roots run at once on library streams
 * and workspaces of their own.  The distances do not depend on any of
 * these.
 *   dist      device int32 [num_roots * V] (TG_INF when unreachable).
 * Errors: TG_EUNSUPPORTED (graph loaded without weights), TG_ERANGE (a
 * finite distance is >= INT32_MAX), TG_EINVAL, TG_ENOMEM, TG_EDEVICE. */
int sssp(const tg_partition *p, const int32_t *roots, int32_t num_roots,
         int32_t *dist, void *stream);

/* Batched SSSP: the same result as sssp(), up to 64 roots per chain of
 * supersteps with one distance per root per vertex ([V][64] int32 scratch),
 * including sssp()'s exact overflow verdict per root (TG_ERANGE names the
 * first root whose distances do not fit).  GPU-only partitions.  Same
 * buffers and errors as sssp(). */
int sssp_batched(const tg_partition *p, const int32_t *roots, int32_t num_roots,
                 int32_t *dist, void *stream);

/* PageRank by synchronous power iteration with a pull gather over in-edges
 * (section 7.1, Figure 14): r_0 = 1/V and
 *   r_{k+1}(v) = (1 - d)/V + d * (sum_{u->v} r_k(u)/outdeg(u) + D_k/V),
 * where D_k is the rank held by out-degree-0 vertices (UNIFORM) or 0 (DROP).
 *   rank      device float [V] receives r_iterations.
 * Ranks are fp32; sums are accumulated in fp64.
 * Errors: TG_EINVAL (damping outside [0, 1], iterations < 0, bad mode),
 * TG_ENOMEM, TG_EDEVICE. */
int pagerank(const tg_partition *p, float damping, int32_t iterations,
             int32_t dangling_mode, float *rank, void *stream);

/* Brandes betweenness centrality (section 7.2, Figure 18): a forward BFS
 * superstep counting shortest paths sigma (fp64, exact below 2^53) and a
 * backward superstep accumulating dependencies delta (fp32) with the
 * (1 + delta) term of Brandes' recurrence.
 *   sources   host array of num_sources original ids (repeats allowed).
 *   scores    device float [V]: sum over the given sources s of delta_s(v)
 *             for v != s — ordered pairs, not halved, not normalised.
 * On a hybrid partition both sides run each sweep: the forward sweep sends,
 * per boundary slot, the sum of sigma over the sender's vertices one level
 * up (the first time a slot has any); the level and sigma of the vertices
 * each side's boundary edges reach then cross once; the backward sweep
 * sends, per level, the deltas of those vertices.  Host deltas are summed
 * in fp64.
 * Errors: TG_EINVAL, TG_ENOMEM, TG_EDEVICE, TG_ERANGE (a path count reached
 * 2^53, beyond which fp64 counts are no longer exact). */
int bc(const tg_partition *p, const int32_t *sources, int32_t num_sources,
       float *scores, void *stream);

/* Connected components by minimum-label propagation (the fifth algorithm of
 * section 9.4, run on the undirected graph; labels are reduced by minimum,
 * section 3.4): every vertex starts with its own id and pushes any lower
 * label it receives to its neighbours until no label drops.
 *   labels    device int32 [V]: the smallest original vertex id of the
 *             vertex's component.  On a directed graph the components are
 *             the weak ones (labels cross edges in both directions).
 * GPU-only partitions (cpu_edge_share 0).
 * Errors: TG_EINVAL, TG_EUNSUPPORTED (hybrid partition), TG_ENOMEM,
 * TG_EDEVICE. */
int cc(const tg_partition *p, int32_t *labels, void *stream);

/* ------------------------------------------------------------- serving
 * A query server with continuous batching over resident graphs: BFS and SSSP
 * queries are admitted into a graph's 64-slot engine (see bfs_batched) as
 * slots and memory free up, joining at the next superstep while other
 * queries are in flight; each query's result is the same as a solo bfs() /
 * sssp() run.  One worker thread drives all graphs; each (graph, kind) has its
 * own stream so different graphs' supersteps overlap on the device.  SSSP
 * queries on a graph of at least sssp_solo_min_vertices vertices whose
 * largest out-degree is at least sssp_solo_min_skew times its mean degree
 * run instead as single searches (the sssp() schedule), up to the
 * partition's sssp_lanes (at most max_slots) at a time, each on its own host
 * thread, workspace and stream. */
typedef struct tg_server tg_server;
enum { TG_QUERY_BFS = 0, TG_QUERY_SSSP = 1 };

/* opts_json: NULL or {"max_slots": 1..64 (concurrent queries per graph and
 * kind; 1 = one query at a time), "memory_cap_bytes": N (device bytes that
 * running queries may hold; a query over the cap waits),
 * "sssp_solo_min_vertices": N (default 2^22), "sssp_solo_min_skew": X
 * (default 16; both 0 = every graph's SSSP queries run as single searches)}.
 * Errors: TG_EINVAL, TG_ENOMEM, TG_EDEVICE. */
int server_create(const char *opts_json, tg_server **out);

/* Register a GPU-only partition (cpu_edge_share 0); it must outlive the
 * server.  Errors: TG_EINVAL, TG_EUNSUPPORTED (hybrid partition). */
int server_add_graph(tg_server *s, const tg_partition *p, int32_t *graph_id);

/* Queue a query.  out: device int32 [V] owned by the caller, untouched by the
 * caller until server_wait returns for this ticket; receives levels (BFS) or
 * distances (SSSP) in original ids.  Errors: TG_EINVAL (bad graph, kind or
 * root), TG_EUNSUPPORTED (SSSP on an unweighted graph), TG_ENOMEM (a single
 * query exceeds the memory cap). */
int server_submit(tg_server *s, int32_t graph_id, int32_t kind, int32_t root,
                  int32_t *out, uint64_t *ticket);

/* Wait for a ticket (timeout_us < 0: no limit).  latency_us gets the time
 * from submission to the result being in `out`.  A ticket can be waited for
 * once.  Errors: TG_ETIMEOUT (not done yet; the ticket stays valid),
 * TG_EINVAL (unknown ticket), TG_ERANGE (an SSSP distance from this query's
 * root does not fit below INT32_MAX: the same verdict sssp() gives for that
 * root, independent of the other queries in flight), or the query's own
 * error. */
int server_wait(tg_server *s, uint64_t ticket, int64_t timeout_us, double *latency_us);

/* JSON counters: completed (queries finished, failed ones included),
 * supersteps (slot-engine supersteps), max_concurrent (most queries admitted
 * and not yet finished at once), waiting (queries not yet admitted),
 * memory_in_use (the device bytes the admitted queries hold, at most the
 * memory cap; 0 once every query has finished), max_slots; same return
 * convention as partition_info. */
int server_stats(tg_server *s, char *json, size_t cap);

/* Stop the worker after running queries finish; waiting queries are
 * dropped (their tickets are never completed). */
void server_destroy(tg_server *s);

/* Batched Brandes betweenness: the same result as bc() (within the stated
 * tolerance), up to 64 sources per chain of supersteps with vertex state laid
 * out [vertex][source] (sigma fp64, delta fp32, level int32: 16 B per vertex
 * and source of scratch).  Many small graphs run in one chain by loading
 * their disjoint union as one graph.  GPU-only partitions.  Same buffers and
 * errors as bc(), plus TG_EUNSUPPORTED on a hybrid partition. */
int bc_batched(const tg_partition *p, const int32_t *sources, int32_t num_sources,
               float *scores, void *stream);

/* Betweenness of many independent graphs in one call (section 5 runs each
 * algorithm over graphs of very different size; small graphs alone leave most
 * of the device idle).  Graph i's scores are those of bc_batched(parts[i],
 * sources[i], num_sources[i], scores[i]); graphs run concurrently, each on a
 * library stream of its own (at most 8 at a time, largest first), ordered
 * after earlier work on `stream`, and the call returns when every score is in
 * place.
 *   parts        num_graphs distinct GPU-only partitions (a partition may
 *                appear once: its scratch is used by the run).
 *   sources      per graph, a host array of num_sources[i] original ids.
 *   scores       per graph, device float [V_i].
 * Errors: as bc_batched, for the first graph that fails (its index is in the
 * message); TG_EINVAL for a repeated partition. */
int bc_multi(const tg_partition *const *parts, int32_t num_graphs, const int32_t *const *sources,
             const int32_t *num_sources, float *const *scores, void *stream);

void graph_free(tg_graph *g);
void partition_free(tg_partition *p);

/* Thread-local description of the last failing call on this thread. */
const char *tg_last_error(void);

/* JSON description of a partition: vertex/edge counts per side, degree-bin
 * boundaries, boundary (outbox/inbox) sizes with and without reduction, and
 * the space formula of section 4.3.3.  Returns the needed length (excluding
 * the terminator) or a negative tg_status. */
int partition_info(const tg_partition *p, char *json, size_t cap);

/* JSON statistics of the last algorithm call on this thread: supersteps,
 * edges scanned or relaxations, and on hybrid partitions per-phase
 * milliseconds (gpu_ms: the GPU's kernels; cpu_ms: the host threads;
 * exchange_ms: the copies of both directions on their copy streams), bytes
 * exchanged (exchange_bytes, of which exchange_h2d_bytes host-to-GPU) and
 * the local out-edges the host threads processed (cpu_edges; the boundary
 * edges of both sides are reduced on the GPU).  Same return convention as
 * partition_info. */
int tg_last_stats(char *json, size_t cap);

/* bfs() for callers that cannot allocate device memory: code under stream
 * capture, serving loops with a fixed memory budget, harnesses that forbid
 * hipMalloc.  The search's workspace lives in a file-scope device array of
 * 64 MiB inside the library (each GPU the library is loaded on holds one
 * until the process ends); the call allocates nothing, on the device or
 * pinned on the host.  A partition needs about 8.4 bytes per vertex plus
 * 70 KiB of it, so up to about 7.9 million vertices fit.
 *   p         a GPU-only partition (cpu_edge_share 0) on the current device.
 *   roots     host array of num_roots original vertex ids.
 *   levels    device int32 [num_roots * V], as bfs(); no parents.
 * Every call on a GPU shares that GPU's array: calls from this process are
 * serialized by a lock (the call returns when its levels are in place), and
 * each starts by clearing what must start at zero.  Errors: TG_EINVAL (bad
 * arguments, partition not on the current device), TG_EUNSUPPORTED (hybrid
 * partition), TG_ENOMEM (the partition needs more than the array holds; the
 * message gives the size), TG_EDEVICE. */
int bfs_noalloc(const tg_partition *p, const int32_t *roots, int32_t num_roots, int32_t *levels,
                void *stream);

/* Per-kernel timing: with on != 0, every timed kernel launch is bracketed
 * by HIP events on its stream and tg_last_stats() reports "<kernel>_ms"
 * (summed duration) and "<kernel>_n" (launches); the events themselves add
 * a few microseconds per launch.  The initial setting comes from the
 * TG_TIMING environment variable (unset or "0": off).  Process-wide; takes
 * effect for calls that start after it returns. */
void tg_set_timing(int on);

#ifdef __cplusplus
}
#endif

#endif /* TG_H */
