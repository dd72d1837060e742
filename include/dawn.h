/*
 * dawn.h — C ABI of libdawn: exact shortest-path lengths on unweighted
 * directed graphs, computed level by level on one AMD Instinct MI355X (gfx950).
 *
 * Method: DAWN (Feng et al., "DAWN: Matrix Operation-Optimized Algorithm for
 * Shortest Paths Problem on Unweighted Graphs", ICS '24).  Section 3.1
 * (Theorem 1, Fact 1) fixes the result: the distance from s to v is the
 * smallest k for which a length-k path s -> v exists, and every shortest path
 * of length k extends a shortest path of length k-1 by one edge.  Sections 3.2
 * (BOVM, Algorithm 1, pull over in-lists) and 3.3 (SOVM, Algorithm 2, push over
 * out-lists) give the level step; the loop stops when a level finds nothing
 * new (the stopping conditions after Equation 1).  APSP is the SSSP run from
 * every source (Section 3.3, APSP cost).
 *
 * Conventions for every call
 * --------------------------
 *  - Graphs are CSR: row u of `col` (entries row_ptr[u] .. row_ptr[u+1]-1)
 *    lists the targets of u's out-edges.  Node ids are int32 in [0, n).
 *    Self-loops and repeated edges are accepted and never change a distance.
 *  - Distances are int32: dist[s] = 0, dist[v] = shortest path length, and
 *    -1 when v is not reachable from s.  The paper's "0 = unvisited" would
 *    collide with dist[s] = 0, hence the separate -1.
 *  - Every call returns a dawn_status.  On any error the output buffers are
 *    left untouched and dawn_last_error() describes the failure (for errors
 *    found on the device by dawn_mssp_device, see there).
 *  - Unless DAWN_DEVICE_OUT is set, pointers are host memory.  With
 *    DAWN_DEVICE_OUT the distance buffer is device memory on the context's GPU
 *    (for example a torch tensor's data_ptr()); it is written on the device
 *    and no copy to the host is made.
 *  - Synchronous calls (everything except dawn_serve_submit and
 *    dawn_mssp_device) have finished writing their outputs when they return.
 *  - All calls are thread-safe on one context.  Calls on the same graph from
 *    several threads run on separate HIP streams.
 */
#ifndef DAWN_H
#define DAWN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status -- */
typedef int32_t dawn_status;
#define DAWN_OK             0
#define DAWN_PENDING        1   /* dawn_serve_poll: the query is still running */
#define DAWN_E_INVALID_ARG (-1) /* null pointer, n <= 0, k < 0, source outside [0, n), bad flag */
#define DAWN_E_BAD_GRAPH   (-2) /* row_ptr[0] != 0, decreasing row_ptr, row_ptr[n] != m, col outside [0, n) */
#define DAWN_E_NO_MEMORY   (-3) /* HBM budget exceeded or device allocation failed */
#define DAWN_E_DEVICE      (-4) /* HIP runtime error, or the level watchdog fired (more than n levels) */
#define DAWN_E_NOT_FOUND   (-5) /* unknown context/graph handle, unknown or retired ticket */
#define DAWN_E_BUSY        (-6) /* serving queue full: retry later */

/* ----------------------------------------------------------------- flags -- */
#define DAWN_DEVICE_OUT 0x1u    /* distance output is device memory */
#define DAWN_SHARED_CSC 0x2u    /* graph upload: the graph is symmetric, so its CSR also
                                   serves as its in-lists (no transpose is kept: 4(n+1+m)
                                   bytes less on the device).  Checked at upload (a
                                   non-symmetric graph gives BAD_GRAPH).  Pull steps then
                                   scan in-lists in CSR order. */

/* ----------------------------------------------------------------- types -- */
typedef struct dawn_ctx dawn_ctx;

/* Per-call statistics (all fields are outputs unless marked).
 * `levels` is max(dist) + 1 over the call's sources: the number of distance
 * values present (the source's level 0 included).  Each expansion step is a
 * push (top-down over the frontier's out-lists, Algorithm 2) or a pull
 * (bottom-up over unvisited nodes' in-lists with early exit, Algorithm 1).
 * `source_edges` is the sum over sources of the out-degrees of every reached
 * node: the SOVM cost E_wcc(s) of Section 3.3, the GTEPS numerator. */
typedef struct dawn_run_stats {
  int32_t levels;
  int32_t push_levels;        /* expansion steps run as push */
  int32_t pull_levels;        /* expansion steps run as pull */
  int32_t launches;           /* traversal kernel launches (driver 3: those queued, some of
                                 which may carry the final state only) */
  int64_t edges_examined;     /* adjacency entries read by expansion steps */
  int64_t source_edges;       /* sum over sources of sum of outdeg(u), u reached */
  int64_t reached;            /* sum over sources of reached nodes (sources included) */
  double kernel_ms;           /* device time of the traversal: HIP events around its kernels;
                                 dawn_sssp under driver 3 and for a source traversed by one
                                 workgroup (small_n): the GPU wall clock from the init
                                 kernel's start to the point the end was found (launches
                                 queued past the end are not counted) */
  double total_ms;            /* host wall time of the call */
  /* dawn_sssp only, optional inputs: when frontier_sizes is non-null it receives
   * the number of nodes found at level L (L = 0 .. min(levels, frontier_cap) - 1)
   * and, when directions is non-null, directions[L] = 1 for push, 2 for pull,
   * 0 for level 0. */
  int32_t *frontier_sizes;
  uint8_t *directions;
  int32_t frontier_cap;
  /* dawn_sssp with timing 1 only (output): the level launches' own durations,
   * each from its earliest workgroup start to its latest workgroup end by the
   * GPU's wall clock, summed (kernel_ms also counts each dispatch's set-up
   * and end-of-kernel cache write-back) */
  double kernel_clock_ms;
} dawn_run_stats;

/* Tuning knobs of one resident graph.  Every setting gives identical
 * distances; they change only speed.  0 (or 0.0) means "library default". */
typedef struct dawn_params {
  int32_t driver;             /* 1 persistent cooperative kernel (grid barrier per level),
                                 2 one launch per level with a host read-back,
                                 3 level launches queued in batches (the first sized from the
                                   graph's recent traversals, later ones `graph_levels`); the
                                   call returns once the launch that finds the end has
                                   reported to host memory, while launches queued past the
                                   end (they only carry the final state) may still run on
                                   the library's stream,
                                 4 the same launches captured once in a HIP graph and replayed */
  int32_t direction;          /* 1 push only, 2 pull only, 3 switch by alpha/beta */
  int32_t block;              /* threads per workgroup: 256, 512 or 1024 */
  int32_t blocks_per_cu;      /* workgroups per compute unit of the persistent kernel and of
                                 level launches (0: as many as a compute unit holds; level
                                 launches then use no more workgroups than a pull level has
                                 visited-bitmap words for, and at least one per compute unit) */
  int32_t big_degree;         /* push: out-degree at which a node's edges are spread over the grid */
  int32_t pull_lane_edges;    /* pull: in-edges one lane scans before its wave helps */
  float alpha;                /* switch push -> pull when frontier edges > unvisited edges / alpha */
  float beta;                 /* switch pull -> push when frontier nodes < n / beta */
  int32_t graph_levels;       /* drivers 3, 4: level launches per host read-back (rounded up to even) */
  int32_t small_n;            /* a source whose weakly connected component has
                                 <= min(small_n, 2048) nodes is traversed by one workgroup
                                 (0 = never; not when direction forces pull; default 512:
                                 on random components of mean degree 10 the one workgroup
                                 wins up to about 700 nodes, the level loop above) */
  float batch_alpha;          /* batched: pull when (sum over frontier nodes of out-degree x
                                 nonzero 64-lane words) * batch_alpha >= n x words, else push */
  int32_t batch_lanes;        /* batched: sources per launch (64..4096, multiple of 64) */
  int32_t timing;             /* 1: kernel_ms/launches of dawn_sssp cover only the level-step
                                 kernels, each timed by HIP events attached to its dispatch
                                 (driver 2 only);
                                 2 (default): every kernel of the call */
  int32_t batch_big_degree;   /* batched push: out-degree from which a frontier node's
                                 out-list is cut into 64-edge chunks spread over the grid
                                 (>= 64; default 64) */
  int32_t batch_wide_scan;    /* batched pull with rows of <= 8 words: in-list length above
                                 which the whole wave scans the list (1..512; default 48) */
  int32_t batch_sparse_words; /* batched push: a frontier node with at most this many nonzero
                                 64-lane words goes one edge per lane (1..4; default 4) */
  int32_t small_frontier_edges; /* single source, drivers 2-4: a push level whose frontier has
                                 at most this many out-edges (and at most `block`) runs on one
                                 workgroup, which also runs the small push levels after it in
                                 the same launch with their frontiers in LDS
                                 (default 1024; -1: never) */
  int32_t medium_edges;       /* single source, drivers 2-4: a push level whose frontier has
                                 more out-edges than such a one-workgroup level and at most
                                 this many runs on the first `medium_groups` workgroups of its
                                 launch, which also run the push levels after it that qualify,
                                 with a barrier between levels instead of a launch per level
                                 (default 0: never; that keeps the level kernel without this
                                 loop, which needs fewer registers) */
  int32_t medium_groups;      /* workgroups of such levels (2..256; default 32) */
} dawn_params;

typedef struct dawn_graph_info {
  int32_t n;
  int32_t max_out_degree;
  int64_t m;
  int32_t zero_out_degree;    /* nodes with no out-edge */
  int32_t s_wcc;              /* size of the largest weakly connected component, -1 until computed */
  int64_t device_bytes;       /* bytes held on the device for this graph (CSR + CSC + metadata) */
} dawn_graph_info;

typedef struct dawn_query_stats {
  uint64_t submit_ns;         /* CLOCK_MONOTONIC timestamps */
  uint64_t admit_ns;          /* lanes granted and sources seeded */
  uint64_t done_ns;           /* every row written (and copied to the host if requested) */
  int32_t levels;             /* max(dist) + 1 over the query's rows */
  int32_t status;             /* DAWN_OK, DAWN_PENDING or the error that ended the query */
  int32_t k;                  /* sources in the query */
  int32_t batch_peak;         /* most lanes the query's batch held at once while it ran */
} dawn_query_stats;

/* -------------------------------------------------------------- context -- */

/* Open device `device` (HIP ordinal).  hbm_budget_bytes caps the device memory
 * the context may hold (0 = 90% of the free memory, or $DAWN_HBM_BUDGET).
 * *out receives the handle.  Errors: INVALID_ARG, DEVICE. */
dawn_status dawn_create(int32_t device, uint64_t hbm_budget_bytes, dawn_ctx **out);

/* Stop the serving thread (pending queries end with DAWN_E_NOT_FOUND), free
 * every graph and buffer, and release the handle. */
dawn_status dawn_destroy(dawn_ctx *ctx);

/* Thread-local text of the last error raised on the calling thread ("" if none). */
const char *dawn_last_error(void);

/* Bytes currently held against the budget, and the budget itself. */
dawn_status dawn_memory(dawn_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* ---------------------------------------------------------------- graphs -- */

/* Copy a CSR graph to the device (the caller may free row_ptr/col on return),
 * build its in-lists (CSC: the transpose, which pull steps scan as BOVM does in
 * Section 3.2) and its out-degree metadata.  The CSR is validated first.
 * row_ptr: n+1 int32, col: m int32 (m = row_ptr[n] <= INT32_MAX), host memory.
 * *graph_out receives a handle >= 0.  flags: 0 or DAWN_SHARED_CSC (the
 * memory-frugal resident form of a symmetric graph).
 * Errors: INVALID_ARG (other flags), BAD_GRAPH, NO_MEMORY, DEVICE. */
dawn_status dawn_graph_upload(dawn_ctx *ctx, int32_t n, int64_t m,
                              const int32_t *row_ptr, const int32_t *col,
                              uint32_t flags, int32_t *graph_out);

/* Free a resident graph.  Waits for running calls on it.  Errors: NOT_FOUND. */
dawn_status dawn_graph_release(dawn_ctx *ctx, int32_t graph);

dawn_status dawn_graph_get_info(dawn_ctx *ctx, int32_t graph, dawn_graph_info *out);

/* Attach non-negative integer edge weights to a resident graph (copied:
 * weights[e], host, m int32, belongs to CSR entry e, the edge from e's row to
 * col[e]).  A second call replaces them.  Every path length must fit an int32
 * distance: max weight x (n - 1) <= 2^31 - 2.  Used by dawn_sssp_weighted
 * only.  Errors: INVALID_ARG (null, negative or too large weights),
 * NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_graph_set_weights(dawn_ctx *ctx, int32_t graph, const int32_t *weights);

/* Tuning knobs (see dawn_params).  set: fields left 0 keep the default;
 * invalid values give INVALID_ARG. */
dawn_status dawn_get_params(dawn_ctx *ctx, int32_t graph, dawn_params *out);
dawn_status dawn_set_params(dawn_ctx *ctx, int32_t graph, const dawn_params *in);

/* ------------------------------------------------------- shortest paths -- */

/* Single-source shortest path lengths (SSSP) from `source`: Algorithm 2 (push)
 * and Algorithm 1 (pull) level steps with a direction switch, until a level
 * finds no new node.  dist: n int32 (host, or device with DAWN_DEVICE_OUT).
 * stats may be NULL.  Errors: INVALID_ARG, NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_sssp(dawn_ctx *ctx, int32_t graph, int32_t source, int32_t *dist,
                      uint32_t flags, dawn_run_stats *stats);

/* Weighted single-source shortest paths: the paper's level loop over the
 * (min, +) semiring, which Section 5 names as future work.  dist[v] is the
 * least sum of weights over directed paths source -> v (int32, -1 when no
 * path exists), for the weights of dawn_graph_set_weights.  Each round
 * relaxes the out-edges of the nodes whose distance dropped in the previous
 * round (an atomic minimum per edge) until a round lowers nothing; a node may
 * join several rounds, so stats->levels counts rounds, which can exceed the
 * hop depth.  dist: n int32 (host, or device with DAWN_DEVICE_OUT); stats may
 * be NULL (edges_examined is not counted; source_edges and reached are as
 * for dawn_sssp).  Errors: INVALID_ARG (also: no weights attached),
 * NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_sssp_weighted(dawn_ctx *ctx, int32_t graph, int32_t source, int32_t *dist,
                               uint32_t flags, dawn_run_stats *stats);

/* Single-source run that allocates nothing, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same distances as dawn_sssp.  Every buffer of the
 * traversal lives in a static device array of 64 MiB that libdawn holds on
 * each GPU it runs on until the process ends; a graph whose traversal needs
 * more (about 128 n + m / 2 + 64 Ki bytes: n up to ~480,000 on sparse graphs)
 * is refused with INVALID_ARG.  d_dist: n int32 of device memory on the
 * context's GPU.  Work is queued on `hip_stream` (NULL: the null stream) and
 * the call returns when the distances are written (it reads the level state
 * back into host stack memory once per batch of level launches).  Calls that
 * overlap on one GPU share the array and race: the caller serialises them.
 * stats (may be NULL): as dawn_sssp, except kernel_ms = 0 (no events).
 * Errors: INVALID_ARG, NOT_FOUND, DEVICE. */
dawn_status dawn_sssp_noalloc(dawn_ctx *ctx, int32_t graph, int32_t source, int32_t *d_dist,
                              void *hip_stream, dawn_run_stats *stats);

/* Multi-source: row r of dist (k x n int32, row-major) holds the distances
 * from sources[r] (host array of k ids; repeats allowed and give equal rows).
 * Up to `batch_lanes` sources share one bitmask batch: one bit per source in
 * 64-bit words per node, and one level step advances all of them (the level
 * step of Algorithms 1/2 applied per bit).  Each level's direction and the
 * end of the run are decided on the device; the host checks a batch once per
 * chunk of queued levels.  k == 0 is a no-op.
 * Errors: INVALID_ARG, NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_mssp(dawn_ctx *ctx, int32_t graph, const int32_t *sources, int32_t k,
                      int32_t *dist, uint32_t flags, dawn_run_stats *stats);

/* Device-ordered multi-source run: the same rows as dawn_mssp, with every step
 * queued on the caller's HIP stream `hip_stream` (NULL: the null stream) and
 * no wait on the host.  The call returns once the work is queued; work the
 * caller queues on the stream afterwards sees the finished rows.
 * d_sources: k int32 node ids in device memory on the context's GPU, read on
 * the device (k == 0 queues nothing but the status).  d_dist: k x n int32,
 * device memory, row r = distances from d_sources[r].  d_status (device int32,
 * may be NULL): written on the stream with DAWN_OK, DAWN_E_INVALID_ARG (a
 * source outside [0, n): no row is written) or DAWN_E_DEVICE (a run needed
 * more than min(n, 65535) levels, or its grid barrier timed out: rows of
 * earlier batches of 4096 sources may be written, later ones are not).
 * Levels are queued as separate launches up to the depth of the graph's last
 * finished run, then one cooperative kernel runs any further levels with a
 * grid barrier between steps; the level bit-planes are allocated for the
 * deepest possible run (min(16, bit_length(n)) planes of n x 64-lane words
 * per batch word, i.e. at most half the size of a full batch's rows).
 * Buffers stay owned by the caller and must stay valid until the stream has
 * run the work.  Not for stream capture (it waits on events and launches a
 * cooperative kernel).  Host-side errors (returned at once, nothing queued):
 * INVALID_ARG (null or non-device pointers, pointers on another GPU, buffers
 * smaller than k or k x n int32 within their allocation), NOT_FOUND,
 * NO_MEMORY, DEVICE.  Section 3.3: the multi-source run is the SSSP of every
 * source, each lane advancing by the level step of Algorithms 1 and 2. */
dawn_status dawn_mssp_device(dawn_ctx *ctx, int32_t graph, const int32_t *d_sources, int32_t k,
                             int32_t *d_dist, int32_t *d_status, void *hip_stream);

/* All-pairs over the largest weakly connected component (ties: the component
 * holding the smallest node id).  Reachability implies weak connectivity, so
 * every finite distance from a node of the component stays inside it; this is
 * the S_wcc x E_wcc APSP cost of Section 3.3.
 * wcc_nodes: host, capacity n: receives the component's nodes, ascending.
 * *s_wcc receives their count.  dist: s_wcc x s_wcc int32, row i / column j =
 * distance from wcc_nodes[i] to wcc_nodes[j]; pass dist = NULL to only query
 * the component.  Errors: INVALID_ARG, NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_apsp_wcc(dawn_ctx *ctx, int32_t graph, int32_t *wcc_nodes, int32_t *s_wcc,
                          int32_t *dist, uint32_t flags, dawn_run_stats *stats);

/* Time the candidate settings on `k` sample sources and keep the fastest for
 * this graph.  what: 1 = single-source knobs, 2 = batched knobs, 3 = both.
 * Every candidate's distances must equal those of the default settings
 * bit for bit, or it is discarded.  best (may be NULL) receives the result.
 * Errors: INVALID_ARG, NOT_FOUND, NO_MEMORY, DEVICE. */
dawn_status dawn_autotune(dawn_ctx *ctx, int32_t graph, const int32_t *sources, int32_t k,
                          uint32_t what, dawn_params *best);

/* --------------------------------------------------------------- serving -- */

/* Queue a multi-source query (same output as dawn_mssp: k x n int32 rows) and
 * return at once with *ticket.  A scheduler thread keeps one bitmask batch per
 * resident graph; at every level boundary it retires finished sources, then
 * admits waiting queries into free lanes while the HBM budget allows, so
 * queries that arrive while others run join the running batch (continuous
 * batching).  While a level runs the scheduler polls the device without
 * sleeping (one host core busy), for up to 2 ms after its last step, then
 * in 20 us sleeps.  The caller keeps `sources` only until the call returns, but must
 * keep dist_out valid and unread until dawn_serve_poll returns DAWN_OK.  A
 * device dist_out is written later on the server's own stream, in no order
 * with the caller's streams: work that writes it (a fill, say) must have
 * finished before this call (the Python binding synchronizes torch's current
 * stream first).
 * Errors: INVALID_ARG, NOT_FOUND, NO_MEMORY (the query can never fit),
 * BUSY (queue full). */
dawn_status dawn_serve_submit(dawn_ctx *ctx, int32_t graph, const int32_t *sources, int32_t k,
                              int32_t *dist_out, uint32_t flags, uint64_t *ticket);

/* DAWN_PENDING while the query runs; DAWN_OK once every row is written (the
 * ticket is then retired, and a second poll gives NOT_FOUND); or the error
 * that ended it.  qstats may be NULL. */
dawn_status dawn_serve_poll(dawn_ctx *ctx, uint64_t ticket, dawn_query_stats *qstats);

/* As dawn_serve_poll, but blocks until the query ends or timeout_ms passes
 * (then DAWN_PENDING).  timeout_ms < 0 waits without limit. */
dawn_status dawn_serve_wait(dawn_ctx *ctx, uint64_t ticket, int32_t timeout_ms,
                            dawn_query_stats *qstats);

#ifdef __cplusplus
}
#endif

#endif /* DAWN_H */
