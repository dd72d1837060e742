/* dawn_host.h — DAWN's SOVM level loop on the host's CPU cores.
 *
 * The paper evaluates DAWN on a multi-core CPU as well as on a GPU (the
 * "DAWN(20)" configuration of its evaluation, and the thread-efficiency
 * measurement of its scalability section).  This library is that CPU
 * configuration: the sparse-vector x CSR step of Section 3.3 (Algorithm 2):
 * the next frontier is the union of the frontier nodes' out-lists minus the
 * nodes already reached, each new node taking the level number as its
 * distance, level by level until a level adds nothing.  It is separate from
 * the GPU library (libdawn) and from the test oracle, and nothing in libdawn
 * calls it.
 *
 * Results are the same as libdawn's: for a source s, dist[v] is the length of
 * a shortest directed path s -> v along out-edges (Theorem 1), dist[s] = 0,
 * and -1 where no path exists.
 *
 * Status codes are libdawn's: 0 ok, -1 invalid argument, -2 bad graph.
 * Every call is thread-safe; a graph handle may be used by several calls at
 * once.
 */
#ifndef DAWN_HOST_H
#define DAWN_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dawn_host_graph dawn_host_graph;

typedef struct {
  int32_t levels;        /* max distance + 1 over the rows computed */
  int64_t source_edges;  /* sum over rows of the out-degrees of the reached nodes */
  int64_t reached;       /* (row, node) pairs with a distance */
  double ms;             /* wall time of the call */
} dawn_host_stats;

/* Wrap a CSR graph: row_ptr int32[n+1], col int32[m], host memory.  The
 * arrays are validated (row_ptr[0] = 0, non-decreasing, row_ptr[n] = m, every
 * col entry in [0, n)) and referenced, not copied: they must stay valid and
 * unchanged until dawn_host_graph_destroy.  *out receives the handle.
 * Errors: -1 (null pointer, n <= 0, m < 0), -2 (invalid CSR). */
int32_t dawn_host_graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                               dawn_host_graph** out);
int32_t dawn_host_graph_destroy(dawn_host_graph* g);

/* One source with `threads` worker threads (1 .. 256) sharing each level:
 * every level's frontier is cut into blocks that the threads take in turn; a
 * target is claimed by an atomic OR on its visited bit, and the claimer
 * writes dist and appends the node to its own list of the next frontier.
 * dist: int32[n], caller-owned; untouched on error.  stats may be NULL.
 * Errors: -1 (null graph/dist, source outside [0, n), threads outside
 * 1 .. 256). */
int32_t dawn_host_sssp(const dawn_host_graph* g, int32_t source, int32_t threads, int32_t* dist,
                       dawn_host_stats* stats);

/* k sources (row r of dist, int32[k][n], is sources[r]), spread over
 * `threads` threads, each running one source at a time single-threaded.
 * k = 0 is a no-op.  Errors as dawn_host_sssp (also a null sources array
 * with k > 0, or a source outside [0, n)). */
int32_t dawn_host_mssp(const dawn_host_graph* g, const int32_t* sources, int32_t k, int32_t threads,
                       int32_t* dist, dawn_host_stats* stats);

/* Message of the calling thread's last error ("" if none). */
const char* dawn_host_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
