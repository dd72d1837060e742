/*
 * CPU oracle for unweighted shortest-path lengths — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this file's library.  It shares no code with the GPU library: no
 * headers, helpers or generated tables.
 *
 * What it computes (the plain definition, not DAWN's steps): for a source s,
 *   dist[v] = length of the shortest directed path s -> v along out-edges
 *             (row u of the CSR lists the targets of u's out-edges),
 *   dist[s] = 0, and dist[v] = -1 when no such path exists.
 * The paper's Theorem 1 (Section 3.1) states that DAWN's level loop returns
 * exactly these lengths; its Algorithm 3 (general BFS, Section 3.5) is the
 * textbook way to compute them.  This file is that BFS with a FIFO queue and
 * an explicit -1 sentinel: the paper's "distance = 0 means unvisited" would
 * collide with dist[s] = 0, so -1 is used instead.
 *
 * Also here: the largest weakly connected component (paper Section 3.3 uses
 * S_wcc / E_wcc in the SOVM cost), found by an undirected BFS sweep over
 * out- and in-edges.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* FIFO BFS from s.  queue must hold n entries.  Returns the number of nodes
 * reached (including s). */
static int64_t bfs_one(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       int32_t s, int32_t *dist, int32_t *queue) {
  for (int32_t v = 0; v < n; ++v) dist[v] = -1;
  int64_t head = 0, tail = 0;
  dist[s] = 0;
  queue[tail++] = s;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      if (dist[v] == -1) {
        dist[v] = dist[u] + 1;
        queue[tail++] = v;
      }
    }
  }
  return tail;
}

/* Single source.  Returns 0, or -1 on a bad argument. */
int oracle_sssp(int32_t n, const int32_t *row_ptr, const int32_t *col,
                int32_t s, int32_t *dist) {
  if (n <= 0 || s < 0 || s >= n || !row_ptr || !col || !dist) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -1;
  bfs_one(n, row_ptr, col, s, dist, queue);
  free(queue);
  return 0;
}

typedef struct {
  int32_t n;
  const int32_t *row_ptr, *col, *sources;
  int32_t k, first, step;
  int32_t *dist;
} mssp_job;

static void *mssp_worker(void *arg) {
  mssp_job *j = (mssp_job *)arg;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)j->n);
  if (!queue) return (void *)1;
  for (int32_t r = j->first; r < j->k; r += j->step)
    bfs_one(j->n, j->row_ptr, j->col, j->sources[r],
            j->dist + (size_t)r * (size_t)j->n, queue);
  free(queue);
  return NULL;
}

/* k sources, one BFS each; row r of dist (k x n) belongs to sources[r].
 * Sources are dealt round-robin to `threads` POSIX threads (threads <= 1 runs
 * on the calling thread).  Returns 0, or -1 on a bad argument. */
int oracle_mssp(int32_t n, const int32_t *row_ptr, const int32_t *col,
                const int32_t *sources, int32_t k, int32_t *dist,
                int32_t threads) {
  if (n <= 0 || k < 0 || !row_ptr || !col || (k && (!sources || !dist))) return -1;
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= n) return -1;
  if (threads < 1) threads = 1;
  if (threads > k) threads = k > 0 ? k : 1;
  mssp_job *jobs = (mssp_job *)calloc((size_t)threads, sizeof(mssp_job));
  pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  if (!jobs || !tids) { free(jobs); free(tids); return -1; }
  int rc = 0;
  for (int32_t t = 0; t < threads; ++t) {
    jobs[t] = (mssp_job){n, row_ptr, col, sources, k, t, threads, dist};
  }
  if (threads == 1) {
    rc = mssp_worker(&jobs[0]) ? -1 : 0;
  } else {
    for (int32_t t = 0; t < threads; ++t)
      pthread_create(&tids[t], NULL, mssp_worker, &jobs[t]);
    for (int32_t t = 0; t < threads; ++t) {
      void *ret = NULL;
      pthread_join(tids[t], &ret);
      if (ret) rc = -1;
    }
  }
  free(jobs);
  free(tids);
  return rc;
}

/* Largest weakly connected component: nodes in ascending id order are written
 * to nodes_out (capacity n) and their count to *s_out.  Components are found
 * by an undirected BFS (out-edges plus in-edges) started from every node not
 * yet labelled, in increasing id order, so ties between equally large
 * components go to the one holding the smallest node id.  Returns 0, or -1. */
int oracle_largest_wcc(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       int32_t *nodes_out, int32_t *s_out) {
  if (n <= 0 || !row_ptr || !col || !nodes_out || !s_out) return -1;
  int64_t m = row_ptr[n];
  int32_t *in_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t *in_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!in_ptr || !in_src || !label || !queue || !fill) {
    free(in_ptr); free(in_src); free(label); free(queue); free(fill);
    return -1;
  }
  /* in-lists by counting */
  for (int64_t e = 0; e < m; ++e) in_ptr[col[e] + 1]++;
  for (int32_t v = 0; v < n; ++v) in_ptr[v + 1] += in_ptr[v];
  memcpy(fill, in_ptr, sizeof(int32_t) * (size_t)n);
  for (int32_t u = 0; u < n; ++u)
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) in_src[fill[col[e]]++] = u;

  for (int32_t v = 0; v < n; ++v) label[v] = -1;
  int32_t best_label = -1;
  int64_t best_size = -1;
  for (int32_t s = 0; s < n; ++s) {
    if (label[s] != -1) continue;
    int64_t head = 0, tail = 0;
    label[s] = s;
    queue[tail++] = s;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        int32_t v = col[e];
        if (label[v] == -1) { label[v] = s; queue[tail++] = v; }
      }
      for (int32_t e = in_ptr[u]; e < in_ptr[u + 1]; ++e) {
        int32_t v = in_src[e];
        if (label[v] == -1) { label[v] = s; queue[tail++] = v; }
      }
    }
    if (tail > best_size) { best_size = tail; best_label = s; }
  }
  int32_t cnt = 0;
  for (int32_t v = 0; v < n; ++v)
    if (label[v] == best_label) nodes_out[cnt++] = v;
  *s_out = cnt;
  free(in_ptr); free(in_src); free(label); free(queue); free(fill);
  return 0;
}
