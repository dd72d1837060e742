/*
 * CPU oracle for weighted shortest-path lengths — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this file's library.  It shares no code with the GPU library.
 *
 * The paper leaves weighted graphs to future work (Section 5: the same level
 * loop over the (min, +) semiring instead of the Boolean one) and defines
 * nothing further, so this oracle computes the plain definition: with
 * non-negative integer edge weights w(e) (weight[e] belongs to CSR entry e,
 * the edge row-of-e -> col[e]),
 *   dist[v] = min over directed paths s -> v of the sum of their weights,
 *   dist[s] = 0, and dist[v] = -1 when no path exists.
 * It is Dijkstra's algorithm with a binary heap and lazy deletion (a node
 * may sit in the heap several times; stale entries are skipped), in 64-bit
 * arithmetic.  Negative weights are refused.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int64_t key;
  int32_t node;
} heap_item;

typedef struct {
  heap_item *a;
  int64_t size, cap;
} heap;

static int heap_push(heap *h, int64_t key, int32_t node) {
  if (h->size == h->cap) {
    int64_t cap = h->cap ? 2 * h->cap : 1024;
    heap_item *na = (heap_item *)realloc(h->a, sizeof(heap_item) * (size_t)cap);
    if (!na) return -1;
    h->a = na;
    h->cap = cap;
  }
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p].key <= key) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i].key = key;
  h->a[i].node = node;
  return 0;
}

static heap_item heap_pop(heap *h) {
  heap_item top = h->a[0];
  heap_item last = h->a[--h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->a[c + 1].key < h->a[c].key) ++c;
    if (h->a[c].key >= last.key) break;
    h->a[i] = h->a[c];
    i = c;
  }
  if (h->size > 0) h->a[i] = last;
  return top;
}

/* Dijkstra from s into dist (n int64, -1 unreachable).  Returns 0 or -1. */
static int dijkstra_one(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        const int32_t *weight, int32_t s, int64_t *dist) {
  for (int32_t v = 0; v < n; ++v) dist[v] = -1;
  heap h = {0, 0, 0};
  dist[s] = 0;
  if (heap_push(&h, 0, s)) return -1;
  while (h.size > 0) {
    heap_item it = heap_pop(&h);
    int32_t u = it.node;
    if (it.key != dist[u]) continue;   /* a stale entry: u was settled closer */
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col[e];
      int64_t nd = it.key + (int64_t)weight[e];
      if (dist[v] == -1 || nd < dist[v]) {
        dist[v] = nd;
        if (heap_push(&h, nd, v)) {
          free(h.a);
          return -1;
        }
      }
    }
  }
  free(h.a);
  return 0;
}

static int weights_ok(int32_t n, const int32_t *row_ptr, const int32_t *weight) {
  for (int64_t e = 0; e < row_ptr[n]; ++e)
    if (weight[e] < 0) return 0;
  return 1;
}

/* Single source.  Returns 0, or -1 on a bad argument (negative weight). */
int oracle_wsssp(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *weight,
                 int32_t s, int64_t *dist) {
  if (n <= 0 || s < 0 || s >= n || !row_ptr || !col || !weight || !dist) return -1;
  if (!weights_ok(n, row_ptr, weight)) return -1;
  return dijkstra_one(n, row_ptr, col, weight, s, dist);
}

typedef struct {
  int32_t n;
  const int32_t *row_ptr, *col, *weight, *sources;
  int32_t k, first, step;
  int64_t *dist;
  int err;
} wmssp_job;

static void *wmssp_worker(void *arg) {
  wmssp_job *j = (wmssp_job *)arg;
  for (int32_t r = j->first; r < j->k; r += j->step)
    if (dijkstra_one(j->n, j->row_ptr, j->col, j->weight, j->sources[r],
                     j->dist + (size_t)r * (size_t)j->n))
      j->err = 1;
  return NULL;
}

/* k sources; row r of dist (k x n int64) belongs to sources[r]; sources are
 * dealt round-robin to `threads` POSIX threads.  Returns 0 or -1. */
int oracle_wmssp(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *weight,
                 const int32_t *sources, int32_t k, int64_t *dist, int32_t threads) {
  if (n <= 0 || k < 0 || !row_ptr || !col || !weight || (k > 0 && (!sources || !dist))) return -1;
  if (!weights_ok(n, row_ptr, weight)) return -1;
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= n) return -1;
  if (threads < 1) threads = 1;
  if (threads > k) threads = k > 0 ? k : 1;
  wmssp_job *jobs = (wmssp_job *)calloc((size_t)threads, sizeof(wmssp_job));
  pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  if (!jobs || !tid) {
    free(jobs);
    free(tid);
    return -1;
  }
  for (int32_t t = 0; t < threads; ++t) {
    wmssp_job j = {n, row_ptr, col, weight, sources, k, t, threads, dist, 0};
    jobs[t] = j;
  }
  for (int32_t t = 1; t < threads; ++t) pthread_create(&tid[t], NULL, wmssp_worker, &jobs[t]);
  wmssp_worker(&jobs[0]);
  int err = jobs[0].err;
  for (int32_t t = 1; t < threads; ++t) {
    pthread_join(tid[t], NULL);
    err |= jobs[t].err;
  }
  free(jobs);
  free(tid);
  return err ? -1 : 0;
}
