// DAWN's SOVM level loop (Section 3.3, Algorithm 2) on the host's CPU cores:
// the paper's CPU configuration, measured for thread efficiency in its
// scalability section.  See include/dawn_host.h for the interface.
//
// One source, N threads: the threads of a team share every level.  The
// frontier is an array of node ids with the exclusive prefix sum of their
// out-degrees, so the level's work is a range of edges.  A level has two
// phases, so that no cache line of the visited bitmap is written by two
// threads (on a many-core host such lines bounce between cores on every
// claim, and every visited test then misses):
//  1. expand: each thread takes blocks of kEdgeBlock edges through one atomic
//     counter (a hub's row is split over many blocks), finds the block's first
//     node by binary search in the prefix and walks the edges; a target whose
//     visited bit is clear (the bitmap is only read in this phase) goes to the
//     bucket of the thread that owns it (thread t owns a contiguous range of
//     nodes, a whole number of 512-node bitmap lines);
//  2. claim: each thread takes the targets bucketed for it by every thread,
//     sets their visited bits (plain stores to its own lines), writes their
//     distance and appends them, with their out-degrees, to its own
//     next-frontier list.
// At the level's end (a spinning barrier) the lists are concatenated in
// parallel into the next frontier at offsets from prefix sums over the
// threads.  The loop ends when a level adds no node.
#include "dawn_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#if defined(__x86_64__)
#include <immintrin.h>
#endif

struct dawn_host_graph {
  int32_t n = 0;
  int64_t m = 0;
  const int32_t* rp = nullptr;
  const int32_t* col = nullptr;
};

namespace {

constexpr int kMaxThreads = 256;
constexpr int64_t kEdgeBlock = 2048;   // edges per claim of the work counter

thread_local char g_err[256] = "";

int32_t fail(int32_t st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

inline void cpu_relax() {
#if defined(__x86_64__)
  _mm_pause();
#endif
}

// Sense-reversing spin barrier for a fixed team.
class SpinBarrier {
 public:
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int gen = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
      count_.store(0, std::memory_order_relaxed);
      gen_.store(gen + 1, std::memory_order_release);
      return;
    }
    int spins = 0;
    while (gen_.load(std::memory_order_acquire) == gen) {
      if (++spins < 4096) cpu_relax();
      else std::this_thread::yield();
    }
  }

 private:
  const int n_;
  alignas(64) std::atomic<int> count_{0};
  alignas(64) std::atomic<int> gen_{0};
};

struct alignas(64) ThreadOut {
  std::vector<std::vector<int32_t>> bucket;   // [owner] targets found for that thread
  std::vector<int32_t> next;   // nodes this thread claimed in the current level
  std::vector<int32_t> deg;    // ... and their out-degrees
  int64_t level_edges = 0;     // sum of deg
  int64_t edges = 0;           // out-degrees of the nodes it claimed (all levels)
  int64_t reached = 0;
  size_t offset = 0;           // where its nodes go in the next frontier
  int64_t edge_offset = 0;     // the edge count before them
};

struct Team {
  const dawn_host_graph* g;
  int nthreads;
  int32_t* dist;
  std::vector<uint64_t> vis;
  int32_t own = 0;                   // nodes owned per thread (multiple of 512)
  std::vector<int32_t> front, next;
  std::vector<int64_t> fpre, npre;   // exclusive prefix of out-degrees over the frontier
  std::vector<ThreadOut> out;
  SpinBarrier bar;
  alignas(64) std::atomic<int64_t> cursor{0};
  size_t fsize = 0;
  int64_t ftotal = 0;                // out-edges of the frontier
  int level = 0;
  bool done = false;

  Team(const dawn_host_graph* gr, int t, int32_t* d)
      : g(gr), nthreads(t), dist(d), out(t), bar(t) {
    const size_t nw = ((size_t)g->n + 63) / 64;
    vis.resize(nw);
    own = (int32_t)((((int64_t)g->n + t - 1) / t + 511) / 512 * 512);
    for (auto& o : out) o.bucket.resize((size_t)t);
    front.resize((size_t)g->n);
    next.resize((size_t)g->n);
    fpre.resize((size_t)g->n);
    npre.resize((size_t)g->n);
  }

  void run(int tid, int32_t source) {
    const int32_t n = g->n;
    const size_t nw = ((size_t)n + 63) / 64;
    // parallel initialisation: dist = -1, nothing visited
    {
      const size_t lo = (size_t)n * tid / nthreads, hi = (size_t)n * (tid + 1) / nthreads;
      for (size_t i = lo; i < hi; ++i) dist[i] = -1;
      const size_t wlo = nw * tid / nthreads, whi = nw * (tid + 1) / nthreads;
      for (size_t i = wlo; i < whi; ++i) vis[i] = 0;
    }
    bar.wait();
    if (tid == 0) {
      dist[source] = 0;
      vis[source >> 6] |= 1ull << (source & 63);
      front[0] = source;
      fpre[0] = 0;
      fsize = 1;
      ftotal = g->rp[source + 1] - g->rp[source];
      out[0].edges += ftotal;
      out[0].reached += 1;
      level = 0;
      cursor.store(0, std::memory_order_relaxed);
    }
    bar.wait();
    ThreadOut& me = out[tid];
    for (;;) {
      const int L = level + 1;
      me.next.clear();
      me.deg.clear();
      me.level_edges = 0;
      for (auto& b : me.bucket) b.clear();
      // 1. expand: blocks of the frontier's edge range taken in turn; the
      // bitmap is read-only until the barrier
      for (;;) {
        const int64_t x = cursor.fetch_add(kEdgeBlock, std::memory_order_relaxed);
        if (x >= ftotal) break;
        const int64_t y = std::min(ftotal, x + kEdgeBlock);
        // first frontier node whose edges reach past x
        size_t i = (size_t)(std::upper_bound(fpre.begin(), fpre.begin() + (ptrdiff_t)fsize, x) -
                            fpre.begin()) - 1;
        int64_t pos = x;
        while (pos < y) {
          const int32_t u = front[i];
          const int64_t row_end = (i + 1 < fsize) ? fpre[i + 1] : ftotal;
          const int64_t stop = std::min(y, row_end);
          const int32_t base = g->rp[u] - (int32_t)fpre[i];
          for (int64_t p = pos; p < stop; ++p) {
            const int32_t v = g->col[base + p];
            if (vis[v >> 6] & (1ull << (v & 63))) continue;
            me.bucket[(size_t)(v / own)].push_back(v);
          }
          pos = stop;
          ++i;
        }
      }
      bar.wait();
      // 2. claim the targets in this thread's range (its own bitmap lines)
      for (int t = 0; t < nthreads; ++t) {
        for (const int32_t v : out[(size_t)t].bucket[(size_t)tid]) {
          const uint64_t bit = 1ull << (v & 63);
          if (vis[v >> 6] & bit) continue;
          vis[v >> 6] |= bit;
          dist[v] = L;
          const int32_t d = g->rp[v + 1] - g->rp[v];
          me.next.push_back(v);
          me.deg.push_back(d);
          me.level_edges += d;
        }
      }
      me.reached += (int64_t)me.next.size();
      me.edges += me.level_edges;
      bar.wait();
      if (tid == 0) {
        size_t off = 0;
        int64_t eoff = 0;
        for (auto& o : out) {
          o.offset = off;
          o.edge_offset = eoff;
          off += o.next.size();
          eoff += o.level_edges;
        }
        fsize = off;
        ftotal = eoff;
        done = off == 0;
        if (!done) level = L;
        cursor.store(0, std::memory_order_relaxed);
      }
      bar.wait();
      if (done) break;
      {
        int64_t e = me.edge_offset;
        for (size_t j = 0; j < me.next.size(); ++j) {
          next[me.offset + j] = me.next[j];
          npre[me.offset + j] = e;
          e += me.deg[j];
        }
      }
      bar.wait();
      if (tid == 0) {
        front.swap(next);
        fpre.swap(npre);
      }
      bar.wait();
    }
  }
};

// Single-threaded SOVM for one source with caller-provided buffers.
struct Serial {
  std::vector<uint64_t> vis;
  std::vector<int32_t> front, next;
  void run(const dawn_host_graph* g, int32_t s, int32_t* dist, int64_t* edges, int64_t* reached,
           int* levels) {
    const int32_t n = g->n;
    vis.assign(((size_t)n + 63) / 64, 0);
    front.resize((size_t)n);
    next.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) dist[i] = -1;
    dist[s] = 0;
    vis[s >> 6] |= 1ull << (s & 63);
    front[0] = s;
    size_t fsize = 1;
    int64_t e_sum = g->rp[s + 1] - g->rp[s], r_sum = 1;
    int L = 0;
    while (fsize) {
      size_t nsize = 0;
      for (size_t i = 0; i < fsize; ++i) {
        const int32_t u = front[i];
        for (int32_t k = g->rp[u], ke = g->rp[u + 1]; k < ke; ++k) {
          const int32_t v = g->col[k];
          const uint64_t bit = 1ull << (v & 63);
          if (vis[v >> 6] & bit) continue;
          vis[v >> 6] |= bit;
          dist[v] = L + 1;
          next[nsize++] = v;
          e_sum += g->rp[v + 1] - g->rp[v];
        }
      }
      if (nsize) ++L;
      r_sum += (int64_t)nsize;
      front.swap(next);
      fsize = nsize;
    }
    *edges += e_sum;
    *reached += r_sum;
    *levels = std::max(*levels, L + 1);
  }
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char* dawn_host_last_error(void) { return g_err; }

int32_t dawn_host_graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                               dawn_host_graph** out) {
  g_err[0] = 0;
  if (!out || !row_ptr || (m > 0 && !col)) return fail(-1, "null pointer");
  if (n <= 0 || m < 0 || m > INT32_MAX) return fail(-1, "n = %d, m = %lld", n, (long long)m);
  if (row_ptr[0] != 0) return fail(-2, "row_ptr[0] = %d, expected 0", row_ptr[0]);
  for (int32_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return fail(-2, "row_ptr decreases at node %d", u);
  if ((int64_t)row_ptr[n] != m) return fail(-2, "row_ptr[n] = %d but m = %lld", row_ptr[n], (long long)m);
  for (int64_t e = 0; e < m; ++e)
    if (col[e] < 0 || col[e] >= n) return fail(-2, "col[%lld] = %d outside [0, %d)", (long long)e, col[e], n);
  dawn_host_graph* g = new dawn_host_graph();
  g->n = n;
  g->m = m;
  g->rp = row_ptr;
  g->col = col;
  *out = g;
  return 0;
}

int32_t dawn_host_graph_destroy(dawn_host_graph* g) {
  g_err[0] = 0;
  if (!g) return fail(-1, "null graph");
  delete g;
  return 0;
}

int32_t dawn_host_sssp(const dawn_host_graph* g, int32_t source, int32_t threads, int32_t* dist,
                       dawn_host_stats* stats) {
  g_err[0] = 0;
  if (!g || !dist) return fail(-1, "null pointer");
  if (source < 0 || source >= g->n) return fail(-1, "source %d outside [0, %d)", source, g->n);
  if (threads < 1 || threads > kMaxThreads) return fail(-1, "threads = %d outside 1 .. %d", threads, kMaxThreads);
  const double t0 = now_ms();
  Team team(g, threads, dist);
  std::vector<std::thread> pool;
  pool.reserve((size_t)threads - 1);
  for (int t = 1; t < threads; ++t) pool.emplace_back([&team, t, source] { team.run(t, source); });
  team.run(0, source);
  for (auto& th : pool) th.join();
  if (stats) {
    int64_t e = 0, r = 0;
    for (auto& o : team.out) {
      e += o.edges;
      r += o.reached;
    }
    stats->levels = team.level + 1;
    stats->source_edges = e;
    stats->reached = r;
    stats->ms = now_ms() - t0;
  }
  return 0;
}

int32_t dawn_host_mssp(const dawn_host_graph* g, const int32_t* sources, int32_t k, int32_t threads,
                       int32_t* dist, dawn_host_stats* stats) {
  g_err[0] = 0;
  if (!g) return fail(-1, "null graph");
  if (k < 0) return fail(-1, "k = %d", k);
  if (threads < 1 || threads > kMaxThreads) return fail(-1, "threads = %d outside 1 .. %d", threads, kMaxThreads);
  if (k > 0 && (!sources || !dist)) return fail(-1, "null pointer");
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= g->n)
      return fail(-1, "sources[%d] = %d outside [0, %d)", r, sources[r], g->n);
  const double t0 = now_ms();
  std::atomic<int32_t> nexti{0};
  const int nt = std::max(1, std::min(threads, k));
  std::vector<int64_t> edges((size_t)nt, 0), reached((size_t)nt, 0);
  std::vector<int> levels((size_t)nt, 0);
  auto work = [&](int t) {
    Serial s;
    for (;;) {
      const int32_t r = nexti.fetch_add(1, std::memory_order_relaxed);
      if (r >= k) break;
      s.run(g, sources[r], dist + (size_t)r * (size_t)g->n, &edges[(size_t)t], &reached[(size_t)t],
            &levels[(size_t)t]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  if (stats) {
    stats->levels = 0;
    stats->source_edges = 0;
    stats->reached = 0;
    for (int t = 0; t < nt; ++t) {
      stats->levels = std::max(stats->levels, levels[(size_t)t]);
      stats->source_edges += edges[(size_t)t];
      stats->reached += reached[(size_t)t];
    }
    stats->ms = now_ms() - t0;
  }
  return 0;
}

}  // extern "C"
