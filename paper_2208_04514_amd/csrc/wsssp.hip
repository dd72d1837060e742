// Weighted single-source shortest paths: DAWN's level loop over the (min, +)
// semiring.
//
// The paper closes (Section 5) by naming weighted graphs, through the same
// vector-matrix step over (min, +) instead of (OR, AND), as future work.  Here
// that step is the SOVM of Algorithm 2 with the Boolean union replaced by a
// minimum of sums: a round takes the nodes whose distance dropped in the
// previous round (the frontier), and for every out-edge (u, v, w) lowers
// dist[v] to dist[u] + w with an atomic minimum; the nodes whose distance
// dropped form the next frontier.  With non-negative weights the loop stops
// at the fixed point dist[v] = min over in-edges of dist[u] + w, which is the
// shortest-path distance (the Bellman-Ford argument: after k rounds every
// shortest path of at most k edges is exact; a frontier node's edges are
// relaxed again whenever its distance drops).  Unlike the Boolean loop a
// node may join several frontiers, so rounds can outnumber BFS levels.
//
// Distances are int32 with -1 for "unreached": compared as unsigned, -1 is
// the largest value, so the atomic minimum needs no sentinel pass.  The
// upload of the weights checks that every path length fits (max weight x
// (n - 1) < 2^31 - 1).
//
// Work per round (64-wide waves): frontier nodes of out-degree below
// kWBig are taken 64 per wave from the queue and the wave walks the union of
// their out-lists four edges per lane and step (owner found by a binary
// search over the wave's prefix sums); larger rows are cut into chunks of
// kWChunk edges listed when the node joins the frontier and spread over the
// waves.  A node joins the next frontier once per round: its bit in the next
// round's membership bitmap is set with an atomic OR, and the claimer stages
// it in its wave's LDS buffer; full buffers go to one of kStripes
// sub-queues with one counter atomic each (the L2 performs atomics one line
// at a time, so every stripe's counter owns a line).  Each round clears the
// bits of the frontier it consumes, so the bitmap of parity p is clear again
// when it is next written.
#include <string.h>

#include <algorithm>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

constexpr int kWBlock = 256;
constexpr int kWBig = 256;      // out-degree from which a frontier node's row goes by chunks
constexpr int kWChunk = 256;    // edges per chunk (four per lane of a wave)

// Counters of one round's output (a ring of three, indexed round % 3: round
// r reads slot r % 3, appends to (r + 1) % 3 and clears (r + 2) % 3).
struct alignas(kLine) WStripe {
  unsigned qn;                  // entries of this stripe's sub-queue
};

struct WSlot {
  WStripe s[kStripes];
  alignas(kLine) unsigned cn;   // chunks of big-degree nodes
};

struct alignas(kLine) WRun {
  int done;                     // 1: a round found its frontier empty; 2: watchdog
  int last_round;               // that round
  // the closing reduction, striped over lines: [s][0] reached nodes, [s][1]
  // the sum of their out-degrees
  alignas(kLine) u64 part[kStripes][kLine / 8];
};

struct WCtrl {
  WSlot slot[3];
  WRun run;
};

struct WArgs {
  int32_t n;
  int32_t nw;
  const int32_t* rp;
  const int32_t* col;
  const int32_t* wt;            // weight of each CSR entry
  int32_t* dist;                // output (device)
  int32_t* q[2];                // frontier queues by round parity: kStripes sub-queues
                                //   of n entries each
  int32_t* cu[2];               // chunk lists: node
  int32_t* ck[2];               //              chunk index within its row
  u64* inq[2];                  // frontier membership bitmaps by parity
  WCtrl* ctrl;
};

__device__ __forceinline__ unsigned umin_atomic(int32_t* p, unsigned v) {
  return __hip_atomic_fetch_min(reinterpret_cast<unsigned*>(p), v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kWWaveBuf = 256;   // entries a wave stages before one reserving atomic

struct WQueue {
  int32_t* buf;                 // this wave's LDS staging area
  int cnt;                      // wave-uniform fill
};

// The wave's staged entries to its stripe's sub-queue of round r + 1.
__device__ __forceinline__ void wq_flush(const WArgs& a, int r, WQueue& q) {
  if (q.cnt == 0) return;
  const int stripe = blockIdx.x % kStripes;
  unsigned base = 0;
  if (lane_id() == 0) base = atom_add(&a.ctrl->slot[(r + 1) % 3].s[stripe].qn, (unsigned)q.cnt);
  base = (unsigned)__shfl((int)base, 0, kWave);
  int32_t* dst = a.q[(r + 1) & 1] + (size_t)stripe * (size_t)a.n + base;
  __builtin_amdgcn_wave_barrier();
  for (int i = lane_id(); i < q.cnt; i += kWave) dst[i] = q.buf[i];
  __builtin_amdgcn_wave_barrier();
  q.cnt = 0;
}

// v's distance dropped in round r (the calling lane, when `hit`): it joins
// the frontier of round r + 1 unless already there.  Wave-uniform call.
__device__ __forceinline__ void join_next(const WArgs& a, int r, int v, bool hit, WQueue& q) {
  const int np = (r + 1) & 1;
  bool first = false;
  int deg = 0;
  if (hit) {
    const u64 bit = 1ull << (v & 63);
    u64* wd = &a.inq[np][v >> 6];
    if (!(ld_relaxed(wd) & bit)) first = !(atom_or(wd, bit) & bit);
    if (first) deg = a.rp[v + 1] - a.rp[v];
  }
  const bool small = first && deg < kWBig;
  const u64 mask = __ballot(small);
  if (mask) {
    if (small) q.buf[q.cnt + __popcll(mask & lanes_below())] = v;
    q.cnt += __popcll(mask);
    if (q.cnt > kWWaveBuf - kWave) wq_flush(a, r, q);
  }
  const int nch = (first && deg >= kWBig) ? (deg + kWChunk - 1) / kWChunk : 0;
  if (__ballot(nch > 0)) {
    const int incl = wave_incl_scan(nch);
    unsigned base = 0;
    if (lane_id() == kWave - 1) base = atom_add(&a.ctrl->slot[(r + 1) % 3].cn, (unsigned)incl);
    base = (unsigned)__shfl((int)base, kWave - 1, kWave) + (unsigned)(incl - nch);
    for (int k = 0; k < nch; ++k) {
      a.cu[np][base + k] = v;
      a.ck[np][base + k] = k;
    }
  }
}

// Relax up to four edges per lane (has[i]: edge i exists; du[i] + wt[i] is
// its candidate).  Wave-uniform call.
__device__ __forceinline__ void relax4(const WArgs& a, int r, const int* v, const unsigned* cand,
                                       const bool* has, WQueue& q) {
  unsigned cur[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cur[i] = has[i] ? (unsigned)a.dist[v[i]] : 0u;
  bool hit[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    hit[i] = false;
    if (has[i] && cand[i] < cur[i]) hit[i] = cand[i] < umin_atomic(&a.dist[v[i]], cand[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) join_next(a, r, v[i], hit[i], q);
}

// Sub-queue holding virtual entry i: largest s with pre[s] <= i.
__device__ __forceinline__ int wstripe_of(const unsigned* pre, unsigned i) {
  int lo = 0;
#pragma unroll
  for (int step = kStripes / 2; step > 0; step >>= 1)
    if (pre[lo + step] <= i) lo += step;
  return lo;
}

// One round: the frontier of slot r % 3 (sub-queues and chunks of parity r & 1).
__global__ __launch_bounds__(kWBlock) void wsssp_round(WArgs a, int r, int max_rounds) {
  __shared__ unsigned pre[kStripes + 1];
  __shared__ int32_t qbuf[kWBlock / kWave][kWWaveBuf];
  WCtrl* c = a.ctrl;
  const WSlot* in = &c->slot[r % 3];
  if (threadIdx.x == 0) {
    unsigned acc = 0;
    for (int t = 0; t < kStripes; ++t) {
      pre[t] = acc;
      acc += ld_relaxed(&in->s[t].qn);
    }
    pre[kStripes] = acc;
  }
  __syncthreads();
  const unsigned qn = pre[kStripes], cn = ld_relaxed(&in->cn);
  if (ld_relaxed(&c->run.done)) return;
  if (qn == 0 && cn == 0) {
    // every workgroup reads the same counts: the run ends here
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->run.done = 1;
      c->run.last_round = r;
    }
    return;
  }
  if (r >= max_rounds) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c->run.done = 2;
    return;
  }
  if (blockIdx.x == 0) {
    // the slot two rounds ahead is next filled by round r + 1
    WSlot* z = &c->slot[(r + 2) % 3];
    if (threadIdx.x < kStripes) z->s[threadIdx.x].qn = 0;
    if (threadIdx.x == kStripes) z->cn = 0;
  }
  const int p = r & 1;
  const int lane = lane_id();
  const unsigned gw = (blockIdx.x * kWBlock + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * kWBlock / kWave;
  WQueue q{qbuf[threadIdx.x / kWave], 0};

  // big-degree rows: one chunk of kWChunk edges per wave, four per lane
  for (unsigned ch = gw; ch < cn; ch += nwaves) {
    const int u = a.cu[p][ch];
    const int k = a.ck[p][ch];
    const unsigned du = (unsigned)a.dist[u];
    const int e0 = a.rp[u] + k * kWChunk;
    const int e1 = min(e0 + kWChunk, a.rp[u + 1]);
    if (k == 0 && lane == 0) atomicAnd(&a.inq[p][u >> 6], ~(1ull << (u & 63)));
    int v[4];
    unsigned cand[4];
    bool has[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = e0 + i * kWave + lane;
      has[i] = e < e1;
      v[i] = has[i] ? a.col[e] : 0;
      cand[i] = has[i] ? du + (unsigned)a.wt[e] : 0u;
    }
    relax4(a, r, v, cand, has, q);
  }

  // small-degree nodes: 64 per wave, the union of their rows
  for (unsigned base = gw * kWave; base < qn; base += nwaves * kWave) {
    const unsigned i = base + lane;
    int rs = 0, deg = 0;
    unsigned du = 0;
    if (i < qn) {
      const int t = wstripe_of(pre, i);
      const int u = a.q[p][(size_t)t * (size_t)a.n + (i - pre[t])];
      rs = a.rp[u];
      deg = a.rp[u + 1] - rs;
      du = (unsigned)a.dist[u];
      atomicAnd(&a.inq[p][u >> 6], ~(1ull << (u & 63)));
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, kWave - 1, kWave);
    for (int eb = 0; eb < total; eb += 4 * kWave) {
      int v[4];
      unsigned cand[4];
      bool has[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int x = eb + t * kWave + lane;
        has[t] = x < total;
        const int j = wave_owner(incl, has[t] ? x : total - 1);
        const int inc_j = __shfl(incl, j, kWave);
        const int deg_j = __shfl(deg, j, kWave);
        const int rs_j = __shfl(rs, j, kWave);
        const unsigned du_j = (unsigned)__shfl((int)du, j, kWave);
        const int e = rs_j + (x - (inc_j - deg_j));
        v[t] = has[t] ? a.col[e] : 0;
        cand[t] = has[t] ? du_j + (unsigned)a.wt[e] : 0u;
      }
      relax4(a, r, v, cand, has, q);
    }
  }
  wq_flush(a, r, q);
}

// dist = -1 everywhere but the source; the frontier of round 0 is the source.
__global__ __launch_bounds__(kWBlock) void wsssp_init(WArgs a, int source) {
  const int tid = blockIdx.x * kWBlock + threadIdx.x;
  const int nt = gridDim.x * kWBlock;
  for (int i = tid; i < a.n; i += nt) a.dist[i] = i == source ? 0 : -1;
  if (tid == 0) {
    WCtrl* c = a.ctrl;
    memset(&c->slot[1], 0, sizeof(WSlot));
    memset(&c->slot[2], 0, sizeof(WSlot));
    memset(&c->run, 0, sizeof(WRun));
    const int deg = a.rp[source + 1] - a.rp[source];
    memset(&c->slot[0], 0, sizeof(WSlot));
    if (deg < kWBig) {
      c->slot[0].s[0].qn = 1;
      a.q[0][0] = source;
    } else {
      const int nch = (deg + kWChunk - 1) / kWChunk;
      c->slot[0].cn = (unsigned)nch;
      for (int k = 0; k < nch; ++k) {
        a.cu[0][k] = source;
        a.ck[0][k] = k;
      }
    }
  }
}

// After the run: reached nodes and the sum of their out-degrees (E_reach,
// the GTEPS numerator).
__global__ __launch_bounds__(kWBlock) void wsssp_close(WArgs a) {
  u64 reached = 0, se = 0;
  const int tid = blockIdx.x * kWBlock + threadIdx.x;
  const int nt = gridDim.x * kWBlock;
  for (int i = tid; i < a.n; i += nt)
    if (a.dist[i] >= 0) {
      reached += 1;
      se += (u64)(a.rp[i + 1] - a.rp[i]);
    }
  __shared__ u64 red[2][kWBlock / kWave];
  reached = wave_sum(reached);
  se = wave_sum(se);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = reached;
    red[1][threadIdx.x / kWave] = se;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    u64 x = 0;
    for (int i = 0; i < kWBlock / kWave; ++i) x += red[threadIdx.x][i];
    if (x) atom_add(&a.ctrl->run.part[blockIdx.x % kStripes][threadIdx.x], x);
  }
}

// ------------------------------------------------------------------ host --
namespace {

struct WWs {
  Ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int32_t* q[2] = {nullptr, nullptr};
  int32_t* cu[2] = {nullptr, nullptr};
  int32_t* ck[2] = {nullptr, nullptr};
  u64* inq[2] = {nullptr, nullptr};
  int32_t* dist = nullptr;
  WCtrl* ctrl = nullptr;
  WCtrl* h_ctrl = nullptr;
  size_t bytes = 0;

  ~WWs() {
    for (int i = 0; i < 2; ++i) {
      dev_free(ctx, q[i], 0);
      dev_free(ctx, cu[i], 0);
      dev_free(ctx, ck[i], 0);
      dev_free(ctx, inq[i], 0);
    }
    dev_free(ctx, dist, 0);
    dev_free(ctx, ctrl, 0);
    if (ctx) ctx->used -= bytes;
    if (h_ctrl) hipHostFree(h_ctrl);
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    if (stream) hipStreamDestroy(stream);
  }
};

dawn_status wws_create(Ctx* ctx, const GraphRec* g, std::unique_ptr<WWs>* out) {
  std::unique_ptr<WWs> w(new WWs());
  w->ctx = ctx;
  const size_t n = (size_t)g->n, nw = (n + 63) / 64;
  // chunks per round: every big node at most once, ceil(deg / kWChunk) each
  const size_t chunk_cap = (size_t)(g->m / kWChunk) + (size_t)(g->m / kWBig) + 64;
  WWs* wp = w.get();
  auto alloc = [&](void** p, size_t bytes) -> dawn_status {
    dawn_status s = dev_alloc(ctx, p, bytes);
    if (s == DAWN_OK) wp->bytes += bytes;
    return s;
  };
  for (int i = 0; i < 2; ++i) {
    DAWN_TRY(alloc((void**)&w->q[i], (size_t)kStripes * n * 4));
    DAWN_TRY(alloc((void**)&w->cu[i], chunk_cap * 4));
    DAWN_TRY(alloc((void**)&w->ck[i], chunk_cap * 4));
    DAWN_TRY(alloc((void**)&w->inq[i], nw * 8 + 64));
    DAWN_HIP(hipMemset(w->inq[i], 0, nw * 8 + 64));
  }
  DAWN_TRY(alloc((void**)&w->dist, n * 4));
  DAWN_TRY(alloc((void**)&w->ctrl, sizeof(WCtrl)));
  DAWN_HIP(hipMemset(w->ctrl, 0, sizeof(WCtrl)));
  DAWN_HIP(hipHostMalloc((void**)&w->h_ctrl, sizeof(WCtrl), hipHostMallocDefault));
  DAWN_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
  DAWN_HIP(hipEventCreate(&w->ev0));
  DAWN_HIP(hipEventCreate(&w->ev1));
  *out = std::move(w);
  return DAWN_OK;
}

}  // namespace

// Rounds queued per host check of the run state: the first batch covers the
// graph's last run, later ones double.
constexpr int kWRoundsFirst = 16;

struct WsspPool {
  std::vector<std::unique_ptr<WWs>> ws;
};

void wsssp_pool_free(GraphRec* g) {
  delete reinterpret_cast<WsspPool*>(g->wpool);
  g->wpool = nullptr;
}

dawn_status wsssp_run(Ctx* ctx, GraphRec* g, int32_t source, int32_t* dist, bool device_out,
                      dawn_run_stats* stats) {
  const uint64_t t0 = now_ns();
  if (!g->wt) return fail(DAWN_E_INVALID_ARG, "graph %d has no weights (dawn_graph_set_weights)", g->id);
  std::unique_ptr<WWs> w;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    WsspPool* pool = reinterpret_cast<WsspPool*>(g->wpool);
    if (pool && !pool->ws.empty()) {
      w = std::move(pool->ws.back());
      pool->ws.pop_back();
    }
  }
  if (!w) DAWN_TRY(wws_create(ctx, g, &w));
  WArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.nw = (g->n + 63) / 64;
  a.rp = g->rp;
  a.col = g->col;
  a.wt = g->wt;
  a.dist = device_out ? dist : w->dist;
  for (int i = 0; i < 2; ++i) {
    a.q[i] = w->q[i];
    a.cu[i] = w->cu[i];
    a.ck[i] = w->ck[i];
    a.inq[i] = w->inq[i];
  }
  a.ctrl = w->ctrl;
  hipStream_t s = w->stream;
  const int fill = std::max(1, std::min((g->n + kWBlock - 1) / kWBlock, ctx->num_cu * 8));
  const int grid = ctx->num_cu * 8;
  const int max_rounds = g->n + 1;
  dawn_status st = DAWN_OK;
  hipError_t e = hipEventRecord(w->ev0, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(wsssp_init, dim3(fill), dim3(kWBlock), 0, s, a, source);
    e = hipGetLastError();
  }
  int launches = 1, queued = 0;
  int batch = std::max(g->wsssp_hint.load(std::memory_order_relaxed) + 1, kWRoundsFirst);
  while (e == hipSuccess) {
    for (int i = 0; i < batch; ++i)
      hipLaunchKernelGGL(wsssp_round, dim3(grid), dim3(kWBlock), 0, s, a, queued + i, max_rounds);
    e = hipGetLastError();
    launches += batch;
    queued += batch;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&w->h_ctrl->run, &w->ctrl->run, sizeof(WRun), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || w->h_ctrl->run.done) break;
    if (queued > max_rounds + 1) {
      st = fail(DAWN_E_DEVICE, "weighted level loop did not terminate");
      break;
    }
    batch = std::min(batch * 2, 1024);
  }
  if (e == hipSuccess && st == DAWN_OK) {
    if (w->h_ctrl->run.done == 2) st = fail(DAWN_E_DEVICE, "watchdog: more than n + 1 rounds");
  }
  if (e == hipSuccess && st == DAWN_OK) {
    hipLaunchKernelGGL(wsssp_close, dim3(fill), dim3(kWBlock), 0, s, a);
    e = hipGetLastError();
    ++launches;
    if (e == hipSuccess) e = hipEventRecord(w->ev1, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(WCtrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !device_out)
      e = hipMemcpyAsync(dist, w->dist, (size_t)g->n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "weighted SSSP: %s", hipGetErrorString(e));
  if (st != DAWN_OK) {
    hipStreamSynchronize(s);
    return st;   // the workspace is dropped (its bitmaps may hold bits)
  }
  const WRun& run = w->h_ctrl->run;
  u64 reached = 0, source_edges = 0;
  for (int i = 0; i < kStripes; ++i) {
    reached += run.part[i][0];
    source_edges += run.part[i][1];
  }
  g->wsssp_hint.store(run.last_round + 1, std::memory_order_relaxed);
  if (stats) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, w->ev0, w->ev1);
    stats->levels = run.last_round;            // rounds that had a frontier
    stats->push_levels = run.last_round;
    stats->pull_levels = 0;
    stats->launches = launches;
    stats->edges_examined = 0;                 // not counted by the weighted rounds
    stats->source_edges = (int64_t)source_edges;
    stats->reached = (int64_t)reached;
    stats->kernel_ms = ms;
    stats->total_ms = (now_ns() - t0) / 1e6;
    stats->kernel_clock_ms = 0.0;
  }
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->wpool) g->wpool = new WsspPool();
    reinterpret_cast<WsspPool*>(g->wpool)->ws.push_back(std::move(w));
  }
  return DAWN_OK;
}

}  // namespace dawn
