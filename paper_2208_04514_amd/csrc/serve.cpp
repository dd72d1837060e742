// Serving: continuous batching of multi-source queries over resident graphs.
//
// APSP is the SSSP from every source (paper Section 3.3), and the paper's
// workload is many sources per graph (Section 4.1); a served query is a set
// of sources on one resident graph.  Each graph with traffic gets an engine:
// one bitmask batch of `batch_lanes` lanes (one lane per source) whose level
// loop runs on its own HIP stream.  A scheduler thread drives every engine:
//
//   after each level of an engine
//     1. lanes whose frontier emptied are finished; a query whose lanes are all
//        finished gets its rows emitted (and the lanes' bits cleared), then is
//        done (after a copy to the host when the caller asked for host rows);
//     2. queued queries for that graph are admitted in arrival order while
//        enough lanes are free and the HBM budget allows: their sources are
//        seeded at the current level, with base = that level, so they join the
//        running batch mid-flight (a source's distance is level - base);
//     3. the next level is launched if any lane is still expanding.
//
// Engines of different graphs overlap on the device; the thread polls their
// events instead of blocking on one.  Timestamps: submit, admit, done.
#include <string.h>
#include <sys/prctl.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"

namespace dawn {

namespace {

struct Query {
  uint64_t id = 0;
  int32_t graph = -1;
  std::shared_ptr<GraphRec> g;
  std::vector<int32_t> src;
  int32_t* out = nullptr;
  bool device_out = false;
  dawn_query_stats qs{};
  int32_t* stage = nullptr;        // device rows for host-destination queries
  size_t stage_bytes = 0;
  std::vector<int> lanes;
  int remaining = 0;
  int base = 0;
  hipEvent_t ev = nullptr;         // rows written (and copied)
  bool emitted = false;
};

struct Engine {
  std::shared_ptr<GraphRec> g;
  BatchWs* ws = nullptr;
  int W = 0;
  int capacity = 0;
  int L = 0;                       // last level merged
  bool running = false;
  bool broken = false;             // a step failed: its queries ended; rebuilt once idle
  hipEvent_t lev_ev = nullptr;
  std::vector<Query*> owner;       // per lane
  std::vector<u64> busy;           // lanes held by a query
  std::vector<u64> act;            // lanes still expanding
  std::vector<Query*> emitting;    // emitted, waiting for their event
  int busy_count = 0;
  BatchLevelSum last{};
  bool have_last = false;
  // pinned host mirrors of what is copied to the device at a level boundary
  // (a boundary's copies have finished before the next boundary starts)
  int32_t** h_rows = nullptr;
  int32_t* h_base = nullptr;
  int32_t* h_src = nullptr;
  int32_t* h_lane = nullptr;
  u64* h_em = nullptr;
  int nseed = 0;
};

}  // namespace

struct Server {
  Ctx* ctx = nullptr;
  std::thread th;
  std::thread copier;
  std::mutex mu;
  std::condition_variable cv;        // new work for the scheduler
  std::condition_variable done_cv;   // a query finished
  std::condition_variable copy_cv;
  bool stop = false;
  std::deque<Query*> pending;
  std::deque<Query*> copies;
  std::map<uint64_t, Query*> tickets;
  std::map<int32_t, Engine*> engines;
  uint64_t next_id = 1;
  size_t max_queue = 1 << 16;
  hipStream_t copy_stream = nullptr;
};

static void finish_query(Server* S, Query* q, dawn_status st) {
  // caller holds S->mu
  q->qs.status = st;
  q->qs.done_ns = now_ns();
  if (q->stage) {
    dev_free(S->ctx, q->stage, q->stage_bytes);
    q->stage = nullptr;
  }
  if (q->ev) {
    hipEventDestroy(q->ev);
    q->ev = nullptr;
  }
  S->done_cv.notify_all();
}

static int bit_length(int x) {
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

static void engine_destroy_raw(Engine* e) {
  if (!e) return;
  if (e->ws) {
    hipStreamSynchronize(e->ws->stream);
    batch_ws_destroy(e->ws);
  }
  if (e->lev_ev) hipEventDestroy(e->lev_ev);
  for (void* p : {(void*)e->h_rows, (void*)e->h_base, (void*)e->h_src, (void*)e->h_lane,
                  (void*)e->h_em})
    if (p) hipHostFree(p);
  delete e;
}

static dawn_status engine_create(Server* S, const std::shared_ptr<GraphRec>& g, Engine** out) {
  Engine* e = new Engine();
  e->g = g;
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    p = g->params;
  }
  e->capacity = p.batch_lanes;
  e->W = (e->capacity + 63) / 64;
  dawn_status st = batch_ws_create(S->ctx, g.get(), e->capacity, &e->ws);
  if (st != DAWN_OK) {
    e->ws = nullptr;
    engine_destroy_raw(e);
    return st;
  }
  // set budget aside for every level plane the engine may need, so a running
  // batch never stalls on memory held by queries waiting to join it
  const size_t plane_bytes = (size_t)g->n * e->ws->Wmax * 8;
  st = dev_reserve(S->ctx, plane_bytes * kMaxPlanes);
  if (st != DAWN_OK) {
    engine_destroy_raw(e);
    return st;
  }
  e->ws->plane_reserve = plane_bytes * kMaxPlanes;
  e->owner.assign(e->capacity, nullptr);
  e->busy.assign(e->W, 0);
  e->act.assign(e->W, 0);
  hipError_t he = hipEventCreateWithFlags(&e->lev_ev, hipEventDisableTiming);
  if (he == hipSuccess) he = hipHostMalloc((void**)&e->h_rows, 4096 * sizeof(int32_t*), 0);
  if (he == hipSuccess) he = hipHostMalloc((void**)&e->h_base, 4096 * 4, 0);
  if (he == hipSuccess) he = hipHostMalloc((void**)&e->h_src, 4096 * 4, 0);
  if (he == hipSuccess) he = hipHostMalloc((void**)&e->h_lane, 4096 * 4, 0);
  if (he == hipSuccess) he = hipHostMalloc((void**)&e->h_em, 64 * 8, 0);
  if (he == hipSuccess) {
    for (int i = 0; i < 4096; ++i) {
      e->h_rows[i] = nullptr;
      e->h_base[i] = 0;
    }
  }
  const size_t nW = (size_t)g->n * e->W;
  BatchWs* w = e->ws;
  if (he == hipSuccess) he = hipMemsetAsync(w->ctrl, 0, sizeof(BatchCtrl), w->stream);
  if (he != hipSuccess) {
    engine_destroy_raw(e);
    return fail(DAWN_E_DEVICE, "serving engine: %s", hipGetErrorString(he));
  }
  dawn_status z = batch_launch_zero(S->ctx, w->vis, nW, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->nxt[0], nW, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->nxt[1], nW, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->touched[0], ((size_t)g->n + 63) / 64, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->touched[1], ((size_t)g->n + 63) / 64, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->fmap[0], (size_t)g->n, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->fmap[1], (size_t)g->n, w->stream);
  if (z == DAWN_OK) z = batch_launch_zero(S->ctx, w->vmap, (size_t)g->n, w->stream);
  if (z == DAWN_OK) {
    he = hipMemcpyAsync(w->base, e->h_base, (size_t)e->capacity * 4, hipMemcpyHostToDevice, w->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(w->rows, e->h_rows, (size_t)e->capacity * sizeof(int32_t*),
                          hipMemcpyHostToDevice, w->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(w->stream);
    if (he != hipSuccess) z = fail(DAWN_E_DEVICE, "serving engine: %s", hipGetErrorString(he));
  }
  if (z != DAWN_OK) {
    engine_destroy_raw(e);
    return z;
  }
  *out = e;
  return DAWN_OK;
}

static void engine_destroy(Engine* e) { engine_destroy_raw(e); }

// A query that does not fit the free lanes lets later, smaller queries of
// its graph pass it while it has waited less than this; after that nothing
// passes it, so the lanes drain for it.
constexpr uint64_t kBypassNs = 20000000;

// Admit queued queries of this engine's graph into free lanes, in arrival
// order, with the bounded bypass above.  Their sources are added to the seeds
// the next launch_level issues.  Returns the query that waits for device
// memory (its host-destination staging), or null; S->mu held.
static Query* admit(Server* S, Engine* e) {
  Query* mem_wait = nullptr;
  BatchWs* w = e->ws;
  if (e->broken) return nullptr;
  int lo = e->capacity, hi = -1;
  bool blocked = false;   // an earlier query of this graph waits for lanes
  const uint64_t now = now_ns();
  for (auto it = S->pending.begin(); it != S->pending.end();) {
    Query* q = *it;
    if (q->g.get() != e->g.get()) {
      ++it;
      continue;
    }
    const int k = (int)q->src.size();
    if (k > e->capacity - e->busy_count) {
      if (!blocked) {
        blocked = true;
        if (now - q->qs.submit_ns >= kBypassNs) break;
      }
      ++it;
      continue;
    }
    if (!q->device_out) {
      const size_t bytes = (size_t)k * e->g->n * 4;
      void* p = nullptr;
      if (dev_alloc(S->ctx, &p, bytes) != DAWN_OK) {   // wait for memory to free up
        mem_wait = q;
        break;
      }
      q->stage = (int32_t*)p;
      q->stage_bytes = bytes;
    }
    // lanes, rows, base
    q->lanes.clear();
    for (int lane = 0; lane < e->capacity && (int)q->lanes.size() < k; ++lane) {
      if (!((e->busy[lane >> 6] >> (lane & 63)) & 1ull)) q->lanes.push_back(lane);
    }
    q->base = e->L;
    for (int i = 0; i < k; ++i) {
      const int lane = q->lanes[i];
      e->busy[lane >> 6] |= 1ull << (lane & 63);
      e->act[lane >> 6] |= 1ull << (lane & 63);
      e->owner[lane] = q;
      e->h_rows[lane] = (q->device_out ? q->out : q->stage) + (size_t)i * e->g->n;
      e->h_base[lane] = q->base;
      e->h_src[e->nseed] = q->src[i];
      e->h_lane[e->nseed] = lane;
      ++e->nseed;
      lo = std::min(lo, lane);
      hi = std::max(hi, lane);
    }
    e->busy_count += k;
    q->remaining = k;
    q->qs.admit_ns = now_ns();
    q->qs.batch_peak = std::max(q->qs.batch_peak, e->busy_count);
    it = S->pending.erase(it);
  }
  if (hi >= lo) {
    hipMemcpyAsync(w->rows + lo, e->h_rows + lo, (size_t)(hi - lo + 1) * sizeof(int32_t*),
                   hipMemcpyHostToDevice, w->stream);
    hipMemcpyAsync(w->base + lo, e->h_base + lo, (size_t)(hi - lo + 1) * 4, hipMemcpyHostToDevice,
                   w->stream);
  }
  return mem_wait;
}

// Launch seeds (if any) and the next level of engine e.  S->mu held.
static dawn_status launch_level(Server* S, Engine* e) {
  BatchWs* w = e->ws;
  hipStream_t s = w->stream;
  const GraphRec* g = e->g.get();
  const int L = e->L;
  // the kernels walk only the words up to the highest busy lane (admission
  // fills the lowest free lanes first)
  int Wa = 1;
  for (int i = e->W - 1; i >= 0; --i)
    if (e->busy[i]) {
      Wa = i + 1;
      break;
    }
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(e->g->mu);
    p = e->g->params;
  }
  BatchArgs a = batch_args(g, w, e->W, Wa);
  batch_knobs(a, p);
  if (e->nseed > 0) {
    const int k = e->nseed;
    DAWN_HIP(hipMemcpyAsync(w->src, e->h_src, (size_t)k * 4, hipMemcpyHostToDevice, s));
    DAWN_HIP(hipMemcpyAsync(w->lane, e->h_lane, (size_t)k * 4, hipMemcpyHostToDevice, s));
    DAWN_TRY(batch_launch_seed(S->ctx, a, w->src, w->lane, k, L, true, s));
    e->nseed = 0;
  }
  // planes for the largest relative level of the next step
  int min_base = L + 1;
  for (int lane = 0; lane < e->capacity; ++lane)
    if (e->owner[lane]) min_base = std::min(min_base, e->owner[lane]->base);
  const int need = bit_length(L + 1 - min_base);
  if (need > w->nplanes) {
    DAWN_TRY(batch_ensure_planes(w, need, e->W));
    a = batch_args(g, w, e->W, Wa);
    batch_knobs(a, p);
  }
  // the merge writes only the planes a running lane's level can reach
  a.nplanes = std::min(a.nplanes, std::max(need, 1));
  BatchActWords aw;
  aw.W = e->W;
  for (int i = 0; i < 64; ++i) aw.w[i] = i < e->W ? e->act[i] : 0ull;
  DAWN_TRY(batch_launch_level_prep(aw, w->act, w->ctrl, (L + 1) & 1, s));
  const bool pull = e->have_last ? batch_choose_pull(p, e->last, g->n, Wa) : false;
  DAWN_TRY(batch_launch_expand(S->ctx, a, pull, L + 1, s));
  DAWN_TRY(batch_launch_merge(S->ctx, a, L + 1, s));
  DAWN_HIP(hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, s));
  DAWN_HIP(hipEventRecord(e->lev_ev, s));
  e->running = true;
  return DAWN_OK;
}

// The level just finished: retire finished lanes, emit finished queries.
static dawn_status level_done(Server* S, Engine* e) {
  BatchWs* w = e->ws;
  e->L += 1;
  const int L = e->L;
  e->last = batch_level_sum(w->h_ctrl->lv[L & 1]);
  e->have_last = true;
  std::vector<Query*> done;
  for (int wd = 0; wd < e->W; ++wd) {
    const u64 still = lane_activity(*w->h_ctrl, L & 1, wd);
    u64 fin = e->busy[wd] & e->act[wd] & ~still;
    e->act[wd] = still & e->busy[wd];
    while (fin) {
      const int b = __builtin_ctzll(fin);
      fin &= fin - 1;
      Query* q = e->owner[wd * 64 + b];
      if (q && --q->remaining == 0) done.push_back(q);
    }
  }
  for (int lane = 0; lane < e->capacity; ++lane)
    if (e->owner[lane]) e->owner[lane]->qs.batch_peak =
        std::max(e->owner[lane]->qs.batch_peak, e->busy_count);
  if (done.empty()) return DAWN_OK;
  for (int i = 0; i < e->W; ++i) e->h_em[i] = 0;
  for (Query* q : done) {
    for (int lane : q->lanes) e->h_em[lane >> 6] |= 1ull << (lane & 63);
    q->qs.levels = L - q->base;
  }
  hipStream_t s = w->stream;
  DAWN_HIP(hipMemcpyAsync(w->emask, e->h_em, (size_t)e->W * 8, hipMemcpyHostToDevice, s));
  int We = 1;
  for (int i = e->W - 1; i >= 0; --i)
    if (e->h_em[i]) {
      We = i + 1;
      break;
    }
  BatchArgs a = batch_args(e->g.get(), w, e->W, We);
  // planes that can hold a bit of a finished lane: its levels reach L - base
  int min_base = L;
  for (Query* q : done) min_base = std::min(min_base, q->base);
  const int D = std::min(w->nplanes, bit_length(L - min_base));
  DAWN_TRY(batch_launch_emit(S->ctx, a, D, w->emask, kEmitClear, s));
  for (Query* q : done) {
    hipEventCreateWithFlags(&q->ev, hipEventDisableTiming);
    hipEventRecord(q->ev, s);
    for (int lane : q->lanes) {
      e->busy[lane >> 6] &= ~(1ull << (lane & 63));
      e->act[lane >> 6] &= ~(1ull << (lane & 63));
      e->owner[lane] = nullptr;
    }
    e->busy_count -= (int)q->lanes.size();
    q->emitted = true;
    e->emitting.push_back(q);
  }
  return DAWN_OK;
}

// A step of the engine failed: its running queries end with `st`, their
// lanes are released, and the engine takes no more work; the scheduler
// destroys it once its last emissions have drained and builds a fresh one
// (with clear bitmaps) for the next query of the graph.
static void engine_fail(Server* S, Engine* e, dawn_status st) {
  for (int lane = 0; lane < e->capacity; ++lane) {
    Query* q = e->owner[lane];
    if (!q) continue;
    for (int l : q->lanes) e->owner[l] = nullptr;
    finish_query(S, q, st);
  }
  std::fill(e->busy.begin(), e->busy.end(), 0ull);
  std::fill(e->act.begin(), e->act.end(), 0ull);
  e->busy_count = 0;
  e->nseed = 0;
  e->broken = true;
}

// Engines of other graphs that hold no work give their memory back.
static void reclaim_idle(Server* S, const Engine* keep) {
  for (auto it = S->engines.begin(); it != S->engines.end();) {
    Engine* x = it->second;
    if (x != keep && !x->running && x->busy_count == 0 && x->emitting.empty()) {
      engine_destroy(x);
      it = S->engines.erase(it);
    } else {
      ++it;
    }
  }
}

static void copier_main(Server* S) {
  hipSetDevice(S->ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->copy_cv.wait(lk, [&] { return S->stop || !S->copies.empty(); });
    if (S->copies.empty() && S->stop) return;
    Query* q = S->copies.front();
    S->copies.pop_front();
    lk.unlock();
    hipError_t he = hipEventSynchronize(q->ev);
    if (he == hipSuccess)
      he = hipMemcpyAsync(q->out, q->stage, q->stage_bytes, hipMemcpyDeviceToHost, S->copy_stream);
    if (he == hipSuccess) he = hipStreamSynchronize(S->copy_stream);
    lk.lock();
    finish_query(S, q, he == hipSuccess ? DAWN_OK : DAWN_E_DEVICE);
  }
}

// Polling without sleeping this long after the last step that made progress.
constexpr uint64_t kSpinNs = 2000000;

static void scheduler_main(Server* S) {
  hipSetDevice(S->ctx->device);
  // timed sleeps of this thread end close to their deadline
  prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
  std::unique_lock<std::mutex> lk(S->mu);
  uint64_t last_progress = now_ns();
  while (!S->stop) {
    bool progressed = false;
    // engines for graphs with waiting queries
    for (auto it = S->pending.begin(); it != S->pending.end();) {
      Query* q = *it;
      if (S->engines.count(q->graph)) {
        ++it;
        continue;
      }
      Engine* e = nullptr;
      dawn_status st = engine_create(S, q->g, &e);
      if (st != DAWN_OK) {
        // give the memory of idle engines back, then try once more
        reclaim_idle(S, nullptr);
        st = engine_create(S, q->g, &e);
      }
      if (st == DAWN_OK) {
        S->engines[q->graph] = e;
        ++it;
      } else if (S->engines.empty() && S->copies.empty()) {
        // nothing else holds memory: this query can never run
        it = S->pending.erase(it);
        finish_query(S, q, st);
      } else {
        break;   // wait for running queries to free memory
      }
    }
    // an idle engine whose lane count no longer matches the graph's setting is rebuilt
    for (auto it = S->engines.begin(); it != S->engines.end();) {
      Engine* e = it->second;
      int want;
      {
        std::lock_guard<std::mutex> gl(e->g->mu);
        want = e->g->params.batch_lanes;
      }
      const bool idle = !e->running && e->busy_count == 0 && e->emitting.empty();
      if ((want != e->capacity || e->broken) && idle) {
        engine_destroy(e);
        it = S->engines.erase(it);
        progressed = true;
      } else {
        ++it;
      }
    }
    Engine* mem_engine = nullptr;
    for (auto& kv : S->engines) {
      Engine* e = kv.second;
      // queries whose rows are written
      for (auto it = e->emitting.begin(); it != e->emitting.end();) {
        Query* q = *it;
        const hipError_t qe = hipEventQuery(q->ev);
        if (qe == hipErrorNotReady) {
          ++it;
          continue;
        }
        if (qe != hipSuccess) {
          (void)hipGetLastError();
          finish_query(S, q, fail(DAWN_E_DEVICE, "serving emission: %s", hipGetErrorString(qe)));
        } else if (q->device_out) {
          finish_query(S, q, DAWN_OK);
        } else {
          S->copies.push_back(q);
          S->copy_cv.notify_one();
        }
        it = e->emitting.erase(it);
        progressed = true;
      }
      if (e->running) {
        const hipError_t le = hipEventQuery(e->lev_ev);
        if (le == hipErrorNotReady) continue;
        e->running = false;
        dawn_status st = le == hipSuccess
                             ? level_done(S, e)
                             : fail(DAWN_E_DEVICE, "serving level: %s", hipGetErrorString(le));
        if (st != DAWN_OK) engine_fail(S, e, st);
        progressed = true;
      }
      if (e->broken) continue;
      if (admit(S, e) && !mem_engine) mem_engine = e;
      bool any = false;
      for (u64 x : e->act) any |= x != 0;
      if (any) {
        dawn_status st = launch_level(S, e);
        if (st != DAWN_OK) engine_fail(S, e, st);
        progressed = true;
      }
    }
    if (mem_engine) {
      // a query waits for staging memory: idle engines of other graphs give
      // theirs back; if nothing else holds memory, it can never be admitted
      reclaim_idle(S, mem_engine);
      Query* q = admit(S, mem_engine);
      if (q) {
        bool others = !S->copies.empty() || mem_engine->running || mem_engine->busy_count > 0 ||
                      !mem_engine->emitting.empty();
        for (auto& kv : S->engines) others |= kv.second != mem_engine;
        if (!others) {
          S->pending.erase(std::find(S->pending.begin(), S->pending.end(), q));
          finish_query(S, q, fail(DAWN_E_NO_MEMORY, "no device memory for the query's rows"));
          progressed = true;
        }
      } else {
        bool any = false;
        for (u64 x : mem_engine->act) any |= x != 0;
        if (any && !mem_engine->running) {
          dawn_status st = launch_level(S, mem_engine);
          if (st != DAWN_OK) engine_fail(S, mem_engine, st);
        }
        progressed = true;
      }
    }
    if (progressed) last_progress = now_ns();
    if (!progressed) {
      bool busy = false;
      for (auto& kv : S->engines) busy |= kv.second->running || !kv.second->emitting.empty();
      if (busy) {
        // a level or an emission is on the device: poll again at once for a
        // while (a level can take tens of microseconds, less than a timed
        // sleep often lasts), then back off to short sleeps
        lk.unlock();
        if (now_ns() - last_progress < kSpinNs) {
          // a few microseconds without the lock, so submitters get it
          const uint64_t until = now_ns() + 5000;
          while (now_ns() < until) std::this_thread::yield();
        } else {
          std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        lk.lock();
      } else {
        S->cv.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
  }
}

static dawn_status server_get(Ctx* ctx, Server** out) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  if (!ctx->server) {
    Server* S = new Server();
    S->ctx = ctx;
    hipError_t e = hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete S;
      return fail(DAWN_E_DEVICE, "serving: %s", hipGetErrorString(e));
    }
    S->th = std::thread(scheduler_main, S);
    S->copier = std::thread(copier_main, S);
    ctx->server = S;
  }
  *out = ctx->server;
  return DAWN_OK;
}

void server_stop(Server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  S->copy_cv.notify_all();
  if (S->th.joinable()) S->th.join();
  if (S->copier.joinable()) S->copier.join();
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& kv : S->engines) {
    hipStreamSynchronize(kv.second->ws->stream);
    for (Query* q : kv.second->emitting) finish_query(S, q, DAWN_E_NOT_FOUND);
    engine_fail(S, kv.second, DAWN_E_NOT_FOUND);
    engine_destroy(kv.second);
  }
  for (Query* q : S->pending) finish_query(S, q, DAWN_E_NOT_FOUND);
  for (auto& kv : S->tickets) delete kv.second;
  if (S->copy_stream) hipStreamDestroy(S->copy_stream);
  delete S;
}

dawn_status serve_submit(Ctx* ctx, int32_t graph, const int32_t* sources, int32_t k,
                         int32_t* dist_out, uint32_t flags, uint64_t* ticket) {
  if (!ticket) return fail(DAWN_E_INVALID_ARG, "null ticket");
  if (k <= 0) return fail(DAWN_E_INVALID_ARG, "k must be positive");
  if (!sources || !dist_out) return fail(DAWN_E_INVALID_ARG, "null pointer");
  if (flags & ~DAWN_DEVICE_OUT) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  int capacity;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    capacity = g->params.batch_lanes;
  }
  if (k > capacity)
    return fail(DAWN_E_INVALID_ARG, "query of %d sources exceeds the %d serving lanes (use dawn_mssp)",
                k, capacity);
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= g->n)
      return fail(DAWN_E_INVALID_ARG, "sources[%d] = %d outside [0, %d)", r, sources[r], g->n);
  // a query that can never fit the budget fails now
  const int W = (capacity + 63) / 64;
  // vis, nxt, planes and the two frontier word maps
  const uint64_t engine_bytes = (uint64_t)g->n * W * 8 * (3 + kMaxPlanes) + (uint64_t)g->n * 16;
  const uint64_t stage = (flags & DAWN_DEVICE_OUT) ? 0 : (uint64_t)k * g->n * 4;
  if (engine_bytes + stage + g->bytes > ctx->budget)
    return fail(DAWN_E_NO_MEMORY, "query needs %llu bytes beyond the graph, budget is %llu",
                (unsigned long long)(engine_bytes + stage), (unsigned long long)ctx->budget);
  Server* S = nullptr;
  DAWN_TRY(server_get(ctx, &S));
  Query* q = new Query();
  q->graph = graph;
  q->g = g;
  q->src.assign(sources, sources + k);
  q->out = dist_out;
  q->device_out = (flags & DAWN_DEVICE_OUT) != 0;
  q->qs.k = k;
  q->qs.status = DAWN_PENDING;
  q->qs.submit_ns = now_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->pending.size() >= S->max_queue) {
      delete q;
      return fail(DAWN_E_BUSY, "serving queue full");
    }
    q->id = S->next_id++;
    S->tickets[q->id] = q;
    S->pending.push_back(q);
    *ticket = q->id;
  }
  S->cv.notify_all();
  return DAWN_OK;
}

dawn_status serve_poll(Ctx* ctx, uint64_t ticket, int32_t timeout_ms, dawn_query_stats* qs) {
  Server* S = nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    S = ctx->server;
  }
  if (!S) return fail(DAWN_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end())
    return fail(DAWN_E_NOT_FOUND, "unknown or retired ticket %llu", (unsigned long long)ticket);
  Query* q = it->second;
  if (timeout_ms != 0 && q->qs.status == DAWN_PENDING) {
    auto pred = [&] { return q->qs.status != DAWN_PENDING; };
    if (timeout_ms < 0)
      S->done_cv.wait(lk, pred);
    else
      S->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  }
  if (qs) *qs = q->qs;
  const dawn_status st = q->qs.status;
  if (st == DAWN_PENDING) return DAWN_PENDING;
  S->tickets.erase(it);
  delete q;
  if (st != DAWN_OK) return fail(st, "query %llu failed", (unsigned long long)ticket);
  return DAWN_OK;
}

}  // namespace dawn
