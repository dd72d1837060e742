// Autotuner: picks the fastest knob settings of one resident graph.
//
// The paper fixes one launch shape (a workgroup of 1024 threads) and notes
// that the best partitioning depends on the graph and the device (Section
// 4.1).  Here every knob is searched by coordinate descent: starting from the
// current settings, each knob in turn takes every candidate value, the
// candidate is timed on the caller's sample sources, and the fastest value is
// kept before moving to the next knob.  A candidate counts only if its
// distances equal, bit for bit, those of the settings the search started
// from (checked on the device); a mismatch would be a library bug, and such a
// candidate is dropped.
#include <string.h>

#include <algorithm>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

__global__ void count_mismatch(const int32_t* a, const int32_t* b, size_t n, unsigned* out) {
  unsigned c = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    c += a[i] != b[i];
  c = wave_sum(c);
  if (lane_id() == 0 && c) atomicAdd(out, c);
}

namespace {

struct Tuner {
  Ctx* ctx;
  GraphRec* g;
  const int32_t* src;
  int k;
  int32_t* ref = nullptr;     // reference rows (k x n) from the starting settings
  int32_t* cand = nullptr;    // candidate rows
  unsigned* bad = nullptr;
  size_t elems = 0;
  bool batched = false;

  dawn_status run(const dawn_params& p, int32_t* out, double* ms) {
    const uint64_t t0 = now_ns();
    if (batched) {
      DAWN_TRY(mssp_run(ctx, g, p, src, k, out, true, g->n, nullptr));
    } else {
      for (int i = 0; i < k; ++i)
        DAWN_TRY(sssp_run(ctx, g, p, src[i], out + (size_t)i * g->n, true, nullptr));
    }
    *ms = (now_ns() - t0) / 1e6;
    return DAWN_OK;
  }

  dawn_status same(bool* ok) {
    DAWN_HIP(hipMemset(bad, 0, 4));
    hipLaunchKernelGGL(count_mismatch, dim3(ctx->num_cu * 4), dim3(256), 0, 0, ref, cand, elems, bad);
    DAWN_HIP(hipGetLastError());
    unsigned h = 1;
    DAWN_HIP(hipMemcpy(&h, bad, 4, hipMemcpyDeviceToHost));
    *ok = h == 0;
    return DAWN_OK;
  }

  // time one candidate: best of `reps` runs after one warm-up
  dawn_status time_candidate(const dawn_params& p, double* best_ms, bool* ok) {
    double ms = 0;
    DAWN_TRY(run(p, cand, &ms));
    DAWN_TRY(same(ok));
    if (!*ok) return DAWN_OK;
    *best_ms = 1e30;
    for (int r = 0; r < 3; ++r) {
      DAWN_TRY(run(p, cand, &ms));
      *best_ms = std::min(*best_ms, ms);
    }
    return DAWN_OK;
  }
};

}  // namespace

dawn_status autotune(Ctx* ctx, GraphRec* g, const int32_t* sources, int32_t k, uint32_t what,
                     dawn_params* best_out) {
  dawn_params cur;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    cur = g->params;
  }
  cur.timing = 2;
  Tuner t{ctx, g, sources, 0};
  const int ks = std::min<int>(k, 32);
  const int kb = std::min<int>(k, 4096);
  const size_t cap = (size_t)((what & 2) ? std::max(ks, kb) : ks) * g->n;
  t.elems = cap;
  DAWN_TRY(dev_alloc_n(ctx, &t.ref, cap));
  dawn_status st = dev_alloc_n(ctx, &t.cand, cap);
  if (st == DAWN_OK) st = dev_alloc_n(ctx, &t.bad, 1);
  auto cleanup = [&]() {
    dev_free(ctx, t.ref, cap * 4);
    dev_free(ctx, t.cand, cap * 4);
    dev_free(ctx, t.bad, 4);
  };
  if (st != DAWN_OK) {
    cleanup();
    return st;
  }

  auto search = [&](const std::vector<std::vector<dawn_params>>& knobs) -> dawn_status {
    double ms = 0;
    DAWN_TRY(t.run(cur, t.ref, &ms));
    bool ok = true;
    double best_ms = 0;
    // baseline time of the starting settings (its rows are the reference)
    std::swap(t.ref, t.cand);
    DAWN_TRY(t.time_candidate(cur, &best_ms, &ok));
    std::swap(t.ref, t.cand);
    for (const auto& vals : knobs) {
      dawn_params keep = cur;
      for (const dawn_params& cand : vals) {
        if (check_params(cand) != DAWN_OK) continue;
        double c_ms = 0;
        bool same = false;
        DAWN_TRY(t.time_candidate(cand, &c_ms, &same));
        if (same && c_ms < best_ms * 0.98) {
          best_ms = c_ms;
          keep = cand;
        }
      }
      cur = keep;
    }
    return DAWN_OK;
  };

  auto variants = [&](auto setter, std::initializer_list<double> vals) {
    std::vector<dawn_params> out;
    for (double v : vals) {
      dawn_params p = cur;
      setter(p, v);
      out.push_back(p);
    }
    return out;
  };

  if (what & 1) {
    t.batched = false;
    t.k = ks;
    t.elems = (size_t)ks * g->n;
    // knobs are searched one after another; each list is built from the
    // settings chosen so far
    st = DAWN_OK;
    const auto one = [&](std::vector<dawn_params> v) -> dawn_status {
      return search({v});
    };
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.driver = (int)v; }, {2, 3, 4}));
    if (st == DAWN_OK && cur.driver >= 3)
      st = one(variants([](dawn_params& p, double v) { p.graph_levels = (int)v; }, {4, 8, 16, 32}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.big_degree = (int)v; },
                        {128, 256, 512, 1024, 2048, 8192}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.alpha = (float)v; },
                        {2, 4, 8, 14, 30, 60, 120}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.beta = (float)v; },
                        {6, 12, 24, 50, 100, 200}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.block = (int)v; }, {256, 512, 1024}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.blocks_per_cu = (int)v; }, {0, 1, 2, 4}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.pull_lane_edges = (int)v; },
                        {4, 16, 32, 128}));
    if (st == DAWN_OK)
      st = one(variants([](dawn_params& p, double v) { p.small_frontier_edges = (int)v; },
                        {-1, 128, 256, 512, 1024}));
    if (st == DAWN_OK && cur.driver >= 2)
      st = one(variants([](dawn_params& p, double v) { p.medium_edges = (int)v; },
                        {0, 4096, 16384, 65536}));
    if (st == DAWN_OK && cur.medium_edges > 0)
      st = one(variants([](dawn_params& p, double v) { p.medium_groups = (int)v; },
                        {8, 16, 32, 64}));
  }
  if (st == DAWN_OK && (what & 2)) {
    t.batched = true;
    t.k = kb;
    t.elems = (size_t)kb * g->n;
    // batch_alpha 1e-4 keeps every batched level push, 1e6 every level pull;
    // then the push chunking threshold, the narrow-row whole-wave scan length
    // and the sparse push width, each from the settings chosen so far
    st = search({variants([](dawn_params& p, double v) { p.batch_alpha = (float)v; },
                          {1e-4, 0.25, 1, 4, 16, 64, 1e6})});
    if (st == DAWN_OK)
      st = search({variants([](dawn_params& p, double v) { p.batch_big_degree = (int)v; },
                            {64, 128, 256, 1024})});
    if (st == DAWN_OK && (kb + 63) / 64 <= 8)
      st = search({variants([](dawn_params& p, double v) { p.batch_wide_scan = (int)v; },
                            {16, 32, 48, 96, 192})});
    if (st == DAWN_OK)
      st = search({variants([](dawn_params& p, double v) { p.batch_sparse_words = (int)v; },
                            {1, 2, 4})});
  }
  cleanup();
  if (st != DAWN_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    g->params = cur;
    if (g->wcc_sub) g->wcc_sub->params = cur;
  }
  if (best_out) *best_out = cur;
  return DAWN_OK;
}

}  // namespace dawn
