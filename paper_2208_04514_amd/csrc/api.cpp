// C ABI entry points of libdawn (declared in include/dawn.h): argument
// checks, the graph table, device-memory accounting and error text.  The
// traversal work itself lives in sssp.hip / mssp.hip / serve.cpp.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "internal.hpp"

namespace dawn {

static thread_local char g_err[512] = "";

dawn_status fail(dawn_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

dawn_status dev_alloc(Ctx* ctx, void** p, size_t bytes, bool from_reserve) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  // failure injection ($DAWN_FAIL_ALLOC_AFTER = N): the allocation after the
  // next N fails once, then allocations succeed again
  long long left = ctx->fail_after.load();
  if (left >= 0) {
    ctx->fail_after.fetch_sub(1);
    if (left == 0) return fail(DAWN_E_NO_MEMORY, "device allocation refused (injected failure)");
  }
  std::lock_guard<std::mutex> lk(ctx->budget_mu);
  const uint64_t used = ctx->used.load(), res = ctx->reserved.load();
  if (from_reserve) {
    if (res < bytes) return fail(DAWN_E_NO_MEMORY, "reservation exhausted");
  } else if (used + res + bytes > ctx->budget) {
    return fail(DAWN_E_NO_MEMORY, "HBM budget exceeded: need %zu more bytes, %llu in use, "
                "%llu reserved, budget %llu", bytes, (unsigned long long)used,
                (unsigned long long)res, (unsigned long long)ctx->budget);
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(DAWN_E_NO_MEMORY, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  ctx->used += bytes;
  if (from_reserve) ctx->reserved -= bytes;
  return DAWN_OK;
}

dawn_status dev_reserve(Ctx* ctx, size_t bytes) {
  std::lock_guard<std::mutex> lk(ctx->budget_mu);
  if (ctx->used.load() + ctx->reserved.load() + bytes > ctx->budget)
    return fail(DAWN_E_NO_MEMORY, "HBM budget exceeded: cannot set aside %zu bytes", bytes);
  ctx->reserved += bytes;
  return DAWN_OK;
}

void dev_unreserve(Ctx* ctx, size_t bytes) {
  std::lock_guard<std::mutex> lk(ctx->budget_mu);
  ctx->reserved -= std::min<uint64_t>(bytes, ctx->reserved.load());
}

void dev_free(Ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  hipFree(p);
  if (ctx && bytes) ctx->used.fetch_sub(bytes == 0 ? 1 : bytes);
}

dawn_status get_graph(Ctx* ctx, int32_t id, std::shared_ptr<GraphRec>* out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->graphs.find(id);
  if (it == ctx->graphs.end()) return fail(DAWN_E_NOT_FOUND, "no resident graph %d", id);
  *out = it->second;
  return DAWN_OK;
}

dawn_params default_params(const GraphRec& g) {
  dawn_params p;
  memset(&p, 0, sizeof(p));
  p.driver = 3;
  p.direction = 3;
  p.block = 256;
  p.blocks_per_cu = 0;
  p.big_degree = 2048;
  p.pull_lane_edges = 32;
  p.alpha = 14.0f;
  p.beta = 24.0f;
  p.graph_levels = 16;
  p.small_n = 512;
  p.batch_alpha = 4.0f;
  p.batch_lanes = 4096;
  p.timing = 2;
  p.batch_big_degree = 64;
  p.batch_wide_scan = 48;
  p.batch_sparse_words = 4;
  p.small_frontier_edges = 1024;
  p.medium_edges = 0;
  p.medium_groups = 32;
  (void)g;
  return p;
}

dawn_status check_params(const dawn_params& p) {
  if (p.driver < 1 || p.driver > 4) return fail(DAWN_E_INVALID_ARG, "driver must be 1, 2, 3 or 4");
  if (p.direction < 1 || p.direction > 3) return fail(DAWN_E_INVALID_ARG, "direction must be 1..3");
  if (p.block != 256 && p.block != 512 && p.block != 1024)
    return fail(DAWN_E_INVALID_ARG, "block must be 256, 512 or 1024");
  if (p.blocks_per_cu < 0 || p.blocks_per_cu > 64) return fail(DAWN_E_INVALID_ARG, "blocks_per_cu");
  if (p.big_degree < 64) return fail(DAWN_E_INVALID_ARG, "big_degree must be >= 64");
  if (p.pull_lane_edges < 1) return fail(DAWN_E_INVALID_ARG, "pull_lane_edges must be >= 1");
  if (!(p.alpha > 0.f) || !(p.beta > 0.f)) return fail(DAWN_E_INVALID_ARG, "alpha, beta > 0");
  if (p.graph_levels < 1 || p.graph_levels > 1024) return fail(DAWN_E_INVALID_ARG, "graph_levels");
  if (p.small_n < 0) return fail(DAWN_E_INVALID_ARG, "small_n");
  if (!(p.batch_alpha > 0.f)) return fail(DAWN_E_INVALID_ARG, "batch_alpha > 0");
  if (p.batch_lanes < 64 || p.batch_lanes > 4096 || p.batch_lanes % 64)
    return fail(DAWN_E_INVALID_ARG, "batch_lanes must be a multiple of 64 in [64, 4096]");
  if (p.timing < 1 || p.timing > 2) return fail(DAWN_E_INVALID_ARG, "timing must be 1 or 2");
  if (p.timing == 1 && p.driver != 2)
    return fail(DAWN_E_INVALID_ARG, "timing 1 needs driver 2 (one launch per level)");
  if (p.batch_big_degree < 64) return fail(DAWN_E_INVALID_ARG, "batch_big_degree must be >= 64");
  if (p.batch_wide_scan < 1 || p.batch_wide_scan > 512)
    return fail(DAWN_E_INVALID_ARG, "batch_wide_scan must be in [1, 512]");
  if (p.batch_sparse_words < 1 || p.batch_sparse_words > 4)
    return fail(DAWN_E_INVALID_ARG, "batch_sparse_words must be in [1, 4]");
  if (p.small_frontier_edges < -1)
    return fail(DAWN_E_INVALID_ARG, "small_frontier_edges must be >= -1");
  if (p.medium_edges < 0) return fail(DAWN_E_INVALID_ARG, "medium_edges must be >= 0");
  if (p.medium_groups < 2 || p.medium_groups > 256)
    return fail(DAWN_E_INVALID_ARG, "medium_groups must be in [2, 256]");
  return DAWN_OK;
}

static dawn_status check_ctx(dawn_ctx* c) {
  if (!c) return fail(DAWN_E_INVALID_ARG, "null context");
  return DAWN_OK;
}

static Ctx* C(dawn_ctx* c) { return reinterpret_cast<Ctx*>(c); }

// `bytes` of device memory at p on the context's GPU, inside one allocation
// (a caching allocator's block may be larger than the tensor: the check then
// only bounds the block).
static dawn_status check_device_span(Ctx* ctx, const void* p, size_t bytes, const char* what) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess || (at.type != hipMemoryTypeDevice && !at.isManaged)) {
    (void)hipGetLastError();
    return fail(DAWN_E_INVALID_ARG, "%s is not device memory", what);
  }
  if (at.device != ctx->device)
    return fail(DAWN_E_INVALID_ARG, "%s is on device %d, the context on %d", what, at.device,
                ctx->device);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) == hipSuccess && base) {
    const size_t off = (size_t)((const char*)p - (const char*)base);
    if (off + bytes > size)
      return fail(DAWN_E_INVALID_ARG, "%s: %zu bytes past %p overrun its allocation of %zu bytes",
                  what, bytes, p, size);
  } else {
    (void)hipGetLastError();
  }
  return DAWN_OK;
}

}  // namespace dawn

using namespace dawn;

extern "C" {

const char* dawn_last_error(void) { return g_err; }

dawn_status dawn_create(int32_t device, uint64_t hbm_budget_bytes, dawn_ctx** out) {
  clear_error();
  if (!out) return fail(DAWN_E_INVALID_ARG, "null output handle");
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0)
    return fail(DAWN_E_DEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (device < 0 || device >= count)
    return fail(DAWN_E_INVALID_ARG, "device %d outside [0, %d)", device, count);
  DAWN_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  DAWN_HIP(hipGetDeviceProperties(&prop, device));
  DAWN_TRY(scratch_init(device));
  size_t freeb = 0, totalb = 0;
  DAWN_HIP(hipMemGetInfo(&freeb, &totalb));
  Ctx* ctx = new Ctx();
  ctx->device = device;
  ctx->num_cu = prop.multiProcessorCount;
  ctx->coop = prop.cooperativeLaunch;
  ctx->lds_per_block = prop.sharedMemPerBlock;
  if (hipDeviceGetAttribute(&ctx->wall_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess)
    ctx->wall_khz = 0;
  uint64_t budget = hbm_budget_bytes;
  if (budget == 0) {
    const char* env = getenv("DAWN_HBM_BUDGET");
    if (env && *env) budget = strtoull(env, nullptr, 10);
  }
  if (budget == 0) budget = (uint64_t)(freeb * 0.9);
  ctx->budget = budget;
  const char* fa = getenv("DAWN_FAIL_ALLOC_AFTER");
  if (fa && *fa) ctx->fail_after = atoll(fa);
  const char* fp = getenv("DAWN_FAIL_PLANE_AFTER");
  if (fp && *fp) ctx->fail_plane_after = atoll(fp);
  *out = reinterpret_cast<dawn_ctx*>(ctx);
  return DAWN_OK;
}

dawn_status dawn_destroy(dawn_ctx* c) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  Ctx* ctx = C(c);
  hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) {
      server_stop(ctx->server);
      ctx->server = nullptr;
    }
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->graphs.clear();
  }
  hipDeviceSynchronize();
  delete ctx;
  return DAWN_OK;
}

dawn_status dawn_memory(dawn_ctx* c, uint64_t* used, uint64_t* budget) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (used) *used = C(c)->used.load();
  if (budget) *budget = C(c)->budget;
  return DAWN_OK;
}

dawn_status dawn_graph_upload(dawn_ctx* c, int32_t n, int64_t m, const int32_t* row_ptr,
                              const int32_t* col, uint32_t flags, int32_t* graph_out) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (n <= 0) return fail(DAWN_E_INVALID_ARG, "n must be positive (got %d)", n);
  if (m < 0 || m > 0x7fffffffLL) return fail(DAWN_E_INVALID_ARG, "m must be in [0, INT32_MAX]");
  if (!row_ptr || (m > 0 && !col) || !graph_out) return fail(DAWN_E_INVALID_ARG, "null pointer");
  if (flags & ~DAWN_SHARED_CSC) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  Ctx* ctx = C(c);
  DAWN_HIP(hipSetDevice(ctx->device));
  auto g = std::make_shared<GraphRec>();
  g->n = n;
  g->m = m;
  g->shared_csc = (flags & DAWN_SHARED_CSC) != 0;
  dawn_status st = graph_build(ctx, g.get(), row_ptr, col);
  if (st != DAWN_OK) return st;
  g->params = default_params(*g);
  std::lock_guard<std::mutex> lk(ctx->mu);
  g->id = ctx->next_graph++;
  ctx->graphs[g->id] = g;
  *graph_out = g->id;
  return DAWN_OK;
}

dawn_status dawn_graph_release(dawn_ctx* c, int32_t graph) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  Ctx* ctx = C(c);
  hipSetDevice(ctx->device);
  std::shared_ptr<GraphRec> g;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->graphs.find(graph);
    if (it == ctx->graphs.end()) return fail(DAWN_E_NOT_FOUND, "no resident graph %d", graph);
    g = it->second;
    ctx->graphs.erase(it);
  }
  // running calls hold their own reference; the buffers go with the last one
  g.reset();
  return DAWN_OK;
}

dawn_status dawn_graph_get_info(dawn_ctx* c, int32_t graph, dawn_graph_info* out) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!out) return fail(DAWN_E_INVALID_ARG, "null output");
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(C(c), graph, &g));
  std::lock_guard<std::mutex> lk(g->mu);
  out->n = g->n;
  out->m = g->m;
  out->max_out_degree = g->max_out_deg;
  out->zero_out_degree = g->zero_out;
  out->s_wcc = g->wcc_ready ? (int32_t)g->wcc_nodes.size() : -1;
  out->device_bytes = (int64_t)g->bytes;
  return DAWN_OK;
}

dawn_status dawn_graph_set_weights(dawn_ctx* c, int32_t graph, const int32_t* weights) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  if (!weights && g->m > 0) return fail(DAWN_E_INVALID_ARG, "null weights");
  int32_t mx = 0;
  for (long long e = 0; e < g->m; ++e) {
    if (weights[e] < 0) return fail(DAWN_E_INVALID_ARG, "weights[%lld] = %d is negative", e, weights[e]);
    mx = std::max(mx, weights[e]);
  }
  // every path length must fit in an int32 distance (and stay below -1 as
  // an unsigned value, which marks "unreached")
  if ((long long)mx * (long long)(g->n - 1) > 0x7ffffffeLL)
    return fail(DAWN_E_INVALID_ARG, "max weight %d x (n - 1) = %lld exceeds int32 distances", mx,
                (long long)mx * (g->n - 1));
  DAWN_HIP(hipSetDevice(ctx->device));
  int32_t* d = nullptr;
  const size_t bytes = (size_t)std::max(g->m, 1LL) * 4;
  DAWN_TRY(dev_alloc(ctx, (void**)&d, bytes));
  hipError_t e = g->m > 0 ? hipMemcpy(d, weights, (size_t)g->m * 4, hipMemcpyHostToDevice) : hipSuccess;
  if (e != hipSuccess) {
    dev_free(ctx, d, bytes);
    return fail(DAWN_E_DEVICE, "weights upload: %s", hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g->mu);
  if (g->wt) dev_free(ctx, g->wt, bytes);
  else g->bytes += bytes;
  g->wt = d;
  g->max_w = mx;
  return DAWN_OK;
}

dawn_status dawn_sssp_weighted(dawn_ctx* c, int32_t graph, int32_t source, int32_t* dist,
                               uint32_t flags, dawn_run_stats* stats) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!dist) return fail(DAWN_E_INVALID_ARG, "null dist");
  if (flags & ~DAWN_DEVICE_OUT) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  if (source < 0 || source >= g->n)
    return fail(DAWN_E_INVALID_ARG, "source %d outside [0, %d)", source, g->n);
  DAWN_HIP(hipSetDevice(ctx->device));
  return wsssp_run(ctx, g.get(), source, dist, (flags & DAWN_DEVICE_OUT) != 0, stats);
}

dawn_status dawn_get_params(dawn_ctx* c, int32_t graph, dawn_params* out) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!out) return fail(DAWN_E_INVALID_ARG, "null output");
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(C(c), graph, &g));
  std::lock_guard<std::mutex> lk(g->mu);
  *out = g->params;
  return DAWN_OK;
}

dawn_status dawn_set_params(dawn_ctx* c, int32_t graph, const dawn_params* in) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!in) return fail(DAWN_E_INVALID_ARG, "null input");
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(C(c), graph, &g));
  dawn_params d = default_params(*g);
  dawn_params p = *in;
#define KEEP(f) \
  if (p.f == 0) p.f = d.f
  KEEP(driver); KEEP(direction); KEEP(block); KEEP(big_degree); KEEP(pull_lane_edges);
  KEEP(alpha); KEEP(beta); KEEP(graph_levels); KEEP(batch_alpha); KEEP(batch_lanes);
  KEEP(timing); KEEP(batch_big_degree); KEEP(batch_wide_scan); KEEP(batch_sparse_words);
  KEEP(small_frontier_edges); KEEP(medium_groups);
#undef KEEP
  DAWN_TRY(check_params(p));
  std::lock_guard<std::mutex> lk(g->mu);
  g->params = p;
  if (g->wcc_sub) g->wcc_sub->params = p;
  return DAWN_OK;
}

dawn_status dawn_sssp(dawn_ctx* c, int32_t graph, int32_t source, int32_t* dist, uint32_t flags,
                      dawn_run_stats* stats) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!dist) return fail(DAWN_E_INVALID_ARG, "null dist");
  if (flags & ~DAWN_DEVICE_OUT) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  if (source < 0 || source >= g->n)
    return fail(DAWN_E_INVALID_ARG, "source %d outside [0, %d)", source, g->n);
  DAWN_HIP(hipSetDevice(ctx->device));
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    p = g->params;
  }
  return sssp_run(ctx, g.get(), p, source, dist, (flags & DAWN_DEVICE_OUT) != 0, stats);
}

dawn_status dawn_sssp_noalloc(dawn_ctx* c, int32_t graph, int32_t source, int32_t* d_dist,
                              void* hip_stream, dawn_run_stats* stats) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!d_dist) return fail(DAWN_E_INVALID_ARG, "null dist");
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  if (source < 0 || source >= g->n)
    return fail(DAWN_E_INVALID_ARG, "source %d outside [0, %d)", source, g->n);
  DAWN_HIP(hipSetDevice(ctx->device));
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    p = g->params;
  }
  return sssp_run_noalloc(ctx, g.get(), p, source, d_dist,
                          reinterpret_cast<hipStream_t>(hip_stream), stats);
}

dawn_status dawn_mssp(dawn_ctx* c, int32_t graph, const int32_t* sources, int32_t k, int32_t* dist,
                      uint32_t flags, dawn_run_stats* stats) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (k < 0) return fail(DAWN_E_INVALID_ARG, "k must be >= 0");
  if (flags & ~DAWN_DEVICE_OUT) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  if (k == 0) {
    if (stats) {
      stats->levels = stats->push_levels = stats->pull_levels = stats->launches = 0;
      stats->edges_examined = stats->source_edges = stats->reached = 0;
      stats->kernel_ms = stats->total_ms = stats->kernel_clock_ms = 0;
    }
    return DAWN_OK;
  }
  if (!sources || !dist) return fail(DAWN_E_INVALID_ARG, "null pointer");
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= g->n)
      return fail(DAWN_E_INVALID_ARG, "sources[%d] = %d outside [0, %d)", r, sources[r], g->n);
  DAWN_HIP(hipSetDevice(ctx->device));
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    p = g->params;
  }
  return mssp_run(ctx, g.get(), p, sources, k, dist, (flags & DAWN_DEVICE_OUT) != 0, g->n, stats);
}

dawn_status dawn_mssp_device(dawn_ctx* c, int32_t graph, const int32_t* d_sources, int32_t k,
                             int32_t* d_dist, int32_t* d_status, void* hip_stream) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (k < 0) return fail(DAWN_E_INVALID_ARG, "k must be >= 0");
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  DAWN_HIP(hipSetDevice(ctx->device));
  if (k > 0) {
    if (!d_sources || !d_dist) return fail(DAWN_E_INVALID_ARG, "null pointer");
    DAWN_TRY(check_device_span(ctx, d_sources, (size_t)k * 4, "sources"));
    DAWN_TRY(check_device_span(ctx, d_dist, (size_t)k * (size_t)g->n * 4, "dist"));
  }
  if (d_status) DAWN_TRY(check_device_span(ctx, d_status, 4, "status"));
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    p = g->params;
  }
  return mssp_device_run(ctx, g.get(), p, d_sources, k, d_dist, d_status,
                         reinterpret_cast<hipStream_t>(hip_stream));
}

dawn_status dawn_apsp_wcc(dawn_ctx* c, int32_t graph, int32_t* wcc_nodes, int32_t* s_wcc,
                          int32_t* dist, uint32_t flags, dawn_run_stats* stats) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (!wcc_nodes || !s_wcc) return fail(DAWN_E_INVALID_ARG, "null pointer");
  if (flags & ~DAWN_DEVICE_OUT) return fail(DAWN_E_INVALID_ARG, "unknown flags 0x%x", flags);
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  DAWN_HIP(hipSetDevice(ctx->device));
  std::shared_ptr<GraphRec> sub;
  std::vector<int32_t> nodes;
  dawn_params p;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->wcc_ready) {
      hipStream_t s = nullptr;
      DAWN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      dawn_status st = graph_wcc(ctx, g.get(), s);
      hipStreamDestroy(s);
      if (st != DAWN_OK) return st;
    }
    sub = g->wcc_sub;
    nodes = g->wcc_nodes;
    p = g->params;
  }
  const int32_t S = (int32_t)nodes.size();
  if (dist && S > 0) {
    std::vector<int32_t> srcs(S);
    for (int32_t i = 0; i < S; ++i) srcs[i] = i;   // subgraph ids are WCC ranks
    DAWN_TRY(mssp_run(ctx, sub.get(), p, srcs.data(), S, dist, (flags & DAWN_DEVICE_OUT) != 0, S,
                      stats));
  } else if (stats) {
    memset(stats, 0, offsetof(dawn_run_stats, frontier_sizes));
  }
  memcpy(wcc_nodes, nodes.data(), (size_t)S * 4);
  *s_wcc = S;
  return DAWN_OK;
}

dawn_status dawn_autotune(dawn_ctx* c, int32_t graph, const int32_t* sources, int32_t k,
                          uint32_t what, dawn_params* best) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  if (k <= 0 || !sources) return fail(DAWN_E_INVALID_ARG, "need k > 0 sample sources");
  if (what == 0 || (what & ~3u)) return fail(DAWN_E_INVALID_ARG, "what must be 1, 2 or 3");
  Ctx* ctx = C(c);
  std::shared_ptr<GraphRec> g;
  DAWN_TRY(get_graph(ctx, graph, &g));
  for (int32_t r = 0; r < k; ++r)
    if (sources[r] < 0 || sources[r] >= g->n)
      return fail(DAWN_E_INVALID_ARG, "sources[%d] outside [0, n)", r);
  DAWN_HIP(hipSetDevice(ctx->device));
  return autotune(ctx, g.get(), sources, k, what, best);
}

dawn_status dawn_serve_submit(dawn_ctx* c, int32_t graph, const int32_t* sources, int32_t k,
                              int32_t* dist_out, uint32_t flags, uint64_t* ticket) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  return serve_submit(C(c), graph, sources, k, dist_out, flags, ticket);
}

dawn_status dawn_serve_poll(dawn_ctx* c, uint64_t ticket, dawn_query_stats* qs) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  return serve_poll(C(c), ticket, 0, qs);
}

dawn_status dawn_serve_wait(dawn_ctx* c, uint64_t ticket, int32_t timeout_ms,
                            dawn_query_stats* qs) {
  clear_error();
  DAWN_TRY(check_ctx(c));
  return serve_poll(C(c), ticket, timeout_ms < 0 ? -1 : std::max(timeout_ms, 1), qs);
}

}  // extern "C"
