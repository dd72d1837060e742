// Batched multi-source level loop: up to 4096 sources advance together.
//
// APSP is the SSSP run from every source (paper Section 3.3, APSP cost), and
// each source's run is the same Boolean level step (Algorithms 1 and 2).  Here
// source r of a batch owns bit r%64 of 64-bit word r/64 in a row of W words
// kept per node, so one pass over the adjacency advances every source:
//
//  * vis[v][w]   bits of the sources that have reached v;
//  * nxt[L&1][v][w] bits that reached v for the first time at level L (the
//    frontier of the next level: the push direction reads them);
//  * act[w]      sources whose frontier is not empty yet.
//
// Pull (BOVM, Section 3.2, per bit):  acc = OR over in-neighbours u of vis[u],
// new = acc & ~vis[v] & act; the scan of v's in-list stops as soon as acc covers
// every still-needed bit (the early exit after Algorithm 1, for all lanes at
// once).  The test uses "visited" rather than "frontier"; both give the same
// bits for the reason given in the single-source kernels, applied per bit.
// Push (SOVM, Section 3.3, per bit): every frontier node u ORs
// nxt[u] & ~vis[v] into the new bits of each out-neighbour v.
//
// After each expansion a merge pass folds the new bits into vis tile by tile
// (64 consecutive nodes), transposes them in LDS and writes the distance
// rows: row r gets L - base[r] at every node whose bit r is new, as one
// coalesced 256-byte masked store per (row, tile).  base[r] is the level at
// which source r joined the batch (0 for dawn_mssp; the serving loop admits
// sources at later levels).
#include <string.h>

#include <algorithm>
#include <vector>

#include "batch.hpp"
#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

constexpr int kBatchBlock = 256;
constexpr int kChunk = 32;        // out-edges per push work item

// group of P lanes per node: lane w of the group handles word w
template <int P>
__device__ __forceinline__ u64 group_mask(int lane) {
  if (P == 64) return ~0ull;
  return ((1ull << P) - 1ull) << (lane & ~(P - 1));
}

// ------------------------------------------------------------- expansion --
template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_pull(BatchArgs a, int L) {
  const int lane = lane_id();
  const int w = lane & (P - 1);
  const int npw = kWave / P;
  const int sub = lane / P;
  const bool wok = w < a.W;
  const u64 gm = group_mask<P>(lane);
  const u64 actw = wok ? a.act[w] : 0ull;
  const size_t W = (size_t)a.W;
  u64* nxt = a.nxt[L & 1];
  u64 edges = 0;
  const unsigned gw = (blockIdx.x * kBatchBlock + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * kBatchBlock / kWave;
  for (unsigned base = gw * npw; base < (unsigned)a.n; base += nwaves * npw) {
    const int v = (int)base + sub;
    const bool valid = v < a.n;
    const u64 vw = (valid && wok) ? a.vis[(size_t)v * W + w] : ~0ull;
    const u64 need = (valid && wok) ? (actw & ~vw) : 0ull;
    const bool gneed = (__ballot(need != 0) & gm) != 0;
    u64 acc = 0;
    if (gneed) {
      const int s = a.ip[v], e = a.ip[v + 1];
      int j = s;
      bool sat = false;
      // four in-neighbours per step: independent loads in flight
      for (; j + 4 <= e; j += 4) {
        const int u0 = a.isrc[j], u1 = a.isrc[j + 1], u2 = a.isrc[j + 2], u3 = a.isrc[j + 3];
        if (wok) {
          acc |= a.vis[(size_t)u0 * W + w] | a.vis[(size_t)u1 * W + w] |
                 a.vis[(size_t)u2 * W + w] | a.vis[(size_t)u3 * W + w];
        }
        acc &= need;
        if ((__ballot(acc != need) & gm) == 0) {
          j += 4;
          sat = true;
          break;
        }
      }
      for (; !sat && j < e; ++j) {
        const int u = a.isrc[j];
        if (wok) acc |= a.vis[(size_t)u * W + w];
        acc &= need;
        if ((__ballot(acc != need) & gm) == 0) {
          ++j;
          break;
        }
      }
      if (w == 0) edges += (u64)(j - s);
    }
    if (acc) nxt[(size_t)v * W + w] = acc;
    const bool any = (__ballot(acc != 0) & gm) != 0;
    if (any && w == 0) atom_or(&a.touched[v >> 6], 1ull << (v & 63));
  }
  edges = wave_sum(edges);
  if (lane == 0 && edges) atom_add(&a.ctrl->lv[L & 1].edges, edges);
}

template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_push(BatchArgs a, int L) {
  const int lane = lane_id();
  const int w = lane & (P - 1);
  const int gpw = kWave / P;
  const bool wok = w < a.W;
  const u64 gm = group_mask<P>(lane);
  const size_t W = (size_t)a.W;
  const int pl = (L - 1) & 1;
  const unsigned nch = ld_relaxed(&a.ctrl->lv[pl].nchunks);
  const int32_t* cu = a.cu[pl];
  const int32_t* ck = a.ck[pl];
  const u64* front = a.nxt[pl];
  u64* out = a.nxt[L & 1];
  u64 edges = 0;
  const unsigned gw = (blockIdx.x * kBatchBlock + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * kBatchBlock / kWave;
  for (unsigned cb = gw * gpw; cb < nch; cb += nwaves * gpw) {
    const unsigned c = cb + (unsigned)(lane / P);
    const bool has = c < nch;
    int e0 = 0, e1 = 0;
    u64 f = 0;
    if (has) {
      const int u = cu[c];
      const int k = ck[c];
      const int r0 = a.rp[u];
      e0 = r0 + k * kChunk;
      e1 = min(e0 + kChunk, a.rp[u + 1]);
      if (wok) f = front[(size_t)u * W + w];
    }
    if (has && w == 0) edges += (u64)(e1 - e0);
    for (int e = e0; e < e1; ++e) {
      const int v = a.col[e];
      u64 b = 0;
      if (wok && f) {
        b = f & ~a.vis[(size_t)v * W + w];
        if (b) atom_or(&out[(size_t)v * W + w], b);
      }
      const bool any = (__ballot(b != 0) & gm) != 0;
      if (any && w == 0) {
        u64* tw = &a.touched[v >> 6];
        const u64 bit = 1ull << (v & 63);
        if (!(*tw & bit)) atom_or(tw, bit);
      }
    }
  }
  edges = wave_sum(edges);
  if (lane == 0 && edges) atom_add(&a.ctrl->lv[L & 1].edges, edges);
}

// ----------------------------------------------------------------- merge --
// One workgroup per touched tile of 64 nodes (grid-stride).  W <= 64.
__global__ __launch_bounds__(kBatchBlock) void batch_merge(BatchArgs a, int L) {
  __shared__ u64 tile[64 * 65];   // tile[w * 65 + j]: new bits of node v0+j, word w
  __shared__ u64 tor[64];         // OR of the tile per word
  __shared__ int tj[64];          // touched node offsets in the tile
  __shared__ int tcount;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  const int W = a.W;
  u64* nxt = a.nxt[L & 1];
  const int cl = L & 1;
  BatchLevel* lv = &a.ctrl->lv[cl];
  u64 act_acc = 0;   // thread w < W: OR of new bits over this block's tiles
  u64 bits = 0, se = 0, mf = 0;
  unsigned nodes = 0;
  const int ntiles = (a.n + 63) / 64;

  // clear the rows of the previous frontier (their bits were consumed by the
  // expansion of this level) and retire that frontier list
  if (L > 0) {
    const int pl = (L - 1) & 1;
    const unsigned nprev = ld_relaxed(&a.ctrl->lv[pl].nfront);
    u64* prev = a.nxt[pl];
    const int32_t* fl = a.fl[pl];
    for (unsigned i = blockIdx.x * (kBatchBlock / 64) + wave; i < nprev;
         i += gridDim.x * (kBatchBlock / 64)) {
      const int u = fl[i];
      if (lane < W) prev[(size_t)u * W + lane] = 0;
    }
  }

  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const u64 tw = a.touched[t];
    if (tw == 0) continue;
    const int v0 = t * 64;
    if (tid == 0) {
      int c = 0;
      u64 m = tw;
      while (m) {
        tj[c++] = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
      }
      tcount = c;
    }
    for (int i = tid; i < W * 65; i += kBatchBlock) tile[i] = 0;
    __syncthreads();
    const int tc = tcount;
    // each wave takes touched nodes; lane = word
    for (int i = wave; i < tc; i += kBatchBlock / kWave) {
      const int j = tj[i];
      const int v = v0 + j;
      u64 nb = 0;
      if (lane < W) {
        const size_t idx = (size_t)v * W + lane;
        nb = nxt[idx];
        a.vis[idx] |= nb;
        tile[lane * 65 + j] = nb;
      }
      const int deg = a.rp[v + 1] - a.rp[v];
      const u64 pc = (u64)__popcll(nb);
      bits += pc;
      se += pc * (u64)deg;
      // v joins the next frontier: node list and out-edge chunks
      if (lane == 0) {
        nodes += 1;
        mf += (u64)deg;
        const unsigned pos = atom_add(&lv->nfront, 1u);
        a.fl[cl][pos] = v;
        if (deg > 0) {
          const unsigned nch = (unsigned)((deg + kChunk - 1) / kChunk);
          const unsigned cb = atom_add(&lv->nchunks, nch);
          for (unsigned k = 0; k < nch; ++k) {
            a.cu[cl][cb + k] = v;
            a.ck[cl][cb + k] = (int32_t)k;
          }
        }
      }
    }
    __syncthreads();
    if (tid < W) {
      u64 o = 0;
      for (int j = 0; j < 64; ++j) o |= tile[tid * 65 + j];
      tor[tid] = o;
      act_acc |= o;
    }
    __syncthreads();
    // distance rows: wave `wave` takes words wave, wave+4, ...
    const int vj = v0 + lane;
    for (int w = wave; w < W; w += kBatchBlock / kWave) {
      u64 m = tor[w];
      const u64 mine = tile[w * 65 + lane];
      while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int r = w * 64 + b;
        if (((mine >> b) & 1ull) && vj < a.n) a.rows[r][vj] = L - a.base[r];
      }
    }
    if (tid == 0) a.touched[t] = 0;
    __syncthreads();
  }
  // lane activity and counters
  if (tid < W && act_acc) {
    u64* g = &a.ctrl->laneact[cl][tid];
    if (act_acc & ~ld_relaxed(g)) atom_or(g, act_acc);
  }
  bits = wave_sum(bits);
  se = wave_sum(se);
  if (lane == 0) {
    if (bits) atom_add(&lv->bits, bits);
    if (se) atom_add(&lv->se, se);
  }
  nodes = wave_sum(nodes);
  mf = wave_sum(mf);
  if (lane == 0) {
    if (nodes) atom_add(&lv->nodes, (u64)nodes);
    if (mf) atom_add(&lv->mf, mf);
  }
}

// ------------------------------------------------------------------ init --
// rows[r][0..n) = -1 for r < k
__global__ __launch_bounds__(kBatchBlock) void batch_fill_rows(BatchArgs a, int k, int r0) {
  const int r = r0 + blockIdx.y;
  if (r >= k) return;
  int32_t* row = a.rows[r];
  if (!row) return;
  const int n = a.n;
  const uintptr_t addr = (uintptr_t)row;
  if ((addr & 15) == 0 && (n & 3) == 0) {
    int4* r4 = (int4*)row;
    const int n4 = n >> 2;
    for (int i = blockIdx.x * kBatchBlock + threadIdx.x; i < n4; i += gridDim.x * kBatchBlock)
      r4[i] = make_int4(-1, -1, -1, -1);
  } else {
    for (int i = blockIdx.x * kBatchBlock + threadIdx.x; i < n; i += gridDim.x * kBatchBlock)
      row[i] = -1;
  }
}

__global__ __launch_bounds__(kBatchBlock) void batch_zero(u64* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kBatchBlock + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kBatchBlock)
    p[i] = 0;
}

// lane r of the batch starts at node src[r]: bit r of nxt[0][src[r]] and the node is touched
__global__ void batch_seed(BatchArgs a, const int32_t* src, int k) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < k; r += gridDim.x * blockDim.x) {
    const int s = src[r];
    const int w = r >> 6;
    atom_or(&a.nxt[0][(size_t)s * a.W + w], 1ull << (r & 63));
    atom_or(&a.touched[s >> 6], 1ull << (s & 63));
  }
}

// ------------------------------------------------------------------ host --
void batch_ws_destroy(BatchWs* w) {
  if (!w) return;
  Ctx* ctx = w->ctx;
  dev_free(ctx, w->vis, 0);
  dev_free(ctx, w->nxt[0], 0);
  dev_free(ctx, w->nxt[1], 0);
  dev_free(ctx, w->touched, 0);
  for (int i = 0; i < 2; ++i) {
    dev_free(ctx, w->fl[i], 0);
    dev_free(ctx, w->cu[i], 0);
    dev_free(ctx, w->ck[i], 0);
  }
  dev_free(ctx, w->ctrl, 0);
  dev_free(ctx, w->act, 0);
  dev_free(ctx, w->rows, 0);
  dev_free(ctx, w->base, 0);
  dev_free(ctx, w->src, 0);
  dev_free(ctx, w->stage, 0);
  if (ctx) ctx->used -= w->bytes;
  if (w->h_ctrl) hipHostFree(w->h_ctrl);
  if (w->ev0) hipEventDestroy(w->ev0);
  if (w->ev1) hipEventDestroy(w->ev1);
  if (w->stream && w->own_stream) hipStreamDestroy(w->stream);
  delete w;
}

dawn_status batch_ws_create(Ctx* ctx, const GraphRec* g, int lanes, size_t stage_ints,
                            BatchWs** out) {
  BatchWs* w = new BatchWs();
  w->ctx = ctx;
  w->n = g->n;
  w->lanes = lanes;
  const int W = (lanes + 63) / 64;
  w->Wmax = W;
  const size_t n = (size_t)g->n;
  const size_t nw = (n + 63) / 64;
  const size_t chunk_cap = (size_t)(g->m / kChunk) + n + 64;
  dawn_status s = DAWN_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (s != DAWN_OK) return;
    s = dev_alloc(ctx, p, bytes);
    if (s == DAWN_OK) w->bytes += bytes;
  };
  alloc((void**)&w->vis, n * W * 8);
  alloc((void**)&w->nxt[0], n * W * 8);
  alloc((void**)&w->nxt[1], n * W * 8);
  alloc((void**)&w->touched, nw * 8 + 64);
  for (int i = 0; i < 2; ++i) {
    alloc((void**)&w->fl[i], n * 4 + 64);
    alloc((void**)&w->cu[i], chunk_cap * 4);
    alloc((void**)&w->ck[i], chunk_cap * 4);
  }
  alloc((void**)&w->ctrl, sizeof(BatchCtrl));
  alloc((void**)&w->act, 64 * 8);
  alloc((void**)&w->rows, (size_t)4096 * sizeof(int32_t*));
  alloc((void**)&w->base, (size_t)4096 * 4);
  alloc((void**)&w->src, (size_t)4096 * 4);
  if (stage_ints) alloc((void**)&w->stage, stage_ints * 4);
  w->stage_ints = stage_ints;
  if (s != DAWN_OK) {
    batch_ws_destroy(w);
    return s;
  }
  hipError_t e = hipHostMalloc((void**)&w->h_ctrl, sizeof(BatchCtrl), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
  w->own_stream = true;
  if (e == hipSuccess) e = hipEventCreate(&w->ev0);
  if (e == hipSuccess) e = hipEventCreate(&w->ev1);
  if (e != hipSuccess) {
    batch_ws_destroy(w);
    return fail(DAWN_E_DEVICE, "batch workspace: %s", hipGetErrorString(e));
  }
  *out = w;
  return DAWN_OK;
}

BatchArgs batch_args(const GraphRec* g, BatchWs* w, int W) {
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.W = W;
  a.m = g->m;
  a.rp = g->rp;
  a.col = g->col;
  a.ip = g->ip;
  a.isrc = g->isrc;
  a.vis = w->vis;
  a.nxt[0] = w->nxt[0];
  a.nxt[1] = w->nxt[1];
  a.touched = w->touched;
  for (int i = 0; i < 2; ++i) {
    a.fl[i] = w->fl[i];
    a.cu[i] = w->cu[i];
    a.ck[i] = w->ck[i];
  }
  a.ctrl = w->ctrl;
  a.act = w->act;
  a.rows = w->rows;
  a.base = w->base;
  return a;
}

static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

dawn_status batch_launch_expand(Ctx* ctx, const BatchArgs& a, bool pull, int L, hipStream_t s) {
  const int P = pow2_at_least(a.W);
  const int grid = ctx->num_cu * 8;
#define DAWN_EXPAND(PP)                                                                  \
  case PP:                                                                               \
    if (pull)                                                                            \
      hipLaunchKernelGGL(batch_pull<PP>, dim3(grid), dim3(kBatchBlock), 0, s, a, L);    \
    else                                                                                 \
      hipLaunchKernelGGL(batch_push<PP>, dim3(grid), dim3(kBatchBlock), 0, s, a, L);    \
    break;
  switch (P) {
    DAWN_EXPAND(1)
    DAWN_EXPAND(2)
    DAWN_EXPAND(4)
    DAWN_EXPAND(8)
    DAWN_EXPAND(16)
    DAWN_EXPAND(32)
    DAWN_EXPAND(64)
    default: return fail(DAWN_E_INVALID_ARG, "batch too wide");
  }
#undef DAWN_EXPAND
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_merge(Ctx* ctx, const BatchArgs& a, int L, hipStream_t s) {
  hipLaunchKernelGGL(batch_merge, dim3(ctx->num_cu * 8), dim3(kBatchBlock), 0, s, a, L);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_fill(Ctx* ctx, const BatchArgs& a, int r0, int k, hipStream_t s) {
  // rows r0 .. k-1, at most 65535 per launch along y
  for (int b = r0; b < k; b += 65535) {
    const int rows = std::min(65535, k - b);
    const int gx = std::max(1, std::min((a.n / 4 + kBatchBlock - 1) / kBatchBlock, 64));
    hipLaunchKernelGGL(batch_fill_rows, dim3(gx, rows), dim3(kBatchBlock), 0, s, a, k, b);
  }
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_zero(Ctx* ctx, u64* p, size_t count, hipStream_t s) {
  if (!count) return DAWN_OK;
  const int grid = (int)std::max<size_t>(1, std::min<size_t>((count + kBatchBlock - 1) / kBatchBlock,
                                                              (size_t)ctx->num_cu * 16));
  hipLaunchKernelGGL(batch_zero, dim3(grid), dim3(kBatchBlock), 0, s, p, count);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_seed(Ctx* ctx, const BatchArgs& a, const int32_t* d_src, int k,
                              hipStream_t s) {
  (void)ctx;
  hipLaunchKernelGGL(batch_seed, dim3((k + 255) / 256), dim3(256), 0, s, a, d_src, k);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

// Choose push or pull for the next level from the counters of the last one.
bool batch_choose_pull(const dawn_params& p, const BatchLevel& last, long long m) {
  if (p.direction == 1) return false;
  if (p.direction == 2) return true;
  return (double)last.mf * (double)p.batch_alpha >= (double)m;
}

// One batch of k <= lanes sources through the per-level loop.
static dawn_status run_batch(Ctx* ctx, const GraphRec* g, BatchWs* w, const dawn_params& p,
                             const int32_t* h_src, int k, int32_t* const* h_rows,
                             BatchTotals* tot) {
  const int W = (k + 63) / 64;
  BatchArgs a = batch_args(g, w, W);
  hipStream_t s = w->stream;
  const size_t nW = (size_t)g->n * W;
  std::vector<int32_t> zeros(k, 0);
  DAWN_HIP(hipMemcpyAsync(w->src, h_src, (size_t)k * 4, hipMemcpyHostToDevice, s));
  DAWN_HIP(hipMemcpyAsync(w->rows, h_rows, (size_t)k * sizeof(int32_t*), hipMemcpyHostToDevice, s));
  DAWN_HIP(hipMemcpyAsync(w->base, zeros.data(), (size_t)k * 4, hipMemcpyHostToDevice, s));
  DAWN_HIP(hipMemsetAsync(w->ctrl, 0, sizeof(BatchCtrl), s));
  DAWN_TRY(batch_launch_zero(ctx, w->vis, nW, s));
  DAWN_TRY(batch_launch_zero(ctx, w->nxt[0], nW, s));
  DAWN_TRY(batch_launch_zero(ctx, w->nxt[1], nW, s));
  DAWN_TRY(batch_launch_zero(ctx, w->touched, ((size_t)g->n + 63) / 64, s));
  DAWN_HIP(hipEventRecord(w->ev0, s));
  DAWN_TRY(batch_launch_fill(ctx, a, 0, k, s));
  DAWN_TRY(batch_launch_seed(ctx, a, w->src, k, s));
  DAWN_TRY(batch_launch_merge(ctx, a, 0, s));
  int launches = 3;
  int last_nonempty = 0;
  for (int L = 1;; ++L) {
    const int pl = (L - 1) & 1;
    DAWN_HIP(hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, s));
    DAWN_HIP(hipStreamSynchronize(s));
    const BatchLevel prev = w->h_ctrl->lv[pl];
    tot->edges += prev.edges;
    tot->reached += prev.bits;
    tot->source_edges += prev.se;
    if (prev.bits) last_nonempty = L - 1;
    bool any = false;
    for (int i = 0; i < W; ++i) any |= w->h_ctrl->laneact[pl][i] != 0;
    if (!any) break;
    if (L > g->n + 1) return fail(DAWN_E_DEVICE, "watchdog: more than n levels");
    // active lanes and a clean slot for this level
    DAWN_HIP(hipMemcpyAsync(w->act, w->h_ctrl->laneact[pl], (size_t)W * 8, hipMemcpyHostToDevice, s));
    DAWN_HIP(hipMemsetAsync(&w->ctrl->lv[L & 1], 0, sizeof(BatchLevel), s));
    DAWN_HIP(hipMemsetAsync(&w->ctrl->laneact[L & 1][0], 0, 64 * 8, s));
    const bool pull = batch_choose_pull(p, prev, g->m);
    DAWN_TRY(batch_launch_expand(ctx, a, pull, L, s));
    DAWN_TRY(batch_launch_merge(ctx, a, L, s));
    launches += 2;
    if (pull) tot->pull_levels++; else tot->push_levels++;
  }
  DAWN_HIP(hipEventRecord(w->ev1, s));
  DAWN_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  DAWN_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
  tot->kernel_ms += ms;
  tot->launches += launches;
  tot->levels = std::max(tot->levels, last_nonempty + 1);
  return DAWN_OK;
}

dawn_status mssp_run(Ctx* ctx, GraphRec* g, const dawn_params& p, const int32_t* sources, int32_t k,
                     int32_t* dist, bool device_out, int64_t row_stride, dawn_run_stats* stats) {
  const uint64_t t0 = now_ns();
  const int lanes = std::min(p.batch_lanes, 4096);
  const int kb_max = std::min(lanes, (int)k);
  const size_t stage = device_out ? 0 : (size_t)kb_max * (size_t)g->n;
  BatchWs* w = nullptr;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    for (size_t i = 0; i < g->batch_pool.size(); ++i) {
      BatchWs* c = g->batch_pool[i];
      if (c->lanes >= kb_max && c->stage_ints >= stage) {
        w = c;
        g->batch_pool.erase(g->batch_pool.begin() + i);
        break;
      }
    }
  }
  if (!w) DAWN_TRY(batch_ws_create(ctx, g, kb_max, stage, &w));
  BatchTotals tot;
  memset(&tot, 0, sizeof(tot));
  dawn_status st = DAWN_OK;
  std::vector<int32_t*> rows(kb_max);
  for (int32_t b0 = 0; b0 < k && st == DAWN_OK; b0 += lanes) {
    const int kb = std::min(lanes, k - b0);
    for (int r = 0; r < kb; ++r)
      rows[r] = device_out ? dist + (size_t)(b0 + r) * row_stride : w->stage + (size_t)r * g->n;
    st = run_batch(ctx, g, w, p, sources + b0, kb, rows.data(), &tot);
    if (st == DAWN_OK && !device_out) {
      hipError_t e = hipMemcpy2DAsync(dist + (size_t)b0 * row_stride, (size_t)row_stride * 4,
                                      w->stage, (size_t)g->n * 4, (size_t)g->n * 4, kb,
                                      hipMemcpyDeviceToHost, w->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
      if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "copy to host: %s", hipGetErrorString(e));
    }
  }
  if (st == DAWN_OK) {
    std::lock_guard<std::mutex> lk(g->mu);
    g->batch_pool.push_back(w);
  } else {
    hipStreamSynchronize(w->stream);
    batch_ws_destroy(w);
    return st;
  }
  if (stats) {
    stats->levels = tot.levels;
    stats->push_levels = tot.push_levels;
    stats->pull_levels = tot.pull_levels;
    stats->launches = tot.launches;
    stats->edges_examined = (int64_t)tot.edges;
    stats->source_edges = (int64_t)tot.source_edges;
    stats->reached = (int64_t)tot.reached;
    stats->kernel_ms = tot.kernel_ms;
    stats->total_ms = (now_ns() - t0) / 1e6;
  }
  return DAWN_OK;
}

}  // namespace dawn
