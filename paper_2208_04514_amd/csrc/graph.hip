// Resident graphs: device CSR, in-lists (CSC) by transpose, and the largest
// weakly connected component with its induced subgraph.
//
// The paper keeps the adjacency as CSR for push (SOVM, Section 3.3) and as CSC
// for pull (BOVM, Section 3.2); both are built here once per upload.  The
// largest WCC (S_wcc, E_wcc in the SOVM cost of Section 3.3) is found on the
// device by lock-free union-find: every edge hooks the larger of its two roots
// under the smaller one with a compare-and-swap, so each component's root ends
// as its smallest node id, which is also the tie-break between equally large
// components.
#include <string.h>

#include <algorithm>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ long long block_excl_scan(long long x, long long* total) {
  __shared__ long long wsum[kScanBlock / kWave];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  // inclusive scan inside the wave (64-bit)
  long long incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    long long y = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  long long off = 0, tot = 0;
  for (int i = 0; i < kScanBlock / kWave; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// Sum of each tile of kScanTile inputs.
__global__ __launch_bounds__(kScanBlock) void scan_tile_sums(const int32_t* in, long long count,
                                                             long long* sums) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < count) s += in[base + i];
  long long tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place (one workgroup); sums[tiles] = total.
__global__ __launch_bounds__(kScanBlock) void scan_tile_offsets(long long* sums, long long tiles) {
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (long long b = 0; b < tiles; b += kScanBlock) {
    const long long i = b + threadIdx.x;
    long long x = i < tiles ? sums[i] : 0;
    long long tot;
    long long ex = block_excl_scan(x, &tot);
    if (i < tiles) sums[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[tiles] = carry;
}

__global__ __launch_bounds__(kScanBlock) void scan_tile_apply(const int32_t* in, long long count,
                                                              const long long* offs, int32_t* out) {
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < count ? in[base + i] : 0;
    s += v[i];
  }
  long long tot;
  long long ex = block_excl_scan(s, &tot) + offs[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) out[base + i] = (int32_t)ex;
    ex += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) out[count] = (int32_t)offs[gridDim.x];
}

// out[0..count] = exclusive prefix sums of in[0..count-1], out[count] = total.
static dawn_status scan_exclusive(Ctx* ctx, const int32_t* in, long long count, int32_t* out,
                                  hipStream_t s) {
  const long long tiles = std::max(1LL, (count + kScanTile - 1) / kScanTile);
  long long* sums = nullptr;
  DAWN_TRY(dev_alloc_n(ctx, &sums, (size_t)tiles + 1));
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, count, sums);
  hipLaunchKernelGGL(scan_tile_offsets, dim3(1), dim3(kScanBlock), 0, s, sums, tiles);
  hipLaunchKernelGGL(scan_tile_apply, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, count,
                     sums, out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(ctx, sums, ((size_t)tiles + 1) * sizeof(long long));
  if (e != hipSuccess) return fail(DAWN_E_DEVICE, "scan: %s", hipGetErrorString(e));
  return DAWN_OK;
}

// Row owning edge e: largest u with rp[u] <= e.
__device__ __forceinline__ int row_of(const int32_t* rp, int n, long long e) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((long long)rp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void count_in_degree(const int32_t* col, long long m, int32_t* cnt) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m;
       e += (long long)gridDim.x * blockDim.x)
    atomicAdd(&cnt[col[e]], 1);
}

// floor(log2(d)) for d >= 1
__device__ __forceinline__ int degree_class(int d) { return 31 - __clz(d); }

// Scatter the out-edges of the sources whose out-degree class is `cls` into
// the in-lists.  Run for cls from the largest class down to 0, it leaves
// every in-list ordered by decreasing source out-degree class (the order
// within a class follows the atomics): a pull that stops at the first hit
// then meets the high-degree in-neighbours, the likeliest to be reached,
// first.  Each wave takes 64 sources and walks the matching ones' out-lists
// with all of its lanes.
__global__ void scatter_in_edges(const int32_t* rp, const int32_t* col, int n, int cls,
                                 const int32_t* ip, int32_t* fill, int32_t* isrc) {
  const int lane = lane_id();
  const int nwaves = gridDim.x * blockDim.x / kWave;
  for (int b = (blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave; b < n; b += nwaves * kWave) {
    const int u = b + lane;
    int s = 0, d = 0;
    if (u < n) {
      s = rp[u];
      d = rp[u + 1] - s;
    }
    u64 match = __ballot(d > 0 && degree_class(d) == cls);
    while (match) {
      const int j = __builtin_ctzll(match);
      match &= match - 1;
      const int sj = __shfl(s, j, kWave), dj = __shfl(d, j, kWave);
      for (int e = lane; e < dj; e += kWave) {
        const int v = col[sj + e];
        const int pos = atomicAdd(&fill[v], 1);
        isrc[ip[v] + pos] = b + j;
      }
    }
  }
}

static int grid_for(Ctx* ctx, long long work, int block) {
  long long g = (work + block - 1) / block;
  return (int)std::max(1LL, std::min(g, (long long)ctx->num_cu * 16));
}

// CSC of (rp, col) into (ip, isrc); all device pointers.
static dawn_status build_csc(Ctx* ctx, int n, long long m, const int32_t* rp, const int32_t* col,
                             int32_t* ip, int32_t* isrc, hipStream_t s) {
  int32_t* cnt = nullptr;
  DAWN_TRY(dev_alloc_n(ctx, &cnt, (size_t)n + 1));
  dawn_status st = DAWN_OK;
  hipError_t e = hipMemsetAsync(cnt, 0, ((size_t)n + 1) * 4, s);
  if (e == hipSuccess && m > 0) {
    hipLaunchKernelGGL(count_in_degree, dim3(grid_for(ctx, m, 256)), dim3(256), 0, s, col, m, cnt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) st = scan_exclusive(ctx, cnt, n, ip, s);
  if (e == hipSuccess && st == DAWN_OK && m > 0) {
    e = hipMemsetAsync(cnt, 0, ((size_t)n + 1) * 4, s);
    const int max_class = 30;
    for (int cls = max_class; cls >= 0 && e == hipSuccess; --cls) {
      hipLaunchKernelGGL(scatter_in_edges, dim3(grid_for(ctx, (long long)n, 256)), dim3(256), 0, s,
                         rp, col, n, cls, ip, cnt, isrc);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  dev_free(ctx, cnt, ((size_t)n + 1) * 4);
  if (st != DAWN_OK) return st;
  if (e != hipSuccess) return fail(DAWN_E_DEVICE, "CSC build: %s", hipGetErrorString(e));
  return DAWN_OK;
}

__global__ void mark_no_in(const int32_t* ip, int n, u64* noin) {
  const int nw = (n + 63) / 64;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += gridDim.x * blockDim.x) {
    u64 bits = 0;
    for (int b = 0; b < 64 && w * 64 + b < n; ++b) {
      const int v = w * 64 + b;
      if (ip[v + 1] == ip[v]) bits |= 1ull << b;
    }
    noin[w] = bits;
  }
}

__global__ void list_pull_chunks(const int32_t* ip, int n, unsigned* count, int32_t* pcv,
                                 int32_t* pck) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int d = ip[v + 1] - ip[v];
    if (d < kPullBig) continue;
    const unsigned nch = (unsigned)((d + kPullChunk - 1) / kPullChunk);
    const unsigned b = atomicAdd(count, nch);
    for (unsigned k = 0; k < nch; ++k) {
      pcv[b + k] = v;
      pck[b + k] = (int32_t)k;
    }
  }
}

static void free_graph_buffers(GraphRec* g) {
  dev_free(g->ctx, g->rp, ((size_t)g->n + 1) * 4);
  dev_free(g->ctx, g->col, (size_t)std::max(g->m, 1LL) * 4);
  if (!g->shared_csc) {
    dev_free(g->ctx, g->ip, ((size_t)g->n + 1) * 4);
    dev_free(g->ctx, g->isrc, (size_t)std::max(g->m, 1LL) * 4);
  }
  dev_free(g->ctx, g->noin, (((size_t)g->n + 63) / 64) * 8);
  dev_free(g->ctx, g->pcv, g->pc_cap * 4);
  dev_free(g->ctx, g->pck, g->pc_cap * 4);
  g->pcv = g->pck = nullptr;
  g->rp = g->col = g->ip = g->isrc = nullptr;
  g->noin = nullptr;
}

GraphRec::~GraphRec() {
  for (auto& w : sssp_pool) w.reset();
  sssp_pool.clear();
  for (BatchWs* b : batch_pool) batch_ws_destroy(b);
  batch_pool.clear();
  if (stage) dev_free(ctx, stage, stage_bytes);
  stage = nullptr;
  wsssp_pool_free(this);
  if (wt) dev_free(ctx, wt, (size_t)std::max(m, 1LL) * 4);
  wt = nullptr;
  wcc_sub.reset();
  if (ctx) free_graph_buffers(this);
}

static dawn_status alloc_graph_buffers(Ctx* ctx, GraphRec* g) {
  const size_t n1 = (size_t)g->n + 1, mm = (size_t)std::max(g->m, 1LL);
  DAWN_TRY(dev_alloc_n(ctx, &g->rp, n1));
  DAWN_TRY(dev_alloc_n(ctx, &g->col, mm));
  if (g->shared_csc) {
    g->ip = g->rp;
    g->isrc = g->col;
  } else {
    DAWN_TRY(dev_alloc_n(ctx, &g->ip, n1));
    DAWN_TRY(dev_alloc_n(ctx, &g->isrc, mm));
  }
  DAWN_TRY(dev_alloc_n(ctx, &g->noin, ((size_t)g->n + 63) / 64));
  // chunks: sum over in-lists of d >= kPullBig entries of ceil(d / kPullChunk)
  g->pc_cap = (size_t)(g->m / kPullChunk) + (size_t)(g->m / kPullBig) + 1;
  DAWN_TRY(dev_alloc_n(ctx, &g->pcv, g->pc_cap));
  DAWN_TRY(dev_alloc_n(ctx, &g->pck, g->pc_cap));
  g->bytes = (g->shared_csc ? 1 : 2) * (n1 + mm) * 4 + (((size_t)g->n + 63) / 64) * 8 +
             g->pc_cap * 8;
  return DAWN_OK;
}

// Per-graph metadata built from the CSC: the no-in-edge bitmap and the
// chunk list of long in-lists.
static dawn_status finish_noin(Ctx* ctx, GraphRec* g, hipStream_t s) {
  const int nw = (g->n + 63) / 64;
  unsigned* count = nullptr;
  DAWN_TRY(dev_alloc_n(ctx, &count, 1));
  hipLaunchKernelGGL(mark_no_in, dim3(grid_for(ctx, nw, 256)), dim3(256), 0, s, g->ip, g->n, g->noin);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemsetAsync(count, 0, sizeof(unsigned), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(list_pull_chunks, dim3(grid_for(ctx, g->n, 256)), dim3(256), 0, s, g->ip,
                       g->n, count, g->pcv, g->pck);
    e = hipGetLastError();
  }
  unsigned npc = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&npc, count, sizeof(unsigned), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(ctx, count, sizeof(unsigned));
  if (e != hipSuccess) return fail(DAWN_E_DEVICE, "graph metadata: %s", hipGetErrorString(e));
  if (npc > g->pc_cap) return fail(DAWN_E_DEVICE, "pull chunk list overflow");
  g->npc = (int32_t)npc;
  return DAWN_OK;
}

// Symmetry check for DAWN_SHARED_CSC: the edge multiset equals its reverse
// iff, for a hash h of ordered pairs, the sums of h(u, v) and of h(v, u)
// over the edges agree (two independent 64-bit mixes; a non-symmetric graph
// passes with probability ~2^-128), and every node's out-degree equals its
// in-degree.
// SplitMix64's output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): the golden-ratio increment,
// then two xor-shift-multiply rounds.
static u64 mix64(u64 x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

static bool is_symmetric(int n, long long m, const int32_t* rp, const int32_t* col) {
  std::vector<int32_t> indeg((size_t)n, 0);
  u64 f1 = 0, r1 = 0, f2 = 0, r2 = 0;
  for (int u = 0; u < n; ++u)
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
      const u64 v = (u64)col[e];
      indeg[(size_t)v] += 1;
      const u64 a = ((u64)u << 32) | v, b = (v << 32) | (u64)u;
      f1 += mix64(a);
      r1 += mix64(b);
      f2 += mix64(a ^ 0x5851f42d4c957f2dull);
      r2 += mix64(b ^ 0x5851f42d4c957f2dull);
    }
  (void)m;
  for (int u = 0; u < n; ++u)
    if (indeg[(size_t)u] != rp[u + 1] - rp[u]) return false;
  return f1 == r1 && f2 == r2;
}

static dawn_status graph_components(Ctx* ctx, GraphRec* g, hipStream_t s);

dawn_status graph_build(Ctx* ctx, GraphRec* g, const int32_t* h_rp, const int32_t* h_col) {
  const int n = g->n;
  const long long m = g->m;
  // validation and degree metadata (host arrays)
  if (h_rp[0] != 0) return fail(DAWN_E_BAD_GRAPH, "row_ptr[0] = %d, expected 0", h_rp[0]);
  int maxdeg = 0, zero = 0;
  for (int u = 0; u < n; ++u) {
    const long long d = (long long)h_rp[u + 1] - h_rp[u];
    if (d < 0) return fail(DAWN_E_BAD_GRAPH, "row_ptr decreases at node %d", u);
    if (d > maxdeg) maxdeg = (int)d;
    if (d == 0) ++zero;
  }
  if ((long long)h_rp[n] != m)
    return fail(DAWN_E_BAD_GRAPH, "row_ptr[n] = %d but m = %lld", h_rp[n], m);
  for (long long e = 0; e < m; ++e)
    if (h_col[e] < 0 || h_col[e] >= n)
      return fail(DAWN_E_BAD_GRAPH, "col[%lld] = %d outside [0, %d)", e, h_col[e], n);
  if (g->shared_csc && !is_symmetric(n, m, h_rp, h_col))
    return fail(DAWN_E_BAD_GRAPH, "DAWN_SHARED_CSC: the graph is not symmetric");
  g->max_out_deg = maxdeg;
  g->zero_out = zero;
  g->ctx = ctx;
  DAWN_TRY(alloc_graph_buffers(ctx, g));
  hipStream_t s = nullptr;
  DAWN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipError_t e = hipMemcpyAsync(g->rp, h_rp, ((size_t)n + 1) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m > 0)
    e = hipMemcpyAsync(g->col, h_col, (size_t)m * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dawn_status st = DAWN_OK;
  if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "upload: %s", hipGetErrorString(e));
  if (st == DAWN_OK && !g->shared_csc) st = build_csc(ctx, n, m, g->rp, g->col, g->ip, g->isrc, s);
  if (st == DAWN_OK) st = finish_noin(ctx, g, s);
  if (st == DAWN_OK) st = graph_components(ctx, g, s);
  hipStreamDestroy(s);
  return st;
}

// ----------------------------------------------------------------- WCC ----
__device__ __forceinline__ int uf_find(int* parent, int x) {
  for (;;) {
    int p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    // path halving: point x at its grandparent (any ancestor is valid)
    int gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp != p)
      __hip_atomic_compare_exchange_strong(&parent[x], &p, gp, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

__global__ void uf_init(int* parent, int n) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    parent[v] = v;
}

__global__ void uf_hook(const int32_t* rp, const int32_t* col, int n, long long m, int* parent) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < m;
       e += (long long)gridDim.x * blockDim.x) {
    int a = row_of(rp, n, e);
    int b = col[e];
    for (;;) {
      a = uf_find(parent, a);
      b = uf_find(parent, b);
      if (a == b) break;
      int hi = a > b ? a : b, lo = a > b ? b : a;
      int expect = hi;
      if (__hip_atomic_compare_exchange_strong(&parent[hi], &expect, lo, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        break;
      a = hi;
      b = lo;
    }
  }
}

// label[v] = root, and component sizes per root.  Lanes of a wave cover
// consecutive nodes, which mostly share one root: that root's count is added
// once per wave.
__global__ void uf_label(int* parent, int n, int32_t* sizes) {
  const int lane = lane_id();
  const int nwaves = gridDim.x * blockDim.x / kWave;
  for (int base = (blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave; base < n;
       base += nwaves * kWave) {
    const int v = base + lane;
    const bool valid = v < n;
    const int r = valid ? uf_find(parent, v) : -1;
    const int r0 = __shfl(r, 0, kWave);
    const u64 same = __ballot(valid && r == r0);
    if (valid) parent[v] = r;
    if (lane == 0) atomicAdd(&sizes[r0], (int)__popcll(same));
    if (valid && r != r0) atomicAdd(&sizes[r], 1);
  }
}

__global__ void comp_size_of(const int* label, const int32_t* sizes, int n, int32_t* out) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    out[v] = sizes[label[v]];
}

// Size of every node's weakly connected component (union-find over the
// edges taken undirected), kept on the host: a source in a small component
// is traversed by one workgroup.
static dawn_status graph_components(Ctx* ctx, GraphRec* g, hipStream_t s) {
  const int n = g->n;
  int* parent = nullptr;
  int32_t *sizes = nullptr, *per = nullptr;
  dawn_status st = DAWN_OK;
  if ((st = dev_alloc_n(ctx, &parent, n)) || (st = dev_alloc_n(ctx, &sizes, n)) ||
      (st = dev_alloc_n(ctx, &per, n))) {
    dev_free(ctx, parent, (size_t)n * 4);
    dev_free(ctx, sizes, (size_t)n * 4);
    dev_free(ctx, per, (size_t)n * 4);
    return st;
  }
  const int gb = grid_for(ctx, n, 256);
  hipError_t e = hipMemsetAsync(sizes, 0, (size_t)n * 4, s);
  hipLaunchKernelGGL(uf_init, dim3(gb), dim3(256), 0, s, parent, n);
  if (g->m > 0)
    hipLaunchKernelGGL(uf_hook, dim3(grid_for(ctx, g->m, 256)), dim3(256), 0, s, g->rp, g->col, n,
                       g->m, parent);
  hipLaunchKernelGGL(uf_label, dim3(gb), dim3(256), 0, s, parent, n, sizes);
  hipLaunchKernelGGL(comp_size_of, dim3(gb), dim3(256), 0, s, parent, sizes, n, per);
  if (e == hipSuccess) e = hipGetLastError();
  g->comp_size.resize((size_t)n);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->comp_size.data(), per, (size_t)n * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(ctx, parent, (size_t)n * 4);
  dev_free(ctx, sizes, (size_t)n * 4);
  dev_free(ctx, per, (size_t)n * 4);
  if (e != hipSuccess) {
    g->comp_size.clear();
    return fail(DAWN_E_DEVICE, "components: %s", hipGetErrorString(e));
  }
  return DAWN_OK;
}

__global__ void uf_best(const int32_t* sizes, int n, u64* best) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int s = sizes[v];
    if (s > 0) {
      const u64 key = ((u64)(unsigned)s << 32) | (u64)(0xffffffffu - (unsigned)v);
      atomicMax(best, key);
    }
  }
}

__global__ void wcc_flags(const int* label, int n, const u64* best, int32_t* flag) {
  const int root = (int)(0xffffffffu - (unsigned)(*best & 0xffffffffull));
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    flag[v] = label[v] == root ? 1 : 0;
}

// pos = exclusive scan of flags: members go to nodes[pos[v]], degrees of the
// induced subgraph to sdeg
__global__ void wcc_compact(const int32_t* flag, const int32_t* pos, const int32_t* rp, int n,
                            int32_t* nodes, int32_t* sdeg) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (flag[v]) {
      nodes[pos[v]] = v;
      sdeg[pos[v]] = rp[v + 1] - rp[v];
    }
  }
}

// copy and renumber the out-lists of the members (every target is a member)
__global__ void wcc_edges(const int32_t* nodes, int s, const int32_t* rp, const int32_t* col,
                          const int32_t* pos, const int32_t* srp, int32_t* scol) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * blockDim.x / kWave;
  const int lane = lane_id();
  for (int i = wave; i < s; i += nwaves) {
    const int v = nodes[i];
    const int b = rp[v], e = rp[v + 1], o = srp[i];
    for (int j = b + lane; j < e; j += kWave) scol[o + (j - b)] = pos[col[j]];
  }
}

dawn_status graph_wcc(Ctx* ctx, GraphRec* g, hipStream_t s) {
  const int n = g->n;
  int* parent = nullptr;
  int32_t *sizes = nullptr, *flag = nullptr, *pos = nullptr, *nodes = nullptr, *sdeg = nullptr;
  u64* best = nullptr;
  dawn_status st = DAWN_OK;
  auto cleanup = [&]() {
    dev_free(ctx, parent, (size_t)n * 4);
    dev_free(ctx, sizes, (size_t)n * 4);
    dev_free(ctx, flag, (size_t)n * 4);
    dev_free(ctx, pos, ((size_t)n + 1) * 4);
    dev_free(ctx, nodes, (size_t)n * 4);
    dev_free(ctx, sdeg, (size_t)n * 4);
    dev_free(ctx, best, 8);
  };
  if ((st = dev_alloc_n(ctx, &parent, n)) || (st = dev_alloc_n(ctx, &sizes, n)) ||
      (st = dev_alloc_n(ctx, &flag, n)) || (st = dev_alloc_n(ctx, &pos, (size_t)n + 1)) ||
      (st = dev_alloc_n(ctx, &nodes, n)) || (st = dev_alloc_n(ctx, &sdeg, n)) ||
      (st = dev_alloc_n(ctx, &best, 1))) {
    cleanup();
    return st;
  }
  const int gb = grid_for(ctx, n, 256);
  hipMemsetAsync(sizes, 0, (size_t)n * 4, s);
  hipMemsetAsync(best, 0, 8, s);
  hipLaunchKernelGGL(uf_init, dim3(gb), dim3(256), 0, s, parent, n);
  if (g->m > 0)
    hipLaunchKernelGGL(uf_hook, dim3(grid_for(ctx, g->m, 256)), dim3(256), 0, s, g->rp, g->col, n,
                       g->m, parent);
  hipLaunchKernelGGL(uf_label, dim3(gb), dim3(256), 0, s, parent, n, sizes);
  hipLaunchKernelGGL(uf_best, dim3(gb), dim3(256), 0, s, sizes, n, best);
  hipLaunchKernelGGL(wcc_flags, dim3(gb), dim3(256), 0, s, parent, n, best, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    cleanup();
    return fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
  }
  if ((st = scan_exclusive(ctx, flag, n, pos, s)) != DAWN_OK) {
    cleanup();
    return st;
  }
  hipLaunchKernelGGL(wcc_compact, dim3(gb), dim3(256), 0, s, flag, pos, g->rp, n, nodes, sdeg);
  int32_t s_wcc = 0;
  e = hipMemcpyAsync(&s_wcc, pos + n, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
  }
  // induced subgraph
  auto sub = std::make_shared<GraphRec>();
  sub->ctx = ctx;
  sub->n = s_wcc;
  sub->params = g->params;
  sub->shared_csc = g->shared_csc;   // an induced subgraph of a symmetric graph is symmetric
  int32_t* srp = nullptr;
  if ((st = dev_alloc_n(ctx, &srp, (size_t)s_wcc + 1)) != DAWN_OK) {
    cleanup();
    sub->ctx = nullptr;
    return st;
  }
  st = scan_exclusive(ctx, sdeg, s_wcc, srp, s);
  int32_t sm = 0;
  if (st == DAWN_OK) {
    e = hipMemcpyAsync(&sm, srp + s_wcc, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
  }
  if (st == DAWN_OK) {
    sub->m = sm;
    st = alloc_graph_buffers(ctx, sub.get());
  }
  if (st == DAWN_OK) {
    hipMemcpyAsync(sub->rp, srp, ((size_t)s_wcc + 1) * 4, hipMemcpyDeviceToDevice, s);
    if (sm > 0)
      hipLaunchKernelGGL(wcc_edges, dim3(grid_for(ctx, (long long)s_wcc * kWave, 256)), dim3(256),
                         0, s, nodes, s_wcc, g->rp, g->col, pos, srp, sub->col);
    e = hipGetLastError();
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
  }
  if (st == DAWN_OK && !sub->shared_csc)
    st = build_csc(ctx, s_wcc, sm, sub->rp, sub->col, sub->ip, sub->isrc, s);
  if (st == DAWN_OK) st = finish_noin(ctx, sub.get(), s);
  std::vector<int32_t> h_nodes(s_wcc);
  if (st == DAWN_OK && s_wcc > 0) {
    e = hipMemcpyAsync(h_nodes.data(), nodes, (size_t)s_wcc * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
  }
  if (st == DAWN_OK) {
    // degree metadata of the subgraph (host copy of its offsets)
    std::vector<int32_t> h_srp((size_t)s_wcc + 1);
    e = hipMemcpy(h_srp.data(), srp, ((size_t)s_wcc + 1) * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "wcc: %s", hipGetErrorString(e));
    int maxd = 0, z = 0;
    for (int i = 0; i < s_wcc; ++i) {
      int d = h_srp[i + 1] - h_srp[i];
      maxd = std::max(maxd, d);
      z += d == 0;
    }
    sub->max_out_deg = maxd;
    sub->zero_out = z;
  }
  dev_free(ctx, srp, ((size_t)s_wcc + 1) * 4);
  cleanup();
  if (st != DAWN_OK) return st;
  g->wcc_nodes = std::move(h_nodes);
  g->wcc_sub = sub;
  g->wcc_ready = true;
  return DAWN_OK;
}

}  // namespace dawn
