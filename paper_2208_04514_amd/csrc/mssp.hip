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
// After each expansion a merge pass folds the new bits into vis and records
// each new bit's relative level L - base[r] in bit-planes: plane b holds bit b
// of that level for every (node, source).  base[r] is the level at which
// source r joined the batch (0 for dawn_mssp; the serving loop admits sources
// at later levels).  Distances are written once, at the end, by an emission
// pass that rebuilds each level from the planes and stores every row as
// whole 256-byte segments (64 consecutive nodes), -1 where the source's bit
// never arrived; no row is touched while the levels run.
//
// dawn_mssp and APSP run the level loop on the device: a one-wave control
// kernel before each level applies the direction rule and ends the run, and
// the host only enqueues levels in chunks.  Serving steps levels from the
// host, where it admits and retires queries.
#include <string.h>

#include <algorithm>
#include <vector>

#include "batch.hpp"
#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

constexpr int kBatchBlock = 256;
constexpr int kBigB = 64;         // least out-degree from which a frontier node's edges may be
                                  //   chunked (the chunk lists are sized for it); the knob
                                  //   batch_big_degree (a.big_b) picks the threshold
constexpr int kChunkB = 64;       // out-edges per chunk of a big-degree node

// group of P lanes per node: lane w of the group handles word w
template <int P>
__device__ __forceinline__ u64 group_mask(int lane) {
  if (P == 64) return ~0ull;
  return ((1ull << (P & 63)) - 1ull) << (lane & ~(P - 1));
}

// the low P bits
template <int P>
__device__ __forceinline__ u64 low_mask() {
  return P == 64 ? ~0ull : (1ull << (P & 63)) - 1ull;
}

__device__ __forceinline__ u64 shfl64(u64 x, int src) {
  unsigned lo = __shfl((unsigned)x, src, kWave), hi = __shfl((unsigned)(x >> 32), src, kWave);
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 shfl_xor64(u64 x, int m) {
  unsigned lo = __shfl_xor((unsigned)x, m, kWave), hi = __shfl_xor((unsigned)(x >> 32), m, kWave);
  return ((u64)hi << 32) | lo;
}

// Append the out-edge chunks of node v (when big) to level L's chunk list,
// one counter atomic per wave (wave-uniform call).
__device__ __forceinline__ void push_chunks_wave(const BatchArgs& a, int L, int v, int deg,
                                                 bool big) {
  const int nch = big ? (deg + kChunkB - 1) / kChunkB : 0;
  const int incl = wave_incl_scan(nch);
  const int total = __shfl(incl, kWave - 1, kWave);
  if (total == 0) return;
  unsigned base = 0;
  if (lane_id() == kWave - 1) base = atom_add(&a.ctrl->lv[L & 1].nchunks, (unsigned)total);
  base = (unsigned)__shfl((int)base, kWave - 1, kWave);
  const unsigned b0 = base + (unsigned)(incl - nch);
  for (int k = 0; k < nch; ++k) {
    a.cu[L & 1][b0 + k] = v;
    a.ck[L & 1][b0 + k] = (int32_t)k;
  }
}

// Sum `edges` over the workgroup and add it to the level's stripe (every
// thread of the workgroup must call it).
__device__ __forceinline__ void block_add_edges(const BatchArgs& a, int L, u64 edges) {
  __shared__ u64 part[kBatchBlock / kWave];
  edges = wave_sum(edges);
  if (lane_id() == 0) part[threadIdx.x / kWave] = edges;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 x = 0;
    for (int i = 0; i < kBatchBlock / kWave; ++i) x += part[i];
    if (x) atom_add(&a.ctrl->lv[L & 1].s[blockIdx.x % kStripes].edges, x);
  }
}

// Big-degree nodes found by a workgroup are staged in LDS and their chunks
// listed with one counter atomic per workgroup (the L2 performs atomics on
// one line at a time, and a dense level has thousands of such nodes).
constexpr int kChunkStage = 1024;

struct ChunkStage {
  int32_t v[kChunkStage];
  int32_t c[kChunkStage];
  unsigned n;
};

// Stage node v (when big) with its chunk count; past the stage's end the
// wave lists its own (wave-uniform call).
__device__ __forceinline__ void stage_chunks_wave(const BatchArgs& a, int L, ChunkStage& cs, int v,
                                                  int deg, bool big) {
  const int nch = big ? (deg + kChunkB - 1) / kChunkB : 0;
  const u64 bm = __ballot(nch > 0);
  if (!bm) return;
  const int lead = __ffsll((unsigned long long)bm) - 1;
  unsigned base = 0;
  if (lane_id() == lead) base = atomicAdd(&cs.n, (unsigned)__popcll(bm));
  base = (unsigned)__shfl((int)base, lead, kWave);
  const unsigned slot = base + (unsigned)__popcll(bm & lanes_below());
  const bool staged = nch > 0 && slot < (unsigned)kChunkStage;
  if (staged) {
    cs.v[slot] = v;
    cs.c[slot] = nch;
  }
  push_chunks_wave(a, L, v, deg, nch > 0 && !staged);
}

// List the staged nodes' chunks (every thread of the workgroup calls it,
// after a barrier that follows the last staging).
__device__ __forceinline__ void flush_chunk_stage(const BatchArgs& a, int L, ChunkStage& cs) {
  constexpr int PER = kChunkStage / kBatchBlock;
  __shared__ int wtot[kBatchBlock / kWave];
  __shared__ unsigned gbase;
  const unsigned nst = min(cs.n, (unsigned)kChunkStage);
  if (nst == 0) return;   // uniform
  const int t = threadIdx.x, lane = lane_id(), wv = t / kWave;
  int mine = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const unsigned i = (unsigned)(t * PER + q);
    if (i < nst) mine += cs.c[i];
  }
  const int incl = wave_incl_scan(mine);
  if (lane == kWave - 1) wtot[wv] = incl;
  __syncthreads();
  if (t == 0) {
    unsigned tot = 0;
    for (int i = 0; i < kBatchBlock / kWave; ++i) {
      const unsigned x = (unsigned)wtot[i];
      wtot[i] = (int)tot;
      tot += x;
    }
    gbase = atom_add(&a.ctrl->lv[L & 1].nchunks, tot);
  }
  __syncthreads();
  unsigned b = gbase + (unsigned)wtot[wv] + (unsigned)(incl - mine);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const unsigned i = (unsigned)(t * PER + q);
    if (i < nst) {
      const int v = cs.v[i], nch = cs.c[i];
      for (int k = 0; k < nch; ++k) {
        a.cu[L & 1][b + k] = v;
        a.ck[L & 1][b + k] = (int32_t)k;
      }
      b += (unsigned)nch;
    }
  }
}

// ------------------------------------------------------------- expansion --
// Lane i of the group reads value x of group lane i (group-uniform call).
template <int P>
__device__ __forceinline__ int group_read(int x, int gb, int i) {
  if (P == 64) return __builtin_amdgcn_readlane(x, i);
  return __shfl(x, gb + i, kWave);
}

template <int P>
__device__ __forceinline__ u64 group_read64(u64 x, int gb, int i) {
  const unsigned lo = (unsigned)group_read<P>((int)(unsigned)x, gb, i);
  const unsigned hi = (unsigned)group_read<P>((int)(unsigned)(x >> 32), gb, i);
  return ((u64)hi << 32) | lo;
}

// OR into acc the visited bits of in-edges [s, e) that lie in `need`,
// stopping once every lane of the group has all of its word's needed bits
// (group-uniform call; gb = the group's first lane).  Returns the number of
// in-edges read.
//
// Per lane r, a node v not yet visited in r after level L - 1 lies at
// distance >= L, and an in-neighbour visited in r lies at <= L - 1, so v is
// at exactly L iff such an in-neighbour exists (the BOVM test of Algorithm 1
// on the visited set, per bit).  The visited rows saturate `need` sooner than
// the last level's new bits would (a hub reached early covers most lanes at
// once; in-lists list high-degree sources first), so the scan stops after
// fewer row reads.  Only the words that the visited word map marks nonzero
// are loaded.  The group reads EPL x P in-edges and their map words at a time
// (lane i takes edges i, i + P, ...: narrow groups take several, so a short
// row still keeps loads in flight), then walks the edges whose source has
// visited bits, each lane loading its own word of those rows.
template <int P>
__device__ __forceinline__ int pull_scan(const BatchArgs& a, const u64* front, const u64* fm, int s,
                                         int e, u64 need, int w, int gb, u64 gm, u64& acc) {
  constexpr int EPL = P >= 16 ? 1 : 16 / P;
  const size_t W = (size_t)a.Ws;
  int j = s;
  while (j < e) {
    int my_u[EPL];
    u64 my_m[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      my_u[k] = 0;
      my_m[k] = 0;
      if (j + k * P + w < e) my_u[k] = a.isrc[j + k * P + w];
    }
#pragma unroll
    for (int k = 0; k < EPL; ++k)
      if (j + k * P + w < e) my_m[k] = fm[my_u[k]];
    j += EPL * P;
    u64 r = 0;
    if constexpr (P <= 8) {
      // narrow group: every (slot k, lane i) edge's word is loaded at once
      const bool want = acc != need;
#pragma unroll
      for (int k = 0; k < EPL; ++k)
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const int u = group_read<P>(my_u[k], gb, i);
          const u64 m = group_read64<P>(my_m[k], gb, i);
          if (want && ((m >> w) & 1ull)) r |= front[(size_t)u * W + w];
        }
      acc |= r & need;
      if ((__ballot(acc != need) & gm) == 0) break;
      continue;
    }
    // wide groups (EPL = 1): the edges whose source has visited words, in
    // list order, in rounds of row loads that are all in flight together;
    // the exit test follows every round (two rows first: a hub early in the
    // list usually covers every needed lane), so a covered node stops after
    // the row that covered it instead of at the end of the P edges.  The
    // groups of a wave run the rounds in step (a group with nothing left
    // idles), so the cover test's ballot sees every lane of the wave.
    const int j0 = j - P;
    u64 hits = (__ballot(my_m[0] != 0) & gm) >> gb;   // bit i: edge j0 + i has visited words
    int round = 2;
    bool covered = false;
    while (__ballot(hits != 0) != 0) {
      u64 val[8];
      int last = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        val[q] = 0;
        if (q < round && hits) {
          const int i = __builtin_ctzll(hits);
          hits &= hits - 1;
          last = i;
          const int u = group_read<P>(my_u[0], gb, i);
          const u64 m = group_read64<P>(my_m[0], gb, i);
          if (((m >> w) & 1ull) && acc != need) val[q] = front[(size_t)u * W + w];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) r |= val[q];
      acc |= r & need;
      const bool group_covered = (__ballot(acc != need) & gm) == 0;
      if (group_covered && !covered) {
        covered = true;
        j = j0 + last + 1;
      }
      if (covered) hits = 0;
      round = 8;
    }
    if (covered) break;
  }
  return min(j, e) - s;
}

// Narrow batched rows (<= 8 words): an in-list longer than this is scanned
// by the whole wave, 64 edges per step.
// (the knob batch_wide_scan, a.wide_scan; 48 by default)

// Narrow rows (W <= P <= 8 words): the whole wave scans in-edges [s, e) of
// one node, one edge per lane and step, and ORs each word's bits across the
// wave.  needw / accw: the node's needed and found bits per word
// (wave-uniform).  Returns the number of in-edges read (wave-uniform call).
template <int P>
__device__ __forceinline__ int wave_scan(const BatchArgs& a, const u64* front, const u64* fm, int s,
                                         int e, const u64* needw, u64* accw) {
  const size_t W = (size_t)a.Ws;
  const int lane = lane_id();
  int j = s;
  while (j < e) {
    int u = 0;
    u64 m = 0;
    if (j + lane < e) {
      u = a.isrc[j + lane];
      m = fm[u];
    }
    j += kWave;
    u64 loc[P];
#pragma unroll
    for (int x = 0; x < P; ++x) {
      loc[x] = 0;
      if (x < a.W && ((m >> x) & 1ull) && accw[x] != needw[x]) loc[x] = front[(size_t)u * W + x];
    }
    bool done = true;
#pragma unroll
    for (int x = 0; x < P; ++x) {
      u64 r = loc[x] & needw[x];
      for (int off = 1; off < kWave; off <<= 1) r |= shfl_xor64(r, off);
      accw[x] |= r;
      done = done && accw[x] == needw[x];
    }
    if (done) break;
  }
  return min(j, e) - s;
}

// In a device-driven loop a level's kernels check the run state first: all
// of them stand down once no lane is active, and only the expansion of the
// chosen direction (dir 0 push, 1 pull; -1 the merge) runs.
__device__ __forceinline__ bool batch_gate_open(const BatchArgs& a, int dir) {
  if (!a.gated) return true;
  const BatchRun& r = a.ctrl->run;
  if (ld_relaxed(&r.done)) return false;
  return dir < 0 || ld_relaxed(&r.pull) == dir;
}

template <int P>
__device__ __forceinline__ void pull_level(const BatchArgs& a, int L) {
  const int lane = lane_id();
  const int w = lane & (P - 1);
  const int npw = kWave / P;
  const int sub = lane / P;
  const bool wok = w < a.W;
  const u64 gm = group_mask<P>(lane);
  const int gb = P == 64 ? 0 : (lane & ~(P - 1));
  const u64 actw = wok ? a.act[w] : 0ull;
  const size_t W = (size_t)a.Ws;
  // the in-neighbours' visited rows (vis is only written by the merge, after
  // this step) and the map of their possibly nonzero words
  const u64* front = a.vis;
  const u64* fm = a.vmap;
  u64* nxt = a.nxt[L & 1];
  u64* T = a.touched[L & 1];
  u64 edges = 0;
  const unsigned gw = (blockIdx.x * kBatchBlock + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * kBatchBlock / kWave;

  if constexpr (P <= 8) {
    // narrow rows: a wave per chunk of a long in-list
    for (unsigned c = gw; c < (unsigned)a.npc; c += nwaves) {
      const int v = a.pcv[c];
      const int s = a.ip[v] + a.pck[c] * kPullChunk;
      const int e = min(s + kPullChunk, a.ip[v + 1]);
      const u64 mine = lane < a.W ? a.act[lane] & ~a.vis[(size_t)v * W + lane] : 0ull;
      u64 needw[P], accw[P];
      bool any_need = false;
#pragma unroll
      for (int x = 0; x < P; ++x) {
        needw[x] = shfl64(mine, x);
        accw[x] = 0;
        any_need = any_need || needw[x] != 0;
      }
      if (!any_need) continue;
      const int nr = wave_scan<P>(a, front, fm, s, e, needw, accw);
      if (lane == 0) edges += (u64)nr;
      u64 got = 0;
#pragma unroll
      for (int x = 0; x < P; ++x)
        if (x == lane) got = accw[x];
      if (got) atom_or(&nxt[(size_t)v * W + lane], got);
      bool any = false;
#pragma unroll
      for (int x = 0; x < P; ++x) any = any || accw[x] != 0;
      if (any && lane == 0) atom_or(&T[v >> 6], 1ull << (v & 63));
    }
  } else {
  // long in-lists: one chunk of kPullChunk in-edges per lane group, the
  // chunks of a node OR their bits into its row
  for (unsigned it = 0; gw + nwaves * npw * it < (unsigned)a.npc; ++it) {
    // spread over the waves first: chunk gw + nwaves (sub + npw it)
    const unsigned c = gw + nwaves * ((unsigned)sub + npw * it);
    const bool has = c < (unsigned)a.npc;
    int v = 0, s = 0, e = 0;
    u64 need = 0;
    if (has) {
      v = a.pcv[c];
      const int k = a.pck[c];
      s = a.ip[v] + k * kPullChunk;
      e = min(s + kPullChunk, a.ip[v + 1]);
      if (wok) need = actw & ~a.vis[(size_t)v * W + w];
    }
    u64 acc = 0;
    if ((__ballot(need != 0) & gm) != 0) {
      const int nr = pull_scan<P>(a, front, fm, s, e, need, w, gb, gm, acc);
      if (w == 0) edges += (u64)nr;
    }
    if (acc) atom_or(&nxt[(size_t)v * W + w], acc);
    const bool any = (__ballot(acc != 0) & gm) != 0;
    if (any && w == 0) atom_or(&T[v >> 6], 1ull << (v & 63));
  }
  }

  for (unsigned base = gw * npw; base < (unsigned)a.n; base += nwaves * npw) {
    const int v = (int)base + sub;
    const bool valid = v < a.n;
    int s = 0, e = 0;
    if (valid) {
      s = a.ip[v];
      e = a.ip[v + 1];
    }
    const bool mine = valid && e - s < kPullBig;     // long in-lists went by chunks
    const u64 vw = (mine && wok) ? a.vis[(size_t)v * W + w] : ~0ull;
    const u64 need = (mine && wok) ? (actw & ~vw) : 0ull;
    const u64 gneed = __ballot(need != 0) & gm;
    // narrow rows: in-lists of more than a.wide_scan entries go to the whole
    // wave below instead of the node's few lanes
    const bool wide = P <= 8 && e - s > a.wide_scan;
    u64 acc = 0;
    if (gneed != 0 && !wide) {
      const int nr = pull_scan<P>(a, front, fm, s, e, need, w, gb, gm, acc);
      if (w == 0) edges += (u64)nr;
    }
    if (acc) nxt[(size_t)v * W + w] = acc;
    const bool any = (__ballot(acc != 0) & gm) != 0;
    if (any && w == 0) atom_or(&T[v >> 6], 1ull << (v & 63));
    if constexpr (P <= 8) {
      u64 lead = __ballot(wide && gneed != 0 && w == 0);
      while (lead) {
        const int ld = __ffsll((unsigned long long)lead) - 1;
        lead &= lead - 1;
        const int vv = __builtin_amdgcn_readlane(v, ld);
        const int ss = __builtin_amdgcn_readlane(s, ld);
        const int ee = __builtin_amdgcn_readlane(e, ld);
        u64 needw[P], accw[P];
#pragma unroll
        for (int x = 0; x < P; ++x) {
          needw[x] = shfl64(need, ld + x);
          accw[x] = 0;
        }
        const int nr = wave_scan<P>(a, front, fm, ss, ee, needw, accw);
        if (lane == 0) edges += (u64)nr;
        u64 got = 0;
#pragma unroll
        for (int x = 0; x < P; ++x)
          if (x == lane) got = accw[x];
        if (got) nxt[(size_t)vv * W + lane] = got;
        bool anyw = false;
#pragma unroll
        for (int x = 0; x < P; ++x) anyw = anyw || accw[x] != 0;
        if (anyw && lane == 0) atom_or(&T[vv >> 6], 1ull << (vv & 63));
      }
    }
  }
  block_add_edges(a, L, edges);
}

// Push bits f[q] of frontier nodes along their edges to v[q], q < 4
// (group-uniform call).  Every load of the four edges is issued before any
// atomic: a stale read of `out` only costs a redundant atomic.
template <int P>
__device__ __forceinline__ void relax4(const BatchArgs& a, u64* out, u64* T, const int* v,
                                       const u64* f, int w, u64 gm) {
  const size_t W = (size_t)a.Ws;
  u64 b[4], o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) b[q] = f[q] ? f[q] & ~a.vis[(size_t)v[q] * W + w] : 0ull;
  // bits already staged for v this level need no atomic
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = b[q] ? out[(size_t)v[q] * W + w] : 0ull;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b[q] &= ~o[q];
    if (b[q]) atom_or(&out[(size_t)v[q] * W + w], b[q]);
  }
  bool any[4];
  u64 tv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    any[q] = (__ballot(b[q] != 0) & gm) != 0 && w == 0;
    tv[q] = any[q] ? T[v[q] >> 6] : 0ull;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const u64 bit = 1ull << (v[q] & 63);
    if (any[q] && !(tv[q] & bit)) atom_or(&T[v[q] >> 6], bit);
  }
}

// A frontier node with at most a.sparse_words (<= kSparseWords, the knob
// batch_sparse_words) nonzero words is pushed one edge
// per lane (over those words) instead of one word per lane.
constexpr int kSparseWords = 4;

// Relax edge (u -> v) over the nonzero words `fmu` of u's frontier row
// (per lane; at most kSparseWords words).
__device__ __forceinline__ void relax_edge_sparse(const BatchArgs& a, const u64* front, u64* out,
                                                  u64* T, int u, int v, u64 fmu) {
  const size_t W = (size_t)a.Ws;
  int wk[kSparseWords];
  u64 f[kSparseWords], b[kSparseWords], o[kSparseWords];
#pragma unroll
  for (int k = 0; k < kSparseWords; ++k) {
    wk[k] = fmu ? __builtin_ctzll(fmu) : -1;
    fmu &= fmu - 1;
  }
#pragma unroll
  for (int k = 0; k < kSparseWords; ++k) f[k] = wk[k] >= 0 ? front[(size_t)u * W + wk[k]] : 0ull;
#pragma unroll
  for (int k = 0; k < kSparseWords; ++k) b[k] = f[k] ? f[k] & ~a.vis[(size_t)v * W + wk[k]] : 0ull;
#pragma unroll
  for (int k = 0; k < kSparseWords; ++k) o[k] = b[k] ? out[(size_t)v * W + wk[k]] : 0ull;
  bool any = false;
#pragma unroll
  for (int k = 0; k < kSparseWords; ++k) {
    b[k] &= ~o[k];
    if (b[k]) {
      atom_or(&out[(size_t)v * W + wk[k]], b[k]);
      any = true;
    }
  }
  if (any) {
    const u64 bit = 1ull << (v & 63);
    if (!(T[v >> 6] & bit)) atom_or(&T[v >> 6], bit);
  }
}

template <int P>
__device__ __forceinline__ void push_level(const BatchArgs& a, int L) {
  const int lane = lane_id();
  const int w = lane & (P - 1);
  const int npw = kWave / P;
  const int sub = lane / P;
  const bool wok = w < a.W;
  const u64 gm = group_mask<P>(lane);
  const size_t W = (size_t)a.Ws;
  const int pl = (L - 1) & 1;
  const u64* F = a.touched[pl];
  const u64* front = a.nxt[pl];
  const u64* fmp = a.fmap[pl];
  u64* out = a.nxt[L & 1];
  u64* T = a.touched[L & 1];
  u64 edges = 0;
  const unsigned gw = (blockIdx.x * kBatchBlock + threadIdx.x) / kWave;
  const unsigned nwaves = gridDim.x * kBatchBlock / kWave;

  // big-degree frontier nodes: chunks of kChunkB out-edges, one per lane
  // group, spread over the waves first (chunk gw + nwaves (sub + npw it))
  const unsigned nch = ld_relaxed(&a.ctrl->lv[pl].nchunks);
  for (unsigned it = 0; gw + nwaves * npw * it < nch; ++it) {
    const unsigned c = gw + nwaves * ((unsigned)sub + npw * it);
    const bool has = c < nch;
    int e0 = 0, e1 = 0, u = 0;
    u64 f = 0, fmu = 0;
    if (has) {
      u = a.cu[pl][c];
      const int k = a.ck[pl][c];
      e0 = a.rp[u] + k * kChunkB;
      e1 = min(e0 + kChunkB, a.rp[u + 1]);
      fmu = fmp[u];
    }
    if (has && w == 0) edges += (u64)(e1 - e0);
    const bool sparse = has && __popcll(fmu) <= a.sparse_words;
    // chunks with few nonzero words: the wave walks the union of its groups'
    // sparse chunks, one edge per lane
    const int cnt = (sparse && w == 0) ? e1 - e0 : 0;
    const int incl = wave_incl_scan(cnt);
    const int total = __shfl(incl, kWave - 1, kWave);
    for (int eb = 0; eb < total; eb += kWave) {
      const int x = eb + lane;
      const bool in = x < total;
      const int j = wave_owner(incl, in ? x : total - 1);
      const int inc_j = __shfl(incl, j, kWave);
      const int cnt_j = __shfl(cnt, j, kWave);
      const int e0_j = __shfl(e0, j, kWave);
      const int u_j = __shfl(u, j, kWave);
      const u64 fm_j = shfl64(fmu, j);
      if (in) relax_edge_sparse(a, front, out, T, u_j, a.col[e0_j + (x - (inc_j - cnt_j))], fm_j);
    }
    if (!has || sparse) continue;
    if (wok && ((fmu >> w) & 1ull)) f = front[(size_t)u * W + w];
    // group-uniform steps of four edges (past e1: no bits)
    for (int e = e0; e < e1; e += 4) {
      int v[4];
      u64 fq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool in = e + q < e1;
        v[q] = in ? a.col[e + q] : 0;
        fq[q] = in ? f : 0ull;
      }
      relax4<P>(a, out, T, v, fq, w, gm);
    }
  }

  // other frontier nodes, 64 per wave (one frontier word): the wave walks the
  // union of their out-lists, each lane group taking one edge per step
  const int nwords = (a.n + 63) / 64;
  for (unsigned t = gw; t < (unsigned)nwords; t += nwaves) {
    const u64 fw = F[t];
    if (!fw) continue;
    const int u = (int)t * 64 + lane;
    int deg = 0, rs = 0, sdeg = 0;
    u64 fmu = 0;
    if ((fw >> lane) & 1ull) {
      rs = a.rp[u];
      deg = a.rp[u + 1] - rs;
      fmu = fmp[u];
      if (deg >= a.big_b) deg = 0;
      if (__popcll(fmu) <= a.sparse_words) {
        sdeg = deg;
        deg = 0;
      }
    }
    // sparse nodes: one edge per lane over the union of their out-lists
    const int sincl = wave_incl_scan(sdeg);
    const int stotal = __shfl(sincl, kWave - 1, kWave);
    for (int eb = 0; eb < stotal; eb += kWave) {
      const int x = eb + lane;
      const bool has = x < stotal;
      const int j = wave_owner(sincl, has ? x : stotal - 1);
      const int inc_j = __shfl(sincl, j, kWave);
      const int deg_j = __shfl(sdeg, j, kWave);
      const int rs_j = __shfl(rs, j, kWave);
      const u64 fm_j = shfl64(fmu, j);
      if (has)
        relax_edge_sparse(a, front, out, T, (int)t * 64 + j, a.col[rs_j + (x - (inc_j - deg_j))],
                          fm_j);
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, kWave - 1, kWave);
    if (lane == 0) edges += (u64)(total + stotal);
    // four edges per lane group and step keep independent loads in flight
    for (int eb = 0; eb < total; eb += 4 * npw) {
      int v[4];
      u64 f[4];
      u64 fmw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int x = eb + q * npw + sub;
        const bool has = x < total;
        const int j = wave_owner(incl, has ? x : total - 1);
        const int inc_j = __shfl(incl, j, kWave);
        const int deg_j = __shfl(deg, j, kWave);
        const int rs_j = __shfl(rs, j, kWave);
        const int uj = (int)t * 64 + j;
        fmw[q] = shfl64(fmu, j);
        v[q] = 0;
        f[q] = 0;
        if (has) {
          v[q] = a.col[rs_j + (x - (inc_j - deg_j))];
          if (wok && ((fmw[q] >> w) & 1ull)) f[q] = front[(size_t)uj * W + w];
        }
      }
      relax4<P>(a, out, T, v, f, w, gm);
    }
  }
  block_add_edges(a, L, edges);
}

// ----------------------------------------------------------------- merge --
// Fold the new bits of level L into vis and the level planes, list the
// big-degree nodes' out-edge chunks for the next push, and clear the rows and
// bitmap of the previous frontier.
template <int P>
__device__ __forceinline__ void merge_level(const BatchArgs& a, int L) {
  __shared__ u64 lmask[kMaxPlanes][64];   // bit b of (L - base) for the lanes of each word
  __shared__ u64 actb[64];
  __shared__ int rank_j[kBatchBlock / kWave][kWave];
  __shared__ u64 red[5][kBatchBlock / kWave];
  __shared__ ChunkStage cstage;
  const int tid = threadIdx.x;
  if (tid == 0) cstage.n = 0;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const int W = a.W;                  // words processed
  const size_t Ws = (size_t)a.Ws;     // row stride
  const int D = a.nplanes;
  // one word per wave: lane r holds source (64 x + r)'s relative level, and a
  // ballot per plane gives that plane's mask
  for (int x = wv; x < W; x += kBatchBlock / kWave) {
    const int rel = L - (a.base ? a.base[x * 64 + lane] : 0);
#pragma unroll
    for (int b = 0; b < kMaxPlanes; ++b) {
      const u64 m = __ballot(b < D && ((rel >> b) & 1));
      if (lane == 0) lmask[b][x] = m;
    }
  }
  if (tid < 64) actb[tid] = 0;
  __syncthreads();

  const int cl = L & 1;
  BatchLevel* lv = &a.ctrl->lv[cl];
  const int w = lane & (P - 1);
  const int npw = kWave / P;
  const int sub = lane / P;
  const bool wok = w < W;
  const int stripe = blockIdx.x % kStripes;
  const int nwords = (a.n + 63) / 64;
  const unsigned gw = (blockIdx.x * kBatchBlock + tid) / kWave;
  const unsigned nwaves = gridDim.x * kBatchBlock / kWave;

  // the previous frontier's bits were consumed by this level's expansion
  if (L > 0) {
    u64* F = a.touched[(L - 1) & 1];
    u64* prev = a.nxt[(L - 1) & 1];
    u64* pmap = a.fmap[(L - 1) & 1];
    for (unsigned t = gw; t < (unsigned)nwords; t += nwaves) {
      const u64 fw = F[t];
      if (!fw) continue;
      const int cnt = __popcll(fw);
      if ((fw >> lane) & 1ull) rank_j[wv][__popcll(fw & lanes_below())] = lane;
      __builtin_amdgcn_wave_barrier();
      // only the words the frontier word map marks nonzero need clearing
      // (a sparse row has one or two of them)
      for (int i0 = 0; i0 < cnt; i0 += 4 * npw) {
        int vq[4];
        u64 pm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + q * npw + sub;
          vq[q] = i < cnt ? (int)t * 64 + rank_j[wv][i] : -1;
          pm[q] = vq[q] >= 0 ? pmap[vq[q]] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (vq[q] < 0) continue;
          if (wok && ((pm[q] >> w) & 1ull)) prev[(size_t)vq[q] * Ws + w] = 0;
          if (w == 0 && pm[q]) pmap[vq[q]] = 0;
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) F[t] = 0;
    }
  }

  u64* nxt = a.nxt[cl];
  u64* fmap = a.fmap[cl];
  const u64* T = a.touched[cl];
  u64 act_acc = 0, bits = 0, se = 0, nodes = 0, mf = 0, mfw = 0;
  // a work unit is a part of a frontier word: with wide rows a quarter (ranks
  // 16 s .. 16 s + 15 of its set bits), so that dense words spread over four
  // waves; with narrow rows (P <= 16: 4 nodes or more per wave and step) the
  // whole word.  Within a unit four nodes' rows per group are loaded before
  // any of them is written back.
  constexpr int kParts = P >= 64 ? 4 : (P >= 32 ? 2 : 1);
  constexpr int kPartNodes = 64 / kParts;
  const unsigned nunits = (unsigned)nwords * (unsigned)kParts;
  for (unsigned ux = gw; ux < nunits; ux += nwaves) {
    const unsigned t = ux / kParts;
    const u64 tw = T[t];
    const int cnt = __popcll(tw);
    const int ib = (int)(ux % kParts) * kPartNodes, ie = min(ib + kPartNodes, cnt);
    if (ib >= ie) continue;
    const int v0 = (int)t * 64;
    const bool bit = (tw >> lane) & 1ull;
    const int rk = __popcll(tw & lanes_below());
    const bool mine = bit && rk >= ib && rk < ie;
    int deg = 0;
    if (bit) rank_j[wv][rk] = lane;
    if (mine) {
      deg = a.rp[v0 + lane + 1] - a.rp[v0 + lane];
      nodes += 1;
      mf += (u64)deg;
    }
    stage_chunks_wave(a, L, cstage, v0 + lane, deg, mine && deg >= a.big_b);
    __builtin_amdgcn_wave_barrier();
    // four nodes' rows per group and step; the next step's rows are loaded
    // before this step's atomic ORs are issued, so the wait for them never
    // covers those atomics
    int jq[4], dq[4];
    bool okq[4];
    u64 nb[4];
    size_t idx[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ib + q * npw + sub;
      okq[q] = i < ie;
      jq[q] = rank_j[wv][okq[q] ? i : ib];
      dq[q] = __shfl(deg, jq[q], kWave);
      idx[q] = (size_t)(v0 + jq[q]) * Ws + w;
      nb[q] = (okq[q] && wok) ? nxt[idx[q]] : 0ull;
    }
    for (int i0 = ib; i0 < ie; i0 += 4 * npw) {
      int jn[4], dn[4];
      bool okn[4];
      u64 nbn[4];
      size_t idn[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * npw + q * npw + sub;
        okn[q] = i < ie;
        jn[q] = rank_j[wv][okn[q] ? i : ib];
        dn[q] = __shfl(deg, jn[q], kWave);
        idn[q] = (size_t)(v0 + jn[q]) * Ws + w;
        nbn[q] = (okn[q] && wok) ? nxt[idn[q]] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // the group's nonzero words of the node: its frontier word map, and
        // the words of its visited row that may now be nonzero
        const u64 nzb = __ballot(nb[q] != 0);
        const u64 fm = (nzb >> ((sub * P) & 63)) & low_mask<P>();
        if (okq[q] && w == 0) {
          fmap[v0 + jq[q]] = fm;
          mfw += (u64)__popcll(fm) * (u64)dq[q];
          if (fm) atom_or(&a.vmap[v0 + jq[q]], fm);
        }
      }
      // vis and the planes take their bits with atomic ORs that return
      // nothing: no (node, word) is touched twice in a level, and the wave
      // never waits for a read-modify-write round trip per plane
      for (int b = 0; b < D; ++b) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const u64 mq = lmask[b][w] & nb[q];
          if (mq) atom_or(&a.planes[b][idx[q]], mq);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (nb[q]) {
          atom_or(&a.vis[idx[q]], nb[q]);
          const u64 pc = (u64)__popcll(nb[q]);
          bits += pc;
          se += pc * (u64)dq[q];
          act_acc |= nb[q];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        jq[q] = jn[q];
        dq[q] = dn[q];
        okq[q] = okn[q];
        nb[q] = nbn[q];
        idx[q] = idn[q];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // lanes w, w+P, ... hold the same word: fold them, then once per block
  for (int off = P; off < kWave; off <<= 1) act_acc |= shfl_xor64(act_acc, off);
  if (lane < P && wok && act_acc) atomicOr(&actb[w], act_acc);
  bits = wave_sum(bits);
  se = wave_sum(se);
  nodes = wave_sum(nodes);
  mf = wave_sum(mf);
  mfw = wave_sum(mfw);
  if (lane == 0) {
    red[0][wv] = bits;
    red[1][wv] = se;
    red[2][wv] = nodes;
    red[3][wv] = mf;
    red[4][wv] = mfw;
  }
  __syncthreads();
  flush_chunk_stage(a, L, cstage);
  if (tid < W && actb[tid]) {
    u64* gp = &a.ctrl->laneact[cl][stripe][tid];
    if (actb[tid] & ~ld_relaxed(gp)) atom_or(gp, actb[tid]);
  }
  if (tid < 5) {
    u64 x = 0;
    for (int i = 0; i < kBatchBlock / kWave; ++i) x += red[tid][i];
    if (x) {
      BatchStripe& st = lv->s[stripe];
      u64* dst = tid == 0 ? &st.bits : tid == 1 ? &st.se : tid == 2 ? &st.nodes
               : tid == 3 ? &st.mf : &st.mfw;
      atom_add(dst, x);
    }
  }
}

template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_pull(BatchArgs a, int L) {
  if (batch_gate_open(a, 1)) pull_level<P>(a, L);
}

template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_push(BatchArgs a, int L) {
  if (batch_gate_open(a, 0)) push_level<P>(a, L);
}

template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_merge(BatchArgs a, int L) {
  if (batch_gate_open(a, -1)) merge_level<P>(a, L);
}

// ------------------------------------------------------------------ emit --
// Write the distance rows of the lanes in emask.  A wave takes a task of 64
// nodes (lane l owns node v0 + l) and a group of EG consecutive words of their
// rows.  Each lane loads its node's EG visited words and EG words of each of
// the D level planes into registers, so a node's 128-byte line is fetched by
// one lane in 16 / EG back-to-back passes (one when EG = 16) instead of being
// re-read later.  Then, for every emitted source b of the group, the lanes
// rebuild b's level at their nodes (-1 where the visited bit is clear) and the
// wave writes the 64 values as one 256-byte run of b's row.  Tasks run
// word-group-major, so waves running side by side write neighbouring runs of
// the same rows.  With `clear` the emitted lanes' bits are removed from vis and
// the planes (serving reuses the lanes).
// One source's 64 values: lane l writes b's level at its node (-1 where the
// visited bit is clear) at byte offset voff of b's row.  b is wave-uniform, so
// the row pointer comes from lane b's register and the store takes a scalar
// base with a 32-bit lane offset.
template <int DMAX>
__device__ __forceinline__ void emit_one(u64 my_row, int b, int bit, unsigned xh,
                                         const unsigned* ph, unsigned voff) {
  typedef __attribute__((address_space(1))) char gchar;
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)my_row, b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(my_row >> 32), b);
  const unsigned long long addr = ((unsigned long long)hi << 32) | lo;
  if (!addr) return;
  int lv = 0;
#pragma unroll
  for (int d = 0; d < DMAX; ++d) lv |= (int)((ph[d] >> bit) & 1u) << d;
  // visited: the level; not visited: -1 (all bits set)
  const int val = lv | ((int)((xh >> bit) & 1u) - 1);
  // written once and not read again by the library
  __builtin_nontemporal_store(val, (__attribute__((address_space(1))) int*)((gchar*)addr + voff));
}

// Planes an emission variant handles: DMAX 3 takes 0..3, 7 takes 4..7, 15
// takes 8..15, 16 takes 16.
template <int DMAX>
__device__ __forceinline__ int emit_dmin() {
  return DMAX <= 3 ? 0 : DMAX <= 7 ? 4 : DMAX <= 15 ? 8 : 16;
}

__device__ __forceinline__ int bit_length_dev(int x) { return x > 0 ? 32 - __clz(x) : 0; }

// Lanes of word w to emit: the mask, or without one every lane < emit_k.
__device__ __forceinline__ u64 emit_word(const BatchArgs& a, const u64* emask, int w) {
  if (emask) return emask[w];
  const int lo = w * 64;
  if (a.emit_k >= lo + 64) return ~0ull;
  return a.emit_k > lo ? (1ull << (a.emit_k - lo)) - 1ull : 0ull;
}

// mode bit 0 (kEmitClear): remove the emitted lanes' bits from vis and the
// planes; bit 1 (kEmitFromRun): the run state decides: emit only after a run
// that finished, with D = bit_length of its last level, and only in the
// variant whose plane range holds D; bit 2 (kEmitMarkClean): every lane is
// emitted with kEmitClear, so the workspace holds no bits afterwards.
template <int DMAX, int EG>
__global__ __launch_bounds__(kBatchBlock) void batch_emit(BatchArgs a, int D,
                                                          const u64* __restrict__ emask,
                                                          int mode, int claim) {
  const int clear = mode & kEmitClear;
  const bool whole_clear = clear && (mode & kEmitMarkClean);
  if (mode & kEmitFromRun) {
    const BatchRun& r = a.ctrl->run;
    if (ld_relaxed(&r.done) != 1 || ld_relaxed(&a.flags[kFlagStatus]) != 0) return;
    D = min(bit_length_dev(ld_relaxed(&r.last_nonempty)), a.nplanes);
    if (D < emit_dmin<DMAX>() || D > DMAX) return;
  }
  if ((mode & kEmitMarkClean) && blockIdx.x == 0 && threadIdx.x == 0) a.flags[kFlagDirty] = 0;
  // the row pointers of all lanes, staged once: a per-word global load in the
  // store loop would wait for every store before it
  __shared__ u64 srow[kMaxBatchLanes];
  const int lane = lane_id();
  const int W = a.W;
  for (int i = threadIdx.x; i < W * 64; i += kBatchBlock)
    srow[i] = a.rows ? (u64)a.rows[i]
                     : (i < a.emit_k ? (u64)(a.row_base + (size_t)i * (size_t)a.row_stride) : 0ull);
  __syncthreads();
  const int gw = __builtin_amdgcn_readfirstlane(
      (int)((blockIdx.x * (unsigned)kBatchBlock + threadIdx.x) / kWave));
  const int nwaves = (int)(gridDim.x * (kBatchBlock / kWave));
  const size_t Ws = (size_t)a.Ws;
  const int ntiles = (a.n + kWave - 1) / kWave;
  const int ngroups = (W + EG - 1) / EG;
  const long long tasks = (long long)ntiles * ngroups;
  // a wave's first task is its index; with `claim` (many tasks per wave)
  // later ones are claimed in order from a counter, so no wave idles while
  // another has several left (with few per wave the claims, serialised on
  // one line, would cost more than they balance)
  auto next_task = [&](long long t) -> long long {
    if (!claim) return t + nwaves;
    unsigned c = 0;
    if (lane == 0) c = atomicAdd(&a.ctrl->emit_next, 1u);
    return nwaves + (unsigned)__builtin_amdgcn_readfirstlane((int)c);
  };
  for (long long t = gw; t < tasks; t = next_task(t)) {
    const int w0 = (int)(t / ntiles) * EG;
    const int v = (int)(t % ntiles) * kWave + lane;
    const int ew = min(EG, W - w0);
    // words of the group with emitted lanes: only those are loaded (serving
    // emits a few lanes at a time)
    unsigned wm = 0;
    for (int e = 0; e < ew; ++e)
      if (emit_word(a, emask, w0 + e)) wm |= 1u << e;
    if (!wm) continue;
    const bool live = v < a.n;
    const bool full = (int)(t % ntiles) * kWave + kWave <= a.n;  // no lane past the last node
    bool cleared = false;     // the group's words were already cleared whole
    const size_t base = (size_t)(live ? v : 0) * Ws + w0;
    u64 x[EG];
    u64 pl[DMAX][EG];
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
#pragma unroll
      for (int e = 0; e < EG; ++e) pl[d][e] = 0;
    if (ew == EG && (Ws & 1) == 0) {
      // whole groups of 16-byte aligned words: each lane reads its node's
      // words of one array in consecutive 16-byte loads, so the requests for
      // a line follow each other closely enough that it is fetched once
      // (lanes past the last node read node 0's row and drop it)
      const ulonglong2* pv = reinterpret_cast<const ulonglong2*>(a.vis + base);
#pragma unroll
      for (int q = 0; q < EG / 2; ++q) {
        x[2 * q] = x[2 * q + 1] = 0;
        if ((wm >> (2 * q)) & 3u) {
          const ulonglong2 t2 = pv[q];
          x[2 * q] = live ? t2.x : 0;
          x[2 * q + 1] = live ? t2.y : 0;
        }
      }
#pragma unroll
      for (int d = 0; d < DMAX; ++d)
        if (d < D) {
          const ulonglong2* pp = reinterpret_cast<const ulonglong2*>(a.planes[d] + base);
#pragma unroll
          for (int q = 0; q < EG / 2; ++q)
            if ((wm >> (2 * q)) & 3u) {
              const ulonglong2 t2 = pp[q];
              pl[d][2 * q] = live ? t2.x : 0;
              pl[d][2 * q + 1] = live ? t2.y : 0;
            }
        }
      if (whole_clear && live) {
        // every lane is emitted: the words just read are cleared with the
        // same 16-byte accesses (the line is still in the cache)
        ulonglong2* wv = reinterpret_cast<ulonglong2*>(a.vis + base);
        const ulonglong2 z = {0ull, 0ull};
#pragma unroll
        for (int q = 0; q < EG / 2; ++q)
          if ((wm >> (2 * q)) & 3u) wv[q] = z;
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
          if (d < D) {
            ulonglong2* wp = reinterpret_cast<ulonglong2*>(a.planes[d] + base);
#pragma unroll
            for (int q = 0; q < EG / 2; ++q)
              if ((wm >> (2 * q)) & 3u) wp[q] = z;
          }
        cleared = true;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EG; ++e) x[e] = live && ((wm >> e) & 1u) ? a.vis[base + e] : 0;
#pragma unroll
      for (int d = 0; d < DMAX; ++d)
        if (d < D) {
#pragma unroll
          for (int e = 0; e < EG; ++e)
            if (live && ((wm >> e) & 1u)) pl[d][e] = a.planes[d][base + e];
        }
    }
#pragma unroll 1
    for (int e = 0; e < ew; ++e) {
      u64 em = emit_word(a, emask, w0 + e);
      if (!em) continue;
      // word e of the staged rows, picked out with selects so that the
      // staging arrays stay in registers
      u64 xe = 0;
      u64 pe[DMAX];
#pragma unroll
      for (int d = 0; d < DMAX; ++d) pe[d] = 0;
#pragma unroll
      for (int k = 0; k < EG; ++k)
        if (k == e) {
          xe = x[k];
#pragma unroll
          for (int d = 0; d < DMAX; ++d) pe[d] = pl[d][k];
        }
      if (clear && live && !cleared) {
        const u64 rem = xe & ~em;
        a.vis[base + e] = rem;
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
          if (d < D) a.planes[d][base + e] = pe[d] & ~em;
        // a word left empty by a partial emission leaves the visited map
        // (a whole emission clears the node's map below)
        if (!rem && xe && !(mode & kEmitMarkClean))
          atomicAnd(&a.vmap[v], ~(1ull << (w0 + e)));
      }
      // lane b holds source (64 w + b)'s row pointer; each row is read from
      // that lane
      const u64 my_row = srow[(w0 + e) * 64 + lane];
      const unsigned voff = (unsigned)v * 4u;
      // one half-word at a time so the bit tests are 32-bit field extracts
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned emh = (unsigned)(em >> (32 * h));
        if (!emh) continue;
        const unsigned xh = (unsigned)(xe >> (32 * h));
        unsigned ph[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d) ph[d] = (unsigned)(pe[d] >> (32 * h));
        if (full) {
          while (emh) {
            const int bit = __builtin_ctz(emh);
            emh &= emh - 1;
            emit_one<DMAX>(my_row, 32 * h + bit, bit, xh, ph, voff);
          }
        } else {
          while (emh) {
            const int bit = __builtin_ctz(emh);
            emh &= emh - 1;
            if (live) emit_one<DMAX>(my_row, 32 * h + bit, bit, xh, ph, voff);
          }
        }
      }
    }
    // every lane of the batch was emitted: the node's visited map is clear too
    if ((mode & kEmitMarkClean) && clear && w0 == 0 && live) a.vmap[v] = 0;
  }
}

// ------------------------------------------------------------------ init --
__global__ __launch_bounds__(kBatchBlock) void batch_zero(u64* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)kBatchBlock + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kBatchBlock)
    p[i] = 0;
}

// Serving's step before a level: the active-lane words (by value) and a
// cleared counter slot for the level, in one launch instead of a copy and
// two fills.
__global__ __launch_bounds__(kWave) void batch_level_prep(BatchActWords act, u64* d_act,
                                                         BatchCtrl* ctrl, int slot) {
  const int lane = lane_id();
  if (lane < act.W) d_act[lane] = act.w[lane];
  for (int i = lane; i < kStripes * 64; i += kWave) ctrl->laneact[slot][i / 64][i % 64] = 0;
  if (lane < kStripes) {
    BatchStripe& st = ctrl->lv[slot].s[lane];
    st.nodes = 0;
    st.bits = 0;
    st.se = 0;
    st.mf = 0;
    st.edges = 0;
    st.mfw = 0;
  }
  if (lane == 0) {
    ctrl->lv[slot].nchunks = 0;
    ctrl->emit_next = 0;
  }
}

// Row y of the grid clears array y of the list.
__global__ __launch_bounds__(kBatchBlock) void batch_zero_list(ZeroList z) {
  u64* p = z.p[blockIdx.y];
  const size_t count = z.count[blockIdx.y];
  for (size_t i = blockIdx.x * (size_t)kBatchBlock + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kBatchBlock)
    p[i] = 0;
}

// The host's per-level step of the batched loop, on the device (one wave):
// level L - 1's counters go into the run totals, the lanes that found new
// bits become the active words, the direction of level L is chosen by the
// batched rule (pull iff the frontier's out-degree x nonzero words times
// alpha reaches n x words), and level L's counter slot is cleared.
//
// The run also stops here (done = 2) when level L would need more level
// planes than the workspace holds or exceeds n levels (the watchdog), and
// (done = 3) when the call's sources were found invalid.  Called by one wave.
__device__ __forceinline__ void control_level(const BatchArgs& a, u64* act, int L, int direction,
                                              double alpha) {
  BatchCtrl* c = a.ctrl;
  BatchRun* r = &c->run;
  if (ld_relaxed(&r->done)) return;
  const int lane = lane_id();
  if (ld_relaxed(&a.flags[kFlagStatus]) != 0) {
    if (lane == 0) r->done = 3;
    return;
  }
  const int pl = (L - 1) & 1, cl = L & 1;
  const int W = a.W;
  u64 x = 0;
  if (lane < W)
    for (int i = 0; i < kStripes; ++i) x |= c->laneact[pl][i][lane];
  const bool any = __ballot(x != 0) != 0;
  if (lane < W) act[lane] = x;
  u64 bits = 0, se = 0, edges = 0, mfw = 0;
  if (lane < kStripes) {
    const BatchStripe& st = c->lv[pl].s[lane];
    bits = st.bits;
    se = st.se;
    edges = st.edges;
    mfw = st.mfw;
  }
  bits = wave_sum(bits);
  se = wave_sum(se);
  edges = wave_sum(edges);
  mfw = wave_sum(mfw);
  for (int i = lane; i < kStripes * 64; i += kWave) c->laneact[cl][i / 64][i % 64] = 0;
  if (lane < kStripes) {
    BatchStripe& st = c->lv[cl].s[lane];
    st.nodes = 0;
    st.bits = 0;
    st.se = 0;
    st.mf = 0;
    st.edges = 0;
    st.mfw = 0;
  }
  if (lane == 0) {
    c->lv[cl].nchunks = 0;
    r->edges += edges;
    r->reached += bits;
    r->source_edges += se;
    if (bits) r->last_nonempty = L - 1;
    if (!any) {
      r->done = 1;
    } else if (L > a.n + 1 || bit_length_dev(L) > a.nplanes) {
      r->done = 2;
      atomicMax(&a.flags[kFlagStatus], 2u);
    } else {
      const bool pull = direction == 2 ||
                        (direction != 1 && (double)mfw * alpha >= (double)a.n * (double)W);
      r->pull = pull ? 1 : 0;
      if (pull)
        r->pull_levels += 1;
      else
        r->push_levels += 1;
    }
  }
}

__global__ __launch_bounds__(kWave) void batch_control(BatchArgs a, u64* act, int L, int direction,
                                                      double alpha) {
  control_level(a, act, L, direction, alpha);
}

// Lane lane[i] starts at node src[i] at level L: its bit joins the new bits
// of level L (nxt) and the node joins that level's frontier bitmap.  With
// `live` (sources admitted after level L's merge ran) the seed also does the
// merge's part: the visited bit and the big-degree chunks.  lane == null:
// source i takes lane i.  A source outside [0, n) is skipped (device-ordered
// calls find it beforehand and stop the run).
__global__ void batch_seed(BatchArgs a, const int32_t* src, const int32_t* lane, int k, int L,
                           int live) {
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flags[kFlagDirty] = 1;
  // whole waves walk the sources so that chunk listing is wave-aggregated
  const int stride = gridDim.x * blockDim.x;
  for (int i0 = blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); i0 < k; i0 += stride) {
    const int i = i0 + lane_id();
    int s = 0, deg = 0;
    bool first = false;
    if (i < k && (unsigned)src[i] < (unsigned)a.n) {
      s = src[i];
      const int l = lane ? lane[i] : i;
      const size_t idx = (size_t)s * a.Ws + (l >> 6);
      const u64 bit = 1ull << (l & 63);
      atom_or(&a.nxt[L & 1][idx], bit);
      atom_or(&a.fmap[L & 1][s], 1ull << (l >> 6));
      const u64 sbit = 1ull << (s & 63);
      const u64 old = atom_or(&a.touched[L & 1][s >> 6], sbit);
      if (live) {
        atom_or(&a.vis[idx], bit);
        atom_or(&a.vmap[s], 1ull << (l >> 6));
        deg = a.rp[s + 1] - a.rp[s];
        first = !(old & sbit);
      }
    }
    push_chunks_wave(a, L, s, deg, first && deg >= a.big_b);
  }
}

// Start of a batched run: the control block is cleared, and the bitmap
// arrays too when the workspace may still hold bits (its first run, or a run
// that stopped before its emission); after a complete run the emission has
// already left them clear.  z.p[0] is the control block.  clear_status:
// reset the run status (device-ordered calls set it once per call instead).
__global__ __launch_bounds__(kBatchBlock) void batch_prepare(ZeroList z, unsigned* flags,
                                                            int clear_status) {
  // nothing in this launch writes the flag, so every workgroup reads the same
  const bool dirty = ld_relaxed(&flags[kFlagDirty]) != 0;
  const size_t t0 = blockIdx.x * (size_t)kBatchBlock + threadIdx.x;
  const size_t nt = (size_t)gridDim.x * kBatchBlock;
  for (int y = 0; y < z.k; ++y) {
    if (y > 0 && !dirty) break;
    u64* p = z.p[y];
    for (size_t i = t0; i < z.count[y]; i += nt) p[i] = 0;
  }
  if (clear_status && t0 == 0) flags[kFlagStatus] = 0;
}

// Device-ordered calls: the run status is 1 when a source lies outside
// [0, n), else 0 (one workgroup; every batch's first control step stops on 1).
__global__ __launch_bounds__(1024) void batch_validate(const int32_t* src, long long k, int n,
                                                      unsigned* flags) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  bool b = false;
  for (long long i = threadIdx.x; i < k; i += blockDim.x) b = b || (unsigned)src[i] >= (unsigned)n;
  if (b) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) flags[kFlagStatus] = bad ? 1u : 0u;
}

// The call's status for the caller (device memory): DAWN_OK, DAWN_E_INVALID_ARG
// (a source outside [0, n): no row was written) or DAWN_E_DEVICE (watchdog).
__global__ void batch_status(const unsigned* flags, int32_t* out) {
  const unsigned f = ld_relaxed(&flags[kFlagStatus]);
  *out = f == 0 ? DAWN_OK : f == 1 ? DAWN_E_INVALID_ARG : DAWN_E_DEVICE;
}

// The levels after the queued ones, in one cooperative launch: per level the
// first wave runs the control step, then every workgroup the chosen
// expansion and the merge, with a grid barrier between the steps.  Returns at
// once when the queued levels already reached the end of the run.
template <int P>
__global__ __launch_bounds__(kBatchBlock) void batch_finish_levels(BatchArgs a, u64* act, int L0,
                                                                  int direction, double alpha) {
  BatchRun* r = &a.ctrl->run;
  GridBarrier* bar = &a.ctrl->bar;
  // read before any workgroup can write it (the first write follows the
  // barrier below), so every workgroup takes the same branch
  if (ld_relaxed(&r->done)) return;
  bool ok = grid_sync(bar);
  for (int L = L0; ok; ++L) {
    if (blockIdx.x == 0 && threadIdx.x < kWave) control_level(a, act, L, direction, alpha);
    if (!(ok = grid_sync(bar))) break;
    if (ld_relaxed(&r->done)) return;
    if (ld_relaxed(&r->pull))
      pull_level<P>(a, L);
    else
      push_level<P>(a, L);
    if (!(ok = grid_sync(bar))) break;
    merge_level<P>(a, L);
    ok = grid_sync(bar);
  }
  // a barrier wait timed out: the run stops with the watchdog status
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    r->done = 2;
    atomicMax(&a.flags[kFlagStatus], 2u);
  }
}

// ------------------------------------------------------------------ host --
void batch_ws_destroy(BatchWs* w) {
  if (!w) return;
  Ctx* ctx = w->ctx;
  if (w->busy_set) hipEventSynchronize(w->busy);
  dev_free(ctx, w->vis, 0);
  dev_free(ctx, w->nxt[0], 0);
  dev_free(ctx, w->nxt[1], 0);
  for (int b = 0; b < kMaxPlanes; ++b) dev_free(ctx, w->planes[b], 0);
  for (int i = 0; i < 2; ++i) {
    dev_free(ctx, w->touched[i], 0);
    dev_free(ctx, w->fmap[i], 0);
    dev_free(ctx, i == 0 ? w->vmap : nullptr, 0);
    dev_free(ctx, w->cu[i], 0);
    dev_free(ctx, w->ck[i], 0);
  }
  dev_free(ctx, w->ctrl, 0);
  dev_free(ctx, w->act, 0);
  dev_free(ctx, w->emask, 0);
  dev_free(ctx, w->rows, 0);
  dev_free(ctx, w->base, 0);
  dev_free(ctx, w->src, 0);
  dev_free(ctx, w->lane, 0);
  dev_free(ctx, w->flags, 0);
  if (ctx) ctx->used -= w->bytes;
  if (ctx && w->plane_reserve) dev_unreserve(ctx, w->plane_reserve);
  if (w->h_ctrl) hipHostFree(w->h_ctrl);
  if (w->ev0) hipEventDestroy(w->ev0);
  if (w->ev1) hipEventDestroy(w->ev1);
  if (w->busy) hipEventDestroy(w->busy);
  if (w->stream && w->own_stream) hipStreamDestroy(w->stream);
  delete w;
}

// A new workspace is marked as possibly holding bits, so its first run's
// prepare step clears every array; afterwards complete runs leave it clear.
dawn_status batch_ws_create(Ctx* ctx, const GraphRec* g, int lanes, BatchWs** out) {
  BatchWs* w = new BatchWs();
  w->ctx = ctx;
  w->n = g->n;
  w->lanes = lanes;
  const int W = (lanes + 63) / 64;
  w->Wmax = W;
  const size_t n = (size_t)g->n;
  const size_t nw = (n + 63) / 64;
  // chunks per level: sum over frontier nodes of degree >= kBigB of
  // ceil(deg / kChunkB) <= m / kChunkB + m / kBigB
  const size_t chunk_cap = (size_t)(g->m / kChunkB) + (size_t)(g->m / kBigB) + 64;
  dawn_status s = DAWN_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (s != DAWN_OK) return;
    s = dev_alloc(ctx, p, bytes);
    if (s == DAWN_OK) w->bytes += bytes;
  };
  alloc((void**)&w->vis, n * W * 8);
  alloc((void**)&w->nxt[0], n * W * 8);
  alloc((void**)&w->nxt[1], n * W * 8);
  for (int i = 0; i < 2; ++i) {
    alloc((void**)&w->touched[i], nw * 8 + 64);
    alloc((void**)&w->fmap[i], n * 8);
    alloc((void**)&w->cu[i], chunk_cap * 4);
    alloc((void**)&w->ck[i], chunk_cap * 4);
  }
  alloc((void**)&w->vmap, n * 8);
  alloc((void**)&w->ctrl, sizeof(BatchCtrl));
  alloc((void**)&w->act, 64 * 8);
  alloc((void**)&w->emask, 64 * 8);
  alloc((void**)&w->rows, (size_t)kMaxBatchLanes * sizeof(int32_t*));
  alloc((void**)&w->base, (size_t)kMaxBatchLanes * 4);
  alloc((void**)&w->src, (size_t)kMaxBatchLanes * 4);
  alloc((void**)&w->lane, (size_t)kMaxBatchLanes * 4);
  alloc((void**)&w->flags, 256);
  if (s != DAWN_OK) {
    batch_ws_destroy(w);
    return s;
  }
  hipError_t e = hipHostMalloc((void**)&w->h_ctrl, sizeof(BatchCtrl), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
  w->own_stream = true;
  if (e == hipSuccess) e = hipEventCreate(&w->ev0);
  if (e == hipSuccess) e = hipEventCreate(&w->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&w->busy, hipEventDisableTiming);
  if (e == hipSuccess) {
    static const unsigned init_flags[2] = {1u, 0u};   // dirty, status
    e = hipMemcpy(w->flags, init_flags, sizeof(init_flags), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    batch_ws_destroy(w);
    return fail(DAWN_E_DEVICE, "batch workspace: %s", hipGetErrorString(e));
  }
  *out = w;
  return DAWN_OK;
}

// Make sure planes 0 .. need-1 exist (new planes start zeroed).
dawn_status batch_ensure_planes(BatchWs* w, int need, int W) {
  if (need > kMaxPlanes)
    return fail(DAWN_E_DEVICE, "batched traversal exceeds %d levels", (1 << kMaxPlanes) - 1);
  const size_t bytes = (size_t)w->n * (size_t)w->Wmax * 8;
  while (w->nplanes < need) {
    // failure injection ($DAWN_FAIL_PLANE_AFTER = N): the plane allocation
    // after the next N fails once (a run that fails part-way through)
    const long long left = w->ctx->fail_plane_after.load();
    if (left >= 0) {
      w->ctx->fail_plane_after.fetch_sub(1);
      if (left == 0) return fail(DAWN_E_NO_MEMORY, "level plane refused (injected failure)");
    }
    u64* p = nullptr;
    const bool res = w->plane_reserve >= bytes;
    DAWN_TRY(dev_alloc(w->ctx, (void**)&p, bytes, res));
    if (res) w->plane_reserve -= bytes;
    w->bytes += bytes;
    DAWN_TRY(batch_launch_zero(w->ctx, p, bytes / 8, w->stream));
    w->planes[w->nplanes++] = p;
  }
  (void)W;
  return DAWN_OK;
}

BatchArgs batch_args(const GraphRec* g, BatchWs* w, int Ws, int W) {
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.Ws = Ws;
  a.W = W > 0 ? std::min(W, Ws) : Ws;
  a.m = g->m;
  a.rp = g->rp;
  a.col = g->col;
  a.ip = g->ip;
  a.isrc = g->isrc;
  a.pcv = g->pcv;
  a.pck = g->pck;
  a.npc = g->npc;
  a.vis = w->vis;
  a.nxt[0] = w->nxt[0];
  a.nxt[1] = w->nxt[1];
  for (int b = 0; b < kMaxPlanes; ++b) a.planes[b] = w->planes[b];
  a.nplanes = w->nplanes;
  for (int i = 0; i < 2; ++i) {
    a.touched[i] = w->touched[i];
    a.fmap[i] = w->fmap[i];
  a.vmap = w->vmap;
    a.cu[i] = w->cu[i];
    a.ck[i] = w->ck[i];
  }
  a.ctrl = w->ctrl;
  a.act = w->act;
  a.rows = w->rows;
  a.base = w->base;
  a.flags = w->flags;
  return a;
}

void batch_knobs(BatchArgs& a, const dawn_params& p) {
  a.big_b = std::max(p.batch_big_degree, kBigB);
  a.wide_scan = std::max(p.batch_wide_scan, 1);
  a.sparse_words = std::min(std::max(p.batch_sparse_words, 1), kSparseWords);
}

BatchLevelSum batch_level_sum(const BatchLevel& l) {
  BatchLevelSum s;
  memset(&s, 0, sizeof(s));
  for (int i = 0; i < kStripes; ++i) {
    s.nodes += l.s[i].nodes;
    s.bits += l.s[i].bits;
    s.se += l.s[i].se;
    s.mf += l.s[i].mf;
    s.edges += l.s[i].edges;
    s.mfw += l.s[i].mfw;
  }
  s.nchunks = l.nchunks;
  return s;
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
  const int P = pow2_at_least(a.W);
  const int grid = ctx->num_cu * 8;
#define DAWN_MERGE(PP)                                                                   \
  case PP:                                                                               \
    hipLaunchKernelGGL(batch_merge<PP>, dim3(grid), dim3(kBatchBlock), 0, s, a, L);     \
    break;
  switch (P) {
    DAWN_MERGE(1)
    DAWN_MERGE(2)
    DAWN_MERGE(4)
    DAWN_MERGE(8)
    DAWN_MERGE(16)
    DAWN_MERGE(32)
    DAWN_MERGE(64)
    default: return fail(DAWN_E_INVALID_ARG, "batch too wide");
  }
#undef DAWN_MERGE
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

template <int DMAX, int EG>
static dawn_status launch_emit_t(Ctx* ctx, const BatchArgs& a, int D, const u64* d_emask, int mode,
                                 hipStream_t s) {
  // one resident wave per slot: the tasks are equal, so a grid larger than
  // what fits at once would only add a tail
  static std::atomic<int> occ_cache{0};
  int occ = occ_cache.load(std::memory_order_relaxed);
  if (!occ) {
    DAWN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_emit<DMAX, EG>, kBatchBlock, 0));
    occ = std::max(occ, 1);
    occ_cache.store(occ, std::memory_order_relaxed);
  }
  const long long tasks = (long long)((a.n + kWave - 1) / kWave) * ((a.W + EG - 1) / EG);
  const long long per_block = kBatchBlock / kWave;
  const int grid = (int)std::max<long long>(
      1, std::min<long long>((tasks + per_block - 1) / per_block, (long long)ctx->num_cu * occ));
  const int claim = tasks >= 4 * (long long)grid * per_block ? 1 : 0;
  hipLaunchKernelGGL((batch_emit<DMAX, EG>), dim3(grid), dim3(kBatchBlock), 0, s, a, D, d_emask,
                     mode, claim);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

// The level planes a lane holds take (1 + DMAX) x EG register pairs; the
// word group shrinks as the planes grow so that stays at 64 words.
dawn_status batch_launch_emit(Ctx* ctx, const BatchArgs& a, int nplanes_used, const u64* d_emask,
                              int mode, hipStream_t s) {
  if (mode & kEmitFromRun) {
    // the plane count is known on the device only: every variant is queued
    // and the one whose range holds it runs
    DAWN_TRY((launch_emit_t<3, 16>(ctx, a, 0, d_emask, mode, s)));
    DAWN_TRY((launch_emit_t<7, 8>(ctx, a, 0, d_emask, mode, s)));
    DAWN_TRY((launch_emit_t<15, 4>(ctx, a, 0, d_emask, mode, s)));
    return launch_emit_t<16, 2>(ctx, a, 0, d_emask, mode, s);
  }
  const int D = nplanes_used;
  if (D <= 3) return launch_emit_t<3, 16>(ctx, a, D, d_emask, mode, s);
  if (D <= 7) return launch_emit_t<7, 8>(ctx, a, D, d_emask, mode, s);
  if (D <= 15) return launch_emit_t<15, 4>(ctx, a, D, d_emask, mode, s);
  return launch_emit_t<16, 2>(ctx, a, D, d_emask, mode, s);
}

dawn_status batch_launch_zero(Ctx* ctx, u64* p, size_t count, hipStream_t s) {
  if (!count) return DAWN_OK;
  const int grid = (int)std::max<size_t>(1, std::min<size_t>((count + kBatchBlock - 1) / kBatchBlock,
                                                              (size_t)ctx->num_cu * 16));
  hipLaunchKernelGGL(batch_zero, dim3(grid), dim3(kBatchBlock), 0, s, p, count);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_zero_list(Ctx* ctx, const ZeroList& z, hipStream_t s) {
  if (z.k <= 0) return DAWN_OK;
  if (z.k > kZeroMax) return fail(DAWN_E_INVALID_ARG, "too many arrays to clear");
  size_t most = 1;
  for (int i = 0; i < z.k; ++i) most = std::max(most, z.count[i]);
  const int gx = (int)std::min<size_t>((most + kBatchBlock - 1) / kBatchBlock, (size_t)ctx->num_cu * 4);
  hipLaunchKernelGGL(batch_zero_list, dim3(gx, z.k), dim3(kBatchBlock), 0, s, z);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_level_prep(const BatchActWords& act, u64* d_act, BatchCtrl* ctrl, int slot,
                                    hipStream_t s) {
  hipLaunchKernelGGL(batch_level_prep, dim3(1), dim3(kWave), 0, s, act, d_act, ctrl, slot);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_control(const BatchArgs& a, u64* act, int L, const dawn_params& p,
                                 hipStream_t s) {
  hipLaunchKernelGGL(batch_control, dim3(1), dim3(kWave), 0, s, a, act, L, p.direction,
                     (double)p.batch_alpha);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

dawn_status batch_launch_seed(Ctx* ctx, const BatchArgs& a, const int32_t* d_src,
                              const int32_t* d_lane, int k, int L, bool live, hipStream_t s) {
  (void)ctx;
  hipLaunchKernelGGL(batch_seed, dim3((k + 255) / 256), dim3(256), 0, s, a, d_src, d_lane, k, L,
                     live ? 1 : 0);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

// Choose push or pull for the next level from the counters of the last one.
// A push touches, per frontier node, its out-edges times its nonzero words;
// a pull reads every node's W visited words (and scans in-lists).
bool batch_choose_pull(const dawn_params& p, const BatchLevelSum& last, int n, int W) {
  if (p.direction == 1) return false;
  if (p.direction == 2) return true;
  return (double)last.mfw * (double)p.batch_alpha >= (double)n * (double)W;
}

static int bit_length(int x) {
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

// The prepare step's list: the control block first, then every array a run
// writes, whole (an earlier run may have used a wider row stride).
static ZeroList prepare_list(const GraphRec* g, const BatchWs* w) {
  ZeroList z;
  memset(&z, 0, sizeof(z));
  auto add = [&z](void* p, size_t count) {
    z.p[z.k] = (u64*)p;
    z.count[z.k++] = count;
  };
  const size_t nW = (size_t)g->n * (size_t)w->Wmax;
  const size_t nwords = ((size_t)g->n + 63) / 64;
  add(w->ctrl, sizeof(BatchCtrl) / 8);
  add(w->vis, nW);
  add(w->nxt[0], nW);
  add(w->nxt[1], nW);
  add(w->touched[0], nwords);
  add(w->touched[1], nwords);
  add(w->fmap[0], (size_t)g->n);
  add(w->fmap[1], (size_t)g->n);
  add(w->vmap, (size_t)g->n);
  for (int b = 0; b < w->nplanes; ++b) add(w->planes[b], nW);
  return z;
}

static dawn_status batch_launch_prepare(Ctx* ctx, const GraphRec* g, BatchWs* w, bool clear_status,
                                        hipStream_t s) {
  static_assert(9 + kMaxPlanes <= kZeroMax, "prepare list too long");
  const ZeroList z = prepare_list(g, w);
  const size_t most = (size_t)g->n * (size_t)w->Wmax;
  const int gx = (int)std::max<size_t>(
      1, std::min<size_t>((most + kBatchBlock - 1) / kBatchBlock, (size_t)ctx->num_cu * 4));
  hipLaunchKernelGGL(batch_prepare, dim3(gx), dim3(kBatchBlock), 0, s, z, w->flags,
                     clear_status ? 1 : 0);
  DAWN_HIP(hipGetLastError());
  return DAWN_OK;
}

// The rows of a dawn_mssp batch: lane r writes row_base + r x row_stride, all
// lanes < k are emitted, every source joins at level 0.
static void set_rows(BatchArgs& a, int32_t* row_base, long long row_stride, int k) {
  a.rows = nullptr;
  a.row_base = row_base;
  a.row_stride = row_stride;
  a.emit_k = k;
  a.base = nullptr;
  a.gated = 1;
}

// One batch of k <= lanes sources through the level loop, in steps so that
// several batches (each on its own workspace and stream) can run side by
// side: begin, then chunks of levels (enqueue, and after a stream sync,
// check) until the run state says done, then finish (emission).
struct BatchJob {
  BatchWs* w = nullptr;
  int k = 0;
  int W = 0;
  BatchArgs a;
  int32_t* row_base = nullptr;
  long long row_stride = 0;
  const dawn_params* p = nullptr;
  int L = 1;        // first level of the next chunk
  int Lend = 0;     // last level of the chunk in flight
  int chunk = 4;
  int launches = 0;
  bool done = false;
};

static dawn_status batch_begin(Ctx* ctx, const GraphRec* g, BatchJob& j, const int32_t* h_src,
                               int k) {
  BatchWs* w = j.w;
  j.k = k;
  j.W = (k + 63) / 64;
  hipStream_t s = w->stream;
  DAWN_HIP(hipMemcpyAsync(w->src, h_src, (size_t)k * 4, hipMemcpyHostToDevice, s));
  DAWN_HIP(hipEventRecord(w->ev0, s));
  DAWN_TRY(batch_launch_prepare(ctx, g, w, true, s));
  j.a = batch_args(g, w, j.W);
  batch_knobs(j.a, *j.p);
  set_rows(j.a, j.row_base, j.row_stride, k);
  DAWN_TRY(batch_launch_seed(ctx, j.a, w->src, nullptr, k, 0, false, s));
  DAWN_TRY(batch_launch_merge(ctx, j.a, 0, s));
  j.launches = 3;
  j.L = 1;
  const int hint = g->batch_hint.load(std::memory_order_relaxed);
  j.chunk = hint > 0 ? std::min(hint, 64) : 4;
  j.done = false;
  return DAWN_OK;
}

// Levels go out in chunks without a host round trip: batch_control picks
// each level's direction on the device and stops the run, after which the
// chunk's remaining launches return at once.  The host reads the run state
// once per chunk; the first chunk is as long as the graph's last run.
static dawn_status batch_enqueue(Ctx* ctx, const GraphRec* g, const dawn_params& p, BatchJob& j) {
  BatchWs* w = j.w;
  hipStream_t s = w->stream;
  const int L = j.L;
  if (L > g->n + 1) return fail(DAWN_E_DEVICE, "watchdog: more than n levels");
  if (bit_length(L) > kMaxPlanes)
    return fail(DAWN_E_DEVICE, "batched traversal exceeds %d levels", (1 << kMaxPlanes) - 1);
  int Lend = L + j.chunk - 1;
  while (bit_length(Lend) > kMaxPlanes) --Lend;
  const int need = bit_length(Lend);
  if (need > w->nplanes) {
    DAWN_TRY(batch_ensure_planes(w, need, j.W));
    j.a = batch_args(g, w, j.W);
    batch_knobs(j.a, p);
    set_rows(j.a, j.row_base, j.row_stride, j.k);
  }
  for (int l = L; l <= Lend; ++l) {
    DAWN_TRY(batch_launch_control(j.a, w->act, l, p, s));
    DAWN_TRY(batch_launch_expand(ctx, j.a, false, l, s));
    DAWN_TRY(batch_launch_expand(ctx, j.a, true, l, s));
    DAWN_TRY(batch_launch_merge(ctx, j.a, l, s));
    j.launches += 4;
  }
  DAWN_HIP(hipMemcpyAsync(&w->h_ctrl->run, &w->ctrl->run, sizeof(BatchRun),
                          hipMemcpyDeviceToHost, s));
  j.Lend = Lend;
  return DAWN_OK;
}

// After the stream has drained the chunk.
static dawn_status batch_check(BatchJob& j) {
  const BatchRun& r = j.w->h_ctrl->run;
  if (r.done == 1) {
    j.done = true;
    return DAWN_OK;
  }
  if (r.done) return fail(DAWN_E_DEVICE, "batched level loop stopped (watchdog)");
  j.L = j.Lend + 1;
  j.chunk = std::min(j.chunk * 2, 64);
  return DAWN_OK;
}

static dawn_status batch_finish(Ctx* ctx, const GraphRec* g, BatchJob& j, BatchTotals* tot) {
  BatchWs* w = j.w;
  const BatchRun run = w->h_ctrl->run;
  tot->edges += run.edges;
  tot->reached += run.reached;
  tot->source_edges += run.source_edges;
  tot->push_levels += run.push_levels;
  tot->pull_levels += run.pull_levels;
  const int last_nonempty = run.last_nonempty;
  // expansions 1 .. last_nonempty + 1, then the control step that ends the run
  g->batch_hint.store(std::min(last_nonempty + 2, 64), std::memory_order_relaxed);
  // every lane is emitted and its bits cleared: the workspace is left clear
  DAWN_TRY(batch_launch_emit(ctx, j.a, bit_length(last_nonempty), nullptr,
                             kEmitClear | kEmitMarkClean, w->stream));
  j.launches += 1;
  DAWN_HIP(hipEventRecord(w->ev1, w->stream));
  tot->launches += j.launches;
  tot->levels = std::max(tot->levels, last_nonempty + 1);
  return DAWN_OK;
}

// Batches that run side by side: small graphs leave most of the device idle
// in one batch's level kernels.
constexpr int kConcurrentBatches = 4;

static BatchWs* pool_take(GraphRec* g, int lanes) {
  std::lock_guard<std::mutex> lk(g->mu);
  for (size_t i = 0; i < g->batch_pool.size(); ++i) {
    BatchWs* c = g->batch_pool[i];
    if (c->lanes >= lanes) {
      g->batch_pool.erase(g->batch_pool.begin() + i);
      return c;
    }
  }
  return nullptr;
}

static void pool_give(GraphRec* g, BatchWs* w) {
  std::lock_guard<std::mutex> lk(g->mu);
  g->batch_pool.push_back(w);
}

// A workspace from the pool, or a new one; work on stream s then follows the
// last work queued on it (by a call on any stream).
// (s == null: the workspace's own stream).
static dawn_status ws_acquire(Ctx* ctx, GraphRec* g, int lanes, const hipStream_t* s,
                              BatchWs** out) {
  BatchWs* w = pool_take(g, lanes);
  if (!w) DAWN_TRY(batch_ws_create(ctx, g, lanes, &w));
  if (w->busy_set) {
    hipError_t e = hipStreamWaitEvent(s ? *s : w->stream, w->busy, 0);
    if (e != hipSuccess) {
      pool_give(g, w);
      return fail(DAWN_E_DEVICE, "stream wait: %s", hipGetErrorString(e));
    }
  }
  *out = w;
  return DAWN_OK;
}

// Device staging of host-destination rows, kept per graph between calls.
static dawn_status stage_take(Ctx* ctx, GraphRec* g, size_t bytes, int32_t** out) {
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->stage && g->stage_bytes >= bytes) {
      *out = g->stage;
      g->stage = nullptr;
      return DAWN_OK;
    }
  }
  return dev_alloc(ctx, (void**)out, bytes);
}

static void stage_give(Ctx* ctx, GraphRec* g, int32_t* p, size_t bytes) {
  int32_t* drop = p;
  size_t drop_bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->stage || g->stage_bytes < bytes) {
      drop = g->stage;
      drop_bytes = g->stage_bytes;
      g->stage = p;
      g->stage_bytes = bytes;
    }
  }
  if (drop) dev_free(ctx, drop, drop_bytes);
}

dawn_status mssp_run(Ctx* ctx, GraphRec* g, const dawn_params& p, const int32_t* sources, int32_t k,
                     int32_t* dist, bool device_out, int64_t row_stride, dawn_run_stats* stats) {
  const uint64_t t0 = now_ns();
  if (k <= 0) return DAWN_OK;   // the entry points return before this
  const int lanes = std::min(p.batch_lanes, kMaxBatchLanes);
  const int nbatches = (int)(((int64_t)k + lanes - 1) / lanes);
  const int kb_max = std::min(lanes, (int)k);
  // host destination: every row is staged on the device and copied out once
  // all batches have finished, so a failure leaves dist untouched
  int32_t* stage = nullptr;
  const size_t stage_bytes = device_out ? 0 : (size_t)k * (size_t)g->n * 4;
  if (!device_out) DAWN_TRY(stage_take(ctx, g, stage_bytes, &stage));
  // workspaces: from the pool, then new ones while the budget allows (at
  // least one, or the call fails)
  std::vector<BatchWs*> ws;
  const int want = std::max(1, std::min(nbatches, kConcurrentBatches));
  while ((int)ws.size() < want) {
    BatchWs* w = nullptr;
    dawn_status cs = ws_acquire(ctx, g, kb_max, nullptr, &w);
    if (cs != DAWN_OK) {
      if (ws.empty()) {
        // a failed call keeps no staging: the budget goes back at once
        if (stage) dev_free(ctx, stage, stage_bytes);
        return cs;
      }
      break;
    }
    ws.push_back(w);
  }
  const int conc = (int)ws.size();
  BatchTotals tot;
  memset(&tot, 0, sizeof(tot));
  dawn_status st = DAWN_OK;
  std::vector<BatchJob> jobs(conc);
  for (int bg = 0; bg < nbatches && st == DAWN_OK; bg += conc) {
    const int nj = std::min(conc, nbatches - bg);
    for (int i = 0; i < nj && st == DAWN_OK; ++i) {
      const int64_t b0 = (int64_t)(bg + i) * lanes;
      const int kb = (int)std::min<int64_t>(lanes, k - b0);
      BatchJob& j = jobs[i];
      j = BatchJob();
      j.w = ws[i];
      j.row_base = device_out ? dist + (size_t)b0 * row_stride : stage + (size_t)b0 * g->n;
      j.row_stride = device_out ? row_stride : g->n;
      j.p = &p;
      st = batch_begin(ctx, g, j, sources + b0, kb);
    }
    // chunks of levels, all running batches side by side
    for (bool busy = true; busy && st == DAWN_OK;) {
      busy = false;
      for (int i = 0; i < nj && st == DAWN_OK; ++i)
        if (!jobs[i].done) st = batch_enqueue(ctx, g, p, jobs[i]);
      for (int i = 0; i < nj && st == DAWN_OK; ++i) {
        if (jobs[i].done) continue;
        hipError_t e = hipStreamSynchronize(ws[i]->stream);
        if (e != hipSuccess) {
          st = fail(DAWN_E_DEVICE, "batched level loop: %s", hipGetErrorString(e));
          break;
        }
        st = batch_check(jobs[i]);
        busy |= !jobs[i].done;
      }
    }
    for (int i = 0; i < nj && st == DAWN_OK; ++i) st = batch_finish(ctx, g, jobs[i], &tot);
    float group_ms = 0.f;
    for (int i = 0; i < nj && st == DAWN_OK; ++i) {
      hipError_t e = hipStreamSynchronize(ws[i]->stream);
      // the group's device time: first start to last end
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ws[0]->ev0, ws[i]->ev1);
      if (e != hipSuccess) {
        st = fail(DAWN_E_DEVICE, "batched run: %s", hipGetErrorString(e));
        break;
      }
      group_ms = std::max(group_ms, ms);
    }
    tot.kernel_ms += group_ms;
  }
  if (st == DAWN_OK && !device_out) {
    hipError_t e = hipMemcpy2DAsync(dist, (size_t)row_stride * 4, stage, (size_t)g->n * 4,
                                    (size_t)g->n * 4, (size_t)k, hipMemcpyDeviceToHost,
                                    ws[0]->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ws[0]->stream);
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "copy to host: %s", hipGetErrorString(e));
  }
  if (stage) {
    for (BatchWs* w : ws) hipStreamSynchronize(w->stream);
    if (st == DAWN_OK)
      stage_give(ctx, g, stage, stage_bytes);
    else
      dev_free(ctx, stage, stage_bytes);
  }
  if (st == DAWN_OK) {
    for (BatchWs* w : ws) {
      w->busy_set = false;   // every stream of the call has drained
      pool_give(g, w);
    }
  } else {
    for (BatchWs* w : ws) {
      hipStreamSynchronize(w->stream);
      batch_ws_destroy(w);
    }
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
    stats->kernel_clock_ms = 0.0;
  }
  return DAWN_OK;
}

// ------------------------------------------------- device-ordered batches --
__global__ void write_status(int32_t* out, int32_t v) { *out = v; }

template <int P>
static dawn_status launch_finish_t(Ctx* ctx, const BatchArgs& a, u64* act, int L0,
                                   const dawn_params& p, hipStream_t s) {
  static std::atomic<int> occ_cache{0};
  int occ = occ_cache.load(std::memory_order_relaxed);
  if (!occ) {
    DAWN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_finish_levels<P>, kBatchBlock, 0));
    if (occ < 1) return fail(DAWN_E_DEVICE, "cooperative level kernel cannot be resident");
    occ_cache.store(occ, std::memory_order_relaxed);
  }
  BatchArgs args = a;
  int l0 = L0;
  int dir = p.direction;
  double alpha = (double)p.batch_alpha;
  void* kargs[] = {&args, &act, &l0, &dir, &alpha};
  DAWN_HIP(hipLaunchCooperativeKernel((const void*)batch_finish_levels<P>,
                                      dim3(occ * ctx->num_cu), dim3(kBatchBlock), kargs, 0, s));
  return DAWN_OK;
}

static dawn_status launch_finish(Ctx* ctx, const BatchArgs& a, u64* act, int L0,
                                 const dawn_params& p, hipStream_t s) {
  switch (pow2_at_least(a.W)) {
    case 1: return launch_finish_t<1>(ctx, a, act, L0, p, s);
    case 2: return launch_finish_t<2>(ctx, a, act, L0, p, s);
    case 4: return launch_finish_t<4>(ctx, a, act, L0, p, s);
    case 8: return launch_finish_t<8>(ctx, a, act, L0, p, s);
    case 16: return launch_finish_t<16>(ctx, a, act, L0, p, s);
    case 32: return launch_finish_t<32>(ctx, a, act, L0, p, s);
    case 64: return launch_finish_t<64>(ctx, a, act, L0, p, s);
    default: return fail(DAWN_E_INVALID_ARG, "batch too wide");
  }
}

// Levels queued as separate launches before the cooperative tail takes over.
constexpr int kDeviceHintMax = 256;

dawn_status mssp_device_run(Ctx* ctx, GraphRec* g, const dawn_params& p, const int32_t* d_src,
                            int32_t k, int32_t* d_dist, int32_t* d_status, hipStream_t s) {
  if (k <= 0) {
    if (d_status) {
      hipLaunchKernelGGL(write_status, dim3(1), dim3(1), 0, s, d_status, (int32_t)DAWN_OK);
      DAWN_HIP(hipGetLastError());
    }
    return DAWN_OK;
  }
  const int lanes = std::min(p.batch_lanes, kMaxBatchLanes);
  const int kb_max = std::min(lanes, (int)k);
  BatchWs* w = nullptr;
  DAWN_TRY(ws_acquire(ctx, g, kb_max, &s, &w));
  // the last device-ordered run on this workspace, if it has finished, tells
  // how many levels to queue as separate launches
  if (w->busy_set && hipEventQuery(w->busy) == hipSuccess && w->h_ctrl->run.done == 1)
    g->batch_hint.store(std::min(w->h_ctrl->run.last_nonempty + 2, kDeviceHintMax),
                        std::memory_order_relaxed);
  // planes for the deepest run a graph of n nodes can have (fewer than n
  // levels), up to kMaxPlanes: the planes cannot grow while the run is queued
  const int need = std::min(kMaxPlanes, std::max(1, bit_length(g->n)));
  dawn_status st = DAWN_OK;
  if (need > w->nplanes) {
    // zeroed on the workspace's stream, which the call's stream then follows
    st = batch_ensure_planes(w, need, 0);
    if (st == DAWN_OK) {
      hipError_t e = hipEventRecord(w->busy, w->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, w->busy, 0);
      if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "stream wait: %s", hipGetErrorString(e));
    }
  }
  if (st == DAWN_OK) {
    hipLaunchKernelGGL(batch_validate, dim3(1), dim3(1024), 0, s, d_src, (long long)k, g->n,
                       w->flags);
    if (hipGetLastError() != hipSuccess) st = fail(DAWN_E_DEVICE, "validate launch failed");
  }
  const int hint0 = g->batch_hint.load(std::memory_order_relaxed);
  const int hint = hint0 > 0 ? std::min(hint0, kDeviceHintMax) : 8;
  for (int64_t b0 = 0; b0 < k && st == DAWN_OK; b0 += lanes) {
    const int kb = (int)std::min<int64_t>(lanes, k - b0);
    const int W = (kb + 63) / 64;
    st = batch_launch_prepare(ctx, g, w, false, s);
    BatchArgs a = batch_args(g, w, W);
    batch_knobs(a, p);
    set_rows(a, d_dist + (size_t)b0 * g->n, g->n, kb);
    if (st == DAWN_OK) st = batch_launch_seed(ctx, a, d_src + b0, nullptr, kb, 0, false, s);
    if (st == DAWN_OK) st = batch_launch_merge(ctx, a, 0, s);
    for (int l = 1; l <= hint && st == DAWN_OK; ++l) {
      st = batch_launch_control(a, w->act, l, p, s);
      if (st == DAWN_OK) st = batch_launch_expand(ctx, a, false, l, s);
      if (st == DAWN_OK) st = batch_launch_expand(ctx, a, true, l, s);
      if (st == DAWN_OK) st = batch_launch_merge(ctx, a, l, s);
    }
    if (st == DAWN_OK) st = launch_finish(ctx, a, w->act, hint + 1, p, s);
    if (st == DAWN_OK)
      st = batch_launch_emit(ctx, a, 0, nullptr, kEmitClear | kEmitFromRun | kEmitMarkClean, s);
  }
  if (st == DAWN_OK && d_status) {
    hipLaunchKernelGGL(batch_status, dim3(1), dim3(1), 0, s, w->flags, d_status);
    if (hipGetLastError() != hipSuccess) st = fail(DAWN_E_DEVICE, "status launch failed");
  }
  if (st == DAWN_OK) {
    hipError_t e = hipMemcpyAsync(&w->h_ctrl->run, &w->ctrl->run, sizeof(BatchRun),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(w->busy, s);
    if (e != hipSuccess) st = fail(DAWN_E_DEVICE, "device-ordered batch: %s", hipGetErrorString(e));
  }
  if (st != DAWN_OK) {
    // launches may be queued on the caller's stream: drain it before the
    // workspace goes
    hipStreamSynchronize(s);
    batch_ws_destroy(w);
    return st;
  }
  w->busy_set = true;
  pool_give(g, w);
  return DAWN_OK;
}

}  // namespace dawn
