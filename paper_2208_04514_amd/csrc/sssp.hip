// Single-source level loop of DAWN on gfx950.
//
// One level step turns the set of nodes found at level L-1 into the set found
// at level L, in one of two directions:
//
//  * push (SOVM, paper Section 3.3, Algorithm 2 and the union-of-rows
//    identity): every frontier node's out-list is scanned and each target not
//    yet visited is claimed, gets dist = L and joins the next frontier.  Only
//    the first claimer of a node wins (an atomic OR on its visited bit), so a
//    node is queued once.  Frontier nodes with out-degree 0 are never queued
//    (the paper's processing step 2 skips them).
//  * pull (BOVM, Section 3.2, Algorithm 1 and the compressed Boolean inner
//    product): every unvisited node scans its in-list and stops at the first
//    in-neighbour that is already visited (the early exit after Algorithm 1).
//    Testing "visited" instead of "in the frontier" gives the same answer: an
//    unvisited node has distance >= L, and a visited in-neighbour at distance
//    <= L-1 puts it at exactly L.  New bits go to a second bitmap that becomes
//    current after the step, so nodes found at level L never label others at
//    the same level.
//
// The loop ends when the nodes found at a level have no out-edges at all
// (nothing can be expanded), which covers the paper's "the distance vector did
// not change" stop.  A direction switch in the style of direction-optimising
// BFS picks push or pull per level from counters of the previous level.
//
// Work assignment (64-wide wavefronts):
//  * frontier nodes with out-degree < big_degree are taken 64 at a time by one
//    wave; the wave scans their degrees and walks the union of their out-lists
//    64 edges per step, each lane finding its owner node by a binary search over
//    the wave's prefix sums (coalesced `col` reads, no idle lanes on skewed
//    degrees);
//  * nodes with out-degree >= big_degree are cut into chunks of one workgroup's
//    width when they are found, and the chunks are spread over every workgroup
//    of the grid;
//  * pull gives each wave one 64-bit word of the visited bitmap (64 nodes, one
//    per lane); a lane scans up to lane_edges in-edges, then the whole wave
//    takes over the remaining in-list of each lane still searching.
//
// Drivers: (1) one persistent cooperative kernel with a software grid barrier
// between levels, (2) one kernel per level with the counters read back by the
// host, (3) a HIP graph of level kernels replayed until a device flag says done.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>

#include <hip/hip_ext.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace dawn {

struct Counters {
  unsigned nf;
  u64 mf;
  u64 edges;
};

// Entries each wave stages in LDS before one atomic reserves room in its
// workgroup's sub-queue (an append adds at most 64, so flush above the rest).
constexpr int kWaveBuf = 256;

struct WaveQueue {
  int32_t* buf;   // this wave's LDS staging area (kWaveBuf entries)
  int cnt;        // wave-uniform fill
  // the workgroup's big-degree nodes found this level (LDS, BLOCK entries):
  // node, chunk count; filled through big_n, listed once per workgroup at
  // the end of the level
  int32_t* big_v;
  int32_t* big_c;
  unsigned* big_n;
};

__device__ __forceinline__ int32_t* small_q(const SsspArgs& a, int level) {
  return (level & 1) ? a.qs1 : a.qs0;
}
__device__ __forceinline__ int32_t* chunk_u(const SsspArgs& a, int level) {
  return (level & 1) ? a.cu1 : a.cu0;
}
__device__ __forceinline__ int32_t* chunk_k(const SsspArgs& a, int level) {
  return (level & 1) ? a.ck1 : a.ck0;
}

// Move the staged entries to this workgroup's sub-queue of level L.  Wave-uniform.
// Queue and chunk-list entries: plain accesses, or (CO) coherent ones, for
// a level whose successor runs in the same launch on other XCDs.
template <bool CO>
__device__ __forceinline__ void q_store(int32_t* p, int32_t v) {
  if constexpr (CO) {
    st_relaxed(p, v);
  } else {
    *p = v;
  }
}
template <bool CO>
__device__ __forceinline__ int32_t q_load(const int32_t* p) {
  if constexpr (CO) {
    return ld_relaxed(p);
  } else {
    return *p;
  }
}

template <bool CO>
__device__ __forceinline__ void wq_flush(const SsspArgs& a, int L, WaveQueue& q) {
  if (q.cnt == 0) return;
  const int stripe = blockIdx.x % kStripes;
  const int lane = lane_id();
  unsigned base = 0;
  if (lane == 0) base = atom_add(&a.ctrl->slot[L % 3].s[stripe].small_count, (unsigned)q.cnt);
  base = __shfl(base, 0, kWave);
  int32_t* dst = small_q(a, L) + (size_t)stripe * (size_t)a.n + base;
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < q.cnt; i += kWave) q_store<CO>(&dst[i], q.buf[i]);
  __builtin_amdgcn_wave_barrier();
  q.cnt = 0;
}

// Record node v (claimed at level L by the calling lane when `found`, out-degree
// deg) in the distance vector and in the next frontier.  Must be reached by the
// whole wave.
template <int BLOCK, bool CO>
__device__ __forceinline__ void emit_found_deg(const SsspArgs& a, int L, int v, bool found, int deg,
                                               Counters& c, WaveQueue& q) {
  if (found) {
    a.dist[v] = L;
    c.nf += 1;
    c.mf += (u64)deg;
  }
  const bool small = found && deg > 0 && deg < a.big_degree;
  const u64 mask = __ballot(small);
  if (mask) {
    const int pos = q.cnt + __popcll(mask & lanes_below());
    if (small) q.buf[pos] = v;
    q.cnt += __popcll(mask);
    if (q.cnt > kWaveBuf - kWave) wq_flush<CO>(a, L, q);
  }
  // big-degree nodes (a middle level finds tens of thousands): staged in the
  // workgroup's LDS list, whose chunks are listed with one atomic on the
  // shared chunk counter per workgroup; past the list's end a wave lists its
  // own with one atomic per wave
  const int nch = (found && deg >= a.big_degree) ? (deg + BLOCK - 1) / BLOCK : 0;
  const u64 bm = __ballot(nch > 0);
  if (bm) {
    const int lead = __ffsll((unsigned long long)bm) - 1;
    unsigned base = 0;
    if (lane_id() == lead) base = atomicAdd(q.big_n, (unsigned)__popcll(bm));
    base = (unsigned)__shfl((int)base, lead, kWave);
    const unsigned slot = base + (unsigned)__popcll(bm & lanes_below());
    const bool staged = nch > 0 && slot < (unsigned)BLOCK;
    if (staged) {
      q.big_v[slot] = v;
      q.big_c[slot] = nch;
    }
    const int rest = staged ? 0 : nch;
    if (__ballot(rest > 0)) {
      const int incl = wave_incl_scan(rest);
      unsigned gb = 0;
      if (lane_id() == kWave - 1) gb = atom_add(&a.ctrl->slot[L % 3].big_chunks, (unsigned)incl);
      gb = (unsigned)__shfl((int)gb, kWave - 1, kWave) + (unsigned)(incl - rest);
      int32_t* cu = chunk_u(a, L);
      int32_t* ck = chunk_k(a, L);
      for (int k = 0; k < rest; ++k) {
        q_store<CO>(&cu[gb + k], v);
        q_store<CO>(&ck[gb + k], k);
      }
    }
  }
}

// List the chunks of the workgroup's staged big-degree nodes (every thread
// of the workgroup calls it; resets the staging list).
template <int BLOCK, bool CO>
__device__ __forceinline__ void flush_big(const SsspArgs& a, int L, WaveQueue& q) {
  __shared__ int wsum[BLOCK / kWave];
  __shared__ unsigned gbase;
  __syncthreads();
  const unsigned nst = min(*q.big_n, (unsigned)BLOCK);
  if (nst == 0) return;   // uniform: every thread read the same count
  const int t = threadIdx.x;
  const int lane = lane_id(), wv = t / kWave;
  int v = 0, nch = 0;
  if ((unsigned)t < nst) {
    v = q.big_v[t];
    nch = q.big_c[t];
  }
  const int incl = wave_incl_scan(nch);
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  if (t == 0) {
    unsigned tot = 0;
    for (int i = 0; i < BLOCK / kWave; ++i) {
      const unsigned x = (unsigned)wsum[i];
      wsum[i] = (int)tot;
      tot += x;
    }
    gbase = atom_add(&a.ctrl->slot[L % 3].big_chunks, tot);
    *q.big_n = 0;
  }
  __syncthreads();
  const unsigned b0 = gbase + (unsigned)wsum[wv] + (unsigned)(incl - nch);
  int32_t* cu = chunk_u(a, L);
  int32_t* ck = chunk_k(a, L);
  for (int k = 0; k < nch; ++k) {
    q_store<CO>(&cu[b0 + k], v);
    q_store<CO>(&ck[b0 + k], k);
  }
}

// Prefix offsets of the kStripes sub-queues of level L-1, in LDS.
__device__ __forceinline__ void stripe_prefix(const LevelSlot* in, unsigned* pre) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned acc = 0;
    for (int s = 0; s < kStripes; ++s) {
      pre[s] = acc;
      acc += ld_relaxed(&in->s[s].small_count);
    }
    pre[kStripes] = acc;
  }
  __syncthreads();
}

// Sub-queue holding virtual entry i: largest s with pre[s] <= i.
__device__ __forceinline__ int stripe_of(const unsigned* pre, unsigned i) {
  int lo = 0;
#pragma unroll
  for (int step = kStripes / 2; step > 0; step >>= 1)
    if (pre[lo + step] <= i) lo += step;
  return lo;
}

// Claim up to four targets per lane (has[i]): every visited word, then every
// claiming atomic, then the claimed nodes' degrees are loaded as one batch
// of independent requests before the nodes are recorded.  Wave-uniform call.
template <int BLOCK, bool CO>
__device__ __forceinline__ void visit4(const SsspArgs& a, int L, u64* vis, const int* v,
                                       const bool* has, Counters& c, WaveQueue& q) {
  u64 w[4], old[4], bit[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bit[i] = 1ull << (v[i] & 63);
    w[i] = has[i] ? vis[v[i] >> 6] : bit[i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) old[i] = (w[i] & bit[i]) ? bit[i] : atom_or(&vis[v[i] >> 6], bit[i]);
  bool claim[4];
  int deg[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (has[i]) c.edges += 1;
    claim[i] = !(old[i] & bit[i]);
    deg[i] = claim[i] ? a.rp[v[i] + 1] - a.rp[v[i]] : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) emit_found_deg<BLOCK, CO>(a, L, v[i], claim[i], deg[i], c, q);
}

// Largest visited bitmap a pull level copies to LDS.
constexpr size_t kPullLdsMax = 64 << 10;

// Waves that share one group of 64 small-degree frontier nodes: enough to
// give every wave of the grid a share when the frontier has few groups
// (at most 64, one step of 256 edges each for a group of up to 16 K edges).
__device__ __forceinline__ unsigned small_split(unsigned nsmall, unsigned nwaves) {
  const unsigned groups = (nsmall + kWave - 1) / kWave;
  return groups == 0 || groups >= nwaves ? 1u : min(nwaves / groups, 64u);
}

// pre: the sub-queue offsets of level L-1 in LDS; `nch` its chunk count, or
// ~0u to have them read here.  The level's work is dealt over `nblk`
// workgroups, this one being `bid` (the grid, or one workgroup alone).
template <int BLOCK, bool CO>
__device__ void push_step(const SsspArgs& a, int L, u64* vis, Counters& c, WaveQueue& q,
                          unsigned* pre, unsigned nch, unsigned bid, unsigned nblk) {
  const LevelSlot* in = &a.ctrl->slot[(L - 1) % 3];
  if (nch == ~0u) {
    stripe_prefix(in, pre);
    nch = ld_relaxed(&in->big_chunks);
  }
  const unsigned nsmall = pre[kStripes];
  const unsigned nchunks = nch;

  // big-degree nodes: chunks of BLOCK edges, four chunks per workgroup
  // iteration (one edge of each per thread)
  const int32_t* cu = chunk_u(a, L - 1);
  const int32_t* ck = chunk_k(a, L - 1);
  for (unsigned g = bid; g < nchunks; g += 4 * nblk) {
    int v[4];
    bool has[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned gi = g + (unsigned)i * nblk;
      has[i] = false;
      v[i] = 0;
      if (gi < nchunks) {
        const int u = q_load<CO>(&cu[gi]);
        const int start = a.rp[u] + q_load<CO>(&ck[gi]) * BLOCK;
        const int end = min(start + BLOCK, a.rp[u + 1]);
        const int e = start + (int)threadIdx.x;
        has[i] = e < end;
        if (has[i]) v[i] = a.col[e];
      }
    }
    visit4<BLOCK, CO>(a, L, vis, v, has, c, q);
  }

  // small-degree nodes: groups of 64, the union of a group's rows walked 256
  // edges a step; a frontier of fewer groups than the grid has waves splits
  // each group's steps over `split` waves
  const int lane = lane_id();
  const int wpb = BLOCK / kWave;
  const unsigned gw = bid * wpb + threadIdx.x / kWave;
  const unsigned nwaves = nblk * wpb;
  const int32_t* q_in = small_q(a, L - 1);
  const unsigned split = small_split(nsmall, nwaves);
  const unsigned nvirt = (nsmall + kWave - 1) / kWave * split;
  for (unsigned vw = gw; vw < nvirt; vw += nwaves) {
    const unsigned part = vw % split;
    const unsigned i = (vw / split) * kWave + lane;
    int rs = 0, deg = 0;
    if (i < nsmall) {
      const int s = stripe_of(pre, i);
      const int u = q_load<CO>(&q_in[(size_t)s * (size_t)a.n + (i - pre[s])]);
      rs = a.rp[u];
      deg = a.rp[u + 1] - rs;
    }
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, kWave - 1, kWave);
    // four edges per lane and step; this wave takes steps part, part + split, ...
    for (int eb = (int)part * 4 * kWave; eb < total; eb += (int)split * 4 * kWave) {
      int v[4];
      bool has[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = eb + i * kWave + lane;
        has[i] = x < total;
        const int j = wave_owner(incl, has[i] ? x : total - 1);
        const int inc_j = __shfl(incl, j, kWave);
        const int deg_j = __shfl(deg, j, kWave);
        const int rs_j = __shfl(rs, j, kWave);
        v[i] = has[i] ? a.col[rs_j + (x - (inc_j - deg_j))] : 0;
      }
      visit4<BLOCK, CO>(a, L, vis, v, has, c, q);
    }
  }
}

// LDS the pull step needs per wave: a rank -> lane table and hit flags.
struct PullScratch {
  int rank_lane[kWave];
};

// `vin` is the visited bitmap of the previous level, read from LDS when the
// level kernel staged a copy there.
template <int BLOCK>
__device__ void pull_step(const SsspArgs& a, int L, const u64* vin, u64* vout, Counters& c,
                          WaveQueue& q, PullScratch* ps) {
  const int lane = lane_id();
  const int wpb = BLOCK / kWave;
  const unsigned gw = blockIdx.x * wpb + threadIdx.x / kWave;
  const unsigned nwaves = gridDim.x * wpb;
  PullScratch& sc = ps[threadIdx.x / kWave];
  // the wave's next bitmap word (and its no-in-edge word) is loaded one
  // iteration ahead, so a word's loads wait on nothing of the word before
  u64 nword = 0, nnoin = 0;
  if (gw < (unsigned)a.nw) {
    nword = vin[gw];
    nnoin = a.noin[gw];
  }
  for (unsigned w = gw; w < (unsigned)a.nw; w += nwaves) {
    const u64 word = nword;
    // nodes without in-edges can only be the source: treat them as settled
    const u64 settled = word | nnoin;
    if (w + nwaves < (unsigned)a.nw) {
      nword = vin[w + nwaves];
      nnoin = a.noin[w + nwaves];
    }
    const int v = (int)(w * kWave) + lane;
    const int valid_n = min(kWave, a.n - (int)(w * kWave));
    const u64 full = valid_n >= kWave ? ~0ull : ((1ull << valid_n) - 1ull);
    if ((settled & full) == full) {
      if (lane == 0) vout[w] = word;
      continue;
    }
    bool found = false;
    int cur = 0, e = 0, deg = 0;
    const bool unvisited = lane < valid_n && !((settled >> lane) & 1ull);
    if (unvisited) {
      cur = a.ip[v];
      e = a.ip[v + 1];
      // the out-degree, needed if the node is found, loaded with the in-list
      // bounds rather than after the search
      deg = a.rp[v + 1] - a.rp[v];
      // the lane's own first in-edges, four loads in flight per step
      const int lim = min(e, cur + a.lane_edges);
      for (; cur + 4 <= lim; cur += 4) {
        const int u0 = a.isrc[cur], u1 = a.isrc[cur + 1], u2 = a.isrc[cur + 2], u3 = a.isrc[cur + 3];
        const u64 b0 = vin[u0 >> 6] >> (u0 & 63), b1 = vin[u1 >> 6] >> (u1 & 63);
        const u64 b2 = vin[u2 >> 6] >> (u2 & 63), b3 = vin[u3 >> 6] >> (u3 & 63);
        c.edges += 4;
        if ((b0 | b1 | b2 | b3) & 1ull) {
          found = true;
          break;
        }
      }
      for (; !found && cur < lim; ++cur) {
        const int u = a.isrc[cur];
        c.edges += 1;
        if ((vin[u >> 6] >> (u & 63)) & 1ull) found = true;
      }
    }
    // lanes still searching share the wave: each round hands the 64 lanes out
    // round-robin over the searching nodes, so every round checks 64 in-edges
    // and a node leaves as soon as one of its edges hits
    bool searching = unvisited && !found && cur < e;
    u64 um = __ballot(searching);
    while (um) {
      const int cnt = __popcll(um);
      const int rank = __popcll(um & lanes_below());
      if (searching) sc.rank_lane[rank] = lane;
      __builtin_amdgcn_wave_barrier();
      const int owner = sc.rank_lane[lane % cnt];
      const int off = lane / cnt;
      const int oc = __shfl(cur, owner, kWave);
      const int oe = __shfl(e, owner, kWave);
      const int idx = oc + off;
      bool hit = false;
      if (idx < oe) {
        const int u = a.isrc[idx];
        c.edges += 1;
        hit = (vin[u >> 6] >> (u & 63)) & 1ull;
      }
      // the helpers of the node of rank r are lanes r, r + cnt, ...: fold
      // the wave's hit mask onto the ranks
      const u64 hm = __ballot(hit);
      u64 fold = 0;
      for (int sft = 0; sft < kWave; sft += cnt) fold |= hm >> sft;
      __builtin_amdgcn_wave_barrier();
      if (searching) {
        if ((fold >> rank) & 1ull) found = true;
        cur += (kWave - rank + cnt - 1) / cnt;
        searching = !found && cur < e;
      }
      um = __ballot(searching);
    }
    const u64 newbits = __ballot(found);
    if (lane == 0) vout[w] = word | newbits;
    emit_found_deg<BLOCK, false>(a, L, v, found, found ? deg : 0, c, q);
  }
}

// End of a level step for one workgroup: staged queue entries out, counters
// summed over the workgroup and added to its stripe.
template <int BLOCK, bool CO>
__device__ __forceinline__ void finish_level(const SsspArgs& a, int L, Counters& c, WaveQueue& q) {
  wq_flush<CO>(a, L, q);
  flush_big<BLOCK, CO>(a, L, q);
  block_sum3<BLOCK>(c.nf, c.mf, c.edges);
  if (threadIdx.x == 0) {
    LevelSlot* out = &a.ctrl->slot[L % 3];
    const int stripe = blockIdx.x % kStripes;
    if (c.nf) atom_add(&out->s[stripe].nf, c.nf);
    if (c.mf) atom_add(&out->s[stripe].mf, c.mf);
    if (c.edges) atom_add(&out->s[stripe].edges, c.edges);
  }
  c.nf = 0;
  c.mf = 0;
  c.edges = 0;
}

struct SlotSum {
  unsigned nf;
  u64 mf;
  u64 edges;
};

__device__ __forceinline__ SlotSum sum_slot(const LevelSlot* s) {
  SlotSum r{0, 0, 0};
  for (int i = 0; i < kStripes; ++i) {
    r.nf += ld_relaxed(&s->s[i].nf);
    r.mf += ld_relaxed(&s->s[i].mf);
    r.edges += ld_relaxed(&s->s[i].edges);
  }
  return r;
}

// Zero a slot with the calling workgroup's threads (tid / nthreads): with
// plain stores, or (CO) by atomics, done where every XCD counts, for a slot
// that other XCDs count into before this launch ends.
template <bool CO>
__device__ __forceinline__ void zero_slot(LevelSlot* s, int tid, int nthreads) {
  if constexpr (CO) {
    for (int i = tid; i < kStripes; i += nthreads) {
      SlotStripe& sp = s->s[i];
      __hip_atomic_fetch_and(&sp.nf, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_and(&sp.small_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_and(&sp.mf, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_and(&sp.edges, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) __hip_atomic_fetch_and(&s->big_chunks, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    unsigned* w = (unsigned*)s;
    const int words = (int)(sizeof(LevelSlot) / 4);
    for (int i = tid; i < words; i += nthreads) w[i] = 0;
  }
}

// Fold level st.level's counters into the state and choose level st.level+1.
// Direction switch in the style of direction-optimising BFS: go bottom-up
// (pull) when the frontier's out-edges exceed the unvisited out-edges / alpha
// while the frontier grows, and back top-down (push) when the frontier falls
// under n / beta while it shrinks.
__device__ void decide(const SsspArgs& a, LevelState& st, const SlotSum& sl, bool record) {
  const int L = st.level;
  if (sl.nf > 0) st.last_nonempty = L;
  st.mu -= (long long)sl.mf;
  st.edges_total += sl.edges;
  st.source_edges += sl.mf;
  st.reached += sl.nf;
  if (record && L < a.lrec) a.level_nf[L] = (int32_t)sl.nf;
  const unsigned prev = st.prev_nf;
  st.prev_nf = sl.nf;
  if (sl.mf == 0) {
    st.done = 1;
    return;
  }
  if (L + 1 > a.n) {
    st.done = 2;
    return;
  }
  bool pull = st.pull;
  if (a.mode == 1) {
    pull = false;
  } else if (a.mode == 2) {
    pull = true;
  } else if (!pull) {
    if ((double)sl.mf * (double)a.alpha > (double)st.mu && sl.nf > prev) pull = true;
  } else {
    if ((double)sl.nf * (double)a.beta < (double)a.n && sl.nf < prev) pull = false;
  }
  st.pull = pull ? 1 : 0;
  st.level = L + 1;
  if (pull) st.pull_levels++; else st.push_levels++;
  if (record && st.level < a.lrec) a.level_dir[st.level] = pull ? 2 : 1;
}

// Seed the source (one thread; slots 1 and 2 are zeroed by the caller).
template <int BLOCK>
__device__ void seed(const SsspArgs& a, int s) {
  const int deg = a.rp[s + 1] - a.rp[s];
  LevelSlot* sl = &a.ctrl->slot[0];
  sl->s[0].nf = 1;
  sl->s[0].mf = (u64)deg;
  if (deg > 0 && deg < a.big_degree) {
    a.qs0[0] = s;
    sl->s[0].small_count = 1;
  } else if (deg >= a.big_degree) {
    unsigned nch = (unsigned)((deg + BLOCK - 1) / BLOCK);
    for (unsigned k = 0; k < nch; ++k) {
      a.cu0[k] = s;
      a.ck0[k] = (int32_t)k;
    }
    sl->big_chunks = nch;
  }
  LevelState& st = a.ctrl->st[1];
  st.level = 0;
  st.cur = 0;
  st.pull = 0;
  st.done = 0;
  st.mu = a.m;
  st.last_nonempty = 0;
  st.push_levels = 0;
  st.pull_levels = 0;
  st.launches = 0;
  st.prev_nf = 0;
  st.mbar = 0;
  st.edges_total = 0;
  st.source_edges = 0;
  st.reached = 0;
  if (a.lrec > 0) a.level_dir[0] = 0;
}

// dist = -1 except dist[s] = 0, visited = {s}, all counter slots zero.
__device__ __forceinline__ void init_fill(const SsspArgs& a, int s) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned nt = gridDim.x * blockDim.x;
  for (unsigned i = tid; i < (unsigned)a.n; i += nt) a.dist[i] = (int)i == s ? 0 : -1;
  for (unsigned w = tid; w < (unsigned)a.nw; w += nt)
    a.vis0[w] = (int)w == (s >> 6) ? (1ull << (s & 63)) : 0ull;
  if (blockIdx.x == 0) {
    for (int i = 0; i < 3; ++i) zero_slot<false>(&a.ctrl->slot[i], threadIdx.x, blockDim.x);
    if (threadIdx.x < kStripes) a.ctrl->arrive[threadIdx.x].n = 0;
    if (threadIdx.x == 0) a.ctrl->mcount = 0;
  }
}

// ------------------------------------------------------- persistent driver --
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_persistent(SsspArgs a0) {
  SsspArgs a = a0;
  a.dist = a0.ctrl->dist;
  __shared__ int32_t qbuf[BLOCK / kWave][kWaveBuf];
  __shared__ unsigned pre[kStripes + 1];
  __shared__ PullScratch ps[BLOCK / kWave];
  __shared__ int32_t big_v[BLOCK], big_c[BLOCK];
  __shared__ unsigned big_n;
  if (threadIdx.x == 0) big_n = 0;
  WaveQueue q{qbuf[threadIdx.x / kWave], 0, big_v, big_c, &big_n};
  init_fill(a, a0.ctrl->source);
  if (!grid_sync(&a.ctrl->bar)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) seed<BLOCK>(a, a0.ctrl->source);
  if (!grid_sync(&a.ctrl->bar)) return;

  LevelState st;
  st.level = 0; st.cur = 0; st.pull = 0; st.done = 0; st.mu = a.m; st.last_nonempty = 0;
  st.push_levels = 0; st.pull_levels = 0; st.launches = 0; st.prev_nf = 0; st.edges_total = 0;
  st.source_edges = 0; st.reached = 0;
  Counters c{0, 0, 0};
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  for (;;) {
    const SlotSum prev = sum_slot(&a.ctrl->slot[st.level % 3]);
    decide(a, st, prev, leader);
    if (st.done) break;
    const int L = st.level;
    u64* vcur = st.cur ? a.vis1 : a.vis0;
    if (st.pull) {
      u64* vnext = st.cur ? a.vis0 : a.vis1;
      pull_step<BLOCK>(a, L, vcur, vnext, c, q, ps);
      st.cur ^= 1;
    } else {
      push_step<BLOCK, false>(a, L, vcur, c, q, pre, ~0u, blockIdx.x, gridDim.x);
    }
    finish_level<BLOCK, false>(a, L, c, q);
    if (blockIdx.x == 0) zero_slot<false>(&a.ctrl->slot[(L + 1) % 3], threadIdx.x, BLOCK);
    if (!grid_sync(&a.ctrl->bar)) return;
  }
  if (leader) a.ctrl->st[1] = st;
}

// The state a launch of parity `parity` leaves, to the host mirror (one
// thread).  `ended`: this launch found the end of the traversal, so the end
// stamp and tag follow, the tag ordered after the rest by a system-scope
// release, which also writes back this XCD's L2: the host returns on the tag
// and its caller may read the distances at once.  Distances stored by other
// waves of the workgroup must be complete before (their waves wait for
// their stores ahead of the barrier that precedes the report); those of
// earlier launches were written back when those launches ended.
__device__ __forceinline__ void report(const SsspArgs& a, int parity, const LevelState& s,
                                       bool ended) {
  if (!a.hm) return;
  a.hm->st[parity] = s;
  if (ended) {
    a.hm->t_end = wall_clock64();
    __hip_atomic_store(&a.hm->end_tag, (a.seq << 1) | (unsigned)parity, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ------------------------------------------------- one-workgroup traversal --
// A source whose weakly connected component has at most kCompMax nodes reaches
// at most that many: one workgroup runs its whole push level loop after the
// grid-wide init kernel (dist = -1).  The frontier lives in LDS, and so does
// the visited set: an open-addressing hash set of every node found so far
// (at most kCompMax in kCompHash slots, so probing always ends), which also
// deduplicates a level's new nodes without a global atomic per edge.  A level
// scans the frontier's degrees over the workgroup and gives each thread four
// edges per step, their target loads in flight together.
constexpr int kCompMax = 2048;
constexpr int kCompHash = 4096;    // power of two >= 2 x kCompMax

// Insert v into the LDS hash set (Knuth's multiplicative hash, linear
// probing); true if it was not there.
__device__ __forceinline__ bool comp_insert(int32_t* set, int v) {
  unsigned h = ((unsigned)v * 2654435761u) & (kCompHash - 1);
  for (;;) {
    const int old = atomicCAS(&set[h], -1, v);
    if (old == -1) return true;
    if (old == v) return false;
    h = (h + 1) & (kCompHash - 1);
  }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_component(SsspArgs a0) {
  SsspArgs a = a0;
  a.dist = a0.ctrl->dist;
  // frontier and next: node, row start, out-degree (the frontier's degrees
  // become their inclusive prefix sums while it is expanded)
  __shared__ int32_t qa[kCompMax], qb[kCompMax], ra[kCompMax], rb[kCompMax], da[kCompMax],
      db[kCompMax];
  __shared__ int32_t seen[kCompHash];
  __shared__ unsigned nnew;
  __shared__ int wscan[BLOCK / kWave];
  __shared__ int ftotal;
  __shared__ u64 wsum[2][BLOCK / kWave];
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  constexpr int NW = BLOCK / kWave;
  constexpr int PER = kCompMax / BLOCK;    // frontier entries per thread in the scan
  const int src = a0.ctrl->source;
  int32_t *cur = qa, *nxt = qb, *cur_r = ra, *nxt_r = rb, *cur_d = da, *nxt_d = db;
  for (int i = tid; i < kCompHash; i += BLOCK) seen[i] = -1;
  __syncthreads();
  if (tid == 0) {
    comp_insert(seen, src);
    qa[0] = src;
    ra[0] = a.rp[src];
    da[0] = a.rp[src + 1] - ra[0];
  }
  unsigned fsize = 1;
  u64 edges_total = 0, source_edges = (u64)(a.rp[src + 1] - a.rp[src]), reached = 1;
  int L = 0, last = 0, expansions = 0;
  for (;;) {
    if (tid == 0) nnew = 0;
    __syncthreads();
    ++L;
    ++expansions;
    // inclusive prefix sums of the frontier's degrees, in place: thread t
    // sums entries t PER .. t PER + PER - 1, the workgroup scans the sums
    int loc[PER];
    int run = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const unsigned i = (unsigned)(tid * PER + k);
      run += i < fsize ? cur_d[i] : 0;
      loc[k] = run;
    }
    int incl = wave_incl_scan(run);
    if (lane == kWave - 1) wscan[wv] = incl;
    __syncthreads();
    if (tid < kWave) {
      const int y = tid < NW ? wscan[tid] : 0;
      const int ys = wave_incl_scan(y);
      if (tid < NW) wscan[tid] = ys - y;
      if (tid == kWave - 1) ftotal = ys;
    }
    __syncthreads();
    const int excl = incl - run + wscan[wv];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const unsigned i = (unsigned)(tid * PER + k);
      if (i < fsize) cur_d[i] = excl + loc[k];
    }
    __syncthreads();
    const int total = ftotal;
    // expand: edge x of the union of the frontier's rows belongs to the
    // smallest j with prefix[j] > x
    for (int base = 0; base < total; base += 4 * BLOCK) {
      int v[4];
      bool has[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int x = base + q * BLOCK + tid;
        has[q] = x < total;
        v[q] = 0;
        if (has[q]) {
          int lo = 0, hi = (int)fsize - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cur_d[mid] > x) hi = mid; else lo = mid + 1;
          }
          const int before = lo ? cur_d[lo - 1] : 0;
          v[q] = a.col[cur_r[lo] + (x - before)];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (has[q] && comp_insert(seen, v[q])) nxt[atomicAdd(&nnew, 1u)] = v[q];
    }
    u64 my_edges = tid == 0 ? (u64)total : 0ull;
    __syncthreads();
    const unsigned found = nnew;
    // mark the new nodes: distance, out-degree sum
    u64 my_mf = 0;
    for (unsigned i = (unsigned)tid; i < found; i += BLOCK) {
      const int v = nxt[i];
      a.dist[v] = L;
      const int rs = a.rp[v], d = a.rp[v + 1] - rs;
      nxt_r[i] = rs;
      nxt_d[i] = d;
      my_mf += (u64)d;
    }
    my_edges = wave_sum(my_edges);
    my_mf = wave_sum(my_mf);
    if (lane == 0) {
      wsum[0][wv] = my_edges;
      wsum[1][wv] = my_mf;
    }
    __syncthreads();
    u64 le = 0, lm = 0;
    for (int i = 0; i < NW; ++i) {
      le += wsum[0][i];
      lm += wsum[1][i];
    }
    edges_total += le;
    if (tid == 0 && L < a.lrec) {
      a.level_nf[L] = (int32_t)found;
      a.level_dir[L] = 1;
    }
    if (found == 0) break;
    last = L;
    source_edges += lm;
    reached += found;
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    t = cur_r;
    cur_r = nxt_r;
    nxt_r = t;
    t = cur_d;
    cur_d = nxt_d;
    nxt_d = t;
    fsize = found;
    if (lm == 0) break;   // the new nodes have no out-edge: nothing left to expand
    __syncthreads();
  }
  // every wave's distance stores are complete before the end report's
  // release (a workgroup barrier alone does not wait for them)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    if (a.lrec > 0) {
      a.level_nf[0] = 1;
      a.level_dir[0] = 0;
    }
    LevelState st;
    st.level = last;
    st.cur = 0;
    st.pull = 0;
    st.done = 1;
    st.mu = 0;
    st.last_nonempty = last;
    st.push_levels = expansions;
    st.pull_levels = 0;
    st.launches = 1;
    st.prev_nf = 0;
    st.edges_total = edges_total;
    st.source_edges = source_edges;
    st.reached = reached;
    a.ctrl->st[1] = st;
    report(a, 1, st, true);
  }
}

// ------------------------------------------------------ per-level drivers --
// Initial state of one traversal.  The output row and source come as
// arguments (direct launches), or with dist == nullptr from the control
// block, where the host copied them (a captured graph or the persistent
// kernel must not depend on them).  Direct launches publish them there for
// the level kernels.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void sssp_init(SsspArgs a0, int32_t* dist, int source) {
  if (a0.hm && blockIdx.x == 0 && threadIdx.x == 0) a0.hm->t_start = wall_clock64();
  SsspArgs a = a0;
  int s = source;
  if (dist) {
    a.dist = dist;
  } else {
    a.dist = a0.ctrl->dist;
    s = a0.ctrl->source;
  }
  init_fill(a, s);
  if (blockIdx.x == 0) {
    __syncthreads();
    if (threadIdx.x == 0) {
      if (dist) {
        a0.ctrl->dist = dist;
        a0.ctrl->source = source;
      }
      seed<BLOCK>(a, s);
    }
  }
}

// One level per launch.  Launch i has parity p = i & 1: it reads the state
// left by the previous launch (st[p ^ 1]) and the counters of that level, and
// every workgroup takes the same decision for the next level (no separate
// decide launch, no fences: the kernel boundary orders the two launches).
// Workgroup 0 stores the new state in st[p].  Once the loop is done, later
// launches only carry the final state forward.
// The first wave of a workgroup reads the level state of the last launch
// and, in the same round trip, the counters of all three slots (lane 16 s + i:
// stripe i of slot s; lanes 48..50 the chunk counts), keeps the slot of level
// `level` and reduces it: the sub-queue offsets and chunk count of that
// level's frontier go to LDS (pre, *nchunks).  Returns the slot's sums in
// lane 0.
__device__ __forceinline__ SlotSum read_level_slot(const SsspArgs& a, int level, unsigned* pre,
                                                   unsigned* nchunks) {
  const int lane = threadIdx.x;
  unsigned nf = 0, sc = 0, bc = 0;
  u64 mf = 0, ed = 0;
  if (lane < 3 * kStripes) {
    const SlotStripe& sp = a.ctrl->slot[lane / kStripes].s[lane % kStripes];
    nf = ld_relaxed(&sp.nf);
    sc = ld_relaxed(&sp.small_count);
    mf = ld_relaxed(&sp.mf);
    ed = ld_relaxed(&sp.edges);
  } else if (lane < 3 * kStripes + 3) {
    bc = ld_relaxed(&a.ctrl->slot[lane - 3 * kStripes].big_chunks);
  }
  const int sel = level % 3;
  const bool mine = lane < 3 * kStripes && lane / kStripes == sel;
  if (!mine) {
    nf = sc = 0;
    mf = ed = 0;
  }
  const int sc_incl = wave_incl_scan((int)sc);
  if (mine) pre[lane % kStripes] = (unsigned)(sc_incl - (int)sc);
  const unsigned nsmall = (unsigned)__shfl(sc_incl, kWave - 1, kWave);
  const SlotSum sum{wave_sum(nf), wave_sum(mf), wave_sum(ed)};
  const unsigned nch = (unsigned)__shfl((int)bc, 3 * kStripes + sel, kWave);
  if (lane == 0) {
    pre[kStripes] = nsmall;
    *nchunks = nch;
  }
  return sum;
}


// Frontier nodes the one-workgroup loop holds: one per thread, as a pair
// (row start, out-degree) in each of two LDS lists.
template <int BLOCK>
__device__ constexpr int small_cap() {
  return BLOCK;
}

// A push level whose frontier has at most min(a.small_edges, small_cap)
// out-edges is run by workgroup 0 alone.  The bound also bounds the nodes the
// level can find (each is the target of one of those edges), so they fit in
// one LDS list, and it gives every thread at most one edge.
template <int BLOCK>
__device__ __forceinline__ bool small_push(const SsspArgs& a, const LevelState& st, const SlotSum& sum) {
  return a.small_edges > 0 && !st.done && !st.pull &&
         sum.mf <= (u64)min(a.small_edges, small_cap<BLOCK>());
}

// LDS of the one-workgroup loop besides its lists.
struct SmallShared {
  int arrived;         // every other workgroup of the launch has read its counters
  int go;              // 1 while the next level is small (medium) as well
  int ok;              // the multi-workgroup barrier completed in time
  unsigned n_next;     // nodes listed for the next level
  unsigned n_small;    // this level's small-degree queue entries
  unsigned n_chunks;   // this level's big-degree chunks
  unsigned nf;         // this level's counters
  u64 mf;
  int total;           // frontier edges of this level
  int wsum[16];        // per-wave scan totals
  LevelState st;
};

// Workgroup 0 of a launch whose levels run on some workgroups only: wait
// (bounded) until the `want` others have counted themselves in ctrl->arrive,
// then zero the count.  Every thread calls it; sh.arrived = 0 if the wait
// timed out.
template <int BLOCK>
__device__ __forceinline__ void wait_arrivals(const SsspArgs& a, SmallShared& sh, unsigned want) {
  if (threadIdx.x == 0) {
    const unsigned long long t0 = wall_clock64();
    int ok = 1;
    for (;;) {
      unsigned tot = 0;
#pragma unroll
      for (int i = 0; i < kStripes; ++i) tot += ld_relaxed(&a.ctrl->arrive[i].n);
      if (tot >= want) break;
      if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    for (int i = 0; i < kStripes; ++i) a.ctrl->arrive[i].n = 0;
    sh.arrived = ok;
  }
  __syncthreads();
}

// Workgroup-wide inclusive scan of one int per thread; returns the thread's
// prefix and leaves the total in sh.total.  Every thread calls it.
template <int BLOCK>
__device__ __forceinline__ int small_scan(int x, SmallShared& sh) {
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  int incl = wave_incl_scan(x);
  if (lane == kWave - 1) sh.wsum[wv] = incl;
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int y = threadIdx.x < BLOCK / kWave ? sh.wsum[threadIdx.x] : 0;
    const int ys = wave_incl_scan(y);
    if (threadIdx.x < BLOCK / kWave) sh.wsum[threadIdx.x] = ys - y;
    if (threadIdx.x == kWave - 1) sh.total = ys;
  }
  __syncthreads();
  return incl + sh.wsum[wv];
}

// Small push levels, one after another, by this workgroup alone (the rest of
// the grid has left).  The frontier of level st.level - 1 is read from its
// global queues once; after that each level's frontier is an LDS list of
// (row start, out-degree) pairs.  A level scans the degrees, gives thread e
// edge e of the union of the rows (at most one per thread), claims its target
// with one bitmap atomic, writes the distance, loads the target's row bounds
// and lists it for the next level; its queue entry goes straight to the
// level's global queue (sub-queue 0, or the chunk list), positions counted in
// LDS.  Counters are summed in LDS and the direction rule is applied right
// here.  When the next level is no longer small, the last level's counters go
// to its slot as the grid-wide step leaves them (one stripe) and the state
// stays at that level, so the next launch folds its counters and takes the
// same decision; a finished traversal stores its final state instead.
template <int BLOCK>
__device__ __forceinline__ void small_levels(const SsspArgs& a, LevelState st, int parity,
                                             u64* vis, const unsigned* pre, unsigned nchunks,
                                             int32_t* lists, SmallShared& sh) {
  constexpr int cap = small_cap<BLOCK>();
  const int t = threadIdx.x, lane = lane_id();
  // list b: row starts at lists[2 cap b ...], degrees (then their prefix
  // sums) at lists[2 cap b + cap ...]
  int32_t* cur = lists;
  int32_t* nxt = lists + 2 * cap;
  // the frontier from the global queues: the sub-queue entries, then each
  // big-degree node once (its chunk 0); then the nodes' rows
  {
    const int L = st.level;
    const unsigned nsmall = pre[kStripes];
    if ((unsigned)t < nsmall && t < cap) {
      const int s = stripe_of(pre, (unsigned)t);
      cur[t] = small_q(a, L - 1)[(size_t)s * (size_t)a.n + ((unsigned)t - pre[s])];
    }
    if (t == 0) sh.n_next = nsmall;
    __syncthreads();
    const int32_t* cu = chunk_u(a, L - 1);
    const int32_t* ck = chunk_k(a, L - 1);
    for (unsigned g = (unsigned)t; g < nchunks; g += BLOCK) {
      if (ck[g] == 0) {
        const unsigned pos = atomicAdd(&sh.n_next, 1u);
        if (pos < (unsigned)cap) cur[pos] = cu[g];
      }
    }
    __syncthreads();
    const unsigned nin = min(sh.n_next, (unsigned)cap);
    if ((unsigned)t < nin) {
      const int u = cur[t];
      const int rs = a.rp[u];
      cur[t] = rs;
      cur[cap + t] = a.rp[u + 1] - rs;
    }
  }
  unsigned ncur = min(sh.n_next, (unsigned)cap);
  for (;;) {
    const int L = st.level;
    __syncthreads();
    if (t == 0) {
      sh.n_next = 0;
      sh.n_small = 0;
      sh.n_chunks = 0;
      sh.nf = 0;
      sh.mf = 0;
    }
    // prefix sums of the frontier's degrees, in place
    const int incl = small_scan<BLOCK>((unsigned)t < ncur ? cur[cap + t] : 0, sh);
    if ((unsigned)t < ncur) cur[cap + t] = incl;
    __syncthreads();
    const int total = sh.total;
    const int* inc = cur + cap;
    int v = 0, rsv = 0, dv = -1;
    if (t < total) {
      // the row holding edge t: smallest j with inc[j] > t
      int lo = 0, hi = (int)ncur - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (inc[mid] > t) hi = mid; else lo = mid + 1;
      }
      const int excl = lo ? inc[lo - 1] : 0;
      v = a.col[cur[lo] + (t - excl)];
      const u64 bit = 1ull << (v & 63);
      if (!(atom_or(&vis[v >> 6], bit) & bit)) {
        a.dist[v] = L;
        rsv = a.rp[v];
        dv = a.rp[v + 1] - rsv;
      }
    }
    // the claimed nodes: counters, next list, this level's queue
    const unsigned cnf = wave_sum((unsigned)(dv >= 0 ? 1 : 0));
    const u64 cmf = wave_sum((u64)(dv > 0 ? dv : 0));
    if (lane == 0 && cnf) {
      atomicAdd(&sh.nf, cnf);
      atomicAdd(&sh.mf, cmf);
    }
    const u64 mk = __ballot(dv > 0);
    if (mk) {
      const int lead = __ffsll((unsigned long long)mk) - 1;
      unsigned b = 0;
      if (lane == lead) b = atomicAdd(&sh.n_next, (unsigned)__popcll(mk));
      b = (unsigned)__shfl((int)b, lead, kWave);
      const unsigned pos = b + (unsigned)__popcll(mk & lanes_below());
      if (dv > 0 && pos < (unsigned)cap) {
        nxt[pos] = rsv;
        nxt[cap + pos] = dv;
      }
    }
    const bool small = dv > 0 && dv < a.big_degree;
    const u64 ms = __ballot(small);
    if (ms) {
      const int lead = __ffsll((unsigned long long)ms) - 1;
      unsigned b = 0;
      if (lane == lead) b = atomicAdd(&sh.n_small, (unsigned)__popcll(ms));
      b = (unsigned)__shfl((int)b, lead, kWave);
      if (small) small_q(a, L)[b + (unsigned)__popcll(ms & lanes_below())] = v;
    }
    if (dv >= a.big_degree && dv > 0) {
      const int nch = (dv + BLOCK - 1) / BLOCK;
      const unsigned b = atomicAdd(&sh.n_chunks, (unsigned)nch);
      for (int k = 0; k < nch; ++k) {
        chunk_u(a, L)[b + k] = v;
        chunk_k(a, L)[b + k] = k;
      }
    }
    __syncthreads();
    if (t == 0) {
      LevelState nx = st;
      const SlotSum sum{sh.nf, sh.mf, (u64)total};
      decide(a, nx, sum, true);
      // (each branch stores one named struct: a select between two of
      // them would put both in scratch memory)
      const int go = small_push<BLOCK>(a, nx, sum) ? 1 : 0;
      sh.go = go;
      if (go || nx.done) {
        sh.st = nx;
      } else {
        sh.st = st;
      }
    }
    __syncthreads();
    if (!sh.go) break;
    st = sh.st;
    ncur = min(sh.n_next, (unsigned)cap);
    int32_t* sw = cur;
    cur = nxt;
    nxt = sw;
  }
  // the other workgroups decided from the slot of the level before this
  // launch's first one, which the hand-over below may overwrite.  Every wave
  // first waits for its own stores (a workgroup barrier does not), so that
  // the end report's release covers the distances of the last levels: the
  // caller may read the row as soon as the report is seen, before this
  // launch has ended
  __builtin_amdgcn_s_waitcnt(0);
  wait_arrivals<BLOCK>(a, sh, gridDim.x - 1);
  LevelState fin = sh.st;
  if (!sh.arrived) fin.done = 2;
  if (fin.done) {
    if (t == 0) {
      a.ctrl->st[parity] = fin;
      report(a, parity, fin, true);
    }
    return;
  }
  // hand over level L = fin.level (its queue is written): its counters to
  // stripe 0 of its slot, the other stripes zero, and the slot of level
  // L + 1 zeroed for the launch that runs it
  const int L = fin.level;
  {
    LevelSlot* sl = &a.ctrl->slot[L % 3];
    unsigned* w = (unsigned*)&sl->s[1];
    const int words = (int)((sizeof(SlotStripe) * (kStripes - 1)) / 4);
    for (int i = t; i < words; i += BLOCK) w[i] = 0;
    zero_slot<false>(&a.ctrl->slot[(L + 1) % 3], t, BLOCK);
  }
  if (t == 0) {
    SlotStripe& s0 = a.ctrl->slot[L % 3].s[0];
    s0.nf = sh.nf;
    s0.small_count = sh.n_small;
    s0.mf = sh.mf;
    s0.edges = (u64)sh.total;
    a.ctrl->slot[L % 3].big_chunks = sh.n_chunks;
    a.ctrl->st[parity] = fin;
    report(a, parity, fin, false);
  }
}

// Whether the push level decided in st (frontier sums `sum`) runs on a few
// workgroups with the levels after it: more out-edges than a one-workgroup
// level takes and at most a.medium_edges.
__device__ __forceinline__ bool medium_push(const SsspArgs& a, const LevelState& st,
                                            const SlotSum& sum) {
  return a.medium_edges > 0 && a.medium_groups > 1 && !st.done && !st.pull &&
         sum.mf <= (u64)a.medium_edges;
}

template <int BLOCK, bool MEDIUM>
__device__ __forceinline__ void level_step(const SsspArgs& a0, int parity) {
  SsspArgs a = a0;
  a.dist = a0.ctrl->dist;
  __shared__ int32_t qbuf[BLOCK / kWave][kWaveBuf];
  __shared__ unsigned pre[kStripes + 1];
  __shared__ PullScratch ps[BLOCK / kWave];
  __shared__ LevelState sst;
  __shared__ int idle, small, medium, ended;
  __shared__ int32_t big_v[BLOCK], big_c[BLOCK];
  __shared__ unsigned big_n, nchunks;
  if (threadIdx.x < kWave) {
    const LevelState st0 = a.ctrl->st[parity ^ 1];
    const SlotSum sum = read_level_slot(a, st0.level, pre, &nchunks);
    if (threadIdx.x == 0) {
      big_n = 0;
      ended = 0;
      LevelState st = st0;
      int sm = 0, md = 0;
      if (!st.done) {
        decide(a, st, sum, blockIdx.x == 0);
        ended = st.done ? 1 : 0;
        sm = small_push<BLOCK>(a, st, sum) ? 1 : 0;
        if constexpr (MEDIUM) md = !sm && gridDim.x > 1 && medium_push(a, st, sum) ? 1 : 0;
        // a push level with nothing for this workgroup lets it leave at once
        const unsigned nwaves = gridDim.x * (BLOCK / kWave);
        const unsigned nvirt = (pre[kStripes] + kWave - 1) / kWave *
                               small_split(pre[kStripes], nwaves);
        idle = !st.done && !st.pull && blockIdx.x * (BLOCK / kWave) >= nvirt &&
               blockIdx.x >= nchunks;
        if (sm) idle = blockIdx.x != 0;
        if (md) idle = blockIdx.x >= min(gridDim.x, (unsigned)a.medium_groups);
      } else {
        idle = 1;
      }
      small = sm;
      medium = md;
      sst = st;
    }
  }
  __syncthreads();
  LevelState st = sst;
  const bool one_group = small != 0;
  const bool few_groups = MEDIUM && medium != 0;
  if ((one_group && blockIdx.x != 0) || (few_groups && idle)) {
    // counted in: workgroup 0 may now overwrite the counters read above
    if (threadIdx.x == 0) atom_add(&a.ctrl->arrive[blockIdx.x % kStripes].n, 1u);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && !one_group) {
    LevelState out = st;
    if (!st.done && st.pull) out.cur ^= 1;
    if (!st.done || ended) out.launches += 1;
    a.ctrl->st[parity] = out;
    report(a, parity, out, ended != 0);
  }
  if (st.done) return;
  const int L0 = st.level;
  if (blockIdx.x == 0) zero_slot<MEDIUM>(&a.ctrl->slot[(L0 + 1) % 3], threadIdx.x, BLOCK);
  if (idle) return;
  WaveQueue q{qbuf[threadIdx.x / kWave], 0, big_v, big_c, &big_n};
  u64* vcur = st.cur ? a.vis1 : a.vis0;
  if (!few_groups) {
    Counters c{0, 0, 0};
    if (!one_group) {
      if (st.pull) {
        u64* vnext = st.cur ? a.vis0 : a.vis1;
        const u64* look = vcur;
        if (a.lds_words) {
          // every in-edge check of the sweep reads the bitmap: copy it to LDS
          extern __shared__ u64 lds_vis[];
          for (int i = threadIdx.x; i < a.lds_words; i += BLOCK) lds_vis[i] = vcur[i];
          __syncthreads();
          look = lds_vis;
        }
        pull_step<BLOCK>(a, L0, look, vnext, c, q, ps);
      } else {
        push_step<BLOCK, MEDIUM>(a, L0, vcur, c, q, pre, nchunks, blockIdx.x, gridDim.x);
      }
      finish_level<BLOCK, MEDIUM>(a, L0, c, q);
      return;
    }
    st.launches += 1;
    __shared__ SmallShared sh;
    small_levels<BLOCK>(a, st, parity, vcur, pre, nchunks, &qbuf[0][0], sh);
    return;
  }
  if constexpr (MEDIUM) {
    // A medium session: the first K workgroups run this push level and the
    // medium push levels after it, one after another.  A level's work is
    // dealt over the K workgroups as a grid-wide step deals it over the
    // grid; between levels they meet at a counting barrier (ctrl->mcount,
    // which only grows during a traversal: the k-th barrier of a session
    // that found it at st.mbar waits for st.mbar + k K).  What one level
    // hands to the next (queue entries, chunk lists, counters) is written
    // with coherent stores or atomics and read with coherent loads, and
    // every wave waits for its own stores before it arrives, so the barrier
    // needs no cache write-back; distances are plain stores nothing reads
    // during the traversal.  Each workgroup reads the level's counters and
    // takes the same decision.  When the next level is not a medium push
    // level (a pull level, a larger frontier, or the end), the state stays
    // at the last level run, so the next launch folds its counters, takes
    // the same decision and, at the end, reports it once every distance of
    // this launch has been written back.
    __shared__ SmallShared sh;
    const unsigned K = min(gridDim.x, (unsigned)a.medium_groups);
    const unsigned base = st.mbar;
    if (threadIdx.x == 0) {
      LevelState run = st;
      run.launches += 1;
      sh.st = run;
      sh.ok = 1;
    }
    unsigned gen = 0;
    bool waited = false;
    int L = L0;
    for (;;) {
      Counters c{0, 0, 0};
      push_step<BLOCK, true>(a, L, vcur, c, q, pre, nchunks, blockIdx.x, K);
      finish_level<BLOCK, true>(a, L, c, q);
      ++gen;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        atom_add(&a.ctrl->mcount, 1u);
        const unsigned long long t0 = wall_clock64();
        while (ld_relaxed(&a.ctrl->mcount) - base < gen * K) {
          if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
            sh.ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __syncthreads();
      if (!sh.ok) break;
      if (threadIdx.x < kWave) {
        const SlotSum sum = read_level_slot(a, L, pre, &nchunks);
        if (threadIdx.x == 0) {
          LevelState nx = sh.st;
          decide(a, nx, sum, blockIdx.x == 0);
          const int go = medium_push(a, nx, sum) ? 1 : 0;
          sh.go = go;
          if (go) sh.st = nx;   // else the state stays at level L
        }
      }
      __syncthreads();
      if (!sh.go) break;
      L = sh.st.level;
      if (blockIdx.x == 0) {
        // the slot level L + 1 counts into held the counters of level L - 2,
        // which the workgroups that left read before they left
        if (!waited) wait_arrivals<BLOCK>(a, sh, gridDim.x - K);
        waited = true;
        zero_slot<true>(&a.ctrl->slot[(L + 1) % 3], threadIdx.x, BLOCK);
      }
    }
    if (blockIdx.x != 0) return;
    if (!waited) wait_arrivals<BLOCK>(a, sh, gridDim.x - K);
    if (threadIdx.x == 0) {
      LevelState hand = sh.st;
      hand.mbar = base + gen * K;
      const bool broken = !sh.ok || !sh.arrived;
      if (broken) hand.done = 2;
      a.ctrl->st[parity] = hand;
      report(a, parity, hand, broken);
    }
  }
}

// In timing mode (a.clk set) every workgroup stamps its start and end with
// the GPU wall clock into the line of its stripe (so that the stamps of
// hundreds of workgroups do not queue on one line): the launch's own
// duration, without its dispatch gap, is the latest end minus the earliest
// start over the stripes.
// MEDIUM: the variant that can run medium push levels on a few workgroups
// (its loop around the push step costs registers, so a graph whose levels
// never qualify keeps the variant without it).
template <int BLOCK, bool MEDIUM>
__global__ __launch_bounds__(BLOCK) void sssp_level(SsspArgs a0, int parity) {
  unsigned long long* line = a0.clk ? a0.clk + (blockIdx.x % kClkStripes) * kClkWords : nullptr;
  if (line && threadIdx.x == 0) atomicMin(&line[0], (unsigned long long)wall_clock64());
  level_step<BLOCK, MEDIUM>(a0, parity);
  if (line) {
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&line[1], (unsigned long long)wall_clock64());
  }
}

// Stamp lines of `launches` launches: starts at the largest value, ends at 0.
__global__ void clk_reset(unsigned long long* clk, int launches) {
  const int lines = launches * kClkStripes;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < lines; i += gridDim.x * blockDim.x) {
    clk[(size_t)i * kClkWords] = ~0ull;
    clk[(size_t)i * kClkWords + 1] = 0ull;
  }
}

// ------------------------------------------------------------------ host --
using LevelKernel = void (*)(SsspArgs, int);

// The level kernel for these arguments: the variant with the medium-level
// loop when the medium bound is set.
template <int BLOCK>
static LevelKernel level_kernel(const SsspArgs& a) {
  return a.medium_edges > 0 ? sssp_level<BLOCK, true> : sssp_level<BLOCK, false>;
}

SsspWs::~SsspWs() {
  // a direct-launch traversal returns once its end is reported, while level
  // launches queued past the end (they only carry the final state) may still
  // be running on this stream
  if (stream) hipStreamSynchronize(stream);
  if (gexec) hipGraphExecDestroy(gexec);
  if (gexec_more) hipGraphExecDestroy(gexec_more);
  for (int i = 0; i < 2; ++i) {
    dev_free(ctx, vis[i], 0);
    dev_free(ctx, qs[i], 0);
    dev_free(ctx, cu[i], 0);
    dev_free(ctx, ck[i], 0);
  }
  dev_free(ctx, ctrl, 0);
  dev_free(ctx, dist, 0);
  dev_free(ctx, level_nf, 0);
  dev_free(ctx, level_dir, 0);
  dev_free(ctx, clk, 0);
  if (ctx) ctx->used -= bytes;
  if (h_ctrl) hipHostFree(h_ctrl);
  if (h_m) hipHostFree(h_m);
  if (ev0) hipEventDestroy(ev0);
  if (ev1) hipEventDestroy(ev1);
  if (stream) hipStreamDestroy(stream);
}

static dawn_status ws_create(Ctx* ctx, GraphRec* g, std::unique_ptr<SsspWs>* out) {
  std::unique_ptr<SsspWs> w(new SsspWs());
  w->ctx = ctx;
  const int n = g->n;
  const size_t nw = ((size_t)n + 63) / 64;
  // chunk lists: every node of out-degree >= 64 could be "big" at the smallest
  // block size; sum of ceil(deg/64) <= m/64 + n/64 + 1
  // at most m/64 big nodes (big_degree >= 64), and at most m/256 chunks of
  // >= 256 edges plus one partial chunk per big node
  const size_t chunk_cap = (size_t)(g->m / 32) + 64;
  w->chunk_cap = chunk_cap;
  w->lrec = std::min(n + 1, 1 << 16);
  SsspWs* wp = w.get();
  auto alloc = [&](void** p, size_t bytes) -> dawn_status {
    dawn_status s = dev_alloc(ctx, p, bytes);
    if (s == DAWN_OK) wp->bytes += bytes;
    return s;
  };
  dawn_status s = DAWN_OK;
  for (int i = 0; i < 2 && s == DAWN_OK; ++i) {
    if ((s = alloc((void**)&w->vis[i], nw * 8 + 256)) != DAWN_OK) break;
    if ((s = alloc((void**)&w->qs[i], (size_t)kStripes * n * 4 + 256)) != DAWN_OK) break;
    if ((s = alloc((void**)&w->cu[i], chunk_cap * 4)) != DAWN_OK) break;
    if ((s = alloc((void**)&w->ck[i], chunk_cap * 4)) != DAWN_OK) break;
  }
  if (s == DAWN_OK) s = alloc((void**)&w->ctrl, sizeof(SsspCtrl));
  if (s == DAWN_OK) s = alloc((void**)&w->dist, (size_t)n * 4);
  if (s == DAWN_OK) s = alloc((void**)&w->level_nf, (size_t)w->lrec * 4);
  if (s == DAWN_OK) s = alloc((void**)&w->level_dir, (size_t)w->lrec);

  // the destructor frees each buffer and returns `bytes` to the budget at once
  if (s != DAWN_OK) return s;
  DAWN_HIP(hipMemset(w->ctrl, 0, sizeof(SsspCtrl)));
  DAWN_HIP(hipHostMalloc((void**)&w->h_ctrl, sizeof(SsspCtrl), hipHostMallocDefault));
  DAWN_HIP(hipHostMalloc((void**)&w->h_m, sizeof(HostMirror),
                         hipHostMallocCoherent | hipHostMallocMapped));
  memset(w->h_m, 0, sizeof(HostMirror));
  DAWN_HIP(hipHostGetDevicePointer((void**)&w->d_m, w->h_m, 0));
  DAWN_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
  DAWN_HIP(hipEventCreate(&w->ev0));
  DAWN_HIP(hipEventCreate(&w->ev1));
  *out = std::move(w);
  return DAWN_OK;
}

static void fill_args(SsspArgs& a, GraphRec* g, SsspWs* w, const dawn_params& p,
                      int32_t source, int32_t* dist) {
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.nw = (g->n + 63) / 64;
  a.m = g->m;
  a.rp = g->rp;
  a.col = g->col;
  a.ip = g->ip;
  a.isrc = g->isrc;
  a.noin = g->noin;
  a.vis0 = w->vis[0];
  a.vis1 = w->vis[1];
  a.qs0 = w->qs[0];
  a.qs1 = w->qs[1];
  a.cu0 = w->cu[0];
  a.cu1 = w->cu[1];
  a.ck0 = w->ck[0];
  a.ck1 = w->ck[1];
  a.ctrl = w->ctrl;
  a.hm = w->d_m;
  a.dist = nullptr;
  (void)source;
  (void)dist;
  a.mode = p.direction;
  a.alpha = p.alpha;
  a.beta = p.beta;
  a.big_degree = std::max(p.big_degree, 64);
  a.lane_edges = std::max(p.pull_lane_edges, 1);
  a.small_edges = std::max(p.small_frontier_edges, 0);
  a.medium_edges = std::max(p.medium_edges, 0);
  a.medium_groups = std::max(p.medium_groups, 2);
  a.level_nf = w->level_nf;
  a.level_dir = w->level_dir;
  a.lrec = w->lrec;
}

template <int BLOCK>
static dawn_status launch_persistent(Ctx* ctx, SsspWs* w, const SsspArgs& a, int blocks_per_cu,
                                     bool single) {
  int occ = 0;
  DAWN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sssp_persistent<BLOCK>, BLOCK, 0));
  if (occ < 1) return fail(DAWN_E_DEVICE, "persistent kernel cannot be resident");
  int per_cu = blocks_per_cu > 0 ? std::min(blocks_per_cu, occ) : occ;
  if (single) {
    // one workgroup: its barriers are workgroup barriers, so a plain launch
    // does (a cooperative launch costs tens of microseconds more here)
    hipLaunchKernelGGL(sssp_persistent<BLOCK>, dim3(1), dim3(BLOCK), 0, w->stream, a);
    DAWN_HIP(hipGetLastError());
    return DAWN_OK;
  }
  int grid = per_cu * ctx->num_cu;
  SsspArgs args = a;
  void* kargs[] = {&args};
  DAWN_HIP(hipLaunchCooperativeKernel((const void*)sssp_persistent<BLOCK>, dim3(grid),
                                      dim3(BLOCK), kargs, 0, w->stream));
  return DAWN_OK;
}

static dawn_status capture(hipGraphExec_t* out, const std::function<void(hipStream_t)>& body) {
  hipStream_t cs = nullptr;
  DAWN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    body(cs);
    e = hipStreamEndCapture(cs, &graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  if (graph) hipGraphDestroy(graph);
  hipStreamDestroy(cs);
  if (e != hipSuccess) return fail(DAWN_E_DEVICE, "HIP graph build: %s", hipGetErrorString(e));
  return DAWN_OK;
}

// Number of the next traversal a workspace reports to its host mirror (never 0).
static unsigned next_seq(SsspWs* w) {
  w->seq = w->seq % 0x7fffffffu + 1;
  return w->seq;
}

// Spin until traversal `seq` reports its end in the host mirror (*parity: the
// parity of the state it left), or until the work queued before ev1 has all
// run without it (*parity = -1).  The event is queried every 64 spins.
static dawn_status wait_end(SsspWs* w, unsigned seq, int* parity) {
  *parity = -1;
  for (unsigned spin = 1;; ++spin) {
    const unsigned tag = __atomic_load_n(&w->h_m->end_tag, __ATOMIC_ACQUIRE);
    if ((tag >> 1) == seq) {
      *parity = (int)(tag & 1);
      return DAWN_OK;
    }
    if ((spin & 63) == 0) {
      const hipError_t e = hipEventQuery(w->ev1);
      if (e == hipSuccess) {
        // the queued work is over: the tag, if any, is in place
        const unsigned t2 = __atomic_load_n(&w->h_m->end_tag, __ATOMIC_ACQUIRE);
        if ((t2 >> 1) == seq) *parity = (int)(t2 & 1);
        return DAWN_OK;
      }
      if (e != hipErrorNotReady) DAWN_HIP(e);
    }
    __builtin_ia32_pause();
  }
}

// Direct-launch driver: level launches queued beyond what the graph's recent
// traversals needed (with none, R-MAT 20 calls ran out of launches often
// enough to cost 25 us per call on average).
constexpr int kSpareLaunches = 1;

template <int BLOCK>
static dawn_status run_levels(Ctx* ctx, GraphRec* g, SsspWs* w, const SsspArgs& a, int grid,
                              size_t shmem, int driver, int graph_levels, int32_t* d_dist,
                              int source, int* launches, double* level_ms, int* final_parity,
                              double* clock_ms) {
  const int fill_grid = std::max(1, std::min((a.n + BLOCK - 1) / BLOCK, ctx->num_cu * 8));
  const long long max_launch = (long long)a.n + 2;
  const LevelKernel kern = level_kernel<BLOCK>(a);
  if (driver == 2) {
    hipLaunchKernelGGL(sssp_init<BLOCK>, dim3(fill_grid), dim3(BLOCK), 0, w->stream, a, d_dist,
                       source);
    DAWN_HIP(hipGetLastError());
    if (level_ms) {
      if (!w->clk) {
        // stamp lines for the first 4096 launches of a traversal (2 MiB per
        // 1024 launches), kept with the workspace once timing is used
        const int cap = std::min(w->lrec, 4096);
        const size_t bytes = (size_t)cap * kClkStripes * kLine;
        DAWN_TRY(dev_alloc(ctx, (void**)&w->clk, bytes));
        w->bytes += bytes;
        w->clk_cap = cap;
      }
      hipLaunchKernelGGL(clk_reset, dim3(std::max(1, (w->clk_cap * kClkStripes + 255) / 256)),
                         dim3(256), 0, w->stream, w->clk, w->clk_cap);
      DAWN_HIP(hipGetLastError());
    }
    *launches = 1;
    int level_launches = 0;
    for (long long it = 0; it <= max_launch; ++it) {
      const int parity = (int)(it & 1);
      SsspArgs al = a;
      if (level_ms && it < w->clk_cap) al.clk = w->clk + (size_t)it * kClkStripes * kClkWords;
      if (level_ms) {
        // events attached to the dispatch itself: their timestamps are the
        // kernel's own begin and end, without the marker packets' dispatch gap
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), (uint32_t)shmem,
                              w->stream, w->ev0, w->ev1, 0, al, parity);
      } else {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), shmem, w->stream, al,
                           parity);
      }
      DAWN_HIP(hipGetLastError());
      *launches += 1;
      ++level_launches;
      if (!level_ms) DAWN_HIP(hipEventRecord(w->ev1, w->stream));
      DAWN_HIP(hipStreamSynchronize(w->stream));
      if (level_ms) {
        float ms = 0.f;
        DAWN_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
        *level_ms += ms;
      }
      if (w->h_m->st[parity].done) {
        *final_parity = parity;
        if (level_ms) {
          *launches = level_launches;
          const int nl = std::min(level_launches, w->clk_cap);
          std::vector<unsigned long long> stamps((size_t)nl * kClkStripes * kClkWords);
          DAWN_HIP(hipMemcpy(stamps.data(), w->clk, stamps.size() * 8, hipMemcpyDeviceToHost));
          double ticks = 0.0;
          for (int i = 0; i < nl; ++i) {
            unsigned long long t0 = ~0ull, t1 = 0;
            for (int sl = 0; sl < kClkStripes; ++sl) {
              const unsigned long long* ln = &stamps[((size_t)i * kClkStripes + sl) * kClkWords];
              t0 = std::min(t0, ln[0]);
              t1 = std::max(t1, ln[1]);
            }
            if (t1 > t0) ticks += (double)(t1 - t0);
          }
          if (clock_ms && ctx->wall_khz > 0) *clock_ms = ticks / (double)ctx->wall_khz;
        }
        return DAWN_OK;
      }
    }
    return fail(DAWN_E_DEVICE, "level loop did not terminate");
  }
  graph_levels += graph_levels & 1;
  if (driver == 3) {
    // K level launches queued per host check.  The first batch covers what
    // the graph's recent traversals needed (one more than their level
    // launches, for the launch that sees the end), so a typical traversal
    // costs one batch and few launches past its end; a launch after the end
    // only carries the final state along.  The host waits for the end tag in
    // the host mirror, not for the stream: it returns as soon as the launch
    // that found the end has reported (every level's writes are complete by
    // then, the launches being stream-ordered), and the launches still queued
    // behind it overlap with what the caller does next.  The stream is waited
    // on only when a batch has run out without the end.
    SsspArgs ad = a;
    ad.seq = next_seq(w);
    hipLaunchKernelGGL(sssp_init<BLOCK>, dim3(fill_grid), dim3(BLOCK), 0, w->stream, ad, d_dist,
                       source);
    *launches = 1;
    const int hint = g->launch_hint.load(std::memory_order_relaxed);
    int batch = hint > 0 ? std::min(hint + kSpareLaunches, graph_levels * 4) : graph_levels;
    long long queued = 0;
    while (queued <= max_launch) {
      for (int i = 0; i < batch; ++i)
        hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), shmem, w->stream, ad,
                           (int)((queued + i) & 1));
      DAWN_HIP(hipGetLastError());
      *launches += batch;
      queued += batch;
      DAWN_HIP(hipEventRecord(w->ev1, w->stream));
      int parity = -1;
      DAWN_TRY(wait_end(w, ad.seq, &parity));
      if (parity >= 0) {
        // launches this traversal needed: every one up to the one that
        // found the end
        const int need = w->h_m->st[parity].launches;
        g->launch_hint.store(std::max(need, hint - 1), std::memory_order_relaxed);
        *final_parity = parity;
        return DAWN_OK;
      }
      batch = graph_levels;
    }
    return fail(DAWN_E_DEVICE, "level loop did not terminate");
  }
  // driver 4: one HIP graph holds the init kernel and an even number of level
  // launches (parities 0, 1, 0, 1, ...); a second graph of level launches
  // alone continues a traversal that needs more levels
  if (w->gexec && (w->gexec_levels != graph_levels || w->gexec_block != BLOCK ||
                   memcmp(&w->gexec_args, &a, sizeof(SsspArgs)) != 0)) {
    hipGraphExecDestroy(w->gexec);
    w->gexec = nullptr;
    if (w->gexec_more) hipGraphExecDestroy(w->gexec_more);
    w->gexec_more = nullptr;
  }
  if (!w->gexec) {
    DAWN_TRY(capture(&w->gexec, [&](hipStream_t cs) {
      hipLaunchKernelGGL(sssp_init<BLOCK>, dim3(fill_grid), dim3(BLOCK), 0, cs, a,
                         (int32_t*)nullptr, 0);
      for (int i = 0; i < graph_levels; ++i)
        hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), shmem, cs, a, i & 1);
    }));
    DAWN_TRY(capture(&w->gexec_more, [&](hipStream_t cs) {
      for (int i = 0; i < graph_levels; ++i)
        hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), shmem, cs, a, i & 1);
    }));
    w->gexec_levels = graph_levels;
    w->gexec_block = BLOCK;
    w->gexec_args = a;
  }
  *launches = 0;
  for (long long it = 0; it * graph_levels <= max_launch; ++it) {
    DAWN_HIP(hipGraphLaunch(it == 0 ? w->gexec : w->gexec_more, w->stream));
    *launches += graph_levels + (it == 0 ? 1 : 0);
    DAWN_HIP(hipEventRecord(w->ev1, w->stream));
    DAWN_HIP(hipStreamSynchronize(w->stream));
    if (w->h_m->st[1].done) {
      *final_parity = 1;
      return DAWN_OK;
    }
  }
  return fail(DAWN_E_DEVICE, "level loop did not terminate");
}

// A source whose weakly connected component has at most small_n nodes (it
// reaches no more) is traversed by one workgroup (sssp_component) after the
// grid-wide init kernel.  Forced pull keeps the general path.
static bool small_component(const GraphRec* g, const dawn_params& p, int32_t source) {
  return p.small_n > 0 && p.direction != 2 && !g->comp_size.empty() &&
         g->comp_size[(size_t)source] <= std::min(p.small_n, kCompMax);
}

// Launch shape of the level kernel on a graph of nw bitmap words: the
// visited bitmap goes to LDS for pull levels when it fits next to the
// kernel's own LDS and is at most kPullLdsMax bytes (every workgroup copies
// it at each pull level; on R-MAT 20, 128 KiB, the copy costs what the
// faster in-edge checks save).  Gives the dynamic LDS, the words copied and
// the workgroups a CU holds.
// Workgroups of a level launch: blocks_per_cu per compute unit when set;
// else as many as a compute unit holds (occ), but no more than a pull level
// has bitmap words for (one wave each) and no fewer than one per compute
// unit: a small graph's launch then does not dispatch workgroups that could
// only read the state and leave (uniform4096: 75 -> 68 us per source).
template <int BLOCK>
static int level_grid(const Ctx* ctx, const dawn_params& p, const SsspArgs& a, int occ) {
  if (p.blocks_per_cu > 0) return std::min(p.blocks_per_cu, occ) * ctx->num_cu;
  const int useful = (a.nw + BLOCK / kWave - 1) / (BLOCK / kWave);
  return std::min(occ * ctx->num_cu, std::max(ctx->num_cu, useful));
}

template <int BLOCK>
static dawn_status level_shape(Ctx* ctx, LevelKernel kern, int32_t nw, size_t* lds,
                               int32_t* words, int* occ) {
  hipFuncAttributes fa;
  DAWN_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)));
  const size_t bitmap = (size_t)nw * 8;
  *lds = 0;
  *words = 0;
  if (bitmap <= kPullLdsMax && fa.sharedSizeBytes + bitmap <= ctx->lds_per_block) {
    *lds = bitmap;
    *words = nw;
    // the largest dynamic LDS any graph's launch can ask for, so graphs
    // sharing the kernel never lower each other's limit
    DAWN_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void*>(kern),
        hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)std::min(kPullLdsMax, ctx->lds_per_block - fa.sharedSizeBytes)));
  }
  int o = 0;
  DAWN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, BLOCK, *lds));
  *occ = std::max(o, 1);
  return DAWN_OK;
}

template <int BLOCK>
static dawn_status sssp_dispatch(Ctx* ctx, GraphRec* g, SsspWs* w, const dawn_params& p,
                                 SsspArgs& a, int32_t source, int32_t* d_dist, int* launches,
                                 double* level_ms, int* final_parity, double* clock_ms) {
  if (small_component(g, p, source)) {
    // the one-workgroup kernel reports its end to the host mirror too
    const int fill_grid = std::max(1, std::min((a.n + BLOCK - 1) / BLOCK, ctx->num_cu * 8));
    SsspArgs ad = a;
    ad.seq = next_seq(w);
    hipLaunchKernelGGL(sssp_init<BLOCK>, dim3(fill_grid), dim3(BLOCK), 0, w->stream, ad, d_dist,
                       source);
    hipLaunchKernelGGL(sssp_component<BLOCK>, dim3(1), dim3(BLOCK), 0, w->stream, ad);
    DAWN_HIP(hipGetLastError());
    DAWN_HIP(hipEventRecord(w->ev1, w->stream));
    int parity = -1;
    DAWN_TRY(wait_end(w, ad.seq, &parity));
    if (parity < 0) return fail(DAWN_E_DEVICE, "one-workgroup traversal ended without a report");
    *launches = 2;
    *final_parity = parity;
    return DAWN_OK;
  }
  if (p.driver == 1) {
    *launches = 1;
    *final_parity = 1;
    return launch_persistent<BLOCK>(ctx, w, a, p.blocks_per_cu, false);
  }
  // the shape depends on the graph, block size and kernel variant only:
  // found once per workspace, block size and variant
  const int bi = (BLOCK == 256 ? 0 : BLOCK == 512 ? 1 : 2) * 2 + (a.medium_edges > 0 ? 1 : 0);
  if (w->shape_grid[bi] == 0)
    DAWN_TRY(level_shape<BLOCK>(ctx, level_kernel<BLOCK>(a), a.nw, &w->shape_lds[bi],
                                &w->shape_words[bi], &w->shape_grid[bi]));
  const size_t shmem = w->shape_lds[bi];
  a.lds_words = w->shape_words[bi];
  const int occ = w->shape_grid[bi];
  return run_levels<BLOCK>(ctx, g, w, a, level_grid<BLOCK>(ctx, p, a, occ), shmem, p.driver,
                           std::max(p.graph_levels, 1), d_dist, source, launches, level_ms,
                           final_parity, clock_ms);
}

dawn_status sssp_run(Ctx* ctx, GraphRec* g, const dawn_params& p, int32_t source, int32_t* dist,
                     bool device_out, dawn_run_stats* stats) {
  const uint64_t t0 = now_ns();
  std::unique_ptr<SsspWs> w;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->sssp_pool.empty()) {
      w = std::move(g->sssp_pool.back());
      g->sssp_pool.pop_back();
    }
  }
  if (!w) DAWN_TRY(ws_create(ctx, g, &w));
  struct Return {
    GraphRec* g;
    std::unique_ptr<SsspWs>& w;
    ~Return() {
      if (w && !w->poisoned) {
        std::lock_guard<std::mutex> lk(g->mu);
        g->sssp_pool.push_back(std::move(w));
      }
    }
  } ret{g, w};

  int32_t* d_dist = device_out ? dist : w->dist;
  SsspArgs a;
  fill_args(a, g, w.get(), p, source, d_dist);
  int launches = 0;
  const bool small = small_component(g, p, source);
  const bool level_timing = p.timing == 1 && p.driver == 2 && !small;
  double level_ms = 0.0, clock_ms = 0.0;
  double* lm = level_timing ? &level_ms : nullptr;
  int fp = 1;
  const uint64_t t_setup = now_ns();
  // the persistent kernel and captured graphs read the row and source from
  // the control block; direct launches hand them to the init kernel
  if (!small && (p.driver == 1 || p.driver == 4)) {
    w->h_ctrl->dist = d_dist;
    w->h_ctrl->source = source;
    DAWN_HIP(hipMemcpyAsync(&w->ctrl->dist, &w->h_ctrl->dist, sizeof(int32_t*) + sizeof(int),
                            hipMemcpyHostToDevice, w->stream));
  }
  // the direct-launch driver times a traversal by the GPU wall clock (the
  // init kernel's start to the start of the launch that found the end), so
  // its host wait never covers the launches queued past the end; the other
  // drivers by events around everything they queue
  const bool mirrored = small || p.driver == 3;
  const bool stamped = mirrored && ctx->wall_khz > 0;
  if (!stamped) DAWN_HIP(hipEventRecord(w->ev0, w->stream));
  dawn_status st;
  switch (p.block) {
    case 512: st = sssp_dispatch<512>(ctx, g, w.get(), p, a, source, d_dist, &launches, lm, &fp, &clock_ms); break;
    case 1024: st = sssp_dispatch<1024>(ctx, g, w.get(), p, a, source, d_dist, &launches, lm, &fp, &clock_ms); break;
    default: st = sssp_dispatch<256>(ctx, g, w.get(), p, a, source, d_dist, &launches, lm, &fp, &clock_ms); break;
  }
  // the level drivers and the one-workgroup path record the end event after
  // their last launch, before the host waits; the persistent kernel here
  if (!small && p.driver == 1) DAWN_HIP(hipEventRecord(w->ev1, w->stream));
  if (st != DAWN_OK) {
    hipStreamSynchronize(w->stream);
    w->poisoned = true;
    return st;
  }
  const uint64_t t_loop = now_ns();
  // the per-level and graph drivers and the one-workgroup path already read
  // the final state back; the persistent driver's state (and its barrier's
  // abort flag) is read here
  const bool persistent = p.driver == 1 && !small;
  const int32_t cap = (stats && stats->frontier_cap > 0) ? std::min(stats->frontier_cap, w->lrec) : 0;
  std::vector<int32_t> lnf;
  std::vector<uint8_t> ldir;
  if (persistent)
    DAWN_HIP(hipMemcpyAsync(w->h_ctrl, w->ctrl, sizeof(SsspCtrl), hipMemcpyDeviceToHost,
                            w->stream));
  if (cap > 0) {
    lnf.resize(cap);
    ldir.resize(cap);
    DAWN_HIP(hipMemcpyAsync(lnf.data(), w->level_nf, cap * 4, hipMemcpyDeviceToHost, w->stream));
    DAWN_HIP(hipMemcpyAsync(ldir.data(), w->level_dir, cap, hipMemcpyDeviceToHost, w->stream));
  }
  if (persistent || cap > 0) DAWN_HIP(hipStreamSynchronize(w->stream));
  const LevelState& rs = persistent ? w->h_ctrl->st[fp] : w->h_m->st[fp];
  if (rs.done != 1) w->poisoned = true;
  if (persistent && w->h_ctrl->bar.abort) return fail(DAWN_E_DEVICE, "grid barrier timed out");
  if (rs.done == 2) return fail(DAWN_E_DEVICE, "watchdog: more than n levels");
  if (rs.done != 1) return fail(DAWN_E_DEVICE, "level loop ended without finishing");
  if (!device_out) {
    DAWN_HIP(hipMemcpyAsync(dist, w->dist, (size_t)g->n * 4, hipMemcpyDeviceToHost, w->stream));
    DAWN_HIP(hipStreamSynchronize(w->stream));
  }
  if (stats) {
    float ms = 0.f;
    if (level_timing) {
      ms = (float)level_ms;
    } else if (stamped) {
      ms = (float)((double)(w->h_m->t_end - w->h_m->t_start) / (double)ctx->wall_khz);
    } else {
      DAWN_HIP(hipEventSynchronize(w->ev1));
      DAWN_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
    }
    stats->levels = rs.last_nonempty + 1;
    stats->push_levels = rs.push_levels;
    stats->pull_levels = rs.pull_levels;
    stats->launches = launches;
    stats->edges_examined = (int64_t)rs.edges_total;
    stats->source_edges = (int64_t)rs.source_edges;
    stats->reached = (int64_t)rs.reached;
    stats->kernel_ms = ms;
    stats->kernel_clock_ms = level_timing ? clock_ms : 0.0;
    const int32_t nl = std::min(cap, stats->levels);
    if (cap > 0 && stats->frontier_sizes)
      for (int i = 0; i < nl; ++i) stats->frontier_sizes[i] = lnf[i];
    if (cap > 0 && stats->directions)
      for (int i = 0; i < nl; ++i) stats->directions[i] = ldir[i];
    stats->total_ms = (now_ns() - t0) / 1e6;
  }
  static const bool host_timing = getenv("DAWN_HOST_TIMING") != nullptr;
  if (host_timing) {
    const uint64_t t_end = now_ns();
    fprintf(stderr, "[dawn_sssp] setup %.1f us, launch+loop %.1f us, tail %.1f us\n",
            (t_setup - t0) / 1e3, (t_loop - t_setup) / 1e3, (t_end - t_loop) / 1e3);
  }
  return DAWN_OK;
}

// ------------------------------------------------ no-allocation variant --
// Callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it) run a single source with
// every buffer of the traversal carved out of this file-scope array: one per
// GPU, held until the process ends.  Calls that overlap on one GPU share it
// and race.  The host never uses the array's name as an address: each
// device's address comes from hipGetSymbolAddress at set-up.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[kScratchDevices] = {};

// With `device` current: look up this GPU's copy of the array (once).
dawn_status scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices)
    return fail(DAWN_E_INVALID_ARG, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return DAWN_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(DAWN_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch_ptr[device] = (unsigned char*)ptr;
  return DAWN_OK;
}

// Bytes of scratch a graph's traversal takes, and its layout.
struct ScratchLayout {
  size_t ctrl, vis0, vis1, qs0, qs1, cu0, cu1, ck0, ck1, lnf, ldir, total;
};

static ScratchLayout scratch_layout(const GraphRec* g) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t n = (size_t)g->n, nw = (n + 63) / 64;
  const size_t chunk_cap = (size_t)(g->m / 32) + 64;
  const size_t lrec = std::min<size_t>(n + 1, 1 << 16);
  ScratchLayout L;
  size_t o = 0;
  L.ctrl = o;  o += up(sizeof(SsspCtrl));
  L.vis0 = o;  o += up(nw * 8 + 256);
  L.vis1 = o;  o += up(nw * 8 + 256);
  L.qs0 = o;   o += up((size_t)kStripes * n * 4 + 256);
  L.qs1 = o;   o += up((size_t)kStripes * n * 4 + 256);
  L.cu0 = o;   o += up(chunk_cap * 4);
  L.cu1 = o;   o += up(chunk_cap * 4);
  L.ck0 = o;   o += up(chunk_cap * 4);
  L.ck1 = o;   o += up(chunk_cap * 4);
  L.lnf = o;   o += up(lrec * 4);
  L.ldir = o;  o += up(lrec);
  L.total = o;
  return L;
}

template <int BLOCK>
static dawn_status noalloc_levels(Ctx* ctx, GraphRec* g, const dawn_params& p, SsspArgs& a,
                                  int32_t source, int32_t* d_dist, hipStream_t s,
                                  LevelState* fin, int* launches) {
  const int fill_grid = std::max(1, std::min((a.n + BLOCK - 1) / BLOCK, ctx->num_cu * 8));
  hipLaunchKernelGGL(sssp_init<BLOCK>, dim3(fill_grid), dim3(BLOCK), 0, s, a, d_dist, source);
  DAWN_HIP(hipGetLastError());
  *launches = 1;
  if (small_component(g, p, source)) {
    hipLaunchKernelGGL(sssp_component<BLOCK>, dim3(1), dim3(BLOCK), 0, s, a);
    DAWN_HIP(hipGetLastError());
    *launches = 2;
    DAWN_HIP(hipMemcpyAsync(fin, &a.ctrl->st[1], sizeof(LevelState), hipMemcpyDeviceToHost, s));
    DAWN_HIP(hipStreamSynchronize(s));
    return DAWN_OK;
  }
  size_t shmem = 0;
  int occ = 1;
  const LevelKernel kern = level_kernel<BLOCK>(a);
  DAWN_TRY(level_shape<BLOCK>(ctx, kern, a.nw, &shmem, &a.lds_words, &occ));
  const int grid = level_grid<BLOCK>(ctx, p, a, occ);
  // level launches queued per host check, as the direct-launch driver does
  const int hint = g->launch_hint.load(std::memory_order_relaxed);
  const int gl = std::max(p.graph_levels, 1) + (std::max(p.graph_levels, 1) & 1);
  int batch = hint > 0 ? std::min(hint + 1, gl * 4) : gl;
  batch += batch & 1;
  for (long long queued = 0; queued <= (long long)a.n + 2;) {
    for (int i = 0; i < batch; ++i)
      hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), shmem, s, a, i & 1);
    DAWN_HIP(hipGetLastError());
    *launches += batch;
    queued += batch;
    // pageable host memory: the copy returns once the stream has reached it
    DAWN_HIP(hipMemcpyAsync(fin, &a.ctrl->st[1], sizeof(LevelState), hipMemcpyDeviceToHost, s));
    DAWN_HIP(hipStreamSynchronize(s));
    if (fin->done) {
      g->launch_hint.store(std::max(fin->launches, hint - 1), std::memory_order_relaxed);
      return DAWN_OK;
    }
    batch = gl;
  }
  return fail(DAWN_E_DEVICE, "level loop did not terminate");
}

dawn_status sssp_run_noalloc(Ctx* ctx, GraphRec* g, const dawn_params& p, int32_t source,
                             int32_t* d_dist, hipStream_t s, dawn_run_stats* stats) {
  const uint64_t t0 = now_ns();
  const ScratchLayout L = scratch_layout(g);
  if (L.total > kScratchBytes)
    return fail(DAWN_E_INVALID_ARG, "graph needs %zu bytes of traversal buffers; the "
                "no-allocation entry point holds %zu (n = %d, m = %lld)", L.total, kScratchBytes,
                g->n, (long long)g->m);
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = ctx->device < kScratchDevices ? g_scratch_ptr[ctx->device] : nullptr;
  }
  if (!base) return fail(DAWN_E_DEVICE, "scratch of device %d not set up", ctx->device);
  SsspArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.nw = (g->n + 63) / 64;
  a.m = g->m;
  a.rp = g->rp;
  a.col = g->col;
  a.ip = g->ip;
  a.isrc = g->isrc;
  a.noin = g->noin;
  a.ctrl = (SsspCtrl*)(base + L.ctrl);
  a.vis0 = (u64*)(base + L.vis0);
  a.vis1 = (u64*)(base + L.vis1);
  a.qs0 = (int32_t*)(base + L.qs0);
  a.qs1 = (int32_t*)(base + L.qs1);
  a.cu0 = (int32_t*)(base + L.cu0);
  a.cu1 = (int32_t*)(base + L.cu1);
  a.ck0 = (int32_t*)(base + L.ck0);
  a.ck1 = (int32_t*)(base + L.ck1);
  a.level_nf = (int32_t*)(base + L.lnf);
  a.level_dir = (uint8_t*)(base + L.ldir);
  a.lrec = (int32_t)std::min<size_t>((size_t)g->n + 1, 1 << 16);
  a.mode = p.direction;
  a.alpha = p.alpha;
  a.beta = p.beta;
  a.big_degree = std::max(p.big_degree, 64);
  a.lane_edges = std::max(p.pull_lane_edges, 1);
  a.small_edges = std::max(p.small_frontier_edges, 0);
  LevelState fin;
  memset(&fin, 0, sizeof(fin));
  int launches = 0;
  dawn_status st;
  switch (p.block) {
    case 512: st = noalloc_levels<512>(ctx, g, p, a, source, d_dist, s, &fin, &launches); break;
    case 1024: st = noalloc_levels<1024>(ctx, g, p, a, source, d_dist, s, &fin, &launches); break;
    default: st = noalloc_levels<256>(ctx, g, p, a, source, d_dist, s, &fin, &launches); break;
  }
  if (st != DAWN_OK) {
    hipStreamSynchronize(s);
    return st;
  }
  if (fin.done == 2) return fail(DAWN_E_DEVICE, "watchdog: more than n levels");
  if (fin.done != 1) return fail(DAWN_E_DEVICE, "level loop ended without finishing");
  if (stats) {
    stats->levels = fin.last_nonempty + 1;
    stats->push_levels = fin.push_levels;
    stats->pull_levels = fin.pull_levels;
    stats->launches = launches;
    stats->edges_examined = (int64_t)fin.edges_total;
    stats->source_edges = (int64_t)fin.source_edges;
    stats->reached = (int64_t)fin.reached;
    stats->kernel_ms = 0.0;
    stats->total_ms = (now_ns() - t0) / 1e6;
    stats->kernel_clock_ms = 0.0;
  }
  return DAWN_OK;
}

}  // namespace dawn
