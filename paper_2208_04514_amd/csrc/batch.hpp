// Shared declarations of the batched (bitmask-lane) traversal, used by the
// multi-source driver (mssp.hip) and the serving scheduler (serve.cpp).
#pragma once

#include "internal.hpp"

namespace dawn {

constexpr int kMaxPlanes = 16;    // relative levels up to 2^16 - 1 per source
constexpr int kMaxBatchLanes = 4096;  // sources one batch carries: 64 words of 64 lanes

// One stripe (a whole cache line) of the counters of one level of a batch.
struct alignas(kLine) BatchStripe {
  u64 nodes;                    // nodes that received a new bit
  u64 bits;                     // new (node, source) pairs
  u64 se;                       // sum over new pairs of the node's out-degree
  u64 mf;                       // sum of out-degrees of the nodes with a new bit
  u64 edges;                    // adjacency entries read by the expansion
  u64 mfw;                      // sum over nodes with a new bit of out-degree x nonzero words
};

// Counters of one level of a batch (two slots, indexed level & 1), striped
// over kStripes lines like the single-source counters.
struct BatchLevel {
  BatchStripe s[kStripes];
  alignas(kLine) unsigned nchunks;   // entries of the big-degree out-edge chunk list
};

struct BatchLevelSum {
  u64 nodes, bits, se, mf, edges, mfw;
  unsigned nchunks;
};

// State of a level loop that runs without the host: batch_control, run once
// before each level's expansion, folds the previous level's counters into the
// totals, sets the active-lane words and the direction, and raises `done`
// when no lane is active; the expansion and merge kernels of that level and
// of every later one then return at once.
struct alignas(kLine) BatchRun {
  int done;                     // 0 running, 1 finished, 2 watchdog (too many levels or a
                                //   grid barrier timed out), 3 stopped by an invalid source
  int pull;                     // 1: the level being expanded pulls
  int last_nonempty;            // last level that found new bits
  int push_levels, pull_levels;
  u64 edges, reached, source_edges;
};

struct BatchCtrl {
  BatchLevel lv[2];
  BatchRun run;
  GridBarrier bar;              // the cooperative tail of a device-ordered run
  // next emission task to claim (cleared before every emission: at the start
  // of a batched run, and by serving's per-level prep)
  alignas(kLine) unsigned emit_next;
  // OR of the new bits of each word, per level parity, striped like the
  // counters (a workgroup ORs into stripe blockIdx % kStripes)
  u64 laneact[2][kStripes][64];
};

// Lanes of word w that found new bits at a level of parity `par`.
inline u64 lane_activity(const BatchCtrl& c, int par, int w) {
  u64 x = 0;
  for (int i = 0; i < kStripes; ++i) x |= c.laneact[par][i][w];
  return x;
}

struct BatchArgs {
  int32_t n;
  int32_t W;                    // 64-bit words processed per node (lanes in use / 64, rounded up)
  int32_t Ws;                   // row stride in words (>= W)
  long long m;
  const int32_t* rp;
  const int32_t* col;
  const int32_t* ip;
  const int32_t* isrc;
  const int32_t* pcv;           // chunks of long in-lists: node
  const int32_t* pck;           //                          chunk index
  int32_t npc;
  u64* vis;                     // [n][W]
  u64* nxt[2];                  // [n][W] new bits per level parity
  u64* planes[kMaxPlanes];      // [n][W] bit b of each source's relative level
  int32_t nplanes;              // planes in use (levels < 2^nplanes)
  u64* touched[2];              // one bit per node with new bits at a level of that
                                //   parity: the frontier of the next level
  u64* vmap;                    // [n] bit w set when word w of the node's vis row may be
                                //   nonzero (set by merges and live seeds; cleared with vis)
  u64* fmap[2];                 // [n] bit w set iff word w of the node's nxt row of
                                //   that parity is nonzero (W <= 64)
  int32_t* cu[2];               // out-edge chunks of big-degree frontier nodes: node
  int32_t* ck[2];               //                                             chunk index
  BatchCtrl* ctrl;
  const u64* act;               // [W] sources still expanding
  int32_t* const* rows;         // [lanes] distance row of each source (device), or null:
  int32_t* row_base;            //   then lane r < emit_k writes row_base + r x row_stride
  long long row_stride;
  int32_t emit_k;               // with a null emission mask: lanes < emit_k are emitted
  const int32_t* base;          // [lanes] level at which each source joined (null: all 0)
  int32_t gated;                // expansion and merge obey ctrl->run (device-driven loop)
  int32_t big_b;                // push: out-degree from which a node's edges go by chunks
  int32_t wide_scan;            // narrow rows: in-list length scanned by the whole wave
  int32_t sparse_words;         // push one edge per lane for nodes with <= this many words
  unsigned* flags;              // [0] the workspace may hold bits (set by the seed, cleared by
                                //   a complete emission), [1] run status: 0 ok, 1 invalid
                                //   source, 2 watchdog (device-ordered calls report it)
};

constexpr int kFlagDirty = 0;
constexpr int kFlagStatus = 1;

struct BatchWs {
  Ctx* ctx = nullptr;
  int n = 0;
  int lanes = 0;
  int Wmax = 0;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  u64* vis = nullptr;
  u64* nxt[2] = {nullptr, nullptr};
  u64* planes[kMaxPlanes] = {};
  int nplanes = 0;              // allocated
  size_t plane_reserve = 0;     // budget set aside for planes not yet allocated
  u64* touched[2] = {nullptr, nullptr};
  u64* fmap[2] = {nullptr, nullptr};
  u64* vmap = nullptr;
  int32_t* cu[2] = {nullptr, nullptr};
  int32_t* ck[2] = {nullptr, nullptr};
  BatchCtrl* ctrl = nullptr;
  u64* act = nullptr;
  u64* emask = nullptr;         // [64] lanes to emit
  int32_t** rows = nullptr;
  int32_t* base = nullptr;
  int32_t* src = nullptr;
  int32_t* lane = nullptr;      // lane of each seeded source
  unsigned* flags = nullptr;    // see BatchArgs::flags
  BatchCtrl* h_ctrl = nullptr;
  // the last work enqueued on the workspace (by a call on any stream); whoever
  // takes it next makes its stream wait for this event first
  hipEvent_t busy = nullptr;
  bool busy_set = false;
};

struct BatchTotals {
  int levels, push_levels, pull_levels, launches;
  u64 edges, source_edges, reached;
  double kernel_ms;
};

dawn_status batch_ws_create(Ctx* ctx, const GraphRec* g, int lanes, BatchWs** out);
dawn_status batch_ensure_planes(BatchWs* w, int need, int W);
// Ws = row stride (the batch's width); W = words the kernels process (<= Ws;
// 0 = Ws).
BatchArgs batch_args(const GraphRec* g, BatchWs* w, int Ws, int W = 0);
BatchLevelSum batch_level_sum(const BatchLevel& l);
// The batched knobs of dawn_params into the kernels' arguments.
void batch_knobs(BatchArgs& a, const dawn_params& p);
dawn_status batch_launch_expand(Ctx* ctx, const BatchArgs& a, bool pull, int L, hipStream_t s);
dawn_status batch_launch_merge(Ctx* ctx, const BatchArgs& a, int L, hipStream_t s);
// mode: kEmitClear | kEmitFromRun | kEmitMarkClean (mssp.hip)
constexpr int kEmitClear = 1;        // remove the emitted lanes' bits from vis and the planes
constexpr int kEmitFromRun = 2;      // plane count and go-ahead from the run state (device)
constexpr int kEmitMarkClean = 4;    // every lane emitted with kEmitClear: workspace is clear
dawn_status batch_launch_emit(Ctx* ctx, const BatchArgs& a, int nplanes_used, const u64* d_emask,
                              int mode, hipStream_t s);
dawn_status batch_launch_zero(Ctx* ctx, u64* p, size_t count, hipStream_t s);
// Clear up to kZeroMax arrays in one launch.
constexpr int kZeroMax = 26;
struct ZeroList {
  u64* p[kZeroMax];
  size_t count[kZeroMax];
  int k;
};
dawn_status batch_launch_zero_list(Ctx* ctx, const ZeroList& z, hipStream_t s);
// Active-lane words passed by value to a kernel.
struct BatchActWords {
  u64 w[64];
  int W;
};
// Set the active words and clear counter slot `slot` (serving, before a level).
dawn_status batch_launch_level_prep(const BatchActWords& act, u64* d_act, BatchCtrl* ctrl, int slot,
                                    hipStream_t s);
// One level's control step of the device-driven loop (see BatchRun).
dawn_status batch_launch_control(const BatchArgs& a, u64* act, int L, const dawn_params& p,
                                 hipStream_t s);
dawn_status batch_launch_seed(Ctx* ctx, const BatchArgs& a, const int32_t* d_src,
                              const int32_t* d_lane, int k, int L, bool live, hipStream_t s);
bool batch_choose_pull(const dawn_params& p, const BatchLevelSum& last, int n, int W);

}  // namespace dawn
