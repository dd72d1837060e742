// Internal declarations of libdawn (host runtime + device helpers).
// Nothing here is part of the C ABI; include/dawn.h is.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dawn.h"

namespace dawn {

// ------------------------------------------------------------------ errors --
dawn_status fail(dawn_status st, const char* fmt, ...);
void clear_error();

#define DAWN_HIP(expr)                                                          \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess)                                                       \
      return ::dawn::fail(DAWN_E_DEVICE, "%s failed: %s (%s:%d)", #expr,       \
                          hipGetErrorString(_e), __FILE__, __LINE__);           \
  } while (0)

#define DAWN_TRY(expr)                  \
  do {                                  \
    dawn_status _s = (expr);            \
    if (_s != DAWN_OK) return _s;       \
  } while (0)

inline uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ------------------------------------------------------------ device data --
typedef unsigned long long u64;

// Software grid barrier state (zeroed once at allocation; self-resetting).
struct GridBarrier {
  unsigned int count;
  unsigned int gen;
  unsigned int abort;         // set when a wait timed out; every later wait returns at once
  unsigned int pad;
};

// Counters of one level step are striped over kStripes cache lines (a
// workgroup adds into stripe blockIdx % kStripes) so that no single line
// takes more than a few hundred atomics per level; readers sum the stripes.
// The L2 performs atomics one cache line at a time, so every stripe owns a
// whole 128-byte line.
constexpr int kStripes = 16;
constexpr int kLine = 128;
constexpr int kClkStripes = 16;        // lines of wall-clock stamps per timed launch
constexpr int kClkWords = kLine / 8;   // u64 per line

constexpr int kPullBig = 512;     // in-degree from which a batched pull splits the in-list
constexpr int kPullChunk = 256;   // in-edges per chunk of a split in-list

// One stripe of a level step's counters.
struct alignas(kLine) SlotStripe {
  unsigned int nf;                      // nodes found at this level
  unsigned int small_count;             // entries appended to this stripe's small-degree sub-queue
  u64 mf;                               // sum of out-degrees of the nodes found
  u64 edges;                            // adjacency entries examined
};

// Counters produced by one level step (ring of three, indexed level % 3).
struct LevelSlot {
  SlotStripe s[kStripes];
  alignas(kLine) unsigned int big_chunks;   // chunks appended to the big-degree queue
};

// Level-loop state shared by every workgroup of a traversal.
struct LevelState {
  int level;                  // last level executed (0 = seeded)
  int cur;                    // which visited bitmap is current (0/1)
  int pull;                   // direction of the last level executed
  int done;                   // 0 running, 1 finished, 2 watchdog
  long long mu;               // out-degree sum of the still-unvisited nodes
  int last_nonempty;          // last level that found a node
  int push_levels, pull_levels;
  int launches;               // launches that found the state unfinished (ran levels or
                              //   found the end)
  unsigned prev_nf;           // nodes found by the level before the last
  unsigned mbar;              // arrivals counted so far by the multi-workgroup level barrier
  u64 edges_total;
  u64 source_edges;
  u64 reached;
};

// Coherent host memory a direct-launch traversal reports to, so the host
// learns of the end without a stream synchronisation.  The launch that finds
// the end stores its state in st[parity] and the GPU wall clock in t_end,
// then (after a system-scope fence) end_tag = (seq << 1) | parity, seq being
// the traversal's number (never 0).  Launches that only carry a finished
// state forward write nothing here.  t_start is the init kernel's start.
struct HostMirror {
  LevelState st[2];
  unsigned long long t_start;
  unsigned long long t_end;
  unsigned end_tag;
};

// st[p]: the state after the level run by the last launch of parity p (the
// per-level kernels alternate parities, so a launch reads st[p ^ 1] and
// writes st[p] without racing its own readers).
// One stripe of the arrival count of a one-workgroup launch.
struct alignas(kLine) ArriveStripe {
  unsigned n;
};

struct SsspCtrl {
  GridBarrier bar;
  int32_t* dist;              // output rows and source: written by the host (one copy)
  int source;                 //   before the init kernel, so launches and captured
  int pad;                    //   graphs do not depend on them
  LevelSlot slot[3];
  LevelState st[2];
  // the barrier of multi-workgroup launches: arrivals, counted up through a
  // traversal (zeroed by its init kernel)
  alignas(kLine) unsigned mcount;
  // a launch that runs its levels on some of its workgroups only (one or a
  // few): every other workgroup adds one here (stripe blockIdx % kStripes)
  // once it has read the counters it decides from; workgroup 0 waits for all
  // of them before it writes a slot they read, then zeroes the count
  ArriveStripe arrive[kStripes];
};

// Everything a single-source traversal kernel needs (passed by value).
struct SsspArgs {
  int32_t n;
  int32_t nw;                 // 64-bit words in a visited bitmap
  long long m;
  const int32_t* rp;          // CSR row offsets (n+1)
  const int32_t* col;         // CSR targets (m)
  const int32_t* ip;          // CSC column offsets (n+1)
  const int32_t* isrc;        // CSC sources (m)
  const u64* noin;            // bit per node with no in-edge (never reached unless the source)
  u64* vis0;
  u64* vis1;
  int32_t* qs0;               // small-degree queues (level parity 0/1): kStripes
  int32_t* qs1;               //   sub-queues of n entries each
  int32_t* cu0;               // big-degree chunk lists: node of each chunk
  int32_t* cu1;
  int32_t* ck0;               // ... and the chunk's index within the node's row
  int32_t* ck1;
  SsspCtrl* ctrl;
  int32_t* dist;              // filled in by each kernel from ctrl->dist
  int32_t mode;               // 1 push, 2 pull, 3 switch
  float alpha, beta;
  int32_t big_degree;
  int32_t lane_edges;
  int32_t* level_nf;          // per-level discovered counts (lrec entries)
  uint8_t* level_dir;
  int32_t lrec;
  int32_t lds_words;          // pull levels copy the visited bitmap (this many words,
                              //   = nw) into LDS; 0 = read it from global memory
  int32_t medium_edges;       // push levels whose frontier has more out-edges than a small
                              //   level and at most this many run on the first
  int32_t medium_groups;      //   medium_groups workgroups of a launch, one after another
                              //   with a barrier between them (0: never)
  int32_t small_edges;        // a push level whose frontier has at most this many out-edges
                              //   runs on one workgroup, with the small levels after it in
                              //   the same launch (0: never)
  HostMirror* hm;             // host-mapped report of the traversal (device address of a
                              //   coherent host allocation); null: none
  unsigned seq;               // this traversal's number in hm->end_tag (direct launches)
  unsigned long long* clk;    // timing mode: this launch's kClkStripes lines; in line s,
                              //   [0] the earliest start and [1] the latest end (GPU wall
                              //   clock) of the workgroups b with b % kClkStripes = s;
                              //   null otherwise
};

// ----------------------------------------------------------- host objects --
struct Ctx;
struct GraphRec;

// Device memory accounted against the context's budget.  Budget can be set
// aside with dev_reserve; an allocation `from_reserve` draws on it.
dawn_status dev_alloc(Ctx* ctx, void** p, size_t bytes, bool from_reserve = false);
dawn_status dev_reserve(Ctx* ctx, size_t bytes);
void dev_unreserve(Ctx* ctx, size_t bytes);
void dev_free(Ctx* ctx, void* p, size_t bytes);

template <class T>
dawn_status dev_alloc_n(Ctx* ctx, T** p, size_t count) {
  return dev_alloc(ctx, (void**)p, count * sizeof(T));
}

// Per-call buffers of a single-source traversal (pooled per graph).
struct SsspWs {
  Ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  u64* vis[2] = {nullptr, nullptr};
  int32_t* qs[2] = {nullptr, nullptr};
  int32_t* cu[2] = {nullptr, nullptr};
  int32_t* ck[2] = {nullptr, nullptr};
  SsspCtrl* ctrl = nullptr;
  int32_t* dist = nullptr;      // internal output for host-destination calls
  int32_t* level_nf = nullptr;
  uint8_t* level_dir = nullptr;
  unsigned long long* clk = nullptr;   // timing mode: wall-clock stamps of the level launches
  int32_t clk_cap = 0;                 //   (allocated on first use, clk_cap launches)
  int32_t lrec = 0;
  bool poisoned = false;        // a launch failed: never reuse these buffers
  size_t chunk_cap = 0;
  size_t bytes = 0;
  SsspCtrl* h_ctrl = nullptr;   // pinned read-back
  HostMirror* h_m = nullptr;    // coherent host memory the level launches report to
  HostMirror* d_m = nullptr;    //   ... and its device address
  unsigned seq = 0;             // number of the last direct-launch traversal
  // launch shape of the level kernel on this graph, per block size (256, 512,
  // 1024) and variant (without, with medium levels), found on first use:
  // grid, dynamic LDS, bitmap words copied to LDS
  int shape_grid[6] = {0, 0, 0, 0, 0, 0};
  size_t shape_lds[6] = {0, 0, 0, 0, 0, 0};
  int32_t shape_words[6] = {0, 0, 0, 0, 0, 0};
  // HIP graph driver cache: init + levels, and levels alone for long runs
  hipGraphExec_t gexec = nullptr;
  hipGraphExec_t gexec_more = nullptr;
  int gexec_levels = 0;
  int gexec_block = 0;
  SsspArgs gexec_args{};        // launch arguments baked into the captured graph
  ~SsspWs();
};

struct BatchWs;   // batched traversal buffers (mssp.hip)
void batch_ws_destroy(BatchWs* ws);

struct GraphRec {
  Ctx* ctx = nullptr;
  int32_t id = -1;
  int32_t n = 0;
  long long m = 0;
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  int32_t* ip = nullptr;
  int32_t* isrc = nullptr;
  u64* noin = nullptr;                    // nodes with no in-edge, one bit each
  bool shared_csc = false;                // symmetric graph: ip/isrc alias rp/col
  std::vector<int32_t> comp_size;         // host copy: nodes in each node's weakly
                                          //   connected component
  // in-lists of at least kPullBig entries cut into chunks of kPullChunk, so
  // that a batched pull scans one long in-list with many waves: node, chunk
  int32_t* pcv = nullptr;
  int32_t* pck = nullptr;
  int32_t npc = 0;
  size_t pc_cap = 0;
  int32_t max_out_deg = 0;
  int32_t zero_out = 0;
  // level launches the recent traversals needed (the direct-launch driver
  // queues about this many before its first host check)
  std::atomic<int> launch_hint{0};
  // batched level loop: levels the last run launched before it saw the end
  // (its expansions + 1), the size of the next run's first chunk
  mutable std::atomic<int> batch_hint{0};
  size_t bytes = 0;
  dawn_params params{};
  std::mutex mu;                          // guards the pools and the WCC cache
  std::vector<std::unique_ptr<SsspWs>> sssp_pool;
  std::vector<BatchWs*> batch_pool;
  // weighted graphs (dawn_graph_set_weights): weight of each CSR entry
  int32_t* wt = nullptr;
  int32_t max_w = 0;
  std::atomic<int> wsssp_hint{0};         // rounds the last weighted run needed
  void* wpool = nullptr;                  // pooled weighted-run workspaces (wsssp.hip)
  // device staging of host-destination batched rows, kept between calls
  int32_t* stage = nullptr;
  size_t stage_bytes = 0;
  // largest-WCC cache (apsp_wcc)
  bool wcc_ready = false;
  std::vector<int32_t> wcc_nodes;
  std::shared_ptr<GraphRec> wcc_sub;      // induced subgraph on the WCC, ids renumbered
  ~GraphRec();
};

struct Server;   // serving scheduler (serve.cpp)
void server_stop(Server* s);

struct Ctx {
  int device = 0;
  int num_cu = 0;
  int coop = 0;
  int wall_khz = 0;                        // the GPU wall clock's rate (timing mode)
  size_t lds_per_block = 0;                // LDS bytes a workgroup may use
  uint64_t budget = 0;
  std::atomic<uint64_t> used{0};
  std::atomic<uint64_t> reserved{0};       // budget set aside (serving engines' level planes)
  std::atomic<long long> fail_after{-1};   // failure injection: allocations left before failing
  std::atomic<long long> fail_plane_after{-1};   // ... level-plane allocations left before failing
  std::mutex mu;
  std::mutex budget_mu;
  std::map<int32_t, std::shared_ptr<GraphRec>> graphs;
  int32_t next_graph = 0;
  Server* server = nullptr;
  std::mutex server_mu;
};

dawn_status get_graph(Ctx* ctx, int32_t id, std::shared_ptr<GraphRec>* out);
dawn_params default_params(const GraphRec& g);
dawn_status check_params(const dawn_params& p);

// graph.hip
dawn_status graph_build(Ctx* ctx, GraphRec* g, const int32_t* h_rp, const int32_t* h_col);
dawn_status graph_wcc(Ctx* ctx, GraphRec* g, hipStream_t stream);

// sssp.hip
dawn_status sssp_run(Ctx* ctx, GraphRec* g, const dawn_params& p, int32_t source,
                     int32_t* dist, bool device_out, dawn_run_stats* stats);
// The no-allocation variant: buffers from the file-scope scratch array of
// sssp.hip, whose per-device address scratch_init (device current) looks up.
dawn_status scratch_init(int device);
dawn_status sssp_run_noalloc(Ctx* ctx, GraphRec* g, const dawn_params& p, int32_t source,
                             int32_t* d_dist, hipStream_t s, dawn_run_stats* stats);

// wsssp.hip: the (min, +) level loop over a weighted graph
dawn_status wsssp_run(Ctx* ctx, GraphRec* g, int32_t source, int32_t* dist, bool device_out,
                      dawn_run_stats* stats);
void wsssp_pool_free(GraphRec* g);

// mssp.hip
dawn_status mssp_run(Ctx* ctx, GraphRec* g, const dawn_params& p, const int32_t* sources,
                     int32_t k, int32_t* dist, bool device_out, int64_t row_stride,
                     dawn_run_stats* stats);
// Everything queued on stream s: sources and rows are device memory.
dawn_status mssp_device_run(Ctx* ctx, GraphRec* g, const dawn_params& p, const int32_t* d_src,
                            int32_t k, int32_t* d_dist, int32_t* d_status, hipStream_t s);

// tune.cpp
dawn_status autotune(Ctx* ctx, GraphRec* g, const int32_t* sources, int32_t k, uint32_t what,
                     dawn_params* best);

// serve.cpp
dawn_status serve_submit(Ctx* ctx, int32_t graph, const int32_t* sources, int32_t k,
                         int32_t* dist_out, uint32_t flags, uint64_t* ticket);
dawn_status serve_poll(Ctx* ctx, uint64_t ticket, int32_t timeout_ms, dawn_query_stats* qs);

}  // namespace dawn
