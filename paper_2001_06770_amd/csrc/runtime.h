// runtime.h -- host-side state of the RAKS library: the context (graph,
// allocator) and its lanes (per-query workspaces, each with its own HIP
// stream), plus the serving queue.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/raks.h"
#include "common.h"
#include "kernels.h"

namespace raks {

constexpr int kTimers = 5;
constexpr size_t kSpecNodes = 1 << 16;   // output read back with the headers
constexpr size_t kSpecArcs = 1 << 16;
constexpr int kMaxLanes = 64;
constexpr int kMaxViews = 4;       // cached activation views for per-query alphas

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;   // a slice of the allocation-free scratch: never freed
};

template <typename T>
T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

struct Ctx;

// Activation levels for one alpha (Section 3.1, Eqs. 1-3): per-arc levels in
// CSR order, per-node levels (NODE mode), and the traversal copy of the graph
// with every row sorted by level (col_s, act_s, eid_s, row_amax, level
// table).  The context's own alpha has one; queries with another alpha use
// cached ones.
struct AlphaView {
  double alpha = 0;
  DevBuf act, act_node, col_s, act_s, eid_s, row_amax, bnd;
  int refs = 0;           // queries using it
  uint64_t last_use = 0;
};

// Recovery capacities of one phase (Algorithm 2 over CGs, or over RPGs plus
// the output): per instance node / arc list capacities and the kind of node
// set, the per-layer work-list capacity, and the derived layout uploaded to
// the device (InstCap table, CG list offsets, sort scratch offsets).
struct RecPhase {
  int32_t n_inst = 0, n_res = 0, T = 0;
  bool grown = false;                 // capacities differ from the defaults
  std::vector<uint32_t> ncap, acap;
  std::vector<uint8_t> dense;
  uint32_t lcap = 0;
  // derived
  std::vector<InstCap> caps;
  std::vector<uint64_t> cg_noff, cg_aoff, soff;   // [n_res + 1]
  uint64_t h_words = 0, n_total = 0, a_total = 0;
  uint64_t cg_nmax = 0, cg_amax = 0;              // largest CG lists (phase 0)
  uint64_t out_n = 0, out_a = 0;                  // output bound (phase 1)
  bool dirty = true;                              // layout not uploaded yet
  DevBuf layout;                                  // caps | cg_noff | cg_aoff | soff
  size_t lay_cg_noff = 0, lay_cg_aoff = 0, lay_soff = 0;
  void* stage = nullptr;                          // pinned staging of the layout
  size_t stage_bytes = 0;
  DevBuf cnt, iflag, lcnt;                        // device counters of the phase
  // labelled mode (one search per keyword column for all results): chosen
  // after a first attempt found large or overflowing instances
  bool labelled = false;
  uint32_t tcap = 0;                              // capacity of the labelled-node list
  DevBuf touch, tcnt;
};

// Everything one query needs besides the graph.  A lane runs one query at a
// time on its own stream.
struct Lane {
  Ctx* ctx = nullptr;
  int id = 0;
  hipStream_t stream = nullptr;
  const AlphaView* view = nullptr;   // activation levels of the current query
  bool own_stream = false;
  bool no_alloc = false;   // the allocation-free lane: no event timing, buffers from scratch

  int32_t n_pad = 0, nblocks = 0, cpw = 1;
  DevBuf Hc, Hm, R, tot, sb, q_off, q_rs, q_lo, q_mask, tile_first, cand, s_item, s_cand;
  DevBuf sel_node, sel_sc, sel_sumh, has_rpg, sm, key, dmin, ranked;
  DevBuf vc_cnt, vc_tmp, vc_off, vc_nodes;
  // recovery storage, shared by both phases (sized for the larger one)
  DevBuf hpool, nl, al, items, sort_a, sort_b;
  DevBuf cg_nodes, cg_arcs, cg_cnt;   // CG lists, kept for the marginal phase
  DevBuf hdr, out_nodes, out_arcs, status;
  DevBuf Hq;                          // cohort path: the query's hitting levels, [n_pad][TPq]
  DevBuf bigf, big_bm, big_chunk, big_slot;   // bitmap path of large results
  RecPhase ph[2];                     // [0] CG recovery, [1] RPG recovery + output
  DevBuf lab;                         // labels of the labelled mode, [T * G][n] words
  bool lab_dirty = true;              // lab may hold non-zero words
  Status* h_status = nullptr;   // pinned
  RunStatus* h_run = nullptr;   // pinned [2]: per-level status, double-buffered
  uint64_t ctl_seq = 0;         // control launches so far (stamps of h_run)
  RunStatus* d_run = nullptr;   // the same memory as the device addresses it
  ResultHdr* h_hdr = nullptr;   // pinned [kMaxW]
  int32_t* h_nodes = nullptr;   // pinned [kSpecNodes]
  int32_t* h_arcs = nullptr;    // pinned [3 * kSpecArcs]
  void* xfer = nullptr;         // pinned staging of outputs beyond the buffers above (grown)
  size_t xfer_bytes = 0;
  // device addresses of the pinned buffers above (results are written there
  // by a kernel)
  Status* d_status = nullptr;
  ResultHdr* d_hdr = nullptr;
  uint32_t* d_nodes = nullptr;
  uint32_t* d_arcs = nullptr;
  hipEvent_t q_start = nullptr, q_end = nullptr;

  // event timing (enabled by the context)
  struct Pending { hipEvent_t a, b; int kind; double bytes; int level, run; };
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<Pending> pending;
};

struct Job {
  uint64_t ticket = 0;
  std::vector<int32_t> central, marginal;
  raks_query_desc desc = {};
  raks_results* res = nullptr;
  int rc = 0;
  std::string err;
  bool done = false;
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct ServeState {
  bool running = false;
  bool stop = false;
  int32_t queue_cap = 0;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, Job*> jobs;
  uint64_t next_ticket = 1;
  int in_flight = 0;
  bool cohort = false;   // served by the cohort engine (else one worker per lane)
};

struct Ctx {
  int device = 0;
  int num_cu = 256;
  raks_alloc_fn alloc = nullptr;
  raks_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  uint64_t budget = 0;
  uint64_t in_use = 0;
  std::mutex mem_mu;
  hipStream_t user_stream = nullptr;
  uint32_t rec_nc0 = 4096, rec_ac0 = 16384, rec_lcap0 = 1u << 16;   // initial recovery capacities
  uint64_t big_list = 1u << 20;   // results with longer lists are merged through bitmaps

  // graph
  bool loaded = false;
  int32_t n = 0;
  uint32_t A = 0;
  int32_t vocab = 0;
  int32_t mode = 0;
  double abar = 0, alpha = 0;
  DevBuf row_ptr, col, label, nw, kw_nodes, arc_src;
  // internal (degree-ordered) node numbering: original row starts, both id maps
  DevBuf row_ptr_o, orig_id, int_id, node_tmp;
  DevBuf rev;            // CSR position of every arc's reverse arc
  DevBuf cweight;        // EDGE: label count c of every arc, kept for other alphas
  DevBuf wstat;          // Status holding the c (or node weight) range of the graph
  uint64_t wmin = 0, wmax = 0;   // the same range on the host
  DevBuf lut;            // levels of every c (or node weight) in the range, for one alpha
  int32_t nbnd = 1;
  AlphaView base;        // levels for the context's alpha
  std::vector<std::unique_ptr<AlphaView>> views;   // other alphas, least recently used evicted
  std::mutex view_mu;
  uint64_t view_clock = 0;
  std::vector<int64_t> kw_ptr;

  std::vector<std::unique_ptr<Lane>> lanes;
  std::unique_ptr<Lane> na_lane;   // the lane of raks_query_noalloc (made at raks_create)
  void* na_scratch = nullptr;      // that lane's device scratch (the device's static array)
  size_t na_scratch_bytes = 0;
  // batches and serving: 0 = cohort engine (many queries in one level loop),
  // 1 = independent single-query runs on the lanes
  int32_t batch_mode = 0;
  void* engine = nullptr;   // the cohort engine (engine.hip), created on first use
  // cohort tuning: expansion workgroups per CU; a batch admits new queries
  // only while at most admit_below queries of the cohort are exploring
  int32_t co_wpc = 8, co_admit_below = 32, co_tile = 1024, co_cols = 64;

  // timing
  std::atomic<uint32_t> timing{0};   // bit k: timer k is recorded
  std::mutex timing_mu;
  raks_kernel_timing acc[kTimers] = {};

  ServeState serve;
};

}  // namespace raks
