// api.hip -- host runtime and C ABI of the RAKS gfx950 library.
//
// A query runs both runs of the unified framework (Section 4.1) on one HIP
// stream:
//   central run   level loop (scan / control / enqueue / expand) until >= w
//                 CGs, the level bound or an empty frontier; top-w selection;
//   recovery      Algorithm 2 for every (CG, central keyword); union, sort,
//                 V_C per CG;
//   marginal run  level loop with the RPG check over V_C and Theorem 4;
//   ranking       Eq. 6 order, top-k;
//   recovery      Algorithm 2 for every (RPG, marginal keyword) from the V_C
//                 nodes at distance D_j; union with the CG; output.
// Only the small per-level status (a few dozen bytes) and the final results
// cross to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/raks.h"
#include "common.h"
#include "kernels.h"

using namespace raks;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(RAKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

#define RAKS_TRY(expr)          \
  do {                          \
    int _rc = (expr);           \
    if (_rc != RAKS_OK) return _rc; \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

constexpr int kTimers = 5;
constexpr size_t kSpecNodes = 1 << 16;   // output read back with the headers
constexpr size_t kSpecArcs = 1 << 16;

}  // namespace

struct raks_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  raks_alloc_fn alloc = nullptr;
  raks_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  uint64_t budget = 0;
  uint64_t in_use = 0;
  int num_cu = 256;

  // graph
  bool loaded = false;
  int32_t n = 0;
  uint32_t A = 0;
  int32_t vocab = 0;
  int32_t mode = 0;
  double abar = 0, alpha = 0;
  DevBuf row_ptr, col, label, act, act_node, nw, kw_nodes, col_s, act_s, eid_s, row_amax, bnd, arc_src;
  int32_t nbnd = 1;
  std::vector<int64_t> kw_ptr;

  // workspace
  int32_t n_pad = 0, nblocks = 0;
  DevBuf Hc, Hm, F, tot, off, q_off, q_rs, q_lo, q_mask, cand;
  DevBuf sel_node, sel_sc, sel_sumh, has_rpg, sm, key, dmin, ranked;
  DevBuf vc_cnt, vc_tmp, vc_off, vc_nodes;
  DevBuf ht, nl, al, icnt, cg_nodes, cg_arcs, cg_cnt, sort_a, sort_b, items, lcnt;
  DevBuf hdr, out_nodes, out_arcs;
  DevBuf status;
  Status* h_status = nullptr;   // pinned
  RunStatus* h_run = nullptr;   // pinned [2]: per-level status, double-buffered
  ResultHdr* h_hdr = nullptr;   // pinned [kMaxW]
  int32_t* h_nodes = nullptr;   // pinned [kSpecNodes]
  int32_t* h_arcs = nullptr;    // pinned [3 * kSpecArcs]
  hipEvent_t lvl_ev[2] = {nullptr, nullptr};
  uint32_t nc = 4096, ac = 16384;  // recovery capacities per instance
  uint32_t lcap = 1u << 16;        // recovery work chunks per layer

  // timing
  bool timing = false;
  raks_kernel_timing acc[kTimers] = {};
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Pending { hipEvent_t a, b; int kind; double bytes; int level, run; };
  std::vector<Pending> pending;
  hipEvent_t q_start = nullptr, q_end = nullptr;
};

namespace {

int dev_alloc(raks_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return RAKS_OK;
  if (b.p) {
    if (c->free_fn) c->free_fn(b.p, b.bytes, c->alloc_user);
    else (void)hipFree(b.p);
    c->in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  if (c->budget && c->in_use + bytes > c->budget)
    return fail(RAKS_ENOMEM, "device memory budget exceeded");
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->alloc_user);
    if (!p) return fail(RAKS_ENOMEM, "device allocator returned NULL");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(RAKS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.p = p;
  b.bytes = bytes;
  c->in_use += bytes;
  return RAKS_OK;
}

void dev_free(raks_ctx* c, DevBuf& b) {
  if (!b.p) return;
  if (c->free_fn) c->free_fn(b.p, b.bytes, c->alloc_user);
  else (void)hipFree(b.p);
  c->in_use -= b.bytes;
  b = DevBuf();
}

template <typename T>
T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

int tp_for(int T) { return T <= 4 ? 4 : (T <= 8 ? 8 : 16); }

DevGraphView graph_view(raks_ctx* c) {
  DevGraphView g;
  g.n = c->n;
  g.A = c->A;
  g.row_ptr = P<uint32_t>(c->row_ptr);
  g.col = P<int32_t>(c->col);
  g.label = P<uint16_t>(c->label);
  g.act = P<uint8_t>(c->act);
  g.act_node = c->mode ? P<uint8_t>(c->act_node) : nullptr;
  g.mode = c->mode;
  g.col_s = P<int32_t>(c->col_s);
  g.act_s = P<uint8_t>(c->act_s);
  g.row_amax = P<uint8_t>(c->row_amax);
  g.eid_s = P<uint32_t>(c->eid_s);
  g.arc_src = P<int32_t>(c->arc_src);
  g.bnd = P<uint32_t>(c->bnd);
  g.nbnd = c->nbnd;
  return g;
}

// ------------------------------------------------------------ timing ---
hipEvent_t next_event(raks_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

struct Timed {
  raks_ctx* c;
  int kind;
  double bytes;
  int level, run;
  hipEvent_t a = nullptr;
  Timed(raks_ctx* c_, int kind_, double bytes_ = 0, int level_ = -1, int run_ = -1)
      : c(c_), kind(kind_), bytes(bytes_), level(level_), run(run_) {
    if (c->timing) {
      a = next_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timed() {
    if (c->timing && a) {
      hipEvent_t b = next_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->pending.push_back({a, b, kind, bytes, level, run});
      }
    }
  }
};

void harvest_timing(raks_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0;
    if (p.kind < 0) continue;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->acc[p.kind].launches += 1;
      c->acc[p.kind].ms += ms;
      c->acc[p.kind].bytes += p.bytes;
    }
  }
  c->pending.clear();
  c->ev_used = 0;
}

// -------------------------------------------------------------- graph ---

int compute_activation(raks_ctx* c) {
  DevGraphView g = graph_view(c);
  Status* st = P<Status>(c->status);
  RAKS_TRY(dev_alloc(c, c->arc_src, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  if (c->mode == RAKS_ACT_EDGE) {
    DevBuf ctmp;
    RAKS_TRY(dev_alloc(c, ctmp, (size_t)std::max<uint32_t>(c->A, 1) * 4));
    launch_check_and_count(g, P<uint32_t>(ctmp), P<int32_t>(c->arc_src), st, c->stream);
    HIP_OK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (c->h_status->err) {
      dev_free(c, ctmp);
      char msg[160];
      snprintf(msg, sizeof msg,
               "graph violates the input contract (bits 0x%x: 1 col range, 2 self-loop, "
               "4 row order, 8 missing reverse arc)", c->h_status->err);
      return fail(RAKS_EINVAL, msg);
    }
    launch_act_edge(g, P<uint32_t>(ctmp), st, c->abar, c->alpha, P<uint8_t>(c->act), c->stream);
    HIP_OK(hipStreamSynchronize(c->stream));
    dev_free(c, ctmp);
  } else {
    DevBuf ctmp;
    RAKS_TRY(dev_alloc(c, ctmp, (size_t)std::max<uint32_t>(c->A, 1) * 4));
    launch_check_and_count(g, P<uint32_t>(ctmp), P<int32_t>(c->arc_src), st, c->stream);
    HIP_OK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    dev_free(c, ctmp);
    if (c->h_status->err)
      return fail(RAKS_EINVAL, "graph violates the input contract");
    launch_act_node(g, P<uint8_t>(c->nw), st, c->abar, c->alpha, P<uint8_t>(c->act_node),
                    P<uint8_t>(c->act), c->stream);
    HIP_OK(hipStreamSynchronize(c->stream));
  }
  // traversal copy sorted by activation level within each row
  RAKS_TRY(dev_alloc(c, c->col_s, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->act_s, (size_t)std::max<uint32_t>(c->A, 1)));
  RAKS_TRY(dev_alloc(c, c->eid_s, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->row_amax, (size_t)c->n));
  // levels never exceed Round(2 * a_bar) (x <= 1 in Eqs. 1-3)
  c->nbnd = (int32_t)std::min(16.0, std::floor(2.0 * c->abar + 0.5) + 1.0);
  RAKS_TRY(dev_alloc(c, c->bnd, (size_t)c->n * c->nbnd * 4));
  g = graph_view(c);
  launch_sort_rows(g, P<int32_t>(c->col_s), P<uint8_t>(c->act_s), P<uint32_t>(c->eid_s),
                   P<uint8_t>(c->row_amax), P<uint32_t>(c->bnd), c->nbnd, c->stream);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(c->stream));
  return RAKS_OK;
}

// ------------------------------------------------------------- query ---

struct QueryPlan {
  int C, M, TPc, TPm, k, w, L, gn, gd;
  std::vector<int32_t> central, marginal;
};

int validate_query(raks_ctx* c, const raks_query_desc* q, QueryPlan& p) {
  if (!q) return fail(RAKS_EINVAL, "query descriptor is NULL");
  p.C = q->n_central;
  p.M = q->n_marginal;
  if (p.C < 1 || p.C > kMaxKw) return fail(RAKS_EINVAL, "need 1..16 central keywords");
  if (p.M < 0 || p.M > kMaxKw) return fail(RAKS_EINVAL, "need 0..16 marginal keywords");
  if (!q->central || (p.M > 0 && !q->marginal)) return fail(RAKS_EINVAL, "keyword array is NULL");
  p.central.assign(q->central, q->central + p.C);
  p.marginal.assign(q->marginal ? q->marginal : q->central, (q->marginal ? q->marginal : q->central) + p.M);
  std::vector<int32_t> all = p.central;
  all.insert(all.end(), p.marginal.begin(), p.marginal.end());
  for (int32_t t : all)
    if (t < 0 || t >= c->vocab) return fail(RAKS_EINVAL, "keyword id out of range");
  std::vector<int32_t> s = all;
  std::sort(s.begin(), s.end());
  if (std::adjacent_find(s.begin(), s.end()) != s.end())
    return fail(RAKS_EINVAL, "duplicate keyword (within or across central/marginal)");
  p.k = q->k;
  p.w = q->w ? q->w : q->k;
  if (p.k < 1 || p.w < p.k || p.w > kMaxW) return fail(RAKS_EINVAL, "need 1 <= k <= w <= 256");
  p.gn = q->gamma_num;
  p.gd = q->gamma_den;
  if (p.gn == 0 && p.gd == 0) { p.gn = 1; p.gd = 2; }
  if (p.gd < 1 || p.gd > 1000000 || p.gn < 0 || p.gn > p.gd)
    return fail(RAKS_EINVAL, "gamma must be gamma_num/gamma_den in [0,1]");
  p.L = q->max_level ? q->max_level : 20;
  if (p.L < 1 || p.L > 250) return fail(RAKS_EINVAL, "max_level must be in 1..250");
  p.TPc = tp_for(p.C);
  p.TPm = tp_for(std::max(p.M, 1));
  return RAKS_OK;
}

int ensure_node_buffers(raks_ctx* c) {
  c->n_pad = (int32_t)(((int64_t)c->n + kScanNodes - 1) / kScanNodes * kScanNodes);
  c->nblocks = c->n_pad / kScanNodes;
  const size_t np = (size_t)c->n_pad;
  RAKS_TRY(dev_alloc(c, c->F, np));
  RAKS_TRY(dev_alloc(c, c->tot, (size_t)c->nblocks * sizeof(ScanTot)));
  RAKS_TRY(dev_alloc(c, c->off, (size_t)c->nblocks * sizeof(ScanOff)));
  RAKS_TRY(dev_alloc(c, c->q_off, (np + 1) * 4));
  RAKS_TRY(dev_alloc(c, c->q_rs, np * 4));
  RAKS_TRY(dev_alloc(c, c->q_lo, np * 4));
  RAKS_TRY(dev_alloc(c, c->q_mask, np * 4));
  RAKS_TRY(dev_alloc(c, c->cand, np * 8));
  RAKS_TRY(dev_alloc(c, c->sel_node, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->sel_sc, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->sel_sumh, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->has_rpg, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->sm, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->key, kMaxW * 8));
  RAKS_TRY(dev_alloc(c, c->dmin, kMaxW * kMaxKw));
  RAKS_TRY(dev_alloc(c, c->ranked, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->vc_cnt, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, c->vc_off, (kMaxW + 1) * 4));
  return RAKS_OK;
}

SeedList seeds_for(raks_ctx* c, const std::vector<int32_t>& kws) {
  SeedList s = {};
  s.T = (int32_t)kws.size();
  uint32_t acc = 0;
  for (int i = 0; i < s.T; ++i) {
    s.start[i] = (uint32_t)c->kw_ptr[kws[i]];
    s.count[i] = (uint32_t)(c->kw_ptr[kws[i] + 1] - c->kw_ptr[kws[i]]);
    s.prefix[i] = acc;
    acc += s.count[i];
  }
  s.prefix[s.T] = acc;
  return s;
}

RunView run_view(raks_ctx* c, int kind, int T, DevBuf& H, const QueryPlan& p) {
  RunView r = {};
  r.kind = kind;
  r.T = T;
  r.tmask = (T >= 32) ? 0xFFFFFFFFu : ((1u << T) - 1);
  r.block_rule = (kind == RUN_CENTRAL) ? 1 : (T >= 2 ? 1 : 0);
  r.H = P<uint8_t>(H);
  r.F = P<uint8_t>(c->F);
  r.n_pad = c->n_pad;
  r.st = &P<Status>(c->status)->run[kind];
  r.tot = P<ScanTot>(c->tot);
  r.off = P<ScanOff>(c->off);
  r.nblocks = c->nblocks;
  r.q_lo = P<uint32_t>(c->q_lo);
  r.q_off = P<uint32_t>(c->q_off);
  r.q_rs = P<uint32_t>(c->q_rs);
  r.q_mask = P<uint32_t>(c->q_mask);
  r.cand = P<uint64_t>(c->cand);
  r.max_level = p.L;
  r.w = p.w;
  r.k = p.k;
  r.gamma_num = p.gn;
  r.gamma_den = p.gd;
  r.nsel = &P<Status>(c->status)->nsel;
  r.sel_sc = P<int32_t>(c->sel_sc);
  r.vc_off = P<uint32_t>(c->vc_off);
  r.vc_nodes = P<int32_t>(c->vc_nodes);
  r.has_rpg = P<int32_t>(c->has_rpg);
  r.sm = P<int32_t>(c->sm);
  r.key = P<int64_t>(c->key);
  r.dmin = P<uint8_t>(c->dmin);
  return r;
}

__global__ void k_query_reset(Status* st) {
  st->nsel = 0;
  st->nres = 0;
  st->overflow = 0;
  st->out_nodes = 0;
  st->out_arcs = 0;
}

// One exploration run: the level loop of Figure 3.  The host enqueues level
// l+1 before it waits for the status of level l, so the GPU never idles on
// the host's decision; the kernels of a level after the run's end return at
// once.  Returns the run's final status in *last.
int run_levels(raks_ctx* c, RunView& r, int TP, const std::vector<int32_t>& kws, int T,
               RunStatus* last) {
  DevGraphView g = graph_view(c);
  const SeedList seeds = seeds_for(c, kws);
  {
    Timed t(c, 4);
    launch_run_init(r, TP, c->n, P<int32_t>(c->kw_nodes), seeds, c->stream);
  }
  const int grid = c->num_cu * 8;
  auto enqueue = [&](int level, int slot) -> int {
    {
      Timed t(c, 1, 0, level, r.kind);
      launch_front_count(r, TP, g, level, c->stream);
    }
    {
      Timed t(c, 2, 0, level, r.kind);
      launch_front_control(r, TP, level, c->stream);
    }
    {
      Timed t(c, 1, 0, level, r.kind);
      launch_front_write(r, TP, g, level, c->stream);
    }
    {
      Timed t(c, 0, 0, level, r.kind);
      launch_expand(r, TP, g, level, grid, c->stream);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(&c->h_run[slot], r.st, sizeof(RunStatus), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipEventRecord(c->lvl_ev[slot], c->stream));
    return RAKS_OK;
  };
  RAKS_TRY(enqueue(0, 0));
  for (int level = 0;; ++level) {
    const int slot = level & 1;
    if (level + 1 <= r.max_level) RAKS_TRY(enqueue(level + 1, slot ^ 1));
    HIP_OK(hipEventSynchronize(c->lvl_ev[slot]));
    const RunStatus s = c->h_run[slot];
    if (c->timing) {
      for (auto& pe : c->pending) {
        if (pe.kind != 0 || pe.level != level || pe.run != r.kind) continue;
        if (s.end_level == INT32_MAX) {
          // algorithmic bytes of this expansion: per examined arc the neighbour
          // id (4) and its T hitting levels; per queue entry 16
          pe.bytes = (4.0 + T) * s.W + 16.0 * s.nactive;
        } else {
          pe.kind = -1;   // the level ended before expanding: no work launched
        }
      }
    }
    if (s.end_level != INT32_MAX || level >= r.max_level) {
      *last = s;
      break;
    }
  }
  return RAKS_OK;
}

int ensure_recovery(raks_ctx* c, int n_inst, int n_cg, int C, int M, int n_res, int max_level) {
  const uint32_t hc = [&] { uint32_t h = 1; while (h < 2 * c->nc) h <<= 1; return h; }();
  RAKS_TRY(dev_alloc(c, c->ht, (size_t)std::max(n_inst, 1) * hc * 4));
  RAKS_TRY(dev_alloc(c, c->nl, (size_t)std::max(n_inst, 1) * c->nc * 4));
  RAKS_TRY(dev_alloc(c, c->al, (size_t)std::max(n_inst, 1) * c->ac * 4));
  RAKS_TRY(dev_alloc(c, c->icnt, (size_t)std::max(n_inst, 1) * 8));
  RAKS_TRY(dev_alloc(c, c->items, (size_t)(max_level + 1) * c->lcap * sizeof(RecItem)));
  RAKS_TRY(dev_alloc(c, c->lcnt, (size_t)(max_level + 1) * 4));
  const size_t cg_ncap = (size_t)C * c->nc, cg_acap = (size_t)C * c->ac;
  RAKS_TRY(dev_alloc(c, c->cg_nodes, (size_t)std::max(n_cg, 1) * cg_ncap * 4));
  RAKS_TRY(dev_alloc(c, c->cg_arcs, (size_t)std::max(n_cg, 1) * cg_acap * 4));
  RAKS_TRY(dev_alloc(c, c->cg_cnt, (size_t)std::max(n_cg, 1) * 8));
  RAKS_TRY(dev_alloc(c, c->vc_tmp, (size_t)std::max(n_cg, 1) * cg_ncap * 4));
  RAKS_TRY(dev_alloc(c, c->vc_nodes, (size_t)std::max(n_cg, 1) * cg_ncap * 4));
  const size_t scap = std::max({cg_acap, cg_ncap + (size_t)M * c->nc, cg_acap + (size_t)M * c->ac});
  const int nw = std::max(n_cg, n_res);
  RAKS_TRY(dev_alloc(c, c->sort_a, (size_t)std::max(nw, 1) * scap * 4));
  RAKS_TRY(dev_alloc(c, c->sort_b, (size_t)std::max(nw, 1) * scap * 4));
  const size_t ncap = (size_t)n_res * ((size_t)C * c->nc + (size_t)M * c->nc);
  const size_t acap = (size_t)n_res * ((size_t)C * c->ac + (size_t)M * c->ac);
  RAKS_TRY(dev_alloc(c, c->hdr, (size_t)std::max(n_res, 1) * sizeof(ResultHdr)));
  RAKS_TRY(dev_alloc(c, c->out_nodes, std::max<size_t>(ncap, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->out_arcs, std::max<size_t>(acap, 1) * 12));
  return RAKS_OK;
}

RecoverView recover_view(raks_ctx* c, int marginal, DevBuf& H, int TP, int T, int n_inst,
                         const int32_t* n_valid, int max_layer) {
  RecoverView v = {};
  v.items = P<RecItem>(c->items);
  v.lcnt = P<uint32_t>(c->lcnt);
  v.lcap = c->lcap;
  v.max_layer = max_layer;
  v.g = graph_view(c);
  v.H = P<uint8_t>(H);
  v.TP = TP;
  v.T = T;
  v.marginal = marginal;
  v.n_inst = n_inst;
  v.n_valid = n_valid;
  v.sel_node = P<int32_t>(c->sel_node);
  v.ranked = P<int32_t>(c->ranked);
  v.vc_off = P<uint32_t>(c->vc_off);
  v.vc_nodes = P<int32_t>(c->vc_nodes);
  v.dmin = P<uint8_t>(c->dmin);
  v.ht = P<uint32_t>(c->ht);
  v.nl = P<int32_t>(c->nl);
  v.al = P<uint32_t>(c->al);
  v.cnt = P<uint32_t>(c->icnt);
  uint32_t hc = 1;
  while (hc < 2 * c->nc) hc <<= 1;
  v.hc = hc;
  v.nc = c->nc;
  v.ac = c->ac;
  v.gst = P<Status>(c->status);
  return v;
}

FinalizeView finalize_view(raks_ctx* c, int marginal, int T, int n_res, const int32_t* n_valid,
                           int C, int TPc, int M) {
  FinalizeView v = {};
  v.g = graph_view(c);
  v.T = T;
  v.marginal = marginal;
  v.n_res = n_res;
  v.n_valid = n_valid;
  v.sel_node = P<int32_t>(c->sel_node);
  v.ranked = P<int32_t>(c->ranked);
  v.nl = P<int32_t>(c->nl);
  v.al = P<uint32_t>(c->al);
  v.cnt = P<uint32_t>(c->icnt);
  v.nc = c->nc;
  v.ac = c->ac;
  v.cg_nodes = P<uint32_t>(c->cg_nodes);
  v.cg_arcs = P<uint32_t>(c->cg_arcs);
  v.cg_cnt = P<uint32_t>(c->cg_cnt);
  v.cg_ncap = (uint32_t)C * c->nc;
  v.cg_acap = (uint32_t)C * c->ac;
  v.Hc = P<uint8_t>(c->Hc);
  v.TPc = TPc;
  v.Tc = C;
  v.vc_cnt = P<uint32_t>(c->vc_cnt);
  v.vc_tmp = P<int32_t>(c->vc_tmp);
  v.sort_a = P<uint32_t>(c->sort_a);
  v.sort_b = P<uint32_t>(c->sort_b);
  v.scap = (uint32_t)std::max({(size_t)v.cg_acap, (size_t)v.cg_ncap + (size_t)M * c->nc,
                               (size_t)v.cg_acap + (size_t)M * c->ac});
  v.write_output = marginal;
  v.hdr = P<ResultHdr>(c->hdr);
  v.out_nodes = P<int32_t>(c->out_nodes);
  v.out_arcs = P<int32_t>(c->out_arcs);
  v.sel_sc = P<int32_t>(c->sel_sc);
  v.sm = P<int32_t>(c->sm);
  v.key = P<int64_t>(c->key);
  v.gst = P<Status>(c->status);
  return v;
}

// One attempt at a query with the current recovery capacities; *overflow is
// set when a capacity ran out (the caller grows them and repeats).
int query_attempt(raks_ctx* c, const QueryPlan& p, raks_results** out, bool* overflow) {
  *overflow = false;
  Status* st = P<Status>(c->status);
  HIP_OK(hipEventRecord(c->q_start, c->stream));
  k_query_reset<<<1, 1, 0, c->stream>>>(st);

  // ---- central run and top-w selection
  RunView r1 = run_view(c, RUN_CENTRAL, p.C, c->Hc, p);
  RunStatus s1 = {}, s2 = {};
  RAKS_TRY(run_levels(c, r1, p.TPc, p.central, p.C, &s1));
  SelectView sv;
  sv.cand = P<uint64_t>(c->cand);
  sv.st = r1.st;
  sv.gst = st;
  sv.w = p.w;
  sv.sel_node = P<int32_t>(c->sel_node);
  sv.sel_sc = P<int32_t>(c->sel_sc);
  sv.sel_sumh = P<int32_t>(c->sel_sumh);
  {
    Timed t(c, 2);
    launch_select(sv, c->stream);
  }

  // ---- recovery of the selected CGs (instances beyond nsel exit at once)
  const int top1 = std::max(0, s1.levels - 1);   // central levels are at most this
  RAKS_TRY(ensure_recovery(c, std::max(p.w * p.C, p.k * p.M), p.w, p.C, p.M, p.k, p.L));
  {
    Timed t(c, 3);
    launch_recover(recover_view(c, 0, c->Hc, p.TPc, p.C, p.w * p.C, &st->nsel, top1), c->stream);
    launch_finalize(finalize_view(c, 0, p.C, p.w, &st->nsel, p.C, p.TPc, p.M), c->stream);
    if (p.M > 0)
      launch_pack_vc(P<uint32_t>(c->vc_cnt), P<int32_t>(c->vc_tmp), (uint32_t)p.C * c->nc,
                     &st->nsel, P<uint32_t>(c->vc_off), P<int32_t>(c->vc_nodes), c->stream);
  }
  HIP_OK(hipGetLastError());

  // ---- marginal run (ends before level 0 when no CG was selected)
  int top2 = 0;
  if (p.M > 0) {
    RunView r2 = run_view(c, RUN_MARGINAL, p.M, c->Hm, p);
    RAKS_TRY(run_levels(c, r2, p.TPm, p.marginal, p.M, &s2));
    top2 = std::max(0, s2.levels - 1);
  }

  // ---- ranking, marginal recovery, output
  RankView rv;
  rv.gst = st;
  rv.nsel = &st->nsel;
  rv.M = p.M;
  rv.k = p.k;
  rv.gamma_num = p.gn;
  rv.gamma_den = p.gd;
  rv.sel_sc = P<int32_t>(c->sel_sc);
  rv.has_rpg = P<int32_t>(c->has_rpg);
  rv.sm = P<int32_t>(c->sm);
  rv.key = P<int64_t>(c->key);
  rv.ranked = P<int32_t>(c->ranked);
  {
    Timed t(c, 2);
    launch_rank(rv, c->stream);
  }
  {
    Timed t(c, 3);
    if (p.M > 0)
      launch_recover(recover_view(c, 1, c->Hm, p.TPm, p.M, p.k * p.M, &st->nres, top2), c->stream);
    FinalizeView fv = finalize_view(c, 1, p.M, p.k, &st->nres, p.C, p.TPc, p.M);
    fv.out_ncap = (uint32_t)std::min<size_t>(c->out_nodes.bytes / 4, UINT32_MAX);
    fv.out_acap = (uint32_t)std::min<size_t>(c->out_arcs.bytes / 12, UINT32_MAX);
    launch_finalize(fv, c->stream);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(c->q_end, c->stream));

  // ---- results to the host: status, headers and a first slice of the
  // output in one round trip
  HIP_OK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipMemcpyAsync(c->h_hdr, c->hdr.p, sizeof(ResultHdr) * p.k, hipMemcpyDeviceToHost, c->stream));
  const size_t spec_n = std::min(c->out_nodes.bytes / 4, (size_t)kSpecNodes);
  const size_t spec_a = std::min(c->out_arcs.bytes / 12, (size_t)kSpecArcs);
  HIP_OK(hipMemcpyAsync(c->h_nodes, c->out_nodes.p, 4 * spec_n, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipMemcpyAsync(c->h_arcs, c->out_arcs.p, 12 * spec_a, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  const Status hs = *c->h_status;
  if (hs.overflow) {
    *overflow = true;
    if (c->timing) harvest_timing(c);
    return RAKS_OK;
  }
  const int nres = hs.nres, nsel = hs.nsel;
  const uint32_t tn = hs.out_nodes, ta = hs.out_arcs;
  std::vector<int32_t> big_nodes, big_arcs;
  const int32_t* nodes = c->h_nodes;
  const int32_t* arcs = c->h_arcs;
  if (tn > spec_n) {
    big_nodes.resize(tn);
    HIP_OK(hipMemcpyAsync(big_nodes.data(), c->out_nodes.p, 4 * (size_t)tn, hipMemcpyDeviceToHost, c->stream));
    nodes = big_nodes.data();
  }
  if (ta > spec_a) {
    big_arcs.resize((size_t)ta * 3);
    HIP_OK(hipMemcpyAsync(big_arcs.data(), c->out_arcs.p, 12 * (size_t)ta, hipMemcpyDeviceToHost, c->stream));
    arcs = big_arcs.data();
  }
  if (tn > spec_n || ta > spec_a) HIP_OK(hipStreamSynchronize(c->stream));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, c->q_start, c->q_end);
  if (c->timing) harvest_timing(c);

  raks_results* res = (raks_results*)calloc(1, sizeof(raks_results));
  if (!res) return fail(RAKS_ENOMEM, "host allocation failed");
  res->n = nres;
  res->r = (raks_result*)calloc(std::max(nres, 1), sizeof(raks_result));
  for (int t = 0; t < nres; ++t) {
    raks_result& o = res->r[t];
    const ResultHdr& h = c->h_hdr[t];
    o.central_node = h.central;
    o.score_c = h.score_c;
    o.score_m = h.score_m;
    o.key = h.key;
    o.n_nodes = (int32_t)h.n_nodes;
    int32_t* nd = (int32_t*)malloc(sizeof(int32_t) * std::max<uint32_t>(h.n_nodes, 1));
    memcpy(nd, nodes + h.node_off, sizeof(int32_t) * h.n_nodes);
    o.nodes = nd;
    o.n_arcs = (int32_t)h.n_arcs;
    raks_arc* ar = (raks_arc*)malloc(sizeof(raks_arc) * std::max<uint32_t>(h.n_arcs, 1));
    memcpy(ar, arcs + 3 * (size_t)h.arc_off, sizeof(raks_arc) * h.n_arcs);
    o.arcs = ar;
  }
  const RunStatus* rs2[2] = {&hs.run[0], &hs.run[1]};
  for (int k = 0; k < 2; ++k) {
    const RunStatus& rs = *rs2[k];
    const bool ran = (k == 0) || (p.M > 0 && nsel > 0);
    res->stats.levels[k] = ran ? rs.levels : 0;
    res->stats.end_reason[k] = ran ? rs.end_reason : END_NONE;
    res->stats.frontier[k] = ran ? (int64_t)rs.frontier_sum : 0;
    res->stats.e_arc[k] = ran ? (int64_t)rs.e_arc : 0;
    res->stats.e_alg[k] = ran ? (int64_t)rs.e_alg : 0;
    res->stats.gate_pass[k] = ran ? (int64_t)rs.gate_pass : 0;
    res->stats.h_writes[k] = ran ? (int64_t)rs.h_writes : 0;
  }
  res->stats.n_cg = (int32_t)hs.run[0].ncand_total;
  res->stats.device_ms = ms;
  int status = 0;
  if (hs.run[0].end_reason == END_LEVEL_BOUND) status |= RAKS_STATUS_CG_LEVEL_BOUND;
  if (p.M > 0 && nsel > 0 && hs.run[1].end_reason == END_LEVEL_BOUND) status |= RAKS_STATUS_RPG_LEVEL_BOUND;
  res->status = status;
  *out = res;
  return RAKS_OK;
}

int query_one(raks_ctx* c, const raks_query_desc* q, raks_results** out) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (!out) return fail(RAKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  QueryPlan p;
  RAKS_TRY(validate_query(c, q, p));
  RAKS_TRY(ensure_node_buffers(c));
  RAKS_TRY(dev_alloc(c, c->Hc, (size_t)c->n_pad * p.TPc));
  if (p.M > 0) RAKS_TRY(dev_alloc(c, c->Hm, (size_t)c->n_pad * p.TPm));
  for (int attempt = 0;; ++attempt) {
    bool overflow = false;
    RAKS_TRY(query_attempt(c, p, out, &overflow));
    if (!overflow) return RAKS_OK;
    if (attempt >= 6) return fail(RAKS_ENOMEM, "recovered subgraphs exceed the recovery capacity");
    c->nc *= 4;
    c->ac *= 4;
    c->lcap *= 4;
  }
}

}  // namespace

// =================================================================== ABI ===

extern "C" {

const char* raks_last_error(void) { return g_err.c_str(); }

const char* raks_version(void) { return "raks-gfx950 0.1"; }

int raks_create(raks_ctx** out, const raks_ctx_opts* opts) {
  if (!out) return fail(RAKS_EINVAL, "out is NULL");
  *out = nullptr;
  raks_ctx_opts o = {};
  if (opts) o = *opts;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(RAKS_EDEVICE, "no HIP device");
  if (o.device < 0 || o.device >= ndev) return fail(RAKS_EINVAL, "device ordinal out of range");
  hipDeviceProp_t prop;
  HIP_OK(hipGetDeviceProperties(&prop, o.device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(RAKS_EDEVICE, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");
  HIP_OK(hipSetDevice(o.device));
  raks_ctx* c = new raks_ctx();
  c->device = o.device;
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->alloc = o.alloc;
  c->free_fn = o.free;
  c->alloc_user = o.alloc_user;
  c->budget = o.mem_budget;
  if (o.stream) {
    c->stream = (hipStream_t)o.stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(RAKS_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (hipHostMalloc((void**)&c->h_status, sizeof(Status), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_run, 2 * sizeof(RunStatus), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_hdr, kMaxW * sizeof(ResultHdr), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_nodes, kSpecNodes * 4, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_arcs, kSpecArcs * 12, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&c->lvl_ev[0]) != hipSuccess || hipEventCreate(&c->lvl_ev[1]) != hipSuccess ||
      hipEventCreate(&c->q_start) != hipSuccess || hipEventCreate(&c->q_end) != hipSuccess) {
    raks_destroy(c);
    return fail(RAKS_EDEVICE, "host status / event allocation failed");
  }
  int rc = dev_alloc(c, c->status, sizeof(Status));
  if (rc) { raks_destroy(c); return rc; }
  *out = c;
  return RAKS_OK;
}

int raks_destroy(raks_ctx* c) {
  if (!c) return RAKS_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->row_ptr, &c->col, &c->label, &c->act, &c->act_node, &c->nw, &c->kw_nodes,
                    &c->col_s, &c->act_s, &c->eid_s, &c->row_amax, &c->bnd,
                    &c->arc_src, &c->Hc, &c->Hm, &c->F, &c->tot, &c->off, &c->q_lo, &c->q_off, &c->q_rs,
                    &c->q_mask, &c->cand, &c->sel_node, &c->sel_sc, &c->sel_sumh, &c->has_rpg,
                    &c->sm, &c->key, &c->dmin, &c->ranked, &c->vc_cnt, &c->vc_tmp, &c->vc_off,
                    &c->vc_nodes, &c->ht, &c->nl, &c->al, &c->icnt, &c->cg_nodes, &c->cg_arcs,
                    &c->cg_cnt, &c->sort_a, &c->sort_b, &c->items, &c->lcnt, &c->hdr, &c->out_nodes, &c->out_arcs,
                    &c->status};
  for (DevBuf* b : bufs) dev_free(c, *b);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->q_start) (void)hipEventDestroy(c->q_start);
  if (c->q_end) (void)hipEventDestroy(c->q_end);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_run) (void)hipHostFree(c->h_run);
  if (c->h_hdr) (void)hipHostFree(c->h_hdr);
  if (c->h_nodes) (void)hipHostFree(c->h_nodes);
  if (c->h_arcs) (void)hipHostFree(c->h_arcs);
  for (hipEvent_t e : c->lvl_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return RAKS_OK;
}

int raks_load_graph(raks_ctx* c, const raks_graph_desc* g) {
  if (!c || !g) return fail(RAKS_EINVAL, "NULL argument");
  HIP_OK(hipSetDevice(c->device));
  const int64_t n = g->n_nodes, A = g->n_arcs;
  if (n < 1 || n >= INT32_MAX) return fail(RAKS_EINVAL, "n_nodes out of range");
  if (A < 0 || A >= (int64_t)UINT32_MAX) return fail(RAKS_EINVAL, "n_arcs must be below 2^32");
  if (!g->row_ptr || (A > 0 && (!g->col || !g->label))) return fail(RAKS_EINVAL, "NULL graph array");
  if (g->act_mode != RAKS_ACT_EDGE && g->act_mode != RAKS_ACT_NODE)
    return fail(RAKS_EINVAL, "act_mode must be EDGE or NODE");
  if (g->act_mode == RAKS_ACT_NODE && !g->node_weight)
    return fail(RAKS_EINVAL, "NODE mode needs node weights");
  if (!(g->alpha > 0.0 && g->alpha < 1.0)) return fail(RAKS_EINVAL, "alpha must be in (0,1)");
  if (!(g->a_bar > 0.0 && g->a_bar <= 100.0)) return fail(RAKS_EINVAL, "a_bar must be in (0,100]");
  if (g->n_keywords < 0 || (g->n_keywords > 0 && (!g->kw_ptr || !g->kw_nodes)))
    return fail(RAKS_EINVAL, "bad keyword index");
  if (g->row_ptr[0] != 0 || g->row_ptr[n] != A) return fail(RAKS_EINVAL, "row_ptr ends do not match n_arcs");
  for (int64_t v = 0; v < n; ++v)
    if (g->row_ptr[v + 1] < g->row_ptr[v]) return fail(RAKS_EINVAL, "row_ptr not monotone");
  const int64_t nkw = g->n_keywords > 0 ? g->kw_ptr[g->n_keywords] : 0;
  if (g->n_keywords > 0) {
    if (g->kw_ptr[0] != 0) return fail(RAKS_EINVAL, "kw_ptr[0] must be 0");
    for (int32_t t = 0; t < g->n_keywords; ++t) {
      if (g->kw_ptr[t + 1] < g->kw_ptr[t]) return fail(RAKS_EINVAL, "kw_ptr not monotone");
      for (int64_t i = g->kw_ptr[t]; i < g->kw_ptr[t + 1]; ++i) {
        if (g->kw_nodes[i] < 0 || g->kw_nodes[i] >= n) return fail(RAKS_EINVAL, "keyword node out of range");
        if (i > g->kw_ptr[t] && g->kw_nodes[i] <= g->kw_nodes[i - 1])
          return fail(RAKS_EINVAL, "keyword node lists must be strictly increasing");
      }
    }
  }
  if (nkw >= (int64_t)UINT32_MAX) return fail(RAKS_EINVAL, "keyword index too large");
  c->loaded = false;
  c->n = (int32_t)n;
  c->A = (uint32_t)A;
  c->vocab = g->n_keywords;
  c->mode = g->act_mode;
  c->abar = g->a_bar;
  c->alpha = g->alpha;
  std::vector<uint32_t> rp32(n + 1);
  for (int64_t v = 0; v <= n; ++v) rp32[v] = (uint32_t)g->row_ptr[v];
  RAKS_TRY(dev_alloc(c, c->row_ptr, (n + 1) * 4));
  RAKS_TRY(dev_alloc(c, c->col, std::max<int64_t>(A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->label, std::max<int64_t>(A, 1) * 2));
  RAKS_TRY(dev_alloc(c, c->act, std::max<int64_t>(A, 1)));
  RAKS_TRY(dev_alloc(c, c->kw_nodes, std::max<int64_t>(nkw, 1) * 4));
  HIP_OK(hipMemcpyAsync(c->row_ptr.p, rp32.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->stream));
  if (A > 0) {
    HIP_OK(hipMemcpyAsync(c->col.p, g->col, A * 4, hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->label.p, g->label, A * 2, hipMemcpyHostToDevice, c->stream));
  }
  if (nkw > 0) HIP_OK(hipMemcpyAsync(c->kw_nodes.p, g->kw_nodes, nkw * 4, hipMemcpyHostToDevice, c->stream));
  if (g->act_mode == RAKS_ACT_NODE) {
    RAKS_TRY(dev_alloc(c, c->nw, n));
    RAKS_TRY(dev_alloc(c, c->act_node, n));
    HIP_OK(hipMemcpyAsync(c->nw.p, g->node_weight, n, hipMemcpyHostToDevice, c->stream));
  }
  c->kw_ptr.assign(g->kw_ptr, g->kw_ptr + (g->n_keywords > 0 ? g->n_keywords + 1 : 0));
  if (c->kw_ptr.empty()) c->kw_ptr.push_back(0);
  HIP_OK(hipStreamSynchronize(c->stream));
  RAKS_TRY(compute_activation(c));
  c->loaded = true;
  return RAKS_OK;
}

int raks_set_alpha(raks_ctx* c, double alpha) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(RAKS_EINVAL, "alpha must be in (0,1)");
  HIP_OK(hipSetDevice(c->device));
  c->alpha = alpha;
  return compute_activation(c);
}

int raks_get_activations(raks_ctx* c, uint8_t* out, int64_t n) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (n != (int64_t)c->A) return fail(RAKS_EINVAL, "n must equal n_arcs");
  HIP_OK(hipSetDevice(c->device));
  if (n > 0) HIP_OK(hipMemcpyAsync(out, c->act.p, n, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return RAKS_OK;
}

int raks_query(raks_ctx* c, const raks_query_desc* q, raks_results** out) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  HIP_OK(hipSetDevice(c->device));
  return query_one(c, q, out);
}

int raks_query_batch(raks_ctx* c, const raks_query_desc* qs, int32_t n, raks_results** outs) {
  if (!c || (n > 0 && (!qs || !outs))) return fail(RAKS_EINVAL, "NULL argument");
  if (n < 0) return fail(RAKS_EINVAL, "n < 0");
  HIP_OK(hipSetDevice(c->device));
  for (int32_t i = 0; i < n; ++i) outs[i] = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    int rc = query_one(c, &qs[i], &outs[i]);
    if (rc != RAKS_OK) {
      for (int32_t j = 0; j <= i; ++j) { raks_results_free(outs[j]); outs[j] = nullptr; }
      return rc;
    }
  }
  return RAKS_OK;
}

void raks_results_free(raks_results* r) {
  if (!r) return;
  for (int32_t i = 0; i < r->n; ++i) {
    free((void*)r->r[i].nodes);
    free((void*)r->r[i].arcs);
  }
  free(r->r);
  free(r);
}

int raks_set_timing(raks_ctx* c, int32_t enable) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  c->timing = enable != 0;
  if (c->timing)
    for (auto& a : c->acc) a = raks_kernel_timing{};
  return RAKS_OK;
}

int raks_get_timing(raks_ctx* c, int32_t kernel, raks_kernel_timing* out) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  if (kernel < 0 || kernel >= kTimers) return fail(RAKS_EINVAL, "kernel id out of range");
  *out = c->acc[kernel];
  return RAKS_OK;
}

}  // extern "C"
