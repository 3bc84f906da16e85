// api.hip -- host runtime and C ABI of the RAKS gfx950 library.
//
// A query runs both runs of the unified framework (Section 4.1) on one lane
// (one HIP stream and one workspace):
//   central run   level loop (scan / control / enqueue / expand) until >= w
//                 CGs, the level bound or an empty frontier; top-w selection;
//   recovery      Algorithm 2 for every (CG, central keyword); union, sort,
//                 V_C per CG;
//   marginal run  level loop with the RPG check over V_C and Theorem 4;
//   ranking       Eq. 6 order, top-k;
//   recovery      Algorithm 2 for every (RPG, marginal keyword) from the V_C
//                 nodes at distance D_j; union with the CG; output.
// Only the per-level status (a few dozen bytes) and the final results cross
// to the host.  A context holds the graph once and one or more lanes; batches
// and the serving loop run queries on several lanes at once, so the kernels
// of different queries overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>
#include <tuple>

#include "host.h"
#include "runtime.h"

using namespace raks;

struct raks_ctx : public raks::Ctx {};

namespace raks {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------- memory ---

// Device buffers grow on demand and are kept.  The context's allocator and
// budget are shared by all lanes, so allocation is serialised.
thread_local Arena* g_arena = nullptr;

int dev_alloc(Ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return RAKS_OK;
  if (g_arena) {
    Arena& a = *g_arena;
    bytes = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
    if (bytes > a.cap - a.used)
      return fail(RAKS_ENOMEM, "allocation-free query: its device state exceeds the " +
                                   std::to_string(a.cap >> 20) + " MiB scratch (" +
                                   std::to_string(a.used + bytes) + " bytes needed so far)");
    b.p = a.base + a.used;
    b.bytes = bytes;
    b.borrowed = true;
    a.used += bytes;
    return RAKS_OK;
  }
  std::lock_guard<std::mutex> lk(c->mem_mu);
  if (b.p && !b.borrowed) {
    if (c->free_fn) c->free_fn(b.p, b.bytes, c->alloc_user);
    else (void)hipFree(b.p);
    c->in_use -= b.bytes;
  }
  b = DevBuf();
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

void dev_free(Ctx* c, DevBuf& b) {
  if (!b.p || b.borrowed) {
    b = DevBuf();
    return;
  }
  std::lock_guard<std::mutex> lk(c->mem_mu);
  if (c->free_fn) c->free_fn(b.p, b.bytes, c->alloc_user);
  else (void)hipFree(b.p);
  c->in_use -= b.bytes;
  b = DevBuf();
}

int tp_for(int T) { return T <= 4 ? 4 : (T <= 8 ? 8 : 16); }

DevGraphView graph_view(const Ctx* c, const AlphaView& v) {
  DevGraphView g;
  g.n = c->n;
  g.A = c->A;
  g.row_ptr = reinterpret_cast<const uint32_t*>(c->row_ptr.p);
  g.row_ptr_o = reinterpret_cast<const uint32_t*>(c->row_ptr_o.p);
  g.orig_id = reinterpret_cast<const int32_t*>(c->orig_id.p);
  g.int_id = reinterpret_cast<const int32_t*>(c->int_id.p);
  g.col = reinterpret_cast<const int32_t*>(c->col.p);
  g.label = reinterpret_cast<const uint16_t*>(c->label.p);
  g.act = reinterpret_cast<const uint8_t*>(v.act.p);
  g.act_node = c->mode ? reinterpret_cast<const uint8_t*>(v.act_node.p) : nullptr;
  g.mode = c->mode;
  g.col_s = reinterpret_cast<const int32_t*>(v.col_s.p);
  g.act_s = reinterpret_cast<const uint8_t*>(v.act_s.p);
  g.row_amax = reinterpret_cast<const uint8_t*>(v.row_amax.p);
  g.eid_s = reinterpret_cast<const uint32_t*>(v.eid_s.p);
  g.arc_src = reinterpret_cast<const int32_t*>(c->arc_src.p);
  g.rev = reinterpret_cast<const uint32_t*>(c->rev.p);
  g.bnd = reinterpret_cast<const uint32_t*>(v.bnd.p);
  g.nbnd = c->nbnd;
  return g;
}

DevGraphView graph_view(const Lane* L) { return graph_view(L->ctx, *L->view); }

// -------------------------------------------------------------- lanes ---

std::vector<DevBuf*> lane_buffers(Lane* L) {
  std::vector<DevBuf*> v = {
      &L->Hc, &L->Hm, &L->Hq, &L->R, &L->tot, &L->sb, &L->q_off, &L->q_rs, &L->q_lo,
      &L->q_mask, &L->tile_first, &L->cand, &L->s_item, &L->s_cand, &L->sel_node, &L->sel_sc,
      &L->sel_sumh, &L->has_rpg, &L->sm, &L->key, &L->dmin, &L->ranked, &L->vc_cnt,
      &L->vc_tmp, &L->vc_off, &L->vc_nodes, &L->hpool, &L->nl, &L->al, &L->items, &L->sort_a,
      &L->sort_b, &L->cg_nodes, &L->cg_arcs, &L->cg_cnt, &L->hdr, &L->out_nodes, &L->out_arcs,
      &L->bigf, &L->big_bm, &L->big_chunk, &L->big_slot};
  for (RecPhase& P : L->ph)
    for (DevBuf* b : {&P.layout, &P.cnt, &P.iflag, &P.lcnt, &P.touch, &P.tcnt}) v.push_back(b);
  v.push_back(&L->lab);
  return v;
}

void lane_destroy(Ctx* c, Lane* L) {
  if (!L) return;
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  for (DevBuf* b : lane_buffers(L)) dev_free(c, *b);
  dev_free(c, L->status);
  for (RecPhase& P : L->ph) {
    if (P.stage) (void)hipHostFree(P.stage);
    P.stage = nullptr;
  }
  for (hipEvent_t e : L->ev_pool) (void)hipEventDestroy(e);
  L->ev_pool.clear();
  if (L->q_start) (void)hipEventDestroy(L->q_start);
  if (L->q_end) (void)hipEventDestroy(L->q_end);
  if (L->h_status) (void)hipHostFree(L->h_status);
  if (L->h_run) (void)hipHostFree(L->h_run);
  if (L->h_hdr) (void)hipHostFree(L->h_hdr);
  if (L->h_nodes) (void)hipHostFree(L->h_nodes);
  if (L->h_arcs) (void)hipHostFree(L->h_arcs);
  if (L->xfer) (void)hipHostFree(L->xfer);
  L->xfer = nullptr;
  L->xfer_bytes = 0;
  if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
  L->stream = nullptr;
}

// Lane 0 runs on the caller's stream when one was given; every other lane
// owns a non-blocking stream of default priority.
int lane_create(Ctx* c, int id, Lane** out) {
  std::unique_ptr<Lane> L(new Lane());
  L->ctx = c;
  L->id = id;
  if (id == 0 && c->user_stream) {
    L->stream = c->user_stream;
  } else {
    if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
      return fail(RAKS_EDEVICE, "hipStreamCreate failed");
    L->own_stream = true;
  }
  if (hipHostMalloc((void**)&L->h_status, sizeof(Status), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&L->h_run, 2 * sizeof(RunStatus), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&L->h_hdr, kMaxW * sizeof(ResultHdr), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&L->h_nodes, kSpecNodes * 4, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&L->h_arcs, kSpecArcs * 12, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&L->q_start) != hipSuccess || hipEventCreate(&L->q_end) != hipSuccess ||
      hipHostGetDevicePointer((void**)&L->d_run, L->h_run, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&L->d_status, L->h_status, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&L->d_hdr, L->h_hdr, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&L->d_nodes, L->h_nodes, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&L->d_arcs, L->h_arcs, 0) != hipSuccess) {
    lane_destroy(c, L.get());
    return fail(RAKS_EDEVICE, "lane pinned memory / event allocation failed");
  }
  std::memset(L->h_run, 0, 2 * sizeof(RunStatus));   // no stamp matches before a launch
  const int rc = dev_alloc(c, L->status, sizeof(Status));
  if (rc) {
    lane_destroy(c, L.get());
    return rc;
  }
  *out = L.release();
  return RAKS_OK;
}

int ensure_lanes(Ctx* c, int n) {
  n = std::min(n, kMaxLanes);
  while ((int)c->lanes.size() < n) {
    Lane* L = nullptr;
    RAKS_TRY(lane_create(c, (int)c->lanes.size(), &L));
    c->lanes.emplace_back(L);
  }
  return RAKS_OK;
}

// ------------------------------------------------------------- timing ---

// Timing events skip the system-scope fence: they are read only after the
// query's final stream synchronisation.
hipEvent_t next_event(Lane* L) {
  if (L->ev_used == L->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    L->ev_pool.push_back(e);
  }
  return L->ev_pool[L->ev_used++];
}

uint32_t timing_mask(const Lane* L) { return L->no_alloc ? 0u : L->ctx->timing.load(); }

// Brackets the launches of its scope with events on the lane's stream while
// timing is enabled.
struct Timed {
  Lane* L;
  int kind, level, run;
  hipEvent_t a = nullptr;
  Timed(Lane* L_, int kind_, int level_ = -1, int run_ = -1)
      : L(L_), kind(kind_), level(level_), run(run_) {
    if ((timing_mask(L) >> kind) & 1u) {
      a = next_event(L);
      if (a) (void)hipEventRecord(a, L->stream);
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = next_event(L);
    if (b) {
      (void)hipEventRecord(b, L->stream);
      L->pending.push_back({a, b, kind, 0.0, level, run});
    }
  }
};

void harvest_timing(Lane* L) {
  Ctx* c = L->ctx;
  {
    std::lock_guard<std::mutex> lk(c->timing_mu);
    for (auto& p : L->pending) {
      float ms = 0;
      if (p.kind < 0) continue;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        c->acc[p.kind].launches += 1;
        c->acc[p.kind].ms += ms;
        c->acc[p.kind].bytes += p.bytes;
      }
    }
  }
  L->pending.clear();
  L->ev_used = 0;
}

// -------------------------------------------------------------- graph ---

// Eqs. 1-3 for a rescaled weight x in [0, 1]: reward below alpha, penalty
// above, round half up (IEEE binary64, operations in the order written).
int level_of_x(double x, double abar, double alpha) {
  double v;
  if (x <= alpha) {
    const double reward = abar * (alpha - x) / alpha;
    v = abar - reward;
  } else {
    const double penalty = abar * (x - alpha) / (1.0 - alpha);
    v = abar + penalty;
  }
  double r = std::floor(v + 0.5);
  r = r < 0.0 ? 0.0 : (r > 254.0 ? 254.0 : r);
  return (int)r;
}

// Levels of every value in [lo, hi]: label counts c in EDGE mode (the
// fine-grained weight is ln c, min-max rescaled over the graph's counts), node
// weights in NODE mode (rescaled directly).  Evaluated once per value on the
// host, so every arc with the same count gets the same level.
void level_table(int mode, int64_t lo, int64_t hi, double abar, double alpha, uint8_t* out) {
  if (mode == RAKS_ACT_EDGE) {
    const double wmin = std::log((double)lo), wmax = std::log((double)hi);
    for (int64_t c = lo; c <= hi; ++c) {
      const double w = std::log((double)c);
      const double x = (hi == lo) ? 0.0 : (w - wmin) / (wmax - wmin);
      out[c - lo] = (uint8_t)level_of_x(x, abar, alpha);
    }
  } else {
    for (int64_t wt = lo; wt <= hi; ++wt) {
      const double x = (hi == lo) ? 0.0 : ((double)wt - (double)lo) / ((double)hi - (double)lo);
      out[wt - lo] = (uint8_t)level_of_x(x, abar, alpha);
    }
  }
}

// Checks the input contract and computes what every alpha's levels derive
// from: the label count c of every arc (EDGE) and the range of c or of the
// node weights (in ctx->wstat).
int check_graph(Ctx* c, Lane* L) {
  hipStream_t s = L->stream;
  RAKS_TRY(dev_alloc(c, c->wstat, sizeof(Status)));
  Status* st = P<Status>(c->wstat);
  RAKS_TRY(dev_alloc(c, c->arc_src, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->cweight, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->rev, (size_t)std::max<uint32_t>(c->A, 1) * 4));
  const DevGraphView g = graph_view(c, c->base);
  launch_check_and_count(g, P<uint32_t>(c->cweight), P<int32_t>(c->arc_src), P<uint32_t>(c->rev),
                         st, s);
  HIP_OK(hipMemcpyAsync(L->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (L->h_status->err) {
    char msg[160];
    snprintf(msg, sizeof msg,
             "graph violates the input contract (bits 0x%x: 1 col range, 2 self-loop, "
             "4 row order, 8 missing reverse arc)", L->h_status->err);
    return fail(RAKS_EINVAL, msg);
  }
  if (c->mode == RAKS_ACT_NODE) {
    launch_node_weight_range(g, P<uint8_t>(c->nw), st, s);
    HIP_OK(hipMemcpyAsync(L->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  c->wmin = L->h_status->cmin;
  c->wmax = L->h_status->cmax;
  if (c->A == 0 && c->mode == RAKS_ACT_EDGE) c->wmin = c->wmax = 1;
  // levels never exceed Round(2 * a_bar) (x <= 1 in Eqs. 1-3)
  c->nbnd = (int32_t)std::min(16.0, std::floor(2.0 * c->abar + 0.5) + 1.0);
  return RAKS_OK;
}

// Activation levels for `alpha` (Eqs. 1-3) and the traversal copy with every
// row sorted by level, on lane L's stream.
int build_view(Ctx* c, Lane* L, AlphaView& v, double alpha) {
  hipStream_t s = L->stream;
  const size_t A1 = std::max<uint32_t>(c->A, 1);
  RAKS_TRY(dev_alloc(c, v.act, A1));
  if (c->mode == RAKS_ACT_NODE) RAKS_TRY(dev_alloc(c, v.act_node, (size_t)c->n));
  RAKS_TRY(dev_alloc(c, v.col_s, A1 * 4));
  RAKS_TRY(dev_alloc(c, v.act_s, A1));
  RAKS_TRY(dev_alloc(c, v.eid_s, A1 * 4));
  // padded to whole scan chunks, which read it in node order
  const size_t n_pad = ((size_t)c->n + kScanNodes - 1) / kScanNodes * kScanNodes;
  RAKS_TRY(dev_alloc(c, v.row_amax, n_pad));
  HIP_OK(hipMemsetAsync(v.row_amax.p, 0, n_pad, s));
  RAKS_TRY(dev_alloc(c, v.bnd, (size_t)c->n * c->nbnd * 4));
  DevGraphView g = graph_view(c, v);
  // the level of every label count (or node weight) of the graph, on the host
  const uint64_t span = c->wmax - c->wmin + 1;
  if (span > kMaxLevelTable)
    return fail(RAKS_EINVAL, "label-count range too large for the level table");
  std::vector<uint8_t> lut(span);
  level_table(c->mode, (int64_t)c->wmin, (int64_t)c->wmax, c->abar, alpha, lut.data());
  RAKS_TRY(dev_alloc(c, c->lut, span));
  HIP_OK(hipMemcpyAsync(c->lut.p, lut.data(), span, hipMemcpyHostToDevice, s));
  if (c->mode == RAKS_ACT_EDGE) {
    launch_act_edge(g, P<uint32_t>(c->cweight), P<uint8_t>(c->lut), c->wmin, P<uint8_t>(v.act), s);
  } else {
    // node levels by original id (they give the per-arc levels), then by internal id
    RAKS_TRY(dev_alloc(c, c->node_tmp, (size_t)c->n));
    launch_act_node(g, P<uint8_t>(c->nw), P<uint8_t>(c->lut), (uint32_t)c->wmin,
                    P<uint8_t>(c->node_tmp), P<uint8_t>(v.act), s);
    launch_to_internal_u8(g, P<uint8_t>(c->node_tmp), P<uint8_t>(v.act_node), s);
  }
  launch_sort_rows(g, P<int32_t>(v.col_s), P<uint8_t>(v.act_s), P<uint32_t>(v.eid_s),
                   P<uint8_t>(v.row_amax), P<uint32_t>(v.bnd), c->nbnd, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  v.alpha = alpha;
  return RAKS_OK;
}

void free_view(Ctx* c, AlphaView& v) {
  DevBuf* bufs[] = {&v.act, &v.act_node, &v.col_s, &v.act_s, &v.eid_s, &v.row_amax, &v.bnd};
  for (DevBuf* b : bufs) dev_free(c, *b);
}

void drop_views(Ctx* c) {
  std::lock_guard<std::mutex> lk(c->view_mu);
  for (auto& v : c->views) free_view(c, *v);
  c->views.clear();
}

// The levels a query runs on: the context's own, or a cached view for the
// query's alpha (built on the lane's stream the first time; the least
// recently used unused view is dropped beyond kMaxViews).
int acquire_view(Lane* L, double alpha) {
  Ctx* c = L->ctx;
  if (alpha == 0.0 || alpha == c->alpha) {
    L->view = &c->base;
    return RAKS_OK;
  }
  std::lock_guard<std::mutex> lk(c->view_mu);
  for (auto& v : c->views) {
    if (v->alpha == alpha) {
      ++v->refs;
      v->last_use = ++c->view_clock;
      L->view = v.get();
      return RAKS_OK;
    }
  }
  if ((int)c->views.size() >= kMaxViews) {
    int victim = -1;
    for (int i = 0; i < (int)c->views.size(); ++i)
      if (c->views[i]->refs == 0 &&
          (victim < 0 || c->views[i]->last_use < c->views[victim]->last_use))
        victim = i;
    if (victim >= 0) {
      free_view(c, *c->views[victim]);
      c->views.erase(c->views.begin() + victim);
    }
  }
  std::unique_ptr<AlphaView> v(new AlphaView());
  const int rc = build_view(c, L, *v, alpha);
  if (rc) {
    free_view(c, *v);
    return rc;
  }
  v->refs = 1;
  v->last_use = ++c->view_clock;
  L->view = v.get();
  c->views.push_back(std::move(v));
  return RAKS_OK;
}

bool view_ready(Ctx* c, double alpha) {
  if (alpha == 0.0 || alpha == c->alpha) return true;
  std::lock_guard<std::mutex> lk(c->view_mu);
  for (auto& v : c->views)
    if (v->alpha == alpha) return true;
  return false;
}

void release_view(Lane* L) {
  Ctx* c = L->ctx;
  if (L->view && L->view != &c->base) {
    std::lock_guard<std::mutex> lk(c->view_mu);
    --const_cast<AlphaView*>(L->view)->refs;
  }
  L->view = nullptr;
}

// ------------------------------------------------------------- query ---

int validate_query(Ctx* c, const raks_query_desc* q, QueryPlan& p) {
  if (!q) return fail(RAKS_EINVAL, "query descriptor is NULL");
  p.C = q->n_central;
  p.M = q->n_marginal;
  if (p.C < 1 || p.C > kMaxKw) return fail(RAKS_EINVAL, "need 1..16 central keywords");
  if (p.M < 0 || p.M > kMaxKw) return fail(RAKS_EINVAL, "need 0..16 marginal keywords");
  if (!q->central || (p.M > 0 && !q->marginal)) return fail(RAKS_EINVAL, "keyword array is NULL");
  p.central.assign(q->central, q->central + p.C);
  p.marginal.clear();
  if (p.M > 0) p.marginal.assign(q->marginal, q->marginal + p.M);
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
  p.score_mode = q->score_mode;
  p.rerank = q->rerank;
  if ((p.score_mode != 0 && p.score_mode != 1) || (p.rerank != 0 && p.rerank != 1))
    return fail(RAKS_EINVAL, "score_mode and rerank must be 0 or 1");
  p.alpha = q->alpha;
  if (!(p.alpha == 0.0 || (p.alpha > 0.0 && p.alpha < 1.0)))
    return fail(RAKS_EINVAL, "alpha must be 0 (the context's) or in (0,1)");
  p.L = q->max_level ? q->max_level : 20;
  if (p.L < 1 || p.L > 250) return fail(RAKS_EINVAL, "max_level must be in 1..250");
  p.TPc = tp_for(p.C);
  p.TPm = tp_for(std::max(p.M, 1));
  p.n_build = p.rerank ? p.w : p.k;
  return RAKS_OK;
}

// Per-query arrays of a lane that do not scale with the graph.
int ensure_small_buffers(Lane* L) {
  Ctx* c = L->ctx;
  RAKS_TRY(dev_alloc(c, L->sel_node, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->sel_sc, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->sel_sumh, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->has_rpg, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->sm, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->key, kMaxW * 8));
  RAKS_TRY(dev_alloc(c, L->dmin, kMaxW * kMaxKw));
  RAKS_TRY(dev_alloc(c, L->ranked, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->vc_cnt, kMaxW * 4));
  RAKS_TRY(dev_alloc(c, L->vc_off, (kMaxW + 1) * 4));
  return RAKS_OK;
}

int ensure_node_buffers(Lane* L) {
  Ctx* c = L->ctx;
  L->n_pad = (int32_t)(((int64_t)c->n + kScanNodes - 1) / kScanNodes * kScanNodes);
  // at most kScanGroups scan workgroups, so the control step's share of
  // the totals stays the same on any graph
  const int32_t chunks = L->n_pad / kScanNodes;
  L->cpw = (chunks + kScanGroups - 1) / kScanGroups;
  L->nblocks = (chunks + L->cpw - 1) / L->cpw;
  const size_t np = (size_t)L->n_pad;
  RAKS_TRY(dev_alloc(c, L->R, np * 2));
  RAKS_TRY(dev_alloc(c, L->tot, (size_t)L->nblocks * sizeof(ScanTot)));
  RAKS_TRY(dev_alloc(c, L->sb, (size_t)2 * kSupers * 3 * 4));
  RAKS_TRY(dev_alloc(c, L->q_off, (np + 1) * 4));
  RAKS_TRY(dev_alloc(c, L->q_rs, np * 4));
  RAKS_TRY(dev_alloc(c, L->q_lo, np * 4));
  RAKS_TRY(dev_alloc(c, L->q_mask, np * 4));
  RAKS_TRY(dev_alloc(c, L->tile_first, ((size_t)c->A / kExpandTile + 2) * 4));
  RAKS_TRY(dev_alloc(c, L->cand, np * 8));
  RAKS_TRY(dev_alloc(c, L->s_item, np * 16));
  RAKS_TRY(dev_alloc(c, L->s_cand, np * 8));
  return ensure_small_buffers(L);
}

SeedList seeds_for(Ctx* c, const std::vector<int32_t>& kws) {
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

RunView run_view(Lane* L, int kind, int T, DevBuf& H, const QueryPlan& p) {
  RunView r = {};
  r.kind = kind;
  r.T = T;
  r.tmask = (T >= 32) ? 0xFFFFFFFFu : ((1u << T) - 1);
  r.block_rule = (kind == RUN_CENTRAL) ? 1 : (T >= 2 ? 1 : 0);
  r.H = P<uint8_t>(H);
  r.R = L->R.p;
  r.n_pad = L->n_pad;
  r.st = &P<Status>(L->status)->run[kind];
  r.tot = P<ScanTot>(L->tot);
  r.sb = P<uint32_t>(L->sb);
  r.nblocks = L->nblocks;
  r.cpw = L->cpw;
  r.s_item = P<uint4>(L->s_item);
  r.s_cand = P<uint64_t>(L->s_cand);
  r.q_lo = P<uint32_t>(L->q_lo);
  r.q_off = P<uint32_t>(L->q_off);
  r.q_rs = P<uint32_t>(L->q_rs);
  r.q_mask = P<uint32_t>(L->q_mask);
  r.tile_first = P<uint32_t>(L->tile_first);
  r.cand = P<uint64_t>(L->cand);
  r.max_level = p.L;
  r.w = p.w;
  r.k = p.k;
  r.gamma_num = p.gn;
  r.gamma_den = p.gd;
  r.score_mode = p.score_mode;
  r.rerank = p.rerank;
  r.nsel = &P<Status>(L->status)->nsel;
  r.sel_sc = P<int32_t>(L->sel_sc);
  r.vc_off = P<uint32_t>(L->vc_off);
  r.vc_nodes = P<int32_t>(L->vc_nodes);
  r.has_rpg = P<int32_t>(L->has_rpg);
  r.sm = P<int32_t>(L->sm);
  r.key = P<int64_t>(L->key);
  r.dmin = P<uint8_t>(L->dmin);
  return r;
}

__global__ void k_query_reset(Status* st) {
  st->nsel = 0;
  st->nres = 0;
  st->overflow = 0;
  st->out_nodes = 0;
  st->out_arcs = 0;
}

void launch_query_reset(Status* st, hipStream_t s) { k_query_reset<<<1, 1, 0, s>>>(st); }

// Waits until the control launch numbered `want` has published its status in
// pinned slot `slot`.  The stream is queried now and then, so that a failed
// stream ends the wait with an error, and so does a stream that has finished
// without the status (which would mean the launch never ran).  A wait that
// lasts (a level of a very large query) sleeps between looks instead of
// spinning.
int wait_status(Lane* L, int slot, uint64_t want) {
  const volatile uint64_t* seq = &L->h_run[slot].seq;
  for (uint32_t spin = 1;; ++spin) {
    if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) return RAKS_OK;
    if ((spin & 1023u) == 0) {
      const hipError_t e = hipStreamQuery(L->stream);
      if (e != hipSuccess && e != hipErrorNotReady)
        return fail(RAKS_EDEVICE, std::string("stream failed: ") + hipGetErrorString(e));
      if (e == hipSuccess && __atomic_load_n(seq, __ATOMIC_ACQUIRE) != want)
        return fail(RAKS_EDEVICE, "the level status was not published");
      if (spin >= (1u << 16)) std::this_thread::sleep_for(std::chrono::microseconds(20));
      else std::this_thread::yield();
    } else {
      __builtin_ia32_pause();
    }
  }
}

// One exploration run: the level loop of Figure 3.  The host enqueues level
// l+1 before it waits for the status of level l, so the GPU never idles on
// the host's decision; the kernels of a level after the run's end return at
// once.  Returns the run's final status in *last.
int run_levels(Lane* L, RunView& r, int TP, const std::vector<int32_t>& kws, int T,
               RunStatus* last) {
  Ctx* c = L->ctx;
  hipStream_t s = L->stream;
  const DevGraphView g = graph_view(L);
  const SeedList seeds = seeds_for(c, kws);
  {
    Timed t(L, 4);
    launch_run_init(r, TP, c->n, P<int32_t>(c->kw_nodes), seeds, s);
  }
  const int grid = c->num_cu * 8;
  // The control step writes the level's status into the pinned slot and
  // then stamps it with the launch's number, so the host learns the decision
  // while the level's enqueue and expansion still run, without an event
  // (an event record after every control launch costs the stream several
  // microseconds per level).
  uint64_t want[2] = {0, 0};
  auto enqueue = [&](int level, int slot) -> int {
    {
      Timed t(L, 1, level, r.kind);
      launch_front_count(r, TP, g, level, s);
    }
    {
      Timed t(L, 2, level, r.kind);
      want[slot] = ++L->ctl_seq;
      launch_front_enqueue(r, TP, level, &L->d_run[slot], want[slot], s);
    }
    if (timing_mask(L) & 1u) {
      // expansion timing: the launch itself stamps the two events
      hipEvent_t a = next_event(L), b = next_event(L);
      launch_expand(r, TP, g, level, grid, s, a, b);
      if (a && b) L->pending.push_back({a, b, 0, 0.0, level, r.kind});
    } else {
      launch_expand(r, TP, g, level, grid, s);
    }
    HIP_OK(hipGetLastError());
    return RAKS_OK;
  };
  RAKS_TRY(enqueue(0, 0));
  for (int level = 0;; ++level) {
    const int slot = level & 1;
    if (level + 1 <= r.max_level) RAKS_TRY(enqueue(level + 1, slot ^ 1));
    RAKS_TRY(wait_status(L, slot, want[slot]));
    const RunStatus rs = L->h_run[slot];
    if (timing_mask(L)) {
      for (auto& pe : L->pending) {
        if (pe.kind != 0 || pe.level != level || pe.run != r.kind) continue;
        if (rs.end_level == INT32_MAX) {
          // algorithmic bytes of this expansion: per examined arc the neighbour
          // id (4) and its T hitting levels; per queue entry 16
          pe.bytes = (4.0 + T) * rs.W + 16.0 * rs.nactive;
        } else {
          pe.kind = -1;   // the level ended before expanding: no work launched
        }
      }
    }
    if (rs.end_level != INT32_MAX || level >= r.max_level) {
      // the launches queued past the run's end return at once: not timed
      for (auto& pe : L->pending)
        if (pe.kind == 0 && pe.run == r.kind && pe.level > level) pe.kind = -1;
      *last = rs;
      break;
    }
  }
  return RAKS_OK;
}

// ------------------------------------------------------------ recovery ---

constexpr int kMaxAttempts = 24;
// a phase whose instances counted more nodes than this in all (or whose node
// tables filled up) is repeated in the labelled mode
constexpr uint64_t kLabelNodes = 1u << 16;

uint32_t pow2_at_least(uint64_t x) {
  uint32_t h = 64;
  while (h < x && h < (1u << 31)) h <<= 1;
  return h;
}

uint32_t dense_words(const Ctx* c) { return (uint32_t)(((uint64_t)c->n + 31) / 32); }

// Initial capacities for a phase of n_res results with T instances each.
void phase_reset(const Ctx* c, RecPhase& P, int n_res, int T) {
  phase_reset(P, n_res, T, c->rec_nc0, c->rec_ac0, c->rec_lcap0);
}

void phase_reset(RecPhase& P, int n_res, int T, uint32_t nc0, uint32_t ac0, uint32_t lc0) {
  const int n_inst = n_res * T;
  if (!P.grown && P.n_res == n_res && P.T == T && P.lcap) return;
  P.n_inst = n_inst;
  P.n_res = n_res;
  P.T = T;
  P.ncap.assign(n_inst, nc0);
  P.acap.assign(n_inst, ac0);
  P.dense.assign(n_inst, 0);
  P.lcap = lc0;
  P.labelled = false;
  P.tcap = 0;
  P.grown = false;
  P.dirty = true;
}

// Derives the device layout of a phase.  Phase 0 (CG recovery) also fixes
// where each CG's lists live; phase 1 sizes its sort scratch and the output
// from phase 0's largest CG lists.
void phase_layout(const Ctx* c, RecPhase& P, const RecPhase* cg_phase) {
  const uint32_t dw = dense_words(c);
  P.caps.resize(P.n_inst);
  uint64_t h = 0, nn = 0, aa = 0;
  for (int i = 0; i < P.n_inst; ++i) {
    InstCap& ic = P.caps[i];
    // the labelled mode keeps no per-instance node sets
    ic.dense = P.labelled ? 0 : P.dense[i];
    ic.hcap = (ic.dense || P.labelled) ? 0u : pow2_at_least(2ull * P.ncap[i]);
    ic.ncap = P.ncap[i];
    ic.acap = P.acap[i];
    ic.hoff = h;
    ic.noff = nn;
    ic.aoff = aa;
    if (!P.labelled) h += ((ic.dense ? (uint64_t)dw : (uint64_t)ic.hcap) + 63) & ~uint64_t(63);
    nn += ic.ncap;
    aa += ic.acap;
  }
  P.h_words = h;
  P.n_total = nn;
  P.a_total = aa;
  P.cg_noff.assign(P.n_res + 1, 0);
  P.cg_aoff.assign(P.n_res + 1, 0);
  P.soff.assign(P.n_res + 1, 0);
  P.cg_nmax = P.cg_amax = 0;
  P.out_n = P.out_a = 0;
  for (int r = 0; r < P.n_res; ++r) {
    uint64_t sn = 0, sa = 0;
    for (int j = 0; j < P.T; ++j) {
      sn += P.ncap[r * P.T + j];
      sa += P.acap[r * P.T + j];
    }
    uint64_t scratch = std::max(sn, sa);
    if (cg_phase) {
      // an RPG is its CG's lists plus its own instances
      sn += cg_phase->cg_nmax;
      sa += cg_phase->cg_amax;
      scratch = std::max(sn, sa);
      P.out_n += sn;
      P.out_a += sa;
    } else {
      P.cg_nmax = std::max(P.cg_nmax, sn);
      P.cg_amax = std::max(P.cg_amax, sa);
    }
    P.cg_noff[r + 1] = P.cg_noff[r] + sn;
    P.cg_aoff[r + 1] = P.cg_aoff[r] + sa;
    P.soff[r + 1] = P.soff[r] + scratch;
  }
}

// Uploads a phase's layout (after a change) and sizes its counters.
int phase_upload(Lane* L, RecPhase& P, int max_level) {
  Ctx* c = L->ctx;
  RAKS_TRY(dev_alloc(c, P.cnt, (size_t)std::max(P.n_inst, 1) * 8));
  RAKS_TRY(dev_alloc(c, P.iflag, (size_t)std::max(P.n_inst, 1) * 4));
  RAKS_TRY(dev_alloc(c, P.lcnt, (size_t)(max_level + 1) * 4));
  if (P.labelled) {
    RAKS_TRY(dev_alloc(c, P.touch, (size_t)std::max<uint32_t>(P.tcap, 1) * 8));
    RAKS_TRY(dev_alloc(c, P.tcnt, 4));
  }
  if (!P.dirty) return RAKS_OK;
  const size_t nr = (size_t)P.n_res + 1;
  P.lay_cg_noff = ((size_t)P.n_inst * sizeof(InstCap) + 63) & ~size_t(63);
  P.lay_cg_aoff = P.lay_cg_noff + nr * 8;
  P.lay_soff = P.lay_cg_aoff + nr * 8;
  const size_t bytes = P.lay_soff + nr * 8;
  if (P.stage_bytes < bytes) {
    if (P.stage) (void)hipHostFree(P.stage);
    P.stage = nullptr;
    P.stage_bytes = 0;
    if (hipHostMalloc(&P.stage, bytes, hipHostMallocDefault) != hipSuccess)
      return fail(RAKS_ENOMEM, "pinned staging allocation failed");
    P.stage_bytes = bytes;
  }
  char* st = static_cast<char*>(P.stage);
  if (P.n_inst) memcpy(st, P.caps.data(), (size_t)P.n_inst * sizeof(InstCap));
  memcpy(st + P.lay_cg_noff, P.cg_noff.data(), nr * 8);
  memcpy(st + P.lay_cg_aoff, P.cg_aoff.data(), nr * 8);
  memcpy(st + P.lay_soff, P.soff.data(), nr * 8);
  RAKS_TRY(dev_alloc(c, P.layout, bytes));
  HIP_OK(hipMemcpyAsync(P.layout.p, st, bytes, hipMemcpyHostToDevice, L->stream));
  P.dirty = false;
  return RAKS_OK;
}

// Layouts and device storage for both phases (grown, never shrunk).  Called
// only where no kernel of the lane is in flight, since a buffer may move.
int ensure_recovery(Lane* L, const QueryPlan& p) {
  Ctx* c = L->ctx;
  RecPhase& P0 = L->ph[0];
  RecPhase& P1 = L->ph[1];
  if (P0.dirty) {
    phase_layout(c, P0, nullptr);
    P1.dirty = true;   // its scratch and output sizes follow the CG lists
  }
  if (P1.dirty) phase_layout(c, P1, &P0);
  RAKS_TRY(phase_upload(L, P0, p.L));
  RAKS_TRY(phase_upload(L, P1, p.L));
  const uint64_t hw = std::max(P0.h_words, P1.h_words);
  const uint64_t nt = std::max(P0.n_total, P1.n_total), at = std::max(P0.a_total, P1.a_total);
  const uint64_t lc = std::max(P0.lcap, P1.lcap);
  RAKS_TRY(dev_alloc(c, L->hpool, std::max<uint64_t>(hw, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->nl, std::max<uint64_t>(nt, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->al, std::max<uint64_t>(at, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->items, (size_t)(p.L + 1) * lc * sizeof(RecItem)));
  const uint64_t cgn = P0.cg_noff[P0.n_res], cga = P0.cg_aoff[P0.n_res];
  RAKS_TRY(dev_alloc(c, L->cg_nodes, std::max<uint64_t>(cgn, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->cg_arcs, std::max<uint64_t>(cga, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->cg_cnt, (size_t)std::max(P0.n_res, 1) * 8));
  RAKS_TRY(dev_alloc(c, L->vc_tmp, std::max<uint64_t>(cgn, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->vc_nodes, std::max<uint64_t>(cgn, 1) * 4));
  const uint64_t sc = std::max(P0.soff[P0.n_res], P1.soff[P1.n_res]);
  RAKS_TRY(dev_alloc(c, L->sort_a, std::max<uint64_t>(sc, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->sort_b, std::max<uint64_t>(sc, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->hdr, (size_t)std::max(P1.n_res, 1) * sizeof(ResultHdr)));
  RAKS_TRY(dev_alloc(c, L->bigf, (size_t)std::max({P0.n_res, P1.n_res, 1}) * 4));
  RAKS_TRY(dev_alloc(c, L->out_nodes, std::max<uint64_t>(P1.out_n, 1) * 4));
  RAKS_TRY(dev_alloc(c, L->out_arcs, std::max<uint64_t>(P1.out_a, 1) * 12));
  // labels of the labelled mode: [T * G][n] words for the larger phase
  uint64_t lw = 0;
  for (const RecPhase* P : {&P0, &P1})
    if (P->labelled) lw = std::max<uint64_t>(lw, (uint64_t)P->T * ((P->n_res + 63) / 64) * c->n);
  if (lw) {
    // new memory holds anything, also when it comes back at the old address
    const void* before = L->lab.p;
    const size_t before_bytes = L->lab.bytes;
    RAKS_TRY(dev_alloc(c, L->lab, lw * 8));
    if (L->lab.p != before || L->lab.bytes != before_bytes) L->lab_dirty = true;
  }
  return RAKS_OK;
}

// After an overflow of phase `ph`: every instance that ran out gets at least
// twice its capacities and twice what it counted; one whose node table
// filled up switches to a bitmap; the layer lists grow to twice the largest
// request.  Only what the phase's kernels cleared is read: the instances of
// the n_valid existing results and the layers 1..max_layer.
int grow_phase(Lane* L, int ph, int n_valid, int max_layer) {
  Ctx* c = L->ctx;
  RecPhase& P = L->ph[ph];
  const int live = std::min(P.n_inst, n_valid * P.T);
  const int layers = std::max(max_layer, 0) + 1;
  std::vector<uint32_t> cnt((size_t)std::max(live, 1) * 2), fl(std::max(live, 1)), lc(layers);
  hipStream_t s = L->stream;
  if (live > 0) {
    HIP_OK(hipMemcpyAsync(cnt.data(), P.cnt.p, (size_t)live * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(fl.data(), P.iflag.p, (size_t)live * 4, hipMemcpyDeviceToHost, s));
  }
  HIP_OK(hipMemcpyAsync(lc.data(), P.lcnt.p, (size_t)layers * 4, hipMemcpyDeviceToHost, s));
  uint32_t tc = 0;
  if (P.labelled) HIP_OK(hipMemcpyAsync(&tc, P.tcnt.p, 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  uint32_t lmax = 0;
  for (int h = 1; h < layers; ++h) lmax = std::max(lmax, lc[h]);
  const bool chunks_fit = lmax <= P.lcap;
  const uint32_t dw = dense_words(c);
  uint64_t counted = 0;
  bool lost = false;
  for (int i = 0; i < live; ++i) {
    const uint32_t cn = cnt[2 * i], ca = cnt[2 * i + 1];
    counted += cn;
    lost |= fl[i] != 0;
    if (cn <= P.ncap[i] && ca <= P.acap[i] && !fl[i]) continue;
    // a bitmap instance that lost no work chunk counted exactly, and so did a
    // labelled search that lost neither chunks nor labelled nodes
    const bool exact = P.labelled ? (chunks_fit && tc <= P.tcap) : (P.dense[i] && !fl[i] && chunks_fit);
    const uint64_t wn = exact ? cn + cn / 8 + 64 : 2ull * std::max(P.ncap[i], cn);
    const uint64_t wa = exact ? ca + ca / 8 + 64 : 2ull * std::max(P.acap[i], ca);
    const uint64_t nn = std::min<uint64_t>((uint64_t)c->n, std::max<uint64_t>(wn, P.ncap[i]));
    const uint64_t na = std::min<uint64_t>((uint64_t)std::max<uint32_t>(c->A, 1),
                                           std::max<uint64_t>(wa, P.acap[i]));
    P.ncap[i] = (uint32_t)nn;
    P.acap[i] = (uint32_t)na;
    if (fl[i] || pow2_at_least(2ull * nn) >= dw) P.dense[i] = 1;
  }
  const uint64_t lab_entries = (uint64_t)P.T * ((P.n_res + 63) / 64) * (uint64_t)c->n;
  if (P.labelled) {
    if (tc > P.tcap) {
      // labelled nodes were lost, and their labels were not cleared
      P.tcap = (uint32_t)std::min<uint64_t>({lab_entries, 2ull * tc, 1ull << 31});
      L->lab_dirty = true;
    }
  } else if (lost || counted > kLabelNodes) {
    // large instances: one search per keyword column from now on; a node
    // labelled in a column is in at least one instance's node list
    P.labelled = true;
    uint64_t sum = 0;
    for (int i = 0; i < P.n_inst; ++i) sum += P.ncap[i];
    P.tcap = (uint32_t)std::min<uint64_t>({lab_entries, std::max<uint64_t>(sum, 1024), 1ull << 31});
  }
  // a layer holds at most every node's chunks once per instance
  const uint64_t bound = (uint64_t)std::max(live, 1) *
                         ((uint64_t)c->n + (uint64_t)c->A / kRecChunk + 1);
  if (!chunks_fit)
    P.lcap = (uint32_t)std::min<uint64_t>({2ull * lmax, bound, 1ull << 30});
  P.grown = true;
  P.dirty = true;
  return RAKS_OK;
}

RecoverView recover_view(Lane* L, int ph, const uint8_t* H, int TP, const int32_t* n_valid,
                         int max_layer) {
  RecPhase& Ph = L->ph[ph];
  RecoverView v = {};
  v.g = graph_view(L);
  v.H = H;
  v.TP = TP;
  v.T = Ph.T;
  v.marginal = ph;
  v.n_inst = Ph.n_inst;
  v.n_valid = n_valid;
  v.sel_node = P<int32_t>(L->sel_node);
  v.ranked = P<int32_t>(L->ranked);
  v.vc_off = P<uint32_t>(L->vc_off);
  v.vc_nodes = P<int32_t>(L->vc_nodes);
  v.dmin = P<uint8_t>(L->dmin);
  v.caps = P<InstCap>(Ph.layout);
  v.hpool = P<uint32_t>(L->hpool);
  v.nl = P<int32_t>(L->nl);
  v.al = P<uint32_t>(L->al);
  v.cnt = P<uint32_t>(Ph.cnt);
  v.iflag = P<uint32_t>(Ph.iflag);
  v.dwords = dense_words(L->ctx);
  v.items = P<RecItem>(L->items);
  v.lcnt = P<uint32_t>(Ph.lcnt);
  v.lcap = Ph.lcap;
  v.max_layer = max_layer;
  v.ovf_bit = ph == 0 ? 1 : 2;
  v.gst = P<Status>(L->status);
  if (Ph.labelled) {
    v.labelled = 1;
    v.G = (Ph.n_res + 63) / 64;
    // the whole allocation, not only this phase's [T * G][n] words: a later
    // phase of the same lane may use more columns or result groups, and it
    // takes every word outside a phase for zero
    v.wipe_words = L->lab_dirty ? L->lab.bytes / 8 : 0;
    L->lab_dirty = false;   // the launch clears it first
    v.lab = P<uint64_t>(L->lab);
    v.touch = P<uint64_t>(Ph.touch);
    v.tcnt = P<uint32_t>(Ph.tcnt);
    v.tcap = Ph.tcap;
  }
  return v;
}

FinalizeView finalize_view(Lane* L, int ph, const int32_t* n_valid, int C, const uint8_t* Hc,
                           int TPc) {
  RecPhase& Ph = L->ph[ph];
  RecPhase& P0 = L->ph[0];
  char* lay = static_cast<char*>(Ph.layout.p);
  char* lay0 = static_cast<char*>(P0.layout.p);
  FinalizeView v = {};
  v.g = graph_view(L);
  v.T = Ph.T;
  v.marginal = ph;
  v.n_res = Ph.n_res;
  v.n_valid = n_valid;
  v.sel_node = P<int32_t>(L->sel_node);
  v.ranked = P<int32_t>(L->ranked);
  v.caps = reinterpret_cast<const InstCap*>(lay);
  v.nl = P<int32_t>(L->nl);
  v.al = P<uint32_t>(L->al);
  v.cnt = P<uint32_t>(Ph.cnt);
  v.cg_nodes = P<uint32_t>(L->cg_nodes);
  v.cg_arcs = P<uint32_t>(L->cg_arcs);
  v.cg_cnt = P<uint32_t>(L->cg_cnt);
  v.cg_noff = reinterpret_cast<const uint64_t*>(lay0 + P0.lay_cg_noff);
  v.cg_aoff = reinterpret_cast<const uint64_t*>(lay0 + P0.lay_cg_aoff);
  v.Hc = Hc;
  v.TPc = TPc;
  v.Tc = C;
  v.vc_cnt = P<uint32_t>(L->vc_cnt);
  v.vc_tmp = P<int32_t>(L->vc_tmp);
  v.sort_a = P<uint32_t>(L->sort_a);
  v.sort_b = P<uint32_t>(L->sort_b);
  v.soff = reinterpret_cast<const uint64_t*>(lay + Ph.lay_soff);
  v.write_output = ph;
  v.skip_bits = ph == 0 ? 1 : 3;
  v.big = P<uint32_t>(L->bigf);
  v.big_list = L->ctx->big_list;
  v.hdr = P<ResultHdr>(L->hdr);
  v.out_nodes = P<int32_t>(L->out_nodes);
  v.out_arcs = P<int32_t>(L->out_arcs);
  v.out_ncap = (uint32_t)std::min<size_t>(L->out_nodes.bytes / 4, UINT32_MAX);
  v.out_acap = (uint32_t)std::min<size_t>(L->out_arcs.bytes / 12, UINT32_MAX);
  v.sel_sc = P<int32_t>(L->sel_sc);
  v.sm = P<int32_t>(L->sm);
  v.key = P<int64_t>(L->key);
  v.gst = P<Status>(L->status);
  return v;
}

// ---------------------------------------------------------------- query ---

// Clears the flags and output counters before a phase is repeated.
__global__ void k_retry_reset(Status* st) {
  st->overflow = 0;
  st->out_nodes = 0;
  st->out_arcs = 0;
}

void launch_retry_reset(Status* st, hipStream_t s) { k_retry_reset<<<1, 1, 0, s>>>(st); }

// Ranking input of the lane's query (selected CGs and their RPG records).
RankView rank_view(Lane* L, const QueryPlan& p) {
  Status* st = P<Status>(L->status);
  RankView rv;
  rv.gst = st;
  rv.nsel = &st->nsel;
  rv.M = p.M;
  rv.k = p.k;
  rv.gamma_num = p.gn;
  rv.gamma_den = p.gd;
  rv.score_mode = p.score_mode;
  rv.rerank = p.rerank;
  rv.sel_sc = P<int32_t>(L->sel_sc);
  rv.has_rpg = P<int32_t>(L->has_rpg);
  rv.sm = P<int32_t>(L->sm);
  rv.key = P<int64_t>(L->key);
  rv.ranked = P<int32_t>(L->ranked);
  return rv;
}

struct QueryRun {
  RunStatus s1 = {}, s2 = {};
  int top1 = 0, top2 = 0;
  bool big0 = false;   // some CG needs the bitmap path: finish CGs before the marginal run
};

__global__ void k_clear_flag(Status* st, int32_t bits) { st->overflow &= ~bits; }

// Runs the bitmap path for every result of phase `ph` that its finalize
// flagged.  Waits for the stream first (the flags are read on the host).
int big_finalize(Lane* L, int ph, const QueryPlan& p, int n_res, const uint8_t* Hc, int TPc) {
  Ctx* c = L->ctx;
  hipStream_t s = L->stream;
  std::vector<uint32_t> flags((size_t)std::max(n_res, 1), 0u);
  if (n_res > 0)
    HIP_OK(hipMemcpyAsync(flags.data(), L->bigf.p, (size_t)n_res * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(L->h_status, L->status.p, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // only results that exist: the flags of the others are not written
  n_res = std::min(n_res, ph == 0 ? L->h_status->nsel : L->h_status->nres);
  const uint64_t bits = std::max<uint64_t>((uint64_t)c->n, (uint64_t)c->A) + 32;
  const uint64_t words = (bits + 31) / 32;
  RAKS_TRY(dev_alloc(c, L->big_bm, words * 4));
  RAKS_TRY(dev_alloc(c, L->big_chunk, (words / 1024 + 2) * 4));
  RAKS_TRY(dev_alloc(c, L->big_slot, 8));
  const FinalizeView fv = finalize_view(L, ph, ph == 0 ? &P<Status>(L->status)->nsel
                                                       : &P<Status>(L->status)->nres, p.C, Hc, TPc);
  {
    Timed t(L, 3);
    for (int r = 0; r < n_res; ++r)
      if (flags[r])
        launch_big_finalize(fv, r, P<uint32_t>(L->big_bm), P<uint32_t>(L->big_chunk),
                            P<uint64_t>(L->big_slot), s);
    k_clear_flag<<<1, 1, 0, s>>>(P<Status>(L->status), ph == 0 ? kOvfBig0 : kOvfBig1);
  }
  HIP_OK(hipGetLastError());
  return RAKS_OK;
}

// Central run and top-w selection.
int stage_central(Lane* L, const QueryPlan& p, QueryRun& q) {
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  HIP_OK(hipEventRecord(L->q_start, s));
  k_query_reset<<<1, 1, 0, s>>>(st);
  RunView r1 = run_view(L, RUN_CENTRAL, p.C, L->Hc, p);
  RAKS_TRY(run_levels(L, r1, p.TPc, p.central, p.C, &q.s1));
  q.top1 = std::max(0, q.s1.levels - 1);   // central levels are at most this
  SelectView sv;
  sv.int_id = P<int32_t>(L->ctx->int_id);
  sv.cand = P<uint64_t>(L->cand);
  sv.st = r1.st;
  sv.gst = st;
  sv.w = p.w;
  sv.sel_node = P<int32_t>(L->sel_node);
  sv.sel_sc = P<int32_t>(L->sel_sc);
  sv.sel_sumh = P<int32_t>(L->sel_sumh);
  Timed t(L, 2);
  launch_select(sv, s);
  return RAKS_OK;
}

// CG recovery (instances beyond nsel exit at once), CG lists and V_C.
int stage_cg_recovery(Lane* L, const QueryPlan& p, const QueryRun& q) {
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  {
    Timed t(L, 3);
    launch_recover(recover_view(L, 0, P<uint8_t>(L->Hc), p.TPc, &st->nsel, q.top1), s);
    launch_finalize(finalize_view(L, 0, &st->nsel, p.C, P<uint8_t>(L->Hc), p.TPc), s);
  }
  if (q.big0) RAKS_TRY(big_finalize(L, 0, p, p.w, P<uint8_t>(L->Hc), p.TPc));
  {
    Timed t(L, 3);
    if (p.M > 0) {
      const char* lay0 = static_cast<const char*>(L->ph[0].layout.p);
      launch_pack_vc(P<uint32_t>(L->vc_cnt), P<int32_t>(L->vc_tmp),
                     reinterpret_cast<const uint64_t*>(lay0 + L->ph[0].lay_cg_noff), &st->nsel,
                     P<uint32_t>(L->vc_off), P<int32_t>(L->vc_nodes), p.w, s);
    }
  }
  HIP_OK(hipGetLastError());
  return RAKS_OK;
}

// Marginal run (ends before level 0 when no CG was selected) and ranking.
int stage_marginal(Lane* L, const QueryPlan& p, QueryRun& q) {
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  q.top2 = 0;
  if (p.M > 0) {
    RunView r2 = run_view(L, RUN_MARGINAL, p.M, L->Hm, p);
    RAKS_TRY(run_levels(L, r2, p.TPm, p.marginal, p.M, &q.s2));
    q.top2 = std::max(0, q.s2.levels - 1);
  }
  (void)st;
  Timed t(L, 2);
  launch_rank(rank_view(L, p), s);
  return RAKS_OK;
}

// RPG recovery and the output.
int stage_output(Lane* L, const QueryPlan& p, const QueryRun& q) {
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  {
    Timed t(L, 3);
    if (p.M > 0)
      launch_recover(recover_view(L, 1, P<uint8_t>(L->Hm), p.TPm, &st->nres, q.top2), s);
    launch_finalize(finalize_view(L, 1, &st->nres, p.C, P<uint8_t>(L->Hc), p.TPc), s);
    if (p.rerank) launch_rerank(P<ResultHdr>(L->hdr), st, p.k, s);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipEventRecord(L->q_end, s));
  return RAKS_OK;
}

// Status, headers and a first slice of the output in one round trip; the
// rest of the output only when it is larger.  *ovf receives the overflow
// bits (1 CG recovery, 2 RPG recovery, 4 output arena); results are built
// only when it is 0.
// Work counters, end reasons, device time and status bits of a finished query.
void fill_stats(Lane* L, const QueryPlan& p, const Status& hs, raks_query_stats* st,
                int32_t* status) {
  float ms = 0;
  (void)hipEventElapsedTime(&ms, L->q_start, L->q_end);
  const int nsel = hs.nsel;
  for (int k = 0; k < 2; ++k) {
    const RunStatus& rs = hs.run[k];
    const bool ran = (k == 0) || (p.M > 0 && nsel > 0);
    st->levels[k] = ran ? rs.levels : 0;
    st->end_reason[k] = ran ? rs.end_reason : END_NONE;
    st->frontier[k] = ran ? (int64_t)rs.frontier_sum : 0;
    st->e_arc[k] = ran ? (int64_t)rs.e_arc : 0;
    st->e_alg[k] = ran ? (int64_t)rs.e_alg : 0;
    st->gate_pass[k] = ran ? (int64_t)rs.gate_pass : 0;
    st->h_writes[k] = ran ? (int64_t)rs.h_writes : 0;
  }
  st->n_cg = (int32_t)hs.run[0].ncand_total;
  st->device_ms = ms;
  int bits = 0;
  if (hs.run[0].end_reason == END_LEVEL_BOUND) bits |= RAKS_STATUS_CG_LEVEL_BOUND;
  if (p.M > 0 && nsel > 0 && hs.run[1].end_reason == END_LEVEL_BOUND) bits |= RAKS_STATUS_RPG_LEVEL_BOUND;
  *status = bits;
}

// Host copies of the pieces (dst, src, bytes) by several threads: the result
// arrays are fresh allocations, so the copy also takes their first-touch page
// faults, which the kernel serves in parallel.
void parallel_copy(const std::vector<std::tuple<void*, const void*, size_t>>& pieces) {
  size_t total = 0;
  for (const auto& x : pieces) total += std::get<2>(x);
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = (unsigned)std::min<size_t>({(size_t)8, (size_t)hw, total / (4u << 20) + 1});
  auto part = [&](unsigned t) {
    // thread t copies bytes [t * total / nt, (t + 1) * total / nt) of the concatenation
    const size_t lo = total * t / nt, hi = total * (t + 1) / nt;
    size_t at = 0;
    for (const auto& x : pieces) {
      const size_t b = std::get<2>(x);
      const size_t s0 = std::max(lo, at), s1 = std::min(hi, at + b);
      if (s0 < s1)
        memcpy(static_cast<char*>(std::get<0>(x)) + (s0 - at),
               static_cast<const char*>(std::get<1>(x)) + (s0 - at), s1 - s0);
      at += b;
      if (at >= hi) break;
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(part, t);
  part(0);
  for (auto& x : th) x.join();
}

int collect(Lane* L, const QueryPlan& p, raks_results** out, int* ovf) {
  Ctx* c = L->ctx;
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  const size_t spec_n = std::min(L->out_nodes.bytes / 4, (size_t)kSpecNodes);
  const size_t spec_a = std::min(L->out_arcs.bytes / 12, (size_t)kSpecArcs);
  CollectView cv;
  cv.st = st;
  cv.hdr = P<ResultHdr>(L->hdr);
  cv.n_hdr = (uint32_t)p.k;
  cv.nodes = P<uint32_t>(L->out_nodes);
  cv.arcs = P<uint32_t>(L->out_arcs);
  cv.cap_nodes = (uint32_t)spec_n;
  cv.cap_arcs = (uint32_t)spec_a;
  cv.h_st = L->d_status;
  cv.h_hdr = L->d_hdr;
  cv.h_nodes = L->d_nodes;
  cv.h_arcs = L->d_arcs;
  launch_collect(cv, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(s));
  const Status hs = *L->h_status;
  *ovf = hs.overflow;
  if (hs.overflow) {
    if (timing_mask(L)) harvest_timing(L);
    return RAKS_OK;
  }
  const int nres = hs.nres, nsel = hs.nsel;
  const uint32_t tn = hs.out_nodes, ta = hs.out_arcs;
  // lists that did not fit the pinned buffers are copied from the device
  // straight into each result's own arrays
  const bool dev_nodes = tn > spec_n, dev_arcs = ta > spec_a;
  raks_results* res = (raks_results*)calloc(1, sizeof(raks_results));
  if (!res) return fail(RAKS_ENOMEM, "host allocation failed");
  res->n = nres;
  res->r = (raks_result*)calloc(std::max(nres, 1), sizeof(raks_result));
  if (!res->r) {
    raks_results_free(res);
    return fail(RAKS_ENOMEM, "host allocation failed");
  }
  // lists beyond the pinned buffers: one copy of the whole output into the
  // lane's pinned staging (a copy into pageable memory goes through small
  // staging buffers of the runtime), then host copies into the result arrays
  const size_t big_bytes = (dev_nodes ? (size_t)tn * 4 : 0) + (dev_arcs ? (size_t)ta * 12 : 0);
  char* stage = nullptr;
  if (big_bytes) {
    if (L->xfer_bytes < big_bytes) {
      if (L->xfer) (void)hipHostFree(L->xfer);
      L->xfer = nullptr;
      L->xfer_bytes = 0;
      const size_t want = big_bytes + big_bytes / 4;
      if (hipHostMalloc(&L->xfer, want, hipHostMallocDefault) == hipSuccess) L->xfer_bytes = want;
      else (void)hipGetLastError();
    }
    if (L->xfer) {
      stage = static_cast<char*>(L->xfer);
      hipError_t e = hipSuccess;
      if (dev_nodes) e = hipMemcpyAsync(stage, L->out_nodes.p, (size_t)tn * 4, hipMemcpyDeviceToHost, s);
      if (dev_arcs && e == hipSuccess)
        e = hipMemcpyAsync(stage + (dev_nodes ? (size_t)tn * 4 : 0), L->out_arcs.p, (size_t)ta * 12,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        raks_results_free(res);
        return fail(RAKS_EDEVICE, std::string("result copy: ") + hipGetErrorString(e));
      }
    }
  }
  const int32_t* st_nodes = reinterpret_cast<const int32_t*>(stage);
  const int32_t* st_arcs = reinterpret_cast<const int32_t*>(stage + (dev_nodes ? (size_t)tn * 4 : 0));
  std::vector<std::tuple<void*, const void*, size_t>> pieces;
  for (int t = 0; t < nres; ++t) {
    raks_result& o = res->r[t];
    const ResultHdr& h = L->h_hdr[t];
    o.central_node = h.central;
    o.score_c = h.score_c;
    o.score_m = h.score_m;
    o.key = h.key;
    o.weight_sum = h.wsum;
    o.n_nodes = (int32_t)h.n_nodes;
    o.n_arcs = (int32_t)h.n_arcs;
    int32_t* nd = (int32_t*)malloc(sizeof(int32_t) * std::max<uint32_t>(h.n_nodes, 1));
    raks_arc* ar = (raks_arc*)malloc(sizeof(raks_arc) * std::max<uint32_t>(h.n_arcs, 1));
    o.nodes = nd;
    o.arcs = ar;
    if (!nd || !ar) {
      raks_results_free(res);
      return fail(RAKS_ENOMEM, "host allocation failed");
    }
    hipError_t e = hipSuccess;
    if (h.n_nodes) {
      if (dev_nodes && stage)
        pieces.emplace_back(nd, st_nodes + h.node_off, sizeof(int32_t) * h.n_nodes);
      else if (dev_nodes)
        e = hipMemcpyAsync(nd, P<int32_t>(L->out_nodes) + h.node_off, sizeof(int32_t) * h.n_nodes,
                           hipMemcpyDeviceToHost, s);
      else
        memcpy(nd, L->h_nodes + h.node_off, sizeof(int32_t) * h.n_nodes);
    }
    if (h.n_arcs && e == hipSuccess) {
      if (dev_arcs && stage)
        pieces.emplace_back(ar, st_arcs + 3 * (size_t)h.arc_off, sizeof(raks_arc) * h.n_arcs);
      else if (dev_arcs)
        e = hipMemcpyAsync(ar, P<int32_t>(L->out_arcs) + 3 * (size_t)h.arc_off,
                           sizeof(raks_arc) * h.n_arcs, hipMemcpyDeviceToHost, s);
      else
        memcpy(ar, L->h_arcs + 3 * (size_t)h.arc_off, sizeof(raks_arc) * h.n_arcs);
    }
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s);
      raks_results_free(res);
      return fail(RAKS_EDEVICE, std::string("result copy: ") + hipGetErrorString(e));
    }
  }
  if (!pieces.empty()) parallel_copy(pieces);
  if ((dev_nodes || dev_arcs) && !stage) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      raks_results_free(res);
      return fail(RAKS_EDEVICE, std::string("result copy: ") + hipGetErrorString(e));
    }
  }
  if (timing_mask(L)) harvest_timing(L);
  fill_stats(L, p, hs, &res->stats, &res->status);
  *out = res;
  return RAKS_OK;
}

// A whole query on one lane.  The common case is one pass with one host wait
// at the end.  When a recovery capacity ran out, only that phase is repeated
// (the CG phase together with everything after it, since V_C feeds the
// marginal run), with the overflowing instances grown.
int query_plan_on_lane(Lane* L, const QueryPlan& p, raks_results** out, raks_results_buf* buf,
                       double t0) {
  Ctx* c = L->ctx;
  auto gather = [&](int* ovf) { return buf ? collect_into(L, p, buf, ovf) : collect(L, p, out, ovf); };
  RAKS_TRY(ensure_node_buffers(L));
  RAKS_TRY(dev_alloc(c, L->Hc, (size_t)L->n_pad * p.TPc));
  if (p.M > 0) RAKS_TRY(dev_alloc(c, L->Hm, (size_t)L->n_pad * p.TPm));
  if (L->no_alloc) {
    // the context's initial recovery capacities, halved until both phases'
    // first layouts take at most a quarter of the scratch (they grow on
    // demand like any lane's)
    uint32_t nc = c->rec_nc0, ac = c->rec_ac0, lc = c->rec_lcap0;
    const uint64_t inst = (uint64_t)p.w * p.C + (uint64_t)p.n_build * std::max(p.M, 1);
    const uint64_t share = c->na_scratch_bytes / 4;
    while ((nc > 64 || ac > 64) && inst * (32ull * nc + 24ull * ac) > share) {
      nc = std::max(64u, nc / 2);
      ac = std::max(64u, ac / 2);
    }
    while (lc > 1024 && (uint64_t)(p.L + 1) * lc * sizeof(RecItem) > share / 2) lc /= 2;
    phase_reset(L->ph[0], p.w, p.C, nc, ac, lc);
    phase_reset(L->ph[1], p.n_build, p.M, nc, ac, lc);
  } else {
    phase_reset(c, L->ph[0], p.w, p.C);
    phase_reset(c, L->ph[1], p.n_build, p.M);
  }
  QueryRun qr;
  RAKS_TRY(ensure_recovery(L, p));   // before any kernel of this query is queued
  RAKS_TRY(stage_central(L, p, qr));
  RAKS_TRY(stage_cg_recovery(L, p, qr));
  RAKS_TRY(stage_marginal(L, p, qr));
  RAKS_TRY(stage_output(L, p, qr));
  int ovf = 0;
  RAKS_TRY(gather(&ovf));
  for (int attempt = 1; ovf; ++attempt) {
    if (attempt >= kMaxAttempts)
      return fail(RAKS_ENOMEM, "recovered subgraphs exceed the recovery capacity");
    // collect() waited for the stream, so buffers may move now
    if (ovf & 4) return fail(RAKS_EDEVICE, "output arena smaller than the recovered lists (internal error)");
    const bool redo_cg = (ovf & (1 | kOvfBig0)) != 0;
    if (!redo_cg && !(ovf & 2)) {
      // only RPGs too large for the sort path: their lists are all there
      RAKS_TRY(big_finalize(L, 1, p, p.n_build, P<uint8_t>(L->Hc), p.TPc));
      if (p.rerank) launch_rerank(P<ResultHdr>(L->hdr), P<Status>(L->status), p.k, L->stream);
      HIP_OK(hipEventRecord(L->q_end, L->stream));
      RAKS_TRY(gather(&ovf));
      continue;
    }
    if (ovf & 1) RAKS_TRY(grow_phase(L, 0, L->h_status->nsel, qr.top1));
    if (ovf & kOvfBig0) qr.big0 = true;   // finish the CG lists before the marginal run
    if (!redo_cg) RAKS_TRY(grow_phase(L, 1, L->h_status->nres, qr.top2));
    RAKS_TRY(ensure_recovery(L, p));
    k_retry_reset<<<1, 1, 0, L->stream>>>(P<Status>(L->status));
    if (redo_cg) {
      RAKS_TRY(stage_cg_recovery(L, p, qr));
      RAKS_TRY(stage_marginal(L, p, qr));
    }
    RAKS_TRY(stage_output(L, p, qr));
    RAKS_TRY(gather(&ovf));
  }
  (buf ? &buf->stats : &(*out)->stats)->host_ms = now_ms() - t0;
  return RAKS_OK;
}

int query_on_lane(Lane* L, const raks_query_desc* q, raks_results** out) {
  Ctx* c = L->ctx;
  if (!out) return fail(RAKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  const double t0 = now_ms();
  QueryPlan p;
  RAKS_TRY(validate_query(c, q, p));
  RAKS_TRY(acquire_view(L, p.alpha));
  const int rc = query_plan_on_lane(L, p, out, nullptr, t0);
  release_view(L);
  // a query that failed may have left labels behind (a phase that lost node-log
  // entries and was not repeated): the lane's next labelled search clears them
  if (rc != RAKS_OK) L->lab_dirty = true;
  return rc;
}

int query_on_lane_into(Lane* L, const raks_query_desc* q, raks_results_buf* out) {
  Ctx* c = L->ctx;
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  const double t0 = now_ms();
  QueryPlan p;
  RAKS_TRY(validate_query(c, q, p));
  if (out->cap_results < p.k) return fail(RAKS_EINVAL, "cap_results is smaller than k");
  if (!view_ready(c, p.alpha))
    return fail(RAKS_ESTATE, "the levels of this query's alpha are not built (a query with "
                             "that alpha through raks_query builds them)");
  RAKS_TRY(acquire_view(L, p.alpha));
  const int rc = query_plan_on_lane(L, p, nullptr, out, t0);
  release_view(L);
  if (rc != RAKS_OK) L->lab_dirty = true;   // as in query_on_lane
  return rc;
}

// ------------------------------------------------------------ serving ---
//
// One worker thread per lane takes the oldest waiting query as soon as its
// lane is free, so queries that arrive while others run start on the device
// beside them.  Admission is by lanes; the queue may be bounded.

void serve_worker(Ctx* c, Lane* L) {
  (void)hipSetDevice(c->device);
  ServeState& S = c->serve;
  for (;;) {
    Job* job = nullptr;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_work.wait(lk, [&] { return S.stop || !S.queue.empty(); });
      if (S.queue.empty()) return;   // stop requested and nothing left
      job = S.queue.front();
      S.queue.pop_front();
      ++S.in_flight;
    }
    job->t_start = now_ms();
    g_err.clear();
    job->rc = query_on_lane(L, &job->desc, &job->res);
    if (job->rc) job->err = g_err;
    job->t_done = now_ms();
    if (job->res) {
      job->res->stats.queue_ms = job->t_start - job->t_submit;
      job->res->stats.host_ms = job->t_done - job->t_submit;
    }
    {
      std::lock_guard<std::mutex> lk(S.mu);
      job->done = true;
      --S.in_flight;
    }
    S.cv_done.notify_all();
  }
}

// Device bytes one lane holds on this graph: per node the two H matrices for
// up to 16 keywords per run, the reached masks, the expansion queue, the
// candidate keys and the scan's staging; the tile map; a recovery allowance.
size_t lane_bytes_estimate(const Ctx* c) {
  const size_t np = (size_t)c->n + kScanNodes;
  return np * (16 + 16 + 2 + 16 + 8 + 16 + 8) + ((size_t)c->A / kExpandTile + 2) * 4 +
         ((size_t)64 << 20);
}

// Drains the queue: queries already submitted still run; their results are
// freed with the jobs nobody collected.
void stop_serving(Ctx* c) {
  ServeState& S = c->serve;
  if (!S.running) return;
  if (S.cohort) {
    cohort_serve_stop(c);
    for (auto& kv : S.jobs) {
      raks_results_free(kv.second->res);
      delete kv.second;
    }
    S.jobs.clear();
    S.running = false;
    S.cohort = false;
    S.stop = false;
    return;
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv_work.notify_all();
  for (auto& t : S.workers) t.join();
  S.workers.clear();
  for (auto& kv : S.jobs) {
    raks_results_free(kv.second->res);
    delete kv.second;
  }
  S.jobs.clear();
  S.queue.clear();
  S.running = false;
  S.stop = false;
}

int take_job(Ctx* c, uint64_t ticket, raks_results** out, bool wait) {
  ServeState& S = c->serve;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.jobs.find(ticket);
  if (it == S.jobs.end()) return fail(RAKS_EINVAL, "unknown ticket");
  Job* job = it->second;
  if (wait) S.cv_done.wait(lk, [&] { return job->done; });
  if (!job->done) return fail(RAKS_EAGAIN, "query still running");
  S.jobs.erase(it);
  lk.unlock();
  const int rc = job->rc;
  if (rc == RAKS_OK) *out = job->res;
  else fail(rc, job->err);
  delete job;
  return rc;
}

}  // namespace raks

// =================================================================== ABI ===

extern "C" {

const char* raks_last_error(void) { return g_err.c_str(); }

const char* raks_version(void) { return "raks-gfx950 0.2"; }

int raks_create(raks_ctx** out, const raks_ctx_opts* opts) {
  if (!out) return fail(RAKS_EINVAL, "out is NULL");
  *out = nullptr;
  raks_ctx_opts o = {};
  if (opts) o = *opts;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(RAKS_EDEVICE, "no HIP device");
  if (o.device < 0 || o.device >= ndev) return fail(RAKS_EINVAL, "device ordinal out of range");
  if (o.lanes < 0 || o.lanes > kMaxLanes) return fail(RAKS_EINVAL, "lanes must be in 0..32");
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
  c->user_stream = (hipStream_t)o.stream;
  if (o.rec_nodes) c->rec_nc0 = o.rec_nodes;
  if (o.rec_arcs) c->rec_ac0 = o.rec_arcs;
  if (o.rec_chunks) c->rec_lcap0 = o.rec_chunks;
  if (o.big_list) c->big_list = o.big_list;
  int rc = ensure_lanes(c, std::max(1, (int)o.lanes));
  if (rc == RAKS_OK) rc = noalloc_setup(c);
  if (rc) {
    const std::string msg = g_err;
    raks_destroy(c);
    return fail(rc, msg);
  }
  *out = c;
  return RAKS_OK;
}

int raks_destroy(raks_ctx* c) {
  if (!c) return RAKS_OK;
  (void)hipSetDevice(c->device);
  stop_serving(c);
  cohort_destroy(c);
  for (auto& L : c->lanes) lane_destroy(c, L.get());
  c->lanes.clear();
  if (c->na_lane) lane_destroy(c, c->na_lane.get());
  c->na_lane.reset();
  drop_views(c);
  free_view(c, c->base);
  DevBuf* bufs[] = {&c->row_ptr, &c->col, &c->label, &c->nw, &c->kw_nodes, &c->arc_src,
                    &c->rev, &c->cweight, &c->wstat, &c->lut, &c->row_ptr_o, &c->orig_id,
                    &c->int_id, &c->node_tmp};
  for (DevBuf* b : bufs) dev_free(c, *b);
  delete c;
  return RAKS_OK;
}

int raks_load_graph(raks_ctx* c, const raks_graph_desc* g) {
  if (!c || !g) return fail(RAKS_EINVAL, "NULL argument");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running");
  HIP_OK(hipSetDevice(c->device));
  cohort_destroy(c);
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
  Lane* L = c->lanes[0].get();
  hipStream_t s = L->stream;
  c->loaded = false;
  c->n = (int32_t)n;
  c->A = (uint32_t)A;
  c->vocab = g->n_keywords;
  c->mode = g->act_mode;
  c->abar = g->a_bar;
  c->alpha = g->alpha;
  std::vector<uint32_t> rp32(n + 1);
  for (int64_t v = 0; v <= n; ++v) rp32[v] = (uint32_t)g->row_ptr[v];
  // internal numbering: nodes by degree, largest first, ties by original id
  // (a counting sort), and the internal row starts
  std::vector<int32_t> orig_id(n), int_id(n);
  std::vector<uint32_t> rpi(n + 1);
  {
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; ++v) maxd = std::max(maxd, g->row_ptr[v + 1] - g->row_ptr[v]);
    std::vector<int64_t> start((size_t)maxd + 1, 0);
    for (int64_t v = 0; v < n; ++v) ++start[g->row_ptr[v + 1] - g->row_ptr[v]];
    int64_t acc = 0;
    for (int64_t d = maxd; d >= 0; --d) {
      const int64_t k = start[d];
      start[d] = acc;
      acc += k;
    }
    for (int64_t v = 0; v < n; ++v) {
      const int64_t u = start[g->row_ptr[v + 1] - g->row_ptr[v]]++;
      orig_id[u] = (int32_t)v;
      int_id[v] = (int32_t)u;
    }
    rpi[0] = 0;
    for (int64_t u = 0; u < n; ++u)
      rpi[u + 1] = rpi[u] + (uint32_t)(g->row_ptr[orig_id[u] + 1] - g->row_ptr[orig_id[u]]);
  }
  RAKS_TRY(dev_alloc(c, c->row_ptr, (n + 1) * 4));
  RAKS_TRY(dev_alloc(c, c->row_ptr_o, (n + 1) * 4));
  RAKS_TRY(dev_alloc(c, c->orig_id, n * 4));
  RAKS_TRY(dev_alloc(c, c->int_id, n * 4));
  RAKS_TRY(dev_alloc(c, c->col, std::max<int64_t>(A, 1) * 4));
  RAKS_TRY(dev_alloc(c, c->label, std::max<int64_t>(A, 1) * 2));
  drop_views(c);
  RAKS_TRY(dev_alloc(c, c->kw_nodes, std::max<int64_t>(nkw, 1) * 4));
  HIP_OK(hipMemcpyAsync(c->row_ptr_o.p, rp32.data(), (n + 1) * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(c->row_ptr.p, rpi.data(), (n + 1) * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(c->orig_id.p, orig_id.data(), n * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(c->int_id.p, int_id.data(), n * 4, hipMemcpyHostToDevice, s));
  if (A > 0) {
    HIP_OK(hipMemcpyAsync(c->col.p, g->col, A * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(c->label.p, g->label, A * 2, hipMemcpyHostToDevice, s));
  }
  if (nkw > 0) {
    HIP_OK(hipMemcpyAsync(c->kw_nodes.p, g->kw_nodes, nkw * 4, hipMemcpyHostToDevice, s));
    launch_map_ids(P<int32_t>(c->int_id), P<int32_t>(c->kw_nodes), (uint64_t)nkw, s);
  }
  if (g->act_mode == RAKS_ACT_NODE) {
    RAKS_TRY(dev_alloc(c, c->nw, n));
    HIP_OK(hipMemcpyAsync(c->nw.p, g->node_weight, n, hipMemcpyHostToDevice, s));
  }
  c->kw_ptr.assign(g->kw_ptr, g->kw_ptr + (g->n_keywords > 0 ? g->n_keywords + 1 : 0));
  if (c->kw_ptr.empty()) c->kw_ptr.push_back(0);
  HIP_OK(hipStreamSynchronize(s));
  RAKS_TRY(check_graph(c, L));
  RAKS_TRY(build_view(c, L, c->base, c->alpha));
  c->loaded = true;
  return RAKS_OK;
}

int raks_set_alpha(raks_ctx* c, double alpha) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(RAKS_EINVAL, "alpha must be in (0,1)");
  HIP_OK(hipSetDevice(c->device));
  RAKS_TRY(build_view(c, c->lanes[0].get(), c->base, alpha));
  c->alpha = alpha;
  return RAKS_OK;
}

int raks_get_activations(raks_ctx* c, uint8_t* out, int64_t n) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (n != (int64_t)c->A) return fail(RAKS_EINVAL, "n must equal n_arcs");
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->lanes[0]->stream;
  if (n > 0) HIP_OK(hipMemcpyAsync(out, c->base.act.p, n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return RAKS_OK;
}

int raks_query(raks_ctx* c, const raks_query_desc* q, raks_results** out) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running: use raks_submit");
  HIP_OK(hipSetDevice(c->device));
  return query_on_lane(c->lanes[0].get(), q, out);
}

int raks_query_batch(raks_ctx* c, const raks_query_desc* qs, int32_t n, raks_results** outs) {
  if (!c || (n > 0 && (!qs || !outs))) return fail(RAKS_EINVAL, "NULL argument");
  if (n < 0) return fail(RAKS_EINVAL, "n < 0");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running: use raks_submit");
  HIP_OK(hipSetDevice(c->device));
  for (int32_t i = 0; i < n; ++i) outs[i] = nullptr;
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (c->batch_mode == 0) return cohort_query_batch(c, qs, n, outs);
  const int lanes = std::min<int>((int)c->lanes.size(), std::max(n, 1));
  std::atomic<int32_t> next{0};
  std::vector<int> rcs(lanes, RAKS_OK);
  std::vector<std::string> errs(lanes);
  // Each lane takes the next query index until none is left; a failure stops
  // the others from taking more.
  auto work = [&](int li) {
    (void)hipSetDevice(c->device);
    Lane* L = c->lanes[li].get();
    for (;;) {
      const int32_t i = next.fetch_add(1);
      if (i >= n) return;
      const int rc = query_on_lane(L, &qs[i], &outs[i]);
      if (rc) {
        rcs[li] = rc;
        errs[li] = g_err;
        next.store(n);
        return;
      }
    }
  };
  if (lanes <= 1) {
    work(0);
  } else {
    std::vector<std::thread> ts;
    for (int li = 1; li < lanes; ++li) ts.emplace_back(work, li);
    work(0);
    for (auto& t : ts) t.join();
  }
  for (int li = 0; li < lanes; ++li) {
    if (rcs[li] != RAKS_OK) {
      for (int32_t j = 0; j < n; ++j) {
        raks_results_free(outs[j]);
        outs[j] = nullptr;
      }
      return fail(rcs[li], errs[li]);
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

int raks_serve_start(raks_ctx* c, const raks_serve_opts* o) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(RAKS_ESTATE, "no graph loaded");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is already running");
  int lanes = o ? o->lanes : 0;
  const int32_t cap = o ? o->queue_cap : 0;
  if (lanes < 0 || lanes > kMaxLanes || cap < 0) return fail(RAKS_EINVAL, "bad serving options");
  HIP_OK(hipSetDevice(c->device));
  if (c->batch_mode == 0) {
    c->serve.cohort = true;
    const int rc = cohort_serve_start(c, cap);
    if (rc) c->serve.cohort = false;
    return rc;
  }
  if (lanes == 0) {
    // as many lanes as half of the free device memory holds, 1..8
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    lanes = (int)std::max<size_t>(1, std::min<size_t>(8, free_b / 2 / lane_bytes_estimate(c)));
  }
  RAKS_TRY(ensure_lanes(c, lanes));
  ServeState& S = c->serve;
  S.queue_cap = cap;
  S.stop = false;
  S.running = true;
  for (int li = 0; li < lanes; ++li)
    S.workers.emplace_back(serve_worker, static_cast<Ctx*>(c), c->lanes[li].get());
  return RAKS_OK;
}

int raks_submit(raks_ctx* c, const raks_query_desc* q, uint64_t* ticket) {
  if (!c || !q || !ticket) return fail(RAKS_EINVAL, "NULL argument");
  ServeState& S = c->serve;
  if (!S.running) return fail(RAKS_ESTATE, "serving is not running");
  if (q->n_central < 0 || q->n_central > kMaxKw || q->n_marginal < 0 || q->n_marginal > kMaxKw ||
      (q->n_central > 0 && !q->central) || (q->n_marginal > 0 && !q->marginal))
    return fail(RAKS_EINVAL, "bad keyword arrays");
  if (S.cohort) return cohort_submit(c, q, ticket);
  Job* job = new Job();
  job->central.assign(q->central, q->central + q->n_central);
  if (q->n_marginal > 0) job->marginal.assign(q->marginal, q->marginal + q->n_marginal);
  job->desc = *q;
  job->desc.central = job->central.data();
  job->desc.marginal = job->marginal.empty() ? nullptr : job->marginal.data();
  job->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.queue_cap > 0 && (int32_t)S.queue.size() >= S.queue_cap) {
      delete job;
      return fail(RAKS_EAGAIN, "serving queue is full");
    }
    job->ticket = S.next_ticket++;
    S.jobs[job->ticket] = job;
    S.queue.push_back(job);
  }
  S.cv_work.notify_one();
  *ticket = job->ticket;
  return RAKS_OK;
}

int raks_poll(raks_ctx* c, uint64_t ticket, raks_results** out) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  *out = nullptr;
  if (!c->serve.running) return fail(RAKS_ESTATE, "serving is not running");
  return take_job(c, ticket, out, false);
}

int raks_wait(raks_ctx* c, uint64_t ticket, raks_results** out) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  *out = nullptr;
  if (!c->serve.running) return fail(RAKS_ESTATE, "serving is not running");
  return take_job(c, ticket, out, true);
}

int raks_serve_stop(raks_ctx* c) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  stop_serving(c);
  return RAKS_OK;
}

int raks_level_table(int32_t mode, int64_t lo, int64_t hi, double a_bar, double alpha,
                     uint8_t* out) {
  if (mode != RAKS_ACT_EDGE && mode != RAKS_ACT_NODE) return fail(RAKS_EINVAL, "unknown mode");
  if (!out || hi < lo || (mode == RAKS_ACT_EDGE && lo < 1) ||
      (uint64_t)(hi - lo) >= kMaxLevelTable)
    return fail(RAKS_EINVAL, "bad value range");
  if (!(alpha > 0.0 && alpha < 1.0) || !(a_bar > 0.0)) return fail(RAKS_EINVAL, "bad a_bar or alpha");
  level_table(mode, lo, hi, a_bar, alpha, out);
  return RAKS_OK;
}

int raks_set_tuning(raks_ctx* c, const raks_tuning* t) {
  if (!c || !t) return fail(RAKS_EINVAL, "NULL argument");
  if (t->expand_wg_per_cu < 0 || t->expand_wg_per_cu > 64 || t->admit_below < 0 ||
      (t->expand_tile != 0 && t->expand_tile != 512 && t->expand_tile != 1024 &&
       t->expand_tile != 2048) ||
      (t->cohort_cols != 0 && t->cohort_cols != 16 && t->cohort_cols != 32 && t->cohort_cols != 64))
    return fail(RAKS_EINVAL, "tuning values out of range");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running");
  c->co_wpc = t->expand_wg_per_cu ? t->expand_wg_per_cu : 8;
  c->co_admit_below = t->admit_below;
  c->co_tile = t->expand_tile ? t->expand_tile : 1024;
  c->co_cols = t->cohort_cols ? t->cohort_cols : 64;
  return RAKS_OK;
}

int raks_set_batch_mode(raks_ctx* c, int32_t mode) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (mode != RAKS_BATCH_COHORT && mode != RAKS_BATCH_LANES) return fail(RAKS_EINVAL, "unknown batch mode");
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running");
  c->batch_mode = mode;
  return RAKS_OK;
}

int raks_set_timing(raks_ctx* c, int32_t mask) {
  if (!c) return fail(RAKS_EINVAL, "ctx is NULL");
  if (mask < 0 || mask >= (1 << kTimers)) return fail(RAKS_EINVAL, "timer mask out of range");
  std::lock_guard<std::mutex> lk(c->timing_mu);
  if (mask)
    for (auto& a : c->acc) a = raks_kernel_timing{};
  c->timing.store((uint32_t)mask);
  return RAKS_OK;
}

int raks_get_timing(raks_ctx* c, int32_t kernel, raks_kernel_timing* out) {
  if (!c || !out) return fail(RAKS_EINVAL, "NULL argument");
  if (kernel < 0 || kernel >= kTimers) return fail(RAKS_EINVAL, "kernel id out of range");
  std::lock_guard<std::mutex> lk(c->timing_mu);
  *out = c->acc[kernel];
  return RAKS_OK;
}

}  // extern "C"
