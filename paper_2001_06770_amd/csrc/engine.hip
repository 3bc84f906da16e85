// engine.hip -- the cohort engine: batches and serving with many queries in
// one level loop on the device (kernels in cohort.hip, layout in cohort.h).
//
// One host thread drives the cohort stream level by level:
//   admission   a waiting query gets a slot, |C|+|M| free columns of one
//               segment and a lane (its post-processing workspace), at the
//               next level boundary; its columns are INF already, so only its
//               keyword nodes are written (level 0);
//   level       scan, control, expansion for every slot; level l+1 is
//               enqueued before the host reads level l's status (pinned);
//   CG stage    when a query's central run has ended: its CG selection,
//               recovery (Algorithm 2) and V_C on the cohort stream, so its
//               marginal run's RPG check can start (the control step replays
//               the levels it missed);
//   hand-off    when both runs have ended and the CG stage succeeded, a post
//               worker finishes the query on its lane's stream: final
//               marginal decision, counters, ranking, RPG recovery, output,
//               results; then it resets the query's columns to INF and
//               returns slot, columns and lane.
// Results are those of the single-query path, query by query.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "cohort.h"
#include "host.h"
#include "runtime.h"

namespace raks {

namespace {

constexpr int kPostWorkers = 8;

struct CoQuery {
  raks_query_desc desc = {};
  std::vector<int32_t> central, marginal;
  int32_t index = -1;      // position in a batch
  Job* job = nullptr;      // serving job
  QueryPlan p;
  bool single = false;     // runs on the single-query path (not cohort-eligible)
  // placement
  Lane* L = nullptr;
  int lane = -1, slot = -1, seg = -1, c0 = -1, T = 0, start = 0;
  // progress
  bool c_done = false, cg_sent = false, cg_ok = false, x_done = false, handed = false;
  bool big0 = false;
  int c_end = 0, m_bound = 0, cg_attempts = 0;
  uint64_t cg_seq = 0;
  hipEvent_t ready = nullptr;     // lane stream: counters, copy-out and reset done
  hipEvent_t fin = nullptr;       // cohort stream: the final marginal decision is written
  double t_submit = 0, t_admit = 0;
  // outcome
  raks_results* res = nullptr;
  int rc = RAKS_OK;
  std::string err;
};

struct TimedEv {
  hipEvent_t a, b;
  int kind;
  double bytes;
  int level;
};

}  // namespace

struct Engine {
  Ctx* c = nullptr;
  hipStream_t stream = nullptr;
  CohortView v = {};
  DevBuf H, R, slots, acc, tot, wpre, qpre, wtot, stage, cand, ccnt, coff, ccur, cst, dmin;
  bool any_vc = false;   // some slot's marginal run is checked (V_C ready): minima each level
  CoMirror* h_mir = nullptr;
  CoMirror* d_mir = nullptr;
  uint64_t seq = 0, cg_no = 0;
  int level = 0;
  CoQuery* slot[kCoSlots] = {};
  uint16_t used[kCoSegs] = {};
  std::vector<int> free_lanes;
  int lanes_made = 0;
  std::vector<hipEvent_t> ev_pool;
  // timing of the level kernels
  std::vector<hipEvent_t> tev_pool;
  size_t tev_used = 0;
  std::vector<TimedEv> timed;

  std::mutex mu;
  std::condition_variable cv;        // post queue, releases, new input
  std::deque<CoQuery*> post_q;
  std::vector<CoQuery*> released;
  std::vector<std::thread> workers;
  bool stop_workers = false;
  std::deque<CoQuery*> pending;
  bool input_closed = false;
  bool failed = false;
  std::string fail_msg;
  int fail_rc = RAKS_OK;
  std::function<void(CoQuery*)> on_done;
  std::thread serve_thr;
  bool batch = false;   // admission follows the batch policy (waves)
};

namespace {

int engine_alloc(Engine& E) {
  Ctx* c = E.c;
  const int32_t n_pad = (int32_t)(((int64_t)c->n + kScanNodes - 1) / kScanNodes * kScanNodes);
  const int32_t chunks = n_pad / kScanNodes;
  const int32_t cpw = (chunks + kScanGroups - 1) / kScanGroups;
  const int32_t nb = (chunks + cpw - 1) / cpw;
  RAKS_TRY(dev_alloc(c, E.H, (size_t)kCoSegs * n_pad * 16));
  RAKS_TRY(dev_alloc(c, E.R, (size_t)n_pad * 8));
  RAKS_TRY(dev_alloc(c, E.slots, sizeof(CoSlot) * kCoSlots));
  RAKS_TRY(dev_alloc(c, E.acc, sizeof(CoAcc)));
  RAKS_TRY(dev_alloc(c, E.tot, (size_t)nb * sizeof(uint2)));
  RAKS_TRY(dev_alloc(c, E.wpre, (size_t)(nb + 1) * 4));
  RAKS_TRY(dev_alloc(c, E.qpre, (size_t)(nb + 1) * 4));
  RAKS_TRY(dev_alloc(c, E.wtot, 16));
  RAKS_TRY(dev_alloc(c, E.stage, (size_t)n_pad * sizeof(CoEntry)));
  RAKS_TRY(dev_alloc(c, E.cand, (size_t)n_pad * 8));
  RAKS_TRY(dev_alloc(c, E.ccnt, (size_t)nb * 4));
  RAKS_TRY(dev_alloc(c, E.coff, (size_t)nb * 4));
  RAKS_TRY(dev_alloc(c, E.ccur, 16));
  RAKS_TRY(dev_alloc(c, E.cst, sizeof(RunStatus)));
  RAKS_TRY(dev_alloc(c, E.dmin, (size_t)kCoSlots * kMaxW * kMaxKw * 4));
  if (!E.h_mir) {
    void* hp = nullptr;
    if (hipHostMalloc(&hp, sizeof(CoMirror), hipHostMallocDefault) != hipSuccess)
      return fail(RAKS_ENOMEM, "pinned allocation failed");
    E.h_mir = static_cast<CoMirror*>(hp);
    memset(E.h_mir, 0, sizeof(CoMirror));
    void* dp = nullptr;
    HIP_OK(hipHostGetDevicePointer(&dp, hp, 0));
    E.d_mir = static_cast<CoMirror*>(dp);
  }
  CohortView& v = E.v;
  v.n = c->n;
  v.n_pad = n_pad;
  v.nblocks = nb;
  v.cpw = cpw;
  v.H = P<uint8_t>(E.H);
  v.R = P<unsigned long long>(E.R);
  v.rbytes = 8;
  v.slots = P<CoSlot>(E.slots);
  v.acc = P<CoAcc>(E.acc);
  v.tot = P<uint2>(E.tot);
  v.wpre = P<uint32_t>(E.wpre);
  v.qpre = P<uint32_t>(E.qpre);
  v.wtot = P<uint32_t>(E.wtot);
  v.stage = P<CoEntry>(E.stage);
  v.mirror = E.d_mir;
  v.dmin = P<uint32_t>(E.dmin);
  HIP_OK(hipMemsetAsync(E.ccur.p, 0, 16, E.stream));
  HIP_OK(hipMemsetAsync(E.wtot.p, 0, 16, E.stream));
  launch_co_init(v, E.stream);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(E.stream));
  return RAKS_OK;
}

// The level loop's stream.  A process has few hardware queues (4 by
// default), and streams beyond that share them; packets of one queue run in
// order, so a level's control step queued behind another query's recovery
// layer on a shared queue would wait for all of it.  A stream made with a CU
// mask gets a hardware queue of its own; the mask holds every CU.
int make_level_stream(const Ctx* c, hipStream_t* s) {
  std::vector<uint32_t> mask(((size_t)std::max(c->num_cu, 1) + 31) / 32, 0u);
  for (int i = 0; i < c->num_cu; ++i) mask[(size_t)i / 32] |= 1u << (i % 32);
  if (hipExtStreamCreateWithCUMask(s, (uint32_t)c->num_cu, mask.data()) == hipSuccess)
    return RAKS_OK;
  (void)hipGetLastError();
  if (hipStreamCreateWithFlags(s, hipStreamNonBlocking) == hipSuccess) return RAKS_OK;
  return fail(RAKS_EDEVICE, "stream creation failed");
}

int engine_create(Ctx* c, Engine** out) {
  Engine* E = new Engine();
  E->c = c;
  if (make_level_stream(c, &E->stream) != RAKS_OK) {
    delete E;
    return RAKS_EDEVICE;
  }
  const int rc = engine_alloc(*E);
  if (rc) {
    for (DevBuf* b : {&E->H, &E->R, &E->slots, &E->acc, &E->tot, &E->wpre, &E->qpre, &E->wtot, &E->stage,
                      &E->cand, &E->ccnt, &E->coff, &E->ccur, &E->cst, &E->dmin})
      dev_free(c, *b);
    if (E->h_mir) (void)hipHostFree(E->h_mir);
    (void)hipStreamDestroy(E->stream);
    delete E;
    return rc;
  }
  *out = E;
  return RAKS_OK;
}

hipEvent_t take_event(Engine& E) {
  if (!E.ev_pool.empty()) {
    hipEvent_t e = E.ev_pool.back();
    E.ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t timing_event(Engine& E) {
  if (E.tev_used == E.tev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    E.tev_pool.push_back(e);
  }
  return E.tev_pool[E.tev_used++];
}

void harvest(Engine& E) {
  Ctx* c = E.c;
  std::lock_guard<std::mutex> lk(c->timing_mu);
  for (auto& t : E.timed) {
    float ms = 0;
    if (t.kind < 0) continue;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->acc[t.kind].launches += 1;
      c->acc[t.kind].ms += ms;
      c->acc[t.kind].bytes += t.bytes;
    }
  }
  E.timed.clear();
  E.tev_used = 0;
}

bool eligible(const Ctx* c, const QueryPlan& p) {
  if (p.C + p.M > 16 || p.L > kCoMaxLevel) return false;
  if (!(p.alpha == 0.0 || p.alpha == c->alpha)) return false;
  for (int32_t t : p.central)
    if (c->kw_ptr[t + 1] == c->kw_ptr[t]) return false;
  for (int32_t t : p.marginal)
    if (c->kw_ptr[t + 1] == c->kw_ptr[t]) return false;
  return true;
}

// A free lane for a query's post-processing (created while fewer than
// kMaxLanes exist and device memory allows).
int take_lane(Engine& E) {
  if (!E.free_lanes.empty()) {
    const int i = E.free_lanes.back();
    E.free_lanes.pop_back();
    return i;
  }
  Ctx* c = E.c;
  if ((int)c->lanes.size() >= kMaxLanes) return -1;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b < ((size_t)1 << 30)) return -1;
  const int id = (int)c->lanes.size();
  if (ensure_lanes(c, id + 1) != RAKS_OK) return -1;
  ++E.lanes_made;
  return id;
}

// First free run of T columns within one segment of the cohort's width.
bool find_cols(Engine& E, int T, int* seg, int* c0) {
  const uint32_t m = (1u << T) - 1u;
  for (int s = 0; s < E.v.rbytes / 2; ++s)
    for (int x = 0; x + T <= 16; ++x)
      if (!((E.used[s] >> x) & m)) {
        *seg = s;
        *c0 = x;
        return true;
      }
  return false;
}

uint8_t* seg_ptr(Engine& E, int seg, int c0) {
  return E.v.H + (size_t)seg * E.v.n_pad * 16 + c0;
}

// Borrows the cohort stream for the lane's helper calls (allocation layout
// uploads, recovery, selection) so that they are ordered with the level loop.
struct Borrow {
  Lane* L;
  hipStream_t saved;
  Borrow(Lane* L_, hipStream_t s) : L(L_), saved(L_->stream) { L->stream = s; }
  ~Borrow() { L->stream = saved; }
};

int explorers(const Engine& E) {
  int k = 0;
  for (int i = 0; i < kCoSlots; ++i) k += E.slot[i] && !E.slot[i]->x_done;
  return k;
}

bool slots_busy(const Engine& E) {
  for (int i = 0; i < kCoSlots; ++i)
    if (E.slot[i]) return true;
  return false;
}

void finish(Engine& E, CoQuery* q, int rc, const std::string& err) {
  q->rc = rc;
  q->err = err;
  // a failed query may have left labels behind on its lane (a phase that lost
  // node-log entries and was not repeated): the lane's next labelled search
  // clears the whole label array
  if (rc != RAKS_OK && q->L) q->L->lab_dirty = true;
  if (E.on_done) E.on_done(q);
}

int admit(Engine& E) {
  Ctx* c = E.c;
  std::vector<CoSlot> adm;
  std::vector<int32_t> idx;
  for (;;) {
    CoQuery* q = nullptr;
    {
      std::lock_guard<std::mutex> lk(E.mu);
      if (E.pending.empty()) break;
      q = E.pending.front();
    }
    if (q->single) {
      const int li = take_lane(E);
      if (li < 0) break;
      {
        std::lock_guard<std::mutex> lk(E.mu);
        E.pending.pop_front();
        q->lane = li;
        q->L = c->lanes[li].get();
        q->t_admit = now_ms();
        q->handed = true;
        E.post_q.push_back(q);
      }
      E.cv.notify_all();
      continue;
    }
    if (E.batch && explorers(E) > c->co_admit_below) break;
    int qs = -1;
    for (int i = 0; i < kCoSlots; ++i)
      if (!E.slot[i]) { qs = i; break; }
    int seg = 0, c0 = 0;
    const int T = q->p.C + q->p.M;
    if (qs < 0 || !find_cols(E, T, &seg, &c0)) break;
    const int li = take_lane(E);
    if (li < 0) break;
    Lane* L = c->lanes[li].get();
    L->view = &c->base;
    int rc = RAKS_OK;
    {
      Borrow b(L, E.stream);
      rc = ensure_small_buffers(L);
      if (!rc) rc = dev_alloc(c, L->Hq, (size_t)E.v.n_pad * 16);
      if (!rc) {
        phase_reset(c, L->ph[0], q->p.w, q->p.C);
        phase_reset(c, L->ph[1], q->p.n_build, q->p.M);
        rc = ensure_recovery(L, q->p);
      }
      if (!rc) {
        launch_query_reset(P<Status>(L->status), E.stream);
        (void)hipEventRecord(L->q_start, E.stream);
      }
    }
    if (rc == RAKS_ENOMEM) {
      // the query's post-processing state does not fit now: wait for running
      // queries to finish, unless none runs
      E.free_lanes.push_back(li);
      bool busy = slots_busy(E);
      {
        std::lock_guard<std::mutex> lk(E.mu);
        busy |= !E.post_q.empty();
      }
      if (busy) break;
    } else if (rc) {
      E.free_lanes.push_back(li);
    }
    {
      std::lock_guard<std::mutex> lk(E.mu);
      E.pending.pop_front();
    }
    if (rc) {
      finish(E, q, rc, g_err);
      delete q;
      continue;
    }
    q->L = L;
    q->lane = li;
    q->slot = qs;
    q->seg = seg;
    q->c0 = c0;
    q->T = T;
    q->start = E.level;
    q->t_admit = now_ms();
    E.slot[qs] = q;
    E.used[seg] |= (uint16_t)(((1u << T) - 1u) << c0);
    CoSlot s = {};
    s.active = 1;
    s.seg = seg;
    s.c0 = c0;
    s.C = q->p.C;
    s.M = q->p.M;
    s.start = E.level;
    s.max_level = q->p.L;
    s.w = q->p.w;
    s.k = q->p.k;
    s.gn = q->p.gn;
    s.gd = q->p.gd;
    s.score_mode = q->p.score_mode;
    s.rerank = q->p.rerank;
    s.m_block = q->p.M >= 2 ? 1 : 0;
    s.c_run = 1;
    s.m_run = q->p.M > 0 ? 1 : 0;
    s.c_end = -1;
    s.m_xend = -1;
    s.m_end = -1;
    s.checked = -1;
    s.sel_sc = P<int32_t>(L->sel_sc);
    s.vc_off = P<uint32_t>(L->vc_off);
    s.vc_nodes = P<int32_t>(L->vc_nodes);
    s.has_rpg = P<int32_t>(L->has_rpg);
    s.sm = P<int32_t>(L->sm);
    s.key = P<int64_t>(L->key);
    s.dmin = P<uint8_t>(L->dmin);
    adm.push_back(s);
    idx.push_back(qs);
    std::vector<int32_t> kws = q->p.central;
    kws.insert(kws.end(), q->p.marginal.begin(), q->p.marginal.end());
    launch_co_seed(E.v, seg, c0, P<int32_t>(c->kw_nodes), seeds_for(c, kws), E.stream);
  }
  if (!adm.empty()) launch_co_admit(E.v, adm.data(), idx.data(), (int)adm.size(), E.stream);
  HIP_OK(hipGetLastError());
  return RAKS_OK;
}

bool any_exploring(const Engine& E) {
  for (int i = 0; i < kCoSlots; ++i)
    if (E.slot[i] && !E.slot[i]->x_done) return true;
  return false;
}

int enqueue_level(Engine& E, int level, uint64_t seq) {
  Ctx* c = E.c;
  hipStream_t s = E.stream;
  const DevGraphView g = graph_view(c, c->base);
  const uint32_t tm = c->timing.load();
  auto timed = [&](int kind, auto&& launch) {
    if ((tm >> kind) & 1u) {
      hipEvent_t a = timing_event(E), b = timing_event(E);
      if (a && b) {
        (void)hipEventRecord(a, s);
        launch();
        (void)hipEventRecord(b, s);
        E.timed.push_back({a, b, kind, 0.0, level});
        return;
      }
    }
    launch();
  };
  timed(1, [&] { launch_co_scan(E.v, g, level, s); });
  if (E.any_vc) launch_co_dmin(E.v, -1, c->num_cu * 4, s);
  timed(2, [&] { launch_co_control(E.v, level, seq, s); });
  if (tm & 1u) {
    hipEvent_t a = timing_event(E), b = timing_event(E);
    launch_co_expand(E.v, g, level, c->num_cu * c->co_wpc, c->co_tile, s, a, b);
    if (a && b) E.timed.push_back({a, b, 0, 0.0, level});
  } else {
    launch_co_expand(E.v, g, level, c->num_cu * c->co_wpc, c->co_tile, s);
  }
  HIP_OK(hipGetLastError());
  return RAKS_OK;
}

// Waits until level `level`'s control launch (number `want`) has published
// its status in the level's mirror section.  A stream that failed, or that
// has finished without the status, ends the wait with an error.
int wait_level(Engine& E, int level, uint64_t want) {
  const CoLevelMirror* m = &E.h_mir->lvl[level & (kCoMirrors - 1)];
  auto published = [&] {
    bool done = __atomic_load_n(&m->seq, __ATOMIC_ACQUIRE) == want;
    for (int q = 0; done && q < kCoSlots; ++q)
      done = __atomic_load_n(&m->slot[q].seq, __ATOMIC_ACQUIRE) == want;
    return done;
  };
  for (uint32_t spin = 1;; ++spin) {
    if (published()) return RAKS_OK;
    if ((spin & 1023u) == 0) {
      const hipError_t e = hipStreamQuery(E.stream);
      if (e != hipSuccess && e != hipErrorNotReady)
        return fail(RAKS_EDEVICE, std::string("cohort stream failed: ") + hipGetErrorString(e));
      if (e == hipSuccess && !published())
        return fail(RAKS_EDEVICE, "the cohort level status was not published");
      if (spin >= (1u << 16)) std::this_thread::sleep_for(std::chrono::microseconds(20));
      else std::this_thread::yield();
    } else {
      __builtin_ia32_pause();
    }
  }
}

// The CG stage of a query whose central run has ended (cohort stream).
int enqueue_cg(Engine& E, CoQuery* q) {
  Ctx* c = E.c;
  Lane* L = q->L;
  Borrow b(L, E.stream);
  hipStream_t s = E.stream;
  Status* st = P<Status>(L->status);
  const uint8_t* Hc = seg_ptr(E, q->seg, q->c0);
  CoCandView cv;
  cv.Hc = Hc;
  cv.C = q->p.C;
  cv.end = q->c_end;
  cv.cnt = P<uint32_t>(E.ccnt);
  cv.off = P<uint32_t>(E.coff);
  cv.cursor = P<uint32_t>(E.ccur);
  cv.cand = P<uint64_t>(E.cand);
  cv.st = P<RunStatus>(E.cst);
  cv.orig_id = P<int32_t>(c->orig_id);
  launch_co_cand(cv, E.v, s);
  SelectView sv;
  sv.int_id = P<int32_t>(c->int_id);
  sv.cand = P<uint64_t>(E.cand);
  sv.st = P<RunStatus>(E.cst);
  sv.gst = st;
  sv.w = q->p.w;
  sv.sel_node = P<int32_t>(L->sel_node);
  sv.sel_sc = P<int32_t>(L->sel_sc);
  sv.sel_sumh = P<int32_t>(L->sel_sumh);
  launch_select(sv, s);
  launch_recover(recover_view(L, 0, Hc, 16, &st->nsel, q->c_end), s);
  launch_finalize(finalize_view(L, 0, &st->nsel, q->p.C, Hc, 16), s);
  HIP_OK(hipGetLastError());
  if (q->big0) RAKS_TRY(big_finalize(L, 0, q->p, q->p.w, Hc, 16));
  if (q->p.M > 0) {
    const char* lay0 = static_cast<const char*>(L->ph[0].layout.p);
    launch_pack_vc(P<uint32_t>(L->vc_cnt), P<int32_t>(L->vc_tmp),
                   reinterpret_cast<const uint64_t*>(lay0 + L->ph[0].lay_cg_noff), &st->nsel,
                   P<uint32_t>(L->vc_off), P<int32_t>(L->vc_nodes), q->p.w, s);
  }
  q->cg_seq = ++E.cg_no;
  launch_co_cg_done(E.v, q->slot, st, q->cg_seq, s);
  HIP_OK(hipGetLastError());
  q->cg_sent = true;
  (void)c;
  return RAKS_OK;
}

__global__ void k_co_set_vc(CoSlot* slots, int q, const int32_t* vc_nodes) {
  slots[q].vc_nodes = vc_nodes;
}

// A CG stage ran out of recovery capacity: grow and repeat it.
int redo_cg(Engine& E, CoQuery* q, int ovf, int nsel) {
  Lane* L = q->L;
  if (++q->cg_attempts >= 24) return fail(RAKS_ENOMEM, "recovered subgraphs exceed the recovery capacity");
  {
    Borrow b(L, E.stream);
    if (ovf & 1) RAKS_TRY(grow_phase(L, 0, nsel, q->c_end));
    if (ovf & kOvfBig0) q->big0 = true;
    HIP_OK(hipStreamSynchronize(E.stream));
    RAKS_TRY(ensure_recovery(L, q->p));
    k_co_set_vc<<<1, 1, 0, E.stream>>>(E.v.slots, q->slot, P<int32_t>(L->vc_nodes));
    launch_retry_reset(P<Status>(L->status), E.stream);
  }
  return enqueue_cg(E, q);
}

int process_level(Engine& E, int level) {
  {
    // algorithmic bytes of the level's expansion: per examined arc its
    // neighbour id, its level and the neighbour's reached mask; per entry 24
    const CoLevelMirror& lm = E.h_mir->lvl[level & (kCoMirrors - 1)];
    for (auto& t : E.timed)
      if (t.kind == 0 && t.level == level) t.bytes = (4.0 + 1.0 + 8.0) * lm.W + 24.0 * lm.nq;
  }
  for (int i = 0; i < kCoSlots; ++i) {
    CoQuery* q = E.slot[i];
    if (!q || q->x_done || q->start > level) continue;
    const CoSlotMirror m = E.h_mir->lvl[level & (kCoMirrors - 1)].slot[i];
    if (!q->c_done && !m.c_run) {
      q->c_done = true;
      q->c_end = m.c_end;
      RAKS_TRY(enqueue_cg(E, q));
    }
    if (!m.c_run && !m.m_run) {
      q->x_done = true;
      q->m_bound = m.m_end >= 0 ? m.m_end : std::max(m.m_xend, 0);
    }
  }
  return RAKS_OK;
}

// CG stage outcomes and hand-offs to the post workers.
int poll_cg(Engine& E) {
  for (int i = 0; i < kCoSlots; ++i) {
    CoQuery* q = E.slot[i];
    if (!q || !q->cg_sent || q->cg_ok) continue;
    if (__atomic_load_n(&E.h_mir->cg_seq[i], __ATOMIC_ACQUIRE) != q->cg_seq) continue;
    const int ovf = E.h_mir->cg_ovf[i];
    if (!ovf) q->cg_ok = true;
    else RAKS_TRY(redo_cg(E, q, ovf, E.h_mir->cg_nsel[i]));
  }
  for (int i = 0; i < kCoSlots; ++i) {
    CoQuery* q = E.slot[i];
    if (!q || q->handed || !q->x_done || !q->cg_ok) continue;
    // the final marginal decision on the cohort stream; the counters, the
    // copy of the query's levels to its lane and the reset of its columns on
    // the lane's stream, beside the next levels (they touch only its columns,
    // which no level kernel reads or writes any more); slot and columns are
    // free once that is done
    if (q->p.M > 0) launch_co_dmin(E.v, q->slot, E.c->num_cu * 4, E.stream);
    launch_co_rpg_final(E.v, q->slot, E.stream);
    q->fin = take_event(E);
    if (!q->fin) return fail(RAKS_EDEVICE, "event creation failed");
    HIP_OK(hipEventRecord(q->fin, E.stream));
    HIP_OK(hipStreamWaitEvent(q->L->stream, q->fin, 0));
    CoFinishView fv;
    fv.seg = E.v.H + (size_t)q->seg * E.v.n_pad * 16;
    fv.c0 = q->c0;
    fv.C = q->p.C;
    fv.M = q->p.M;
    fv.m_block = q->p.M >= 2 ? 1 : 0;
    fv.n_pad = E.v.n_pad;
    fv.TPq = tp_for(q->p.C + q->p.M);
    fv.slot = E.v.slots + q->slot;
    fv.gst = P<Status>(q->L->status);
    fv.Hq = P<uint8_t>(q->L->Hq);
    launch_co_finish(fv, graph_view(E.c, E.c->base), q->L->stream);
    HIP_OK(hipGetLastError());
    q->ready = take_event(E);
    if (!q->ready) return fail(RAKS_EDEVICE, "event creation failed");
    HIP_OK(hipEventRecord(q->ready, q->L->stream));
    q->handed = true;
    {
      std::lock_guard<std::mutex> lk(E.mu);
      E.post_q.push_back(q);
    }
    E.cv.notify_all();
  }
  return RAKS_OK;
}

// Slots and columns of handed-off queries whose lane has finished with them.
void reap_finished(Engine& E) {
  for (int i = 0; i < kCoSlots; ++i) {
    CoQuery* q = E.slot[i];
    if (!q || !q->handed || !q->ready) continue;
    if (hipEventQuery(q->ready) != hipSuccess) continue;
    E.used[q->seg] &= (uint16_t)~(((1u << q->T) - 1u) << q->c0);
    E.slot[i] = nullptr;
    q->slot = -1;
  }
}

bool cg_outstanding(const Engine& E) {
  for (int i = 0; i < kCoSlots; ++i)
    if (E.slot[i] && E.slot[i]->cg_sent && !E.slot[i]->cg_ok) return true;
  return false;
}

void take_releases(Engine& E) {
  std::vector<CoQuery*> rel;
  {
    std::lock_guard<std::mutex> lk(E.mu);
    rel.swap(E.released);
  }
  for (CoQuery* q : rel) {
    if (q->slot >= 0) {
      E.used[q->seg] &= (uint16_t)~(((1u << q->T) - 1u) << q->c0);
      E.slot[q->slot] = nullptr;
    }
    if (q->ready) E.ev_pool.push_back(q->ready);
    if (q->fin) E.ev_pool.push_back(q->fin);
    if (q->lane >= 0) E.free_lanes.push_back(q->lane);
    delete q;
  }
}

// ------------------------------------------------------------- post ---

int post_output(Engine& E, CoQuery* q, raks_results** out) {
  Lane* L = q->L;
  hipStream_t s = L->stream;
  Status* st = P<Status>(L->status);
  const QueryPlan& p = q->p;
  const uint8_t* Hc = P<uint8_t>(L->Hq);
  const uint8_t* Hm = Hc + p.C;
  const int TPq = tp_for(p.C + p.M);   // row bytes of the lane's copy
  HIP_OK(hipStreamWaitEvent(s, q->ready, 0));
  launch_rank(rank_view(L, p), s);
  auto stage_out = [&]() -> int {
    if (p.M > 0) launch_recover(recover_view(L, 1, Hm, TPq, &st->nres, q->m_bound), s);
    launch_finalize(finalize_view(L, 1, &st->nres, p.C, Hc, TPq), s);
    if (p.rerank) launch_rerank(P<ResultHdr>(L->hdr), st, p.k, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(L->q_end, s));
    return RAKS_OK;
  };
  RAKS_TRY(stage_out());
  int ovf = 0;
  RAKS_TRY(collect(L, p, out, &ovf));
  for (int attempt = 1; ovf; ++attempt) {
    if (attempt >= 24) return fail(RAKS_ENOMEM, "recovered subgraphs exceed the recovery capacity");
    if (ovf & (4 | 1 | kOvfBig0))
      return fail(RAKS_EDEVICE, "unexpected overflow after the CG stage (internal error)");
    if (!(ovf & 2)) {
      RAKS_TRY(big_finalize(L, 1, p, p.n_build, Hc, TPq));
      if (p.rerank) launch_rerank(P<ResultHdr>(L->hdr), st, p.k, s);
      HIP_OK(hipEventRecord(L->q_end, s));
      RAKS_TRY(collect(L, p, out, &ovf));
      continue;
    }
    RAKS_TRY(grow_phase(L, 1, L->h_status->nres, q->m_bound));
    RAKS_TRY(ensure_recovery(L, p));
    launch_retry_reset(st, s);
    RAKS_TRY(stage_out());
    RAKS_TRY(collect(L, p, out, &ovf));
  }
  return RAKS_OK;
}

void post_worker(Engine* E) {
  (void)hipSetDevice(E->c->device);
  for (;;) {
    CoQuery* q = nullptr;
    {
      std::unique_lock<std::mutex> lk(E->mu);
      E->cv.wait(lk, [&] { return E->stop_workers || !E->post_q.empty(); });
      if (E->post_q.empty()) return;
      q = E->post_q.front();
      E->post_q.pop_front();
    }
    g_err.clear();
    raks_results* res = nullptr;
    int rc = RAKS_OK;
    if (q->single) {
      rc = query_on_lane(q->L, &q->desc, &res);
    } else {
      rc = post_output(*E, q, &res);
    }
    if (rc != RAKS_OK) {
      raks_results_free(res);
      res = nullptr;
    }
    q->res = res;
    if (res) {
      const double t = now_ms();
      res->stats.queue_ms = q->t_admit - q->t_submit;
      res->stats.host_ms = t - q->t_submit;
    }
    finish(*E, q, rc, rc ? g_err : std::string());
    {
      std::lock_guard<std::mutex> lk(E->mu);
      E->released.push_back(q);
    }
    E->cv.notify_all();
  }
}

void start_workers(Engine& E) {
  E.stop_workers = false;
  for (int i = 0; i < kPostWorkers; ++i) E.workers.emplace_back(post_worker, &E);
}

void stop_workers(Engine& E) {
  {
    std::lock_guard<std::mutex> lk(E.mu);
    E.stop_workers = true;
  }
  E.cv.notify_all();
  for (auto& t : E.workers) t.join();
  E.workers.clear();
}

bool posts_busy(Engine& E) {
  std::lock_guard<std::mutex> lk(E.mu);
  return !E.post_q.empty() || !E.released.empty();
}

// The level loop: runs until the input is closed and every query is done.
int engine_loop(Engine& E) {
  Ctx* c = E.c;
  (void)hipSetDevice(c->device);
  // levels queued and not yet read, oldest first: the host reads level l while
  // up to kCoAhead later levels are queued, so the device does not wait for
  // the host's admissions and hand-offs between levels (every run decision is
  // the control step's, on the device)
  std::deque<std::pair<int, uint64_t>> inflight;
  for (;;) {
    take_releases(E);
    reap_finished(E);
    RAKS_TRY(admit(E));
    if (any_exploring(E)) {
      E.any_vc = false;
      for (int i = 0; i < kCoSlots; ++i)
        E.any_vc |= E.slot[i] && !E.slot[i]->x_done && E.slot[i]->cg_sent && E.slot[i]->p.M > 0;
      const uint64_t sq = ++E.seq;
      RAKS_TRY(enqueue_level(E, E.level, sq));
      inflight.emplace_back(E.level, sq);
      ++E.level;
      if ((int)inflight.size() > kCoAhead) {
        const auto lv = inflight.front();
        inflight.pop_front();
        RAKS_TRY(wait_level(E, lv.first, lv.second));
        RAKS_TRY(process_level(E, lv.first));
      }
      RAKS_TRY(poll_cg(E));
      continue;
    }
    if (!inflight.empty()) {
      const auto lv = inflight.front();
      inflight.pop_front();
      RAKS_TRY(wait_level(E, lv.first, lv.second));
      RAKS_TRY(process_level(E, lv.first));
      RAKS_TRY(poll_cg(E));
      continue;
    }
    RAKS_TRY(poll_cg(E));
    if (cg_outstanding(E)) {
      const hipError_t e = hipStreamQuery(E.stream);
      if (e != hipSuccess && e != hipErrorNotReady)
        return fail(RAKS_EDEVICE, std::string("cohort stream failed: ") + hipGetErrorString(e));
      if (e == hipSuccess) {
        // the stream is idle: every CG stage has published its outcome
        RAKS_TRY(poll_cg(E));
        if (cg_outstanding(E)) return fail(RAKS_EDEVICE, "a CG stage outcome was not published");
        continue;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      continue;
    }
    // nothing on the device for the level loop: wait for input or releases
    std::unique_lock<std::mutex> lk(E.mu);
    const bool busy = slots_busy(E) || !E.post_q.empty();
    if (E.input_closed && E.pending.empty() && !busy && E.released.empty()) break;
    E.cv.wait_for(lk, std::chrono::milliseconds(1), [&] {
      return !E.released.empty() || (!E.pending.empty()) || (E.input_closed && !busy);
    });
  }
  harvest(E);
  return RAKS_OK;
}

// The cohort's width (columns) from the context's tuning; set while the
// cohort is empty, with the reached masks cleared for the new entry size.
int set_width(Engine& E) {
  const int rb = E.c->co_cols / 8;
  if (E.v.rbytes == rb) return RAKS_OK;
  E.v.rbytes = rb;
  launch_co_init(E.v, E.stream);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize(E.stream));
  return RAKS_OK;
}

Engine* get_engine(Ctx* c, int* rc) {
  *rc = RAKS_OK;
  Engine* E = static_cast<Engine*>(c->engine);
  if (E && E->v.n == c->n) return E;
  if (E) cohort_destroy(c);
  *rc = engine_create(c, &E);
  if (*rc) return nullptr;
  // the context's lanes serve as post-processing workspaces; more are made
  // on demand
  for (int i = (int)c->lanes.size() - 1; i >= 0; --i) E->free_lanes.push_back(i);
  c->engine = E;
  return E;
}

}  // namespace

// ---------------------------------------------------------------- API ---

void cohort_destroy(Ctx* c) {
  Engine* E = static_cast<Engine*>(c->engine);
  if (!E) return;
  c->engine = nullptr;
  if (E->serve_thr.joinable()) {
    {
      std::lock_guard<std::mutex> lk(E->mu);
      E->input_closed = true;
    }
    E->cv.notify_all();
    E->serve_thr.join();
  }
  stop_workers(*E);
  (void)hipStreamSynchronize(E->stream);
  for (DevBuf* b : {&E->H, &E->R, &E->slots, &E->acc, &E->tot, &E->wpre, &E->qpre, &E->wtot, &E->stage,
                    &E->cand, &E->ccnt, &E->coff, &E->ccur, &E->cst, &E->dmin})
    dev_free(c, *b);
  for (hipEvent_t e : E->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : E->tev_pool) (void)hipEventDestroy(e);
  if (E->h_mir) (void)hipHostFree(E->h_mir);
  (void)hipStreamDestroy(E->stream);
  delete E;
}

int cohort_query_batch(Ctx* c, const raks_query_desc* qs, int32_t n, raks_results** outs) {
  std::vector<QueryPlan> plans((size_t)std::max(n, 0));
  for (int32_t i = 0; i < n; ++i) RAKS_TRY(validate_query(c, &qs[i], plans[i]));
  int rc = RAKS_OK;
  Engine* E = get_engine(c, &rc);
  if (!E) return rc;
  RAKS_TRY(set_width(*E));
  std::vector<int> rcs((size_t)std::max(n, 0), RAKS_OK);
  std::vector<std::string> errs((size_t)std::max(n, 0));
  E->on_done = [&](CoQuery* q) {
    outs[q->index] = q->res;
    q->res = nullptr;
    rcs[q->index] = q->rc;
    errs[q->index] = q->err;
  };
  const double t0 = now_ms();
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->input_closed = true;
    for (int32_t i = 0; i < n; ++i) {
      CoQuery* q = new CoQuery();
      q->index = i;
      q->desc = qs[i];
      q->p = plans[i];
      q->single = !eligible(c, q->p);
      q->t_submit = t0;
      E->pending.push_back(q);
    }
  }
  start_workers(*E);
  E->batch = true;
  rc = engine_loop(*E);
  E->batch = false;
  if (rc) {
    // stop: queries not finished are abandoned with the batch
    std::lock_guard<std::mutex> lk(E->mu);
    for (CoQuery* q : E->pending) delete q;
    E->pending.clear();
  }
  const std::string loop_err = g_err;
  stop_workers(*E);
  take_releases(*E);
  E->on_done = nullptr;
  E->input_closed = false;
  if (!rc) {
    for (int32_t i = 0; i < n; ++i)
      if (rcs[i] != RAKS_OK) { rc = rcs[i]; g_err = errs[i]; break; }
  } else {
    g_err = loop_err;
    // the device state of an aborted loop is not reused
    (void)hipStreamSynchronize(E->stream);
    cohort_destroy(c);
  }
  if (rc) {
    for (int32_t j = 0; j < n; ++j) {
      raks_results_free(outs[j]);
      outs[j] = nullptr;
    }
  }
  return rc;
}

int cohort_serve_start(Ctx* c, int32_t queue_cap) {
  int rc = RAKS_OK;
  Engine* E = get_engine(c, &rc);
  if (E) RAKS_TRY(set_width(*E));
  if (!E) return rc;
  ServeState& S = c->serve;
  S.queue_cap = queue_cap;
  S.stop = false;
  S.running = true;
  E->input_closed = false;
  E->on_done = [c](CoQuery* q) {
    ServeState& S2 = c->serve;
    Job* job = q->job;
    {
      std::lock_guard<std::mutex> lk(S2.mu);
      job->res = q->res;
      q->res = nullptr;
      job->rc = q->rc;
      job->err = q->err;
      job->t_done = now_ms();
      job->done = true;
      --S2.in_flight;
    }
    S2.cv_done.notify_all();
  };
  start_workers(*E);
  E->serve_thr = std::thread([E, c] {
    const int r = engine_loop(*E);
    if (r) {
      // fail every query still waiting or running
      const std::string msg = g_err;
      std::vector<CoQuery*> left;
      {
        std::lock_guard<std::mutex> lk(E->mu);
        left.assign(E->pending.begin(), E->pending.end());
        E->pending.clear();
        E->failed = true;
        E->fail_rc = r;
        E->fail_msg = msg;
      }
      for (int i = 0; i < kCoSlots; ++i)
        if (E->slot[i] && !E->slot[i]->handed) left.push_back(E->slot[i]);
      for (CoQuery* q : left) {
        q->res = nullptr;
        finish(*E, q, r, msg);
      }
    }
  });
  return RAKS_OK;
}

int cohort_submit(Ctx* c, const raks_query_desc* d, uint64_t* ticket) {
  Engine* E = static_cast<Engine*>(c->engine);
  ServeState& S = c->serve;
  if (!E) return fail(RAKS_ESTATE, "serving is not running");
  CoQuery* q = new CoQuery();
  q->central.assign(d->central, d->central + d->n_central);
  if (d->n_marginal > 0) q->marginal.assign(d->marginal, d->marginal + d->n_marginal);
  q->desc = *d;
  q->desc.central = q->central.data();
  q->desc.marginal = q->marginal.empty() ? nullptr : q->marginal.data();
  q->t_submit = now_ms();
  Job* job = new Job();
  job->t_submit = q->t_submit;
  q->job = job;
  const int vrc = validate_query(c, &q->desc, q->p);
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.queue_cap > 0 && S.in_flight >= S.queue_cap) {
      delete job;
      delete q;
      return fail(RAKS_EAGAIN, "serving queue is full");
    }
    job->ticket = S.next_ticket++;
    S.jobs[job->ticket] = job;
    ++S.in_flight;
  }
  *ticket = job->ticket;
  if (vrc != RAKS_OK) {
    // invalid queries fail at raks_poll / raks_wait
    const std::string msg = g_err;
    q->res = nullptr;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      job->rc = vrc;
      job->err = msg;
      job->done = true;
      --S.in_flight;
    }
    S.cv_done.notify_all();
    delete q;
    return RAKS_OK;
  }
  q->single = !eligible(c, q->p);
  {
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->failed) {
      const int frc = E->fail_rc;
      const std::string msg = E->fail_msg;
      delete q;
      {
        std::lock_guard<std::mutex> lk2(S.mu);
        job->rc = frc;
        job->err = msg;
        job->done = true;
        --S.in_flight;
      }
      S.cv_done.notify_all();
      return RAKS_OK;
    }
    E->pending.push_back(q);
  }
  E->cv.notify_all();
  return RAKS_OK;
}

void cohort_serve_stop(Ctx* c) {
  Engine* E = static_cast<Engine*>(c->engine);
  if (!E) return;
  {
    std::lock_guard<std::mutex> lk(E->mu);
    E->input_closed = true;
  }
  E->cv.notify_all();
  if (E->serve_thr.joinable()) E->serve_thr.join();
  stop_workers(*E);
  take_releases(*E);
  E->on_done = nullptr;
  E->input_closed = false;
  const bool bad = E->failed;
  E->failed = false;
  if (bad) cohort_destroy(c);
}

}  // namespace raks
