// noalloc.hip -- raks_query_noalloc: one query like raks_query, for callers
// that cannot allocate.  It runs the same kernels on a lane of its own whose
// device buffers are all carved from one static device array per GPU (the
// scratch below); the results go into arrays the caller passes.  Everything
// that allocates (the lane's stream, events, pinned buffers, the scratch's
// address) is set up once by raks_create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace raks {

constexpr size_t kScratchBytes = size_t(256) << 20;

// The allocation-free lane's device state: node buffers, hitting levels,
// recovery storage and output staging of one query.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device ordinal

struct ArenaScope {
  explicit ArenaScope(Arena* a) { g_arena = a; }
  ~ArenaScope() { g_arena = nullptr; }
};
}  // namespace

// Called by raks_create with c->device current.
int noalloc_setup(Ctx* c) {
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= c->device) g_scratch_ptr.resize(c->device + 1, nullptr);
    if (!g_scratch_ptr[c->device]) {
      // each device holds its own copy of the array; the host-side name is
      // not a device address, so only this pointer is ever handed to kernels
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(RAKS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_ptr[c->device] = p;
    }
    ptr = g_scratch_ptr[c->device];
  }
  c->na_scratch = ptr;
  c->na_scratch_bytes = kScratchBytes;
  Lane* L = nullptr;
  RAKS_TRY(lane_create(c, -1, &L));
  c->na_lane.reset(L);
  L->no_alloc = true;
  // pinned staging of the recovery layouts at their largest size (w <= 256
  // results, <= 16 keywords each), so a query never grows it
  const size_t stage = ((size_t)kMaxW * kMaxKw * sizeof(InstCap) + 63) / 64 * 64 +
                       3 * ((size_t)kMaxW + 1) * 8;
  for (RecPhase& P : L->ph) {
    if (hipHostMalloc(&P.stage, stage, hipHostMallocDefault) != hipSuccess)
      return fail(RAKS_ENOMEM, "pinned staging allocation failed");
    P.stage_bytes = stage;
  }
  return RAKS_OK;
}

// collect() with the caller's arrays as the destination: one kernel gathers
// the headers and the lists that fit the lane's pinned buffers, the rest is
// copied from the device.
int collect_into(Lane* L, const QueryPlan& p, raks_results_buf* out, int* ovf) {
  hipStream_t s = L->stream;
  const size_t spec_n = std::min(L->out_nodes.bytes / 4, (size_t)kSpecNodes);
  const size_t spec_a = std::min(L->out_arcs.bytes / 12, (size_t)kSpecArcs);
  CollectView cv;
  cv.st = P<Status>(L->status);
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
  if (hs.overflow) return RAKS_OK;
  const int nres = hs.nres;
  const bool dev_nodes = hs.out_nodes > spec_n, dev_arcs = hs.out_arcs > spec_a;
  int64_t need_n = 0, need_a = 0;
  for (int t = 0; t < nres; ++t) {
    need_n += L->h_hdr[t].n_nodes;
    need_a += L->h_hdr[t].n_arcs;
  }
  out->n_nodes = need_n;
  out->n_arcs = need_a;
  if (need_n > out->cap_nodes || need_a > out->cap_arcs)
    return fail(RAKS_ENOMEM, "output arrays too small: the results hold " + std::to_string(need_n) +
                                 " nodes and " + std::to_string(need_a) + " arcs");
  int64_t on = 0, oa = 0;
  for (int t = 0; t < nres; ++t) {
    const ResultHdr& h = L->h_hdr[t];
    raks_result& o = out->r[t];
    o.central_node = h.central;
    o.score_c = h.score_c;
    o.score_m = h.score_m;
    o.key = h.key;
    o.weight_sum = h.wsum;
    o.n_nodes = (int32_t)h.n_nodes;
    o.n_arcs = (int32_t)h.n_arcs;
    int32_t* nd = out->nodes ? out->nodes + on : nullptr;
    raks_arc* ar = out->arcs ? out->arcs + oa : nullptr;
    o.nodes = nd;
    o.arcs = ar;
    if (h.n_nodes) {
      if (dev_nodes)
        HIP_OK(hipMemcpyAsync(nd, P<int32_t>(L->out_nodes) + h.node_off, sizeof(int32_t) * h.n_nodes,
                              hipMemcpyDeviceToHost, s));
      else
        memcpy(nd, L->h_nodes + h.node_off, sizeof(int32_t) * h.n_nodes);
    }
    if (h.n_arcs) {
      if (dev_arcs)
        HIP_OK(hipMemcpyAsync(ar, P<int32_t>(L->out_arcs) + 3 * (size_t)h.arc_off,
                              sizeof(raks_arc) * h.n_arcs, hipMemcpyDeviceToHost, s));
      else
        memcpy(ar, L->h_arcs + 3 * (size_t)h.arc_off, sizeof(raks_arc) * h.n_arcs);
    }
    on += h.n_nodes;
    oa += h.n_arcs;
  }
  if (dev_nodes || dev_arcs) HIP_OK(hipStreamSynchronize(s));
  fill_stats(L, p, hs, &out->stats, &out->status);
  out->n = nres;
  return RAKS_OK;
}

}  // namespace raks

using namespace raks;

// the context handle of the ABI is the runtime's context
struct raks_ctx : public raks::Ctx {};

extern "C" int raks_query_noalloc(raks_ctx* c, const raks_query_desc* q, raks_results_buf* out) {
  if (!c || !q || !out) return fail(RAKS_EINVAL, "NULL argument");
  if (out->cap_results < 0 || out->cap_nodes < 0 || out->cap_arcs < 0 ||
      (out->cap_results > 0 && !out->r) || (out->cap_nodes > 0 && !out->nodes) ||
      (out->cap_arcs > 0 && !out->arcs))
    return fail(RAKS_EINVAL, "output capacities must be >= 0, with non-NULL arrays where > 0");
  out->n = 0;
  out->status = 0;
  out->n_nodes = out->n_arcs = 0;
  memset(&out->stats, 0, sizeof(out->stats));
  if (c->serve.running) return fail(RAKS_ESTATE, "serving is running: use raks_submit");
  if (!c->na_lane || !c->na_scratch) return fail(RAKS_ESTATE, "allocation-free lane not set up");
  HIP_OK(hipSetDevice(c->device));
  Lane* L = c->na_lane.get();
  // the scratch keeps the last call's contents: every buffer is carved anew
  // from its start and initialised by the query's own kernels, and the
  // recovery capacities restart from the context's initial values
  for (DevBuf* b : lane_buffers(L)) *b = DevBuf();
  L->lab_dirty = true;
  for (RecPhase& P : L->ph) {
    P.grown = true;
    P.dirty = true;
  }
  Arena a;
  a.base = static_cast<uint8_t*>(c->na_scratch);
  a.cap = c->na_scratch_bytes;
  int rc;
  {
    ArenaScope scope(&a);
    rc = query_on_lane_into(L, q, out);
  }
  if (rc != RAKS_OK) {
    out->n = 0;
    (void)hipStreamSynchronize(L->stream);   // nothing of a failed call keeps running
  }
  return rc;
}
