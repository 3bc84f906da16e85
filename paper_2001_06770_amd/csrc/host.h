// host.h -- host runtime pieces shared by the single-query path (api.hip)
// and the cohort engine (engine.hip): errors, device memory, query plans,
// recovery phases, result collection.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "runtime.h"

namespace raks {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
double now_ms();

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(RAKS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

#define RAKS_TRY(expr)              \
  do {                              \
    int _rc = (expr);               \
    if (_rc != RAKS_OK) return _rc; \
  } while (0)

// Device scratch of the allocation-free entry point.  While a thread has one
// set, dev_alloc carves its buffers from it (256-byte aligned, bump order)
// instead of allocating, and fails with RAKS_ENOMEM once it is used up.
struct Arena {
  uint8_t* base = nullptr;
  size_t cap = 0, used = 0;
};
extern thread_local Arena* g_arena;

int dev_alloc(Ctx* c, DevBuf& b, size_t bytes);
void dev_free(Ctx* c, DevBuf& b);
uint32_t timing_mask(const Lane* L);   // the context's timing mask; 0 on the allocation-free lane
DevGraphView graph_view(const Ctx* c, const AlphaView& v);
DevGraphView graph_view(const Lane* L);
int ensure_lanes(Ctx* c, int n);
int lane_create(Ctx* c, int id, Lane** out);
void lane_destroy(Ctx* c, Lane* L);
std::vector<DevBuf*> lane_buffers(Lane* L);   // every device buffer of a lane but its status
bool view_ready(Ctx* c, double alpha);        // levels for this query alpha exist (no build needed)
void harvest_timing(Lane* L);

struct QueryPlan {
  int C, M, TPc, TPm, k, w, L, gn, gd;
  double alpha;   // 0: the context's
  int score_mode, rerank;
  int n_build;    // RPGs recovered: k, or w when equal scores are re-ranked
  std::vector<int32_t> central, marginal;
};

int tp_for(int T);   // row bytes (4, 8 or 16) of a hitting-level matrix for T keywords
int validate_query(Ctx* c, const raks_query_desc* q, QueryPlan& p);

// activation levels (Eqs. 1-3) of every value in [lo, hi], built on the host
constexpr uint64_t kMaxLevelTable = 1ull << 28;
int level_of_x(double x, double abar, double alpha);
void level_table(int mode, int64_t lo, int64_t hi, double abar, double alpha, uint8_t* out);
SeedList seeds_for(Ctx* c, const std::vector<int32_t>& kws);
int ensure_small_buffers(Lane* L);
int query_on_lane(Lane* L, const raks_query_desc* q, raks_results** out);
// the same with results copied into a caller's buffers instead (raks_query_noalloc)
int query_on_lane_into(Lane* L, const raks_query_desc* q, raks_results_buf* out);
int noalloc_setup(Ctx* c);   // raks_create: the device's scratch address and the lane

// recovery phases (Algorithm 2): [0] central graphs, [1] radial pattern graphs
void phase_reset(const Ctx* c, RecPhase& P, int n_res, int T);
void phase_reset(RecPhase& P, int n_res, int T, uint32_t nc0, uint32_t ac0, uint32_t lc0);
int ensure_recovery(Lane* L, const QueryPlan& p);
int grow_phase(Lane* L, int ph, int n_valid, int max_layer);
RecoverView recover_view(Lane* L, int ph, const uint8_t* H, int TP, const int32_t* n_valid,
                         int max_layer);
FinalizeView finalize_view(Lane* L, int ph, const int32_t* n_valid, int C, const uint8_t* Hc,
                           int TPc);
int big_finalize(Lane* L, int ph, const QueryPlan& p, int n_res, const uint8_t* Hc, int TPc);
int collect(Lane* L, const QueryPlan& p, raks_results** out, int* ovf);
int collect_into(Lane* L, const QueryPlan& p, raks_results_buf* out, int* ovf);
void fill_stats(Lane* L, const QueryPlan& p, const Status& hs, raks_query_stats* st,
                int32_t* status);
void launch_query_reset(Status* st, hipStream_t s);
void launch_retry_reset(Status* st, hipStream_t s);
RankView rank_view(Lane* L, const QueryPlan& p);

// the cohort engine (engine.hip)
int cohort_query_batch(Ctx* c, const raks_query_desc* qs, int32_t n, raks_results** outs);
int cohort_serve_start(Ctx* c, int32_t queue_cap);
int cohort_submit(Ctx* c, const raks_query_desc* q, uint64_t* ticket);
void cohort_serve_stop(Ctx* c);
void cohort_destroy(Ctx* c);

}  // namespace raks
