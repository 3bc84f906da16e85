// kernels.h -- views passed to the kernels and the host-side launchers.
#pragma once

#include "common.h"

namespace raks {

struct DevGraphView {
  int32_t n;
  uint32_t A;
  const uint32_t* row_ptr;  // [n+1]
  const int32_t* col;       // [A]
  const uint16_t* label;    // [A]
  const uint8_t* act;       // [A] activation level per arc
  const uint8_t* act_node;  // [n] NODE mode, else nullptr
  int32_t mode;             // 0 EDGE, 1 NODE
};

// State of one exploration run (Section 4.2), laid out for one query.
struct RunView {
  int32_t kind;          // RUN_CENTRAL / RUN_MARGINAL
  int32_t T;             // keywords of the run
  uint32_t tmask;        // (1 << T) - 1
  int32_t block_rule;    // 1: a node reached by every keyword stops expanding (CF)
  uint8_t* H;            // node-keyword matrix [n_pad][TP]; INF = 0xFF, padding bytes 0
  uint8_t* F;            // frontier flags [n_pad]
  int32_t n_pad;         // n rounded up to kScanNodes
  RunStatus* st;
  ScanTot* tot;          // [nblocks]
  ScanOff* off;          // [nblocks]
  int32_t nblocks;
  int32_t* q_node;       // expansion queue: node
  uint32_t* q_off;       // exclusive prefix of degrees [nactive+1]
  uint32_t* q_rs;        // row start of the node
  uint32_t* q_mask;      // keywords the node expands for
  uint64_t* cand;        // central run: identified central nodes (S<<48 | sum<<32 | node)
  int32_t max_level;
  int32_t w, k, gamma_num, gamma_den;
  // marginal run: RPG identification over the selected CGs
  int32_t nsel;
  const int32_t* sel_sc;     // [nsel] S^c of the selected CGs, in CG rank order
  const uint32_t* vc_off;    // [nsel+1]
  const int32_t* vc_nodes;   // central-keyword nodes of each CG
  int32_t* has_rpg;          // [nsel]
  int32_t* sm;               // [nsel]
  int64_t* key;              // [nsel]
  uint8_t* dmin;             // [nsel][kMaxKw]
};

struct SeedList {
  uint32_t start[kMaxKw];   // offset into kw_nodes
  uint32_t count[kMaxKw];
  uint32_t prefix[kMaxKw + 1];
  int32_t T;
};

struct SelectView {
  const uint64_t* cand;
  RunStatus* st;
  Status* gst;
  int32_t w;
  int32_t* sel_node;   // [w]
  int32_t* sel_sc;     // [w]
  int32_t* sel_sumh;   // [w]
};

struct RankView {
  Status* gst;
  int32_t nsel, M, k, gamma_num, gamma_den;
  const int32_t* sel_sc;
  int32_t* has_rpg;
  int32_t* sm;
  int64_t* key;
  int32_t* ranked;     // [k] CG rank of result t
};

// Recovery (Algorithm 2) of one (result, keyword) instance per workgroup.
struct RecoverView {
  DevGraphView g;
  const uint8_t* H;
  int32_t TP;
  int32_t T;            // keywords per result (instances per result)
  int32_t marginal;     // 0: start at the central node; 1: start at V_C nodes at distance D_j
  int32_t n_inst;
  const int32_t* sel_node;   // central node of CG r
  const int32_t* ranked;     // marginal: CG rank of result t
  const uint32_t* vc_off;
  const int32_t* vc_nodes;
  const uint8_t* dmin;       // [nsel][kMaxKw]
  uint32_t* ht;              // [n_inst][hc]
  int32_t* nl;               // [n_inst][nc]
  uint32_t* al;              // [n_inst][ac]
  uint32_t* cnt;             // [n_inst][2]: nodes, arcs
  uint32_t hc, nc, ac;
  Status* gst;
};

// Union, sort and unique per result.
struct FinalizeView {
  DevGraphView g;
  int32_t T;                 // instances per result
  int32_t marginal;          // 1: merge the CG lists of ranked[t] first
  int32_t n_res;
  const int32_t* sel_node;
  const int32_t* ranked;
  const int32_t* nl;
  const uint32_t* al;
  const uint32_t* cnt;
  uint32_t nc, ac;
  // CG lists (written when marginal == 0, read when marginal == 1)
  uint32_t* cg_nodes;        // [nsel][cg_ncap]
  uint32_t* cg_arcs;         // [nsel][cg_acap]
  uint32_t* cg_cnt;          // [nsel][2]
  uint32_t cg_ncap, cg_acap;
  // V_C (marginal == 0): nodes with some central hitting level 0
  const uint8_t* Hc;
  int32_t TPc, Tc;
  uint32_t* vc_cnt;          // [nsel]
  int32_t* vc_tmp;           // [nsel][cg_ncap]
  // sort scratch, per workgroup
  uint32_t* sort_a;          // [n_res][scap]
  uint32_t* sort_b;
  uint32_t scap;
  // final output (marginal == 1 or no marginal keywords)
  int32_t write_output;
  ResultHdr* hdr;
  int32_t* out_nodes;
  int32_t* out_arcs;         // (src, dst, label) triples
  uint32_t out_ncap, out_acap;
  const int32_t* sel_sc;
  const int32_t* sm;
  const int64_t* key;
  Status* gst;
};

// Position of arc (src -> dst, lab) in row src (rows sorted by (label, dst)),
// or kEmpty when absent.
__device__ inline uint32_t find_arc_dev(const uint32_t* row_ptr, const int32_t* col,
                                        const uint16_t* label, int32_t src, uint16_t lab,
                                        int32_t dst) {
  uint32_t a = row_ptr[src], b = row_ptr[src + 1];
  const uint32_t hi = b;
  while (a < b) {
    uint32_t m = (a + b) >> 1;
    if (label[m] < lab || (label[m] == lab && col[m] < dst)) a = m + 1; else b = m;
  }
  return (a < hi && label[a] == lab && col[a] == dst) ? a : kEmpty;
}

__device__ inline uint32_t row_of(const uint32_t* row_ptr, int32_t n, uint32_t e) {
  return (uint32_t)upper_index<uint32_t>(row_ptr, 0, n + 1, e);
}

void launch_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp, uint32_t cg_ncap, int32_t nsel,
                    uint32_t* vc_off, int32_t* vc_nodes, hipStream_t s);
void launch_check_and_count(const DevGraphView& g, uint32_t* c_tmp, Status* st, hipStream_t s);
void launch_act_edge(const DevGraphView& g, const uint32_t* c_tmp, const Status* st, double abar,
                     double alpha, uint8_t* act, hipStream_t s);
void launch_act_node(const DevGraphView& g, const uint8_t* nw, Status* st, double abar,
                     double alpha, uint8_t* act_node, uint8_t* act, hipStream_t s);

void launch_run_init(const RunView& r, int TP, int32_t n, const int32_t* kw_nodes,
                     const SeedList& seeds, hipStream_t s);
void launch_front_count(const RunView& r, int TP, const DevGraphView& g, int level, hipStream_t s);
void launch_front_control(const RunView& r, int TP, int level, hipStream_t s);
void launch_front_write(const RunView& r, int TP, const DevGraphView& g, int level, hipStream_t s);
void launch_expand(const RunView& r, int TP, const DevGraphView& g, int level, int grid,
                   hipStream_t s);
void launch_count_writes(const RunView& r, int TP, int32_t n, hipStream_t s);
void launch_select(const SelectView& v, hipStream_t s);
void launch_rank(const RankView& v, hipStream_t s);
void launch_recover(const RecoverView& v, hipStream_t s);
void launch_finalize(const FinalizeView& v, hipStream_t s);

}  // namespace raks
