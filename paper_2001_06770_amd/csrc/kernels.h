// kernels.h -- views passed to the kernels and the host-side launchers.
#pragma once

#include "common.h"

namespace raks {

// Two numberings of the nodes.  The caller's ("original") ids and CSR
// positions are kept for everything that leaves the library and for the
// load-time checks; the search runs on internal ids that order the nodes by
// degree (largest first), so the hitting levels and reached masks of the
// nodes that most arcs point to share a few cache lines.
struct DevGraphView {
  int32_t n;
  uint32_t A;
  const uint32_t* row_ptr;  // [n+1] internal rows (the traversal copy's row starts)
  const uint32_t* row_ptr_o;// [n+1] original rows
  const int32_t* orig_id;   // [n] internal id -> original id
  const int32_t* int_id;    // [n] original id -> internal id
  const int32_t* col;       // [A] original CSR: destination (original id)
  const uint16_t* label;    // [A] original CSR
  const uint8_t* act;       // [A] activation level per arc, original CSR order
  const uint8_t* act_node;  // [n] NODE mode, by internal id, else nullptr
  int32_t mode;             // 0 EDGE, 1 NODE
  // traversal copy, internal rows: each row's arcs ordered by activation level
  const int32_t* col_s;     // [A] destination (internal id)
  const uint8_t* act_s;     // [A]
  const uint32_t* eid_s;    // [A] original CSR position of the arc
  const int32_t* arc_src;   // [A] source node of each arc (original id, original CSR order)
  const uint32_t* rev;      // [A] original CSR position of each arc's reverse arc
  const uint8_t* row_amax;  // [n_pad] largest activation level of the row, internal ids (0 if
                            // empty; 0 past n, up to a multiple of kScanNodes)
  const uint32_t* bnd;      // [nbnd][n] arcs of the internal row with level <= l, l < nbnd
                            // (level-major: a level's counts of all nodes are contiguous)
  int32_t nbnd;             // levels covered by bnd (1..16)
};

// Number of arcs of row v with activation level <= x (x may be negative).
__device__ inline uint32_t count_le(const DevGraphView& g, int32_t v, int x) {
  if (x < 0) return 0;
  const uint32_t rs = g.row_ptr[v], re = g.row_ptr[v + 1];
  if (x >= (int)g.row_amax[v]) return re - rs;
  if (x < g.nbnd) return g.bnd[(size_t)x * g.n + v];
  uint32_t a = rs, b = re;
  while (a < b) {
    const uint32_t m = (a + b) >> 1;
    if ((int)g.act_s[m] <= x) a = m + 1; else b = m;
  }
  return a - rs;
}

// State of one exploration run (Section 4.2), laid out for one query.
struct RunView {
  int32_t kind;          // RUN_CENTRAL / RUN_MARGINAL
  int32_t T;             // keywords of the run
  uint32_t tmask;        // (1 << T) - 1
  int32_t block_rule;    // 1: a node reached by every keyword stops expanding (CF)
  uint8_t* H;            // node-keyword matrix [n_pad][TP]; INF = 0xFF, padding bytes 0
  void* R;               // reached-keyword mask per node [n_pad] (4 bits, two nodes per byte,
                         // when TP == 4; u8 when TP == 8; u16 when TP == 16): bit i set
                         // iff h_vi is finite at the start of the level
  int32_t n_pad;         // n rounded up to kScanNodes
  RunStatus* st;
  ScanTot* tot;          // [nblocks]
  uint32_t* sb;          // [2][kScanGroups / 64][3] sums of nq, work, ncand per 64 scan
                         // workgroups, double-buffered by level parity
  int32_t nblocks;       // frontier-scan workgroups
  int32_t cpw;           // kScanNodes-chunks per scan workgroup
  uint4* s_item;         // [n_pad] staged queue entries (local arc prefix, rs, lo, mask)
  uint64_t* s_cand;      // [n_pad] staged central-node keys
  uint32_t* q_off;       // expansion queue: exclusive prefix of examined arcs [nactive+1]
  uint32_t* q_rs;        // first examined arc (position in the level-sorted row)
  uint32_t* q_lo;        // from here on the arcs have level == l: old keywords join
  uint32_t* q_mask;      // keywords reached at level l | keywords reached before << 16
  uint32_t* tile_first;  // [A / kExpandTile + 2] queue entry holding each expansion tile's
                         // first arc (| kTileAtEntry when the tile starts with the entry)
  uint64_t* cand;        // central run: identified central nodes (S<<48 | sum<<32 | original id)
  int32_t max_level;
  int32_t w, k, gamma_num, gamma_den;
  int32_t score_mode;        // 0: Eq. 6, 1: S^c * S^m
  int32_t rerank;            // 1: ties re-ranked by the arcs' level sum (Theorem 4 strict)
  // marginal run: RPG identification over the selected CGs
  const int32_t* nsel;       // device: number of selected CGs (marginal run)
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
  const int32_t* int_id;    // original id (in the keys) -> internal id
  const uint64_t* cand;
  RunStatus* st;
  Status* gst;
  int32_t w;
  int32_t* sel_node;   // [w] internal ids
  int32_t* sel_sc;     // [w]
  int32_t* sel_sumh;   // [w]
};

struct RankView {
  Status* gst;
  const int32_t* nsel;       // device: number of selected CGs
  int32_t M, k, gamma_num, gamma_den;
  int32_t score_mode, rerank;
  const int32_t* sel_sc;
  int32_t* has_rpg;
  int32_t* sm;
  int64_t* key;
  int32_t* ranked;     // [k] (re-ranking: [w]) CG rank of result t
};

// Recovery (Algorithm 2) of every (result, keyword) instance of a phase at
// once, layer by layer (hitting level h from the largest down to 1).
struct RecItem {
  uint32_t inst;   // instance = result * T + keyword column
  int32_t q;       // node whose in-arcs are examined
  uint32_t start;  // first arc of the chunk (CSR position in q's row)
  uint32_t len;    // arcs in the chunk (<= kRecChunk)
};

constexpr uint32_t kRecChunk = 256;

// Storage of one recovery instance.  Its node set is an open-addressing table
// of hcap slots, or (dense) a bitmap of n bits; its node and arc lists hold
// ncap / acap entries.  Counts continue past the capacities, so after an
// overflow the host knows (or bounds from below) what the instance needs.
struct InstCap {
  uint64_t hoff;   // node set at hpool + hoff
  uint64_t noff;   // node list at nl + noff
  uint64_t aoff;   // arc list at al + aoff
  uint32_t hcap, ncap, acap, dense;
};

struct RecoverView {
  DevGraphView g;
  const uint8_t* H;
  int32_t TP;
  int32_t T;            // keywords per result (instances per result)
  int32_t marginal;     // 0: start at the central node; 1: start at V_C nodes at distance D_j
  int32_t n_inst;            // launched instances: results x T
  const int32_t* n_valid;    // device: results that exist (instances of later ones exit)
  const int32_t* sel_node;   // central node of CG r
  const int32_t* ranked;     // marginal: CG rank of result t
  const uint32_t* vc_off;
  const int32_t* vc_nodes;
  const uint8_t* dmin;       // [nsel][kMaxKw]
  const InstCap* caps;       // [n_inst]
  uint32_t* hpool;           // node sets
  int32_t* nl;               // node lists
  uint32_t* al;              // arc lists (CSR position of n -> q)
  uint32_t* cnt;             // [n_inst][2] nodes / arcs found
  uint32_t* iflag;           // [n_inst] 1: the node table filled up (nodes were lost)
  uint32_t dwords;           // words of a dense node set
  RecItem* items;            // [max_layer + 1][lcap] work chunks per layer
  uint32_t* lcnt;            // [max_layer + 1] chunks requested per layer
  uint32_t lcap;
  int32_t max_layer;
  int32_t ovf_bit;           // bit set in gst->overflow when a capacity runs out
  Status* gst;
  // labelled mode: one search per keyword column serves up to 64 results
  int32_t labelled;
  int32_t G;                 // label words per node and column (results / 64, rounded up)
  uint64_t wipe_words;       // words of `lab` to clear first: all of its allocation when it
                             // may hold stale bits (new memory, lost labels), else 0
  uint64_t* lab;             // [T * G][n] result bits per node; zero outside a phase
  uint64_t* touch;           // [tcap] (column group << 32) | node, per labelled node
  uint32_t* tcnt;            // entries of `touch` requested (counted past tcap)
  uint32_t tcap;
};

// Union, sort and unique per result.
struct FinalizeView {
  DevGraphView g;
  int32_t T;                 // instances per result
  int32_t marginal;          // 1: merge the CG lists of ranked[t] first
  int32_t n_res;             // launched workgroups
  const int32_t* n_valid;    // device: results that exist
  const int32_t* sel_node;
  const int32_t* ranked;
  const InstCap* caps;       // [n_res * T]
  const int32_t* nl;
  const uint32_t* al;
  const uint32_t* cnt;
  // CG lists (written when marginal == 0, read when marginal == 1); CG r owns
  // cg_nodes / vc_tmp from cg_noff[r] and cg_arcs from cg_aoff[r]
  uint32_t* cg_nodes;
  uint32_t* cg_arcs;
  uint32_t* cg_cnt;          // [nsel][2]
  const uint64_t* cg_noff;
  const uint64_t* cg_aoff;
  // V_C (marginal == 0): nodes with some central hitting level 0
  const uint8_t* Hc;
  int32_t TPc, Tc;
  uint32_t* vc_cnt;          // [nsel]
  int32_t* vc_tmp;
  // sort scratch of result t: sort_a / sort_b from soff[t] to soff[t + 1]
  uint32_t* sort_a;
  uint32_t* sort_b;
  const uint64_t* soff;
  // final output (marginal == 1 or no marginal keywords)
  int32_t write_output;
  int32_t skip_bits;         // overflow bits that make this finalize pointless (phase repeats)
  uint32_t* big;             // [n_res] 1: the result's lists go to the bitmap path
  uint64_t big_list;         // lists longer than this take the bitmap path
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

// max_sel: an upper bound of the device-side nsel (one workgroup per CG)
void launch_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp, const uint64_t* cg_noff,
                    const int32_t* nsel, uint32_t* vc_off, int32_t* vc_nodes, int max_sel,
                    hipStream_t s);
void launch_check_and_count(const DevGraphView& g, uint32_t* c_tmp, int32_t* arc_src, uint32_t* rev,
                            Status* st,
                            hipStream_t s);
// act[e] = lut[c[e] - cmin] (lut: levels of the label counts, built on the host)
void launch_act_edge(const DevGraphView& g, const uint32_t* c_tmp, const uint8_t* lut,
                     uint64_t cmin, uint8_t* act, hipStream_t s);
void launch_sort_rows(const DevGraphView& g, int32_t* col_s, uint8_t* act_s, uint32_t* eid_s,
                      uint8_t* row_amax, uint32_t* bnd, int32_t nbnd, hipStream_t s);
// out[u] = in[orig_id[u]] for every internal id u (per-node arrays to internal order)
void launch_to_internal_u8(const DevGraphView& g, const uint8_t* in, uint8_t* out, hipStream_t s);
// ids[i] = int_id[ids[i]] (original node ids to internal ones, in place)
void launch_map_ids(const int32_t* int_id, int32_t* ids, uint64_t count, hipStream_t s);
// node weight range into st->cmin / st->cmax (NODE mode, once per graph)
void launch_node_weight_range(const DevGraphView& g, const uint8_t* nw, Status* st,
                              hipStream_t s);
// act_node[v] = lut[nw[v] - wmin]; act[e] = act_node[col[e]]
void launch_act_node(const DevGraphView& g, const uint8_t* nw, const uint8_t* lut, uint32_t wmin,
                     uint8_t* act_node, uint8_t* act, hipStream_t s);

void launch_run_init(const RunView& r, int TP, int32_t n, const int32_t* kw_nodes,
                     const SeedList& seeds, hipStream_t s);
void launch_front_count(const RunView& r, int TP, const DevGraphView& g, int level, hipStream_t s);
// The level's control step and Frontier Enqueue in one launch.  mirror:
// device-visible pinned host memory that receives the level's status,
// stamped with seq once the rest of it is visible to the host.
void launch_front_enqueue(const RunView& r, int TP, int level, RunStatus* mirror, uint64_t seq,
                          hipStream_t s);
// ev0 / ev1 (optional): events that receive the kernel's start and end times
void launch_expand(const RunView& r, int TP, const DevGraphView& g, int level, int grid,
                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_select(const SelectView& v, hipStream_t s);
void launch_rank(const RankView& v, hipStream_t s);
// Re-ranking of equal scores by the arcs' level sum; keeps the first k.
void launch_rerank(ResultHdr* hdr, Status* gst, int32_t k, hipStream_t s);
void launch_recover(const RecoverView& v, hipStream_t s);   // all layers of one phase
void launch_finalize(const FinalizeView& v, hipStream_t s);

// Results to pinned host memory (device addresses of the host buffers).
struct CollectView {
  const Status* st;
  const ResultHdr* hdr;
  uint32_t n_hdr;                    // headers to copy
  const uint32_t* nodes;             // output arena, 1 word per node
  const uint32_t* arcs;              // output arena, 3 words per arc
  uint32_t cap_nodes, cap_arcs;      // what the host buffers hold (and the arena has)
  Status* h_st;
  ResultHdr* h_hdr;
  uint32_t* h_nodes;
  uint32_t* h_arcs;
};
constexpr int kCollectGroups = 64;
void launch_collect(const CollectView& v, hipStream_t s);
// Bitmap path for result t (flagged in v.big): bm holds max(n, A) bits, chunk
// one count per kBigChunk words, slot one 64-bit list start.
void launch_big_finalize(const FinalizeView& v, int t, uint32_t* bm, uint32_t* chunk, uint64_t* slot,
                         hipStream_t s);

}  // namespace raks
