// cohort.h -- many queries explored together (the batched and served path).
//
// A cohort holds up to kCoSlots queries at once in one node x column
// hitting-level matrix of kCoCols columns, split into kCoSegs segments of 16
// columns (segment-major: segment s is an [n_pad][16] byte array, so a level
// reads only the segments whose columns still expand).  A query owns the
// contiguous columns [c0, c0 + |C| + |M|) of one segment: its central keywords
// first, then its marginal keywords.  Both of its runs (Section 4.1) advance
// in the same level loop (the marginal search does not depend on the central
// graphs, Section 4.2.3), every query at its own local level: a query admitted
// at cohort level s is at local level L - s when the cohort is at level L, and
// its hitting levels are stored in local units, exactly the values the
// single-query path writes.  One frontier scan, one control step and one
// expansion per cohort level serve every query; an arc of a frontier node is
// read once for all queries that expand the node.
#pragma once

#include "common.h"
#include "kernels.h"

namespace raks {

constexpr int kCoCols = 64;
constexpr int kCoSegs = kCoCols / 16;
constexpr int kCoSlots = 32;
constexpr int kCoMaxLevel = 125;   // hitting levels are kept below 127 (7-bit compares)

// One query slot, in device memory.  The host writes it at admission; the
// control step of every level updates the run fields.
struct CoSlot {
  int32_t active;        // holds a query
  int32_t seg, c0;       // segment and first column of the query in it
  int32_t C, M;          // central / marginal keyword counts
  int32_t start;         // cohort level of admission (local level = L - start)
  int32_t max_level, w, k, gn, gd, score_mode, rerank;
  int32_t m_block;       // the marginal run blocks complete rows (|M| >= 2)
  // run state
  int32_t c_run, m_run;          // the run still expands
  int32_t c_end, c_reason;       // central run: end level and reason
  int32_t m_xend, m_xreason;     // marginal exploration ended (empty frontier / level bound)
  int32_t m_end, m_reason;       // marginal run's end once decided (-1: not yet)
  int32_t checked;               // marginal levels whose stop rule is decided
  int32_t vc_ready;              // the CGs' V_C lists are in place
  int32_t nsel;                  // selected CGs (valid once vc_ready)
  uint32_t ncand;                // central nodes identified so far
  int32_t pad0;
  // the query's post-processing buffers (its lane)
  const int32_t* sel_sc;
  const uint32_t* vc_off;
  const int32_t* vc_nodes;
  int32_t* has_rpg;
  int32_t* sm;
  int64_t* key;
  uint8_t* dmin;
};

// What the host learns of a slot after each level (pinned memory).
struct CoSlotMirror {
  int32_t active, c_run, m_run, c_end, c_reason, m_xend, m_xreason, m_end, m_reason, checked,
      vc_ready, nsel;
  uint32_t ncand;
  int32_t pad;
  uint64_t seq;
};

// One level's status.  Level l writes section l % kCoMirrors: the host reads
// level l while up to kCoAhead later levels are already queued, so fewer
// sections could be overwritten before the host saw them.
struct CoLevelMirror {
  uint32_t W, nq;
  uint32_t pad[2];
  uint64_t seq;
  uint64_t pad2;
  CoSlotMirror slot[kCoSlots];
};

constexpr int kCoAhead = 2;     // levels the host keeps queued beyond the one it reads
constexpr int kCoMirrors = 4;   // > kCoAhead, a power of two

struct CoMirror {
  CoLevelMirror lvl[kCoMirrors];
  // outcome of each slot's central-graph stage (recovery overflow bits, nsel)
  int32_t cg_ovf[kCoSlots];
  int32_t cg_nsel[kCoSlots];
  uint64_t cg_seq[kCoSlots];
};

// Per-level accumulators of the frontier scan, double-buffered by level
// parity: bit 2q (2q+1) of gfront is set when slot q's central (marginal)
// run has a frontier node; ncand counts each slot's central nodes.
struct CoAcc {
  unsigned long long gfront[2];
  uint32_t ncand[2][kCoSlots];
};

// A staged expansion entry: the node's examined arcs are the level-sorted row
// positions [arc, arc + work); columns in nmask expand over arcs of level <=
// their query's level, columns in omask only over arcs of exactly that level.
struct CoEntry {
  uint32_t pre;    // exclusive prefix of examined arcs within the scan workgroup
  uint32_t arc;    // first examined arc
  uint32_t nlo, nhi, olo, ohi;
};

struct CohortView {
  int32_t n, n_pad;
  int32_t nblocks, cpw;          // scan workgroups and 1024-node chunks per workgroup
  uint8_t* H;                    // [kCoSegs][n_pad][16]
  unsigned long long* R;         // [n_pad] reached mask: bit c set iff column c expands and
                                 // its hitting level is finite at the start of the level;
                                 // entries of rbytes bytes (the cohort's width / 8)
  int32_t rbytes;                // 2, 4 or 8: the cohort uses the first rbytes / 2 segments
  CoSlot* slots;                 // [kCoSlots]
  CoAcc* acc;
  uint2* tot;                    // [nblocks] per scan workgroup: entries, examined arcs
  uint32_t* wpre;                // [nblocks + 1] exclusive prefix of examined arcs
  uint32_t* qpre;                // [nblocks + 1] exclusive prefix of entries
  uint32_t* wtot;                // [2] arcs and entries of the level
  CoEntry* stage;                // [n_pad] entries, in each scan workgroup's node range
  CoMirror* mirror;              // device address of the pinned mirror
  uint32_t* dmin;                // [kCoSlots][kMaxW][kMaxKw] running minima of the marginal
                                 // levels over each CG's V_C (the RPG check's D_j)
};

// Candidate keys of one slot's central run (CG selection after the run).
struct CoCandView {
  const uint8_t* Hc;             // segment base + c0 (stride 16)
  int32_t C, end;                // central keywords, end level of the central run
  uint32_t* cnt;                 // [nblocks] last-level candidates per workgroup
  uint32_t* off;                 // [nblocks] their offsets
  uint32_t* cursor;              // [2]: earlier-level candidates placed / counted
  uint64_t* cand;                // keys: earlier levels first, then the last level in node order
  RunStatus* st;                 // receives ncand_total / ncand_level for the selection
  const int32_t* orig_id;        // internal id -> original id (the keys' node ids)
};

// End of a query's exploration: the work counters of both runs from its
// final hitting levels, its columns copied out to its lane (rows of TPq = 4, 8
// or 16 bytes, the smallest that holds its |C| + |M| levels: its levels first,
// then INF) and reset to INF in the cohort matrix.
struct CoFinishView {
  uint8_t* seg;                  // the query's segment [n_pad][16]
  int32_t c0, C, M, m_block;
  int32_t n_pad;
  int32_t TPq;                   // row bytes of the copy
  const CoSlot* slot;            // end levels
  Status* gst;                   // the lane's status: run[0], run[1] counters
  uint8_t* Hq;                   // the lane's copy [n_pad][TPq]
};

void launch_co_init(const CohortView& v, hipStream_t s);
void launch_co_admit(const CohortView& v, const CoSlot* slots, const int32_t* idx, int n,
                     hipStream_t s);
void launch_co_seed(const CohortView& v, int seg, int c0, const int32_t* kw_nodes,
                    const SeedList& seeds, hipStream_t s);
void launch_co_scan(const CohortView& v, const DevGraphView& g, int level, hipStream_t s);
void launch_co_control(const CohortView& v, int level, uint64_t seq, hipStream_t s);
// tile: examined arcs per expansion tile (512, 1024 or 2048)
void launch_co_expand(const CohortView& v, const DevGraphView& g, int level, int grid, int tile,
                      hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// CG selection input of slot q (three launches), then the selection kernel
void launch_co_cand(const CoCandView& cv, const CohortView& v, hipStream_t s);
// After slot q's CG recovery: V_C ready unless a recovery capacity ran out
void launch_co_cg_done(const CohortView& v, int q, const Status* gst, uint64_t seq,
                       hipStream_t s);
// Final marginal decision (Theorem 4 replayed up to the exploration's end)
void launch_co_rpg_final(const CohortView& v, int q, hipStream_t s);
// D_j minima over V_C for every slot whose marginal run is checked (q < 0), or
// for slot q alone; many workgroups, before the control step reads them
void launch_co_dmin(const CohortView& v, int q, int grid, hipStream_t s);
void launch_co_finish(const CoFinishView& fv, const DevGraphView& g, hipStream_t s);

}  // namespace raks
