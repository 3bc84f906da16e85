// explore.hip -- exploration phase (Section 4.2) on gfx950.
//
// One level of a run is three launches:
//   k_front_count   frontier scan: every workgroup takes a run of 1024-node
//                   chunks (4 nodes per thread), reads their H rows and row
//                   levels in node order, decides frontier membership from
//                   them, inspects every frontier node once (complete row ->
//                   central node / PTC block, keywords with h <= level, level
//                   slice of the row), stages its queue entry and central-node
//                   key in node order and refreshes its reached mask; then
//                   writes its totals;
//   k_front_enqueue workgroup 0 sums the totals, applies the run's
//                   identification and termination rules (Theorem identifyCG,
//                   >= w CGs; the RPG check over each CG's V_C rows and
//                   Theorem 4) and decides whether this level expands; the
//                   other workgroups, one per scan workgroup, do Frontier
//                   Enqueue: they copy the staged entries to the expansion
//                   queue (node order, arc prefix) and the central nodes to
//                   the candidate list;
//   k_expand        Algorithm 1 for every (frontier, arc) pair, balanced by
//                   arcs: each workgroup takes tiles of 1024 consecutive arcs
//                   of the concatenated frontier rows, so a hub's arcs spread
//                   over many workgroups; one H-row gather serves all keywords
//                   of the frontier at once.
// Writes need no atomics (Theorem "lockfree"): every H write of a level
// stores level+1 into a byte that was INF.  Neither the frontier flags nor
// the joining flag array is stored, both are implied by H: a node is blocked
// exactly when its row is complete, and it is identified at the level equal
// to its row maximum.
#include <hip/hip_ext.h>

#include <climits>

#include "common.h"
#include "kernels.h"

namespace raks {

template <int TP> struct RowVec;
template <> struct RowVec<4> { using T = uint32_t; };
template <> struct RowVec<8> { using T = uint2; };
template <> struct RowVec<16> { using T = uint4; };

// Per-node mask of the keywords whose hitting level is finite: 4 bits per
// node for up to 4 keywords (two nodes per byte, so the array that every
// expansion gathers from is half as large), 8 or 16 bits otherwise.  W holds
// the masks of the kScanPer consecutive nodes of one scan thread.
template <int TP> struct RMask { using T = uint8_t; };
template <> struct RMask<16> { using T = uint16_t; };
template <int TP> using RMaskT = typename RMask<TP>::T;

template <int Bits> struct UintOf;
template <> struct UintOf<8> { using T = uint8_t; };
template <> struct UintOf<16> { using T = uint16_t; };
template <> struct UintOf<32> { using T = uint32_t; };
template <> struct UintOf<64> { using T = uint64_t; };

template <int TP> struct RBits {
  static constexpr int kBits = TP == 4 ? 4 : (TP == 8 ? 8 : 16);   // bits per node
  using W = typename UintOf<kBits * kScanPer>::T;
  __device__ static uint32_t get(const void* R, int64_t v) {
    if constexpr (kBits == 4)
      return (reinterpret_cast<const uint8_t*>(R)[v >> 1] >> ((v & 1) * 4)) & 0xFu;
    else if constexpr (kBits == 8)
      return reinterpret_cast<const uint8_t*>(R)[v];
    else
      return reinterpret_cast<const uint16_t*>(R)[v];
  }
  // the word of node v's scan thread (v a multiple of kScanPer)
  __device__ static W* group(void* R, int64_t v) {
    return reinterpret_cast<W*>(reinterpret_cast<uint8_t*>(R) + v * kBits / 8);
  }
  __device__ static uint32_t unpack(W w, int k) {
    return (uint32_t)(w >> (kBits * k)) & ((1u << kBits) - 1u);
  }
  __device__ static W pack(const uint32_t (&m)[kScanPer]) {
    W w = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) w |= (W)(m[k] & ((1u << kBits) - 1u)) << (kBits * k);
    return w;
  }
};

template <int TP>
__device__ inline void load_row(const uint8_t* H, int64_t v, uint8_t (&b)[TP]) {
  using V = typename RowVec<TP>::T;
  V x = *reinterpret_cast<const V*>(H + v * TP);
  __builtin_memcpy(b, &x, TP);
}

// ------------------------------------------------------------- run init ---

// A run with a keyword that has no node ends before level 0; the marginal
// run does not run at all when the central run selected no CG.
__global__ void k_run_reset(RunStatus* st, int32_t empty, const int32_t* nsel, uint32_t* sb) {
  for (int i = 0; i < 2 * kSupers * 3; ++i) sb[i] = 0;
  RunStatus s = {};
  const bool skip = nsel != nullptr && *nsel == 0;
  s.end_level = (skip || empty) ? -1 : INT32_MAX;
  s.end_reason = skip ? END_NONE : (empty ? END_EMPTY_KEYWORD : END_NONE);
  *st = s;
}

template <int TP>
__global__ __launch_bounds__(kBlock) void k_init_rows(uint8_t* H, RMaskT<TP>* R, int32_t n,
                                                      int32_t n_pad, int32_t T) {
  uint8_t b[TP];
#pragma unroll
  for (int i = 0; i < TP; ++i) b[i] = i < T ? kInf : 0;
  typename RowVec<TP>::T pat;
  __builtin_memcpy(&pat, b, TP);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n_pad; v += stride) {
    reinterpret_cast<typename RowVec<TP>::T*>(H)[v] = pat;
    R[v] = 0;
  }
}

template <int TP>
__global__ __launch_bounds__(kBlock) void k_seed(uint8_t* H, const int32_t* kw_nodes, SeedList s) {
  const uint32_t total = s.prefix[s.T];
  for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < total; p += gridDim.x * kBlock) {
    int i = 0;
    while (p >= s.prefix[i + 1]) ++i;
    const int32_t v = kw_nodes[s.start[i] + (p - s.prefix[i])];
    H[(int64_t)v * TP + i] = 0;   // keyword nodes are at distance 0: the first frontier
  }
}

// --------------------------------------------------------- frontier scan ---
//
// Work-efficient form of Algorithm 1 (same H, frontiers and counters).
// Algorithm 1 keeps a frontier f in the frontier after level l exactly when
// it expands and its row has an arc of level > l (an arc it could not cross
// yet): a property of the row, precomputed as row_amax.  A keyword i with h_fi < l expanded f at level l-1 over all arcs
// of level <= l-1, so only arcs of level exactly l can reach new nodes for it;
// a keyword with h_fi = l needs all arcs of level <= l.  With rows sorted by
// level these are the row slices [lo, hi) and [0, hi), read from the level
// table.
//
// No frontier flags are stored.  By induction over the levels, v is in the
// level-l frontier exactly when some keyword reached it at level l (the
// expansion set its flag), or it was reached before l, its row has an arc of level
// > l-1 and it was not blocked at l-1: from the level it is first reached on,
// a node stays a frontier for as long as it expands and keeps arcs of higher
// levels, and blocking (a complete row) never ends.  All of this is in the H
// row and row_amax, which the scan reads in node order.

// What one H row says at level l.
struct RowState {
  uint32_t mn, mo, rm;   // keywords with h == l / h < l / h finite
  uint32_t mx, sum;      // largest finite h and sum of finite h
  bool complete;         // every byte finite (padding bytes are 0)
};

template <int TP>
__device__ inline RowState row_state(const uint8_t (&b)[TP], uint32_t tmask, int level) {
  RowState st;
  st.complete = true;
  uint32_t mn = 0, mo = 0, mx = 0, sum = 0, rm = 0;
#pragma unroll
  for (int i = 0; i < TP; ++i) {
    const uint32_t h = b[i];
    const bool inf = h == kInf;
    st.complete &= !inf;
    rm |= (inf ? 0u : 1u) << i;
    if (h == (uint32_t)level) mn |= 1u << i;
    if (h < (uint32_t)level) mo |= 1u << i;
    mx = (!inf && h > mx) ? h : mx;
    sum += inf ? 0u : h;
  }
  st.mn = mn & tmask;
  st.mo = mo & tmask;
  st.rm = rm & tmask;
  st.mx = mx;
  st.sum = sum;
  return st;
}

__device__ inline bool in_frontier(const RowState& st, uint32_t tmask, uint32_t amax, int level,
                                   int block_rule) {
  if (st.mn) return true;   // reached at level l
  // reached before l, not complete by l-1 where blocking applies, and an arc
  // of level > l-1 left
  return st.mo != 0 && (int)amax > level - 1 && !(block_rule && st.mo == tmask);
}

struct NodeInfo {
  uint32_t mask_new, mask_old;  // keywords with h == level / h < level
  uint32_t deg;                 // row degree if the node expands (Algorithm 1 scans it)
  uint32_t rs, lo, hi, start;   // row start; arcs of level < l end at lo, <= l end at hi
  uint32_t work;                // hi - start if the node expands
  uint32_t hw;                  // entries written at the previous level
  uint32_t reached;             // keywords with a finite hitting level
  bool active, cand;
  uint64_t key;
};

// A frontier node at level l: central-node test, block rule and the slice of
// its row that the expansion examines.
__device__ inline NodeInfo inspect_node(const RunView& r, const DevGraphView& g, int32_t v,
                                        const RowState& st, uint32_t amax, int level) {
  NodeInfo o;
  o.mask_new = st.mn;
  o.mask_old = st.mo;
  o.reached = st.rm;
  o.hw = level >= 1 ? __popc(o.mask_new) : 0;
  const bool blocked = r.block_rule && st.complete;
  // the row bounds and both level-table entries in one round of loads (the
  // table entries are in bounds whenever their level is below nbnd)
  const int xl = level - 1, xh = level;
  const uint32_t blo = (xl >= 0 && xl < g.nbnd) ? g.bnd[(size_t)xl * g.n + v] : 0u;
  const uint32_t bhi = (xh < g.nbnd) ? g.bnd[(size_t)xh * g.n + v] : 0u;
  o.rs = g.row_ptr[v];
  const uint32_t d = g.row_ptr[v + 1] - o.rs;
  o.active = !blocked && (o.mask_new | o.mask_old) != 0 && d > 0;
  o.deg = o.active ? d : 0;
  o.cand = (r.kind == RUN_CENTRAL) && st.complete && st.mx == (uint32_t)level;
  o.key = ((uint64_t)st.mx << 48) | ((uint64_t)st.sum << 32) | (uint32_t)g.orig_id[v];
  o.lo = o.hi = o.start = o.work = 0;
  if (o.active) {
    // arcs of level <= x: none below 0, the whole row from its largest level
    // on, else the level table (or a search of the row past the table)
    o.lo = xl < 0 ? 0u : (xl >= (int)amax ? d : (xl < g.nbnd ? blo : count_le(g, v, xl)));
    o.hi = xh >= (int)amax ? d : (xh < g.nbnd ? bhi : count_le(g, v, xh));
    o.start = o.mask_new ? 0 : o.lo;
    o.work = o.hi - o.start;
  }
  return o;
}

// Every workgroup takes cpw consecutive chunks of kScanNodes nodes (kScanPer
// per thread), reads their H rows and levels in node order, inspects each
// frontier node once and, in node order, stages its queue entry and its
// central-node key in the workgroup's own slots of the staging arrays
// (slot = first node of the workgroup + local index).  It also refreshes the
// reached mask R of every frontier node: every node whose H row changed in
// the previous expansion is a frontier now, so R stays equal to H's finite
// set.
template <int TP>
__global__ __launch_bounds__(kBlock) void k_front_count(RunView r, DevGraphView g, int level) {
  if (level > r.st->end_level) return;
  __shared__ uint64_t s_multi[(kBlock / kWave + 1) * 5];
  __shared__ uint32_t s_m32[(kBlock / kWave + 1) * 3];
  const int64_t wg0 = (int64_t)blockIdx.x * r.cpw * kScanNodes;
  const int64_t wg1 = min(wg0 + (int64_t)r.cpw * kScanNodes, (int64_t)r.n_pad);
  uint32_t cq = 0, cc = 0, cw = 0;   // block-uniform running counts of the workgroup
  uint32_t nf = 0, hw = 0;
  uint64_t dg = 0, dk = 0, gt = 0;
  // the next chunk's rows and levels are loaded while this chunk is inspected
  using AmW = typename UintOf<8 * kScanPer>::T;   // the row levels of a thread's nodes
  uint8_t nrows[kScanPer][TP];
  uint32_t nam2 = 0;
  {
    const int64_t b0 = wg0 + threadIdx.x * kScanPer;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) load_row<TP>(r.H, b0 + k, nrows[k]);
    nam2 = *reinterpret_cast<const AmW*>(g.row_amax + b0);
  }
#pragma unroll 1
  for (int64_t c0 = wg0; c0 < wg1; c0 += kScanNodes) {
    const int64_t base = c0 + threadIdx.x * kScanPer;
    uint8_t rows[kScanPer][TP];
    __builtin_memcpy(rows, nrows, sizeof(rows));
    const uint32_t am2 = nam2;
    if (c0 + kScanNodes < wg1) {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) load_row<TP>(r.H, base + kScanNodes + k, nrows[k]);
      nam2 = *reinterpret_cast<const AmW*>(g.row_amax + base + kScanNodes);
    }
    uint32_t fw = 0;   // frontier bit per node
    // what the staging step needs of each node, kept across the block scan
    uint4 item[kScanPer];        // examined arcs (0: no queue entry), slice start, split, masks
    uint64_t key[kScanPer];
    uint32_t bits[kScanPer];     // reached mask | central node << 17
    uint32_t v[3] = {0, 0, 0};   // queue entries, central nodes, examined arcs
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      item[k] = make_uint4(0, 0, 0, 0);
      key[k] = 0;
      bits[k] = 0;
      const RowState st = row_state<TP>(rows[k], r.tmask, level);
      const uint32_t amax = (am2 >> (8 * k)) & 0xFFu;
      if (!in_frontier(st, r.tmask, amax, level, r.block_rule)) continue;
      fw |= 1u << k;
      const NodeInfo o = inspect_node(r, g, (int32_t)(base + k), st, amax, level);
      ++nf;
      hw += o.hw;
      if (o.active) {
        dg += o.deg;
        dk += (uint64_t)o.deg * __popc(o.mask_new | o.mask_old);
        gt += o.hi;
      }
      item[k] = make_uint4(o.work, o.rs + o.start, o.rs + o.lo, o.mask_new | (o.mask_old << 16));
      key[k] = o.key;
      bits[k] = o.reached | (o.cand ? 1u << 17 : 0u);
      v[0] += o.work != 0;
      v[1] += o.cand;
      v[2] += o.work;
    }
    uint32_t t[3];
    block_exclusive_scan_multi<3, kBlock, uint32_t>(v, t, s_m32);
    if (fw) {
      using RB = RBits<TP>;
      typename RB::W* rp = RB::group(r.R, base);
      const typename RB::W cur = *rp;
      uint32_t mk[kScanPer];
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) mk[k] = RB::unpack(cur, k);
      uint32_t q = cq + (uint32_t)v[0], cd = cc + (uint32_t)v[1], wk = cw + (uint32_t)v[2];
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        if (!((fw >> k) & 1u)) continue;
        mk[k] = bits[k] & 0xFFFFu;
        if (item[k].x) {
          const uint32_t work = item[k].x;
          item[k].x = wk;
          r.s_item[wg0 + q] = item[k];
          ++q;
          wk += work;
        }
        if (bits[k] & (1u << 17)) r.s_cand[wg0 + cd++] = key[k];
      }
      *rp = RB::pack(mk);
    }
    cq += (uint32_t)t[0];
    cc += (uint32_t)t[1];
    cw += (uint32_t)t[2];
  }
  uint64_t v5[5] = {nf, hw, dg, dk, gt}, t5[5];
  block_exclusive_scan_multi<5, kBlock>(v5, t5, s_multi);
  if (threadIdx.x == 0) {
    ScanTot t;
    t.nfront = (uint32_t)t5[0];
    t.nq = cq;
    t.ncand = cc;
    t.work = cw;
    t.hw = (uint32_t)t5[1];
    t.pad = 0;
    t.deg = t5[2];
    t.degk = t5[3];
    t.gate = t5[4];
    r.tot[blockIdx.x] = t;
    // superblock sums, so that every copying workgroup of the enqueue finds
    // its offsets with at most kSupers + kSuper loads
    uint32_t* sb = r.sb + ((level & 1) * kSupers + blockIdx.x / kSuper) * 3;
    if (t.nq) atomicAdd(&sb[0], t.nq);
    if (t.work) atomicAdd(&sb[1], t.work);
    if (t.ncand) atomicAdd(&sb[2], t.ncand);
  }
}

constexpr int kCtl = 1024;
constexpr uint32_t kTileAtEntry = 0x80000000u;   // tile_first: the tile starts with the entry

// Marginal run identification (Section 4.2.3): for every selected CG without
// an RPG, D_j = min over its central-keyword nodes of h_j; all finite -> RPG
// with S^m = max_j D_j (Eq. 5) and key gamma_num*S^c + (gamma_den-gamma_num)*S^m
// (Eq. 6 scaled by gamma_den).  Then the stop rules: every CG has an RPG, or
// Theorem 4 with the k-th RPG in (key, S^c, CG rank) order.
template <int TP>
__device__ int rpg_identify(const RunView& r, uint32_t* nrpg_io, int level) {
  __shared__ uint32_t s_dm[kMaxW * kMaxKw];
  __shared__ int32_t s_has[kMaxW], s_sm[kMaxW], s_sc[kMaxW];
  __shared__ uint32_t s_vc[kMaxW + 1];
  __shared__ int64_t s_key[kMaxW];
  __shared__ int32_t s_new, s_nrpg, s_kth, s_minsc, s_stop;
  const int nsel = *r.nsel, M = r.T;
  const int64_t gn = r.gamma_num, gd = r.gamma_den;
  for (int i = threadIdx.x; i < nsel * kMaxKw; i += kCtl) s_dm[i] = kInf;
  for (int i = threadIdx.x; i < nsel; i += kCtl) {
    s_has[i] = r.has_rpg[i]; s_sm[i] = r.sm[i]; s_key[i] = r.key[i]; s_sc[i] = r.sel_sc[i];
  }
  for (int i = threadIdx.x; i <= nsel; i += kCtl) s_vc[i] = r.vc_off[i];
  if (threadIdx.x == 0) { s_new = 0; s_kth = -1; s_minsc = INT32_MAX; s_stop = 0; }
  __syncthreads();
  // D_j of every CG without an RPG: minimum over its V_C rows
  const uint32_t total = s_vc[nsel];
  for (uint32_t p = threadIdx.x; p < total; p += kCtl) {
    const int rr = upper_index<uint32_t>(s_vc, 0, nsel + 1, p);
    if (s_has[rr]) continue;
    uint8_t b[TP];
    load_row<TP>(r.H, r.vc_nodes[p], b);
#pragma unroll
    for (int j = 0; j < TP; ++j)
      if (j < M) atomicMin(&s_dm[rr * kMaxKw + j], (uint32_t)b[j]);
  }
  __syncthreads();
  for (int rr = threadIdx.x; rr < nsel; rr += kCtl) {
    if (s_has[rr]) continue;
    bool all = true;
    int smax = 0;
    for (int j = 0; j < M; ++j) {
      const int d = (int)s_dm[rr * kMaxKw + j];
      r.dmin[rr * kMaxKw + j] = (uint8_t)d;
      all &= d != kInf;
      smax = d > smax ? d : smax;
    }
    if (all) {
      s_has[rr] = 1;
      s_sm[rr] = smax;
      s_key[rr] = r.score_mode ? (int64_t)s_sc[rr] * smax : gn * s_sc[rr] + (gd - gn) * smax;
      atomicAdd(&s_new, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) { s_nrpg = (int)*nrpg_io + s_new; *nrpg_io = (uint32_t)s_nrpg; }
  __syncthreads();
  const int nrpg = s_nrpg;
  if (nrpg == nsel) {
    s_stop = 1;
  } else if (nrpg >= r.k) {
    for (int rr = threadIdx.x; rr < nsel; rr += kCtl) {
      if (s_has[rr]) {
        int rank = 0;
        for (int o = 0; o < nsel; ++o) {
          if (!s_has[o]) continue;
          const bool less = s_key[o] < s_key[rr] ||
                            (s_key[o] == s_key[rr] && (s_sc[o] < s_sc[rr] ||
                                                       (s_sc[o] == s_sc[rr] && o < rr)));
          rank += less;
        }
        if (rank == r.k - 1) s_kth = rr;
      } else {
        atomicMin(&s_minsc, s_sc[rr]);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int kth = s_kth;
      // Theorem 4; strict when equal scores are re-ranked
      const int64_t bound = r.score_mode ? (int64_t)s_minsc * s_sm[kth]
                                         : gn * (int64_t)s_minsc + (gd - gn) * (int64_t)s_sm[kth];
      if (r.rerank ? s_key[kth] < bound : s_key[kth] <= bound) s_stop = 1;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nsel; i += kCtl) {
    r.has_rpg[i] = s_has[i]; r.sm[i] = s_sm[i]; r.key[i] = s_key[i];
  }
  return s_stop;
}

// The final status of the level also goes to `mirror` (pinned host memory),
// so the host learns it without a copy or an event: the status is written,
// made visible to the host, and then stamped with `seq`, the launch's number,
// which the host polls for.  Every thread loads its scan totals
// (at most two workgroups' worth) before anything else, so the kernel waits
// for memory about once before the scan.
static_assert(kScanGroups <= 2 * kCtl, "the control step keeps two scan totals per thread");

__device__ inline void publish(RunStatus* mirror, const RunStatus& st, uint64_t seq) {
  *mirror = st;
  __threadfence_system();
  *reinterpret_cast<volatile uint64_t*>(&mirror->seq) = seq;
}

template <int TP>
__device__ void control_level(const RunView& r, int level, RunStatus* mirror, uint64_t seq) {
  RunStatus* st = r.st;
  const int nb = r.nblocks;
  const int per = (nb + kCtl - 1) / kCtl;   // 1 or 2
  const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
  ScanTot t[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (b0 + i < b1) t[i] = r.tot[b0 + i];
    else t[i] = ScanTot{};
  }
  // thread 0 keeps the run's status in LDS (not in private memory, which
  // every launch of the kernel would then have to set up) and stores it once
  __shared__ RunStatus cur;
  if (threadIdx.x == 0) cur = *st;
  if (level > st->end_level) {
    if (threadIdx.x == 0) publish(mirror, cur, seq);
    return;
  }
  __shared__ int32_t s_end;
  __shared__ uint32_t s_nrpg;
  // one pass for all eight values: q, work, cand prefixes; the rest totals
  __shared__ uint64_t s_multi[(kCtl / kWave + 1) * 8];
  uint64_t vals[8] = {(uint64_t)t[0].nq + t[1].nq, (uint64_t)t[0].work + t[1].work,
                      (uint64_t)t[0].ncand + t[1].ncand, (uint64_t)t[0].nfront + t[1].nfront,
                      (uint64_t)t[0].hw + t[1].hw, t[0].deg + t[1].deg, t[0].degk + t[1].degk,
                      t[0].gate + t[1].gate};
  uint64_t tots[8];
  block_exclusive_scan_multi<8, kCtl>(vals, tots, s_multi);
  const uint32_t tnq = (uint32_t)tots[0], twk = (uint32_t)tots[1], tnc = (uint32_t)tots[2];
  const uint32_t tnf = (uint32_t)tots[3], thw = (uint32_t)tots[4];
  const uint64_t tdg = tots[5], tdk = tots[6], tgt = tots[7];
  if (threadIdx.x == 0) {
    cur.levels = level + 1;
    cur.nfront = tnf;
    cur.nactive = tnq;
    cur.W = twk;
    cur.ncand_level = tnc;
    cur.frontier_sum += tnf;
    cur.h_writes += thw;
    r.q_off[tnq] = twk;
    s_end = END_NONE;
    if (tnf == 0) {
      s_end = END_EXHAUSTED;
    } else if (r.kind == RUN_CENTRAL) {
      cur.ncand_total += tnc;
      if (cur.ncand_total >= (uint32_t)r.w) s_end = END_STOP;
    }
    // where the next level's central nodes start (the other slot is read by
    // this launch's copying workgroups)
    cur.cand_base[(level + 1) & 1] = cur.cand_base[level & 1] + tnc;
    s_nrpg = cur.nrpg;
  }
  // the next level's superblock sums start from zero (this level's are read
  // by the copying workgroups of this launch)
  if (threadIdx.x < kSupers * 3) r.sb[((level + 1) & 1) * kSupers * 3 + threadIdx.x] = 0;
  __syncthreads();
  if (s_end == END_NONE && r.kind == RUN_MARGINAL) {
    if (rpg_identify<TP>(r, &s_nrpg, level) && threadIdx.x == 0) s_end = END_STOP;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cur.nrpg = s_nrpg;
    int end = s_end;
    if (end == END_NONE && level >= r.max_level) end = END_LEVEL_BOUND;
    if (end != END_NONE) {
      cur.end_level = level;
      cur.end_reason = end;
      cur.expand_on = 0;
    } else {
      cur.expand_on = 1;
      cur.e_arc += tdg;
      cur.e_alg += tdk;
      cur.gate_pass += tgt;
    }
    *st = cur;
    publish(mirror, cur, seq);
  }
}

// Frontier Enqueue in the same launch: workgroup 0 runs the level's control
// step; workgroup 1 + b copies scan workgroup b's staged queue entries to
// its place in the expansion queue (its offsets are the sums of the totals
// of the scan workgroups before it, read by all its threads at once), its
// central nodes to the level's place in the candidate list, and, for every
// expansion tile whose first arc falls in one of its entries, that entry to
// the tile map.  The copies do not wait for the control step: if the level
// does not expand, nothing reads the queue.
template <int TP>
__global__ __launch_bounds__(kCtl) void k_front_enqueue(RunView r, int level, RunStatus* mirror,
                                                        uint64_t seq) {
  if (blockIdx.x == 0) {
    control_level<TP>(r, level, mirror, seq);
    return;
  }
  const RunStatus* st = r.st;
  const int b = (int)blockIdx.x - 1;
  if (level > st->end_level) return;   // (set to this level at most, by workgroup 0)
  const ScanTot t = r.tot[b];
  if (t.nq == 0 && t.ncand == 0) return;
  __shared__ uint32_t s_m32[(kCtl / kWave + 1) * 3];
  // offsets: the superblocks before b's, then the scan workgroups of b's
  // superblock before b (one load per thread)
  uint32_t v[3] = {0, 0, 0}, tot[3];
  const int sup = b / kSuper, first = sup * kSuper;
  const uint32_t* sb = r.sb + (level & 1) * kSupers * 3;
  if ((int)threadIdx.x < sup) {
    v[0] = sb[threadIdx.x * 3]; v[1] = sb[threadIdx.x * 3 + 1]; v[2] = sb[threadIdx.x * 3 + 2];
  } else if ((int)threadIdx.x >= kSupers && (int)threadIdx.x - kSupers < b - first) {
    const ScanTot x = r.tot[first + threadIdx.x - kSupers];
    v[0] = x.nq; v[1] = x.work; v[2] = x.ncand;
  }
  block_exclusive_scan_multi<3, kCtl, uint32_t>(v, tot, s_m32);
  const uint32_t oq = tot[0], ow = tot[1];
  const uint32_t oc = st->cand_base[level & 1] + tot[2];
  const int64_t wg0 = (int64_t)b * r.cpw * kScanNodes;
  for (uint32_t j = threadIdx.x; j < t.nq; j += kCtl) {
    const uint4 e = r.s_item[wg0 + j];
    const uint32_t start = ow + e.x;
    const uint32_t end = ow + (j + 1 < t.nq ? r.s_item[wg0 + j + 1].x : t.work);
    r.q_off[oq + j] = start;
    r.q_rs[oq + j] = e.y;
    r.q_lo[oq + j] = e.z;
    r.q_mask[oq + j] = e.w;
    // expansion tiles whose first arc falls in this entry start at it
    for (uint32_t tl = (start + kExpandTile - 1) / kExpandTile; tl * kExpandTile < end; ++tl)
      r.tile_first[tl] = (oq + j) | (tl * kExpandTile == start ? kTileAtEntry : 0u);
  }
  for (uint32_t j = threadIdx.x; j < t.ncand; j += kCtl) r.cand[oc + j] = r.s_cand[wg0 + j];
}


// Algorithm 1 at level `level` over the queued row slices (all of them have
// level <= l).  For arc f -> n every keyword i that f expands for and that has
// not reached n gets h_ni = level + 1, which makes n a frontier of the next
// level.  One gather of the neighbour's reached mask serves
// every keyword at once.  Tile of 1024 consecutive arcs of the concatenated
// slices: the tile map gives its first and last queue entry, the entries go
// to LDS, each entry marks the tile item where it starts and a block max-scan
// turns the marks into the owner entry of every item; item i of the tile is
// handled by thread i mod 256, so consecutive lanes read consecutive arcs.
template <int TP>
__global__ __launch_bounds__(kBlock) void k_expand(RunView r, DevGraphView g, int level) {
  RunStatus* st = r.st;
  if (level > st->end_level || !st->expand_on) return;
  constexpr int IPT = kExpandTile / kBlock;
  const uint32_t W = st->W;
  const int nq = (int)st->nactive;
  __shared__ uint32_t s_base[kExpandTile];
  __shared__ uint32_t s_lo[kExpandTile];
  __shared__ uint32_t s_mask[kExpandTile];
  __shared__ uint16_t s_own[kExpandTile];
  __shared__ uint32_t s_scan[kBlock / kWave + 1];
  const uint32_t ntiles = (W + kExpandTile - 1) / kExpandTile;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t w0 = tile * kExpandTile;
    const uint32_t w1 = min(W, w0 + (uint32_t)kExpandTile);
    // first entry: the one holding arc w0; last: the one holding arc w1 - 1,
    // which is the next tile's first entry unless that entry starts there
    const int e0 = (int)(r.tile_first[tile] & ~kTileAtEntry);
    int e1 = nq - 1;
    if (tile + 1 < ntiles) {
      const uint32_t f1 = r.tile_first[tile + 1];
      e1 = (int)(f1 & ~kTileAtEntry) - ((f1 & kTileAtEntry) ? 1 : 0);
    }
    for (int i = threadIdx.x; i < kExpandTile; i += kBlock) s_own[i] = 0;
    __syncthreads();
    const int cnt = e1 - e0 + 1;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
      const uint32_t off = r.q_off[e0 + j];
      s_base[j] = r.q_rs[e0 + j] - off + w0;   // arc of tile item i is s_base[j] + i
      s_lo[j] = r.q_lo[e0 + j];
      s_mask[j] = r.q_mask[e0 + j];
      s_own[off > w0 ? off - w0 : 0] = (uint16_t)j;
    }
    __syncthreads();
    uint32_t loc[IPT];
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const uint32_t o = s_own[threadIdx.x * IPT + k];
      m = o > m ? o : m;
      loc[k] = m;
    }
    const uint32_t pre = block_exclusive_max(m, s_scan);
#pragma unroll
    for (int k = 0; k < IPT; ++k) s_own[threadIdx.x * IPT + k] = (uint16_t)(pre > loc[k] ? pre : loc[k]);
    __syncthreads();
    // all of the thread's arcs at once: their targets, then the targets'
    // reached masks, then the writes, so that a wavefront keeps IPT
    // independent gathers in flight instead of one dependent chain per arc
    int32_t nbv[IPT];
    uint32_t wantv[IPT], rv[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const uint32_t i = k * kBlock + threadIdx.x;
      wantv[k] = 0;
      nbv[k] = 0;
      if (w0 + i < w1) {
        const int j = s_own[i];
        const uint32_t e = s_base[j] + i;
        const uint32_t mk = s_mask[j];
        wantv[k] = (e < s_lo[j]) ? (mk & 0xFFFFu) : ((mk & 0xFFFFu) | (mk >> 16));
        nbv[k] = g.col_s[e];
      }
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) rv[k] = wantv[k] ? RBits<TP>::get(r.R, nbv[k]) : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // keywords that have not reached the target (as of the start of this level)
      const uint32_t mm = ~rv[k] & wantv[k];
      if (mm) {
#pragma unroll
        for (int t = 0; t < TP; ++t)
          if ((mm >> t) & 1u) r.H[(int64_t)nbv[k] * TP + t] = (uint8_t)(level + 1);
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- top-w ---
// Top-w central graphs by (S^c, sum of central levels, node id).  All CGs of
// earlier levels are kept (they are fewer than w); the remaining slots go to
// the last level's CGs with the smallest sums, ties to smaller node ids.  The
// keys hold original node ids; the selected nodes are stored by internal id.
__global__ __launch_bounds__(kCtl) void k_select(SelectView v) {
  __shared__ uint64_t s_sel[kMaxW];
  __shared__ uint32_t s_hist[4096];
  __shared__ uint32_t s_cnt, s_thr, s_take, s_nsel;
  const RunStatus* st = v.st;
  const uint32_t total = st->ncand_total, last = st->ncand_level;
  const uint32_t prev = total - last;
  const uint32_t w = (uint32_t)v.w;
  if (total <= w) {
    for (uint32_t i = threadIdx.x; i < total; i += kCtl) s_sel[i] = v.cand[i];
    if (threadIdx.x == 0) s_nsel = total;
  } else {
    const uint32_t need = w - prev;
    for (uint32_t i = threadIdx.x; i < prev; i += kCtl) s_sel[i] = v.cand[i];
    for (int i = threadIdx.x; i < 4096; i += kCtl) s_hist[i] = 0;
    __syncthreads();
    // the level's sums crowd into a few bins: one LDS atomic per distinct bin
    // of a wavefront instead of one per candidate
    for (uint32_t base = prev; base < total; base += kCtl) {
      const uint32_t i = base + threadIdx.x;
      const int bin = i < total ? (int)((v.cand[i] >> 32) & 0xFFF) : -1;
      uint64_t pending = __ballot(bin >= 0);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lb = __shfl(bin, leader, kWave);
        const uint64_t same = __ballot(bin == lb);
        if (lane_id() == leader) atomicAdd(&s_hist[lb], (uint32_t)__popcll(same));
        pending &= ~same;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t cum = 0, thr = 0;
      for (uint32_t s = 0; s < 4096; ++s) {
        if (cum + s_hist[s] >= need) { thr = s; break; }
        cum += s_hist[s];
      }
      s_thr = thr;
      s_take = need - cum;
      s_cnt = prev;
      s_nsel = w;
    }
    __syncthreads();
    const uint32_t thr = s_thr;
    // ties at the threshold sum go to the smallest node ids: unless every tie
    // is kept, a byte-wise radix select finds the take-th smallest id T among
    // them (ids are unique, so exactly `take` ties have an id <= T)
    uint32_t T = 0xFFFFFFFFu;
    if (s_hist[thr] != s_take) {
      uint32_t prefix = 0, mask = 0, rem = s_take;
      for (int sh = 24; sh >= 0; sh -= 8) {
        __syncthreads();
        for (int i = threadIdx.x; i < 256; i += kCtl) s_hist[i] = 0;
        __syncthreads();
        for (uint32_t i = prev + threadIdx.x; i < total; i += kCtl) {
          const uint64_t key = v.cand[i];
          const uint32_t id = (uint32_t)key;
          if (((uint32_t)(key >> 32) & 0xFFFF) == thr && (id & mask) == prefix)
            atomicAdd(&s_hist[(id >> sh) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          uint32_t cum = 0;
          for (uint32_t d = 0; d < 256; ++d) {
            if (cum + s_hist[d] >= rem) { s_thr = prefix | (d << sh); s_take = rem - cum; break; }
            cum += s_hist[d];
          }
        }
        __syncthreads();
        prefix = s_thr;
        rem = s_take;
        mask |= 255u << sh;
      }
      T = prefix;
    }
    for (uint32_t i = prev + threadIdx.x; i < total; i += kCtl) {
      const uint64_t key = v.cand[i];
      const uint32_t s = (uint32_t)(key >> 32) & 0xFFFF;
      if (s < thr || (s == thr && (uint32_t)key <= T)) s_sel[atomicAdd(&s_cnt, 1u)] = key;
    }
  }
  __syncthreads();
  const uint32_t nsel = s_nsel;
  for (uint32_t i = threadIdx.x; i < nsel; i += kCtl) {
    const uint64_t key = s_sel[i];
    uint32_t rank = 0;
    for (uint32_t j = 0; j < nsel; ++j) rank += s_sel[j] < key;
    v.sel_node[rank] = v.int_id[key & 0xFFFFFFFFu];
    v.sel_sc[rank] = (int32_t)(key >> 48);
    v.sel_sumh[rank] = (int32_t)((key >> 32) & 0xFFFF);
  }
  if (threadIdx.x == 0) v.gst->nsel = (int32_t)nsel;
}

// Ranking of the results: RPGs by (key, S^c, CG rank); without marginal
// keywords every selected CG is a result with S^m = 0.
__global__ __launch_bounds__(kBlock) void k_rank(RankView v) {
  __shared__ int32_t s_has[kMaxW];
  __shared__ int64_t s_key[kMaxW];
  __shared__ int32_t s_cnt, s_build;
  __shared__ int64_t s_kkey;
  const int nsel = *v.nsel;
  if (threadIdx.x == 0) { s_cnt = 0; s_build = 0; }
  __syncthreads();
  for (int r = threadIdx.x; r < nsel; r += kBlock) {
    if (v.M == 0) {
      v.has_rpg[r] = 1;
      v.sm[r] = 0;
      v.key[r] = v.score_mode ? (int64_t)v.sel_sc[r] : (int64_t)v.gamma_num * v.sel_sc[r];
    }
    s_has[r] = v.has_rpg[r];
    s_key[r] = v.key[r];
    if (s_has[r]) atomicAdd(&s_cnt, 1);
  }
  __syncthreads();
  // results built: the top k; when re-ranking, every RPG whose key does not
  // exceed the k-th one's
  int myrank[kMaxW / kBlock + 1];
  for (int r = threadIdx.x, i = 0; r < nsel; r += kBlock, ++i) {
    myrank[i] = -1;
    if (!s_has[r]) continue;
    int rank = 0;
    for (int o = 0; o < nsel; ++o) {
      if (!s_has[o]) continue;
      rank += s_key[o] < s_key[r] ||
              (s_key[o] == s_key[r] && (v.sel_sc[o] < v.sel_sc[r] ||
                                        (v.sel_sc[o] == v.sel_sc[r] && o < r)));
    }
    myrank[i] = rank;
    if (rank == v.k - 1) s_kkey = s_key[r];
  }
  __syncthreads();
  const bool full = s_cnt >= v.k;
  for (int r = threadIdx.x, i = 0; r < nsel; r += kBlock, ++i) {
    if (myrank[i] < 0) continue;
    const bool build = v.rerank ? (!full || s_key[r] <= s_kkey) : myrank[i] < v.k;
    if (build) {
      v.ranked[myrank[i]] = r;
      atomicAdd(&s_build, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) v.gst->nres = s_build;
}

// Re-ranking (Section 3.3): results of equal score ordered by the sum of
// their arcs' activation levels, then S^c and CG rank; the first k are kept.
__global__ __launch_bounds__(kBlock) void k_rerank(ResultHdr* hdr, Status* gst, int32_t k) {
  __shared__ ResultHdr s_h[kMaxW];
  if (gst->overflow) return;   // the pass is incomplete: the host repeats or finishes it first
  const int n = gst->nres;
  for (int i = threadIdx.x; i < n; i += kBlock) s_h[i] = hdr[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const ResultHdr& a = s_h[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const ResultHdr& b = s_h[j];
      rank += b.key < a.key ||
              (b.key == a.key && (b.wsum < a.wsum ||
              (b.wsum == a.wsum && (b.score_c < a.score_c ||
              (b.score_c == a.score_c && b.cg_rank < a.cg_rank)))));
    }
    hdr[rank] = a;
  }
  if (threadIdx.x == 0) gst->nres = min(n, k);
}

__global__ void k_clear_rpg(int32_t* has, int32_t* sm, int64_t* key, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) { has[i] = 0; sm[i] = 0; key[i] = 0; }
}

// ------------------------------------------------------------ launchers ---

#define RAKS_TP_DISPATCH(TP, ...)                         \
  switch (TP) {                                           \
    case 4: { constexpr int kTP = 4; __VA_ARGS__; } break;  \
    case 8: { constexpr int kTP = 8; __VA_ARGS__; } break;  \
    default: { constexpr int kTP = 16; __VA_ARGS__; } break; \
  }

void launch_run_init(const RunView& r, int TP, int32_t n, const int32_t* kw_nodes,
                     const SeedList& seeds, hipStream_t s) {
  int empty = 0;
  for (int i = 0; i < seeds.T; ++i) empty |= seeds.count[i] == 0;
  k_run_reset<<<1, 1, 0, s>>>(r.st, empty, r.kind == RUN_MARGINAL ? r.nsel : nullptr, r.sb);
  const unsigned g = (unsigned)std::min<int64_t>(8192, (r.n_pad + kBlock - 1) / kBlock);
  RAKS_TP_DISPATCH(TP, k_init_rows<kTP><<<g, kBlock, 0, s>>>(
                           r.H, reinterpret_cast<RMaskT<kTP>*>(r.R), n, r.n_pad, r.T));
  const uint32_t total = seeds.prefix[seeds.T];
  if (total > 0) {
    const unsigned gs = (unsigned)std::min<uint32_t>(4096, (total + kBlock - 1) / kBlock);
    RAKS_TP_DISPATCH(TP, k_seed<kTP><<<gs, kBlock, 0, s>>>(r.H, kw_nodes, seeds));
  }
  if (r.kind == RUN_MARGINAL) k_clear_rpg<<<1, kBlock, 0, s>>>(r.has_rpg, r.sm, r.key, kMaxW);
}

void launch_front_count(const RunView& r, int TP, const DevGraphView& g, int level, hipStream_t s) {
  RAKS_TP_DISPATCH(TP, k_front_count<kTP><<<r.nblocks, kBlock, 0, s>>>(r, g, level));
}

void launch_front_enqueue(const RunView& r, int TP, int level, RunStatus* mirror, uint64_t seq,
                          hipStream_t s) {
  RAKS_TP_DISPATCH(TP, k_front_enqueue<kTP><<<r.nblocks + 1, kCtl, 0, s>>>(r, level, mirror, seq));
}


void launch_expand(const RunView& r, int TP, const DevGraphView& g, int level, int grid,
                   hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 && ev1) {
    // the events take the kernel's own start and end times
    RAKS_TP_DISPATCH(TP, hipExtLaunchKernelGGL(k_expand<kTP>, dim3(grid), dim3(kBlock), 0, s,
                                               ev0, ev1, 0, r, g, level));
  } else {
    RAKS_TP_DISPATCH(TP, k_expand<kTP><<<grid, kBlock, 0, s>>>(r, g, level));
  }
}

void launch_select(const SelectView& v, hipStream_t s) { k_select<<<1, kCtl, 0, s>>>(v); }

void launch_rank(const RankView& v, hipStream_t s) { k_rank<<<1, kBlock, 0, s>>>(v); }

void launch_rerank(ResultHdr* hdr, Status* gst, int32_t k, hipStream_t s) {
  k_rerank<<<1, kBlock, 0, s>>>(hdr, gst, k);
}

}  // namespace raks
