// recover.hip -- recovering phase (Section 4.3, Algorithm 2, Lemma 1) on the
// GPU, and the per-result union / sort / unique of the recovered subgraphs.
//
// Every (result, keyword) instance of a phase is recovered at once: a
// backward search from the start nodes over in-arcs n -> q (the reverses of
// q's arcs on the bi-directed graph) keeps (n, e_nq) when
// h_q = 1 + max(a_nq, h_n) and continues from n unless h_n = 0.  Along a
// recovered arc h strictly drops, so the search runs layer by layer, h from
// the largest level down to 1, one launch per layer: every node of layer h is
// discovered while layers above h run.  A node's arcs are cut into chunks of
// at most 256 that go to the work list of its layer; one wavefront takes a
// chunk, so a hub's arcs spread over the whole GPU.  Only arcs of level below
// the layer can qualify; they are a prefix of the node's level-sorted row, so
// a hub whose arcs all have high levels costs nothing.  Each instance has its
// own node set (open addressing, or a bitmap of n bits once a table was too
// small), node list and arc list, with capacities of its own.  Nodes and arcs
// are counted even when a list is full, and the search goes on, so an
// overflow tells the host how much the instance needs; the host then repeats
// only the phase that overflowed, with only the overflowing instances grown.
#include "common.h"
#include "kernels.h"

namespace raks {

constexpr uint32_t kLdsSort = 4096;   // lists up to this size are sorted in LDS

// Linear probing over at most kMaxProbe slots.  Within its capacity a table is
// at most half full, so a run that long means it has filled up: the node is
// reported lost (the instance switches to a bitmap on the next attempt)
// instead of every later insert walking the whole table with atomics.
constexpr uint32_t kMaxProbe = 64;

__device__ inline bool ht_insert(uint32_t* ht, uint32_t hc, uint32_t key, int* full) {
  uint32_t h = (key * 2654435761u) & (hc - 1);
  const uint32_t probes = hc < kMaxProbe ? hc : kMaxProbe;
  for (uint32_t probe = 0; probe < probes; ++probe) {
    const uint32_t old = atomicCAS(&ht[h], kEmpty, key);
    if (old == kEmpty) return true;
    if (old == key) return false;
    h = (h + 1) & (hc - 1);
  }
  *full = 1;
  return false;
}

// Lanes with `fresh` set queue the in-arcs of node n (hitting level hn) that
// can be recovered arcs as work chunks of layer hn, tagged `inst`.  Called by
// all lanes of a wavefront together.
__device__ inline void rec_queue(const RecoverView& v, bool fresh, uint32_t inst, int32_t n,
                                 uint32_t hn) {
  const int lane = lane_id();
  uint32_t k = 0, rs = 0, deg = 0;
  if (fresh && hn >= 1 && (int)hn <= v.max_layer) {
    // in-arcs m -> n that can meet h_n = 1 + max(a, h_m) have a <= h_n - 1:
    // a prefix of n's level-sorted row (EDGE), or all arcs when the node's
    // own level is below h_n (NODE: every in-arc of n has the level of n)
    rs = v.g.row_ptr[n];
    deg = v.g.mode ? ((uint32_t)v.g.act_node[n] < hn ? v.g.row_ptr[n + 1] - rs : 0u)
                   : count_le(v.g, n, (int)hn - 1);
    k = (deg + kRecChunk - 1) / kRecChunk;
  }
  uint64_t pend = __ballot(k > 0);
  while (pend) {
    const int l0 = __ffsll((unsigned long long)pend) - 1;
    const uint32_t hv = __shfl(hn, l0, kWave);
    const bool mine = k > 0 && hn == hv && ((pend >> lane) & 1ull);
    const uint64_t grp = __ballot(mine);
    const uint32_t inc = wave_inclusive_scan<uint32_t>(mine ? k : 0u);
    const uint32_t tot = __shfl(inc, kWave - 1, kWave);
    uint32_t b0 = 0;
    if (lane == l0) b0 = atomicAdd(&v.lcnt[hv], tot);
    b0 = __shfl(b0, l0, kWave);
    if (mine) {
      const uint32_t first = b0 + inc - k;
      if (first + k > v.lcap) {
        atomicOr(&v.gst->overflow, v.ovf_bit);
      } else {
        RecItem* dst = v.items + (size_t)hv * v.lcap + first;
        for (uint32_t c = 0; c < k; ++c) {
          RecItem it;
          it.inst = inst;
          it.q = n;
          it.start = rs + c * kRecChunk;
          it.len = min(kRecChunk, deg - c * kRecChunk);
          dst[c] = it;
        }
      }
    }
    pend &= ~grp;
  }
}

// Lanes with `act` set have recovered node n (hitting level hn in instance
// inst's column): record each node once per instance and queue its arcs on
// layer hn.  Called by all lanes of a wavefront together (the counters are
// bumped once per wavefront, not once per lane: every wave of a large
// instance would otherwise queue on the same two addresses).
__device__ inline void rec_discover(const RecoverView& v, bool act, uint32_t inst,
                                    const InstCap& ic, int32_t n, uint32_t hn) {
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1;
  bool fresh = false;
  if (act) {
    if (ic.dense) {
      uint32_t* w = v.hpool + ic.hoff + ((uint32_t)n >> 5);
      const uint32_t bit = 1u << ((uint32_t)n & 31u);
      fresh = (atomicOr(w, bit) & bit) == 0;
    } else {
      int full = 0;
      fresh = ht_insert(v.hpool + ic.hoff, ic.hcap, (uint32_t)n, &full);
      if (full) {
        v.iflag[inst] = 1;
        atomicOr(&v.gst->overflow, v.ovf_bit);
      }
    }
  }
  // node list slots
  const uint64_t fb = __ballot(fresh);
  if (fb == 0) return;
  const int lead = __ffsll((unsigned long long)fb) - 1;
  uint32_t base = 0;
  if (lane == lead) base = atomicAdd(&v.cnt[inst * 2], (uint32_t)__popcll(fb));
  base = __shfl(base, lead, kWave);
  if (fresh) {
    const uint32_t slot = base + (uint32_t)__popcll(fb & below);
    if (slot < ic.ncap) v.nl[ic.noff + slot] = n;
    else atomicOr(&v.gst->overflow, v.ovf_bit);
  }
  rec_queue(v, fresh, inst, n, hn);
}

// Clears the node sets and counters of the live instances: row y of the grid
// takes instance y.
__global__ __launch_bounds__(kBlock) void k_rec_clear(RecoverView v) {
  const uint32_t inst = blockIdx.y;
  if (inst == 0 && blockIdx.x == 0)
    for (int i = threadIdx.x; i <= v.max_layer; i += kBlock) v.lcnt[i] = 0;
  if ((int)(inst / v.T) >= *v.n_valid) return;
  const InstCap ic = v.caps[inst];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.cnt[inst * 2] = 0;
    v.cnt[inst * 2 + 1] = 0;
    v.iflag[inst] = 0;
  }
  const size_t words = ic.dense ? (size_t)v.dwords : (size_t)ic.hcap;
  const uint32_t fill = ic.dense ? 0u : kEmpty;
  uint32_t* p = v.hpool + ic.hoff;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += (size_t)gridDim.x * kBlock)
    p[i] = fill;
}

// Start nodes: the central node (central graphs), or the V_C nodes whose
// level for the marginal keyword equals D_j (radial pattern graphs).
template <int TP>
__global__ __launch_bounds__(kBlock) void k_rec_seed(RecoverView v) {
  const uint32_t inst = blockIdx.x;
  const int res = inst / v.T, col = inst % v.T;
  if (res >= *v.n_valid) return;
  const InstCap ic = v.caps[inst];
  if (!v.marginal) {
    if (wave_id() == 0) {
      const int32_t c = v.sel_node[res];
      rec_discover(v, lane_id() == 0, inst, ic, c, v.H[(int64_t)c * TP + col]);
    }
  } else {
    const int r = v.ranked[res];
    const uint8_t d = v.dmin[r * kMaxKw + col];
    const uint32_t p0 = v.vc_off[r], p1 = v.vc_off[r + 1];
    for (uint32_t p = p0 + (threadIdx.x & ~(uint32_t)(kWave - 1)); p < p1; p += kBlock) {
      const uint32_t q = p + lane_id();
      const int32_t x = q < p1 ? v.vc_nodes[q] : 0;
      rec_discover(v, q < p1 && v.H[(int64_t)x * TP + col] == d, inst, ic, x, d);
    }
  }
}

template <int TP>
__global__ __launch_bounds__(kBlock) void k_rec_layer(RecoverView v, int h) {
  // A layer whose chunk requests ran past its capacity has unwritten slots
  // below the capacity (a request that did not fit was dropped whole), so it
  // is not searched at all: the phase is repeated with room for every chunk.
  if (v.lcnt[h] > v.lcap) return;
  const uint32_t n_items = v.lcnt[h];
  const uint32_t waves = gridDim.x * (kBlock / kWave);
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1;
  const RecItem* list = v.items + (size_t)h * v.lcap;
  const DevGraphView& g = v.g;
  for (uint32_t it = blockIdx.x * (kBlock / kWave) + wave_id(); it < n_items; it += waves) {
    const RecItem item = list[it];
    // an instance whose node table filled up has lost nodes: this pass only
    // tells the host to give it a bitmap, so its remaining work is skipped
    if (v.iflag[item.inst]) continue;
    const InstCap ic = v.caps[item.inst];
    const int col = item.inst % v.T;
    const int32_t q = item.q;
    const uint32_t aq = g.mode ? g.act_node[q] : 0u;   // NODE mode: level of the in-arc's target q
    for (uint32_t k0 = 0; k0 < item.len; k0 += kWave) {
      const uint32_t k = k0 + lane;
      bool take = false;
      int32_t n = 0;
      uint32_t hn = 0, fwd = 0;
      if (k < item.len) {
        const uint32_t e = item.start + k;                 // position in q's level-sorted row
        const uint32_t a = g.mode ? aq : g.act_s[e];       // EDGE: level of q -> n = level of n -> q
        if (a < (uint32_t)h) {
          n = g.col_s[e];
          hn = v.H[(int64_t)n * TP + col];
          // h = 1 + max(a, h_n)
          take = hn < (uint32_t)h && (a + 1 == (uint32_t)h || hn + 1 == (uint32_t)h);
          if (take) fwd = g.rev[g.eid_s[e]];               // the arc n -> q, CSR position
        }
      }
      const uint64_t tb = __ballot(take);
      if (tb == 0) continue;
      const int lead = __ffsll((unsigned long long)tb) - 1;
      uint32_t base = 0;
      if (lane == lead) base = atomicAdd(&v.cnt[item.inst * 2 + 1], (uint32_t)__popcll(tb));
      base = __shfl(base, lead, kWave);
      if (take) {
        const uint32_t sa = base + (uint32_t)__popcll(tb & below);
        if (sa < ic.acap) v.al[ic.aoff + sa] = fwd;
        else atomicOr(&v.gst->overflow, v.ovf_bit);
      }
      rec_discover(v, take, item.inst, ic, n, hn);
    }
  }
}

// ------------------------------------------------------ labelled mode
//
// The instances of one keyword column differ only in their start nodes, and a
// search from a set of start nodes reaches the union of what the searches
// from each of them reach, over the same recovered arcs.  So one search per
// column (and group of 64 results) stands for all of the column's instances:
// every reached node carries a label with one bit per result whose search
// reaches it, and a recovered arc n -> q passes q's label on to n.  A node of
// layer h gets bits only from nodes of higher layers, so its label is final
// when layer h runs: its recovered in-arcs are then written to the arc list of
// every result in the label.  The node lists are written from the final
// labels once the last layer has run, which also clears them.  Each
// instance's lists hold the same sets as in the per-instance search; the work
// is that of the column's union instead of the sum of its instances.

__device__ inline uint64_t* lab_row(const RecoverView& v, uint32_t jg) {
  return v.lab + (size_t)jg * (uint32_t)v.g.n;
}

// Lanes with `fresh` set gave node n its first label bits in column group jg:
// record (jg, n) for the node pass and queue n's in-arcs on layer hn.
__device__ inline void lr_fresh(const RecoverView& v, bool fresh, uint32_t jg, int32_t n,
                                uint32_t hn) {
  const int lane = lane_id();
  const uint64_t fb = __ballot(fresh);
  if (fb == 0) return;
  const int lead = __ffsll((unsigned long long)fb) - 1;
  uint32_t base = 0;
  if (lane == lead) base = atomicAdd(v.tcnt, (uint32_t)__popcll(fb));
  base = __shfl(base, lead, kWave);
  if (fresh) {
    const uint32_t slot = base + (uint32_t)__popcll(fb & ((1ull << lane) - 1));
    if (slot < v.tcap) v.touch[slot] = ((uint64_t)jg << 32) | (uint32_t)n;
    else atomicOr(&v.gst->overflow, v.ovf_bit);
  }
  rec_queue(v, fresh, jg, n, hn);
}

__global__ __launch_bounds__(kBlock) void k_lr_clear(RecoverView v, size_t wipe_words) {
  const uint32_t tid = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
  for (uint32_t i = tid; i < (uint32_t)v.n_inst * 2u; i += stride) v.cnt[i] = 0;
  for (uint32_t i = tid; i < (uint32_t)v.n_inst; i += stride) v.iflag[i] = 0;
  for (uint32_t i = tid; i <= (uint32_t)v.max_layer; i += stride) v.lcnt[i] = 0;
  if (tid == 0) *v.tcnt = 0;
  for (size_t i = tid; i < wipe_words; i += stride) v.lab[i] = 0;
}

// Start nodes as in k_rec_seed, labelled with their result's bit.
template <int TP>
__global__ __launch_bounds__(kBlock) void k_lr_seed(RecoverView v) {
  const uint32_t inst = blockIdx.x;
  const int res = inst / v.T, col = inst % v.T;
  if (res >= *v.n_valid) return;
  const uint32_t jg = (uint32_t)(col * v.G + res / 64);
  const unsigned long long bit = 1ull << (res % 64);
  unsigned long long* lab = reinterpret_cast<unsigned long long*>(lab_row(v, jg));
  if (!v.marginal) {
    if (wave_id() == 0) {
      const int32_t c = v.sel_node[res];
      const bool fresh = lane_id() == 0 && atomicOr(&lab[c], bit) == 0;
      lr_fresh(v, fresh, jg, c, v.H[(int64_t)c * TP + col]);
    }
  } else {
    const int r = v.ranked[res];
    const uint8_t d = v.dmin[r * kMaxKw + col];
    const uint32_t p0 = v.vc_off[r], p1 = v.vc_off[r + 1];
    for (uint32_t p = p0 + (threadIdx.x & ~(uint32_t)(kWave - 1)); p < p1; p += kBlock) {
      const uint32_t q = p + lane_id();
      const int32_t x = q < p1 ? v.vc_nodes[q] : 0;
      const bool act = q < p1 && v.H[(int64_t)x * TP + col] == d;
      const bool fresh = act && atomicOr(&lab[x], bit) == 0;
      lr_fresh(v, fresh, jg, x, d);
    }
  }
}

// A labelled layer in batches of kLrBatch work chunks per workgroup, one
// wavefront per chunk (at most kRecChunk = 4 x 64 arcs of q's row), so that a
// batch makes one global reservation per arc list, per layer queue and for
// the node log instead of one per chunk: these counters are few, and every
// wavefront of the GPU adds to them (atomics on device memory are performed
// at the memory side, so one address takes them one at a time).
//   A  each wavefront examines its chunks: recovered arcs (h = 1 + max(a, h_n)),
//      labels or-ed into their nodes (a label that already holds all of q's
//      bits needs no atomic, and its node is not fresh: bits are only added
//      during a layer), and the batch's local offsets from LDS counters;
//   B  one global reservation per touched arc list, per layer with queued
//      chunks and for the node log;
//   C  the writes.
// All of a chunk's recovered arcs go to the arc lists of the results in q's
// final label.
constexpr int kLrGI = 2;                                 // chunks per wavefront per batch
constexpr int kLrBatch = kLrGI * (kBlock / kWave);      // chunks per workgroup per batch
constexpr int kLrMaxInst = kMaxW * kMaxKw;               // instances of a phase
constexpr int kLrMaxLayer = 256;
static_assert(kRecChunk == 4 * kWave, "a recovery chunk is four wavefront rounds");

template <int TP>
__global__ __launch_bounds__(kBlock) void k_lr_layer(RecoverView v, int h) {
  if (v.lcnt[h] > v.lcap) return;   // as in k_rec_layer: the phase is repeated
  __shared__ uint32_t s_cnt[kLrMaxInst];     // batch's arcs per instance, then its global base
  __shared__ uint16_t s_list[kLrBatch * 64]; // instances touched by the batch
  __shared__ uint32_t s_lay[kLrMaxLayer];    // chunks queued per layer, then the global base
  __shared__ uint32_t s_nt, s_touch, s_tbase;
  const uint32_t n_items = v.lcnt[h];
  const int lane = lane_id(), wv = wave_id();
  const uint64_t below = (1ull << lane) - 1;
  const RecItem* list = v.items + (size_t)h * v.lcap;
  const DevGraphView& g = v.g;
  for (int i = threadIdx.x; i < v.n_inst; i += kBlock) s_cnt[i] = 0;
  for (int i = threadIdx.x; i <= v.max_layer; i += kBlock) s_lay[i] = 0;
  if (threadIdx.x == 0) { s_nt = 0; s_touch = 0; }
  __syncthreads();
  for (uint32_t b0 = blockIdx.x * (uint32_t)kLrBatch; b0 < n_items; b0 += gridDim.x * (uint32_t)kLrBatch) {
    // ---- A
    uint32_t fwd[kLrGI][4];
    int32_t nn[kLrGI][4];
    uint32_t hh[kLrGI][4], toff[kLrGI][4], qoff[kLrGI][4];
    uint32_t take = 0, fresh = 0;             // bit 4 g + r
    uint32_t pos[kLrGI][4];
    uint64_t lqs[kLrGI];
    uint32_t jgs[kLrGI], tots[kLrGI];         // per chunk (the same in every lane)
    uint32_t lbase[kLrGI];                    // lane j: local offset in its j-th result's list
#pragma unroll
    for (int gi = 0; gi < kLrGI; ++gi) {
      const uint32_t it = b0 + (uint32_t)(wv * kLrGI + gi);
      lqs[gi] = 0;
      jgs[gi] = 0;
      lbase[gi] = 0;
      RecItem item = {0, 0, 0, 0};
      if (it < n_items) item = list[it];
      const uint32_t jg = item.inst;
      const int col = (int)jg / v.G, grp = (int)jg % v.G;
      unsigned long long* lab = reinterpret_cast<unsigned long long*>(lab_row(v, jg));
      const uint64_t lq = it < n_items ? lab[item.q] : 0ull;   // final: q is on this layer
      const uint32_t aq = (g.mode && it < n_items) ? g.act_node[item.q] : 0u;
      lqs[gi] = lq;
      jgs[gi] = jg;
      uint32_t tot = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t k = (uint32_t)r * kWave + lane;
        bool tk = false;
        nn[gi][r] = 0;
        hh[gi][r] = 0;
        fwd[gi][r] = 0;
        if (k < item.len) {
          const uint32_t e = item.start + k;
          const uint32_t a = g.mode ? aq : g.act_s[e];
          if (a < (uint32_t)h) {
            nn[gi][r] = g.col_s[e];
            hh[gi][r] = v.H[(int64_t)nn[gi][r] * TP + col];
            // h = 1 + max(a, h_n)
            tk = hh[gi][r] < (uint32_t)h && (a + 1 == (uint32_t)h || hh[gi][r] + 1 == (uint32_t)h);
            if (tk) fwd[gi][r] = g.rev[g.eid_s[e]];
          }
        }
        const uint64_t tb = __ballot(tk);
        pos[gi][r] = tot + (uint32_t)__popcll(tb & below);
        tot += (uint32_t)__popcll(tb);
        if (tk) take |= 1u << (4 * gi + r);
        bool fr = false;
        if (tk) {
          const uint64_t cur = __atomic_load_n(&lab[nn[gi][r]], __ATOMIC_RELAXED);
          if ((cur & lq) != lq) fr = atomicOr(&lab[nn[gi][r]], (unsigned long long)lq) == 0;
        }
        // local offsets of a fresh node: its node-log entry and its queued chunks
        toff[gi][r] = 0;
        qoff[gi][r] = 0;
        const uint64_t fb = __ballot(fr);
        if (fb) {
          const int lead = __ffsll((unsigned long long)fb) - 1;
          uint32_t t0 = 0;
          if (lane == lead) t0 = atomicAdd(&s_touch, (uint32_t)__popcll(fb));
          t0 = __shfl(t0, lead, kWave);
          if (fr) {
            fresh |= 1u << (4 * gi + r);
            toff[gi][r] = t0 + (uint32_t)__popcll(fb & below);
            const uint32_t hn = hh[gi][r];
            if (hn >= 1 && (int)hn <= v.max_layer) {
              const int32_t n = nn[gi][r];
              const uint32_t deg = g.mode ? ((uint32_t)g.act_node[n] < hn ? g.row_ptr[n + 1] - g.row_ptr[n] : 0u)
                                          : count_le(g, n, (int)hn - 1);
              const uint32_t kc = (deg + kRecChunk - 1) / kRecChunk;
              if (kc) qoff[gi][r] = atomicAdd(&s_lay[hn], kc);
            }
          }
        }
      }
      tots[gi] = tot;
      // lane j: room for this chunk's arcs in the list of q's j-th label bit
      if (tot && lane < __popcll(lq)) {
        uint64_t m = lq;
        for (int j = 0; j < lane; ++j) m &= m - 1;
        const int b = __ffsll((unsigned long long)m) - 1;
        const uint32_t inst = (uint32_t)(grp * 64 + b) * (uint32_t)v.T + (uint32_t)col;
        lbase[gi] = atomicAdd(&s_cnt[inst], tot);
        if (lbase[gi] == 0) s_list[atomicAdd(&s_nt, 1u)] = (uint16_t)inst;
      }
    }
    __syncthreads();
    // ---- B
    for (uint32_t t = threadIdx.x; t < s_nt; t += kBlock) {
      const uint32_t inst = s_list[t];
      const uint32_t c = s_cnt[inst];
      const uint32_t base = atomicAdd(&v.cnt[inst * 2 + 1], c);
      if (base + c > v.caps[inst].acap) atomicOr(&v.gst->overflow, v.ovf_bit);
      s_cnt[inst] = base;
    }
    for (int t = threadIdx.x; t <= v.max_layer; t += kBlock)
      if (s_lay[t]) s_lay[t] = atomicAdd(&v.lcnt[t], s_lay[t]);
    if (threadIdx.x == 0 && s_touch) s_tbase = atomicAdd(v.tcnt, s_touch);
    __syncthreads();
    // ---- C
#pragma unroll
    for (int gi = 0; gi < kLrGI; ++gi) {
      const uint64_t lq = lqs[gi];
      const uint32_t jg = jgs[gi];
      const int col = (int)jg / v.G, grp = (int)jg % v.G;
      if (tots[gi]) {
        uint64_t m = lq;
        for (int j = 0; m; ++j, m &= m - 1) {
          const int b = __ffsll((unsigned long long)m) - 1;
          const uint32_t inst = (uint32_t)(grp * 64 + b) * (uint32_t)v.T + (uint32_t)col;
          const InstCap ic = v.caps[inst];
          const uint32_t base = s_cnt[inst] + __shfl(lbase[gi], j, kWave);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (((take >> (4 * gi + r)) & 1u) && base + pos[gi][r] < ic.acap)
              v.al[ic.aoff + base + pos[gi][r]] = fwd[gi][r];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!((fresh >> (4 * gi + r)) & 1u)) continue;
        const int32_t n = nn[gi][r];
        const uint32_t hn = hh[gi][r];
        const uint32_t slot = s_tbase + toff[gi][r];
        if (slot < v.tcap) v.touch[slot] = ((uint64_t)jg << 32) | (uint32_t)n;
        else atomicOr(&v.gst->overflow, v.ovf_bit);
        if (hn >= 1 && (int)hn <= v.max_layer) {
          const uint32_t rs = g.row_ptr[n];
          const uint32_t deg = g.mode ? ((uint32_t)g.act_node[n] < hn ? g.row_ptr[n + 1] - rs : 0u)
                                      : count_le(g, n, (int)hn - 1);
          const uint32_t kc = (deg + kRecChunk - 1) / kRecChunk;
          const uint32_t first = s_lay[hn] + qoff[gi][r];
          if (kc && first + kc > v.lcap) {
            atomicOr(&v.gst->overflow, v.ovf_bit);
          } else {
            RecItem* dst = v.items + (size_t)hn * v.lcap + first;
            for (uint32_t c = 0; c < kc; ++c) {
              RecItem ri;
              ri.inst = jg;
              ri.q = n;
              ri.start = rs + c * kRecChunk;
              ri.len = min(kRecChunk, deg - c * kRecChunk);
              dst[c] = ri;
            }
          }
        }
      }
    }
    __syncthreads();
    // reset the batch's counters
    for (uint32_t t = threadIdx.x; t < s_nt; t += kBlock) s_cnt[s_list[t]] = 0;
    for (int t = threadIdx.x; t <= v.max_layer; t += kBlock) s_lay[t] = 0;
    __syncthreads();
    if (threadIdx.x == 0) { s_nt = 0; s_touch = 0; }
    __syncthreads();
  }
}

// Node lists from the final labels; the labels are cleared on the way.
__global__ __launch_bounds__(kBlock) void k_lr_nodes(RecoverView v) {
  const uint32_t total = min(*v.tcnt, v.tcap);
  const uint32_t waves = gridDim.x * (kBlock / kWave);
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1;
  for (uint32_t w0 = (blockIdx.x * (kBlock / kWave) + wave_id()) * kWave; w0 < total;
       w0 += waves * kWave) {
    const uint32_t i = w0 + lane;
    uint32_t jg = 0;
    int32_t n = 0;
    uint64_t my = 0;
    if (i < total) {
      const uint64_t e = v.touch[i];
      jg = (uint32_t)(e >> 32);
      n = (int32_t)(uint32_t)e;
      uint64_t* lab = lab_row(v, jg);
      my = lab[n];
      lab[n] = 0;
    }
    // one counter update per (wavefront, instance)
    for (;;) {
      const uint64_t act = __ballot(my != 0);
      if (act == 0) break;
      const int lead = __ffsll((unsigned long long)act) - 1;
      const uint32_t ljg = __shfl(jg, lead, kWave);
      const uint32_t lo = __shfl((uint32_t)my, lead, kWave);
      const uint32_t hi = __shfl((uint32_t)(my >> 32), lead, kWave);
      const int b = lo ? __ffs(lo) - 1 : 32 + __ffs(hi) - 1;
      const bool sel = jg == ljg && ((my >> b) & 1ull);
      const uint64_t sm = __ballot(sel);
      const uint32_t inst = (uint32_t)((int)(ljg % (uint32_t)v.G) * 64 + b) * (uint32_t)v.T +
                            ljg / (uint32_t)v.G;
      const InstCap ic = v.caps[inst];
      uint32_t base = 0;
      if (lane == lead) base = atomicAdd(&v.cnt[inst * 2], (uint32_t)__popcll(sm));
      base = __shfl(base, lead, kWave);
      if (sel) {
        const uint32_t slot = base + (uint32_t)__popcll(sm & below);
        if (slot < ic.ncap) v.nl[ic.noff + slot] = n;
        else atomicOr(&v.gst->overflow, v.ovf_bit);
        my &= ~(1ull << b);
      }
    }
  }
}

// Per result: gather the node lists (and arc lists) of its instances (and,
// for an RPG, of its CG), radix sort, keep distinct keys.  For CGs also the
// central-keyword nodes V_C (some central level 0).  Final results go to the
// output arena with their header; arcs are written as (src, dst, label).
__global__ __launch_bounds__(kBlock) void k_finalize(FinalizeView v) {
  const int t = blockIdx.x;
  if (t >= *v.n_valid) {
    if (threadIdx.x == 0) v.big[t] = 0;
    return;
  }
  bool skip = (v.gst->overflow & v.skip_bits) != 0;
  uint64_t nn = 0, na = 0;   // input sizes of the node and arc lists
  if (!skip) {
    // inputs beyond big_list go to the bitmap path (k_big_*), run by the host
    // once this launch has finished
    const int r0 = v.marginal ? v.ranked[t] : t;
    nn = v.marginal ? v.cg_cnt[r0 * 2] : 0u;
    na = v.marginal ? v.cg_cnt[r0 * 2 + 1] : 0u;
    for (int j = 0; j < v.T; ++j) {
      const InstCap ic = v.caps[t * v.T + j];
      nn += min(v.cnt[(t * v.T + j) * 2], ic.ncap);
      na += min(v.cnt[(t * v.T + j) * 2 + 1], ic.acap);
    }
    if (nn > v.big_list || na > v.big_list) {
      if (threadIdx.x == 0) {
        v.big[t] = 1;
        atomicOr(&v.gst->overflow, v.marginal ? kOvfBig1 : kOvfBig0);
      }
      skip = true;
    } else if (threadIdx.x == 0) {
      v.big[t] = 0;
    }
  } else if (threadIdx.x == 0) {
    v.big[t] = 0;
  }
  if (skip) {
    // the phase is repeated or finished elsewhere: record empty CG lists so
    // nothing reads stale sizes
    if (!v.marginal && threadIdx.x == 0) {
      v.cg_cnt[t * 2] = 0;
      v.cg_cnt[t * 2 + 1] = 0;
      v.vc_cnt[t] = 0;
    }
    return;
  }
  __shared__ RadixLds lds;
  __shared__ uint32_t s_off;
  __shared__ uint64_t s_ws[kBlock / kWave + 1];
  __shared__ uint32_t s_sa[kLdsSort], s_sb[kLdsSort];
  uint32_t* A_g = v.sort_a + v.soff[t];
  uint32_t* B_g = v.sort_b + v.soff[t];
  const int r = v.marginal ? v.ranked[t] : t;
  const DevGraphView& g = v.g;

  // When both lists fit LDS, the result's two workgroups (y = 0, 1) take the
  // node and the arc pass at once; otherwise workgroup 0 takes both, since
  // they share the result's global sort scratch.
  const bool split = nn <= kLdsSort && na <= kLdsSort;
  if (!split && blockIdx.y == 1) return;
  const int p0 = split ? (int)blockIdx.y : 0, p1 = split ? p0 + 1 : 2;
  for (int pass = p0; pass < p1; ++pass) {   // 0: nodes, 1: arcs
    // total input size first: small lists are sorted in LDS
    uint32_t n = v.marginal ? v.cg_cnt[r * 2 + pass] : 0u;
    for (int j = 0; j < v.T; ++j)
      n += min(v.cnt[(t * v.T + j) * 2 + pass],
               pass == 0 ? v.caps[t * v.T + j].ncap : v.caps[t * v.T + j].acap);
    const bool small = n <= kLdsSort;
    uint32_t* A = small ? s_sa : A_g;
    uint32_t* B = small ? s_sb : B_g;
    __syncthreads();
    n = 0;
    if (v.marginal) {
      const uint32_t cnt = v.cg_cnt[r * 2 + pass];
      const uint32_t* src = pass == 0 ? v.cg_nodes + v.cg_noff[r] : v.cg_arcs + v.cg_aoff[r];
      for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) A[i] = src[i];
      n = cnt;
    }
    for (int j = 0; j < v.T; ++j) {
      const int inst = t * v.T + j;
      const InstCap ic = v.caps[inst];
      const uint32_t cnt = min(v.cnt[inst * 2 + pass], pass == 0 ? ic.ncap : ic.acap);
      if (pass == 0) {
        // recovered nodes are internal ids; results list original ids
        const int32_t* src = v.nl + ic.noff;
        for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) A[n + i] = (uint32_t)g.orig_id[src[i]];
      } else {
        const uint32_t* src = v.al + ic.aoff;
        for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) A[n + i] = src[i];
      }
      n += cnt;
    }
    __syncthreads();
    uint32_t* sorted = wg_radix_sort_u32(A, B, n, lds);
    uint32_t* uniq = (sorted == A) ? B : A;
    const uint32_t m = wg_unique_u32(sorted, n, uniq, lds.scan);
    __syncthreads();
    if (!v.marginal) {
      uint32_t* dst = pass == 0 ? v.cg_nodes + v.cg_noff[r] : v.cg_arcs + v.cg_aoff[r];
      for (uint32_t i = threadIdx.x; i < m; i += kBlock) dst[i] = uniq[i];
      if (threadIdx.x == 0) v.cg_cnt[r * 2 + pass] = m;
      if (pass == 0) {
        // V_C in node order, stored as internal ids
        int32_t* vc = v.vc_tmp + v.cg_noff[r];
        uint32_t written = 0;
        for (uint32_t t0 = 0; t0 < m; t0 += kBlock) {
          const uint32_t i = t0 + threadIdx.x;
          uint32_t keep = 0;
          int64_t x = 0;
          if (i < m) {
            x = g.int_id[uniq[i]];
            for (int c = 0; c < v.Tc; ++c) keep |= v.Hc[x * v.TPc + c] == 0;
          }
          uint32_t tot;
          const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(keep, lds.scan, &tot);
          if (keep) vc[written + ex] = (int32_t)x;
          written += tot;
        }
        if (threadIdx.x == 0) v.vc_cnt[r] = written;
      }
    }
    if (v.write_output) {
      // sum of the arcs' activation levels (the re-ranking weight); integer, so
      // any summation order gives the same value
      uint64_t ws = 0;
      if (pass == 1)
        for (uint32_t i = threadIdx.x; i < m; i += kBlock) ws += g.act[uniq[i]];
      ws = block_sum<uint64_t, kBlock>(ws, s_ws);
      if (threadIdx.x == 0) {
        const uint32_t off = atomicAdd(pass == 0 ? &v.gst->out_nodes : &v.gst->out_arcs, m);
        const uint32_t cap = pass == 0 ? v.out_ncap : v.out_acap;
        if (off + m > cap) atomicOr(&v.gst->overflow, 4);
        s_off = off;
        ResultHdr& hd = v.hdr[t];
        if (pass == 0) {
          hd.central = v.g.orig_id[v.sel_node[r]];
          hd.score_c = v.sel_sc[r];
          hd.score_m = v.sm[r];
          hd.cg_rank = r;
          hd.key = v.key[r];
          hd.node_off = off;
          hd.n_nodes = m;
        } else {
          hd.arc_off = off;
          hd.n_arcs = m;
          hd.wsum = (int64_t)ws;
        }
      }
      __syncthreads();
      const uint32_t off = s_off;
      const uint32_t cap = pass == 0 ? v.out_ncap : v.out_acap;
      if (off + m <= cap) {
        if (pass == 0) {
          for (uint32_t i = threadIdx.x; i < m; i += kBlock) v.out_nodes[off + i] = (int32_t)uniq[i];
        } else {
          for (uint32_t i = threadIdx.x; i < m; i += kBlock) {
            const uint32_t e = uniq[i];
            int32_t* o = v.out_arcs + 3 * (size_t)(off + i);
            o[0] = g.arc_src[e];
            o[1] = g.col[e];
            o[2] = g.label[e];
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------- large results
//
// A result whose lists exceed big_list is not sorted by one workgroup: its
// node ids (or arc positions) are set in a bitmap over all nodes (arcs) by the
// whole GPU, counted per chunk of kBigChunk words, scanned, and written in id
// order -- the same sorted, distinct list, in O(n + A) work.  Pass 0 takes the
// nodes, pass 1 the arcs, pass 2 (CGs only) the V_C nodes: the set nodes with
// some central hitting level 0.

constexpr uint32_t kBigChunk = 4 * kBlock;   // bitmap words per count / write block

__global__ __launch_bounds__(kBlock) void k_big_clear(uint32_t* bm, uint32_t words) {
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < words; i += gridDim.x * kBlock) bm[i] = 0;
}

// Sets the ids of every input list of result t (ids outside the node or arc
// range are never produced; the test only guards the bitmap).
__global__ __launch_bounds__(kBlock) void k_big_mark(FinalizeView v, int t, int pass, uint32_t* bm) {
  const uint32_t stride = gridDim.x * kBlock, tid = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t limit = (pass & 1) ? v.g.A : (uint32_t)v.g.n;
  if (v.marginal) {
    const int r = v.ranked[t];
    const uint32_t cnt = v.cg_cnt[r * 2 + (pass & 1)];
    const uint32_t* src = (pass & 1) ? v.cg_arcs + v.cg_aoff[r] : v.cg_nodes + v.cg_noff[r];
    for (uint32_t i = tid; i < cnt; i += stride) {
      const uint32_t x = src[i];
      if (x < limit) atomicOr(&bm[x >> 5], 1u << (x & 31u));
    }
  }
  for (int j = 0; j < v.T; ++j) {
    const int inst = t * v.T + j;
    const InstCap ic = v.caps[inst];
    if (pass & 1) {
      const uint32_t cnt = min(v.cnt[inst * 2 + 1], ic.acap);
      const uint32_t* src = v.al + ic.aoff;
      for (uint32_t i = tid; i < cnt; i += stride) {
        const uint32_t x = src[i];
        if (x < limit) atomicOr(&bm[x >> 5], 1u << (x & 31u));
      }
    } else {
      const uint32_t cnt = min(v.cnt[inst * 2], ic.ncap);
      const int32_t* src = v.nl + ic.noff;
      for (uint32_t i = tid; i < cnt; i += stride) {
        const uint32_t x = (uint32_t)v.g.orig_id[src[i]];   // internal -> original id
        if (x < limit) atomicOr(&bm[x >> 5], 1u << (x & 31u));
      }
    }
  }
}

// Set bits of one word that count for the pass (pass 2: V_C nodes only).
__device__ inline uint32_t big_bits(const FinalizeView& v, int pass, uint32_t word, uint32_t wi) {
  if (pass != 2 || word == 0) return word;
  uint32_t keep = 0;
  for (uint32_t b = word; b; b &= b - 1) {
    const int bit = __ffs(b) - 1;
    const int64_t x = v.g.int_id[wi * 32 + (uint32_t)bit];   // the bitmap is over original ids
    bool vc = false;
    for (int c = 0; c < v.Tc; ++c) vc |= v.Hc[x * v.TPc + c] == 0;
    keep |= (vc ? 1u : 0u) << bit;
  }
  return keep;
}

__global__ __launch_bounds__(kBlock) void k_big_count(FinalizeView v, int pass, const uint32_t* bm,
                                                      uint32_t words, uint32_t* chunk) {
  __shared__ uint32_t s32[kBlock / kWave + 1];
  const uint32_t w0 = blockIdx.x * kBigChunk + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (w0 + k < words) c += __popc(big_bits(v, pass, bm[w0 + k], w0 + k));
  const uint32_t tot = block_sum<uint32_t, kBlock>(c, s32);
  if (threadIdx.x == 0) chunk[blockIdx.x] = tot;
}

// One workgroup: chunk counts -> chunk offsets; places the list (output arena
// or the CG's lists) and writes its size.  slot[0] receives the list start.
__global__ __launch_bounds__(kBlock) void k_big_scan(FinalizeView v, int t, int pass, uint32_t* chunk,
                                                     uint32_t nchunks, uint64_t* slot) {
  __shared__ uint32_t s32[kBlock / kWave + 1];
  __shared__ uint32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nchunks; b0 += kBlock) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t x = i < nchunks ? chunk[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(x, s32, &tot);
    if (i < nchunks) chunk[i] = s_carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const uint32_t m = s_carry;
  const int r = v.marginal ? v.ranked[t] : t;
  if (!v.marginal) {
    if (pass == 2) {
      v.vc_cnt[r] = m;
      slot[0] = v.cg_noff[r];
    } else {
      v.cg_cnt[r * 2 + pass] = m;
      slot[0] = pass == 0 ? v.cg_noff[r] : v.cg_aoff[r];
    }
    return;
  }
  const uint32_t off = atomicAdd(pass == 0 ? &v.gst->out_nodes : &v.gst->out_arcs, m);
  const uint32_t cap = pass == 0 ? v.out_ncap : v.out_acap;
  if ((uint64_t)off + m > cap) atomicOr(&v.gst->overflow, 4);
  slot[0] = off;
  ResultHdr& hd = v.hdr[t];
  if (pass == 0) {
    hd.central = v.g.orig_id[v.sel_node[r]];
    hd.score_c = v.sel_sc[r];
    hd.score_m = v.sm[r];
    hd.cg_rank = r;
    hd.key = v.key[r];
    hd.node_off = off;
    hd.n_nodes = m;
  } else {
    hd.arc_off = off;
    hd.n_arcs = m;
    hd.wsum = 0;   // k_big_write adds the arcs' levels
  }
}

__global__ __launch_bounds__(kBlock) void k_big_write(FinalizeView v, int t, int pass,
                                                      const uint32_t* bm, uint32_t words,
                                                      const uint32_t* chunk, const uint64_t* slot) {
  __shared__ uint32_t s32[kBlock / kWave + 1];
  __shared__ uint64_t s_ws[kBlock / kWave + 1];
  const uint32_t w0 = blockIdx.x * kBigChunk + threadIdx.x * 4;
  uint32_t bits[4], c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    bits[k] = w0 + k < words ? big_bits(v, pass, bm[w0 + k], w0 + k) : 0u;
    c += __popc(bits[k]);
  }
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(c, s32, &tot);
  const uint64_t base = slot[0] + chunk[blockIdx.x] + ex;
  const DevGraphView& g = v.g;
  if (v.marginal && pass == 1) {
    uint64_t ws = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      for (uint32_t b = bits[k]; b; b &= b - 1) ws += g.act[(w0 + k) * 32 + (uint32_t)(__ffs(b) - 1)];
    ws = block_sum<uint64_t, kBlock>(ws, s_ws);
    if (threadIdx.x == 0 && ws) atomicAdd((unsigned long long*)&v.hdr[t].wsum, (unsigned long long)ws);
  }
  if (v.marginal && base + c > (pass == 0 ? v.out_ncap : v.out_acap)) return;   // overflow flagged
  uint64_t pos = base;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    for (uint32_t b = bits[k]; b; b &= b - 1) {
      const uint32_t id = (w0 + k) * 32 + (uint32_t)(__ffs(b) - 1);
      if (!v.marginal) {
        if (pass == 0) v.cg_nodes[pos] = id;
        else if (pass == 1) v.cg_arcs[pos] = id;
        else v.vc_tmp[pos] = g.int_id[id];
      } else if (pass == 0) {
        v.out_nodes[pos] = (int32_t)id;
      } else {
        int32_t* o = v.out_arcs + 3 * pos;
        o[0] = g.arc_src[id];
        o[1] = g.col[id];
        o[2] = g.label[id];
      }
      ++pos;
    }
  }
}

// V_C of every selected CG packed in CG order: workgroup r sums the counts of
// the CGs before it and copies CG r's list there.
__global__ __launch_bounds__(kBlock) void k_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp,
                                                    const uint64_t* cg_noff, const int32_t* nsel_p,
                                                    uint32_t* vc_off, int32_t* vc_nodes) {
  __shared__ uint32_t s32[kBlock / kWave + 1];
  const int nsel = *nsel_p;
  const int r = blockIdx.x;
  if (r >= nsel) {
    if (r == 0 && threadIdx.x == 0) vc_off[0] = 0;   // no CG: empty lists
    return;
  }
  uint32_t part = 0;
  for (int i = threadIdx.x; i < r; i += kBlock) part += vc_cnt[i];
  const uint32_t off = block_sum<uint32_t, kBlock>(part, s32);
  const uint32_t cnt = vc_cnt[r];
  if (threadIdx.x == 0) {
    vc_off[r] = off;
    if (r == nsel - 1) vc_off[nsel] = off + cnt;
  }
  const int32_t* src = vc_tmp + cg_noff[r];
  for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) vc_nodes[off + i] = src[i];
}

void launch_recover(const RecoverView& v, hipStream_t s) {
  if (v.n_inst <= 0) return;
  if (v.labelled) {
    const size_t wipe = (size_t)v.wipe_words;
    const unsigned gc = wipe ? 4096u : 64u;
    k_lr_clear<<<gc, kBlock, 0, s>>>(v, wipe);
    const unsigned grid = 1024;
    switch (v.TP) {
      case 4:
        k_lr_seed<4><<<v.n_inst, kBlock, 0, s>>>(v);
        for (int h = v.max_layer; h >= 1; --h) k_lr_layer<4><<<grid, kBlock, 0, s>>>(v, h);
        break;
      case 8:
        k_lr_seed<8><<<v.n_inst, kBlock, 0, s>>>(v);
        for (int h = v.max_layer; h >= 1; --h) k_lr_layer<8><<<grid, kBlock, 0, s>>>(v, h);
        break;
      default:
        k_lr_seed<16><<<v.n_inst, kBlock, 0, s>>>(v);
        for (int h = v.max_layer; h >= 1; --h) k_lr_layer<16><<<grid, kBlock, 0, s>>>(v, h);
        break;
    }
    k_lr_nodes<<<grid, kBlock, 0, s>>>(v);
    return;
  }
  // enough blocks per instance for a dense node set; tables of sparse ones
  // are small
  const unsigned gx = (unsigned)std::min<size_t>(64, ((size_t)v.dwords + kBlock - 1) / kBlock + 1);
  k_rec_clear<<<dim3(gx, (unsigned)v.n_inst), kBlock, 0, s>>>(v);
  const unsigned grid = 1024;
  switch (v.TP) {
    case 4:
      k_rec_seed<4><<<v.n_inst, kBlock, 0, s>>>(v);
      for (int h = v.max_layer; h >= 1; --h) k_rec_layer<4><<<grid, kBlock, 0, s>>>(v, h);
      break;
    case 8:
      k_rec_seed<8><<<v.n_inst, kBlock, 0, s>>>(v);
      for (int h = v.max_layer; h >= 1; --h) k_rec_layer<8><<<grid, kBlock, 0, s>>>(v, h);
      break;
    default:
      k_rec_seed<16><<<v.n_inst, kBlock, 0, s>>>(v);
      for (int h = v.max_layer; h >= 1; --h) k_rec_layer<16><<<grid, kBlock, 0, s>>>(v, h);
      break;
  }
}

void launch_finalize(const FinalizeView& v, hipStream_t s) {
  if (v.n_res > 0) k_finalize<<<dim3(v.n_res, 2), kBlock, 0, s>>>(v);
}

// The query's status, its result headers and as much of its output lists as
// the pinned staging buffers hold go straight into host memory: only the
// bytes that the query produced cross the bus, and no copy is launched.  The
// host copies a larger output itself.
__global__ __launch_bounds__(kBlock) void k_collect(CollectView v) {
  const uint32_t tn = min(v.st->out_nodes, v.cap_nodes);
  const uint32_t ta = min(v.st->out_arcs, v.cap_arcs) * 3u;   // 3 words per arc
  const uint32_t gt = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
  for (uint32_t i = gt; i < tn; i += stride) v.h_nodes[i] = v.nodes[i];
  for (uint32_t i = gt; i < ta; i += stride) v.h_arcs[i] = v.arcs[i];
  if (blockIdx.x == 0) {
    const uint32_t hw = v.n_hdr * (uint32_t)(sizeof(ResultHdr) / 4);
    for (uint32_t i = threadIdx.x; i < hw; i += kBlock)
      reinterpret_cast<uint32_t*>(v.h_hdr)[i] = reinterpret_cast<const uint32_t*>(v.hdr)[i];
    for (uint32_t i = threadIdx.x; i < sizeof(Status) / 4; i += kBlock)
      reinterpret_cast<uint32_t*>(v.h_st)[i] = reinterpret_cast<const uint32_t*>(v.st)[i];
  }
  __threadfence_system();
}

void launch_collect(const CollectView& v, hipStream_t s) {
  k_collect<<<kCollectGroups, kBlock, 0, s>>>(v);
}

void launch_big_finalize(const FinalizeView& v, int t, uint32_t* bm, uint32_t* chunk, uint64_t* slot,
                         hipStream_t s) {
  const uint32_t nw = (uint32_t)(((uint64_t)v.g.n + 31) / 32);
  const uint32_t aw = (uint32_t)(((uint64_t)v.g.A + 31) / 32);
  // CGs: nodes, V_C (from the node bitmap), then arcs
  const int order[3] = {0, 2, 1};
  for (int oi = 0; oi < (v.marginal ? 2 : 3); ++oi) {
    const int pass = v.marginal ? oi : order[oi];
    const uint32_t words = (pass == 1) ? aw : nw;
    const uint32_t nchunks = (words + kBigChunk - 1) / kBigChunk;
    const unsigned gc = (unsigned)std::min<uint32_t>(4096, (words + kBlock - 1) / kBlock);
    if (pass != 2) {   // pass 2 reuses the node bitmap of pass 0
      k_big_clear<<<gc, kBlock, 0, s>>>(bm, words);
      k_big_mark<<<2048, kBlock, 0, s>>>(v, t, pass, bm);
    }
    k_big_count<<<nchunks, kBlock, 0, s>>>(v, pass, bm, words, chunk);
    k_big_scan<<<1, kBlock, 0, s>>>(v, t, pass, chunk, nchunks, slot);
    k_big_write<<<nchunks, kBlock, 0, s>>>(v, t, pass, bm, words, chunk, slot);
  }
}

void launch_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp, const uint64_t* cg_noff,
                    const int32_t* nsel, uint32_t* vc_off, int32_t* vc_nodes, int max_sel,
                    hipStream_t s) {
  if (max_sel > 0) k_pack_vc<<<max_sel, kBlock, 0, s>>>(vc_cnt, vc_tmp, cg_noff, nsel, vc_off, vc_nodes);
}

}  // namespace raks
