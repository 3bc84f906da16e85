// cohort.hip -- kernels of the batched and served path: one level loop for
// every query of a cohort (layout and slot state in cohort.h).
//
// Per cohort level, three launches serve all queries:
//   k_co_scan     frontier scan over the segments that hold an expanding run:
//                 per node and query the frontier rule of Algorithm 1 (the
//                 same rule as the single-query scan, at the query's own
//                 level), the central-node test (Theorem identifyCG), the
//                 joining-flag block, and one staged expansion entry per node
//                 with the columns it expands for;
//   k_co_control  workgroup 0 turns the scan totals into the level's queue
//                 prefixes; workgroup 1 + q applies slot q's identification
//                 and termination rules (>= w CGs; the RPG check over V_C
//                 with Theorem 4, replayed over the levels it has missed);
//   k_co_expand   Algorithm 1 over tiles of 1024 consecutive examined arcs,
//                 reading the staged entries in place; an arc is read once
//                 for every query that expands its source node.
// After a query's runs: its CG selection input (k_co_cand_*), the final
// marginal decision (k_co_rpg_final) and its work counters (k_co_counters)
// come from its final hitting levels; recovery, ranking and output are the
// single-query kernels on views of its columns.
#include <hip/hip_ext.h>

#include <climits>

#include "cohort.h"
#include "common.h"
#include "kernels.h"

namespace raks {

namespace {

// Threads of the one-workgroup-per-slot kernels (control step, final RPG
// decision, candidate scan): small, so that such a workgroup finds room on a
// CU beside the recovery kernels of other queries' lanes, which it otherwise
// waits for on the level loop's critical path.
constexpr int kCtlT = 256;

__device__ inline uint8_t* seg_base(const CohortView& v, int seg) {
  return v.H + (size_t)seg * v.n_pad * 16;
}

// A node's reached mask in the cohort's width: a narrower cohort keeps its
// masks in 2 or 4 bytes per node, so that the expansion's random gathers touch
// a smaller array (it fits the 256 MB Infinity Cache on larger graphs).
__device__ inline uint64_t r_get(const CohortView& v, int64_t i) {
  if (v.rbytes == 2) return reinterpret_cast<const uint16_t*>(v.R)[i];
  if (v.rbytes == 4) return reinterpret_cast<const uint32_t*>(v.R)[i];
  return v.R[i];
}

__device__ inline void r_put(const CohortView& v, int64_t i, uint64_t x) {
  if (v.rbytes == 2) reinterpret_cast<uint16_t*>(v.R)[i] = (uint16_t)x;
  else if (v.rbytes == 4) reinterpret_cast<uint32_t*>(v.R)[i] = (uint32_t)x;
  else v.R[i] = x;
}

// Bit 7 of each byte of x (only those bits set) -> 4-bit mask.
__device__ inline uint32_t msb4(uint32_t x) { return ((x >> 7) * 0x10204080u) >> 28; }

// Per-column masks of a 16-byte row against per-column levels (7-bit
// compares: hitting levels stay below 127, INF 0xFF reads as 127).
struct RowMasks {
  uint32_t fin, eq, lt, inf;
};

__device__ inline RowMasks row_masks(const uint4 row, const uint32_t (&lvw)[4]) {
  RowMasks m = {0, 0, 0, 0};
  const uint32_t w[4] = {row.x, row.y, row.z, row.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t A = w[k] & 0x7F7F7F7Fu, B = lvw[k];
    const uint32_t ge = ((A | 0x80808080u) - B) & 0x80808080u;        // A >= B
    const uint32_t le = ((B | 0x80808080u) - A) & 0x80808080u;        // B >= A
    const uint32_t fn = (0xFEFEFEFEu - A) & 0x80808080u;              // A <= 126
    m.eq |= msb4(ge & le) << (4 * k);
    m.lt |= msb4(le & ~ge) << (4 * k);
    m.fin |= msb4(fn) << (4 * k);
  }
  m.inf = ~m.fin & 0xFFFFu;
  return m;
}

// Arcs of row v with level <= x, given its degree d and largest level.
__device__ inline uint32_t cnt_le(const DevGraphView& g, int32_t v, int x, uint32_t rs,
                                  uint32_t d, uint32_t amax) {
  if (x < 0) return 0;
  if (x >= (int)amax) return d;
  if (x < g.nbnd) return g.bnd[(size_t)x * g.n + v];
  uint32_t a = rs, b = rs + d;
  while (a < b) {
    const uint32_t m = (a + b) >> 1;
    if ((int)g.act_s[m] <= x) a = m + 1; else b = m;
  }
  return a - rs;
}

// The cohort's queries as one level's kernels see them.
struct SlotCfg {
  uint16_t gc, gm;      // central / marginal columns within the segment (running runs only)
  uint8_t q, seg, lq, blk_m;
};

struct CoCfg {
  int32_t nslot;
  uint32_t seg_mask;               // segments with a running run
  int32_t first[kCoSegs + 1];      // slots of segment s: sl[first[s] .. first[s+1])
  SlotCfg sl[kCoSlots];
  uint32_t lvw[kCoSegs][4];        // per-column local level (127 where no run expands)
  unsigned long long run;          // columns of running runs
};

// The fields of a slot that the level kernels use.
struct SlotLite {
  int32_t on, seg, c0, C, M, start, c_run, m_run, m_block;
};

// Loads the slot table, one slot per thread (threads 0..kCoSlots-1).
__device__ inline void load_lite(const CohortView& v, SlotLite* lite) {
  const int q = threadIdx.x;
  if (q < kCoSlots) {
    const CoSlot& s = v.slots[q];
    SlotLite x;
    x.on = s.active && (s.c_run || s.m_run);
    x.seg = s.seg; x.c0 = s.c0; x.C = s.C; x.M = s.M; x.start = s.start;
    x.c_run = s.c_run; x.m_run = s.m_run; x.m_block = s.m_block;
    lite[q] = x;
  }
}

// Built by thread 0 from the loaded slot table.
__device__ void build_cfg(const SlotLite* lite, int level, CoCfg& cfg) {
  uint8_t lv[kCoCols];
  for (int c = 0; c < kCoCols; ++c) lv[c] = 0x7F;
  int cnt[kCoSegs] = {0, 0, 0, 0};
  SlotCfg tmp[kCoSlots];
  int nt = 0;
  uint32_t segm = 0;
  for (int q = 0; q < kCoSlots; ++q) {
    const SlotLite& s = lite[q];
    if (!s.on) continue;
    SlotCfg c;
    c.q = (uint8_t)q;
    c.seg = (uint8_t)s.seg;
    c.lq = (uint8_t)(level - s.start);
    c.blk_m = (uint8_t)s.m_block;
    c.gc = s.c_run ? (uint16_t)(((1u << s.C) - 1u) << s.c0) : 0;
    c.gm = (s.m_run && s.M > 0) ? (uint16_t)(((1u << s.M) - 1u) << (s.c0 + s.C)) : 0;
    for (int j = 0; j < s.C + s.M; ++j) lv[s.seg * 16 + s.c0 + j] = c.lq;
    tmp[nt++] = c;
    ++cnt[s.seg];
    segm |= 1u << s.seg;
  }
  int acc = 0;
  for (int s = 0; s < kCoSegs; ++s) {
    cfg.first[s] = acc;
    acc += cnt[s];
  }
  cfg.first[kCoSegs] = acc;
  int pos[kCoSegs];
  for (int s = 0; s < kCoSegs; ++s) pos[s] = cfg.first[s];
  for (int i = 0; i < nt; ++i) cfg.sl[pos[tmp[i].seg]++] = tmp[i];
  cfg.nslot = nt;
  cfg.seg_mask = segm;
  unsigned long long run = 0;
  for (int i = 0; i < nt; ++i)
    run |= (unsigned long long)(tmp[i].gc | tmp[i].gm) << (16 * tmp[i].seg);
  cfg.run = run;
  for (int s = 0; s < kCoSegs; ++s)
    for (int k = 0; k < 4; ++k)
      cfg.lvw[s][k] = (uint32_t)lv[s * 16 + 4 * k] | ((uint32_t)lv[s * 16 + 4 * k + 1] << 8) |
                      ((uint32_t)lv[s * 16 + 4 * k + 2] << 16) |
                      ((uint32_t)lv[s * 16 + 4 * k + 3] << 24);
}

// Last index j in [lo, hi) with a[j * stride] <= x (non-decreasing, a[lo] <= x),
// by one wavefront, 64 probes per round.
__device__ inline int wave_search_s(const uint32_t* a, int lo, int hi, int stride, uint32_t x) {
  const int lane = lane_id();
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int idx = lo + lane * step;
    const bool ok = idx < hi && a[(size_t)idx * stride] <= x;
    const uint64_t b = __ballot(ok);
    const int L = 63 - __clzll((long long)b);
    lo += L * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

}  // namespace

// ------------------------------------------------------------- set-up ---

__global__ __launch_bounds__(kBlock) void k_co_init(CohortView v) {
  const size_t words = (size_t)kCoSegs * v.n_pad * 16 / 16;
  uint4* h = reinterpret_cast<uint4*>(v.H);
  const uint4 inf = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += (size_t)gridDim.x * kBlock)
    h[i] = inf;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < (size_t)v.n_pad;
       i += (size_t)gridDim.x * kBlock)
    v.R[i] = 0;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < kCoSlots; i += kBlock) v.slots[i] = CoSlot{};
    if (threadIdx.x == 0) *v.acc = CoAcc{};
  }
}

struct AdmitArgs {
  CoSlot s[8];
  int32_t idx[8];
  int32_t n;
};

// Writes the admitted slots and clears their RPG records.
__global__ __launch_bounds__(kBlock) void k_co_admit(CohortView v, AdmitArgs a) {
  for (int i = 0; i < a.n; ++i) {
    for (int r = threadIdx.x; r < kMaxW; r += kBlock) {
      a.s[i].has_rpg[r] = 0;
      a.s[i].sm[r] = 0;
      a.s[i].key[r] = 0;
    }
  }
  if ((int)threadIdx.x < a.n) v.slots[a.idx[threadIdx.x]] = a.s[threadIdx.x];
}

// Keyword nodes at level 0 in the query's columns (the columns are INF).
__global__ __launch_bounds__(kBlock) void k_co_seed(uint8_t* Hs, const int32_t* kw_nodes, SeedList s) {
  const uint32_t total = s.prefix[s.T];
  for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < total; p += gridDim.x * kBlock) {
    int i = 0;
    while (p >= s.prefix[i + 1]) ++i;
    const int32_t n = kw_nodes[s.start[i] + (p - s.prefix[i])];
    Hs[(int64_t)n * 16 + i] = 0;
  }
}

// --------------------------------------------------------- frontier scan ---
//
// Node v is in run g's level-l frontier (l the query's local level) exactly
// when some keyword of g reached it at l, or it was reached before l, its row
// has an arc of level > l-1 and it was not blocked (row of g complete) by
// l-1: the rule of the single-query scan, applied per run.  A frontier node
// that is not blocked expands for the run's keywords with h <= l.  The entry
// covers the union of the row slices its runs need; the expansion filters
// every arc by its level and each column's level.
__global__ __launch_bounds__(kBlock) void k_co_scan(CohortView v, DevGraphView g, int level) {
  __shared__ CoCfg cfg;
  __shared__ SlotLite s_lite[kCoSlots];
  __shared__ uint32_t s_ncand[kCoSlots];
  __shared__ unsigned long long s_gf;
  __shared__ uint32_t s_m32[(kBlock / kWave + 1) * 2];
  load_lite(v, s_lite);
  __syncthreads();
  if (threadIdx.x == 0) {
    build_cfg(s_lite, level, cfg);
    s_gf = 0;
  }
  if (threadIdx.x < kCoSlots) s_ncand[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t segm = cfg.seg_mask;
  const int64_t wg0 = (int64_t)blockIdx.x * v.cpw * kScanNodes;
  const int64_t wg1 = min(wg0 + (int64_t)v.cpw * kScanNodes, (int64_t)v.n_pad);
  uint32_t cq = 0, cw = 0;
  unsigned long long gf = 0;
  if (segm) {
#pragma unroll 1
    for (int64_t b0 = wg0; b0 < wg1; b0 += kBlock) {
      const int64_t vv = b0 + threadIdx.x;
      const int32_t node = (int32_t)vv;
      unsigned long long en = 0, eo = 0, rfin = 0;
      int hi_lv = -1, lo_lv = INT_MAX;
      uint32_t amax = 0;
      if (vv < v.n) {
        amax = g.row_amax[vv];
#pragma unroll 1
        for (int s = 0; s < kCoSegs; ++s) {
          if (!((segm >> s) & 1u)) continue;
          const uint4 row = reinterpret_cast<const uint4*>(seg_base(v, s))[vv];
          if ((row.x & row.y & row.z & row.w) == 0xFFFFFFFFu) continue;
          const RowMasks m = row_masks(row, cfg.lvw[s]);
          rfin |= (unsigned long long)m.fin << (16 * s);
          for (int i = cfg.first[s]; i < cfg.first[s + 1]; ++i) {
            const SlotCfg sc = cfg.sl[i];
#pragma unroll
            for (int grp = 0; grp < 2; ++grp) {
              const uint32_t G = grp ? sc.gm : sc.gc;
              const uint32_t mn = m.eq & G, mo = m.lt & G;
              if (!(mn | mo)) continue;
              const bool blk = grp ? sc.blk_m != 0 : true;
              const bool inF = mn != 0 || ((int)amax >= (int)sc.lq && !(blk && mo == G));
              if (!inF) continue;
              gf |= 1ull << (2 * sc.q + grp);
              const bool complete = (m.fin & G) == G;
              if (!grp && complete && mn) atomicAdd(&s_ncand[sc.q], 1u);
              if (blk && complete) continue;
              en |= (unsigned long long)mn << (16 * s);
              eo |= (unsigned long long)mo << (16 * s);
              hi_lv = max(hi_lv, (int)sc.lq);
              if (mo) lo_lv = min(lo_lv, (int)sc.lq);
            }
          }
        }
      }
      if (vv < v.n) {
        // the reached mask of the running columns, as the expansion reads it
        const unsigned long long rnew = rfin & cfg.run;
        if (r_get(v, vv) != rnew) r_put(v, vv, rnew);
      }
      CoEntry e = {};
      uint32_t work = 0;
      if (en | eo) {
        const uint32_t rs = g.row_ptr[node];
        const uint32_t d = g.row_ptr[node + 1] - rs;
        if (d) {
          const uint32_t hi = cnt_le(g, node, hi_lv, rs, d, amax);
          const uint32_t st = en ? 0u : cnt_le(g, node, lo_lv - 1, rs, d, amax);
          work = hi > st ? hi - st : 0u;
          e.arc = rs + st;
          e.nlo = (uint32_t)en;
          e.nhi = (uint32_t)(en >> 32);
          e.olo = (uint32_t)eo;
          e.ohi = (uint32_t)(eo >> 32);
        }
      }
      uint32_t x[2] = {work ? 1u : 0u, work}, t[2];
      block_exclusive_scan_multi<2, kBlock, uint32_t>(x, t, s_m32);
      if (work) {
        e.pre = cw + x[1];
        v.stage[wg0 + cq + x[0]] = e;
      }
      cq += t[0];
      cw += t[1];
    }
  }
  if (gf) atomicOr(&s_gf, gf);
  __syncthreads();
  if (threadIdx.x == 0) {
    v.tot[blockIdx.x] = make_uint2(cq, cw);
    if (s_gf) atomicOr(&v.acc->gfront[level & 1], s_gf);
  }
  if (threadIdx.x < kCoSlots && s_ncand[threadIdx.x])
    atomicAdd(&v.acc->ncand[level & 1][threadIdx.x], s_ncand[threadIdx.x]);
}

// ---------------------------------------------------------- marginal run ---
//
// RPG identification of a slot (Section 4.2.3) for levels from..to, given
// hitting levels up to `to`: D_j = min over a CG's central-keyword nodes of
// h_j (Definition 3), S^m = max_j D_j (Eq. 5).  A CG gets its RPG at level
// S^m (values never change once written, and later ones are larger), so the
// RPG set at any level lv <= to is {CG : S^m <= lv}; the stop rules (every CG
// has an RPG; Theorem 4 with the k-th RPG in (key, S^c, CG rank) order) are
// checked level by level from `from` on.  Returns the first level where a
// rule holds, or -1.  The CGs with an RPG at that level (or at `to`) are
// written back with S^m, key and D_j.  One workgroup of kCtlT threads.
__device__ int co_rpg_eval(const CohortView& v, int q, const CoSlot& s, int from, int to) {
  __shared__ uint32_t s_dm[kMaxW * kMaxKw];
  __shared__ int32_t s_lvl[kMaxW], s_sc[kMaxW], s_old[kMaxW];
  __shared__ int64_t s_key[kMaxW];
  __shared__ int32_t s_stop, s_n, s_kth, s_minsc;
  const int nsel = s.nsel, M = s.M;
  const int64_t gn = s.gn, gd = s.gd;
  for (int i = threadIdx.x; i < nsel * kMaxKw; i += kCtlT) s_dm[i] = kInf;
  for (int i = threadIdx.x; i < nsel; i += kCtlT) {
    s_old[i] = s.has_rpg[i];
    s_lvl[i] = s_old[i] ? s.sm[i] : INT_MAX;
    s_sc[i] = s.sel_sc[i];
  }
  if (threadIdx.x == 0) s_stop = -1;
  __syncthreads();
  // D_j: the running minima that k_co_dmin keeps (every level written so far
  // is <= to)
  const uint32_t* gdm = v.dmin + (size_t)q * kMaxW * kMaxKw;
  for (int i = threadIdx.x; i < nsel * kMaxKw; i += kCtlT) {
    const uint32_t h = gdm[i];
    if (!s_old[i / kMaxKw] && h <= (uint32_t)to) s_dm[i] = h;
  }
  __syncthreads();
  for (int rr = threadIdx.x; rr < nsel; rr += kCtlT) {
    if (s_old[rr]) {
      s_key[rr] = s.key[rr];
      continue;
    }
    int mx = 0;
    bool all = true;
    for (int j = 0; j < M; ++j) {
      const int d = (int)s_dm[rr * kMaxKw + j];
      all &= d != kInf;
      mx = d > mx ? d : mx;
    }
    s_lvl[rr] = all ? mx : INT_MAX;
    s_key[rr] = all ? (s.score_mode ? (int64_t)s_sc[rr] * mx : gn * s_sc[rr] + (gd - gn) * mx) : 0;
  }
  __syncthreads();
  for (int lv = from; lv <= to; ++lv) {
    if (threadIdx.x == 0) { s_n = 0; s_kth = -1; s_minsc = INT_MAX; }
    __syncthreads();
    for (int rr = threadIdx.x; rr < nsel; rr += kCtlT)
      if (s_lvl[rr] <= lv) atomicAdd(&s_n, 1);
    __syncthreads();
    const int n = s_n;
    bool stop = n == nsel;
    if (!stop && n >= s.k) {
      for (int rr = threadIdx.x; rr < nsel; rr += kCtlT) {
        if (s_lvl[rr] <= lv) {
          int rank = 0;
          for (int o = 0; o < nsel; ++o) {
            if (s_lvl[o] > lv) continue;
            rank += s_key[o] < s_key[rr] ||
                    (s_key[o] == s_key[rr] && (s_sc[o] < s_sc[rr] || (s_sc[o] == s_sc[rr] && o < rr)));
          }
          if (rank == s.k - 1) s_kth = rr;
        } else {
          atomicMin(&s_minsc, s_sc[rr]);
        }
      }
      __syncthreads();
      const int kth = s_kth;
      const int64_t bound = s.score_mode ? (int64_t)s_minsc * s_lvl[kth]
                                         : gn * (int64_t)s_minsc + (gd - gn) * (int64_t)s_lvl[kth];
      stop = s.rerank ? s_key[kth] < bound : s_key[kth] <= bound;
    }
    if (stop) {
      if (threadIdx.x == 0) s_stop = lv;
      break;
    }
    __syncthreads();
  }
  __syncthreads();
  const int fin = s_stop >= 0 ? s_stop : to;
  for (int rr = threadIdx.x; rr < nsel; rr += kCtlT) {
    if (s_old[rr]) continue;
    const bool has = s_lvl[rr] <= fin;
    s.has_rpg[rr] = has ? 1 : 0;
    s.sm[rr] = has ? s_lvl[rr] : 0;
    s.key[rr] = has ? s_key[rr] : 0;
    for (int j = 0; j < M; ++j) s.dmin[rr * kMaxKw + j] = (uint8_t)s_dm[rr * kMaxKw + j];
  }
  __syncthreads();
  return s_stop;
}

// ------------------------------------------------------------- control ---

__device__ inline void co_publish_slot(CoLevelMirror* mir, int q, const CoSlot& s, uint64_t seq) {
  CoSlotMirror m;
  m.active = s.active;
  m.c_run = s.c_run;
  m.m_run = s.m_run;
  m.c_end = s.c_end;
  m.c_reason = s.c_reason;
  m.m_xend = s.m_xend;
  m.m_xreason = s.m_xreason;
  m.m_end = s.m_end;
  m.m_reason = s.m_reason;
  m.checked = s.checked;
  m.vc_ready = s.vc_ready;
  m.nsel = s.nsel;
  m.ncand = s.ncand;
  m.pad = 0;
  m.seq = 0;
  mir->slot[q] = m;
  __threadfence_system();
  *reinterpret_cast<volatile uint64_t*>(&mir->slot[q].seq) = seq;
}

__global__ __launch_bounds__(kCtlT) void k_co_control(CohortView v, int level, uint64_t seq) {
  if (blockIdx.x == 0) {
    // queue prefixes of the level: each thread takes a run of `per` scan
    // workgroups
    __shared__ uint32_t s_m32[(kCtlT / kWave + 1) * 2];
    const int nb = v.nblocks;
    const int per = (nb + kCtlT - 1) / kCtlT;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t x[2] = {0, 0}, tt[2];
    for (int b = b0; b < b1; ++b) {
      const uint2 t = v.tot[b];
      x[0] += t.x;
      x[1] += t.y;
    }
    block_exclusive_scan_multi<2, kCtlT, uint32_t>(x, tt, s_m32);
    uint32_t q = x[0], w = x[1];
    for (int b = b0; b < b1; ++b) {
      const uint2 t = v.tot[b];
      v.qpre[b] = q;
      v.wpre[b] = w;
      q += t.x;
      w += t.y;
    }
    if (threadIdx.x == 0) {
      v.qpre[nb] = tt[0];
      v.wpre[nb] = tt[1];
      v.wtot[0] = tt[1];
      v.wtot[1] = tt[0];
      v.acc->gfront[(level + 1) & 1] = 0;
    }
    if (threadIdx.x < kCoSlots) v.acc->ncand[(level + 1) & 1][threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      CoLevelMirror* mir = &v.mirror->lvl[level & (kCoMirrors - 1)];
      mir->W = tt[1];
      mir->nq = tt[0];
      __threadfence_system();
      *reinterpret_cast<volatile uint64_t*>(&mir->seq) = seq;
    }
    return;
  }
  const int q = (int)blockIdx.x - 1;
  __shared__ CoSlot s;
  __shared__ int32_t s_go, s_live;
  if (threadIdx.x == 0) {
    s = v.slots[q];
    s_go = 0;
    s_live = s.active && (s.c_run || s.m_run);
    if (s_live) {
      const int l = level - s.start;
      const unsigned long long gf = v.acc->gfront[level & 1];
      if (s.c_run) {
        if (!((gf >> (2 * q)) & 1ull)) {
          s.c_end = l; s.c_reason = END_EXHAUSTED; s.c_run = 0;
        } else {
          s.ncand += v.acc->ncand[level & 1][q];
          if (s.ncand >= (uint32_t)s.w) {
            s.c_end = l; s.c_reason = END_STOP; s.c_run = 0;
          } else if (l >= s.max_level) {
            s.c_end = l; s.c_reason = END_LEVEL_BOUND; s.c_run = 0;
          }
        }
      }
      if (s.m_run) {
        if (!((gf >> (2 * q + 1)) & 1ull)) {
          s.m_xend = l; s.m_xreason = END_EXHAUSTED; s.m_run = 0;
        } else if (s.vc_ready) {
          if (s.nsel == 0) {
            s.m_run = 0;   // no CG: the marginal run does not take place
          } else {
            s_go = 1;      // RPG check below
          }
        } else if (l >= s.max_level) {
          s.m_xend = l; s.m_xreason = END_LEVEL_BOUND; s.m_run = 0;
        }
      }
    }
  }
  __syncthreads();
  if (s_go) {
    const int l = level - s.start;
    const int stop = co_rpg_eval(v, q, s, s.checked + 1, l);
    if (threadIdx.x == 0) {
      s.checked = l;
      if (stop >= 0) {
        s.m_end = stop; s.m_reason = END_STOP; s.m_run = 0;
      } else if (l >= s.max_level) {
        s.m_xend = l; s.m_xreason = END_LEVEL_BOUND; s.m_run = 0;
      }
    }
    __syncthreads();
  }
  // only a slot whose runs were still going is written back: a finished
  // query's slot belongs to its post-processing (other streams) until reuse
  if (threadIdx.x == 0) {
    if (s_live) v.slots[q] = s;
    co_publish_slot(&v.mirror->lvl[level & (kCoMirrors - 1)], q, s, seq);
  }
}

// ------------------------------------------------------------ expansion ---
//
// Algorithm 1 at cohort level `level`.  Tile of 1024 consecutive examined
// arcs; the scan workgroups holding its first and last arc are found in the
// level's arc prefix, its entries in their staging slots, and an owner map
// gives every arc its entry.  For arc f -> n with level a the columns to
// relax are the entry's new columns whose query level is >= a and its old
// columns whose query level equals a (precomputed per a); every one of them
// still INF at n gets its query's level + 1.  Writes need no atomics: every
// write of a level stores the same value into a byte that was INF (Theorem
// "lockfree").
template <int TILE>
__global__ __launch_bounds__(kBlock) void k_co_expand(CohortView v, DevGraphView g, int level) {
  __shared__ unsigned long long s_ge[256], s_eq[256];
  __shared__ uint8_t s_lv1[kCoCols];
  __shared__ uint8_t s_lvc[kCoCols];
  __shared__ unsigned long long s_run;
  __shared__ uint32_t s_base[TILE];
  __shared__ unsigned long long s_nm[TILE], s_om[TILE];
  __shared__ uint16_t s_own[TILE];
  __shared__ uint32_t s_scan[kBlock / kWave + 1];
  __shared__ int32_t s_e[4];
  __shared__ SlotLite s_lite[kCoSlots];
  const uint32_t W = v.wtot[0];
  if (W == 0) return;
  load_lite(v, s_lite);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int c = 0; c < kCoCols; ++c) { s_lvc[c] = 0xFF; s_lv1[c] = 0; }
    for (int q = 0; q < kCoSlots; ++q) {
      const SlotLite& s = s_lite[q];
      if (!s.on) continue;
      const int lq = level - s.start;
      for (int j = 0; j < s.C + s.M; ++j) {
        const bool on = j < s.C ? s.c_run != 0 : s.m_run != 0;
        const int c = s.seg * 16 + s.c0 + j;
        s_lvc[c] = (uint8_t)lq;
        s_lv1[c] = (uint8_t)(lq + 1);
        if (on) run |= 1ull << c;
      }
    }
    s_run = run;
  }
  __syncthreads();
  {
    const int a = threadIdx.x;   // kBlock == 256 levels
    unsigned long long ge = 0, eq = 0;
    const unsigned long long run = s_run;
    for (int c = 0; c < kCoCols; ++c) {
      if (!((run >> c) & 1ull)) continue;
      if ((int)s_lvc[c] >= a) ge |= 1ull << c;
      if ((int)s_lvc[c] == a) eq |= 1ull << c;
    }
    s_ge[a] = ge;
    s_eq[a] = eq;
  }
  __syncthreads();
  if (s_run == 0) return;
  constexpr int IPT = TILE / kBlock;
  const int nb = v.nblocks;
  const int64_t per_wg = (int64_t)v.cpw * kScanNodes;
  const uint32_t ntiles = (W + TILE - 1) / TILE;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t w0 = tile * TILE;
    const uint32_t w1 = min(W, w0 + (uint32_t)TILE);
    if (wave_id() == 0) {
      // entries holding the tile's first and last arcs (global entry numbers)
#pragma unroll 1
      for (int k = 0; k < 2; ++k) {
        const uint32_t x = k == 0 ? w0 : w1 - 1;
        const int b = wave_search_s(v.wpre, 0, nb + 1, 1, x);
        const uint32_t nqb = v.qpre[b + 1] - v.qpre[b];
        const int j = wave_search_s(&v.stage[b * per_wg].pre, 0, (int)nqb,
                                    (int)(sizeof(CoEntry) / 4), x - v.wpre[b]);
        if (lane_id() == 0) { s_e[2 * k] = (int)(v.qpre[b] + j); s_e[2 * k + 1] = b; }
      }
    }
    for (int i = threadIdx.x; i < TILE; i += kBlock) s_own[i] = 0;
    __syncthreads();
    const int E0 = s_e[0], bA = s_e[1], E1 = s_e[2], bB = s_e[3];
    const int cnt = E1 - E0 + 1;
    for (int t = threadIdx.x; t < cnt; t += kBlock) {
      const uint32_t E = (uint32_t)(E0 + t);
      // scan workgroup of entry E: last b in [bA, bB] with qpre[b] <= E
      int b = bA;
      if (bB > bA) b = upper_index<uint32_t>(v.qpre, bA, bB + 1, E);
      const CoEntry e = v.stage[b * per_wg + (E - v.qpre[b])];
      const uint32_t off = v.wpre[b] + e.pre;
      s_base[t] = e.arc - off + w0;   // arc of tile item i is s_base[t] + i
      s_nm[t] = ((unsigned long long)e.nhi << 32) | e.nlo;
      s_om[t] = ((unsigned long long)e.ohi << 32) | e.olo;
      s_own[off > w0 ? off - w0 : 0] = (uint16_t)t;
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
    for (int k = 0; k < IPT; ++k)
      s_own[threadIdx.x * IPT + k] = (uint16_t)(pre > loc[k] ? pre : loc[k]);
    __syncthreads();
    // all of the thread's arcs at once: their levels and targets, then the
    // targets' reached masks, then the writes, so that a wavefront has IPT
    // independent gathers in flight instead of one dependent chain per arc
    int32_t nbv[IPT];
    unsigned long long wantv[IPT], rv[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const uint32_t i = k * kBlock + threadIdx.x;
      wantv[k] = 0;
      nbv[k] = 0;
      if (w0 + i < w1) {
        const int j = s_own[i];
        const uint32_t e = s_base[j] + i;
        const uint32_t a = g.act_s[e];
        nbv[k] = g.col_s[e];
        wantv[k] = (s_nm[j] & s_ge[a]) | (s_om[j] & s_eq[a]);
      }
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) rv[k] = wantv[k] ? r_get(v, nbv[k]) : ~0ull;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // columns that have not reached the target (as of the start of the level)
      unsigned long long mm = ~rv[k] & wantv[k];
      while (mm) {
        const int c = __ffsll(mm) - 1;
        mm &= mm - 1;
        seg_base(v, c >> 4)[(size_t)nbv[k] * 16 + (c & 15)] = s_lv1[c];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- CG selection ---
//
// After slot q's central run ended at level `end`, its CGs are exactly the
// nodes whose central row is complete with a maximum <= end (each was
// identified at the level of its row maximum).  Those of earlier levels (fewer
// than w) go first in any order, those of the last level follow in node
// order, which is what the top-w selection expects.

__global__ __launch_bounds__(kBlock) void k_co_cand_count(CoCandView cv, int32_t n, int32_t n_pad,
                                                          int32_t cpw) {
  __shared__ uint32_t s_red[kBlock / kWave + 1];
  const int64_t wg0 = (int64_t)blockIdx.x * cpw * kScanNodes;
  const int64_t wg1 = min(wg0 + (int64_t)cpw * kScanNodes, (int64_t)n);
  uint32_t last = 0, prev = 0;
  for (int64_t v = wg0 + threadIdx.x; v < wg1; v += kBlock) {
    const uint8_t* r = cv.Hc + v * 16;
    bool complete = true;
    int mx = 0;
    for (int j = 0; j < cv.C; ++j) {
      const int h = r[j];
      complete &= h != kInf;
      mx = h > mx ? h : mx;
    }
    if (complete && mx <= cv.end) {
      if (mx == cv.end) ++last; else ++prev;
    }
  }
  const uint32_t tl = block_sum<uint32_t, kBlock>(last, s_red);
  const uint32_t tp = block_sum<uint32_t, kBlock>(prev, s_red);
  if (threadIdx.x == 0) {
    cv.cnt[blockIdx.x] = tl;
    if (tp) atomicAdd(&cv.cursor[1], tp);
  }
}

__global__ __launch_bounds__(kCtlT) void k_co_cand_scan(CoCandView cv, int32_t nb) {
  __shared__ uint32_t s_m32[kCtlT / kWave + 1];
  const uint32_t prev = cv.cursor[1];
  const int per = (nb + kCtlT - 1) / kCtlT;
  const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += cv.cnt[b];
  uint32_t tot;
  uint32_t ex = block_exclusive_scan<uint32_t, kCtlT>(sum, s_m32, &tot);
  for (int b = b0; b < b1; ++b) {
    cv.off[b] = prev + ex;
    ex += cv.cnt[b];
  }
  if (threadIdx.x == 0) {
    RunStatus st = {};
    st.ncand_total = prev + tot;
    st.ncand_level = tot;
    *cv.st = st;
    cv.cursor[0] = 0;
    cv.cursor[1] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_co_cand_write(CoCandView cv, int32_t n, int32_t cpw) {
  __shared__ uint32_t s_red[kBlock / kWave + 1];
  const int64_t wg0 = (int64_t)blockIdx.x * cpw * kScanNodes;
  const int64_t wg1 = min(wg0 + (int64_t)cpw * kScanNodes, (int64_t)n);
  uint32_t base = cv.off[blockIdx.x];
  for (int64_t b0 = wg0; b0 < wg1; b0 += kBlock) {
    const int64_t v = b0 + threadIdx.x;
    bool keep = false, last = false;
    uint64_t key = 0;
    if (v < wg1) {
      const uint8_t* r = cv.Hc + v * 16;
      bool complete = true;
      int mx = 0, sum = 0;
      for (int j = 0; j < cv.C; ++j) {
        const int h = r[j];
        complete &= h != kInf;
        mx = h > mx ? h : mx;
        sum += h == kInf ? 0 : h;
      }
      keep = complete && mx <= cv.end;
      last = keep && mx == cv.end;
      key = ((uint64_t)mx << 48) | ((uint64_t)sum << 32) | (uint32_t)cv.orig_id[v];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(last ? 1u : 0u, s_red, &tot);
    if (last) cv.cand[base + ex] = key;
    else if (keep) cv.cand[atomicAdd(&cv.cursor[0], 1u)] = key;
    base += tot;
  }
}

__global__ __launch_bounds__(kBlock) void k_co_cg_done(CohortView v, int q, const Status* gst,
                                                       uint64_t seq) {
  const int32_t ovf = gst->overflow & (1 | kOvfBig0);
  const int32_t nsel = gst->nsel;
  // the D_j minima of the new V_C lists start at INF
  uint32_t* dm = v.dmin + (size_t)q * kMaxW * kMaxKw;
  for (int i = threadIdx.x; i < kMaxW * kMaxKw; i += kBlock) dm[i] = kInf;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!ovf) {
      v.slots[q].nsel = nsel;
      v.slots[q].vc_ready = 1;
    }
    v.mirror->cg_ovf[q] = ovf;
    v.mirror->cg_nsel[q] = nsel;
    __threadfence_system();
    *reinterpret_cast<volatile uint64_t*>(&v.mirror->cg_seq[q]) = seq;
  }
}

// D_j = min over a CG's V_C nodes of its marginal level j (Definition 3),
// kept as running minima: levels never change once written, so a rescan
// only lowers them.  Grid-stride over the V_C entries of every slot whose
// marginal run is checked at this level (or of slot `only`), skipping CGs
// that already have their RPG.
__global__ __launch_bounds__(kBlock) void k_co_dmin(CohortView v, int only) {
  for (int q = 0; q < kCoSlots; ++q) {
    if (only >= 0 && q != only) continue;
    const CoSlot& s = v.slots[q];
    if (!s.active || !s.vc_ready || s.M == 0 || s.nsel == 0) continue;
    if (only < 0 && !s.m_run) continue;
    const int nsel = s.nsel, M = s.M;
    const uint32_t total = s.vc_off[nsel];
    const uint8_t* Hm = seg_base(v, s.seg) + s.c0 + s.C;
    uint32_t* dm = v.dmin + (size_t)q * kMaxW * kMaxKw;
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < total; p += gridDim.x * kBlock) {
      const int rr = upper_index<uint32_t>(s.vc_off, 0, nsel + 1, p);
      if (s.has_rpg[rr]) continue;
      const uint8_t* row = Hm + (size_t)s.vc_nodes[p] * 16;
      for (int j = 0; j < M; ++j) {
        const uint32_t h = row[j];
        if (h != kInf && h < dm[rr * kMaxKw + j]) atomicMin(&dm[rr * kMaxKw + j], h);
      }
    }
  }
}

// ------------------------------------------------- after the exploration ---

// The marginal run's end: decided already by a control step (Theorem 4 or
// every CG with an RPG), or replayed here up to where the exploration ended
// (the level before an empty frontier, or the level bound).
__global__ __launch_bounds__(kCtlT) void k_co_rpg_final(CohortView v, int q) {
  __shared__ CoSlot s;
  __shared__ int32_t s_go;
  if (threadIdx.x == 0) {
    s = v.slots[q];
    s_go = 0;
    if (s.M == 0 || !s.vc_ready || s.nsel == 0) {
      s.m_end = -1;
      s.m_reason = END_NONE;
    } else if (s.m_end < 0) {
      s_go = 1;
    }
  }
  __syncthreads();
  if (s_go) {
    const int to = s.m_xreason == END_EXHAUSTED ? s.m_xend - 1 : s.m_xend;
    const int stop = co_rpg_eval(v, q, s, s.checked + 1, to);
    if (threadIdx.x == 0) {
      if (stop >= 0) { s.m_end = stop; s.m_reason = END_STOP; }
      else { s.m_end = s.m_xend; s.m_reason = s.m_xreason; }
      s.checked = max(s.checked, to);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) v.slots[q] = s;
}

// The lane's run status from the slot: levels, end reasons, CG count; the
// counters are added by k_co_counters.
__global__ void k_co_post_init(const CoSlot* slot, Status* gst) {
  const CoSlot s = *slot;
  RunStatus a = {}, b = {};
  a.end_level = s.c_end;
  a.end_reason = s.c_reason;
  a.levels = s.c_end + 1;
  a.ncand_total = s.ncand;
  if (s.m_end >= 0) {
    b.end_level = s.m_end;
    b.end_reason = s.m_reason;
    b.levels = s.m_end + 1;
  } else {
    b.end_level = -1;
    b.end_reason = END_NONE;
  }
  gst->run[0] = a;
  gst->run[1] = b;
}

// Counters of one run at one node from its final hitting levels h[0..T)
// (entries above the run's end level L are not part of the run).  The node is
// a frontier at the levels where a keyword reached it, and at every level l in
// (hmin, U] with U = min(L, largest arc level, the level its row became
// complete when the run blocks); at each such level below L where it is not
// blocked it expands: its whole row is scanned (e_arc), once per keyword with
// h <= l (e_alg), and its arcs of level <= l pass the gate.
struct RunCnt {
  uint64_t fr, ea, eg, gp, hw;
};

__device__ inline void run_counts(const uint8_t* h, int T, int L, bool blk, const DevGraphView& g,
                                  int32_t v, uint32_t rs, uint32_t d, uint32_t amax, RunCnt& o) {
  int vals[kMaxKw];
  int nv = 0;
  bool complete = true;
  for (int j = 0; j < T; ++j) {
    const int x = h[j];
    if (x == kInf || x > L) { complete = false; continue; }
    // insertion into the sorted list
    int p = nv++;
    while (p > 0 && vals[p - 1] > x) { vals[p] = vals[p - 1]; --p; }
    vals[p] = x;
    if (x >= 1) ++o.hw;
  }
  if (nv == 0) return;
  const int hmin = vals[0];
  const int done = complete ? vals[nv - 1] : INT_MAX;
  const int U = min(min(L, (int)amax), blk ? done : INT_MAX);
  int p = 0;   // values <= l: vals[0..p)
  for (int l = hmin; l <= L; ++l) {
    bool point = false;
    while (p < nv && vals[p] <= l) { point |= vals[p] == l; ++p; }
    const bool inF = point || (l > hmin && l <= U);
    if (!inF) {
      if (l > U && p == nv) break;   // no value left above l and no retention
      continue;
    }
    ++o.fr;
    if (l < L && !(blk && done <= l)) {
      o.ea += d;
      o.eg += (uint64_t)d * p;
      o.gp += cnt_le(g, v, l, rs, d, amax);
    }
  }
}

// One pass over the query's rows: counters, copy-out and reset.  Runs on the
// query's lane stream while the next levels run: the level kernels may write
// other columns of the same rows, so the reset stores only the query's own
// bytes (and only those that are not INF already).
__global__ __launch_bounds__(kBlock) void k_co_finish(CoFinishView fv, DevGraphView g) {
  __shared__ uint64_t s_multi[(kBlock / kWave + 1) * 10];
  const CoSlot s = *fv.slot;
  const int Lc = s.c_end, Lm = s.m_end;
  const int T = fv.C + fv.M;
  uint64_t acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < fv.n_pad;
       v += (int64_t)gridDim.x * kBlock) {
    uint4* rowp = reinterpret_cast<uint4*>(fv.seg) + v;
    const uint4 row = *rowp;
    uint8_t b[16], out[16];
    __builtin_memcpy(b, &row, 16);
#pragma unroll
    for (int j = 0; j < 16; ++j) out[j] = kInf;
    for (int j = 0; j < T; ++j) out[j] = b[fv.c0 + j];
    if (v < g.n && ((row.x & row.y & row.z & row.w) != 0xFFFFFFFFu)) {
      const uint32_t rs = g.row_ptr[v], d = g.row_ptr[v + 1] - rs, amax = g.row_amax[v];
      RunCnt a = {0, 0, 0, 0, 0};
      run_counts(out, fv.C, Lc, true, g, (int32_t)v, rs, d, amax, a);
      acc[0] += a.fr; acc[1] += a.ea; acc[2] += a.eg; acc[3] += a.gp; acc[4] += a.hw;
      if (Lm >= 0) {
        RunCnt c = {0, 0, 0, 0, 0};
        run_counts(out + fv.C, fv.M, Lm, fv.m_block != 0, g, (int32_t)v, rs, d, amax, c);
        acc[5] += c.fr; acc[6] += c.ea; acc[7] += c.eg; acc[8] += c.gp; acc[9] += c.hw;
      }
    }
    uint4 o;
    __builtin_memcpy(&o, out, 16);
    if (fv.TPq == 4) reinterpret_cast<uint32_t*>(fv.Hq)[v] = o.x;
    else if (fv.TPq == 8) reinterpret_cast<uint2*>(fv.Hq)[v] = make_uint2(o.x, o.y);
    else reinterpret_cast<uint4*>(fv.Hq)[v] = o;
    uint8_t* rb = reinterpret_cast<uint8_t*>(rowp);
    for (int j = 0; j < T; ++j)
      if (out[j] != kInf) rb[fv.c0 + j] = kInf;
  }
  uint64_t tot[10];
  block_exclusive_scan_multi<10, kBlock>(acc, tot, s_multi);
  if (threadIdx.x < 10 && tot[threadIdx.x]) {
    const int k = threadIdx.x;
    RunStatus& rs = fv.gst->run[k / 5];
    unsigned long long* dst = nullptr;
    switch (k % 5) {
      case 0: dst = reinterpret_cast<unsigned long long*>(&rs.frontier_sum); break;
      case 1: dst = reinterpret_cast<unsigned long long*>(&rs.e_arc); break;
      case 2: dst = reinterpret_cast<unsigned long long*>(&rs.e_alg); break;
      case 3: dst = reinterpret_cast<unsigned long long*>(&rs.gate_pass); break;
      default: dst = reinterpret_cast<unsigned long long*>(&rs.h_writes); break;
    }
    atomicAdd(dst, (unsigned long long)tot[k]);
  }
}

// ------------------------------------------------------------ launchers ---

void launch_co_init(const CohortView& v, hipStream_t s) {
  const size_t words = (size_t)kCoSegs * v.n_pad;
  const unsigned g = (unsigned)std::min<size_t>(8192, (words + kBlock - 1) / kBlock);
  k_co_init<<<g, kBlock, 0, s>>>(v);
}

void launch_co_admit(const CohortView& v, const CoSlot* slots, const int32_t* idx, int n,
                     hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 8) {
    AdmitArgs a = {};
    a.n = std::min(8, n - i0);
    for (int i = 0; i < a.n; ++i) {
      a.s[i] = slots[i0 + i];
      a.idx[i] = idx[i0 + i];
    }
    k_co_admit<<<1, kBlock, 0, s>>>(v, a);
  }
}

void launch_co_seed(const CohortView& v, int seg, int c0, const int32_t* kw_nodes,
                    const SeedList& seeds, hipStream_t s) {
  const uint32_t total = seeds.prefix[seeds.T];
  if (!total) return;
  const unsigned g = (unsigned)std::min<uint32_t>(4096, (total + kBlock - 1) / kBlock);
  k_co_seed<<<g, kBlock, 0, s>>>(v.H + (size_t)seg * v.n_pad * 16 + c0, kw_nodes, seeds);
}

void launch_co_scan(const CohortView& v, const DevGraphView& g, int level, hipStream_t s) {
  k_co_scan<<<v.nblocks, kBlock, 0, s>>>(v, g, level);
}

void launch_co_control(const CohortView& v, int level, uint64_t seq, hipStream_t s) {
  k_co_control<<<1 + kCoSlots, kCtlT, 0, s>>>(v, level, seq);
}

template <int TILE>
void co_expand_at(const CohortView& v, const DevGraphView& g, int level, int grid, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(k_co_expand<TILE>, dim3(grid), dim3(kBlock), 0, s, ev0, ev1, 0, v, g,
                          level);
  else
    k_co_expand<TILE><<<grid, kBlock, 0, s>>>(v, g, level);
}

void launch_co_expand(const CohortView& v, const DevGraphView& g, int level, int grid, int tile,
                      hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (tile == 512) co_expand_at<512>(v, g, level, grid, s, ev0, ev1);
  else if (tile == 2048) co_expand_at<2048>(v, g, level, grid, s, ev0, ev1);
  else co_expand_at<1024>(v, g, level, grid, s, ev0, ev1);
}

void launch_co_cand(const CoCandView& cv, const CohortView& v, hipStream_t s) {
  k_co_cand_count<<<v.nblocks, kBlock, 0, s>>>(cv, v.n, v.n_pad, v.cpw);
  k_co_cand_scan<<<1, kCtlT, 0, s>>>(cv, v.nblocks);
  k_co_cand_write<<<v.nblocks, kBlock, 0, s>>>(cv, v.n, v.cpw);
}

void launch_co_cg_done(const CohortView& v, int q, const Status* gst, uint64_t seq,
                       hipStream_t s) {
  k_co_cg_done<<<1, kBlock, 0, s>>>(v, q, gst, seq);
}

void launch_co_dmin(const CohortView& v, int q, int grid, hipStream_t s) {
  k_co_dmin<<<grid, kBlock, 0, s>>>(v, q);
}

void launch_co_rpg_final(const CohortView& v, int q, hipStream_t s) {
  k_co_rpg_final<<<1, kCtlT, 0, s>>>(v, q);
}

void launch_co_finish(const CoFinishView& fv, const DevGraphView& g, hipStream_t s) {
  k_co_post_init<<<1, 1, 0, s>>>(fv.slot, fv.gst);
  const unsigned grid = (unsigned)std::min<int64_t>(8192, ((int64_t)fv.n_pad + kBlock - 1) / kBlock);
  k_co_finish<<<std::max(1u, grid), kBlock, 0, s>>>(fv, g);
}

}  // namespace raks
