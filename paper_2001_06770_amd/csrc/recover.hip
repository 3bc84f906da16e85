// recover.hip -- recovering phase (Section 4.3, Algorithm 2, Lemma 1) on the
// GPU, and the per-result union / sort / unique of the recovered subgraphs.
//
// One workgroup recovers one (result, keyword) instance: a backward search
// from the start nodes over in-arcs n -> q (the reverses of q's arcs on the
// bi-directed graph), keeping (n, e_nq) when h_q = 1 + max(a_nq, h_n) and
// continuing from n unless h_n = 0.  Along a recovered arc h strictly drops,
// so the search runs layer by layer from the largest level down to 1; every
// node of a layer is discovered before its layer is processed.  A hash set in
// global memory (open addressing) keeps each node once per instance; a
// node's arcs are spread over the 256 lanes by a prefix sum over degrees.
// Capacities are fixed per launch; running out sets a flag and the host
// repeats the phase with larger buffers.
#include "common.h"
#include "kernels.h"

namespace raks {

__device__ inline bool ht_insert(uint32_t* ht, uint32_t hc, uint32_t key, int* full) {
  uint32_t h = (key * 2654435761u) & (hc - 1);
  for (uint32_t probe = 0; probe < hc; ++probe) {
    const uint32_t old = atomicCAS(&ht[h], kEmpty, key);
    if (old == kEmpty) return true;
    if (old == key) return false;
    h = (h + 1) & (hc - 1);
  }
  *full = 1;
  return false;
}

template <int TP>
__global__ __launch_bounds__(kBlock) void k_recover(RecoverView v) {
  const int inst = blockIdx.x;
  const int res = inst / v.T, col = inst % v.T;
  uint32_t* ht = v.ht + (size_t)inst * v.hc;
  int32_t* nl = v.nl + (size_t)inst * v.nc;
  uint32_t* al = v.al + (size_t)inst * v.ac;
  const uint8_t* H = v.H;
  const DevGraphView& g = v.g;
  __shared__ uint32_t s_nn, s_na;
  __shared__ int s_over, s_hmax;
  __shared__ int32_t s_q[kBlock];
  __shared__ uint32_t s_off[kBlock], s_rs[kBlock];
  __shared__ uint32_t s_scan[kBlock / kWave + 1];

  for (uint32_t i = threadIdx.x; i < v.hc; i += kBlock) ht[i] = kEmpty;
  if (threadIdx.x == 0) { s_nn = 0; s_na = 0; s_over = 0; s_hmax = 0; }
  __syncthreads();

  // start nodes
  if (!v.marginal) {
    if (threadIdx.x == 0) {
      const int32_t c = v.sel_node[res];
      int full = 0;
      ht_insert(ht, v.hc, (uint32_t)c, &full);
      nl[0] = c;
      s_nn = 1;
      s_hmax = H[(int64_t)c * TP + col];
    }
  } else {
    const int r = v.ranked[res];
    const uint8_t d = v.dmin[r * kMaxKw + col];
    for (uint32_t p = v.vc_off[r] + threadIdx.x; p < v.vc_off[r + 1]; p += kBlock) {
      const int32_t x = v.vc_nodes[p];
      if (H[(int64_t)x * TP + col] != d) continue;
      int full = 0;
      if (ht_insert(ht, v.hc, (uint32_t)x, &full)) {
        const uint32_t slot = atomicAdd(&s_nn, 1u);
        if (slot < v.nc) nl[slot] = x; else s_over = 1;
      }
      if (full) s_over = 1;
    }
    if (threadIdx.x == 0) s_hmax = d;
  }
  __syncthreads();

  for (int h = s_hmax; h >= 1 && !s_over; --h) {
    const uint32_t total = min(s_nn, v.nc);
    for (uint32_t c0 = 0; c0 < total; c0 += kBlock) {
      const uint32_t idx = c0 + threadIdx.x;
      int32_t q = -1;
      uint32_t deg = 0, rs = 0;
      if (idx < total) {
        q = nl[idx];
        if (H[(int64_t)q * TP + col] == h) {
          rs = g.row_ptr[q];
          deg = g.row_ptr[q + 1] - rs;
        }
      }
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(deg, s_scan, &tot);
      s_q[threadIdx.x] = q;
      s_off[threadIdx.x] = ex;
      s_rs[threadIdx.x] = rs;
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < tot; k += kBlock) {
        const int j = upper_index<uint32_t>(s_off, 0, kBlock, k);
        const int32_t qq = s_q[j];
        const uint32_t e = s_rs[j] + (k - s_off[j]);
        const int32_t n = g.col[e];
        const uint32_t a = g.mode ? g.act_node[qq] : g.act[e];   // level of the in-arc n -> qq
        const uint32_t hn = H[(int64_t)n * TP + col];
        if ((uint32_t)h == 1u + (a > hn ? a : hn)) {
          const uint32_t fwd = find_arc_dev(g.row_ptr, g.col, g.label, n, g.label[e], qq);
          const uint32_t sa = atomicAdd(&s_na, 1u);
          if (sa < v.ac) al[sa] = fwd; else s_over = 1;
          int full = 0;
          if (ht_insert(ht, v.hc, (uint32_t)n, &full)) {
            const uint32_t sn = atomicAdd(&s_nn, 1u);
            if (sn < v.nc) nl[sn] = n; else s_over = 1;
          }
          if (full) s_over = 1;
        }
      }
      __syncthreads();
      if (s_over) break;
    }
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    v.cnt[inst * 2] = min(s_nn, v.nc);
    v.cnt[inst * 2 + 1] = min(s_na, v.ac);
    if (s_over) atomicOr(&v.gst->overflow, 1);
  }
}

// Per result: gather the node lists (and arc lists) of its instances (and,
// for an RPG, of its CG), radix sort, keep distinct keys.  For CGs also the
// central-keyword nodes V_C (some central level 0).  Final results go to the
// output arena with their header; arcs are written as (src, dst, label).
__global__ __launch_bounds__(kBlock) void k_finalize(FinalizeView v) {
  const int t = blockIdx.x;
  __shared__ RadixLds lds;
  __shared__ uint32_t s_n, s_off;
  uint32_t* A = v.sort_a + (size_t)t * v.scap;
  uint32_t* B = v.sort_b + (size_t)t * v.scap;
  const int r = v.marginal ? v.ranked[t] : t;
  const DevGraphView& g = v.g;

  for (int pass = 0; pass < 2; ++pass) {   // 0: nodes, 1: arcs
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint32_t n = 0;
    if (v.marginal) {
      const uint32_t cnt = v.cg_cnt[r * 2 + pass];
      const uint32_t* src = pass == 0 ? v.cg_nodes + (size_t)r * v.cg_ncap
                                      : v.cg_arcs + (size_t)r * v.cg_acap;
      for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) A[i] = src[i];
      n = cnt;
    }
    for (int j = 0; j < v.T; ++j) {
      const int inst = t * v.T + j;
      const uint32_t cnt = v.cnt[inst * 2 + pass];
      if (pass == 0) {
        const int32_t* src = v.nl + (size_t)inst * v.nc;
        for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) A[n + i] = (uint32_t)src[i];
      } else {
        const uint32_t* src = v.al + (size_t)inst * v.ac;
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
      uint32_t* dst = pass == 0 ? v.cg_nodes + (size_t)r * v.cg_ncap : v.cg_arcs + (size_t)r * v.cg_acap;
      for (uint32_t i = threadIdx.x; i < m; i += kBlock) dst[i] = uniq[i];
      if (threadIdx.x == 0) v.cg_cnt[r * 2 + pass] = m;
      if (pass == 0) {
        // V_C in node order
        int32_t* vc = v.vc_tmp + (size_t)r * v.cg_ncap;
        uint32_t written = 0;
        for (uint32_t t0 = 0; t0 < m; t0 += kBlock) {
          const uint32_t i = t0 + threadIdx.x;
          uint32_t keep = 0;
          if (i < m) {
            const int64_t x = uniq[i];
            for (int c = 0; c < v.Tc; ++c) keep |= v.Hc[x * v.TPc + c] == 0;
          }
          uint32_t tot;
          const uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(keep, lds.scan, &tot);
          if (keep) vc[written + ex] = (int32_t)uniq[i];
          written += tot;
        }
        if (threadIdx.x == 0) v.vc_cnt[r] = written;
      }
    }
    if (v.write_output) {
      if (threadIdx.x == 0) {
        const uint32_t off = atomicAdd(pass == 0 ? &v.gst->out_nodes : &v.gst->out_arcs, m);
        const uint32_t cap = pass == 0 ? v.out_ncap : v.out_acap;
        if (off + m > cap) atomicOr(&v.gst->overflow, 2);
        s_off = off;
        ResultHdr& hd = v.hdr[t];
        if (pass == 0) {
          hd.central = v.sel_node[r];
          hd.score_c = v.sel_sc[r];
          hd.score_m = v.sm[r];
          hd.cg_rank = r;
          hd.key = v.key[r];
          hd.node_off = off;
          hd.n_nodes = m;
        } else {
          hd.arc_off = off;
          hd.n_arcs = m;
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
            o[0] = (int32_t)row_of(g.row_ptr, g.n, e);
            o[1] = g.col[e];
            o[2] = g.label[e];
          }
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp,
                                                    uint32_t cg_ncap, int32_t nsel,
                                                    uint32_t* vc_off, int32_t* vc_nodes) {
  __shared__ uint32_t s_off[kMaxW + 1];
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int r = 0; r < nsel; ++r) { s_off[r] = acc; acc += vc_cnt[r]; }
    s_off[nsel] = acc;
  }
  __syncthreads();
  for (int r = threadIdx.x; r <= nsel; r += kBlock) vc_off[r] = s_off[r];
  for (int r = 0; r < nsel; ++r) {
    const int32_t* src = vc_tmp + (size_t)r * cg_ncap;
    for (uint32_t i = threadIdx.x; i < vc_cnt[r]; i += kBlock) vc_nodes[s_off[r] + i] = src[i];
  }
}

void launch_recover(const RecoverView& v, hipStream_t s) {
  if (v.n_inst <= 0) return;
  switch (v.TP) {
    case 4: k_recover<4><<<v.n_inst, kBlock, 0, s>>>(v); break;
    case 8: k_recover<8><<<v.n_inst, kBlock, 0, s>>>(v); break;
    default: k_recover<16><<<v.n_inst, kBlock, 0, s>>>(v); break;
  }
}

void launch_finalize(const FinalizeView& v, hipStream_t s) {
  if (v.n_res > 0) k_finalize<<<v.n_res, kBlock, 0, s>>>(v);
}

void launch_pack_vc(const uint32_t* vc_cnt, const int32_t* vc_tmp, uint32_t cg_ncap, int32_t nsel,
                    uint32_t* vc_off, int32_t* vc_nodes, hipStream_t s) {
  k_pack_vc<<<1, kBlock, 0, s>>>(vc_cnt, vc_tmp, cg_ncap, nsel, vc_off, vc_nodes);
}

}  // namespace raks
