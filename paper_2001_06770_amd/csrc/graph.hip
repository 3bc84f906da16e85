// graph.hip -- graph upload checks and activation levels (Section 3.1).
//
// EDGE mode: for arc e = (i -> j, l) the fine weight is the log of
//   c_e = |arcs of i with label l| + |arcs into j with label l|
// (on the bi-directed graph the arcs into j with label l are the reverses of
// j's arcs with label l), min-max rescaled to x in [0,1], then coarsened by the
// reward/penalty rule (Eqs. 1-3) around a_bar and rounded half up.
// NODE mode: the node weights are min-max rescaled and coarsened the same way;
// an arc u -> v gets the level of v.
// Rows are sorted by (label, destination), so a label's arcs in a row are one
// run found by binary search.  Built with -ffp-contract=off: the fp64
// expressions are evaluated exactly as written.
#include "common.h"
#include "kernels.h"

namespace raks {

// number of arcs in row x with label lab
__device__ inline uint32_t label_run(const uint32_t* row_ptr, const uint16_t* label, uint32_t x,
                                     uint16_t lab) {
  uint32_t lo = row_ptr[x], hi = row_ptr[x + 1];
  uint32_t a = lo, b = hi;
  while (a < b) { uint32_t m = (a + b) >> 1; if (label[m] < lab) a = m + 1; else b = m; }
  const uint32_t first = a;
  b = hi;
  while (a < b) { uint32_t m = (a + b) >> 1; if (label[m] <= lab) a = m + 1; else b = m; }
  return a - first;
}

// Checks every arc against the input contract and computes its label count c.
__global__ __launch_bounds__(kBlock) void k_check_and_count(const uint32_t* row_ptr,
                                                            const int32_t* col,
                                                            const uint16_t* label, int32_t n,
                                                            uint32_t A, uint32_t* c_out,
                                                            int32_t* arc_src, uint32_t* rev,
                                                            Status* st) {
  uint32_t err = 0;
  uint64_t cmin = ~0ull, cmax = 0;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < A; e += gridDim.x * kBlock) {
    const uint32_t i = row_of(row_ptr, n, e);
    arc_src[e] = (int32_t)i;
    const int32_t j = col[e];
    const uint16_t lab = label[e];
    if (j < 0 || j >= n) { err |= 1; c_out[e] = 0; rev[e] = kEmpty; continue; }
    if ((uint32_t)j == i) err |= 2;
    if (e > row_ptr[i]) {
      const uint16_t pl = label[e - 1];
      const int32_t pc = col[e - 1];
      if (pl > lab || (pl == lab && pc >= j)) err |= 4;
    }
    const uint32_t r = find_arc_dev(row_ptr, col, label, j, lab, (int32_t)i);
    rev[e] = r;
    if (r == kEmpty) err |= 8;
    const uint64_t c = (uint64_t)label_run(row_ptr, label, i, lab) + label_run(row_ptr, label, j, lab);
    c_out[e] = (uint32_t)c;
    cmin = c < cmin ? c : cmin;
    cmax = c > cmax ? c : cmax;
  }
  // wave reductions, then one atomic per wave
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    uint64_t a = __shfl_xor(cmin, d, kWave), b = __shfl_xor(cmax, d, kWave);
    cmin = a < cmin ? a : cmin;
    cmax = b > cmax ? b : cmax;
    err |= __shfl_xor(err, d, kWave);
  }
  if (lane_id() == 0) {
    if (err) atomicOr(&st->err, (int32_t)err);
    atomicMin((unsigned long long*)&st->cmin, (unsigned long long)cmin);
    atomicMax((unsigned long long*)&st->cmax, (unsigned long long)cmax);
  }
}

// Activation level of every arc: a lookup of its label count c in the table
// of levels the host built for c in [cmin, cmax] (Eqs. 1-3 evaluated once per
// count, on the host).
__global__ __launch_bounds__(kBlock) void k_act_edge(const uint32_t* c, uint32_t A,
                                                     const uint8_t* lut, uint64_t cmin,
                                                     uint8_t* act) {
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < A; e += gridDim.x * kBlock)
    act[e] = lut[c[e] - cmin];
}

__global__ __launch_bounds__(kBlock) void k_node_weight_range(const uint8_t* nw, int32_t n,
                                                              Status* st) {
  uint32_t mn = 255, mx = 0;
  for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
    mn = min(mn, (uint32_t)nw[v]);
    mx = max(mx, (uint32_t)nw[v]);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor(mn, d, kWave));
    mx = max(mx, (uint32_t)__shfl_xor(mx, d, kWave));
  }
  if (lane_id() == 0) {
    atomicMin((unsigned long long*)&st->cmin, (unsigned long long)mn);
    atomicMax((unsigned long long*)&st->cmax, (unsigned long long)mx);
  }
}

// NODE mode: the level of every node from the host's table over the node
// weights in [wmin, wmax].
__global__ __launch_bounds__(kBlock) void k_act_node(const uint8_t* nw, int32_t n,
                                                     const uint8_t* lut, uint32_t wmin,
                                                     uint8_t* act_node) {
  for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock)
    act_node[v] = lut[nw[v] - wmin];
}

__global__ __launch_bounds__(kBlock) void k_act_gather(const uint8_t* act_node,
                                                       const int32_t* col, uint32_t A,
                                                       uint8_t* act) {
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < A; e += gridDim.x * kBlock)
    act[e] = act_node[col[e]];
}

// Traversal copy of the graph: each row's arcs re-ordered by activation level
// (counting sort per row, one wavefront per row), plus the row's largest
// level and its entries of the level-major level table.  At level l a
// frontier's arcs with level <= l form a row prefix.
__global__ __launch_bounds__(kBlock) void k_sort_rows(const uint32_t* row_ptr_o,
                                                      const uint32_t* row_ptr,
                                                      const int32_t* orig_id, const int32_t* int_id,
                                                      const int32_t* col, const uint8_t* act,
                                                      int32_t n, int32_t* col_s, uint8_t* act_s,
                                                      uint32_t* eid_s, uint8_t* row_amax,
                                                      uint32_t* bnd, int32_t nbnd) {
  __shared__ uint32_t s_hist[kBlock / kWave][256];
  uint32_t* hist = s_hist[wave_id()];
  const int lane = lane_id();
  const int waves = gridDim.x * (kBlock / kWave);
  for (int32_t u = blockIdx.x * (kBlock / kWave) + wave_id(); u < n; u += waves) {
    // internal row u holds original row v's arcs
    const int32_t v = orig_id[u];
    const uint32_t rs_o = row_ptr_o[v], re_o = row_ptr_o[v + 1];
    const uint32_t rs = row_ptr[u];
    for (int b = lane; b < 256; b += kWave) hist[b] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t amax = 0;
    for (uint32_t e = rs_o + lane; e < re_o; e += kWave) {
      const uint32_t a = act[e];
      atomicAdd(&hist[a], 1u);
      amax = a > amax ? a : amax;
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
      const uint32_t o = __shfl_xor(amax, d, kWave);
      amax = o > amax ? o : amax;
    }
    __builtin_amdgcn_wave_barrier();
    // exclusive prefix over the 256 bins: lane owns bins 4*lane .. 4*lane+3
    uint32_t c0 = hist[4 * lane], c1 = hist[4 * lane + 1], c2 = hist[4 * lane + 2], c3 = hist[4 * lane + 3];
    const uint32_t tot = c0 + c1 + c2 + c3;
    const uint32_t ex = wave_inclusive_scan(tot) - tot;
    hist[4 * lane] = ex;
    hist[4 * lane + 1] = ex + c0;
    hist[4 * lane + 2] = ex + c0 + c1;
    hist[4 * lane + 3] = ex + c0 + c1 + c2;
    __builtin_amdgcn_wave_barrier();
    // arcs with level <= l = start of level l + 1
    if (lane < nbnd) bnd[(size_t)lane * n + u] = hist[lane + 1];
    __builtin_amdgcn_wave_barrier();
    for (uint32_t e = rs_o + lane; e < re_o; e += kWave) {
      const uint32_t a = act[e];
      const uint32_t pos = rs + atomicAdd(&hist[a], 1u);
      col_s[pos] = int_id[col[e]];
      act_s[pos] = (uint8_t)a;
      eid_s[pos] = e;
    }
    if (lane == 0) row_amax[u] = (uint8_t)amax;
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(kBlock) void k_to_internal_u8(const int32_t* orig_id, int32_t n,
                                                           const uint8_t* in, uint8_t* out) {
  for (int32_t u = blockIdx.x * kBlock + threadIdx.x; u < n; u += gridDim.x * kBlock)
    out[u] = in[orig_id[u]];
}

__global__ __launch_bounds__(kBlock) void k_map_ids(const int32_t* int_id, int32_t* ids,
                                                    uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * kBlock)
    ids[i] = int_id[ids[i]];
}

void launch_sort_rows(const DevGraphView& g, int32_t* col_s, uint8_t* act_s, uint32_t* eid_s,
                      uint8_t* row_amax, uint32_t* bnd, int32_t nbnd, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>(16384, ((int64_t)g.n + 3) / 4);
  k_sort_rows<<<grid, kBlock, 0, s>>>(g.row_ptr_o, g.row_ptr, g.orig_id, g.int_id, g.col, g.act,
                                      g.n, col_s, act_s, eid_s, row_amax, bnd, nbnd);
}

__global__ void k_status_reset_minmax(Status* st) {
  st->cmin = ~0ull;
  st->cmax = 0;
  st->err = 0;
}

// ------------------------------------------------------------ launchers ---

static unsigned grid_for(uint64_t items, unsigned cap = 8192) {
  uint64_t g = (items + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

void launch_check_and_count(const DevGraphView& g, uint32_t* c_tmp, int32_t* arc_src, uint32_t* rev,
                            Status* st, hipStream_t s) {
  k_status_reset_minmax<<<1, 1, 0, s>>>(st);
  if (g.A > 0)
    k_check_and_count<<<grid_for(g.A), kBlock, 0, s>>>(g.row_ptr_o, g.col, g.label, g.n, g.A, c_tmp,
                                                        arc_src, rev, st);
}

void launch_act_edge(const DevGraphView& g, const uint32_t* c_tmp, const uint8_t* lut,
                     uint64_t cmin, uint8_t* act, hipStream_t s) {
  if (g.A > 0) k_act_edge<<<grid_for(g.A), kBlock, 0, s>>>(c_tmp, g.A, lut, cmin, act);
}

void launch_node_weight_range(const DevGraphView& g, const uint8_t* nw, Status* st,
                              hipStream_t s) {
  k_status_reset_minmax<<<1, 1, 0, s>>>(st);
  k_node_weight_range<<<grid_for(g.n), kBlock, 0, s>>>(nw, g.n, st);
}

void launch_to_internal_u8(const DevGraphView& g, const uint8_t* in, uint8_t* out, hipStream_t s) {
  k_to_internal_u8<<<grid_for(g.n), kBlock, 0, s>>>(g.orig_id, g.n, in, out);
}

void launch_map_ids(const int32_t* int_id, int32_t* ids, uint64_t count, hipStream_t s) {
  if (count) k_map_ids<<<grid_for(count), kBlock, 0, s>>>(int_id, ids, count);
}

void launch_act_node(const DevGraphView& g, const uint8_t* nw, const uint8_t* lut, uint32_t wmin,
                     uint8_t* act_node, uint8_t* act, hipStream_t s) {
  k_act_node<<<grid_for(g.n), kBlock, 0, s>>>(nw, g.n, lut, wmin, act_node);
  if (g.A > 0) k_act_gather<<<grid_for(g.A), kBlock, 0, s>>>(act_node, g.col, g.A, act);
}

}  // namespace raks
