// common.h -- internal declarations of the RAKS gfx950 library: device
// utilities (wave/block scans, workgroup radix sort), run status layout and
// kernel argument blocks shared by the kernel files and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace raks {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup for most kernels
constexpr int kScanPer = 4;        // nodes per frontier-scan thread
constexpr int kScanNodes = 1024;   // nodes per frontier-scan chunk (kBlock * kScanPer)
constexpr int kScanGroups = 2048;  // at most this many frontier-scan workgroups
constexpr int kSuper = 64;         // scan workgroups per superblock of the enqueue prefix
constexpr int kSupers = kScanGroups / kSuper;
constexpr int kExpandTile = 1024;  // arcs per expansion tile
constexpr int kMaxKw = 16;         // keywords per run
constexpr int kMaxW = 256;         // beam width limit
constexpr uint8_t kInf = 0xFF;     // "not reached" in the node-keyword matrix
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int32_t kOvfBig0 = 8;    // a CG's lists exceed the sort path (Status::overflow)
constexpr int32_t kOvfBig1 = 16;   // an RPG's lists exceed the sort path

enum RunKind : int { RUN_CENTRAL = 0, RUN_MARGINAL = 1 };
enum EndReason : int { END_NONE = 0, END_EXHAUSTED = 1, END_STOP = 2, END_LEVEL_BOUND = 3,
                       END_EMPTY_KEYWORD = 4 };

// Device-resident state of one run (central or marginal), updated by the
// control step (workgroup 0 of the enqueue launch) at every level.
struct RunStatus {
  int32_t end_level;     // level at which the run ended; INT32_MAX while running
  int32_t end_reason;
  int32_t expand_on;     // 1 if the expansion of the current level runs
  int32_t levels;        // identification passes made
  uint32_t nfront;       // |frontier| of the current level
  uint32_t nactive;      // queue entries (frontiers with arcs to examine at this level)
  uint32_t W;            // arcs examined by the expansion of this level
  uint32_t ncand_level;  // central nodes identified at the current level
  uint32_t ncand_total;  // central nodes identified so far
  uint32_t nrpg;         // CGs with an RPG so far (marginal run)
  uint32_t cand_base[2]; // [l & 1]: central nodes identified before level l
  uint64_t frontier_sum, e_arc, e_alg, gate_pass, h_writes;
  uint64_t seq;          // host mirror only: number of the control launch that wrote it
};

struct Status {
  RunStatus run[2];
  int32_t nsel;          // selected CGs (<= w)
  int32_t nres;          // ranked results (<= k)
  int32_t overflow;      // 1/2: CG/RPG recovery capacity ran out, 4: output arena; 8/16: CG/RPG lists for the bitmap path
  int32_t err;           // graph contract violation bits (load)
  uint64_t cmin, cmax;   // label-count extremes (load)
  uint32_t out_nodes, out_arcs;  // output arena use
  uint32_t pad[2];
};

// Per-workgroup totals of the frontier scan.
struct ScanTot {
  uint32_t nfront;       // flagged nodes
  uint32_t nq;           // queue entries (nodes with arcs to examine at this level)
  uint32_t ncand;        // central nodes identified
  uint32_t work;         // arcs the GPU examines (sum of queue entry ranges)
  uint32_t hw;           // hitting levels written by the previous expansion
  uint32_t pad;
  uint64_t deg;          // sum of degrees of expanding frontiers (Algorithm 1 scans)
  uint64_t degk;         // sum of degree * expanding keywords
  uint64_t gate;         // arcs with level <= l of expanding frontiers
};


// Output header of one result.
struct ResultHdr {
  int32_t central, score_c, score_m, cg_rank;
  int64_t key;
  uint32_t node_off, n_nodes, arc_off, n_arcs;
  int64_t wsum;          // sum of the activation levels of the result's arcs
};

// ------------------------------------------------------------------------
// wave / block primitives (wave64; blocks of kBlock threads = 4 waves)

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ inline int wave_id() { return threadIdx.x / kWave; }

template <typename T>
__device__ inline T wave_inclusive_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Exclusive scan over a block of NT threads (NT multiple of 64, <= 1024);
// `scratch` holds NT/64 + 1 elements of T in LDS.  Returns the exclusive
// prefix; *total receives the block total.  Contains __syncthreads.
template <typename T, int NT>
__device__ inline T block_exclusive_scan(T v, T* scratch, T* total) {
  constexpr int NW = NT / kWave;
  T inc = wave_inclusive_scan(v);
  if (lane_id() == kWave - 1) scratch[wave_id()] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < NW; ++w) { T t = scratch[w]; scratch[w] = acc; acc += t; }
    scratch[NW] = acc;
  }
  __syncthreads();
  T res = scratch[wave_id()] + inc - v;
  *total = scratch[NW];
  __syncthreads();
  return res;
}

template <typename T, int NT>
__device__ inline T block_sum(T v, T* scratch) {
  T tot;
  (void)block_exclusive_scan<T, NT>(v, scratch, &tot);
  return tot;
}

// Exclusive scans of N values at once over a block of NT threads: one LDS
// exchange (two barriers) for all of them.  `scratch` holds (NT/64 + 1) * N
// 64-bit words.  v[] is replaced by the exclusive prefixes, tot[] gets the
// block totals.
template <int N, int NT, typename T = uint64_t>
__device__ inline void block_exclusive_scan_multi(T (&v)[N], T (&tot)[N], T* scratch) {
  constexpr int NW = NT / kWave;
  T inc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) inc[k] = wave_inclusive_scan(v[k]);
  if (lane_id() == kWave - 1)
#pragma unroll
    for (int k = 0; k < N; ++k) scratch[wave_id() * N + k] = inc[k];
  __syncthreads();
  if (threadIdx.x < N) {
    const int k = threadIdx.x;
    T acc = 0;
    for (int w = 0; w < NW; ++w) { const T t = scratch[w * N + k]; scratch[w * N + k] = acc; acc += t; }
    scratch[NW * N + k] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const T x = v[k];
    v[k] = scratch[wave_id() * N + k] + inc[k] - x;
    tot[k] = scratch[NW * N + k];
  }
  __syncthreads();
}

// Exclusive max-scan over a block of kBlock threads of non-negative values;
// `scratch` holds kBlock/64 + 1 words of LDS.  Contains __syncthreads.
__device__ inline uint32_t block_exclusive_max(uint32_t v, uint32_t* scratch) {
  const int lane = lane_id();
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, kWave);
    if (lane >= d) inc = inc > o ? inc : o;
  }
  if (lane == kWave - 1) scratch[wave_id()] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < kBlock / kWave; ++w) { const uint32_t t = scratch[w]; scratch[w] = acc; acc = acc > t ? acc : t; }
  }
  __syncthreads();
  uint32_t ex = __shfl_up(inc, 1, kWave);
  if (lane == 0) ex = 0;
  const uint32_t w = scratch[wave_id()];
  __syncthreads();
  return ex > w ? ex : w;
}

// Last index j in [0, n) with a[j] <= x (a non-decreasing, a[0] <= x), found
// by one wavefront: each round the 64 lanes probe 64 evenly spaced entries,
// so the search takes ceil(log64 n) dependent memory round trips.
__device__ inline int wave_search(const uint32_t* a, int n, uint32_t x) {
  int lo = 0, hi = n;
  const int lane = lane_id();
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int idx = lo + lane * step;
    const bool ok = idx < hi && a[idx] <= x;
    const uint64_t b = __ballot(ok);
    const int L = 63 - __clzll((long long)b);
    lo += L * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// Last index j in [lo, hi) with a[j] <= x, given a[lo] <= x (a non-decreasing).
template <typename T>
__device__ inline int upper_index(const T* a, int lo, int hi, T x) {
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------------
// Workgroup stable LSD radix sort of n 32-bit keys (kBlock threads), keys in
// `a`, `b` same-size scratch; the sorted keys end in the returned pointer
// (a or b).  Digits are 8 bits; a pass whose digit is constant is skipped.
struct RadixLds {
  uint32_t hist[256];
  uint32_t base[256];
  uint32_t cnt[kBlock / kWave][256];
  uint32_t scan[kBlock / kWave + 1];
  int32_t skip;
};

__device__ inline uint32_t* wg_radix_sort_u32(uint32_t* a, uint32_t* b, uint32_t n, RadixLds& s) {
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  for (int shift = 0; shift < 32; shift += 8) {
    s.hist[tid] = 0;
    if (tid == 0) s.skip = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kBlock) atomicAdd(&s.hist[(a[i] >> shift) & 0xFF], 1u);
    __syncthreads();
    uint32_t h = s.hist[tid];
    if (h == n) s.skip = 1;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(h, s.scan, &tot);
    s.base[tid] = ex;
    __syncthreads();
    if (s.skip) { __syncthreads(); continue; }
    for (uint32_t t0 = 0; t0 < n; t0 += kBlock) {
      for (int w = 0; w < kBlock / kWave; ++w) s.cnt[w][tid] = 0;
      __syncthreads();
      const uint32_t i = t0 + tid;
      const bool valid = i < n;
      const uint32_t key = valid ? a[i] : 0u;
      const uint32_t d = (key >> shift) & 0xFF;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        uint64_t bb = __ballot(valid && ((d >> bit) & 1));
        peers &= ((d >> bit) & 1) ? bb : ~bb;
      }
      const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
      const uint32_t rank = __popcll(peers & lt);
      if (valid && rank == 0) s.cnt[wv][d] = __popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t off = s.base[d] + rank;
        for (int w = 0; w < wv; ++w) off += s.cnt[w][d];
        b[off] = key;
      }
      __syncthreads();
      uint32_t add = 0;
      for (int w = 0; w < kBlock / kWave; ++w) add += s.cnt[w][tid];
      s.base[tid] += add;
      __syncthreads();
    }
    uint32_t* t = a; a = b; b = t;
  }
  return a;
}

// Writes the distinct keys of the sorted array `in` (length n) to `out` in
// order; returns their number.  Uses `scan` LDS of kBlock/64+1 words.
__device__ inline uint32_t wg_unique_u32(const uint32_t* in, uint32_t n, uint32_t* out,
                                        uint32_t* scan) {
  uint32_t written = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += kBlock) {
    const uint32_t i = t0 + threadIdx.x;
    uint32_t keep = (i < n && (i == 0 || in[i] != in[i - 1])) ? 1u : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<uint32_t, kBlock>(keep, scan, &tot);
    if (keep) out[written + ex] = in[i];
    written += tot;
  }
  return written;
}

}  // namespace raks
