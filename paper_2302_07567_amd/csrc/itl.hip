// Interaction lists on the GPU: a breadth-first form of the list-filling
// dual tree traversal (Alg. dualtraversefillitl with Alg. diam, dist and
// admissible), followed by grouping of the pairs by target node (Sec. 10:
// sort by target plus a start-offset array, so that one workgroup owns one
// target and no atomics touch the fields).
//
// Each iteration takes the frontier of undecided (target, source) node pairs
// and classifies every pair exactly as the recursive traversal would: leaf-
// leaf pairs go to P2P, admissible pairs to M2L, and the rest are replaced by
// their two child pairs.  The set of emitted pairs is the recursive
// traversal's; only the order differs, and the final sort fixes that.
#include "internal.hpp"

namespace relfmm {

constexpr int kThreads = 256;
constexpr int kStepBlocks = 1024;

__global__ void k_itl_init(int *counters, int2 *front0) {
  int i = threadIdx.x;
  if (i < kCounters) counters[i] = 0;
  __syncthreads();
  if (i == 0) {
    front0[0] = make_int2(1, 1);
    counters[kCntFront + 0] = 1;
  }
}

// Alg. admissible in squared form: max(r_t^2, r_s^2) < eta^2 d^2, with d the
// stretched distance between box centres (Alg. dist).
__device__ inline bool admissible(const double *bmin, const double *bmax,
                                  const double *r2, int t, int s, double gb,
                                  double eta) {
  bool res;
  {
#pragma clang fp contract(off)
    const double sv[3] = {1.0, 1.0, gb};
    double d2 = 0.0;
    for (int g = 0; g < 3; ++g) {
      double ci = (bmin[3 * t + g] + bmax[3 * t + g]) * 0.5;
      double cj = (bmin[3 * s + g] + bmax[3 * s + g]) * 0.5;
      double d = sv[g] * (ci - cj);
      d2 = d2 + d * d;
    }
    double r = r2[t] > r2[s] ? r2[t] : r2[s];
    res = r < (eta * eta) * d2;
  }
  return res;
}

__global__ void __launch_bounds__(kThreads)
k_itl_step(int it, const int2 *front, int2 *next, int fcap, int *counters,
           uint64_t *p2p, int p2p_cap, uint64_t *m2l, int m2l_cap,
           const int32_t *kind, const double *bmin, const double *bmax,
           const double *r2, const double *gbar, double eta, int bits) {
  const int cnt = min(counters[kCntFront + it], fcap);
  const double gb = *gbar;
  const int lane = lane_id();
  const int wave_first = (blockIdx.x * kThreads + (int)threadIdx.x) - lane;
  const int stride = gridDim.x * kThreads;
  for (int base = wave_first; base < cnt; base += stride) {
    const int k = base + lane;
    const bool valid = k < cnt;
    int t = 1, s = 1, action = -1;  // 0 p2p, 1 m2l, 2 split t, 3 split s
    if (valid) {
      int2 pr = front[k];
      t = pr.x;
      s = pr.y;
      const bool lt = kind[t] == 1, ls = kind[s] == 1;
      if (lt && ls)
        action = 0;
      else if (admissible(bmin, bmax, r2, t, s, gb, eta))
        action = 1;
      else if (lt)
        action = 3;
      else if (ls)
        action = 2;
      else
        action = (r2[t] > r2[s]) ? 2 : 3;
    }
    const uint64_t key = ((uint64_t)t << bits) | (uint64_t)s;
    int slot = wave_alloc(action == 0, 1, &counters[kCntP2P]);
    if (action == 0) {
      if (slot < p2p_cap)
        p2p[slot] = key;
      else
        atomicOr(&counters[kCntOverflow], 1);
    }
    slot = wave_alloc(action == 1, 1, &counters[kCntM2L]);
    if (action == 1) {
      if (slot < m2l_cap)
        m2l[slot] = key;
      else
        atomicOr(&counters[kCntOverflow], 2);
    }
    slot = wave_alloc(action >= 2, 2, &counters[kCntFront + it + 1]);
    if (action >= 2) {
      if (slot + 1 < fcap) {
        if (action == 2) {
          next[slot] = make_int2(2 * t, s);
          next[slot + 1] = make_int2(2 * t + 1, s);
        } else {
          next[slot] = make_int2(t, 2 * s);
          next[slot + 1] = make_int2(t, 2 * s + 1);
        }
      } else {
        atomicOr(&counters[kCntOverflow], 4);
      }
    }
  }
}

// Start offsets of each target's group in a list sorted by key.
__global__ void k_rowptr(int ns, const uint64_t *keys, const int *cnt_ptr,
                         int cap, int bits, int32_t *row) {
  int v = blockIdx.x * kThreads + threadIdx.x;
  if (v > ns) return;
  const int cnt = min(*cnt_ptr, cap);
  const uint64_t want = (uint64_t)v << bits;
  int a = 0, b = cnt;
  while (a < b) {
    int mid = (a + b) >> 1;
    if (keys[mid] < want)
      a = mid + 1;
    else
      b = mid;
  }
  row[v] = a;
}

__global__ void k_count_inter(const uint64_t *keys, const int *cnt_ptr,
                              int cap, int bits, const int32_t *lo,
                              const int32_t *hi,
                              unsigned long long *inter) {
  const int cnt = min(*cnt_ptr, cap);
  const uint64_t mask = (1ull << bits) - 1ull;
  unsigned long long acc = 0;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < cnt;
       k += gridDim.x * kThreads) {
    int t = (int)(keys[k] >> bits), s = (int)(keys[k] & mask);
    acc += (unsigned long long)(hi[t] - lo[t]) * (unsigned long long)(hi[s] - lo[s]);
  }
  if (acc) atomicAdd(inter, acc);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0; }

// Swap (t, s) keys into (s, t) keys.
__global__ void k_swap_keys(const uint64_t *keys, const int *cnt_ptr, int cap,
                            int bits, uint64_t *out) {
  const int cnt = min(*cnt_ptr, cap);
  const uint64_t mask = (1ull << bits) - 1ull;
  for (int k = blockIdx.x * kThreads + threadIdx.x; k < cnt;
       k += gridDim.x * kThreads) {
    const uint64_t t = keys[k] >> bits, s = keys[k] & mask;
    out[k] = (s << bits) | t;
  }
}

static int nblocks(int n) { return (n + kThreads - 1) / kThreads; }

// Node slots ordered by decreasing length of their list row, so that the
// workgroups with the most work start first (list lengths vary by two orders
// of magnitude on a core + halo bunch).  The key is the row length clamped to
// 16 bits, complemented, above the node index; ties keep the node order.  Only
// the launch order of workgroups depends on it, never a result.
constexpr int kOrderThreads = 1024;
constexpr int kOrderSmall = 16384;  // node slots sorted in one workgroup's LDS

__device__ inline uint32_t cost_bits(const int32_t *row, int v) {
  const int32_t len = row[v + 1] - row[v];
  return 0xFFFFu - (uint32_t)min(max(len, 0), 0xFFFF);
}

struct OrderJob {
  const int32_t *row[2];
  int32_t *order[2];
};

// Bitonic sort of up to kOrderSmall 32-bit keys (cost << 16 | node) in LDS;
// workgroup b orders job b.
__global__ void __launch_bounds__(kOrderThreads)
k_order_small(int ns, OrderJob job) {
  __shared__ uint32_t key[kOrderSmall];
  const int tid = threadIdx.x;
  const int32_t *row = job.row[blockIdx.x];
  int P = 1;
  while (P < ns) P <<= 1;
  for (int v = tid; v < P; v += kOrderThreads)
    key[v] = v < ns ? (cost_bits(row, v) << 16) | (uint32_t)v : 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += kOrderThreads) {
        const int l = i ^ j;
        if (l > i) {
          const uint32_t a = key[i], b = key[l];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[l] = a;
          }
        }
      }
      __syncthreads();
    }
  int32_t *order = job.order[blockIdx.x];
  for (int v = tid; v < ns; v += kOrderThreads) order[v] = (int32_t)(key[v] & 0xFFFFu);
}

__global__ void k_cost_keys(int ns, const int32_t *row, int bits,
                            uint64_t *keys) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns) return;
  keys[v] = ((uint64_t)cost_bits(row, v) << bits) | (uint64_t)v;
}

__global__ void k_extract_order(int ns, const uint64_t *keys, int bits,
                                int32_t *order) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns) return;
  order[v] = (int32_t)(keys[v] & ((1ull << bits) - 1ull));
}

static void order_by_cost(const Dev &d, const int32_t *row0, int32_t *order0,
                          const int32_t *row1, int32_t *order1, int ns,
                          int bits, hipStream_t st) {
  if (ns <= kOrderSmall) {
    OrderJob job{{row0, row1}, {order0, order1}};
    hipLaunchKernelGGL(k_order_small, dim3(2), dim3(kOrderThreads), 0, st, ns,
                       job);
    return;
  }
  const int32_t *rows[2] = {row0, row1};
  int32_t *orders[2] = {order0, order1};
  for (int b = 0; b < 2; ++b) {
    hipLaunchKernelGGL(k_cost_keys, dim3(nblocks(ns)), dim3(kThreads), 0, st,
                       ns, rows[b], bits, d.okey);
    radix_sort(d.okey, nullptr, d.okey_tmp, nullptr, ns, 0, 16 + bits, d.hist,
               d.partial, st);
    hipLaunchKernelGGL(k_extract_order, dim3(nblocks(ns)), dim3(kThreads), 0,
                       st, ns, d.okey, bits, orders[b]);
  }
}

void build_transposed_lists_dev(const Dev &d, const ListArgs &a,
                                hipStream_t st) {
  const int key_bits = 2 * a.bits;
  hipLaunchKernelGGL(k_swap_keys, dim3(kStepBlocks), dim3(kThreads), 0, st,
                     d.p2p, d.counters + kCntP2P, a.p2p_cap, a.bits, d.p2p_T);
  hipLaunchKernelGGL(k_swap_keys, dim3(kStepBlocks), dim3(kThreads), 0, st,
                     d.m2l, d.counters + kCntM2L, a.m2l_cap, a.bits, d.m2l_T);
  // only the live prefix of each list (device-side count) is sorted
  radix_sort(d.p2p_T, nullptr, d.p2p_tmp, nullptr, a.p2p_cap, 0, key_bits,
             d.hist, d.partial, st, 1, d.counters + kCntP2P);
  radix_sort(d.m2l_T, nullptr, d.m2l_tmp, nullptr, a.m2l_cap, 0, key_bits,
             d.hist, d.partial, st, 1, d.counters + kCntM2L);
  hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0, st,
                     a.ns, d.p2p_T, d.counters + kCntP2P, a.p2p_cap, a.bits,
                     d.p2p_row_T);
  hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0, st,
                     a.ns, d.m2l_T, d.counters + kCntM2L, a.m2l_cap, a.bits,
                     d.m2l_row_T);
  order_by_cost(d, d.p2p_row_T, d.order_p2p_T, d.m2l_row_T, d.order_m2l_T,
                a.ns, a.bits, st);
}

void build_lists_dev(const Dev &d, const ListArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_itl_init, dim3(1), dim3(128), 0, st, d.counters,
                     d.front[0]);
  const int iters = 2 * a.depth + 1;
  for (int it = 0; it < iters; ++it) {
    const int2 *cur = d.front[it & 1];
    int2 *nxt = d.front[(it + 1) & 1];
    hipLaunchKernelGGL(k_itl_step, dim3(kStepBlocks), dim3(kThreads), 0, st,
                       it, cur, nxt, a.fcap, d.counters, d.p2p, a.p2p_cap,
                       d.m2l, a.m2l_cap, d.kind, d.bmin, d.bmax, d.r2, d.gbar,
                       a.eta, a.bits);
  }
  const int key_bits = 2 * a.bits;
  // only the live prefix of each list (device-side count) is sorted
  radix_sort(d.p2p, nullptr, d.p2p_tmp, nullptr, a.p2p_cap, 0, key_bits,
             d.hist, d.partial, st, 1, d.counters + kCntP2P);
  radix_sort(d.m2l, nullptr, d.m2l_tmp, nullptr, a.m2l_cap, 0, key_bits,
             d.hist, d.partial, st, 1, d.counters + kCntM2L);
  hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0, st,
                     a.ns, d.p2p, d.counters + kCntP2P, a.p2p_cap, a.bits,
                     d.p2p_row);
  hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0, st,
                     a.ns, d.m2l, d.counters + kCntM2L, a.m2l_cap, a.bits,
                     d.m2l_row);
  order_by_cost(d, d.p2p_row, d.order_p2p, d.m2l_row, d.order_m2l, a.ns,
                a.bits, st);

}

// Sum over P2P pairs of |t||s| for the statistics (run on request, not on
// every evaluation).
void count_interactions_dev(const Dev &d, const ListArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, d.inter);
  hipLaunchKernelGGL(k_count_inter, dim3(256), dim3(kThreads), 0, st, d.p2p,
                     d.counters + kCntP2P, a.p2p_cap, a.bits, d.lo, d.hi,
                     d.inter);
}

}  // namespace relfmm
