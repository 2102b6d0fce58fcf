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
// traversal's; only the order differs, and the grouping by row (which sorts
// every row) fixes that.
#include <algorithm>

#include "internal.hpp"

namespace relfmm {

constexpr int kThreads = 256;
constexpr int kStepBlocks = 1024;

// Alg. admissible in squared form: max(r_t^2, r_s^2) < eta^2 d^2, with d the
// stretched distance between the centres of the nodes' boxes (Alg. dist) and
// r the stretched half-diagonals of those boxes (Alg. diam).
__device__ inline bool admissible(const double *cen, const double *r2, int t,
                                  int s, double gb, double eta) {
  bool res;
  {
#pragma clang fp contract(off)
    const double sv[3] = {1.0, 1.0, gb};
    double d2 = 0.0;
    for (int g = 0; g < 3; ++g) {
      double d = sv[g] * (cen[3 * t + g] - cen[3 * s + g]);
      d2 = d2 + d * d;
    }
    double r = r2[t] > r2[s] ? r2[t] : r2[s];
    res = r < (eta * eta) * d2;
  }
  return res;
}

// One traversal iteration over the cnt frontier pairs, in waves whose lane 0
// starts at pair wave_first and steps by stride.
__device__ inline void itl_classify(int it, int cnt, const int2 *front,
                                    int2 *next, int fcap, int *counters,
                                    uint64_t *p2p, int p2p_cap, uint64_t *m2l,
                                    int m2l_cap, const int32_t *kind,
                                    const double *cen,
                                    const double *r2, double gb, double eta,
                                    int bits, int wave_first, int stride) {
  const int lane = lane_id();
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
      else if (admissible(cen, r2, t, s, gb, eta))
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

__global__ void __launch_bounds__(kThreads)
k_itl_step(int it, const int2 *front, int2 *next, int fcap, int *counters,
           uint64_t *p2p, int p2p_cap, uint64_t *m2l, int m2l_cap,
           const int32_t *kind, const double *cen,
           const double *r2, const double *gbar, double eta, int bits) {
  const int cnt = min(counters[kCntFront + it], fcap);
  const int wave_first =
      (blockIdx.x * kThreads + (int)threadIdx.x) - lane_id();
  itl_classify(it, cnt, front, next, fcap, counters, p2p, p2p_cap, m2l,
               m2l_cap, kind, cen, r2, *gbar, eta, bits, wave_first,
               gridDim.x * kThreads);
}

// The first iterations in one workgroup, with the counters' reset: the
// frontier of iteration it holds at most 2^it pairs (every pair is replaced
// by at most two), so up to kHeadIters iterations it stays within one pair
// per thread and a launch per iteration would cost more than the work.
constexpr int kHeadThreads = 1024;
constexpr int kHeadIters = 11;

__global__ void __launch_bounds__(kHeadThreads)
k_itl_head(int iters, int2 *f0, int2 *f1, int fcap, int *counters,
           uint64_t *p2p, int p2p_cap, uint64_t *m2l, int m2l_cap,
           const int32_t *kind, const double *cen,
           const double *r2, const double *gbar, double eta, int bits) {
  const int tid = threadIdx.x;
  if (tid < kCounters) counters[tid] = 0;
  __syncthreads();
  if (tid == 0) {
    f0[0] = make_int2(1, 1);
    counters[kCntFront + 0] = 1;
  }
  __syncthreads();
  const double gb = *gbar;
  for (int it = 0; it < iters; ++it) {
    const int cnt = min(__hip_atomic_load(&counters[kCntFront + it],
                                          __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT),
                        fcap);
    itl_classify(it, cnt, (it & 1) ? f1 : f0, (it & 1) ? f0 : f1, fcap,
                 counters, p2p, p2p_cap, m2l, m2l_cap, kind, cen, r2,
                 gb, eta, bits, tid - lane_id(), kHeadThreads);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Grouping by row: each list's live prefix (keys (r << bits) | c, r the node
// the row belongs to) is counted per row, the counts are scanned into the row
// start offsets, the keys are scattered into their rows (in arbitrary order
// inside a row), and every row is then sorted in LDS.  The list ends up in
// ascending key order, exactly as a sort of the whole list leaves it, and the
// start offsets come with it.
// ---------------------------------------------------------------------------
struct ListGroup {
  uint64_t *keys[2];       // in: live prefix; out: sorted
  uint64_t *tmp[2];        // scratch, cap entries
  const int *cnt_ptr[2];   // device-side entry counts
  int cap[2];
  int32_t *rows[2];        // [ns + 1] row start offsets (out)
  int32_t *fill[2];        // [ns + 1] per-row counters (scratch)
};

__global__ void k_group_zero(int ns, ListGroup g) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v > ns) return;
  g.fill[0][v] = 0;
  g.fill[1][v] = 0;
}

__global__ void k_group_count(int bits, ListGroup g) {
  for (int l = 0; l < 2; ++l) {
    const int cnt = min(*g.cnt_ptr[l], g.cap[l]);
    for (int k = blockIdx.x * kThreads + threadIdx.x; k < cnt;
         k += gridDim.x * kThreads)
      atomicAdd(&g.fill[l][(int)(g.keys[l][k] >> bits)], 1);
  }
}

// Each key takes one of its row's slots; the counters run back down to zero.
__global__ void k_group_scatter(int bits, ListGroup g) {
  for (int l = 0; l < 2; ++l) {
    const int cnt = min(*g.cnt_ptr[l], g.cap[l]);
    for (int k = blockIdx.x * kThreads + threadIdx.x; k < cnt;
         k += gridDim.x * kThreads) {
      const uint64_t key = g.keys[l][k];
      const int r = (int)(key >> bits);
      const int pos = g.rows[l][r] + atomicSub(&g.fill[l][r], 1) - 1;
      g.tmp[l][pos] = key;
    }
  }
}

constexpr int kRowThreads = 256;
constexpr int kRowChunk = 2048;  // keys sorted at once in LDS (16 KB)

// One workgroup per row (blockIdx.x) of list blockIdx.y: the row is sorted
// in chunks of kRowChunk keys by a bitonic network in LDS; a row of several
// chunks is then merged by rank: a key's place is its place in its own chunk
// plus, in every other chunk, the number of keys below it (at most equal to
// it for the chunks before its own, so equal keys keep their chunk order).
__global__ void __launch_bounds__(kRowThreads) k_group_sort(ListGroup g) {
  __shared__ uint64_t sh[kRowChunk];
  const int l = blockIdx.y, r = blockIdx.x, tid = threadIdx.x;
  const int b = g.rows[l][r], len = g.rows[l][r + 1] - b;
  if (len <= 0) return;
  uint64_t *src = g.tmp[l] + b, *dst = g.keys[l] + b;
  const bool single = len <= kRowChunk;
  for (int c0 = 0; c0 < len; c0 += kRowChunk) {
    const int m = min(kRowChunk, len - c0);
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = tid; i < P; i += kRowThreads)
      sh[i] = i < m ? src[c0 + i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = tid; i < P; i += kRowThreads) {
          const int q = i ^ j;
          if (q > i) {
            const uint64_t x = sh[i], y = sh[q];
            if ((x > y) == ((i & k) == 0)) {
              sh[i] = y;
              sh[q] = x;
            }
          }
        }
        __syncthreads();
      }
    uint64_t *o = single ? dst : src + c0;
    for (int i = tid; i < m; i += kRowThreads) o[i] = sh[i];
    __syncthreads();
  }
  if (single) return;
  for (int i = tid; i < len; i += kRowThreads) {
    const int ci = i / kRowChunk;
    const uint64_t key = src[i];
    int rank = i - ci * kRowChunk;
    for (int c = 0; c * kRowChunk < len; ++c) {
      if (c == ci) continue;
      const uint64_t *ch = src + c * kRowChunk;
      int a = 0, z = min(kRowChunk, len - c * kRowChunk);
      while (a < z) {
        const int mid = (a + z) >> 1;
        const uint64_t v = ch[mid];
        if (c < ci ? v <= key : v < key)
          a = mid + 1;
        else
          z = mid;
      }
      rank += a;
    }
    dst[rank] = key;
  }
}

// Start offsets of each row in a list sorted by key (the radix-sort path).
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

// Trees of up to kGroupMaxSlots node slots group their lists by row (six
// launches; a row then holds at most kGroupMaxSlots keys, so its LDS sort
// stays short); larger trees sort the lists with the radix sort (measured on
// 8.7M-entry lists, where rows of ten thousand keys occur, 4.4 ms vs 0.7 ms).
constexpr int kGroupMaxSlots = 8192;

// Sort the live prefixes of two lists of (row << bits) | column keys and
// write their row start offsets.
static void group_lists(const Dev &d, const ListArgs &a, uint64_t *k0,
                        int32_t *r0, uint64_t *k1, int32_t *r1,
                        hipStream_t st) {
  if (a.ns > kGroupMaxSlots) {
    const int key_bits = 2 * a.bits;
    radix_sort(k0, nullptr, d.p2p_tmp, nullptr, a.p2p_cap, 0, key_bits,
               d.hist, d.partial, st, 1, d.counters + kCntP2P);
    radix_sort(k1, nullptr, d.m2l_tmp, nullptr, a.m2l_cap, 0, key_bits,
               d.hist, d.partial, st, 1, d.counters + kCntM2L);
    hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0,
                       st, a.ns, k0, d.counters + kCntP2P, a.p2p_cap, a.bits,
                       r0);
    hipLaunchKernelGGL(k_rowptr, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0,
                       st, a.ns, k1, d.counters + kCntM2L, a.m2l_cap, a.bits,
                       r1);
    return;
  }
  ListGroup g;
  g.keys[0] = k0;
  g.keys[1] = k1;
  g.tmp[0] = d.p2p_tmp;
  g.tmp[1] = d.m2l_tmp;
  g.cnt_ptr[0] = d.counters + kCntP2P;
  g.cnt_ptr[1] = d.counters + kCntM2L;
  g.cap[0] = a.p2p_cap;
  g.cap[1] = a.m2l_cap;
  g.rows[0] = r0;
  g.rows[1] = r1;
  g.fill[0] = d.lfill;
  g.fill[1] = d.lfill + (a.ns + 1);
  hipLaunchKernelGGL(k_group_zero, dim3(nblocks(a.ns + 1)), dim3(kThreads), 0,
                     st, a.ns, g);
  hipLaunchKernelGGL(k_group_count, dim3(kStepBlocks), dim3(kThreads), 0, st,
                     a.bits, g);
  for (int l = 0; l < 2; ++l)
    scan_exclusive_u32(reinterpret_cast<const uint32_t *>(g.fill[l]),
                       reinterpret_cast<uint32_t *>(g.rows[l]), a.ns + 1,
                       d.partial, st);
  hipLaunchKernelGGL(k_group_scatter, dim3(kStepBlocks), dim3(kThreads), 0,
                     st, a.bits, g);
  hipLaunchKernelGGL(k_group_sort, dim3(a.ns, 2), dim3(kRowThreads), 0, st, g);
}

// Node order of the list-driven kernels: longest list row first (list
// lengths vary by two orders of magnitude on a core + halo bunch).
// Spatial form (large P2P grids): each level of the tree is cut into eight
// runs of consecutive slots (neighbouring clusters) of about equal total list
// length, one per XCD, so that the workgroups of an XCD work on one region of
// the bunch and its L2 keeps the source leaves that neighbouring targets
// share (P2P HBM traffic on the 1M bunch 1.9 GB -> 0.26 GB per launch), while
// the XCDs get equal work; within an XCD, nodes run by decreasing class of
// list length (two classes per doubling) and in slot order within a class.
// Measured, the spatial form costs 5-9 % of P2P time on grids split into row
// parts (131k and 262k bunches) and is neutral on the unsplit 1M grid.  M2L
// takes it together with grouped row blocks (m2l_grouped).  The result is laid
// out for sched_idx: with c the smallest node count of an XCD, slot p * 8 + x
// (p < c) holds the p-th node of XCD x, and the nodes beyond the first c of
// each XCD (the cheapest ones, run last) follow from slot 8 c on, so the
// active nodes fill the first slots without holes (the rest is -1).  Only the
// launch order of workgroups depends on it, never a result.
constexpr int kOrderThreads = 1024;
constexpr int kOrderXcd = 32768;  // node slots ordered in one workgroup's LDS
constexpr int kOrderPer = kOrderXcd / kOrderThreads;

__device__ inline uint32_t row_len(const int32_t *row, int v, int ns) {
  return (v >= 1 && v < ns) ? (uint32_t)max(row[v + 1] - row[v], 0) : 0u;
}

// 14-bit sort keys of a row length, decreasing length first: exact (up to
// 16,383) or by class
__device__ inline uint32_t cost_key_exact(uint32_t len) {
  return 16383u - min(len, 16383u);
}
__device__ inline uint32_t cost_key_class(uint32_t len) {
  if (len == 0) return 63u;
  const int b = 31 - __clz(len);
  const uint32_t half = b >= 1 ? (len >> (b - 1)) & 1u : 0u;
  return 63u - min(2u * (uint32_t)b + half + 1u, 63u);
}

struct OrderJob {
  const int32_t *row[2];
  int32_t *order[2];
  int skip_empty[2];  // leave out slots with an empty row (P2P: non-leaves)
  int spatial[2];     // per-XCD regions (else one plain longest-first order)
};

// Per-level prefix sums of the list lengths give each slot's XCD; then a
// bitonic sort of the 32-bit keys (XCD << 29 | cost key << 15 | slot) in
// LDS, and each node is written to its XCD's next position.  Workgroup b
// orders job b.
__global__ void __launch_bounds__(kOrderThreads)
k_order_xcd(int ns, int olen, OrderJob job) {
  __shared__ uint32_t key[kOrderXcd];
  __shared__ uint32_t part[kOrderThreads];
  __shared__ int first[kXcds], cnt[kXcds];
  const int tid = threadIdx.x;
  const int32_t *row = job.row[blockIdx.x];
  int32_t *order = job.order[blockIdx.x];
  const bool skip = job.skip_empty[blockIdx.x] != 0;
  const bool spatial = job.spatial[blockIdx.x] != 0;
  int P = 1;
  while (P < ns) P <<= 1;
  // thread tid owns slots [tid * C, tid * C + C)
  const int C = P > kOrderThreads ? P / kOrderThreads : 1;
  const int v0 = tid * C;
  uint32_t sum = 0;
  if (v0 < P)
    for (int i = 0; i < C; ++i) sum += row_len(row, v0 + i, ns);
  part[tid] = sum;
  if (tid < kXcds) cnt[tid] = 0;
  for (int i = tid; i < olen; i += kOrderThreads) order[i] = -1;
  __syncthreads();
  for (int o = 1; o < kOrderThreads; o <<= 1) {
    const uint32_t a = tid >= o ? part[tid - o] : 0u;
    __syncthreads();
    part[tid] += a;
    __syncthreads();
  }
  const uint32_t total = part[kOrderThreads - 1];
  if (v0 < P) {
    uint32_t run = tid > 0 ? part[tid - 1] : 0u;
    for (int i = 0; i < C; ++i) {
      key[v0 + i] = run;  // exclusive prefix of the list lengths
      run += row_len(row, v0 + i, ns);
    }
  }
  __syncthreads();
  // XCD of every slot: midpoint of its cost within its level
  uint32_t kk[kOrderPer];
#pragma unroll
  for (int i = 0; i < kOrderPer; ++i) {
    const int v = v0 + i;
    kk[i] = 0xFFFFFFFFu;
    if (i < C && v >= 1 && v < ns) {
      const uint32_t len = row_len(row, v, ns);
      if (skip && len == 0) continue;
      const int lev = 31 - __clz(v);
      const int b = 1 << lev, e = min(b << 1, ns);
      const uint32_t tot = (e < P ? key[e] : total) - key[b];
      uint32_t x;
      if (!spatial) {
        x = 0;
      } else if (tot > 0) {
        const uint64_t mid = 2ull * (key[v] - key[b]) + len;  // twice the midpoint
        x = (uint32_t)min((uint64_t)(kXcds - 1), (kXcds * mid) / (2ull * tot));
      } else {
        const int anc = lev >= 3 ? (v >> (lev - 3)) : (v << (3 - lev));
        x = (uint32_t)(anc - kXcds);
      }
      atomicAdd(&cnt[x], 1);
      kk[i] = (x << 29) |
              ((spatial ? cost_key_class(len) : cost_key_exact(len)) << 15) |
              (uint32_t)v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kOrderPer; ++i)
    if (i < C && v0 + i < P) key[v0 + i] = kk[i];
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
  // the active node slots now lead, grouped by XCD
  int na = 0, cmin = cnt[0], excess[kXcds];
  for (int x = 0; x < kXcds; ++x) {
    na += cnt[x];
    cmin = min(cmin, cnt[x]);
  }
  for (int x = 0, e = 0; x < kXcds; ++x) {
    excess[x] = e;
    e += cnt[x] - cmin;
  }
  for (int i = tid; i < na; i += kOrderThreads) {
    const uint32_t x = key[i] >> 29;
    if (i == 0 || (key[i - 1] >> 29) != x) first[x] = i;
  }
  __syncthreads();
  for (int i = tid; i < na; i += kOrderThreads) {
    const int x = (int)(key[i] >> 29), r = i - first[x];
    const int pos = r < cmin ? r * kXcds + x : kXcds * cmin + excess[x] + (r - cmin);
    order[pos] = (int32_t)(key[i] & 0x7FFFu);
  }
}

// Above kOrderXcd slots: decreasing row length (key complemented length <<
// bits | slot, radix-sorted), in plain order (the sched_idx layout then
// reads it as eight interleaved queues).
__device__ inline uint32_t cost_bits(const int32_t *row, int v) {
  const int32_t len = row[v + 1] - row[v];
  return 0xFFFFu - (uint32_t)min(max(len, 0), 0xFFFF);
}

__global__ void k_cost_keys(int ns, const int32_t *row, int bits,
                            uint64_t *keys) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns) return;
  keys[v] = ((uint64_t)cost_bits(row, v) << bits) | (uint64_t)v;
}

__global__ void k_extract_order(int ns, int olen, const uint64_t *keys,
                                int bits, int32_t *order) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= olen) return;
  order[v] = v < ns ? (int32_t)(keys[v] & ((1ull << bits) - 1ull)) : -1;
}

static void order_by_cost(const Dev &d, const int32_t *row0, int32_t *order0,
                          const int32_t *row1, int32_t *order1, int ns,
                          int bits, bool spatial0, bool spatial1,
                          hipStream_t st) {
  const int olen = order_len(ns);
  if (ns <= kOrderXcd) {
    OrderJob job{{row0, row1}, {order0, order1}, {1, 0},
                 {spatial0 ? 1 : 0, spatial1 ? 1 : 0}};
    hipLaunchKernelGGL(k_order_xcd, dim3(2), dim3(kOrderThreads), 0, st, ns,
                       olen, job);
    return;
  }
  const int32_t *rows[2] = {row0, row1};
  int32_t *orders[2] = {order0, order1};
  for (int b = 0; b < 2; ++b) {
    hipLaunchKernelGGL(k_cost_keys, dim3(nblocks(ns)), dim3(kThreads), 0, st,
                       ns, rows[b], bits, d.okey);
    radix_sort(d.okey, nullptr, d.okey_tmp, nullptr, ns, 0, 16 + bits, d.hist,
               d.partial, st);
    hipLaunchKernelGGL(k_extract_order, dim3(nblocks(olen)), dim3(kThreads), 0,
                       st, ns, olen, d.okey, bits, orders[b]);
  }
}

void build_transposed_lists_dev(const Dev &d, const ListArgs &a,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_swap_keys, dim3(kStepBlocks), dim3(kThreads), 0, st,
                     d.p2p, d.counters + kCntP2P, a.p2p_cap, a.bits, d.p2p_T);
  hipLaunchKernelGGL(k_swap_keys, dim3(kStepBlocks), dim3(kThreads), 0, st,
                     d.m2l, d.counters + kCntM2L, a.m2l_cap, a.bits, d.m2l_T);
  // only the live prefix of each list (device-side count) is grouped
  group_lists(d, a, d.p2p_T, d.p2p_row_T, d.m2l_T, d.m2l_row_T, st);
  order_by_cost(d, d.p2p_row_T, d.order_p2p_T, d.m2l_row_T, d.order_m2l_T,
                a.ns, a.bits, a.p2p_spatial != 0, a.m2l_spatial != 0, st);
}

void build_lists_dev(const Dev &d, const ListArgs &a, hipStream_t st) {
  const int iters = 2 * a.depth + 1;
  const int head = std::min(iters, kHeadIters);
  hipLaunchKernelGGL(k_itl_head, dim3(1), dim3(kHeadThreads), 0, st, head,
                     d.front[0], d.front[1], a.fcap, d.counters, d.p2p,
                     a.p2p_cap, d.m2l, a.m2l_cap, d.kind, d.cen,
                     d.r2, d.gbar, a.eta, a.bits);
  for (int it = head; it < iters; ++it) {
    const int2 *cur = d.front[it & 1];
    int2 *nxt = d.front[(it + 1) & 1];
    hipLaunchKernelGGL(k_itl_step, dim3(kStepBlocks), dim3(kThreads), 0, st,
                       it, cur, nxt, a.fcap, d.counters, d.p2p, a.p2p_cap,
                       d.m2l, a.m2l_cap, d.kind, d.cen, d.r2, d.gbar,
                       a.eta, a.bits);
  }
  // only the live prefix of each list (device-side count) is grouped
  group_lists(d, a, d.p2p, d.p2p_row, d.m2l, d.m2l_row, st);
  order_by_cost(d, d.p2p_row, d.order_p2p, d.m2l_row, d.order_m2l, a.ns,
                a.bits, a.p2p_spatial != 0, a.m2l_spatial != 0, st);

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
