// Device-wide exclusive scan, stable LSD radix sort (8-bit digits) and a
// merge sort of (key, value) pairs for gfx950.  The merge sort presorts the
// k-d tree's three coordinate orders; the radix sort orders the node slots
// of large trees by cost; the scan serves both builds.
#include "internal.hpp"

namespace relfmm {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / kWave;

// Exclusive scan of one value per thread across a 256-thread block.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds,
                                                uint32_t *total) {
  const int tid = threadIdx.x;
  const int lane = lane_id(), wave = tid / kWave;
  uint32_t x = v;
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) lds[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    uint32_t s = lds[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const uint32_t *in, int n, uint32_t *partial) {
  __shared__ uint32_t lds[kScanThreads / kWave];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Single-block exclusive scan of the per-block partial sums, in chunks.
__global__ void __launch_bounds__(kScanThreads)
k_scan_partials(uint32_t *partial, int nb) {
  __shared__ uint32_t lds[kScanThreads / kWave];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += kScanThreads) {
    int i = base + threadIdx.x;
    uint32_t v = i < nb ? partial[i] : 0;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, lds, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_down(const uint32_t *in, uint32_t *out, int n, const uint32_t *partial) {
  __shared__ uint32_t lds[kScanThreads / kWave];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(s, lds, &tot) + partial[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

int scan_blocks(int n) { return (n + kScanTile - 1) / kScanTile; }

// One-workgroup exclusive scan for small arrays (the histograms of the radix
// sort): the array is staged through LDS with coalesced loads, each of the
// 1024 threads scans a contiguous run there, and the run totals are scanned
// across the workgroup.  One padding word every 32 keeps the runs of
// neighbouring threads in different LDS banks.
constexpr int kSmallScanThreads = 1024;
constexpr int kSmallScanMax = 32768;

__device__ inline int pad32(int i) { return i + (i >> 5); }

__global__ void __launch_bounds__(kSmallScanThreads)
k_scan_small(const uint32_t *in, uint32_t *out, int n) {
  __shared__ uint32_t buf[kSmallScanMax + kSmallScanMax / 32];
  __shared__ uint32_t wsum[kSmallScanThreads / kWave];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
#pragma unroll 8
  for (int i = tid; i < n; i += kSmallScanThreads) buf[pad32(i)] = in[i];
  __syncthreads();
  const int per = (n + kSmallScanThreads - 1) / kSmallScanThreads;
  const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
  uint32_t s = 0;
  for (int i = b0; i < b1; ++i) s += buf[pad32(i)];
  uint32_t inc = s;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off);
    if (lane >= off) inc += t;
  }
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t run = inc - s;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int i = b0; i < b1; ++i) {
    const uint32_t t = buf[pad32(i)];
    buf[pad32(i)] = run;
    run += t;
  }
  __syncthreads();
#pragma unroll 8
  for (int i = tid; i < n; i += kSmallScanThreads) out[i] = buf[pad32(i)];
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int n,
                        uint32_t *partial, hipStream_t st) {
  if (n <= 0) return;
  if (n <= kSmallScanMax) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallScanThreads), 0, st,
                       in, out, n);
    return;
  }
  int nb = scan_blocks(n);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, in, n,
                     partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st,
                     partial, nb);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, st, in, out,
                     n, partial);
}

// ---------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------

// nseg independent arrays of length n are sorted together: block b covers
// tile (b % nblk) of segment (b / nblk); histograms are laid out
// [segment][digit][tile], so one exclusive scan over all of them yields each
// element's global destination inside its own segment.
__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const uint64_t *keys, int n, const int *count, int nblk,
             int shift, uint32_t *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  if (count) n = min(n, *count);  // sort only the live prefix
  __syncthreads();
  const int seg = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  const uint64_t *kp = keys + (size_t)seg * n;
  const int base = blk * kSortTile;
  for (int i = 0; i < kSortItems; ++i) {
    int idx = base + i * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(kp[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[((size_t)seg * 256 + threadIdx.x) * nblk + blk] = h[threadIdx.x];
}

// Stable scatter: inside a tile, elements keep their input order.  Ranks of
// equal digits inside a wave come from a ballot match over the 8 digit bits.
// The whole tile is loaded into registers first, so the global-load latency
// is paid once per tile rather than once per 256-element chunk.
template <bool kVals>
__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                uint32_t *vout, int n, const int *count, int nblk, int shift,
                const uint32_t *offs) {
  if (count) n = min(n, *count);
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kSortWaves][256];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int seg = blockIdx.x / nblk, blk = blockIdx.x % nblk;
  const size_t sbase = (size_t)seg * n;
  const int base = blk * kSortTile;
  if (base >= n) return;  // whole tile beyond the live prefix (uniform)
  uint64_t keys[kSortItems];
  uint32_t vals[kSortItems];
#pragma unroll
  for (int c = 0; c < kSortItems; ++c) {
    const int idx = base + c * kSortThreads + tid;
    keys[c] = idx < n ? kin[sbase + idx] : 0;
    vals[c] = (kVals && idx < n) ? vin[sbase + idx] : 0;
  }
  run[tid] = offs[((size_t)seg * 256 + tid) * nblk + blk];
#pragma unroll
  for (int c = 0; c < kSortItems; ++c) {
    for (int k = tid; k < kSortWaves * 256; k += kSortThreads)
      (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const int idx = base + c * kSortThreads + tid;
    const bool valid = idx < n;
    const uint64_t key = keys[c];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(m & ((1ull << lane) - 1ull));
    if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t off = run[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][d];
      kout[off] = key;
      if (kVals) vout[off] = vals[c];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortWaves; ++w) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
}

template <typename T>
__global__ void k_copy(const T *in, T *out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

size_t radix_hist_entries(int n_max) {
  return (size_t)256 * ((n_max + kSortTile - 1) / kSortTile + 1);
}

void radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *ktmp, uint32_t *vtmp,
                int n, int bit_lo, int bit_hi, uint32_t *hist,
                uint32_t *partial, hipStream_t st, int nseg,
                const int *count) {
  if (n <= 1) return;
  const int nblk = (n + kSortTile - 1) / kSortTile;
  const int grid = nblk * nseg;
  uint64_t *ka = keys, *kb = ktmp;
  uint32_t *va = vals, *vb = vtmp;
  int passes = 0;
  for (int shift = bit_lo; shift < bit_hi; shift += 8, ++passes) {
    hipLaunchKernelGGL(k_radix_hist, dim3(grid), dim3(kSortThreads), 0, st, ka,
                       n, count, nblk, shift, hist);
    scan_exclusive_u32(hist, hist, 256 * grid, partial, st);
    if (vals)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(grid), dim3(kSortThreads),
                         0, st, ka, va, kb, vb, n, count, nblk, shift, hist);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3(grid),
                         dim3(kSortThreads), 0, st, ka, va, kb, vb, n, count,
                         nblk, shift, hist);
    uint64_t *kt = ka; ka = kb; kb = kt;
    uint32_t *vt = va; va = vb; vb = vt;
  }
  if (passes & 1) {
    const int tot = n * nseg;
    const int nb = (tot + 255) / 256;
    hipLaunchKernelGGL(k_copy<uint64_t>, dim3(nb), dim3(256), 0, st, ka, keys,
                       tot);
    if (vals)
      hipLaunchKernelGGL(k_copy<uint32_t>, dim3(nb), dim3(256), 0, st, va,
                         vals, tot);
  }
}

// ---------------------------------------------------------------------------
// Merge sort of (key, value) pairs by the pair order (key first, then value),
// nseg independent arrays of length n back to back: tiles of kMTile pairs are
// sorted in LDS by a bitonic network, then sorted runs are merged pairwise,
// each thread finding where its kMergeItems outputs start by a binary search
// along the merge path.  With the particle index as value this is the order
// a stable sort by key leaves.
// ---------------------------------------------------------------------------
constexpr int kMTile = 4096;
constexpr int kMThreads = 1024;
constexpr int kMergeThreads = 256;
constexpr int kMergeItems = 4;

__device__ inline bool pair_less(uint64_t ka, uint32_t va, uint64_t kb,
                                 uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

__global__ void __launch_bounds__(kMThreads)
k_tile_sort(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
            uint32_t *vout, int n, int ntile) {
  __shared__ uint64_t sk[kMTile];
  __shared__ uint32_t sv[kMTile];
  const int seg = blockIdx.x / ntile, t = blockIdx.x % ntile;
  const size_t base = (size_t)seg * n + (size_t)t * kMTile;
  const int m = min(kMTile, n - t * kMTile);
  for (int i = threadIdx.x; i < kMTile; i += kMThreads) {
    sk[i] = i < m ? kin[base + i] : ~0ull;  // padding sorts last
    sv[i] = i < m ? vin[base + i] : ~0u;
  }
  __syncthreads();
  for (int k = 2; k <= kMTile; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < kMTile; i += kMThreads) {
        const int q = i ^ j;
        if (q > i) {
          const uint64_t ka = sk[i], kb = sk[q];
          const uint32_t va = sv[i], vb = sv[q];
          if (pair_less(kb, vb, ka, va) == ((i & k) == 0)) {
            sk[i] = kb;
            sv[i] = vb;
            sk[q] = ka;
            sv[q] = va;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < m; i += kMThreads) {
    kout[base + i] = sk[i];
    vout[base + i] = sv[i];
  }
}

// Sorted runs of length w (the last one possibly shorter) merged pairwise.
__global__ void __launch_bounds__(kMergeThreads)
k_merge_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
             uint32_t *vout, int n, int w, int nblk) {
  const int seg = blockIdx.x / nblk, b = blockIdx.x % nblk;
  const int o = (b * kMergeThreads + (int)threadIdx.x) * kMergeItems;
  if (o >= n) return;
  const uint64_t *K = kin + (size_t)seg * n;
  const uint32_t *V = vin + (size_t)seg * n;
  uint64_t *KO = kout + (size_t)seg * n;
  uint32_t *VO = vout + (size_t)seg * n;
  const int p0 = o / (2 * w) * (2 * w);
  const int a0 = p0, na = min(w, n - p0);
  const int b0 = a0 + na, nb = min(w, n - b0);  // nb = 0 for a lone run
  const int d = o - p0;  // outputs of this pair before this thread's first
  // i = how many of the first d outputs come from the first run
  int lo = max(0, d - nb), hi = min(d, na);
  while (lo < hi) {
    const int i = (lo + hi) >> 1, j = d - i;
    if (pair_less(K[a0 + i], V[a0 + i], K[b0 + j - 1], V[b0 + j - 1]))
      lo = i + 1;
    else
      hi = i;
  }
  int ia = lo, ib = d - lo;
  const int cnt = min(kMergeItems, n - o);
  for (int k = 0; k < cnt; ++k) {
    bool from_a;
    if (ia >= na)
      from_a = false;
    else if (ib >= nb)
      from_a = true;
    else
      from_a = !pair_less(K[b0 + ib], V[b0 + ib], K[a0 + ia], V[a0 + ia]);
    if (from_a) {
      KO[o + k] = K[a0 + ia];
      VO[o + k] = V[a0 + ia];
      ++ia;
    } else {
      KO[o + k] = K[b0 + ib];
      VO[o + k] = V[b0 + ib];
      ++ib;
    }
  }
}

void merge_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *ktmp,
                      uint32_t *vtmp, int n, int nseg, hipStream_t st) {
  if (n <= 1) return;
  const int ntile = (n + kMTile - 1) / kMTile;
  int passes = 0;
  for (int64_t w = kMTile; w < n; w *= 2) ++passes;
  // the tile sort writes where the last merge pass must read from, so that
  // the result ends in keys / vals
  uint64_t *ka = keys, *kb = ktmp;
  uint32_t *va = vals, *vb = vtmp;
  if (passes & 1) {
    ka = ktmp;
    kb = keys;
    va = vtmp;
    vb = vals;
  }
  hipLaunchKernelGGL(k_tile_sort, dim3(ntile * nseg), dim3(kMThreads), 0, st,
                     keys, vals, ka, va, n, ntile);
  const int per_blk = kMergeThreads * kMergeItems;
  const int nblk = (n + per_blk - 1) / per_blk;
  for (int64_t w = kMTile; w < n; w *= 2) {
    hipLaunchKernelGGL(k_merge_pass, dim3(nblk * nseg), dim3(kMergeThreads), 0,
                       st, ka, va, kb, vb, n, (int)w, nblk);
    uint64_t *kt = ka; ka = kb; kb = kt;
    uint32_t *vt = va; va = vb; vb = vt;
  }
}

}  // namespace relfmm
