// Mean Lorentz factor, level-synchronous k-d tree build and leaf-order
// particle preparation (Sec. 3; Alg. direction4split and subdivide with the
// index split of App. B; array tree of Sec. 8).
//
// The tree is built from three presorted orders of the particles, one per
// axis, sorted by (coordinate, particle index).  A node's members occupy the
// same contiguous range [lo, hi) in all three orders, so its bounding box is
// read off the ends of the ranges, and its split along axis k keeps the first
// ceil(|S|/2) members of order k.  Each level then stably partitions every
// order by the per-particle "left" flag, which keeps all three orders sorted
// inside the children.  Decisions are FP64 without contraction so they match
// a plain serial evaluation bit for bit.
#include "internal.hpp"

namespace relfmm {

constexpr int kThreads = 256;
// Largest particle count presorted by the merge sort (measured: 131k and 262k
// particles faster than with the radix sort, 1M slower).
constexpr int kMergePresortMax = 1 << 18;

// --------------------------------------------------------------------------
// Mean Lorentz factor: gbar^2 = 1 + pbar.pbar (Sec. 3), deterministic order.
// --------------------------------------------------------------------------

__global__ void __launch_bounds__(kThreads)
k_gamma_partial(const double *u, int n, double *part) {
  __shared__ double sh[3][kThreads];
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n;
       i += kGammaBlocks * kThreads)
    for (int c = 0; c < 3; ++c) s[c] += u[3 * (size_t)i + c];
  for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_gamma_finish(const double *part, int n, double given,
                               double *gbar) {
  if (threadIdx.x != 0) return;
  if (given > 0.0) {
    *gbar = given;
    return;
  }
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < kGammaBlocks; ++b)
    for (int c = 0; c < 3; ++c) s[c] += part[3 * b + c];
  double p0 = s[0] / (double)n, p1 = s[1] / (double)n, p2 = s[2] / (double)n;
  *gbar = sqrt(1.0 + (p0 * p0 + p1 * p1 + p2 * p2));
}

// --------------------------------------------------------------------------
// Presort and per-level split
// --------------------------------------------------------------------------

__global__ void k_init_keys(const double *x, int n, uint64_t *key,
                            uint32_t *ord) {
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  for (int g = 0; g < 3; ++g) {
    key[(size_t)g * n + i] = double_key(x[3 * (size_t)i + g]);
    ord[(size_t)g * n + i] = (uint32_t)i;
  }
}

__global__ void k_init_nodes(int ns, int n, int32_t *lo, int32_t *hi,
                             int32_t *kind, int32_t *axis, int32_t *nleft) {
  int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns) return;
  lo[v] = (v == 1) ? 0 : -1;
  hi[v] = (v == 1) ? n : -1;
  kind[v] = 0;
  axis[v] = -1;
  nleft[v] = 0;
}

__global__ void k_init_seg(int n, int32_t *seg) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p < n) seg[p] = 1;
}

struct Ord3 {
  const uint32_t *o[3];
};
struct Ord3w {
  uint32_t *o[3];
};

// Alg. direction4split: the axis of the largest stretched box extent (ties to
// the lowest axis), FP64 without contraction.
__device__ inline int split_axis(const double (&a)[3], const double (&b)[3],
                                 double gb) {
  int k = 0;
  {
#pragma clang fp contract(off)
    const double s[3] = {1.0, 1.0, gb};
    double best = s[0] * (b[0] - a[0]);
    for (int g = 1; g < 3; ++g) {
      double wg = s[g] * (b[g] - a[g]);
      if (wg > best) {
        best = wg;
        k = g;
      }
    }
  }
  return k;
}

// Alg. direction4split and the split decision of Alg. subdivide for every
// node of one level; the bounding box (bbox of Sec. 2) is exact.
__global__ void k_level_nodes(int level, int depth, int leaf_size,
                              const double *x, Ord3 ord, int32_t *lo,
                              int32_t *hi, int32_t *kind, int32_t *axis,
                              int32_t *nleft, double *bmin, double *bmax,
                              const double *gbar) {
  int v = (1 << level) + blockIdx.x * kThreads + threadIdx.x;
  if (v >= (2 << level) || lo[v] < 0) return;
  const int l0 = lo[v], h0 = hi[v], cnt = h0 - l0;
  double a[3], b[3];
  for (int g = 0; g < 3; ++g) {
    a[g] = x[3 * (size_t)ord.o[g][l0] + g];
    b[g] = x[3 * (size_t)ord.o[g][h0 - 1] + g];
    bmin[3 * v + g] = a[g];
    bmax[3 * v + g] = b[g];
  }
  if (cnt > leaf_size && level < depth) {
    const int k = split_axis(a, b, *gbar);
    const int nl = (cnt + 1) / 2;
    kind[v] = 2;
    axis[v] = k;
    nleft[v] = nl;
    lo[2 * v] = l0;
    hi[2 * v] = l0 + nl;
    lo[2 * v + 1] = l0 + nl;
    hi[2 * v + 1] = h0;
  } else {
    kind[v] = 1;
    axis[v] = -1;
    nleft[v] = cnt;
  }
}

// The node decisions of one level (as k_level_nodes) and every position's
// flag (1 if it stays in the first part of its node) in one pass: the thread
// of every position works out its node's decision itself (the same
// arithmetic, from the node's ends in the three orders), the node's first
// position writes the node, and every thread writes its flag.  Positions
// still in a leaf of an earlier level keep flag 1.
__global__ void k_level_flags(int n, int level, int depth, int leaf_size,
                              const double *x, Ord3 ord, const int32_t *seg,
                              int32_t *lo, int32_t *hi, int32_t *kind,
                              int32_t *axis, int32_t *nleft, double *bmin,
                              double *bmax, const double *gbar,
                              uint8_t *flag) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int v = seg[p];
  if (v < (1 << level)) {
    flag[ord.o[0][p]] = 1;
    return;
  }
  const int l0 = lo[v], h0 = hi[v], cnt = h0 - l0;
  double a[3], b[3];
  for (int g = 0; g < 3; ++g) {
    a[g] = x[3 * (size_t)ord.o[g][l0] + g];
    b[g] = x[3 * (size_t)ord.o[g][h0 - 1] + g];
  }
  const bool split = cnt > leaf_size && level < depth;
  const int k = split ? split_axis(a, b, *gbar) : -1;
  const int nl = split ? (cnt + 1) / 2 : cnt;
  if (p == l0) {
    for (int g = 0; g < 3; ++g) {
      bmin[3 * v + g] = a[g];
      bmax[3 * v + g] = b[g];
    }
    kind[v] = split ? 2 : 1;
    axis[v] = k;
    nleft[v] = nl;
    if (split) {
      lo[2 * v] = l0;
      hi[2 * v] = l0 + nl;
      lo[2 * v + 1] = l0 + nl;
      hi[2 * v + 1] = h0;
    }
  }
  if (split)
    flag[ord.o[k][p]] = (p - l0 < nl) ? 1 : 0;
  else
    flag[ord.o[0][p]] = 1;
}

// The partition leaves two kinds of segment in place: the order along a
// splitting node's axis (its first nleft members are the left child) and
// every order of a leaf.  Only the two other orders of a splitting node
// move; their flags are gathered through the particle id into f2, the order
// of lower axis number in the first half, the other in the second (leaves
// fill both with 1, unused).
__device__ inline void other_axes(int k, int &a1, int &a2) {
  a1 = k == 0 ? 1 : 0;
  a2 = k == 2 ? 1 : 2;
}

__global__ void k_gather_flags(int n, Ord3 ord, const int32_t *seg,
                               const int32_t *kind, const int32_t *axis,
                               const uint8_t *flag, uint32_t *f2) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int v = seg[p];
  uint32_t f0 = 1u, f1 = 1u;
  if (kind[v] == 2) {
    int a1, a2;
    other_axes(axis[v], a1, a2);
    f0 = flag[ord.o[a1][p]];
    f1 = flag[ord.o[a2][p]];
  }
  f2[p] = f0;
  f2[(size_t)n + p] = f1;
}

// Stable partition of the moving orders inside every node by the flags.
// scanv is the exclusive scan of f2, so the flag at position i is
// scanv[i + 1] - scanv[i] (read next to scanv[i] rather than gathered again;
// the very last position takes the gathered flag).
__global__ void k_part_scatter(int n, const int32_t *seg, const int32_t *kind,
                               const int32_t *axis, const int32_t *lo,
                               const int32_t *nleft, Ord3 ord,
                               const uint8_t *flag, const uint32_t *scanv,
                               Ord3w out, int32_t *seg_out) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int v = seg[p], l0 = lo[v], nl = nleft[v];
  const bool split = kind[v] == 2;
  const int k = split ? axis[v] : -1;
  int a1 = 0, a2 = 0;
  if (split) other_axes(k, a1, a2);
  for (int a = 0; a < 3; ++a) {
    const uint32_t e = ord.o[a][p];
    int np = p;
    if (split && a != k) {
      const size_t h = a == a1 ? 0 : (size_t)n;
      const size_t i = h + p;
      const uint32_t sp = scanv[i];
      const bool left =
          i + 1 < 2 * (size_t)n ? scanv[i + 1] != sp : flag[e] != 0;
      const int sl = (int)(sp - scanv[h + l0]);
      np = left ? l0 + sl : l0 + nl + (p - l0 - sl);
    }
    out.o[a][np] = e;
  }
  seg_out[p] = split ? ((p - l0 < nl) ? 2 * v : 2 * v + 1) : v;
}

template <typename T>
__global__ void k_copy_t(const T *in, T *out, int n) {
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// Interpolation box of every node: the bounding box, except on an axis g
// whose half-width is below R/(8 s_g), R = max_g s_g h_g the node's largest
// stretched half-width, where the half-width becomes R/(8 s_g) about the
// bounding-box centre and the interval is clipped to the parent's box; a node
// of one particle (R = 0) takes its parent's box, a root of one particle
// gets R = 1.  The paper interpolates over the bounding box and is silent on
// zero widths, where the basis derivative of the adjoint divides by the
// width.  Each thread walks its node's ancestry from the root, so the boxes
// come out in one launch; every operation is that of the top-down
// definition, in FP64 without contraction.  Also the stretched
// half-diagonal squared of Alg. diam over this box.
__global__ void k_node_geom(int ns, const int32_t *kind, const double *bmin,
                            const double *bmax, double *cen, double *hw,
                            double *r2, const double *gbar) {
  int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns || v < 1 || kind[v] == 0) return;
  {
#pragma clang fp contract(off)
  const double s[3] = {1.0, 1.0, *gbar};
  const int lv = 31 - __clz(v);
  double lo[3], hi[3];
  for (int l = 0; l <= lv; ++l) {
    const int a = v >> (lv - l);
    double R = 0.0;
    for (int g = 0; g < 3; ++g) {
      double h = s[g] * ((bmax[3 * a + g] - bmin[3 * a + g]) * 0.5);
      if (h > R) R = h;
    }
    if (R == 0.0 && l > 0) continue;  // the parent's box, already in lo, hi
    if (R == 0.0) R = 1.0;
    for (int g = 0; g < 3; ++g) {
      double x0 = bmin[3 * a + g], x1 = bmax[3 * a + g];
      const double h = (x1 - x0) * 0.5;
      const double fl = ldexp(R, -3) / s[g];
      if (h < fl) {
        const double c = (x0 + x1) * 0.5;
        x0 = c - fl;
        x1 = c + fl;
        if (l > 0) {
          if (x0 < lo[g]) x0 = lo[g];
          if (x1 > hi[g]) x1 = hi[g];
        }
      }
      lo[g] = x0;
      hi[g] = x1;
    }
  }
  double rr = 0.0;
  for (int g = 0; g < 3; ++g) {
    cen[3 * v + g] = (lo[g] + hi[g]) * 0.5;
    const double h = (hi[g] - lo[g]) * 0.5;
    // coordinates equal to the last bits: keep the reference coordinate
    // defined
    const double hv = h > 0.0 ? h : ldexp(1.0, -40) / s[g];
    hw[3 * v + g] = hv;
    const double hs = s[g] * hv;
    rr = rr + hs * hs;
  }
  r2[v] = rr;
  }
}

static int nblocks(int n) { return (n + kThreads - 1) / kThreads; }

// --------------------------------------------------------------------------
// Bottom of the tree in one workgroup per node: once every node of a level
// holds at most kSubMax particles, each such node's three orders are loaded
// into LDS and all remaining levels (bounding box, axis, split, stable
// partition of the three orders) are done there, with the same decisions as
// the level-synchronous path.  A member e of a split node goes left iff
// (x_k(e), e) <= (x_k(pivot), pivot) in the presort order (coordinate, then
// particle index), the pivot being the ceil(|S|/2)-th member of order k; this
// is exactly the first ceil(|S|/2) members of order k.
// --------------------------------------------------------------------------
constexpr int kSubMax = 2048;
constexpr int kSubThreads = 1024;

__device__ inline void wg_exclusive_scan(uint32_t *v, int N, uint32_t *wsum) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int per = (N + kSubThreads - 1) / kSubThreads;
  const int b0 = min(N, tid * per), b1 = min(N, b0 + per);
  uint32_t s = 0;
  for (int i = b0; i < b1; ++i) s += v[i];
  uint32_t inc = s;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += t;
  }
  if (lane == kWave - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  uint32_t run = base + inc - s;
  for (int i = b0; i < b1; ++i) {
    const uint32_t t = v[i];
    v[i] = run;
    run += t;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kSubThreads)
k_subtree(int level0, int depth, int leaf_size, const double *x, Ord3 ord,
          int32_t *lo, int32_t *hi, int32_t *kind, int32_t *axis,
          int32_t *nleft, double *bmin, double *bmax, const double *gbar,
          uint32_t *ord_out, int32_t *seg_out) {
  __shared__ uint32_t so[2][3][kSubMax];    // the three orders, double buffer
  __shared__ uint32_t scan[3 * kSubMax];    // flags, then their prefix sums
  __shared__ uint8_t flg[3 * kSubMax];
  __shared__ int32_t hlo[2 * kSubMax], hhi[2 * kSubMax];  // heap of ranges
  __shared__ int16_t seg[kSubMax];          // heap index of each position
  __shared__ double pvx[kSubMax];           // per node of the level: pivot
  __shared__ uint32_t pve[kSubMax];
  __shared__ int8_t pax[kSubMax];           // split axis, -1 leaf, -2 none
  __shared__ uint32_t wsum[kSubThreads / kWave];
  __shared__ int any_split;
  const int vroot = (1 << level0) + blockIdx.x;
  if (lo[vroot] < 0) return;  // no such node
  const int tid = threadIdx.x;
  const int l0 = lo[vroot], cnt = hi[vroot] - l0;
  const double gb = *gbar;
  for (int i = tid; i < 3 * cnt; i += kSubThreads) {
    const int a = i / cnt, p = i - a * cnt;
    so[0][a][p] = ord.o[a][l0 + p];
  }
  for (int p = tid; p < cnt; p += kSubThreads) seg[p] = 1;
  for (int h = tid; h < 2 * kSubMax; h += kSubThreads) hlo[h] = hhi[h] = -1;
  __syncthreads();
  if (tid == 0) {
    hlo[1] = 0;
    hhi[1] = cnt;
  }
  int cur = 0;
  for (int d = 0;; ++d) {
    const int level = level0 + d, first = 1 << d;
    if (tid == 0) any_split = 0;
    __syncthreads();
    for (int k = tid; k < first; k += kSubThreads) {
      const int h = first + k, nlo = hlo[h];
      if (nlo < 0) {
        pax[k] = -2;
        continue;
      }
      const int nhi = hhi[h], c = nhi - nlo;
      const int v = (vroot << d) + k;
      double a[3], b[3];
      for (int g = 0; g < 3; ++g) {
        a[g] = x[3 * (size_t)so[cur][g][nlo] + g];
        b[g] = x[3 * (size_t)so[cur][g][nhi - 1] + g];
        bmin[3 * v + g] = a[g];
        bmax[3 * v + g] = b[g];
      }
      lo[v] = l0 + nlo;
      hi[v] = l0 + nhi;
      if (c > leaf_size && level < depth) {
        int kx = 0;
        {
#pragma clang fp contract(off)
          const double s[3] = {1.0, 1.0, gb};
          double best = s[0] * (b[0] - a[0]);
          for (int g = 1; g < 3; ++g) {
            const double wg = s[g] * (b[g] - a[g]);
            if (wg > best) {
              best = wg;
              kx = g;
            }
          }
        }
        const int nl = (c + 1) / 2;
        kind[v] = 2;
        axis[v] = kx;
        nleft[v] = nl;
        const uint32_t pe = so[cur][kx][nlo + nl - 1];
        pvx[k] = x[3 * (size_t)pe + kx];
        pve[k] = pe;
        pax[k] = (int8_t)kx;
        hlo[2 * h] = nlo;
        hhi[2 * h] = nlo + nl;
        hlo[2 * h + 1] = nlo + nl;
        hhi[2 * h + 1] = nhi;
        any_split = 1;
      } else {
        kind[v] = 1;
        axis[v] = -1;
        nleft[v] = c;
        pax[k] = -1;
      }
    }
    __syncthreads();
    if (!any_split) break;
    for (int i = tid; i < 3 * cnt; i += kSubThreads) {
      const int a = i / cnt, p = i - a * cnt;
      const int h = seg[p];
      int f = 1;
      if (h >= first) {
        const int k = h - first, ax = pax[k];
        if (ax >= 0) {
          const uint32_t e = so[cur][a][p];
          const double xv = x[3 * (size_t)e + ax];
          f = (xv < pvx[k]) || (xv == pvx[k] && e <= pve[k]);
        }
      }
      flg[i] = (uint8_t)f;
      scan[i] = (uint32_t)f;
    }
    __syncthreads();
    wg_exclusive_scan(scan, 3 * cnt, wsum);
    for (int i = tid; i < 3 * cnt; i += kSubThreads) {
      const int a = i / cnt, p = i - a * cnt;
      const int h = seg[p];
      int np = p;
      if (h >= first && pax[h - first] >= 0) {
        const int nlo = hlo[h], nl = hhi[2 * h] - hlo[2 * h];
        const int sl = (int)(scan[i] - scan[a * cnt + nlo]);
        np = flg[i] ? nlo + sl : nlo + nl + (p - nlo - sl);
      }
      so[cur ^ 1][a][np] = so[cur][a][p];
    }
    __syncthreads();
    for (int p = tid; p < cnt; p += kSubThreads) {
      const int h = seg[p];
      if (h >= first && pax[h - first] >= 0)
        seg[p] = (int16_t)(p < hhi[2 * h] ? 2 * h : 2 * h + 1);
    }
    cur ^= 1;
  }
  for (int p = tid; p < cnt; p += kSubThreads) {
    ord_out[l0 + p] = so[cur][0][p];
    const int h = seg[p];
    const int dd = 31 - __clz(h);
    seg_out[l0 + p] = (vroot << dd) + (h - (1 << dd));
  }
}


void build_tree_dev(const Dev &d, const TreeArgs &a, const double *x,
                    const double *u, hipStream_t st) {
  const int n = a.n, ns = a.ns;
  hipLaunchKernelGGL(k_gamma_partial, dim3(kGammaBlocks), dim3(kThreads), 0,
                     st, u, n, d.gpart);
  hipLaunchKernelGGL(k_gamma_finish, dim3(1), dim3(64), 0, st, d.gpart, n,
                     a.given_gbar, d.gbar);
  // presort by each coordinate with the particle index as tie-break: the
  // three orders are sorted together as three segments of one sort (a merge
  // sort, fewer launches, up to kMergePresortMax particles; an LSD radix sort,
  // less traffic, above)
  hipLaunchKernelGGL(k_init_keys, dim3(nblocks(n)), dim3(kThreads), 0, st, x,
                     n, d.key, d.ord_all);
  if (n <= kMergePresortMax)
    merge_sort_pairs(d.key, d.ord_all, d.key_tmp, d.ord_tmp_all, n, 3, st);
  else
    radix_sort(d.key, d.ord_all, d.key_tmp, d.ord_tmp_all, n, 0, 64, d.hist,
               d.partial, st, 3);
  hipLaunchKernelGGL(k_init_nodes, dim3(nblocks(ns)), dim3(kThreads), 0, st,
                     ns, n, d.lo, d.hi, d.kind, d.axis, d.nleft);
  hipLaunchKernelGGL(k_init_seg, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                     d.seg);
  Ord3 cur = {{d.ord_all, d.ord_all + n, d.ord_all + 2 * (size_t)n}};
  Ord3w nxt = {{d.ord_tmp_all, d.ord_tmp_all + n,
                d.ord_tmp_all + 2 * (size_t)n}};
  int32_t *seg = d.seg, *seg2 = d.seg_tmp;
  // levels above the first one whose nodes all fit kSubMax: level-synchronous
  int level0 = 0;
  while (level0 < a.depth && (n + (1 << level0) - 1) / (1 << level0) > kSubMax)
    ++level0;
  for (int l = 0; l < level0; ++l) {
    hipLaunchKernelGGL(k_level_flags, dim3(nblocks(n)), dim3(kThreads), 0, st,
                       n, l, a.depth, a.leaf_size, x, cur, seg, d.lo, d.hi,
                       d.kind, d.axis, d.nleft, d.bmin, d.bmax, d.gbar,
                       d.flag);
    hipLaunchKernelGGL(k_gather_flags, dim3(nblocks(n)), dim3(kThreads), 0, st,
                       n, cur, seg, d.kind, d.axis, d.flag, d.scanv);
    scan_exclusive_u32(d.scanv, d.scanv, 2 * n, d.partial, st);
    hipLaunchKernelGGL(k_part_scatter, dim3(nblocks(n)), dim3(kThreads), 0, st,
                       n, seg, d.kind, d.axis, d.lo, d.nleft, cur, d.flag,
                       d.scanv, nxt, seg2);
    Ord3 t = {{nxt.o[0], nxt.o[1], nxt.o[2]}};
    nxt = Ord3w{{const_cast<uint32_t *>(cur.o[0]),
                 const_cast<uint32_t *>(cur.o[1]),
                 const_cast<uint32_t *>(cur.o[2])}};
    cur = t;
    int32_t *ts = seg;
    seg = seg2;
    seg2 = ts;
  }
  if ((n + (1 << level0) - 1) / (1 << level0) <= kSubMax) {
    // the rest, one workgroup per node of level0; writes the final leaf
    // order (order 0) and the leaf of every position
    hipLaunchKernelGGL(k_subtree, dim3(1 << level0), dim3(kSubThreads), 0, st,
                       level0, a.depth, a.leaf_size, x, cur, d.lo, d.hi,
                       d.kind, d.axis, d.nleft, d.bmin, d.bmax, d.gbar,
                       d.ord_all, d.seg);
  } else {
    // leaves larger than kSubMax (level0 == depth): last level here
    hipLaunchKernelGGL(k_level_nodes, dim3(nblocks(1 << level0)),
                       dim3(kThreads), 0, st, level0, a.depth, a.leaf_size, x,
                       cur, d.lo, d.hi, d.kind, d.axis, d.nleft, d.bmin,
                       d.bmax, d.gbar);
    if (cur.o[0] != d.ord_all)
      hipLaunchKernelGGL(k_copy_t<uint32_t>, dim3(nblocks(n)), dim3(kThreads),
                         0, st, cur.o[0], d.ord_all, n);
    if (seg != d.seg)
      hipLaunchKernelGGL(k_copy_t<int32_t>, dim3(nblocks(n)), dim3(kThreads),
                         0, st, seg, d.seg, n);
  }
  hipLaunchKernelGGL(k_node_geom, dim3(nblocks(ns)), dim3(kThreads), 0, st, ns,
                     d.kind, d.bmin, d.bmax, d.cen, d.hw, d.r2, d.gbar);
}

// --------------------------------------------------------------------------
// Leaf-order particle data: coordinates relative to the leaf centre and the
// source weights (q gamma, q u) of the effective masses (Sec. 3).
// --------------------------------------------------------------------------

__global__ void k_prep(int n, const uint32_t *ord, const int32_t *seg,
                       const double *cen, const double *x, const double *u,
                       const double *q, double *xl, double *w, double *us,
                       float *w32, float *us32, int fp32) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const size_t i = ord[p];
  const int v = seg[p];
  double uu[3], xv[3];
  for (int g = 0; g < 3; ++g) {
    uu[g] = u[3 * i + g];
    xv[g] = x[3 * i + g] - cen[3 * v + g];
  }
  const double gam = sqrt(1.0 + (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]));
  const double qi = q[i];
  double wv[4] = {qi * gam, qi * uu[0], qi * uu[1], qi * uu[2]};
  for (int g = 0; g < 3; ++g) {
    xl[(size_t)g * n + p] = xv[g];
    us[(size_t)g * n + p] = uu[g];
  }
  for (int c = 0; c < 4; ++c) w[(size_t)c * n + p] = wv[c];
  if (fp32) {
    for (int g = 0; g < 3; ++g) us32[(size_t)g * n + p] = (float)uu[g];
    for (int c = 0; c < 4; ++c) w32[(size_t)c * n + p] = (float)wv[c];
  }
}

void prep_leaf_order(const Dev &d, int n, int ns, const double *x,
                     const double *u, const double *q, bool need_fp32,
                     hipStream_t st) {
  (void)ns;
  hipLaunchKernelGGL(k_prep, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                     d.ord_all, d.seg, d.cen, x, u, q, d.xl, d.w, d.us, d.w32,
                     d.us32, need_fp32 ? 1 : 0);
}

}  // namespace relfmm
