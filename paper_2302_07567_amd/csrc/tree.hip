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
    int k = 0;
    {
#pragma clang fp contract(off)
      const double s[3] = {1.0, 1.0, *gbar};
      double best = s[0] * (b[0] - a[0]);
      for (int g = 1; g < 3; ++g) {
        double wg = s[g] * (b[g] - a[g]);
        if (wg > best) {
          best = wg;
          k = g;
        }
      }
    }
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

// Per-particle flag: 1 if it stays in the first (left) part of its node.
__global__ void k_flags(int n, const int32_t *seg, const int32_t *kind,
                        const int32_t *axis, const int32_t *lo,
                        const int32_t *nleft, Ord3 ord, uint8_t *flag) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  int v = seg[p];
  if (kind[v] == 2) {
    int k = axis[v];
    flag[ord.o[k][p]] = (p - lo[v] < nleft[v]) ? 1 : 0;
  } else {
    flag[ord.o[0][p]] = 1;
  }
}

__global__ void k_gather_flags(int n, Ord3 ord, const uint8_t *flag,
                               uint32_t *f3) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  for (int a = 0; a < 3; ++a) f3[(size_t)a * n + p] = flag[ord.o[a][p]];
}

// Stable partition of the three orders inside every node by the flags.
__global__ void k_part_scatter(int n, const int32_t *seg, const int32_t *kind,
                               const int32_t *lo, const int32_t *nleft,
                               Ord3 ord, const uint8_t *flag,
                               const uint32_t *scanv, Ord3w out,
                               int32_t *seg_out) {
  int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const int v = seg[p], l0 = lo[v], nl = nleft[v];
  for (int a = 0; a < 3; ++a) {
    const uint32_t e = ord.o[a][p];
    const int sl = (int)(scanv[(size_t)a * n + p] - scanv[(size_t)a * n + l0]);
    const int np = flag[e] ? l0 + sl : l0 + nl + (p - l0 - sl);
    out.o[a][np] = e;
  }
  seg_out[p] = (kind[v] == 2) ? ((p - l0 < nl) ? 2 * v : 2 * v + 1) : v;
}

template <typename T>
__global__ void k_copy_t(const T *in, T *out, int n) {
  int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// Box centre and half-width for interpolation (zero widths get a floor of
// 2^-40 times the root's largest half-width) and the stretched
// half-diagonal squared of Alg. diam.
__global__ void k_node_geom(int ns, const int32_t *kind, const double *bmin,
                            const double *bmax, double *cen, double *hw,
                            double *r2, const double *gbar) {
  int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= ns || v < 1 || kind[v] == 0) return;
  {
#pragma clang fp contract(off)
  double hroot = 0.0;
  for (int g = 0; g < 3; ++g) {
    double h = (bmax[3 + g] - bmin[3 + g]) * 0.5;
    if (h > hroot) hroot = h;
  }
  const double hfloor = hroot > 0.0 ? ldexp(hroot, -40) : 1.0;
  const double s[3] = {1.0, 1.0, *gbar};
  double rr = 0.0;
  for (int g = 0; g < 3; ++g) {
    cen[3 * v + g] = (bmin[3 * v + g] + bmax[3 * v + g]) * 0.5;
    double h = (bmax[3 * v + g] - bmin[3 * v + g]) * 0.5;
    hw[3 * v + g] = h > 0.0 ? h : hfloor;
    double hs = s[g] * ((bmax[3 * v + g] - bmin[3 * v + g]) * 0.5);
    rr = rr + hs * hs;
  }
  r2[v] = rr;
  }
}

static int nblocks(int n) { return (n + kThreads - 1) / kThreads; }

void build_tree_dev(const Dev &d, const TreeArgs &a, const double *x,
                    const double *u, hipStream_t st) {
  const int n = a.n, ns = a.ns;
  hipLaunchKernelGGL(k_gamma_partial, dim3(kGammaBlocks), dim3(kThreads), 0,
                     st, u, n, d.gpart);
  hipLaunchKernelGGL(k_gamma_finish, dim3(1), dim3(64), 0, st, d.gpart, n,
                     a.given_gbar, d.gbar);
  // presort by each coordinate with the particle index as tie-break: the
  // three orders are sorted together as three segments of one radix sort
  hipLaunchKernelGGL(k_init_keys, dim3(nblocks(n)), dim3(kThreads), 0, st, x,
                     n, d.key, d.ord_all);
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
  for (int l = 0; l <= a.depth; ++l) {
    const int nodes = 1 << l;
    hipLaunchKernelGGL(k_level_nodes, dim3(nblocks(nodes)), dim3(kThreads), 0,
                       st, l, a.depth, a.leaf_size, x, cur, d.lo, d.hi,
                       d.kind, d.axis, d.nleft, d.bmin, d.bmax, d.gbar);
    if (l == a.depth) break;
    hipLaunchKernelGGL(k_flags, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                       seg, d.kind, d.axis, d.lo, d.nleft, cur, d.flag);
    hipLaunchKernelGGL(k_gather_flags, dim3(nblocks(n)), dim3(kThreads), 0, st,
                       n, cur, d.flag, d.scanv);
    scan_exclusive_u32(d.scanv, d.scanv, 3 * n, d.partial, st);
    hipLaunchKernelGGL(k_part_scatter, dim3(nblocks(n)), dim3(kThreads), 0, st,
                       n, seg, d.kind, d.lo, d.nleft, cur, d.flag, d.scanv,
                       nxt, seg2);
    Ord3 t = {{nxt.o[0], nxt.o[1], nxt.o[2]}};
    nxt = Ord3w{{const_cast<uint32_t *>(cur.o[0]),
                 const_cast<uint32_t *>(cur.o[1]),
                 const_cast<uint32_t *>(cur.o[2])}};
    cur = t;
    int32_t *ts = seg;
    seg = seg2;
    seg2 = ts;
  }
  // keep the final leaf order (any of the three orders) in the primary array
  if (cur.o[0] != d.ord_all)
    hipLaunchKernelGGL(k_copy_t<uint32_t>, dim3(nblocks(n)), dim3(kThreads), 0,
                       st, cur.o[0], d.ord_all, n);
  if (seg != d.seg)
    hipLaunchKernelGGL(k_copy_t<int32_t>, dim3(nblocks(n)), dim3(kThreads), 0,
                       st, seg, d.seg, n);
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
