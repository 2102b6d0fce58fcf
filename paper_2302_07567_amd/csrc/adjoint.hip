// Adjoint of the FMM with frozen structure: gradients of
//   L = sum_i (gE_i . E_i + gB_i . B_i)
// with respect to the positions x and the charges q.  The tree, boxes,
// proxies, mean Lorentz factor and lists are held fixed; the transposes of the
// operators of Alg. FMM run in reverse order:
//   L2P^T (anterpolation of the scaled cotangents, upward.hip),
//   L2L^T (children into parents, the form of M2M),
//   M2L^T (this file, grouped by SOURCE so each workgroup owns its outputs),
//   M2M^T (parent into children, the form of L2L),
//   P2M^T with the derivatives of the interpolation bases at the particles
//   (target side through the cumulative local fields, source side through
//   the multipole cotangents), and
//   P2P^T on the target side (grouped by target) and the source side
//   (grouped by source).
// For one pair term g(r) . C with g = r D^{-3/2} and D = r^T S r,
//   d/dr = D^{-3/2} C - 3 D^{-5/2} (C . r) S r,
// S = diag(1, 1, gbar^2) for the mean kernel, I + u_j u_j^T per source.
// With m_j = q_j (gamma_j, u_j), dL/dq_j = gamma_j mbar_j[0] + u_j . mbar_j[1:].
//
// Momenta (optional): u_j enters m_j (dgamma_j/du_j = u_j/gamma_j), the
// per-source denominator D = |r|^2 + (u_j.r)^2, whose derivative adds
// -3 (u_j.r) D^{-5/2} (C.r) r per pair on the source side, and, when the mean
// Lorentz factor is the function of u of Sec. 3, every mean kernel:
//   dL/dgbar = sum over near pairs of -3 gbar rz^2 D^{-5/2} (C.r)
//            + the same derivative of the far field (m2l.hip),
//   dgbar/du_j = pbar / (n gbar).
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace relfmm {

constexpr int kQ = kMaxDegree + 1;
constexpr int kMaxM = kQ * kQ * kQ;
constexpr int kThreads = 256;

// Scaled cotangents in leaf order: ebar = (ke gE, ke/c0 gB).
__global__ void k_adj_prep(int n, const uint32_t *ord, const double *gE,
                           const double *gB, double ke, double kb,
                           double *ebar, float *ebar32) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const size_t i = ord[p];
  for (int c = 0; c < 3; ++c) {
    const double e = ke * gE[3 * i + c], b = kb * gB[3 * i + c];
    ebar[(size_t)c * n + p] = e;
    ebar[(size_t)(3 + c) * n + p] = b;
    ebar32[(size_t)c * n + p] = (float)e;
    ebar32[(size_t)(3 + c) * n + p] = (float)b;
  }
}

__device__ inline float adj_rsq(float D) { return __builtin_amdgcn_rsqf(D); }
__device__ inline double adj_rsq(double D) { return 1.0 / sqrt(D); }

// M2L^T: for every source node s and source proxy nu,
//   Mbar_s[nu] = sum over targets t with (t, s) in the M2L list, over mu:
//                (g . Lbar^E_t[mu], g x Lbar^B_t[mu]),  g = g(xi_t,mu - xi_s,nu).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_m2l_adj(Cheb cb, int bits, const int32_t *kind, const double *cen,
          const double *hw, const int32_t *rowT, const uint64_t *keysT,
          const int32_t *order, const double *Lbar, const double *gbar,
          double *Mbar) {
  __shared__ T dX[3][kQ][kQ];  // [axis][target index][source index]
  __shared__ T sL[kMaxM][6];
  const int s = sched_idx(order, 1, 1, false).node;
  if (s < 0 || kind[s] == 0) return;
  const int tid = threadIdx.x;
  const int q = cb.p + 1, m = q * q * q;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const int r0 = rowT[s], r1 = rowT[s + 1];
  for (int nu0 = 0; nu0 < m; nu0 += kThreads) {
    const int nu = nu0 + tid;
    const bool act = nu < m;
    const int a2 = act ? nu / (q * q) : 0, b2 = act ? (nu / q) % q : 0,
              c2 = act ? nu % q : 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = r0; r < r1; ++r) {
      const int t = (int)(keysT[r] & mask);
      __syncthreads();
      for (int i = tid; i < 3 * q * q; i += kThreads) {
        const int g = i / (q * q), a1 = (i / q) % q, a3 = i % q;
        dX[g][a1][a3] = (T)((cen[3 * t + g] - cen[3 * s + g]) +
                            (hw[3 * t + g] * cb.t[a1] - hw[3 * s + g] * cb.t[a3]));
      }
      for (int i = tid; i < m; i += kThreads)
        for (int k = 0; k < 6; ++k) sL[i][k] = (T)Lbar[((size_t)t * m + i) * 6 + k];
      __syncthreads();
      if (act) {
        T ae = (T)0, ab[3] = {(T)0, (T)0, (T)0};
        int mu = 0;
        for (int a = 0; a < q; ++a) {
          const T rx = dX[0][a][a2];
          for (int b = 0; b < q; ++b) {
            const T ry = dX[1][b][b2];
            const T dxy = rx * rx + ry * ry;
            for (int c = 0; c < q; ++c, ++mu) {
              const T rz = dX[2][c][c2];
              const T iv = adj_rsq(dxy + g2 * (rz * rz));
              const T inv3 = iv * iv * iv;
              const T gx = rx * inv3, gy = ry * inv3, gz = rz * inv3;
              ae += gx * sL[mu][0] + gy * sL[mu][1] + gz * sL[mu][2];
              ab[0] += gy * sL[mu][5] - gz * sL[mu][4];
              ab[1] += gz * sL[mu][3] - gx * sL[mu][5];
              ab[2] += gx * sL[mu][4] - gy * sL[mu][3];
            }
          }
        }
        acc[0] += (double)ae;
        for (int k = 0; k < 3; ++k) acc[1 + k] += (double)ab[k];
      }
    }
    if (act)
      for (int k = 0; k < 4; ++k) Mbar[((size_t)s * m + nu) * 4 + k] = acc[k];
  }
}

// P2M^T and the basis derivatives at the particles of one leaf chunk:
//   mbar_j = sum_nu l_nu(x_j) Mbar[nu]
//   gx_j   = sum_nu grad l_nu(x_j) (m_j . Mbar[nu] + ebar_j . Lcum[nu]).
// The 1-D derivatives are l_k'(x) = sum_j D[j][k] l_j(x) / h: the derivative
// of a degree-n polynomial interpolated at the nodes (Theorem 1), with the
// differentiation matrix D[j][k] = l_k'(t_j).
constexpr int kLeafThreads = 256;

// One thread per particle of a 256-particle chunk of one leaf; the bases and
// their derivatives in registers, the leaf's multipole cotangents (4) and
// cumulative locals (6) staged in LDS and read as broadcasts.  Per proxy:
//   s = w . Mbar[nu] + ebar . Lcum[nu],  grad += grad l_nu s,
//   mbar += l_nu Mbar[nu].
template <int Q>
__global__ void __launch_bounds__(kLeafThreads)
k_adj_leaf(Cheb cb, int n, const int32_t *kind, const int32_t *lo,
           const int32_t *hi, const double *hw, const double *xl,
           const double *w, const double *ebar, const double *Mbar,
           const double *Lcum, double *gx, double *mbar) {
  constexpr int MM = Q * Q * Q;
  __shared__ double Ms[MM * 4];
  __shared__ double Ls[MM * 6];
  __shared__ double xa[2][Q][kLeafThreads];  // x basis and derivative
  const int v = blockIdx.x;
  if (kind[v] != 1) return;
  const int l0 = lo[v], cnt = hi[v] - l0;
  const int i0 = blockIdx.y * kLeafThreads;
  if (i0 >= cnt) return;
  const int tid = threadIdx.x;
  const int ii = i0 + tid;
  const bool act = ii < cnt;
  const int p = l0 + (act ? ii : 0);
  for (int i = tid; i < MM * 4; i += kLeafThreads)
    Ms[i] = Mbar[(size_t)v * MM * 4 + i];
  for (int i = tid; i < MM * 6; i += kLeafThreads)
    Ls[i] = Lcum[(size_t)v * MM * 6 + i];
  // bases and derivatives: x axis to LDS (indexed by the runtime loop), y and
  // z in registers (fully unrolled loops)
  double lb[3][Q], db[3][Q];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const double h = hw[3 * v + g];
    basis1d_q<Q>(cb, xl[(size_t)g * n + p] / h, lb[g]);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < Q; ++j) s += cb.D[j][k] * lb[g][j];
      db[g][k] = s / h;
    }
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    xa[0][k][tid] = lb[0][k];
    xa[1][k][tid] = db[0][k];
  }
  double wt[10];
#pragma unroll
  for (int k = 0; k < 4; ++k) wt[k] = w[(size_t)k * n + p];
#pragma unroll
  for (int k = 0; k < 6; ++k) wt[4 + k] = ebar[(size_t)k * n + p];
  __syncthreads();
  double grad[3] = {0.0, 0.0, 0.0}, mb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int a = 0; a < Q; ++a) {
    const double la = xa[0][a][tid], da = xa[1][a][tid];
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      const double lab = la * lb[1][b], dab = da * lb[1][b], ladb = la * db[1][b];
      const int mu0 = (a * Q + b) * Q;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const double *mr = Ms + (mu0 + c) * 4, *lr = Ls + (mu0 + c) * 6;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) s += wt[k] * mr[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) s += wt[4 + k] * lr[k];
        const double lcs = lb[2][c] * s;
        grad[0] += dab * lcs;
        grad[1] += ladb * lcs;
        grad[2] += lab * (db[2][c] * s);
        const double l = lab * lb[2][c];
#pragma unroll
        for (int k = 0; k < 4; ++k) mb[k] += l * mr[k];
      }
    }
  }
  if (act) {
    for (int c = 0; c < 3; ++c) gx[(size_t)c * n + p] = grad[c];
    for (int k = 0; k < 4; ++k) mbar[(size_t)k * n + p] = mb[k];
  }
}

template <int Q>
struct AdjLeafLaunch {
  static void run(const Dev &d, const Cheb &cb, int n, int ns, int max_leaf,
                  hipStream_t st) {
    const dim3 grid(ns, (max_leaf + kLeafThreads - 1) / kLeafThreads);
    hipLaunchKernelGGL(k_adj_leaf<Q>, grid, dim3(kLeafThreads), 0, st, cb, n,
                       d.kind, d.lo, d.hi, d.hw, d.xl, d.w, d.ebar, d.Mbar,
                       d.L, d.gx, d.mbar);
  }
};

// ---------------------------------------------------------------------------
// P2P^T.  Target side: lanes are targets, staged tiles are sources (as in the
// forward P2P).  Source side: lanes are sources, staged tiles are targets of
// the source-grouped list.  Both split each tile over four waves and add the
// wave partials in a fixed order; offsets are formed in FP64 and rounded once.
// ---------------------------------------------------------------------------

// 64 partners per wave and tile; workgroups of one, two or four waves by
// leaf size (tiles of 64 WAVES partners).
constexpr int kAdjPerWave = kWave;

// Staged partners; coordinates in the lane particles' leaf frame, C = double
// (exact offsets) or, in the FP32 kernels, C = float for partner leaves well
// separated from the own leaf (the criterion of the forward P2P).
template <typename T, typename C>
struct AdjSrc {  // a staged source for the target side
  C x, y, z;
  T w0, w1, w2, w3, u0, u1, u2;
};
template <typename T, typename C>
struct AdjTgt {  // a staged target for the source side
  C x, y, z;
  T e0, e1, e2, b0, b1, b2;
};
constexpr double kAdjFarRatio = 8.0;
// Pair-loop unroll by particles per lane; with two per lane, split launches
// take no unrolling (as in the forward P2P; 1 % faster on the 262k bunch).
constexpr int kAdjUnroll[3] = {0, 4, 2};

// Gradient of g(r).C for one pair (D set to 1 and the pair zeroed for the
// self term, SELF), accumulated into acc; g itself is returned in gvec.
// Also returns t5 = 3 D^{-5/2} (C.r) and, for the per-source kernel,
// ur = u_j.r (the parts of the momentum and gbar derivatives).
template <typename T, int MODE, bool SELF>
__device__ inline void pair_grad_s(T rx, T ry, T rz, T u0, T u1, T u2, T g2,
                                   T cx, T cy, T cz, bool self, T *acc,
                                   T *gvec, T &t5o, T &uro) {
  T sx, sy, sz;
  if constexpr (MODE == 0) {
    sx = rx;
    sy = ry;
    sz = g2 * rz;
    uro = (T)0;
  } else {
    const T ur = u0 * rx + u1 * ry + u2 * rz;
    sx = rx + ur * u0;
    sy = ry + ur * u1;
    sz = rz + ur * u2;
    uro = ur;
  }
  T D = rx * sx + ry * sy + rz * sz;
  if (SELF && self) D = (T)1;
  T iv = adj_rsq(D);
  if (SELF && self) iv = (T)0;
  const T iv2 = iv * iv;
  const T inv3 = iv * iv2;
  const T t5 = (T)3 * inv3 * iv2 * (cx * rx + cy * ry + cz * rz);
  t5o = t5;
  // two fused multiply-adds per component (not a product, an FMA and an add)
  acc[0] = fma(-t5, sx, fma(inv3, cx, acc[0]));
  acc[1] = fma(-t5, sy, fma(inv3, cy, acc[1]));
  acc[2] = fma(-t5, sz, fma(inv3, cz, acc[2]));
  gvec[0] = rx * inv3;
  gvec[1] = ry * inv3;
  gvec[2] = rz * inv3;
}

// Tile cursor over the entries of one list row: (entry r, first member j0 of
// the staged tile) and the partner leaf's range and centre offset.
struct AdjCursor {
  int r, r1, j0, p, pl, pc;
  bool far;
  double dx, dy, dz;
};

// Opens list entry c.r.  far: the partner leaf is well separated from the own
// leaf o (largest coordinate magnitude of the two boxes in o's frame at most
// kAdjFarRatio times their distance, z stretched by zs) and hybrid is set.
__device__ inline void adj_open(AdjCursor &c, const uint64_t *keys,
                                uint64_t mask, const int32_t *lo,
                                const int32_t *hi, const double *cen,
                                const double *hw, int o,
                                const double (&co)[3], double zs,
                                bool hybrid) {
  c.p = (int)(keys[c.r] & mask);
  c.pl = lo[c.p];
  c.pc = hi[c.p] - c.pl;
  c.dx = cen[3 * c.p] - co[0];
  c.dy = cen[3 * c.p + 1] - co[1];
  c.dz = cen[3 * c.p + 2] - co[2];
  c.far = false;
  if (hybrid && c.p != o) {
    const double dd[3] = {c.dx, c.dy, c.dz}, sz[3] = {1.0, 1.0, zs};
    double gap2 = 0.0, mx = 0.0;
    for (int g = 0; g < 3; ++g) {
      const double hp = hw[3 * c.p + g], ho = hw[3 * o + g];
      const double gap = fmax(fabs(dd[g]) - hp - ho, 0.0) * sz[g];
      gap2 += gap * gap;
      mx = fmax(mx, fmax(fabs(dd[g]) + hp, ho) * sz[g]);
    }
    c.far = mx * mx <= kAdjFarRatio * kAdjFarRatio * gap2;
  }
}

// GB (mean kernel only): also the gbar derivative of the target's near sum,
// sum_j t5 rz^2 (times -gbar), into gG.  TPL targets per lane (64 TPL per
// workgroup): each staged source is read from LDS once for TPL pairs.
template <typename T, int MODE, bool GB, int TPL, int WAVES, int UNR>
__global__ void __launch_bounds__(WAVES * kWave)
k_p2p_adj_tgt(int n, int bits, const int32_t *kind, const int32_t *lo,
              const int32_t *hi, const double *cen, const double *hw,
              const int32_t *row, const uint64_t *keys, const int32_t *order,
              const double *xl, const T *w, const T *us, const T *eb,
              const double *gbar, double *gx, double *gG, int ny, int nsplit,
              double *parts) {
  constexpr bool kHybrid = sizeof(T) == 4 && MODE == 0;
  constexpr int NR = GB ? 4 : 3;
  constexpr int kTile = WAVES * kWave;
  __shared__ union {
    AdjSrc<T, double> d[kTile];
    AdjSrc<T, float> f[kTile];
  } sh;
  __shared__ double red[WAVES > 1 ? WAVES - 1 : 1][NR][TPL * kWave];
  const SchedIdx si = sched_idx(order, ny, nsplit, true);
  const int t = si.node;
  if (t < 0 || kind[t] != 1) return;
  const int tl = lo[t], tc = hi[t] - tl;
  const int i0 = si.y * kWave * TPL;
  if (i0 >= tc) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  int ii[TPL], pi[TPL];
  double xi[TPL], yi[TPL], zi[TPL];
  T e[TPL][6];
  double acc[TPL][NR];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    ii[k] = i0 + k * kWave + lane;
    pi[k] = tl + (ii[k] < tc ? ii[k] : 0);
    xi[k] = xl[pi[k]];
    yi[k] = xl[(size_t)n + pi[k]];
    zi[k] = xl[2 * (size_t)n + pi[k]];
#pragma unroll
    for (int c = 0; c < 6; ++c) e[k][c] = eb[(size_t)c * n + pi[k]];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[k][q] = 0.0;
  }
  AdjCursor c;
  {
    const int part = si.z, rlen = row[t + 1] - row[t];
    c.r = row[t] + rlen * part / nsplit;
    c.r1 = row[t] + rlen * (part + 1) / nsplit;
  }
  c.j0 = 0;
  // raw source data of this thread for the next tile (prefetched)
  double rx_ = 1.0e12, ry_ = 1.0e12, rz_ = 1.0e12;
  T rw[7] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
  auto load = [&]() {
    const bool in = c.j0 + tid < c.pc;
    const size_t q = (size_t)c.pl + c.j0 + tid;
    rx_ = in ? xl[q] + c.dx : 1.0e12;
    ry_ = in ? xl[n + q] + c.dy : 1.0e12;
    rz_ = in ? xl[2 * (size_t)n + q] + c.dz : 1.0e12;
    rw[0] = in ? w[q] : (T)0;
    rw[1] = in ? w[n + q] : (T)0;
    rw[2] = in ? w[2 * (size_t)n + q] : (T)0;
    rw[3] = in ? w[3 * (size_t)n + q] : (T)0;
    rw[4] = in ? us[q] : (T)0;
    rw[5] = in ? us[n + q] : (T)0;
    rw[6] = in ? us[2 * (size_t)n + q] : (T)0;
  };
  if (c.r < c.r1) {
    adj_open(c, keys, mask, lo, hi, cen, hw, t, ct, gbd, kHybrid);
    load();
  }
  while (c.r < c.r1) {
    const int s = c.p, j0 = c.j0, sc = c.pc;
    const bool far = c.far;
    __syncthreads();
    if (far) {
      AdjSrc<T, float> v;
      v.x = (float)rx_;
      v.y = (float)ry_;
      v.z = (float)rz_;
      v.w0 = rw[0];
      v.w1 = rw[1];
      v.w2 = rw[2];
      v.w3 = rw[3];
      v.u0 = rw[4];
      v.u1 = rw[5];
      v.u2 = rw[6];
      sh.f[tid] = v;
    } else {
      AdjSrc<T, double> v;
      v.x = rx_;
      v.y = ry_;
      v.z = rz_;
      v.w0 = rw[0];
      v.w1 = rw[1];
      v.w2 = rw[2];
      v.w3 = rw[3];
      v.u0 = rw[4];
      v.u1 = rw[5];
      v.u2 = rw[6];
      sh.d[tid] = v;
    }
    __syncthreads();
    c.j0 += kTile;
    if (c.j0 >= c.pc) {
      ++c.r;
      c.j0 = 0;
      if (c.r < c.r1) adj_open(c, keys, mask, lo, hi, cen, hw, t, ct, gbd, kHybrid);
    }
    if (c.r < c.r1) load();
    const int kb = wave * kAdjPerWave;
    if (j0 + kb >= sc) continue;
    T a[TPL][3], ag[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      a[k][0] = a[k][1] = a[k][2] = (T)0;
      ag[k] = (T)0;
    }
    auto body = [&](auto self_tag, const auto *shp, const auto &px,
                    const auto &py, const auto &pz) {
      constexpr bool SELF = decltype(self_tag)::value;
#pragma unroll UNR
      for (int k = 0; k < kAdjPerWave; ++k) {
        const auto &sj = shp[kb + k];
#pragma unroll
        for (int tp = 0; tp < TPL; ++tp) {
          const T rx = (T)(px[tp] - sj.x), ry = (T)(py[tp] - sj.y),
                  rz = (T)(pz[tp] - sj.z);
          // C = w0_j ebar_i + bbar_i x wu_j
          const T cx = sj.w0 * e[tp][0] + (e[tp][4] * sj.w3 - e[tp][5] * sj.w2);
          const T cy = sj.w0 * e[tp][1] + (e[tp][5] * sj.w1 - e[tp][3] * sj.w3);
          const T cz = sj.w0 * e[tp][2] + (e[tp][3] * sj.w2 - e[tp][4] * sj.w1);
          T gv[3], t5, ur;
          pair_grad_s<T, MODE, SELF>(rx, ry, rz, sj.u0, sj.u1, sj.u2, g2, cx,
                                     cy, cz, j0 + kb + k == ii[tp], a[tp], gv,
                                     t5, ur);
          if constexpr (GB) ag[tp] += t5 * (rz * rz);
        }
      }
    };
    if (s == t) {
      body(std::true_type{}, sh.d, xi, yi, zi);
    } else if (far) {
      if constexpr (kHybrid) {
        float xf[TPL], yf[TPL], zf[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
          xf[k] = (float)xi[k];
          yf[k] = (float)yi[k];
          zf[k] = (float)zi[k];
        }
        body(std::false_type{}, sh.f, xf, yf, zf);
      }
    } else {
      body(std::false_type{}, sh.d, xi, yi, zi);
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[k][q] += (double)a[k][q];
      if constexpr (GB) acc[k][3] += (double)ag[k];
    }
  }
  if (wave > 0)
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) red[wave - 1][q][k * kWave + lane] = acc[k][q];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (ii[k] >= tc) continue;
      for (int wv = 0; wv < WAVES - 1; ++wv)
        for (int q = 0; q < NR; ++q) acc[k][q] += red[wv][q][k * kWave + lane];
      if (si.z > 0) {
        // a later part of the row: its own slice, added by k_adj_tgt_combine
        double *pp = parts + (size_t)(si.z - 1) * NR * n;
        for (int q = 0; q < NR; ++q) pp[(size_t)q * n + pi[k]] = acc[k][q];
        continue;
      }
      for (int q = 0; q < 3; ++q) gx[(size_t)q * n + pi[k]] += acc[k][q];
      if constexpr (GB) gG[pi[k]] = acc[k][3];
    }
  }
}

// GU (per-source kernel only): also the derivative through the source's
// own denominator, -sum_i t5 (u_j.r) r, into gu.  TPL sources per lane.
template <typename T, int MODE, bool GU, int TPL, int WAVES, int UNR>
__global__ void __launch_bounds__(WAVES * kWave)
k_p2p_adj_src(int n, int bits, const int32_t *kind, const int32_t *lo,
              const int32_t *hi, const double *cen, const double *hw,
              const int32_t *rowT, const uint64_t *keysT,
              const int32_t *order, const double *xl, const T *w, const T *us,
              const T *eb, const double *gbar, double *gx, double *mbar,
              double *gu, int ny, int nsplit, double *parts) {
  constexpr bool kHybrid = sizeof(T) == 4 && MODE == 0;
  constexpr int NR = GU ? 10 : 7;
  constexpr int kTile = WAVES * kWave;
  __shared__ union {
    AdjTgt<T, double> d[kTile];
    AdjTgt<T, float> f[kTile];
  } sh;
  __shared__ double red[WAVES > 1 ? WAVES - 1 : 1][NR][TPL * kWave];
  const SchedIdx si = sched_idx(order, ny, nsplit, true);
  const int s = si.node;
  if (s < 0 || kind[s] != 1) return;
  const int sl = lo[s], sc = hi[s] - sl;
  const int j0s = si.y * kWave * TPL;
  if (j0s >= sc) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const double cs[3] = {cen[3 * s], cen[3 * s + 1], cen[3 * s + 2]};
  int jj[TPL], pj[TPL];
  double xj[TPL], yj[TPL], zj[TPL];
  T w0[TPL], w1[TPL], w2[TPL], w3[TPL], u0[TPL], u1[TPL], u2[TPL];
  double acc[TPL][NR];  // -grad x (3), mbar (4), [grad u (3)]
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    jj[k] = j0s + k * kWave + lane;
    pj[k] = sl + (jj[k] < sc ? jj[k] : 0);
    const int p = pj[k];
    xj[k] = xl[p];
    yj[k] = xl[(size_t)n + p];
    zj[k] = xl[2 * (size_t)n + p];
    w0[k] = w[p];
    w1[k] = w[(size_t)n + p];
    w2[k] = w[2 * (size_t)n + p];
    w3[k] = w[3 * (size_t)n + p];
    u0[k] = us[p];
    u1[k] = us[(size_t)n + p];
    u2[k] = us[2 * (size_t)n + p];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[k][q] = 0.0;
  }
  AdjCursor c;
  {
    const int part = si.z, rlen = rowT[s + 1] - rowT[s];
    c.r = rowT[s] + rlen * part / nsplit;
    c.r1 = rowT[s] + rlen * (part + 1) / nsplit;
  }
  c.j0 = 0;
  double rx_ = 1.0e12, ry_ = 1.0e12, rz_ = 1.0e12;
  T re[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
  auto load = [&]() {
    const bool in = c.j0 + tid < c.pc;
    const size_t q = (size_t)c.pl + c.j0 + tid;
    rx_ = in ? xl[q] + c.dx : 1.0e12;
    ry_ = in ? xl[n + q] + c.dy : 1.0e12;
    rz_ = in ? xl[2 * (size_t)n + q] + c.dz : 1.0e12;
#pragma unroll
    for (int k = 0; k < 6; ++k) re[k] = in ? eb[(size_t)k * n + q] : (T)0;
  };
  if (c.r < c.r1) {
    adj_open(c, keysT, mask, lo, hi, cen, hw, s, cs, gbd, kHybrid);
    load();
  }
  while (c.r < c.r1) {
    const int t = c.p, i0 = c.j0, tc = c.pc;
    const bool far = c.far;
    __syncthreads();
    if (far) {
      AdjTgt<T, float> v;
      v.x = (float)rx_;
      v.y = (float)ry_;
      v.z = (float)rz_;
      v.e0 = re[0];
      v.e1 = re[1];
      v.e2 = re[2];
      v.b0 = re[3];
      v.b1 = re[4];
      v.b2 = re[5];
      sh.f[tid] = v;
    } else {
      AdjTgt<T, double> v;
      v.x = rx_;
      v.y = ry_;
      v.z = rz_;
      v.e0 = re[0];
      v.e1 = re[1];
      v.e2 = re[2];
      v.b0 = re[3];
      v.b1 = re[4];
      v.b2 = re[5];
      sh.d[tid] = v;
    }
    __syncthreads();
    c.j0 += kTile;
    if (c.j0 >= c.pc) {
      ++c.r;
      c.j0 = 0;
      if (c.r < c.r1) adj_open(c, keysT, mask, lo, hi, cen, hw, s, cs, gbd, kHybrid);
    }
    if (c.r < c.r1) load();
    const int kb = wave * kAdjPerWave;
    if (i0 + kb >= tc) continue;
    // Per pair, with the lane's source weights w0, wu = (w1, w2, w3) fixed:
    //   C = w0 ebar_i + bbar_i x wu,  C.r = w0 (ebar_i.r) + wu.(r x bbar_i),
    //   sum_i D^{-3/2} C = w0 sum D^{-3/2} ebar_i + (sum D^{-3/2} bbar_i) x wu,
    // so the pair loop keeps sum D^{-3/2} ebar (se), sum D^{-3/2} bbar (sb)
    // and sum D^{-5/2} (C.r) S r (ss) and forms C only once per tile; the
    // factor 3 of the D^{-5/2} terms is applied there too.
    T se[TPL][3], sb[TPL][3], ss[TPL][3], mg[TPL], mu3[TPL][3], au[TPL][3];
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      mg[k] = (T)0;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        se[k][q] = sb[k][q] = ss[k][q] = mu3[k][q] = au[k][q] = (T)0;
    }
    auto body = [&](auto self_tag, const auto *shp, const auto &px,
                    const auto &py, const auto &pz) {
      constexpr bool SELF = decltype(self_tag)::value;
#pragma unroll UNR
      for (int k = 0; k < kAdjPerWave; ++k) {
        const auto &ti = shp[kb + k];
#pragma unroll
        for (int tp = 0; tp < TPL; ++tp) {
          const T rx = (T)(ti.x - px[tp]), ry = (T)(ti.y - py[tp]),
                  rz = (T)(ti.z - pz[tp]);
          T sx, sy, sz, ur = (T)0;
          if constexpr (MODE == 0) {
            sx = rx;
            sy = ry;
            sz = g2 * rz;
          } else {
            ur = u0[tp] * rx + u1[tp] * ry + u2[tp] * rz;
            sx = rx + ur * u0[tp];
            sy = ry + ur * u1[tp];
            sz = rz + ur * u2[tp];
          }
          T D = rx * sx + ry * sy + rz * sz;
          const bool self = SELF && i0 + kb + k == jj[tp];
          if (self) D = (T)1;
          T iv = adj_rsq(D);
          if (self) iv = (T)0;
          const T iv2 = iv * iv;
          const T inv3 = iv * iv2;
          const T er = ti.e0 * rx + ti.e1 * ry + ti.e2 * rz;
          const T rb0 = ry * ti.b2 - rz * ti.b1;
          const T rb1 = rz * ti.b0 - rx * ti.b2;
          const T rb2 = rx * ti.b1 - ry * ti.b0;
          const T cr = w0[tp] * er + (w1[tp] * rb0 + w2[tp] * rb1 + w3[tp] * rb2);
          const T f5 = inv3 * iv2 * cr;
          se[tp][0] += inv3 * ti.e0;
          se[tp][1] += inv3 * ti.e1;
          se[tp][2] += inv3 * ti.e2;
          sb[tp][0] += inv3 * ti.b0;
          sb[tp][1] += inv3 * ti.b1;
          sb[tp][2] += inv3 * ti.b2;
          ss[tp][0] += f5 * sx;
          ss[tp][1] += f5 * sy;
          ss[tp][2] += f5 * sz;
          if constexpr (GU) {
            const T fu = f5 * ur;
            au[tp][0] += fu * rx;
            au[tp][1] += fu * ry;
            au[tp][2] += fu * rz;
          }
          mg[tp] += inv3 * er;
          mu3[tp][0] += inv3 * rb0;
          mu3[tp][1] += inv3 * rb1;
          mu3[tp][2] += inv3 * rb2;
        }
      }
    };
    if (s == t) {
      body(std::true_type{}, sh.d, xj, yj, zj);
    } else if (far) {
      if constexpr (kHybrid) {
        float xf[TPL], yf[TPL], zf[TPL];
#pragma unroll
        for (int k = 0; k < TPL; ++k) {
          xf[k] = (float)xj[k];
          yf[k] = (float)yj[k];
          zf[k] = (float)zj[k];
        }
        body(std::false_type{}, sh.f, xf, yf, zf);
      }
    } else {
      body(std::false_type{}, sh.d, xj, yj, zj);
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      // sum over the tile of D^{-3/2} C - 3 D^{-5/2} (C.r) S r
      const T a0 = (w0[k] * se[k][0] + (sb[k][1] * w3[k] - sb[k][2] * w2[k])) -
                   (T)3 * ss[k][0];
      const T a1 = (w0[k] * se[k][1] + (sb[k][2] * w1[k] - sb[k][0] * w3[k])) -
                   (T)3 * ss[k][1];
      const T a2 = (w0[k] * se[k][2] + (sb[k][0] * w2[k] - sb[k][1] * w1[k])) -
                   (T)3 * ss[k][2];
      acc[k][0] += (double)a0;
      acc[k][1] += (double)a1;
      acc[k][2] += (double)a2;
      acc[k][3] += (double)mg[k];
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[k][4 + q] += (double)mu3[k][q];
      if constexpr (GU)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[k][7 + q] += (double)((T)3 * au[k][q]);
    }
  }
  if (wave > 0)
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) red[wave - 1][q][k * kWave + lane] = acc[k][q];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (jj[k] >= sc) continue;
      for (int wv = 0; wv < WAVES - 1; ++wv)
        for (int q = 0; q < NR; ++q) acc[k][q] += red[wv][q][k * kWave + lane];
      if (si.z > 0) {
        // a later part of the row: its own slice, added by k_adj_src_combine
        double *pp = parts + (size_t)(si.z - 1) * NR * n;
        for (int q = 0; q < NR; ++q) pp[(size_t)q * n + pj[k]] = acc[k][q];
        continue;
      }
      for (int q = 0; q < 3; ++q) gx[(size_t)q * n + pj[k]] -= acc[k][q];
      for (int q = 0; q < 4; ++q) mbar[(size_t)q * n + pj[k]] += acc[k][3 + q];
      if constexpr (GU)
        for (int q = 0; q < 3; ++q) gu[(size_t)q * n + pj[k]] = -acc[k][7 + q];
    }
  }
}

// The later row parts of a split P2P^T launch, added in part order after the
// first part's direct update: target side gx += parts, gG += parts.
__global__ void k_adj_tgt_combine(int n, int nsplit, int nr,
                                  const double *parts, double *gx,
                                  double *gG) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  for (int q = 0; q < nr; ++q) {
    double *o = q < 3 ? gx + (size_t)q * n + p : gG + p;
    double v = *o;
    for (int k = 1; k < nsplit; ++k)
      v += parts[((size_t)(k - 1) * nr + q) * n + p];
    *o = v;
  }
}

// Source side: gx -= parts (3), mbar += parts (4), gu -= parts (3, if nr 10).
__global__ void k_adj_src_combine(int n, int nsplit, int nr,
                                  const double *parts, double *gx,
                                  double *mbar, double *gu) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  for (int q = 0; q < nr; ++q) {
    double *o = q < 3   ? gx + (size_t)q * n + p
                : q < 7 ? mbar + (size_t)(q - 3) * n + p
                        : gu + (size_t)(q - 7) * n + p;
    const bool add = q >= 3 && q < 7;
    double v = *o;
    for (int k = 1; k < nsplit; ++k) {
      const double a = parts[((size_t)(k - 1) * nr + q) * n + p];
      v = add ? v + a : v - a;
    }
    *o = v;
  }
}

// Scatter to the caller's order: grad_x, and grad_q = gamma mbar0 + u . mbar.
// (Lists that overflowed their capacity dropped interactions: the gradients
// are NaN rather than silently wrong.)
__global__ void k_adj_final(int n, const uint32_t *ord, const double *us,
                            const double *gx, const double *mbar,
                            const int *ovf, double *grad_x, double *grad_q) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const size_t i = ord[p];
  const double u0 = us[p], u1 = us[(size_t)n + p], u2 = us[2 * (size_t)n + p];
  const double gam = sqrt(1.0 + (u0 * u0 + u1 * u1 + u2 * u2));
  const bool bad = *ovf != 0;
  for (int c = 0; c < 3; ++c)
    grad_x[3 * i + c] = bad ? __builtin_nan("") : gx[(size_t)c * n + p];
  const double g = gam * mbar[p] + u0 * mbar[(size_t)n + p] +
                   u1 * mbar[2 * (size_t)n + p] + u2 * mbar[3 * (size_t)n + p];
  grad_q[i] = bad ? __builtin_nan("") : g;
}

// Momentum gradient in the caller's order:
//   grad_u = q (mbar0 u/gamma + mbar[1:]) + [gu] + [G dgbar/du],
// q = w0/gamma; gs = (G, dgbar/du (3)) from k_gsum_final or null.
__global__ void k_adj_final_u(int n, const uint32_t *ord, const double *us,
                              const double *w, const double *mbar,
                              const double *gu, const double *gs,
                              const int *ovf, double *grad_u) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  const size_t i = ord[p];
  const double u[3] = {us[p], us[(size_t)n + p], us[2 * (size_t)n + p]};
  const double gam = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  const double q = w[p] / gam, m0 = mbar[p];
  for (int c = 0; c < 3; ++c) {
    double v = q * (m0 * u[c] / gam + mbar[(size_t)(1 + c) * n + p]);
    if (gu) v += gu[(size_t)c * n + p];
    if (gs) v += gs[0] * gs[1 + c];
    grad_u[3 * i + c] = *ovf != 0 ? __builtin_nan("") : v;
  }
}

// dL/dgbar and dgbar/du, deterministic two-stage sums.  Stage 1: block b
// sums a fixed contiguous slice of the particles (near-field gbar
// derivatives gG when present, the momenta) and of the nodes (the far-field
// partials gdot, nblk per node with kind != 0), in a fixed order.
constexpr int kGsThreads = 256;
__device__ inline double block_sum(double v, double *sh) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < kGsThreads / kWave; ++k) s += sh[k];
  return s;
}

__global__ void __launch_bounds__(kGsThreads)
k_gsum_partial(int n, int ns, int nblk, const int32_t *kind, const double *gG,
               const double *gdot, const double *us, double *part) {
  __shared__ double sh[kGsThreads / kWave];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t p0 = (int64_t)n * b / kGsBlocks, p1 = (int64_t)n * (b + 1) / kGsBlocks;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t p = p0 + tid; p < p1; p += kGsThreads) {
    if (gG) v[0] += gG[p];
    for (int c = 0; c < 3; ++c) v[1 + c] += us[(size_t)c * n + p];
  }
  double vd = 0.0;
  if (gdot) {
    const int t0 = (int)((int64_t)ns * b / kGsBlocks),
              t1 = (int)((int64_t)ns * (b + 1) / kGsBlocks);
    for (int t = t0 + tid; t < t1; t += kGsThreads)
      if (kind[t] != 0)
        for (int k = 0; k < nblk; ++k) vd += gdot[(size_t)t * kGdotStride + k];
  }
  for (int c = 0; c < 4; ++c) {
    const double s = block_sum(v[c], sh);
    if (tid == 0) part[5 * b + c] = s;
  }
  const double s = block_sum(vd, sh);
  if (tid == 0) part[5 * b + 4] = s;
}

// Stage 2: G = -gbar sum gG - (3/gbar) sum gdot (the kernels' gbar),
// dgbar/du = pbar/(n gamma(pbar)) with pbar the mean momentum.
__global__ void __launch_bounds__(kGsThreads)
k_gsum_final(int n, const double *part, const double *gbar, double *gs) {
  __shared__ double sh[kGsThreads / kWave];
  const int tid = threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < kGsBlocks; b += kGsThreads)
    for (int c = 0; c < 5; ++c) v[c] += part[5 * b + c];
  double s[5];
  for (int c = 0; c < 5; ++c) s[c] = block_sum(v[c], sh);
  if (tid == 0) {
    const double gb = *gbar;
    const double pb[3] = {s[1] / n, s[2] / n, s[3] / n};
    const double gp = sqrt(1.0 + (pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2]));
    gs[0] = -gb * s[0] - (3.0 / gb) * s[4];
    for (int c = 0; c < 3; ++c) gs[1 + c] = pb[c] / ((double)n * gp);
  }
}

static int nblocks(int n) { return (n + kThreads - 1) / kThreads; }

void launch_adj_prep(const Dev &d, int n, const double *gE, const double *gB,
                     double ke, double kb, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_prep, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                     d.ord_all, gE, gB, ke, kb, d.ebar, d.ebar32);
}

void launch_m2l_adjoint(const Dev &d, const Cheb &cb, const M2LArgs &a,
                        hipStream_t st) {
  if (a.prec == 0)
    hipLaunchKernelGGL(k_m2l_adj<double>, dim3(order_len(a.ns)), dim3(kThreads), 0, st,
                       cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row_T, d.m2l_T,
                       d.order_m2l_T, d.Lbar, d.gbar, d.Mbar);
  else
    launch_m2l_adjoint_mfma(d, cb, a, st);
}

void launch_adj_leaf(const Dev &d, const Cheb &cb, int n, int ns, int max_leaf,
                     hipStream_t st) {
  dispatch_q<AdjLeafLaunch>(cb.p + 1, d, cb, n, ns, max_leaf, st);
}

// Rows of a small grid are split into parts (as for the forward P2P): the
// first part updates the gradients directly, the later parts write slices of
// the near-field buffer beyond its first 6 n entries (which keep the forward
// near field), and a combine kernel adds them in part order.
#ifndef RELFMM_ADJ_MINWAVES
#define RELFMM_ADJ_MINWAVES 32768
#endif
constexpr int kAdjSplitWaves = RELFMM_ADJ_MINWAVES;

static int adj_nsplit(const Dev &d, int n, int64_t waves, int nr) {
  const int64_t extra = (int64_t)((d.near_cap - 6 * (size_t)n) /
                                  ((size_t)nr * (size_t)n));
  int nsplit = 1;
  while (2 * nsplit <= kP2PMaxSplit && 2 * nsplit - 1 <= extra &&
         waves * nsplit < kAdjSplitWaves)
    nsplit *= 2;
  return nsplit;
}

template <typename T, int MODE, int TPL, int WAVES, int UNR>
static void adj_tgt_kernel(const Dev &d, const P2PArgs &a, int n, const T *w,
                           const T *us, const T *eb, bool tgb, dim3 grid,
                           int ny, int nsplit, double *parts, hipStream_t st) {
  const dim3 block(WAVES * kWave);
  if (tgb)
    hipLaunchKernelGGL((k_p2p_adj_tgt<T, MODE, MODE == 0, TPL, WAVES, UNR>),
                       grid, block, 0, st, n, a.bits, d.kind, d.lo, d.hi,
                       d.cen, d.hw, d.p2p_row, d.p2p, d.order_p2p, d.xl, w, us,
                       eb, d.gbar, d.gx, d.gG, ny, nsplit, parts);
  else
    hipLaunchKernelGGL((k_p2p_adj_tgt<T, MODE, false, TPL, WAVES, UNR>), grid,
                       block, 0, st, n, a.bits, d.kind, d.lo, d.hi, d.cen,
                       d.hw, d.p2p_row, d.p2p, d.order_p2p, d.xl, w, us, eb,
                       d.gbar, d.gx, nullptr, ny, nsplit, parts);
}

template <typename T, int MODE, int TPL, int WAVES, int UNR>
static void adj_src_kernel(const Dev &d, const P2PArgs &a, int n, const T *w,
                           const T *us, const T *eb, bool sgu, dim3 grid,
                           int ny, int nsplit, double *parts, hipStream_t st) {
  const dim3 block(WAVES * kWave);
  if (sgu)
    hipLaunchKernelGGL((k_p2p_adj_src<T, MODE, MODE == 1, TPL, WAVES, UNR>),
                       grid, block, 0, st, n, a.bits, d.kind, d.lo, d.hi,
                       d.cen, d.hw, d.p2p_row_T, d.p2p_T, d.order_p2p_T, d.xl,
                       w, us, eb, d.gbar, d.gx, d.mbar, d.gu, ny, nsplit, parts);
  else
    hipLaunchKernelGGL((k_p2p_adj_src<T, MODE, false, TPL, WAVES, UNR>), grid,
                       block, 0, st, n, a.bits, d.kind, d.lo, d.hi, d.cen,
                       d.hw, d.p2p_row_T, d.p2p_T, d.order_p2p_T, d.xl, w, us,
                       eb, d.gbar, d.gx, d.mbar, nullptr, ny, nsplit, parts);
}

// gb: the mean-kernel target side also forms the near-field gbar
// derivative; gu: the per-source side also forms the denominator term.
template <typename T, int MODE, int TPL, int WAVES>
static void launch_p2p_adj_t(const Dev &d, const P2PArgs &a, int n, const T *w,
                             const T *us, const T *eb, bool gb, bool gu,
                             hipStream_t st) {
  constexpr int U = kAdjUnroll[TPL];
  const int chunks = (a.max_leaf + kWave * TPL - 1) / (kWave * TPL);
  const int64_t waves = (int64_t)std::max(a.ns / 2, 1) * chunks * WAVES;
  double *parts = d.near + 6 * (size_t)n;
  const bool tgb = MODE == 0 && gb, sgu = MODE == 1 && gu;
  const int nrt = tgb ? 4 : 3, nrs = sgu ? 10 : 7;
  const int st_split = adj_nsplit(d, n, waves, nrt);
  const dim3 gt(order_len(a.ns) * chunks * st_split);
  if constexpr (TPL == 2) {
    if (st_split > 1)
      adj_tgt_kernel<T, MODE, TPL, WAVES, 1>(d, a, n, w, us, eb, tgb, gt,
                                             chunks, st_split, parts, st);
    else
      adj_tgt_kernel<T, MODE, TPL, WAVES, U>(d, a, n, w, us, eb, tgb, gt,
                                             chunks, st_split, parts, st);
  } else {
    adj_tgt_kernel<T, MODE, TPL, WAVES, U>(d, a, n, w, us, eb, tgb, gt,
                                           chunks, st_split, parts, st);
  }
  if (st_split > 1)
    hipLaunchKernelGGL(k_adj_tgt_combine, dim3(nblocks(n)), dim3(kThreads), 0,
                       st, n, st_split, nrt, parts, d.gx, d.gG);
  const int ss_split = adj_nsplit(d, n, waves, nrs);
  const dim3 gs(order_len(a.ns) * chunks * ss_split);
  if constexpr (TPL == 2) {
    if (ss_split > 1)
      adj_src_kernel<T, MODE, TPL, WAVES, 1>(d, a, n, w, us, eb, sgu, gs,
                                             chunks, ss_split, parts, st);
    else
      adj_src_kernel<T, MODE, TPL, WAVES, U>(d, a, n, w, us, eb, sgu, gs,
                                             chunks, ss_split, parts, st);
  } else {
    adj_src_kernel<T, MODE, TPL, WAVES, U>(d, a, n, w, us, eb, sgu, gs,
                                           chunks, ss_split, parts, st);
  }
  if (ss_split > 1)
    hipLaunchKernelGGL(k_adj_src_combine, dim3(nblocks(n)), dim3(kThreads), 0,
                       st, n, ss_split, nrs, parts, d.gx, d.mbar, d.gu);
}

// Workgroup size by leaf size (tiles of 64 partners per wave).
template <typename T, int MODE, int TPL>
static void launch_p2p_adj_w(const Dev &d, const P2PArgs &a, int n, const T *w,
                             const T *us, const T *eb, bool gb, bool gu,
                             hipStream_t st) {
  if (a.max_leaf <= kWave)
    launch_p2p_adj_t<T, MODE, TPL, 1>(d, a, n, w, us, eb, gb, gu, st);
  else if (a.max_leaf <= 2 * kWave)
    launch_p2p_adj_t<T, MODE, TPL, 2>(d, a, n, w, us, eb, gb, gu, st);
  else
    launch_p2p_adj_t<T, MODE, TPL, 4>(d, a, n, w, us, eb, gb, gu, st);
}

// Waves wanted in flight before two particles per lane pay off.
constexpr int kAdjMinWaves = 8192;

void launch_p2p_adjoint(const Dev &d, const P2PArgs &a, int n, bool gb,
                        bool gu, hipStream_t st) {
  // the FP32 kernels take two particles per lane (half the LDS broadcast
  // bytes per pair) for leaves larger than one wave when the grid stays large
  const int waves = a.max_leaf <= kWave ? 1 : a.max_leaf <= 2 * kWave ? 2 : 4;
  const int64_t waves2 = (int64_t)std::max(a.ns / 2, 1) *
                         ((a.max_leaf + 2 * kWave - 1) / (2 * kWave)) * waves;
  const bool two = a.max_leaf > kWave && waves2 >= kAdjMinWaves;
  if (a.prec == 0) {
    if (a.mode == 0)
      launch_p2p_adj_w<double, 0, 1>(d, a, n, d.w, d.us, d.ebar, gb, gu, st);
    else
      launch_p2p_adj_w<double, 1, 1>(d, a, n, d.w, d.us, d.ebar, gb, gu, st);
  } else if (two) {
    if (a.mode == 0)
      launch_p2p_adj_w<float, 0, 2>(d, a, n, d.w32, d.us32, d.ebar32, gb, gu, st);
    else
      launch_p2p_adj_w<float, 1, 2>(d, a, n, d.w32, d.us32, d.ebar32, gb, gu, st);
  } else {
    if (a.mode == 0)
      launch_p2p_adj_w<float, 0, 1>(d, a, n, d.w32, d.us32, d.ebar32, gb, gu, st);
    else
      launch_p2p_adj_w<float, 1, 1>(d, a, n, d.w32, d.us32, d.ebar32, gb, gu, st);
  }
}

void launch_gbar_sums(const Dev &d, int n, int ns, int nblk, bool near,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_gsum_partial, dim3(kGsBlocks), dim3(kGsThreads), 0, st,
                     n, ns, nblk, d.kind, near ? d.gG : nullptr, d.gdot, d.us,
                     d.gspart);
  hipLaunchKernelGGL(k_gsum_final, dim3(1), dim3(kGsThreads), 0, st, n,
                     d.gspart, d.gbar, d.gsum);
}

void launch_adj_final(const Dev &d, int n, double *grad_x, double *grad_q,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_adj_final, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                     d.ord_all, d.us, d.gx, d.mbar, d.counters + kCntOverflow,
                     grad_x, grad_q);
}

void launch_adj_final_u(const Dev &d, int n, bool gu, bool gs, double *grad_u,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_adj_final_u, dim3(nblocks(n)), dim3(kThreads), 0, st, n,
                     d.ord_all, d.us, d.w, d.mbar, gu ? d.gu : nullptr,
                     gs ? d.gsum : nullptr, d.counters + kCntOverflow, grad_u);
}

}  // namespace relfmm
