// P2P near field (Alg. P2P) over the target-grouped P2P list (Sec. 10).
//
// Target-grouped: the targets of one leaf are handled by workgroups that loop
// over that leaf's P2P sources (no atomics).  Particles are stored in leaf
// order, so each source leaf is a contiguous range that is
// staged through LDS with coalesced loads (the gather of the paper's
// index-array layout disappears).  Coordinates are relative to the target
// leaf centre, kept in FP64 (the source leaf's local coordinates plus the
// offset of the two centres); each pair offset r = x_i - x_j is formed in FP64
// and rounded once to the kernel precision T, so the FP32 path loses no
// accuracy to the size of the leaf.  The rest of the pair arithmetic runs in
// T; each wave's partial sums over its 64 sources of a tile are flushed into
// FP64 accumulators.
//
// Kernels (r = x_i - x_j):
//   MEAN   (eq. fmm_relativistic_kernel) D = rx^2 + ry^2 + gbar^2 rz^2
//   SOURCE (per-source momentum)          D = |r|^2 + (u_j . r)^2
//   E_i += (q gamma)_j r D^{-3/2},  B_i += ((q u)_j x r) D^{-3/2},  j != i.
#include "internal.hpp"

namespace relfmm {

constexpr int kP2PThreads = 256;

__device__ inline float inv_d32(float D) {
  const float r = __builtin_amdgcn_rsqf(D);
  return r * r * r;
}
__device__ inline double inv_d32(double D) { return 1.0 / (D * sqrt(D)); }

// A staged source: position in the target leaf's frame (FP64) and the
// weights (q gamma, q u) and momentum u in the kernel precision.
template <typename T, int MODE>
struct Src {
  double x, y, z;
  T w0, w1, w2, w3;
};
template <typename T>
struct Src<T, 1> {
  double x, y, z;
  T w0, w1, w2, w3;
  T u0, u1, u2;
};

// Pair field of one staged source on TPL targets of this lane.
template <typename T, int MODE, int TPL, bool SELF>
__device__ inline void p2p_pair(const Src<T, MODE> &sj, const double (&xi)[TPL],
                                const double (&yi)[TPL],
                                const double (&zi)[TPL], T g2,
                                const int (&tidx)[TPL], int jidx, T (&e)[TPL][3],
                                T (&b)[TPL][3]) {
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const T rx = (T)(xi[k] - sj.x), ry = (T)(yi[k] - sj.y),
            rz = (T)(zi[k] - sj.z);
    T D;
    if constexpr (MODE == 0) {
      D = rx * rx + ry * ry + g2 * (rz * rz);
    } else {
      const T ur = sj.u0 * rx + sj.u1 * ry + sj.u2 * rz;
      D = rx * rx + ry * ry + rz * rz + ur * ur;
    }
    if (SELF && tidx[k] == jidx) D = (T)1;
    T inv3 = inv_d32(D);
    if (SELF && tidx[k] == jidx) inv3 = (T)0;
    const T sg = sj.w0 * inv3;
    e[k][0] += sg * rx;
    e[k][1] += sg * ry;
    e[k][2] += sg * rz;
    b[k][0] += inv3 * (sj.w2 * rz - sj.w3 * ry);
    b[k][1] += inv3 * (sj.w3 * rx - sj.w1 * rz);
    b[k][2] += inv3 * (sj.w1 * ry - sj.w2 * rx);
  }
}

// One workgroup = 4 waves per chunk of 64*TPL targets of one leaf (TPL per
// lane).  Source leaves are staged in tiles of 256 (padded with zero-weight
// sources far away, so every wave runs a fixed, fully unrolled loop); each
// wave takes a quarter of every tile for the same targets, flushes its FP32
// partial sums into FP64 after each tile, and the four partial results are
// added in a fixed order at the end.  No atomics; the result is
// deterministic.
constexpr int kP2PWaves = kP2PThreads / kWave;
constexpr int kP2PTile = kP2PThreads;
constexpr int kP2PPerWave = kP2PTile / kP2PWaves;

template <typename T, int MODE, int TPL>
__global__ void __launch_bounds__(kP2PThreads)
k_p2p(int n, int bits, const int32_t *kind, const int32_t *lo,
      const int32_t *hi, const double *cen, const int32_t *row,
      const uint64_t *keys, const double *xl, const T *w, const T *us,
      const double *gbar, double *near) {
  __shared__ Src<T, MODE> sh[kP2PTile];
  __shared__ double red[kP2PWaves - 1][6][TPL * kWave];
  const int t = blockIdx.x;
  if (kind[t] != 1) return;
  const int tl = lo[t], tc = hi[t] - tl;
  const int i0 = blockIdx.y * kWave * TPL;
  if (i0 >= tc) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  const int r0 = row[t], r1 = row[t + 1];
  double xi[TPL], yi[TPL], zi[TPL];
  int tidx[TPL];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int ii = i0 + k * kWave + lane;
    tidx[k] = ii;
    const int pi = tl + (ii < tc ? ii : 0);
    xi[k] = xl[pi];
    yi[k] = xl[(size_t)n + pi];
    zi[k] = xl[2 * (size_t)n + pi];
  }
  double acc[TPL][6];
#pragma unroll
  for (int k = 0; k < TPL; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[k][c] = 0.0;
  for (int r = r0; r < r1; ++r) {
    const int s = (int)(keys[r] & mask);
    const int sl = lo[s], sc = hi[s] - sl;
    const double dx = cen[3 * s] - ct[0];
    const double dy = cen[3 * s + 1] - ct[1];
    const double dz = cen[3 * s + 2] - ct[2];
    for (int j0 = 0; j0 < sc; j0 += kP2PTile) {
      __syncthreads();
      {
        Src<T, MODE> v;
        if (j0 + tid < sc) {
          const size_t p = (size_t)sl + j0 + tid;
          v.x = xl[p] + dx;
          v.y = xl[n + p] + dy;
          v.z = xl[2 * (size_t)n + p] + dz;
          v.w0 = w[p];
          v.w1 = w[n + p];
          v.w2 = w[2 * (size_t)n + p];
          v.w3 = w[3 * (size_t)n + p];
          if constexpr (MODE == 1) {
            v.u0 = us[p];
            v.u1 = us[n + p];
            v.u2 = us[2 * (size_t)n + p];
          }
        } else {
          // padding: zero weight, far away (finite pair terms, no effect)
          v.x = v.y = v.z = 1.0e12;
          v.w0 = v.w1 = v.w2 = v.w3 = (T)0;
          if constexpr (MODE == 1) v.u0 = v.u1 = v.u2 = (T)0;
        }
        sh[tid] = v;
      }
      __syncthreads();
      const int kb = wave * kP2PPerWave;
      if (j0 + kb >= sc) continue;  // wave-uniform: this quarter is padding
      T e[TPL][3], b[TPL][3];
#pragma unroll
      for (int k = 0; k < TPL; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[k][c] = b[k][c] = (T)0;
      if (s == t) {
#pragma unroll 8
        for (int k = 0; k < kP2PPerWave; ++k)
          p2p_pair<T, MODE, TPL, true>(sh[kb + k], xi, yi, zi, g2, tidx,
                                       j0 + kb + k, e, b);
      } else {
#pragma unroll 8
        for (int k = 0; k < kP2PPerWave; ++k)
          p2p_pair<T, MODE, TPL, false>(sh[kb + k], xi, yi, zi, g2, tidx,
                                        -1, e, b);
      }
#pragma unroll
      for (int k = 0; k < TPL; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[k][c] += (double)e[k][c];
          acc[k][3 + c] += (double)b[k][c];
        }
    }
  }
  if (wave > 0)
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int c = 0; c < 6; ++c) red[wave - 1][c][k * kWave + lane] = acc[k][c];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const int ii = i0 + k * kWave + lane;
      if (ii >= tc) continue;
      for (int wv = 0; wv < kP2PWaves - 1; ++wv)
        for (int c = 0; c < 6; ++c) acc[k][c] += red[wv][c][k * kWave + lane];
      for (int c = 0; c < 6; ++c) near[(size_t)c * n + tl + ii] = acc[k][c];
    }
  }
}

template <typename T, int MODE, int TPL>
static void launch_p2p_t(const Dev &d, const P2PArgs &a, int n, const T *w,
                         const T *us, hipStream_t st) {
  const int per_wg = kWave * TPL;
  const dim3 grid(a.ns, (a.max_leaf + per_wg - 1) / per_wg), block(kP2PThreads);
  hipLaunchKernelGGL((k_p2p<T, MODE, TPL>), grid, block, 0, st, n, a.bits,
                     d.kind, d.lo, d.hi, d.cen, d.p2p_row, d.p2p, d.xl, w, us,
                     d.gbar, d.near);
}

void launch_p2p(const Dev &d, const P2PArgs &a, int n, hipStream_t st) {
  if (a.prec == 0) {
    if (a.mode == 0)
      launch_p2p_t<double, 0, 1>(d, a, n, d.w, d.us, st);
    else
      launch_p2p_t<double, 1, 1>(d, a, n, d.w, d.us, st);
  } else {
    if (a.mode == 0)
      launch_p2p_t<float, 0, 1>(d, a, n, d.w32, d.us32, st);
    else
      launch_p2p_t<float, 1, 1>(d, a, n, d.w32, d.us32, st);
  }
}

}  // namespace relfmm
