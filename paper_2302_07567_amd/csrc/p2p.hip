// P2P near field (Alg. P2P) over the target-grouped P2P list (Sec. 10).
//
// One workgroup per target leaf, one thread per target particle.  Particles
// are stored in leaf order, so each source leaf is a contiguous range that is
// staged through LDS with coalesced loads (the gather of the paper's
// index-array layout disappears).  Coordinates are relative to the target
// leaf centre, kept in FP64 (the source leaf's local coordinates plus the
// offset of the two centres); each pair offset r = x_i - x_j is formed in FP64
// and rounded once to the kernel precision T, so the FP32 path loses no
// accuracy to the size of the leaf.  The rest of the pair arithmetic runs in
// T, and partial sums are flushed into FP64 accumulators every kFlush
// sources.
//
// Kernels (r = x_i - x_j):
//   MEAN   (eq. fmm_relativistic_kernel) D = rx^2 + ry^2 + gbar^2 rz^2
//   SOURCE (per-source momentum)          D = |r|^2 + (u_j . r)^2
//   E_i += (q gamma)_j r D^{-3/2},  B_i += ((q u)_j x r) D^{-3/2},  j != i.
#include "internal.hpp"

namespace relfmm {

constexpr int kP2PThreads = 256;
constexpr int kFlush = 64;

__device__ inline float inv_d32(float D) {
  const float r = __builtin_amdgcn_rsqf(D);
  return r * r * r;
}
__device__ inline double inv_d32(double D) { return 1.0 / (D * sqrt(D)); }

template <typename T>
struct SrcTile {
  double x[kP2PThreads], y[kP2PThreads], z[kP2PThreads];
  T w0[kP2PThreads], w1[kP2PThreads], w2[kP2PThreads], w3[kP2PThreads];
  T u0[kP2PThreads], u1[kP2PThreads], u2[kP2PThreads];
};

template <typename T, int MODE, bool SELF>
__device__ inline void p2p_tile(const SrcTile<T> &s, int k0, int k1, int skip,
                                double xi, double yi, double zi, T g2, T *e,
                                T *b) {
  for (int k = k0; k < k1; ++k) {
    const T rx = (T)(xi - s.x[k]), ry = (T)(yi - s.y[k]), rz = (T)(zi - s.z[k]);
    T D;
    if (MODE == 0) {
      D = rx * rx + ry * ry + g2 * (rz * rz);
    } else {
      const T ur = s.u0[k] * rx + s.u1[k] * ry + s.u2[k] * rz;
      D = rx * rx + ry * ry + rz * rz + ur * ur;
    }
    T w0 = s.w0[k];
    if (SELF && k == skip) {
      D = (T)1;
      w0 = (T)0;
    }
    T inv3 = inv_d32(D);
    if (SELF && k == skip) inv3 = (T)0;
    const T sg = w0 * inv3;
    e[0] += sg * rx;
    e[1] += sg * ry;
    e[2] += sg * rz;
    const T cx = s.w2[k] * rz - s.w3[k] * ry;
    const T cy = s.w3[k] * rx - s.w1[k] * rz;
    const T cz = s.w1[k] * ry - s.w2[k] * rx;
    b[0] += inv3 * cx;
    b[1] += inv3 * cy;
    b[2] += inv3 * cz;
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kP2PThreads)
k_p2p(int n, int bits, const int32_t *kind, const int32_t *lo,
      const int32_t *hi, const double *cen, const int32_t *row,
      const uint64_t *keys, const double *xl, const T *w, const T *us,
      const double *gbar, double *near) {
  __shared__ SrcTile<T> sh;
  const int t = blockIdx.x;
  if (kind[t] != 1) return;
  const int tid = threadIdx.x;
  const int tl = lo[t], tc = hi[t] - tl;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  const int r0 = row[t], r1 = row[t + 1];
  for (int i0 = 0; i0 < tc; i0 += kP2PThreads) {
    const int ii = i0 + tid;
    const bool act = ii < tc;
    const int pi = tl + (act ? ii : 0);
    const double xi = xl[pi], yi = xl[(size_t)n + pi],
                 zi = xl[2 * (size_t)n + pi];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = r0; r < r1; ++r) {
      const int s = (int)(keys[r] & mask);
      const int sl = lo[s], sc = hi[s] - sl;
      const double dx = cen[3 * s] - ct[0];
      const double dy = cen[3 * s + 1] - ct[1];
      const double dz = cen[3 * s + 2] - ct[2];
      for (int j0 = 0; j0 < sc; j0 += kP2PThreads) {
        __syncthreads();
        if (j0 + tid < sc) {
          const size_t p = (size_t)sl + j0 + tid;
          sh.x[tid] = xl[p] + dx;
          sh.y[tid] = xl[n + p] + dy;
          sh.z[tid] = xl[2 * (size_t)n + p] + dz;
          sh.w0[tid] = w[p];
          sh.w1[tid] = w[n + p];
          sh.w2[tid] = w[2 * (size_t)n + p];
          sh.w3[tid] = w[3 * (size_t)n + p];
          if (MODE == 1) {
            sh.u0[tid] = us[p];
            sh.u1[tid] = us[n + p];
            sh.u2[tid] = us[2 * (size_t)n + p];
          }
        }
        __syncthreads();
        const int nj = min(kP2PThreads, sc - j0);
        for (int k0 = 0; k0 < nj; k0 += kFlush) {
          const int k1 = min(nj, k0 + kFlush);
          T e[3] = {(T)0, (T)0, (T)0}, b[3] = {(T)0, (T)0, (T)0};
          if (s == t)
            p2p_tile<T, MODE, true>(sh, k0, k1, ii - j0, xi, yi, zi, g2, e, b);
          else
            p2p_tile<T, MODE, false>(sh, k0, k1, -1, xi, yi, zi, g2, e, b);
          for (int c = 0; c < 3; ++c) {
            acc[c] += (double)e[c];
            acc[3 + c] += (double)b[c];
          }
        }
      }
    }
    if (act)
      for (int c = 0; c < 6; ++c) near[(size_t)c * n + pi] = acc[c];
  }
}

void launch_p2p(const Dev &d, const P2PArgs &a, int n, hipStream_t st) {
  const dim3 grid(a.ns), block(kP2PThreads);
  if (a.prec == 0) {
    if (a.mode == 0)
      hipLaunchKernelGGL((k_p2p<double, 0>), grid, block, 0, st, n, a.bits,
                         d.kind, d.lo, d.hi, d.cen, d.p2p_row, d.p2p, d.xl,
                         d.w, d.us, d.gbar, d.near);
    else
      hipLaunchKernelGGL((k_p2p<double, 1>), grid, block, 0, st, n, a.bits,
                         d.kind, d.lo, d.hi, d.cen, d.p2p_row, d.p2p, d.xl,
                         d.w, d.us, d.gbar, d.near);
  } else {
    if (a.mode == 0)
      hipLaunchKernelGGL((k_p2p<float, 0>), grid, block, 0, st, n, a.bits,
                         d.kind, d.lo, d.hi, d.cen, d.p2p_row, d.p2p, d.xl,
                         d.w32, d.us32, d.gbar, d.near);
    else
      hipLaunchKernelGGL((k_p2p<float, 1>), grid, block, 0, st, n, a.bits,
                         d.kind, d.lo, d.hi, d.cen, d.p2p_row, d.p2p, d.xl,
                         d.w32, d.us32, d.gbar, d.near);
  }
}

}  // namespace relfmm
