// M2L (Alg. M2L, effective fields of Sec. 3) over the target-grouped M2L list
// (Sec. 10), always with the mean kernel of eq. (fmm_relativistic_kernel):
//   E_{t,mu} += sum_nu M^gamma_{s,nu} g(xi_{t,mu} - xi_{s,nu})
//   B_{t,mu} += sum_nu M^u_{s,nu} x g(xi_{t,mu} - xi_{s,nu}).
//
// One workgroup per target node, one thread per target proxy.  Proxies are
// tensor products of three (p+1)-point axes, so the pair offsets
// xi_{t,mu} - xi_{s,nu} take only 3 (p+1)^2 distinct per-axis values per pair;
// they are formed in FP64 and rounded once to the kernel precision T.  The
// per-source partial sums run in T and are flushed into FP64 after each
// source.
#include "internal.hpp"

namespace relfmm {

constexpr int kM2LThreads = 256;
constexpr int kQ = kMaxDegree + 1;
constexpr int kMaxM = kQ * kQ * kQ;

__device__ inline float m2l_inv(float D) {
  const float r = __builtin_amdgcn_rsqf(D);
  return r * r * r;
}
__device__ inline double m2l_inv(double D) { return 1.0 / (D * sqrt(D)); }

template <typename T>
__global__ void __launch_bounds__(kM2LThreads)
k_m2l_valu(Cheb cb, int bits, const int32_t *kind, const double *cen,
           const double *hw, const int32_t *row, const uint64_t *keys,
           const double *M, const double *gbar, double *L) {
  // dX[g][a][a2] = xi^g_{t,a} - xi^g_{s,a2}, formed in FP64, rounded once
  __shared__ T dX[3][kQ][kQ];
  __shared__ T sM[kMaxM][4];
  const int t = blockIdx.x;
  if (kind[t] == 0) return;
  const int tid = threadIdx.x;
  const int q = cb.p + 1, m = q * q * q;
  const double gbd = *gbar;
  const T g2 = (T)(gbd * gbd);
  const uint64_t mask = (1ull << bits) - 1ull;
  const int r0 = row[t], r1 = row[t + 1];
  for (int mu0 = 0; mu0 < m; mu0 += kM2LThreads) {
    const int mu = mu0 + tid;
    const bool act = mu < m;
    const int a = act ? mu / (q * q) : 0, b = act ? (mu / q) % q : 0,
              c = act ? mu % q : 0;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = r0; r < r1; ++r) {
      const int s = (int)(keys[r] & mask);
      __syncthreads();
      for (int i = tid; i < 3 * q * q; i += kM2LThreads) {
        const int g = i / (q * q), a1 = (i / q) % q, a2 = i % q;
        dX[g][a1][a2] = (T)((cen[3 * t + g] - cen[3 * s + g]) +
                            (hw[3 * t + g] * cb.t[a1] - hw[3 * s + g] * cb.t[a2]));
      }
      for (int i = tid; i < m; i += kM2LThreads)
        for (int k = 0; k < 4; ++k) sM[i][k] = (T)M[((size_t)s * m + i) * 4 + k];
      __syncthreads();
      if (act) {
        T e[3] = {(T)0, (T)0, (T)0}, bb[3] = {(T)0, (T)0, (T)0};
        int nu = 0;
        for (int a2 = 0; a2 < q; ++a2) {
          const T rx = dX[0][a][a2];
          for (int b2 = 0; b2 < q; ++b2) {
            const T ry = dX[1][b][b2];
            const T dxy = rx * rx + ry * ry;
            for (int c2 = 0; c2 < q; ++c2, ++nu) {
              const T rz = dX[2][c][c2];
              const T inv3 = m2l_inv(dxy + g2 * (rz * rz));
              const T sg = sM[nu][0] * inv3;
              e[0] += sg * rx;
              e[1] += sg * ry;
              e[2] += sg * rz;
              bb[0] += inv3 * (sM[nu][2] * rz - sM[nu][3] * ry);
              bb[1] += inv3 * (sM[nu][3] * rx - sM[nu][1] * rz);
              bb[2] += inv3 * (sM[nu][1] * ry - sM[nu][2] * rx);
            }
          }
        }
        for (int k = 0; k < 3; ++k) {
          acc[k] += (double)e[k];
          acc[3 + k] += (double)bb[k];
        }
      }
    }
    if (act)
      for (int k = 0; k < 6; ++k) L[((size_t)t * m + mu) * 6 + k] = acc[k];
  }
}

void launch_m2l(const Dev &d, const Cheb &cb, const M2LArgs &a,
                hipStream_t st) {
  const dim3 grid(a.ns), block(kM2LThreads);
  if (a.prec == 0)
    hipLaunchKernelGGL(k_m2l_valu<double>, grid, block, 0, st, cb, a.bits,
                       d.kind, d.cen, d.hw, d.m2l_row, d.m2l, d.M, d.gbar,
                       d.L);
  else
    hipLaunchKernelGGL(k_m2l_valu<float>, grid, block, 0, st, cb, a.bits,
                       d.kind, d.cen, d.hw, d.m2l_row, d.m2l, d.M, d.gbar,
                       d.L);
}

}  // namespace relfmm
