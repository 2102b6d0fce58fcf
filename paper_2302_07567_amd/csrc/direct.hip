// FP64 direct sum of eq. (fmm_pp_force_field) over all sources j != i at a
// set of target particles (the brute force of Sec. 6), for accuracy
// measurement of the FMM against its own definition.  One thread per target;
// sources are staged through LDS in tiles.
#include "internal.hpp"

namespace relfmm {

constexpr int kDirThreads = 256;

template <int MODE>
__global__ void __launch_bounds__(kDirThreads)
k_direct(int n, const double *x, const double *u, const double *q, int nt,
         const int64_t *tgt, double gb, double ke, double kb, double *E,
         double *B) {
  __shared__ double sx[kDirThreads][3], su[kDirThreads][3], sw[kDirThreads][4];
  const int a = blockIdx.x * kDirThreads + threadIdx.x;
  const bool act = a < nt;
  const int64_t i = act ? (tgt ? tgt[a] : a) : 0;
  const double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
  const double g2 = gb * gb;
  double e[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < n; j0 += kDirThreads) {
    __syncthreads();
    const int j = j0 + threadIdx.x;
    if (j < n) {
      double uu[3];
      for (int c = 0; c < 3; ++c) {
        sx[threadIdx.x][c] = x[3 * (size_t)j + c];
        uu[c] = u[3 * (size_t)j + c];
        su[threadIdx.x][c] = uu[c];
      }
      const double gam =
          sqrt(1.0 + (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]));
      sw[threadIdx.x][0] = q[j] * gam;
      for (int c = 0; c < 3; ++c) sw[threadIdx.x][1 + c] = q[j] * uu[c];
    }
    __syncthreads();
    const int nj = min(kDirThreads, n - j0);
    for (int k = 0; k < nj; ++k) {
      if (j0 + k == i) continue;
      const double rx = xi[0] - sx[k][0], ry = xi[1] - sx[k][1],
                   rz = xi[2] - sx[k][2];
      double D;
      if (MODE == 0) {
        D = rx * rx + ry * ry + g2 * (rz * rz);
      } else {
        const double ur = su[k][0] * rx + su[k][1] * ry + su[k][2] * rz;
        D = (rx * rx + ry * ry + rz * rz) + ur * ur;
      }
      const double inv = 1.0 / (D * sqrt(D));
      const double gx = rx * inv, gy = ry * inv, gz = rz * inv;
      e[0] += sw[k][0] * gx;
      e[1] += sw[k][0] * gy;
      e[2] += sw[k][0] * gz;
      b[0] += sw[k][2] * gz - sw[k][3] * gy;
      b[1] += sw[k][3] * gx - sw[k][1] * gz;
      b[2] += sw[k][1] * gy - sw[k][2] * gx;
    }
  }
  if (act)
    for (int c = 0; c < 3; ++c) {
      E[3 * (size_t)a + c] = ke * e[c];
      B[3 * (size_t)a + c] = kb * b[c];
    }
}

void launch_direct(int n, const double *x, const double *u, const double *q,
                   int nt, const int64_t *tgt, int kernel, double gb,
                   double ke, double kb, double *E, double *B,
                   hipStream_t st) {
  const dim3 grid((nt + kDirThreads - 1) / kDirThreads), block(kDirThreads);
  if (kernel == 0)
    hipLaunchKernelGGL(k_direct<0>, grid, block, 0, st, n, x, u, q, nt, tgt,
                       gb, ke, kb, E, B);
  else
    hipLaunchKernelGGL(k_direct<1>, grid, block, 0, st, n, x, u, q, nt, tgt,
                       gb, ke, kb, E, B);
}

}  // namespace relfmm
