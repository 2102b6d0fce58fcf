// Downward pass (Alg. downwardpass): L2L into the cumulative local fields
// (eq. L2L; the lemma of App. A) and L2P (Alg. L2P) at the leaves, then the
// near field is added, the prefactors of eq. (fmm_pp_force_field) applied and
// the result scattered to the caller's particle order.  FP64.
//
// Locals are [node][mu][6] = (E, B) before the prefactors.  L2L applies the
// transpose of the tensor-product transfer of M2M:
//   L_C[a'][b'][c'] += sum_{a,b,c} T_x[a][a'] T_y[b][b'] T_z[c][c'] L_S[a][b][c]
// with T_g[a][b] = l^g_{S,a}(xi^g_{C,b}).
#include "internal.hpp"

namespace relfmm {

constexpr int kQ = kMaxDegree + 1;
// threads per node of the M2M / L2L kernels (the upper levels have few
// nodes, so the passes of one node are spread over many threads)
#ifndef RELFMM_TRANS_THREADS
#define RELFMM_TRANS_THREADS 1024
#endif
constexpr int kTransThreads = RELFMM_TRANS_THREADS;
constexpr int kL2PThreads = 256;

// One workgroup per child C at one level, all NC components at once: the
// parent's block L_S[m][NC] is loaded into LDS with coalesced reads, the
// three mode products run on the [mu][k] layout in LDS, and the child's block
// is updated with coalesced read-modify-writes (one workgroup per (child,
// component) with strided accesses moved 4.4x the pass's bytes).
template <int Q, int NC>
__global__ void __launch_bounds__(kTransThreads)
k_l2l(Cheb cb, int level, const int32_t *kind, const double *cen,
      const double *hw, double *L) {
  constexpr int QQ = Q * Q, MM = QQ * Q, W = MM * NC;
  __shared__ double T[3][kQ][kQ];
  __shared__ double P[W], B1[W];
  const int C = (1 << level) + blockIdx.x;
  if (kind[C] == 0) return;
  const int S = C >> 1;
  const int tid = threadIdx.x;
  if (tid < 3 * Q) {
    const int g = tid / Q, bb = tid % Q;
    double l[kQ];
    const double xb = cen[3 * C + g] + hw[3 * C + g] * cb.t[bb];
    basis1d(cb, (xb - cen[3 * S + g]) / hw[3 * S + g], l);
    for (int a = 0; a < Q; ++a) T[g][a][bb] = l[a];
  }
  const double *in = L + (size_t)S * W;
  for (int i = tid; i < W; i += kTransThreads) P[i] = in[i];
  __syncthreads();
  // z: B1[a][b][c'] = sum_c T_z[c][c'] P[a][b][c]
  for (int i = tid; i < W; i += kTransThreads) {
    const int k = i % NC, mu = i / NC, ab = mu / Q, c2 = mu % Q;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < Q; ++c) s += T[2][c][c2] * P[(ab * Q + c) * NC + k];
    B1[i] = s;
  }
  __syncthreads();
  // y: P[a][b'][c'] = sum_b T_y[b][b'] B1[a][b][c']
  for (int i = tid; i < W; i += kTransThreads) {
    const int k = i % NC, mu = i / NC, a = mu / QQ, b2 = (mu / Q) % Q, c2 = mu % Q;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < Q; ++b) s += T[1][b][b2] * B1[(a * QQ + b * Q + c2) * NC + k];
    P[i] = s;
  }
  __syncthreads();
  // x: L_C[a'][b'][c'] += sum_a T_x[a][a'] P[a][b'][c']
  double *out = L + (size_t)C * W;
  for (int i = tid; i < W; i += kTransThreads) {
    const int k = i % NC, mu = i / NC, a2 = mu / QQ, bc = mu % QQ;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) s += T[0][a][a2] * P[(a * QQ + bc) * NC + k];
    out[i] += s;
  }
}

template <int NC>
struct L2LLaunch {
  template <int Q>
  struct F {
    static void run(const Cheb &cb, int level, const int32_t *kind,
                    const double *cen, const double *hw, double *L,
                    hipStream_t st) {
      hipLaunchKernelGGL((k_l2l<Q, NC>), dim3(1 << level), dim3(kTransThreads), 0, st,
                         cb, level, kind, cen, hw, L);
    }
  };
};

void launch_l2l_level(const Dev &d, const Cheb &cb, int level,
                      hipStream_t st) {
  dispatch_q<L2LLaunch<6>::F>(cb.p + 1, cb, level, d.kind, d.cen, d.hw, d.L,
                              st);
}

// The transpose of M2M has the form of L2L (parent into the children), here
// on the four components of the multipole cotangents.
void launch_m2m_transpose_level(const Dev &d, const Cheb &cb, int level,
                                hipStream_t st) {
  dispatch_q<L2LLaunch<4>::F>(cb.p + 1, cb, level, d.kind, d.cen, d.hw,
                              d.Mbar, st);
}

// L2P for a chunk of 256 particles of one leaf (one thread each, the bases in
// registers; the leaf's six local components are the same for every lane and
// are read from memory at wave-uniform addresses, so they arrive through the
// scalar cache into scalar registers instead of as LDS broadcasts, which at
// 8 bytes per lane and value held the kernel to the LDS bandwidth), plus the
// near field and the prefactors, written to the caller's order.
template <int Q>
__global__ void __launch_bounds__(kL2PThreads)
k_l2p_fin(Cheb cb, int n, const int32_t *kind, const int32_t *lo,
          const int32_t *hi, const double *hw, const double *xl,
          const double *L, const double *near, const uint32_t *ord, double ke,
          double kb, const int *ovf, double *E, double *B) {
  constexpr int MM = Q * Q * Q;
  const int v = blockIdx.x;
  if (kind[v] != 1) return;
  const int l0 = lo[v], cnt = hi[v] - l0;
  const int i0 = blockIdx.y * kL2PThreads;
  if (i0 >= cnt) return;
  const int tid = threadIdx.x;
  const int ii = i0 + tid;
  const bool act = ii < cnt;
  const int p = l0 + (act ? ii : 0);
  const double *__restrict__ Lv = L + (size_t)v * MM * 6;
  double lx[Q], ly[Q], lz[Q];
  basis1d_q<Q>(cb, xl[p] / hw[3 * v], lx);
  basis1d_q<Q>(cb, xl[(size_t)n + p] / hw[3 * v + 1], ly);
  basis1d_q<Q>(cb, xl[2 * (size_t)n + p] / hw[3 * v + 2], lz);
  double far[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int a = 0; a < Q; ++a) {
#pragma unroll 1
    for (int b = 0; b < Q; ++b) {
      const double lab = lx[a] * ly[b];
      const double *row = Lv + (a * Q + b) * Q * 6;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const double l = lab * lz[c];
#pragma unroll
        for (int k = 0; k < 6; ++k) far[k] += l * row[c * 6 + k];
      }
    }
  }
  if (act) {
    const size_t i = ord[p];
    // lists that overflowed their capacity dropped interactions: the fields
    // are NaN rather than silently wrong
    const bool bad = *ovf != 0;
    for (int k = 0; k < 3; ++k) {
      const double e = ke * (far[k] + near[(size_t)k * n + p]);
      const double b = kb * (far[3 + k] + near[(size_t)(3 + k) * n + p]);
      E[3 * i + k] = bad ? __builtin_nan("") : e;
      B[3 * i + k] = bad ? __builtin_nan("") : b;
    }
  }
}

template <int Q>
struct L2PLaunch {
  static void run(const Dev &d, const Cheb &cb, int n, int ns, int max_leaf,
                  double ke, double kb, double *E, double *B, hipStream_t st) {
    const dim3 grid(ns, (max_leaf + kL2PThreads - 1) / kL2PThreads);
    hipLaunchKernelGGL(k_l2p_fin<Q>, grid, dim3(kL2PThreads), 0, st, cb, n,
                       d.kind, d.lo, d.hi, d.hw, d.xl, d.L, d.near, d.ord_all,
                       ke, kb, d.counters + kCntOverflow, E, B);
  }
};

void launch_l2p_finalize(const Dev &d, const Cheb &cb, int n, int ns,
                         int max_leaf, double ke, double kb, double *E,
                         double *B, hipStream_t st) {
  dispatch_q<L2PLaunch>(cb.p + 1, d, cb, n, ns, max_leaf, ke, kb, E, B, st);
}

}  // namespace relfmm
