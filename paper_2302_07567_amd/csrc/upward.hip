// Upward pass (Alg. upwardpass): P2M at the leaves (Alg. P2M with the
// effective masses of Sec. 3) and M2M from children to parents (eq. M2M,
// Alg. M2M), in FP64.
//
// Proxy index nu = (a*(p+1) + b)*(p+1) + c for per-axis node indices (a, b, c)
// along (x, y, z).  Multipoles are [node][nu][4] = (q gamma, q u_x, q u_y,
// q u_z).  M2M applies the tensor-product transfer T_x (x) T_y (x) T_z one
// axis at a time, T_g[a][b] = l^g_{parent,a}(xi^g_{child,b}).
#include "internal.hpp"

namespace relfmm {

constexpr int kQ = kMaxDegree + 1;
// threads per node of the M2M / L2L kernels (the upper levels have few
// nodes, so the passes of one node are spread over many threads)
#ifndef RELFMM_TRANS_THREADS
#define RELFMM_TRANS_THREADS 1024
#endif
constexpr int kTransThreads = RELFMM_TRANS_THREADS;

// One workgroup per leaf; thread (a, b) of each of S thread groups owns the
// proxies (a, b, 0..p) and all NC components, so each particle's basis values
// are read once per thread (the z basis and the weights as broadcasts):
//   out[v][nu][k] = sum_{j in leaf v} l_{v,nu}(x_j) wts[k][j],  k < NC.
// P2M uses the weights (q gamma, q u) (NC = 4); the transpose of L2P uses the
// scaled field cotangents (NC = 6).  Group s takes the chunks s, s + S, ...
// of 64 particles; the per-axis bases of a chunk are computed by the group's
// threads and shared through LDS; the S partial sums are added in group
// order at the end, one group at a time through LDS.
constexpr int kAnterpChunk = 64;

template <int Q>
constexpr int anterp_threads() {
  return (Q * Q + kWave - 1) / kWave * kWave;
}
// thread groups per leaf: four up to n = 6, two above (LDS)
template <int Q>
constexpr int anterp_groups() {
  return Q <= 7 ? 4 : 2;
}

template <int Q, int NC>
__global__ void __launch_bounds__(anterp_threads<Q>() * anterp_groups<Q>())
k_anterp(Cheb cb, int n, const int32_t *kind, const int32_t *lo,
         const int32_t *hi, const double *hw, const double *xl,
         const double *wts, double *out) {
  constexpr int NT = anterp_threads<Q>(), S = anterp_groups<Q>();
  constexpr int kStage = S * kAnterpChunk * (3 * Q + NC);
  constexpr int kRed = Q * Q * Q * NC;
  __shared__ double sh[kStage > kRed ? kStage : kRed];
  const int v = blockIdx.x;
  if (kind[v] != 1) return;
  const int grp = threadIdx.x / NT, tid = threadIdx.x % NT;
  double(*lb)[3][Q] =
      reinterpret_cast<double(*)[3][Q]>(sh + grp * kAnterpChunk * 3 * Q);
  double(*lw)[NC] = reinterpret_cast<double(*)[NC]>(
      sh + S * kAnterpChunk * 3 * Q + grp * kAnterpChunk * NC);
  const int l0 = lo[v], cnt = hi[v] - l0;
  const double h[3] = {hw[3 * v], hw[3 * v + 1], hw[3 * v + 2]};
  const bool own = tid < Q * Q;
  const int a = own ? tid / Q : 0, b = own ? tid % Q : 0;
  double acc[Q][NC];
#pragma unroll
  for (int c = 0; c < Q; ++c)
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[c][k] = 0.0;
  // every group runs the same number of rounds (barriers are block-wide)
  for (int r0 = 0; r0 < cnt; r0 += S * kAnterpChunk) {
    const int j0 = r0 + grp * kAnterpChunk;
    const int nj = max(0, min(kAnterpChunk, cnt - j0));
    __syncthreads();
    for (int i = tid; i < 3 * nj; i += NT) {
      const int g = i / nj, jj = i - g * nj, p = l0 + j0 + jj;
      double l[Q];
      basis1d_q<Q>(cb, xl[(size_t)g * n + p] / h[g], l);
#pragma unroll
      for (int k = 0; k < Q; ++k) lb[jj][g][k] = l[k];
    }
    for (int i = tid; i < NC * nj; i += NT) {
      const int k = i / nj, jj = i - k * nj;
      lw[jj][k] = wts[(size_t)k * n + l0 + j0 + jj];
    }
    __syncthreads();
    for (int jj = 0; jj < nj; ++jj) {
      const double lab = lb[jj][0][a] * lb[jj][1][b];
      double wk[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) wk[k] = lw[jj][k];
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const double l = lab * lb[jj][2][c];
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[c][k] += l * wk[k];
      }
    }
  }
  // groups 1..S-1 hand their sums to group 0 one after another
  double *red = sh + (size_t)(a * Q + b) * Q * NC;
  for (int s = 1; s < S; ++s) {
    __syncthreads();
    if (grp == s && own)
#pragma unroll
      for (int c = 0; c < Q; ++c)
#pragma unroll
        for (int k = 0; k < NC; ++k) red[c * NC + k] = acc[c][k];
    __syncthreads();
    if (grp == 0 && own)
#pragma unroll
      for (int c = 0; c < Q; ++c)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[c][k] += red[c * NC + k];
  }
  if (grp == 0 && own) {
    double *o = out + ((size_t)v * Q * Q * Q + (size_t)(a * Q + b) * Q) * NC;
#pragma unroll
    for (int c = 0; c < Q; ++c)
#pragma unroll
      for (int k = 0; k < NC; ++k) o[c * NC + k] = acc[c][k];
  }
}

template <int NC>
struct AnterpLaunch {
  template <int Q>
  struct F {
    static void run(const Dev &d, const Cheb &cb, int n, int ns,
                    const double *wts, double *out, hipStream_t st) {
      hipLaunchKernelGGL((k_anterp<Q, NC>), dim3(ns),
                         dim3(anterp_threads<Q>() * anterp_groups<Q>()), 0, st,
                         cb, n, d.kind, d.lo, d.hi, d.hw, d.xl, wts, out);
    }
  };
};

void launch_p2m(const Dev &d, const Cheb &cb, int n, int ns, hipStream_t st) {
  dispatch_q<AnterpLaunch<4>::F>(cb.p + 1, d, cb, n, ns, d.w, d.M, st);
}

void launch_l2p_transpose(const Dev &d, const Cheb &cb, int n, int ns,
                          hipStream_t st) {
  dispatch_q<AnterpLaunch<6>::F>(cb.p + 1, d, cb, n, ns, d.ebar, d.Lbar, st);
}

// T_g[a][b] = l^g_{S,a}(xi^g_{C,b}): basis of node S at the proxies of C.
__device__ inline void transfer_tables(const Cheb &cb, const double *cen,
                                       const double *hw, int S, int C,
                                       double (*T)[kQ][kQ]) {
  const int q = cb.p + 1;
  const int tid = threadIdx.x;
  if (tid < 3 * q) {
    const int g = tid / q, b = tid % q;
    double l[kQ];
    const double xb = cen[3 * C + g] + hw[3 * C + g] * cb.t[b];
    basis1d(cb, (xb - cen[3 * S + g]) / hw[3 * S + g], l);
    for (int a = 0; a < q; ++a) T[g][a][b] = l[a];
  }
}

// One workgroup per parent S at one level, all NC components at once:
// M_S[mu][k] = sum over children C of (T_x (x) T_y (x) T_z) M_C[.][k].
// A child's block M_C[m][NC] is contiguous, so it is loaded into LDS with
// coalesced reads, the three mode products run on the [mu][k] layout in LDS,
// and the parent's block is written (first child) and updated (second) with
// coalesced accesses: every byte of the pass moves once (one workgroup per
// (parent, component) with strided accesses moved 2.8x that).
template <int Q, int NC>
__global__ void __launch_bounds__(kTransThreads)
k_m2m(Cheb cb, int level, const int32_t *kind, const double *cen,
      const double *hw, double *M) {
  constexpr int QQ = Q * Q, MM = QQ * Q, W = MM * NC;
  __shared__ double T[2][3][kQ][kQ];
  __shared__ double P[W], B1[W];
  const int S = (1 << level) + blockIdx.x;
  if (kind[S] != 2) return;
  const int tid = threadIdx.x;
  transfer_tables(cb, cen, hw, S, 2 * S, T[0]);
  if (tid >= 64) {
    // a second group of threads builds the table of the second child
    const int t2 = tid - 64;
    if (t2 < 3 * Q) {
      const int g = t2 / Q, b = t2 % Q;
      double l[kQ];
      const double xb = cen[3 * (2 * S + 1) + g] + hw[3 * (2 * S + 1) + g] * cb.t[b];
      basis1d(cb, (xb - cen[3 * S + g]) / hw[3 * S + g], l);
      for (int a = 0; a < Q; ++a) T[1][g][a][b] = l[a];
    }
  }
  double *out = M + (size_t)S * W;
  for (int ci = 0; ci < 2; ++ci) {
    const double *in = M + (size_t)(2 * S + ci) * W;
    __syncthreads();
    for (int i = tid; i < W; i += kTransThreads) P[i] = in[i];
    __syncthreads();
    // z: B1[a'][b'][c] = sum_c' T_z[c][c'] P[a'][b'][c']
    for (int i = tid; i < W; i += kTransThreads) {
      const int k = i % NC, mu = i / NC, ab = mu / Q, c = mu % Q;
      double s = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < Q; ++c2) s += T[ci][2][c][c2] * P[(ab * Q + c2) * NC + k];
      B1[i] = s;
    }
    __syncthreads();
    // y: P[a'][b][c] = sum_b' T_y[b][b'] B1[a'][b'][c]
    for (int i = tid; i < W; i += kTransThreads) {
      const int k = i % NC, mu = i / NC, a = mu / QQ, b = (mu / Q) % Q, c = mu % Q;
      double s = 0.0;
#pragma unroll
      for (int b2 = 0; b2 < Q; ++b2)
        s += T[ci][1][b][b2] * B1[(a * QQ + b2 * Q + c) * NC + k];
      P[i] = s;
    }
    __syncthreads();
    // x: M_S[a][b][c] (+)= sum_a' T_x[a][a'] P[a'][b][c]
    for (int i = tid; i < W; i += kTransThreads) {
      const int k = i % NC, mu = i / NC, a = mu / QQ, bc = mu % QQ;
      double s = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < Q; ++a2) s += T[ci][0][a][a2] * P[(a2 * QQ + bc) * NC + k];
      out[i] = ci == 0 ? s : out[i] + s;
    }
  }
}

template <int NC>
struct M2MLaunch {
  template <int Q>
  struct F {
    static void run(const Cheb &cb, int level, const int32_t *kind,
                    const double *cen, const double *hw, double *M,
                    hipStream_t st) {
      hipLaunchKernelGGL((k_m2m<Q, NC>), dim3(1 << level), dim3(kTransThreads), 0, st,
                         cb, level, kind, cen, hw, M);
    }
  };
};

void launch_m2m_level(const Dev &d, const Cheb &cb, int level,
                      hipStream_t st) {
  dispatch_q<M2MLaunch<4>::F>(cb.p + 1, cb, level, d.kind, d.cen, d.hw, d.M,
                              st);
}

// The transpose of L2L has the form of M2M (children into the parent), here
// on the six components of the local-field cotangents.
void launch_l2l_transpose_level(const Dev &d, const Cheb &cb, int level,
                                hipStream_t st) {
  dispatch_q<M2MLaunch<6>::F>(cb.p + 1, cb, level, d.kind, d.cen, d.hw,
                              d.Lbar, st);
}

}  // namespace relfmm
