// Shared device helpers of the relfmm HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace relfmm {

constexpr int kMaxDegree = 10;
constexpr int kWave = 64;

// Chebyshev points of the second kind on [-1, 1] and their barycentric
// weights, passed to kernels by value.  t_k = cos(k pi / p) is written as
// sin(pi (p - 2k) / (2p)) so that t_0 = 1, t_p = -1, t_{p/2} = 0 exactly.
// D[j][k] = l_k'(t_j) on [-1, 1] is the differentiation matrix of the nodes.
struct Cheb {
  double t[kMaxDegree + 1];
  double w[kMaxDegree + 1];
  double D[kMaxDegree + 1][kMaxDegree + 1];
  int p;
};

// Order-preserving map of a finite double to an unsigned 64-bit key.
// -0.0 is folded into +0.0 so that equal values get equal keys.
__device__ inline uint64_t double_key(double v) {
  v = v + 0.0;
  uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// One-dimensional Lagrange basis over [c - h, c + h] at reference coordinate
// tau = (x - c)/h, second (true) barycentric form (Berrut & Trefethen 2004).
// An exact node hit returns the Kronecker delta.
__device__ inline void basis1d(const Cheb &cb, double tau, double *l) {
  const int p = cb.p;
  int hit = -1;
  for (int k = 0; k <= p; ++k)
    if (tau == cb.t[k]) hit = k;
  if (hit >= 0) {
    for (int k = 0; k <= p; ++k) l[k] = (k == hit) ? 1.0 : 0.0;
    return;
  }
  double s = 0.0;
  for (int k = 0; k <= p; ++k) {
    l[k] = cb.w[k] / (tau - cb.t[k]);
    s += l[k];
  }
  for (int k = 0; k <= p; ++k) l[k] = l[k] / s;
}

// The same basis for a degree known at compile time (Q = p + 1 nodes), into
// registers.
template <int Q>
__device__ inline void basis1d_q(const Cheb &cb, double tau, double (&l)[Q]) {
  int hit = -1;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (tau == cb.t[k]) hit = k;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    l[k] = cb.w[k] / (tau - cb.t[k]);
    s += l[k];
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) l[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : l[k] / s;
}

// Dispatch a functor templated on Q = p + 1 (2..11).
template <template <int> class F, typename... A>
inline void dispatch_q(int q, A &&...args) {
  switch (q) {
    case 2: F<2>::run(args...); break;
    case 3: F<3>::run(args...); break;
    case 4: F<4>::run(args...); break;
    case 5: F<5>::run(args...); break;
    case 6: F<6>::run(args...); break;
    case 7: F<7>::run(args...); break;
    case 8: F<8>::run(args...); break;
    case 9: F<9>::run(args...); break;
    case 10: F<10>::run(args...); break;
    default: F<11>::run(args...); break;
  }
}

__device__ inline int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Workgroup schedule of the list-driven kernels (P2P, M2L and their
// transposes).  The launch is one-dimensional; consecutive workgroup ids are
// dealt to the eight XCDs in turn, so id L runs on XCD L % 8.  The order
// array is read in slices of eight: with ids taken in order, slot p * 8 + x
// runs on XCD x.  A node has ny * nz workgroups (chunks y, parts z).
// GROUPED: they take consecutive positions of one XCD, so they run together
// and share that XCD's L2 for the source data they all stage (P2P: every
// chunk and row part of a leaf stages the same source leaves; M2L: every row
// block of a node stages the same source multipoles).  Otherwise the launch
// is ny * nz passes over the order (M2L with a small last row block, which
// measured better as a pass of its own).
constexpr int kXcds = 8;
struct SchedIdx {
  int node, y, z;
};
__device__ inline SchedIdx sched_idx(const int32_t *order, int ny, int nz,
                                    bool grouped) {
  SchedIdx r;
  const int L = (int)blockIdx.x, U = ny * nz;
  int sub;
  if (grouped) {
    const int x = L & (kXcds - 1), k = L / kXcds, p = k / U;
    sub = k - p * U;
    r.node = order[p * kXcds + x];
  } else {
    const int olen = (int)gridDim.x / U;
    sub = L / olen;
    r.node = order[L - sub * olen];
  }
  r.y = sub % ny;
  r.z = sub / ny;
  return r;
}

// Wave-aggregated append: every lane of the wave must call this.  Lanes with
// pred reserve n_each consecutive slots of *counter; returns the first slot
// (or -1 for lanes without pred).
__device__ inline int wave_alloc(bool pred, int n_each, int *counter) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return -1;
  int leader = __ffsll((unsigned long long)mask) - 1;
  int lane = lane_id();
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask) * n_each);
  base = __shfl(base, leader);
  int rank = __popcll(mask & ((1ull << lane) - 1ull));
  return pred ? base + rank * n_each : -1;
}

}  // namespace relfmm
