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
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace relfmm {

constexpr int kP2PThreads = 256;

__device__ inline float inv_d32(float D) {
  const float r = __builtin_amdgcn_rsqf(D);
  return r * r * r;
}
__device__ inline double inv_d32(double D) { return 1.0 / (D * sqrt(D)); }

// A staged source with exact offsets: position in the target leaf's frame in
// FP64 and the weights (q gamma, q u) and momentum u in the kernel precision.
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

// A separated source of the mean kernel in FP32 (see k_p2p): position in the
// target leaf's frame, weights (q gamma, q u), and a = (q u) x x, each
// rounded once from FP64.
struct SrcSep {
  float x, y, z;
  float w0, w1, w2, w3;
  float a0, a1, a2;
};

// Orders this wave's LDS writes before its later reads (and the reads before
// the next writes): each wave of k_p2p stages and reads only its own slice,
// so the tile loop needs no workgroup barrier.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave-uniform double, marked as such (it then lives in scalar registers).
__device__ inline double wave_uniform(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Pair field of one staged source on TPL targets of this lane.  For the mean
// kernel the z coordinates arrive multiplied by gbar (see k_p2p), so that
// D = rx^2 + ry^2 + rz'^2 with rz' = gbar rz.
template <typename T, int MODE, int TPL, bool SELF>
__device__ inline void p2p_pair(const Src<T, MODE> &sj, const double (&xi)[TPL],
                                const double (&yi)[TPL], const double (&zi)[TPL],
                                const int (&tidx)[TPL], int jidx, T (&e)[TPL][3],
                                T (&b)[TPL][3]) {
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const T rx = (T)(xi[k] - sj.x), ry = (T)(yi[k] - sj.y),
            rz = (T)(zi[k] - sj.z);
    T D;
    if constexpr (MODE == 0) {
      D = rx * rx + ry * ry + rz * rz;
    } else {
      const T ur = sj.u0 * rx + sj.u1 * ry + sj.u2 * rz;
      D = rx * rx + ry * ry + rz * rz + ur * ur;
    }
    if (SELF && tidx[k] == jidx) D = (T)1;
    T inv3 = inv_d32(D);
    if (SELF && tidx[k] == jidx) inv3 = (T)0;
    // g = r D^{-3/2} is shared: E += (q gamma) g, B += (q u) x g
    const T gx = inv3 * rx, gy = inv3 * ry, gz = inv3 * rz;
    e[k][0] += sj.w0 * gx;
    e[k][1] += sj.w0 * gy;
    e[k][2] += sj.w0 * gz;
    b[k][0] += sj.w2 * gz;
    b[k][0] -= sj.w3 * gy;
    b[k][1] += sj.w3 * gx;
    b[k][1] -= sj.w1 * gz;
    b[k][2] += sj.w1 * gy;
    b[k][2] -= sj.w2 * gx;
  }
}

// Pair field of one separated source on TPL targets (mean kernel, FP32,
// target leaf frame).  The magnetic sum is taken apart as
// sum_j D^{-3/2} (q u)_j x (x_i - x_j) = W_i x x_i - A_i with
// W_i = sum_j D^{-3/2} (q u)_j and A_i = sum_j D^{-3/2} a_j, so a pair costs
// three fused multiply-adds for W and three for A instead of the cross
// product; k_p2p adds W_i x x_i once per slice.  The separation of the slice
// bounds |x_i| and |x_j| by kFarRatio times the pair distance, which bounds
// the cancellation between the two sums like the FP32 rounding of the
// offsets.
template <int TPL>
__device__ inline void p2p_pair_sep(const SrcSep &sj, const float (&xi)[TPL],
                                    const float (&yi)[TPL],
                                    const float (&zi)[TPL], float (&e)[TPL][3],
                                    float (&b)[TPL][3], float (&wq)[TPL][3]) {
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const float rx = xi[k] - sj.x, ry = yi[k] - sj.y, rz = zi[k] - sj.z;
    const float D = rx * rx + ry * ry + rz * rz;
    const float inv3 = inv_d32(D);
    const float t = sj.w0 * inv3;
    e[k][0] += t * rx;
    e[k][1] += t * ry;
    e[k][2] += t * rz;
    wq[k][0] += inv3 * sj.w1;
    wq[k][1] += inv3 * sj.w2;
    wq[k][2] += inv3 * sj.w3;
    b[k][0] -= inv3 * sj.a0;
    b[k][1] -= inv3 * sj.a1;
    b[k][2] -= inv3 * sj.a2;
  }
}

// Raw global data of the source this thread stages for one tile; the loads of
// the next tile are issued before the current tile is computed, so their
// latency hides behind the pair loop.
template <typename T, int MODE>
struct SrcRaw {
  double x, y, z;
  T w0, w1, w2, w3;
  T u0, u1, u2;
};

template <typename T, int MODE>
__device__ inline void load_src(SrcRaw<T, MODE> &v, bool in, size_t p, int n,
                                const double *xl, const T *w, const T *us) {
  if (in) {
    v.x = xl[p];
    v.y = xl[n + p];
    v.z = xl[2 * (size_t)n + p];
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
}

// One workgroup = WAVES waves per chunk of 64*TPL targets of one leaf (TPL
// per lane) and one part of the leaf's list row (sched_idx: the chunks and
// parts of a leaf run together on one XCD); with nsplit > 1
// the parts of every row write separate near-field buffers that are added
// afterwards in a fixed order.  Source leaves are staged in tiles of
// 64 WAVES (padded with zero-weight sources far away, so every wave runs a
// fixed, fully unrolled loop); each wave stages and takes its own 64 sources
// of every tile for the same targets, flushes its partial sums into FP64
// after each tile, and the WAVES partial results are added in a fixed order
// at the end.  Since no wave reads another's sources, the waves run through
// the tiles without workgroup barriers (one wave's FP32 slice does not wait
// for another's FP64 one).  No atomics; the result is deterministic.
// Workgroups are launched longest list first.
//
// Mean kernel: coordinates are used as (x, y, gbar z) and the weights as
// (q gamma, q u_x, q u_y, gbar q u_z); then E_z and B_x, B_y come out
// multiplied by gbar and are divided once per target at the end.
//
// FP32 kernel: the separation test runs once per list entry between the
// bounding box of the workgroup's targets and the source leaf's box, and for
// entries that fail it, per wave and tile, against the box of the wave's 64
// sources (slices of 64 consecutive particles of a leaf, from k_slice_box).
// A slice that is well separated from the targets (largest coordinate
// magnitude M of either box in the target frame at most kFarRatio times the
// distance d between the boxes) is staged with its coordinates rounded once
// to FP32, the pair offsets formed in FP32 and the magnetic sum taken apart
// (p2p_pair_sep); the representation
// error of both coordinates is then at most eps M <= kFarRatio eps d relative
// to |r| >= d, and the terms of the two parts of the magnetic sum exceed the
// pair's own by at most the same factor.  Slices close to or overlapping the
// targets keep the FP64 offsets and the direct cross product.  Particles are in x order inside a leaf, so slices are thin slabs
// and the test separates much more than one between whole leaves: on the
// flat 1M bunch 14 % of the pairs keep FP64 offsets (43 % with a test per
// source leaf), on the 131k Gaussian bunch 10 % (18 %).  Mean kernel only.
constexpr double kFarRatio = 8.0;
// Sources per wave and tile slice; a workgroup of WAVES waves stages tiles of
// 64 WAVES sources (4 waves when the built tree's largest leaf holds more
// than 128 particles, 2 up to 128, 1 up to 64, so that small leaves do not
// leave waves idle on padding).
constexpr int kP2PPerWave = kWave;
#ifndef RELFMM_P2P_UNROLL
#define RELFMM_P2P_UNROLL 4
#endif
// Each staged source is one LDS broadcast read per wave (40 bytes, an FP32
// separated source with its a = (q u) x x or one with FP64 coordinates): with one target per lane the LDS return path (128 bytes per
// clock per CU) is as busy as the VALU, so the FP32 kernels take two targets
// per lane when the grid stays large enough.  Sources per loop iteration
// (UNR): 4 with one target per lane; with two, 4 on unsplit launches and 1
// (no unrolling) on split ones.  Measured:
// without unrolling the pair loop issues twice the LDS reads (no paired
// ds_read2) but one VALU instruction every 3.1 instead of 3.2 cycles, 3 %
// faster on the 131k bunch (rows split in eight); on the unsplit 1M bunch
// unrolling by 4 beat 2 by 0.8 % and 1 by 3 %.
#ifndef RELFMM_P2P_UNROLL2
#define RELFMM_P2P_UNROLL2 4
#endif
constexpr int kP2PUnroll[3] = {0, RELFMM_P2P_UNROLL, RELFMM_P2P_UNROLL2};

// Bounding boxes of the slices of 64 consecutive particles of every leaf
// (from the leaf's first particle, in leaf order), in the leaf's own frame:
// sbox[(s * kmax + k) * 6 + g] = min and [.. + 3 + g] = max of coordinate g
// over slice k of leaf s.  One wave per slice.
constexpr int kBoxWaves = 4;
__global__ void __launch_bounds__(kBoxWaves * kWave)
k_slice_box(int n, int nslices, int kmax, const int32_t *kind,
            const int32_t *lo, const int32_t *hi, const double *xl,
            double *sbox) {
  const int slice = blockIdx.x * kBoxWaves + (int)threadIdx.x / kWave;
  if (slice >= nslices) return;
  const int s = slice / kmax, k = slice - s * kmax;
  if (kind[s] != 1) return;
  const int p0 = lo[s] + k * kWave;
  if (p0 >= hi[s]) return;
  const int p = p0 + lane_id();
  const int pp = p < hi[s] ? p : p0;
  double mn[3], mx[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) mn[g] = mx[g] = xl[(size_t)g * n + pp];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1)
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      mn[g] = fmin(mn[g], __shfl_xor(mn[g], o));
      mx[g] = fmax(mx[g], __shfl_xor(mx[g], o));
    }
  if (lane_id() == 0)
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      sbox[(size_t)slice * 6 + g] = mn[g];
      sbox[(size_t)slice * 6 + 3 + g] = mx[g];
    }
}

// HALF (leaves of at most 64 particles, one wave): each lane takes two of
// the 64 targets (lane % 32 and lane % 32 + 32) and the two half-waves take
// alternate sources of every tile, so that one LDS read of a source serves
// two pairs as with two targets per lane on larger leaves; the halves' sums
// are added at the end.
template <typename T, int MODE, int TPL, int WAVES, int UNR, bool HALF = false>
__global__ void __launch_bounds__(WAVES * kWave)
k_p2p(int n, int bits, const int32_t *kind, const int32_t *lo,
      const int32_t *hi, const double *cen, const double *hw,
      const int32_t *row,
      const uint64_t *keys, const int32_t *order, const double *xl,
      const T *w, const T *us, const double *gbar, const double *sbox,
      int kmax, double *near, int ny, int nsplit) {
  constexpr int kTile = WAVES * kWave;
  // wave w stages and reads slice w of every tile, as FP64 or FP32 records
  __shared__ union {
    Src<T, MODE> d[kWave];
    SrcSep f[kWave];
  } sh[WAVES];
  __shared__ double red[WAVES > 1 ? WAVES - 1 : 1][6][TPL * kWave];
  // the mean kernel only: the per-source momenta of the source kernel stretch
  // the metric along u_j, which the box test does not see
  constexpr bool kHybrid = sizeof(T) == 4 && MODE == 0;
  const SchedIdx si = sched_idx(order, ny, nsplit, true);
  const int t = si.node;
  if (t < 0 || kind[t] != 1) return;
  const int tl = lo[t], tc = hi[t] - tl;
  static_assert(!HALF || (TPL == 2 && WAVES == 1), "half-wave mode");
  const int i0 = si.y * kWave * (HALF ? 1 : TPL);
  if (i0 >= tc) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const double zs = MODE == 0 ? *gbar : 1.0;  // z stretch of the mean kernel
  const uint64_t mask = (1ull << bits) - 1ull;
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  const int part = si.z;
  const int rlen = row[t + 1] - row[t];
  const int r0 = row[t] + rlen * part / nsplit,
            r1 = row[t] + rlen * (part + 1) / nsplit;
  near += (size_t)part * 6 * n;
  double xi[TPL], yi[TPL], zi[TPL];
  int tidx[TPL];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int ii = i0 + (HALF ? (lane & 31) + 32 * k : k * kWave + lane);
    tidx[k] = ii;
    const int pi = tl + (ii < tc ? ii : 0);
    xi[k] = xl[pi];
    yi[k] = xl[(size_t)n + pi];
    zi[k] = zs * xl[2 * (size_t)n + pi];
  }
  double acc[TPL][6];
#pragma unroll
  for (int k = 0; k < TPL; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[k][c] = 0.0;
  // bounding box of this workgroup's targets (its TPL slices of the leaf),
  // in the kernel's coordinates (x, y, zs z) of the target frame
  double alo[3] = {0.0, 0.0, 0.0}, ahi[3] = {0.0, 0.0, 0.0};
  if constexpr (kHybrid) {
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      alo[g] = __builtin_inf();
      ahi[g] = -__builtin_inf();
    }
#pragma unroll
    for (int k = 0; k < (HALF ? 1 : TPL); ++k) {
      const int sk = HALF ? si.y : si.y * TPL + k;
      if (sk * kWave < tc) {
        const double *b = sbox + ((size_t)t * kmax + sk) * 6;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
          alo[g] = fmin(alo[g], b[g]);
          ahi[g] = fmax(ahi[g], b[3 + g]);
        }
      }
    }
    alo[2] *= zs;
    ahi[2] *= zs;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      alo[g] = wave_uniform(alo[g]);
      ahi[g] = wave_uniform(ahi[g]);
    }
  }

  // tile cursor over (list entry r, first source j0 of the tile)
  int r = r0, j0 = 0, s = 0, sl = 0, sc = 0;
  bool far_leaf = false;
  double dx = 0.0, dy = 0.0, dz = 0.0;
  auto open_entry = [&](int rr) {
    s = (int)(keys[rr] & mask);
    sl = lo[s];
    sc = hi[s] - sl;
    dx = cen[3 * s] - ct[0];
    dy = cen[3 * s + 1] - ct[1];
    dz = cen[3 * s + 2] - ct[2];
    far_leaf = false;
    if (kHybrid && s != t) {
      // the same test between the whole source leaf and the targets' box
      // first: it settles most entries once, with no test per tile
      const double dd[3] = {dx, dy, dz}, sz[3] = {1.0, 1.0, zs};
      double gap2 = 0.0, mx = 0.0;
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        const double hs = hw[3 * s + g];
        const double bl = (dd[g] - hs) * sz[g], bh = (dd[g] + hs) * sz[g];
        const double gap = fmax(fmax(bl - ahi[g], alo[g] - bh), 0.0);
        gap2 += gap * gap;
        mx = fmax(mx, fmax(fmax(fabs(bl), fabs(bh)),
                           fmax(fabs(alo[g]), fabs(ahi[g]))));
      }
      far_leaf = gap2 > 0.0 && mx * mx <= kFarRatio * kFarRatio * gap2;
    }
  };
  // box of this wave's slice of the next tile (source leaf frame), for
  // entries the leaf test leaves close
  double blo[3] = {0.0, 0.0, 0.0}, bhi[3] = {0.0, 0.0, 0.0};
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  auto load_box = [&]() {
    if constexpr (kHybrid) {
      if (!far_leaf && j0 + wave_u * kWave < sc) {
        const double *b = sbox + ((size_t)s * kmax + j0 / kWave + wave_u) * 6;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
          blo[g] = b[g];
          bhi[g] = b[3 + g];
        }
      }
    }
  };
  SrcRaw<T, MODE> raw;
  if (r < r1) {
    open_entry(r);
    load_src(raw, tid < sc, (size_t)sl + tid, n, xl, w, us);
    load_box();
  }
  while (r < r1) {
    const int s_tile = s, j_tile = j0, sc_tile = sc;
    const double ddx = dx, ddy = dy, ddz = dz;
    const bool live = j_tile + wave * kWave < sc_tile;  // wave-uniform
    // separation of this wave's slice from the targets: box gap and largest
    // coordinate magnitude, in the kernel's coordinates of the target frame
    bool far = far_leaf;
    if constexpr (kHybrid) {
      if (live && !far) {
        const double dd[3] = {ddx, ddy, ddz}, sz[3] = {1.0, 1.0, zs};
        double gap2 = 0.0, mx = 0.0;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
          const double bl = (blo[g] + dd[g]) * sz[g], bh = (bhi[g] + dd[g]) * sz[g];
          const double gap = fmax(fmax(bl - ahi[g], alo[g] - bh), 0.0);
          gap2 += gap * gap;
          mx = fmax(mx, fmax(fmax(fabs(bl), fabs(bh)),
                             fmax(fabs(alo[g]), fabs(ahi[g]))));
        }
        // strictly separated boxes only (two boxes collapsed onto the
        // target centre have mx = gap = 0)
        far = gap2 > 0.0 && mx * mx <= kFarRatio * kFarRatio * gap2;
      }
    }
    wave_lds_sync();
    {
      const bool pad = j_tile + tid >= sc_tile;
      const double px = pad ? raw.x : raw.x + ddx;
      const double py = pad ? raw.y : raw.y + ddy;
      const double pz = pad ? raw.z : zs * (raw.z + ddz);
      const T w3 = MODE == 0 ? (T)(zs * (double)raw.w3) : raw.w3;
      if (far) {
        // with a = (q u) x x
        const double q1 = (double)raw.w1, q2 = (double)raw.w2, q3 = (double)w3;
        SrcSep v;
        v.x = (float)px;
        v.y = (float)py;
        v.z = (float)pz;
        v.w0 = (float)raw.w0;
        v.w1 = (float)raw.w1;
        v.w2 = (float)raw.w2;
        v.w3 = (float)w3;
        v.a0 = (float)(q2 * pz - q3 * py);
        v.a1 = (float)(q3 * px - q1 * pz);
        v.a2 = (float)(q1 * py - q2 * px);
        sh[wave].f[lane] = v;
      } else {
        Src<T, MODE> v;
        v.x = px;
        v.y = py;
        v.z = pz;
        v.w0 = raw.w0;
        v.w1 = raw.w1;
        v.w2 = raw.w2;
        v.w3 = w3;
        if constexpr (MODE == 1) {
          v.u0 = raw.u0;
          v.u1 = raw.u1;
          v.u2 = raw.u2;
        }
        sh[wave].d[lane] = v;
      }
    }
    wave_lds_sync();
    // advance the cursor and issue the loads of the next tile
    j0 += kTile;
    if (j0 >= sc) {
      ++r;
      j0 = 0;
      if (r < r1) open_entry(r);
    }
    if (r < r1) {
      load_src(raw, j0 + tid < sc, (size_t)sl + j0 + tid, n, xl, w, us);
      load_box();
    }

    if (!live) continue;  // wave-uniform: this wave's slice is padding
    const int kb = wave * kWave;
    const int hw2 = lane >> 5;  // HALF: this lane's half-wave
    // valid sources of this wave's slice (the padding after them is not
    // computed; with HALF an odd count meets one zero-weight padding record)
    const int nv = min(kP2PPerWave, sc_tile - (j_tile + kb));
    T e[TPL][3], b[TPL][3];
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) e[k][c] = b[k][c] = (T)0;
    // the pair loops over this wave's sources: FULL slices with a fixed trip
    // count, a leaf's last partial slice over its valid sources only
    auto pairs = [&](auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int cnt = FULL ? (HALF ? kP2PPerWave / 2 : kP2PPerWave)
                           : (HALF ? (nv + 1) >> 1 : nv);
      if (far) {
        // a separated slice never holds one of the targets
        if constexpr (kHybrid) {
          float xf[TPL], yf[TPL], zf[TPL], wq[TPL][3];
#pragma unroll
          for (int k = 0; k < TPL; ++k) {
            xf[k] = (float)xi[k];
            yf[k] = (float)yi[k];
            zf[k] = (float)zi[k];
            wq[k][0] = wq[k][1] = wq[k][2] = 0.0f;
          }
          if constexpr (HALF) {
#pragma unroll UNR
            for (int k = 0; k < cnt; ++k)
              p2p_pair_sep<TPL>(sh[wave].f[2 * k + hw2], xf, yf, zf, e, b, wq);
          } else {
#pragma unroll UNR
            for (int k = 0; k < cnt; ++k)
              p2p_pair_sep<TPL>(sh[wave].f[k], xf, yf, zf, e, b, wq);
          }
          // B += W x x_i
#pragma unroll
          for (int k = 0; k < TPL; ++k) {
            b[k][0] += wq[k][1] * zf[k] - wq[k][2] * yf[k];
            b[k][1] += wq[k][2] * xf[k] - wq[k][0] * zf[k];
            b[k][2] += wq[k][0] * yf[k] - wq[k][1] * xf[k];
          }
        }
      } else if (s_tile == t) {
        if constexpr (HALF) {
#pragma unroll UNR
          for (int k = 0; k < cnt; ++k)
            p2p_pair<T, MODE, TPL, true>(sh[wave].d[2 * k + hw2], xi, yi, zi,
                                         tidx, j_tile + kb + 2 * k + hw2, e, b);
        } else {
#pragma unroll UNR
          for (int k = 0; k < cnt; ++k)
            p2p_pair<T, MODE, TPL, true>(sh[wave].d[k], xi, yi, zi, tidx,
                                         j_tile + kb + k, e, b);
        }
      } else {
        if constexpr (HALF) {
#pragma unroll UNR
          for (int k = 0; k < cnt; ++k)
            p2p_pair<T, MODE, TPL, false>(sh[wave].d[2 * k + hw2], xi, yi, zi,
                                          tidx, -1, e, b);
        } else {
#pragma unroll UNR
          for (int k = 0; k < cnt; ++k)
            p2p_pair<T, MODE, TPL, false>(sh[wave].d[k], xi, yi, zi, tidx, -1,
                                          e, b);
        }
      }
    };
    if (nv == kP2PPerWave)  // wave-uniform
      pairs(std::true_type{});
    else
      pairs(std::false_type{});
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[k][c] += (double)e[k][c];
        acc[k][3 + c] += (double)b[k][c];
      }
  }
  if constexpr (HALF)
    // the other half-wave's sums over the other sources, in a fixed order
#pragma unroll
    for (int k = 0; k < TPL; ++k)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double o = __shfl_xor(acc[k][c], 32);
        acc[k][c] = lane < 32 ? acc[k][c] + o : o + acc[k][c];
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
      // HALF: both halves hold the sums; each lane writes one of its targets
      if (HALF && k != (lane >> 5)) continue;
      const int ii = i0 + (HALF ? (lane & 31) + 32 * k : k * kWave + lane);
      if (ii >= tc) continue;
      for (int wv = 0; wv < WAVES - 1; ++wv)
        for (int c = 0; c < 6; ++c) acc[k][c] += red[wv][c][k * kWave + lane];
      if (MODE == 0) {
        acc[k][2] /= zs;
        acc[k][3] /= zs;
        acc[k][4] /= zs;
      }
      for (int c = 0; c < 6; ++c) near[(size_t)c * n + tl + ii] = acc[k][c];
    }
  }
}

// near[0..6n) += near[6n..12n) + ...: the later row parts' sums, in order.
__global__ void k_near_combine(int n6, int nsplit, double *near) {
  const int i = blockIdx.x * kP2PThreads + threadIdx.x;
  if (i >= n6) return;
  double s = near[i];
  for (int p = 1; p < nsplit; ++p) s += near[(size_t)p * n6 + i];
  near[i] = s;
}

// Waves wanted per launch: rows are split (up to kP2PMaxSplit parts, as far
// as the near-field buffer holds them) until the grid has this many, i.e.
// eight rounds of four workgroups of four waves per CU, so that the last
// round's uneven rows leave a short tail.
#ifndef RELFMM_P2P_MINWAVES
#define RELFMM_P2P_MINWAVES 32768
#endif
constexpr int kP2PMinWaves = RELFMM_P2P_MINWAVES;

template <typename T, int MODE, int TPL, int WAVES, bool HALF = false>
static void launch_p2p_t(const Dev &d, const P2PArgs &a, int n, const T *w,
                         const T *us, hipStream_t st) {
  const int per_wg = kWave * (HALF ? 1 : TPL);
  const int chunks = (a.max_leaf + per_wg - 1) / per_wg;
  const int kmax = (a.max_leaf + kWave - 1) / kWave;
  // leaves: the index split puts every leaf on the last level (ns / 2 slots)
  const int64_t waves = (int64_t)std::max(a.ns / 2, 1) * chunks * WAVES;
  const int64_t parts = (int64_t)(d.near_cap / (6 * (size_t)n));
  int nsplit = 1;
  while (2 * nsplit <= kP2PMaxSplit && 2 * nsplit <= parts &&
         waves * nsplit < kP2PMinWaves)
    nsplit *= 2;
  const dim3 grid(order_len(a.ns) * chunks * nsplit), block(WAVES * kWave);
  bool split2 = false;
  if constexpr (TPL == 2) split2 = nsplit > 1;
  if (split2) {
    if constexpr (TPL == 2)
      hipLaunchKernelGGL((k_p2p<T, MODE, TPL, WAVES, 1, HALF>), grid, block, 0, st,
                         n, a.bits, d.kind, d.lo, d.hi, d.cen, d.hw,
                         d.p2p_row, d.p2p, d.order_p2p, d.xl, w, us, d.gbar,
                         d.sbox, kmax, d.near, chunks, nsplit);
  } else {
    hipLaunchKernelGGL((k_p2p<T, MODE, TPL, WAVES, kP2PUnroll[TPL], HALF>), grid,
                       block, 0, st, n, a.bits, d.kind, d.lo, d.hi, d.cen,
                       d.hw, d.p2p_row, d.p2p, d.order_p2p, d.xl, w, us,
                       d.gbar, d.sbox, kmax, d.near, chunks, nsplit);
  }
  if (nsplit > 1)
    hipLaunchKernelGGL(k_near_combine, dim3((6 * n + kP2PThreads - 1) / kP2PThreads),
                       dim3(kP2PThreads), 0, st, 6 * n, nsplit, d.near);
}

// Workgroup size by leaf size.
template <typename T, int MODE, int TPL>
static void launch_p2p_w(const Dev &d, const P2PArgs &a, int n, const T *w,
                         const T *us, hipStream_t st) {
  if (a.max_leaf <= kWave)
    launch_p2p_t<T, MODE, TPL, 1>(d, a, n, w, us, st);
  else if (a.max_leaf <= 2 * kWave)
    launch_p2p_t<T, MODE, TPL, 2>(d, a, n, w, us, st);
  else
    launch_p2p_t<T, MODE, TPL, 4>(d, a, n, w, us, st);
}

void launch_p2p(const Dev &d, const P2PArgs &a, int n, hipStream_t st) {
  if (a.prec != 0 && a.mode == 0) {
    // slice boxes for the separation test of the FP32 mean kernel
    const int nslices = a.ns * ((a.max_leaf + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_slice_box, dim3((nslices + kBoxWaves - 1) / kBoxWaves),
                       dim3(kBoxWaves * kWave), 0, st, n, nslices,
                       (a.max_leaf + kWave - 1) / kWave, d.kind, d.lo, d.hi,
                       d.xl, d.sbox);
  }
  // two targets per lane for the FP32 kernels once a leaf spans more than
  // one wave (two-wave workgroups up to 128, four above)
  const bool two = a.max_leaf > kWave;
  if (a.prec == 0) {
    if (a.mode == 0)
      launch_p2p_w<double, 0, 1>(d, a, n, d.w, d.us, st);
    else
      launch_p2p_w<double, 1, 1>(d, a, n, d.w, d.us, st);
  } else if (two && a.max_leaf <= 2 * kWave) {
    if (a.mode == 0)
      launch_p2p_t<float, 0, 2, 2>(d, a, n, d.w32, d.us32, st);
    else
      launch_p2p_t<float, 1, 2, 2>(d, a, n, d.w32, d.us32, st);
  } else if (two) {
    if (a.mode == 0)
      launch_p2p_t<float, 0, 2, 4>(d, a, n, d.w32, d.us32, st);
    else
      launch_p2p_t<float, 1, 2, 4>(d, a, n, d.w32, d.us32, st);
  } else {
    // leaves of at most 64: one wave, two targets per lane on half-waves
    if (a.mode == 0)
      launch_p2p_t<float, 0, 2, 1, true>(d, a, n, d.w32, d.us32, st);
    else
      launch_p2p_t<float, 1, 2, 1, true>(d, a, n, d.w32, d.us32, st);
  }
}

}  // namespace relfmm
