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

// DG = false: L_t = the M2L sums above.  DG = true: the same sums with
// D^{-3/2} replaced by gbar^2 dz^2 D^{-5/2} (= -gbar/3 times the gbar
// derivative of D^{-3/2}) are not stored but dotted with the local
// cotangents Lbar_t; the block's sum goes to gdot[t * kGdotStride].
__device__ inline double block_sum_m2l(double v, double *sh, int nthreads) {
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nthreads / kWave; ++k) s += sh[k];
  return s;
}

template <typename T, bool DG>
__global__ void __launch_bounds__(kM2LThreads)
k_m2l_valu(Cheb cb, int bits, const int32_t *kind, const double *cen,
           const double *hw, const int32_t *row, const uint64_t *keys,
           const int32_t *order, const double *M, const double *gbar,
           double *L, const double *lbar) {
  // dX[g][a][a2] = xi^g_{t,a} - xi^g_{s,a2}, formed in FP64, rounded once
  __shared__ T dX[3][kQ][kQ];
  __shared__ T sM[kMaxM][4];
  __shared__ double wsum[kM2LThreads / kWave];
  double dsum = 0.0;
  const int t = sched_idx(order, 1, 1, false).node;
  if (t < 0 || kind[t] == 0) return;
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
              T inv3;
              if constexpr (DG) {
                const T z2 = g2 * (rz * rz), D = dxy + z2;
                inv3 = z2 * m2l_inv(D) / D;
              } else {
                inv3 = m2l_inv(dxy + g2 * (rz * rz));
              }
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
    if (act) {
      if constexpr (DG) {
        for (int k = 0; k < 6; ++k)
          dsum += acc[k] * lbar[((size_t)t * m + mu) * 6 + k];
      } else {
        for (int k = 0; k < 6; ++k) L[((size_t)t * m + mu) * 6 + k] = acc[k];
      }
    }
  }
  if constexpr (DG) {
    const double s = block_sum_m2l(dsum, wsum, kM2LThreads);
    if (threadIdx.x == 0) L[(size_t)t * kGdotStride] = s;
  }
}

// ---------------------------------------------------------------------------
// FP32 M2L on the matrix cores.
//
// With origin at the target centre c_t and xi' = xi - c_t, the M2L sums
// factor exactly into one scalar kernel matrix times ten source columns:
//   Phi[mu][nu] = D_{mu nu}^{-3/2},  D = dx^2 + dy^2 + gbar^2 dz^2,
//   W[nu] = (Mg, Mg xi'_s (3), Mu (3), Mu x xi'_s (3)),   C = sum_s Phi W,
//   E_mu = xi'_{t,mu} C0 - C[1..3],   B_mu = C[4..6] x xi'_{t,mu} - C[7..9].
// Phi is generated on the VALU and fed straight into v_mfma_f32_16x16x4f32 as
// the A operand; W (staged in LDS per pair) is the B operand.  Because proxies
// are tensor products, D = X[mu1][nu1] + Y[mu2][nu2] + Z[mu3][nu3] with three
// (p+1) x (p+1) tables of squared per-axis offsets (formed in FP64, rounded
// once).  The K dimension (source proxies) is ordered so that a lane keeps
// (nu1, nu2) fixed for p+1 consecutive steps: X + Y is formed once per block
// and each entry costs one add, one rsq and two multiplies.  Each pair's
// products are flushed from the FP32 accumulators into FP64 registers.
// ---------------------------------------------------------------------------

typedef float v4f __attribute__((ext_vector_type(4)));


// Launch shape of the FP32 kernel: 8 waves, TPW 16-row tiles per wave, as
// many row blocks as needed to cover the (p+1)^3 target proxies; the source
// cluster of the next pair is staged (second LDS buffer, its multipoles
// prefetched into registers one pair earlier) while the current one is
// multiplied, so each pair costs one barrier.
#ifndef RELFMM_M2L_WAVES
#define RELFMM_M2L_WAVES 8
#endif
#ifndef RELFMM_M2L_TPW
#define RELFMM_M2L_TPW 2
#endif
constexpr int kM2LWaves = RELFMM_M2L_WAVES;
constexpr int kM2LBlock = kM2LWaves * kWave;

template <int Q>
struct M2LShape {
  static constexpr int MM = Q * Q * Q;
  static constexpr int tiles = (MM + 15) / 16;
  static constexpr int tpw0 = (tiles + kM2LWaves - 1) / kM2LWaves;
  static constexpr int TPW = tpw0 < RELFMM_M2L_TPW ? tpw0 : RELFMM_M2L_TPW;
  static constexpr int rows = kM2LWaves * TPW * 16;
  static constexpr int blocks = (MM + rows - 1) / rows;
  static constexpr int KS = (MM + kM2LBlock - 1) / kM2LBlock;  // nu per thread
  static_assert(blocks <= kGdotStride, "partials per node of the gbar derivative");
};

// ADJ = false: output node o = target t, partner p = source s, partner data
//   M_s[nu][4], output L_t[mu][6] (the forward M2L above).
// ADJ = true: the transpose, grouped by source.  Output node o = source s,
//   partner p = target t of the source-grouped list, partner data the local
//   cotangents Lbar_t[mu][6] = (Ebar, Bbar), output Mbar_s[nu][4]:
//     Mbar^g_s[nu] = sum_t sum_mu g(xi_{t,mu} - xi_{s,nu}) . Ebar_t[mu],
//     Mbar^u_s[nu] = sum_t sum_mu g(xi_{t,mu} - xi_{s,nu}) x Bbar_t[mu].
//   With x = xi_{s,nu} - c_s and xi' = xi_{t,mu} - c_s the same Phi applies
//   to W = (xi'.Ebar, Ebar (3), xi' x Bbar (3), Bbar (3)), and
//     Mbar^g = C0 - x.C[1..3],   Mbar^u = C[4..6] - x x C[7..9].
// DG (forward only): Phi replaced by gbar^2 dz^2 D^{-5/2}; the output rows
// are dotted with the local cotangents lbar instead of stored, and the
// block's sum goes to out[t * kGdotStride + row block].
template <int Q, bool ADJ, bool DG = false, bool PIPE = false>
__global__ void __launch_bounds__(kM2LBlock)
k_m2l_mfma(Cheb cb, int bits, const int32_t *kind, const double *cen,
           const double *hw, const int32_t *row, const uint64_t *keys,
           const int32_t *order, const double *part, const double *gbar,
           double *out, const double *lbar, int grouped) {
  static_assert(!(ADJ && DG), "the gbar derivative runs on the forward form");
  constexpr int PC = ADJ ? 6 : 4;  // components of the partner data
  constexpr int OC = ADJ ? 4 : 6;  // components of the output
  using S = M2LShape<Q>;
  constexpr int QQ = Q * Q, MM = S::MM, TPW = S::TPW, KS = S::KS;
  constexpr int NBLK = (QQ + 3) / 4;
  constexpr int WC = 10;  // used columns of W
  constexpr int WSZ = MM * WC + 16;
  constexpr int CSZ = kM2LWaves * 16 * 17;  // epilogue tile per wave (doubles)
  // two W buffers (float) during the loop; the epilogue reuses them as double
  __shared__ double shbuf[(2 * WSZ + 1) / 2 > CSZ ? (2 * WSZ + 1) / 2 : CSZ];
  __shared__ float tab[2][3][Q][Q];
  __shared__ double wsum[kM2LWaves];
  float *Wb = reinterpret_cast<float *>(shbuf);
  const SchedIdx si = sched_idx(order, S::blocks, 1, grouped != 0);
  const int t = si.node, rblk = si.y;
  if (t < 0 || kind[t] == 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int g = lane >> 4, j = lane & 15;
  const double gbd = *gbar, gb2 = gbd * gbd;
  const uint64_t mask = (1ull << bits) - 1ull;
  const int r0 = row[t], r1 = row[t + 1];
  if (r0 == r1) {
    if constexpr (DG) {
      if (tid == 0) out[(size_t)t * kGdotStride + rblk] = 0.0;
      return;
    }
    // no partners: zero output for this row block
    for (int i = tid; i < S::rows; i += kM2LBlock) {
      const int mu = rblk * S::rows + i;
      if (mu < MM)
        for (int k = 0; k < OC; ++k) out[((size_t)t * MM + mu) * OC + k] = 0.0;
    }
    return;
  }
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  const double ht[3] = {hw[3 * t], hw[3 * t + 1], hw[3 * t + 2]};

  // this lane's A rows (target proxies) for its tiles
  const int row_base = rblk * S::rows + wave * TPW * 16;
  const bool wave_active = row_base < MM;
  int mu1[TPW], mu2[TPW], mu3[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int mu = min(row_base + 16 * k + j, MM - 1);
    mu1[k] = mu / QQ;
    mu2[k] = (mu / Q) % Q;
    mu3[k] = mu % Q;
  }
  double acc64[TPW][4];
#pragma unroll
  for (int k = 0; k < TPW; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc64[k][e] = 0.0;

  // staging of one source cluster into buffer b: W relative to the target
  // centre (FP64, rounded once) from prefetched multipoles, and the tables
  double pm[KS][PC];
  double pc[3], ph[3];
  auto prefetch = [&](int rr) {
    const int s = (int)(keys[rr] & mask);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pc[a] = cen[3 * s + a];
      ph[a] = hw[3 * s + a];
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int nu = tid + k * kM2LBlock;
      if (nu < MM) {
        const double *m4 = part + ((size_t)s * MM + nu) * PC;
#pragma unroll
        for (int c = 0; c < PC; ++c) pm[k][c] = m4[c];
      }
    }
  };
  auto stage = [&](int b) {
    for (int i = tid; i < 3 * QQ; i += kM2LBlock) {
      const int ax = i / QQ, a1 = (i / Q) % Q, a2 = i % Q;
      const double dd = (ct[ax] - pc[ax]) + (ht[ax] * cb.t[a1] - ph[ax] * cb.t[a2]);
      double v = dd * dd;
      if (ax == 2) v *= gb2;
      tab[b][ax][a1][a2] = (float)v;
    }
    float *W = Wb + b * WSZ;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int nu = tid + k * kM2LBlock;
      if (nu < MM) {
        const int n1 = nu / QQ, n2 = (nu / Q) % Q, n3 = nu % Q;
        const double xs = (pc[0] - ct[0]) + ph[0] * cb.t[n1];
        const double ys = (pc[1] - ct[1]) + ph[1] * cb.t[n2];
        const double zs = (pc[2] - ct[2]) + ph[2] * cb.t[n3];
        float *w = W + nu * WC;
        if constexpr (!ADJ) {
          const double mg = pm[k][0], ux = pm[k][1], uy = pm[k][2],
                       uz = pm[k][3];
          w[0] = (float)mg;
          w[1] = (float)(mg * xs);
          w[2] = (float)(mg * ys);
          w[3] = (float)(mg * zs);
          w[4] = (float)ux;
          w[5] = (float)uy;
          w[6] = (float)uz;
          w[7] = (float)(uy * zs - uz * ys);
          w[8] = (float)(uz * xs - ux * zs);
          w[9] = (float)(ux * ys - uy * xs);
        } else {
          const double ex = pm[k][0], ey = pm[k][1], ez = pm[k][2],
                       bx = pm[k][3], by = pm[k][4], bz = pm[k][5];
          w[0] = (float)(xs * ex + ys * ey + zs * ez);
          w[1] = (float)ex;
          w[2] = (float)ey;
          w[3] = (float)ez;
          w[4] = (float)(ys * bz - zs * by);
          w[5] = (float)(zs * bx - xs * bz);
          w[6] = (float)(xs * by - ys * bx);
          w[7] = (float)bx;
          w[8] = (float)by;
          w[9] = (float)bz;
        }
      }
    }
  };

  prefetch(r0);
  stage(0);
  if (r0 + 1 < r1) prefetch(r0 + 1);
  __syncthreads();
  for (int r = r0; r < r1; ++r) {
    const int b = (r - r0) & 1;
    if (wave_active) {
      const float *W = Wb + b * WSZ;
      float zrow[TPW][Q];
#pragma unroll
      for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int c = 0; c < Q; ++c) zrow[k][c] = tab[b][2][mu3[k]][c];
      v4f acc[TPW];
#pragma unroll
      for (int k = 0; k < TPW; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
      // lanes j >= 10 read a valid W column too: the output columns >= 10
      // are never used; K slots beyond (p+1)^2 get Phi = rsq(inf)^3 = 0
      const int jc = j < WC ? j : WC - 1;
      if constexpr (PIPE && Q <= 7) {
      // Phi of the next block of K slots is generated before the current
      // block's MFMAs are issued back to back (two register sets, the block
      // loop unrolled, scheduling barriers keep the order), so the VALU work
      // runs in the MFMAs' shadow.  The extra registers leave three waves
      // per SIMD at n = 6 instead of four: measured, that pays on small grids
      // (M2L -8 % on the 131k bunch, 2,048 workgroups) and costs on larger
      // ones (+8 % on the 262k bunch); launched only for small grids, and
      // never at n >= 7, where two waves per SIMD would remain.
      float ph[2][TPW][Q], bvp[2][Q];
      auto gen = [&](int bb, float (&p)[TPW][Q], float (&bv)[Q]) {
        const int n12 = 4 * bb + g;
        const bool ok = n12 < QQ;
        const int n1 = ok ? n12 / Q : 0, n2 = ok ? n12 % Q : 0;
        float xy[TPW];
#pragma unroll
        for (int k = 0; k < TPW; ++k)
          xy[k] = ok ? tab[b][0][mu1[k]][n1] + tab[b][1][mu2[k]][n2]
                     : __builtin_inff();
        const float *wrow = W + (ok ? n12 : 0) * Q * WC + jc;
#pragma unroll
        for (int c = 0; c < Q; ++c) bv[c] = wrow[c * WC];
#pragma unroll
        for (int c = 0; c < Q; ++c)
#pragma unroll
          for (int k = 0; k < TPW; ++k) {
            const float rs = __builtin_amdgcn_rsqf(xy[k] + zrow[k][c]);
            if constexpr (DG) {
              const float r2 = rs * rs;
              p[k][c] = zrow[k][c] * (r2 * r2 * rs);
            } else {
              p[k][c] = rs * rs * rs;
            }
          }
      };
      gen(0, ph[0], bvp[0]);
#pragma unroll
      for (int bb = 0; bb < NBLK; ++bb) {
        const int cur = bb & 1;
        if (bb + 1 < NBLK) gen(bb + 1, ph[cur ^ 1], bvp[cur ^ 1]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < Q; ++c)
#pragma unroll
          for (int k = 0; k < TPW; ++k)
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(ph[cur][k][c], bvp[cur][c],
                                                          acc[k], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      } else {
      for (int bb = 0; bb < NBLK; ++bb) {
        const int n12 = 4 * bb + g;
        const bool ok = n12 < QQ;
        const int n1 = ok ? n12 / Q : 0, n2 = ok ? n12 % Q : 0;
        float xy[TPW];
#pragma unroll
        for (int k = 0; k < TPW; ++k)
          xy[k] = ok ? tab[b][0][mu1[k]][n1] + tab[b][1][mu2[k]][n2]
                     : __builtin_inff();
        const float *wrow = W + (ok ? n12 : 0) * Q * WC + jc;
        float bvs[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) bvs[c] = wrow[c * WC];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          const float bv = bvs[c];
#pragma unroll
          for (int k = 0; k < TPW; ++k) {
            const float rs = __builtin_amdgcn_rsqf(xy[k] + zrow[k][c]);
            float phi;
            if constexpr (DG) {
              const float r2 = rs * rs;
              phi = zrow[k][c] * (r2 * r2 * rs);
            } else {
              phi = rs * rs * rs;
            }
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(phi, bv, acc[k], 0, 0, 0);
          }
        }
      }
      }
#pragma unroll
      for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc64[k][e] += (double)acc[k][e];
    }
    if (r + 1 < r1) {
      stage(b ^ 1);
      if (r + 2 < r1) prefetch(r + 2);
    }
    __syncthreads();
  }

  // Epilogue, one tile at a time in each wave's own LDS slot: C rows to LDS
  // (FP64), then one lane per target proxy row combines the ten columns.
  // Only lanes of the same wave exchange data here, so wave-level ordering
  // suffices.
  double *Cs = shbuf + wave * 16 * 17;  // [16 rows][17]
  double dsum = 0.0;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int rb = row_base + 16 * k;
    if (rb >= MM) break;  // wave-uniform
#pragma unroll
    for (int e = 0; e < 4; ++e) Cs[(4 * g + e) * 17 + j] = acc64[k][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16) {
      const int mu = rb + lane;
      if (mu < MM) {
        const double *C = Cs + lane * 17;
        const double x = ht[0] * cb.t[mu / QQ], y = ht[1] * cb.t[(mu / Q) % Q],
                     z = ht[2] * cb.t[mu % Q];
        if constexpr (DG) {
          const double *lb = lbar + ((size_t)t * MM + mu) * 6;
          dsum += lb[0] * (x * C[0] - C[1]) + lb[1] * (y * C[0] - C[2]) +
                  lb[2] * (z * C[0] - C[3]) +
                  lb[3] * ((C[5] * z - C[6] * y) - C[7]) +
                  lb[4] * ((C[6] * x - C[4] * z) - C[8]) +
                  lb[5] * ((C[4] * y - C[5] * x) - C[9]);
        } else if constexpr (!ADJ) {
          double *o = out + ((size_t)t * MM + mu) * OC;
          o[0] = x * C[0] - C[1];
          o[1] = y * C[0] - C[2];
          o[2] = z * C[0] - C[3];
          o[3] = (C[5] * z - C[6] * y) - C[7];
          o[4] = (C[6] * x - C[4] * z) - C[8];
          o[5] = (C[4] * y - C[5] * x) - C[9];
        } else {
          double *o = out + ((size_t)t * MM + mu) * OC;
          o[0] = C[0] - (x * C[1] + y * C[2] + z * C[3]);
          o[1] = C[4] - (y * C[9] - z * C[8]);
          o[2] = C[5] - (z * C[7] - x * C[9]);
          o[3] = C[6] - (x * C[8] - y * C[7]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if constexpr (DG) {
    // lanes 0..15 hold row sums; wave sums, then waves in order
    for (int o = 32; o > 0; o >>= 1) dsum += __shfl_xor(dsum, o);
    if (lane == 0) wsum[wave] = dsum;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kM2LWaves; ++w) s += wsum[w];
      out[(size_t)t * kGdotStride + rblk] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 M2L: the same factorization with bf16 operands and FP32 accumulation
// (v_mfma_f32_16x16x16_bf16), in the launch shape of the FP32 kernel.  Per
// pair, the squared-offset tables are scaled by 2^(2k) so that Phi comes out
// as D^{-3/2} 2^(-3k) ~ O(1) at the distance of the two centres, and each of
// the ten W columns is scaled by 2^(-e) with 2^e above a bound of the column's
// magnitude over the source cluster: |M| per component (max over the proxies,
// computed once per node) times |c_s - c_t| + h_s per axis for the columns
// that carry xi'.  The exact powers of two are undone when the FP32 products
// are flushed into FP64.  The K slots of one lane are four consecutive nu3 of
// one (nu1, nu2): nu3 is padded to a multiple of 4 with zero W entries.
// ---------------------------------------------------------------------------

typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// Four floats to bf16 (round to nearest even) as two packed conversions;
// element 2i goes to the low half of word i.
__device__ inline v4bf pack4_bf16(const float (&f)[4]) {
  const v2bf lo = __builtin_convertvector((v2f{f[0], f[1]}), v2bf);
  const v2bf hi = __builtin_convertvector((v2f{f[2], f[3]}), v2bf);
  v2u w;
  w[0] = __builtin_bit_cast(unsigned int, lo);
  w[1] = __builtin_bit_cast(unsigned int, hi);
  return __builtin_bit_cast(v4bf, w);
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Eight floats to bf16 (round to nearest even), element i in slot i.
__device__ inline v8bf pack8_bf16(const float (&f)[8]) {
  const float lo[4] = {f[0], f[1], f[2], f[3]}, hi[4] = {f[4], f[5], f[6], f[7]};
  return __builtin_shufflevector(pack4_bf16(lo), pack4_bf16(hi), 0, 1, 2, 3, 4,
                                 5, 6, 7);
}

constexpr int kMaxThreads = 256;

// mmax[s][c] = max over proxies nu of |M[s][nu][c]| (NC components: the
// multipoles of the forward M2L, or the local-field cotangents of its
// transpose)
template <int NC>
__global__ void __launch_bounds__(kMaxThreads)
k_mmax(int MM, const int32_t *kind, const double *M, double *mmax) {
  __shared__ double red[kMaxThreads / kWave][NC];
  const int s = blockIdx.x;
  if (kind[s] == 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  double m[NC];
  for (int c = 0; c < NC; ++c) m[c] = 0.0;
  for (int nu = tid; nu < MM; nu += kMaxThreads)
    for (int c = 0; c < NC; ++c)
      m[c] = fmax(m[c], fabs(M[((size_t)s * MM + nu) * NC + c]));
  for (int c = 0; c < NC; ++c) {
    for (int o = 32; o > 0; o >>= 1) m[c] = fmax(m[c], __shfl_xor(m[c], o));
    if (lane == 0) red[wave][c] = m[c];
  }
  __syncthreads();
  if (tid < NC) {
    double v = 0.0;
    for (int w = 0; w < kMaxThreads / kWave; ++w) v = fmax(v, red[w][tid]);
    mmax[NC * s + tid] = v;
  }
}

// e with v < 2^e for finite v > 0 (0 otherwise): the biased exponent of v
// less 1022, the exponent frexp gives for a normal v (a subnormal v gets
// -1022, still above it).
__device__ inline int pow2_exponent_above(double v) {
  if (!(v > 0.0)) return 0;
  return (int)((unsigned long long)__double_as_longlong(v) >> 52) - 1022;
}

// ADJ: the transpose, as in k_m2l_mfma (output node o = source s of the
// source-grouped list, partner data the local cotangents Lbar_t[mu][6] with
// their maxima per component in mmax, output Mbar_s[nu][4]); the column
// bounds of W = (xi'.Ebar, Ebar, xi' x Bbar, Bbar) follow from the same
// per-axis magnitudes of xi'.
template <int Q, bool SPLIT, bool ADJ = false>
__global__ void __launch_bounds__(kM2LBlock, 4)
k_m2l_bf16(Cheb cb, int bits, const int32_t *kind, const double *cen,
           const double *hw, const int32_t *row, const uint64_t *keys,
           const int32_t *order, const double *M, const double *mmax,
           const double *gbar, double *L, int grouped) {
  constexpr int PC = ADJ ? 6 : 4;  // components of the partner data
  constexpr int OC = ADJ ? 4 : 6;  // components of the output
  using S = M2LShape<Q>;
  constexpr int QQ = Q * Q, MM = S::MM, TPW = S::TPW, KS = S::KS;
  constexpr int QP = (Q + 3) / 4 * 4;  // nu3 padded to a multiple of 4
  constexpr int NBLK = (QQ + 3) / 4;
  constexpr int WC = 10;
  constexpr int WSZ = QQ * WC * QP;      // bf16 per buffer, [nu12][col][nu3]
  constexpr int NW = SPLIT ? 2 : 1;      // hi (and lo) parts of W
  constexpr int CSZ = kM2LWaves * 16 * 17;
  constexpr int WBYTES = 2 * NW * WSZ * 2;
  __shared__ double shbuf[(WBYTES + 7) / 8 > CSZ ? (WBYTES + 7) / 8 : CSZ];
  __shared__ float tab[2][3][Q][Q];
  __shared__ int scl[2][WC + 1];  // column exponents and the Phi exponent k
  __bf16 *Wb = reinterpret_cast<__bf16 *>(shbuf);
  const SchedIdx si = sched_idx(order, S::blocks, 1, grouped != 0);
  const int t = si.node, rblk = si.y;
  if (t < 0 || kind[t] == 0) return;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int g = lane >> 4, j = lane & 15;
  const double gbd = *gbar, gb2 = gbd * gbd;
  const uint64_t mask = (1ull << bits) - 1ull;
  const int r0 = row[t], r1 = row[t + 1];
  if (r0 == r1) {
    for (int i = tid; i < S::rows; i += kM2LBlock) {
      const int mu = rblk * S::rows + i;
      if (mu < MM)
        for (int k = 0; k < OC; ++k) L[((size_t)t * MM + mu) * OC + k] = 0.0;
    }
    return;
  }
  const double ct[3] = {cen[3 * t], cen[3 * t + 1], cen[3 * t + 2]};
  const double ht[3] = {hw[3 * t], hw[3 * t + 1], hw[3 * t + 2]};
  const int row_base = rblk * S::rows + wave * TPW * 16;
  const bool wave_active = row_base < MM;
  int mu1[TPW], mu2[TPW], mu3[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int mu = min(row_base + 16 * k + j, MM - 1);
    mu1[k] = mu / QQ;
    mu2[k] = (mu / Q) % Q;
    mu3[k] = mu % Q;
  }
  double acc64[TPW][4];
#pragma unroll
  for (int k = 0; k < TPW; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc64[k][e] = 0.0;
  // the padded nu3 slots stay zero in both buffers
  for (int i = tid; i < 2 * NW * QQ * WC; i += kM2LBlock)
    for (int n3 = Q; n3 < QP; ++n3) Wb[i * QP + n3] = (__bf16)0.0f;

  // the partner data of the next pair, prefetched in registers across the
  // current pair's loop: FP64 multipoles for the forward form; the six local
  // cotangents of the transpose are kept as FP32 (their W columns are split
  // to about 16 bits anyway), which keeps that form within 128 VGPRs
  using PT = typename std::conditional<ADJ, float, double>::type;
  PT pm[KS][PC];
  double pmax[PC];
  double pc[3], ph[3];
  auto prefetch = [&](int rr) {
    const int s = (int)(keys[rr] & mask);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      pc[a] = cen[3 * s + a];
      ph[a] = hw[3 * s + a];
    }
#pragma unroll
    for (int c = 0; c < PC; ++c) pmax[c] = mmax[PC * s + c];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int nu = tid + k * kM2LBlock;
      if (nu < MM) {
        const double *m4 = M + ((size_t)s * MM + nu) * PC;
#pragma unroll
        for (int c = 0; c < PC; ++c) pm[k][c] = (PT)m4[c];
      }
    }
  };
  auto stage = [&](int b) {
    const double del[3] = {pc[0] - ct[0], pc[1] - ct[1], pc[2] - ct[2]};
    // Phi scale: D_c = stretched squared distance of the centres
    const double dc = del[0] * del[0] + del[1] * del[1] + gb2 * del[2] * del[2];
    int edc;
    frexp(dc, &edc);
    const int kexp = (edc > 0 ? edc : edc - 1) / 2 * -1;  // 2^(2k) D_c ~ 1
    // column exponents from bounds of |W| over the cluster
    double ax[3];
    for (int a = 0; a < 3; ++a) ax[a] = fabs(del[a]) + ph[a];
    int e[WC];
    if constexpr (!ADJ) {
      e[0] = pow2_exponent_above(pmax[0]);
      for (int a = 0; a < 3; ++a) {
        e[1 + a] = pow2_exponent_above(pmax[0] * ax[a]);
        e[4 + a] = pow2_exponent_above(pmax[1 + a]);
      }
      e[7] = pow2_exponent_above(pmax[2] * ax[2] + pmax[3] * ax[1]);
      e[8] = pow2_exponent_above(pmax[3] * ax[0] + pmax[1] * ax[2]);
      e[9] = pow2_exponent_above(pmax[1] * ax[1] + pmax[2] * ax[0]);
    } else {
      // pmax = (|Ebar| and |Bbar| per axis)
      e[0] = pow2_exponent_above(ax[0] * pmax[0] + ax[1] * pmax[1] + ax[2] * pmax[2]);
      for (int a = 0; a < 3; ++a) {
        e[1 + a] = pow2_exponent_above(pmax[a]);
        e[7 + a] = pow2_exponent_above(pmax[3 + a]);
      }
      e[4] = pow2_exponent_above(ax[1] * pmax[5] + ax[2] * pmax[4]);
      e[5] = pow2_exponent_above(ax[2] * pmax[3] + ax[0] * pmax[5]);
      e[6] = pow2_exponent_above(ax[0] * pmax[4] + ax[1] * pmax[3]);
    }
    if (tid <= WC) scl[b][tid] = tid < WC ? e[tid] : kexp;
    for (int i = tid; i < 3 * QQ; i += kM2LBlock) {
      const int a = i / QQ, a1 = (i / Q) % Q, a2 = i % Q;
      const double dd = (ct[a] - pc[a]) + (ht[a] * cb.t[a1] - ph[a] * cb.t[a2]);
      double v = dd * dd;
      if (a == 2) v *= gb2;
      tab[b][a][a1][a2] = (float)ldexp(v, 2 * kexp);
    }
    __bf16 *W = Wb + b * NW * WSZ;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int nu = tid + k * kM2LBlock;
      if (nu < MM) {
        const int n1 = nu / QQ, n2 = (nu / Q) % Q, n3 = nu % Q;
        // the columns in FP32: their rounding (2^-24 of the column bound) is
        // far below the 2^-17 that the hi + lo bf16 pair keeps
        const float xs = (float)(del[0] + ph[0] * cb.t[n1]);
        const float ys = (float)(del[1] + ph[1] * cb.t[n2]);
        const float zs = (float)(del[2] + ph[2] * cb.t[n3]);
        float wv[WC];
        if constexpr (!ADJ) {
          const float mg = (float)pm[k][0], ux = (float)pm[k][1],
                      uy = (float)pm[k][2], uz = (float)pm[k][3];
          const float w0[WC] = {mg, mg * xs, mg * ys, mg * zs, ux, uy, uz,
                                uy * zs - uz * ys, uz * xs - ux * zs,
                                ux * ys - uy * xs};
#pragma unroll
          for (int c = 0; c < WC; ++c) wv[c] = w0[c];
        } else {
          const float ex = pm[k][0], ey = pm[k][1], ez = pm[k][2],
                      bx = pm[k][3], by = pm[k][4], bz = pm[k][5];
          const float w0[WC] = {xs * ex + ys * ey + zs * ez, ex, ey, ez,
                                ys * bz - zs * by, zs * bx - xs * bz,
                                xs * by - ys * bx, bx, by, bz};
#pragma unroll
          for (int c = 0; c < WC; ++c) wv[c] = w0[c];
        }
        __bf16 *w = W + (n1 * Q + n2) * WC * QP + n3;
#pragma unroll
        for (int c = 0; c < WC; ++c) {
          const float v = ldexpf(wv[c], -e[c]);
          const __bf16 hv = (__bf16)v;
          w[c * QP] = hv;
          if constexpr (SPLIT) w[WSZ + c * QP] = (__bf16)(v - (float)hv);
        }
      }
    }
  };

  prefetch(r0);
  stage(0);
  if (r0 + 1 < r1) prefetch(r0 + 1);
  __syncthreads();
  const int jc = j < WC ? j : WC - 1;
  for (int r = r0; r < r1; ++r) {
    const int b = (r - r0) & 1;
    if (wave_active) {
      const __bf16 *W = Wb + b * NW * WSZ;
      float zrow[TPW][QP];
#pragma unroll
      for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int c = 0; c < QP; ++c) zrow[k][c] = tab[b][2][mu3[k]][c < Q ? c : Q - 1];
      v4f acc[TPW];
#pragma unroll
      for (int k = 0; k < TPW; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
      for (int bb = 0; bb < NBLK; ++bb) {
        const int n12 = 4 * bb + g;
        const bool ok = n12 < QQ;
        const int n1 = ok ? n12 / Q : 0, n2 = ok ? n12 % Q : 0;
        float xy[TPW];
#pragma unroll
        for (int k = 0; k < TPW; ++k)
          xy[k] = ok ? tab[b][0][mu1[k]][n1] + tab[b][1][mu2[k]][n2]
                     : __builtin_inff();
        const __bf16 *wp = W + ((ok ? n12 : 0) * WC + jc) * QP;
        v4bf bvs[QP / 4], bls[QP / 4];
#pragma unroll
        for (int c4 = 0; c4 < QP / 4; ++c4) {
          bvs[c4] = *reinterpret_cast<const v4bf *>(wp + 4 * c4);
          if constexpr (SPLIT)
            bls[c4] = *reinterpret_cast<const v4bf *>(wp + WSZ + 4 * c4);
        }
        // nu3 in slices of eight on the K = 32 instruction (which takes the
        // cycles of the K = 16 one for twice the products), a last slice of
        // four on the K = 16 instruction
#pragma unroll
        for (int c8 = 0; c8 < QP / 8; ++c8) {
          const v8bf bv8 = __builtin_shufflevector(bvs[2 * c8], bvs[2 * c8 + 1],
                                                   0, 1, 2, 3, 4, 5, 6, 7);
          v8bf bl8;
          if constexpr (SPLIT)
            bl8 = __builtin_shufflevector(bls[2 * c8], bls[2 * c8 + 1], 0, 1,
                                          2, 3, 4, 5, 6, 7);
#pragma unroll
          for (int k = 0; k < TPW; ++k) {
            float phi[8];
#pragma unroll
            for (int i2 = 0; i2 < 8; ++i2) {
              const float rs = __builtin_amdgcn_rsqf(xy[k] + zrow[k][8 * c8 + i2]);
              phi[i2] = rs * rs * rs;
            }
            const v8bf av = pack8_bf16(phi);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv8, acc[k], 0,
                                                             0, 0);
            if constexpr (SPLIT) {
              // phi = hi + lo: the low parts from the rounding residuals
              float res[8];
#pragma unroll
              for (int i2 = 0; i2 < 8; ++i2) res[i2] = phi[i2] - (float)av[i2];
              const v8bf al = pack8_bf16(res);
              acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl8, acc[k],
                                                               0, 0, 0);
              acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bv8, acc[k],
                                                               0, 0, 0);
            }
          }
        }
        if constexpr (QP % 8 != 0) {
          constexpr int c4 = QP / 4 - 1;
#pragma unroll
          for (int k = 0; k < TPW; ++k) {
            float phi[4];
#pragma unroll
            for (int i2 = 0; i2 < 4; ++i2) {
              const float rs = __builtin_amdgcn_rsqf(xy[k] + zrow[k][4 * c4 + i2]);
              phi[i2] = rs * rs * rs;
            }
            const v4bf av = pack4_bf16(phi);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bvs[c4],
                                                               acc[k], 0, 0, 0);
            if constexpr (SPLIT) {
              float res[4];
#pragma unroll
              for (int i2 = 0; i2 < 4; ++i2) res[i2] = phi[i2] - (float)av[i2];
              const v4bf al = pack4_bf16(res);
              acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bls[c4],
                                                                 acc[k], 0, 0, 0);
              acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bvs[c4],
                                                                 acc[k], 0, 0, 0);
            }
          }
        }
      }
      // undo the scales: Phi carried 2^(-3k), column j carried 2^(-e_j)
      const int ej = scl[b][jc] + 3 * scl[b][WC];
#pragma unroll
      for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc64[k][e] += ldexp((double)acc[k][e], ej);
    }
    if (r + 1 < r1) {
      stage(b ^ 1);
      if (r + 2 < r1) prefetch(r + 2);
    }
    __syncthreads();
  }

  double *Cs = shbuf + wave * 16 * 17;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int rb = row_base + 16 * k;
    if (rb >= MM) break;  // wave-uniform
#pragma unroll
    for (int e = 0; e < 4; ++e) Cs[(4 * g + e) * 17 + j] = acc64[k][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16) {
      const int mu = rb + lane;
      if (mu < MM) {
        const double *C = Cs + lane * 17;
        const double x = ht[0] * cb.t[mu / QQ], y = ht[1] * cb.t[(mu / Q) % Q],
                     z = ht[2] * cb.t[mu % Q];
        double *o = L + ((size_t)t * MM + mu) * OC;
        if constexpr (!ADJ) {
          o[0] = x * C[0] - C[1];
          o[1] = y * C[0] - C[2];
          o[2] = z * C[0] - C[3];
          o[3] = (C[5] * z - C[6] * y) - C[7];
          o[4] = (C[6] * x - C[4] * z) - C[8];
          o[5] = (C[4] * y - C[5] * x) - C[9];
        } else {
          o[0] = C[0] - (x * C[1] + y * C[2] + z * C[3]);
          o[1] = C[4] - (y * C[9] - z * C[8]);
          o[2] = C[5] - (z * C[7] - x * C[9]);
          o[3] = C[6] - (x * C[8] - y * C[7]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// The software-pipelined FP32 form (n <= 6) for grids of at most 2,048
// workgroups.
template <int Q>
static bool m2l_pipelined(const M2LArgs &a) {
  return Q <= 7 && (int64_t)a.ns * M2LShape<Q>::blocks <= 2048;
}

template <int Q>
static void launch_mfma_q(const Dev &d, const Cheb &cb, const M2LArgs &a,
                          hipStream_t st) {
  constexpr int MM = Q * Q * Q;
  const int g = m2l_grouped(a.ns, Q - 1) ? 1 : 0;
  if (a.prec == 2 || a.prec == 3) {
    hipLaunchKernelGGL(k_mmax<4>, dim3(a.ns), dim3(kMaxThreads), 0, st, MM,
                       d.kind, d.M, d.mmax);
    const dim3 grid(order_len(a.ns) * M2LShape<Q>::blocks);
    if (a.prec == 2)
      hipLaunchKernelGGL((k_m2l_bf16<Q, false>), grid, dim3(kM2LBlock), 0, st,
                         cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row, d.m2l,
                         d.order_m2l, d.M, d.mmax, d.gbar, d.L, g);
    else
      hipLaunchKernelGGL((k_m2l_bf16<Q, true>), grid, dim3(kM2LBlock), 0, st,
                         cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row, d.m2l,
                         d.order_m2l, d.M, d.mmax, d.gbar, d.L, g);
  } else {
    const dim3 grid(order_len(a.ns) * M2LShape<Q>::blocks);
    if (m2l_pipelined<Q>(a))
      hipLaunchKernelGGL((k_m2l_mfma<Q, false, false, true>), grid,
                         dim3(kM2LBlock), 0, st, cb, a.bits, d.kind, d.cen,
                         d.hw, d.m2l_row, d.m2l, d.order_m2l, d.M, d.gbar, d.L,
                         nullptr, g);
    else
      hipLaunchKernelGGL((k_m2l_mfma<Q, false>), grid, dim3(kM2LBlock), 0, st,
                         cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row, d.m2l,
                         d.order_m2l, d.M, d.gbar, d.L, nullptr, g);
  }
}

template <int Q>
static void launch_mfma_adj_q(const Dev &d, const Cheb &cb, const M2LArgs &a,
                              hipStream_t st) {
  const int g = m2l_grouped(a.ns, Q - 1) ? 1 : 0;
  const dim3 grid(order_len(a.ns) * M2LShape<Q>::blocks);
  if (a.prec == 2 || a.prec == 3) {
    constexpr int MM = Q * Q * Q;
    hipLaunchKernelGGL(k_mmax<6>, dim3(a.ns), dim3(kMaxThreads), 0, st, MM,
                       d.kind, d.Lbar, d.lmax);
    if (a.prec == 2)
      hipLaunchKernelGGL((k_m2l_bf16<Q, false, true>), grid, dim3(kM2LBlock),
                         0, st, cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row_T,
                         d.m2l_T, d.order_m2l_T, d.Lbar, d.lmax, d.gbar, d.Mbar,
                         g);
    else
      hipLaunchKernelGGL((k_m2l_bf16<Q, true, true>), grid, dim3(kM2LBlock), 0,
                         st, cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row_T,
                         d.m2l_T, d.order_m2l_T, d.Lbar, d.lmax, d.gbar, d.Mbar,
                         g);
    return;
  }
  if (m2l_pipelined<Q>(a))
    hipLaunchKernelGGL((k_m2l_mfma<Q, true, false, true>), grid,
                       dim3(kM2LBlock), 0, st, cb, a.bits, d.kind, d.cen, d.hw,
                       d.m2l_row_T, d.m2l_T, d.order_m2l_T, d.Lbar, d.gbar,
                       d.Mbar, nullptr, g);
  else
    hipLaunchKernelGGL((k_m2l_mfma<Q, true>), grid, dim3(kM2LBlock), 0, st, cb,
                       a.bits, d.kind, d.cen, d.hw, d.m2l_row_T, d.m2l_T,
                       d.order_m2l_T, d.Lbar, d.gbar, d.Mbar, nullptr, g);
}

template <int Q>
static int launch_mfma_dg_q(const Dev &d, const Cheb &cb, const M2LArgs &a,
                            hipStream_t st) {
  const int g = m2l_grouped(a.ns, Q - 1) ? 1 : 0;
  const dim3 grid(order_len(a.ns) * M2LShape<Q>::blocks);
  if (m2l_pipelined<Q>(a))
    hipLaunchKernelGGL((k_m2l_mfma<Q, false, true, true>), grid,
                       dim3(kM2LBlock), 0, st, cb, a.bits, d.kind, d.cen, d.hw,
                       d.m2l_row, d.m2l, d.order_m2l, d.M, d.gbar, d.gdot,
                       d.Lbar, g);
  else
    hipLaunchKernelGGL((k_m2l_mfma<Q, false, true>), grid, dim3(kM2LBlock), 0,
                       st, cb, a.bits, d.kind, d.cen, d.hw, d.m2l_row, d.m2l,
                       d.order_m2l, d.M, d.gbar, d.gdot, d.Lbar, g);
  return M2LShape<Q>::blocks;
}

// gbar derivative of the far field dotted with the local cotangents, per
// node (needs M and Lbar): FP64 on the VALU for an FP64 plan, else the FP32
// MFMA form.  Returns the number of partial sums per node.
int launch_m2l_dgbar(const Dev &d, const Cheb &cb, const M2LArgs &a,
                     hipStream_t st) {
  if (a.prec == 0) {
    hipLaunchKernelGGL((k_m2l_valu<double, true>), dim3(order_len(a.ns)),
                       dim3(kM2LThreads), 0, st, cb, a.bits, d.kind, d.cen,
                       d.hw, d.m2l_row, d.m2l, d.order_m2l, d.M, d.gbar,
                       d.gdot, d.Lbar);
    return 1;
  }
  switch (cb.p + 1) {
    case 2: return launch_mfma_dg_q<2>(d, cb, a, st);
    case 3: return launch_mfma_dg_q<3>(d, cb, a, st);
    case 4: return launch_mfma_dg_q<4>(d, cb, a, st);
    case 5: return launch_mfma_dg_q<5>(d, cb, a, st);
    case 6: return launch_mfma_dg_q<6>(d, cb, a, st);
    case 7: return launch_mfma_dg_q<7>(d, cb, a, st);
    case 8: return launch_mfma_dg_q<8>(d, cb, a, st);
    case 9: return launch_mfma_dg_q<9>(d, cb, a, st);
    case 10: return launch_mfma_dg_q<10>(d, cb, a, st);
    default: return launch_mfma_dg_q<11>(d, cb, a, st);
  }
}

// M2L^T on the matrix cores (FP32 operands, FP64 flush), grouped by source.
void launch_m2l_adjoint_mfma(const Dev &d, const Cheb &cb, const M2LArgs &a,
                             hipStream_t st) {
  switch (cb.p + 1) {
    case 2: launch_mfma_adj_q<2>(d, cb, a, st); break;
    case 3: launch_mfma_adj_q<3>(d, cb, a, st); break;
    case 4: launch_mfma_adj_q<4>(d, cb, a, st); break;
    case 5: launch_mfma_adj_q<5>(d, cb, a, st); break;
    case 6: launch_mfma_adj_q<6>(d, cb, a, st); break;
    case 7: launch_mfma_adj_q<7>(d, cb, a, st); break;
    case 8: launch_mfma_adj_q<8>(d, cb, a, st); break;
    case 9: launch_mfma_adj_q<9>(d, cb, a, st); break;
    case 10: launch_mfma_adj_q<10>(d, cb, a, st); break;
    default: launch_mfma_adj_q<11>(d, cb, a, st); break;
  }
}

void launch_m2l(const Dev &d, const Cheb &cb, const M2LArgs &a,
                hipStream_t st) {
  const dim3 grid(order_len(a.ns)), block(kM2LThreads);
  if (a.prec == 0) {
    hipLaunchKernelGGL((k_m2l_valu<double, false>), grid, block, 0, st, cb,
                       a.bits, d.kind, d.cen, d.hw, d.m2l_row, d.m2l,
                       d.order_m2l, d.M, d.gbar, d.L, nullptr);
    return;
  }
  switch (cb.p + 1) {
    case 2: launch_mfma_q<2>(d, cb, a, st); break;
    case 3: launch_mfma_q<3>(d, cb, a, st); break;
    case 4: launch_mfma_q<4>(d, cb, a, st); break;
    case 5: launch_mfma_q<5>(d, cb, a, st); break;
    case 6: launch_mfma_q<6>(d, cb, a, st); break;
    case 7: launch_mfma_q<7>(d, cb, a, st); break;
    case 8: launch_mfma_q<8>(d, cb, a, st); break;
    case 9: launch_mfma_q<9>(d, cb, a, st); break;
    case 10: launch_mfma_q<10>(d, cb, a, st); break;
    default: launch_mfma_q<11>(d, cb, a, st); break;
  }
}

}  // namespace relfmm
