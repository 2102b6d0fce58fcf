// Internal declarations of the relfmm HIP library: device-array bundle and
// host-side launchers implemented in the per-stage .hip files.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace relfmm {

// Most parts a P2P list row is split into when the grid is small (each part
// sums into its own near-field buffer; the parts are added in a fixed order).
#ifndef RELFMM_P2P_MAXSPLIT
#define RELFMM_P2P_MAXSPLIT 8
#endif
constexpr int kP2PMaxSplit = RELFMM_P2P_MAXSPLIT;

// All device arrays live in the caller's workspace.  Particle arrays are in
// leaf order (position p in the final permutation) unless noted.
struct Dev {
  // scalars and counters
  double *gbar;     // [1] mean Lorentz factor
  double *gpart;    // [3 * kGammaBlocks] partial momentum sums
  int *counters;    // [kCounters]
  unsigned long long *inter;  // [1] sum over p2p pairs of |t||s|
  // tree build scratch
  uint64_t *key, *key_tmp;    // [3 * n_max]
  uint32_t *ord_all;          // [3][n] particle ids sorted by each axis; the
                              // first n entries are the leaf-order permutation
  uint32_t *ord_tmp_all;      // [3][n]
  uint8_t *flag;              // [n_max] per particle: goes to the left child
  uint32_t *scanv;            // [3 * n_max] exclusive scans of the flags
  int32_t *seg, *seg_tmp;     // [n_max] node owning each position
  uint32_t *hist;             // radix histograms
  uint32_t *partial;          // scan partial sums
  // nodes [ns_max]
  int32_t *lo, *hi, *kind, *axis, *nleft;
  double *bmin, *bmax, *cen, *hw;  // [3 * ns_max]
  double *r2;                      // [ns_max] stretched half-diagonal^2
  // leaf-order particle data
  double *xl;     // [3][n_max] x - centre of the leaf (fp64)
  double *w;      // [4][n_max] (q gamma, q u)
  double *us;     // [3][n_max] u (for the per-source kernel)
  float *w32, *us32;       // FP32 copies of w and us
  double *near;   // [near_cap / (6 n)][6][n] P2P part of (E, B); the
                  // rest holds the later row parts of split P2P and P2P^T
                  // launches until they are added
  size_t near_cap;  // doubles in near
  double *sbox;     // [ns_max][kslices][6] boxes of the 64-particle slices
                    // of the leaves (FP32 P2P separation test)
  // interaction lists
  int2 *front[2];           // [fcap]
  uint64_t *p2p, *p2p_tmp;  // [p2p_cap] key (t << bits) | s
  uint64_t *m2l, *m2l_tmp;  // [m2l_cap]
  int32_t *p2p_row, *m2l_row;  // [ns_max + 1]
  int32_t *lfill;              // [2][ns_max + 1] per-row counters (grouping)
  // node orders of the list-driven kernels (sched_idx layout, longest rows
  // first within each XCD's eighth of the tree)
  int32_t *order_p2p, *order_m2l;      // [order_len(ns_max)]
  uint64_t *okey, *okey_tmp;           // [ns_max] sort scratch
  // expansions
  double *M;  // [ns_max][m][4]
  double *mmax;  // [ns_max][4] max over proxies of |M| per component
  double *L;  // [ns_max][m][6]
  // adjoint
  uint64_t *p2p_T, *m2l_T;       // lists keyed (s << bits) | t, sorted
  int32_t *p2p_row_T, *m2l_row_T;  // start offsets per source
  int32_t *order_p2p_T, *order_m2l_T;  // the same for the source-grouped lists
  double *ebar;    // [6][n_max] (ke gE, kb gB) in leaf order
  float *ebar32;   // [6][n_max]
  double *Lbar;    // [ns_max][m][6] cotangents of the local fields
  double *lmax;    // [ns_max][6] max over proxies of |Lbar| per component
  double *Mbar;    // [ns_max][m][4] cotangents of the multipoles (aliases M)
  double *gx;      // [3][n_max] position gradient in leaf order
  double *mbar;    // [4][n_max] cotangents of the particle weights
  // momentum gradient
  double *gu;      // [3][n_max] per-source denominator term (leaf order)
  double *gG;      // [n_max] near-field gbar derivative per target
  double *gdot;    // [ns_max][kGdotStride] far-field gbar derivative partials
  double *gspart;  // [kGsBlocks][5] stage-1 sums
  double *gsum;    // [4] dL/dgbar, dgbar/du
};

enum {
  kCntFront = 0,   // [0, 64): frontier size per traversal iteration
  kCntP2P = 64,
  kCntM2L = 65,
  kCntOverflow = 66,
  kCounters = 80
};
constexpr int kGammaBlocks = 256;
constexpr int kGdotStride = 8;  // >= row blocks of any M2L launch shape
constexpr int kGsBlocks = 512;

// Length of a node-order array (sched_idx layout): the node slots, rounded up
// to whole slices of eight.
inline int order_len(int ns) { return ((ns + kXcds - 1) / kXcds) * kXcds; }

// sort.hip
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int n,
                        uint32_t *partial, hipStream_t st);
int scan_blocks(int n);
size_t radix_hist_entries(int n_max);
// Sorts nseg arrays of n (key, value) pairs stored back to back by key, then
// value (a strict order for distinct values); ktmp / vtmp: scratch of the
// same size.
void merge_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *ktmp,
                      uint32_t *vtmp, int n, int nseg, hipStream_t st);
// Sorts nseg arrays of length n stored back to back (keys[nseg][n]) by bits
// [bit_lo, bit_hi) of the keys, stably, carrying vals when non-NULL.
void radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *ktmp, uint32_t *vtmp,
                int n, int bit_lo, int bit_hi, uint32_t *hist,
                uint32_t *partial, hipStream_t st, int nseg = 1,
                const int *count = nullptr);

// tree.hip
struct TreeArgs {
  int n, depth, leaf_size, ns;
  double given_gbar;  // > 0: use as gamma_bar
};
void build_tree_dev(const Dev &d, const TreeArgs &a, const double *x,
                    const double *u, hipStream_t st);
void prep_leaf_order(const Dev &d, int n, int ns, const double *x,
                     const double *u, const double *q, bool need_fp32,
                     hipStream_t st);

// itl.hip
struct ListArgs {
  int ns, depth, bits;
  int fcap, p2p_cap, m2l_cap;
  double eta;
  int p2p_spatial;  // P2P order by XCD regions (large unsplit grids)
  int m2l_spatial;  // the same for M2L (m2l_grouped)
};
void count_interactions_dev(const Dev &d, const ListArgs &a, hipStream_t st);
void build_lists_dev(const Dev &d, const ListArgs &a, hipStream_t st);
// Source-grouped copies of both lists, for the adjoint.
void build_transposed_lists_dev(const Dev &d, const ListArgs &a,
                                hipStream_t st);

// upward.hip
void launch_p2m(const Dev &d, const Cheb &cb, int n, int ns, hipStream_t st);
void launch_m2m_level(const Dev &d, const Cheb &cb, int level, hipStream_t st);
void launch_l2p_transpose(const Dev &d, const Cheb &cb, int n, int ns,
                          hipStream_t st);
void launch_l2l_transpose_level(const Dev &d, const Cheb &cb, int level,
                                hipStream_t st);

// p2p.hip
struct P2PArgs {
  int ns, bits, mode, prec, max_leaf;
};
void launch_p2p(const Dev &d, const P2PArgs &a, int n, hipStream_t st);

// m2l.hip
// The matrix-core M2L kernels take rows of 256 target proxies per workgroup
// (one block when there are at most 128).  A node's row blocks run grouped
// on one XCD, and the M2L order takes XCD regions, when the grid is large
// (4,096 node slots or more) and the last block is at least half full.
inline bool m2l_grouped(int ns, int degree) {
  const int m = (degree + 1) * (degree + 1) * (degree + 1);
  const int blocks = m <= 128 ? 1 : (m + 255) / 256;
  return ns >= 4096 && blocks >= 2 && 2 * (m - 256 * (blocks - 1)) >= 256;
}
struct M2LArgs {
  int ns, bits, prec;
};
void launch_m2l(const Dev &d, const Cheb &cb, const M2LArgs &a,
                hipStream_t st);
int launch_m2l_dgbar(const Dev &d, const Cheb &cb, const M2LArgs &a,
                     hipStream_t st);

// downward.hip
void launch_l2l_level(const Dev &d, const Cheb &cb, int level, hipStream_t st);
void launch_l2p_finalize(const Dev &d, const Cheb &cb, int n, int ns,
                         int max_leaf, double ke, double kb, double *E,
                         double *B, hipStream_t st);

void launch_m2m_transpose_level(const Dev &d, const Cheb &cb, int level,
                                hipStream_t st);

// adjoint.hip
void launch_adj_prep(const Dev &d, int n, const double *gE, const double *gB,
                     double ke, double kb, hipStream_t st);
void launch_m2l_adjoint_mfma(const Dev &d, const Cheb &cb, const M2LArgs &a,
                             hipStream_t st);
void launch_m2l_adjoint(const Dev &d, const Cheb &cb, const M2LArgs &a,
                        hipStream_t st);
void launch_adj_leaf(const Dev &d, const Cheb &cb, int n, int ns, int max_leaf,
                     hipStream_t st);
void launch_p2p_adjoint(const Dev &d, const P2PArgs &a, int n, bool gb,
                        bool gu, hipStream_t st);
void launch_gbar_sums(const Dev &d, int n, int ns, int nblk, bool near,
                      hipStream_t st);
void launch_adj_final(const Dev &d, int n, double *grad_x, double *grad_q,
                      hipStream_t st);
void launch_adj_final_u(const Dev &d, int n, bool gu, bool gs, double *grad_u,
                        hipStream_t st);

// direct.hip
void launch_direct(int n, const double *x, const double *u, const double *q,
                   int nt, const int64_t *tgt, int kernel, double gb,
                   double ke, double kb, double *E, double *B, hipStream_t st);

}  // namespace relfmm
