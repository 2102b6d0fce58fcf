/*
 * relfmm.h -- C-ABI of the MI355X (gfx950) library for the lab-frame,
 * interpolation-based FMM of the relativistic space-charge field
 * (Kan, Kaertner, Le Borne, Zemke, arXiv 2302.07567).
 *
 * The library computes, for N macro-particles with positions x_i, momenta
 * u_i = gamma_i beta_i and charges q_i, the fields
 *   E_i = ke   * sum_{j != i} q_j gamma_j g(x_i, x_j)
 *   B_i = ke/c0 * sum_{j != i} q_j u_j x g(x_i, x_j)
 * of eq. (fmm_pp_force_field) in Sec. 3, with the FMM of Alg. FMM (Sec. 5):
 * a cardinality-balanced k-d tree split along the longest stretched side
 * (Alg. direction4split / subdivide, App. B), P2M/M2M upward pass, a dual
 * tree traversal under the stretched admissibility condition
 * (eq. fmm_stretched_admc, Alg. diam/dist/admissible) producing P2P and M2L
 * interaction lists (Alg. dualtraversefillitl), target-grouped P2P and M2L
 * (Sec. 10), and the L2L/L2P downward pass.
 *
 * Conventions for every entry point:
 *  - Particle arrays are DEVICE pointers owned by the caller.  x, u, E, B,
 *    grad arrays are n x 3 row-major contiguous float64; q is n float64.
 *  - All work is enqueued on the plan's HIP stream; calls do not
 *    synchronize except relfmm_get_stats and relfmm_export.
 *  - Device memory is the caller's workspace; the library allocates no
 *    device memory.  The plan object owns host metadata only.  (The one
 *    exception, relfmm_compute_fields_static, works in a fixed device array
 *    of the library instead.)
 *  - Errors are returned as relfmm_status; the message is available from
 *    relfmm_last_error() (thread-local, valid until the next call on that
 *    thread).  No C++ exception crosses this boundary.  Arguments are
 *    validated before anything is enqueued.  Asynchronous device faults are
 *    reported by a later call as RELFMM_EDEVICE.
 *  - Interaction lists have a capacity (relfmm_params.max_p2p_per_leaf,
 *    max_m2l_per_node).  A build whose lists overflow it writes NaN to every
 *    field and gradient computed on that structure.  Its flag is copied to
 *    host memory after the lists are built and read by the next call on the
 *    plan, which waits for that copy: that call (whatever it is) returns
 *    RELFMM_ECAPACITY and enqueues nothing; calls that reuse the structure
 *    (rebuild = 0) keep returning it until the next build; relfmm_get_stats
 *    returns it as well.
 *  - Preconditions that are not checked: finite inputs, and distinct
 *    positions (two particles at one point divide by zero, as the pair field
 *    itself does).
 */
#ifndef RELFMM_H
#define RELFMM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define RELFMM_API __attribute__((visibility("default")))
#else
#define RELFMM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct relfmm_plan relfmm_plan;

typedef enum {
  RELFMM_OK = 0,
  RELFMM_EINVAL = 1,    /* invalid argument or parameter */
  RELFMM_ECAPACITY = 2, /* n > n_max, workspace too small, or an interaction
                           list overflowed its capacity (raise the caps) */
  RELFMM_EDEVICE = 3,   /* HIP runtime error or device fault */
  RELFMM_ESTATE = 4     /* call out of order (e.g. rebuild=0 with no tree) */
} relfmm_status;

/* Pair kernel used by P2P (Alg. P2P).  The far field (M2L) always uses the
 * mean kernel of eq. (fmm_relativistic_kernel), since its proxies cannot
 * carry per-source momenta. */
typedef enum {
  RELFMM_KERNEL_MEAN = 0,  /* g = r / (rx^2 + ry^2 + gbar^2 rz^2)^{3/2}     */
  RELFMM_KERNEL_SOURCE = 1 /* g = r / (|r|^2 + (u_j . r)^2)^{3/2}: the field
                              of a uniformly moving source, per-source u_j */
} relfmm_kernel;

typedef enum {
  RELFMM_FP64 = 0,
  RELFMM_FP32 = 1,
  RELFMM_BF16 = 2,  /* M2L only: bf16 operands, fp32 accumulation        */
  RELFMM_BF16X3 = 3 /* M2L only: each operand split into two bf16 terms
                       (hi + lo, 16 significant bits), three bf16 products
                       (hi hi + hi lo + lo hi), fp32 accumulation         */
} relfmm_prec;

typedef struct {
  int32_t degree;    /* interpolation degree n, 1..10; (n+1)^3 proxies per
                        cluster (Sec. 2, Sec. 6)                            */
  int32_t leaf_size; /* N0 >= 1: max particles per leaf (Alg. subdivide)   */
  double eta;        /* admissibility parameter > 0 (eq. fmm_stretched_admc)*/
  double gamma_bar;  /* > 0: mean Lorentz factor to use; <= 0: computed from
                        the unweighted mean momentum (Sec. 3)               */
  int32_t kernel;    /* relfmm_kernel for P2P                               */
  int32_t p2p_prec;  /* RELFMM_FP64 or RELFMM_FP32                          */
  int32_t m2l_prec;  /* RELFMM_FP64, RELFMM_FP32, RELFMM_BF16 or
                        RELFMM_BF16X3; the reduced-precision tiers are
                        specified for eta <= 0.5 (their rounding error grows
                        with eta above that): with eta > 0.5 only
                        RELFMM_FP64 is accepted, else RELFMM_EINVAL.  The
                        FP32 and BF16 tiers of both operators carry the
                        weights q gamma, q u and the multipoles (formed in
                        FP64) as FP32 values, so these must lie within
                        FP32's normal range (about 1e-38 to 3e38), as SI
                        charges of particle bunches do by many decades.  */
  int32_t max_p2p_per_leaf; /* list capacity per leaf; <= 0: default 1024  */
  int32_t max_m2l_per_node; /* list capacity per node; <= 0: default 256   */
  int32_t reserved;
  double ke; /* E prefactor, 1/(4 pi eps0); <= 0: SI value with
                eps0 = 8.8541878128e-12 F/m                                  */
  double c0; /* speed of light for B = ke/c0 ...; <= 0: 299792458 m/s       */
} relfmm_params;

typedef struct {
  int64_t n;                /* particles of the last build                  */
  int32_t depth;            /* tree depth kappa (Sec. 8)                    */
  int32_t overflow;         /* nonzero if a list overflowed its capacity    */
  int64_t n_nodes;          /* node slots 2^(kappa+1), index 0 unused       */
  int64_t n_p2p_pairs;      /* |p2p_itl|                                    */
  int64_t n_m2l_pairs;      /* |m2l_itl|                                    */
  int64_t p2p_interactions; /* sum over p2p pairs of |t||s| (incl. i = j)   */
  int64_t m2l_entries;      /* |m2l_itl| * ((n+1)^3)^2                      */
  double gamma_bar;         /* mean Lorentz factor used                     */
} relfmm_stats;

/* Bytes of device workspace a plan for up to n_max particles needs
 * (1 <= n_max <= 2^28). Host only, pure; returns 0 for invalid parameters. */
RELFMM_API size_t relfmm_workspace_bytes(const relfmm_params *params, int64_t n_max);

/* Create a plan.  workspace: device buffer of at least
 * relfmm_workspace_bytes(params, n_max) bytes, 256-byte aligned, owned by
 * the caller and kept alive until relfmm_plan_destroy.  stream: hipStream_t
 * (NULL = default stream).  The device is the current HIP device. */
RELFMM_API relfmm_status relfmm_plan_create(relfmm_plan **plan,
                                 const relfmm_params *params, int64_t n_max,
                                 void *workspace, size_t workspace_bytes,
                                 void *stream);
RELFMM_API void relfmm_plan_destroy(relfmm_plan *plan);

/* Set the stream later work is enqueued on. */
RELFMM_API relfmm_status relfmm_set_stream(relfmm_plan *plan, void *stream);

/* Build the structure for n particles from positions x and momenta u (both
 * device, n x 3 float64): mean Lorentz factor (unless given), k-d tree
 * (Alg. subdivide with s = (1, 1, gbar)), node boxes and proxies, and the
 * P2P / M2L interaction lists grouped by target (Alg. dualtraversefillitl,
 * Sec. 10). */
RELFMM_API relfmm_status relfmm_build_tree(relfmm_plan *plan, int64_t n, const double *x,
                                const double *u);

/* Compute E and B (device, n x 3 float64, overwritten) at every particle.
 * rebuild = 1: build the structure from x and u first (the whole Alg. FMM).
 * rebuild = 0: keep the structure of the last build (same n) and evaluate
 * with the given x, u, q: particles keep their leaves, boxes, proxies and
 * lists (frozen structure). */
RELFMM_API relfmm_status relfmm_compute_fields(relfmm_plan *plan, int64_t n,
                                    const double *x, const double *u,
                                    const double *q, double *E, double *B,
                                    int32_t rebuild);

/* Gradients of L = sum_i (gE_i . E_i + gB_i . B_i) with respect to the
 * positions, the charges and (optionally) the momenta, for the FMM with
 * frozen structure: the tree, boxes, proxies and lists are held fixed and
 * the transposes of the operators of Alg. FMM are applied in reverse order
 * (L2P^T, L2L^T, M2L^T grouped by source, M2M^T, P2M^T with the derivatives
 * of the interpolation bases, P2P^T on both sides).  gE, gB: device n x 3
 * float64 cotangents; grad_x (n x 3) and grad_q (n): device float64,
 * overwritten.  grad_u (n x 3, device float64, overwritten) may be NULL;
 * otherwise it receives dL/du through the weights q gamma and q u of
 * Sec. 3, the per-source denominator (RELFMM_KERNEL_SOURCE) and, when the
 * plan's gamma_bar parameter is <= 0 (mean Lorentz factor computed from u,
 * Sec. 3), the derivative of every mean kernel (near and far field) with
 * respect to gamma_bar times dgamma_bar/du = pbar / (n gamma_bar); the value
 * of gamma_bar is that of the last build, the derivative the one at the u
 * passed here.  A given gamma_bar (> 0) is a constant.  grad_x and grad_q
 * do not depend on whether grad_u is requested.  rebuild = 1 builds the
 * structure from x and u first (the same structure the forward call builds
 * from the same inputs); rebuild = 0 reuses the last build (same n).
 * Precisions follow the plan (P2P^T in p2p_prec; M2L^T in m2l_prec, like the
 * forward M2L; the far-field gamma_bar derivative in FP64 for an FP64 plan,
 * else FP32). */
RELFMM_API relfmm_status relfmm_adjoint(relfmm_plan *plan, int64_t n,
                                        const double *x, const double *u,
                                        const double *q, const double *gE,
                                        const double *gB, double *grad_x,
                                        double *grad_q, double *grad_u,
                                        int32_t rebuild);

/* Synchronize the plan's stream and report counts of the last build.
 * Returns RELFMM_ECAPACITY if an interaction list overflowed. */
RELFMM_API relfmm_status relfmm_get_stats(relfmm_plan *plan, relfmm_stats *out);

/* Debug / test export of internal state into a HOST buffer (synchronizes).
 * Layouts, for S = n_nodes slots, m = (degree+1)^3, n particles:
 *  RELFMM_EXPORT_NODES    int32  [S][4]  (lo, hi, kind, axis); kind 0 empty,
 *                                        1 leaf, 2 internal; [lo, hi) into
 *                                        the leaf-order permutation
 *  RELFMM_EXPORT_BOXES    float64[S][6]  (min x, y, z, max x, y, z)
 *  RELFMM_EXPORT_PERM     int32  [n]     original index at each position
 *  RELFMM_EXPORT_P2P      int32  [n_p2p][2] (target, source), sorted
 *  RELFMM_EXPORT_M2L      int32  [n_m2l][2] (target, source), sorted
 *  RELFMM_EXPORT_MULTIPOLES float64[S][m][4] (q gamma, q u)
 *  RELFMM_EXPORT_LOCALS   float64[S][m][6] cumulative local fields (after
 *                                        L2L), before the prefactors
 *  RELFMM_EXPORT_NEAR     float64[n][6]  P2P part of (E, B) in the caller's
 *                                        particle order, before prefactors
 *  RELFMM_EXPORT_GAMMA_BAR float64[1]
 *  RELFMM_EXPORT_LOCAL_COTANGENTS float64[S][m][6] after relfmm_adjoint: the
 *                                        cotangents of the local fields;
 *                                        MULTIPOLES then holds the multipole
 *                                        cotangents
 *  RELFMM_EXPORT_INTERP_BOXES float64[S][6] (centre x, y, z, half-width x,
 *                                        y, z) of each node's box: the
 *                                        bounding box, with an axis below
 *                                        1/8 of the node's largest stretched
 *                                        half-width widened to it and
 *                                        clipped to the parent's box, and the
 *                                        parent's box for a node of one
 *                                        particle; the interpolation (Sec. 2)
 *                                        and Alg. diam / dist use it
 * relfmm_export_bytes gives the byte count for the last build. */
typedef enum {
  RELFMM_EXPORT_NODES = 0,
  RELFMM_EXPORT_BOXES = 1,
  RELFMM_EXPORT_PERM = 2,
  RELFMM_EXPORT_P2P = 3,
  RELFMM_EXPORT_M2L = 4,
  RELFMM_EXPORT_MULTIPOLES = 5,
  RELFMM_EXPORT_LOCALS = 6,
  RELFMM_EXPORT_NEAR = 7,
  RELFMM_EXPORT_GAMMA_BAR = 8,
  RELFMM_EXPORT_LOCAL_COTANGENTS = 9,
  RELFMM_EXPORT_INTERP_BOXES = 10
} relfmm_export_what;
RELFMM_API size_t relfmm_export_bytes(relfmm_plan *plan, int32_t what);
RELFMM_API relfmm_status relfmm_export(relfmm_plan *plan, int32_t what, void *host_dst,
                            size_t bytes);

/* Phase timing.  With timing enabled, HIP events are recorded on the plan's
 * stream at the start of every phase of relfmm_compute_fields and at the end
 * of the call; relfmm_get_timings waits for the last timed call and returns
 * the milliseconds of each phase (skipped phases, e.g. the tree with
 * rebuild = 0, take 0), indexed by relfmm_phase. */
typedef enum {
  RELFMM_PHASE_TREE = 0,  /* mean Lorentz factor, presort, k-d levels, boxes */
  RELFMM_PHASE_LISTS = 1, /* dual traversal and grouping by target          */
  RELFMM_PHASE_PREP = 2,  /* leaf-order particle data                        */
  RELFMM_PHASE_P2M = 3,
  RELFMM_PHASE_M2M = 4,
  RELFMM_PHASE_M2L = 5,
  RELFMM_PHASE_P2P = 6,
  RELFMM_PHASE_L2L = 7,
  RELFMM_PHASE_L2P = 8,   /* L2P, near + far, prefactors, original order    */
  RELFMM_N_PHASES = 9
} relfmm_phase;
RELFMM_API relfmm_status relfmm_set_timing(relfmm_plan *plan, int32_t enable);
RELFMM_API relfmm_status relfmm_get_timings(relfmm_plan *plan, double *ms,
                                            int32_t count);

/* Sums of the phase times (ms, indexed by relfmm_phase) over every
 * relfmm_compute_fields call timed since timing was enabled or since the
 * sums were last read, and the number of those calls (*calls); resets both.
 * Each call records its own events (a ring of 64 sets, read back before a
 * set is reused), so a loop of calls is timed without a synchronization per
 * call; this waits for the calls.  ms: host array of count >=
 * RELFMM_N_PHASES doubles. */
RELFMM_API relfmm_status relfmm_get_timing_sums(relfmm_plan *plan, double *ms,
                                                int32_t count, int64_t *calls);

/* FP64 direct sum of eq. (fmm_pp_force_field) over all j != i at selected
 * targets (the brute force of Sec. 6), on the GPU: the reference the FMM's
 * accuracy is measured against.  1 <= n <= 2^28, 0 <= n_targets <= 2^28.
 * x, u (n x 3), q (n): device float64;
 * targets: device int64 indices into the particles (NULL: all n, then
 * n_targets must equal n); E, B: device n_targets x 3 float64, overwritten.
 * kernel: RELFMM_KERNEL_MEAN (needs gamma_bar > 0) or RELFMM_KERNEL_SOURCE
 * (per-source momentum; gamma_bar unused).  ke, c0 <= 0 select the SI
 * defaults.  Enqueued on stream; O(n * n_targets). */
RELFMM_API relfmm_status relfmm_direct_fields(
    int64_t n, const double *x, const double *u, const double *q,
    int64_t n_targets, const int64_t *targets, int32_t kernel,
    double gamma_bar, double ke, double c0, double *E, double *B,
    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the fields
 * of relfmm_compute_fields with rebuild = 1, without a plan or a workspace.
 * The structure and every intermediate live in a device array inside the
 * library, RELFMM_STATIC_SCRATCH_BYTES (64 MiB) on each GPU the library runs
 * on, held until the process ends.  params as for relfmm_plan_create; n, x,
 * u, q, E, B as for relfmm_compute_fields (device float64; E and B
 * overwritten); stream: the hipStream_t the work is enqueued on (NULL: the
 * default stream); the device is the current HIP device.  The call allocates
 * nothing (no device or pinned memory, no events) and does not synchronize.
 * Returns RELFMM_ECAPACITY, enqueuing nothing, when the parameters and n need
 * more than RELFMM_STATIC_SCRATCH_BYTES (never when relfmm_workspace_bytes
 * (params, n) is at most that).  With no plan to keep the flag, a list
 * overflow is reported only through E and B, which are then NaN.  Every call
 * on one GPU uses that GPU's one array, whose contents the next call
 * overwrites: calls on one stream are ordered and safe, calls that overlap
 * on one GPU (other streams, other host threads) race and give wrong
 * results. */
#define RELFMM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
RELFMM_API relfmm_status relfmm_compute_fields_static(
    const relfmm_params *params, int64_t n, const double *x, const double *u,
    const double *q, double *E, double *B, void *stream);

RELFMM_API const char *relfmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
