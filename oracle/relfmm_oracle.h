/*
 * relfmm_oracle.h -- plain FP64 CPU oracle for the relativistic space-charge
 * FMM of Kan, Kaertner, Le Borne and Zemke (arXiv 2302.07567).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this library: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the HIP library.
 *
 * Everything is FP64 and compiled with -ffp-contract=off so that decisions
 * (split axis, admissibility, traversal order) are reproducible bit for bit.
 *
 * Layouts: positions x and momenta u are n x 3 row-major; charges q are n;
 * fields E, B are n x 3 row-major in the caller's particle order.
 * Proxy index nu = (i*(p+1) + j)*(p+1) + k for per-axis node indices
 * (i, j, k) along (x, y, z), p = interpolation degree.
 * Multipoles: [node][nu][4] = (q*gamma, q*u_x, q*u_y, q*u_z) weights.
 * Locals:     [node][mu][6] = (E_x, E_y, E_z, B_x, B_y, B_z) before the
 *             physical prefactors ke and ke/c0.
 */
#ifndef RELFMM_ORACLE_H
#define RELFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_KERNEL_MEAN 0  /* eq. (fmm_relativistic_kernel): beam-average gamma */
#define ORC_KERNEL_EXACT 1 /* per-source momentum in the denominator */

/* OpenMP threads of the loops over independent targets (and the current
 * setting). */
void orc_set_num_threads(int n);
int orc_get_num_threads(void);

/* Mean Lorentz factor from the unweighted mean momentum (Sec. 3). */
double orc_gamma_bar(int64_t n, const double *u);

/* Pair kernel g for one (target, source) offset r = x_i - x_j. */
void orc_pair_kernel(int mode, double gamma_bar, const double *r,
                     const double *uj, double *g);

/* O(N^2) direct sum (Alg. P2P with S_t = S_s = S, i != j).  If tgt is NULL
 * all n targets are evaluated and E, B are n x 3; otherwise E, B are
 * ntgt x 3 for the listed targets. */
void orc_direct(int64_t n, const double *x, const double *u, const double *q,
                double gamma_bar, int mode, double ke, double c0,
                int64_t ntgt, const int64_t *tgt, double *E, double *B);

/* Chebyshev points of the second kind on [-1, 1] and barycentric basis. */
void orc_cheb_nodes(int p, double *t);
void orc_basis_1d(int p, double c, double h, double x, double *out);

typedef struct orc_fmm orc_fmm;

orc_fmm *orc_fmm_create(int64_t n, int degree, int leaf_size, double eta,
                        double gamma_bar, int mode, double ke, double c0);
void orc_fmm_destroy(orc_fmm *f);

/* Steps of Alg. FMM, in order.  Each step needs the previous ones. */
int orc_fmm_build_tree(orc_fmm *f, const double *x);       /* Alg. subdivide */
int orc_fmm_build_lists(orc_fmm *f);                        /* Alg. dual traversal (ITL form) */
int orc_fmm_upward(orc_fmm *f, const double *u, const double *q); /* P2M + M2M */
int orc_fmm_m2l(orc_fmm *f);                                /* Alg. M2L over m2l list */
int orc_fmm_p2p(orc_fmm *f);                                /* Alg. P2P over p2p list */
int orc_fmm_downward(orc_fmm *f);                           /* L2L + L2P + prefactors */

/* Frozen structure: replace the positions (same particles, same order) and
 * rerun orc_fmm_upward .. orc_fmm_downward on the tree, boxes, proxies and
 * lists built from the previous positions. */
int orc_fmm_set_positions(orc_fmm *f, const double *x);
/* Frozen structure: the mean Lorentz factor the kernels of the next run use. */
int orc_fmm_set_gamma_bar(orc_fmm *f, double gamma_bar);

/* Derivative d l_k/dx of the one-dimensional basis over c +- h. */
void orc_basis_deriv_1d(int p, double c, double h, double x, double *dl);

/* Gradients of L = sum_i (gE_i . E_i + gB_i . B_i): the analytic O(N^2)
 * gradient of the direct sum, and the transpose of the FMM with frozen
 * structure (needs a completed forward run). grad_x is n x 3, grad_q n. */
void orc_direct_grad(int64_t n, const double *x, const double *u,
                     const double *q, double gamma_bar, int mode, double ke,
                     double c0, const double *gE, const double *gB,
                     double *grad_x, double *grad_q);
int orc_fmm_adjoint(orc_fmm *f, const double *gE, const double *gB,
                    double *grad_x, double *grad_q, double *grad_u,
                    int gbar_from_u);
/* Gradient with respect to the momenta (n x 3).  gbar_from_u: gamma_bar is
 * the function of u of Sec. 3 and its derivative is included; otherwise it
 * is a fixed parameter.  orc_fmm_adjoint computes the same for the FMM when
 * grad_u is not NULL (structure frozen, gamma_bar enters only the kernels). */
void orc_direct_grad_u(int64_t n, const double *x, const double *u,
                       const double *q, double gamma_bar, int mode, double ke,
                       double c0, const double *gE, const double *gB,
                       int gbar_from_u, double *grad_u);

/* Sizes: out[0]=depth, out[1]=nslots, out[2]=n_p2p, out[3]=n_m2l,
 * out[4]=sum over p2p pairs of |t||s|, out[5]=n_m2l*m*m, out[6]=m. */
void orc_fmm_sizes(const orc_fmm *f, int64_t *out);

/* Copies of the internal state (arrays sized by orc_fmm_sizes). */
void orc_fmm_get_tree(const orc_fmm *f, int64_t *perm, int64_t *lo,
                      int64_t *hi, int8_t *kind, int8_t *axis, double *bmin,
                      double *bmax, double *cen, double *hw);
void orc_fmm_get_lists(const orc_fmm *f, int64_t *p2p, int64_t *m2l);
void orc_fmm_get_multipoles(const orc_fmm *f, double *M);
void orc_fmm_get_locals(const orc_fmm *f, double *L, double *Lcum);
void orc_fmm_get_fields(const orc_fmm *f, double *E, double *B,
                        double *Enear, double *Bnear);

#ifdef __cplusplus
}
#endif
#endif
