/*
 * relfmm_oracle.c -- plain, slow, FP64 CPU oracle of the lab-frame
 * interpolation-based FMM for the relativistic space-charge field
 * (Kan, Kaertner, Le Borne, Zemke, arXiv 2302.07567).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares
 * no code with the HIP library.
 *
 * Each function follows one passage of the paper and is written to be
 * checked against it by eye.  Readings of silent or garbled passages:
 *  - P2P kernel: MEAN uses the two-argument kernel of Sec. 3 with the mean
 *    Lorentz factor; EXACT uses the per-source momentum u_j, i.e. the
 *    field of a uniformly moving charge, g = r / (|r|^2 + (u_j.r)^2)^{3/2}.
 *    The far field (M2L) can only carry the mean factor and always uses MEAN.
 *  - Mean momentum: unweighted arithmetic mean over all particles.
 *  - Per-particle charges q_j: the multipole weights are (q_j gamma_j,
 *    q_j u_j), which reduces to the paper's common q when all are equal.
 *  - Split: members sorted by (coordinate, original index); the first
 *    ceil(|S|/2) go to child 2i (index split of App. B).  Axis ties go to
 *    the lowest axis.
 *  - Stretched radius: the half-diagonal of Alg. diam; distance between box
 *    centres of Alg. dist; admissible iff max(r_t^2, r_s^2) < eta^2 d^2.
 *  - Traversal: split the target only if r_t^2 > r_s^2 (ties split source).
 *  - Interpolation: Chebyshev points of the second kind with barycentric
 *    weights (Berrut and Trefethen 2004); exact node hits give a Kronecker
 *    delta.
 *  - Boxes: the bounding box, with an axis narrower than 1/8 of the node's
 *    largest stretched half-width widened to that and clipped to the
 *    parent's box; a one-particle node takes its parent's box (interp_box).
 *  - M2M, M2L and L2L accumulate (+=) and the momentum line of M2M uses the
 *    child's momentum multipole.
 */
#include "relfmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Sec. 3: kinematics and the pair kernels.                                  */
/* ------------------------------------------------------------------------ */

/* Threads of the OpenMP loops over independent targets (the CPU-baseline
 * timing runs the serial FMM on one). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_get_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sec. 3: gamma_bar^2 = 1 + pbar.pbar with pbar the mean momentum. */
double orc_gamma_bar(int64_t n, const double *u) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t j = 0; j < n; ++j) {
    s[0] += u[3 * j + 0];
    s[1] += u[3 * j + 1];
    s[2] += u[3 * j + 2];
  }
  double p[3] = {s[0] / (double)n, s[1] / (double)n, s[2] / (double)n};
  return sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
}

/* gamma_j = 1/sqrt(1 - beta_j^2) written through u_j = gamma_j beta_j. */
static double lorentz(const double *uj) {
  return sqrt(1.0 + (uj[0] * uj[0] + uj[1] * uj[1] + uj[2] * uj[2]));
}

/* eq. (fmm_relativistic_kernel) for MEAN; field of a uniformly moving
 * charge for EXACT.  D^{3/2} is formed as D*sqrt(D). */
void orc_pair_kernel(int mode, double gamma_bar, const double *r,
                     const double *uj, double *g) {
  double D;
  if (mode == ORC_KERNEL_MEAN) {
    double gb2 = gamma_bar * gamma_bar;
    D = r[0] * r[0] + r[1] * r[1] + gb2 * (r[2] * r[2]);
  } else {
    double ur = uj[0] * r[0] + uj[1] * r[1] + uj[2] * r[2];
    D = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) + ur * ur;
  }
  double inv = 1.0 / (D * sqrt(D));
  g[0] = r[0] * inv;
  g[1] = r[1] * inv;
  g[2] = r[2] * inv;
}

static void cross(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* eq. (fmm_pp_force_field) summed over j != i: the brute force of Sec. 6. */
void orc_direct(int64_t n, const double *x, const double *u, const double *q,
                double gamma_bar, int mode, double ke, double c0,
                int64_t ntgt, const int64_t *tgt, double *E, double *B) {
  int64_t nt = tgt ? ntgt : n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < nt; ++a) {
    int64_t i = tgt ? tgt[a] : a;
    double e[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                     x[3 * i + 2] - x[3 * j + 2]};
      double g[3], ug[3];
      orc_pair_kernel(mode, gamma_bar, r, u + 3 * j, g);
      double qg = q[j] * lorentz(u + 3 * j);
      cross(u + 3 * j, g, ug);
      for (int c = 0; c < 3; ++c) {
        e[c] += qg * g[c];
        b[c] += q[j] * ug[c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      E[3 * a + c] = ke * e[c];
      B[3 * a + c] = (ke / c0) * b[c];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2: tensor-product Lagrange interpolation on the bounding box.        */
/* ------------------------------------------------------------------------ */

/* Chebyshev points of the second kind, t_k = cos(k pi / p), written as a
 * sine so that t_0 = 1, t_p = -1 and t_{p/2} = 0 hold exactly. */
void orc_cheb_nodes(int p, double *t) {
  for (int k = 0; k <= p; ++k)
    t[k] = sin(M_PI * (double)(p - 2 * k) / (2.0 * (double)p));
}

/* Barycentric weights of the second-kind points: (-1)^k, halved at ends. */
static void cheb_weights(int p, double *w) {
  for (int k = 0; k <= p; ++k) {
    w[k] = (k % 2 == 0) ? 1.0 : -1.0;
    if (k == 0 || k == p) w[k] *= 0.5;
  }
}

/* One-dimensional Lagrange basis l_k(x) over the interval c +- h, in the
 * second (true) barycentric form. */
void orc_basis_1d(int p, double c, double h, double x, double *out) {
  double t[32], w[32];
  orc_cheb_nodes(p, t);
  cheb_weights(p, w);
  double tau = (x - c) / h;
  for (int k = 0; k <= p; ++k) {
    if (tau == t[k]) {
      for (int m = 0; m <= p; ++m) out[m] = (m == k) ? 1.0 : 0.0;
      return;
    }
  }
  double s = 0.0;
  for (int k = 0; k <= p; ++k) {
    out[k] = w[k] / (tau - t[k]);
    s += out[k];
  }
  for (int k = 0; k <= p; ++k) out[k] = out[k] / s;
}

/* ------------------------------------------------------------------------ */
/* FMM state.                                                               */
/* ------------------------------------------------------------------------ */

struct orc_fmm {
  int64_t n;
  int p, leaf_size, mode;
  double eta, gamma_bar, ke, c0;
  int depth;
  int64_t nslots, m;
  const double *x; /* borrowed positions (valid during the run) */
  int64_t *perm;
  int64_t *lo, *hi;
  int8_t *kind; /* 0 empty, 1 leaf, 2 internal */
  int8_t *axis; /* split axis, -1 if not split */
  double *bmin, *bmax, *cen, *hw;
  int64_t np2p, nm2l, cap_p2p, cap_m2l;
  int64_t *p2p, *m2l;
  double *mw;  /* per particle weights (q gamma, q u) in caller order */
  double *uu;  /* per particle momenta (caller order), for EXACT P2P */
  double *qq;  /* per particle charges (caller order) */
  double *M, *L, *Lcum;
  double *Enear, *Bnear, *E, *B;
};

orc_fmm *orc_fmm_create(int64_t n, int degree, int leaf_size, double eta,
                        double gamma_bar, int mode, double ke, double c0) {
  if (n < 1 || degree < 1 || degree > 30 || leaf_size < 1 || !(eta > 0))
    return NULL;
  orc_fmm *f = (orc_fmm *)calloc(1, sizeof(orc_fmm));
  f->n = n;
  f->p = degree;
  f->leaf_size = leaf_size;
  f->eta = eta;
  f->gamma_bar = gamma_bar;
  f->mode = mode;
  f->ke = ke;
  f->c0 = c0;
  f->m = (int64_t)(degree + 1) * (degree + 1) * (degree + 1);
  /* Sec. 8: depth kappa = 0 for N <= N0, else ceil(log2(N/N0)). */
  int depth = 0;
  while ((int64_t)leaf_size << depth < n) ++depth;
  f->depth = depth;
  f->nslots = (int64_t)1 << (depth + 1);
  return f;
}

void orc_fmm_destroy(orc_fmm *f) {
  if (!f) return;
  free(f->perm); free(f->lo); free(f->hi); free(f->kind); free(f->axis);
  free(f->bmin); free(f->bmax); free(f->cen); free(f->hw);
  free(f->p2p); free(f->m2l); free(f->mw); free(f->uu); free(f->qq);
  free(f->M); free(f->L); free(f->Lcum);
  free(f->Enear); free(f->Bnear); free(f->E); free(f->B);
  free(f);
}

/* ------------------------------------------------------------------------ */
/* Alg. direction4split / subdivide and App. B (index split).               */
/* ------------------------------------------------------------------------ */

typedef struct {
  double key;
  int64_t idx;
} keyed;

static int cmp_keyed(const void *a, const void *b) {
  const keyed *x = (const keyed *)a, *y = (const keyed *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

/* bbox(S): componentwise min and max over the members. */
static void bbox(orc_fmm *f, int64_t node) {
  const double *x = f->x;
  for (int g = 0; g < 3; ++g) {
    double a = x[3 * f->perm[f->lo[node]] + g], b = a;
    for (int64_t k = f->lo[node]; k < f->hi[node]; ++k) {
      double v = x[3 * f->perm[k] + g];
      if (v < a) a = v;
      if (v > b) b = v;
    }
    f->bmin[3 * node + g] = a;
    f->bmax[3 * node + g] = b;
  }
}

/* Alg. direction4split: argmax_g s_g (b_g - a_g), s = (1, 1, gamma_bar). */
static int direction4split(const orc_fmm *f, int64_t node) {
  double s[3] = {1.0, 1.0, f->gamma_bar};
  int k = 0;
  double best = s[0] * (f->bmax[3 * node] - f->bmin[3 * node]);
  for (int g = 1; g < 3; ++g) {
    double w = s[g] * (f->bmax[3 * node + g] - f->bmin[3 * node + g]);
    if (w > best) {
      best = w;
      k = g;
    }
  }
  return k;
}

/* Alg. subdivide, recursive, with the index split of App. B. */
static void subdivide(orc_fmm *f, int64_t node, keyed *scratch) {
  bbox(f, node);
  int64_t cnt = f->hi[node] - f->lo[node];
  if (cnt <= f->leaf_size) {
    f->kind[node] = 1;
    f->axis[node] = -1;
    return;
  }
  int k = direction4split(f, node);
  f->kind[node] = 2;
  f->axis[node] = (int8_t)k;
  for (int64_t a = 0; a < cnt; ++a) {
    int64_t idx = f->perm[f->lo[node] + a];
    scratch[a].key = f->x[3 * idx + k];
    scratch[a].idx = idx;
  }
  qsort(scratch, (size_t)cnt, sizeof(keyed), cmp_keyed);
  for (int64_t a = 0; a < cnt; ++a) f->perm[f->lo[node] + a] = scratch[a].idx;
  int64_t nleft = (cnt + 1) / 2;
  int64_t c1 = 2 * node, c2 = 2 * node + 1;
  f->lo[c1] = f->lo[node];
  f->hi[c1] = f->lo[node] + nleft;
  f->lo[c2] = f->lo[node] + nleft;
  f->hi[c2] = f->hi[node];
  subdivide(f, c1, scratch);
  subdivide(f, c2, scratch);
}

/* Interpolation box of a node and, recursively, of its subtree (the paper
 * interpolates over the bounding box and is silent on boxes of zero or
 * near-zero width, where the basis derivative of the adjoint divides by the
 * width).  Reading: the box is the bounding box, except on an axis g whose
 * half-width h_g is below R/(8 s_g), R = max_g s_g h_g the node's largest
 * stretched half-width: there the half-width becomes R/(8 s_g) about the
 * bounding-box centre and the interval is clipped to the parent's, so that
 * every box stays inside its parent's.  A node of one particle (R = 0)
 * takes its parent's box; a root of one particle gets R = 1.  Alg. diam,
 * Alg. dist and the interpolation all use this box. */
static void interp_box(orc_fmm *f, int64_t node, const double *plo,
                       const double *phi, double *ilo, double *ihi) {
  if (node >= f->nslots || !f->kind[node]) return;
  const double s[3] = {1.0, 1.0, f->gamma_bar};
  double *lo = ilo + 3 * node, *hi = ihi + 3 * node;
  double R = 0.0;
  for (int g = 0; g < 3; ++g) {
    double v = s[g] * ((f->bmax[3 * node + g] - f->bmin[3 * node + g]) * 0.5);
    if (v > R) R = v;
  }
  if (R == 0.0 && plo) {
    for (int g = 0; g < 3; ++g) {
      lo[g] = plo[g];
      hi[g] = phi[g];
    }
  } else {
    if (R == 0.0) R = 1.0;
    for (int g = 0; g < 3; ++g) {
      double a = f->bmin[3 * node + g], b = f->bmax[3 * node + g];
      double h = (b - a) * 0.5;
      double fl = ldexp(R, -3) / s[g];
      if (h < fl) {
        double c = (a + b) * 0.5;
        a = c - fl;
        b = c + fl;
        if (plo) {
          if (a < plo[g]) a = plo[g];
          if (b > phi[g]) b = phi[g];
        }
      }
      lo[g] = a;
      hi[g] = b;
    }
  }
  for (int g = 0; g < 3; ++g) {
    f->cen[3 * node + g] = (lo[g] + hi[g]) * 0.5;
    double h = (hi[g] - lo[g]) * 0.5;
    /* coordinates equal to the last bits: keep the reference coordinate
     * defined */
    f->hw[3 * node + g] = h > 0.0 ? h : ldexp(1.0, -40) / s[g];
  }
  interp_box(f, 2 * node, lo, hi, ilo, ihi);
  interp_box(f, 2 * node + 1, lo, hi, ilo, ihi);
}

int orc_fmm_build_tree(orc_fmm *f, const double *x) {
  int64_t ns = f->nslots;
  f->x = x;
  f->perm = (int64_t *)malloc(sizeof(int64_t) * f->n);
  f->lo = (int64_t *)malloc(sizeof(int64_t) * ns);
  f->hi = (int64_t *)malloc(sizeof(int64_t) * ns);
  f->kind = (int8_t *)calloc(ns, 1);
  f->axis = (int8_t *)malloc(ns);
  f->bmin = (double *)calloc(3 * ns, sizeof(double));
  f->bmax = (double *)calloc(3 * ns, sizeof(double));
  f->cen = (double *)calloc(3 * ns, sizeof(double));
  f->hw = (double *)calloc(3 * ns, sizeof(double));
  for (int64_t i = 0; i < ns; ++i) {
    f->lo[i] = -1;
    f->hi[i] = -1;
    f->axis[i] = -1;
  }
  for (int64_t i = 0; i < f->n; ++i) f->perm[i] = i;
  f->lo[1] = 0;
  f->hi[1] = f->n;
  keyed *scratch = (keyed *)malloc(sizeof(keyed) * f->n);
  subdivide(f, 1, scratch);
  free(scratch);
  double *ilo = (double *)calloc(3 * ns, sizeof(double));
  double *ihi = (double *)calloc(3 * ns, sizeof(double));
  interp_box(f, 1, NULL, NULL, ilo, ihi);
  free(ilo);
  free(ihi);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. diam, dist, admissible and the list-filling dual traversal.          */
/* ------------------------------------------------------------------------ */

/* Alg. diam, squared: ||s o (a - b)/2||^2, the stretched half-diagonal of
 * the node's box (the interpolation box above). */
static double diam2(const orc_fmm *f, int64_t i) {
  double s[3] = {1.0, 1.0, f->gamma_bar};
  double r2 = 0.0;
  for (int g = 0; g < 3; ++g) {
    double h = s[g] * f->hw[3 * i + g];
    r2 = r2 + h * h;
  }
  return r2;
}

/* Alg. dist, squared: ||s o (c1 - c2)||^2 with c the box centres. */
static double dist2(const orc_fmm *f, int64_t i, int64_t j) {
  double s[3] = {1.0, 1.0, f->gamma_bar};
  double d2 = 0.0;
  for (int g = 0; g < 3; ++g) {
    double d = s[g] * (f->cen[3 * i + g] - f->cen[3 * j + g]);
    d2 = d2 + d * d;
  }
  return d2;
}

/* Alg. admissible: max(r1, r2)/d < eta, in squared form (d = 0 never). */
static int admissible(const orc_fmm *f, int64_t i, int64_t j) {
  double r1 = diam2(f, i), r2 = diam2(f, j);
  double r = r1 > r2 ? r1 : r2;
  double d2 = dist2(f, i, j);
  return r < (f->eta * f->eta) * d2;
}

static void push(int64_t **arr, int64_t *cnt, int64_t *cap, int64_t a,
                 int64_t b) {
  if (*cnt == *cap) {
    *cap = *cap ? 2 * *cap : 1024;
    *arr = (int64_t *)realloc(*arr, sizeof(int64_t) * 2 * (*cap));
  }
  (*arr)[2 * *cnt] = a;
  (*arr)[2 * *cnt + 1] = b;
  ++*cnt;
}

/* Alg. dualtraversefillitl. */
static void fill_itl(orc_fmm *f, int64_t i, int64_t j) {
  int leaf_i = f->kind[i] == 1, leaf_j = f->kind[j] == 1;
  if (leaf_i && leaf_j) {
    push(&f->p2p, &f->np2p, &f->cap_p2p, i, j);
    return;
  }
  if (admissible(f, i, j)) {
    push(&f->m2l, &f->nm2l, &f->cap_m2l, i, j);
  } else if (leaf_i) {
    fill_itl(f, i, 2 * j);
    fill_itl(f, i, 2 * j + 1);
  } else if (leaf_j) {
    fill_itl(f, 2 * i, j);
    fill_itl(f, 2 * i + 1, j);
  } else if (diam2(f, i) > diam2(f, j)) {
    fill_itl(f, 2 * i, j);
    fill_itl(f, 2 * i + 1, j);
  } else {
    fill_itl(f, i, 2 * j);
    fill_itl(f, i, 2 * j + 1);
  }
}

int orc_fmm_build_lists(orc_fmm *f) {
  f->np2p = f->nm2l = 0;
  fill_itl(f, 1, 1);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Interpolation helpers: proxies and per-axis basis tables.                 */
/* ------------------------------------------------------------------------ */

/* Proxy coordinate xi_{S,k} along axis g. */
static double proxy(const orc_fmm *f, int64_t node, int g, int k,
                    const double *t) {
  return f->cen[3 * node + g] + f->hw[3 * node + g] * t[k];
}

/* Per-axis basis of node S evaluated at a point. */
static void basis3(const orc_fmm *f, int64_t node, const double *pt,
                   double *lx, double *ly, double *lz) {
  int p = f->p;
  orc_basis_1d(p, f->cen[3 * node], f->hw[3 * node], pt[0], lx);
  orc_basis_1d(p, f->cen[3 * node + 1], f->hw[3 * node + 1], pt[1], ly);
  orc_basis_1d(p, f->cen[3 * node + 2], f->hw[3 * node + 2], pt[2], lz);
}

/* T_g[a][b] = l^g_{S,a}(xi^g_{C,b}): parent S basis at the child C proxies. */
static void transfer_tables(const orc_fmm *f, int64_t S, int64_t C,
                            const double *t, double *T) {
  int p = f->p, q = p + 1;
  double tmp[32];
  for (int g = 0; g < 3; ++g)
    for (int b = 0; b < q; ++b) {
      orc_basis_1d(p, f->cen[3 * S + g], f->hw[3 * S + g],
                   proxy(f, C, g, b, t), tmp);
      for (int a = 0; a < q; ++a) T[(g * q + a) * q + b] = tmp[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. upwardpass: P2M at leaves, M2M to parents (eq. M2M).                 */
/* ------------------------------------------------------------------------ */

/* Alg. P2M with the effective masses of Sec. 3. */
static void p2m(orc_fmm *f, int64_t S) {
  int q = f->p + 1;
  double lx[32], ly[32], lz[32];
  double *M = f->M + S * f->m * 4;
  for (int64_t k = f->lo[S]; k < f->hi[S]; ++k) {
    int64_t j = f->perm[k];
    basis3(f, S, f->x + 3 * j, lx, ly, lz);
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b)
        for (int c = 0; c < q; ++c) {
          double l = lx[a] * ly[b] * lz[c];
          int64_t nu = (a * q + b) * q + c;
          for (int w = 0; w < 4; ++w) M[nu * 4 + w] += l * f->mw[4 * j + w];
        }
  }
}

/* Alg. M2M: M_S[nu] += sum_nu' l_{S,nu}(xi_{C,nu'}) M_C[nu']. */
static void m2m(orc_fmm *f, int64_t S, int64_t C, const double *t) {
  int q = f->p + 1;
  double T[3 * 32 * 32];
  transfer_tables(f, S, C, t, T);
  double *MS = f->M + S * f->m * 4;
  const double *MC = f->M + C * f->m * 4;
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c) {
        int64_t nu = (a * q + b) * q + c;
        for (int a2 = 0; a2 < q; ++a2)
          for (int b2 = 0; b2 < q; ++b2)
            for (int c2 = 0; c2 < q; ++c2) {
              int64_t nu2 = (a2 * q + b2) * q + c2;
              double l = T[(0 * q + a) * q + a2] * T[(1 * q + b) * q + b2] *
                         T[(2 * q + c) * q + c2];
              for (int w = 0; w < 4; ++w) MS[nu * 4 + w] += l * MC[nu2 * 4 + w];
            }
      }
}

int orc_fmm_upward(orc_fmm *f, const double *u, const double *q) {
  int64_t n = f->n, ns = f->nslots;
  free(f->mw);
  free(f->uu);
  free(f->qq);
  free(f->M);
  f->mw = (double *)malloc(sizeof(double) * 4 * n);
  f->uu = (double *)malloc(sizeof(double) * 3 * n);
  f->qq = (double *)malloc(sizeof(double) * n);
  for (int64_t j = 0; j < n; ++j) {
    double gj = lorentz(u + 3 * j);
    f->qq[j] = q[j];
    f->mw[4 * j] = q[j] * gj;
    for (int c = 0; c < 3; ++c) {
      f->mw[4 * j + 1 + c] = q[j] * u[3 * j + c];
      f->uu[3 * j + c] = u[3 * j + c];
    }
  }
  f->M = (double *)calloc((size_t)(ns * f->m * 4), sizeof(double));
  double t[32];
  orc_cheb_nodes(f->p, t);
  /* Leaves at every level first (P2M), then parents level by level from
   * the deepest (post-order of Alg. upwardpass, level-synchronous). */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t S = 1; S < ns; ++S)
    if (f->kind[S] == 1) p2m(f, S);
  for (int l = f->depth - 1; l >= 0; --l) {
    int64_t a = (int64_t)1 << l, b = (int64_t)1 << (l + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t S = a; S < b; ++S) {
      if (f->kind[S] != 2) continue;
      m2m(f, S, 2 * S, t);
      m2m(f, S, 2 * S + 1, t);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. M2L and Alg. P2P over the interaction lists.                         */
/* ------------------------------------------------------------------------ */

/* Group list entries by target, keeping traversal order inside a group. */
static void group_by_target(const int64_t *pairs, int64_t np, int64_t ns,
                            int64_t **start_out, int64_t **order_out) {
  int64_t *start = (int64_t *)calloc(ns + 1, sizeof(int64_t));
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
  for (int64_t k = 0; k < np; ++k) start[pairs[2 * k] + 1]++;
  for (int64_t i = 0; i < ns; ++i) start[i + 1] += start[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ns);
  memcpy(fill, start, sizeof(int64_t) * ns);
  for (int64_t k = 0; k < np; ++k) order[fill[pairs[2 * k]]++] = k;
  free(fill);
  *start_out = start;
  *order_out = order;
}

/* Alg. M2L: E_{t,mu} += sum_nu gamma_{s,nu} g(xi_t,mu, xi_s,nu) and
 * B_{t,mu} += sum_nu p_{s,nu} x g(...), always with the MEAN kernel. */
static void m2l_pair(orc_fmm *f, int64_t T, int64_t S, const double *t) {
  int q = f->p + 1;
  double *L = f->L + T * f->m * 6;
  const double *M = f->M + S * f->m * 4;
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c) {
        int64_t mu = (a * q + b) * q + c;
        double xt[3] = {proxy(f, T, 0, a, t), proxy(f, T, 1, b, t),
                        proxy(f, T, 2, c, t)};
        for (int a2 = 0; a2 < q; ++a2)
          for (int b2 = 0; b2 < q; ++b2)
            for (int c2 = 0; c2 < q; ++c2) {
              int64_t nu = (a2 * q + b2) * q + c2;
              double r[3] = {xt[0] - proxy(f, S, 0, a2, t),
                             xt[1] - proxy(f, S, 1, b2, t),
                             xt[2] - proxy(f, S, 2, c2, t)};
              double g[3], ug[3];
              orc_pair_kernel(ORC_KERNEL_MEAN, f->gamma_bar, r, NULL, g);
              cross(M + nu * 4 + 1, g, ug);
              for (int w = 0; w < 3; ++w) {
                L[mu * 6 + w] += M[nu * 4] * g[w];
                L[mu * 6 + 3 + w] += ug[w];
              }
            }
      }
}

int orc_fmm_m2l(orc_fmm *f) {
  int64_t ns = f->nslots;
  free(f->L);
  f->L = (double *)calloc((size_t)(ns * f->m * 6), sizeof(double));
  double t[32];
  orc_cheb_nodes(f->p, t);
  int64_t *start, *order;
  group_by_target(f->m2l, f->nm2l, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t T = 1; T < ns; ++T)
    for (int64_t k = start[T]; k < start[T + 1]; ++k)
      m2l_pair(f, T, f->m2l[2 * order[k] + 1], t);
  free(start);
  free(order);
  return 0;
}

/* Alg. P2P: E_i += gamma_j g(x_i, x_j, p_j), B_i += p_j x g, j != i. */
static void p2p_pair(orc_fmm *f, int64_t T, int64_t S) {
  const double *x = f->x;
  for (int64_t a = f->lo[T]; a < f->hi[T]; ++a) {
    int64_t i = f->perm[a];
    for (int64_t b = f->lo[S]; b < f->hi[S]; ++b) {
      int64_t j = f->perm[b];
      if (j == i) continue;
      double r[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                     x[3 * i + 2] - x[3 * j + 2]};
      double g[3], ug[3];
      orc_pair_kernel(f->mode, f->gamma_bar, r, f->uu + 3 * j, g);
      cross(f->mw + 4 * j + 1, g, ug);
      for (int w = 0; w < 3; ++w) {
        f->Enear[3 * i + w] += f->mw[4 * j] * g[w];
        f->Bnear[3 * i + w] += ug[w];
      }
    }
  }
}

int orc_fmm_p2p(orc_fmm *f) {
  int64_t ns = f->nslots, n = f->n;
  free(f->Enear);
  free(f->Bnear);
  f->Enear = (double *)calloc((size_t)(3 * n), sizeof(double));
  f->Bnear = (double *)calloc((size_t)(3 * n), sizeof(double));
  int64_t *start, *order;
  group_by_target(f->p2p, f->np2p, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t T = 1; T < ns; ++T)
    for (int64_t k = start[T]; k < start[T + 1]; ++k)
      p2p_pair(f, T, f->p2p[2 * order[k] + 1]);
  free(start);
  free(order);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. downwardpass: L2L (cumulative local field, eq. L2L) and L2P.        */
/* ------------------------------------------------------------------------ */

/* Alg. L2L: L_C[mu'] += sum_mu l_{S,mu}(xi_{C,mu'}) L_S[mu]. */
static void l2l(orc_fmm *f, int64_t C, int64_t S, const double *t) {
  int q = f->p + 1;
  double T[3 * 32 * 32];
  transfer_tables(f, S, C, t, T);
  double *LC = f->Lcum + C * f->m * 6;
  const double *LS = f->Lcum + S * f->m * 6;
  for (int a2 = 0; a2 < q; ++a2)
    for (int b2 = 0; b2 < q; ++b2)
      for (int c2 = 0; c2 < q; ++c2) {
        int64_t mu2 = (a2 * q + b2) * q + c2;
        for (int a = 0; a < q; ++a)
          for (int b = 0; b < q; ++b)
            for (int c = 0; c < q; ++c) {
              int64_t mu = (a * q + b) * q + c;
              double l = T[(0 * q + a) * q + a2] * T[(1 * q + b) * q + b2] *
                         T[(2 * q + c) * q + c2];
              for (int w = 0; w < 6; ++w) LC[mu2 * 6 + w] += l * LS[mu * 6 + w];
            }
      }
}

/* Alg. L2P: E_i += sum_mu l_{S,mu}(x_i) E_{S,mu}, same for B. */
static void l2p(orc_fmm *f, int64_t S) {
  int q = f->p + 1;
  double lx[32], ly[32], lz[32];
  const double *L = f->Lcum + S * f->m * 6;
  for (int64_t k = f->lo[S]; k < f->hi[S]; ++k) {
    int64_t i = f->perm[k];
    basis3(f, S, f->x + 3 * i, lx, ly, lz);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b)
        for (int c = 0; c < q; ++c) {
          double l = lx[a] * ly[b] * lz[c];
          int64_t mu = (a * q + b) * q + c;
          for (int w = 0; w < 6; ++w) acc[w] += l * L[mu * 6 + w];
        }
    for (int w = 0; w < 3; ++w) {
      f->E[3 * i + w] += acc[w];
      f->B[3 * i + w] += acc[3 + w];
    }
  }
}

int orc_fmm_downward(orc_fmm *f) {
  int64_t ns = f->nslots, n = f->n;
  size_t nl = (size_t)(ns * f->m * 6);
  free(f->Lcum);
  free(f->E);
  free(f->B);
  f->Lcum = (double *)malloc(sizeof(double) * nl);
  memcpy(f->Lcum, f->L, sizeof(double) * nl);
  double t[32];
  orc_cheb_nodes(f->p, t);
  for (int l = 0; l < f->depth; ++l) {
    int64_t a = (int64_t)1 << l, b = (int64_t)1 << (l + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t S = a; S < b; ++S) {
      if (f->kind[S] != 2) continue;
      l2l(f, 2 * S, S, t);
      l2l(f, 2 * S + 1, S, t);
    }
  }
  f->E = (double *)calloc((size_t)(3 * n), sizeof(double));
  f->B = (double *)calloc((size_t)(3 * n), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t S = 1; S < ns; ++S)
    if (f->kind[S] == 1) l2p(f, S);
  /* Near field plus far field, then the prefactors of
   * eq. (fmm_pp_force_field): ke for E and ke/c0 for B. */
  for (int64_t i = 0; i < 3 * n; ++i) {
    f->E[i] = f->ke * (f->E[i] + f->Enear[i]);
    f->B[i] = (f->ke / f->c0) * (f->B[i] + f->Bnear[i]);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Frozen structure: new positions, same tree, boxes, proxies and lists.     */
/* ------------------------------------------------------------------------ */

int orc_fmm_set_positions(orc_fmm *f, const double *x) {
  f->x = x;
  return 0;
}

/* The mean Lorentz factor used by the kernels of the next run; the tree,
 * boxes and lists stay those of the build. */
int orc_fmm_set_gamma_bar(orc_fmm *f, double gamma_bar) {
  f->gamma_bar = gamma_bar;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Derivative of the one-dimensional Lagrange basis.                         */
/* ------------------------------------------------------------------------ */

/* d l_k / dx over c +- h.  Off the nodes, from the logarithmic derivative of
 * the second barycentric form, l_k' = l_k (sum_m l_m/(tau - t_m)
 * - 1/(tau - t_k)) / h, written with the partition of unity as
 * l_k sum_{m != k} l_m (t_m - t_k) / ((tau - t_m)(tau - t_k)) / h so that no
 * two large terms cancel near a node.  At a node t_j the entries of the
 * differentiation matrix: (w_k / w_j)/(t_j - t_k) for k != j and minus
 * their sum for k = j. */
void orc_basis_deriv_1d(int p, double c, double h, double x, double *dl) {
  double t[32], w[32], l[32];
  orc_cheb_nodes(p, t);
  cheb_weights(p, w);
  double tau = (x - c) / h;
  for (int j = 0; j <= p; ++j) {
    if (tau == t[j]) {
      double diag = 0.0;
      for (int k = 0; k <= p; ++k) {
        if (k == j) continue;
        dl[k] = (w[k] / w[j]) / (t[j] - t[k]) / h;
        diag += dl[k];
      }
      dl[j] = -diag;
      return;
    }
  }
  orc_basis_1d(p, c, h, x, l);
  for (int k = 0; k <= p; ++k) {
    double s = 0.0;
    for (int m = 0; m <= p; ++m) {
      if (m == k) continue;
      s += l[m] * (t[m] - t[k]) / ((tau - t[m]) * (tau - t[k]));
    }
    dl[k] = l[k] * s / h;
  }
}

/* ------------------------------------------------------------------------ */
/* Gradients of L = sum_i (gE_i . E_i + gB_i . B_i) with respect to the      */
/* positions and charges.                                                   */
/* ------------------------------------------------------------------------ */

/* For one pair term g(r) . C with g = r D^{-3/2}, D = r^T S r:
 * d/dr = D^{-3/2} C - 3 D^{-5/2} (C . r) S r, S = diag(1, 1, gbar^2) for
 * MEAN and I + u_j u_j^T for EXACT. */
static void pair_grad(int mode, double gamma_bar, const double *r,
                      const double *uj, const double *C, double *out) {
  double Sr[3], D;
  if (mode == ORC_KERNEL_MEAN) {
    double gb2 = gamma_bar * gamma_bar;
    Sr[0] = r[0];
    Sr[1] = r[1];
    Sr[2] = gb2 * r[2];
  } else {
    double ur = uj[0] * r[0] + uj[1] * r[1] + uj[2] * r[2];
    for (int c = 0; c < 3; ++c) Sr[c] = r[c] + ur * uj[c];
  }
  D = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
  double d32 = 1.0 / (D * sqrt(D));
  double d52 = d32 / D;
  double cr = C[0] * r[0] + C[1] * r[1] + C[2] * r[2];
  for (int c = 0; c < 3; ++c) out[c] = d32 * C[c] - 3.0 * d52 * cr * Sr[c];
}

/* d/dgamma_bar of g(r) . C for the MEAN kernel: g = r D^{-3/2} with
 * D = rx^2 + ry^2 + gbar^2 rz^2, so dD/dgbar = 2 gbar rz^2 and
 * d(g . C)/dgbar = -3 gbar rz^2 D^{-5/2} (C . r).  The EXACT kernel does not
 * contain gamma_bar. */
static double pair_dgbar(int mode, double gamma_bar, const double *r,
                         const double *C) {
  if (mode != ORC_KERNEL_MEAN) return 0.0;
  double D = r[0] * r[0] + r[1] * r[1] + gamma_bar * gamma_bar * (r[2] * r[2]);
  double d52 = 1.0 / (D * D * sqrt(D));
  double cr = C[0] * r[0] + C[1] * r[1] + C[2] * r[2];
  return -3.0 * gamma_bar * (r[2] * r[2]) * d52 * cr;
}

/* d/du_j of g(r) . C through the denominator of the EXACT kernel,
 * D = |r|^2 + (u_j . r)^2, dD/du_j = 2 (u_j . r) r:
 * -3 (u_j . r) D^{-5/2} (C . r) r.  Zero for MEAN. */
static void pair_grad_u(int mode, const double *r, const double *uj,
                        const double *C, double *out) {
  out[0] = out[1] = out[2] = 0.0;
  if (mode == ORC_KERNEL_MEAN) return;
  double ur = uj[0] * r[0] + uj[1] * r[1] + uj[2] * r[2];
  double D = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) + ur * ur;
  double d52 = 1.0 / (D * D * sqrt(D));
  double cr = C[0] * r[0] + C[1] * r[1] + C[2] * r[2];
  for (int c = 0; c < 3; ++c) out[c] = -3.0 * ur * d52 * cr * r[c];
}

/* d gamma_bar / d u_j for gamma_bar^2 = 1 + |pbar|^2, pbar = (1/n) sum u:
 * pbar / (n gamma_bar), the same for every particle. */
static void dgbar_du(int64_t n, const double *u, double *out) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t j = 0; j < n; ++j)
    for (int c = 0; c < 3; ++c) s[c] += u[3 * j + c];
  double p[3] = {s[0] / (double)n, s[1] / (double)n, s[2] / (double)n};
  double gb = sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
  for (int c = 0; c < 3; ++c) out[c] = p[c] / ((double)n * gb);
}

/* Analytic O(N^2) gradient of the direct sum with respect to the momenta.
 * u_j enters the source weights q_j gamma_j (dgamma_j/du_j = u_j/gamma_j)
 * and q_j u_j, the EXACT denominator, and, if gbar_from_u, the mean Lorentz
 * factor of the MEAN kernel. */
void orc_direct_grad_u(int64_t n, const double *x, const double *u,
                       const double *q, double gamma_bar, int mode, double ke,
                       double c0, const double *gE, const double *gB,
                       int gbar_from_u, double *grad_u) {
  double kb = ke / c0;
  double *Gj = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < n; ++j) {
    double acc[3] = {0, 0, 0}, G = 0.0;
    double gj = lorentz(u + 3 * j);
    double wu[3] = {q[j] * u[3 * j], q[j] * u[3 * j + 1], q[j] * u[3 * j + 2]};
    for (int64_t i = 0; i < n; ++i) {
      if (i == j) continue;
      double r[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                     x[3 * i + 2] - x[3 * j + 2]};
      double eb[3] = {kb * gB[3 * i], kb * gB[3 * i + 1], kb * gB[3 * i + 2]};
      double g[3], gxb[3], bxw[3], C[3], du[3];
      orc_pair_kernel(mode, gamma_bar, r, u + 3 * j, g);
      /* through gamma_j in q_j gamma_j: ke q_j (gE_i . g) u_j / gamma_j */
      double eg = gE[3 * i] * g[0] + gE[3 * i + 1] * g[1] + gE[3 * i + 2] * g[2];
      for (int c = 0; c < 3; ++c) acc[c] += ke * q[j] * eg * u[3 * j + c] / gj;
      /* through q_j u_j in B: b . (u x g) = u . (g x b) */
      cross(g, eb, gxb);
      for (int c = 0; c < 3; ++c) acc[c] += q[j] * gxb[c];
      /* the pair's cotangent vector and the kernel's own dependence */
      cross(eb, wu, bxw);
      for (int c = 0; c < 3; ++c) C[c] = ke * q[j] * gj * gE[3 * i + c] + bxw[c];
      pair_grad_u(mode, r, u + 3 * j, C, du);
      for (int c = 0; c < 3; ++c) acc[c] += du[c];
      G += pair_dgbar(mode, gamma_bar, r, C);
    }
    for (int c = 0; c < 3; ++c) grad_u[3 * j + c] = acc[c];
    Gj[j] = G;
  }
  if (gbar_from_u) {
    double G = 0.0, dg[3];
    for (int64_t j = 0; j < n; ++j) G += Gj[j];
    dgbar_du(n, u, dg);
    for (int64_t j = 0; j < n; ++j)
      for (int c = 0; c < 3; ++c) grad_u[3 * j + c] += G * dg[c];
  }
  free(Gj);
}

/* Analytic O(N^2) gradient of the direct sum. */
void orc_direct_grad(int64_t n, const double *x, const double *u,
                     const double *q, double gamma_bar, int mode, double ke,
                     double c0, const double *gE, const double *gB,
                     double *grad_x, double *grad_q) {
  double kb = ke / c0;
  /* target side: d/dx_i of the terms with target i */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double acc[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                     x[3 * i + 2] - x[3 * j + 2]};
      double wu[3] = {q[j] * u[3 * j], q[j] * u[3 * j + 1],
                      q[j] * u[3 * j + 2]};
      double bxw[3], C[3], gr[3];
      double eb[3] = {kb * gB[3 * i], kb * gB[3 * i + 1], kb * gB[3 * i + 2]};
      cross(eb, wu, bxw);
      double w0 = q[j] * lorentz(u + 3 * j);
      for (int c = 0; c < 3; ++c) C[c] = ke * w0 * gE[3 * i + c] + bxw[c];
      pair_grad(mode, gamma_bar, r, u + 3 * j, C, gr);
      for (int c = 0; c < 3; ++c) acc[c] += gr[c];
    }
    for (int c = 0; c < 3; ++c) grad_x[3 * i + c] = acc[c];
  }
  /* source side: d/dx_j and d/dq_j of the terms with source j */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < n; ++j) {
    double acc[3] = {0, 0, 0}, aq = 0.0;
    double gj = lorentz(u + 3 * j);
    double wu[3] = {q[j] * u[3 * j], q[j] * u[3 * j + 1], q[j] * u[3 * j + 2]};
    double w0 = q[j] * gj;
    for (int64_t i = 0; i < n; ++i) {
      if (i == j) continue;
      double r[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1],
                     x[3 * i + 2] - x[3 * j + 2]};
      double eb[3] = {kb * gB[3 * i], kb * gB[3 * i + 1], kb * gB[3 * i + 2]};
      double bxw[3], bxu[3], C[3], gr[3], g[3];
      cross(eb, wu, bxw);
      for (int c = 0; c < 3; ++c) C[c] = ke * w0 * gE[3 * i + c] + bxw[c];
      pair_grad(mode, gamma_bar, r, u + 3 * j, C, gr);
      for (int c = 0; c < 3; ++c) acc[c] -= gr[c];
      orc_pair_kernel(mode, gamma_bar, r, u + 3 * j, g);
      cross(eb, u + 3 * j, bxu);
      for (int c = 0; c < 3; ++c) aq += (ke * gj * gE[3 * i + c] + bxu[c]) * g[c];
    }
    grad_q[j] = aq;
    for (int c = 0; c < 3; ++c) grad_x[3 * j + c] += acc[c];
  }
}

/* Transpose of the FMM with frozen structure, step by step: L2P^T, L2L^T,
 * M2L^T, M2M^T, P2M^T, the derivatives of the interpolation bases at the
 * particles (target and source side), and the transpose of P2P.  Needs a
 * completed forward run on the same positions (it reads the cumulative
 * local fields and the multipole weights). */
int orc_fmm_adjoint(orc_fmm *f, const double *gE, const double *gB,
                    double *grad_x, double *grad_q, double *grad_u,
                    int gbar_from_u) {
  const int64_t n = f->n, ns = f->nslots, m = f->m;
  const int q = f->p + 1;
  const double kb = f->ke / f->c0;
  double t[32];
  orc_cheb_nodes(f->p, t);
  double *eb = (double *)malloc(sizeof(double) * 6 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      eb[6 * i + c] = f->ke * gE[3 * i + c];
      eb[6 * i + 3 + c] = kb * gB[3 * i + c];
    }
  double *Lbar = (double *)calloc((size_t)(ns * m * 6), sizeof(double));
  double *Mbar = (double *)calloc((size_t)(ns * m * 4), sizeof(double));
  double *mbar = (double *)calloc((size_t)(4 * n), sizeof(double));
  /* momentum gradient: the EXACT denominator term per source, and the
   * gamma_bar derivative of the near (MEAN) and far sums per target node */
  double *gu = (double *)calloc((size_t)(3 * n), sizeof(double));
  double *Gp = (double *)calloc((size_t)ns, sizeof(double));
  double *Gm = (double *)calloc((size_t)ns, sizeof(double));
  for (int64_t i = 0; i < 3 * n; ++i) grad_x[i] = 0.0;
  /* L2P^T: Lbar_leaf[mu] = sum_i l_mu(x_i) (gE'_i, gB'_i) */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t S = 1; S < ns; ++S) {
    if (f->kind[S] != 1) continue;
    double lx[32], ly[32], lz[32];
    for (int64_t k = f->lo[S]; k < f->hi[S]; ++k) {
      int64_t i = f->perm[k];
      basis3(f, S, f->x + 3 * i, lx, ly, lz);
      for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
          for (int c = 0; c < q; ++c) {
            double l = lx[a] * ly[b] * lz[c];
            int64_t mu = (a * q + b) * q + c;
            for (int w = 0; w < 6; ++w)
              Lbar[(S * m + mu) * 6 + w] += l * eb[6 * i + w];
          }
    }
  }
  /* L2L^T: children to parents, deepest level first */
  for (int l = f->depth - 1; l >= 0; --l) {
    int64_t a0 = (int64_t)1 << l, b0 = (int64_t)1 << (l + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t S = a0; S < b0; ++S) {
      if (f->kind[S] != 2) continue;
      for (int64_t C = 2 * S; C <= 2 * S + 1; ++C) {
        double T[3 * 32 * 32];
        transfer_tables(f, S, C, t, T);
        for (int64_t mu = 0; mu < m; ++mu) {
          int a = (int)(mu / (q * q)), b = (int)((mu / q) % q), c = (int)(mu % q);
          for (int64_t mu2 = 0; mu2 < m; ++mu2) {
            int a2 = (int)(mu2 / (q * q)), b2 = (int)((mu2 / q) % q),
                c2 = (int)(mu2 % q);
            double tt = T[(0 * q + a) * q + a2] * T[(1 * q + b) * q + b2] *
                        T[(2 * q + c) * q + c2];
            for (int w = 0; w < 6; ++w)
              Lbar[(S * m + mu) * 6 + w] += tt * Lbar[(C * m + mu2) * 6 + w];
          }
        }
      }
    }
  }
  /* M2L^T: Mbar_s[nu] += sum_mu (g . Ebar_t[mu], g x Bbar_t[mu]) */
  {
    int64_t *start, *order;
    int64_t *swapped = (int64_t *)malloc(sizeof(int64_t) * 2 * (f->nm2l ? f->nm2l : 1));
    for (int64_t k = 0; k < f->nm2l; ++k) {
      swapped[2 * k] = f->m2l[2 * k + 1];
      swapped[2 * k + 1] = f->m2l[2 * k];
    }
    group_by_target(swapped, f->nm2l, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t Sn = 1; Sn < ns; ++Sn)
      for (int64_t k = start[Sn]; k < start[Sn + 1]; ++k) {
        int64_t T = swapped[2 * order[k] + 1];
        for (int64_t nu = 0; nu < m; ++nu) {
          int a2 = (int)(nu / (q * q)), b2 = (int)((nu / q) % q), c2 = (int)(nu % q);
          double xs[3] = {proxy(f, Sn, 0, a2, t), proxy(f, Sn, 1, b2, t),
                          proxy(f, Sn, 2, c2, t)};
          for (int64_t mu = 0; mu < m; ++mu) {
            int a = (int)(mu / (q * q)), b = (int)((mu / q) % q), c = (int)(mu % q);
            double r[3] = {proxy(f, T, 0, a, t) - xs[0],
                           proxy(f, T, 1, b, t) - xs[1],
                           proxy(f, T, 2, c, t) - xs[2]};
            double g[3], gxb[3];
            orc_pair_kernel(ORC_KERNEL_MEAN, f->gamma_bar, r, NULL, g);
            const double *Lb = Lbar + (T * m + mu) * 6;
            cross(g, Lb + 3, gxb);
            Mbar[(Sn * m + nu) * 4] += g[0] * Lb[0] + g[1] * Lb[1] + g[2] * Lb[2];
            for (int w = 0; w < 3; ++w) Mbar[(Sn * m + nu) * 4 + 1 + w] += gxb[w];
          }
        }
      }
    free(start);
    free(order);
    free(swapped);
  }
  /* M2M^T: parents to children, top level first */
  for (int l = 0; l < f->depth; ++l) {
    int64_t a0 = (int64_t)1 << l, b0 = (int64_t)1 << (l + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t S = a0; S < b0; ++S) {
      if (f->kind[S] != 2) continue;
      for (int64_t C = 2 * S; C <= 2 * S + 1; ++C) {
        double T[3 * 32 * 32];
        transfer_tables(f, S, C, t, T);
        for (int64_t nu2 = 0; nu2 < m; ++nu2) {
          int a2 = (int)(nu2 / (q * q)), b2 = (int)((nu2 / q) % q),
              c2 = (int)(nu2 % q);
          for (int64_t nu = 0; nu < m; ++nu) {
            int a = (int)(nu / (q * q)), b = (int)((nu / q) % q), c = (int)(nu % q);
            double tt = T[(0 * q + a) * q + a2] * T[(1 * q + b) * q + b2] *
                        T[(2 * q + c) * q + c2];
            for (int w = 0; w < 4; ++w)
              Mbar[(C * m + nu2) * 4 + w] += tt * Mbar[(S * m + nu) * 4 + w];
          }
        }
      }
    }
  }
  /* P2M^T and the basis derivatives at every particle of every leaf:
   * mbar_j = sum_nu l_nu(x_j) Mbar[nu];
   * grad_x_j += sum_nu grad l_nu(x_j) (m_j . Mbar[nu] + gE'_j . Lcum^E[nu]
   *                                    + gB'_j . Lcum^B[nu]) */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t S = 1; S < ns; ++S) {
    if (f->kind[S] != 1) continue;
    double lx[32], ly[32], lz[32], dx[32], dy[32], dz[32];
    for (int64_t k = f->lo[S]; k < f->hi[S]; ++k) {
      int64_t j = f->perm[k];
      const double *xj = f->x + 3 * j;
      basis3(f, S, xj, lx, ly, lz);
      orc_basis_deriv_1d(f->p, f->cen[3 * S], f->hw[3 * S], xj[0], dx);
      orc_basis_deriv_1d(f->p, f->cen[3 * S + 1], f->hw[3 * S + 1], xj[1], dy);
      orc_basis_deriv_1d(f->p, f->cen[3 * S + 2], f->hw[3 * S + 2], xj[2], dz);
      double gx[3] = {0, 0, 0};
      for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
          for (int c = 0; c < q; ++c) {
            int64_t nu = (a * q + b) * q + c;
            const double *Mb = Mbar + (S * m + nu) * 4;
            const double *Lc = f->Lcum + (S * m + nu) * 6;
            double l = lx[a] * ly[b] * lz[c];
            for (int w = 0; w < 4; ++w) mbar[4 * j + w] += l * Mb[w];
            double s = 0.0;
            for (int w = 0; w < 4; ++w) s += f->mw[4 * j + w] * Mb[w];
            for (int w = 0; w < 6; ++w) s += eb[6 * j + w] * Lc[w];
            gx[0] += dx[a] * ly[b] * lz[c] * s;
            gx[1] += lx[a] * dy[b] * lz[c] * s;
            gx[2] += lx[a] * ly[b] * dz[c] * s;
          }
      for (int w = 0; w < 3; ++w) grad_x[3 * j + w] += gx[w];
    }
  }
  /* P2P^T, target side (grouped by target) */
  {
    int64_t *start, *order;
    group_by_target(f->p2p, f->np2p, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t T = 1; T < ns; ++T)
      for (int64_t k = start[T]; k < start[T + 1]; ++k) {
        int64_t S = f->p2p[2 * order[k] + 1];
        for (int64_t a = f->lo[T]; a < f->hi[T]; ++a) {
          int64_t i = f->perm[a];
          for (int64_t b = f->lo[S]; b < f->hi[S]; ++b) {
            int64_t j = f->perm[b];
            if (j == i) continue;
            double r[3] = {f->x[3 * i] - f->x[3 * j], f->x[3 * i + 1] - f->x[3 * j + 1],
                           f->x[3 * i + 2] - f->x[3 * j + 2]};
            double bxw[3], C[3], gr[3];
            cross(eb + 6 * i + 3, f->mw + 4 * j + 1, bxw);
            for (int c = 0; c < 3; ++c) C[c] = f->mw[4 * j] * eb[6 * i + c] + bxw[c];
            pair_grad(f->mode, f->gamma_bar, r, f->uu + 3 * j, C, gr);
            for (int c = 0; c < 3; ++c) grad_x[3 * i + c] += gr[c];
            Gp[T] += pair_dgbar(f->mode, f->gamma_bar, r, C);
          }
        }
      }
    free(start);
    free(order);
  }
  /* P2P^T, source side (grouped by source) */
  {
    int64_t *start, *order;
    int64_t *swapped = (int64_t *)malloc(sizeof(int64_t) * 2 * (f->np2p ? f->np2p : 1));
    for (int64_t k = 0; k < f->np2p; ++k) {
      swapped[2 * k] = f->p2p[2 * k + 1];
      swapped[2 * k + 1] = f->p2p[2 * k];
    }
    group_by_target(swapped, f->np2p, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t S = 1; S < ns; ++S)
      for (int64_t k = start[S]; k < start[S + 1]; ++k) {
        int64_t T = swapped[2 * order[k] + 1];
        for (int64_t b = f->lo[S]; b < f->hi[S]; ++b) {
          int64_t j = f->perm[b];
          for (int64_t a = f->lo[T]; a < f->hi[T]; ++a) {
            int64_t i = f->perm[a];
            if (j == i) continue;
            double r[3] = {f->x[3 * i] - f->x[3 * j], f->x[3 * i + 1] - f->x[3 * j + 1],
                           f->x[3 * i + 2] - f->x[3 * j + 2]};
            double bxw[3], C[3], gr[3], g[3], gxb[3];
            cross(eb + 6 * i + 3, f->mw + 4 * j + 1, bxw);
            for (int c = 0; c < 3; ++c) C[c] = f->mw[4 * j] * eb[6 * i + c] + bxw[c];
            pair_grad(f->mode, f->gamma_bar, r, f->uu + 3 * j, C, gr);
            for (int c = 0; c < 3; ++c) grad_x[3 * j + c] -= gr[c];
            double du[3];
            pair_grad_u(f->mode, r, f->uu + 3 * j, C, du);
            for (int c = 0; c < 3; ++c) gu[3 * j + c] += du[c];
            orc_pair_kernel(f->mode, f->gamma_bar, r, f->uu + 3 * j, g);
            cross(g, eb + 6 * i + 3, gxb);
            mbar[4 * j] += g[0] * eb[6 * i] + g[1] * eb[6 * i + 1] + g[2] * eb[6 * i + 2];
            for (int c = 0; c < 3; ++c) mbar[4 * j + 1 + c] += gxb[c];
          }
        }
      }
    free(start);
    free(order);
    free(swapped);
  }
  /* charges: m_j = q_j (gamma_j, u_j) */
  for (int64_t j = 0; j < n; ++j) {
    double gj = lorentz(f->uu + 3 * j);
    grad_q[j] = gj * mbar[4 * j] + f->uu[3 * j] * mbar[4 * j + 1] +
                f->uu[3 * j + 1] * mbar[4 * j + 2] + f->uu[3 * j + 2] * mbar[4 * j + 3];
  }
  if (grad_u) {
    /* far field: d/dgamma_bar of sum over M2L pairs and proxies of
     * Lbar_t[mu] . (M^g_s[nu] g, M^u_s[nu] x g), g = g(xi_t,mu - xi_s,nu),
     * i.e. g . C with C = M^g Lbar^E + Lbar^B x M^u */
    int64_t *start, *order;
    group_by_target(f->m2l, f->nm2l, ns, &start, &order);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t T = 1; T < ns; ++T)
      for (int64_t k = start[T]; k < start[T + 1]; ++k) {
        int64_t S = f->m2l[2 * order[k] + 1];
        for (int64_t mu = 0; mu < m; ++mu) {
          int a = (int)(mu / (q * q)), b = (int)((mu / q) % q), c = (int)(mu % q);
          double xt[3] = {proxy(f, T, 0, a, t), proxy(f, T, 1, b, t),
                          proxy(f, T, 2, c, t)};
          const double *Lb = Lbar + (T * m + mu) * 6;
          for (int64_t nu = 0; nu < m; ++nu) {
            int a2 = (int)(nu / (q * q)), b2 = (int)((nu / q) % q), c2 = (int)(nu % q);
            double r[3] = {xt[0] - proxy(f, S, 0, a2, t), xt[1] - proxy(f, S, 1, b2, t),
                           xt[2] - proxy(f, S, 2, c2, t)};
            const double *Ms = f->M + (S * m + nu) * 4;
            double bxm[3], C[3];
            cross(Lb + 3, Ms + 1, bxm);
            for (int w = 0; w < 3; ++w) C[w] = Ms[0] * Lb[w] + bxm[w];
            Gm[T] += pair_dgbar(ORC_KERNEL_MEAN, f->gamma_bar, r, C);
          }
        }
      }
    free(start);
    free(order);
    double G = 0.0, dg[3] = {0.0, 0.0, 0.0};
    for (int64_t T = 1; T < ns; ++T) G += Gp[T] + Gm[T];
    if (gbar_from_u) dgbar_du(n, f->uu, dg);
    /* u_j enters q_j gamma_j and q_j u_j (mbar), the EXACT denominator (gu)
     * and gamma_bar (G) */
    for (int64_t j = 0; j < n; ++j) {
      double gj = lorentz(f->uu + 3 * j);
      for (int c = 0; c < 3; ++c)
        grad_u[3 * j + c] = f->qq[j] * (mbar[4 * j] * f->uu[3 * j + c] / gj +
                                        mbar[4 * j + 1 + c]) +
                            gu[3 * j + c] + G * dg[c];
    }
  }
  free(gu);
  free(Gp);
  free(Gm);
  free(eb);
  free(Lbar);
  free(Mbar);
  free(mbar);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Accessors.                                                               */
/* ------------------------------------------------------------------------ */

void orc_fmm_sizes(const orc_fmm *f, int64_t *out) {
  out[0] = f->depth;
  out[1] = f->nslots;
  out[2] = f->np2p;
  out[3] = f->nm2l;
  int64_t inter = 0;
  if (f->lo)
    for (int64_t k = 0; k < f->np2p; ++k) {
      int64_t T = f->p2p[2 * k], S = f->p2p[2 * k + 1];
      inter += (f->hi[T] - f->lo[T]) * (f->hi[S] - f->lo[S]);
    }
  out[4] = inter;
  out[5] = f->nm2l * f->m * f->m;
  out[6] = f->m;
}

void orc_fmm_get_tree(const orc_fmm *f, int64_t *perm, int64_t *lo,
                      int64_t *hi, int8_t *kind, int8_t *axis, double *bmin,
                      double *bmax, double *cen, double *hw) {
  int64_t ns = f->nslots;
  memcpy(perm, f->perm, sizeof(int64_t) * f->n);
  memcpy(lo, f->lo, sizeof(int64_t) * ns);
  memcpy(hi, f->hi, sizeof(int64_t) * ns);
  memcpy(kind, f->kind, ns);
  memcpy(axis, f->axis, ns);
  memcpy(bmin, f->bmin, sizeof(double) * 3 * ns);
  memcpy(bmax, f->bmax, sizeof(double) * 3 * ns);
  memcpy(cen, f->cen, sizeof(double) * 3 * ns);
  memcpy(hw, f->hw, sizeof(double) * 3 * ns);
}

void orc_fmm_get_lists(const orc_fmm *f, int64_t *p2p, int64_t *m2l) {
  if (f->np2p) memcpy(p2p, f->p2p, sizeof(int64_t) * 2 * f->np2p);
  if (f->nm2l) memcpy(m2l, f->m2l, sizeof(int64_t) * 2 * f->nm2l);
}

void orc_fmm_get_multipoles(const orc_fmm *f, double *M) {
  memcpy(M, f->M, sizeof(double) * f->nslots * f->m * 4);
}

void orc_fmm_get_locals(const orc_fmm *f, double *L, double *Lcum) {
  size_t nl = (size_t)(f->nslots * f->m * 6);
  if (L) memcpy(L, f->L, sizeof(double) * nl);
  if (Lcum) memcpy(Lcum, f->Lcum, sizeof(double) * nl);
}

void orc_fmm_get_fields(const orc_fmm *f, double *E, double *B, double *Enear,
                        double *Bnear) {
  size_t k = (size_t)(3 * f->n);
  if (E) memcpy(E, f->E, sizeof(double) * k);
  if (B) memcpy(B, f->B, sizeof(double) * k);
  if (Enear) memcpy(Enear, f->Enear, sizeof(double) * k);
  if (Bnear) memcpy(Bnear, f->Bnear, sizeof(double) * k);
}
