// C-ABI entry points of the relfmm library (declared in include/relfmm.h):
// parameter validation, workspace carving, and the order of the stages of
// Alg. FMM (Sec. 5): subdivide, upward pass, dual traversal lists, P2P and
// M2L, downward pass.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/relfmm.h"
#include "internal.hpp"

using namespace relfmm;

namespace {

thread_local std::string g_err;

relfmm_status fail(relfmm_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

constexpr double kDefaultKe = 1.0 / (4.0 * M_PI * 8.8541878128e-12);
constexpr double kDefaultC0 = 299792458.0;
constexpr int kDefaultP2PPerLeaf = 1024;
constexpr int kDefaultM2LPerNode = 256;

int tree_depth(int64_t n, int leaf) {
  int d = 0;
  while ((int64_t)leaf << d < n) ++d;
  return d;
}

// Largest leaf population of the tree the index split builds for n
// particles (App. B): the populations at level l are floor or ceil of
// n / 2^l, a node splits while it holds more than leaf_size particles and
// is above the last level, so leaves above the last level hold at most
// leaf_size and exist only where floor(n / 2^l) <= leaf_size.  The launch
// shapes of the leaf kernels follow this bound rather than leaf_size (after
// a depth transition the leaves hold about half of leaf_size).
int max_leaf_population(int64_t n, int leaf, int depth) {
  int64_t m = (n + ((int64_t)1 << depth) - 1) >> depth;  // last level
  for (int l = 0; l < depth; ++l)
    if ((n >> l) <= leaf) {  // floor(n / 2^l): leaves possible at level l
      m = std::max<int64_t>(m, std::min<int64_t>(leaf, (n + ((int64_t)1 << l) - 1) >> l));
      break;
    }
  return (int)std::min<int64_t>(m, n);
}

struct Sizes {
  int64_t n_max;
  int depth, ns, leaves;
  int64_t p2p_cap, m2l_cap, fcap;
  int m;
  int kslices;  // 64-particle slices of the largest leaf
  size_t hist, partial;
};

bool resolve(const relfmm_params *in, int64_t n_max, relfmm_params *out,
             Sizes *sz, std::string *why) {
  if (!in) return *why = "params is NULL", false;
  relfmm_params p = *in;
  if (p.degree < 1 || p.degree > kMaxDegree)
    return *why = "degree must be in 1.." + std::to_string(kMaxDegree), false;
  if (p.leaf_size < 1) return *why = "leaf_size must be >= 1", false;
  if (!(p.eta > 0.0) || !isfinite(p.eta))
    return *why = "eta must be finite and > 0", false;
  if (!isfinite(p.gamma_bar)) return *why = "gamma_bar must be finite", false;
  if (p.kernel != RELFMM_KERNEL_MEAN && p.kernel != RELFMM_KERNEL_SOURCE)
    return *why = "kernel must be RELFMM_KERNEL_MEAN or _SOURCE", false;
  if (p.p2p_prec != RELFMM_FP64 && p.p2p_prec != RELFMM_FP32)
    return *why = "p2p_prec must be RELFMM_FP64 or RELFMM_FP32", false;
  if (p.m2l_prec != RELFMM_FP64 && p.m2l_prec != RELFMM_FP32 &&
      p.m2l_prec != RELFMM_BF16 && p.m2l_prec != RELFMM_BF16X3)
    return *why = "m2l_prec must be RELFMM_FP64, RELFMM_FP32, RELFMM_BF16 or "
                  "RELFMM_BF16X3",
           false;
  // the factored M2L of the reduced-precision tiers loses accuracy to
  // cancellation as eta grows (measured 3e-6..9e-5 at eta = 0.6..0.7 against
  // <= 2e-6 up to 0.5); beyond the paper's range only FP64 M2L is offered
  if (p.m2l_prec != RELFMM_FP64 && p.eta > 0.5)
    return *why = "eta > 0.5 needs m2l_prec = RELFMM_FP64 (the FP32 and BF16 "
                  "M2L tiers are specified for eta <= 0.5)",
           false;
  if (!isfinite(p.ke) || !isfinite(p.c0))
    return *why = "ke and c0 must be finite", false;
  if (p.ke <= 0.0) p.ke = kDefaultKe;
  if (p.c0 <= 0.0) p.c0 = kDefaultC0;
  if (p.max_p2p_per_leaf <= 0) p.max_p2p_per_leaf = kDefaultP2PPerLeaf;
  if (p.max_m2l_per_node <= 0) p.max_m2l_per_node = kDefaultM2LPerNode;
  // 2^28 keeps every per-particle index (up to 6 n) in 32-bit integers; the
  // workspace for it (~950 bytes per particle) is within one MI355X's HBM
  if (n_max < 1 || n_max > (int64_t)1 << 28)
    return *why = "n_max must be in 1..2^28", false;
  Sizes s;
  s.n_max = n_max;
  s.depth = tree_depth(n_max, p.leaf_size);
  if (s.depth > 26) return *why = "tree too deep (n_max / leaf_size)", false;
  s.ns = 1 << (s.depth + 1);
  s.leaves = 1 << s.depth;
  const int64_t L = s.leaves, S = s.ns;
  s.p2p_cap = std::min(L * L, L * (int64_t)p.max_p2p_per_leaf);
  s.m2l_cap = std::min(S * S, S * (int64_t)p.max_m2l_per_node);
  s.fcap = s.p2p_cap + s.m2l_cap + 2;
  if (s.fcap > ((int64_t)1 << 31) - 4096)
    return *why = "interaction-list capacity exceeds 2^31", false;
  s.m = (p.degree + 1) * (p.degree + 1) * (p.degree + 1);
  s.kslices = (int)((std::min<int64_t>(n_max, p.leaf_size) + kWave - 1) / kWave);
  int64_t sort_n = std::max<int64_t>(3 * n_max + 3 * 4096, std::max(s.p2p_cap, s.m2l_cap));
  s.hist = radix_hist_entries((int)sort_n);
  int64_t scan_n = std::max<int64_t>(3 * n_max, (int64_t)s.hist);
  s.partial = (size_t)scan_blocks((int)scan_n) + 64;
  *out = p;
  *sz = s;
  return true;
}

struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Lay out the buffers of one plan in a workspace starting at base (NULL:
// only count).  adjoint = false leaves out the buffers only relfmm_adjoint
// uses (their pointers stay NULL) and near_parts > 0 bounds the near-field
// buffer to that many row parts per particle (at least 1).
size_t carve(const Sizes &s, bool fp32, char *base, Dev *d,
             bool adjoint = true, int near_parts = 0) {
  *d = Dev{};
  Carver c{base};
  const size_t n = (size_t)s.n_max, ns = (size_t)s.ns, m = (size_t)s.m;
  d->gbar = c.take<double>(1);
  d->gpart = c.take<double>(3 * kGammaBlocks);
  d->counters = c.take<int>(kCounters);
  d->inter = c.take<unsigned long long>(1);
  d->key = c.take<uint64_t>(3 * n);
  d->key_tmp = c.take<uint64_t>(3 * n);
  d->ord_all = c.take<uint32_t>(3 * n);
  d->ord_tmp_all = c.take<uint32_t>(3 * n);
  d->flag = c.take<uint8_t>(n);
  d->scanv = c.take<uint32_t>(3 * n);
  d->seg = c.take<int32_t>(n);
  d->seg_tmp = c.take<int32_t>(n);
  d->hist = c.take<uint32_t>(s.hist);
  d->partial = c.take<uint32_t>(s.partial);
  d->lo = c.take<int32_t>(ns);
  d->hi = c.take<int32_t>(ns);
  d->kind = c.take<int32_t>(ns);
  d->axis = c.take<int32_t>(ns);
  d->nleft = c.take<int32_t>(ns);
  d->bmin = c.take<double>(3 * ns);
  d->bmax = c.take<double>(3 * ns);
  d->cen = c.take<double>(3 * ns);
  d->hw = c.take<double>(3 * ns);
  d->r2 = c.take<double>(ns);
  d->xl = c.take<double>(3 * n);
  d->w = c.take<double>(4 * n);
  d->us = c.take<double>(3 * n);
  d->w32 = fp32 ? c.take<float>(4 * n) : nullptr;
  d->us32 = fp32 ? c.take<float>(3 * n) : nullptr;
  // one part per particle plus room for the extra row parts of small grids
  // (a split is only taken while the grid is small, so the extra room needed
  // is bounded): at least 2 parts, at most 2^21 extra particle-parts
  d->near_cap = 6 * (n + std::max(n, std::min(8 * n, (size_t)1 << 21)));
  if (near_parts > 0) d->near_cap = 6 * n * (size_t)near_parts;
  d->near = c.take<double>(d->near_cap);
  d->sbox = fp32 ? c.take<double>(6 * ns * (size_t)s.kslices) : nullptr;
  d->front[0] = c.take<int2>((size_t)s.fcap);
  d->front[1] = c.take<int2>((size_t)s.fcap);
  d->p2p = c.take<uint64_t>((size_t)s.p2p_cap);
  d->p2p_tmp = c.take<uint64_t>((size_t)s.p2p_cap);
  d->m2l = c.take<uint64_t>((size_t)s.m2l_cap);
  d->m2l_tmp = c.take<uint64_t>((size_t)s.m2l_cap);
  d->p2p_row = c.take<int32_t>(ns + 1);
  d->m2l_row = c.take<int32_t>(ns + 1);
  d->lfill = c.take<int32_t>(2 * (ns + 1));
  d->order_p2p = c.take<int32_t>(order_len((int)ns));
  d->order_m2l = c.take<int32_t>(order_len((int)ns));
  d->okey = c.take<uint64_t>(ns);
  d->okey_tmp = c.take<uint64_t>(ns);
  d->M = c.take<double>(ns * m * 4);
  d->mmax = c.take<double>(ns * 4);
  d->L = c.take<double>(ns * m * 6);
  if (!adjoint) return c.off + 256;
  // adjoint
  d->p2p_T = c.take<uint64_t>((size_t)s.p2p_cap);
  d->m2l_T = c.take<uint64_t>((size_t)s.m2l_cap);
  d->p2p_row_T = c.take<int32_t>(ns + 1);
  d->m2l_row_T = c.take<int32_t>(ns + 1);
  d->order_p2p_T = c.take<int32_t>(order_len((int)ns));
  d->order_m2l_T = c.take<int32_t>(order_len((int)ns));
  d->ebar = c.take<double>(6 * n);
  d->ebar32 = c.take<float>(6 * n);
  d->Lbar = c.take<double>(ns * m * 6);
  d->lmax = c.take<double>(ns * 6);
  d->Mbar = d->M;
  d->gx = c.take<double>(3 * n);
  d->mbar = c.take<double>(4 * n);
  d->gu = c.take<double>(3 * n);
  d->gG = c.take<double>(n);
  d->gdot = c.take<double>(ns * kGdotStride);
  d->gspart = c.take<double>(5 * kGsBlocks);
  d->gsum = c.take<double>(4);
  return c.off + 256;
}

Cheb make_cheb(int p) {
  Cheb cb;
  memset(&cb, 0, sizeof(cb));
  cb.p = p;
  for (int k = 0; k <= p; ++k) {
    cb.t[k] = sin(M_PI * (double)(p - 2 * k) / (2.0 * (double)p));
    double wk = (k % 2 == 0) ? 1.0 : -1.0;
    if (k == 0 || k == p) wk *= 0.5;
    cb.w[k] = wk;
  }
  // differentiation matrix of the barycentric interpolant at the nodes
  for (int j = 0; j <= p; ++j) {
    double diag = 0.0;
    for (int k = 0; k <= p; ++k) {
      if (k == j) continue;
      cb.D[j][k] = (cb.w[k] / cb.w[j]) / (cb.t[j] - cb.t[k]);
      diag += cb.D[j][k];
    }
    cb.D[j][j] = -diag;
  }
  return cb;
}

relfmm_status check_hip(hipError_t e, const char *where) {
  if (e == hipSuccess) return RELFMM_OK;
  return fail(RELFMM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

struct relfmm_plan {
  relfmm_params p;
  Sizes sz;
  bool fp32;
  void *ws;
  size_t ws_bytes;
  hipStream_t stream;
  int device;
  Dev d;
  Cheb cb;
  // last build
  int built_n = -1;
  int depth = 0, ns = 0, bits = 0, max_leaf = 0;
  ListArgs la = {};
  bool transposed = false;  // source-grouped lists exist for the last build
  // optional phase timing of relfmm_compute_fields: in the event set of the
  // call, ev[k] is recorded when phase k starts and ev[RELFMM_N_PHASES] when
  // the call ends (skipped phases take 0 ms).  Calls use a ring of kRing
  // sets; a set is read (harvested into sum_ms) before it is reused, so the
  // sums cover every timed call without a synchronization per call.
  static constexpr int kRing = 64;
  bool timing = false;
  bool in_call = false;
  hipEvent_t ev[kRing][RELFMM_N_PHASES + 1] = {};
  int64_t calls = 0;      // timed calls since the sums were last read
  int64_t harvested = 0;  // of them, added to sum_ms
  int cur = 0, last = -1; // set of the current and of the last timed call
  double sum_ms[RELFMM_N_PHASES] = {};
  // list overflow of a build: its flag is copied to pinned host memory after
  // the lists (ovf_ev) and read at the start of the next call on the plan
  int *ovf_host = nullptr;
  hipEvent_t ovf_ev = nullptr;
  bool ovf_pending = false;  // a build's flag is in flight
  bool ovf_struct = false;   // the current structure's lists overflowed
  bool ovf_report = false;   // ... and no call has reported it yet
  ~relfmm_plan() {
    for (auto &set : ev)
      for (auto &e : set)
        if (e) (void)hipEventDestroy(e);
    if (ovf_ev) (void)hipEventDestroy(ovf_ev);
    if (ovf_host) (void)hipHostFree(ovf_host);
  }
  void mark(int k) {
    if (timing && in_call) (void)hipEventRecord(ev[cur][k], stream);
  }
  // milliseconds of the phases of event set k (waits for it)
  hipError_t read_set(int k, double *ms) {
    hipError_t e = hipEventSynchronize(ev[k][RELFMM_N_PHASES]);
    for (int ph = 0; ph < RELFMM_N_PHASES && e == hipSuccess; ++ph) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, ev[k][ph], ev[k][ph + 1]);
      ms[ph] = (double)t;
    }
    return e;
  }
  hipError_t harvest_one() {
    double ms[RELFMM_N_PHASES];
    hipError_t e = read_set((int)(harvested % kRing), ms);
    if (e != hipSuccess) return e;
    for (int ph = 0; ph < RELFMM_N_PHASES; ++ph) sum_ms[ph] += ms[ph];
    ++harvested;
    return hipSuccess;
  }
  hipError_t begin_timed_call() {
    if (!timing) return hipSuccess;
    if (calls - harvested >= kRing) {
      hipError_t e = harvest_one();
      if (e != hipSuccess) return e;
    }
    cur = (int)(calls % kRing);
    in_call = true;
    return hipSuccess;
  }
  void end_timed_call() {
    if (!in_call) return;
    mark(RELFMM_N_PHASES);
    in_call = false;
    last = cur;
    ++calls;
  }
};

namespace {

// Make the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
      (void)hipSetDevice(prev);
  }
};

const char *kOverflowMsg =
    "the interaction lists of the last structure build overflowed their "
    "capacity (its fields and gradients are NaN); raise max_p2p_per_leaf / "
    "max_m2l_per_node";

// Read the overflow flag of the last build once its lists are done.  The
// first call after an overflowing build reports it (and does nothing else);
// calls that would reuse that structure keep reporting it.
relfmm_status settle_overflow(relfmm_plan *P, bool uses_structure) {
  if (P->ovf_pending) {
    relfmm_status st =
        check_hip(hipEventSynchronize(P->ovf_ev), "overflow event");
    if (st != RELFMM_OK) return st;
    P->ovf_pending = false;
    P->ovf_struct = *P->ovf_host != 0;
    P->ovf_report = P->ovf_struct;
  }
  if (P->ovf_report || (uses_structure && P->ovf_struct)) {
    P->ovf_report = false;
    return fail(RELFMM_ECAPACITY, kOverflowMsg);
  }
  return RELFMM_OK;
}

relfmm_status do_build(relfmm_plan *P, int n, const double *x,
                       const double *u) {
  const int depth = tree_depth(n, P->p.leaf_size);
  const int ns = 1 << (depth + 1);
  TreeArgs ta;
  ta.n = n;
  ta.depth = depth;
  ta.leaf_size = P->p.leaf_size;
  ta.ns = ns;
  ta.given_gbar = P->p.gamma_bar;
  P->mark(RELFMM_PHASE_TREE);
  build_tree_dev(P->d, ta, x, u, P->stream);
  P->mark(RELFMM_PHASE_LISTS);
  ListArgs la;
  la.ns = ns;
  la.depth = depth;
  la.bits = depth + 1;
  const int64_t L = (int64_t)1 << depth, S = ns;
  la.p2p_cap = (int)std::min(P->sz.p2p_cap,
                             std::min(L * L, L * (int64_t)P->p.max_p2p_per_leaf));
  la.m2l_cap = (int)std::min(P->sz.m2l_cap,
                             std::min(S * S, S * (int64_t)P->p.max_m2l_per_node));
  la.fcap = (int)P->sz.fcap;
  la.eta = P->p.eta;
  // XCD regions for the P2P order once the grid holds 8,192 chunks of 128
  // targets (the P2P launch is then not split into row parts)
  la.p2p_spatial = L * ((std::min(n, P->p.leaf_size) + 127) / 128) >= 8192;
  la.m2l_spatial = m2l_grouped(ns, P->p.degree);
  build_lists_dev(P->d, la, P->stream);
  relfmm_status st = check_hip(hipGetLastError(), "structure build launch");
  if (st != RELFMM_OK) return st;
  // (a plan without a host flag, that of relfmm_compute_fields_static,
  // reports an overflow through the NaN fields only)
  if (P->ovf_host) {
    st = check_hip(hipMemcpyAsync(P->ovf_host, P->d.counters + kCntOverflow,
                                  sizeof(int), hipMemcpyDeviceToHost,
                                  P->stream),
                   "overflow flag copy");
    if (st == RELFMM_OK)
      st = check_hip(hipEventRecord(P->ovf_ev, P->stream), "overflow event");
    if (st != RELFMM_OK) return st;
  }
  P->ovf_pending = P->ovf_host != nullptr;
  P->ovf_struct = false;
  P->ovf_report = false;
  P->la = la;
  P->transposed = false;
  P->built_n = n;
  P->depth = depth;
  P->ns = ns;
  P->bits = depth + 1;
  P->max_leaf = max_leaf_population(n, P->p.leaf_size, depth);
  return RELFMM_OK;
}

relfmm_status do_evaluate(relfmm_plan *P, int n, const double *x,
                          const double *u, const double *q, double *E,
                          double *B) {
  const Dev &d = P->d;
  hipStream_t st = P->stream;
  P->mark(RELFMM_PHASE_PREP);
  prep_leaf_order(d, n, P->ns, x, u, q, P->fp32, st);
  P->mark(RELFMM_PHASE_P2M);
  launch_p2m(d, P->cb, n, P->ns, st);
  P->mark(RELFMM_PHASE_M2M);
  for (int l = P->depth - 1; l >= 0; --l) launch_m2m_level(d, P->cb, l, st);
  P->mark(RELFMM_PHASE_M2L);
  M2LArgs ma;
  ma.ns = P->ns;
  ma.bits = P->bits;
  ma.prec = P->p.m2l_prec;
  launch_m2l(d, P->cb, ma, st);
  P->mark(RELFMM_PHASE_P2P);
  P2PArgs pa;
  pa.ns = P->ns;
  pa.bits = P->bits;
  pa.mode = P->p.kernel;
  pa.prec = P->p.p2p_prec;
  pa.max_leaf = P->max_leaf;
  launch_p2p(d, pa, n, st);
  P->mark(RELFMM_PHASE_L2L);
  for (int l = 1; l <= P->depth; ++l) launch_l2l_level(d, P->cb, l, st);
  P->mark(RELFMM_PHASE_L2P);
  launch_l2p_finalize(d, P->cb, n, P->ns, P->max_leaf, P->p.ke,
                      P->p.ke / P->p.c0, E, B, st);
  P->end_timed_call();
  return check_hip(hipGetLastError(), "evaluation launch");
}

relfmm_status do_adjoint(relfmm_plan *P, int n, const double *x,
                         const double *u, const double *q, const double *gE,
                         const double *gB, double *grad_x, double *grad_q,
                         double *grad_u) {
  const Dev &d = P->d;
  hipStream_t st = P->stream;
  if (!P->transposed) {
    build_transposed_lists_dev(d, P->la, st);
    P->transposed = true;
  }
  // forward far field on the frozen structure (the cumulative local fields
  // enter the target-side basis derivatives)
  prep_leaf_order(d, n, P->ns, x, u, q, P->fp32, st);
  launch_p2m(d, P->cb, n, P->ns, st);
  for (int l = P->depth - 1; l >= 0; --l) launch_m2m_level(d, P->cb, l, st);
  M2LArgs ma;
  ma.ns = P->ns;
  ma.bits = P->bits;
  ma.prec = P->p.m2l_prec;
  launch_m2l(d, P->cb, ma, st);
  for (int l = 1; l <= P->depth; ++l) launch_l2l_level(d, P->cb, l, st);
  // transposes, in reverse order
  launch_adj_prep(d, n, gE, gB, P->p.ke, P->p.ke / P->p.c0, st);
  launch_l2p_transpose(d, P->cb, n, P->ns, st);
  for (int l = P->depth - 1; l >= 0; --l)
    launch_l2l_transpose_level(d, P->cb, l, st);
  // M2L^T in the forward M2L's tier (FP64 VALU, FP32 MFMA, BF16, BF16x3);
  // the gbar-derivative M2L runs in FP32 for every reduced tier
  M2LArgs mt = ma;
  M2LArgs mg = ma;
  mg.prec = P->p.m2l_prec == RELFMM_FP64 ? 0 : 1;
  // momenta: the mean Lorentz factor is a function of u unless given; its
  // far-field derivative needs M and Lbar, before M2L^T overwrites M
  const bool gbar_u = grad_u && !(P->p.gamma_bar > 0.0);
  int nblk = 0;
  if (gbar_u) nblk = launch_m2l_dgbar(d, P->cb, mg, st);
  launch_m2l_adjoint(d, P->cb, mt, st);
  for (int l = 1; l <= P->depth; ++l)
    launch_m2m_transpose_level(d, P->cb, l, st);
  launch_adj_leaf(d, P->cb, n, P->ns, P->max_leaf, st);
  P2PArgs pa;
  pa.ns = P->ns;
  pa.bits = P->bits;
  pa.mode = P->p.kernel;
  pa.prec = P->p.p2p_prec;
  pa.max_leaf = P->max_leaf;
  const bool mean = P->p.kernel == RELFMM_KERNEL_MEAN;
  launch_p2p_adjoint(d, pa, n, gbar_u && mean, grad_u && !mean, st);
  launch_adj_final(d, n, grad_x, grad_q, st);
  if (grad_u) {
    if (gbar_u) launch_gbar_sums(d, n, P->ns, nblk, mean, st);
    launch_adj_final_u(d, n, !mean, gbar_u, grad_u, st);
  }
  return check_hip(hipGetLastError(), "adjoint launch");
}

}  // namespace

extern "C" {

const char *relfmm_last_error(void) { return g_err.c_str(); }

size_t relfmm_workspace_bytes(const relfmm_params *params, int64_t n_max) {
  relfmm_params p;
  Sizes s;
  std::string why;
  if (!resolve(params, n_max, &p, &s, &why)) return 0;
  Dev d;
  return carve(s, p.p2p_prec == RELFMM_FP32 || p.m2l_prec != RELFMM_FP64,
               nullptr, &d);
}

relfmm_status relfmm_plan_create(relfmm_plan **plan,
                                 const relfmm_params *params, int64_t n_max,
                                 void *workspace, size_t workspace_bytes,
                                 void *stream) {
  try {
    if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
    *plan = nullptr;
    relfmm_params p;
    Sizes s;
    std::string why;
    if (!resolve(params, n_max, &p, &s, &why)) return fail(RELFMM_EINVAL, why);
    if (!workspace) return fail(RELFMM_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0)
      return fail(RELFMM_EINVAL, "workspace must be 256-byte aligned");
    const bool fp32 = p.p2p_prec == RELFMM_FP32 || p.m2l_prec != RELFMM_FP64;
    Dev d;
    const size_t need = carve(s, fp32, nullptr, &d);
    if (workspace_bytes < need)
      return fail(RELFMM_ECAPACITY, "workspace too small: need " +
                                        std::to_string(need) + " bytes");
    relfmm_plan *P = new relfmm_plan();
    P->p = p;
    P->sz = s;
    P->fp32 = fp32;
    P->ws = workspace;
    P->ws_bytes = workspace_bytes;
    P->stream = (hipStream_t)stream;
    if (hipGetDevice(&P->device) != hipSuccess) {
      delete P;
      return fail(RELFMM_EDEVICE, "hipGetDevice failed");
    }
    carve(s, fp32, (char *)workspace, &P->d);
    P->cb = make_cheb(p.degree);
    if (hipHostMalloc((void **)&P->ovf_host, sizeof(int)) != hipSuccess ||
        hipEventCreateWithFlags(&P->ovf_ev, hipEventDisableTiming) !=
            hipSuccess) {
      delete P;
      return fail(RELFMM_EDEVICE, "cannot create the plan's overflow flag");
    }
    *P->ovf_host = 0;
    *plan = P;
    g_err.clear();
    return RELFMM_OK;
  } catch (const std::exception &e) {
    return fail(RELFMM_EINVAL, e.what());
  } catch (...) {
    return fail(RELFMM_EINVAL, "unknown error");
  }
}

void relfmm_plan_destroy(relfmm_plan *plan) { delete plan; }

relfmm_status relfmm_set_stream(relfmm_plan *plan, void *stream) {
  if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
  plan->stream = (hipStream_t)stream;
  return RELFMM_OK;
}

relfmm_status relfmm_build_tree(relfmm_plan *plan, int64_t n, const double *x,
                                const double *u) {
  try {
    if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
    if (n < 1) return fail(RELFMM_EINVAL, "n must be >= 1");
    if (n > plan->sz.n_max) return fail(RELFMM_ECAPACITY, "n exceeds n_max");
    if (!x || !u) return fail(RELFMM_EINVAL, "x and u must be non-NULL");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(RELFMM_EDEVICE, "cannot select the plan's device");
    relfmm_status st = check_hip(hipGetLastError(), "pending device error");
    if (st != RELFMM_OK) return st;
    st = settle_overflow(plan, false);
    if (st != RELFMM_OK) return st;
    return do_build(plan, (int)n, x, u);
  } catch (...) {
    return fail(RELFMM_EDEVICE, "unexpected exception");
  }
}

relfmm_status relfmm_compute_fields(relfmm_plan *plan, int64_t n,
                                    const double *x, const double *u,
                                    const double *q, double *E, double *B,
                                    int32_t rebuild) {
  try {
    if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
    if (n < 1) return fail(RELFMM_EINVAL, "n must be >= 1");
    if (n > plan->sz.n_max) return fail(RELFMM_ECAPACITY, "n exceeds n_max");
    if (!x || !u || !q || !E || !B)
      return fail(RELFMM_EINVAL, "x, u, q, E and B must be non-NULL");
    if (rebuild != 0 && rebuild != 1)
      return fail(RELFMM_EINVAL, "rebuild must be 0 or 1");
    if (!rebuild && plan->built_n != (int)n)
      return fail(RELFMM_ESTATE,
                  "rebuild=0 needs a structure built for the same n");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(RELFMM_EDEVICE, "cannot select the plan's device");
    relfmm_status st = check_hip(hipGetLastError(), "pending device error");
    if (st != RELFMM_OK) return st;
    st = settle_overflow(plan, !rebuild);
    if (st != RELFMM_OK) return st;
    st = check_hip(plan->begin_timed_call(), "timing events");
    if (st != RELFMM_OK) return st;
    if (rebuild) {
      st = do_build(plan, (int)n, x, u);
      if (st != RELFMM_OK) {
        plan->in_call = false;
        return st;
      }
    } else {
      plan->mark(RELFMM_PHASE_TREE);
      plan->mark(RELFMM_PHASE_LISTS);
    }
    return do_evaluate(plan, (int)n, x, u, q, E, B);
  } catch (...) {
    return fail(RELFMM_EDEVICE, "unexpected exception");
  }
}

relfmm_status relfmm_adjoint(relfmm_plan *plan, int64_t n, const double *x,
                             const double *u, const double *q,
                             const double *gE, const double *gB,
                             double *grad_x, double *grad_q, double *grad_u,
                             int32_t rebuild) {
  try {
    if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
    if (n < 1) return fail(RELFMM_EINVAL, "n must be >= 1");
    if (n > plan->sz.n_max) return fail(RELFMM_ECAPACITY, "n exceeds n_max");
    if (!x || !u || !q || !gE || !gB || !grad_x || !grad_q)
      return fail(RELFMM_EINVAL,
                  "x, u, q, gE, gB, grad_x and grad_q must be non-NULL");
    if (rebuild != 0 && rebuild != 1)
      return fail(RELFMM_EINVAL, "rebuild must be 0 or 1");
    if (!rebuild && plan->built_n != (int)n)
      return fail(RELFMM_ESTATE,
                  "rebuild=0 needs a structure built for the same n");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(RELFMM_EDEVICE, "cannot select the plan's device");
    relfmm_status st = check_hip(hipGetLastError(), "pending device error");
    if (st != RELFMM_OK) return st;
    st = settle_overflow(plan, !rebuild);
    if (st != RELFMM_OK) return st;
    if (rebuild) {
      st = do_build(plan, (int)n, x, u);
      if (st != RELFMM_OK) return st;
    }
    return do_adjoint(plan, (int)n, x, u, q, gE, gB, grad_x, grad_q, grad_u);
  } catch (...) {
    return fail(RELFMM_EDEVICE, "unexpected exception");
  }
}

relfmm_status relfmm_set_timing(relfmm_plan *plan, int32_t enable) {
  if (!plan) return fail(RELFMM_EINVAL, "plan is NULL");
  if (enable && !plan->ev[0][0]) {
    DeviceGuard g(plan->device);
    for (auto &set : plan->ev)
      for (auto &e : set) {
        relfmm_status st = check_hip(hipEventCreate(&e), "hipEventCreate");
        if (st != RELFMM_OK) return st;
      }
  }
  if (enable && !plan->timing) {
    plan->calls = plan->harvested = 0;
    plan->last = -1;
    for (double &v : plan->sum_ms) v = 0.0;
  }
  plan->timing = enable != 0;
  return RELFMM_OK;
}

relfmm_status relfmm_get_timings(relfmm_plan *plan, double *ms, int32_t count) {
  if (!plan || !ms) return fail(RELFMM_EINVAL, "plan and ms must be non-NULL");
  if (count < RELFMM_N_PHASES)
    return fail(RELFMM_EINVAL, "ms must hold RELFMM_N_PHASES values");
  if (!plan->timing || plan->last < 0)
    return fail(RELFMM_ESTATE, "timing is not enabled or no call was timed");
  DeviceGuard g(plan->device);
  return check_hip(plan->read_set(plan->last, ms), "timing events");
}

relfmm_status relfmm_get_timing_sums(relfmm_plan *plan, double *ms,
                                     int32_t count, int64_t *calls) {
  if (!plan || !ms || !calls)
    return fail(RELFMM_EINVAL, "plan, ms and calls must be non-NULL");
  if (count < RELFMM_N_PHASES)
    return fail(RELFMM_EINVAL, "ms must hold RELFMM_N_PHASES values");
  if (!plan->timing) return fail(RELFMM_ESTATE, "timing is not enabled");
  DeviceGuard g(plan->device);
  while (plan->harvested < plan->calls) {
    relfmm_status st = check_hip(plan->harvest_one(), "timing events");
    if (st != RELFMM_OK) return st;
  }
  for (int k = 0; k < RELFMM_N_PHASES; ++k) {
    ms[k] = plan->sum_ms[k];
    plan->sum_ms[k] = 0.0;
  }
  *calls = plan->calls;
  plan->calls = plan->harvested = 0;
  return RELFMM_OK;
}

relfmm_status relfmm_direct_fields(int64_t n, const double *x, const double *u,
                                   const double *q, int64_t n_targets,
                                   const int64_t *targets, int32_t kernel,
                                   double gamma_bar, double ke, double c0,
                                   double *E, double *B, void *stream) {
  if (n < 1 || n > ((int64_t)1 << 28))
    return fail(RELFMM_EINVAL, "n must be in 1..2^28");
  if (n_targets < 0 || n_targets > ((int64_t)1 << 28))
    return fail(RELFMM_EINVAL, "n_targets must be in 0..2^28");
  if (!x || !u || !q || !E || !B)
    return fail(RELFMM_EINVAL, "x, u, q, E and B must be non-NULL");
  if (kernel != RELFMM_KERNEL_MEAN && kernel != RELFMM_KERNEL_SOURCE)
    return fail(RELFMM_EINVAL, "kernel must be RELFMM_KERNEL_MEAN or _SOURCE");
  if (kernel == RELFMM_KERNEL_MEAN && !(gamma_bar > 0.0 && isfinite(gamma_bar)))
    return fail(RELFMM_EINVAL, "the mean kernel needs gamma_bar > 0");
  if (!isfinite(ke) || !isfinite(c0))
    return fail(RELFMM_EINVAL, "ke and c0 must be finite");
  if (n_targets == 0) return RELFMM_OK;
  if (ke <= 0.0) ke = kDefaultKe;
  if (c0 <= 0.0) c0 = kDefaultC0;
  relfmm_status st = check_hip(hipGetLastError(), "pending device error");
  if (st != RELFMM_OK) return st;
  launch_direct((int)n, x, u, q, (int)n_targets, targets, kernel, gamma_bar,
                ke, ke / c0, E, B, (hipStream_t)stream);
  return check_hip(hipGetLastError(), "direct-sum launch");
}

relfmm_status relfmm_get_stats(relfmm_plan *plan, relfmm_stats *out) {
  if (!plan || !out) return fail(RELFMM_EINVAL, "plan and out must be non-NULL");
  if (plan->built_n < 0) return fail(RELFMM_ESTATE, "no structure built yet");
  DeviceGuard g(plan->device);
  int cnt[kCounters];
  unsigned long long inter = 0;
  double gb = 0.0;
  count_interactions_dev(plan->d, plan->la, plan->stream);
  relfmm_status st = check_hip(
      hipMemcpyAsync(cnt, plan->d.counters, sizeof(cnt), hipMemcpyDeviceToHost,
                     plan->stream),
      "stats copy");
  if (st == RELFMM_OK)
    st = check_hip(hipMemcpyAsync(&inter, plan->d.inter, sizeof(inter),
                                  hipMemcpyDeviceToHost, plan->stream),
                   "stats copy");
  if (st == RELFMM_OK)
    st = check_hip(hipMemcpyAsync(&gb, plan->d.gbar, sizeof(gb),
                                  hipMemcpyDeviceToHost, plan->stream),
                   "stats copy");
  if (st == RELFMM_OK)
    st = check_hip(hipStreamSynchronize(plan->stream), "stream synchronize");
  if (st != RELFMM_OK) return st;
  const int64_t m = (int64_t)(plan->p.degree + 1) * (plan->p.degree + 1) *
                    (plan->p.degree + 1);
  out->n = plan->built_n;
  out->depth = plan->depth;
  out->overflow = cnt[kCntOverflow];
  out->n_nodes = plan->ns;
  out->n_p2p_pairs = cnt[kCntP2P];
  out->n_m2l_pairs = cnt[kCntM2L];
  out->p2p_interactions = (int64_t)inter;
  out->m2l_entries = (int64_t)cnt[kCntM2L] * m * m;
  out->gamma_bar = gb;
  // the stream is drained: the last build's overflow flag is known, and this
  // call reports it
  if (plan->ovf_pending) {
    plan->ovf_pending = false;
    plan->ovf_struct = *plan->ovf_host != 0;
  }
  plan->ovf_report = false;
  if (cnt[kCntOverflow])
    return fail(RELFMM_ECAPACITY,
                "an interaction list overflowed its capacity (flags " +
                    std::to_string(cnt[kCntOverflow]) +
                    "); raise max_p2p_per_leaf / max_m2l_per_node");
  return RELFMM_OK;
}

size_t relfmm_export_bytes(relfmm_plan *plan, int32_t what) {
  if (!plan || plan->built_n < 0) return 0;
  const size_t ns = plan->ns, n = plan->built_n;
  const size_t m = (size_t)(plan->p.degree + 1) * (plan->p.degree + 1) *
                   (plan->p.degree + 1);
  int cnt[kCounters];
  switch (what) {
    case RELFMM_EXPORT_NODES: return ns * 4 * sizeof(int32_t);
    case RELFMM_EXPORT_BOXES: return ns * 6 * sizeof(double);
    case RELFMM_EXPORT_PERM: return n * sizeof(int32_t);
    case RELFMM_EXPORT_P2P:
    case RELFMM_EXPORT_M2L: {
      DeviceGuard g(plan->device);
      if (hipMemcpyAsync(cnt, plan->d.counters, sizeof(cnt),
                         hipMemcpyDeviceToHost, plan->stream) != hipSuccess ||
          hipStreamSynchronize(plan->stream) != hipSuccess)
        return 0;
      int c = cnt[what == RELFMM_EXPORT_P2P ? kCntP2P : kCntM2L];
      return (size_t)c * 2 * sizeof(int32_t);
    }
    case RELFMM_EXPORT_MULTIPOLES: return ns * m * 4 * sizeof(double);
    case RELFMM_EXPORT_LOCALS: return ns * m * 6 * sizeof(double);
    case RELFMM_EXPORT_NEAR: return n * 6 * sizeof(double);
    case RELFMM_EXPORT_GAMMA_BAR: return sizeof(double);
    case RELFMM_EXPORT_LOCAL_COTANGENTS: return ns * m * 6 * sizeof(double);
    case RELFMM_EXPORT_INTERP_BOXES: return ns * 6 * sizeof(double);
    default: return 0;
  }
}

relfmm_status relfmm_export(relfmm_plan *plan, int32_t what, void *host_dst,
                            size_t bytes) {
  try {
    if (!plan || !host_dst) return fail(RELFMM_EINVAL, "NULL argument");
    if (plan->built_n < 0) return fail(RELFMM_ESTATE, "no structure built yet");
    const size_t need = relfmm_export_bytes(plan, what);
    if (need == 0 && what != RELFMM_EXPORT_P2P && what != RELFMM_EXPORT_M2L)
      return fail(RELFMM_EINVAL, "unknown export id");
    if (bytes < need)
      return fail(RELFMM_ECAPACITY, "destination too small: need " +
                                        std::to_string(need) + " bytes");
    DeviceGuard g(plan->device);
    const Dev &d = plan->d;
    const size_t ns = plan->ns, n = plan->built_n;
    hipStream_t st = plan->stream;
    auto get = [&](void *dst, const void *src, size_t b) {
      return hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, st);
    };
    hipError_t e = hipSuccess;
    switch (what) {
      case RELFMM_EXPORT_NODES: {
        std::vector<int32_t> a(ns), b(ns), c(ns), dd(ns);
        e = get(a.data(), d.lo, ns * 4);
        if (!e) e = get(b.data(), d.hi, ns * 4);
        if (!e) e = get(c.data(), d.kind, ns * 4);
        if (!e) e = get(dd.data(), d.axis, ns * 4);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        int32_t *o = (int32_t *)host_dst;
        for (size_t i = 0; i < ns; ++i) {
          const bool ex = c[i] != 0;
          o[4 * i] = ex ? a[i] : -1;
          o[4 * i + 1] = ex ? b[i] : -1;
          o[4 * i + 2] = c[i];
          o[4 * i + 3] = ex ? dd[i] : -1;
        }
        break;
      }
      case RELFMM_EXPORT_BOXES: {
        std::vector<double> a(3 * ns), b(3 * ns);
        e = get(a.data(), d.bmin, ns * 24);
        if (!e) e = get(b.data(), d.bmax, ns * 24);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        double *o = (double *)host_dst;
        for (size_t i = 0; i < ns; ++i)
          for (int g2 = 0; g2 < 3; ++g2) {
            o[6 * i + g2] = a[3 * i + g2];
            o[6 * i + 3 + g2] = b[3 * i + g2];
          }
        break;
      }
      case RELFMM_EXPORT_INTERP_BOXES: {
        std::vector<double> a(3 * ns), b(3 * ns);
        e = get(a.data(), d.cen, ns * 24);
        if (!e) e = get(b.data(), d.hw, ns * 24);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        std::vector<int32_t> k(ns);
        e = get(k.data(), d.kind, ns * 4);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        double *o = (double *)host_dst;
        for (size_t i = 0; i < ns; ++i)
          for (int g2 = 0; g2 < 3; ++g2) {
            o[6 * i + g2] = k[i] ? a[3 * i + g2] : 0.0;
            o[6 * i + 3 + g2] = k[i] ? b[3 * i + g2] : 0.0;
          }
        break;
      }
      case RELFMM_EXPORT_PERM:
        e = get(host_dst, d.ord_all, n * 4);
        if (!e) e = hipStreamSynchronize(st);
        break;
      case RELFMM_EXPORT_P2P:
      case RELFMM_EXPORT_M2L: {
        const size_t c = need / 8;
        std::vector<uint64_t> k(c);
        if (c) e = get(k.data(), what == RELFMM_EXPORT_P2P ? d.p2p : d.m2l, c * 8);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        int32_t *o = (int32_t *)host_dst;
        const uint64_t mask = (1ull << plan->bits) - 1ull;
        for (size_t i = 0; i < c; ++i) {
          o[2 * i] = (int32_t)(k[i] >> plan->bits);
          o[2 * i + 1] = (int32_t)(k[i] & mask);
        }
        break;
      }
      case RELFMM_EXPORT_MULTIPOLES:
        e = get(host_dst, d.M, need);
        if (!e) e = hipStreamSynchronize(st);
        break;
      case RELFMM_EXPORT_LOCALS:
        e = get(host_dst, d.L, need);
        if (!e) e = hipStreamSynchronize(st);
        break;
      case RELFMM_EXPORT_NEAR: {
        std::vector<double> a(6 * n);
        std::vector<uint32_t> o(n);
        e = get(a.data(), d.near, 6 * n * 8);
        if (!e) e = get(o.data(), d.ord_all, n * 4);
        if (!e) e = hipStreamSynchronize(st);
        if (e) break;
        double *out = (double *)host_dst;
        for (size_t p = 0; p < n; ++p)
          for (int k2 = 0; k2 < 6; ++k2) out[6 * (size_t)o[p] + k2] = a[k2 * n + p];
        break;
      }
      case RELFMM_EXPORT_GAMMA_BAR:
        e = get(host_dst, d.gbar, 8);
        if (!e) e = hipStreamSynchronize(st);
        break;
      case RELFMM_EXPORT_LOCAL_COTANGENTS:
        e = get(host_dst, d.Lbar, need);
        if (!e) e = hipStreamSynchronize(st);
        break;
      default:
        return fail(RELFMM_EINVAL, "unknown export id");
    }
    return check_hip(e, "export");
  } catch (...) {
    return fail(RELFMM_EDEVICE, "unexpected exception");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// relfmm_compute_fields_static: the workspace of a one-shot forward plan in a
// device array of the library, for callers that cannot allocate.  In host
// code the array's name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress, once per device (with that device
// current), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[RELFMM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the current device's), looked
// up on its first use.
relfmm_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(RELFMM_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    relfmm_status st = check_hip(
        hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (st != RELFMM_OK) return st;
    if (!ptr || ((uintptr_t)ptr & 255) != 0)
      return fail(RELFMM_EDEVICE, "scratch symbol address is not aligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RELFMM_OK;
}
}  // namespace

extern "C" relfmm_status relfmm_compute_fields_static(
    const relfmm_params *params, int64_t n, const double *x, const double *u,
    const double *q, double *E, double *B, void *stream) {
  try {
    if (n < 1) return fail(RELFMM_EINVAL, "n must be >= 1");
    relfmm_params p;
    Sizes s;
    std::string why;
    if (!resolve(params, n, &p, &s, &why)) return fail(RELFMM_EINVAL, why);
    if (!x || !u || !q || !E || !B)
      return fail(RELFMM_EINVAL, "x, u, q, E and B must be non-NULL");
    const bool fp32 = p.p2p_prec == RELFMM_FP32 || p.m2l_prec != RELFMM_FP64;
    // forward buffers only; near field in at most two row parts
    Dev d;
    const size_t need = carve(s, fp32, nullptr, &d, false, 2);
    if (need > (size_t)RELFMM_STATIC_SCRATCH_BYTES)
      return fail(RELFMM_ECAPACITY,
                  "relfmm_compute_fields_static: these parameters and n need " +
                      std::to_string(need) + " bytes of scratch, more than "
                      "its " + std::to_string((size_t)RELFMM_STATIC_SCRATCH_BYTES) +
                      " (use a plan with a workspace)");
    int dev = -1;
    relfmm_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != RELFMM_OK) return st;
    st = check_hip(hipGetLastError(), "pending device error");
    if (st != RELFMM_OK) return st;
    void *base = nullptr;
    st = scratch_address(dev, &base);
    if (st != RELFMM_OK) return st;
    // a plan on the host stack: no events, no host flag, nothing allocated
    relfmm_plan P;
    P.p = p;
    P.sz = s;
    P.fp32 = fp32;
    P.ws = base;
    P.ws_bytes = RELFMM_STATIC_SCRATCH_BYTES;
    P.stream = (hipStream_t)stream;
    P.device = dev;
    carve(s, fp32, (char *)base, &P.d, false, 2);
    P.cb = make_cheb(p.degree);
    st = do_build(&P, (int)n, x, u);
    if (st != RELFMM_OK) return st;
    return do_evaluate(&P, (int)n, x, u, q, E, B);
  } catch (...) {
    return fail(RELFMM_EDEVICE, "unexpected exception");
  }
}
