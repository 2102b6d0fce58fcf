"""FP64 CPU oracle of the relativistic space-charge FMM (arXiv 2302.07567).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and the
two share no code.

This module is a thin ctypes wrapper over ``relfmm_oracle.c``; the arithmetic
lives there.  Physical constants (SI, CODATA 2018):
  ke = 1/(4 pi eps0), eps0 = 8.8541878128e-12 F/m;  c0 = 299792458 m/s.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

EPS0 = 8.8541878128e-12
KE = 1.0 / (4.0 * np.pi * EPS0)
C0 = 299792458.0

MEAN = 0
EXACT = 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or (
                os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build()
        _lib = load(path)
    return _lib


def load(path):
    """Load an oracle library from path with its signatures declared (the
    tests also load deliberately mutated builds through this)."""
    L = C.CDLL(path)
    i64, dbl, vp = C.c_int64, C.c_double, C.c_void_p
    L.orc_set_num_threads.restype = None
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_get_num_threads.restype = C.c_int
    L.orc_get_num_threads.argtypes = []
    L.orc_gamma_bar.restype = dbl
    L.orc_gamma_bar.argtypes = [i64, vp]
    L.orc_pair_kernel.restype = None
    L.orc_pair_kernel.argtypes = [C.c_int, dbl, vp, vp, vp]
    L.orc_direct.restype = None
    L.orc_direct.argtypes = [i64, vp, vp, vp, dbl, C.c_int, dbl, dbl, i64,
                             vp, vp, vp]
    L.orc_cheb_nodes.restype = None
    L.orc_cheb_nodes.argtypes = [C.c_int, vp]
    L.orc_basis_1d.restype = None
    L.orc_basis_1d.argtypes = [C.c_int, dbl, dbl, dbl, vp]
    L.orc_fmm_create.restype = vp
    L.orc_fmm_create.argtypes = [i64, C.c_int, C.c_int, dbl, dbl, C.c_int,
                                 dbl, dbl]
    L.orc_fmm_destroy.restype = None
    L.orc_fmm_destroy.argtypes = [vp]
    for name in ("orc_fmm_build_lists", "orc_fmm_m2l", "orc_fmm_p2p",
                 "orc_fmm_downward"):
        getattr(L, name).restype = C.c_int
        getattr(L, name).argtypes = [vp]
    L.orc_fmm_build_tree.restype = C.c_int
    L.orc_fmm_build_tree.argtypes = [vp, vp]
    L.orc_fmm_upward.restype = C.c_int
    L.orc_fmm_upward.argtypes = [vp, vp, vp]
    L.orc_fmm_sizes.restype = None
    L.orc_fmm_sizes.argtypes = [vp, vp]
    L.orc_fmm_get_tree.restype = None
    L.orc_fmm_get_tree.argtypes = [vp] * 10
    L.orc_fmm_get_lists.restype = None
    L.orc_fmm_get_lists.argtypes = [vp] * 3
    L.orc_fmm_get_multipoles.restype = None
    L.orc_fmm_get_multipoles.argtypes = [vp] * 2
    L.orc_fmm_get_locals.restype = None
    L.orc_fmm_get_locals.argtypes = [vp] * 3
    L.orc_fmm_get_fields.restype = None
    L.orc_fmm_get_fields.argtypes = [vp] * 5
    L.orc_fmm_set_positions.restype = C.c_int
    L.orc_fmm_set_positions.argtypes = [vp, vp]
    L.orc_basis_deriv_1d.restype = None
    L.orc_basis_deriv_1d.argtypes = [C.c_int, dbl, dbl, dbl, vp]
    L.orc_direct_grad.restype = None
    L.orc_direct_grad.argtypes = [i64, vp, vp, vp, dbl, C.c_int, dbl, dbl,
                                  vp, vp, vp, vp]
    L.orc_fmm_adjoint.restype = C.c_int
    L.orc_fmm_adjoint.argtypes = [vp] * 6 + [C.c_int]
    L.orc_fmm_set_gamma_bar.restype = C.c_int
    L.orc_fmm_set_gamma_bar.argtypes = [vp, dbl]
    L.orc_direct_grad_u.restype = None
    L.orc_direct_grad_u.argtypes = [i64, vp, vp, vp, dbl, C.c_int, dbl,
                                    dbl, vp, vp, C.c_int, vp]
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def set_threads(n):
    """OpenMP threads of the oracle's loops over independent targets."""
    lib().orc_set_num_threads(int(n))


def threads():
    return int(lib().orc_get_num_threads())


def gamma_bar(u):
    """Sec. 3: mean Lorentz factor from the unweighted mean momentum."""
    u = _f64(u, (-1, 3))
    return lib().orc_gamma_bar(u.shape[0], _p(u))


def pair_kernel(r, uj=None, gamma_bar_=1.0, mode=MEAN):
    r = _f64(r, (3,))
    uj = _f64(uj if uj is not None else np.zeros(3), (3,))
    g = np.zeros(3)
    lib().orc_pair_kernel(mode, float(gamma_bar_), _p(r), _p(uj), _p(g))
    return g


def direct(x, u, q, gamma_bar_, mode=MEAN, targets=None, ke=KE, c0=C0):
    """O(N^2) direct sum of eq. (fmm_pp_force_field), j != i."""
    x = _f64(x, (-1, 3))
    u = _f64(u, (-1, 3))
    q = _f64(q, (-1,))
    n = x.shape[0]
    if targets is None:
        nt, tg = n, None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.shape[0]
    E = np.zeros((nt, 3))
    B = np.zeros((nt, 3))
    lib().orc_direct(n, _p(x), _p(u), _p(q), float(gamma_bar_), int(mode),
                     float(ke), float(c0), nt, _p(tg), _p(E), _p(B))
    return E, B


def cheb_nodes(p):
    t = np.zeros(p + 1)
    lib().orc_cheb_nodes(int(p), _p(t))
    return t


def basis_1d(p, c, h, x):
    out = np.zeros(p + 1)
    lib().orc_basis_1d(int(p), float(c), float(h), float(x), _p(out))
    return out


def basis_deriv_1d(p, c, h, x):
    out = np.zeros(p + 1)
    lib().orc_basis_deriv_1d(int(p), float(c), float(h), float(x), _p(out))
    return out


def direct_grad(x, u, q, gE, gB, gamma_bar_, mode=MEAN, ke=KE, c0=C0):
    """Analytic gradient of L = sum_i gE_i.E_i + gB_i.B_i of the direct sum
    with respect to positions (n x 3) and charges (n)."""
    x = _f64(x, (-1, 3))
    u = _f64(u, (-1, 3))
    q = _f64(q, (-1,))
    gE = _f64(gE, (-1, 3))
    gB = _f64(gB, (-1, 3))
    n = x.shape[0]
    gx = np.zeros((n, 3))
    gq = np.zeros(n)
    lib().orc_direct_grad(n, _p(x), _p(u), _p(q), float(gamma_bar_), int(mode),
                          float(ke), float(c0), _p(gE), _p(gB), _p(gx), _p(gq))
    return gx, gq


def direct_grad_u(x, u, q, gE, gB, gamma_bar_, mode=MEAN, gbar_from_u=True,
                  ke=KE, c0=C0):
    """Analytic gradient of L = sum_i gE_i.E_i + gB_i.B_i of the direct sum
    with respect to the momenta (n x 3).  gbar_from_u: gamma_bar is the mean
    Lorentz factor of u (Sec. 3) and its derivative is included."""
    x = _f64(x, (-1, 3))
    u = _f64(u, (-1, 3))
    q = _f64(q, (-1,))
    gE = _f64(gE, (-1, 3))
    gB = _f64(gB, (-1, 3))
    gu = np.zeros((x.shape[0], 3))
    lib().orc_direct_grad_u(x.shape[0], _p(x), _p(u), _p(q), float(gamma_bar_),
                            int(mode), float(ke), float(c0), _p(gE), _p(gB),
                            int(bool(gbar_from_u)), _p(gu))
    return gu


class FMM:
    """Serial FP64 FMM (Alg. FMM) with access to every intermediate.

    ``run()`` performs subdivide, the list-filling dual traversal, the upward
    pass, M2L, P2P and the downward pass.  Fields come back in the caller's
    particle order with the physical prefactors applied.
    """

    def __init__(self, x, u, q, degree, leaf_size, eta, gamma_bar_=None,
                 mode=MEAN, ke=KE, c0=C0):
        self.x = _f64(x, (-1, 3))
        self.u = _f64(u, (-1, 3))
        self.q = _f64(q, (-1,))
        self.n = self.x.shape[0]
        self.degree = int(degree)
        self.leaf_size = int(leaf_size)
        self.eta = float(eta)
        # gamma_bar is a function of u unless it is given
        self.gbar_from_u = gamma_bar_ is None
        self.gamma_bar = float(gamma_bar(self.u) if gamma_bar_ is None
                               else gamma_bar_)
        self.mode = int(mode)
        self.h = lib().orc_fmm_create(self.n, self.degree, self.leaf_size,
                                      self.eta, self.gamma_bar, self.mode,
                                      float(ke), float(c0))
        if not self.h:
            raise ValueError("invalid oracle FMM parameters")
        self._done = set()  # steps run on the current structure

    def _need(self, what, *steps):
        missing = [st for st in steps if st not in self._done]
        if missing:
            raise RuntimeError("oracle FMM: %s needs %s first"
                               % (what, ", ".join(missing)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_fmm_destroy(h)
            self.h = None

    # individual steps -----------------------------------------------------
    def build_tree(self):
        lib().orc_fmm_build_tree(self.h, _p(self.x))
        self._done = {"build_tree"}
        return self

    def build_lists(self):
        self._need("build_lists", "build_tree")
        lib().orc_fmm_build_lists(self.h)
        self._done.add("build_lists")
        return self

    def upward(self):
        self._need("upward", "build_tree")
        lib().orc_fmm_upward(self.h, _p(self.u), _p(self.q))
        self._done.add("upward")
        return self

    def m2l(self):
        self._need("m2l", "build_lists", "upward")
        lib().orc_fmm_m2l(self.h)
        self._done.add("m2l")
        return self

    def p2p(self):
        self._need("p2p", "build_lists", "upward")
        lib().orc_fmm_p2p(self.h)
        self._done.add("p2p")
        return self

    def downward(self):
        self._need("downward", "m2l", "p2p")
        lib().orc_fmm_downward(self.h)
        self._done.add("downward")
        return self

    def run(self):
        return (self.build_tree().build_lists().upward().m2l().p2p()
                .downward())

    def rerun_frozen(self, x, u=None):
        """Evaluate at new positions (and momenta) with the structure built
        from the old ones (tree, boxes, proxies and lists kept).  New momenta
        also move gamma_bar when it is a function of u."""
        self._need("rerun_frozen", "build_lists")
        self.x = _f64(x, (-1, 3))
        lib().orc_fmm_set_positions(self.h, _p(self.x))
        if u is not None:
            self.u = _f64(u, (-1, 3))
            if self.gbar_from_u:
                self.gamma_bar = float(gamma_bar(self.u))
                lib().orc_fmm_set_gamma_bar(self.h, self.gamma_bar)
        return self.upward().m2l().p2p().downward()

    def adjoint(self, gE, gB):
        """Gradient of sum_i gE_i.E_i + gB_i.B_i with respect to positions
        and charges, with the structure frozen (needs run() first)."""
        self._need("adjoint", "downward")
        gE = _f64(gE, (-1, 3))
        gB = _f64(gB, (-1, 3))
        gx = np.zeros((self.n, 3))
        gq = np.zeros(self.n)
        lib().orc_fmm_adjoint(self.h, _p(gE), _p(gB), _p(gx), _p(gq), None, 0)
        return gx, gq

    def adjoint_u(self, gE, gB):
        """Gradients with respect to positions, charges and momenta (frozen
        structure; gamma_bar's derivative included when it is a function of
        u).  Needs run() first."""
        self._need("adjoint_u", "downward")
        gE = _f64(gE, (-1, 3))
        gB = _f64(gB, (-1, 3))
        gx = np.zeros((self.n, 3))
        gq = np.zeros(self.n)
        gu = np.zeros((self.n, 3))
        lib().orc_fmm_adjoint(self.h, _p(gE), _p(gB), _p(gx), _p(gq), _p(gu),
                              int(self.gbar_from_u))
        return gx, gq, gu

    # accessors -----------------------------------------------------------
    def sizes(self):
        out = np.zeros(7, dtype=np.int64)
        lib().orc_fmm_sizes(self.h, _p(out))
        keys = ("depth", "nslots", "n_p2p", "n_m2l", "p2p_interactions",
                "m2l_entries", "m")
        return dict(zip(keys, (int(v) for v in out)))

    def tree(self):
        self._need("tree", "build_tree")
        s = self.sizes()
        ns = s["nslots"]
        t = dict(perm=np.zeros(self.n, np.int64), lo=np.zeros(ns, np.int64),
                 hi=np.zeros(ns, np.int64), kind=np.zeros(ns, np.int8),
                 axis=np.zeros(ns, np.int8), bmin=np.zeros((ns, 3)),
                 bmax=np.zeros((ns, 3)), cen=np.zeros((ns, 3)),
                 hw=np.zeros((ns, 3)))
        lib().orc_fmm_get_tree(self.h, *(_p(t[k]) for k in (
            "perm", "lo", "hi", "kind", "axis", "bmin", "bmax", "cen", "hw")))
        t["depth"] = s["depth"]
        return t

    def lists(self):
        self._need("lists", "build_lists")
        s = self.sizes()
        p2p = np.zeros((s["n_p2p"], 2), np.int64)
        m2l = np.zeros((s["n_m2l"], 2), np.int64)
        lib().orc_fmm_get_lists(self.h, _p(p2p), _p(m2l))
        return p2p, m2l

    def multipoles(self):
        self._need("multipoles", "upward")
        s = self.sizes()
        M = np.zeros((s["nslots"], s["m"], 4))
        lib().orc_fmm_get_multipoles(self.h, _p(M))
        return M

    def locals(self):
        self._need("locals", "downward")
        s = self.sizes()
        L = np.zeros((s["nslots"], s["m"], 6))
        Lc = np.zeros((s["nslots"], s["m"], 6))
        lib().orc_fmm_get_locals(self.h, _p(L), _p(Lc))
        return L, Lc

    def fields(self):
        self._need("fields", "downward")
        E = np.zeros((self.n, 3))
        B = np.zeros((self.n, 3))
        lib().orc_fmm_get_fields(self.h, _p(E), _p(B), None, None)
        return E, B

    def near_fields(self):
        """P2P part only, before the prefactors."""
        self._need("near_fields", "p2p")
        E = np.zeros((self.n, 3))
        B = np.zeros((self.n, 3))
        lib().orc_fmm_get_fields(self.h, None, None, _p(E), _p(B))
        return E, B


def rel_error(f, ref):
    """eq. (fmm_error) for one field: global relative L2 error."""
    f = np.asarray(f, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.sum(ref * ref)
    return float(np.sqrt(np.sum((f - ref) ** 2) / den)) if den > 0 else 0.0


def fmm_error(E, B, Eref, Bref):
    """eq. (fmm_error): max over f in {E, B}; B is skipped when its
    reference is identically zero (u = 0)."""
    eb = rel_error(B, Bref) if np.any(np.asarray(Bref) != 0) else 0.0
    return max(rel_error(E, Eref), eb)
