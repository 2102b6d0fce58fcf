"""ctypes binding of the relfmm C-ABI (include/relfmm.h).

Argument marshalling only: every step of the FMM runs in the HIP library.
PyTorch supplies device memory (inputs, outputs and the plan's workspace)
and the stream.  If the library has not been built the binding raises; there
is no fallback path.
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librelfmm.so")

OK, EINVAL, ECAPACITY, EDEVICE, ESTATE = 0, 1, 2, 3, 4
_STATUS = {EINVAL: ValueError, ECAPACITY: MemoryError, EDEVICE: RuntimeError,
           ESTATE: RuntimeError}

KERNEL = {"mean": 0, "source": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}

EXPORT = {"nodes": 0, "boxes": 1, "perm": 2, "p2p": 3, "m2l": 4,
          "multipoles": 5, "locals": 6, "near": 7, "gamma_bar": 8,
          "local_cotangents": 9, "interp_boxes": 10}

API = ("relfmm_workspace_bytes", "relfmm_plan_create", "relfmm_plan_destroy",
       "relfmm_set_stream", "relfmm_build_tree", "relfmm_compute_fields",
       "relfmm_get_stats", "relfmm_export_bytes", "relfmm_export",
       "relfmm_set_timing", "relfmm_get_timings", "relfmm_get_timing_sums",
       "relfmm_direct_fields",
       "relfmm_adjoint", "relfmm_compute_fields_static", "relfmm_last_error")

STATIC_SCRATCH_BYTES = 64 << 20  # RELFMM_STATIC_SCRATCH_BYTES

PHASES = ("tree", "lists", "prep", "p2m", "m2m", "m2l", "p2p", "l2l", "l2p")


class CParams(C.Structure):
    _fields_ = [("degree", C.c_int32), ("leaf_size", C.c_int32),
                ("eta", C.c_double), ("gamma_bar", C.c_double),
                ("kernel", C.c_int32), ("p2p_prec", C.c_int32),
                ("m2l_prec", C.c_int32), ("max_p2p_per_leaf", C.c_int32),
                ("max_m2l_per_node", C.c_int32), ("reserved", C.c_int32),
                ("ke", C.c_double), ("c0", C.c_double)]


class CStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("depth", C.c_int32),
                ("overflow", C.c_int32), ("n_nodes", C.c_int64),
                ("n_p2p_pairs", C.c_int64), ("n_m2l_pairs", C.c_int64),
                ("p2p_interactions", C.c_int64), ("m2l_entries", C.c_int64),
                ("gamma_bar", C.c_double)]


_lib = None


def load():
    """Load the HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "relfmm HIP library not found at %s; build it with "
            "`python -m paper_2302_07567_amd.build`" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.relfmm_workspace_bytes.restype = C.c_size_t
    L.relfmm_workspace_bytes.argtypes = [C.POINTER(CParams), i64]
    L.relfmm_plan_create.restype = C.c_int
    L.relfmm_plan_create.argtypes = [C.POINTER(vp), C.POINTER(CParams), i64,
                                     vp, C.c_size_t, vp]
    L.relfmm_plan_destroy.restype = None
    L.relfmm_plan_destroy.argtypes = [vp]
    L.relfmm_set_stream.restype = C.c_int
    L.relfmm_set_stream.argtypes = [vp, vp]
    L.relfmm_build_tree.restype = C.c_int
    L.relfmm_build_tree.argtypes = [vp, i64, vp, vp]
    L.relfmm_compute_fields.restype = C.c_int
    L.relfmm_compute_fields.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32]
    L.relfmm_get_stats.restype = C.c_int
    L.relfmm_get_stats.argtypes = [vp, C.POINTER(CStats)]
    L.relfmm_export_bytes.restype = C.c_size_t
    L.relfmm_export_bytes.argtypes = [vp, i32]
    L.relfmm_export.restype = C.c_int
    L.relfmm_export.argtypes = [vp, i32, vp, C.c_size_t]
    L.relfmm_set_timing.restype = C.c_int
    L.relfmm_set_timing.argtypes = [vp, i32]
    L.relfmm_get_timings.restype = C.c_int
    L.relfmm_get_timings.argtypes = [vp, C.POINTER(C.c_double), i32]
    L.relfmm_get_timing_sums.restype = C.c_int
    L.relfmm_get_timing_sums.argtypes = [vp, C.POINTER(C.c_double), i32,
                                         C.POINTER(C.c_int64)]
    L.relfmm_direct_fields.restype = C.c_int
    L.relfmm_direct_fields.argtypes = [i64, vp, vp, vp, i64, vp, i32,
                                       C.c_double, C.c_double, C.c_double,
                                       vp, vp, vp]
    L.relfmm_adjoint.restype = C.c_int
    L.relfmm_adjoint.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, i32]
    L.relfmm_compute_fields_static.restype = C.c_int
    L.relfmm_compute_fields_static.argtypes = [C.POINTER(CParams), i64, vp,
                                               vp, vp, vp, vp, vp]
    L.relfmm_last_error.restype = C.c_char_p
    L.relfmm_last_error.argtypes = []
    _lib = L
    return L


def check(status):
    if status != OK:
        msg = load().relfmm_last_error().decode(errors="replace")
        raise _STATUS.get(status, RuntimeError)(
            "relfmm status %d: %s" % (status, msg))


@dataclass(frozen=True)
class Params:
    """Method parameters (Alg. FMM): degree n, leaf size N0, eta; the P2P
    kernel ('mean' or 'source') and the precisions of P2P and M2L."""
    degree: int
    leaf_size: int
    eta: float
    gamma_bar: float = 0.0
    kernel: str = "mean"
    p2p_prec: str = "fp32"
    m2l_prec: str = "fp32"
    max_p2p_per_leaf: int = 0
    max_m2l_per_node: int = 0
    ke: float = 0.0
    c0: float = 0.0

    def to_c(self):
        return CParams(int(self.degree), int(self.leaf_size), float(self.eta),
                       float(self.gamma_bar), KERNEL[self.kernel],
                       PREC[self.p2p_prec], PREC[self.m2l_prec],
                       int(self.max_p2p_per_leaf), int(self.max_m2l_per_node),
                       0, float(self.ke), float(self.c0))


def workspace_bytes(params, n_max):
    cp = params.to_c()
    nb = load().relfmm_workspace_bytes(C.byref(cp), int(n_max))
    if nb == 0:
        raise ValueError("invalid relfmm parameters: %r" % (params,))
    return nb


def _dev_ptr(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be contiguous with shape %s" % (name, shape))
    return C.c_void_p(t.data_ptr())


class Plan:
    """A relfmm plan for up to ``n_max`` particles on one device.  The
    workspace is a torch uint8 tensor owned by the plan."""

    def __init__(self, params, n_max, device=None):
        import torch
        self.lib = load()
        self.params = params
        self.n_max = int(n_max)
        self.device = torch.device(device if device is not None else "cuda")
        self.nbytes = workspace_bytes(params, self.n_max)
        with torch.cuda.device(self.device):
            self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8,
                                  device=self.device)
            base = self.ws.data_ptr()
            aligned = (base + 255) & ~255
            self._cp = params.to_c()
            self.h = C.c_void_p()
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(self.lib.relfmm_plan_create(
                C.byref(self.h), C.byref(self._cp), self.n_max,
                C.c_void_p(aligned), self.nbytes, C.c_void_p(stream)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.relfmm_plan_destroy(h)
            self.h = None

    def _sync_stream(self):
        import torch
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.relfmm_set_stream(self.h, C.c_void_p(s)))

    def build_tree(self, x, u):
        n = x.shape[0]
        self._sync_stream()
        check(self.lib.relfmm_build_tree(self.h, n, _dev_ptr(x, (n, 3), "x"),
                                         _dev_ptr(u, (n, 3), "u")))

    def compute(self, x, u, q, E=None, B=None, rebuild=True):
        import torch
        n = x.shape[0]
        if E is None:
            E = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        if B is None:
            B = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        self._sync_stream()
        check(self.lib.relfmm_compute_fields(
            self.h, n, _dev_ptr(x, (n, 3), "x"), _dev_ptr(u, (n, 3), "u"),
            _dev_ptr(q, (n,), "q"), _dev_ptr(E, (n, 3), "E"),
            _dev_ptr(B, (n, 3), "B"), 1 if rebuild else 0))
        return E, B

    def adjoint(self, x, u, q, gE, gB, grad_x=None, grad_q=None,
                rebuild=True, with_u=False, grad_u=None):
        """Gradients of sum_i gE_i.E_i + gB_i.B_i with respect to x and q
        (frozen structure), and with respect to u if with_u (then returns
        (grad_x, grad_q, grad_u))."""
        import torch
        n = x.shape[0]
        if grad_x is None:
            grad_x = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        if grad_q is None:
            grad_q = torch.empty((n,), dtype=torch.float64, device=x.device)
        if with_u and grad_u is None:
            grad_u = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        self._sync_stream()
        check(self.lib.relfmm_adjoint(
            self.h, n, _dev_ptr(x, (n, 3), "x"), _dev_ptr(u, (n, 3), "u"),
            _dev_ptr(q, (n,), "q"), _dev_ptr(gE, (n, 3), "gE"),
            _dev_ptr(gB, (n, 3), "gB"), _dev_ptr(grad_x, (n, 3), "grad_x"),
            _dev_ptr(grad_q, (n,), "grad_q"),
            _dev_ptr(grad_u, (n, 3), "grad_u") if with_u else None,
            1 if rebuild else 0))
        return (grad_x, grad_q, grad_u) if with_u else (grad_x, grad_q)

    def set_timing(self, enable=True):
        check(self.lib.relfmm_set_timing(self.h, 1 if enable else 0))

    def timings(self):
        """Milliseconds of each phase of the last call (waits for it)."""
        buf = (C.c_double * len(PHASES))()
        check(self.lib.relfmm_get_timings(self.h, buf, len(PHASES)))
        return dict(zip(PHASES, list(buf)))

    def timing_means(self):
        """Mean milliseconds of each phase over the compute calls timed since
        timing was enabled or since this was last called (waits for them),
        and the number of calls."""
        buf = (C.c_double * len(PHASES))()
        calls = C.c_int64(0)
        check(self.lib.relfmm_get_timing_sums(self.h, buf, len(PHASES),
                                              C.byref(calls)))
        k = max(calls.value, 1)
        return {p: v / k for p, v in zip(PHASES, list(buf))}, calls.value

    def stats(self):
        s = CStats()
        check(self.lib.relfmm_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in CStats._fields_}

    def export(self, what):
        wid = EXPORT[what]
        nb = self.lib.relfmm_export_bytes(self.h, wid)
        m = (self.params.degree + 1) ** 3
        dtype = np.int32 if what in ("nodes", "perm", "p2p", "m2l") \
            else np.float64
        buf = np.zeros(max(nb, 8) // np.dtype(dtype).itemsize, dtype=dtype)
        check(self.lib.relfmm_export(self.h, wid,
                                     buf.ctypes.data_as(C.c_void_p), nb))
        buf = buf[: nb // np.dtype(dtype).itemsize]
        if what == "nodes":
            return buf.reshape(-1, 4)
        if what in ("boxes", "interp_boxes"):
            return buf.reshape(-1, 6)
        if what in ("p2p", "m2l"):
            return buf.reshape(-1, 2)
        if what == "multipoles":
            return buf.reshape(-1, m, 4)
        if what in ("locals", "local_cotangents"):
            return buf.reshape(-1, m, 6)
        if what == "near":
            return buf.reshape(-1, 6)
        if what == "gamma_bar":
            return float(buf[0])
        return buf


def direct_fields(x, u, q, targets=None, kernel="mean", gamma_bar=0.0,
                  ke=0.0, c0=0.0):
    """FP64 direct sum (all j != i) at the given targets on the GPU."""
    import torch
    n = x.shape[0]
    if targets is None:
        nt, tp = n, C.c_void_p(0)
    else:
        if targets.dtype != torch.int64 or not targets.is_cuda:
            raise TypeError("targets must be a CUDA int64 tensor")
        targets = targets.contiguous()
        nt, tp = targets.shape[0], C.c_void_p(targets.data_ptr())
    E = torch.empty((nt, 3), dtype=torch.float64, device=x.device)
    B = torch.empty((nt, 3), dtype=torch.float64, device=x.device)
    s = torch.cuda.current_stream(x.device).cuda_stream
    check(load().relfmm_direct_fields(
        n, _dev_ptr(x, (n, 3), "x"), _dev_ptr(u, (n, 3), "u"),
        _dev_ptr(q, (n,), "q"), nt, tp, KERNEL[kernel], float(gamma_bar),
        float(ke), float(c0), _dev_ptr(E, (nt, 3), "E"),
        _dev_ptr(B, (nt, 3), "B"), C.c_void_p(s)))
    return E, B


def compute_fields_static(x, u, q, params, E=None, B=None):
    """E, B at every particle through relfmm_compute_fields_static: the
    structure is built and the fields evaluated in the library's fixed
    device scratch, with no workspace (nothing is allocated but E and B when
    they are not given).  On torch's current stream of x's device."""
    import torch
    n = x.shape[0]
    if E is None:
        E = torch.empty((n, 3), dtype=torch.float64, device=x.device)
    if B is None:
        B = torch.empty((n, 3), dtype=torch.float64, device=x.device)
    cp = params.to_c()
    with torch.cuda.device(x.device):
        s = torch.cuda.current_stream(x.device).cuda_stream
        check(load().relfmm_compute_fields_static(
            C.byref(cp), n, _dev_ptr(x, (n, 3), "x"),
            _dev_ptr(u, (n, 3), "u"), _dev_ptr(q, (n,), "q"),
            _dev_ptr(E, (n, 3), "E"), _dev_ptr(B, (n, 3), "B"),
            C.c_void_p(s)))
    return E, B


_plans = {}


def _plan_for(params, n, device):
    key = (params, str(device))
    plan = _plans.get(key)
    if plan is None or plan.n_max < n:
        plan = Plan(params, n, device)
        _plans[key] = plan
    return plan


def compute_fields(x, u, q, params, rebuild=True):
    """E, B (float64 CUDA tensors, n x 3) at every particle."""
    return _plan_for(params, x.shape[0], x.device).compute(x, u, q,
                                                           rebuild=rebuild)


def _fields_function():
    import torch

    class FieldsFunction(torch.autograd.Function):
        """(E, B) = FMM(x, q, u; params) with a hand-written backward: the
        adjoint of the FMM with frozen structure, recomputing the tree,
        lists and far field from the saved inputs instead of storing them.
        Gradients flow to x, q and (when it requires grad) u; params get
        none."""

        @staticmethod
        def forward(ctx, x, q, u, params):
            x_, q_, u_ = (t.detach().contiguous() for t in (x, q, u))
            E, B = _plan_for(params, x_.shape[0], x_.device).compute(x_, u_, q_)
            ctx.save_for_backward(x_, q_, u_)
            ctx.params = params
            return E, B

        @staticmethod
        def backward(ctx, gE, gB):
            x, q, u = ctx.saved_tensors
            n = x.shape[0]
            if gE is None:
                gE = torch.zeros((n, 3), dtype=torch.float64, device=x.device)
            if gB is None:
                gB = torch.zeros((n, 3), dtype=torch.float64, device=x.device)
            plan = _plan_for(ctx.params, n, x.device)
            if ctx.needs_input_grad[2]:
                gx, gq, gu = plan.adjoint(x, u, q, gE.contiguous(),
                                          gB.contiguous(), with_u=True)
                return gx, gq, gu, None
            gx, gq = plan.adjoint(x, u, q, gE.contiguous(), gB.contiguous())
            return gx, gq, None, None

    return FieldsFunction


_FF = None


def fields(x, q, u, params):
    """Differentiable (E, B) with respect to x, q and u."""
    global _FF
    if _FF is None:
        _FF = _fields_function()
    return _FF.apply(x, q, u, params)
