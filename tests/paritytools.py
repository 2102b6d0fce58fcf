"""Element-wise parity measures shared by the GPU tests.

Besides the global relative L2 error of eq. (fmm_error), every value test
bounds the worst single particle (or node):

    pointwise(a, ref) = max_i |a_i - ref_i| / max(|ref_i|, rms_i |ref_i|)

with |.| the Euclidean norm of the row (a particle's 3-vector field or
gradient, a node's expansion).  Rows whose reference is far below the RMS
are measured against the RMS, so that a field that nearly cancels does not
turn rounding into a large relative error; everywhere else the bound is
the particle's own relative error.  A mis-staged tile, a wrong row part or
a dropped pair moves a few rows by far more than the global L2 sees.

Bars (derivations next to each tier):
  FP64  fields 1e-11, gradients 1e-9: same sums in another order and with
        FMA contraction; a row's error is a few hundred ulps of the sum of
        the magnitudes of its terms, which stays within 1e-12 of the row
        for these inputs; gradients add the derivative of the interpolation
        basis (up to ~n^2 / h relative to the box scale).
  FP32  fields 2e-5, gradients 1e-4: per pair ~3e-7 relative (one rounding
        of the offsets, rsqrt, products), summed with FP64 accumulation per
        tile; a row whose field is a near-cancelling sum of many terms
        sees that error relative to the sum of its terms' magnitudes, which
        the cancellation ratio (below ~30 for these bunches) turns into the
        bar.
  BF16  fields 5e-2: 8 significant bits per operand (2^-9 relative).
"""
import numpy as np

import oracle


def pointwise(a, ref):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    a = a.reshape(ref.shape[0], -1)
    ref = ref.reshape(ref.shape[0], -1)
    d = np.sqrt(np.sum((a - ref) ** 2, axis=1))
    r = np.sqrt(np.sum(ref * ref, axis=1))
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    if rms == 0.0:
        return float(d.max()) if d.size else 0.0
    return float((d / np.maximum(r, rms)).max())


def check(label, a, ref, tol_l2, tol_pw):
    """Global relative L2 (eq. fmm_error for one field) and the worst row."""
    e2 = oracle.rel_error(a, ref)
    ep = pointwise(a, ref)
    print("%s: L2 %.3e worst row %.3e" % (label, e2, ep), flush=True)
    assert e2 < tol_l2, (label, "L2", e2)
    assert ep < tol_pw, (label, "row", ep)
    return e2, ep


def check_fields(label, E, B, Eo, Bo, tol_l2, tol_pw):
    """eq. (fmm_error) (max over E and B, B skipped when its reference is
    zero) and the worst particle of each field."""
    assert oracle.fmm_error(E, B, Eo, Bo) < tol_l2
    check(label + " E", E, Eo, tol_l2, tol_pw)
    if np.any(np.asarray(Bo) != 0):
        check(label + " B", B, Bo, tol_l2, tol_pw)


FIELDS = {"fp64": (1e-12, 1e-11), "fp32": (2e-6, 2e-5),
          "bf16x3": (2e-6, 2e-5), "bf16": (5e-3, 5e-2)}
GRADS = {"fp64": (1e-11, 1e-9), "fp32": (1e-5, 1e-4),
         "bf16x3": (1e-5, 1e-4), "bf16": (5e-3, 5e-2)}
