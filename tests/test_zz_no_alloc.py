"""relfmm_compute_fields_static (the entry point that allocates nothing and
works in the library's fixed device scratch) against relfmm_compute_fields
on a plan with its own workspace, through the C-ABI: two calls in a row, the
second on a smaller bunch, for FP64 and FP32.  Both run the same kernels on
the same structure; the only difference is how many row parts the P2P
near field is split into (at most two in the scratch), which changes the
order of FP64 additions of identical per-tile partial sums, so every
particle agrees to FP64 rounding."""
import numpy as np
import pytest

from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

from paritytools import check

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = (1e-13, 1e-12)  # global L2, worst particle


def _gpu(arr):
    return torch.tensor(np.ascontiguousarray(arr), dtype=torch.float64,
                        device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_matches_plan_two_calls(prec):
    p = B.Params(degree=5, leaf_size=128, eta=0.4, gamma_bar=0.0,
                 p2p_prec=prec, m2l_prec=prec)
    for call, (name, n, seed) in enumerate((("gauss131k", 20000, 41),
                                            ("chirp1m", 5000, 42))):
        assert B.workspace_bytes(p, n) <= B.STATIC_SCRATCH_BYTES
        w = W.make(name, seed=seed, n=n)
        x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
        print("static entry point: call %d, %s n=%d %s" % (call, name, n, prec),
              flush=True)
        Es, Bs = B.compute_fields_static(x, u, q, p)
        torch.cuda.synchronize()
        plan = B.Plan(p, n)
        Ep, Bp = plan.compute(x, u, q)
        torch.cuda.synchronize()
        assert plan.stats()["overflow"] == 0
        Es, Bs, Ep, Bp = (t.cpu().numpy() for t in (Es, Bs, Ep, Bp))
        assert np.all(np.isfinite(Es)) and np.all(np.isfinite(Bs))
        lab = "static vs plan call %d n=%d %s" % (call, n, prec)
        check(lab + " E", Es, Ep, *TOL)
        check(lab + " B", Bs, Bp, *TOL)
