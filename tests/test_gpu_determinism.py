"""Run-to-run reproducibility of every precision tier.  The library sums in
fixed orders and uses no floating-point atomics, so evaluating the same
inputs again, on the same plan or on a fresh one, gives the same bits: the
fields of every tier and the gradient of every reduced tier.  The bunches
are large enough for the launch shapes of the benchmark (unsplit
two-targets-per-lane P2P, grouped M2L row blocks on the flat bunch, many M2L
pairs per node on the halo bunch, split rows and the degree-6 kernels on the
Gaussian one), where a race between waves would show up as a changed bit."""
import numpy as np
import pytest

import oracle
from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIERS = [("fp64", "fp64"), ("fp32", "fp32"), ("fp32", "bf16x3"),
         ("fp32", "bf16")]


def _gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                        device="cuda")


@pytest.mark.parametrize("name,n", [("chirp1m", 262144), ("halo8m", 524288),
                                    ("gauss131k", 262144)])
def test_bitwise_reproducible(name, n):
    w = W.make(name, seed=5, n=n)
    gb = oracle.gamma_bar(w.u)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    rng = np.random.default_rng(5)
    gE = _gpu(rng.standard_normal((n, 3)))
    gB = _gpu(rng.standard_normal((n, 3)) * oracle.C0)
    print("reproducibility", name, n, flush=True)
    for p2p, m2l in TIERS:
        p = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=w.eta,
                     gamma_bar=gb, p2p_prec=p2p, m2l_prec=m2l)
        runs = []
        for fresh in (True, False, True):
            if fresh:
                plan = B.Plan(p, n)
            E, Bf = plan.compute(x, u, q)
            runs.append((E.cpu().numpy(), Bf.cpu().numpy()))
        for E, Bf in runs[1:]:
            assert np.array_equal(E, runs[0][0]), (name, p2p, m2l, "E")
            assert np.array_equal(Bf, runs[0][1]), (name, p2p, m2l, "B")
        if p2p == "fp32":
            g = [plan.adjoint(x, u, q, gE, gB, rebuild=False)
                 for _ in range(2)]
            for a, b in zip(g[0], g[1]):
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), \
                    (name, "adjoint")
        del plan
        torch.cuda.empty_cache()
