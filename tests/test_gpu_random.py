"""Seeded random configurations against the oracle: workload shape, particle
count (1 to 5,000), leaf size, degree, eta (0.3-0.5, the range of the
reduced-precision tiers) and kernel drawn at random, covering the small-grid
launch shapes (split rows, grouped lists, merge presort, one-workgroup
traversal head).  FP64: structure bit-identical, fields <= 1e-12, gradient
<= 1e-11; FP32: fields <= 2e-6, gradient <= 1e-5 (the bars of the fixed-case
tests), plus the worst particle of every field and gradient
(tests/paritytools.py)."""
import numpy as np
import pytest

import oracle
from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

from paritytools import FIELDS, GRADS, check, check_fields
from test_gpu_parity import check_structure

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ["gauss4k", "chirp1m", "halo8m", "cube", "gauss131k"]


def _gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                        device="cuda")


def _config(seed):
    rng = np.random.default_rng(seed)
    name = NAMES[rng.integers(len(NAMES))]
    n = int(rng.choice([1, 2, 17, 100, 513, 1000, 2000, 3000, 5000]))
    leaf = int(rng.choice([8, 16, 37, 64, 100, 129, 200, 300]))
    deg = int(rng.integers(1, 6))
    eta = float(rng.choice([0.3, 0.4, 0.5]))
    kernel = str(rng.choice(["mean", "source"]))
    return name, n, leaf, deg, eta, kernel, int(rng.integers(1000))


@pytest.mark.parametrize("seed", range(24))
def test_random_configuration(seed):
    name, n, leaf, deg, eta, kernel, wseed = _config(1000 + seed)
    print("config", name, n, leaf, deg, eta, kernel, flush=True)
    w = W.make(name, seed=wseed, n=n)
    gb = oracle.gamma_bar(w.u)
    mode = oracle.MEAN if kernel == "mean" else oracle.EXACT
    rng = np.random.default_rng(seed)
    gE = rng.standard_normal((n, 3))
    gB = rng.standard_normal((n, 3)) * oracle.C0
    f = oracle.FMM(w.x, w.u, w.q, deg, leaf, eta, gb, mode).run()
    Eo, Bo = f.fields()
    gxo, gqo = f.adjoint(gE, gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta, gamma_bar=gb,
                     kernel=kernel, p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, n)
        E, Bf = plan.compute(x, u, q)
        gx, gq = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB), rebuild=False)
        torch.cuda.synchronize()
        if prec == "fp64":
            check_structure(plan, f)
        E, Bf = E.cpu().numpy(), Bf.cpu().numpy()
        if n == 1:
            assert np.all(E == 0) and np.all(Bf == 0)
            continue
        lab = "random %d %s" % (seed, prec)
        check_fields(lab, E, Bf, Eo, Bo, *FIELDS[prec])
        check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS[prec])
        check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS[prec])
