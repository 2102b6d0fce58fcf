"""GPU adjoint (relfmm_adjoint) against the oracle's serial FMM adjoint on
the identical structure, against central finite differences of the GPU FMM
with frozen structure (rebuild=0), and against the analytic gradient of the
direct sum.

Tolerances: the FP64 adjoint computes the same sums as the oracle's in
another order, so 1e-11 (global relative L2).  The FP32 adjoint (P2P^T and
M2L^T in FP32 with FP64 pair offsets) keeps ~1e-6 relative per pair term;
1e-5 globally.  Against finite differences: 1e-4 (the FD step trades
truncation against rounding of the FP64 loss), the target of the adjoint
workload."""
import numpy as np
import pytest

import oracle
from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64,
                        device="cuda")


def _cotangents(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3)), rng.standard_normal((n, 3)) * oracle.C0


CASES = [("gauss4k", 4096, 4, 64, 0.5), ("gauss4k", 1000, 3, 37, 0.5),
         ("chirp1m", 20000, 8, 512, 0.4), ("halo8m", 30000, 5, 100, 0.45)]


@pytest.mark.parametrize("name,n,deg,leaf,eta", CASES)
@pytest.mark.parametrize("kernel", ["mean", "source"])
def test_adjoint_against_oracle(name, n, deg, leaf, eta, kernel):
    w = W.make(name, seed=31, n=n)
    gb = oracle.gamma_bar(w.u)
    gE, gB = _cotangents(n, 1)
    mode = oracle.MEAN if kernel == "mean" else oracle.EXACT
    f = oracle.FMM(w.x, w.u, w.q, deg, leaf, eta, gb, mode).run()
    gxo, gqo = f.adjoint(gE, gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-5)):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta, gamma_bar=gb,
                     kernel=kernel, p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, n)
        gx, gq = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB))
        torch.cuda.synchronize()
        ex = oracle.rel_error(gx.cpu().numpy(), gxo)
        eq = oracle.rel_error(gq.cpu().numpy(), gqo)
        print("adjoint %s %s %s: grad_x %.3e grad_q %.3e" % (name, kernel,
                                                             prec, ex, eq))
        assert ex < tol and eq < tol


def test_adjoint_linear_in_q_and_autograd():
    w = W.make("gauss131k", seed=5, n=20000)
    gb = oracle.gamma_bar(w.u)
    p = B.Params(degree=5, leaf_size=128, eta=0.4, gamma_bar=gb,
                 p2p_prec="fp64", m2l_prec="fp64")
    x = _gpu(w.x).requires_grad_(True)
    q = _gpu(w.q).requires_grad_(True)
    u = _gpu(w.u)
    gE, gB = _cotangents(w.n, 2)
    gE, gB = _gpu(gE), _gpu(gB)
    E, Bf = B.fields(x, q, u, p)
    L = (E * gE).sum() + (Bf * gB).sum()
    L.backward()
    gx, gq = B.Plan(p, w.n).adjoint(x.detach(), u, q.detach(), gE, gB)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gx) and torch.equal(q.grad, gq)
    # the fields are linear in q: L = sum_j q_j dL/dq_j
    assert abs(L.item() - float((q.detach() * gq).sum())) < 1e-12 * abs(L.item())


def _loss(plan, x, u, q, gE, gB):
    E, Bf = plan.compute(x, u, q, rebuild=False)
    return float((E * gE).sum() + (Bf * gB).sum())


def test_adjoint_finite_differences_adjoint262k():
    """The adjoint workload: 262,144 particles, loss sum_i w_i (E_i.a_i +
    B_i.b_i); central differences of the FP64 FMM with frozen structure on
    64 seeded coordinates."""
    w = W.make("adjoint262k", seed=0)
    gb = oracle.gamma_bar(w.u)
    ww, a, b = w.extra["w"], w.extra["a"], w.extra["b"]
    gE, gB = _gpu(ww[:, None] * a), _gpu(ww[:, None] * b)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    results = {}
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=0.35,
                     gamma_bar=gb, p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, w.n)
        gx, gq = plan.adjoint(x, u, q, gE, gB)
        results[prec] = (gx.cpu().numpy(), gq.cpu().numpy())
    p64 = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=0.35,
                   gamma_bar=gb, p2p_prec="fp64", m2l_prec="fp64")
    plan = B.Plan(p64, w.n)
    plan.build_tree(x, u)
    rng = np.random.default_rng(123)
    idx = rng.choice(w.n, 64, replace=False)
    axes = rng.integers(0, 3, 64)
    # step: 1e-3 of the particle's nearest-neighbour distance (the scale on
    # which its pair terms vary), with one Richardson step on h and h/2
    from scipy.spatial import cKDTree
    dnn = cKDTree(w.x).query(w.x[idx], k=2)[0][:, 1]

    def central(i, c, h):
        xp = x.clone()
        xp[i, c] += h
        Lp = _loss(plan, xp, u, q, gE, gB)
        xp[i, c] -= 2 * h
        Lm = _loss(plan, xp, u, q, gE, gB)
        return (Lp - Lm) / (2 * h)

    fd, g64, g32 = [], [], []
    for i, c, dn in zip(idx, axes, dnn):
        h = 1e-3 * dn
        f1, f2 = central(i, c, h), central(i, c, h / 2)
        fd.append((4.0 * f2 - f1) / 3.0)
        g64.append(results["fp64"][0][i, c])
        g32.append(results["fp32"][0][i, c])
    fd, g64, g32 = map(np.array, (fd, g64, g32))
    e64 = np.sqrt(np.sum((g64 - fd) ** 2) / np.sum(fd ** 2))
    e32 = np.sqrt(np.sum((g32 - fd) ** 2) / np.sum(fd ** 2))
    print("adjoint262k FD: fp64 %.3e fp32 %.3e" % (e64, e32))
    assert e64 < 1e-4 and e32 < 1e-4
    # charges: exact linearity, L = q . dL/dq
    L = _loss(plan, x, u, q, gE, gB)
    for prec in ("fp64", "fp32"):
        lin = float(w.q @ results[prec][1])
        assert abs(L - lin) < (1e-10 if prec == "fp64" else 1e-5) * abs(L)


def test_adjoint_against_direct_gradient_16k():
    w = W.make("adjoint262k", seed=1, n=16384)
    gb = oracle.gamma_bar(w.u)
    ww, a, b = w.extra["w"], w.extra["a"], w.extra["b"]
    gE, gB = ww[:, None] * a, ww[:, None] * b
    gxd, gqd = oracle.direct_grad(w.x, w.u, w.q, gE, gB, gb)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=0.35,
                     gamma_bar=gb, p2p_prec=prec, m2l_prec=prec)
        gx, gq = B.Plan(p, w.n).adjoint(x, u, q, _gpu(gE), _gpu(gB))
        ex = oracle.rel_error(gx.cpu().numpy(), gxd)
        eq = oracle.rel_error(gq.cpu().numpy(), gqd)
        print("direct-gradient 16k %s: grad_x %.3e grad_q %.3e" % (prec, ex, eq))
        assert ex < 1e-4 and eq < 1e-4


@pytest.mark.parametrize("deg", list(range(1, 11)))
def test_adjoint_every_degree(deg):
    """Each compile-time degree of the adjoint kernels (L2P^T, M2L^T on MFMA,
    the basis-derivative leaf kernel) against the oracle's adjoint."""
    w = W.make("cube", seed=60 + deg, n=2000)
    gb = oracle.gamma_bar(w.u)
    leaf, eta = 40, 0.5
    gE, gB = _cotangents(w.n, 2)
    f = oracle.FMM(w.x, w.u, w.q, deg, leaf, eta, gb, oracle.MEAN).run()
    gxo, gqo = f.adjoint(gE, gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-5)):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta, gamma_bar=gb,
                     p2p_prec=prec, m2l_prec=prec)
        gx, gq = B.Plan(p, w.n).adjoint(x, u, q, _gpu(gE), _gpu(gB))
        torch.cuda.synchronize()
        ex = oracle.rel_error(gx.cpu().numpy(), gxo)
        eq = oracle.rel_error(gq.cpu().numpy(), gqo)
        print("adjoint degree %d %s: grad_x %.3e grad_q %.3e" % (deg, prec,
                                                                 ex, eq))
        assert ex < tol and eq < tol
