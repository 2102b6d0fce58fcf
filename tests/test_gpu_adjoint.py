"""GPU adjoint (relfmm_adjoint) against the oracle's serial FMM adjoint on
the identical structure, against central finite differences of the GPU FMM
with frozen structure (rebuild=0), and against the analytic gradient of the
direct sum.

Tolerances: the FP64 adjoint computes the same sums as the oracle's in
another order, so 1e-11 (global relative L2).  The FP32 adjoint (P2P^T and
M2L^T in FP32 with FP64 pair offsets) keeps ~1e-6 relative per pair term;
1e-5 globally.  Against finite differences: 1e-4 (the FD step trades
truncation against rounding of the FP64 loss), the target of the adjoint
workload.  Every comparison with the oracle also bounds the worst particle
(tests/paritytools.py)."""
import numpy as np
import pytest

import oracle
from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

from paritytools import FIELDS, GRADS, check, check_fields

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
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta, gamma_bar=gb,
                     kernel=kernel, p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, n)
        gx, gq = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB))
        torch.cuda.synchronize()
        lab = "adjoint %s %s %s" % (name, kernel, prec)
        check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS[prec])
        check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS[prec])


@pytest.mark.parametrize("leaf,deg", [(1, 2), (1, 3), (2, 3), (2, 5)])
def test_adjoint_tiny_leaves_against_oracle(leaf, deg):
    """Leaves of one or two particles: boxes of zero or near-zero width on
    some axis, widened to 1/8 of the node's largest stretched half-width (and
    clipped to the parent's box) or, for one particle, the parent's box.
    Fields and gradients against the oracle, FP64 and FP32."""
    w = W.make("gauss4k", seed=70 + 10 * leaf + deg, n=3000)
    gb = oracle.gamma_bar(w.u)
    gE, gB = _cotangents(w.n, 11)
    f = oracle.FMM(w.x, w.u, w.q, deg, leaf, 0.5, gb).run()
    Eo, Bo = f.fields()
    gxo, gqo = f.adjoint(gE, gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=deg, leaf_size=leaf, eta=0.5, gamma_bar=gb,
                     p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, w.n)
        E, Bf = plan.compute(x, u, q)
        gx, gq = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB), rebuild=False)
        torch.cuda.synchronize()
        assert plan.stats()["overflow"] == 0
        lab = "tiny leaves %d degree %d %s" % (leaf, deg, prec)
        check_fields(lab, E.cpu().numpy(), Bf.cpu().numpy(), Eo, Bo,
                     *FIELDS[prec])
        check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS[prec])
        check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS[prec])


def test_adjoint_two_per_lane_split_rows_against_oracle():
    """The FP32 P2P^T kernels with two particles per lane, which the grid
    takes from 8,192 waves on (leaves of 129-256 in a tree of 2,048 node
    slots: 1,024 leaves of 130 here), with rows split into parts: grad_x,
    grad_q and grad_u against the oracle's adjoint on the same structure."""
    n = 1024 * 130
    w = W.make("gauss131k", seed=17, n=n)
    u_np = _spread(w, 12, (0.05, 0.05, 0.5))
    gb = oracle.gamma_bar(u_np)
    gE, gB = _cotangents(n, 12)
    print("oracle adjoint, n=%d" % n, flush=True)
    f = oracle.FMM(w.x, u_np, w.q, 2, 130, 0.5, None).run()
    gxo, gqo, guo = f.adjoint_u(gE, gB)
    x, u, q = _gpu(w.x), _gpu(u_np), _gpu(w.q)
    p = B.Params(degree=2, leaf_size=130, eta=0.5, gamma_bar=0.0,
                 p2p_prec="fp32", m2l_prec="fp32")
    plan = B.Plan(p, n)
    gx, gq, gu = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB), with_u=True)
    torch.cuda.synchronize()
    st = plan.stats()
    assert st["overflow"] == 0 and st["n_nodes"] == 2048
    assert abs(st["gamma_bar"] - gb) <= 1e-13 * gb
    lab = "two per lane n=%d fp32" % n
    check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS["fp32"])
    check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS["fp32"])
    check(lab + " grad_u", gu.cpu().numpy(), guo, *GRADS["fp32"])


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
    """Each compile-time degree of the adjoint kernels (L2P^T, M2L^T on MFMA
    in FP32, BF16 and split BF16, the basis-derivative leaf kernel) against
    the oracle's adjoint."""
    w = W.make("cube", seed=60 + deg, n=2000)
    gb = oracle.gamma_bar(w.u)
    leaf, eta = 40, 0.5
    gE, gB = _cotangents(w.n, 2)
    f = oracle.FMM(w.x, w.u, w.q, deg, leaf, eta, gb, oracle.MEAN).run()
    gxo, gqo = f.adjoint(gE, gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    for prec in ("fp64", "fp32", "bf16x3", "bf16"):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta, gamma_bar=gb,
                     p2p_prec="fp64" if prec == "fp64" else "fp32",
                     m2l_prec=prec)
        gx, gq = B.Plan(p, w.n).adjoint(x, u, q, _gpu(gE), _gpu(gB))
        torch.cuda.synchronize()
        lab = "adjoint degree %d %s" % (deg, prec)
        check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS[prec])
        check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS[prec])


# --- gradient with respect to the momenta ----------------------------------

def _spread(w, seed, s=(0.2, 0.2, 1.0)):
    """Momenta with a spread well beyond the bunch's, so that the weight,
    denominator and gamma_bar terms all carry weight."""
    rng = np.random.default_rng(seed)
    return w.u + rng.standard_normal((w.n, 3)) * np.array(s)


U_CASES = [("gauss4k", 4096, 4, 64, 0.5, "mean"),
           ("chirp1m", 20000, 8, 512, 0.4, "mean"),
           ("halo8m", 30000, 5, 100, 0.45, "source"),
           ("gauss4k", 1000, 3, 37, 0.5, "source")]


@pytest.mark.parametrize("name,n,deg,leaf,eta,kernel", U_CASES)
@pytest.mark.parametrize("given", [False, True])
def test_momentum_gradient_against_oracle(name, n, deg, leaf, eta, kernel,
                                          given):
    """grad_u against the oracle's FMM adjoint on the identical structure,
    gamma_bar computed from u (its derivative included) or given (a
    constant); grad_x and grad_q are unchanged by requesting grad_u."""
    w = W.make(name, seed=33, n=n)
    u_np = _spread(w, 7)
    gb = oracle.gamma_bar(u_np)
    gE, gB = _cotangents(n, 3)
    mode = oracle.MEAN if kernel == "mean" else oracle.EXACT
    f = oracle.FMM(w.x, u_np, w.q, deg, leaf, eta, gb if given else None,
                   mode).run()
    gxo, gqo, guo = f.adjoint_u(gE, gB)
    x, u, q = _gpu(w.x), _gpu(u_np), _gpu(w.q)
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=deg, leaf_size=leaf, eta=eta,
                     gamma_bar=gb if given else 0.0, kernel=kernel,
                     p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, n)
        gx, gq, gu = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB), with_u=True)
        torch.cuda.synchronize()
        # the device sums the momenta in another order
        assert abs(plan.stats()["gamma_bar"] - gb) <= 1e-13 * gb
        if prec == "fp64":
            st, s = plan.stats(), f.sizes()
            assert st["n_p2p_pairs"] == s["n_p2p"]
            assert st["n_m2l_pairs"] == s["n_m2l"]
        lab = "grad_u %s %s %s given=%s" % (name, kernel, prec, given)
        check(lab + " grad_u", gu.cpu().numpy(), guo, *GRADS[prec])
        check(lab + " grad_x", gx.cpu().numpy(), gxo, *GRADS[prec])
        check(lab + " grad_q", gq.cpu().numpy(), gqo, *GRADS[prec])
        gx2, gq2 = plan.adjoint(x, u, q, _gpu(gE), _gpu(gB), rebuild=False)
        torch.cuda.synchronize()
        assert oracle.rel_error(gx2.cpu().numpy(), gx.cpu().numpy()) <= 1e-13
        assert oracle.rel_error(gq2.cpu().numpy(), gq.cpu().numpy()) <= 1e-13


def test_momentum_gradient_finite_differences():
    """Central differences of the FP64 GPU FMM in the momenta with gamma_bar
    computed from u: each evaluation rebuilds from the perturbed momenta and
    must find the same tree and lists, so the differences see the weights,
    and gamma_bar in every near and far kernel."""
    w = W.make("gauss131k", seed=34, n=20000)
    u_np = _spread(w, 8)
    gE, gB = _cotangents(w.n, 4)
    gE, gB = _gpu(gE), _gpu(gB)
    x, u, q = _gpu(w.x), _gpu(u_np), _gpu(w.q)
    res = {}
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=5, leaf_size=128, eta=0.4, gamma_bar=0.0,
                     p2p_prec=prec, m2l_prec=prec)
        res[prec] = B.Plan(p, w.n).adjoint(x, u, q, gE, gB,
                                           with_u=True)[2].cpu().numpy()
    p = B.Params(degree=5, leaf_size=128, eta=0.4, gamma_bar=0.0,
                 p2p_prec="fp64", m2l_prec="fp64")
    plan = B.Plan(p, w.n)
    plan.compute(x, u, q)
    ref = [plan.export(k) for k in ("nodes", "p2p", "m2l")]

    def L(uu):
        E, Bf = plan.compute(x, uu, q, rebuild=True)
        for k, r in zip(("nodes", "p2p", "m2l"), ref):
            assert np.array_equal(plan.export(k), r)
        return float((E * gE).sum() + (Bf * gB).sum())

    def central(j, c, h):
        up = u.clone()
        up[j, c] += h
        Lp = L(up)
        up[j, c] -= 2 * h
        return (Lp - L(up)) / (2 * h)

    rng = np.random.default_rng(5)
    idx = rng.choice(w.n, 24, replace=False)
    axes = rng.integers(0, 3, 24)
    fd, g64, g32 = [], [], []
    for j, c in zip(idx, axes):
        h = 1e-3 * max(1.0, abs(u_np[j, c]))
        f1, f2 = central(j, c, h), central(j, c, h / 2)
        fd.append((4.0 * f2 - f1) / 3.0)
        g64.append(res["fp64"][j, c])
        g32.append(res["fp32"][j, c])
    fd, g64, g32 = map(np.array, (fd, g64, g32))
    e64 = np.sqrt(np.sum((g64 - fd) ** 2) / np.sum(fd ** 2))
    e32 = np.sqrt(np.sum((g32 - fd) ** 2) / np.sum(fd ** 2))
    print("grad_u FD: fp64 %.3e fp32 %.3e" % (e64, e32))
    assert e64 < 1e-4 and e32 < 1e-4


@pytest.mark.parametrize("kernel", ["mean", "source"])
def test_momentum_gradient_against_direct_16k(kernel):
    """grad_u of the FMM against the analytic direct-sum gradient (gamma_bar
    from u).  The source kernel's far field carries gamma_bar through the
    mean kernel, which the direct sum does not contain: a modelling
    difference of the size of the momentum spread's effect on the far field,
    so that case is held to the far-field approximation's level."""
    w = W.make("adjoint262k", seed=1, n=16384)
    u_np = _spread(w, 9, (0.05, 0.05, 0.2))
    gb = oracle.gamma_bar(u_np)
    ww, a, b = w.extra["w"], w.extra["a"], w.extra["b"]
    gE, gB = ww[:, None] * a, ww[:, None] * b
    mode = oracle.MEAN if kernel == "mean" else oracle.EXACT
    gud = oracle.direct_grad_u(w.x, u_np, w.q, gE, gB, gb, mode, True)
    x, u, q = _gpu(w.x), _gpu(u_np), _gpu(w.q)
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=0.35,
                     gamma_bar=0.0, kernel=kernel, p2p_prec=prec,
                     m2l_prec=prec)
        gu = B.Plan(p, w.n).adjoint(x, u, q, _gpu(gE), _gpu(gB),
                                    with_u=True)[2]
        eu = oracle.rel_error(gu.cpu().numpy(), gud)
        print("grad_u vs direct 16k %s %s: %.3e" % (kernel, prec, eu))
        assert eu < (1e-4 if kernel == "mean" else 1e-2)


def test_momentum_gradient_autograd():
    w = W.make("chirp1m", seed=35, n=12000)
    p = B.Params(degree=6, leaf_size=256, eta=0.4, gamma_bar=0.0,
                 kernel="source", p2p_prec="fp32", m2l_prec="fp32")
    x = _gpu(w.x).requires_grad_(True)
    q = _gpu(w.q)
    u = _gpu(_spread(w, 10)).requires_grad_(True)
    gE, gB = _cotangents(w.n, 6)
    gE, gB = _gpu(gE), _gpu(gB)
    E, Bf = B.fields(x, q, u, p)
    ((E * gE).sum() + (Bf * gB).sum()).backward()
    gx, gq, gu = B.Plan(p, w.n).adjoint(x.detach(), u.detach(), q, gE, gB,
                                        with_u=True)
    torch.cuda.synchronize()
    assert q.grad is None
    assert torch.equal(x.grad, gx) and torch.equal(u.grad, gu)


def test_adjoint_full_size_fp32_against_fp64():
    """The 262k workload in the launch configuration the benchmark times
    (FP32 P2P^T with two particles per lane, MFMA M2L^T and the gamma_bar
    derivative of the far field): every component of grad_x, grad_q and
    grad_u of the FP32 plan, and of the benchmark's plan (split-BF16 M2L and
    M2L^T), against the FP64 plan on the same structure (gamma_bar computed
    from u on the device by all)."""
    w = W.make("adjoint262k", seed=0)
    ww, a, b = w.extra["w"], w.extra["a"], w.extra["b"]
    gE, gB = _gpu(ww[:, None] * a), _gpu(ww[:, None] * b)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    out = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        p = B.Params(degree=w.degree, leaf_size=w.leaf_size, eta=0.35,
                     gamma_bar=0.0, p2p_prec="fp64" if prec == "fp64" else "fp32",
                     m2l_prec=prec)
        plan = B.Plan(p, w.n)
        g = plan.adjoint(x, u, q, gE, gB, with_u=True)
        torch.cuda.synchronize()
        out[prec] = [t.cpu().numpy() for t in g]
        del plan, g
        torch.cuda.empty_cache()
    for prec in ("fp32", "bf16x3"):
        errs = [oracle.rel_error(a, a64) for a, a64 in zip(out[prec], out["fp64"])]
        print("adjoint262k %s vs fp64: grad_x %.3e grad_q %.3e grad_u %.3e"
              % ((prec,) + tuple(errs)))
        assert max(errs) < 1e-5


def test_two_per_lane_two_wave_launches():
    """Leaves of 100 on 600k particles: the FP32 forward P2P and both P2P^T
    kernels run with two particles per lane in two-wave workgroups on an
    unsplit grid (8,192 leaves); fields and all gradients against the FP64
    plan (one particle per lane) on the same structure."""
    w = W.make("gauss131k", seed=7, n=600000)
    gE, gB = _cotangents(w.n, 8)
    gE, gB = _gpu(gE), _gpu(gB)
    x, u, q = _gpu(w.x), _gpu(w.u), _gpu(w.q)
    out = {}
    for prec in ("fp64", "fp32"):
        p = B.Params(degree=4, leaf_size=100, eta=0.5, gamma_bar=0.0,
                     p2p_prec=prec, m2l_prec=prec)
        plan = B.Plan(p, w.n)
        E, Bf = plan.compute(x, u, q)
        g = plan.adjoint(x, u, q, gE, gB, rebuild=False, with_u=True)
        torch.cuda.synchronize()
        assert plan.stats()["overflow"] == 0
        out[prec] = [t.cpu().numpy() for t in (E, Bf) + tuple(g)]
        del plan, E, Bf, g
        torch.cuda.empty_cache()
    errs = [oracle.rel_error(a32, a64) for a32, a64 in zip(out["fp32"], out["fp64"])]
    print("600k leaf 100 fp32 vs fp64: E %.2e B %.2e grad_x %.2e grad_q %.2e "
          "grad_u %.2e" % tuple(errs))
    assert max(errs[:2]) < 5e-7 and max(errs[2:]) < 1e-5
