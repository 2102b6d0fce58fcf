"""Pins of the oracle's gradients: the derivative of the interpolation basis
(Theorem 1 applied to P'), central finite differences of the direct sum and
of the frozen-structure FMM, exact linearity in the charges, and agreement
of the FMM gradient with the direct-sum gradient within the FMM's accuracy."""
import numpy as np
import pytest

import oracle
from paper_2302_07567_amd import workloads as W


def loss(E, B, gE, gB):
    return float(np.sum(E * gE) + np.sum(B * gB))


@pytest.mark.parametrize("p", [1, 3, 4, 6, 8])
def test_basis_derivative_reproduces_polynomial_derivatives(p):
    t = oracle.cheb_nodes(p)
    c, h = -0.2, 0.7
    nodes = c + h * t
    rng = np.random.default_rng(p)
    pts = np.concatenate([rng.uniform(c - h, c + h, 10), nodes,
                          [c + h * (1 - 1e-15), c - h * (1 - 1e-15)]])
    for xv in pts:
        dl = oracle.basis_deriv_1d(p, c, h, xv)
        for deg in range(p + 1):
            got = dl @ (((nodes - c) / h) ** deg)
            want = deg * ((xv - c) / h) ** max(deg - 1, 0) / h if deg else 0.0
            assert abs(got - want) < 1e-11 * max(1.0, abs(want)), (xv, deg)
        eps = 1e-6 * h
        fd = (oracle.basis_1d(p, c, h, xv + eps) -
              oracle.basis_1d(p, c, h, xv - eps)) / (2 * eps)
        if abs((xv - c) / h) < 1 - 1e-5:
            np.testing.assert_allclose(dl, fd, rtol=1e-6, atol=1e-6 / h)


@pytest.mark.parametrize("mode", [oracle.MEAN, oracle.EXACT])
def test_direct_gradient_finite_differences(mode):
    rng = np.random.default_rng(3)
    w = W.make("chirp1m", seed=3, n=30)
    gb = oracle.gamma_bar(w.u)
    q = w.q * rng.uniform(0.5, 1.5, w.n)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    gx, gq = oracle.direct_grad(w.x, w.u, q, gE, gB, gb, mode)
    L0 = lambda x, qq: loss(*oracle.direct(x, w.u, qq, gb, mode), gE, gB)
    for (i, c) in [(0, 0), (5, 1), (17, 2), (29, 2)]:
        h = 1e-7 * np.abs(w.x[:, c]).max()
        xp, xm = w.x.copy(), w.x.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (L0(xp, q) - L0(xm, q)) / (2 * h)
        assert abs(fd - gx[i, c]) < 1e-6 * np.abs(gx).max()
    # linear in q: L = sum_j q_j dL/dq_j
    assert abs(L0(w.x, q) - float(q @ gq)) < 1e-12 * abs(L0(w.x, q))


def _frozen_fd(f, x, gE, gB, i, c, h):
    xp, xm = x.copy(), x.copy()
    xp[i, c] += h
    xm[i, c] -= h
    Lp = loss(*f.rerun_frozen(xp).fields(), gE, gB)
    Lm = loss(*f.rerun_frozen(xm).fields(), gE, gB)
    f.rerun_frozen(x)
    return (Lp - Lm) / (2 * h)


@pytest.mark.parametrize("mode", [oracle.MEAN, oracle.EXACT])
def test_fmm_adjoint_finite_differences_frozen(mode):
    rng = np.random.default_rng(8)
    w = W.make("gauss131k", seed=8, n=1500)
    gb = oracle.gamma_bar(w.u)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    f = oracle.FMM(w.x, w.u, w.q, 4, 40, 0.5, gb, mode).run()
    assert f.sizes()["n_m2l"] > 0
    gx, gq = f.adjoint(gE, gB)
    scale = np.abs(gx).max()
    for (i, c) in [(0, 0), (100, 1), (777, 2), (1499, 0), (640, 2)]:
        h = 1e-6 * (w.x[:, c].max() - w.x[:, c].min())
        fd = _frozen_fd(f, w.x, gE, gB, i, c, h)
        assert abs(fd - gx[i, c]) < 2e-6 * scale, (i, c, fd, gx[i, c])
    L = loss(*f.fields(), gE, gB)
    assert abs(L - float(w.q @ gq)) < 1e-12 * abs(L)


def test_fmm_adjoint_matches_direct_gradient():
    rng = np.random.default_rng(9)
    w = W.make("gauss4k", seed=9, n=3000)
    gb = oracle.gamma_bar(w.u)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    gxd, gqd = oracle.direct_grad(w.x, w.u, w.q, gE, gB, gb)
    errs = []
    for p in (4, 6):
        f = oracle.FMM(w.x, w.u, w.q, p, 50, 0.3, gb).run()
        gx, gq = f.adjoint(gE, gB)
        errs.append((oracle.rel_error(gx, gxd), oracle.rel_error(gq, gqd)))
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]
    assert errs[1][0] < 1e-5 and errs[1][1] < 1e-6
