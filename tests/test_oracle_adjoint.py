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


@pytest.mark.parametrize("leaf,degree", [(1, 3), (2, 3), (2, 5)])
def test_fmm_adjoint_finite_differences_tiny_leaves(leaf, degree):
    """Leaves of one or two particles: boxes of zero or near-zero width on
    some axis, where the interpolation-box rule keeps the basis derivative
    finite and well conditioned (a half-width of 2^-40 times the root's made
    the derivative of the interpolant, and central differences of it,
    differ by orders of magnitude).  Central differences of the FMM with
    frozen structure, including particles whose leaf box was widened or
    inherited from the parent."""
    rng = np.random.default_rng(40 + leaf + degree)
    w = W.make("gauss4k", seed=40 + leaf, n=300)
    gb = oracle.gamma_bar(w.u)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    f = oracle.FMM(w.x, w.u, w.q, degree, leaf, 0.5, gb).run()
    assert f.sizes()["n_m2l"] > 0
    t = f.tree()
    # particles in leaves whose box is not their own bounding box
    span = t["bmax"] - t["bmin"]
    widened = np.where((t["kind"] == 1)
                       & np.any(np.abs(2 * t["hw"] - span) > 0, axis=1))[0]
    assert len(widened) > 0
    picks = [int(t["perm"][t["lo"][v]]) for v in widened[:6]]
    gx, gq = f.adjoint(gE, gB)
    scale = np.abs(gx).max()
    for k, i in enumerate(picks + [0, 150, 299]):
        c = k % 3
        h = 1e-7 * (w.x[:, c].max() - w.x[:, c].min())
        fd = _frozen_fd(f, w.x, gE, gB, i, c, h)
        assert abs(fd - gx[i, c]) < 1e-6 * scale, (i, c, fd, gx[i, c])
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


# --- gradient with respect to the momenta ----------------------------------

@pytest.mark.parametrize("mode,from_u", [(oracle.MEAN, True),
                                         (oracle.MEAN, False),
                                         (oracle.EXACT, True)])
def test_direct_momentum_gradient_finite_differences(mode, from_u):
    """u enters q gamma and q u, the EXACT denominator and (MEAN, gamma_bar
    a function of u) the stretch of the kernel; central differences of the
    direct sum with gamma_bar recomputed from the perturbed momenta."""
    rng = np.random.default_rng(21)
    w = W.make("chirp1m", seed=21, n=24)
    # momentum spread well beyond the bunch's so that every term matters
    u = w.u + rng.standard_normal((w.n, 3)) * np.array([0.3, 0.3, 2.0])
    q = w.q * rng.uniform(0.5, 1.5, w.n)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    gb0 = oracle.gamma_bar(u)
    gu = oracle.direct_grad_u(w.x, u, q, gE, gB, gb0, mode, from_u)

    def L(uu):
        gb = oracle.gamma_bar(uu) if from_u else gb0
        return loss(*oracle.direct(w.x, uu, q, gb, mode), gE, gB)

    scale = np.abs(gu).max()
    for (j, c) in [(0, 0), (3, 1), (11, 2), (23, 2), (17, 0)]:
        h = 1e-6 * max(1.0, abs(u[j, c]))
        up, um = u.copy(), u.copy()
        up[j, c] += h
        um[j, c] -= h
        fd = (L(up) - L(um)) / (2 * h)
        assert abs(fd - gu[j, c]) < 1e-7 * scale, (j, c, fd, gu[j, c])


def test_direct_momentum_gradient_gamma_bar_term():
    """With gamma_bar a function of u, the MEAN gradient differs from the
    fixed-gamma_bar one by the same vector G pbar/(n gamma_bar) for every
    particle (G = dL/dgamma_bar); the EXACT sum does not contain gamma_bar."""
    rng = np.random.default_rng(22)
    w = W.make("gauss4k", seed=22, n=40)
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    gb = oracle.gamma_bar(w.u)
    d = (oracle.direct_grad_u(w.x, w.u, w.q, gE, gB, gb, oracle.MEAN, True)
         - oracle.direct_grad_u(w.x, w.u, w.q, gE, gB, gb, oracle.MEAN, False))
    assert np.abs(d - d[0]).max() <= 1e-12 * np.abs(d[0]).max()
    pbar = w.u.mean(axis=0)
    assert np.abs(np.cross(d[0], pbar)).max() <= 1e-10 * np.linalg.norm(d[0]) * np.linalg.norm(pbar)
    # G from a central difference in gamma_bar
    L = lambda g: loss(*oracle.direct(w.x, w.u, w.q, g, oracle.MEAN), gE, gB)
    h = 1e-6 * gb
    G = (L(gb + h) - L(gb - h)) / (2 * h)
    want = G * pbar / (w.n * gb)
    assert np.abs(d[0] - want).max() < 1e-6 * np.abs(want).max()
    e = (oracle.direct_grad_u(w.x, w.u, w.q, gE, gB, gb, oracle.EXACT, True)
         - oracle.direct_grad_u(w.x, w.u, w.q, gE, gB, gb, oracle.EXACT, False))
    assert np.all(e == 0.0)


@pytest.mark.parametrize("mode", [oracle.MEAN, oracle.EXACT])
def test_fmm_momentum_gradient_finite_differences_frozen(mode):
    """Frozen structure: perturbed momenta change the weights, the EXACT
    near-field denominators and gamma_bar in every MEAN kernel (near and
    far), while the tree, boxes and lists stay."""
    rng = np.random.default_rng(23)
    w = W.make("gauss131k", seed=23, n=1200)
    u = w.u + rng.standard_normal((w.n, 3)) * np.array([0.2, 0.2, 1.0])
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    f = oracle.FMM(w.x, u, w.q, 4, 40, 0.5, None, mode).run()
    assert f.sizes()["n_m2l"] > 0
    gx, gq, gu = f.adjoint_u(gE, gB)
    gx0, gq0 = f.adjoint(gE, gB)
    assert np.array_equal(gx, gx0) and np.array_equal(gq, gq0)
    scale = np.abs(gu).max()
    for (j, c) in [(0, 0), (100, 1), (777, 2), (1199, 2), (640, 0)]:
        h = 1e-6 * max(1.0, abs(u[j, c]))
        up, um = u.copy(), u.copy()
        up[j, c] += h
        um[j, c] -= h
        Lp = loss(*f.rerun_frozen(w.x, up).fields(), gE, gB)
        Lm = loss(*f.rerun_frozen(w.x, um).fields(), gE, gB)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gu[j, c]) < 1e-6 * scale, (j, c, fd, gu[j, c])
    f.rerun_frozen(w.x, u)


def test_fmm_momentum_gradient_matches_direct():
    rng = np.random.default_rng(24)
    w = W.make("gauss4k", seed=24, n=3000)
    u = w.u + rng.standard_normal((w.n, 3)) * np.array([0.1, 0.1, 0.5])
    gE = rng.standard_normal((w.n, 3))
    gB = rng.standard_normal((w.n, 3)) * oracle.C0
    gb = oracle.gamma_bar(u)
    gud = oracle.direct_grad_u(w.x, u, w.q, gE, gB, gb, oracle.MEAN, True)
    errs = []
    for p in (4, 6):
        f = oracle.FMM(w.x, u, w.q, p, 50, 0.3).run()
        errs.append(oracle.rel_error(f.adjoint_u(gE, gB)[2], gud))
    assert errs[1] < errs[0] and errs[1] < 1e-5, errs
