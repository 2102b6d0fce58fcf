"""Full-size checks in the launch configuration the benchmark times.

At 131k to 8.4M particles the oracle's serial FMM is out of reach, so the
HIP FMM is checked at seeded sampled targets against the oracle's FP64
direct sum (eq. fmm_error over the sample, 1,024 seeded targets), which the
oracle evaluates target by target.  The bound is the accuracy the method is run at: relative error
<= 1e-6 against the FP64 direct sum for the FP32 path and for the FP64 path,
with the interpolation degree, leaf size and admissibility parameter of the
benchmark configuration.  FP32 against FP64 (same structure, all targets) is
bounded by the per-pair FP32 rounding (few ulps, averaged in the L2 sum).
"""
import numpy as np
import pytest

import bench
import oracle
from paper_2302_07567_amd import binding as B
from paper_2302_07567_amd import workloads as W

from paritytools import check

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_SAMPLE = 1024


def _gpu(arr):
    return torch.tensor(np.ascontiguousarray(arr), dtype=torch.float64,
                        device="cuda")


def _fields(w, spec, prec, m2l_prec=None):
    p = B.Params(degree=spec["degree"], leaf_size=spec["leaf_size"],
                 eta=spec["eta"], gamma_bar=0.0, kernel="mean",
                 p2p_prec=prec, m2l_prec=m2l_prec or prec)
    plan = B.Plan(p, w.n)
    E, Bf = plan.compute(_gpu(w.x), _gpu(w.u), _gpu(w.q))
    torch.cuda.synchronize()
    st = plan.stats()
    assert st["overflow"] == 0
    out = E.cpu().numpy(), Bf.cpu().numpy(), st["gamma_bar"]
    del plan, E, Bf
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("name", ["gauss131k", "adjoint262k", "chirp1m",
                                  "halo8m"])
def test_full_size_against_direct_sum(name):
    """FP64, FP32 and the benchmark's default tiers (FP32 P2P with split-BF16
    M2L) at full size: each against the oracle's direct sum at the sampled
    targets, and the reduced tiers against the FP64 plan at every particle
    (global and worst row)."""
    spec = bench.BENCH[name]
    w = W.make(name, seed=0)
    print("full size", name, w.n, spec, flush=True)
    E64, B64, gb = _fields(w, spec, "fp64")
    s = w.sample[:N_SAMPLE]
    Ed, Bd = oracle.direct(w.x, w.u, w.q, gb, oracle.MEAN, targets=s)
    e64 = oracle.fmm_error(E64[s], B64[s], Ed, Bd)
    print("%s fp64 vs direct %.3e" % (name, e64), flush=True)
    assert e64 <= 1e-6
    for m2l in ("fp32", "bf16x3"):
        E, Bf, gbr = _fields(w, spec, "fp32", m2l)
        assert gbr == gb
        e = oracle.fmm_error(E[s], Bf[s], Ed, Bd)
        e_64 = oracle.fmm_error(E, Bf, E64, B64)
        print("%s fp32 P2P + %s M2L: vs direct %.3e, vs fp64 %.3e"
              % (name, m2l, e, e_64), flush=True)
        assert e <= 1e-6
        assert e_64 <= 5e-7
        # every particle, against FP64 on the same structure
        check("%s %s vs fp64 E" % (name, m2l), E, E64, 5e-7, 2e-5)
        check("%s %s vs fp64 B" % (name, m2l), Bf, B64, 5e-7, 2e-5)
        del E, Bf


def test_full_size_bf16_m2l():
    """BF16 M2L operands on the 1M bunch: reported accuracy tier, bounded by
    bf16's 8 significant bits, and clearly coarser than FP32."""
    name = "chirp1m"
    spec = bench.BENCH[name]
    w = W.make(name, seed=0)
    Eb, Bb, gb = _fields(w, spec, "fp32", "bf16")
    s = w.sample[:N_SAMPLE]
    Ed, Bd = oracle.direct(w.x, w.u, w.q, gb, oracle.MEAN, targets=s)
    err = oracle.fmm_error(Eb[s], Bb[s], Ed, Bd)
    print("chirp1m bf16 M2L vs direct %.3e" % err, flush=True)
    assert err < 5e-3
