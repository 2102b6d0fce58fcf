"""Mutation check of the oracle's pins: a copy of the oracle with one
planted mistake (admissibility, traversal tie rule, box rule, mean
momentum) is compiled on the CPU and must fail at least one golden fixture.
The fixtures themselves are hand-worked from the paper's algorithms
(tests/golden); this shows that they discriminate the readings they pin.
"""
import os
import shutil
import subprocess

import pytest

import oracle
from oracle import build as orcbuild

import test_oracle as T

# (name, text in relfmm_oracle.c, replacement)
MUTATIONS = [
    ("full diameter instead of the half-diagonal of Alg. diam",
     "double h = s[g] * f->hw[3 * i + g];",
     "double h = s[g] * (2.0 * f->hw[3 * i + g]);"),
    ("ties split the target",
     "} else if (diam2(f, i) > diam2(f, j)) {",
     "} else if (diam2(f, i) >= diam2(f, j)) {"),
    ("admissibility not strict",
     "return r < (f->eta * f->eta) * d2;",
     "return r <= (f->eta * f->eta) * d2;"),
    ("box floor not applied",
     "if (h < fl) {",
     "if (h < 0.0 * fl) {"),
    ("widened interval not clipped to the parent",
     "if (a < plo[g]) a = plo[g];",
     "if (0) a = plo[g];"),
    ("one-particle node not given its parent's box",
     "if (R == 0.0 && plo) {",
     "if (R == 0.0 && plo && 0) {"),
    ("mean Lorentz factor from u_z only",
     "return sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));",
     "return sqrt(1.0 + (p[2] * p[2]));"),
    ("unstretched distance",
     "double d = s[g] * (f->cen[3 * i + g] - f->cen[3 * j + g]);",
     "double d = (f->cen[3 * i + g] - f->cen[3 * j + g]);"),
]


def all_goldens_pass():
    return (all(T.golden_lists_match(f) for f in T.GOLDEN_TRAVERSALS)
            and T.golden_boxes_match() and T.golden_gamma_bar_matches())


def test_unmutated_oracle_passes_every_golden():
    assert all_goldens_pass()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_golden(tmp_path, name, old, new):
    src = open(orcbuild.SRC).read()
    assert src.count(old) == 1, "mutation site not unique: " + old
    d = tmp_path / "orc"
    d.mkdir()
    shutil.copy(os.path.join(os.path.dirname(orcbuild.SRC), "relfmm_oracle.h"),
                d / "relfmm_oracle.h")
    (d / "relfmm_oracle.c").write_text(src.replace(old, new))
    lib = str(d / "liborc_mut.so")
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-ffp-contract=off", "-fPIC",
                    "-shared", str(d / "relfmm_oracle.c"), "-o", lib, "-lm"],
                   check=True)
    saved = oracle.lib()
    try:
        oracle._lib = oracle.load(lib)
        assert not all_goldens_pass(), "planted mistake not caught: " + name
    finally:
        oracle._lib = saved
