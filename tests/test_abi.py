"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every symbol that include/relfmm.h declares, its structs have the layout
the ctypes binding assumes, and arguments are validated before any device
work (these calls need no GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2302_07567_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "relfmm.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"RELFMM_API\s+[\w\s\*]*?\b(relfmm_\w+)\s*\(",
                                 text)))


def test_header_declares_the_binding_api():
    assert declared_symbols() == sorted(B.API)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (relfmm_\w+)", out))
    assert set(declared_symbols()) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "lay.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "relfmm.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n",'
                   'sizeof(relfmm_params), offsetof(relfmm_params, ke),'
                   'offsetof(relfmm_params, max_m2l_per_node),'
                   'sizeof(relfmm_stats), offsetof(relfmm_stats, gamma_bar));'
                   'return 0;}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o",
                    str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True,
                                       text=True).stdout.split()))
    assert got == [C.sizeof(B.CParams), B.CParams.ke.offset,
                   B.CParams.max_m2l_per_node.offset, C.sizeof(B.CStats),
                   B.CStats.gamma_bar.offset]


def _create(params, n_max=1000, ws=4096, nbytes=10 ** 9):
    lib = B.load()
    h = C.c_void_p()
    cp = params.to_c() if isinstance(params, B.Params) else params
    st = lib.relfmm_plan_create(C.byref(h), C.byref(cp), n_max,
                                C.c_void_p(ws), nbytes, None)
    return st, lib.relfmm_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(degree=0), "degree"), (dict(degree=11), "degree"),
    (dict(leaf_size=0), "leaf_size"), (dict(eta=0.0), "eta"),
    (dict(eta=float("nan")), "eta"), (dict(eta=float("inf")), "eta"),
    (dict(kernel="source", p2p_prec="bf16"), "p2p_prec"),
    (dict(eta=0.6, p2p_prec="fp32", m2l_prec="fp32"), "eta > 0.5"),
    (dict(eta=0.51, m2l_prec="bf16x3"), "eta > 0.5"),
    (dict(eta=0.7, m2l_prec="bf16"), "eta > 0.5"),
])
def test_invalid_parameters_rejected(kw, msg):
    base = dict(degree=4, leaf_size=64, eta=0.5)
    base.update(kw)
    st, err = _create(B.Params(**base))
    assert st == B.EINVAL and msg in err


def test_invalid_plan_arguments_rejected():
    p = B.Params(4, 64, 0.5)
    assert _create(p, n_max=0)[0] == B.EINVAL
    assert _create(p, ws=None)[0] == B.EINVAL
    st, err = _create(p, ws=4097)
    assert st == B.EINVAL and "aligned" in err
    st, err = _create(p, nbytes=100)
    assert st == B.ECAPACITY and "workspace" in err
    lib = B.load()
    assert lib.relfmm_compute_fields(None, 10, None, None, None, None, None,
                                     1) == B.EINVAL
    assert lib.relfmm_build_tree(None, 10, None, None) == B.EINVAL
    assert lib.relfmm_get_stats(None, None) == B.EINVAL
    assert lib.relfmm_export(None, 0, None, 0) == B.EINVAL


def test_reduced_precision_m2l_limited_to_eta_one_half():
    """The FP32 and BF16 M2L tiers are specified for eta <= 0.5; above it
    only the FP64 M2L is accepted (host-side check, no device work)."""
    for prec in ("fp32", "bf16", "bf16x3"):
        assert B.workspace_bytes(B.Params(4, 64, 0.5, m2l_prec=prec), 4096) > 0
        with pytest.raises(ValueError):
            B.workspace_bytes(B.Params(4, 64, 0.55, m2l_prec=prec), 4096)
    assert B.workspace_bytes(B.Params(4, 64, 0.9, m2l_prec="fp64"), 4096) > 0


def test_workspace_bytes_grow_with_n_and_degree():
    a = B.workspace_bytes(B.Params(4, 64, 0.5), 4096)
    b = B.workspace_bytes(B.Params(4, 64, 0.5), 65536)
    c = B.workspace_bytes(B.Params(8, 64, 0.5), 65536)
    assert 0 < a < b < c
    with pytest.raises(ValueError):
        B.workspace_bytes(B.Params(4, 64, -1.0), 4096)


def test_particle_count_limit():
    """n_max up to 2^28 (every per-particle index fits in 32 bits); beyond
    it the plan is refused before any device work."""
    p = B.Params(4, 512, 0.5)
    assert B.workspace_bytes(p, 1 << 28) > 0
    with pytest.raises(ValueError):
        B.workspace_bytes(p, (1 << 28) + 1)
    st, err = _create(p, n_max=(1 << 28) + 1)
    assert st == B.EINVAL and "2^28" in err


def test_static_entry_point_validates_before_device_work():
    """relfmm_compute_fields_static refuses bad arguments and, with
    RELFMM_ECAPACITY, any call whose structure does not fit its fixed
    scratch, before it touches the device (the pointers here are never
    dereferenced)."""
    lib = B.load()
    fake = C.c_void_p(4096)
    cp = B.Params(4, 64, 0.5).to_c()
    args = [fake] * 5 + [None]
    assert lib.relfmm_compute_fields_static(C.byref(cp), 0, *args) == B.EINVAL
    assert lib.relfmm_compute_fields_static(None, 10, *args) == B.EINVAL
    assert lib.relfmm_compute_fields_static(
        C.byref(cp), 10, None, fake, fake, fake, fake, None) == B.EINVAL
    bad = B.Params(0, 64, 0.5).to_c()
    assert lib.relfmm_compute_fields_static(C.byref(bad), 10, *args) == B.EINVAL
    # 2^20 particles in leaves of 64 need far more than the scratch
    assert B.workspace_bytes(B.Params(4, 64, 0.5), 1 << 20) > \
        B.STATIC_SCRATCH_BYTES
    st = lib.relfmm_compute_fields_static(C.byref(cp), 1 << 20, *args)
    err = lib.relfmm_last_error().decode()
    assert st == B.ECAPACITY and "scratch" in err


def test_static_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define RELFMM_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)",
                  text)
    assert m and int(m.group(1)) << int(m.group(2)) == B.STATIC_SCRATCH_BYTES
