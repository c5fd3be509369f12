"""The C-ABI library loads and exports every symbol include/trg.h declares (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trg.h")
LIB = os.path.join(ROOT, "paper_2507_21909_amd", "libtrg.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|size_t|char)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2507_21909_amd.build import build
        build()
    return LIB


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tensor_init", "atrg_step", "triad_atrg_step", "log_z_per_site", "trg_create", "trg_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path]).decode()
    exported = set(re.findall(r"\sT\s+(\w+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_rejects_bad_arguments(lib_path):
    import ctypes
    from paper_2507_21909_amd import binding
    lib = binding.load_library(lib_path)
    assert lib.trg_strerror(-1).decode() == "invalid argument"
    # argument checks run before any device call
    assert lib.trg_create(None, None) == -1
    o = binding.Options()
    lib.trg_default_options(ctypes.byref(o))
    assert (o.dim, o.r, o.sketch_mult, o.power_iters) == (4, 7, 2, 1)
    o.dim = 5
    s = ctypes.c_void_p()
    assert lib.trg_create(ctypes.byref(o), ctypes.byref(s)) == -1
    assert lib.trg_destroy(None) == 0
    assert lib.tensor_init(None, 0, 0.1, 0.0, 4) == -1
    assert lib.atrg_step(None, 0) == -1
    out = ctypes.c_double()
    assert lib.log_z_per_site(None, ctypes.byref(out)) == -1


def test_graph_and_batch_entry_points_reject_bad_arguments(lib_path):
    import ctypes
    from paper_2507_21909_amd import binding
    lib = binding.load_library(lib_path)
    g = ctypes.c_void_p()
    assert lib.trg_graph_capture(None, 1, 0, ctypes.byref(g)) == -1
    assert lib.trg_graph_launch(None, 0) == -1
    assert lib.trg_graph_launch(None, 1) == -1
    assert lib.trg_graph_destroy(None) == 0
    assert lib.trg_batch_run_graphs(None, 4, None) == -1
    assert lib.trg_batch_run(None, 4, None) == -1
    assert lib.trg_strerror(-7).decode().startswith("truncation cut inside a multiplet")


def test_selftest_entry_points_reject_bad_arguments(lib_path):
    import ctypes
    from paper_2507_21909_amd import binding
    lib = binding.load_library(lib_path)
    ip = lambda *v: (ctypes.c_int * len(v))(*v)
    buf = (ctypes.c_double * 8)()
    dp = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    # the permute check runs before any device call: rank, sizes, a true permutation
    assert lib.trg_selftest_permute(0, ip(2), ip(0), dp, dp) == -1
    assert lib.trg_selftest_permute(9, ip(*[1] * 9), ip(*range(9)), dp, dp) == -1
    assert lib.trg_selftest_permute(2, ip(2, 0), ip(1, 0), dp, dp) == -1
    assert lib.trg_selftest_permute(2, ip(2, 3), ip(0, 0), dp, dp) == -1
    assert lib.trg_selftest_permute(2, ip(2, 3), ip(0, 2), dp, dp) == -1
    assert lib.trg_selftest_permute(2, None, ip(1, 0), dp, dp) == -1
    assert lib.trg_selftest_tsqr(5, 6, dp, dp, dp) == -1      # m < n
    assert lib.trg_selftest_tsqr(6, 0, dp, dp, dp) == -1
