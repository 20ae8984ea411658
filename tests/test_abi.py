"""CPU checks of the C ABI: the built library loads and exports every
function include/hfx.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hfx.h")
LIB = os.path.join(ROOT, "paper_1708_00033_amd", "libhfx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hfx_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfx.so not built")
def test_binding_covers_header():
    from paper_1708_00033_amd import hfx
    assert set(declared_functions()) == set(hfx.EXPORTED)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhfx.so not built")
def test_defaults_and_null_handling_without_gpu():
    from paper_1708_00033_amd import hfx
    o = hfx.default_options()
    assert o.schwarz_tau == 1e-10 and o.task_quartets % 256 == 0
    s = hfx.default_scf_options()
    assert s.max_iter == 100 and s.diis_max == 8
    assert hfx.hfx_default_options(None) == hfx.HFX_ERR_INVALID_ARG
    assert hfx.hfx_create(None, None) == hfx.HFX_ERR_INVALID_ARG


def test_generator_class_table():
    import sys
    sys.path.insert(0, os.path.join(ROOT, "paper_1708_00033_amd", "csrc"))
    import gen_eri
    assert len(gen_eri.CLASSES) == 21
    # every class is in canonical orientation
    for B, K in gen_eri.CLASSES:
        la, lb = gen_eri.PAIR_CLASSES[B]
        lc, ld = gen_eri.PAIR_CLASSES[K]
        assert la >= lb and lc >= ld and B >= K
    g = gen_eri.ClassGen(0, 0, 0, 0)
    g.emit("x")
    assert g.flops == 0 and g.hrr_flops == 0
