"""The C ABI library loads and exports every entry point of include/hyb.h
(CPU only: no compute calls)."""
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hyb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hyb_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def P():
    import paper_2107_01723_amd as P
    P.lib()
    return P


def test_library_exports_every_declared_symbol(P):
    decl = _header_functions()
    assert len(decl) >= 20
    L = P.lib()
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(P.hyb.ABI_FUNCTIONS) == decl


def test_struct_layouts_match(P):
    P.check_abi()


def test_footprint_and_validation(P):
    cfg, _, _ = W.config_small()
    b = P.footprint(cfg)
    assert 1e6 < b < 1e8
    big, _, _ = W.config_huge()
    assert 2e10 < P.footprint(big) < 4e10          # 512^3 cells, 2e8 particles
    bad = dict(cfg, x_lo=2.5e-6)                  # slab face off the cell faces
    with pytest.raises(P.HybError) as e:
        P.footprint(bad)
    assert e.value.status == 1
    with pytest.raises(P.HybError):
        P.footprint(dict(cfg, nx=4096))
    with pytest.raises(P.HybError):
        P.footprint(dict(cfg, brem_boost=0.5))


def test_status_strings(P):
    L = P.lib()
    assert L.hyb_status_string(0) == b"ok"
    assert L.hyb_status_string(7) == b"busy"
