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
    # 512^3 cells, 2e8 particles: E, B (run precision) and J plus its
    # accumulator (int64) per node; Te, Ti, two eta, heat and its
    # accumulator (FP64) and F_sigma per cell; two particle buffers of
    # records (cell, id, 8 values); per tile of 4^3 cells the current
    # partials (3 x 150 words), 64 heat partials, a claim and a mark of
    # atomics into its accumulators; per particle
    # a scatter offset, per chunk of 256 its 125 destination counts
    ts = 8 if big["precision"] == W.FP64 else 4
    nodes = (big["nx"] + 1) * (big["ny"] + 1) * (big["nz"] + 1)
    cells = big["nx"] * big["ny"] * big["nz"]
    tiles = -(-big["nx"] // 4) * -(-big["ny"] // 4) * -(-big["nz"] // 4)
    cap = big["max_particles"]
    need = (nodes * (6 * ts + 6 * 8) + cells * (6 * 8 + ts) + 2 * cap * (8 + 8 * ts)
            + tiles * (3 * 150 * ts + 64 * 8 + 8) + cap * 4 + -(-cap // 256) * 125 * 4)
    assert need <= P.footprint(big) <= 1.02 * need + 1e8
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


def test_binding_fails_loudly_without_the_library():
    """No CPU fallback: without libhyb.so the binding raises."""
    import subprocess
    import sys
    code = ("import paper_2107_01723_amd.hyb as H\n"
            "H.LIB_PATH = '/nonexistent/libhyb.so'\n"
            "try:\n    H.lib()\nexcept RuntimeError as e:\n    print('raised', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert "raised" in out.stdout and "missing" in out.stdout, (out.stdout, out.stderr[-2000:])
