"""CPU-side checks of the HIP library: it loads, exports every entry point of
include/lst.h, and its host-built module map equals the oracle's."""
import re
import os

import numpy as np
import pytest

import oracle
from synth import geometry as G
from synth import params as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "lst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lst_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    import paper_2209_13711_amd as lst
    lib = lst.load_library()
    declared = _header_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(lst.lst.EXPORTS)


@pytest.mark.parametrize("geo_name,w", [("barrel_toy", 1.0), ("full", 1.0), ("barrel_toy", 1.5)])
def test_library_module_map_equals_oracle(geo_name, w):
    import paper_2209_13711_amd as lst
    geo = G.get(geo_name)
    params = PR.make(w=w)
    ptr, col = lst.lst_build_map(params, geo.f32, geo.i32)
    optr, ocol = oracle.Oracle(params, geo.f32, geo.i32).module_map()
    np.testing.assert_array_equal(ptr, optr)
    np.testing.assert_array_equal(col, ocol)
