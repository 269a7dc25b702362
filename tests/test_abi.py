"""The C ABI library loads and exports every symbol include/velognn.h declares
(no compute call: this runs without a GPU)."""
import os
import re

import pytest

from paper_2407_12119_amd import synth, velo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "velognn.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"\b(velo_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = velo.lib()
    declared = _declared()
    assert set(declared) == set(velo.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_param_count_matches_the_generator_layout():
    for H, n in ((32, 5), (64, 4), (64, 6), (64, 0)):
        assert velo.param_count(H, n) == synth.param_count(H, n)
    assert velo.param_count(0, 4) == -1
    assert velo.param_count(64, 17) == -1


def test_status_strings():
    L = velo.lib()
    for st in range(8):
        assert L.velo_status_str(st)
