"""The C-ABI library loads and exports every symbol include/bh.h declares (no GPU needed)."""
import os
import re

import pytest

from paper_2010_08735_amd import bh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bh_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bh.LIB_PATH):
        from paper_2010_08735_amd import build
        build.build()
    return bh.lib()


def test_header_declares_the_binding_names():
    assert declared_symbols() == sorted(bh.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_tile_configs_are_wave_multiples(lib):
    n = bh.bh_tile_config_count()
    assert n >= 4
    for i in range(n):
        t = bh.bh_tile_config_get(i)
        assert t.tile_w % 8 == 0 and t.tile_h % 8 == 0
        assert t.waves * t.ppt * 64 == t.tile_w * t.tile_h
    with pytest.raises(bh.BhError):
        bh.bh_tile_config_get(n)


def test_structs_match_header_layout(lib):
    import ctypes as C
    # bh_view: 3 doubles of position ... stars pointer last; 8-byte aligned record
    assert C.sizeof(bh.View) % 8 == 0
    assert bh.View.stars.offset == C.sizeof(bh.View) - 8
    assert C.sizeof(bh.TableParams) == 32
    assert C.sizeof(bh.StarField) == 48
