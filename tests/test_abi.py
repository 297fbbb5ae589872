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


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a bh.h record, from a C program compiled against the header."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bh.h"', "int main(void) {",
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                            text=True).stdout.split()]
    return vals[0], dict(zip(fields, vals[1:]))


@pytest.mark.parametrize("name", ["View", "TableParams", "TileConfig", "ServeParams"])
def test_structs_match_header_layout(tmp_path, name):
    """The ctypes records of the binding have the C layout of include/bh.h, field by field."""
    import ctypes as C
    cls = getattr(bh, name)
    cname = {"View": "bh_view", "TableParams": "bh_table_params",
             "TileConfig": "bh_tile_config", "ServeParams": "bh_serve_params"}[name]
    fields = [f[0] for f in cls._fields_]
    size, offs = _c_layout(tmp_path, cname, fields)
    assert C.sizeof(cls) == size
    for f in fields:
        assert getattr(cls, f).offset == offs[f], f


def test_serve_start_rejects_launches_past_the_work_item_range(lib):
    """A serving launch holds at most 4194303 tiles (1024 pixels each at most, fewer than
    2^32 work-items); a larger max_tiles_per_launch is refused before any device work."""
    import ctypes as C
    p = bh.ServeParams(0, 0, 1 << 22)
    rc = lib.bh_serve_start(None, C.byref(p))
    assert rc == bh.BH_EINVAL
    assert b"max_tiles_per_launch" in lib.bh_last_error(None)
    p = bh.ServeParams(0, 0, (1 << 22) - 1)
    assert lib.bh_serve_start(None, C.byref(p)) == bh.BH_EINVAL
    assert b"NULL context" in lib.bh_last_error(None)


def test_generic_release_rejects_addresses_that_are_not_handles(lib):
    """bh_release looks an address up among the live handles before touching it: NULL, a
    host buffer and a misaligned address are refused with BH_EINVAL and a message."""
    import ctypes as C
    buf = (C.c_uint64 * 8)()
    for addr in (None, C.addressof(buf), C.addressof(buf) + 3):
        assert lib.bh_release(addr) == bh.BH_EINVAL
        assert b"not a live handle" in lib.bh_last_error(None)
