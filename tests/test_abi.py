"""The C ABI: libxy.so loads and exports every function include/xy.h declares,
and the binding's struct layouts match the header (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xy.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xy_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = _declared()
    for n in ("xy_alloc", "xy_sweep", "xy_measure", "xy_pcc_step", "xy_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1210_6116_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def test_struct_sizes_match_header():
    from paper_1210_6116_amd import _lib
    assert ctypes.sizeof(_lib.xy_params) == 40
    assert ctypes.sizeof(_lib.xy_obs) == 104
    assert ctypes.sizeof(_lib.xy_pcc) == 48


def test_bytes_required_and_argument_errors():
    from paper_1210_6116_amd import _lib
    p = _lib.xy_params(L=64, beta=1.12, seed=1, replica=0, label_bits=0, start=0, tile_rows=0)
    n64 = _lib.xy_bytes_required([p])
    assert n64 > 64 * 64 * 8
    big = _lib.xy_params(L=65536, beta=1.0, seed=1, replica=0, label_bits=0, start=0, tile_rows=0)
    nbig = _lib.xy_bytes_required([big])
    # spins (8 B) + two planes of 16-bit tile-local labels (4 B) per site, and
    # well inside 288 GB
    assert 12 * 65536 ** 2 < nbig < 100e9
    for bad in (dict(L=48), dict(L=1), dict(L=131072), dict(beta=-1.0), dict(label_bits=16),
                dict(L=65536, label_bits=32), dict(tile_rows=8), dict(start=7)):
        kw = dict(L=64, beta=1.0, seed=1, replica=0, label_bits=0, start=0, tile_rows=0)
        kw.update(bad)
        with pytest.raises(_lib.XYError) as ei:
            _lib.xy_bytes_required([_lib.xy_params(**kw)])
        assert ei.value.code == _lib.XY_EINVAL
