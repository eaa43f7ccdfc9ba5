"""The C ABI library loads and exports every function include/sambaten.h declares
(CPU only: nothing here calls into the GPU)."""

import ctypes
import os
import re

from paper_1709_00668_amd import sambaten

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sambaten.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sbt_init_dense", "sbt_init_coo", "sbt_update_batch_dense",
                     "sbt_update_batch_coo", "sbt_get_factors", "sbt_fit", "sbt_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sambaten.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == set(sambaten.exported_symbols())


def test_config_struct_layout():
    # int32 x 10, uint64, uint32 x 2, int64 x 3 with natural alignment
    assert ctypes.sizeof(sambaten.sbt_config) == 80
    assert sambaten.sbt_config.seed.offset == 40
    assert sambaten.sbt_config.k_capacity.offset == 56


def test_status_strings_without_gpu():
    lib = sambaten.load()
    for s in range(7):
        assert lib.sbt_status_str(s)
