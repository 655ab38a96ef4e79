"""The C-ABI library loads and exports every symbol include/ck.h declares;
host-only calls (no GPU work) behave as documented."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1605_05236_amd", "libck.so")


def declared():
    src = open(os.path.join(ROOT, "include", "ck.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ck_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1605_05236_amd import build
        build.build()
    from paper_1605_05236_amd import table
    return table.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\b(ck_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_binding_covers_the_header(lib):
    from paper_1605_05236_amd import table
    assert sorted(table.EXPORTED) == declared()


def test_storage_bytes_and_geometry_checks(lib):
    from paper_1605_05236_amd import table
    size = ctypes.c_size_t()
    assert lib.ck_storage_bytes(1 << 16, 4, 2, ctypes.byref(size)) == 0
    # 16-byte slots, 4-byte metadata word and 8-byte claim word per bin
    assert size.value == (1 << 16) * (4 * 16 + 4 + 8)
    for bins, B, d in [(0, 4, 2), (1 << 10, 3, 2), (1 << 10, 4, 3), (1 << 10, 1, 5),
                       (1 << 32, 1, 2), (1, 1, 2)]:
        assert lib.ck_storage_bytes(bins, B, d, ctypes.byref(size)) == -1
    opt = table.CkOptions()
    lib.ck_default_options(ctypes.byref(opt))
    assert (opt.max_chain, opt.max_search, opt.batch_ops) == (500, 500, 1 << 20)
    h = ctypes.c_void_p()
    # invalid requests are refused before any device work
    assert lib.ck_create(1 << 10, 4, 3, 0, ctypes.byref(opt), ctypes.c_void_p(256), 1 << 20,
                         None, ctypes.byref(h)) == -1
    assert lib.ck_create(1 << 10, 4, 2, 4, ctypes.byref(opt), ctypes.c_void_p(256), 1 << 20,
                         None, ctypes.byref(h)) == -1  # rattle needs single-slot bins
    assert lib.ck_create(1 << 10, 4, 2, 0, ctypes.byref(opt), None, 1 << 20, None,
                         ctypes.byref(h)) == -1
    assert lib.ck_strerror(-1) == b"invalid argument"
    assert lib.ck_insert(None, None, None, 0, None, None) == -1


def test_stash_and_bias_options_are_checked_before_device_work(lib):
    from paper_1605_05236_amd import table
    opt = table.CkOptions()
    lib.ck_default_options(ctypes.byref(opt))
    assert (opt.stash, opt.hash_bias) == (0, 0)  # no stash, uniform hashes
    h = ctypes.c_void_p()
    for field, bad in [("stash", 65), ("hash_bias", 5)]:
        o = table.CkOptions()
        lib.ck_default_options(ctypes.byref(o))
        setattr(o, field, bad)
        assert lib.ck_create(1 << 10, 4, 2, 0, ctypes.byref(o), ctypes.c_void_p(256), 1 << 20,
                             None, ctypes.byref(h)) == -1, field
    # the calls on a null handle are refused, whatever the size
    assert lib.ck_upsert(None, None, None, 5, None, None, None, None, None) == -1
    assert lib.ck_overwrite(None, None, None, 5, None, None) == -1
    assert lib.ck_export_stash(None, None, None, None) == -1
    assert lib.ck_import_stash(None, None, None, None) == -1
    assert lib.ck_group_upsert(None, None, None, None, 5, None, None, None, None, None) == -1
    assert lib.ck_group_export_stash(None, 0, None, None, None) == -1


def test_spawn_k_option_is_checked_before_device_work(lib):
    # k-at-a-time spawning: BFS (1) and sorted search (2) only, two hash
    # functions, 4- or 8-slot bins, k <= 32 / slots_per_bin
    from paper_1605_05236_amd import table
    h = ctypes.c_void_p()
    for bins, B, d, scheme, k, want in [(1 << 10, 8, 2, 2, 5, -1), (1 << 10, 4, 2, 1, 9, -1),
                                        (1 << 10, 4, 2, 0, 2, -5), (1 << 10, 4, 2, 5, 2, -5),
                                        (1 << 10, 2, 2, 2, 2, -5), (1 << 10, 1, 3, 1, 2, -5)]:
        o = table.CkOptions()
        lib.ck_default_options(ctypes.byref(o))
        o.spawn_k = k
        assert lib.ck_create(bins, B, d, scheme, ctypes.byref(o), ctypes.c_void_p(256), 1 << 30,
                             None, ctypes.byref(h)) == want, (B, d, scheme, k)
    assert lib.ck_delete_noalloc(None, None, 5, None, None) == -1
