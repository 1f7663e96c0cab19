"""The C ABI without a GPU: the library loads, exports every entry point that
include/dbbc.h declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2609_21848_amd as dbbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^[A-Za-z_][\w \*]*?\b(dbbc_\w+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported():
    lib = dbbc.load()
    declared = _declared()
    assert declared == set(dbbc.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    assert dbbc.dbbc_version() == "0.2.0"
    lib = dbbc.load()
    for code, word in [(0, "ok"), (-2, "range"), (-3, "sign"), (-4, "duplicate"), (-8, "gfx950")]:
        assert word in lib.dbbc_status_string(code).decode()


def _create(n_u, n_v, u, v, s, flags=0):
    lib = dbbc.load()
    out = ctypes.c_void_p()
    u = np.asarray(u, np.int32)
    v = np.asarray(v, np.int32)
    s = np.asarray(s, np.int8)
    rc = lib.dbbc_graph_create(n_u, n_v, len(u), u.ctypes.data, v.ctypes.data, s.ctypes.data,
                               flags, None, None, ctypes.byref(out))
    return rc, out.value, lib.dbbc_last_error().decode()


def test_argument_errors_need_no_device():
    # (ids, signs and duplicates are checked by the device build: GPU tests)
    assert _create(0, 2, [], [], [])[0] == dbbc.DBBC_E_INVALID_ARG
    assert _create(2**29, 2**29, [0], [0], [1])[0] == dbbc.DBBC_E_TOO_LARGE
    lib = dbbc.load()
    assert lib.dbbc_graph_create(2, 2, 1, None, None, None, 0, None, None, None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_graph_create(2, 2, 0, None, None, None, 0x80, None, None,
                                 ctypes.byref(ctypes.c_void_p())) == dbbc.DBBC_E_INVALID_ARG
    # an allocator needs both functions
    half = dbbc.Allocator()
    assert lib.dbbc_graph_create(2, 2, 0, None, None, None, 0, ctypes.byref(half), None,
                                 ctypes.byref(ctypes.c_void_p())) == dbbc.DBBC_E_INVALID_ARG
    out = ctypes.c_void_p()
    assert lib.dbbc_graph_create_text(None, 5, 0, None, None, ctypes.byref(out), None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_graph_create_text(b"1 2 1", 5, 0x80, None, None, ctypes.byref(out),
                                      None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_graph_create_text(b"1 2 1", 5, 0, None, None, None, None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_graph_create_text(b"1 2 1", 1 << 40, 0, None, None, ctypes.byref(out),
                                      None) == dbbc.DBBC_E_TOO_LARGE
    assert lib.dbbc_graph_raw_ids(None, 0, None, None) == dbbc.DBBC_E_INVALID_ARG
    # NULL handles are rejected or ignored
    assert lib.dbbc_count(None, None, None, None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_count_async(None, None, None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_count_read(None, None) == dbbc.DBBC_E_INVALID_ARG
    lib.dbbc_graph_destroy(None)
    # batches: bad arguments are rejected before any device work
    out = ctypes.c_void_p()
    assert lib.dbbc_batch_create(None, 1, None, 0, None, ctypes.byref(out)) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_batch_create(None, -1, None, 0, None, ctypes.byref(out)) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_batch_create(None, 0, None, 0x80, None, ctypes.byref(out)) == dbbc.DBBC_E_INVALID_ARG
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.dbbc_batch_create(arr, 1, None, 0, None, ctypes.byref(out)) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_batch_launch(None, None) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_batch_size(None) == 0
    lib.dbbc_batch_destroy(None)
    # servers
    assert lib.dbbc_server_create(None, None, None) == dbbc.DBBC_E_INVALID_ARG
    t = ctypes.c_int64()
    assert lib.dbbc_server_submit(None, 0, ctypes.byref(t)) == dbbc.DBBC_E_INVALID_ARG
    assert lib.dbbc_server_wait(None, 1, None, None) == dbbc.DBBC_E_INVALID_ARG
    lib.dbbc_server_destroy(None)
    assert lib.dbbc_now_ns() > 0


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(dbbc, "_lib", None)
    with pytest.raises(ImportError):
        dbbc.load(str(tmp_path / "nope.so"))


def test_plain_c_consumer(tmp_path):
    # the header compiles as strict C99 and a C program links against the
    # library and gets argument errors without a device
    import subprocess
    lib_dir = os.path.dirname(dbbc.LIB_PATH)
    exe = str(tmp_path / "abi_c")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                           f"-I{os.path.join(ROOT, 'include')}", "-o", exe,
                           os.path.join(ROOT, "tests", "native", "abi_c.c"), f"-L{lib_dir}", "-ldbbc",
                           f"-Wl,-rpath,{lib_dir}"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
