"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/bang.h declares, and rejects invalid arguments before
touching a device (validation is host-side and synchronous)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2401_11324_amd as bang

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NONE = 0xFFFFFFFF


def header_functions():
    src = open(os.path.join(ROOT, "include", "bang.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bang_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    assert header_functions() == sorted(bang.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = bang.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_library_is_hip_for_gfx950():
    # the code object inside the library targets gfx950
    data = open(bang.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _desc(n=100, d=32, m=16, R=8, dtype=np.uint8, medoid=0, adj=None,
          flags=0):
    rng = np.random.default_rng(0)
    rows = max(n, 1)
    base = rng.integers(0, 255, size=(rows, d)).astype(dtype)
    if adj is None:
        adj = np.stack([rng.choice(max(n, R), R, replace=False)
                        for _ in range(rows)])
    adj = np.ascontiguousarray(adj, dtype=np.uint32)
    cb = np.zeros((m, 256, d // m), dtype=np.float32)
    codes = np.zeros((rows, m), dtype=np.uint8)
    keep = (base, adj, cb, codes)
    dt = {np.dtype(np.float32): 0, np.dtype(np.uint8): 1,
          np.dtype(np.int8): 2}[np.dtype(dtype)]
    desc = bang.IndexDesc(n, d, dt, base.ctypes.data, adj.shape[1],
                          adj.ctypes.data, medoid, m, cb.ctypes.data,
                          codes.ctypes.data, flags)
    return desc, keep


def _create(desc):
    h = ctypes.c_void_p()
    rc = bang.lib().bang_index_create(ctypes.byref(desc), ctypes.byref(h))
    return rc, h, bang.lib().bang_last_error().decode()


@pytest.mark.parametrize("mutate,code,msg", [
    (dict(n=0), -1, "n must be"),
    (dict(m=5), -1, "m must divide d"),
    (dict(R=65, adj=np.zeros((100, 65))), -1, "R must be"),
    (dict(medoid=100), -1, "medoid"),
    (dict(flags=4), -1, "flags"),            # HOST_ADJ | BF16_BASE only
    (dict(flags=2), -4, "BF16_BASE"),        # bfloat16 base: float data
    (dict(m=4), -4, "no kernel"),            # d/m = 8 not compiled
])
def test_create_rejects_bad_descriptions(mutate, code, msg):
    desc, keep = _desc(**mutate)
    rc, h, err = _create(desc)
    assert rc == code and msg in err
    assert not h.value


def test_create_rejects_out_of_range_and_repeated_ids():
    n, R = 50, 4
    adj = np.tile(np.arange(R, dtype=np.uint32), (n, 1))
    adj[7, 2] = n + 3
    desc, keep = _desc(n=n, R=R, adj=adj)
    rc, _, err = _create(desc)
    assert rc == -1 and "row 7" in err and ">= n" in err
    adj[7, 2] = 1                         # row 7 now holds id 1 twice
    desc, keep = _desc(n=n, R=R, adj=adj)
    rc, _, err = _create(desc)
    assert rc == -1 and "twice" in err
    adj[7, 2] = NONE                      # empty slots are fine
    desc, keep = _desc(n=n, R=R, adj=adj)
    rc, h, err = _create(desc)
    assert rc in (0, -3)                  # -3: no GPU in this container
    if rc == 0:
        bang.lib().bang_index_destroy(h)


def test_calls_with_null_index_fail_cleanly():
    L = bang.lib()
    assert L.bang_search(None, None, 1, 10, 10, None, None, None, None) == -1
    assert L.bang_build_pq_tables(None, None, 1, None, None) == -1
    assert L.bang_rerank(None, None, 1, None, 4, 1, None, None, None) == -1
    assert L.bang_index_probe(None, 10, 0, None, None, None) == -1
    assert b"null index" in L.bang_last_error()
    assert L.bang_index_destroy(None) == 0


def test_server_calls_with_null_arguments_fail_cleanly():
    import ctypes
    L = bang.lib()
    o = bang.ServerOpts(16, 1, 10, 64, 0, 0)
    h = ctypes.c_void_p()
    assert L.bang_server_create(None, ctypes.byref(o), ctypes.byref(h)) == -1
    assert not h.value
    t = ctypes.c_uint64()
    assert L.bang_server_submit(None, None, 1, 1, 1, ctypes.byref(t)) == -1
    assert L.bang_server_wait(None, 1, None, None, 0) == -1
    assert L.bang_server_replay(None, None, 0, None, None, None, None, 1,
                                None, None, None) == -1
    assert L.bang_server_stats(None, None, 0) == -1
    assert L.bang_server_destroy(None) == 0
    assert "null" in L.bang_last_error().decode()


def test_python_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(bang, "_lib", None)
    monkeypatch.setattr(bang, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        bang.lib()
