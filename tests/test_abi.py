"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/tsqr.h, and rejects invalid arguments before touching
the device.  Also the host-side tree geometry (Sec. 2.1 trees)."""
import ctypes
import os
import re

import pytest

from paper_0808_2664_amd import _lib
from paper_0808_2664_amd.tsqr import plan_geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b((?:tsqr|caqr)_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert "tsqr_factor" in names and "tsqr_apply_qt" in names and "tsqr_form_q" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib.load()
    assert lib.tsqr_status_string(0) == b"success"
    assert lib.tsqr_status_string(-3) == b"invalid argument"


def test_factor_argument_errors_without_launch():
    lib = _lib.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: every call below fails its checks first
    h = vp()
    f = lib.tsqr_factor
    assert f(7, 100, 4, fake, 4, fake, 4, None, ctypes.byref(h), None) == -1       # dtype
    assert f(1, 0, 4, fake, 4, fake, 4, None, ctypes.byref(h), None) == -2         # m
    assert f(1, 3, 4, fake, 4, fake, 4, None, ctypes.byref(h), None) == -2         # m < n
    assert f(1, 100, 0, fake, 4, fake, 4, None, ctypes.byref(h), None) == -3       # n
    assert f(1, 100, 65, fake, 65, fake, 65, None, ctypes.byref(h), None) == _lib.TSQR_ERR_UNSUPPORTED
    assert f(1, 100, 4, None, 4, fake, 4, None, ctypes.byref(h), None) == -4       # A
    assert f(1, 100, 4, fake, 3, fake, 4, None, ctypes.byref(h), None) == -5       # lda
    assert f(1, 100, 4, fake, 4, fake, 3, None, ctypes.byref(h), None) == -7       # ldr
    bad = _lib.opts(flags=8)  # not a defined flag
    assert f(1, 100, 4, fake, 4, fake, 4, ctypes.byref(bad), ctypes.byref(h), None) == -8
    assert f(1, 100, 4, fake, 4, None, 4, None, None, None) == -9                  # nothing to return
    bad_h = _lib.opts(block_rows=100)
    assert f(1, 100, 4, fake, 4, fake, 4, ctypes.byref(bad_h), ctypes.byref(h), None) == _lib.TSQR_ERR_UNSUPPORTED


def test_apply_argument_errors():
    lib = _lib.load()
    vp = ctypes.c_void_p
    assert lib.tsqr_apply_qt(None, 4, vp(0x1000), 4, None) == -1
    assert lib.tsqr_apply_q(None, 4, vp(0x1000), 4, None) == -1
    assert lib.tsqr_form_q(None, vp(0x1000), 4, None) == -1
    assert lib.tsqr_qtree_destroy(None) == 0
    assert lib.tsqr_sign_normalize(5, 10, 4, None, 4, vp(0x1000), 4, None) == -1
    assert lib.tsqr_sign_normalize(1, 10, 4, None, 4, None, 4, None) == -6


@pytest.mark.parametrize("m,n,h,chains,arity", [
    (4096, 16, 64, 16, 0), (1 << 20, 64, 64, 0, 0), (1000, 8, 64, 0, 3),
    (300, 64, 64, 0, 0), (64, 64, 64, 0, 0), (129, 64, 64, 0, 0), (10000, 33, 64, 7, 4),
    (65536 + 17, 32, 64, 100, 2), (5000, 20, 64, 0, 2), (5000, 16, 64, 0, 5),
    (1 << 24, 8, 64, 0, 2), (777, 1, 64, 3, 0),
])
def test_plan_geometry_covers_rows(m, n, h, chains, arity):
    g = plan_geometry(m, n, block_rows=h, chains=chains, arity=arity)
    assert g["block_rows"] == h
    S, W = g["chain_rows"], g["chains"]
    assert S % h == 0 and W >= 1
    last = m - (W - 1) * S
    assert last >= n                      # every chain's first block holds an n x n leaf
    assert (W - 1) * S < m
    assert g["blocks"] == (W - 1) * (S // h) + (last + h - 1) // h
    # tree levels: smallest L with arity^L >= W
    a = g["arity"]
    assert a ** g["levels"] >= W and (g["levels"] == 0 or a ** (g["levels"] - 1) < W)
    assert g["padded_n"] in (8, 16, 32, 64) and g["padded_n"] >= n


def test_plan_geometry_config1_is_binary_tree_over_256_row_leaves():
    # leaves of 256 rows (chains of four 64-row blocks), binary tree
    g = plan_geometry(4096, 16, chains=16)
    assert g["block_rows"] == 64 and g["chains"] == 16 and g["chain_rows"] == 256
    assert g["arity"] == 2 and g["levels"] == 4


def test_plan_geometry_default_block_rows():
    # 64-row blocks; one wave per chain, 1024 chains at most by default
    for n in (1, 9, 32, 64):
        assert plan_geometry(1 << 20, n)["block_rows"] == 64
    assert plan_geometry(1 << 20, 64)["chains"] == 1024
    assert plan_geometry(1000, 64)["chains"] == 15


def test_plan_geometry_rejects_other_block_heights():
    for n, h in [(64, 128), (16, 256), (8, 32)]:
        with pytest.raises(_lib.TsqrError):
            plan_geometry(4096, n, block_rows=h)


def test_plan_geometry_short_last_chain_merges():
    # 3 chains of 256 rows would leave 10 rows (< n = 16) for a fourth chain
    g = plan_geometry(3 * 256 + 10, 16, chains=4)
    assert g["chains"] == 3
    assert 3 * 256 + 10 - 2 * g["chain_rows"] >= 16


def test_implicit_q_parameter_count():
    """Sec. 5.2: TSQR stores as many reflector entries as Householder QR,
    mn - n(n+1)/2, when every leaf is n x n or taller: each leaf stores the
    below-diagonal part of its block, each tree step an upper triangle of a
    combined triangle."""
    for (m, n, h) in [(4096, 16, 64), (1024, 8, 64), (2048, 64, 64), (4096, 32, 64)]:
        g = plan_geometry(m, n, block_rows=h, chains=m // h)
        W = g["chains"]
        leaves = W * (h * n - n * (n + 1) // 2)
        steps = (W - 1) * (n * (n + 1) // 2)
        assert leaves + steps == m * n - n * (n + 1) // 2


def test_lstsq_argument_errors_without_launch():
    lib = _lib.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: every call below fails its checks first
    f = lib.tsqr_lstsq
    assert f(7, 100, 4, fake, 4, 2, fake, 2, None, None, None) == -1           # dtype
    assert f(1, 3, 4, fake, 4, 2, fake, 2, None, None, None) == -2             # m < n
    assert f(1, 100, 0, fake, 4, 2, fake, 2, None, None, None) == -3           # n
    assert f(1, 100, 65, fake, 65, 2, fake, 2, None, None, None) == _lib.TSQR_ERR_UNSUPPORTED
    assert f(1, 100, 4, None, 4, 2, fake, 2, None, None, None) == -4           # A
    assert f(1, 100, 4, fake, 3, 2, fake, 2, None, None, None) == -5           # lda
    assert f(1, 100, 4, fake, 4, -1, fake, 2, None, None, None) == -6          # k
    assert f(1, 100, 4, fake, 4, 2, None, 2, None, None, None) == -7           # B
    assert f(1, 100, 4, fake, 4, 2, fake, 1, None, None, None) == -8           # ldb
    bad = _lib.opts(flags=8)
    assert f(1, 100, 4, fake, 4, 2, fake, 2, None, ctypes.byref(bad), None) == -10


def test_cholqr_argument_errors_without_launch():
    lib = _lib.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: every call below fails its checks first
    f = lib.tsqr_cholqr
    assert f(7, 100, 4, fake, 4, fake, 4, fake, 4, 1, None) == -1         # dtype
    assert f(1, 3, 4, fake, 4, fake, 4, fake, 4, 1, None) == -2           # m < n
    assert f(1, 100, 0, fake, 4, fake, 4, fake, 4, 1, None) == -3         # n
    assert f(1, 100, 65, fake, 65, fake, 65, fake, 65, 1, None) == _lib.TSQR_ERR_UNSUPPORTED
    assert f(1, 100, 4, None, 4, fake, 4, fake, 4, 1, None) == -4         # A
    assert f(1, 100, 4, fake, 3, fake, 4, fake, 4, 1, None) == -5         # lda
    assert f(1, 100, 4, fake, 4, None, 4, fake, 4, 1, None) == -6         # Q
    assert f(1, 100, 4, fake, 4, fake, 3, fake, 4, 1, None) == -7         # ldq
    assert f(1, 100, 4, fake, 4, fake, 4, None, 4, 1, None) == -8         # R
    assert f(1, 100, 4, fake, 4, fake, 4, fake, 3, 1, None) == -9         # ldr
    assert f(1, 100, 4, fake, 4, fake, 4, fake, 4, 3, None) == -10        # passes


def test_header_is_plain_c():
    # the boundary is a C ABI: the header must compile as C99 (no C++ or torch types)
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    hdr = os.path.join(ROOT, "include", "tsqr.h")
    p = subprocess.run([gcc, "-fsyntax-only", "-x", "c", "-std=c99", "-Wall", "-Werror", hdr],
                       capture_output=True, text=True)
    assert p.returncode == 0, p.stderr


def test_status_and_layout_calls_without_device_work():
    lib = _lib.load()
    assert lib.tsqr_status_string(_lib.TSQR_ERR_TIMEOUT).startswith(b"a bounded wait")
    assert lib.tsqr_apply_layout(None, 0, 32) == -1


def test_environment_does_not_change_the_tree(monkeypatch):
    # tuning comes only from tsqr_opts: the library reads no environment variable
    ref = plan_geometry(1 << 20, 64)
    for name, val in (("TSQR_CHAINS", "7"), ("TSQR_ARITY", "4"), ("TSQR_BLOCK_ROWS", "32")):
        monkeypatch.setenv(name, val)
    assert plan_geometry(1 << 20, 64) == ref
    assert ref["chains"] == 1024 and ref["arity"] == 2


def test_opts_struct_matches_header():
    src = open(os.path.join(ROOT, "include", "tsqr.h")).read()
    body = re.search(r"typedef struct tsqr_opts \{(.*?)\} tsqr_opts;", src, flags=re.S).group(1)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert fields == [f for f, _ in _lib.TsqrOpts._fields_]


def test_mgs_argument_errors():
    lib = _lib.load()
    vp = ctypes.c_void_p
    f = vp(0x1000)  # never dereferenced: every call fails its checks first
    assert lib.tsqr_mgs(7, 10, 4, f, 4, f, 4, f, 4, None) == -1
    assert lib.tsqr_mgs(1, 3, 4, f, 4, f, 4, f, 4, None) == -2
    assert lib.tsqr_mgs(1, 100, 65, f, 65, f, 65, f, 65, None) == _lib.TSQR_ERR_UNSUPPORTED
    assert lib.tsqr_mgs(1, 100, 4, f, 4, f, 5, f, 4, None) == -7  # Q is A with another ld
    assert lib.tsqr_mgs(1, 100, 4, f, 4, vp(0x2000), 4, None, 4, None) == -8


def test_noalloc_argument_errors_without_launch():
    lib = _lib.load()
    vp = ctypes.c_void_p
    f = vp(0x1000)  # never dereferenced: every call fails its checks first
    g = lib.tsqr_factor_noalloc
    assert g(7, 100, 4, f, 4, f, 4, None, None) == -1
    assert g(1, 3, 4, f, 4, f, 4, None, None) == -2
    assert g(1, 100, 4, None, 4, f, 4, None, None) == -4
    assert g(1, 100, 4, f, 4, None, 4, None, None) == -6   # R is required
    big = _lib.opts(chains=4096)  # 4096 chain R slots of 64 x 64 FP64 exceed the fixed scratch
    assert g(1, 1 << 20, 64, f, 64, f, 64, ctypes.byref(big), None) == _lib.TSQR_ERR_SCRATCH
    assert lib.tsqr_factor_noalloc_scratch_bytes() == 40 << 20


def test_caqr_left_argument_errors_without_launch():
    lib = _lib.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)  # never dereferenced: every call below fails its checks first
    h = vp()
    f = lib.caqr_factor_left
    F64, F32 = _lib.TSQR_F64, _lib.TSQR_F32
    assert f(7, 100, 50, fake, 50, 64, 64, F64, None, ctypes.byref(h), None) == -1     # dtype
    assert f(F64, 0, 50, fake, 50, 64, 64, F64, None, ctypes.byref(h), None) == -2     # m
    assert f(F64, 40, 50, fake, 50, 64, 64, F64, None, ctypes.byref(h), None) == -2    # m < n
    assert f(F64, 100, 0, fake, 50, 64, 64, F64, None, ctypes.byref(h), None) == -3    # n
    assert f(F64, 100, 50, None, 50, 64, 64, F64, None, ctypes.byref(h), None) == -4   # A
    assert f(F64, 100, 50, fake, 49, 64, 64, F64, None, ctypes.byref(h), None) == -5   # lda
    assert f(F64, 100, 50, fake, 50, 65, 65, F64, None, ctypes.byref(h), None) == -6   # panel > 64
    assert f(F64, 100, 50, fake, 50, 64, 100, F64, None, ctypes.byref(h), None) == -7  # not a multiple
    assert f(F64, 100, 50, fake, 50, 64, 32, F64, None, ctypes.byref(h), None) == -7   # below the panel
    assert f(F32, 100, 50, fake, 50, 64, 64, F64, None, ctypes.byref(h), None) == -8   # FP64 update, FP32 storage
    assert f(F64, 100, 50, fake, 50, 64, 64, 9, None, ctypes.byref(h), None) == -8     # update dtype
    bad = _lib.opts(flags=64)  # not a defined flag
    assert f(F64, 100, 50, fake, 50, 64, 64, F64, ctypes.byref(bad), ctypes.byref(h), None) == -9


def test_form_q_signed_argument_errors_without_launch():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    assert lib.tsqr_form_q_signed(None, fake, 64, fake, 64, 0, None) == -1


def test_release_workspace_pools_without_device_work():
    # no pool exists before any call that allocates: no HIP call is made
    assert _lib.load().tsqr_release_workspace_pools() == 0
