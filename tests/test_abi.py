"""The C-ABI library loads on any host and exports what include/lbm.h
declares; argument checks that touch no device memory behave as documented.
No compute calls: these run without a GPU."""
import ctypes
import os
import subprocess

import pytest

from paper_2012_11075_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2012_11075_amd import build
        build.build()
    return lbm.load()


def test_exports_every_declared_symbol(lib):
    names = lbm.header_functions()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_workspace_bytes_rejects_bad_params(lib):
    P = lbm.make_params
    for bad in [P(0, 4, 1.0, 0.1, 0.02, 1, 0.1), P(4, -1, 1.0, 0.1, 0.02, 1, 0.1),
                P(4, 4, 0.5, 0.1, 0.02, 1, 0.1), P(4, 4, float("nan"), 0.1, 0.02, 1, 0.1),
                P(4, 4, 1.0, -0.1, 0.02, 1, 0.1), P(4, 4, 1.0, 0.1, -1.0, 1, 0.1),
                P(4, 4, 1.0, 0.1, 0.02, 1, 0.1, precision=7),
                P(4, 4, 1.0, 0.1, 0.02, 1, 0.1, force_stencil=2),
                P(4, 70000, 1.0, 0.1, 0.02, 1, 0.1, force_stencil=1),
                P(4, 4, 1.0, 0.1, 0.02, 1, 0.1, nz=-1),
                P(4, 4, 1.0, 0.1, 0.02, 1, 0.1, nz=8, force_stencil=1),
                P(2048, 2048, 1.0, 0.1, 0.02, 1, 0.1, nz=1024),
                # a z-plane of 19 * 4096 * 8192 * 8 bytes is over 4 GiB
                P(8192, 4096, 1.0, 0.1, 0.02, 1, 0.1, nz=2)]:
        assert lib.lbm_workspace_bytes(ctypes.byref(bad)) == 0
    # the largest z-plane: 19 * 4096 * 6880 * 8 bytes, just below 4 GiB
    assert lib.lbm_workspace_bytes(ctypes.byref(P(6880, 4096, 1.0, 0.1, 0.02, 1, 0.1, nz=2))) > 0
    assert lib.lbm_workspace_bytes(ctypes.byref(P(6912, 4096, 1.0, 0.1, 0.02, 1, 0.1, nz=2))) == 0
    # a 3-D (D3Q19) lattice: two copies of 19 populations + 5 fields of staging
    p3 = P(64, 48, 1.0, 0.1, 0.02, 1, 0.1, nz=40)
    n3 = lib.lbm_workspace_bytes(ctypes.byref(p3))
    assert 2 * 19 * 64 * 48 * 40 * 8 + 5 * 64 * 48 * 40 * 8 <= n3 < 1.05 * (2 * 19 + 5) * 64 * 48 * 40 * 8
    # 3-D lattices in FP32-shifted storage (half the bytes of FP64)
    p3f = P(64, 48, 1.0, 0.1, 0.02, 1, 0.1, nz=40, precision="fp32s")
    n3f = lib.lbm_workspace_bytes(ctypes.byref(p3f))
    assert 2 * 19 * 64 * 48 * 40 * 4 + 5 * 64 * 48 * 40 * 8 <= n3f < n3
    # the fourth-order force stencil is accepted in FP64 and FP32-shifted
    for prec in ("fp64", "fp32s"):
        good = P(64, 48, 1.0, 0.1, 0.02, 1, 0.1, force_stencil=1, precision=prec)
        assert lib.lbm_workspace_bytes(ctypes.byref(good)) > 0


def test_row_pitch_overflow_rejected(lib):
    """A 2-D lattice whose row pitch (9 * nx rounded up to 32 elements) does
    not fit in 32 bits is rejected before any memory is touched, although it
    is under the 2^31-node limit."""
    P = lbm.make_params
    bad = P(300_000_000, 2, 1.0, 0.1, 0.02, 1, 0.1)
    assert lib.lbm_workspace_bytes(ctypes.byref(bad)) == 0
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(bad), 0x100000, 1 << 40, None, ctypes.byref(h)) == -1
    assert b"2^31" in lib.lbm_last_error(None) and not h.value
    # the widest accepted row: 9 * 238,609,280 = 2,147,483,520 elements
    ok = P(238_609_280, 2, 1.0, 0.1, 0.02, 1, 0.1)
    assert lib.lbm_workspace_bytes(ctypes.byref(ok)) > 0
    assert lib.lbm_workspace_bytes(ctypes.byref(P(238_609_312, 2, 1.0, 0.1, 0.02, 1, 0.1))) == 0


def test_lattice3_selector(lib):
    """lattice3 picks the 3-D velocity set: 0 or 19 D3Q19, 27 D3Q27 (two
    population copies of 27 instead of 19 per node); any other value, or a
    non-zero value on a 2-D lattice, is rejected."""
    P = lbm.make_params
    n19 = lib.lbm_workspace_bytes(ctypes.byref(P(64, 64, 1.0, 0.1, 0.02, 1, 0.1, nz=64)))
    n27 = lib.lbm_workspace_bytes(ctypes.byref(P(64, 64, 1.0, 0.1, 0.02, 1, 0.1, nz=64, q3=27)))
    p19 = P(64, 64, 1.0, 0.1, 0.02, 1, 0.1, nz=64)
    p19.lattice3 = 19
    assert lib.lbm_workspace_bytes(ctypes.byref(p19)) == n19
    assert n27 - n19 == 2 * 8 * 8 * 64 ** 3
    for bad in (1, 9, 26, 28, -1):
        q = P(64, 64, 1.0, 0.1, 0.02, 1, 0.1, nz=64)
        q.lattice3 = bad
        assert lib.lbm_workspace_bytes(ctypes.byref(q)) == 0
    flat = P(64, 64, 1.0, 0.1, 0.02, 1, 0.1)
    flat.lattice3 = 27
    assert lib.lbm_workspace_bytes(ctypes.byref(flat)) == 0
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(flat), 0x100000, 1 << 40, None, ctypes.byref(h)) == -1
    assert b"lattice3" in lib.lbm_last_error(None)
    # a z-plane of 27 populations must stay below 4 GiB: 27 * 2048 * 2048 * 8
    # bytes is 864 MiB; 27 * 65535 * 512 * 8 bytes = 6.7 GiB is rejected
    assert lib.lbm_workspace_bytes(ctypes.byref(P(512, 65535, 1.0, 0.1, 0.02, 1, 0.1, nz=2,
                                                  q3=27))) == 0
    assert lib.lbm_workspace_bytes(ctypes.byref(P(2048, 2048, 1.0, 0.1, 0.02, 1, 0.1, nz=2,
                                                  q3=27))) > 0


def test_params_struct_matches_header(lib):
    """lbm_params as ctypes lays it out: the field order of include/lbm.h."""
    import re
    with open(os.path.join(ROOT, "include", "lbm.h")) as fh:
        text = fh.read()
    body = re.search(r"typedef struct \{(.*?)\} lbm_params;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)\s*[,;]", body)
    assert names == [f[0] for f in lbm.Params._fields_], names


def test_workspace_bytes_layout(lib):
    # two population copies + 4 double fields of staging + reduction partials
    for prec, elem in [("fp64", 8), ("fp32s", 4)]:
        p = lbm.make_params(4096, 4096, 0.8, 0.1, 0.02, 1.0, 0.01, precision=prec)
        n = lib.lbm_workspace_bytes(ctypes.byref(p))
        assert n >= 2 * 9 * 4096 * 4096 * elem + 4 * 4096 * 4096 * 8
        assert n < 1.01 * (2 * 9 * 4096 * 4096 * elem + 4 * 4096 * 4096 * 8)


def test_create_argument_errors(lib):
    p = lbm.make_params(8, 8, 1.0, 0.1, 0.02, 1.0, 0.1)
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(p), None, 1 << 20, None, ctypes.byref(h)) == -1
    assert b"workspace" in lib.lbm_last_error(None)
    assert lib.lbm_create(ctypes.byref(p), 0x1001, 1 << 20, None, ctypes.byref(h)) == -1
    assert b"aligned" in lib.lbm_last_error(None)
    assert lib.lbm_create(ctypes.byref(p), 0x100000, 16, None, ctypes.byref(h)) == -2
    assert lib.lbm_create(None, 0x100000, 1 << 20, None, ctypes.byref(h)) == -1
    assert lib.lbm_create(ctypes.byref(p), 0x100000, 1 << 20, None, None) == -1
    assert not h.value


def test_null_context_calls(lib):
    assert lib.lbm_step(None, 1, 1) == -1
    assert lib.lbm_observe(None, None, None, None, None, None) == -1
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_status_string(-4) == b"non-finite state"
