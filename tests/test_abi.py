"""The C-ABI library: it loads, exports every symbol include/relax.h declares, and its
pure host-side logic (configuration checks, workspace sizing, status texts) behaves.
No GPU and no compute calls here."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1405_0942_amd as R
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "relax.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(relax_[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding_exports():
    assert declared_functions() == sorted(R.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = R.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (relax_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_library_is_gfx950_code_object():
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", R.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_strerror_texts():
    for code in (R.RELAX_OK, R.RELAX_E_ARG, R.RELAX_E_HIP, R.RELAX_E_FOLD, R.RELAX_E_DT, R.RELAX_E_NAN,
                 R.RELAX_E_STATE, R.RELAX_E_SPACE):
        assert R.relax_strerror(code) and R.relax_strerror(code) != "unknown status"
    assert R.relax_strerror(12345) == "unknown status"


def _cfg(**kw):
    g = W.make_grid((16, 16, 16), [(-1.0, 1.0)] * 3, (0, 0, 0))
    return R.make_config(g, **kw)


def test_workspace_bytes_valid_and_invalid():
    c = _cfg()
    n64 = R.relax_workspace_bytes(c)
    N3 = 3 * 16 ** 3
    # at least: two position buffers, k_1..k_3, y_5, three partial sums and B0, all FP64
    assert n64 >= 10 * N3 * 8
    cm = _cfg(precision=R.RELAX_FP32_MIXED)
    nm = R.relax_workspace_bytes(cm)
    assert 0 < nm < n64 + N3 * 8
    cr = _cfg(record=True, checkpoint_every=20)
    assert R.relax_workspace_bytes(cr, 200) >= n64 + 200 * 8 + 11 * N3 * 8
    bad = _cfg()
    bad.n[0] = 3
    assert R.relax_workspace_bytes(bad) == 0
    bad = _cfg()
    bad.h[1] = 0.0
    assert R.relax_workspace_bytes(bad) == 0
    bad = _cfg()
    bad.bc[2] = 7
    assert R.relax_workspace_bytes(bad) == 0
    bad = _cfg(tol=-1.0)
    assert R.relax_workspace_bytes(bad) == 0
    for sf in (0.0, 1.5, float("nan")):
        assert R.relax_workspace_bytes(_cfg(safety=sf)) == 0
    assert R.relax_workspace_bytes(_cfg(), -1) == 0
    # plane size limit: n[0] * n[1] < 2^28 (32-bit buffer offsets within a plane)
    big = _cfg()
    big.n[0], big.n[1], big.n[2] = 1 << 14, 1 << 14, 4
    assert R.relax_workspace_bytes(big) == 0
    big.n[1] = (1 << 14) - 1
    assert R.relax_workspace_bytes(big) >= 10 * 3 * big.n[0] * big.n[1] * 4 * 8


def test_init_rejects_bad_arguments_without_touching_the_gpu():
    c = _cfg()
    bad = _cfg()
    bad.n[0] = 2
    rc, ctx = R.relax_init(bad, 0, 1 << 20, 1 << 20, 1 << 20, 1 << 30, None)
    assert rc == R.RELAX_E_ARG and not ctx.value
    # misaligned workspace
    rc, ctx = R.relax_init(c, 0, 1 << 20, 1 << 20, (1 << 20) + 8, 1 << 30, None)
    assert rc == R.RELAX_E_ARG and not ctx.value
    # too small a workspace
    rc, ctx = R.relax_init(c, 0, 1 << 20, 1 << 20, 1 << 20, 1024, None)
    assert rc == R.RELAX_E_SPACE and not ctx.value
    # null context handles
    assert R.lib().relax_step(None, 1, None, None) == R.RELAX_E_ARG
    assert R.lib().relax_diagnostics(None, None) == R.RELAX_E_ARG
    assert R.lib().relax_velocity(None, None) == R.RELAX_E_ARG
    assert R.lib().relax_fields(None, None, None) == R.RELAX_E_ARG
    assert R.lib().relax_monitors(None, None, None) == R.RELAX_E_ARG
    assert R.relax_last_error(None) == ""
    R.relax_destroy(None)


def test_config_struct_layout_matches_header():
    # n[3] int, h[3] double, bc[3] int, precision int, gamma, dt0, dt_min, tol double,
    # adaptive, record, checkpoint_every int, xi_null_tau double, safety double, curl int (+4 pad)
    assert ctypes.sizeof(R.relax_config) == 12 + 4 + 24 + 12 + 4 + 32 + 12 + 4 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(R.relax_diag) == 7 * 8 + 8


def test_noalloc_rejects_without_touching_the_gpu():
    """relax_diagnostics_noalloc checks its arguments and its scratch limit (16384 workgroups
    of 64 x 8 nodes) on the host, before any GPU work."""
    c = _cfg()
    assert R.relax_diagnostics_noalloc(c, 0, 1 << 20, None)[0] == R.RELAX_E_ARG
    bad = _cfg()
    bad.n[0] = 3
    assert R.relax_diagnostics_noalloc(bad, 1 << 20, 1 << 20, None)[0] == R.RELAX_E_ARG
    big = _cfg()
    big.n[0], big.n[1], big.n[2] = 4096, 4096, 4  # 32768 tiles of 64 x 8
    assert R.relax_workspace_bytes(big) > 0
    assert R.relax_diagnostics_noalloc(big, 1 << 20, 1 << 20, None)[0] == R.RELAX_E_SPACE
