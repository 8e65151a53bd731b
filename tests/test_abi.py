"""The C-ABI library loads and exports every entry point include/ranky.h declares; the host-side
argument checks answer before any device work.  No GPU needed (no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ranky.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ranky_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2009_09767_amd import ranky

    if not os.path.exists(ranky.LIB_PATH):
        from paper_2009_09767_amd import build

        build.build()
    return ranky.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ranky_svd", "ranky_workspace_bytes", "ranky_ctx_create", "ranky_occupancy", "ranky_gram",
                 "ranky_eigh", "ranky_backproject", "ranky_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_default_opts_and_version(L):
    from paper_2009_09767_amd import ranky

    o = ranky.Opts()
    assert L.ranky_default_opts(ctypes.byref(o)) == 0
    assert (o.gram_prec, o.validate, o.v_dtype, o.max_sweeps) == (0, 1, 1, 40)
    assert o.refine == -1 and o.graph == 0    # refinement chosen per call; no graph replay by default
    assert b"gfx950" in L.ranky_version()


def test_workspace_sizing(L):
    from paper_2009_09767_amd import ranky

    o = ranky.make_opts()
    small = ranky.workspace_bytes(64, 4096, 5000, 64, o)
    big = ranky.workspace_bytes(1024, 1 << 20, 1_050_000, 128, o)
    assert 0 < small < big
    # G and the eigenvector matrix dominate: 2 * 1024^2 doubles plus the row-major copy (8 B / nnz)
    assert big >= 2 * 1024 * 1024 * 8 + 8 * 1_050_000
    assert ranky.workspace_bytes(0, 10, 0, 1, o) == 0
    assert ranky.workspace_bytes(10, 10, 0, 11, o) == 0      # k > M
    assert ranky.workspace_bytes(9000, 10, 0, 1, o) == 0     # M above the 8192 cap
    o.n_blocks = 11
    assert ranky.workspace_bytes(10, 10, 0, 1, o) == 0       # D > N


def test_host_checks_return_before_device_work(L):
    from paper_2009_09767_amd import ranky

    csc = ranky.Csc(0, 0, 0, 0, 1)
    info = ranky.Info()
    o = ranky.make_opts()
    st = L.ranky_svd(None, ctypes.byref(csc), 4, 4, 1, 0.0, ctypes.byref(o), None, 0, None, None, None,
                     ctypes.byref(info), None)
    assert st == ranky.E_INVALID and info.status == ranky.E_INVALID
    assert L.ranky_last_error()
    assert L.ranky_eigh(0, None, None, None, 0, None, None, 0, None) == ranky.E_INVALID
    t = ctypes.c_uint64(7)
    assert L.ranky_svd_async(None, ctypes.byref(csc), 4, 4, 1, 0.0, ctypes.byref(o), None, 0, None, None, None, None,
                             ctypes.byref(t)) == ranky.E_INVALID
    assert t.value == 7   # untouched on an error
    assert L.ranky_query(None, 1, None) == ranky.E_INVALID
    assert L.ranky_eigh_workspace_bytes(0) == 0 and L.ranky_eigh_workspace_bytes(100) > 2 * 128 * 128 * 8


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2009_09767_amd import ranky

    monkeypatch.setattr(ranky, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ranky, "_lib", None)
    with pytest.raises(ranky.RankyError):
        ranky.lib()


def test_struct_layouts_match_the_binding(tmp_path):
    """Every field offset and struct size of the C header, as gcc lays them out, equals the
    ctypes binding's (a drift would pass garbage across the boundary)."""
    import shutil
    import subprocess

    from paper_2009_09767_amd import ranky

    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"ranky_csc": ranky.Csc, "ranky_opts": ranky.Opts, "ranky_info": ranky.Info,
               "ranky_batch_item": ranky.BatchItem, "ranky_serve_cfg": ranky.ServeCfg,
               "ranky_request": ranky.Request, "ranky_serve_summary": ranky.ServeStats,
               "ranky_tune_report": ranky.TuneReport, "ranky_paper_info": ranky.PaperInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ranky.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = str(tmp_path / "layout")
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
