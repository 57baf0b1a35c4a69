"""The C-ABI library loads and exports every entry point declared in
include/*.h, and the ctypes structs match the C layout (CPU only: no compute
call is made)."""

import ctypes
import glob
import os
import re
import subprocess

import pytest

import paper_1407_1785_amd as lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for header in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(header).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("tsvt", "tsvd_complete", "trpca", "tsvd_create", "tsvd_destroy", "tsvd_set_stream",
               "tsvd_status_string", "tsvd_last_error", "tsvd_batch_run", "tsvd_submit", "tsvd_poll",
               "tsvd_serve_stats_read", "tsvd_factors", "tsvd_compress", "tsvd_cancel"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lib.library_path()):
        pytest.skip("libtsvd.so not built")
    so = ctypes.CDLL(lib.library_path())
    missing = [n for n in sorted(declared_functions()) if not hasattr(so, n)]
    assert not missing, missing
    # every declared function has a binding signature
    assert declared_functions() <= set(lib._SIGNATURES)


def test_status_strings_without_gpu():
    if not os.path.exists(lib.library_path()):
        pytest.skip("libtsvd.so not built")
    so = lib.load_library()
    assert so.tsvd_status_string(0) == b"ok"
    assert so.tsvd_status_string(-5) == b"non-finite value"


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tsvd.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\\n\", sizeof(tsvd_shape), sizeof(tsvd_admm_opts),"
        " sizeof(tsvd_info), offsetof(tsvd_shape, n), offsetof(tsvd_info, primal),"
        " offsetof(tsvd_admm_opts, max_sweeps));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    want = [ctypes.sizeof(lib.Shape), ctypes.sizeof(lib.AdmmOpts), ctypes.sizeof(lib.Info),
            lib.Shape.n.offset, lib.Info.primal.offset, lib.AdmmOpts.max_sweeps.offset]
    assert got == want


def test_batch_struct_layouts_match_c(tmp_path):
    src = tmp_path / "layout2.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tsvd.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(tsvd_problem),"
        " offsetof(tsvd_problem, shape), offsetof(tsvd_problem, x), offsetof(tsvd_problem, penalty),"
        " offsetof(tsvd_problem, opts), offsetof(tsvd_problem, out_s), sizeof(tsvd_serve_stats),"
        " offsetof(tsvd_serve_stats, peak_running));return 0;}\n")
    exe = tmp_path / "layout2"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    P = lib.ProblemRecord
    want = [ctypes.sizeof(P), P.shape.offset, P.x.offset, P.penalty.offset, P.opts.offset, P.out_s.offset,
            ctypes.sizeof(lib.ServeStats), lib.ServeStats.peak_running.offset]
    assert got == want


def test_state_and_stat_layouts_match_c(tmp_path):
    src = tmp_path / "layout3.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "tsvd.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(tsvd_state),"
        " offsetof(tsvd_state, penalty), offsetof(tsvd_state, iter), offsetof(tsvd_state, save),"
        " offsetof(tsvd_admm_opts, state), sizeof(tsvd_kernel_stat), offsetof(tsvd_kernel_stat, slice_sweeps),"
        " offsetof(tsvd_kernel_stat, rotations), offsetof(tsvd_problem, deadline_s));return 0;}\n")
    exe = tmp_path / "layout3"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()))
    S, K = lib.StateRecord, lib.KernelStat
    want = [ctypes.sizeof(S), S.penalty.offset, S.iter.offset, S.save.offset, lib.AdmmOpts.state.offset,
            ctypes.sizeof(K), K.slice_sweeps.offset, K.rotations.offset, lib.ProblemRecord.deadline_s.offset]
    assert got == want


def test_serving_status_strings():
    if not os.path.exists(lib.library_path()):
        pytest.skip("libtsvd.so not built")
    so = lib.load_library()
    assert so.tsvd_status_string(-8) == b"cancelled"
    assert so.tsvd_status_string(-9) == b"deadline passed"


def test_busy_status_string():
    if not os.path.exists(lib.library_path()):
        pytest.skip("libtsvd.so not built")
    assert lib.load_library().tsvd_status_string(-7) == b"not finished"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setenv("TSVD_LIBRARY", str(tmp_path / "absent.so"))
    with pytest.raises(lib.LibraryNotBuilt):
        lib.load_library()
