"""The C-ABI library loads and exports every entry point include/sa.h declares
(no device needed)."""
import ctypes
import os
import re

from paper_1502_03701_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "sa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sa_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["sa_base_set", "sa_op_apply", "sa_precond_setup", "sa_precond_apply",
              "sa_gmres_solve", "sa_arnoldi_eigs"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_native.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert set(declared()) == set(_native.EXPORTED)


def test_version_and_null_context_errors():
    lib = _native.load()
    assert b"gfx950" in lib.sa_version()
    assert lib.sa_op_apply(None, 0, 1, None, None, 0.0) == _native.SA_EINVAL
    assert lib.sa_gmres_solve(None, None, 1, None, None, None, None) == _native.SA_EINVAL


def test_variant_names_match_the_header():
    text = open(os.path.join(ROOT, "include", "sa.h")).read()
    n = int(re.search(r"SA_JV_NVARIANTS\s*=\s*(\d+)", text).group(1))
    assert len(_native.JV_VARIANTS) == n
    for i, name in enumerate(_native.JV_VARIANTS):
        kind, depth = name.split("_z")
        assert re.search(r"SA_JV_%s_Z%s\s*=\s*%d\b" % (kind.upper(), depth, i), text), name


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: N > 1 exits with a message, before any GPU
    work (so this runs on the CPU)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
