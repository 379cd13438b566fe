"""The C-ABI library loads and exports every function include/*.h declares (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["dirac_create", "dirac_destroy", "dirac_apply", "dirac_apply_eo", "clover_invert", "dirac_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2502_02490_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdirac.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2502_02490_amd import _lib

    with pytest.raises(RuntimeError):
        _lib.load.__wrapped__(str(tmp_path / "missing.so")) if hasattr(_lib.load, "__wrapped__") else _load_missing(tmp_path)


def _load_missing(tmp_path):
    import importlib

    from paper_2502_02490_amd import _lib

    saved = _lib._lib
    try:
        _lib._lib = None
        _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved


def test_hop_shape_count_matches_table_and_bench_names():
    """DIRAC_HOP_SHAPE indexes the hop kernel's shape table: the GPU tests that run every shape,
    and bench.py's shape names, have as many entries as the table."""
    import ast
    import sys

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import N_HOP_SHAPES

    src = open(os.path.join(ROOT, "paper_2502_02490_amd", "csrc", "hop_kernels.h")).read()
    table = re.search(r"const HopShape kShapes\[\] = \{(.*?)\};", src, flags=re.S).group(1)
    assert len(re.findall(r"\{[^{}]*\}", table)) == N_HOP_SHAPES
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    names = [n for n in tree.body if isinstance(n, ast.Assign) and getattr(n.targets[0], "id", "") == "HOP_SHAPES"]
    assert len(names) == 1 and len(names[0].value.elts) == N_HOP_SHAPES
