"""The C-ABI library loads on a machine without a GPU and exports every
entry point that include/prot.h declares; its pure host functions work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "prot.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prot_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    syms = declared_symbols()
    for s in ("prot_solve_rounded", "prot_solve_points", "prot_solve_cost",
              "prot_round_costs", "prot_build_costs", "prot_ctx_create"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2203_03732_amd import _lib
    lib = _lib.load()
    for s in declared_symbols():
        assert hasattr(lib, s), f"{s} is declared in prot.h but not exported"
    assert set(_lib.EXPORTS) == set(declared_symbols())


def test_host_helpers():
    import paper_2203_03732_amd as prot
    assert prot.pitch(1) == 128 and prot.pitch(128) == 128 and prot.pitch(129) == 256
    assert prot.pitch(10000) == 10112
    assert prot.threshold(0.01, 10000) == 100
    assert prot.threshold(0.1, 1000) == 100
    assert prot.threshold(0.005, 50000) == 250
    assert prot.threshold(0.05, 64) == 3
    lib = prot.load()
    assert lib.prot_status_string(-2) == b"cost out of range or not finite"


def test_null_context_is_rejected():
    import paper_2203_03732_amd as prot
    lib = prot.load()
    assert lib.prot_solve_rounded(None, None, 0, 0, 0, None, 0, None, None, None, None, None) == -1
    assert lib.prot_last_error(None) == b"null context"


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message (the library has no
    multi-GPU path), before touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout == ""
