"""The C-ABI library loads and exports every symbol include/dgs.h declares.

No compute call is made here (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dgs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dgs_solve", "dgs_solve_ex", "dgs_solve_batched", "dgs_server_create",
                     "dgs_server_submit", "dgs_server_poll", "dgs_server_wait",
                     "dgs_server_destroy", "dgs_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1106_5694_amd as dgs
    if not os.path.exists(dgs.LIB_PATH):
        pytest.skip("libdgs.so not built")
    L = ctypes.CDLL(dgs.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(dgs.EXPORTS) == declared_functions()


def test_status_strings_without_gpu():
    import paper_1106_5694_amd as dgs
    if not os.path.exists(dgs.LIB_PATH):
        pytest.skip("libdgs.so not built")
    L = dgs.lib()
    assert L.dgs_status_string(0) == b"ok"
    assert L.dgs_status_string(2) == b"benefit out of range"
    assert L.dgs_version().startswith(b"dgs-gfx950")


def test_oracle_library_exports():
    import oracle
    L = oracle.lib()
    for name in ("orc_objective", "orc_greedy", "orc_scan", "orc_dgs_full", "orc_dgs_incr",
                 "orc_hungarian", "orc_is_permutation"):
        assert hasattr(L, name)


def test_product_does_not_reference_the_oracle():
    # the GPU library and its binding never load, import or link the oracle
    pkg = os.path.join(ROOT, "paper_1106_5694_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f


def test_binding_flags_and_result_fields_match_header():
    import paper_1106_5694_amd as dgs
    text = open(HEADER).read()
    for name, val in re.findall(r"#define (DGS_[A-Z_]+) (0x[0-9a-fA-F]+)u", text):
        assert getattr(dgs, name) == int(val, 16), name
    body = re.search(r"typedef struct dgs_result \{(.*?)\} dgs_result;", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b([a-z_]+)(?:\[[A-Z_]+\])?;", body)
    assert fields == [f for f, _ in dgs.Result._fields_]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no CPU fallback: without the built library every call raises
    import paper_1106_5694_amd as dgs
    monkeypatch.setattr(dgs, "LIB_PATH", str(tmp_path / "libdgs.so"))
    monkeypatch.setattr(dgs, "_lib", None, raising=False)
    with pytest.raises(RuntimeError):
        dgs.lib()
    with pytest.raises(RuntimeError):
        dgs.solve(np.zeros((4, 4), dtype=np.int32))
