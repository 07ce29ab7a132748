"""Host-side checks of the C ABI library (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppq.h")
LIB = os.path.join(ROOT, "paper_1606_04004_amd", "libppq.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ppq_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ppq_create", "ppq_destroy", "ppq_set_grid", "ppq_add_potential_term", "ppq_set_state",
                     "ppq_get_state", "ppq_init_gaussian", "ppq_apply_h", "ppq_step", "ppq_prune",
                     "ppq_propagate", "ppq_observables"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ppq_[a-z_0-9]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_binding_matches_header():
    from paper_1606_04004_amd import _ppq
    lib = _ppq.load()
    assert set(_ppq.SIGNATURES) == set(declared_functions())
    for name in _ppq.SIGNATURES:
        assert getattr(lib, name) is not None


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_1606_04004_amd import _ppq
    monkeypatch.setattr(_ppq, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_ppq, "_LIB", None)
    with pytest.raises(RuntimeError):
        _ppq.load()


def test_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1606_04004_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("no oracle", ""), f
