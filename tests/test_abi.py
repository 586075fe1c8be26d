"""The C-ABI library builds, loads and exports every entry point the header declares
(no GPU calls: these run on the CPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmpcast.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rmpc_status|const char \*)\s*(rmpc_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2301_08068_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rmpc_create", "rmpc_destroy", "rmpc_map_upload", "rmpc_map_release", "rmpc_query",
                 "rmpc_scan_query", "rmpc_trace_debug", "rmpc_directions", "rmpc_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(rmpc_\w+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_resolves(lib_path):
    from paper_2301_08068_amd import binding
    assert set(binding.exported_symbols()) == set(_declared())
    assert binding._lib.rmpc_last_error() == b""


def test_library_has_no_oracle_dependency(lib_path):
    """The product library neither links nor names the oracle."""
    out = subprocess.run(["nm", "-D", lib_path], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", lib_path], capture_output=True, text=True).stdout
    assert "rmp_oracle" not in ldd
    for f in os.listdir(os.path.join(ROOT, "paper_2301_08068_amd")):
        if f.endswith(".py"):
            src = open(os.path.join(ROOT, "paper_2301_08068_amd", f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f
