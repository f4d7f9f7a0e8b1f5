"""The C-ABI library builds for gfx950, loads, and exports every declared symbol (CPU only)."""
import os
import re
import subprocess

import pytest

import paper_2106_00454_amd as wp
from paper_2106_00454_amd import build as wbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(wp.LIB_PATH):
        wbuild.build()
    return wp.LIB_PATH


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wpcd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wpcd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(wp.EXPORTS)


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (wpcd_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_library_loads_and_reports_version(libpath):
    L = wp.lib()
    for name in wp.EXPORTS:
        assert hasattr(L, name)
    assert wp.version().startswith("wpcd-gfx950")


def test_code_object_targets_gfx950(libpath, tmp_path):
    # the offload bundle header in .hip_fatbin names every device target
    out = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", libpath, str(out)], check=True)
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", out.read_bytes()))
    assert targets == {b"gfx950"}
