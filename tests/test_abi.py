"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/cblp.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cblp.h")
LIB = os.path.join(ROOT, "paper_2602_22421_amd", "libcblp.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2602_22421_amd.csrc import build as b
        b.build()
    return LIB


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("cblp_create", "spfom_iterate", "spfom_solve", "cblp_gap", "cblp_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], check=True,
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_agrees(lib_path):
    lib = ctypes.CDLL(lib_path)
    for n in _declared():
        assert hasattr(lib, n)
    from paper_2602_22421_amd import cblp
    assert set(cblp.EXPORTS) == set(_declared())
    assert lib.cblp_last_error is not None


def test_library_is_gfx950_only(lib_path, tmp_path):
    import shutil
    local = tmp_path / "lib.so"
    shutil.copy(lib_path, local)
    out = subprocess.run(["/opt/rocm/llvm/bin/llvm-objdump", "--offloading", str(local)],
                         capture_output=True, text=True, cwd=tmp_path)
    if out.returncode != 0:
        pytest.skip("llvm-objdump cannot list the offload bundles")
    targets = re.findall(r"amdgcn-amd-amdhsa-+(\w+)", out.stdout)
    assert targets and all(t == "gfx950" for t in targets), out.stdout


def test_oracle_shares_no_code_with_library():
    """The oracle and the HIP path are independent: no includes or imports
    across the boundary."""
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".c", ".py")):
            text = open(os.path.join(ROOT, "oracle", fn)).read()
            assert "paper_2602_22421_amd.cblp" not in text and "cblp.h" not in text
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2602_22421_amd")):
        for fn in files:
            if fn.endswith((".hip", ".py", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text
                assert "spfom_oracle" not in text
