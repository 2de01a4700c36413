"""CPU checks of the C ABI: the library loads and exports every declared call."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2109_04131_amd", "libusfft.so")
HEADER = os.path.join(ROOT, "include", "usfft.h")


def declared():
    txt = open(HEADER).read()
    pat = r"^\s*(?:usfft_status|void|int64_t|const char\s*\*)\s*(usfft_\w+)\s*\("
    return sorted(set(re.findall(pat, txt, flags=re.M)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    return LIB


def test_header_declares_stage_calls():
    names = declared()
    for need in ["usfft_plan_create", "usfft_detect", "usfft_eval", "usfft_sample", "usfft_line_dft",
                 "usfft_lattice_dft", "usfft_select", "usfft_product", "usfft_compact", "usfft_family",
                 "usfft_nodes"]:
        assert need in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (usfft_[a-z_0-9]+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_loads_and_covers_abi(built):
    import paper_2109_04131_amd as U
    assert U.version().startswith("usfft")
    assert set(U.EXPORTED) == set(declared())


def test_binding_shares_torchs_hip_runtime(built):
    # one HIP runtime per process: the library binds to the one PyTorch
    # ships (same soname), whichever module the caller imports first
    code = ("import paper_2109_04131_amd\n"
            "m = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(m))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True).stdout
    assert out.strip() == "1"
