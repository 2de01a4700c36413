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


def test_tuning_cache_json_round_trip(built, tmp_path):
    """usfft_tune_load / usfft_tune_save (host only): the JSON format keeps
    every entry's key and numbers; loading merges, the file's entries win."""
    import json

    import paper_2109_04131_amd as U
    src = tmp_path / "in.json"
    src.write_text(json.dumps({"version": 1, "entries": [
        {"key": "rader L=2592 fp32=1 G=3969", "a": 256, "b": 1, "time_ms": 0.081},
        {"key": "dst n=64 d=10 prec=1 model=0", "a": 2, "b": 0, "time_ms": 2.5}]}))
    U.tune_clear()
    U.tune_load(str(src))
    U.tune_load(str(src))  # merging the same entries again changes nothing
    out = tmp_path / "out.json"
    U.tune_save(str(out))
    got = {e["key"]: e for e in json.loads(out.read_text())["entries"]}
    assert set(got) == {"rader L=2592 fp32=1 G=3969", "dst n=64 d=10 prec=1 model=0"}
    assert (got["rader L=2592 fp32=1 G=3969"]["a"], got["rader L=2592 fp32=1 G=3969"]["b"]) == (256, 1)
    assert got["dst n=64 d=10 prec=1 model=0"]["a"] == 2
    U.tune_clear()
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"key": "x", "a": 1')
    with pytest.raises(U.UsfftError):
        U.tune_load(str(bad))
