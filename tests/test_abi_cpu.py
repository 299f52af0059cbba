"""CPU checks of the C ABI boundary: the built library loads and exports every
function that include/vecchia.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vecchia.h")
LIB = os.path.join(ROOT, "paper_2410_04477_amd", "libvecchia.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(vecchia_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for f in ("vecchia_blocks", "vecchia_neighbors", "vecchia_loglik", "vecchia_loglik_grad"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_version_without_gpu():
    from paper_2410_04477_amd import _lib as L
    lib = L.lib()
    assert lib.vecchia_version() >= 10000
    assert lib.vecchia_status_string(L.EINVAL).decode() == "invalid argument"
    # workspace-size queries are host-only arithmetic
    assert lib.vecchia_plan_workspace_size(100, 2) > 100 * 2 * 8
    assert lib.vecchia_plan_workspace_size(0, 1) == 0


def test_binding_signatures_cover_header():
    from paper_2410_04477_amd import _lib as L
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_fp32_wave_kernels_keep_their_tiles_in_registers():
    """The build records each kernel's register use (compiler resource remarks).
    No FP32 closed-form one-wave kernel may spill (its tiles would go through
    scratch), and the FP32 classes up to G = 9 must keep two waves per SIMD.
    (The Bessel-form kernels, for nu outside the closed forms, call a
    non-inlined function and keep a call frame in scratch.)"""
    import json
    import re
    path = os.path.join(ROOT, "paper_2410_04477_amd", "_build", "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("library not built")
    res = json.load(open(path))
    seen = 0
    for name, r in res.items():
        mt = re.search(r"bv_wave_kernelIfLi(\d+)ELi(\d)ELb0E", name)
        if not mt:
            continue
        seen += 1
        g = int(mt.group(1))
        assert r["scratch"] == 0, (name, r)
        if g <= 9:
            assert r["occupancy"] >= 2, (name, r)
    assert seen == 24   # value G = 1..11, fused gradient G = 1..9, split gradient G = 10, 11 (two kernels)
