"""CPU checks of the C ABI boundary: the built library loads and exports every
function that include/vecchia.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import numpy as np
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
    # value G = 1..11; gradient: tile buffer G = 1..9, registers G = 1..10, split G = 11
    assert seen == 32


def test_fp64_gradient_kernels_do_not_spill():
    """The FP64 closed-form gradient kernels the plans use keep their working
    set in registers: the register-resident adjoint (mode 5, G <= 9), and for
    the classes above G = 9 the left-looking factorisation (mode 6, one tile
    column in the registers at a time, two waves per SIMD) and the adjoint from
    the stored tiles (mode 3)."""
    import json
    import re
    path = os.path.join(ROOT, "paper_2410_04477_amd", "_build", "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("library not built")
    res = json.load(open(path))
    seen = {}
    for name, r in res.items():
        mt = re.search(r"bv_wave_kernelIdLi(\d+)ELi([356])ELb0E", name)
        if not mt:
            continue
        g, mode = int(mt.group(1)), int(mt.group(2))
        seen[(g, mode)] = r
        assert r["scratch"] == 0, (name, r)
        if mode == 6:
            assert r["occupancy"] >= 2, (name, r)
    assert {(g, 5) for g in range(1, 10)} <= set(seen)
    assert {(10, 6), (11, 6), (10, 3), (11, 3)} <= set(seen)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_plan_layout_matches_binding_and_mismatch_is_caught():
    """The ctypes mirror of vecchia_plan must have the library's layout; a
    mirror with a field missing or a field of the wrong width is reported."""
    import ctypes
    from paper_2410_04477_amd import _lib as L
    lib = L.lib()   # raises on a mismatch
    assert L.plan_layout_mismatch(lib) is None
    fields = list(L.Plan._fields_)

    class Dropped(ctypes.Structure):
        _fields_ = [f for f in fields if f[0] != "lsum"]

    class Narrow(ctypes.Structure):
        _fields_ = [(nm, ctypes.c_int32 if nm == "nlarge" else t) for nm, t in fields]

    for bad in (Dropped, Narrow):
        msg = L.plan_layout_mismatch(lib, bad)
        assert msg is not None and msg.startswith("vecchia_plan "), msg


def test_mle_parameter_map_stays_in_domain():
    """L-BFGS works on eta = log(sigma2, range, nugget); every eta, however far
    the line search moves it, maps to positive parameters, the map's gradient
    is the chain rule of exp, and a zero starting nugget starts at the floor."""
    import torch
    from paper_2410_04477_amd import mle
    eta = torch.tensor([0.3, -3.0, -80.0], dtype=torch.float64, requires_grad=True)
    th = mle.to_natural(eta)
    assert torch.all(th > 0)
    assert float(th[2]) == pytest.approx(float(torch.exp(torch.tensor(-80.0, dtype=torch.float64))), rel=1e-15)
    (th * torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)).sum().backward()
    np_grad = eta.grad.numpy()
    assert np_grad[0] == pytest.approx(float(th[0]), rel=1e-15)
    assert np_grad[1] == pytest.approx(2.0 * float(th[1]), rel=1e-15)
    assert np_grad[2] == pytest.approx(3.0 * float(th[2]), rel=1e-15)
    e0 = mle.to_eta((1.5, 0.08, 0.0))
    assert e0[2] == pytest.approx(np.log(mle.NUGGET_FLOOR))
    back = mle.to_natural(torch.tensor(mle.to_eta((1.5, 0.08, 0.01)), dtype=torch.float64))
    np.testing.assert_allclose(back.numpy(), [1.5, 0.08, 0.01], rtol=1e-14)
    nu_eta = torch.tensor([0.0, 0.0, 0.0, 40.0], dtype=torch.float64)
    nu = float(mle.to_natural(nu_eta, estimate_nu=True)[3])
    assert mle.NU_LO < nu <= mle.NU_HI
