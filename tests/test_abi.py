"""The C-ABI library loads and exports every symbol include/neig.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "neig.h")
LIB = os.path.join(ROOT, "paper_2002_05024_amd", "libneig.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(neig_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["neig_schur", "neig_schur_batched", "neig_sweep", "neig_aed", "neig_small_schur",
                     "neig_set_params", "neig_get_params", "neig_get_stats", "neig_finalize", "neig_version"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libneig.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libneig.so not built")
def test_params_roundtrip_and_validation():
    from paper_2002_05024_amd import binding

    before = binding.get_params()
    binding.set_params(ns=32, nw=48, deflation=1)
    p = binding.get_params()
    assert p["ns"] == 32 and p["nw"] == 48 and p["deflation"] == 1
    with pytest.raises(binding.NeigError):
        binding.set_params(ns=3)  # odd shift count
    with pytest.raises(binding.NeigError):
        binding.set_params(deflation=5)
    binding.set_params(**before)
    assert binding.get_params() == before


@pytest.mark.skipif(not os.path.exists(LIB), reason="libneig.so not built")
def test_argument_errors_without_gpu_work():
    lib = ctypes.CDLL(LIB)
    lib.neig_schur.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    # n < 0, null H, small ld: rejected before any HIP call
    assert lib.neig_schur(-1, None, 1, None, 1, None, None, None) == -1
    assert lib.neig_schur(4, None, 4, None, 4, None, None, None) == -2
    assert lib.neig_schur(4, ctypes.c_void_p(8), 3, ctypes.c_void_p(8), 4, None, None, None) == -3
    assert lib.neig_schur(4, ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 2, None, None, None) == -5
    assert lib.neig_schur(0, None, 1, None, 1, None, None, None) == 0


def test_product_path_has_no_cpu_fallback():
    """The binding refuses CPU tensors instead of computing anything itself."""
    torch = pytest.importorskip("torch")
    from paper_2002_05024_amd import binding

    if not os.path.exists(LIB):
        with pytest.raises(binding.NeigError):
            binding.load_library()
        return
    H = torch.zeros((4, 4), dtype=torch.float64).t()
    with pytest.raises(binding.NeigError):
        binding.schur(H)
