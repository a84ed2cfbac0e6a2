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
                     "neig_set_params", "neig_get_params", "neig_get_stats", "neig_finalize", "neig_version",
                     "neig_set_batched_tune", "neig_get_batched_tune", "neig_reorder", "neig_hessenberg", "neig_policy_set",
                     "neig_mlp_grad", "neig_mlp_infer"]:
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
    with pytest.raises(binding.NeigError):
        binding.set_params(overlap=3)
    with pytest.raises(binding.NeigError):
        binding.set_params(aed_ends=2)
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
    lib.neig_hessenberg.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p]
    assert lib.neig_hessenberg(-1, None, 1, None, 1, None) == -1
    assert lib.neig_hessenberg(4, None, 4, None, 4, None) == -2
    assert lib.neig_hessenberg(4, ctypes.c_void_p(8), 3, None, 4, None) == -3
    assert lib.neig_hessenberg(4, ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 3, None) == -5
    assert lib.neig_hessenberg(0, None, 1, None, 1, None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libneig.so not built")
def test_batched_tune_roundtrip_and_validation():
    from paper_2002_05024_amd import binding

    before = binding.get_batched_tune()
    assert len(before["nw"]) == 6 and before["n_hi"][-1] >= 1 << 30
    binding.set_batched_tune([100, 400, 0], [32, 48, 64], [8, 16, 32], [40, 64, 96], [50, 80, 96])
    t = binding.get_batched_tune()
    assert t["n_hi"][:2] == [100, 400] and t["n_hi"][2] >= 1 << 30
    assert t["nw"] == [32, 48, 64, 64, 64, 64] and t["ns"][5] == 32 and t["chase_w"][0] == 50
    for bad in ([[100, 50, 0], [32] * 3, [8] * 3, [40] * 3, [50] * 3],  # n_hi not increasing
                [[0], [1], [8], [40], [50]],  # nw < 2
                [[0], [32], [7], [40], [50]],  # odd ns
                [[0], [32], [34], [40], [96]],  # ns > 32
                [[0], [32], [32], [97], [96]],  # nmin too large
                [[0], [32], [32], [40], [49]]):  # chase window cannot hold 16 bulges
        with pytest.raises(binding.NeigError):
            binding.set_batched_tune(*bad)
    assert binding.get_batched_tune() == t  # unchanged on error
    k = len(before["nw"])
    binding.set_batched_tune(before["n_hi"], before["nw"], before["ns"], before["nmin"], before["chase_w"])
    assert binding.get_batched_tune() == before and k == 6


@pytest.mark.skipif(not os.path.exists(LIB), reason="libneig.so not built")
def test_batched_argument_errors_without_gpu_work():
    lib = ctypes.CDLL(LIB)
    lib.neig_schur_batched.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 9
    assert lib.neig_schur_batched(-1, *([None] * 9)) == -1
    assert lib.neig_schur_batched(65537, *([None] * 9)) == -1
    assert lib.neig_schur_batched(0, *([None] * 9)) == 0
    assert lib.neig_schur_batched(3, *([None] * 9)) == -2
    lib.neig_schur_batched_noalloc.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 9
    assert lib.neig_schur_batched_noalloc(-1, *([None] * 9)) == -1
    assert lib.neig_schur_batched_noalloc(4097, *([None] * 9)) == -1  # above its fixed capacity
    assert lib.neig_schur_batched_noalloc(0, *([None] * 9)) == 0
    assert lib.neig_schur_batched_noalloc(3, *([None] * 9)) == -2
    lib.neig_batched_flops.argtypes = [ctypes.c_void_p]
    assert lib.neig_batched_flops(None) == -1


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


def header_struct_fields(name):
    """(field, C type) in declaration order of `typedef struct name {...} name;`
    in the header (comments removed; one type per declaration, several names)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        m = re.match(r"(long long|double|int)\s+(.*)", decl)
        assert m, decl
        for f in m.group(2).split(","):
            f = f.strip()
            arr = re.match(r"(\w+)\[(\d+)\]", f)
            fields.append((arr.group(1), m.group(1), int(arr.group(2))) if arr else (f, m.group(1), 1))
    return fields


@pytest.mark.parametrize("cname,pyname", [("neig_params", "Params"), ("neig_stats", "Stats")])
def test_binding_structs_match_the_header(cname, pyname):
    """The binding's ctypes mirrors of the parameter and statistics structs have
    the header's fields, in its order, with its types."""
    from paper_2002_05024_amd import binding

    ctype = {"int": ctypes.c_int, "double": ctypes.c_double, "long long": ctypes.c_longlong}
    want = header_struct_fields(cname)
    got = getattr(binding, pyname)._fields_
    assert [f for f, _ in got] == [f for f, _, _ in want]
    for (f, t), (_, ct, cnt) in zip(got, want):
        assert t == (ctype[ct] * cnt if cnt > 1 else ctype[ct]), f
