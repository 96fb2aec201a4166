"""The C-ABI library loads on a machine without a GPU and exports every entry
point include/rbfib.h declares (no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rbfib.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rbfib_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_all_declared_symbols():
    path = os.path.join(ROOT, "paper_1901_06427_amd", "librbfib.so")
    assert os.path.exists(path), "build the library first: python paper_1901_06427_amd/build.py"
    lib = ctypes.CDLL(path)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    import paper_1901_06427_amd as rb
    assert sorted(rb.EXPORTS) == _declared()
    o = rb.rbfib_default_opts()
    assert o.tol == 1e-6 and o.restart == 100 and o.use_graphs == 1
    # the last fields land where the C struct has them
    assert o.mg_cheby == 0.27 and o.krylov_s == 2 and o.mg_first2 == 1
    assert rb._lib.rbfib_strerror(-2).decode().startswith("unphysical")
