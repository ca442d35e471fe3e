"""The C-ABI library loads without a GPU and exports every symbol include/*.h declares."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(stk_[a-z_0-9]+)\s*\(", src, re.M))
    return names


def test_header_declares_entry_points():
    d = _declared()
    for need in ("stk_build_tree", "stk_compute_moments", "stk_evaluate", "stk_evaluate_tree", "stk_last_error"):
        assert need in d


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1811_12498_amd", "libstokestree.so"))
    missing = [s for s in sorted(_declared()) if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_match_header():
    from paper_1811_12498_amd import native
    assert set(native.EXPORTS) == _declared()
