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


def test_tiles_file_round_trip(tmp_path):
    """The kernel-variant table's text format: a valid file merges, save writes it back,
    and a malformed or invalid line rejects the whole file (no device needed)."""
    from paper_1811_12498_amd import native
    good = tmp_path / "tiles.txt"
    good.write_text("# arch p K precision far_kb near_kb near_mfma far_mfma far_cm far_split\n"
                    "gfx950 8 16 1 4 4 1 1 0 0\n"
                    "gfx950 6 1 0 1 1 0 0 1 3\n"
                    "gfx950 5 4 1 2 2 0 0 2\n")    # written before far_split existed: automatic
    assert native.tiles_load(str(good)) == 3
    out = tmp_path / "saved.txt"
    native.tiles_save(str(out))
    lines = {ln for ln in out.read_text().splitlines() if not ln.startswith("#")}
    assert {"gfx950 8 16 1 4 4 1 1 0 0", "gfx950 6 1 0 1 1 0 0 1 3", "gfx950 5 4 1 2 2 0 0 2 0"} <= lines
    for bad in ("gfx950 8 16 1 4 4 1 1\n",      # too few fields
                "gfx950 8 16 0 4 1 0 0 0\n",    # FP64 with 4 right-hand sides per pass
                "gfx950 8 16 0 1 1 0 1 0\n",    # FP64 on the matrix cores
                "gfx950 8 6 1 4 1 0 0 0\n",     # 4 does not divide K = 6
                "gfx950 8 16 1 1 1 0 1 1\n",    # matrix-core far field with the cluster-major split
                "gfx950 8 16 1 1 1 0 0 3\n",    # unknown far_cm mode
                "gfx950 8 1 1 1 1 0 0 0 5\n",   # more than four far-list parts
                "gfx950 8 1 1 1 1 0 0 0 -1\n",  # negative far-list parts
                "gfx950 8 16 1 1 1 0 1 0 2\n",  # matrix-core far field with split lists
                "gfx950 8 16 7 1 1 0 0 0\n"):   # unknown precision
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        try:
            native.tiles_load(str(f))
        except native.StkError as e:
            assert e.status == -1
        else:
            raise AssertionError(f"accepted {bad!r}")
