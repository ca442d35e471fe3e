"""Build libstokestree.so (HIP, gfx950) in-tree.

Every .hip file under csrc/ is compiled to an object with hipcc (in parallel) and the
objects are linked into paper_1811_12498_amd/libstokestree.so.  Packed FP32 VALU
instructions are disabled (-packed-fp32-ops); the code is written for gfx950 only.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import json
import os
import re
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libstokestree.so")
OBJDIR = os.path.join(ROOT, "_build", "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]


TIMES = os.path.join(ROOT, "_build", "compile_seconds.json")


def _compile(src: str) -> tuple[str, float]:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    t0 = time.perf_counter()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj, time.perf_counter() - t0


def _order_key(path: str, times: dict) -> tuple:
    """Longest compile first (last build's times; else the Taylor order in the name)."""
    name = os.path.basename(path)
    if name in times:
        return (-times[name], name)
    m = re.search(r"_p(\d+)\.hip$", name)
    return (-(1000 + int(m.group(1))) if m else 0.0, name)


def _stale(src: str, newest_header: float) -> bool:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    return os.path.getmtime(obj) < max(os.path.getmtime(src), newest_header)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every .hip under csrc/ and link the library.  incremental=True recompiles
    only sources older than their object or than any header (csrc/*.hpp, include/*.h)."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = glob.glob(os.path.join(CSRC, "*.hip"))
    all_srcs = sorted(srcs)
    if incremental:
        headers = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
        newest = max((os.path.getmtime(h) for h in headers), default=0.0)
        srcs = [sp for sp in srcs if _stale(sp, newest)]
    try:
        with open(TIMES) as fh:
            times = json.load(fh)
    except (OSError, ValueError):
        times = {}
    srcs.sort(key=lambda p: _order_key(p, times))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        res = list(ex.map(_compile, srcs))
    objs = [os.path.join(OBJDIR, os.path.basename(sp) + ".o") for sp in all_srcs]
    times.update({os.path.basename(sp): round(dt, 1) for sp, (_, dt) in zip(srcs, res)})
    with open(TIMES, "w") as fh:
        json.dump(times, fh, indent=0, sort_keys=True)
    tmp = OUT + f".tmp{os.getpid()}"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
