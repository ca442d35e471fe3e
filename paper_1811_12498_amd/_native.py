"""ctypes binding of libstokestree (include/stokestree.h).

Argument marshalling only: torch tensors supply device memory and the current HIP
stream; every step of the computation runs in the library's kernels.  There is no
fallback: if the built library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokestree.so")

STK_OK, STK_EINVAL, STK_ENOMEM, STK_EDEVICE, STK_ESTATE = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
P_MAX = 10

_STATUS_NAMES = {STK_EINVAL: "STK_EINVAL", STK_ENOMEM: "STK_ENOMEM", STK_EDEVICE: "STK_EDEVICE",
                 STK_ESTATE: "STK_ESTATE"}

# every symbol include/stokestree.h declares
EXPORTS = ["stk_build_tree", "stk_compute_moments", "stk_evaluate_tree", "stk_evaluate", "stk_evaluate_adjoint",
           "stk_direct", "stk_direct_noalloc", "stk_evaluate_regularized",
           "stk_tree_info", "stk_tree_export", "stk_tree_export_moments", "stk_plan_counts", "stk_plan_info",
           "stk_plan_export_lists", "stk_plan_far_split", "stk_tiles_set", "stk_tiles_get", "stk_autotune", "stk_tiles_save",
           "stk_tiles_load", "stk_plan_tiles",
           "stk_profile_enable", "stk_profile_read", "stk_tree_destroy", "stk_plan_destroy",
           "stk_plan_cache_clear", "stk_last_error"]

PHASES = ["tree", "moments", "targets", "lists", "near", "far", "direct", "adjoint", "far_sparse", "finish"]


class StkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1811_12498_amd.build` "
                      "(there is no fallback implementation)")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_i32p, _i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
_i64, _i32, _d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double

_lib.stk_last_error.restype = ctypes.c_char_p
_lib.stk_build_tree.argtypes = [_vp, _i64, _i32, _vp, ctypes.POINTER(_vp)]
_lib.stk_compute_moments.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, ctypes.c_int, _vp]
_lib.stk_evaluate_tree.argtypes = [_vp, _vp, _i64, _d, _vp, ctypes.POINTER(_vp), _vp]
_lib.stk_evaluate.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _i32, _d, _i32, ctypes.c_int, _vp,
                              ctypes.POINTER(_vp), _vp]
_lib.stk_direct.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _vp]
_lib.stk_direct_noalloc.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _vp]
_lib.stk_evaluate_regularized.argtypes = [_vp, _i64, _vp, _i64, _vp, _vp, _vp, ctypes.c_double, _i32,
                                          ctypes.c_double, _i32, _vp, _vp]
_lib.stk_evaluate_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.stk_tree_info.argtypes = [_vp, _i64p, _i32p, _dp]
_lib.stk_tree_export.argtypes = [_vp] + [_vp] * 11
_lib.stk_tree_export_moments.argtypes = [_vp, _i32, _vp, _vp]
_lib.stk_plan_export_lists.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp]
_lib.stk_plan_far_split.argtypes = [_vp, _i32p, _i64p]


class Tiles(ctypes.Structure):
    """stk_tiles: kernel variants of the far and near fields."""
    _fields_ = [("far_kb", ctypes.c_int32), ("near_kb", ctypes.c_int32), ("near_mfma", ctypes.c_int32),
                ("far_mfma", ctypes.c_int32), ("far_cm", ctypes.c_int32), ("far_split", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"far_kb": self.far_kb, "near_kb": self.near_kb, "near_mfma": bool(self.near_mfma),
                "far_mfma": bool(self.far_mfma), "far_cm": int(self.far_cm), "far_split": int(self.far_split)}


_lib.stk_tiles_set.argtypes = [_i32, _i32, ctypes.c_int, ctypes.POINTER(Tiles)]
_lib.stk_tiles_get.argtypes = [_i32, _i32, ctypes.c_int, ctypes.POINTER(Tiles), _i32p]
_lib.stk_autotune.argtypes = [_i32, _i32, ctypes.c_int, _i64, _d, _i32, ctypes.POINTER(Tiles), _dp, _vp]
_lib.stk_tiles_save.argtypes = [ctypes.c_char_p]
_lib.stk_tiles_load.argtypes = [ctypes.c_char_p, _i32p]
_lib.stk_plan_tiles.argtypes = [_vp, ctypes.POINTER(Tiles)]
_lib.stk_plan_counts.argtypes = [_vp, _vp, _vp, _vp]
_lib.stk_plan_info.argtypes = [_vp, _i64p, _i64p, _i64p]
_lib.stk_profile_enable.argtypes = [ctypes.c_int]
_lib.stk_profile_read.argtypes = [_vp, _vp]
_lib.stk_tree_destroy.argtypes = [_vp]
_lib.stk_plan_destroy.argtypes = [_vp]
for _name in EXPORTS:
    _lib[_name].restype = ctypes.c_int if _name != "stk_last_error" else ctypes.c_char_p
_lib.stk_tree_destroy.restype = None
_lib.stk_plan_destroy.restype = None
_lib.stk_plan_cache_clear.restype = None


def _check(st: int) -> None:
    if st != STK_OK:
        raise StkError(st, _lib.stk_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, shape_last: int | None = 3) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and t.shape[-1] != shape_last:
        raise ValueError(f"{name} must have last dimension {shape_last}")
    return t


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _prec(precision) -> int:
    if precision in (FP64, "fp64", "float64"):
        return FP64
    if precision in (MIXED, "mixed", "fp32", "float32"):
        return MIXED
    raise ValueError(f"unknown precision {precision!r}")


class Tree:
    """Owning wrapper of an stk_tree handle."""

    def __init__(self, handle: int, n: int):
        self.handle = ctypes.c_void_p(handle)
        self.n = n

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.stk_tree_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)


class Plan:
    """Owning wrapper of an stk_plan handle (keeps its tree alive)."""

    def __init__(self, handle: int, m: int, tree: Tree | None):
        self.handle = ctypes.c_void_p(handle)
        self.m = m
        self.tree = tree

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.stk_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)


def build_tree(sources: torch.Tensor, n0: int) -> Tree:
    _dev(sources, "sources")
    h = ctypes.c_void_p()
    _check(_lib.stk_build_tree(_ptr(sources), sources.shape[0], int(n0), _stream(), ctypes.byref(h)))
    return Tree(h.value, sources.shape[0])


def compute_moments(tree: Tree, f: torch.Tensor, h: torch.Tensor, nu: torch.Tensor, p: int,
                    precision="fp64") -> None:
    for t, nm in ((f, "f"), (h, "h"), (nu, "nu")):
        _dev(t, nm)
    k = f.shape[0] if f.dim() == 3 else 1
    _check(_lib.stk_compute_moments(tree.handle, _ptr(f), _ptr(h), _ptr(nu), k, int(p), _prec(precision),
                                    _stream()))
    tree.k_rhs = k


def evaluate_tree(tree: Tree, targets: torch.Tensor, theta: float, keep_plan: bool = False,
                  out: torch.Tensor | None = None):
    _dev(targets, "targets")
    m = targets.shape[0]
    k = getattr(tree, "k_rhs", 1)
    shape = (m, 3) if k == 1 else (k, m, 3)
    u = out if out is not None else torch.empty(shape, dtype=torch.float64, device=targets.device)
    _dev(u, "out")
    if u.numel() != k * m * 3:
        raise ValueError(f"out must hold {k} x {m} x 3 values")
    ph = ctypes.c_void_p()
    _check(_lib.stk_evaluate_tree(tree.handle, _ptr(targets), m, float(theta), _ptr(u),
                                  ctypes.byref(ph) if keep_plan else None, _stream()))
    return (u, Plan(ph.value, m, tree)) if keep_plan else u


def evaluate(targets, sources, f, h, nu, p: int, theta: float, n0: int, precision="fp64",
             keep_plan: bool = False):
    for t, nm in ((targets, "targets"), (sources, "sources"), (f, "f"), (h, "h"), (nu, "nu")):
        _dev(t, nm)
    m, n = targets.shape[0], sources.shape[0]
    k = f.shape[0] if f.dim() == 3 else 1
    u = torch.empty((m, 3) if k == 1 else (k, m, 3), dtype=torch.float64, device=targets.device)
    ph = ctypes.c_void_p()
    _check(_lib.stk_evaluate(_ptr(targets), m, _ptr(sources), n, _ptr(f), _ptr(h), _ptr(nu), k, int(p),
                             float(theta), int(n0), _prec(precision), _ptr(u),
                             ctypes.byref(ph) if keep_plan else None, _stream()))
    return (u, Plan(ph.value, m, None)) if keep_plan else u


def evaluate_adjoint(plan: Plan, w: torch.Tensor, n_sources: int, want=("f", "h", "targets", "sources")):
    """Gradients of sum(w * u) for the plan's frozen operator: dict of tensors for the
    requested keys among "f", "h", "targets", "sources"."""
    _dev(w, "w")
    if w.shape[0] != plan.m:
        raise ValueError("w must have one row per target")
    dev = w.device
    out = {}
    for k in want:
        rows = plan.m if k == "targets" else n_sources
        out[k] = torch.empty((rows, 3), dtype=torch.float64, device=dev)
    ptr = lambda k: _ptr(out[k]) if k in out else None
    _check(_lib.stk_evaluate_adjoint(plan.handle, _ptr(w), ptr("f"), ptr("h"), ptr("targets"), ptr("sources"),
                                     _stream()))
    return out


def direct(targets, sources, f, h, nu) -> torch.Tensor:
    for t, nm in ((targets, "targets"), (sources, "sources"), (f, "f"), (h, "h"), (nu, "nu")):
        _dev(t, nm)
    m, n = targets.shape[0], sources.shape[0]
    k = f.shape[0] if f.dim() == 3 else 1
    u = torch.empty((m, 3) if k == 1 else (k, m, 3), dtype=torch.float64, device=targets.device)
    _check(_lib.stk_direct(_ptr(targets), m, _ptr(sources), n, _ptr(f), _ptr(h), _ptr(nu), k, _ptr(u),
                           _stream()))
    return u


def evaluate_regularized(targets, sources, f, h, nu, eps: float, p: int, theta: float, n0: int) -> torch.Tensor:
    """stk_evaluate_regularized: the treecode with regularized Stokeslets and stresslets
    (FP64, one right-hand side); u of shape (m, 3)."""
    for t, nm in ((targets, "targets"), (sources, "sources"), (f, "f"), (h, "h"), (nu, "nu")):
        _dev(t, nm)
    m, n = targets.shape[0], sources.shape[0]
    u = torch.empty((m, 3), dtype=torch.float64, device=targets.device)
    _check(_lib.stk_evaluate_regularized(_ptr(targets), m, _ptr(sources), n, _ptr(f), _ptr(h), _ptr(nu), float(eps),
                                         int(p), float(theta), int(n0), _ptr(u), _stream()))
    return u


def direct_noalloc(targets, sources, f, h, nu, out=None) -> torch.Tensor:
    """stk_direct_noalloc: the direct sum with the library's fixed scratch array (the
    library allocates nothing; `out`, if given, receives the result)."""
    for t, nm in ((targets, "targets"), (sources, "sources"), (f, "f"), (h, "h"), (nu, "nu")):
        _dev(t, nm)
    m, n = targets.shape[0], sources.shape[0]
    k = f.shape[0] if f.dim() == 3 else 1
    shape = (m, 3) if k == 1 else (k, m, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=targets.device)
    elif tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float64 tensor of shape {shape}")
    _check(_lib.stk_direct_noalloc(_ptr(targets), m, _ptr(sources), n, _ptr(f), _ptr(h), _ptr(nu), k, _ptr(out),
                                   _stream()))
    return out


def tree_info(tree: Tree):
    nn, nl = ctypes.c_int64(), ctypes.c_int32()
    root = (ctypes.c_double * 4)()
    _check(_lib.stk_tree_info(tree.handle, ctypes.byref(nn), ctypes.byref(nl), root))
    return int(nn.value), int(nl.value), np.array(root[:])


def tree_export(tree: Tree) -> dict:
    nn, _, _ = tree_info(tree)
    out = {"perm": np.zeros(tree.n, np.int32)}
    for k in ("level", "parent", "child0", "nchild", "start", "count"):
        out[k] = np.zeros(nn, np.int32)
    for k in ("bmin", "bmax", "center"):
        out[k] = np.zeros((nn, 3))
    out["radius"] = np.zeros(nn)
    order = ["perm", "level", "parent", "child0", "nchild", "start", "count", "bmin", "bmax", "center", "radius"]
    _check(_lib.stk_tree_export(tree.handle, *[ctypes.c_void_p(out[k].ctypes.data) for k in order]))
    return out


def tree_moments(tree: Tree, p: int, rhs: int = 0):
    nn, _, _ = tree_info(tree)
    nm = (p + 1) * (p + 2) * (p + 3) // 6
    M = np.zeros((nn, nm, 3))
    Mt = np.zeros((nn, nm, 3, 3))
    _check(_lib.stk_tree_export_moments(tree.handle, int(rhs), ctypes.c_void_p(M.ctypes.data),
                                        ctypes.c_void_p(Mt.ctypes.data)))
    return M, Mt


def plan_counts(plan: Plan):
    a, b, c = (np.zeros(plan.m, np.int64) for _ in range(3))
    _check(_lib.stk_plan_counts(plan.handle, ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(b.ctypes.data),
                                ctypes.c_void_p(c.ctypes.data)))
    return a, b, c


def plan_info(plan: Plan) -> dict:
    g, fe, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.stk_plan_info(plan.handle, ctypes.byref(g), ctypes.byref(fe), ctypes.byref(ne)))
    return {"groups": g.value, "far_entries": fe.value, "near_entries": ne.value}


def plan_lists(plan: Plan, kind: str) -> dict:
    """A plan's group lists ("far" or "near"): off (ngroups+1), node, mask (uint64 lane
    masks) and tperm (sorted target -> caller index), as host arrays."""
    info = plan_info(plan)
    k = {"far": 0, "near": 1}[kind]
    ne = info["far_entries" if k == 0 else "near_entries"]
    out = {"off": np.zeros(info["groups"] + 1, np.int32), "node": np.zeros(max(ne, 1), np.int32),
           "mask": np.zeros(max(ne, 1), np.uint64), "tperm": np.zeros(max(plan.m, 1), np.int32)}
    _check(_lib.stk_plan_export_lists(plan.handle, k, *[ctypes.c_void_p(out[n].ctypes.data)
                                                        for n in ("off", "node", "mask", "tperm")]))
    out["node"], out["mask"], out["tperm"] = out["node"][:ne], out["mask"][:ne], out["tperm"][:plan.m]
    return out


def tiles_set(p: int, k_rhs: int, precision: str, far_kb: int = 1, near_kb: int = 1, near_mfma: bool = False,
              far_mfma: bool = False, clear: bool = False, far_cm: int = 0, far_split: int = 0) -> None:
    """far_cm: 0 automatic, 1 every far entry cluster major, 2 only the sparse split.
    far_split: parts of each group's far list (1..4), 0 automatic."""
    t = Tiles(far_kb, near_kb, int(near_mfma), int(far_mfma), int(far_cm), int(far_split))
    _check(_lib.stk_tiles_set(int(p), int(k_rhs), _prec(precision), None if clear else ctypes.byref(t)))


def tiles_get(p: int, k_rhs: int, precision: str) -> tuple[dict, bool]:
    t, hit = Tiles(), ctypes.c_int32()
    _check(_lib.stk_tiles_get(int(p), int(k_rhs), _prec(precision), ctypes.byref(t), ctypes.byref(hit)))
    return t.as_dict(), bool(hit.value)


def autotune(p: int, k_rhs: int, precision: str, n: int, theta: float, n0: int) -> tuple[dict, float]:
    t, ms = Tiles(), ctypes.c_double()
    _check(_lib.stk_autotune(int(p), int(k_rhs), _prec(precision), int(n), float(theta), int(n0), ctypes.byref(t),
                             ctypes.byref(ms), _stream()))
    return t.as_dict(), ms.value


def tiles_save(path: str) -> None:
    _check(_lib.stk_tiles_save(str(path).encode()))


def tiles_load(path: str) -> int:
    k = ctypes.c_int32()
    _check(_lib.stk_tiles_load(str(path).encode(), ctypes.byref(k)))
    return k.value


def plan_tiles(plan: Plan) -> dict:
    t = Tiles()
    _check(_lib.stk_plan_tiles(plan.handle, ctypes.byref(t)))
    return t.as_dict()


def plan_far_split(plan: Plan) -> tuple[int, int]:
    """(max_pc, sparse_interactions): far entries with at most max_pc targets ran cluster major."""
    mp, ns = ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.stk_plan_far_split(plan.handle, ctypes.byref(mp), ctypes.byref(ns)))
    return mp.value, ns.value


def plan_cache_clear() -> None:
    """Free the device memory of the plans parked for reuse by evaluate(keep_plan=True)."""
    _lib.stk_plan_cache_clear()


def profile_enable(on: bool = True) -> None:
    _check(_lib.stk_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{phase: (total ms, number of timed intervals)} since the last read; clears the record."""
    ms = np.zeros(len(PHASES))
    cnt = np.zeros(len(PHASES), np.int64)
    _check(_lib.stk_profile_read(ctypes.c_void_p(ms.ctypes.data), ctypes.c_void_p(cnt.ctypes.data)))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PHASES)}


def exported_symbols() -> list[str]:
    """Names from include/stokestree.h that the loaded library exports."""
    return [s for s in EXPORTS if hasattr(_lib, s)]
