"""FP64 CPU oracle for the Stokeslet/stresslet treecode -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``stokes_oracle.c`` (plain C, ``-O2 -ffp-contract=off``).
It follows Wang, Tlupova & Krasny (arXiv 1811.12498): the direct sum of eq. StoStre
in the contracted form of Sec. 4.1, the octree of Sec. 5, the cluster moments of
Sec. 2, the Coulomb recurrence (recurrence_1), the contracted far field (S_final,
T_final) and Algorithm 1.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP over targets)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_nm.restype = ctypes.c_int
        L.orc_tree_build.restype = ctypes.c_void_p
        L.orc_tree_build.argtypes = [_dp, ctypes.c_int64, ctypes.c_int32]
        L.orc_tree_nnodes.restype = ctypes.c_int64
        L.orc_tree_nnodes.argtypes = [ctypes.c_void_p]
        L.orc_tree_free.argtypes = [ctypes.c_void_p]
        L.orc_tree_export.argtypes = [ctypes.c_void_p, _i64p, _i32p, _i32p, _i32p, _i32p, _i64p, _i64p,
                                      _dp, _dp, _dp, _dp, _dp]
        L.orc_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp]
        L.orc_treecode.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int,
                                   ctypes.c_double, _dp, ctypes.c_int64, _dp, _i64p, _i64p, _i64p,
                                   ctypes.c_int]
        L.orc_direct.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp, _dp]
        L.orc_direct_tensor.argtypes = L.orc_direct.argtypes
        L.orc_coulomb_taylor.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_stokeslet_coeffs.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_stresslet_coeffs.argtypes = [_dp, ctypes.c_int, _dp]
        L.orc_far_contracted.argtypes = [_dp, ctypes.c_int, _dp, _dp, _dp]
        L.orc_far_explicit.argtypes = [_dp, ctypes.c_int, _dp, _dp, _dp]
        L.orc_kindex.argtypes = [ctypes.c_int, _i32p]
        L.orc_lists.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, ctypes.c_int64, _i64p, _i32p,
                                _i64p, _i32p]
        L.orc_frozen_apply.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_int, _dp,
                                       ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _dp]
        L.orc_frozen_adjoint.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, ctypes.c_int, _dp,
                                         ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _dp, _dp, _dp,
                                         _dp, _dp]
        L.orc_direct_grad.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp, _dp,
                                      _dp, _dp, _dp, _dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_reg_taylor.argtypes = [_dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp]
        L.orc_reg_coeffs.argtypes = [_dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.orc_reg_far.argtypes = [_dp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
        L.orc_reg_direct.argtypes = [_dp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_reg_direct_tensor.argtypes = L.orc_reg_direct.argtypes
        L.orc_reg_treecode.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, _dp, ctypes.c_int64, _dp, _i64p, _i64p, _i64p]
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads for the oracle's OpenMP loops (per-target results do not depend on it)."""
    lib().orc_set_num_threads(int(k))


def nm(p: int) -> int:
    """Number of multi-indices with ||k|| <= p."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def kindex(p: int) -> np.ndarray:
    """Graded-lex multi-index table (flattened moment order)."""
    k = np.zeros((nm(p), 3), dtype=np.int32)
    lib().orc_kindex(p, k.ctypes.data_as(_i32p))
    return k


def coulomb_taylor(d, P: int) -> np.ndarray:
    """Dense array b[k1,k2,k3] = (1/k!) D_y^k 1/|x-y| at d = x - y, ||k|| <= P (recurrence_1)."""
    d = _c(d)
    b = np.zeros((P + 1, P + 1, P + 1))
    lib().orc_coulomb_taylor(_d(d), P, _d(b))
    return b


def stokeslet_coeffs(d, p: int) -> np.ndarray:
    """a^k_ij (recurrence_2), shape (nm, 3, 3)."""
    d = _c(d)
    a = np.zeros((nm(p), 3, 3))
    lib().orc_stokeslet_coeffs(_d(d), p, _d(a))
    return a


def stresslet_coeffs(d, p: int) -> np.ndarray:
    """at^k_ijl (recurrence_3), shape (nm, 3, 3, 3)."""
    d = _c(d)
    a = np.zeros((nm(p), 3, 3, 3))
    lib().orc_stresslet_coeffs(_d(d), p, _d(a))
    return a


def far_contracted(d, p, M, Mt) -> np.ndarray:
    """Contracted particle-cluster far field (S_final + T_final) for one cluster."""
    d, M, Mt = _c(d), _c(M), _c(Mt)
    u = np.zeros(3)
    lib().orc_far_contracted(_d(d), p, _d(M), _d(Mt), _d(u))
    return u


def far_explicit(d, p, M, Mt) -> np.ndarray:
    """Far field from explicit coefficients (eq. pc_interaction)."""
    d, M, Mt = _c(d), _c(M), _c(Mt)
    u = np.zeros(3)
    lib().orc_far_explicit(_d(d), p, _d(M), _d(Mt), _d(u))
    return u


def direct(tgt, src, f, h, nu, tensor: bool = False) -> np.ndarray:
    """Direct sum of eq. StoStre (contracted form of Sec. 4.1, or explicit tensors)."""
    tgt, src, f, h, nu = (_c(a) for a in (tgt, src, f, h, nu))
    u = np.zeros_like(tgt)
    fn = lib().orc_direct_tensor if tensor else lib().orc_direct
    fn(_d(tgt), tgt.shape[0], _d(src), src.shape[0], _d(f), _d(h), _d(nu), _d(u))
    return u


def direct_grad(tgt, src, f, h, nu, w):
    """Analytic gradient of sum(w * u_direct) w.r.t. f, h, sources, targets."""
    tgt, src, f, h, nu, w = (_c(a) for a in (tgt, src, f, h, nu, w))
    gf, gh, gs = (np.zeros_like(src) for _ in range(3))
    gt = np.zeros_like(tgt)
    lib().orc_direct_grad(_d(tgt), tgt.shape[0], _d(src), src.shape[0], _d(f), _d(h), _d(nu), _d(w),
                          _d(gf), _d(gh), _d(gs), _d(gt))
    return gf, gh, gs, gt


@dataclass
class Tree:
    """Node table of the oracle octree (breadth-first, children in Morton order)."""
    handle: int
    n: int
    perm: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    child0: np.ndarray
    nchild: np.ndarray
    start: np.ndarray
    count: np.ndarray
    bmin: np.ndarray
    bmax: np.ndarray
    center: np.ndarray
    radius: np.ndarray
    root: np.ndarray

    @property
    def nnodes(self) -> int:
        return int(self.level.shape[0])

    def __del__(self):
        try:
            if self.handle:
                lib().orc_tree_free(ctypes.c_void_p(self.handle))
                self.handle = 0
        except Exception:
            pass


def build_tree(src, n0: int) -> Tree:
    src = _c(src)
    n = src.shape[0]
    h = lib().orc_tree_build(_d(src), n, n0)
    nn = lib().orc_tree_nnodes(ctypes.c_void_p(h))
    perm = np.zeros(n, np.int64)
    level, parent, child0, nchild = (np.zeros(nn, np.int32) for _ in range(4))
    start, count = np.zeros(nn, np.int64), np.zeros(nn, np.int64)
    bmin, bmax, center = (np.zeros((nn, 3)) for _ in range(3))
    radius = np.zeros(nn)
    root = np.zeros(4)
    lib().orc_tree_export(ctypes.c_void_p(h), perm.ctypes.data_as(_i64p), level.ctypes.data_as(_i32p),
                          parent.ctypes.data_as(_i32p), child0.ctypes.data_as(_i32p),
                          nchild.ctypes.data_as(_i32p), start.ctypes.data_as(_i64p),
                          count.ctypes.data_as(_i64p), _d(bmin), _d(bmax), _d(center), _d(radius),
                          _d(root))
    return Tree(h, n, perm, level, parent, child0, nchild, start, count, bmin, bmax, center, radius, root)


def moments(tree: Tree, src, f, h, nu, p: int):
    """Cluster moments M (nnodes, nm, 3) and Mt (nnodes, nm, 3, 3) of Sec. 2."""
    src, f, h, nu = (_c(a) for a in (src, f, h, nu))
    M = np.zeros((tree.nnodes, nm(p), 3))
    Mt = np.zeros((tree.nnodes, nm(p), 3, 3))
    lib().orc_moments(ctypes.c_void_p(tree.handle), _d(src), _d(f), _d(h), _d(nu), p, _d(M), _d(Mt))
    return M, Mt


@dataclass
class TreecodeResult:
    u: np.ndarray
    nfar: np.ndarray
    nnear: np.ndarray
    npairs: np.ndarray


def treecode(tree: Tree, src, f, h, nu, M, Mt, p: int, theta: float, tgt,
             explicit_far: bool = False) -> TreecodeResult:
    """Algorithm 1 at the given targets; also the per-target interaction counts."""
    src, f, h, nu, M, Mt, tgt = (_c(a) for a in (src, f, h, nu, M, Mt, tgt))
    m = tgt.shape[0]
    u = np.zeros((m, 3))
    nfar, nnear, npairs = (np.zeros(m, np.int64) for _ in range(3))
    lib().orc_treecode(ctypes.c_void_p(tree.handle), _d(src), _d(f), _d(h), _d(nu), _d(M), _d(Mt), p,
                       float(theta), _d(tgt), m, _d(u), nfar.ctypes.data_as(_i64p),
                       nnear.ctypes.data_as(_i64p), npairs.ctypes.data_as(_i64p), int(explicit_far))
    return TreecodeResult(u, nfar, nnear, npairs)


@dataclass
class Lists:
    far_ptr: np.ndarray
    far_nodes: np.ndarray
    near_ptr: np.ndarray
    near_nodes: np.ndarray


def lists(tree: Tree, theta: float, tgt) -> Lists:
    """Per-target far-node and near-leaf lists of Algorithm 1 (the frozen plan)."""
    tgt = _c(tgt)
    m = tgt.shape[0]
    fp, np_ = np.zeros(m + 1, np.int64), np.zeros(m + 1, np.int64)
    lib().orc_lists(ctypes.c_void_p(tree.handle), float(theta), _d(tgt), m, fp.ctypes.data_as(_i64p),
                    None, np_.ctypes.data_as(_i64p), None)
    fn = np.zeros(max(int(fp[-1]), 1), np.int32)
    nn = np.zeros(max(int(np_[-1]), 1), np.int32)
    lib().orc_lists(ctypes.c_void_p(tree.handle), float(theta), _d(tgt), m, fp.ctypes.data_as(_i64p),
                    fn.ctypes.data_as(_i32p), np_.ctypes.data_as(_i64p), nn.ctypes.data_as(_i32p))
    return Lists(fp, fn, np_, nn)


def frozen_apply(tree: Tree, L: Lists, src, f, h, nu, p: int, tgt) -> np.ndarray:
    """Frozen-plan operator: lists, membership and centres fixed; moments and kernels re-evaluated."""
    src, f, h, nu, tgt = (_c(a) for a in (src, f, h, nu, tgt))
    u = np.zeros_like(tgt)
    lib().orc_frozen_apply(ctypes.c_void_p(tree.handle), _d(src), _d(f), _d(h), _d(nu), p, _d(tgt),
                           tgt.shape[0], L.far_ptr.ctypes.data_as(_i64p), L.far_nodes.ctypes.data_as(_i32p),
                           L.near_ptr.ctypes.data_as(_i64p), L.near_nodes.ctypes.data_as(_i32p), _d(u))
    return u


def frozen_adjoint(tree: Tree, L: Lists, src, f, h, nu, p: int, tgt, w):
    """Transpose of the frozen-plan operator: gradients of sum(w * u) w.r.t. f, h, sources, targets."""
    src, f, h, nu, tgt, w = (_c(a) for a in (src, f, h, nu, tgt, w))
    gf, gh, gs = (np.zeros_like(src) for _ in range(3))
    gt = np.zeros_like(tgt)
    lib().orc_frozen_adjoint(ctypes.c_void_p(tree.handle), _d(src), _d(f), _d(h), _d(nu), p, _d(tgt),
                             tgt.shape[0], L.far_ptr.ctypes.data_as(_i64p), L.far_nodes.ctypes.data_as(_i32p),
                             L.near_ptr.ctypes.data_as(_i64p), L.near_nodes.ctypes.data_as(_i32p), _d(w),
                             _d(gf), _d(gh), _d(gs), _d(gt))
    return gf, gh, gs, gt


# ---- regularized Stokeslets and stresslets (the extension named in Sec. 7) ----

def reg_taylor(d, eps: float, nu2: int, P: int) -> np.ndarray:
    """Coefficients (1/k!) D_y^k of (|d|^2 + eps^2)^(-nu2/2), dense (P+1)^3 like coulomb_taylor."""
    d = _c(d)
    a = np.zeros((P + 1) ** 3)
    lib().orc_reg_taylor(_d(d), float(eps), int(nu2), int(P), _d(a))
    return a.reshape(P + 1, P + 1, P + 1)


def reg_coeffs(d, eps: float, p: int):
    """a^k_ij (nm,3,3) and at^k_ijl (nm,3,3,3) of the regularized kernels at d."""
    d = _c(d)
    a = np.zeros((nm(p), 3, 3))
    at = np.zeros((nm(p), 3, 3, 3))
    lib().orc_reg_coeffs(_d(d), float(eps), int(p), _d(a), _d(at))
    return a, at


def reg_far(d, eps: float, p: int, M, Mt) -> np.ndarray:
    d, M, Mt = _c(d), _c(M), _c(Mt)
    u = np.zeros(3)
    lib().orc_reg_far(_d(d), float(eps), int(p), _d(M), _d(Mt), _d(u))
    return u


def reg_direct(tgt, src, f, h, nu, eps: float, tensor: bool = False) -> np.ndarray:
    """Regularized direct sum (contracted, or with S^eps and T^eps formed as tensors)."""
    tgt, src, f, h, nu = (_c(a) for a in (tgt, src, f, h, nu))
    u = np.zeros_like(tgt)
    fn = lib().orc_reg_direct_tensor if tensor else lib().orc_reg_direct
    fn(_d(tgt), tgt.shape[0], _d(src), src.shape[0], _d(f), _d(h), _d(nu), float(eps), _d(u))
    return u


def reg_treecode(tree: Tree, src, f, h, nu, M, Mt, p: int, theta: float, eps: float, tgt) -> TreecodeResult:
    """Algorithm 1 with the regularized kernels (same tree, moments and MAC)."""
    src, f, h, nu, M, Mt, tgt = (_c(a) for a in (src, f, h, nu, M, Mt, tgt))
    m = tgt.shape[0]
    u = np.zeros((m, 3))
    nfar, nnear, npairs = (np.zeros(m, np.int64) for _ in range(3))
    lib().orc_reg_treecode(ctypes.c_void_p(tree.handle), _d(src), _d(f), _d(h), _d(nu), _d(M), _d(Mt), p,
                           float(theta), float(eps), _d(tgt), m, _d(u), nfar.ctypes.data_as(_i64p),
                           nnear.ctypes.data_as(_i64p), npairs.ctypes.data_as(_i64p))
    return TreecodeResult(u, nfar, nnear, npairs)


def rel_l2(a, b) -> float:
    """Relative L2 error of eq. L2Err: ||a - b|| / ||b|| over all components."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum((a - b) ** 2)))
