"""Parity of the HIP library (through its C-ABI) with the FP64 oracle.

Integer work (tree topology, sorted order, interaction counts) must match bit for
bit; geometry (boxes, centres, radii) is exact FP64 and must match bit for bit;
moments within 1e-13; the FP64 treecode within 1e-12 relative L2 of the oracle
treecode; the mixed path within the error its FP32 arithmetic allows (1e-5 of the
FP64 treecode, a bound a factor ~20 above what FP32 rounding of each far and near
term accumulates over ~1e4 terms).
"""
import numpy as np
import pytest

from paper_1811_12498_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_12498_amd import native
    return native


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(kind, n, seed, n0):
    if kind == "cube":
        return W.cube(n, seed=seed, n0=n0)
    if kind == "cube_pm1":
        return W.cube(n, seed=seed, lo=-1.0, hi=1.0, n0=n0)
    if kind == "sphere":
        return W.sphere(n, seed=seed, n0=n0)
    if kind == "dups":  # many coincident points
        w = W.cube(n, seed=seed, n0=n0)
        w.src[n // 2:] = w.src[: n - n // 2]
        return w
    if kind == "chain":  # all but ten points coincident: single-child nodes down to the last level
        w = W.cube(n, seed=seed, n0=n0)
        w.src[10:] = w.src[0]
        return w
    raise ValueError(kind)


# level sizes (oracle): the 20,000-point sphere 1, 8, 56, 264, 575 (the sparse top levels
# and the level-by-level build both run); the chain one node per level from level 2 to the
# last (21)
TREE_CASES = [("cube", 1000, 1, 50), ("cube", 5003, 2, 64), ("sphere", 20000, 3, 100), ("cube_pm1", 7777, 4, 500),
              ("dups", 3000, 5, 40), ("cube", 70, 6, 1000), ("chain", 300, 8, 20)]


@pytest.mark.parametrize("kind,n,seed,n0", TREE_CASES)
def test_tree_matches_oracle(nat, orc, kind, n, seed, n0):
    w = _case(kind, n, seed, n0)
    T = orc.build_tree(w.src, n0)
    g = nat.tree_export(nat.build_tree(_t(w.src), n0))
    assert g["level"].shape[0] == T.nnodes
    assert np.array_equal(g["perm"], T.perm)
    for k in ("level", "parent", "child0", "nchild", "start", "count"):
        assert np.array_equal(g[k], getattr(T, k)), k
    for k in ("bmin", "bmax", "center", "radius"):
        assert np.array_equal(g[k], getattr(T, k)), k


def test_tree_all_coincident(nat, orc):
    src = np.tile([[0.25, -0.5, 0.75]], (300, 1))
    g = nat.tree_export(nat.build_tree(_t(src), 10))
    assert g["level"].shape[0] == 1 and g["radius"][0] == 0.0 and g["count"][0] == 300


@pytest.mark.parametrize("p", [0, 3, 8, 10])
def test_moments_match_oracle(nat, orc, p):
    w = W.cube(6000, seed=7, lo=-1.0, hi=1.0, n0=80)
    T = orc.build_tree(w.src, w.n0)
    M, Mt = orc.moments(T, w.src, w.f[0], w.h[0], w.nu, p)
    tr = nat.build_tree(_t(w.src), w.n0)
    nat.compute_moments(tr, _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, "fp64")
    gM, gMt = nat.tree_moments(tr, p)
    for a, b in ((gM, M), (gMt, Mt)):
        scale = np.abs(b).reshape(b.shape[0], -1).max(axis=1)[:, None]
        err = np.abs(a - b).reshape(b.shape[0], -1) / scale
        assert err.max() < 1e-13


def _oracle_tc(orc, w, p, theta, tg):
    T = orc.build_tree(w.src, w.n0)
    M, Mt = orc.moments(T, w.src, w.f[0], w.h[0], w.nu, p)
    return orc.treecode(T, w.src, w.f[0], w.h[0], w.nu, M, Mt, p, theta, tg)


TC_CASES = [
    # kind, n, seed, n0, p, theta, targets ("same" | "disjoint" | "subset")
    ("cube", 1000, 1, 50, 6, 0.5, "same"),
    ("cube_pm1", 20000, 2, 500, 4, 0.5, "same"),
    ("cube_pm1", 20000, 2, 500, 8, 0.7, "same"),
    ("cube_pm1", 20000, 2, 500, 10, 0.5, "subset"),
    ("sphere", 30000, 3, 200, 8, 0.5, "subset"),
    ("cube", 9000, 8, 60, 0, 0.6, "disjoint"),
    ("cube", 9000, 8, 60, 5, 0.3, "disjoint"),
    ("dups", 4000, 9, 30, 6, 0.5, "same"),
]


def _targets(w, how, seed=0):
    if how == "same":
        return w.src
    rng = np.random.default_rng(seed)
    if how == "subset":
        return w.src[np.sort(rng.choice(w.n, 3001, replace=False))]
    lo, hi = w.src.min(0), w.src.max(0)
    return rng.uniform(lo - 0.3 * (hi - lo), hi + 0.3 * (hi - lo), (2501, 3))


@pytest.mark.parametrize("kind,n,seed,n0,p,theta,how", TC_CASES)
def test_treecode_fp64_matches_oracle(nat, orc, kind, n, seed, n0, p, theta, how):
    w = _case(kind, n, seed, n0)
    tg = _targets(w, how)
    ref = _oracle_tc(orc, w, p, theta, tg)
    u, plan = nat.evaluate(_t(tg), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "fp64",
                           keep_plan=True)
    nf, nn, npair = nat.plan_counts(plan)
    assert np.array_equal(nf, ref.nfar)
    assert np.array_equal(nn, ref.nnear)
    assert np.array_equal(npair, ref.npairs)
    assert orc.rel_l2(u.cpu().numpy(), ref.u) < 1e-12


def _per_target(lists, m):
    """Expand group lists (entries with 64-bit lane masks) into per-target sorted node arrays."""
    off, node, mask, tperm = lists["off"], lists["node"], lists["mask"], lists["tperm"]
    grp = np.repeat(np.arange(len(off) - 1), np.diff(off))
    bits = ((mask[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(bool)
    e_idx, lane = np.nonzero(bits)
    sorted_t = grp[e_idx].astype(np.int64) * 64 + lane
    assert np.all(sorted_t < m)
    tgt = tperm[sorted_t]
    order = np.lexsort((node[e_idx], tgt))
    return tgt[order], node[e_idx][order]


@pytest.mark.parametrize("kind,n,seed,n0,p,theta,how", [TC_CASES[i] for i in (0, 2, 4, 6)])
def test_interaction_lists_match_oracle(nat, orc, kind, n, seed, n0, p, theta, how):
    """Alg. 1: every target's far clusters and near leaves are the oracle's, as sets."""
    w = _case(kind, n, seed, n0)
    tg = _targets(w, how)
    T = orc.build_tree(w.src, n0)
    L = orc.lists(T, theta, tg)
    _, plan = nat.evaluate(_t(tg), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "fp64",
                           keep_plan=True)
    m = tg.shape[0]
    for kind_, ptr, nodes in (("far", L.far_ptr, L.far_nodes), ("near", L.near_ptr, L.near_nodes)):
        t_gpu, n_gpu = _per_target(nat.plan_lists(plan, kind_), m)
        t_ref = np.repeat(np.arange(m), np.diff(ptr))
        n_ref = nodes[: int(ptr[-1])]
        order = np.lexsort((n_ref, t_ref))
        assert np.array_equal(t_gpu, t_ref[order]), kind_
        assert np.array_equal(n_gpu, n_ref[order]), kind_


def test_list_build_one_pass_and_second_pass(nat, orc):
    """The lists are written in one traversal into per-group slots sized from the tree's
    previous evaluation (a quarter above its longest group lists), then compacted; a group
    whose lists outgrow their slots (a fresh tree starts at 512 far and 256 near entries)
    makes the build fall back to a second traversal at the scanned offsets.  N = 20,000 in
    the unit cube, N0 = 16, theta = 0.35: the longest group far list (1464 entries, from the
    oracle's per-target lists) exceeds a fresh tree's slots, so a fresh plan's first
    evaluation takes the second pass and the same plan's next one the slots.  Both give
    every target's far clusters and near leaves of Algorithm 1."""
    w = W.cube(20_000, seed=12, n0=16)
    theta, p, n0 = 0.35, 2, 16
    T = orc.build_tree(w.src, n0)
    L = orc.lists(T, theta, w.src)
    X = _t(w.src)
    nat.plan_cache_clear()
    for call in range(2):
        _, plan = nat.evaluate(X, X, _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "fp64", keep_plan=True)
        for kind_, ptr, nodes in (("far", L.far_ptr, L.far_nodes), ("near", L.near_ptr, L.near_nodes)):
            lists = nat.plan_lists(plan, kind_)
            if call == 0 and kind_ == "far":
                assert np.diff(lists["off"]).max() > 512
            t_gpu, n_gpu = _per_target(lists, w.n)
            t_ref = np.repeat(np.arange(w.n), np.diff(ptr))
            n_ref = nodes[: int(ptr[-1])]
            order = np.lexsort((n_ref, t_ref))
            assert np.array_equal(t_gpu, t_ref[order]), (call, kind_)
            assert np.array_equal(n_gpu, n_ref[order]), (call, kind_)
        del plan


def test_large_plan_matches_oracle(nat, orc):
    """150,000 targets (= sources) with small leaves: the device-wide scans of the list
    build take their multi-tile path (more than 65,536 entries); counts, lists and the
    FP64 result still match the oracle."""
    w = W.cube(150_000, seed=10, n0=64)
    p, theta = 3, 0.5
    ref = _oracle_tc(orc, w, p, theta, w.src)
    u, plan = nat.evaluate(_t(w.src), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, 64, "fp64",
                           keep_plan=True)
    nf, nn, npair = nat.plan_counts(plan)
    assert np.array_equal(nf, ref.nfar)
    assert np.array_equal(nn, ref.nnear)
    assert np.array_equal(npair, ref.npairs)
    assert nat.plan_info(plan)["near_entries"] > 65536
    t_gpu, n_gpu = _per_target(nat.plan_lists(plan, "near"), w.n)
    assert np.array_equal(np.bincount(t_gpu, minlength=w.n), ref.nnear)
    assert orc.rel_l2(u.cpu().numpy(), ref.u) < 1e-12


@pytest.mark.parametrize("kind,n,seed,n0,p,theta,how", TC_CASES[:6])
def test_treecode_mixed_close_to_fp64(nat, orc, kind, n, seed, n0, p, theta, how):
    w = _case(kind, n, seed, n0)
    tg = _targets(w, how)
    ref = _oracle_tc(orc, w, p, theta, tg)
    u = nat.evaluate(_t(tg), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "mixed")
    assert orc.rel_l2(u.cpu().numpy(), ref.u) < 1e-5


def test_theta_zero_is_direct_sum(nat, orc):
    w = W.cube(3000, seed=10, n0=40)
    u = nat.evaluate(_t(w.src), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu), 6, 0.0, 40, "fp64")
    ud = orc.direct(w.src, w.src, w.f[0], w.h[0], w.nu)
    assert orc.rel_l2(u.cpu().numpy(), ud) < 1e-13


@pytest.mark.parametrize("n,m", [(1, 1), (2, 65), (1000, 1000), (4097, 333)])
def test_direct_matches_oracle(nat, orc, n, m):
    w = W.cube(n, seed=11)
    tg = W.cube(m, seed=12).src if m != n else w.src
    ud = orc.direct(tg, w.src, w.f[0], w.h[0], w.nu)
    u = nat.direct(_t(tg), _t(w.src), _t(w.f[0]), _t(w.h[0]), _t(w.nu)).cpu().numpy()
    assert orc.rel_l2(u, ud) < 1e-14


def test_reuse_tree_and_moments(nat, orc):
    """Evaluate twice on one tree, with new moments in between (iterative-solve use)."""
    w = W.cube(5000, seed=13, n0=64)
    tr = nat.build_tree(_t(w.src), w.n0)
    for r, prec in enumerate(("fp64", "mixed", "fp64")):
        f = w.f[0] * (r + 1)
        nat.compute_moments(tr, _t(f), _t(w.h[0]), _t(w.nu), 5, prec)
        u = nat.evaluate_tree(tr, _t(w.src), 0.5)
        T = orc.build_tree(w.src, w.n0)
        M, Mt = orc.moments(T, w.src, f, w.h[0], w.nu, 5)
        ref = orc.treecode(T, w.src, f, w.h[0], w.nu, M, Mt, 5, 0.5, w.src)
        assert orc.rel_l2(u.cpu().numpy(), ref.u) < (1e-12 if prec == "fp64" else 1e-5)


def test_argument_errors(nat):
    import torch
    x = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(nat.StkError) as e:
        nat.evaluate(x, x, x, x, x, 11, 0.5, 10)
    assert e.value.status == nat.STK_EINVAL
    with pytest.raises(nat.StkError):
        nat.evaluate(x, x, x, x, x, 4, 1.0, 10)
    with pytest.raises(nat.StkError):
        nat.evaluate(x, x, x, x, x, 4, 0.5, 0)
    tr = nat.build_tree(x + torch.rand_like(x), 4)
    with pytest.raises(nat.StkError) as e:
        nat.evaluate_tree(tr, x, 0.5)
    assert e.value.status == nat.STK_ESTATE


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_target_and_single_source(nat, orc, prec):
    """Degenerate sizes: one target against many sources, many targets against one source
    (a one-point tree: the root is a leaf of radius 0), and one against one."""
    rng = np.random.default_rng(90)
    src = rng.uniform(0, 1, (3000, 3))
    f, h = rng.uniform(-1, 1, (2, 3000, 3))
    nu = rng.normal(size=(3000, 3))
    nu /= np.linalg.norm(nu, axis=1, keepdims=True)
    tol = 1e-12 if prec == "fp64" else 1e-5
    for tg, s, ff, hh, nn in ((rng.uniform(0, 1, (1, 3)), src, f, h, nu),
                              (rng.uniform(0, 1, (500, 3)), src[:1], f[:1], h[:1], nu[:1]),
                              (src[:1] + 0.25, src[:1], f[:1], h[:1], nu[:1])):
        T = orc.build_tree(s, 40)
        M, Mt = orc.moments(T, s, ff, hh, nn, 4)
        ref = orc.treecode(T, s, ff, hh, nn, M, Mt, 4, 0.5, tg)
        u = nat.evaluate(_t(tg), _t(s), _t(ff), _t(hh), _t(nn), 4, 0.5, 40, prec)
        assert orc.rel_l2(u.cpu().numpy(), ref.u) < tol


def test_target_equal_to_only_source_gives_zero(nat):
    """The only source coincides with the target: the pair is skipped (r = 0), u = 0."""
    import torch
    x = torch.tensor([[0.3, 0.4, 0.5]], dtype=torch.float64, device="cuda")
    one = torch.ones_like(x)
    for prec in ("fp64", "mixed"):
        u = nat.evaluate(x, x, one, one, one / 3 ** 0.5, 6, 0.5, 10, prec)
        assert torch.count_nonzero(u) == 0


def test_maximum_rhs_count(nat):
    """K = 64 right-hand sides (the largest accepted) against one-RHS runs, in both
    precisions, with the default kernel variants."""
    w = W.cube(6000, seed=91, n0=80, k=64)
    X = _t(w.src)
    F, H, NU = _t(w.f), _t(w.h), _t(w.nu)
    for prec, tol in (("fp64", 1e-15), ("mixed", 2e-6)):
        u = nat.evaluate(X, X, F, H, NU, 5, 0.5, 80, prec)
        for r in (0, 17, 63):
            u1 = nat.evaluate(X, X, F[r].contiguous(), H[r].contiguous(), NU, 5, 0.5, 80, prec)
            assert float((u[r] - u1).norm() / u1.norm()) <= tol, (prec, r)
    with pytest.raises(nat.StkError):
        bad = _t(np.zeros((65, 10, 3)))
        nat.evaluate(X[:10].contiguous(), X[:10].contiguous(), bad, bad, NU[:10].contiguous(), 5, 0.5, 80)
