"""Adjoint (gradients of L = sum w.u for the frozen plan) on the GPU vs the oracle.

The oracle's frozen-plan adjoint is pinned on the CPU by finite differences, the
dot-product test and the direct-sum gradient at theta = 0 (tests/test_oracle_pins.py).
Here the HIP adjoint is compared with it element by element (same lists: the per-target
interaction counts of both sides are equal), and checked at larger sizes through the
dot-product identity, which holds at any size."""
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


CASES = [
    # n, seed, n0, p, theta, disjoint targets
    (1200, 31, 40, 4, 0.5, False),
    (1500, 32, 64, 3, 0.6, True),
    (900, 33, 30, 6, 0.5, False),
]


@pytest.mark.parametrize("n,seed,n0,p,theta,disjoint", CASES)
def test_adjoint_fp64_matches_oracle(nat, orc, n, seed, n0, p, theta, disjoint):
    w = W.cube(n, seed=seed, n0=n0, with_w=True)
    tg = np.random.default_rng(seed).uniform(-0.2, 1.2, (n - 17, 3)) if disjoint else w.src
    wt = np.random.default_rng(seed + 1).uniform(-1, 1, tg.shape)
    T = orc.build_tree(w.src, n0)
    L = orc.lists(T, theta, tg)
    ref = orc.frozen_adjoint(T, L, w.src, w.f[0], w.h[0], w.nu, p, tg, wt)
    X = _t(tg)
    S = X if not disjoint else _t(w.src)
    u, plan = nat.evaluate(X, S, _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "fp64", keep_plan=True)
    g = nat.evaluate_adjoint(plan, _t(wt), n)
    for key, r in zip(("f", "h", "sources", "targets"), ref):
        err = orc.rel_l2(g[key].cpu().numpy(), r)
        assert err < 1e-11, (key, err)


def test_adjoint_mixed_close_to_oracle(nat, orc):
    n, n0, p, theta = 1500, 40, 5, 0.5
    w = W.cube(n, seed=34, n0=n0, with_w=True)
    T = orc.build_tree(w.src, n0)
    L = orc.lists(T, theta, w.src)
    ref = orc.frozen_adjoint(T, L, w.src, w.f[0], w.h[0], w.nu, p, w.src, w.w)
    X = _t(w.src)
    u, plan = nat.evaluate(X, X, _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, "mixed", keep_plan=True)
    g = nat.evaluate_adjoint(plan, _t(w.w), n)
    for key, r in zip(("f", "h", "sources", "targets"), ref):
        err = orc.rel_l2(g[key].cpu().numpy(), r)
        assert err < 1e-4, (key, err)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_dot_product_identity(nat, prec, tol):
    """L is linear in (f, h): sum(w * u) = sum(grad_f * f) + sum(grad_h * h)."""
    import torch
    w = W.cube(50_000, seed=35, n0=300, with_w=True)
    X = _t(w.src)
    F, H = _t(w.f[0]), _t(w.h[0])
    u, plan = nat.evaluate(X, X, F, H, _t(w.nu), 8, 0.5, 300, prec, keep_plan=True)
    g = nat.evaluate_adjoint(plan, _t(w.w), w.n, ("f", "h"))
    lhs = float(torch.sum(_t(w.w) * u))
    rhs = float(torch.sum(g["f"] * F) + torch.sum(g["h"] * H))
    scale = float(torch.sum(torch.abs(_t(w.w) * u)))
    assert abs(lhs - rhs) <= tol * scale


def test_autograd_function(nat):
    import torch
    from paper_1811_12498_amd.autograd import stokes_treecode
    w = W.cube(3000, seed=36, n0=64, with_w=True)
    X = _t(w.src).requires_grad_(True)
    F = _t(w.f[0]).requires_grad_(True)
    H = _t(w.h[0]).requires_grad_(True)
    NU = _t(w.nu)
    Wt = _t(w.w)
    u = stokes_treecode(X, X, F, H, NU, p=5, theta=0.5, n0=64, precision="fp64")
    (u * Wt).sum().backward()
    _, plan = nat.evaluate(X.detach(), X.detach(), F.detach(), H.detach(), NU, 5, 0.5, 64, "fp64", keep_plan=True)
    g = nat.evaluate_adjoint(plan, Wt, w.n)
    assert torch.allclose(F.grad, g["f"], rtol=1e-12, atol=1e-12)
    assert torch.allclose(H.grad, g["h"], rtol=1e-12, atol=1e-12)
    # the same tensor as targets and sources: autograd adds both position gradients
    assert torch.allclose(X.grad, g["targets"] + g["sources"], rtol=1e-10, atol=1e-10)


def test_finite_differences_full_size(nat):
    """N = 200,000 in the unit cube, p = 8, theta = 0.5, N0 = 2000, L = sum w.u: the FP64
    adjoint against central differences on 50 seeded coordinates (17 of f, 17 of h, 16
    of positions; targets = sources, so a position's gradient is the target part plus
    the source part).  L is linear in f and h, so their difference quotient is exact for
    any step and a unit step keeps rounding out of it; positions use a step of 1e-6 and
    a tolerance that adds the rounding of two evaluations of L (64 ulp of sum |w.u|)
    divided by the step.  A position perturbation that moves a cluster box or changes
    an interaction count leaves the frozen operator; such coordinates are replaced by
    the next draw."""
    import torch
    w = W.c5_cube_adjoint()
    rng = np.random.default_rng(55)
    X, F, H, NU, Wt = (_t(a) for a in (w.src, w.f[0], w.h[0], w.nu, w.w))
    args = (w.p, w.theta, w.n0, "fp64")
    u, plan = nat.evaluate(X, X, F, H, NU, *args, keep_plan=True)
    g = nat.evaluate_adjoint(plan, Wt, w.n)
    counts0 = nat.plan_counts(plan)
    tree0 = nat.tree_export(nat.build_tree(X, w.n0))
    eps = 1e-6
    noise = 64 * np.finfo(np.float64).eps * float(torch.sum(torch.abs(Wt * u))) / (2 * eps)

    def loss(Xp, Fp, Hp):
        return float(torch.sum(Wt * nat.evaluate(Xp, Xp, Fp, Hp, NU, *args)))

    checked = {"f": 0, "h": 0, "x": 0}
    want = {"f": 17, "h": 17, "x": 16}
    while any(checked[k] < want[k] for k in want):
        kind = next(k for k in ("f", "h", "x") if checked[k] < want[k])
        j, ax = int(rng.integers(w.n)), int(rng.integers(3))
        if kind == "x":
            ok = True
            for sgn in (1.0, -1.0):
                Xp = X.clone()
                Xp[j, ax] += sgn * eps
                t1 = nat.tree_export(nat.build_tree(Xp, w.n0))
                same = all(np.array_equal(t1[k], tree0[k]) for k in ("perm", "start", "count", "center", "radius"))
                _, pl1 = nat.evaluate(Xp, Xp, F, H, NU, *args, keep_plan=True)
                c1 = nat.plan_counts(pl1)
                same = same and all(np.array_equal(a, b) for a, b in zip(c1, counts0))
                ok = ok and same
            if not ok:
                continue
            Xp, Xm = X.clone(), X.clone()
            Xp[j, ax] += eps
            Xm[j, ax] -= eps
            fd = (loss(Xp, F, H) - loss(Xm, F, H)) / (2 * eps)
            ad = float(g["targets"][j, ax] + g["sources"][j, ax])
            tol = 1e-5 * abs(ad) + noise
        else:
            A = F if kind == "f" else H
            Ap, Am = A.clone(), A.clone()
            Ap[j, ax] += 1.0
            Am[j, ax] -= 1.0
            lp = loss(X, Ap, H) if kind == "f" else loss(X, F, Ap)
            lm = loss(X, Am, H) if kind == "f" else loss(X, F, Am)
            fd = (lp - lm) / 2.0
            ad = float(g[kind][j, ax])
            tol = 1e-9 * abs(ad) + noise * 2 * eps
        print(kind, j, ax, fd, ad, tol, flush=True)
        assert abs(fd - ad) <= tol, (kind, j, ax, fd, ad, tol)
        checked[kind] += 1


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 1e-4)])
def test_adjoint_after_cluster_major_forward(nat, orc, prec, tol):
    """With tile far_cm the forward builds the cluster-major view of every far entry and the
    adjoint reuses it; gradients against the oracle's adjoint."""
    n, seed, n0, p, theta = 1400, 36, 40, 5, 0.5
    w = W.cube(n, seed=seed, n0=n0, with_w=True)
    T = orc.build_tree(w.src, n0)
    L = orc.lists(T, theta, w.src)
    ref = orc.frozen_adjoint(T, L, w.src, w.f[0], w.h[0], w.nu, p, w.src, w.w)
    X = _t(w.src)
    try:
        nat.tiles_set(p, 1, prec, far_cm=1)
        u, plan = nat.evaluate(X, X, _t(w.f[0]), _t(w.h[0]), _t(w.nu), p, theta, n0, prec, keep_plan=True)
        assert nat.plan_far_split(plan)[0] == 64
        g = nat.evaluate_adjoint(plan, _t(w.w), n)
    finally:
        nat.tiles_set(p, 1, prec, clear=True)
    for key, r in zip(("f", "h", "sources", "targets"), ref):
        err = orc.rel_l2(g[key].cpu().numpy(), r)
        assert err < tol, (key, err)


def test_autograd_rejects_multi_rhs_gradients(nat):
    """K > 1 right-hand sides evaluate through the Function, but asking for gradients fails
    in forward (the adjoint is that of a one-right-hand-side operator)."""
    import torch
    from paper_1811_12498_amd.autograd import stokes_treecode
    w = W.cube(2000, seed=37, n0=64, k=3)
    X, NU = _t(w.src), _t(w.nu)
    F, H = _t(w.f), _t(w.h)
    u = stokes_treecode(X, X, F, H, NU, p=4, theta=0.5, n0=64, precision="fp64")
    assert u.shape == (3, w.n, 3)
    with pytest.raises(ValueError, match="one right-hand side"):
        stokes_treecode(X, X, F.clone().requires_grad_(True), H, NU, p=4, theta=0.5, n0=64, precision="fp64")
    del torch
