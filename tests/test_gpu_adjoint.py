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
