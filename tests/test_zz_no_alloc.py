"""stk_direct_noalloc (the direct sum that allocates nothing: partial sums in the
library's fixed per-device array) against stk_direct through the C-ABI: two calls in a
row, the second smaller, each bit-identical to stk_direct and within 1e-12 relative of
it; the first is large enough that its targets go through the array in two slices.  A
few targets are also checked against the FP64 oracle's direct sum."""
import numpy as np
import pytest

from paper_1811_12498_amd import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = (32 << 20) // 8


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


def _slices(m, n):
    """Target slices the library uses for (m, n): its source chunking (512..8192 sources,
    about 32768 waves) and the partial sums of a slice within the fixed array."""
    ng = -(-m // 64)
    want = -(-32768 // ng)
    c = -(-n // want)
    c = min(max(-(-c // 256) * 256, 512), 8192)
    nch = -(-n // c)
    ms = SCRATCH_DOUBLES // (3 * nch) // 64 * 64
    return -(-m // min(ms, m))


def _check(nat, orc, src, tgt, f, h, nu, sample):
    import torch
    X, T, F, H, NU = _t(src), _t(tgt), _t(f), _t(h), _t(nu)
    ref = nat.direct(T, X, F, H, NU)
    out = nat.direct_noalloc(T, X, F, H, NU)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    rel = float((out - ref).norm() / ref.norm())
    assert rel <= 1e-12, rel
    f0 = f[0] if f.ndim == 3 else f
    h0 = h[0] if h.ndim == 3 else h
    u_o = orc.direct(tgt[sample], src, f0, h0, nu)
    got = (out[0] if f.ndim == 3 else out).cpu().numpy()[sample]
    assert orc.rel_l2(got, u_o) < 1e-13


def test_noalloc_matches_direct_twice(nat, orc):
    big = W.cube(200_000, seed=21, p=8, theta=0.5, n0=2000)
    m1 = 100_000
    assert _slices(m1, big.n) == 2
    _check(nat, orc, big.src, big.src[:m1], big.f[0], big.h[0], big.nu, np.arange(0, m1, 9973))
    small = W.cube(50_000, seed=22, k=2, p=8, theta=0.5, n0=2000)
    m2 = 3_000
    assert _slices(m2, small.n) == 1
    _check(nat, orc, small.src, small.src[-m2:], small.f, small.h, small.nu, np.arange(0, m2, 307))


def test_noalloc_rejects_bad_arguments(nat):
    import torch
    X = _t(np.zeros((4, 3)))
    with pytest.raises(nat.StkError, match="STK_EINVAL"):
        nat._check(nat._lib.stk_direct_noalloc(nat._ptr(X), 4, nat._ptr(X), 4, nat._ptr(X), nat._ptr(X),
                                               None, 1, nat._ptr(X), nat._stream()))
    with pytest.raises(ValueError):
        nat.direct_noalloc(X, X, X, X, X, out=torch.empty((3, 3), dtype=torch.float64, device=X.device))
