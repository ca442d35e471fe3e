"""Parameter sweep on the GPU: the chosen (p, theta, N0) meets the required error and is
the fastest candidate that does; the error grows with theta at fixed p and N0."""
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


def test_tune_small_cube(nat):
    import torch
    from paper_1811_12498_amd import tuning
    w = W.cube(30_000, seed=71)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    X, F, H, NU = t(w.src), t(w.f[0]), t(w.h[0]), t(w.nu)
    best, table = tuning.tune(X, X, F, H, NU, 1e-4, "fp64", ps=(4, 8), thetas=(0.4, 0.7), n0s=(200, 800),
                              n_sample=500, reps=1)
    assert len(table) == 8
    assert best is not None and best.error <= 1e-4
    assert best.ms == min(c.ms for c in table if c.error <= 1e-4)
    for p in (4, 8):
        for n0 in (200, 800):
            e = {c.theta: c.error for c in table if c.p == p and c.n0 == n0}
            assert e[0.4] < e[0.7], (p, n0, e)
