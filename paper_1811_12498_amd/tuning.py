"""Choice of the treecode parameters (p, theta, N0) for the least time at a required
accuracy, the tuning the paper leaves to future work (Sec. 7).

For every candidate on a grid, one `stk_evaluate` of the caller's own problem is timed (after
a warm-up) and its error E = ||u - u_d|| / ||u_d|| is measured on seeded sample targets
against the FP64 direct sum on the GPU; the fastest candidate with E <= e_target wins.  The
sweep only orchestrates library calls: every evaluation runs in the HIP kernels."""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Candidate:
    p: int
    theta: float
    n0: int
    ms: float       # time of one evaluation
    error: float    # E on the sample targets


def select(table: list[Candidate], e_target: float) -> Candidate | None:
    """The fastest candidate whose error is at most e_target (ties: the smaller error, then
    the smaller p); None when no candidate is accurate enough."""
    ok = [c for c in table if c.error <= e_target]
    if not ok:
        return None
    return min(ok, key=lambda c: (c.ms, c.error, c.p))


def sweep(targets, sources, f, h, nu, precision: str = "mixed", ps=(4, 6, 8, 10),
          thetas=(0.4, 0.5, 0.6, 0.7), n0s=(250, 500, 1000, 2000), n_sample: int = 2000, seed: int = 0,
          reps: int = 2) -> list[Candidate]:
    """Time and error of every (p, theta, N0) on the grid for this problem (device tensors
    as for `native.evaluate`, one right-hand side)."""
    import torch

    from . import native
    m = targets.shape[0]
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(m, min(n_sample, m), replace=False))
    S = torch.from_numpy(pick).to(targets.device)
    ud = native.direct(targets[S].contiguous(), sources, f, h, nu)
    nd = torch.linalg.norm(ud)
    table = []
    for n0 in n0s:
        for p in ps:
            for theta in thetas:
                u = native.evaluate(targets, sources, f, h, nu, p, theta, n0, precision)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    u = native.evaluate(targets, sources, f, h, nu, p, theta, n0, precision)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / reps
                err = float(torch.linalg.norm(u[S] - ud) / nd)
                table.append(Candidate(p, theta, n0, round(ms, 4), err))
    return table


def tune(targets, sources, f, h, nu, e_target: float, precision: str = "mixed", **grid):
    """(best candidate or None, full table) for the required error e_target."""
    table = sweep(targets, sources, f, h, nu, precision, **grid)
    return select(table, e_target), table
