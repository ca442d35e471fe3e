"""Host build of the library's far-field header (stk_math.hpp) against the oracle.

The GPU kernels evaluate S_final + T_final in a regrouped, scaled form (G and E blocks
per cluster, recurrence on scaled coefficients).  This CPU test compiles that same
header for the host (tests/hostcheck/far_host.hip; no GPU code runs) and checks it
against the oracle's literal S_final/T_final for p = 0..10."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "hostcheck", "far_host.hip")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def hc(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("hc") / "libhc.so")
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "paper_1811_12498_amd", "csrc"), "-I",
                           os.path.join(ROOT, "include"), "-o", out, SRC])
    L = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    L.hc_rho.restype = ctypes.c_double
    L.hc_rho.argtypes = [ctypes.c_double]
    L.hc_far.argtypes = [dp, ctypes.c_int, dp, ctypes.c_double, dp]
    L.hc_gidx.argtypes = [ctypes.c_int] * 3
    L.hc_set_variant.argtypes = [ctypes.c_int]
    L.hc_stream_ok.argtypes = [ctypes.c_int]
    return L


def test_index_order_matches_oracle(hc, orc):
    for a, (k1, k2, k3) in enumerate(orc.kindex(12)):
        assert hc.hc_gidx(int(k1), int(k2), int(k3)) == a


@pytest.mark.parametrize("p", range(11))
def test_stream_layout_is_a_bijection(hc, p):
    assert hc.hc_stream_ok(p) == 1


@pytest.mark.parametrize("variant,tol", [(0, 1e-14), (1, 1e-4)])
def test_fp32_and_fp64_far_field(hc, orc, variant, tol):
    """FP64 to rounding; FP32 within what FP32 rounding of ~300 coefficients allows."""
    dp = ctypes.POINTER(ctypes.c_double)
    rng = np.random.default_rng(7)
    hc.hc_set_variant(variant)
    try:
        for p in (2, 6, 8, 10):
            kk = orc.kindex(p)
            for trial in range(20):
                ys = rng.uniform(-0.1, 0.1, (50, 3)) * rng.uniform(0.2, 1.0, 3)
                f, h = rng.uniform(-1, 1, (50, 3)), rng.uniform(-1, 1, (50, 3))
                nu = rng.standard_normal((50, 3))
                yc = (ys.min(0) + ys.max(0)) / 2
                dy = ys - yc
                r = np.sqrt((dy ** 2).sum(1)).max()
                mono = np.prod(dy[:, None, :] ** kk[None], axis=2)
                M, Mt = mono.T @ f, np.einsum("na,nj,nl->ajl", mono, h, nu)
                mom = np.ascontiguousarray(np.concatenate([M, Mt.reshape(-1, 9)], axis=1))
                d = rng.standard_normal(3)
                d *= (r / rng.uniform(0.2, 0.5)) / np.linalg.norm(d)
                u = np.zeros(3)
                hc.hc_far(mom.ctypes.data_as(dp), p, d.ctypes.data_as(dp), r, u.ctypes.data_as(dp))
                ref = orc.far_contracted(d, p, M, Mt)
                assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)
    finally:
        hc.hc_set_variant(0)


def test_rho_is_power_of_two_cover(hc):
    for r, want in ((0.0, 1.0), (0.3, 0.5), (0.5, 0.5), (1.0, 1.0), (3.0, 4.0), (1e-9, 2.0 ** -29)):
        assert hc.hc_rho(r) == want


@pytest.mark.parametrize("p", range(11))
def test_regrouped_far_field_equals_s_final_t_final(hc, orc, p):
    rng = np.random.default_rng(100 + p)
    kk = orc.kindex(p)
    dp = ctypes.POINTER(ctypes.c_double)
    for trial in range(4):
        ys = rng.uniform(-0.15, 0.15, (40, 3))
        f, h = rng.uniform(-1, 1, (40, 3)), rng.uniform(-1, 1, (40, 3))
        nu = rng.standard_normal((40, 3))
        yc = ys.mean(0) * 0.3
        dy = ys - yc
        r = np.sqrt((dy ** 2).sum(1)).max()
        mono = np.prod(dy[:, None, :] ** kk[None], axis=2)
        M = mono.T @ f
        Mt = np.einsum("na,nj,nl->ajl", mono, h, nu)
        mom = np.ascontiguousarray(np.concatenate([M, Mt.reshape(-1, 9)], axis=1))
        d = rng.standard_normal(3)
        d *= (r / 0.45) / np.linalg.norm(d) * (1 + trial * 0.7)
        u = np.zeros(3)
        hc.hc_far(mom.ctypes.data_as(dp), p, d.ctypes.data_as(dp), r, u.ctypes.data_as(dp))
        ref = orc.far_contracted(d, p, M, Mt)
        assert np.linalg.norm(u - ref) <= 1e-14 * np.linalg.norm(ref)
