"""The boundary from plain C on the GPU: the C99 caller in tests/c_abi
allocates its own device buffers and workspace with the HIP runtime's C
API, builds the table, computes q0 and runs enl_potential; its energies and
dE/dn equal the oracle's (FP64: 1e-12 / 1e-10, FP32C: 1e-6 / 1e-4)."""
import ctypes as ct
import os

import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "tests", "c_abi", "libenl_from_c.so")


@pytest.fixture(scope="module")
def demo():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ct.CDLL(DEMO)
    P = ct.POINTER
    lib.vdw_c_demo.restype = ct.c_int
    lib.vdw_c_demo.argtypes = [P(ct.c_int32), P(ct.c_double), P(ct.c_int32), P(ct.c_int32), ct.c_double, ct.c_int32,
                               P(ct.c_double), P(ct.c_double), P(ct.c_double)]
    return lib


@pytest.mark.parametrize("prec,etol,vtol", [(0, 1e-12, 1e-10), (1, 1e-6, 1e-4)])
def test_c_caller_matches_oracle(demo, oracle, prec, etol, vtol):
    wl = W.random_small(n=(13, 12, 11), h=(0.4, 0.45, 0.5), periodic=(1, 1, 0), seed=91, n_cut=2.2e-3)
    image_max = (1, 1, 0)
    tp = oracle.table_params(n_D=256, n_sigma=16, D_max=16.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    tab = oracle.build_table(tp)
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, image_max, potential=True)
    n3 = (ct.c_int32 * 3)(*wl.n)
    h = (ct.c_double * 3)(*wl.h)
    per = (ct.c_int32 * 3)(*wl.periodic)
    im = (ct.c_int32 * 3)(*image_max)
    rho = np.ascontiguousarray(wl.rho.reshape(-1), dtype=np.float64)
    E = (ct.c_double * 3)()
    v = np.zeros(wl.G)
    dp = ct.POINTER(ct.c_double)
    print(f"C caller precision={prec}", flush=True)
    rc = demo.vdw_c_demo(n3, h, per, im, wl.n_cut, prec, rho.ctypes.data_as(dp), E, v.ctypes.data_as(dp))
    assert rc == 0
    assert abs(sum(E) - ref.E) <= etol * abs(ref.E)
    for a, b in zip(E, (ref.E_pair0, ref.E_pairL, ref.E_self)):
        assert abs(a - b) <= etol * abs(ref.E)
    assert np.linalg.norm(v - ref.dEdn) <= vtol * np.linalg.norm(ref.dEdn)
