"""Seeded random combinations of the widened options against the oracle,
element by element (FP64: 1e-12 / 1e-10, FP32C: 1e-6 / 1e-4 for the energy
/ dE/dn): orthorhombic or skew cells, the finite-difference or the spectral
gradient on periodic axes, near images and a far image shell, the sphere or
the voxel on-site term, and both table interpolants where offered (the
cubic form in FP64)."""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
FP = {0: (1e-12, 1e-10), 1: (1e-6, 1e-4)}
NCASES = 8


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def V():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0810_2273_amd as V

    return V


def _case(k):
    rng = np.random.default_rng(4000 + k)
    n = tuple(int(v) for v in rng.integers(12, 19, size=3))
    periodic = tuple(int(v) for v in (rng.random(3) < 0.6))
    if not any(periodic):
        periodic = (1, 0, 0)
    skew = rng.random() < 0.5
    if skew:
        C = np.diag(rng.uniform(0.35, 0.5, size=3) * np.array(n))
        C[1, 0] = rng.uniform(-0.3, 0.3) * C[1, 1]
        C[2, 0], C[2, 1] = rng.uniform(-0.2, 0.2, size=2) * C[2, 2]
        wl = W.random_skew(n=n, cell=tuple(map(tuple, C)), periodic=periodic, seed=5000 + k, n_cut=2.2e-3)
    else:
        h = tuple(float(v) for v in rng.uniform(0.35, 0.5, size=3))
        wl = W.random_small(n=n, h=h, periodic=periodic, seed=5000 + k, n_cut=2.2e-3)
    near = tuple(int(rng.integers(1, 3)) if p else 0 for p in periodic)
    far = tuple(m + int(rng.integers(1, 4)) if p else 0 for m, p in zip(near, periodic)) if rng.random() < 0.6 \
        else (0, 0, 0)
    gradient = "spectral" if rng.random() < 0.5 else "fd"
    self_term = int(rng.choice([1, 2]))
    interp = int(rng.random() < 0.3)
    return wl, near, far, gradient, self_term, interp


@pytest.fixture(scope="module")
def tables(oracle):
    out = {}
    for interp in (0, 1):
        tp = oracle.table_params(n_D=256, n_sigma=16, D_max=16.0, interp=interp, **CHEAP_RULE)
        out[interp] = (tp, oracle.build_table(tp))
    return out


@pytest.mark.parametrize("k", range(NCASES))
def test_combined_options(V, oracle, tables, k):
    import torch

    wl, near, far, gradient, self_term, interp = _case(k)
    tp, tab = tables[interp]
    if wl.cell is not None:
        g = V.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell, gradient=gradient)
        og = oracle.grid_of_cell(wl.n, wl.cell, wl.periodic, gradient=gradient)
    else:
        g = V.Grid(wl.n, wl.h, wl.periodic, gradient=gradient)
        og = oracle.Grid(wl.n, wl.h, wl.periodic, gradient=gradient)
    ref = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, near, self_term=self_term, potential=True, far_max=far)
    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0, interp=interp)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    table = V.Table(params, t64, t64.float().contiguous())
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    for prec in ((0,) if interp else (0, 1)):
        etol, vtol = FP[prec]
        opts = V.Opts(n_cut=wl.n_cut, image_max=near, far_max=far, self_term=self_term, precision=prec)
        E, v = V.enl_potential(g, n, qd, table, opts)
        v = v.cpu().numpy()
        rel_e = abs(sum(E) - ref.E) / abs(ref.E)
        rel_v = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
        say(f"combined {k} prec {prec}: n={wl.n} per={wl.periodic} skew={wl.cell is not None} near={near} "
            f"far={far} grad={gradient} self={self_term} interp={interp} dE={rel_e:.1e} dv={rel_v:.1e}")
        assert rel_e <= etol
        for a, b in ((E[0], ref.E_pair0), (E[1], ref.E_pairL), (E[2], ref.E_self)):
            assert abs(a - b) <= etol * abs(ref.E) + 1e-300
        assert rel_v <= vtol
