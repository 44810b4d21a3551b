"""enl_potential_noalloc (the entry point for callers that cannot allocate:
its workspace is the library's static device scratch) against enl_potential
on the same inputs, called through the C ABI: two calls in a row, the second
on a smaller grid, in both precisions, and the rejection of a grid that needs
more scratch than the library holds.  Both paths run the same kernels, whose
results are bitwise reproducible, so the energies and dE/dn must be equal;
the tolerances of the oracle parity tests are checked as well."""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
TOL = {0: (1e-12, 1e-10), 1: (1e-6, 1e-4)}  # (energy, dE/dn in L2) per precision


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def V():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0810_2273_amd as V

    return V


@pytest.fixture(scope="module")
def table(V):
    return V.build_phi_table(V.TableParams(n_D=512, n_sigma=64, D_max=24.0, **CHEAP_RULE), device="cuda:0")


def _both(V, wl, table, prec):
    import torch

    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    opts = V.Opts(n_cut=wl.n_cut, precision=prec)
    Ea, va = V.enl_potential_noalloc(g, n, qd, table, opts)
    Eb, vb = V.enl_potential(g, n, qd, table, opts)
    return Ea, va.cpu().numpy(), Eb, vb.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_enl_potential_twice(V, table, prec):
    etol, vtol = TOL[prec]
    for edge in (32, 24):  # the second call on a smaller grid
        wl = W.scaled_dimer(edge=edge, h=0.4, R=5.0)
        say(f"noalloc vs enl_potential: {edge}^3 dimer, precision {prec}")
        Ea, va, Eb, vb = _both(V, wl, table, prec)
        say(f"  E noalloc {Ea}  E workspace {Eb}")
        for a, b in zip(Ea, Eb):
            assert abs(a - b) <= etol * abs(sum(Eb)) + 1e-300
        assert np.linalg.norm(va - vb) <= vtol * np.linalg.norm(vb)
        assert tuple(Ea) == tuple(Eb)
        assert np.array_equal(va, vb)
        assert V.last_stats()["retained"] > 1000


def test_noalloc_rejects_grids_beyond_the_scratch(V, table):
    import torch

    from paper_0810_2273_amd import _lib as L

    wl = W.scaled_dimer(edge=48, h=0.3, R=5.0)
    g = V.Grid(wl.n, wl.h, wl.periodic)
    opts = V.Opts(n_cut=wl.n_cut, precision=0)
    assert V.enl_workspace_size(g, table, opts) > 64 << 20
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    with pytest.raises(L.VdwError) as ei:
        V.enl_potential_noalloc(g, n, qd, table, opts)
    say(f"  rejected: {ei.value}")
    assert ei.value.code == L.VDW_EWORKSPACE
    assert "scratch" in str(ei.value)
