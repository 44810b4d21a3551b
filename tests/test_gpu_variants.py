"""GPU parity of the pair-kernel variants the other tests reach only at full
size or not at all, element by element against the oracle (energies 1e-12 /
1e-6, dE/dn 1e-10 / 1e-4 in the L2 norm for the FP64 / FP32C forms):

* four i-points per lane on a non-cubic grid (difference form of r^2), and
  eight per lane in 512-thread workgroups on cubic and non-cubic grids;
* the Kahan-compensated FP32 variant, in 1024- and 256-thread workgroups;
* row blocks whose diagonal work is split into several items (chunks
  shorter than the row block);
* a cubic periodic grid whose image-shifted coordinates are too large for
  the exact integer form of r^2 (|x_i|^2 + |x_j|^2 alone passes 2^24 for
  neighbouring points), which the host must route to the difference form.
"""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
FP = {"fp64": (0, 1e-12, 1e-10), "fp32c": (1, 1e-6, 1e-4)}


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
def big(oracle):
    tp = oracle.table_params(n_D=2048, n_sigma=64, D_max=48.0, **CHEAP_RULE)
    return tp, oracle.build_table(tp)


def _table(V, tp, tab):
    import torch

    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    return V.Table(params, t64, t64.float().contiguous())


def _run_check(V, oracle, wl, tp, tab, prec, what, **kw):
    import torch

    p, etol, vtol = FP[prec]
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    E, v = V.enl_potential(g, n, qd, _table(V, tp, tab),
                           V.Opts(n_cut=wl.n_cut, r_cut=wl.r_cut, image_max=wl.image_max, precision=p, **kw))
    v = v.cpu().numpy()
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, wl.image_max, wl.r_cut,
                          potential=True)
    rel_e = abs(sum(E) - ref.E) / abs(ref.E)
    rel_v = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
    say(f"  {what} {prec}: N={V.last_stats()['retained']} |dE|/|E|={rel_e:.2e} |dv|/|v|={rel_v:.2e}")
    assert rel_e <= etol
    for a, b in ((E[0], ref.E_pair0), (E[1], ref.E_pairL), (E[2], ref.E_self)):
        assert abs(a - b) <= etol * abs(ref.E) + 1e-300
    assert rel_v <= vtol
    return V.last_stats()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_non_cubic_grid_four_points_per_lane(V, oracle, big, prec):
    """34 x 30 x 28 grid with h = (0.40, 0.45, 0.35) and the 2048 x 64 table:
    seven row blocks of 4096 (FP32C) with a ragged last one."""
    tp, tab = big
    wl = W.random_small(n=(34, 30, 28), h=(0.40, 0.45, 0.35), seed=21, n_cut=1e-3)
    st = _run_check(V, oracle, wl, tp, tab, prec, "non-cubic", block_threads=1024)
    assert st["retained"] > 4 * 4096 and st["retained"] % 4096 != 0 and st["block_threads"] == 1024


@pytest.mark.parametrize("cubic", [True, False])
def test_eight_points_per_lane(V, oracle, big, cubic):
    """block_threads = 512: eight i-points per lane, same row blocks of 4096,
    on a cubic 30^3 dimer (with the LDS rows cut to 40 so the global-table
    pass runs too) and on the non-cubic grid above."""
    tp, tab = big
    if cubic:
        wl = W.scaled_dimer(edge=30, h=0.4, R=5.0)
        for rows in (-1, 40):
            st = _run_check(V, oracle, wl, tp, tab, "fp32c", f"eight-point cubic rows={rows}", block_threads=512,
                            table_lds_rows=rows)
    else:
        wl = W.random_small(n=(34, 30, 28), h=(0.40, 0.45, 0.35), seed=21, n_cut=1e-3)
        st = _run_check(V, oracle, wl, tp, tab, "fp32c", "eight-point non-cubic", block_threads=512)
    assert st["block_threads"] == 512


@pytest.mark.parametrize("threads", [1024, 256])
def test_kahan_variant(V, oracle, big, threads):
    """kahan = 1 (every FP32 run Kahan-compensated) on a 30^3 dimer, in both
    workgroup shapes the Kahan kernel has."""
    tp, tab = big
    wl = W.scaled_dimer(edge=30, h=0.4, R=5.0)
    st = _run_check(V, oracle, wl, tp, tab, "fp32c", "kahan", kahan=1, block_threads=threads)
    assert st["block_threads"] == threads


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("jc", [1, 2])
def test_split_diagonal(V, oracle, big, prec, jc):
    """1024-thread row blocks with chunks shorter than the block: each row
    block's diagonal work is split into BI / JC items (two or four; one for
    FP64 blocks of 2048 with chunks of 2048), on the non-cubic grid with a
    ragged last block."""
    tp, tab = big
    wl = W.random_small(n=(34, 30, 28), h=(0.40, 0.45, 0.35), seed=23, n_cut=1e-3)
    st = _run_check(V, oracle, wl, tp, tab, prec, f"split diagonal jc={jc}", block_threads=1024, j_chunks=jc)
    bi = 2048 if prec == "fp64" else 4096
    assert st["diag_items"] == max(1, bi // (1024 * jc))


def test_large_coordinates_use_the_difference_form(V, oracle, big):
    """Periodic x on a 3000 x 4 x 4 cubic grid with images |m| <= 1: for a
    point at x = 0 shifted by one cell and its neighbour at x = 2999,
    |x_i|^2 + |x_j|^2 exceeds 2^24, so the exact integer form of r^2 would
    round; the host must fall back to the difference form (FP32C)."""
    tp, tab = big
    wl = W.random_small(n=(3000, 4, 4), h=(0.3, 0.3, 0.3), periodic=(1, 0, 0), seed=22, n_cut=1e-3,
                        image_max=(1, 0, 0))
    assert 2 * 2999 ** 2 > 2 ** 24
    _run_check(V, oracle, wl, tp, tab, "fp32c", "large-coordinates")
