"""Seeded random configurations against the oracle, element by element
(energies 1e-12 / 1e-6, dE/dn 1e-10 / 1e-4 in the L2 norm for the FP64 /
FP32C forms): grid shapes and spacings (cubic or not), periodic axes and
image ranges, distance cuts, table shapes (16 or 64 sigma columns, so both
the generic and the fast kernels run), LDS row limits, j-chunk lengths and
workgroup shapes (with short chunks, 1024-thread row blocks split their
diagonal work into several items), and on periodic grids without a cut a
far image shell in half the cases (drawn from a stream of its own, so the
other choices do not depend on it).  A random cut is moved off any pair distance it would
nearly tie with (a tie may fall either way in FP32)."""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
FP = {0: (1e-12, 1e-10), 1: (1e-6, 1e-4)}
NCASES = 16


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
def tables(oracle):
    out = {}
    for nS, nD, Dmax in ((16, 256, 16.0), (64, 512, 24.0)):
        tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax, **CHEAP_RULE)
        out[nS] = (tp, oracle.build_table(tp))
    return out


def _safe_cut(rng, h, lo=2.0, hi=6.0):
    """A cut radius with no grid distance (any integer offset, any image) within
    1e-5 (relative) of it: only offsets shorter than `hi` can tie."""
    k = [np.arange(-int(np.ceil(hi / ha)) - 1, int(np.ceil(hi / ha)) + 2) for ha in h]
    kx, ky, kz = np.meshgrid(*k, indexing="ij")
    d2 = np.unique((kx * h[0]) ** 2 + (ky * h[1]) ** 2 + (kz * h[2]) ** 2)
    for _ in range(200):
        rc = rng.uniform(lo, hi)
        if np.min(np.abs(d2 - rc * rc)) > 1e-5 * rc * rc:
            return rc
    raise RuntimeError("no tie-free cut found")


def _case(k):
    rng = np.random.default_rng(1000 + k)
    n = tuple(int(v) for v in rng.integers(12, 27, size=3))  # several row blocks: the off-diagonal rings run
    if rng.random() < 0.5:
        h = (float(rng.uniform(0.3, 0.6)),) * 3
    else:
        h = tuple(float(v) for v in rng.uniform(0.3, 0.6, size=3))
    periodic = tuple(int(v) for v in (rng.random(3) < 0.35))
    image_max = tuple(int(rng.integers(0, 2)) if p else 0 for p in periodic)
    wl = W.random_small(n=n, h=h, periodic=periodic, seed=2000 + k, n_cut=float(rng.uniform(1.5e-3, 2.15e-3)),
                        image_max=image_max)
    if rng.random() < 0.4:
        wl.r_cut = _safe_cut(rng, h)
    opts = dict(table_lds_rows=int(rng.choice([-1, 2, 12, 60])), j_chunks=int(rng.choice([0, 1, 2])),
                block_threads=int(rng.choice([0, 256, 512, 1024])))
    nS = int(rng.choice([16, 64]))
    rf = np.random.default_rng(3000 + k)
    far = (0, 0, 0)
    if any(periodic) and wl.r_cut == 0.0 and rf.random() < 0.5:
        far = tuple(m + int(rf.integers(1, 4)) if p else 0 for m, p in zip(image_max, periodic))
    opts["far_max"] = far
    return wl, opts, nS


@pytest.mark.parametrize("k", range(NCASES))
def test_random_configuration(V, oracle, tables, k):
    import torch

    wl, extra, nS = _case(k)
    tp, tab = tables[nS]
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, wl.image_max, wl.r_cut,
                          potential=True, far_max=extra["far_max"])
    assert ref.E != 0.0
    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    table = V.Table(params, t64, t64.float().contiguous())
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    for prec in (0, 1):
        etol, vtol = FP[prec]
        opts = V.Opts(n_cut=wl.n_cut, r_cut=wl.r_cut, image_max=wl.image_max, precision=prec, **extra)
        E, v = V.enl_potential(g, n, qd, table, opts)
        v = v.cpu().numpy()
        st = V.last_stats()
        rel_e = abs(sum(E) - ref.E) / abs(ref.E)
        rel_v = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
        say(f"case {k} prec {prec}: n={wl.n} h={tuple(round(x, 3) for x in wl.h)} per={wl.periodic} "
            f"img={wl.image_max} rc={wl.r_cut:.3f} nS={nS} {extra} N={st['retained']} "
            f"threads={st['block_threads']} diag={st['diag_items']} dE={rel_e:.1e} dv={rel_v:.1e}")
        assert rel_e <= etol
        for a, b in ((E[0], ref.E_pair0), (E[1], ref.E_pairL), (E[2], ref.E_self)):
            assert abs(a - b) <= etol * abs(ref.E) + 1e-300
        assert rel_v <= vtol
