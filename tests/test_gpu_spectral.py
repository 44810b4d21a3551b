"""GPU parity of the spectral (Fourier-derivative) gradient against the
oracle, whose derivative is an FFT along the axis: gradient and q0 point by
point; energies and dE/dn element by element (FP64: 1e-12 / 1e-10, FP32C:
1e-6 / 1e-4), the adjoint including the transposed line operators; the
exchange-correlation energies; on orthorhombic and skew cells, with even
and odd periodic axes and an open axis; and in a batch with a
finite-difference density (the batched call and graph plans)."""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
FP = {0: (1e-12, 1e-10), 1: (1e-6, 1e-4)}


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
def table(oracle):
    tp = oracle.table_params(n_D=256, n_sigma=16, D_max=16.0, **CHEAP_RULE)
    return tp, oracle.build_table(tp)


def _case(k):
    if k == 0:  # even x, odd y periodic, open z
        return W.random_small(n=(20, 17, 12), h=(0.35, 0.4, 0.3), periodic=(1, 1, 0), seed=80, n_cut=2.2e-3,
                              image_max=(1, 1, 0))
    if k == 1:  # fully periodic, odd x
        return W.random_small(n=(15, 14, 16), h=(0.4, 0.35, 0.3), periodic=(1, 1, 1), seed=81, n_cut=2.2e-3)
    return W.random_skew(n=(18, 16, 13), cell=((6.0, 0.0, 0.0), (2.3, 5.2, 0.0), (0.7, -0.6, 4.3)),
                         periodic=(1, 0, 1), seed=82, n_cut=2.2e-3, image_max=(1, 0, 1), r_cut=6.1)


def _grids(V, oracle, wl):
    return (V.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell, gradient="spectral"),
            oracle.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell, gradient="spectral"))


@pytest.mark.parametrize("k", range(3))
def test_spectral_gradient_and_q0(V, oracle, k):
    import torch

    wl = _case(k)
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    ref = oracle.compute_q0(og, wl.rho, wl.n_cut)
    grad = qd["grad"].cpu().numpy().reshape(3, -1)
    for a, key in enumerate(("gx", "gy", "gz")):
        assert np.abs(grad[a] - ref[key]).max() <= 1e-11 * np.abs(ref[key]).max(), key
    for key in ("q0", "dq_dn", "dq_dg"):
        assert np.abs(qd[key].cpu().numpy() - ref[key]).max() <= 1e-11 * np.abs(ref[key]).max(), key
    # the finite-difference gradient is a different operator
    fd = V.compute_q0(V.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell), n, wl.n_cut)
    assert float((fd["grad"] - qd["grad"]).abs().max()) > 1e-8


@pytest.mark.parametrize("k", range(3))
def test_spectral_energy_and_potential(V, oracle, table, k):
    import torch

    tp, tab = table
    wl = _case(k)
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    ref = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, wl.image_max, wl.r_cut, potential=True)
    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    gtab = V.Table(params, t64, t64.float().contiguous())
    for prec in (0, 1):
        etol, vtol = FP[prec]
        E, v = V.enl_potential(g, n, qd, gtab, V.Opts(n_cut=wl.n_cut, r_cut=wl.r_cut, image_max=wl.image_max,
                                                      precision=prec))
        v = v.cpu().numpy()
        rel_e = abs(sum(E) - ref.E) / abs(ref.E)
        rel_v = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
        say(f"spectral case {k} prec {prec}: dE={rel_e:.1e} dv={rel_v:.1e}")
        assert rel_e <= etol
        assert rel_v <= vtol
        # the dropped points next to kept ones get their share through the transposed operators
        drop = wl.rho.reshape(-1) < wl.n_cut
        if drop.any():
            assert np.abs(v[drop] - ref.dEdn[drop]).max() <= max(vtol, 1e-9) * np.abs(ref.dEdn).max()


@pytest.mark.parametrize("k", range(3))
def test_spectral_xc_energies(V, oracle, k):
    import torch

    wl = _case(k)
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    E = V.xc_energies(g, n, 1e-12)
    ref = oracle.xc_energies(og, wl.rho, 1e-12)
    for key in ref:
        assert E[key] == pytest.approx(ref[key], rel=1e-12), key


def test_spectral_in_batched_calls_and_plans(V, oracle, table):
    """A batch of a spectral and a finite-difference density (both periodic
    in x and y, one ring of images): the batched call, a potential plan
    replayed from its graph and an energy-only plan equal the oracle per
    density."""
    import torch

    tp, tab = table
    wls = [W.random_small(n=(20, 17, 12), h=(0.35, 0.4, 0.3), periodic=(1, 1, 0), seed=83, n_cut=2.2e-3),
           W.random_small(n=(14, 15, 13), h=(0.4, 0.35, 0.45), periodic=(1, 1, 0), seed=84, n_cut=2.2e-3)]
    kinds = ("spectral", "fd")
    grids = [V.Grid(w.n, w.h, w.periodic, gradient=k) for w, k in zip(wls, kinds)]
    refs = [oracle.evaluate(oracle.Grid(w.n, w.h, w.periodic, gradient=k), w.rho, tab, tp, w.n_cut, (1, 1, 0),
                            potential=True) for w, k in zip(wls, kinds)]
    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    gt = V.Table(params, t64, t64.float().contiguous())
    ns = [torch.tensor(w.rho.reshape(-1), dtype=torch.float64, device="cuda:0") for w in wls]
    npk, offs = V.pack_batch(grids, ns)

    def check(Eb, vb, etol, vtol, what):
        for b, ref in enumerate(refs):
            assert abs(sum(Eb[b]) - ref.E) <= etol * abs(ref.E), (what, b)
            if vb is not None:
                seg = vb[offs[b]:offs[b + 1]].cpu().numpy()
                assert np.linalg.norm(seg - ref.dEdn) <= vtol * np.linalg.norm(ref.dEdn), (what, b)

    qd = V.compute_q0_batched(grids, npk, offs, wls[0].n_cut)
    for prec in (0, 1):
        etol, vtol = FP[prec]
        say(f"spectral batch precision={prec}")
        Eb, vb = V.enl_potential_batched(grids, npk, offs, qd, gt, V.Opts(n_cut=wls[0].n_cut, image_max=(1, 1, 0),
                                                                         precision=prec))
        check(Eb, vb, etol, vtol, "batched")
    opts = V.Opts(n_cut=wls[0].n_cut, image_max=(1, 1, 0), precision=0)
    say("spectral plan (graph)")
    plan = V.BatchPlan(grids, offs, gt, opts)
    plan.capture(npk)
    for _ in range(2):
        plan.replay()
        torch.cuda.synchronize()
        check(plan.energies(), plan.dEdn, 1e-12, 1e-10, "plan")
    plan.close()
    say("spectral energy-only plan")
    plan = V.BatchPlan(grids, offs, gt, opts, potential=False)
    plan.capture(npk)
    plan.replay()
    torch.cuda.synchronize()
    check(plan.energies(), None, 1e-12, None, "energy plan")
    plan.close()
