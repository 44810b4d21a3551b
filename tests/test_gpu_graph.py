"""Batch plans and HIP-graph replay of the batched evaluation.

A plan's execute launches kernels only (q0 of every density in one launch,
then the same pipeline as enl_potential_batched), so it must agree with the
batched call; a recorded graph must give the eager result on every replay,
with other GPU work and host synchronisations between replays, and follow a
density rewritten in place.  One direct check against the oracle covers the
batched q0 kernel on periodic grids with images.
"""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)


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


def _gpu_table(V, tp, tab):
    import torch

    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    return V.Table(params, t64, t64.float().contiguous())


def _packed(V, mols):
    import torch

    grids = [V.Grid(m.n, m.h, m.periodic) for m in mols]
    ns = [torch.tensor(m.rho.reshape(-1), dtype=torch.float64, device="cuda:0") for m in mols]
    n, offs = V.pack_batch(grids, ns)
    return grids, n, offs


def _eager(V, grids, n, offs, table, opts):
    qd = V.compute_q0_batched(grids, n, offs, opts.n_cut)
    E, v = V.enl_potential_batched(grids, n, offs, qd, table, opts)
    return E, v, qd


def _close(Ea, Eb, rel):
    for a, b in zip(Ea, Eb):
        assert sum(a) == pytest.approx(sum(b), rel=rel, abs=1e-300)


@pytest.mark.parametrize("prec", [1, 0])
def test_plan_execute_matches_batched_call(V, big, prec):
    """64 molecules: execute (q0 inside, one launch for all densities) equals
    compute_q0 per density + enl_potential_batched."""
    import torch

    tp, tab = big
    table = _gpu_table(V, tp, tab)
    mols = W.molecule_batch(64)
    grids, n, offs = _packed(V, mols)
    opts = V.Opts(n_cut=mols[0].n_cut, precision=prec)
    say(f"plan execute vs batched call, 64 molecules, precision={prec}")
    Eb, vb, qd = _eager(V, grids, n, offs, table, opts)
    plan = V.BatchPlan(grids, offs, table, opts)
    plan.execute(n)
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(plan.q0 - qd["q0"]) / torch.clamp(torch.abs(qd["q0"]), min=1e-300))) <= 1e-14
    assert float(torch.max(torch.abs(plan.grad - qd["grad"]))) <= 1e-12 * float(torch.max(torch.abs(qd["grad"])))
    _close(plan.energies(), Eb, 1e-12)
    assert float(torch.linalg.norm(plan.dEdn - vb) / torch.linalg.norm(vb)) <= 1e-12
    assert sum(plan.retained()) == sum(int((n[offs[b]:offs[b + 1]] >= mols[0].n_cut).sum()) for b in range(64))
    plan.close()


def test_graph_replays_match_eager(V, big):
    """Record once, replay three times with eager evaluations and host
    synchronisations in between: every replay equals the first bit for bit
    and the eager result to rounding; then the density is rescaled in place
    and the next replay follows it."""
    import torch

    tp, tab = big
    table = _gpu_table(V, tp, tab)
    mols = W.molecule_batch(64)
    grids, n, offs = _packed(V, mols)
    opts = V.Opts(n_cut=mols[0].n_cut, precision=1)
    plan = V.BatchPlan(grids, offs, table, opts)
    say("capturing the batched evaluation into a HIP graph")
    plan.capture(n)
    first = None
    for r in range(3):
        say(f"  replay {r}")
        plan.replay()
        torch.cuda.synchronize()
        E_r, v_r = plan.energies(), plan.dEdn.clone()
        Eb, vb, _ = _eager(V, grids, n, offs, table, opts)
        torch.cuda.synchronize()
        _close(E_r, Eb, 1e-12)
        assert float(torch.linalg.norm(v_r - vb) / torch.linalg.norm(vb)) <= 1e-12
        if first is None:
            first = (E_r, v_r)
        else:
            assert E_r == first[0]
            assert torch.equal(v_r, first[1])
    n.mul_(1.05)  # a new density in the same buffer
    torch.cuda.synchronize()
    say("  replay after rescaling the density")
    plan.replay()
    torch.cuda.synchronize()
    E_s = plan.energies()
    Eb, vb, _ = _eager(V, grids, n, offs, table, opts)
    _close(E_s, Eb, 1e-12)
    assert float(torch.linalg.norm(plan.dEdn - vb) / torch.linalg.norm(vb)) <= 1e-12
    assert sum(map(sum, E_s)) != sum(map(sum, first[0]))
    plan.close()


def test_energy_only_plan(V, big):
    """potential=0: no derivative buffers, energies equal enl_energy."""
    import torch

    tp, tab = big
    table = _gpu_table(V, tp, tab)
    wl = W.kr_dimer(7.0)
    grids, n, offs = _packed(V, [wl])
    opts = V.Opts(n_cut=wl.n_cut, precision=1)
    plan = V.BatchPlan(grids, offs, table, opts, potential=False)
    assert plan.dEdn is None and plan.grad is None
    say("energy-only plan on the 96^3 dimer (graph)")
    plan.capture(n)
    plan.replay()
    torch.cuda.synchronize()
    Ep = plan.energies()[0]
    qd = V.compute_q0(grids[0], n, wl.n_cut, derivatives=False)
    Ee = V.enl_energy(grids[0], n, qd["q0"], table, opts)
    assert sum(Ep) == pytest.approx(sum(Ee), rel=1e-12)
    plan.close()


def test_plan_on_periodic_slabs_matches_oracle(V, oracle):
    """Two slab densities (periodic x, y, images |m|, |p| <= 3, 30 bohr cut)
    in one plan against the oracle, FP64 and FP32C."""
    import torch

    tp = oracle.table_params(n_D=512, n_sigma=32, D_max=48.0, **CHEAP_RULE)
    tab = oracle.build_table(tp)
    table = _gpu_table(V, tp, tab)
    mols = [W.scaled_slab(seed=3), W.scaled_slab(nxy=10, nz=36, seed=4)]
    grids, n, offs = _packed(V, mols)
    refs = [oracle.evaluate(oracle.Grid(m.n, m.h, m.periodic), m.rho, tab, tp, m.n_cut, image_max=m.image_max,
                            r_cut=m.r_cut, potential=True) for m in mols]
    for prec, etol, vtol in ((0, 1e-12, 1e-10), (1, 1e-6, 1e-4)):
        say(f"slab plan vs oracle precision={prec}")
        opts = V.Opts(n_cut=mols[0].n_cut, r_cut=mols[0].r_cut, image_max=mols[0].image_max, precision=prec)
        plan = V.BatchPlan(grids, offs, table, opts)
        plan.capture(n)
        plan.replay()
        torch.cuda.synchronize()
        E = plan.energies()
        v = plan.dEdn.cpu().numpy()
        for b, ref in enumerate(refs):
            assert abs(sum(E[b]) - ref.E) <= etol * abs(ref.E), (b, sum(E[b]), ref.E)
            assert E[b][1] < 0
            vb = v[offs[b]:offs[b + 1]]
            assert np.linalg.norm(vb - ref.dEdn) <= vtol * np.linalg.norm(ref.dEdn), b
        plan.close()


def test_plan_errors(V, big):
    """Host-side errors: replay before capture, a density of the wrong size,
    offsets that do not match the grids."""
    import torch

    tp, tab = big
    table = _gpu_table(V, tp, tab)
    mols = W.molecule_batch(4)
    grids, n, offs = _packed(V, mols)
    opts = V.Opts(n_cut=mols[0].n_cut)
    plan = V.BatchPlan(grids, offs, table, opts)
    with pytest.raises(V.VdwError, match="no captured graph"):
        plan.replay()
    with pytest.raises(ValueError):
        plan.execute(n[:-1].contiguous())
    bad = list(offs)
    bad[1] += 1
    with pytest.raises(V.VdwError):
        V.BatchPlan(grids, bad, table, opts)
    plan.close()
    torch.cuda.synchronize()
