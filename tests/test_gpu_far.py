"""GPU parity of the far image shell (the images beyond image_max up to
far_max with the kernel's large-D asymptote, folded into one lattice sum
per pair) against the oracle: energies and dE/dn element by element (FP64:
1e-12 / 1e-10, FP32C: 1e-6 / 1e-4 in the L2 norm) on cubic, orthorhombic
and skew cells periodic in one, two or three axes, with and without near
images; the energy-only call; and the Xe slab at full size (48 x 48 x 224,
two rings of near images and the shell out to eight cells, no distance
cut), dE/dn at sampled points."""
import numpy as np
import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
FP = {0: (1e-12, 1e-10), 1: (1e-6, 1e-4)}
CELL = ((6.0, 0.0, 0.0), (2.3, 5.2, 0.0), (0.7, -0.6, 4.3))


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
    for nS, nD, Dmax in ((16, 256, 16.0), (64, 2048, 48.0)):
        tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax, **CHEAP_RULE)
        out[nS] = (tp, oracle.build_table(tp))
    return out


def _gpu_table(V, tp, tab):
    import torch

    params = V.TableParams(n_D=tp.n_D, n_sigma=tp.n_sigma, D_max=tp.D_max, gl_points=tp.gl_points,
                           graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device="cuda:0").contiguous()
    return V.Table(params, t64, t64.float().contiguous())


CASES = [
    # name, workload, near image_max, far_max
    ("cubic-xy", lambda: W.random_small(n=(14, 12, 16), h=(0.4, 0.4, 0.4), periodic=(1, 1, 0), seed=81,
                                        n_cut=2.2e-3), (1, 1, 0), (4, 5, 0)),
    ("ortho-x-no-near", lambda: W.random_small(n=(13, 12, 15), h=(0.35, 0.4, 0.3), periodic=(1, 0, 0), seed=82,
                                               n_cut=2.2e-3), (0, 0, 0), (6, 0, 0)),
    ("skew-xyz", lambda: W.random_skew(n=(16, 13, 12), cell=CELL, periodic=(1, 1, 1), seed=83, n_cut=2.2e-3),
     (1, 0, 1), (2, 2, 2)),
]


def _grids(V, oracle, wl):
    if wl.cell is not None:
        return V.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell), oracle.grid_of_cell(wl.n, wl.cell, wl.periodic)
    return V.Grid(wl.n, wl.h, wl.periodic), oracle.Grid(wl.n, wl.h, wl.periodic)


@pytest.mark.parametrize("nS", [16, 64])
@pytest.mark.parametrize("c", range(len(CASES)))
def test_far_shell_energy_and_potential(V, oracle, tables, c, nS):
    import torch

    name, make, near, far = CASES[c]
    wl = make()
    tp, tab = tables[nS]
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    ref = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, near, potential=True, far_max=far)
    base = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, near)
    assert abs(ref.E_pairL - base.E_pairL) > 1e-4 * abs(ref.E)  # the shell matters at this tolerance
    table = _gpu_table(V, tp, tab)
    for prec in (0, 1):
        etol, vtol = FP[prec]
        opts = V.Opts(n_cut=wl.n_cut, image_max=near, far_max=far, precision=prec)
        E, v = V.enl_potential(g, n, qd, table, opts)
        v = v.cpu().numpy()
        st = V.last_stats()
        rel_e = abs(sum(E) - ref.E) / abs(ref.E)
        rel_v = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
        say(f"far {name} nS {nS} prec {prec}: N={st['retained']} far_pairs={st['far_pairs']:.3g} "
            f"dE={rel_e:.1e} dv={rel_v:.1e}")
        assert st["retained"] > 2048 and st["far_pairs"] == float(st["retained"]) ** 2
        assert rel_e <= etol
        for a, b in ((E[0], ref.E_pair0), (E[1], ref.E_pairL), (E[2], ref.E_self)):
            assert abs(a - b) <= etol * abs(ref.E)
        assert rel_v <= vtol
        Ee = V.enl_energy(g, n, qd["q0"], table, opts)
        assert abs(sum(Ee) - sum(E)) <= 1e-12 * abs(sum(E))


def test_far_shell_matches_the_near_sum_it_replaces(V, oracle):
    """With a table whose D_max lies below every D of the shell, the GPU's
    near sum out to far_max equals its near sum to image_max plus the shell."""
    import torch

    wl = W.random_small(n=(12, 10, 9), h=(0.5, 0.6, 0.45), periodic=(1, 1, 0), seed=84, n_cut=1e-4)
    g, og = _grids(V, oracle, wl)
    Dmax = 1.0
    tp = oracle.table_params(n_D=9, n_sigma=5, D_max=Dmax)
    Dk = np.arange(9) * Dmax / 8
    sl = np.arange(5) / 4
    tab = 0.3 - 0.2 * Dk[:, None] + 0.9 * sl[None, :] + 0.1 * Dk[:, None] * sl[None, :]
    qd0 = oracle.compute_q0(og, wl.rho, wl.n_cut)
    qmin = qd0["q0"][qd0["keep"]].min()
    # nearest far image: two cells away along x or y, less the cell's extent
    assert qmin * min(2 * 12 * 0.5 - 11 * 0.5, 2 * 10 * 0.6 - 9 * 0.6) > Dmax
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    table = _gpu_table(V, tp, tab)
    full, vf = V.enl_potential(g, n, qd, table, V.Opts(n_cut=wl.n_cut, image_max=(3, 3, 0), precision=0))
    split, vs = V.enl_potential(g, n, qd, table, V.Opts(n_cut=wl.n_cut, image_max=(1, 1, 0), far_max=(3, 3, 0),
                                                        precision=0))
    assert sum(split) == pytest.approx(sum(full), rel=1e-12)
    assert split[1] == pytest.approx(full[1], rel=1e-12)
    vf, vs = vf.cpu().numpy(), vs.cpu().numpy()
    assert np.abs(vs - vf).max() <= 1e-10 * np.abs(vf).max()


@pytest.mark.parametrize("prec,vtol", [(1, 1e-4), (0, 1e-10)])
def test_far_shell_slab_full_size_sampled_potential(V, oracle, tables, prec, vtol):
    """Xe slab 48 x 48 x 224 (periodic in x and y), images |m|, |n| <= 2 with
    the table and the shell out to 8 cells with the asymptote, no cut:
    dE/dn at sampled points against the oracle's rows for them."""
    import torch

    tp, tab = tables[64]
    wl = W.xe_slab()
    g, og = _grids(V, oracle, wl)
    near, far = (2, 2, 0), (8, 8, 0)
    say(f"far slab full size precision={prec}")
    rng = np.random.default_rng(12)
    rho = wl.rho.reshape(-1)
    keep = np.flatnonzero(rho >= wl.n_cut)
    ks = np.array(sorted(set(int(k) for k in list(rng.choice(keep, 16, replace=False)) + list(np.argsort(rho)[-3:]))))
    n = torch.tensor(rho, dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    opts = V.Opts(n_cut=wl.n_cut, image_max=near, far_max=far, precision=prec)
    E, v = V.enl_potential(g, n, qd, _gpu_table(V, tp, tab), opts)
    v = v.cpu().numpy()
    say(f"  GPU E = {sum(E):.12e} (pairL {E[1]:.6e}; {V.last_stats()['retained']} kept points)")
    ref = oracle.potential_at(og, wl.rho, ks, tab, tp, wl.n_cut, near, far_max=far)
    rel = np.linalg.norm(v[ks] - ref) / np.linalg.norm(ref)
    say(f"  sampled |dv|/|v| over {len(ks)} points = {rel:.3e}")
    assert rel <= vtol
    assert E[1] < 0


def test_far_shell_approximation_on_the_slab(V):
    """Xe slab at full size, energies only (FP32C): the shell's asymptote in
    place of the table for rings 3-4 moves E_pairL by less than 1e-5 of
    itself, under 1 % of what those rings contribute; the paper's setting
    (three rings, r <= 30 bohr) and the shell out to 32 rings are printed."""
    import torch

    wl = W.xe_slab()
    dev = torch.device("cuda:0")
    table = V.build_phi_table(V.TableParams(n_D=2048, n_sigma=64, D_max=48.0), device=dev)
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device=dev)
    q0 = V.compute_q0(g, n, wl.n_cut)["q0"]

    def e(near, far=(0, 0, 0), r_cut=0.0):
        E = V.enl_energy(g, n, q0, table, V.Opts(n_cut=wl.n_cut, image_max=near, far_max=far, r_cut=r_cut))
        say(f"  near {near} far {far} r_cut {r_cut}: E_pairL = {E[1]:.10e}  E = {sum(E):.10e}")
        return E

    exact4 = e((4, 4, 0))
    near2 = e((2, 2, 0))
    far4 = e((2, 2, 0), (4, 4, 0))
    e((1, 1, 0), (4, 4, 0))  # one near ring: printed for the record
    e((2, 2, 0), (32, 32, 0))
    e((3, 3, 0), r_cut=30.0)
    assert abs(far4[1] - exact4[1]) <= 1e-5 * abs(exact4[1])
    assert abs(far4[1] - exact4[1]) <= 1e-2 * abs(near2[1] - exact4[1])
    assert far4[0] == exact4[0] and far4[2] == exact4[2]


def test_far_shell_in_a_graph_plan(V, oracle, tables):
    """A one-density plan with the far shell, recorded as a HIP graph: three
    replays (eager calls in between) equal each other bit for bit and equal
    the oracle."""
    import torch

    name, make, near, far = CASES[0]
    wl = make()
    tp, tab = tables[16]
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    table = _gpu_table(V, tp, tab)
    opts = V.Opts(n_cut=wl.n_cut, image_max=near, far_max=far, precision=0)
    ref = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, near, potential=True, far_max=far)
    plan = V.BatchPlan([g], [0, wl.G], table, opts)
    plan.capture(n)
    first = None
    for r in range(3):
        plan.replay()
        torch.cuda.synchronize()
        E_r, v_r = plan.energies()[0], plan.dEdn.clone()
        qd = V.compute_q0(g, n, wl.n_cut)
        E_e, v_e = V.enl_potential(g, n, qd, table, opts)
        torch.cuda.synchronize()
        assert sum(E_r) == pytest.approx(ref.E, rel=1e-12)
        assert sum(E_r) == pytest.approx(sum(E_e), rel=1e-14)
        assert np.linalg.norm(v_r.cpu().numpy() - ref.dEdn) <= 1e-10 * np.linalg.norm(ref.dEdn)
        if first is None:
            first = (E_r, v_r)
        else:
            assert E_r == first[0] and torch.equal(v_r, first[1])
    plan.close()


def test_far_shell_in_batches(V, oracle, tables):
    """Two periodic densities of different grids and cells (orthorhombic and
    skew) with the shell: the batched call (FP64 and FP32C) and a graph plan
    equal the oracle per density."""
    import torch

    tp, tab = tables[64]
    table = _gpu_table(V, tp, tab)
    wls = [W.random_small(n=(14, 12, 16), h=(0.4, 0.4, 0.4), periodic=(1, 1, 0), seed=86, n_cut=2.2e-3),
           W.random_skew(n=(13, 15, 11), cell=CELL, periodic=(1, 1, 0), seed=87, n_cut=2.2e-3)]
    near, far = (1, 1, 0), (3, 4, 0)
    pairs = [_grids(V, oracle, w) for w in wls]
    grids = [p[0] for p in pairs]
    refs = [oracle.evaluate(og, w.rho, tab, tp, w.n_cut, near, potential=True, far_max=far)
            for (_, og), w in zip(pairs, wls)]
    ns = [torch.tensor(w.rho.reshape(-1), dtype=torch.float64, device="cuda:0") for w in wls]
    npk, offs = V.pack_batch(grids, ns)

    def check(Eb, vb, etol, vtol, what):
        for b, ref in enumerate(refs):
            assert abs(sum(Eb[b]) - ref.E) <= etol * abs(ref.E), (what, b)
            assert abs(Eb[b][1] - ref.E_pairL) <= etol * abs(ref.E), (what, b)
            seg = vb[offs[b]:offs[b + 1]].cpu().numpy()
            assert np.linalg.norm(seg - ref.dEdn) <= vtol * np.linalg.norm(ref.dEdn), (what, b)

    qd = V.compute_q0_batched(grids, npk, offs, wls[0].n_cut)
    for prec in (0, 1):
        etol, vtol = FP[prec]
        say(f"far batch precision={prec}")
        opts = V.Opts(n_cut=wls[0].n_cut, image_max=near, far_max=far, precision=prec)
        Eb, vb = V.enl_potential_batched(grids, npk, offs, qd, table, opts)
        st = V.last_stats()
        assert st["far_pairs"] == pytest.approx(sum(float(r.q0["keep"].sum()) ** 2 for r in refs))
        check(Eb, vb, etol, vtol, "batched")
    say("far batch plan (graph)")
    plan = V.BatchPlan(grids, offs, table, V.Opts(n_cut=wls[0].n_cut, image_max=near, far_max=far, precision=0))
    plan.capture(npk)
    plan.replay()
    torch.cuda.synchronize()
    check(plan.energies(), plan.dEdn, 1e-12, 1e-10, "plan")
    plan.close()


def test_far_shell_edge_cases(V, oracle, tables):
    """Nothing kept: all zero.  One kept point: its only pair terms are its
    own far images, -C T(0) / (2 q^6) per unit n^2.  Two runs agree bit for
    bit."""
    import torch

    tp, tab = tables[16]
    table = _gpu_table(V, tp, tab)
    wl = W.random_small(n=(9, 8, 7), h=(0.4, 0.45, 0.5), periodic=(1, 1, 0), seed=85, n_cut=2.2e-3)
    g, og = _grids(V, oracle, wl)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")

    def run(n_cut, prec=0):
        qd = V.compute_q0(g, n, n_cut)
        E, v = V.enl_potential(g, n, qd, table, V.Opts(n_cut=n_cut, image_max=(1, 1, 0), far_max=(5, 5, 0),
                                                       precision=prec))
        return E, v.cpu().numpy()

    say("far edge: empty retained set")
    E, v = run(1e6)
    assert E == (0.0, 0.0, 0.0) and np.all(v == 0) and V.last_stats()["far_pairs"] == 0.0
    say("far edge: one retained point")
    top = float(wl.rho.max())
    E, v = run(top)
    ref = oracle.evaluate(og, wl.rho, tab, tp, top, (1, 1, 0), potential=True, far_max=(5, 5, 0))
    assert V.last_stats()["retained"] == 1
    assert E[0] == 0.0
    assert E[1] == pytest.approx(ref.E_pairL, rel=1e-13) and E[1] < 0
    assert np.linalg.norm(v - ref.dEdn) <= 1e-12 * np.linalg.norm(ref.dEdn)
    say("far edge: determinism")
    for prec in (0, 1):
        a, va = run(wl.n_cut, prec)
        b, vb = run(wl.n_cut, prec)
        assert a == b and np.array_equal(va, vb)
    say("far edge: Kahan-compensated FP32 runs")
    qd = V.compute_q0(g, n, wl.n_cut)
    E, v = V.enl_potential(g, n, qd, table, V.Opts(n_cut=wl.n_cut, image_max=(1, 1, 0), far_max=(5, 5, 0),
                                                   precision=1, kahan=1))
    ref = oracle.evaluate(og, wl.rho, tab, tp, wl.n_cut, (1, 1, 0), potential=True, far_max=(5, 5, 0))
    assert abs(sum(E) - ref.E) <= 1e-6 * abs(ref.E)
    assert np.linalg.norm(v.cpu().numpy() - ref.dEdn) <= 1e-4 * np.linalg.norm(ref.dEdn)
