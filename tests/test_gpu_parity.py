"""GPU parity: the HIP library, called through its C ABI, against the FP64
oracle on the same seeded inputs.

Tolerances (relative): energies 1e-12 (FP64 form) and 1e-6 (FP32C form);
dE/dn in L2 norm 1e-10 (FP64) and 1e-4 (FP32C); the table builder 1e-12 of
the table's scale.  Tables passed to the pair kernels are built by the
oracle, so a pair-sum comparison never depends on the GPU table builder.
"""
import math

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
def dev(V):
    import torch

    return torch.device("cuda:0")


def _gpu_table(V, dev, tp_o, tab):
    import torch

    params = V.TableParams(n_D=tp_o.n_D, n_sigma=tp_o.n_sigma, D_max=tp_o.D_max, gl_points=tp_o.gl_points,
                           graded_levels=tp_o.graded_levels, kappa=tp_o.kappa, A0=tp_o.A0)
    t64 = torch.tensor(tab, dtype=torch.float64, device=dev).contiguous()
    return V.Table(params, t64, t64.float().contiguous())


def _run(V, dev, wl, table, prec, potential=True, **kw):
    import torch

    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device=dev)
    opts = V.Opts(n_cut=wl.n_cut, r_cut=wl.r_cut, image_max=wl.image_max, precision=prec, **kw)
    qd = V.compute_q0(g, n, wl.n_cut)
    if potential:
        E, v = V.enl_potential(g, n, qd, table, opts)
        return E, v.cpu().numpy()
    return V.enl_energy(g, n, qd["q0"], table, opts), None


def _check(E, v, ref, etol, vtol, what):
    Eg = sum(E)
    say(f"  {what}: E_gpu={Eg:.15e} E_ref={ref.E:.15e} rel={abs(Eg - ref.E) / abs(ref.E):.2e}")
    assert abs(Eg - ref.E) <= etol * abs(ref.E)
    for a, b in ((E[0], ref.E_pair0), (E[1], ref.E_pairL), (E[2], ref.E_self)):
        assert abs(a - b) <= etol * abs(ref.E) + 1e-300
    if v is not None:
        rel = np.linalg.norm(v - ref.dEdn) / np.linalg.norm(ref.dEdn)
        say(f"  {what}: |dv|/|v| = {rel:.2e}")
        assert rel <= vtol


# ---------------------------------------------------------------------------


def test_table_builder_small_full(V, dev, oracle):
    say("table builder 128 x 16, cheap rule")
    tp = oracle.table_params(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    ref = oracle.build_table(tp)
    t = V.build_phi_table(V.TableParams(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE), device=dev)
    got = t.phi64.cpu().numpy()
    err = np.abs(got - ref).max()
    say(f"  max abs err {err:.2e}, scale {np.abs(ref).max():.3f}")
    assert err <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(t.phi32.cpu().numpy(), got.astype(np.float32))


@pytest.mark.parametrize("shape", [(1024, 32), (2048, 64)])
def test_table_builder_default_rule_sampled(V, dev, oracle, shape):
    """The default rule at the workload table sizes, on sampled nodes (all of
    rows 0, 1, 2 and the last row, plus random nodes)."""
    nD, nS = shape
    say(f"table builder {nD} x {nS}, default rule (sampled nodes)")
    t = V.build_phi_table(V.TableParams(n_D=nD, n_sigma=nS, D_max=48.0), device=dev)
    got = t.phi64.cpu().numpy()
    rng = np.random.default_rng(nD)
    ks = np.concatenate([np.repeat([0, 1, 2, nD - 1], nS), rng.integers(0, nD, 48)])
    ls = np.concatenate([np.tile(np.arange(nS), 4), rng.integers(0, nS, 48)])
    ref = oracle.table_nodes(oracle.table_params(n_D=nD, n_sigma=nS, D_max=48.0), ks, ls)
    err = np.abs(got[ks, ls] - ref)
    say(f"  max abs err {err.max():.2e}")
    assert np.all(err <= 1e-12 * np.maximum(np.abs(ref), 1e-3))


@pytest.mark.parametrize("case", ["dimer_small", "periodic_xy", "periodic_xyz"])
def test_compute_q0_matches_oracle(V, dev, oracle, case):
    import torch

    say(f"compute_q0 {case}")
    if case == "dimer_small":
        wl = W.dimer_small()
    elif case == "periodic_xy":
        wl = W.scaled_slab(nxy=12, nz=40)
    else:
        wl = W.random_small(n=(5, 7, 6), periodic=(1, 1, 1), seed=4)
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device=dev)
    qd = V.compute_q0(g, n, wl.n_cut)
    ref = oracle.compute_q0(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, wl.n_cut)
    G = g.G
    grad = qd["grad"].cpu().numpy()
    for a, comp in enumerate(("gx", "gy", "gz")):
        assert np.allclose(grad[a * G:(a + 1) * G], ref[comp], rtol=1e-13, atol=1e-13 * np.abs(ref[comp]).max())
    for key in ("q0", "dq_dg"):
        got = qd[key].cpu().numpy()
        assert np.allclose(got, ref[key], rtol=1e-13, atol=0), key
    # dq0/dn sums three terms of opposite sign; compare against their scale
    keep = ref["keep"]
    nn = wl.rho.reshape(-1)[keep]
    kF = np.cbrt(3 * np.pi ** 2 * nn)
    scale = kF / (3 * nn) + np.abs(7 * 0.8491 * ref["g"][keep] / (108 * kF * nn ** 3)) + 1.0 / nn
    got = qd["dq_dn"].cpu().numpy()
    assert np.all(np.abs(got[keep] - ref["dq_dn"][keep]) <= 1e-13 * scale)
    assert np.all(got[~keep] == 0)


@pytest.fixture(scope="module")
def small_table(oracle):
    tp = oracle.table_params(n_D=256, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    return tp, oracle.build_table(tp)


@pytest.fixture(scope="module")
def big_table(oracle):
    tp = oracle.table_params(n_D=2048, n_sigma=64, D_max=48.0, **CHEAP_RULE)
    return tp, oracle.build_table(tp)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("case", ["tiny", "ragged_periodic", "images_cut", "all_periodic"])
def test_small_cases_energy_and_potential(V, dev, oracle, small_table, case, prec):
    tp, tab = small_table
    p, etol, vtol = FP[prec]
    if case == "tiny":
        wl = W.random_small(n=(6, 5, 7), seed=1, n_cut=2.5e-3)
    elif case == "ragged_periodic":
        wl = W.random_small(n=(13, 11, 9), periodic=(1, 0, 0), seed=2, n_cut=3e-3, image_max=(2, 0, 0))
    elif case == "images_cut":
        wl = W.random_small(n=(8, 8, 10), periodic=(1, 1, 0), seed=3, n_cut=2e-3, image_max=(2, 2, 0), r_cut=4.17)
    else:
        wl = W.random_small(n=(5, 6, 7), periodic=(1, 1, 1), seed=5, n_cut=1e-3, image_max=(1, 1, 1))
    say(f"{case} {prec}: grid {wl.n} images {wl.image_max} r_cut {wl.r_cut}")
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, wl.image_max, wl.r_cut,
                          potential=True)
    table = _gpu_table(V, dev, tp, tab)
    E, v = _run(V, dev, wl, table, p)
    _check(E, v, ref, etol, vtol, case)
    E2, _ = _run(V, dev, wl, table, p, potential=False)
    assert sum(E2) == pytest.approx(sum(E), rel=1e-13 if p == 0 else 1e-7)  # energy-only kernel


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_dimer_small_full_parity(V, dev, oracle, table_cache, prec):
    """The 24^3 dimer (13 824 points, all kept) with the 1024 x 32 table of the
    default rule; energy and potential at every grid point."""
    say(f"dimer_small {prec}")
    tp, tab = table_cache(n_D=1024, n_sigma=32, D_max=48.0)
    wl = W.dimer_small()
    p, etol, vtol = FP[prec]
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h), wl.rho, tab, tp, wl.n_cut, potential=True)
    E, v = _run(V, dev, wl, _gpu_table(V, dev, tp, tab), p)
    _check(E, v, ref, etol, vtol, "dimer_small")
    st = V.last_stats()
    assert st["retained"] == 13824 and st["pairs"] == 13824 * 13823


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_multi_tile_dimer_parity(V, dev, oracle, big_table, prec):
    """A dimer on 30^3 (several 1024-point i-blocks, ragged last block, many
    j-chunks) with the 2048 x 64 table; LDS rows limited so both table
    sources are exercised."""
    tp, tab = big_table
    wl = W.scaled_dimer(edge=30, h=0.4, R=5.0)
    p, etol, vtol = FP[prec]
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h), wl.rho, tab, tp, wl.n_cut, potential=True)
    for rows in (-1, 40):
        say(f"scaled dimer {prec} lds_rows={rows}")
        E, v = _run(V, dev, wl, _gpu_table(V, dev, tp, tab), p, table_lds_rows=rows)
        _check(E, v, ref, etol, vtol, f"dimer30 rows={rows}")
    assert V.last_stats()["retained"] % 1024 != 0


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_slab_images_parity(V, dev, oracle, big_table, prec):
    """The Xe-slab shape on a coarse 12 x 12 x 40 grid, images |m|, |p| <= 3 and
    the 30 bohr cut; with all LDS rows and with 40 (then most pairs take the
    global-table pass)."""
    tp, tab = big_table
    wl = W.scaled_slab(nxy=12, nz=40)
    p, etol, vtol = FP[prec]
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, wl.image_max, wl.r_cut,
                          potential=True)
    for rows in (-1, 40):
        say(f"slab 12x12x40 {prec} lds_rows={rows}")
        E, v = _run(V, dev, wl, _gpu_table(V, dev, tp, tab), p, table_lds_rows=rows)
        _check(E, v, ref, etol, vtol, f"slab rows={rows}")
        assert abs(E[1]) > 0


def test_edge_cases(V, dev, oracle, small_table):
    tp, tab = small_table
    table = _gpu_table(V, dev, tp, tab)
    # nothing kept
    wl = W.random_small(seed=1)
    wl.n_cut = 1e6
    say("edge: empty retained set")
    E, v = _run(V, dev, wl, table, 0)
    assert E == (0.0, 0.0, 0.0) and np.all(v == 0)
    # one kept point: no pairs, only the on-site term
    wl = W.random_small(seed=1)
    wl.n_cut = float(wl.rho.max())
    say("edge: one retained point")
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h), wl.rho, tab, tp, wl.n_cut, potential=True)
    E, v = _run(V, dev, wl, table, 0)
    assert E[0] == 0.0 and E[1] == 0.0 and abs(E[2] - ref.E_self) <= 1e-13 * abs(ref.E_self)
    assert np.linalg.norm(v - ref.dEdn) <= 1e-12 * np.linalg.norm(ref.dEdn)
    # smallest grid, self term off
    wl = W.random_small(n=(3, 3, 3), seed=2, n_cut=1e-4)
    say("edge: 3x3x3 grid, no self term")
    ref = oracle.evaluate(oracle.Grid(wl.n, wl.h), wl.rho, tab, tp, wl.n_cut, self_term=False, potential=True)
    E, v = _run(V, dev, wl, table, 0, self_term=0)
    _check(E, v, ref, 1e-12, 1e-10, "3^3")


def test_nonfinite_density_is_reported(V, dev, small_table):
    import torch

    tp, tab = small_table
    table = _gpu_table(V, dev, tp, tab)
    wl = W.random_small(seed=1)
    g = V.Grid(wl.n, wl.h)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device=dev)
    q = V.compute_q0(g, n, wl.n_cut)["q0"]
    n[5] = float("nan")
    say("edge: NaN in the density")
    with pytest.raises(V.VdwError) as e:
        V.enl_energy(g, n, q, table, V.Opts(n_cut=wl.n_cut, precision=0))
    assert e.value.code == -6


def test_deterministic_bitwise(V, dev, small_table):
    tp, tab = small_table
    table = _gpu_table(V, dev, tp, tab)
    wl = W.random_small(n=(12, 12, 12), seed=6, n_cut=2e-3)
    say("determinism")
    for p in (0, 1):
        E1, v1 = _run(V, dev, wl, table, p)
        E2, v2 = _run(V, dev, wl, table, p)
        assert E1 == E2 and np.array_equal(v1, v2)


def test_autograd_matches_potential_and_fd(V, dev, small_table):
    import torch

    tp, tab = small_table
    table = _gpu_table(V, dev, tp, tab)
    wl = W.random_small(n=(9, 8, 7), seed=8, n_cut=2e-3)
    g = V.Grid(wl.n, wl.h)
    say("autograd")
    opts = V.Opts(n_cut=wl.n_cut, precision=0)
    n = torch.tensor(wl.rho, dtype=torch.float64, device=dev, requires_grad=True)
    E = V.energy(n, g, table, opts)
    E.backward()
    grad = n.grad.reshape(-1).cpu().numpy()
    qd = V.compute_q0(g, n.detach().reshape(-1).contiguous(), wl.n_cut)
    _, v = V.enl_potential(g, n.detach().reshape(-1).contiguous(), qd, table, opts)
    assert np.array_equal(grad, v.cpu().numpy())
    rho = wl.rho.reshape(-1)
    rng = np.random.default_rng(0)
    for k in rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 6, replace=False):
        eps = 1e-5 * rho[k]
        vals = []
        for s in (1, -1):
            m = torch.tensor(rho, dtype=torch.float64, device=dev)
            m[k] += s * eps
            vals.append(float(V.energy(m, g, table, opts)))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert fd == pytest.approx(grad[k], rel=2e-4, abs=1e-9 * np.abs(grad).max())
