"""The boundary on the GPU: calls on different streams from different host
threads (the binding gives each (device, stream) its own workspace, as the C
ABI requires), a caller-provided workspace, and the image-window fields of
vdw_stats (Sec. 3 periodic repetition; Sec. 7 far cells) against the
oracle's q0 and the host geometry."""
import threading

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
def table(V):
    return V.build_phi_table(V.TableParams(n_D=512, n_sigma=64, D_max=24.0, **CHEAP_RULE), device="cuda:0")


def test_concurrent_streams_from_two_threads(V, table):
    """Two densities evaluated at the same time on two streams from two host
    threads equal their serial evaluations bitwise, and the two streams got
    workspaces of their own."""
    import torch

    from paper_0810_2273_amd import api

    wls = [W.scaled_dimer(edge=32, h=0.4, R=5.0), W.scaled_dimer(edge=32, h=0.4, R=6.5, seed=4)]
    grids = [V.Grid(w.n, w.h, w.periodic) for w in wls]
    ns = [torch.tensor(w.rho.reshape(-1), dtype=torch.float64, device="cuda:0") for w in wls]
    opts = [V.Opts(n_cut=w.n_cut, precision=1) for w in wls]
    qds = [V.compute_q0(g, n, w.n_cut) for g, n, w in zip(grids, ns, wls)]
    serial = [V.enl_potential(g, n, qd, table, o) for g, n, qd, o in zip(grids, ns, qds, opts)]
    serial = [(E, v.cpu().numpy()) for E, v in serial]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]
    errors = []

    def work(k):
        try:
            with torch.cuda.stream(streams[k]):
                for _ in range(3):
                    E, v = V.enl_potential(grids[k], ns[k], qds[k], table, opts[k], stream=streams[k])
                streams[k].synchronize()
                out[k] = (E, v.cpu().numpy())
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        say(f"  stream {k}: E = {out[k][0]}")
        assert tuple(out[k][0]) == tuple(serial[k][0])
        assert np.array_equal(out[k][1], serial[k][1])
    keys = {key for key in api._WS if key[1] in (streams[0].cuda_stream, streams[1].cuda_stream)}
    assert len(keys) == 2


def test_caller_workspace(V, table):
    import torch

    from paper_0810_2273_amd import _lib as L

    wl = W.scaled_dimer(edge=24, h=0.4, R=5.0)
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    qd = V.compute_q0(g, n, wl.n_cut)
    o = V.Opts(n_cut=wl.n_cut, precision=0)
    nbytes = V.enl_workspace_size(g, table, o)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    E1, v1 = V.enl_potential(g, n, qd, table, o, ws=ws)
    E2, v2 = V.enl_potential(g, n, qd, table, o)
    assert tuple(E1) == tuple(E2) and torch.equal(v1, v2)
    assert V.enl_energy(g, n, qd["q0"], table, o, ws=ws) == tuple(E1)
    with pytest.raises(L.VdwError):
        V.enl_potential(g, n, qd, table, o, ws=ws[: nbytes // 2])
    # the cached workspaces can be dropped; the next call allocates again
    from paper_0810_2273_amd import api

    V.release_workspaces()
    assert not api._WS
    E3, v3 = V.enl_potential(g, n, qd, table, o)
    assert tuple(E3) == tuple(E1) and torch.equal(v3, v1) and api._WS


@pytest.mark.parametrize("image_max,r_cut,far", [((3, 3, 0), 30.0, 0), ((4, 4, 0), 30.0, 0), ((1, 1, 0), 0.0, 3)])
def test_image_window_stats(V, oracle, table, image_max, r_cut, far):
    """vdw_stats after a slab evaluation: the window's reach and coverage as
    the host function gives them, q0_min equal to the oracle's smallest q0 over
    the kept points, and far_D_min = q0_min x reach with a far shell."""
    import torch

    wl = W.scaled_slab(nxy=12, nz=40, image_max=image_max, r_cut=r_cut)
    g = V.Grid(wl.n, wl.h, wl.periodic)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    o = V.Opts(n_cut=wl.n_cut, r_cut=r_cut, image_max=image_max, precision=1, far_max=(far, far, 0))
    qd = V.compute_q0(g, n, wl.n_cut)
    V.enl_energy(g, n, qd["q0"], table, o)
    st = V.last_stats()
    reach, covers = V.image_window(g, o)
    qref = oracle.compute_q0(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, wl.n_cut)
    qmin = float(qref["q0"][qref["keep"]].min())
    say(f"  image_max={image_max} r_cut={r_cut} far={far}: reach {st['image_reach']:.4f} covers "
        f"{st['image_cut_covered']} q0_min {st['q0_min']:.6f} far_D_min {st['far_D_min']:.4f}")
    assert st["image_reach"] == reach and st["image_cut_covered"] == covers
    assert covers == (1 if image_max[0] == 4 else 0)
    assert st["q0_min"] == pytest.approx(qmin, rel=1e-12)
    if far:
        assert st["far_D_min"] == pytest.approx(qmin * reach, rel=1e-12)
        assert st["far_D_min"] < 48.0  # this shell takes the asymptote below D_max: an approximation
    else:
        assert st["far_D_min"] == 0.0
