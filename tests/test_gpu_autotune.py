"""The autotuner: it times each (workgroup shape, j-chunk length) candidate
with the pair kernel's HIP events, keeps the fastest, caches the choice, and
the tuned evaluation gives the same result (the tile shape changes the
summation order only).  The FP64 kernel has the 1024- and 256-thread
shapes; the FP32C n_sigma = 64 sweep covers 1024, 512 and 256."""
import json

import pytest

import vdw_workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_picks_and_caches(tmp_path, monkeypatch):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0810_2273_amd as V
    from paper_0810_2273_amd import autotune

    cache = tmp_path / "tune.json"
    monkeypatch.setenv("VDW_AUTOTUNE_CACHE", str(cache))
    wl = W.scaled_dimer(edge=48, h=0.3)
    g = V.Grid(wl.n, wl.h)
    n = torch.tensor(wl.rho.reshape(-1), dtype=torch.float64, device="cuda:0")
    table = V.build_phi_table(V.TableParams(n_D=512, n_sigma=64, D_max=48.0, gl_points=6, graded_levels=8,
                                            kappa=2.0, A0=20.0))
    qd = V.compute_q0(g, n, wl.n_cut)
    kept = int((n >= wl.n_cut).sum())
    print(f"autotune on a 48^3 dimer ({kept} kept points)", flush=True)

    def run(o):
        return V.enl_potential(g, n, qd, table, o)

    base = V.Opts(n_cut=wl.n_cut, precision=0)
    tuned = autotune.tune(run, base, kept=kept, candidates=(1, 2, 4, 8), repeats=1, verbose=True)
    assert tuned.j_chunks in (1, 2, 4, 8) and tuned.block_threads in (1024, 256)
    data = json.loads(cache.read_text())
    (entry,) = data.values()
    assert entry["j_chunks"] == tuned.j_chunks
    assert set(entry["sweep"]) == {f"{bt}/{jc}" for bt in (1024, 256) for jc in (1, 2, 4, 8)}
    assert min(entry["sweep"].values()) == entry["ms"] > 0
    # the cached choice comes back without timing
    again = autotune.tune(lambda o: pytest.fail("re-timed a cached workload"), base, kept=kept)
    assert again.j_chunks == tuned.j_chunks
    E0, v0 = run(base)
    E1, v1 = run(tuned)
    assert sum(E1) == pytest.approx(sum(E0), rel=1e-12)
    assert float(torch.linalg.norm(v1 - v0) / torch.linalg.norm(v0)) <= 1e-12
    assert V.last_stats()["j_chunks"] == tuned.j_chunks
    assert V.last_stats()["block_threads"] == tuned.block_threads
    # FP32C on the same cubic dimer and 64-column table: all three shapes are timed
    f32 = autotune.tune(run, V.Opts(n_cut=wl.n_cut, precision=1), kept=kept, candidates=(4, 8), repeats=1,
                        verbose=True)
    sweep = next(e for k, e in json.loads(cache.read_text()).items() if "|p1|" in k)["sweep"]
    assert set(sweep) == {f"{bt}/{jc}" for bt in (1024, 512, 256) for jc in (4, 8)}
    assert f32.block_threads in (1024, 512, 256)
