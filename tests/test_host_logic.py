"""Host-side logic on the CPU: the autotuner's choice and cache (with the
pair-kernel timing replaced by a known cost function), and the workspace
bounds the library's planner reports (no device call is involved)."""
import json
import os

import pytest


@pytest.fixture()
def tuner(monkeypatch, tmp_path):
    from paper_0810_2273_amd import autotune

    monkeypatch.setenv("VDW_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    state = {}
    monkeypatch.setattr(autotune.api, "set_timing", lambda on: None)
    monkeypatch.setattr(autotune.api, "last_stats", lambda: dict(state))
    return autotune, state, tmp_path / "tune.json"


def _fake_run(state, shapes, calls):
    """A 'kernel' whose time is smallest at 1024 threads and j_chunks = 16;
    shapes the variant does not have fall back to 1024, as the library does."""

    def run(o):
        bt = o.block_threads if o.block_threads in shapes else 1024
        calls.append((bt, o.j_chunks))
        state.update(block_threads=bt, j_chunks=o.j_chunks,
                     pair_kernel_ms=10.0 + abs(o.j_chunks - 16) * 0.5 + (3.0 if bt == 512 else 0.0))

    return run


def test_autotune_picks_the_fastest_and_caches(tuner):
    autotune, state, cache = tuner
    from paper_0810_2273_amd import api

    calls = []
    opts = api.Opts(n_cut=1e-5)
    best = autotune.tune(_fake_run(state, (1024, 512), calls), opts, kept=500_000, candidates=(4, 8, 16, 32))
    assert (best.block_threads, best.j_chunks) == (1024, 16)
    entry = next(iter(json.loads(cache.read_text()).values()))
    assert set(entry["sweep"]) == {f"{bt}/{jc}" for bt in (1024, 512) for jc in (4, 8, 16, 32)}
    assert entry["ms"] == min(entry["sweep"].values()) == 10.0
    # cached: no timing at all, same answer, other options untouched
    again = autotune.tune(lambda o: pytest.fail("re-timed"), api.Opts(n_cut=1e-5, kahan=0), kept=500_000)
    assert (again.block_threads, again.j_chunks, again.n_cut) == (1024, 16, 1e-5)
    # another workload class (kept points in another power-of-two bucket) is tuned afresh
    calls.clear()
    autotune.tune(_fake_run(state, (1024, 512), calls), opts, kept=5_000, candidates=(8, 16))
    assert calls


def test_autotune_skips_shapes_a_variant_lacks(tuner):
    autotune, state, cache = tuner
    from paper_0810_2273_amd import api

    calls = []
    best = autotune.tune(_fake_run(state, (1024,), calls), api.Opts(n_cut=1e-5, precision=0), kept=10_000,
                         candidates=(8, 16))
    assert best.block_threads == 1024 and best.j_chunks == 16
    entry = next(iter(json.loads(cache.read_text()).values()))
    assert set(entry["sweep"]) == {"1024/8", "1024/16"}
    # one probe at 512 and one at 256 showed the variant runs 1024 and ended those sweeps
    assert sum(1 for c in calls if c == (1024, 8)) == 5  # three timed at 1024, one probe each at 512 and 256


def _ws(V, n, h=0.25, periodic=(0, 0, 0), **kw):
    tp = V.TableParams(n_D=2048, n_sigma=64, D_max=48.0)
    return V.enl_workspace_size(V.Grid(n, (h, h, h), periodic), tp, V.Opts(n_cut=1e-5, **kw))


def test_workspace_bounds_from_the_planner():
    import paper_0810_2273_amd as V

    base = _ws(V, (96, 96, 96))
    G = 96 ** 3
    # records (32 B), grid indices and the per-point dE/dq at least
    assert base > G * (32 + 4 + 8)
    assert _ws(V, (48, 48, 48)) < base / 4  # the item partials grow like G^2
    assert _ws(V, (96, 96, 96), precision=0) > base  # FP64 records and j-side partials
    assert _ws(V, (96, 96, 96), periodic=(1, 1, 0), image_max=(3, 3, 0)) > base  # one more accumulator array
    assert _ws(V, (96, 96, 96), j_chunks=1) != base  # the chunk length changes the work list
    assert _ws(V, (96, 96, 96), j_chunks=99) == 0  # invalid options: no size
    g1, g2 = V.Grid((96, 96, 96), (0.25,) * 3), V.Grid((40, 40, 40), (0.25,) * 3)
    tp = V.TableParams(n_D=2048, n_sigma=64, D_max=48.0)
    import ctypes as ct

    from paper_0810_2273_amd import _lib as L

    arr = (L.VdwGrid * 2)(g1.c(), g2.c())
    # the batch's tile shape is chosen for the whole list, so compare at a fixed one
    fixed = dict(block_threads=1024, j_chunks=8)
    o = V.Opts(n_cut=1e-5, **fixed).c()
    both = int(L.lib().enl_batched_workspace_size(2, arr, ct.byref(tp.c()), ct.byref(o)))
    # the sum of the parts, less the per-call items a batch holds once: the
    # FP32 table by cell (one float4 per cell) and the alignment padding
    quad = (2048 - 1) * (64 - 1) * 16
    assert both >= _ws(V, (96, 96, 96), **fixed) + _ws(V, (40, 40, 40), **fixed) - quad - 2 * 4096


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before it imports torch or touches a device."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
