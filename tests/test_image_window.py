"""The near image window (vdw_image_window, host only; Sec. 3 periodic
repetition): the reach below which every pair (i, j, L) is summed, against
the closed form on orthorhombic cells and against brute force over point
pairs and lattice vectors on small orthorhombic and skew grids; the coverage
flag of the Xe-slab setting; and the layout of vdw_stats as C sees it."""
import ctypes as ct
import itertools
import math
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def V():
    from paper_0810_2273_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_0810_2273_amd import build_ext

        build_ext.build()
    import paper_0810_2273_amd as V

    return V


def test_slab_window_does_not_cover_30_bohr(V):
    """The slab setting (8.6 x 8.6 x 40 bohr, 48 x 48 x 224, images |m| <= 3,
    r <= 30): the first left-out lateral image is (3 + 1/48) * 8.6 = 25.98 bohr
    away at the closest, inside the cut; |m| <= 4 reaches 34.58 and covers it."""
    g = V.Grid((48, 48, 224), (8.6 / 48, 8.6 / 48, 40.0 / 224), (1, 1, 0))
    reach, covers = V.image_window(g, V.Opts(n_cut=1e-5, r_cut=30.0, image_max=(3, 3, 0)))
    assert reach == pytest.approx((3 + 1 / 48) * 8.6, rel=1e-14)
    assert covers == 0
    reach, covers = V.image_window(g, V.Opts(n_cut=1e-5, r_cut=30.0, image_max=(4, 4, 0)))
    assert reach == pytest.approx((4 + 1 / 48) * 8.6, rel=1e-14) and covers == 1
    # no cut on a periodic grid: the window truncates the sum
    assert V.image_window(g, V.Opts(n_cut=1e-5, image_max=(4, 4, 0)))[1] == 0
    # no periodic axis: nothing to cover
    open_grid = V.Grid((8, 8, 8), (0.3, 0.3, 0.3))
    reach, covers = V.image_window(open_grid, V.Opts(n_cut=1e-5, r_cut=5.0))
    assert math.isinf(reach) and covers == -1


def _brute_min_distance(cell, n, periodic, image_max, extra=2):
    """Smallest |r_i - r_j - L| over all grid-point pairs and the lattice
    vectors L with |m_a| > image_max[a] on some periodic axis (|m_a| up to
    image_max[a] + extra)."""
    cell = np.asarray(cell, dtype=float)
    E = cell / np.asarray(n, dtype=float)[:, None]
    idx = np.array(list(itertools.product(*(range(k) for k in n))), dtype=float)
    pts = idx @ E
    d = (pts[:, None, :] - pts[None, :, :]).reshape(-1, 3)
    best = math.inf
    rng = [range(-(image_max[a] + extra), image_max[a] + extra + 1) if periodic[a] else range(0, 1) for a in range(3)]
    for m in itertools.product(*rng):
        if all(abs(m[a]) <= image_max[a] for a in range(3) if periodic[a]):
            continue
        L = np.asarray(m, dtype=float) @ cell
        best = min(best, float(np.sqrt(((d - L) ** 2).sum(axis=1)).min()))
    return best


@pytest.mark.parametrize("cell,n,periodic,image_max,exact", [
    (((3.0, 0, 0), (0, 2.5, 0), (0, 0, 4.0)), (4, 3, 5), (1, 1, 0), (1, 0, 0), True),
    (((3.0, 0, 0), (0, 2.5, 0), (0, 0, 4.0)), (3, 4, 3), (1, 1, 1), (0, 2, 1), True),
    (((3.0, 0, 0), (1.5, 2.6, 0), (0.0, 0.0, 3.5)), (4, 4, 3), (1, 1, 0), (1, 1, 0), False),
    (((2.8, 0, 0), (1.1, 2.6, 0), (0.4, -0.3, 2.9)), (3, 4, 3), (1, 1, 1), (1, 0, 1), False),
])
def test_reach_is_a_bound_and_exact_on_orthorhombic_cells(V, cell, n, periodic, image_max, exact):
    g = V.Grid(n, periodic=periodic, cell=cell)
    reach, _ = V.image_window(g, V.Opts(n_cut=1e-5, image_max=image_max))
    brute = _brute_min_distance(cell, n, periodic, image_max)
    assert reach <= brute * (1 + 1e-12)
    if exact:
        assert reach == pytest.approx(brute, rel=1e-12)


def test_vdw_stats_layout_matches_the_header(V, tmp_path):
    """Offsets and size of vdw_stats from a C compiler against the binding."""
    from paper_0810_2273_amd import _lib as L

    fields = [f for f, _ in L.VdwStats._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof(vdw_stats, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "vdwdf.h"\nint main(void) {\n' + body +
                   '    printf("%zu\\n", sizeof(vdw_stats));\n    return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I" + os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[:-1] == [getattr(L.VdwStats, f).offset for f in fields]
    assert out[-1] == ct.sizeof(L.VdwStats)


def test_image_window_rejects_bad_arguments(V):
    from paper_0810_2273_amd import _lib as L

    lib = L.lib()
    g = V.Grid((8, 8, 8), (0.3, 0.3, 0.3), (1, 0, 0)).c()
    o = V.Opts(n_cut=1e-5, image_max=(-1, 0, 0)).c()
    r = ct.c_double()
    assert lib.vdw_image_window(ct.byref(g), ct.byref(o), ct.byref(r), None) == L.VDW_EINVAL
    o = V.Opts(n_cut=1e-5).c()
    assert lib.vdw_image_window(ct.byref(g), None, ct.byref(r), None) == L.VDW_EINVAL
    assert lib.vdw_image_window(ct.byref(g), ct.byref(o), None, None) == L.VDW_EINVAL
