"""The oracle's point-sampled potential equals its full adjoint (it is the
same arithmetic restricted to the rows a point needs)."""
import numpy as np

import vdw_workloads as W

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)


def test_potential_at_matches_full_adjoint(oracle, table_cache):
    tp, tab = table_cache(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    for periodic, image_max, r_cut in [((0, 0, 0), (0, 0, 0), 0.0), ((1, 1, 0), (1, 1, 0), 3.1)]:
        wl = W.random_small(n=(7, 6, 5), periodic=periodic, seed=9, n_cut=4e-3)
        g = oracle.Grid(wl.n, wl.h, wl.periodic)
        full = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, image_max, r_cut, potential=True).dEdn
        ks = np.arange(0, g.G, 7)
        part = oracle.potential_at(g, wl.rho, ks, tab, tp, wl.n_cut, image_max, r_cut)
        assert np.allclose(part, full[ks], rtol=1e-13, atol=1e-16)
