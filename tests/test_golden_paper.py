"""Values the paper prints for its worked example (App. A, the Xe-monolayer
sample run).  The density file of that run is not available, so these pin
only what the printed numbers fix by themselves: the grid volume element and
the bookkeeping identities of the printed energies."""
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "xe_layer_sample_run.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            k, v = line.split("=")
            vals[k.strip()] = [float(x) for x in v.split()]
    return vals


def test_volume_element_from_printed_cell(oracle):
    """dV = |det(a, b, c)| / (nx ny nz) reproduces the printed dV for the printed
    hexagonal cell (App. A output: 28 x 28 x 160 grid)."""
    g = _golden()
    n = [int(x) for x in g["nx ny nz"]]
    dV = oracle.cell_volume_element([g["a"], g["b"], g["c"]], n)
    assert dV == pytest.approx(g["dV"][0], abs=5e-9)
    assert n[0] * n[1] * n[2] == int(g["total_points"][0])
    assert int(g["total_points"][0]) // int(g["processors"][0]) == int(g["points_per_processor"][0])


def test_printed_energy_identities():
    """Printed totals are the sums of their parts; the 'needed number' fixes the
    sign convention of Eq. (3): -E_c^PBE + E_c^LDA + E_c^NL."""
    g = _golden()
    ex, ec, exc = g["E_lda"]
    assert ex + ec == pytest.approx(exc, abs=2e-8)
    ex, ec_pbe, exc = g["E_pbe"]
    assert ex + ec_pbe == pytest.approx(exc, abs=2e-8)
    off, diag, tot = g["E_nl"]
    assert off + diag == pytest.approx(tot, abs=2e-8)
    assert -ec_pbe + g["E_lda"][1] + tot == pytest.approx(g["needed_number"][0], abs=2e-8)


def test_printed_trimming_keeps_almost_all_charge():
    """The density cut-off drops 80 % of the points but < 0.03 % of the charge."""
    g = _golden()
    assert g["points_after_trimming"][0] / g["total_points"][0] < 0.2
    lost = 1 - g["electrons_after_trimming"][0] / g["electrons"][0]
    assert 0 < lost < 3e-4
