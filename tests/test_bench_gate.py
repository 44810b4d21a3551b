"""bench.py's oracle gate on the scan (host logic only, no GPU).

The gate compares, per component over |E| of each density, the energies of
every scan density the oracle has stored at full size with those the GPU
computed.  Here the "GPU" energies are the stored oracle values themselves,
then the same with one component of one density moved: the gate must find
exactly that density and fail only when the move exceeds its tolerance.
"""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import vdw_workloads as W  # noqa: E402


def _stored():
    gold = json.load(open(bench.GOLDEN))["workloads"]
    E, keys = [], []
    for R in W.KR_SEPARATIONS:
        for which in ("both", "A", "B"):
            r = gold.get("kr_dimer_R%g_%s" % (R, which))
            E.append((r["E_pair0"], r["E_pairL"], r["E_self"]) if r else (0.0, 0.0, 1.0))
            if r:
                keys.append("R%g_%s" % (R, which))
    return E, keys


def test_gate_passes_on_the_oracle_values():
    E, keys = _stored()
    g = bench.oracle_gate(W, list(E), list(E))
    assert g is not None and g["passed"]
    assert g["densities_compared"] == len(keys) >= 3
    assert sorted(g["per_density_fp32c_fp64"]) == sorted(keys)
    assert g["fp32c_dE_rel_max"] == 0.0 and g["fp64_dE_rel_max"] == 0.0


@pytest.mark.parametrize("rel, passes", [(5e-7, True), (2e-6, False)])
def test_gate_finds_a_moved_component(rel, passes):
    E, keys = _stored()
    # move E_self of the R = 7 dimer in the FP32C energies by rel of |E|
    t = list(W.KR_SEPARATIONS).index(7.0)
    e = list(E[3 * t])
    e[2] += rel * abs(sum(e))
    E32 = list(E)
    E32[3 * t] = tuple(e)
    g = bench.oracle_gate(W, E32, list(E))
    assert g["passed"] is passes
    d = g["per_density_fp32c_fp64"]["R7_both"]
    assert d[0] == pytest.approx(rel, rel=1e-6) and d[1] == 0.0
    assert all(v == [0.0, 0.0] for k, v in g["per_density_fp32c_fp64"].items() if k != "R7_both")
