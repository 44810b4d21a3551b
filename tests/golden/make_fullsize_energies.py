"""Write tests/golden/fullsize_energies.json: the oracle's energies of the
full-size workloads, for the GPU tests to compare with.

Test infrastructure.  Calls only the oracle (and the seeded input
generators); nothing here runs or reads the HIP library.  The values:

  * the kernel table: 2048 x 64 nodes on D in [0, 48] with the default
    quadrature rule (Sec. 2 kernel, Sec. 7 refinement-converged rule);
  * the 96^3 Kr2-like dimer at R = 7 bohr (the Sec. 6.1 Kr-dimer stand-in) and
    each of its atoms alone at the same position: E_pair0, E_pairL (= 0),
    E_self (sphere on-site term), and for the dimer the norm of dE/dn and its
    projections on four seeded Gaussian vectors;
  * the 48 x 48 x 224 Xe-like slab (the Sec. 6.2 monolayer stand-in; Sec. 3
    periodic repetition) with images |m|, |p| <= 3 and r <= 30 bohr: E_pair0,
    E_self, and E_pairL as twice the sum over one of each image pair (m, -m)
    (the two terms of each pair are equal), one image shift per step;
  * the 64 synthetic molecules of the batch workload, each in full: E_pair0,
    E_self and the kept count;
  * the Xe-like slab on the hexagonal cell (skew cell, r <= 30 bohr): E_pair0
    (the home cell's pairs inside the cut) and E_self; its 80 image cells are
    left out (about five hours of oracle time);
  * the Xe-like slab's far image shell (the large-D asymptote over the cells
    beyond |m|, |p| <= 2 up to 32, no cut): its energy E_far, the part of
    E_pairL that the shell adds;
  * the rest of the Kr2-like scan, energies only: the dimers at R = 6, 8, 10
    and 14 bohr, then their atoms alone (about 20 minutes per dimer).

The run takes hours on a few cores (the slab's image sum is ~4e12 pair
evaluations), so every finished step is written at once and a rerun resumes
after the last one.  The table is kept in a cache file between runs (a
plain .npy written by this script; pass --cache).

    OMP_NUM_THREADS=8 python tests/golden/make_fullsize_energies.py [--cache PATH]
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import vdw_workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "fullsize_energies.json")
TABLE = dict(n_D=2048, n_sigma=64, D_max=48.0)
PROJ_SEEDS = (101, 102, 103, 104)


def _save(doc):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def _host():
    try:
        cpu = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")][0]
    except (OSError, IndexError):
        cpu = platform.processor()
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        nproc = os.cpu_count()
    return dict(cpu=cpu, nproc=nproc, threads=O.num_threads())


def _points(wl):
    g = O.Grid(wl.n, wl.h, wl.periodic)
    qd = O.compute_q0(g, wl.rho, wl.n_cut)
    idx, ix, iy, iz = O._points(g, qd["keep"])
    r = wl.rho.reshape(-1)
    return g, ix, iy, iz, r[idx], qd["q0"][idx]


def _self_energy(g, nS, qS, tab, tp):
    Phi = np.array([O.onsite_phi(g, float(q), tab, tp, 1)[0] for q in qS])
    return 0.5 * g.dV * g.dV * float(np.sum(nS * nS * Phi))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default=os.path.join("/tmp", "vdw_golden_table_2048x64.npy"))
    args = ap.parse_args()

    doc = json.load(open(OUT)) if os.path.exists(OUT) else {}
    tp = O.table_params(**TABLE)
    rule = dict(gl_points=tp.gl_points, graded_levels=tp.graded_levels, kappa=tp.kappa, A0=tp.A0)
    if doc.get("table") != dict(TABLE, **rule):
        doc = {"table": dict(TABLE, **rule), "workloads": {}}
    # the host of the first run (the dimer and slab sections); later sections
    # record their own
    doc.setdefault("host", {}).setdefault(platform.node() or "host", _host())

    if os.path.exists(args.cache):
        tab = np.load(args.cache, allow_pickle=False)
    else:
        t = time.time()
        tab = O.build_table(tp)
        doc["table_build_s"] = time.time() - t
        np.save(args.cache, tab)
    print(f"table ready ({tab.shape})", flush=True)
    wls = doc["workloads"]

    # --- Kr2-like dimer at R = 7 and its two atoms alone ---
    for which in ("both", "A", "B"):
        key = f"kr_dimer_R7_{which}"
        if key in wls:
            continue
        wl = W.kr_dimer(7.0, which=which)
        g = O.Grid(wl.n, wl.h, wl.periodic)
        t = time.time()
        res = O.evaluate(g, wl.rho, tab, tp, wl.n_cut, potential=(which == "both"))
        entry = dict(E_pair0=res.E_pair0, E_pairL=res.E_pairL, E_self=res.E_self,
                     kept=int(res.q0["keep"].sum()), seconds=time.time() - t)
        if which == "both":
            v = res.dEdn
            entry["dEdn_norm"] = float(np.linalg.norm(v))
            entry["dEdn_proj"] = {str(s): float(v @ np.random.default_rng(s).standard_normal(v.size))
                                  for s in PROJ_SEEDS}
        wls[key] = entry
        _save(doc)
        print(key, entry, flush=True)

    # --- Xe-like slab, images |m|, |p| <= 3, r <= 30 ---
    key = "xe_slab"
    wl = W.xe_slab()
    ent = wls.setdefault(key, {"image_max": list(wl.image_max), "r_cut": wl.r_cut, "shifts": {}})
    g, ix, iy, iz, nS, qS = _points(wl)
    ent["kept"] = int(len(nS))
    dV2 = g.dV * g.dV
    if "E_self" not in ent:
        ent["E_self"] = _self_energy(g, nS, qS, tab, tp)
        _save(doc)
    if "E_pair0" not in ent:
        t = time.time()
        ent["E_pair0"] = 0.5 * dV2 * O.image_pair_sum(g, ix, iy, iz, nS, qS, tab, tp, (0, 0, 0), wl.r_cut)
        ent["E_pair0_s"] = time.time() - t
        _save(doc)
        print(key, "E_pair0", ent["E_pair0"], flush=True)
    half = sorted(O.half_image_shifts(g, wl.image_max), key=lambda m: (m[0] ** 2 + m[1] ** 2 + m[2] ** 2, m))
    for m in half:
        mk = "%d,%d,%d" % m
        if mk in ent["shifts"]:
            continue
        t = time.time()
        s = O.image_pair_sum(g, ix, iy, iz, nS, qS, tab, tp, m, wl.r_cut)
        ent["shifts"][mk] = dict(sum=s, seconds=time.time() - t)
        _save(doc)
        print(key, "shift", mk, s, "%.0f s" % (time.time() - t), flush=True)
    # E_pairL = 1/2 dV^2 sum_{m != 0} = dV^2 sum over one of each (m, -m), in the order above
    if "E_pairL" not in ent:
        ent["E_pairL"] = dV2 * sum(ent["shifts"]["%d,%d,%d" % m]["sum"] for m in half)
        _save(doc)
        print(key, "E_pairL", ent["E_pairL"], flush=True)

    # --- the 64-molecule batch, every molecule in full ---
    mols = W.molecule_batch()
    bent = wls.setdefault("molecule_batch", {"count": len(mols), "molecules": [], "host": _host()})
    for b in range(len(bent["molecules"]), len(mols)):
        wl = mols[b]
        g = O.Grid(wl.n, wl.h, wl.periodic)
        t = time.time()
        res = O.evaluate(g, wl.rho, tab, tp, wl.n_cut)
        bent["molecules"].append(dict(E_pair0=res.E_pair0, E_pairL=res.E_pairL, E_self=res.E_self,
                                      kept=int(res.q0["keep"].sum()), seconds=time.time() - t))
        _save(doc)
        print("molecule", b, bent["molecules"][-1], flush=True)

    # --- the hexagonal-cell slab: home cell and on-site term ---
    key = "xe_hex_slab_home"
    if key not in wls:
        wl = W.xe_hex_slab()
        g = O.Grid(wl.n, wl.h, wl.periodic, cell=wl.cell)
        t = time.time()
        qd = O.compute_q0(g, wl.rho, wl.n_cut)
        idx, ix, iy, iz = O._points(g, qd["keep"])
        nS, qS = wl.rho.reshape(-1)[idx], qd["q0"][idx]
        S0, _, _ = O.pair_rows(g, ix, iy, iz, nS, qS, tab, tp, (0, 0, 0), wl.r_cut)
        e0 = 0.5 * g.dV * g.dV * float(np.sum(nS * S0))
        wls[key] = dict(E_pair0=e0, E_self=_self_energy(g, nS, qS, tab, tp), kept=int(len(nS)), r_cut=wl.r_cut,
                        seconds=time.time() - t, host=_host())
        _save(doc)
        print(key, wls[key], flush=True)

    # --- the slab's far image shell ---
    key = "xe_slab_far_shell"
    if key not in wls:
        wl = W.xe_slab()
        near, far = (2, 2, 0), (32, 32, 0)
        g, ix, iy, iz, nS, qS = _points(wl)
        t = time.time()
        F0, _ = O.far_rows(g, ix, iy, iz, nS, qS, near, far)
        wls[key] = dict(E_far=0.5 * g.dV * g.dV * float(np.sum(nS * F0)), image_max=list(near), far_max=list(far),
                        kept=int(len(nS)), seconds=time.time() - t, host=_host())
        _save(doc)
        print(key, wls[key], flush=True)

    # --- the rest of the scan: dimers first, then their atoms ---
    for which in ("both", "A", "B"):
        for R in (6.0, 8.0, 10.0, 14.0):
            key = "kr_dimer_R%g_%s" % (R, which)
            if key in wls:
                continue
            wl = W.kr_dimer(R, which=which)
            g = O.Grid(wl.n, wl.h, wl.periodic)
            t = time.time()
            res = O.evaluate(g, wl.rho, tab, tp, wl.n_cut)
            wls[key] = dict(E_pair0=res.E_pair0, E_pairL=res.E_pairL, E_self=res.E_self,
                            kept=int(res.q0["keep"].sum()), seconds=time.time() - t, host=_host())
            _save(doc)
            print(key, wls[key], flush=True)


if __name__ == "__main__":
    main()
