"""CPU timings of the oracle on the five benchmark workloads.

Test infrastructure, not part of the product: it times the plain FP64
oracle (oracle/oracle.py and its C double sums) on the host cores, to put
the GPU figures in context (the paper reports its own timings, Sec. 5, on
hardware of its time).  Nothing here loads or runs the HIP library.

  * tiny dimer, 24^3 grid, energy only: the 1024 x 32 table with the default
    quadrature rule, q0 and the full double sum;
  * Kr2-like scan, 96^3 grids, R = 6, 7, 8, 10, 14 bohr: q0 on every grid and
    a fixed random sample of rows of the double sum (E and dE/dq row sums)
    against all kept points; the full time is extrapolated from the rate;
  * Xe-like slab (images |m|, |p| <= 3, r <= 30 bohr): the full run that wrote
    tests/golden/fullsize_energies.json (its stored timings), and a live
    sample of image rows on this host;
  * the R = 7 dimer's dE/dn: the full oracle run of the same file (stored),
    and central finite differences of the energy at 64 seeded points;
  * the 64-molecule batch: every molecule in full, energy and dE/dn;
  * the rate of one thread on a sample of the R = 7 rows.

The 2048 x 64 tables are built with a coarser rule than the default one:
the node values do not change the work per pair, and the default rule's
build time is quoted from the stored full run.

    OMP_NUM_THREADS=<n> python oracle/time_oracle.py [--out profiles/oracle_cpu_timings.md]
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
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import vdw_workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden", "fullsize_energies.json")
COARSE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
SCAN_ROWS = 6000
SLAB_ROWS = 300
ONE_THREAD_ROWS = 400


def host_info():
    info = {"python_platform": platform.platform(), "omp_threads": O.num_threads()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        info["nproc"] = os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        keep = ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)", "CPU max MHz",
                "L2 cache", "L3 cache")
        info["lscpu"] = {k.strip(): v.strip() for k, v in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)
                         if k.strip() in keep}
    except OSError:
        info["lscpu"] = {}
    return info


def sample_rows(wl, tab, tp, rows, seed=0, image_max=(0, 0, 0), r_cut=0.0):
    """q0 on the whole grid, then `rows` random rows of the double sum against
    every kept point; returns (q0 seconds, rows seconds, kept, rows)."""
    g = O.Grid(wl.n, wl.h, wl.periodic)
    t0 = time.perf_counter()
    qd = O.compute_q0(g, wl.rho, wl.n_cut)
    t1 = time.perf_counter()
    idx, ix, iy, iz = O._points(g, qd["keep"])
    N = len(idx)
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(N, size=min(rows, N), replace=False)).astype(np.int64)
    r = wl.rho.reshape(-1)
    t2 = time.perf_counter()
    O.pair_rows(g, ix, iy, iz, r[idx], qd["q0"][idx], tab, tp, image_max, r_cut, rows=sel)
    t3 = time.perf_counter()
    return t1 - t0, t3 - t2, N, len(sel)


def cfg_tiny():
    wl = W.dimer_small()
    tp = O.table_params(n_D=1024, n_sigma=32, D_max=48.0)
    t0 = time.perf_counter()
    tab = O.build_table(tp)
    tb = time.perf_counter() - t0
    g = O.Grid(wl.n, wl.h, wl.periodic)
    t0 = time.perf_counter()
    res = O.evaluate(g, wl.rho, tab, tp, wl.n_cut)
    te = time.perf_counter() - t0
    N = int(res.q0["keep"].sum())
    return {"workload": wl.name, "kept": N, "ordered_pairs": N * (N - 1), "table_1024x32_default_rule_s": tb,
            "q0_pair_sum_self_s": te, "pair_evals_per_s": N * (N - 1) / te, "E": res.E}


def cfg_scan(tab, tp):
    out = []
    for R in W.KR_SEPARATIONS:
        wl = W.kr_dimer(R)
        tq, tr, N, rows = sample_rows(wl, tab, tp, SCAN_ROWS, seed=int(R * 10))
        rate = rows * (N - 1) / tr
        # the two atoms alone (the scan's E(inf) = E(A) + E(B)), at the same rate
        NA, NB = (int((W.kr_dimer(R, which=w).rho >= wl.n_cut).sum()) for w in ("A", "B"))
        out.append({"R_bohr": R, "kept": N, "q0_s": tq, "rows": rows, "rows_s": tr, "pair_evals_per_s": rate,
                    "full_sum_s_extrapolated": N * (N - 1) / rate, "kept_A": NA, "kept_B": NB,
                    "atoms_sum_s_extrapolated": (NA * (NA - 1) + NB * (NB - 1)) / rate})
    return out


def cfg_slab(tab, tp):
    gold = json.load(open(GOLDEN))
    ent = gold["workloads"]["xe_slab"]
    shifts = sum(v["seconds"] for v in ent["shifts"].values())
    stored = {"E_pair0_s": ent["E_pair0_s"], "image_shifts": len(ent["shifts"]), "image_shifts_s": shifts,
              "total_s": ent["E_pair0_s"] + shifts, "host": gold.get("host"),
              "note": "one full oracle run: E_pair0 over the home cell, then one of each image pair (m, -m)"}
    wl = W.xe_slab()
    tq, tr, N, rows = sample_rows(wl, tab, tp, SLAB_ROWS, seed=3, image_max=wl.image_max, r_cut=wl.r_cut)
    nimg = (2 * wl.image_max[0] + 1) * (2 * wl.image_max[1] + 1)
    live = {"kept": N, "q0_s": tq, "rows": rows, "rows_s": tr,
            "window_triples_per_s": rows * N * nimg / tr,
            "full_sum_s_extrapolated": N * N * nimg / (rows * N * nimg / tr)}
    return {"stored_full_run": stored, "live_sample": live}


def cfg_adjoint(tab, tp):
    gold = json.load(open(GOLDEN))
    stored = gold["workloads"].get("kr_dimer_R7_both", {}).get("seconds")
    wl = W.kr_dimer(7.0)
    g = O.Grid(wl.n, wl.h, wl.periodic)
    r = wl.rho.reshape(-1)
    rng = np.random.default_rng(7)
    cand = np.flatnonzero(r >= 10 * wl.n_cut)
    pts = rng.choice(cand, size=64, replace=False)
    ops = O.gradient_operators(g)
    t0 = time.perf_counter()
    for k in pts:
        eps = 1e-4 * r[k]
        O.local_energy_change(g, wl.rho, int(k), eps, tab, tp, wl.n_cut, ops=ops)
    tfd = time.perf_counter() - t0
    return {"stored_full_E_and_dEdn_s": stored, "fd_points": 64, "fd_s": tfd,
            "note": "the stored run is the oracle's full E + dE/dn of the R = 7 dimer with the default rule"}


def cfg_batch(tab, tp):
    wls = W.molecule_batch()
    t0 = time.perf_counter()
    pairs = 0
    for wl in wls:
        g = O.Grid(wl.n, wl.h, wl.periodic)
        res = O.evaluate(g, wl.rho, tab, tp, wl.n_cut, potential=True)
        N = int(res.q0["keep"].sum())
        pairs += N * (N - 1)
    dt = time.perf_counter() - t0
    return {"molecules": len(wls), "ordered_pairs": pairs, "E_and_dEdn_s": dt, "pair_evals_per_s": pairs / dt}


def one_thread(tab_path):
    """Rows of the R = 7 dimer on one thread (run in a child process with
    OMP_NUM_THREADS=1)."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json, numpy as np; sys.path.insert(0, %r); from oracle import time_oracle as T, oracle as O; "
            "import vdw_workloads as W; tp = O.table_params(n_D=2048, n_sigma=64, D_max=48.0, **T.COARSE); "
            "tab = np.load(%r); tq, tr, N, rows = T.sample_rows(W.kr_dimer(7.0), tab, tp, %d, seed=70); "
            "print(json.dumps(dict(threads=O.num_threads(), rows=rows, kept=N, rows_s=tr, "
            "pair_evals_per_s=rows * (N - 1) / tr)))") % (ROOT, tab_path, ONE_THREAD_ROWS)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def report(res):
    h = res["host"]
    L = ["# Oracle timings on the host CPU (FP64, OpenMP)", "",
         "Made by `OMP_NUM_THREADS=%d python oracle/time_oracle.py` (the oracle as it stands, not tuned for "
         "speed). Host: %s, nproc %s, %d OpenMP threads." % (h["omp_threads"], h["lscpu"].get("Model name", "?"),
                                                              h["nproc"], h["omp_threads"]), "",
         "lscpu: " + "; ".join("%s = %s" % kv for kv in h["lscpu"].items()), ""]
    t = res["tiny"]
    L += ["## Tiny dimer, 24^3, energy only (in full)", "",
          "%d kept points, %.3g ordered pairs: table 1024 x 32 (default rule) %.1f s; q0 + double sum + "
          "on-site term %.2f s (%.3g pair evaluations/s)." % (t["kept"], t["ordered_pairs"],
                                                              t["table_1024x32_default_rule_s"],
                                                              t["q0_pair_sum_self_s"], t["pair_evals_per_s"]), ""]
    L += ["## Kr2-like scan, 96^3 (sampled rows, E and dE/dq row sums)", "",
          "| R (bohr) | kept | q0 s | rows | rows s | pair evals/s | full double sum s (extrapolated) |",
          "|---|---|---|---|---|---|---|"]
    for s in res["scan"]:
        L.append("| %g | %d | %.2f | %d | %.1f | %.3g | %.0f |" % (s["R_bohr"], s["kept"], s["q0_s"], s["rows"],
                                                                   s["rows_s"], s["pair_evals_per_s"],
                                                                   s["full_sum_s_extrapolated"]))
    tot = sum(s["full_sum_s_extrapolated"] for s in res["scan"])
    atoms = sum(s["atoms_sum_s_extrapolated"] for s in res["scan"])
    L += ["", "Five dimers: %.0f s of double sum (extrapolated); their ten atoms alone %.0f s more, %.0f s (%.1f h) "
          "for the scan's step. The default-rule 2048 x 64 table took %.0f s in the stored run." % (
              tot, atoms, tot + atoms, (tot + atoms) / 3600, res.get("table_2048x64_default_s") or -1), ""]
    s = res["slab"]
    st, lv = s["stored_full_run"], s["live_sample"]
    L += ["## Xe-like slab, images |m|, |p| <= 3, r <= 30 bohr", "",
          "Stored full run (tests/golden/fullsize_energies.json): E_pair0 %.0f s, %d image shifts %.0f s, total "
          "%.0f s (%.2f h) on %s. That run sums one of each image pair (m, -m) and doubles it (the two sums are "
          "equal), so it visits 25 of the 49 cells." % (st["E_pair0_s"], st["image_shifts"], st["image_shifts_s"],
                                                        st["total_s"], st["total_s"] / 3600, json.dumps(st["host"])),
          "Live sample here, all 49 cells per row as the double sum is written: %d rows x %d points x 49 cells in "
          "%.1f s, %.3g (point, image, point) triples/s, full sum about %.0f s." % (
              lv["rows"], lv["kept"], lv["rows_s"], lv["window_triples_per_s"], lv["full_sum_s_extrapolated"]), ""]
    a = res["adjoint"]
    L += ["## R = 7 dimer, dE/dn", "",
          "Stored full oracle run (E + dE/dn, default rule): %.0f s. Central differences of E at 64 points: %.1f s."
          % (a["stored_full_E_and_dEdn_s"] or -1, a["fd_s"]), ""]
    b = res["batch"]
    L += ["## 64-molecule batch (in full, E and dE/dn)", "",
          "%d molecules, %.3g ordered pairs: %.0f s (%.3g pair evaluations/s)." % (b["molecules"], b["ordered_pairs"],
                                                                                  b["E_and_dEdn_s"],
                                                                                  b["pair_evals_per_s"]), ""]
    o = res["one_thread"]
    L += ["## One thread", "",
          "R = 7 dimer, %d rows x %d points on %d thread: %.1f s, %.3g pair evaluations/s." % (
              o["rows"], o["kept"], o["threads"], o["rows_s"], o["pair_evals_per_s"]), ""]
    return "\n".join(L)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "oracle_cpu_timings.md"))
    ap.add_argument("--table-cache", default="/tmp/vdw_time_oracle_table_2048x64.npy")
    a = ap.parse_args()
    res = {"host": host_info()}
    print("host", res["host"], flush=True)
    res["tiny"] = cfg_tiny()
    print("tiny", res["tiny"], flush=True)
    tp = O.table_params(n_D=2048, n_sigma=64, D_max=48.0, **COARSE)
    tab = O.build_table(tp)
    np.save(a.table_cache, tab)
    gold = json.load(open(GOLDEN))
    res["table_2048x64_default_s"] = gold.get("table_build_s")
    res["scan"] = cfg_scan(tab, tp)
    print("scan", res["scan"], flush=True)
    res["slab"] = cfg_slab(tab, tp)
    print("slab", res["slab"], flush=True)
    res["adjoint"] = cfg_adjoint(tab, tp)
    print("adjoint", res["adjoint"], flush=True)
    res["one_thread"] = one_thread(a.table_cache)
    print("one thread", res["one_thread"], flush=True)
    res["batch"] = cfg_batch(tab, tp)
    print("batch", res["batch"], flush=True)
    with open(a.out, "w") as f:
        f.write(report(res))
        f.write("\n<!-- raw: %s -->\n" % json.dumps(res))
    print("written", a.out, flush=True)


if __name__ == "__main__":
    main()
