"""Benchmark: pair evaluations per second of E_c^nl + v_nl on one MI355X.

Default workload (`--workload kr`): the Kr2-like dimer scan.  Five
separations R = 6, 7, 8, 10, 14 bohr, each with its two atoms alone
(E(inf) = E(A) + E(B) on the same grid positions), 15 densities on 96^3
grids (h = 0.25 bohr, n_cut = 1e-5), 2048 x 64 kernel table.  One step is
the whole batched evaluation — gradient and q0 of every density,
compaction, the persistent pair kernel over the shared work list, the
reductions and the adjoint dE/dn — recorded once into a HIP graph and
replayed, inputs resident in HBM.  The table is built once on the GPU
before timing.  Prints one JSON line with the binding curve
E_nl(R) - E_nl(inf), the FP32C-vs-FP64 comparison on the same step, the
roofline of the pair kernel and the CPU oracle's rate on a sample.

Roofline: the pair kernel is bound by vector ALU work.  It evaluates each
unordered pair once for both orders; the algorithmic work of one such
evaluation (energy + adjoint sums, table branch) is FLOP_PER_UNORDERED_PAIR
FP32 operations (FMA counted as 2, transcendental as 1: displacement 3,
squared distance 5, square root 1, a_i + a_j 1, t_D 1, reciprocal 1, u 2,
t_sigma 1, fractions 2, bilinear value 9, sigma slope 3, the two derivative
products 4, the two q-derivatives 4, four accumulations 8), so
achieved = (ordered pairs / 2) x FLOP_PER_UNORDERED_PAIR / (mean pair-kernel
time from HIP events on the launch stream), against the 157.3 TFLOP/s FP32
vector peak of MI355X.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# fused energy + adjoint, table branch, one evaluation for both orders of a pair
FLOP_PER_UNORDERED_PAIR = 45
FLOP_PER_UNORDERED_PAIR_ENERGY = 30
PEAK_FP32_TFLOPS = 157.3
# Counter figures of the same kernel and workload from the rocprofv3 runs in
# profiles/ (executed FP32 FLOP from SQ_INSTS_VALU_FLOPS_FP32 x 64, VALU
# instructions against wave64 issue slots from GRBM_GUI_ACTIVE); reported
# beside the live roofline, not measured by this script.
PROFILE_COUNTERS = {
    "kr": {"source": "profiles/pair_kernel_kr_scan96_fp32c.md", "executed_tflops": 43.6,
           "valu_instructions_per_issue_slot": 1.06, "lane_instructions_per_unordered_pair": 37.6},
    "slab": {"source": "profiles/pair_kernel_xe_slab_literal_fp32c.md", "executed_tflops": 31.9,
             "valu_instructions_per_issue_slot": 0.76, "lane_instructions_per_in_cut_unordered_pair": 39.1},
}
# Far image shell (FP64): algorithmic FLOP per ordered pair of the row pass
# (a_i^2 a_j^2 (a_i^2 + a_j^2), its reciprocal, the weighted sum and the
# q-derivative term) and per (displacement, lattice vector) term of the
# lattice-sum table (the displacement mapped by the step matrix, |.|^2, the
# cube, its reciprocal, the sum); peak: MI355X FP64 vector.
FLOP_PER_FAR_PAIR = 12
FLOP_PER_FAR_TERM = 30
PEAK_FP64_TFLOPS = 78.6
# HBM bytes per pair-kernel launch, from rocprofv3 FETCH_SIZE (x 2.0, the
# factor a plain 512 MiB copy needs) + WRITE_SIZE of the current kernel
# (profiles/); a workload without a profile of the current kernel has none.
TRAFFIC_BYTES = {"kr": (5308970.0 * 2.0 + 8971550.0) * 1024, "slab": (411084.0 * 2.0 + 891907.0) * 1024}
# The metric's accuracy gate: FP32C against the FP64 form (and against the
# oracle's full-size energies where they are stored).
GATE_DE_REL = 1e-6
GATE_DV_REL = 1e-4
GOLDEN = os.path.join(ROOT, "tests", "golden", "fullsize_energies.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--R", type=float, default=7.0, help="separation of the kr1 workload (bohr)")
    p.add_argument("--far", type=int, default=32, help="far image shell of the slabfar workload: |m|,|p| <= far")
    p.add_argument("--workload", default="kr",
                   choices=["kr", "kr1", "slab", "hexslab", "slabfar", "batch", "dimer24"],
                   help="kr: the Kr2-like dimer scan (the reported metric); kr1: one dimer at --R; slab, hexslab, "
                        "slabfar (near images plus the far shell), batch, dimer24: the other cases")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=0, help="oracle rows in the CPU sample (0: auto)")
    p.add_argument("--kahan", type=int, default=0)
    p.add_argument("--no-kahan", action="store_true", help="skip the Kahan-compensated comparison run")
    p.add_argument("--lds-rows", type=int, default=-1)
    p.add_argument("--j-chunks", type=int, default=0)
    p.add_argument("--grid-blocks", type=int, default=0)
    p.add_argument("--block-threads", type=int, default=0,
                   help="pair-kernel workgroup: 0/1024 (four i-points per lane) or 512 (eight)")
    p.add_argument("--no-graph", action="store_true",
                   help="batched workloads: call enl_potential_batched per step instead of replaying a recorded graph")
    p.add_argument("--autotune", action="store_true", help="pick j_chunks with the autotuner before timing")
    p.add_argument("--cpu-only", action="store_true",
                   help="print the CPU oracle's rate on the sample as JSON and exit (no GPU use)")
    p.add_argument("--copy-calib", type=int, default=0,
                   help="MiB: run one plain device-to-device copy of this size first (profiler calibration)")
    return p.parse_args()


def workloads(a, W):
    """(densities, description) of the chosen workload."""
    if a.workload == "kr":
        wls = []
        for R in W.KR_SEPARATIONS:
            wls += [W.kr_dimer(R), W.kr_dimer(R, which="A"), W.kr_dimer(R, which="B")]
        desc = ("Kr2-like dimer scan: R in {6,7,8,10,14} bohr, each with its two atoms alone (E(inf) = E(A)+E(B)); "
                "15 densities on 96^3 grids h=0.25 bohr, n_cut=1e-5, table 2048x64 on D<=48; one batched evaluation "
                "(q0 included, E + dE/dn fused) replayed as a HIP graph")
    elif a.workload == "kr1":
        wls = [W.kr_dimer(a.R)]
        desc = (f"Kr2-like dimer, 96^3 grid h=0.25 bohr, R={a.R:g} bohr, n_cut=1e-5, "
                f"table 2048x64 on D<=48, energy + potential fused")
    elif a.workload == "slab":
        wls = [W.xe_slab()]
        desc = ("Xe-like slab, 48x48x224 grid of an 8.6x8.6x40 bohr cell, periodic x,y, images |m|,|p|<=3, "
                "r<=30 bohr, n_cut=1e-5, table 2048x64, energy + potential fused")
    elif a.workload == "hexslab":
        wls = [W.xe_hex_slab()]
        desc = ("Xe-like slab on the hexagonal cell of a close-packed monolayer (a = (8.6, 0, 0), b = (4.3, 7.45, 0), "
                "c = (0, 0, 40) bohr), 48x48x224 grid, periodic in a and b, images |m|,|p|<=4, r<=30 bohr, n_cut=1e-5, "
                "table 2048x64, energy + potential fused")
    elif a.workload == "slabfar":
        wls = [W.xe_slab()]
        wls[0].image_max, wls[0].r_cut = (2, 2, 0), 0.0
        desc = ("Xe-like slab, 48x48x224 grid of an 8.6x8.6x40 bohr cell, periodic x,y, no distance cut: images "
                "|m|,|p|<=2 with the table, the far shell |m|,|p|<=%d with the large-D asymptote (one lattice-sum "
                "pass), n_cut=1e-5, table 2048x64, energy + potential fused" % a.far)
    elif a.workload == "batch":
        wls = W.molecule_batch(64)
        desc = ("64 molecule densities, 16^3..64^3 grids h=0.3 bohr, n_cut=1e-5, table 2048x64, one batched "
                "evaluation (q0 included) replayed as a HIP graph")
    else:
        wls = [W.dimer_small()]
        desc = "dimer 24^3 grid h=0.5 bohr, n_cut=1e-6, table 1024x32, energy only"
    return wls, desc


def one_thread_baseline(rows):
    """The oracle's rate on one thread: a child process (started before this
    one touches the GPU) with OMP_NUM_THREADS=1 on a smaller sample."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--cpu-rows", str(rows)]
    print("# cpu baseline on one thread (child process)", file=sys.stderr, flush=True)
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        print(r.stderr[-2000:], file=sys.stderr)
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU split is a design "
              "note, not part of this build", file=sys.stderr)
        sys.exit(2)
    if a.cpu_only:
        import vdw_workloads as W

        print(json.dumps(cpu_baseline(W.kr_dimer(7.0), a.cpu_rows)), flush=True)
        return
    one_thread = None
    if not a.no_cpu_baseline and a.workload in ("kr", "kr1"):
        one_thread = one_thread_baseline(400)
    import numpy as np
    import torch

    import paper_0810_2273_amd as V
    import vdw_workloads as W

    dev = torch.device("cuda:0")
    if a.copy_calib > 0:
        src = torch.ones(a.copy_calib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"# building the {a.workload} densities", file=sys.stderr, flush=True)
    wls, desc = workloads(a, W)
    wl = wls[0]
    tparams = V.TableParams(n_D=1024, n_sigma=32, D_max=48.0) if a.workload == "dimer24" else \
        V.TableParams(n_D=2048, n_sigma=64, D_max=48.0)
    print(f"# building table {tparams.n_D}x{tparams.n_sigma} on the GPU", file=sys.stderr, flush=True)
    t0 = time.time()
    table = V.build_phi_table(tparams, device=dev)
    torch.cuda.synchronize()
    t_table = time.time() - t0
    grids = [V.Grid(w.n, w.h, w.periodic, cell=w.cell) for w in wls]
    ns = [torch.tensor(w.rho.reshape(-1), dtype=torch.float64, device=dev) for w in wls]
    n, offs = V.pack_batch(grids, ns)
    del ns
    g = grids[0]
    batched = len(wls) > 1

    def opts(prec):
        far = (a.far, a.far, 0) if a.workload == "slabfar" else (0, 0, 0)
        return V.Opts(n_cut=wl.n_cut, r_cut=wl.r_cut, image_max=wl.image_max, precision=prec, kahan=a.kahan,
                      table_lds_rows=a.lds_rows, j_chunks=a.j_chunks, grid_blocks=a.grid_blocks,
                      block_threads=a.block_threads, far_max=far)

    graph = batched and not a.no_graph
    plans = {}

    def eager(prec):
        """[(E_pair0, E_pairL, E_self)] per density and dE/dn (packed)."""
        if batched:
            qd = V.compute_q0_batched(grids, n, offs, wl.n_cut)
            return V.enl_potential_batched(grids, n, offs, qd, table, opts(prec))
        if a.workload == "dimer24":
            qd = V.compute_q0(g, n, wl.n_cut, derivatives=False)
            return [V.enl_energy(g, n, qd["q0"], table, opts(prec))], n
        qd = V.compute_q0(g, n, wl.n_cut)
        E, v = V.enl_potential(g, n, qd, table, opts(prec))
        return [E], v

    def step(prec):
        if not graph:
            return eager(prec)
        p = plans.get(prec)
        if p is None:
            # the whole batched evaluation (q0 of every density included)
            # recorded once into a HIP graph, replayed per step
            p = plans[prec] = V.BatchPlan(grids, offs, table, opts(prec))
            p.capture(n)
        p.replay()
        return p, None

    def result(out):
        if not graph:
            return out
        p = out[0]
        return p.energies(), p.dEdn

    def timed(prec, steps, warmup):
        V.set_timing(False)
        for i in range(warmup):
            step(prec)
            torch.cuda.synchronize()
            print(f"# warmup {i + 1}/{warmup} precision={prec}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        V.set_timing(not graph)
        kms = []
        t0 = time.perf_counter()
        for i in range(steps):
            out = step(prec)
            if not graph:
                kms.append(V.last_stats()["pair_kernel_ms"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        E, v = result(out)
        if graph:
            # pair-kernel time from HIP events around the same kernel in one
            # eager evaluation (a replayed graph carries no events)
            V.set_timing(True)
            eager(prec)
            kms.append(V.last_stats()["pair_kernel_ms"])
        st = V.last_stats()
        V.set_timing(False)
        print(f"# timed {steps} steps precision={prec}: {dt:.3f} s", file=sys.stderr, flush=True)
        return dt, E, v, float(np.mean(kms)), st

    main_prec = V.VDW_FP64 if a.workload == "dimer24" else V.VDW_FP32C
    if a.autotune:
        from paper_0810_2273_amd import autotune

        base = opts(main_prec)
        tuned = autotune.tune(lambda o: V.enl_potential_batched(grids, n, offs, V.compute_q0_batched(
            grids, n, offs, wl.n_cut), table, o), base, kept=int((n >= wl.n_cut).sum()),
            nimg=int(np.prod([2 * m + 1 if per else 1 for m, per in zip(wl.image_max, wl.periodic)])),
            batch=len(wls), verbose=True)
        a.j_chunks, a.block_threads = tuned.j_chunks, tuned.block_threads
        V.release_workspaces()  # the sweep's largest workspace is not needed again
        print(f"# autotune: block_threads={a.block_threads} j_chunks={a.j_chunks}", file=sys.stderr, flush=True)
    dt, E32, v32, kms32, st = timed(main_prec, a.steps, a.warmup)
    near_pairs = st["pairs"]
    far_pairs = st["far_pairs"]
    pairs = near_pairs + far_pairs  # the far shell's pairs count once each (their lattice sums folded in)
    value = pairs * a.steps / dt
    out = {
        "metric": "pair-evals/s E_nl+v_nl, FP32-compensated vs FP64 on GPU at |dE|/|E|<=1e-6",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.workload == "dimer24" else "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "densities": len(wls),
            "retained_points": st["retained"],
            "pairs_per_step": pairs,
            "lds_rows": st["lds_rows"],
            "j_chunks": st["j_chunks"],
            "grid_blocks": st["grid_blocks"],
            "block_threads": st["block_threads"],
            "kahan": a.kahan,
            "hip_graph": graph,
        },
    }
    fpp = FLOP_PER_UNORDERED_PAIR_ENERGY if a.workload == "dimer24" else FLOP_PER_UNORDERED_PAIR
    # algorithmic work: the pairs inside the distance cut (all of them without one)
    work_pairs = near_pairs
    if wl.r_cut > 0:
        work_pairs = sum(in_cut_pairs(w) for w in wls)
        out["config"]["pairs_in_cut_per_step"] = work_pairs
    achieved = 0.5 * work_pairs * fpp / (kms32 * 1e-3) / 1e12
    out["roofline"] = {
        "bound": "alu",
        "achieved": achieved,
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_TFLOPS,
        "traffic": TRAFFIC_BYTES.get(a.workload) if a.workload != "kr1" or a.R == 7.0 else None,
        "kernel": "pair_kernel<%s, %s, %s>" % ("double" if a.workload == "dimer24" else "float",
                                                "energy" if a.workload == "dimer24" else "ADJ",
                                                "IMG" if a.workload in ("slab", "hexslab", "slabfar") else "noIMG"),
        "kernel_ms": kms32,
        "flop_per_unordered_pair": fpp,
        "pairs_counted": "ordered pairs inside the distance cut" if wl.r_cut > 0 else "ordered pairs",
    }
    if a.workload in PROFILE_COUNTERS:
        out["roofline"]["counters"] = PROFILE_COUNTERS[a.workload]
    if any(wl.periodic):
        out["image_window"] = {"reach_bohr": st["image_reach"], "covers_r_cut": st["image_cut_covered"],
                               "q0_min": st["q0_min"]}
        if far_pairs:
            out["image_window"]["far_D_min_bound"] = st["far_D_min"]
    tot = [sum(e[k] for e in E32) for k in range(3)]
    out["energy_ha"] = {"E_pair0": tot[0], "E_pairL": tot[1], "E_self": tot[2], "E": sum(tot)}
    if a.workload == "kr":
        scan = []
        for t, R in enumerate(W.KR_SEPARATIONS):
            e_ab, e_a, e_b = (sum(E32[3 * t + k]) for k in range(3))
            scan.append({"R_bohr": R, "E_nl": e_ab, "E_nl_minus_E_inf": e_ab - e_a - e_b})
        out["scan"] = scan
    out["table_build_s"] = t_table
    if far_pairs:
        nvec = (2 * a.far + 1) ** 2 - (2 * wl.image_max[0] + 1) * (2 * wl.image_max[1] + 1)
        entries = (2 * wl.n[0] - 1) * (2 * wl.n[1] - 1) * (2 * wl.n[2] - 1)
        flop = far_pairs * FLOP_PER_FAR_PAIR + entries * nvec * FLOP_PER_FAR_TERM
        fms = st["far_kernel_ms"]
        out["far_shell"] = {
            "near_image_max": list(wl.image_max), "far_max": [a.far, a.far, 0], "lattice_vectors": nvec,
            "table_entries": entries, "far_pairs": far_pairs, "image_pairs_covered": far_pairs * nvec,
            "far_kernels_ms": fms, "near_pair_kernel_ms": kms32,
            "roofline": {"bound": "alu", "achieved": flop / (fms * 1e-3) / 1e12 if fms > 0 else None,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": flop / (fms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS if fms > 0 else None,
                         "kernels": "far_table_kernel + far_rows_kernel", "flop_per_pair": FLOP_PER_FAR_PAIR,
                         "flop_per_table_term": FLOP_PER_FAR_TERM},
        }
    if not a.no_fp64 and a.workload != "dimer24":
        steps64 = max(1, a.steps // 2)
        dt64, E64, v64, kms64, _ = timed(V.VDW_FP64, steps64, 1)
        rate64 = pairs * steps64 / dt64
        dE = max(abs(sum(e32) - sum(e64)) / abs(sum(e64)) for e32, e64 in zip(E32, E64))
        # the same error over |E_pair0| + |E_pairL| + |E_self|: the scale of the FP32
        # roundings, apart when a density's components nearly cancel
        dEc = max(abs(sum(e32) - sum(e64)) / sum(abs(x) for x in e64) for e32, e64 in zip(E32, E64))
        dv = float(torch.linalg.norm(v32 - v64) / torch.linalg.norm(v64))
        ach64 = 0.5 * near_pairs * FLOP_PER_UNORDERED_PAIR / (kms64 * 1e-3) / 1e12
        passed = bool(dE <= GATE_DE_REL and dv <= GATE_DV_REL)
        if not passed:
            print(f"# WARNING: FP32C misses the accuracy gate against FP64 (|dE|/|E| = {dE:.2e}, "
                  f"|dv|/|v| = {dv:.2e}; tolerances {GATE_DE_REL}, {GATE_DV_REL}): the rate does not count",
                  file=sys.stderr, flush=True)
        out["accuracy_gate"] = {"dE_rel_tol": GATE_DE_REL, "dv_rel_tol": GATE_DV_REL, "passed": passed,
                                "against": "GPU FP64 form, every density of the step"}
        out["fp64"] = {"value": rate64, "ms_per_step": 1e3 * dt64 / steps64, "kernel_ms": kms64,
                       "speedup_fp32c_over_fp64": value / rate64,
                       "fp32c_vs_fp64": {"dE_rel_max": dE, "dE_rel_max_of_components": dEc, "dv_rel_l2": dv,
                                         "within_gate": passed},
                       "roofline": {"bound": "alu", "achieved": ach64, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                    "frac": ach64 / PEAK_FP64_TFLOPS,
                                    "kernel": "pair_kernel<double, ADJ, %s>" % (
                                        "IMG" if a.workload in ("slab", "hexslab", "slabfar") else "noIMG")}}
        if a.workload == "kr":
            for t, s in enumerate(out["scan"]):
                e_ab, e_a, e_b = (sum(E64[3 * t + k]) for k in range(3))
                s["E_nl_minus_E_inf_fp64"] = e_ab - e_a - e_b
            gate = oracle_gate(W, E32, E64)
            if gate is not None:
                out["accuracy_gate"]["oracle"] = gate
                if not gate["passed"]:
                    out["accuracy_gate"]["passed"] = False
                    print("# WARNING: the stored densities miss the oracle gate", file=sys.stderr, flush=True)
        if a.kahan == 0 and not a.no_kahan and a.workload in ("kr", "kr1", "slab"):
            # the Kahan-compensated form (kahan = 1) beside the headline: rate and accuracy on the same step
            a.kahan = 1
            plans.clear()
            steps_k = max(1, a.steps // 2)
            dtk, Ek, vk, kmsk, _ = timed(V.VDW_FP32C, steps_k, 1)
            a.kahan = 0
            dEk = max(abs(sum(ek) - sum(e64)) / abs(sum(e64)) for ek, e64 in zip(Ek, E64))
            dvk = float(torch.linalg.norm(vk - v64) / torch.linalg.norm(v64))
            out["kahan"] = {"value": pairs * steps_k / dtk, "ms_per_step": 1e3 * dtk / steps_k, "kernel_ms": kmsk,
                            "vs_fp64": {"dE_rel_max": dEk, "dv_rel_l2": dvk,
                                        "within_gate": bool(dEk <= GATE_DE_REL and dvk <= GATE_DV_REL)}}
    if batched and a.workload != "dimer24":
        # energy only (no adjoint sums, no dE/dn): the same step as a plan without the potential
        p = V.BatchPlan(grids, offs, table, opts(main_prec), potential=False)
        p.capture(n)
        p.replay()
        torch.cuda.synchronize()
        steps_e = max(1, a.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps_e):
            p.replay()
        torch.cuda.synchronize()
        dte = time.perf_counter() - t0
        Ee = p.energies()
        out["energy_only"] = {"value": pairs * steps_e / dte, "ms_per_step": 1e3 * dte / steps_e,
                              "dE_rel_max_vs_fused": max(abs(sum(x) - sum(y)) / abs(sum(y)) for x, y in zip(Ee, E32))}
        p.close()
    if a.workload == "kr":
        # the exchange-correlation energies of Eq. (3) for the scan's densities
        # (outside the timed step; one call per density, each ending in a host wait)
        xcs = [V.xc_energies(gb, n[offs[b]:offs[b + 1]]) for b, gb in enumerate(grids)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xcs = [V.xc_energies(gb, n[offs[b]:offs[b + 1]]) for b, gb in enumerate(grids)]
        dtx = time.perf_counter() - t0
        e_nl = [sum(e) for e in E32]
        out["xc_energies"] = {"ms_per_density": 1e3 * dtx / len(grids), "grid_points": int(offs[1] - offs[0]),
                              "R7_dimer": dict(xcs[3], E_nl=e_nl[3],
                                               correction_pbe=V.recombine(xcs[3], e_nl[3], 0.0, "pbe"),
                                               correction_revpbe=V.recombine(xcs[3], e_nl[3], 0.0, "revpbe"))}
    if a.workload == "batch":
        # the same step as one call per density (q0, then energy + potential),
        # each with its own automatic tile shape
        def singles():
            res = []
            for b, gb in enumerate(grids):
                nb = n[offs[b]:offs[b + 1]]
                qb = V.compute_q0(gb, nb, wls[b].n_cut)
                res.append(V.enl_potential(gb, nb, qb, table, opts(main_prec))[0])
            return res
        singles()
        torch.cuda.synchronize()
        steps_s = max(1, a.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps_s):
            Es = singles()
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
        out["single_calls"] = {"value": pairs * steps_s / dts, "ms_per_step": 1e3 * dts / steps_s,
                               "batched_speedup": (pairs * a.steps / dt) / (pairs * steps_s / dts),
                               "dE_rel_max_vs_batched": max(abs(sum(x) - sum(y)) / abs(sum(y))
                                                            for x, y in zip(Es, E32))}
    if not a.no_cpu_baseline and a.workload in ("kr", "kr1"):
        cb = cpu_baseline(W.kr_dimer(7.0) if a.workload == "kr" else wl, a.cpu_rows)
        cb["per_core"] = cb["value"] / cb["cores"]
        if one_thread is not None:
            cb["one_thread"] = {"value": one_thread["value"], "sample": one_thread["sample"]}
        cb["context"] = ("the paper's timing (Sec. 5): 130 000 points in 36 min on one 2.13 GHz Core Duo core, "
                         "i.e. 7.8e6 ordered pairs/s")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def in_cut_pairs(wl):
    """Ordered pairs (i, j, L) of kept points with |r_i - r_j - L| <= r_cut,
    (i, i, 0) excluded, counted exactly from the kept mask: the numbers of
    kept pairs at every grid displacement d (the mask's autocorrelation, by
    FFT), times the number of near images L that keep d inside the cut.
    Host-side bookkeeping for the roofline's algorithmic work."""
    import numpy as np

    n = np.asarray(wl.n)
    mask = (wl.rho >= wl.n_cut).astype(np.float64)  # (nz, ny, nx)
    N = int(mask.sum())
    shape = tuple(2 * n[::-1])
    F = np.fft.rfftn(mask, shape)
    A = np.fft.irfftn(F * np.conj(F), shape)
    A = np.rint(A).astype(np.int64)
    # displacement d_a in (-n_a, n_a) at FFT index d mod 2 n_a
    dz, dy, dx = (np.fft.fftfreq(2 * n[a], 1.0 / (2 * n[a])).astype(np.int64) for a in (2, 1, 0))
    cell = np.asarray(wl.cell, dtype=np.float64) if wl.cell is not None else np.diag(np.asarray(wl.h) * n)
    E = cell / n[:, None]  # step vectors (rows)
    lim = [int(wl.image_max[a]) if wl.periodic[a] else 0 for a in range(3)]
    total = 0
    R2 = wl.r_cut * wl.r_cut
    for mx in range(-lim[0], lim[0] + 1):
        for my in range(-lim[1], lim[1] + 1):
            for mz in range(-lim[2], lim[2] + 1):
                ux = (dx - mx * n[0]).astype(np.float64)
                uy = (dy - my * n[1]).astype(np.float64)
                uz = (dz - mz * n[2]).astype(np.float64)
                X = uz[:, None, None] * E[2, 0] + uy[None, :, None] * E[1, 0] + ux[None, None, :] * E[0, 0]
                Y = uz[:, None, None] * E[2, 1] + uy[None, :, None] * E[1, 1] + ux[None, None, :] * E[0, 1]
                Z = uz[:, None, None] * E[2, 2] + uy[None, :, None] * E[1, 2] + ux[None, None, :] * E[0, 2]
                total += int(A[(X * X + Y * Y + Z * Z) <= R2].sum())
    return total - N


def oracle_gate(W, E32, E64):
    """Every density of the scan whose energies the oracle has stored at full
    size (tests/golden/fullsize_energies.json, written by
    tests/golden/make_fullsize_energies.py with the default table rule, the
    rule this benchmark's table is built with): |dE| per component over |E|
    of the density, FP32C and FP64, the largest of each and per density.
    None when the file or every entry is absent."""
    if not os.path.exists(GOLDEN):
        return None
    gold = json.load(open(GOLDEN)).get("workloads", {})
    res = {"source": os.path.relpath(GOLDEN, ROOT), "tol_fp32c": GATE_DE_REL, "tol_fp64": 1e-11}
    per, worst = {}, {"fp32c": 0.0, "fp64": 0.0}
    ok = True
    for t, R in enumerate(W.KR_SEPARATIONS):
        for k, which in enumerate(("both", "A", "B")):
            ref = gold.get("kr_dimer_R%g_%s" % (R, which))
            if ref is None:
                continue
            Eref = (ref["E_pair0"], ref["E_pairL"], ref["E_self"])
            scale = abs(sum(Eref))
            ds = []
            for name, E, tol in (("fp32c", E32, GATE_DE_REL), ("fp64", E64, 1e-11)):
                e = E[3 * t + k]
                d = max(abs(x - y) for x, y in zip(e, Eref)) / scale
                worst[name] = max(worst[name], d)
                ds.append(d)
                ok = ok and d <= tol
            per["R%g_%s" % (R, which)] = ds
    if not per:
        return None
    res["densities_compared"] = len(per)
    res["fp32c_dE_rel_max"] = worst["fp32c"]
    res["fp64_dE_rel_max"] = worst["fp64"]
    res["per_density_fp32c_fp64"] = per
    res["passed"] = ok
    return res


def cpu_baseline(wl, rows):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    q0 on the whole grid of one dimer, then the double-sum rows of a fixed
    random subset of the kept points against all kept points (energy +
    adjoint sums).  The oracle table (2048 x 64, a coarser quadrature rule: its
    values do not change the work per pair) is built before the clock starts."""
    import numpy as np

    from oracle import oracle as O

    print("# cpu baseline: building the oracle table", file=sys.stderr, flush=True)
    tp = O.table_params(n_D=2048, n_sigma=64, D_max=48.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    tab = O.build_table(tp)
    g = O.Grid(wl.n, wl.h, wl.periodic)
    threads = O.num_threads()
    t0 = time.perf_counter()
    qd = O.compute_q0(g, wl.rho, wl.n_cut)
    idx, ix, iy, iz = O._points(g, qd["keep"])
    N = len(idx)
    if rows <= 0:
        rows = max(64, int(1e9 * threads / N))  # about 15-20 s of oracle work
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(N, size=min(rows, N), replace=False)).astype(np.int64)
    r = wl.rho.reshape(-1)
    print(f"# cpu baseline: {len(sel)} rows x {N} points on {threads} threads", file=sys.stderr, flush=True)
    O.pair_rows(g, ix, iy, iz, r[idx], qd["q0"][idx], tab, tp, rows=sel)
    dt = time.perf_counter() - t0
    pairs = float(len(sel)) * (N - 1)
    return {"value": pairs / dt, "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{wl.name}: q0 on all {g.G} grid points + {len(sel)} of {N} rows of the double sum "
                      f"(E and dE/dq row sums, FP64, OpenMP), {dt:.1f} s"}


if __name__ == "__main__":
    main()
