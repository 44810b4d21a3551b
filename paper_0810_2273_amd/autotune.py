"""Tile autotuner for the pair kernel.

Two tile parameters are free.  The j-chunk length of the off-diagonal work
items (``Opts.j_chunks`` x 1024 points): short chunks give many small items
(good load balance, more partial sums to write and reduce), long chunks the
opposite; chunks shorter than a row block also split its diagonal work.
The workgroup shape (``Opts.block_threads``): 1024 threads (row blocks of
4096 points for the FP32 n_sigma = 64 kernels, 2048 otherwise); 512 with
eight i-points per lane for the FP32 n_sigma = 64 kernels without images
(fewer instructions per pair, half the wavefronts to hide LDS and L2
latency); 256 with row blocks of 512 points for any kernel without images
(more, smaller items for densities too small to fill the chip).  There is
one workgroup per CU in every shape because the table fills the LDS.
``tune`` times the pair kernel (HIP events around the launch, read back
through ``last_stats``) for each candidate and caches the fastest per device
and workload class.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time
from dataclasses import replace

import torch

from . import api

CANDIDATES = (2, 4, 8, 16, 32)
BLOCK_THREADS = (1024, 512, 256)


def _cache_path() -> str:
    base = os.environ.get("VDW_AUTOTUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_0810_2273_amd", "autotune.json")


def _key(kept: int, nimg: int, precision: int, potential: bool, batch: int) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    # workload class: kept points rounded to a power of two, images, form, batch size
    cls = 1 << max(0, int(math.log2(max(kept, 1))))
    return f"{dev}|N~{cls}|img{nimg}|p{precision}|adj{int(potential)}|B{batch}"


def _load() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home: tuning still works, it is just not remembered


def tune(run, opts: api.Opts, kept: int, nimg: int = 1, potential: bool = True, batch: int = 1,
         candidates=CANDIDATES, block_threads=BLOCK_THREADS, repeats: int = 2, use_cache: bool = True,
         verbose: bool = False) -> api.Opts:
    """Pick ``j_chunks`` and ``block_threads`` for ``run(opts)`` (a callable
    doing one evaluation) by timing the pair kernel; returns a copy of
    ``opts`` with the choice.  Workgroup shapes that the options' kernel
    variant does not have (it reports another size) are skipped."""
    key = _key(kept, nimg, opts.precision, potential, batch)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        return replace(opts, j_chunks=int(c["j_chunks"]), block_threads=int(c.get("block_threads", 0)))
    best, best_ms, report = None, math.inf, {}
    api.set_timing(True)
    try:
        for bt in block_threads:
            for jc in candidates:
                o = replace(opts, j_chunks=jc, block_threads=bt)
                run(o)  # warm
                if api.last_stats()["block_threads"] != bt:
                    break  # this variant has one workgroup shape only
                ms = []
                for _ in range(repeats):
                    run(o)
                    ms.append(api.last_stats()["pair_kernel_ms"])
                t = min(ms)
                report[f"{bt}/{jc}"] = t
                if verbose:
                    print(f"# autotune block_threads={bt} j_chunks={jc}: {t:.3f} ms", file=sys.stderr, flush=True)
                if t < best_ms:
                    best, best_ms = (bt, jc), t
    finally:
        api.set_timing(False)
    cache[key] = {"block_threads": best[0], "j_chunks": best[1], "ms": best_ms, "sweep": report,
                  "when": time.time()}
    if use_cache:
        _store(cache)
    return replace(opts, block_threads=best[0], j_chunks=best[1])
