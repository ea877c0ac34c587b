"""Autotuner for the work shape of the pair kernels.

The two knobs of ``gbmc_tuning`` (j blocks walked per work item, independent
wavefronts per workgroup) change only the schedule, never the result (every
64 x 64 tile is rounded into fixed point on its own), so the tuner can pick
them by timing alone.  It times the three pair kernels with the library's HIP
event hook on the caller's actual batch and keeps the fastest shape.  Results
are cached in a JSON file keyed by precision and a size bucket of the batch.
"""
from __future__ import annotations

import json
import math
import os
import statistics
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np
import torch

from . import api

J_BLOCKS = (1, 2, 4, 8, 16)
WAVES = (1, 2, 4, 8)
PAIR_KERNELS = ("radii_pairs", "energy_pairs", "chain_pairs")

_CACHE_ENV = "GBMC_TUNING_CACHE"


def cache_path() -> str:
    return os.environ.get(_CACHE_ENV,
                          os.path.join(os.path.expanduser("~"), ".cache", "gbmc", "tuning.json"))


def bucket_key(atom_offset: Sequence[int], precision: str) -> str:
    """Size bucket of a batch: system count and largest system (powers of two)
    plus the total number of 64 x 64 tiles (powers of two)."""
    n = np.diff(np.asarray(atom_offset, dtype=np.int64))
    nb = (n + 63) // 64
    tiles = int((nb * (nb + 1) // 2).sum())
    lg = lambda v: int(math.ceil(math.log2(max(1, v))))
    return f"{precision}:B{lg(len(n))}:N{lg(int(n.max()) if n.size else 1)}:T{lg(tiles)}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(cache: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def lookup(atom_offset: Sequence[int], precision: str = "fp32"):
    """Cached (j_blocks_per_item, waves_per_group) triples for this size bucket, or None."""
    hit = _load_cache().get(bucket_key(atom_offset, precision))
    return (tuple(hit["j_blocks_per_item"]), tuple(hit["waves_per_group"])) if hit else None


def tune(batch, precision: str = "fp32", order: Optional[np.ndarray] = None,
         params: api.GBParams = api.IGB5, reps: int = 3,
         candidates: Optional[Iterable[Tuple[int, int]]] = None, use_cache: bool = True) -> dict:
    """Time every (j_blocks_per_item, waves_per_group) candidate on ``batch``
    (any object with atom_offset, x, y, z, q, rho, screen), applied to all three
    pair passes, and pick the fastest shape of each pass.  Returns
    {"best": ((jb radii, energy, chain), (wv radii, energy, chain)), ...}."""
    key = bucket_key(batch.atom_offset, precision)
    cands = list(candidates) if candidates is not None else [(j, w) for j in J_BLOCKS for w in WAVES]
    table, per_kernel = {}, {}
    for jb, wv in cands:
        plan = api.Plan(batch.atom_offset, precision, j_blocks_per_item=jb, waves_per_group=wv)
        if order is not None:
            plan.set_order(order)
        atoms = api.Atoms.from_batch(plan, batch)
        api.radii(plan, atoms, params)                  # warm-up (code objects, caches)
        api.energy_forces(plan, atoms, params)
        plan.set_timing(True)
        runs, per = [], {k: [] for k in PAIR_KERNELS}
        for _ in range(reps):
            api.radii(plan, atoms, params)
            api.energy_forces(plan, atoms, params)
            ms = plan.kernel_ms()
            runs.append(sum(ms.get(k, 0.0) for k in PAIR_KERNELS))
            for k in PAIR_KERNELS:
                per[k].append(ms.get(k, 0.0))
        plan.set_timing(False)
        table[f"{jb}x{wv}"] = statistics.median(runs)
        per_kernel[f"{jb}x{wv}"] = {k: statistics.median(v) for k, v in per.items()}
        del plan, atoms
    torch.cuda.synchronize()
    # the passes are separate launches: each takes its own fastest shape
    jbs, wvs, total = [], [], 0.0
    for k in PAIR_KERNELS:
        shape = min(per_kernel, key=lambda c: per_kernel[c][k])
        jb, wv = (int(v) for v in shape.split("x"))
        jbs.append(jb)
        wvs.append(wv)
        total += per_kernel[shape][k]
    best = (tuple(jbs), tuple(wvs))
    if use_cache:
        cache = _load_cache()
        cache[key] = {"j_blocks_per_item": list(jbs), "waves_per_group": list(wvs), "pair_ms": total}
        _save_cache(cache)
    return {"key": key, "best": best, "pair_ms": total, "ms": table, "per_kernel_ms": per_kernel}
