"""Online autotuner of a batch's launch shapes.

The result of a step does not depend on the launch shape (every face flux and every
per-tile partial sum is computed the same way whatever workgroup handles it), so the
tuner times candidate shapes on the live batch: the steps it spends measuring are real
steps of the solves.  Searched: for each face-kernel class present, the persistent grid
(one workgroup per tile, or 4/8/16 workgroups per CU) and, for the 2D classes, the cell-tile
shape of the fused kernel (16 x 15, 32 x 7 or 8 x 28); then the grid of the strain kernel
and, with 3D members, of the update kernel.  The winner is cached in a JSON
file keyed by device, class mix and problem size, and reused without a search.
"""
from __future__ import annotations

import json
import os
import time

KIND_STRAIN, KIND_UPDATE = 0, 5
TILE2_SHAPES = (0, 1, 2)     # GKS_TILE2_16X15, GKS_TILE2_32X7, GKS_TILE2_8X28


def tiles_of(c: int):
    """Tile choices of a face class: the fused 2D kernel's cell-tile shape for the 2D
    classes (0, 1); none for 3D (the fused 3D column and the 3D face kernel of the options
    outside it have fixed tiles)."""
    return TILE2_SHAPES if c < 2 else (0,)


def cls_of(case) -> int:
    return (2 if case.dim == 3 else 0) + (1 if case.precision == "fp32_flux" else 0)


def default_cache_path() -> str:
    return os.environ.get("GKS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gks", "autotune.json"))


def _signature(batch) -> str:
    import torch
    name = torch.cuda.get_device_properties(torch.cuda.current_device()).name
    classes = sorted({cls_of(s.case) for s in batch.solvers})
    cells = sum(s.case.ncells for s in batch.solvers)
    bucket = 1 << max(int(cells).bit_length() - 1, 0)        # power-of-two size class
    return f"{name}|classes={classes}|cells~{bucket}|members~{len(batch.solvers)}|fused2d3d"


def _time_steps(batch, n: int) -> float:
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(n)
    e1.record(batch.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(batch, shape: dict) -> None:
    for c, (grid, tile) in shape.get("face", {}).items():
        batch.set_launch(1 + int(c), grid, tile)
    batch.set_launch(KIND_STRAIN, shape["strain_grid"], 0)
    batch.set_launch(KIND_UPDATE, shape["update_grid"], 0)


def autotune(batch, steps_per_trial: int = 2, cache_path: str | None = None, use_cache: bool = True):
    """Pick launch shapes for `batch` (a paper_1302_2132_amd.Batch).  Returns
    (shape, steps_spent, seconds_spent)."""
    import torch
    cache_path = cache_path or default_cache_path()
    key = _signature(batch)
    cache = _load(cache_path)
    if use_cache and key in cache:
        apply(batch, cache[key])
        return cache[key], 0, 0.0
    t_start = time.perf_counter()
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    grids = (0, 4 * cus, 8 * cus, 16 * cus)
    classes = sorted({cls_of(s.case) for s in batch.solvers})
    steps = 0
    shape = {"face": {}, "strain_grid": 8 * cus, "update_grid": 8 * cus}
    for c in classes:
        trials = []
        for tile in tiles_of(c):
            for g in grids:
                batch.set_launch(1 + c, g, tile)
                batch.step(1)                       # first launch of a new shape: warm
                trials.append((_time_steps(batch, steps_per_trial), g, tile))
                steps += 1 + steps_per_trial
        _, g, tile = min(trials)
        batch.set_launch(1 + c, g, tile)
        shape["face"][str(c)] = [g, tile]
    kinds = [(KIND_STRAIN, "strain_grid")]
    if any(c >= 2 for c in classes):
        kinds.append((KIND_UPDATE, "update_grid"))
    for kind, keyname in kinds:
        trials = []
        for g in grids:
            batch.set_launch(kind, g, 0)
            batch.step(1)
            trials.append((_time_steps(batch, steps_per_trial), g))
            steps += 1 + steps_per_trial
        _, g = min(trials)
        batch.set_launch(kind, g, 0)
        shape[keyname] = g
    cache[key] = shape
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return shape, steps, time.perf_counter() - t_start
