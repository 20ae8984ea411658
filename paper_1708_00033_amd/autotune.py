"""Autotuner for the per-class work decomposition of the Fock build.

For every quartet class the library exposes two scheduling knobs
(``hfx_set_class_tuning``): quartets per workgroup task and XCD striping of
long ket prefixes.  Results do not depend on them.  The tuner times each
candidate setting for all classes at once with the library's per-launch HIP
events, keeps each class's fastest setting, applies it and returns the table
(JSON-serialisable, keyed by class name).
"""
from __future__ import annotations

import json
from typing import Dict, Iterable, Sequence, Tuple

import numpy as np

from . import hfx

DEFAULT_CANDIDATES: Tuple[Tuple[int, int], ...] = (
    (2048, 0), (2048, 1), (8192, 0), (8192, 1), (32768, 0), (32768, 1))


PREFERRED: Tuple[int, int] = (32768, 0)


def autotune(ctx: "hfx.Context", dD_ptr: int, dF_ptr: int, stream: int,
             candidates: Sequence[Tuple[int, int]] = DEFAULT_CANDIDATES, reps: int = 2,
             sync=None, prefer: Tuple[int, int] = PREFERRED, margin: float = 0.03) -> Dict[str, dict]:
    """Return {class name: {"task_quartets", "xcd_stripe", "ms", "candidates_ms"}}.

    A class keeps the ``prefer`` setting (when it is a candidate) unless another
    candidate is faster by more than ``margin`` (relative): timing noise then
    does not flip the launch shape from one run to the next."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times = np.full((len(candidates), 21), np.inf)
    for ci, (tq, st) in enumerate(candidates):
        ctx.set_class_tuning(-1, tq, st)
        ctx.build_fock_dev(dD_ptr, dF_ptr, stream)   # warm-up
        sync()
        ctx.kernel_timing(True)
        for _ in range(reps):
            ctx.build_fock_dev(dD_ptr, dF_ptr, stream)
        sync()
        ms, n = ctx.kernel_times()
        ctx.kernel_timing(False)
        times[ci] = ms / np.maximum(n, 1)
    table = {}
    for k in range(21):
        best = int(np.argmin(times[:, k]))
        if tuple(prefer) in [tuple(c) for c in candidates]:
            pi = [tuple(c) for c in candidates].index(tuple(prefer))
            if times[pi, k] <= times[best, k] * (1.0 + margin):
                best = pi
        tq, st = candidates[best]
        table[hfx.CLASS_NAMES[k]] = {"task_quartets": int(tq), "xcd_stripe": int(st),
                                      "ms": float(times[best, k]),
                                      "candidates_ms": [round(float(x), 4) for x in times[:, k]]}
    apply(ctx, table)
    return table


def apply(ctx: "hfx.Context", table: Dict[str, dict]) -> None:
    for name, v in table.items():
        ctx.set_class_tuning(hfx.CLASS_NAMES.index(name), int(v["task_quartets"]), int(v["xcd_stripe"]))


def save(table: Dict[str, dict], path: str) -> None:
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)


def load(path: str) -> Dict[str, dict]:
    with open(path) as fh:
        return json.load(fh)


def summary(table: Dict[str, dict], classes: Iterable[str] = ()) -> Dict[str, Tuple[int, int]]:
    return {k: (v["task_quartets"], v["xcd_stripe"]) for k, v in table.items() if not classes or k in classes}
