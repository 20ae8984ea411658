"""Autotuner for the per-class work decomposition of the Fock build.

For every quartet class the library exposes four scheduling knobs
(``hfx_set_class_tuning``): quartets per workgroup task, XCD striping of
long ket prefixes, the launch form (one workgroup per task, a persistent
resident grid fed by per-XCD atomic work counters, or such a grid with one
task per wave for short tasks, or register-tiled grids) and the digestion
(bra rows of F staged in LDS, with or without the bra rows of D, global
atomics into one matrix, or into per-XCD private copies).  Results do not depend on them.  The tuner times each
candidate setting for all classes at once with the library's per-launch HIP
events, keeps each class's fastest setting, applies it and returns the table
(JSON-serialisable, keyed by class name).
"""
from __future__ import annotations

import json
from typing import Dict, Iterable, Sequence, Tuple

import numpy as np

from . import hfx

DEFAULT_CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = (
    (2048, 0, 0, -1), (2048, 1, 0, -1), (8192, 0, 0, -1), (8192, 1, 0, -1), (32768, 0, 0, -1), (32768, 1, 0, -1),
    (2048, 1, 1, -1), (8192, 1, 1, -1), (8192, 0, 0, 1), (32768, 0, 0, 1), (8192, 1, 2, -1), (32768, 0, 2, -1),
    (32768, 0, 3, -1), (32768, 0, 4, -1), (8192, 1, 4, -1), (32768, 0, 1, 2), (32768, 0, 1, -1),
    (32768, 0, 1, 0), (8192, 1, 0, 0))


# Kept unless another candidate is clearly faster: the persistent form, whose
# resident workgroups drain the XCD queues in order, re-reads the ket lists
# from HBM several times less than one workgroup per task at about the same
# speed.
PREFERRED: Tuple[int, int, int, int] = (32768, 0, 1, -1)
_PAD = (0, 0, 0, -1)


def _full(c) -> Tuple[int, int, int, int]:
    c = tuple(int(x) for x in c)
    return c + _PAD[len(c):]


def autotune(ctx: "hfx.Context", dD_ptr: int, dF_ptr: int, stream: int,
             candidates: Sequence[Tuple[int, ...]] = DEFAULT_CANDIDATES, reps: int = 2,
             sync=None, prefer: Tuple[int, ...] = PREFERRED, margin: float = 0.03) -> Dict[str, dict]:
    """Return {class name: {"task_quartets", "xcd_stripe", "persistent", "digest", "ms", "candidates_ms"}}.
    A candidate is (task_quartets, xcd_stripe[, persistent[, digest]]).

    A class keeps the ``prefer`` setting (when it is a candidate) unless another
    candidate is faster by more than ``margin`` (relative): timing noise then
    does not flip the launch shape from one run to the next."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times = np.full((len(candidates), 21), np.inf)
    cands = [_full(c) for c in candidates]
    prefer = _full(prefer)
    for ci, (tq, st, pe, dg) in enumerate(cands):
        ctx.set_class_tuning(-1, tq, st, pe, dg)
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
        if prefer in cands:
            pi = cands.index(prefer)
            if times[pi, k] <= times[best, k] * (1.0 + margin):
                best = pi
        tq, st, pe, dg = cands[best]
        table[hfx.CLASS_NAMES[k]] = {"task_quartets": int(tq), "xcd_stripe": int(st), "persistent": int(pe),
                                      "digest": int(dg),
                                      "ms": float(times[best, k]),
                                      "candidates_ms": [round(float(x), 4) for x in times[:, k]]}
    apply(ctx, table)
    return table


def autotune_precision(ctx: "hfx.Context", dD_ptr: int, dF_ptr: int, stream: int, reps: int = 2, sync=None,
                       margin: float = 0.02) -> Dict[str, dict]:
    """For a context configured for mixed builds: time every class with its
    FP32 kernel on and off, keep FP32 where it is faster by more than
    ``margin`` (FP64 is never less accurate), apply and return
    {class name: {"fp32", "ms_fp32", "ms_fp64"}}."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times = np.full((2, 21), np.inf)
    for on in (0, 1):
        ctx.set_class_precision(-1, on)
        ctx.build_fock_dev(dD_ptr, dF_ptr, stream)
        sync()
        ctx.kernel_timing(True)
        for _ in range(reps):
            ctx.build_fock_dev(dD_ptr, dF_ptr, stream)
        sync()
        ms, n = ctx.kernel_times()
        ctx.kernel_timing(False)
        times[on] = ms / np.maximum(n, 1)
    table = {}
    for k in range(21):
        on = int(times[1, k] < times[0, k] * (1.0 - margin))
        ctx.set_class_precision(k, on)
        table[hfx.CLASS_NAMES[k]] = {"fp32": on, "ms_fp32": float(times[1, k]), "ms_fp64": float(times[0, k])}
    return table


def apply(ctx: "hfx.Context", table: Dict[str, dict]) -> None:
    for name, v in table.items():
        ctx.set_class_tuning(hfx.CLASS_NAMES.index(name), int(v["task_quartets"]), int(v["xcd_stripe"]),
                             int(v.get("persistent", 0)), int(v.get("digest", -1)))


def save(table: Dict[str, dict], path: str) -> None:
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)


def load(path: str) -> Dict[str, dict]:
    with open(path) as fh:
        return json.load(fh)


def summary(table: Dict[str, dict], classes: Iterable[str] = ()) -> Dict[str, Tuple[int, int, int, int]]:
    return {k: (v["task_quartets"], v["xcd_stripe"], v.get("persistent", 0), v.get("digest", -1))
            for k, v in table.items() if not classes or k in classes}
