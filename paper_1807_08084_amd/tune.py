"""Autotuner for the launch shapes of the per-call kernels, with a JSON cache.

The inverse kernel is tuned inside the library (polsar_autotune_inv_det:
every block x unroll x grid x non-temporal x access-width candidate, timed
with HIP events on the caller's buffers).  The Wishart kernel is swept here
through polsar_set_launch with the same timing.  A table of winners can be
saved to JSON (keyed by device name and compute-unit count) and installed
again with :func:`load`.
"""
from __future__ import annotations

import itertools
import json

import torch

from . import ops

OPS = {"inv_det": 0, "wishart": 1, "multilook": 2, "batch": 3, "wishart_small": 5}


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_inv_det(z: torch.Tensor, method: str, precision: str, reps: int = 10):
    return ops.autotune_inv_det(z, method, precision, reps=reps)


BPC = (0, 2, 3, 4, 5, 6, 8)  # resident-block caps tried


def wishart_candidates():
    for b, u, g, vb, bpc in itertools.product((64, 128, 256), (1, 2), (0, 8), (16, 8), BPC):
        yield dict(block=b, unroll=u, grid_per_cu=g, nontemporal=1, vector_bytes=vb, blocks_per_cu=bpc)


def tune_wishart(sigma: torch.Tensor, z: torch.Tensor, n_looks: float, reps: int = 10):
    """Sweep the Wishart forward+backward launch; install the best in the
    table entry that calls of this size use (op 1, or op 5 for small
    images) and return it."""
    n = sigma[0].numel()
    op = ops.wishart_launch_op(n)
    ws = torch.empty(ops.workspace_bytes(sigma.dtype, n) // 8 + 1, dtype=torch.float64, device=sigma.device)
    best, best_ms = None, float("inf")
    for cfg in wishart_candidates():
        ops.set_launch(op, sigma.dtype, "adjugate", "plain", cfg)
        ms = _time(lambda: ops.wishart_loglik(sigma, z, n_looks, forward=True, backward=True, workspace=ws), reps)
        if ms < best_ms:
            best, best_ms = cfg, ms
    ops.set_launch(op, sigma.dtype, "adjugate", "plain", best)
    return best, best_ms


def tune_multilook(looks: torch.Tensor, n_looks: int, method: str = "adjugate", precision: str = "compensated",
                   reps: int = 10):
    best, best_ms = None, float("inf")
    for b, g, vb, bpc in itertools.product((64, 128, 256), (0, 8), (16, 8), BPC):
        cfg = dict(block=b, unroll=1, grid_per_cu=g, nontemporal=1, vector_bytes=vb, blocks_per_cu=bpc)
        ops.set_launch(2, looks.dtype, method, precision, cfg)
        ms = _time(lambda: ops.multilook_inv_det(looks, n_looks, method, precision), reps)
        if ms < best_ms:
            best, best_ms = cfg, ms
    ops.set_launch(2, looks.dtype, method, precision, best)
    return best, best_ms


def tune_batch(items, method: str = "adjugate", precision: str = "compensated", reps: int = 5):
    """Sweep the batch launch (block; one block per tile or a persistent
    grid of g blocks per CU; access width; resident-block cap); each
    candidate builds its own plan (and graph)."""
    from .batch import BatchPlan
    dtype = items[0]["z"].dtype
    best, best_ms = None, float("inf")
    for b, g, vb, bpc in itertools.product((64, 128, 256), (0, 2, 4, 8), (16, 8), (0, 4, 8, 16)):
        if bpc and g > bpc:
            continue  # a persistent grid larger than what can be resident
        if bpc * b > 2048:
            continue  # more lanes than a CU holds
        cfg = dict(block=b, unroll=1, grid_per_cu=g, nontemporal=1, vector_bytes=vb, blocks_per_cu=bpc)
        ops.set_launch(3, dtype, method, precision, cfg)
        plan = BatchPlan(items, method, precision, status=False)
        ms = _time(plan.run, reps)
        plan.close()
        if ms < best_ms:
            best, best_ms = cfg, ms
    ops.set_launch(3, dtype, method, precision, best)
    return best, best_ms


def device_key() -> str:
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def save(path: str, table: dict) -> None:
    with open(path, "w") as fh:
        json.dump({"device": device_key(), "entries": table}, fh, indent=1)


def load(path: str, strict_device: bool = True) -> int:
    """Install a saved table; returns the number of entries installed."""
    rec = json.load(open(path))
    if strict_device and rec.get("device") != device_key():
        return 0
    n = 0
    for key, ent in rec["entries"].items():
        op, dt, method, prec = key.split("/")
        ops.set_launch(OPS[op], torch.float32 if dt == "f32" else torch.float64, method, prec, ent["cfg"])
        n += 1
    return n
