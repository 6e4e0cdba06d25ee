"""Autotuner for batched BDIS.

For each image-size class it times the batch kernel on calibration pairs
for every candidate (patch, stride) and keeps the fastest one whose accuracy
stays within a guard of the default (8, 4): end-point error against the
generated ground truth at most `guard` times the default's, coverage at least
`cover` times the default's.  It then picks the batch execution (a graph of per-level launches, or the
persistent kernel at a given number of workgroups per compute unit) for the
tuned batch.  The result is a plain
JSON-able dict; `apply` installs it in a handle (bdis_set_tuning and
bdis_set_batch_mode).
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

from . import bdis

CANDIDATES = [(8, 3), (8, 4), (8, 6), (12, 3), (12, 4), (12, 6)]
DEFAULT = (8, 4)


def _epe(d, gt, valid):
    m = np.isfinite(d) & valid
    if not m.any():
        return float("inf"), 0.0
    return float(np.abs(d[m] - gt[m]).mean()), float(m.sum() / max(valid.sum(), 1))


def _time_batch(h, lefts, rights, outs, dmax, reps):
    import torch
    h.compute_batch(lefts, rights, outs, max_disparity=dmax)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        h.compute_batch(lefts, rights, outs, max_disparity=dmax)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(base: bdis.Params, classes, candidates=CANDIDATES, guard=1.02, cover=0.98,
         reps=5, device=0, log=None):
    """classes: ascending list of (max_width, [calibration StereoPair ...]).
    Returns {"table": [[max_width, patch, stride], ...], "wgs_per_cu": n,
    "report": {...}}."""
    import torch
    dev = torch.device(f"cuda:{device}")
    table, report = [], {}
    for (max_w, pairs) in classes:
        L = [torch.from_numpy(p.left).to(dev) for p in pairs]
        R = [torch.from_numpy(p.right).to(dev) for p in pairs]
        O = [torch.empty(p.left.shape, dtype=torch.float32, device=dev) for p in pairs]
        dm = [p.d_max for p in pairs]
        rows = {}
        for (pa, st) in candidates:
            h = bdis.Bdis(dataclasses.replace(base, patch=pa, stride=st, autotune=0), device)
            h.set_batch_mode(0)
            ms = _time_batch(h, L, R, O, dm, reps)
            errs = [_epe(o.cpu().numpy(), p.disp, p.valid) for o, p in zip(O, pairs)]
            rows[(pa, st)] = (ms, float(np.mean([e[0] for e in errs])), float(np.mean([e[1] for e in errs])))
            h.close()
            if log:
                log(f"autotune {max_w}: patch {pa} stride {st}: {ms:.3f} ms, EPE {rows[(pa, st)][1]:.3f}, "
                    f"coverage {rows[(pa, st)][2]:.3f}")
        ref_ms, ref_epe, ref_cov = rows[DEFAULT]
        ok = [c for c, (ms, e, cv) in rows.items() if e <= guard * ref_epe and cv >= cover * ref_cov]
        best = min(ok, key=lambda c: rows[c][0])
        table.append([int(max_w), int(best[0]), int(best[1])])
        report[str(max_w)] = {f"{c[0]}x{c[1]}": {"ms": v[0], "epe": v[1], "coverage": v[2]}
                              for c, v in rows.items()}
    # batch execution for the tuned batch: the per-level graph, or the
    # persistent kernel at each grid density
    prm = dataclasses.replace(base, autotune=1)
    h = bdis.Bdis(prm, device)
    h.set_tuning([tuple(t) for t in table])
    allp = [p for (_, ps) in classes for p in ps]
    L = [torch.from_numpy(p.left).to(dev) for p in allp]
    R = [torch.from_numpy(p.right).to(dev) for p in allp]
    O = [torch.empty(p.left.shape, dtype=torch.float32, device=dev) for p in allp]
    dm = [p.d_max for p in allp]
    runs = {}
    for mode, w in ((0, 0), (2, 0), (2, 1), (2, 2)):
        if mode == 2 and any(t[1] not in (8, 12) for t in table):
            continue
        h.set_batch_mode(mode, w)
        runs[(mode, w)] = _time_batch(h, L, R, O, dm, reps)
        if log:
            log(f"autotune execution: mode {mode} workgroups/CU {w or 'max'}: {runs[(mode, w)]:.3f} ms")
    h.close()
    mode, wgs = min(runs, key=runs.get)
    return {"table": table, "batch_mode": int(mode), "wgs_per_cu": int(wgs), "report": report,
            "execution_ms": {f"mode{m}_wgs{w}": v for (m, w), v in runs.items()}}


def apply(h: bdis.Bdis, tuned: dict):
    h.set_tuning([tuple(t) for t in tuned["table"]])
    h.set_batch_mode(int(tuned.get("batch_mode", 0)), int(tuned.get("wgs_per_cu", 0)))


def save(tuned: dict, path: str | None = None) -> str:
    path = path or os.environ.get("BDIS_TUNING_CACHE", "bdis_tuning.json")
    with open(path, "w") as f:
        json.dump(tuned, f, indent=1)
    return path


def load(path: str | None = None) -> dict | None:
    path = path or os.environ.get("BDIS_TUNING_CACHE", "bdis_tuning.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)
