"""Tile-class autotuner.

The per-particle kernels map one outer particle to a segment of SEG lanes
with JPT inner particles per lane (dpf_tile_classes).  Several classes hold a
given inner size M; which one is fastest depends on the model (registers per
inner particle, reductions across waves versus work per lane) and on M.  The
tuner times every class that holds M with little idle room (SEG * JPT < 2M,
or the default class) on a probe filter of the model, as replays of a
captured run, and keeps the fastest; tables are saved as JSON keyed by the
device and model.
"""
import json
import os
import time

import numpy as np

from . import Filter, tile_classes


def _torch():
    import torch
    return torch


def candidates(M):
    """Class indices that hold M inner particles without idling half a segment
    or more, plus the default class."""
    cls = tile_classes()
    out = [k for k, (seg, jpt) in enumerate(cls) if M <= seg * jpt < 2 * M]
    default = next(k for k, (seg, jpt) in enumerate(cls[:6]) if M <= seg * jpt)
    if default not in out:
        out.append(default)
    return sorted(out)


def time_class(spec, M, cls, N=1024, steps=16, reps=3, algo="lookahead", device="cuda", simulate=None,
               seed=3, n_filters=32):
    """Milliseconds per step of the model's step with tile class cls on a
    probe batch of n_filters filters of N outer particles (enough work to
    fill the GPU), best of reps graph-replayed runs of `steps` steps."""
    torch = _torch()
    _, _, ys = simulate(spec, steps, 123)
    Y = torch.tensor(np.repeat(ys[:, None, :], n_filters, axis=1), dtype=torch.float32, device=device)
    f = Filter(spec.kind, spec.dx, spec.dz, spec.dy, spec.blob, [N] * n_filters, [M] * n_filters, seed=seed,
               algo=algo, device=device)
    f.set_tiling([cls] * n_filters)
    f.run(Y, trace=False, use_graph=True)  # capture and warm up
    best = float("inf")
    for _ in range(reps):
        f.reset()
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        f.run(Y, trace=False, use_graph=True)
        torch.cuda.synchronize(device)
        best = min(best, (time.perf_counter() - t0) * 1e3 / steps)
    f.close()
    return best


def tune(spec, Ms, N=1024, steps=16, reps=3, algo="lookahead", device="cuda", simulate=None, n_filters=32):
    """{M: {"class": best class, "ms": {class: ms per step}}} for each M."""
    table = {}
    for M in sorted(set(int(m) for m in Ms)):
        ms = {k: time_class(spec, M, k, N, steps, reps, algo, device, simulate, n_filters=n_filters)
              for k in candidates(M)}
        table[M] = {"class": min(ms, key=ms.get), "ms": ms}
    return table


def classes_for(table, Ms):
    """Per-filter class list for inner sizes Ms (-1 where the table has no entry)."""
    return [table[int(m)]["class"] if int(m) in table else -1 for m in Ms]


def save(table, path, spec, algo="lookahead"):
    torch = _torch()
    key = "%s|model%d|%d,%d,%d|%s" % (torch.cuda.get_device_name(0), spec.kind, spec.dx, spec.dz, spec.dy, algo)
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = {str(m): {"class": v["class"], "ms": {str(k): t for k, t in v["ms"].items()}}
                 for m, v in table.items()}
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def load(path, spec, algo="lookahead"):
    torch = _torch()
    key = "%s|model%d|%d,%d,%d|%s" % (torch.cuda.get_device_name(0), spec.kind, spec.dx, spec.dz, spec.dy, algo)
    with open(path) as fh:
        data = json.load(fh).get(key, {})
    return {int(m): {"class": v["class"], "ms": {int(k): t for k, t in v["ms"].items()}} for m, v in data.items()}
