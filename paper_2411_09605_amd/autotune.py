"""Launch-shape autotuner for the batched form.

Times a few steps of the batch for each candidate (threads per workgroup, particles per
work item) on the GPU and keeps the fastest; results are cached in a JSON file keyed by
the batch's shape so later runs skip the search.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Sequence, Tuple

CANDIDATES: Sequence[Tuple[int, int]] = ((256, 8192), (256, 16384), (256, 32768),
                                         (512, 16384), (512, 32768), (512, 65536))


def cache_path() -> str:
    return os.environ.get("PIC_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pic_batch_tune.json"))


def signature(runs) -> str:
    n = sum(r.n_particles for r in runs)
    g = max(r.n_cells for r in runs)
    r0 = runs[0]
    return f"{len(runs)}|{n >> 16}|{g}|{r0.order}|{r0.nv}|{r0.scheme}"


def _load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict):
    try:
        os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
        with open(cache_path(), "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune(runs, steps: int = 4, device="cuda", use_cache: bool = True, packed=None,
         candidates: Sequence[Tuple[int, int]] = CANDIDATES) -> Dict:
    """Return {'block_threads': t, 'chunk': c, 'ms_per_step': ms, 'trials': [...]}.

    ``packed`` (from ``pack_runs``) avoids packing the runs again; every candidate steps
    its own copy of the particles."""
    import torch
    from .binding import PicBatch, pack_runs
    key = signature(runs)
    cache = _load() if use_cache else {}
    if key in cache:
        return dict(cache[key], cached=True)
    if packed is None:
        packed = pack_runs(runs, device)
    trials = []
    best = None
    for bt, chunk in candidates:
        b = PicBatch(packed=packed, block_threads=bt, chunk=chunk)
        b.step(1)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(steps)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        trials.append({"block_threads": bt, "chunk": chunk, "ms_per_step": ms})
        if best is None or ms < best["ms_per_step"]:
            best = trials[-1]
        b.destroy()
        del b
        torch.cuda.empty_cache()
    out = dict(best, trials=trials, tuned_at=time.time())
    if use_cache:
        cache[key] = out
        _store(cache)
    return dict(out, cached=False)
