"""Autotuner for the mixed-request layer launches: picks, per (slot size, precision) bucket,
how many persistent workgroups per compute unit the layer launch uses, by timing candidate
settings on the caller's own requests.  Results are cached as JSON keyed by device name, so a
serving process tunes once and reloads the choice on start.
"""
from __future__ import annotations

import json
import os

from . import anomps, mixed

DEFAULT_CANDIDATES = (1, 2, 4, 8, 0)  # 0 = as many as fit (the library default)


def bucket_of(spec: mixed.RequestSpec) -> int:
    S = anomps.slot_dim(spec.n, spec.chi, spec.layers)
    return 4 * (spec.precision == anomps.PREC_FP32) + {2: 0, 4: 1, 8: 2, 16: 3}[S]


def _time_layers(mr: mixed.MixedRequests, repeats: int) -> float:
    import torch
    best = float("inf")
    for _ in range(repeats):
        mr.init()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(mr.max_layers):
            mr.step()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(specs, candidates=DEFAULT_CANDIDATES, repeats: int = 2) -> dict:
    """Time every candidate on each bucket's requests; returns {bucket: (blocks_per_cu, ms)}."""
    groups: dict = {}
    for sp in specs:
        groups.setdefault(bucket_of(sp), []).append(sp)
    choice = {}
    for b, group in sorted(groups.items()):
        mr = mixed.MixedRequests(group)
        timings = {}
        for c in candidates:
            anomps.set_mixed_tuning(b, c)
            timings[c] = _time_layers(mr, repeats)
        best = min(timings, key=timings.get)
        anomps.set_mixed_tuning(b, best)
        choice[b] = (best, timings[best], timings)
        del mr
    return choice


def device_key() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def save(choice: dict, path: str) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[device_key()] = {str(b): int(c[0]) for b, c in choice.items()}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_and_apply(path: str) -> dict:
    """Apply a cached choice for this device (if any); returns {bucket: blocks_per_cu}."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f).get(device_key(), {})
    for b, c in data.items():
        anomps.set_mixed_tuning(int(b), int(c))
    return {int(b): int(c) for b, c in data.items()}
