"""Autotuner of the library's launch schedules, chosen by timing candidates on the caller's own
work:

* mixed-request layer launches: per (slot size, precision) bucket, how many persistent
  workgroups per compute unit the layer launch uses (``tune``);
* the measurement's 16-wide pair kernel: the launch order (blocks of images, start site major
  inside a block) and a cap on resident workgroups per compute unit (``tune_measure``), for a
  batch shape (sites, bond limit, depth, batch size, precision).

Every candidate runs the same arithmetic per image (only the grid, the order of the workgroups
or their occupancy changes), so the choice never changes a result; tests check that bit for
bit.  Results are cached as JSON keyed by device name, so a process tunes once and reloads the
choice on start.
"""
from __future__ import annotations

import json
import os

from . import anomps, mixed

DEFAULT_CANDIDATES = (1, 2, 4, 8, 0)  # 0 = as many as fit (the library default)
# pair-kernel schedules: (images per block, resident workgroups per CU); the library default is
# (64, 0), (0, 0) one block of the whole batch with no cap
MEASURE_CANDIDATES = tuple((blk, w) for blk in (0, 32, 64, 128, 256) for w in (0, 8, 12, 16))


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


def measure_key(n: int, chi: int, layers: int, batch: int, precision: int) -> str:
    return f"measure/n{n}/chi{chi}/L{layers}/b{batch}/p{precision}"


def tune_measure(n: int, chi: int, layers: int, batch: int, precision: int,
                 candidates=MEASURE_CANDIDATES, repeats: int = 3, seed: int = 12345,
                 p: int | None = None):
    """Time the measurement call (environments + pair expectations of the image-local
    neighbour pairs) for each pair-kernel schedule on a seeded batch of this shape; applies the
    fastest and returns ((pair_block_images, pair_waves_per_cu), ms, {candidate: ms})."""
    import torch
    from . import inputs
    p = p if p is not None else int(round(n ** 0.5))
    assert p * p == n, "square images only"
    x = inputs.blob_images(batch, p, seed)
    th, ph = inputs.layer_angles(layers, n, seed + 1)
    b = anomps.new_batch(n, chi, layers, batch, precision)
    anomps.init_batch(b, torch.as_tensor(x, device="cuda").contiguous())
    if layers:
        anomps.apply_layers(b, torch.as_tensor(th, device="cuda").contiguous(),
                            torch.as_tensor(ph, device="cuda").contiguous())
    pairs = torch.as_tensor(inputs.neighbour_pairs(p), device="cuda").contiguous()
    real = torch.float64 if precision == anomps.PREC_FP64 else torch.float32
    out = torch.empty((batch, pairs.shape[0], 15), dtype=real, device="cuda")
    timings = {}
    for cand in candidates:
        anomps.set_measure_tuning(*cand)
        anomps.pauli_pair_expect(b, pairs, out)  # warm-up
        best = float("inf")
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            anomps.pauli_pair_expect(b, pairs, out)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        timings[cand] = best
    choice = min(timings, key=timings.get)
    anomps.set_measure_tuning(*choice)
    del b, out
    return choice, timings[choice], timings


def save_measure(key: str, choice, path: str) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(device_key(), {})[key] = [int(choice[0]), int(choice[1])]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_measure(key: str, path: str):
    """Apply a cached pair-kernel schedule for this device and shape key; returns it or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        got = json.load(f).get(device_key(), {}).get(key)
    if got is None:
        return None
    anomps.set_measure_tuning(int(got[0]), int(got[1]))
    return tuple(got)


def device_key() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def save(choice: dict, path: str) -> None:
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    dev = data.setdefault(device_key(), {})
    dev.update({str(b): int(c[0]) for b, c in choice.items()})
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def load_and_apply(path: str) -> dict:
    """Apply a cached choice for this device (if any); returns {bucket: blocks_per_cu}."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f).get(device_key(), {})
    mixed_part = {b: c for b, c in data.items() if b.isdigit()}
    for b, c in mixed_part.items():
        anomps.set_mixed_tuning(int(b), int(c))
    return {int(b): int(c) for b, c in mixed_part.items()}
