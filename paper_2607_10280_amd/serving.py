"""Continuous-batching request loop for feature extraction (mixed p, L, chi per request).

Requests arrive over time.  The loop admits them while their device footprint fits in a fixed
HBM arena; keeps each admitted request's MPS resident; advances every resident request by one
layer per iteration through the library's mixed-table calls; measures requests that have all
their layers; returns features (and, where readout weights are given, the reconstruction) to
the host; and frees their memory.  Latency is measured from arrival to features on the host.

The arena allocator and the table bookkeeping are host-side; all arithmetic runs in the
library's kernels.
"""
from __future__ import annotations

import bisect
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import anomps, mixed

ALIGN = 256


def _al(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


class ArenaAllocator:
    """First-fit allocator over [0, size) with coalescing free list (host bookkeeping only)."""

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]  # sorted (offset, length)
        self.used = 0

    def alloc(self, nbytes: int):
        nbytes = _al(nbytes)
        for i, (off, ln) in enumerate(self.free):
            if ln >= nbytes:
                if ln == nbytes:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + nbytes, ln - nbytes)
                self.used += nbytes
                return off
        return None

    def release(self, off: int, nbytes: int):
        nbytes = _al(nbytes)
        self.used -= nbytes
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, nbytes))
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


@dataclass
class Request:
    rid: int
    arrival: float                 # seconds since the start of the run
    spec: mixed.RequestSpec
    readout: tuple | None = None   # (coeff_dev [m][16], W_dev [out][m], bias_dev [out]) or None
    # filled by the server
    offset: int = -1
    nbytes: int = 0
    desc: anomps.MpsRequest | None = None
    layers_done: int = 0
    out_off: int = 0
    ctrl_off: int = 0
    done_time: float = 0.0
    features: np.ndarray | None = None
    y: np.ndarray | None = None
    status: int = 0


def request_layout(spec: mixed.RequestSpec):
    """Byte offsets inside one request's arena block: state, env, out, f64 inputs, i32 inputs."""
    n, L, m = spec.n, spec.layers, spec.m
    real = 8 if spec.precision == anomps.PREC_FP64 else 4
    sb = _al(anomps.state_bytes(n, spec.chi, L, 1, spec.precision))
    eb = _al(anomps.env_bytes(n, spec.chi, L, 1, spec.precision))
    ob = _al(max(m * 15 * real, 1))
    fb = _al(8 * n * (1 + 2 * L))
    ib = _al(4 * (2 * m + 2))
    offs = {"state": 0, "env": sb, "out": sb + eb, "f64": sb + eb + ob, "i32": sb + eb + ob + fb}
    return offs, sb + eb + ob + fb + ib


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    completed: int = 0
    wall_s: float = 0.0
    iterations: int = 0
    peak_bytes: int = 0

    def summary(self):
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"completed": self.completed, "wall_s": round(self.wall_s, 3),
                "throughput_req_per_s": round(self.completed / max(self.wall_s, 1e-9), 1),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                "iterations": self.iterations, "peak_arena_bytes": self.peak_bytes}


class Server:
    """One-GPU continuous-batching loop over a fixed HBM arena."""

    def __init__(self, arena_bytes: int, max_resident: int = 65536, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.base = self.arena.data_ptr()
        self.alloc = ArenaAllocator(arena_bytes)
        rs = ctypes.sizeof(anomps.MpsRequest)
        # one table slot per call of an iteration (encode, layer step, measurement): a slot's
        # pinned staging buffer is rewritten only after the iteration's closing synchronize
        self.table_host = [torch.empty(max_resident * rs, dtype=torch.uint8, pin_memory=True)
                           for _ in range(3)]
        self.table_dev = [torch.empty(max_resident * rs, dtype=torch.uint8, device=self.device)
                          for _ in range(3)]
        self.queue = torch.zeros(anomps.MIXED_BUCKETS, dtype=torch.int32, device=self.device)
        self.max_resident = max_resident
        self.resident: list[Request] = []

    # ---- admission
    def try_admit(self, r: Request) -> bool:
        if len(self.resident) >= self.max_resident:
            return False
        offs, nbytes = request_layout(r.spec)
        off = self.alloc.alloc(nbytes)
        if off is None:
            return False
        r.offset, r.nbytes = off, nbytes
        sp = r.spec
        n, L, m = sp.n, sp.layers, sp.m
        f = np.concatenate([np.asarray(sp.pixels, np.float64).ravel(),
                            np.asarray(sp.theta, np.float64).ravel(),
                            np.asarray(sp.phi, np.float64).ravel()])
        pr = np.ascontiguousarray(sp.pairs, dtype=np.int32).reshape(-1, 2)
        i = np.concatenate([pr.ravel(), np.zeros(2, np.int32)])
        fo, io = off + offs["f64"], off + offs["i32"]
        self.arena[fo:fo + f.nbytes].copy_(self.torch.from_numpy(f.view(np.uint8)))
        self.arena[io:io + i.nbytes].copy_(self.torch.from_numpy(i.view(np.uint8)))
        b = self.base + off
        r.desc = anomps.MpsRequest(
            n, sp.chi, L, sp.precision, m, 0,
            self.base + fo, b + offs["state"], b + offs["env"], self.base + fo + 8 * n,
            self.base + fo + 8 * n * (1 + L), 0, self.base + io, b + offs["out"],
            self.base + io + 8 * m)
        r.out_off, r.ctrl_off = off + offs["out"], io + 8 * m
        r.layers_done = -1  # encode pending
        self.resident.append(r)
        return True

    def _table(self, reqs, slot: int):
        """Plan and upload a table of the given resident requests; returns (table, plan)."""
        descs = [r.desc for r in reqs]
        order, plan = anomps.plan_mixed(descs)
        rs = ctypes.sizeof(anomps.MpsRequest)
        arr = (anomps.MpsRequest * max(len(descs), 1))(*[descs[k] for k in order])
        nb = len(descs) * rs
        host, dev = self.table_host[slot], self.table_dev[slot]
        ctypes.memmove(host.data_ptr(), ctypes.addressof(arr), nb)
        dev[:nb].copy_(host[:nb], non_blocking=True)
        return dev, plan

    # ---- one iteration of the loop
    def iterate(self, now: float, stats: ServeStats, t0: float):
        torch = self.torch
        new = [r for r in self.resident if r.layers_done < 0]
        if new:
            tab, plan = self._table(new, 0)
            anomps.init_mixed(tab, plan)
            for r in new:
                r.layers_done = 0
        stepping = [r for r in self.resident if r.layers_done < r.spec.layers]
        if stepping:
            tab, plan = self._table(stepping, 1)
            anomps.apply_layer_mixed(tab, plan, self.queue)
            for r in stepping:
                r.layers_done += 1
        finished = [r for r in self.resident if r.layers_done == r.spec.layers]
        if not finished:
            torch.cuda.synchronize()
        else:
            tab, plan = self._table(finished, 2)
            anomps.pauli_pair_expect_mixed(tab, plan)
            pieces, ys, ctrls = [], [], []
            for r in finished:
                dt = torch.float64 if r.spec.precision == anomps.PREC_FP64 else torch.float32
                nb = r.spec.m * 15 * (8 if dt == torch.float64 else 4)
                feat = self.arena[r.out_off:r.out_off + nb].view(dt).reshape(1, r.spec.m, 15)
                if r.readout is not None:
                    coeff, W, bias = r.readout
                    y = torch.empty((1, W.shape[0]), dtype=dt, device=self.device)
                    anomps.ano_readout(feat, coeff, W, bias, y)
                    ys.append(y.reshape(-1).double())
                pieces.append(feat.reshape(-1).double())
                ctrls.append(self.arena[r.ctrl_off:r.ctrl_off + 8].view(torch.int32))
            feats = torch.cat(pieces).cpu().numpy()  # one copy back (synchronises the stream)
            yh = torch.cat(ys).cpu().numpy() if ys else None
            ch = torch.cat(ctrls).cpu().numpy().reshape(-1, 2)
            done = time.perf_counter() - t0
            at = yat = 0
            for r, c in zip(finished, ch):
                k = r.spec.m * 15
                r.features = feats[at:at + k].reshape(r.spec.m, 15)
                at += k
                if r.readout is not None:
                    k = r.readout[1].shape[0]
                    r.y = yh[yat:yat + k]
                    yat += k
                r.status = int(c[1])
                r.done_time = done
                stats.latencies_ms.append((done - r.arrival) * 1e3)
                stats.completed += 1
                self.alloc.release(r.offset, r.nbytes)
            self.resident = [r for r in self.resident if r.layers_done != r.spec.layers]
        stats.iterations += 1
        stats.peak_bytes = max(stats.peak_bytes, self.alloc.used)

    def run(self, requests, time_scale: float = 1.0):
        """Serve `requests` (sorted by arrival, seconds) in real time; returns ServeStats."""
        stats = ServeStats()
        pending = list(requests)
        t0 = time.perf_counter()
        k = 0
        while k < len(pending) or self.resident:
            now = (time.perf_counter() - t0) / time_scale
            while k < len(pending) and pending[k].arrival <= now:
                if not self.try_admit(pending[k]):
                    break
                k += 1
            if not self.resident:
                if k < len(pending):  # idle until the next arrival
                    wait = pending[k].arrival * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            self.iterate(now, stats, t0)
        stats.wall_s = time.perf_counter() - t0
        return stats


def serve_plain(requests, time_scale: float = 1.0):
    """The same arrivals through a plain FIFO: one request at a time with the batch calls."""
    import torch
    stats = ServeStats()
    t0 = time.perf_counter()
    for r in requests:
        now = time.perf_counter() - t0
        if r.arrival * time_scale > now:
            time.sleep(r.arrival * time_scale - now)
        sp = r.spec
        out, st = anomps.extract_features(sp.pixels[None], sp.theta, sp.phi, sp.pairs, sp.chi,
                                          sp.precision)
        if r.readout is not None:
            coeff, W, bias = r.readout
            y = torch.empty((1, W.shape[0]), dtype=out.dtype, device=out.device)
            anomps.ano_readout(out, coeff, W, bias, y)
            r.y = y.cpu().numpy()[0]
        r.features = out.cpu().numpy()[0]
        done = time.perf_counter() - t0
        stats.latencies_ms.append((done - r.arrival) * 1e3)
        stats.completed += 1
        stats.iterations += 1
    stats.wall_s = time.perf_counter() - t0
    return stats
