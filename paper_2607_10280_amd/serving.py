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


REJECTED = -2   # Request.status of a request whose footprint exceeds the whole arena


@dataclass
class Request:
    rid: int
    arrival: float                 # arrival time in trace units (wall seconds = arrival * time_scale)
    spec: mixed.RequestSpec
    readout: tuple | None = None   # (coeff_dev [m][16], W_dev [out][m], bias_dev [out]) or None
    # filled by the server
    offset: int = -1
    nbytes: int = 0
    desc: anomps.MpsRequest | None = None
    layers_done: int = 0
    out_off: int = 0
    ctrl_off: int = 0
    staged: tuple | None = None    # host inputs still to be copied into the arena
    lane: int = 0
    admit_time: float = -1.0       # wall seconds since the start of the run
    waited: bool = False           # arrived while the arena had no room for it
    done_time: float = 0.0         # wall seconds since the start of the run
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


def layer_cost(spec: mixed.RequestSpec) -> float:
    """Relative cost of one layer step of a request: n two-site factorisations of up to
    2S x 2S matrices, S the request's slot dimension (used only to pick its lane)."""
    S = anomps.slot_dim(spec.n, spec.chi, spec.layers)
    return float(spec.n) * float(S) ** 3


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    completed: int = 0
    rejected: int = 0
    queued: int = 0          # requests that had arrived but waited for arena space
    wall_s: float = 0.0
    iterations: int = 0
    peak_bytes: int = 0
    peak_resident: int = 0

    def summary(self):
        lat = np.array(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"completed": self.completed, "rejected": self.rejected, "queued": self.queued,
                "wall_s": round(self.wall_s, 3),
                "throughput_req_per_s": round(self.completed / max(self.wall_s, 1e-9), 1),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                "iterations": self.iterations, "peak_arena_bytes": self.peak_bytes,
                "peak_resident": self.peak_resident}


class _Lane:
    """One independent iteration cadence: its own stream, request tables and work queue.  A lane
    has at most one iteration in flight; the host polls its event and never waits on it."""

    def __init__(self, torch, device, max_resident: int):
        rs = ctypes.sizeof(anomps.MpsRequest)
        self.stream = torch.cuda.Stream(device=device)  # default priority
        # one table slot per call of an iteration (encode, layer step, measurement): a slot's
        # pinned staging buffer is rewritten only after the iteration's event has completed
        self.table_host = [torch.empty(max_resident * rs, dtype=torch.uint8, pin_memory=True)
                           for _ in range(3)]
        self.table_dev = [torch.empty(max_resident * rs, dtype=torch.uint8, device=device)
                          for _ in range(3)]
        self.queue = torch.zeros(anomps.MIXED_BUCKETS, dtype=torch.int32, device=device)
        self.resident: list[Request] = []
        self.event = None
        self.inflight = None   # (finished requests, device tensors kept alive, host copies)


class Server:
    """One-GPU continuous-batching loop over a fixed HBM arena.

    Requests are spread over `lanes` by the cost of one of their layer steps (`layer_cost`,
    split at `lane_bounds`); each lane advances its resident requests by one layer per
    iteration on its own stream, so light requests run many iterations while a heavy chain is
    still in its layer step, and the iterations of different lanes overlap on the device."""

    def __init__(self, arena_bytes: int, max_resident: int = 8192, device="cuda",
                 lane_bounds=(2.0 ** 13, 2.0 ** 17)):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena_bytes = arena_bytes
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        self.base = self.arena.data_ptr()
        self.alloc = ArenaAllocator(arena_bytes)
        self.max_resident = max_resident
        self.lane_bounds = tuple(lane_bounds)
        self.lanes = [_Lane(torch, self.device, max_resident)
                      for _ in range(len(self.lane_bounds) + 1)]

    @property
    def resident(self):
        return [r for ln in self.lanes for r in ln.resident]

    # ---- admission
    def footprint(self, r: Request) -> int:
        return request_layout(r.spec)[1]

    def try_admit(self, r: Request) -> bool:
        lane = bisect.bisect_right(self.lane_bounds, layer_cost(r.spec))
        if len(self.lanes[lane].resident) >= self.max_resident:
            return False
        offs, nbytes = request_layout(r.spec)
        off = self.alloc.alloc(nbytes)
        if off is None:
            return False
        r.offset, r.nbytes, r.lane = off, nbytes, lane
        sp = r.spec
        n, L, m = sp.n, sp.layers, sp.m
        f = np.concatenate([np.asarray(sp.pixels, np.float64).ravel(),
                            np.asarray(sp.theta, np.float64).ravel(),
                            np.asarray(sp.phi, np.float64).ravel()])
        pr = np.ascontiguousarray(sp.pairs, dtype=np.int32).reshape(-1, 2)
        i = np.concatenate([pr.ravel(), np.zeros(2, np.int32)])
        fo, io = off + offs["f64"], off + offs["i32"]
        r.staged = ((fo, f), (io, i))   # copied into the arena on the lane's stream at launch
        b = self.base + off
        r.desc = anomps.MpsRequest(
            n, sp.chi, L, sp.precision, m, 0,
            self.base + fo, b + offs["state"], b + offs["env"], self.base + fo + 8 * n,
            self.base + fo + 8 * n * (1 + L), 0, self.base + io, b + offs["out"],
            self.base + io + 8 * m)
        r.out_off, r.ctrl_off = off + offs["out"], io + 8 * m
        r.layers_done = -1  # encode pending
        self.lanes[lane].resident.append(r)
        return True

    def _table(self, lane: _Lane, reqs, slot: int):
        """Plan and upload a table of the given resident requests; returns (table, plan)."""
        descs = [r.desc for r in reqs]
        order, plan = anomps.plan_mixed(descs)
        rs = ctypes.sizeof(anomps.MpsRequest)
        arr = (anomps.MpsRequest * max(len(descs), 1))(*[descs[k] for k in order])
        nb = len(descs) * rs
        host, dev = lane.table_host[slot], lane.table_dev[slot]
        ctypes.memmove(host.data_ptr(), ctypes.addressof(arr), nb)
        dev[:nb].copy_(host[:nb], non_blocking=True)
        return dev, plan

    # ---- one iteration of a lane: launched, then completed by polling
    def _launch(self, lane: _Lane):
        torch = self.torch
        with torch.cuda.stream(lane.stream):
            new = [r for r in lane.resident if r.layers_done < 0]
            for r in new:
                for off, arr in r.staged:
                    src = torch.from_numpy(arr.view(np.uint8))
                    self.arena[off:off + arr.nbytes].copy_(src)
                r.staged = None
            if new:
                tab, plan = self._table(lane, new, 0)
                anomps.init_mixed(tab, plan, lane.stream)
                for r in new:
                    r.layers_done = 0
            stepping = [r for r in lane.resident if r.layers_done < r.spec.layers]
            if stepping:
                tab, plan = self._table(lane, stepping, 1)
                anomps.apply_layer_mixed(tab, plan, lane.queue, lane.stream)
                for r in stepping:
                    r.layers_done += 1
            finished = [r for r in lane.resident if r.layers_done == r.spec.layers]
            keep, host = [], None
            if finished:
                tab, plan = self._table(lane, finished, 2)
                anomps.pauli_pair_expect_mixed(tab, plan, lane.stream)
                pieces, ys, ctrls = [], [], []
                for r in finished:
                    dt = torch.float64 if r.spec.precision == anomps.PREC_FP64 else torch.float32
                    nb = r.spec.m * 15 * (8 if dt == torch.float64 else 4)
                    feat = self.arena[r.out_off:r.out_off + nb].view(dt).reshape(1, r.spec.m, 15)
                    if r.readout is not None:
                        coeff, W, bias = r.readout
                        y = torch.empty((1, W.shape[0]), dtype=dt, device=self.device)
                        anomps.ano_readout(feat, coeff, W, bias, y, lane.stream)
                        ys.append(y.reshape(-1).double())
                    pieces.append(feat.reshape(-1).double())
                    ctrls.append(self.arena[r.ctrl_off:r.ctrl_off + 8].view(torch.int32))
                dev = [torch.cat(pieces), torch.cat(ys) if ys else None, torch.cat(ctrls)]
                host = [None if t is None else torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
                        for t in dev]
                for h, t in zip(host, dev):
                    if t is not None:
                        h.copy_(t, non_blocking=True)
                keep = dev
            lane.event = torch.cuda.Event()
            lane.event.record(lane.stream)
        lane.inflight = (finished, keep, host)

    def _complete(self, lane: _Lane, stats: ServeStats, t0: float, time_scale: float):
        finished, _, host = lane.inflight
        lane.inflight = None
        stats.iterations += 1
        if not finished:
            return
        done = time.perf_counter() - t0
        feats = host[0].numpy()
        yh = host[1].numpy() if host[1] is not None else None
        ch = host[2].numpy().reshape(-1, 2)
        at = yat = 0
        for r, c in zip(finished, ch):
            k = r.spec.m * 15
            r.features = feats[at:at + k].reshape(r.spec.m, 15).copy()
            at += k
            if r.readout is not None:
                k = r.readout[1].shape[0]
                r.y = yh[yat:yat + k].copy()
                yat += k
            r.status = int(c[1])
            r.done_time = done
            stats.latencies_ms.append((done - r.arrival * time_scale) * 1e3)
            stats.completed += 1
            self.alloc.release(r.offset, r.nbytes)
        lane.resident = [r for r in lane.resident if r.layers_done != r.spec.layers]

    def run(self, requests, time_scale: float = 1.0):
        """Serve `requests` (sorted by arrival) in real time, arrival * time_scale wall seconds
        after the start; returns ServeStats.  A request whose footprint exceeds the whole arena
        can never be admitted: it is marked REJECTED (status) and skipped."""
        stats = ServeStats()
        pending = []
        for r in requests:
            if self.footprint(r) > self.arena_bytes:
                r.status = REJECTED
                stats.rejected += 1
            else:
                pending.append(r)
        t0 = time.perf_counter()
        k = 0
        while k < len(pending) or any(ln.resident or ln.inflight for ln in self.lanes):
            now = time.perf_counter() - t0
            while k < len(pending) and pending[k].arrival * time_scale <= now:
                if not self.try_admit(pending[k]):
                    stats.queued += int(not pending[k].waited)
                    pending[k].waited = True
                    break
                pending[k].admit_time = now
                k += 1
            stats.peak_bytes = max(stats.peak_bytes, self.alloc.used)
            stats.peak_resident = max(stats.peak_resident, sum(len(ln.resident) for ln in self.lanes))
            busy = False
            for ln in self.lanes:
                if ln.inflight is not None and ln.event.query():
                    self._complete(ln, stats, t0, time_scale)
                if ln.inflight is None and ln.resident:
                    self._launch(ln)
                busy |= ln.inflight is not None
            if not busy and k < len(pending):  # idle until the next arrival
                wait = pending[k].arrival * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif busy:
                time.sleep(2e-5)
        self.torch.cuda.synchronize()
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
        stats.latencies_ms.append((done - r.arrival * time_scale) * 1e3)
        stats.completed += 1
        stats.iterations += 1
    stats.wall_s = time.perf_counter() - t0
    return stats
