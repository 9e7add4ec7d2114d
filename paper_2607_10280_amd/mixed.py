"""Mixed request tables: many images with different sizes, bond limits, depths and precisions
run together through the library's persistent per-bucket launches (include/anomps.h,
``mps_plan_mixed`` ... ``mps_pauli_pair_expect_mixed``).

`MixedRequests` packs every request's buffers into a few device arenas (one allocation per
kind, offsets aligned to 256 bytes), builds the request table in the library's plan order and
runs the whole path.  All arithmetic happens in the library's kernels; this module only lays
out memory and marshals arguments.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import anomps

ALIGN = 256


def _align(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


@dataclass
class RequestSpec:
    """One image: pixels [n], angles theta/phi [L][n], pairs [m][2], chi, precision."""
    pixels: np.ndarray
    theta: np.ndarray
    phi: np.ndarray
    pairs: np.ndarray
    chi: int
    precision: int = anomps.PREC_FP32

    @property
    def n(self) -> int:
        return int(np.asarray(self.pixels).size)

    @property
    def layers(self) -> int:
        return int(np.asarray(self.theta).reshape(-1, self.n).shape[0]) if np.asarray(self.theta).size else 0

    @property
    def m(self) -> int:
        return int(np.asarray(self.pairs).reshape(-1, 2).shape[0])


def footprint_bytes(spec: RequestSpec) -> int:
    """Device bytes of one request: state + environments + outputs + pixels, angles, pairs and
    control words (each rounded up to the arena alignment)."""
    n, L, m = spec.n, spec.layers, spec.m
    real = 8 if spec.precision == anomps.PREC_FP64 else 4
    return (_align(anomps.state_bytes(n, spec.chi, L, 1, spec.precision)) +
            _align(anomps.env_bytes(n, spec.chi, L, 1, spec.precision)) +
            _align(m * 15 * real) + _align(8 * n * (1 + 2 * L)) + _align(8 * m + 8))


class MixedRequests:
    """Device-resident buffers and the planned request table of a list of RequestSpec."""

    def __init__(self, specs, device="cuda", trunc_err: bool = False):
        import torch
        self.specs = list(specs)
        self.device = torch.device(device)
        N = len(self.specs)
        byte_off, f64_off, i32_off = [], [], []
        nb = nf = ni = 0
        for sp in self.specs:
            n, L, m = sp.n, sp.layers, sp.m
            real = 8 if sp.precision == anomps.PREC_FP64 else 4
            sb = anomps.state_bytes(n, sp.chi, L, 1, sp.precision)
            eb = anomps.env_bytes(n, sp.chi, L, 1, sp.precision)
            if sb == 0 or eb == 0:
                raise anomps.MpsError(-1, anomps.lib().mps_last_error().decode())
            ob = m * 15 * real
            byte_off.append((nb, nb + _align(sb), nb + _align(sb) + _align(eb)))
            nb += _align(sb) + _align(eb) + _align(max(ob, 1))
            te = L * (n - 1) if trunc_err else 0
            f64_off.append((nf, nf + n, nf + n + L * n, nf + n + 2 * L * n))
            nf += n + 2 * L * n + te
            i32_off.append((ni, ni + 2 * m))
            ni += 2 * m + 2
        self.bytes = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)
        host_f = np.zeros(max(nf, 1), dtype=np.float64)
        host_i = np.zeros(max(ni, 1), dtype=np.int32)
        for sp, (p0, t0, f0, e0), (q0, c0) in zip(self.specs, f64_off, i32_off):
            n, L = sp.n, sp.layers
            host_f[p0:p0 + n] = np.asarray(sp.pixels, dtype=np.float64).ravel()
            host_f[t0:t0 + L * n] = np.asarray(sp.theta, dtype=np.float64).ravel()
            host_f[f0:f0 + L * n] = np.asarray(sp.phi, dtype=np.float64).ravel()
            pr = np.asarray(sp.pairs, dtype=np.int32).reshape(-1, 2)
            anomps.validate_pairs(pr, n)
            host_i[q0:q0 + 2 * sp.m] = pr.ravel()
        self.f64 = torch.as_tensor(host_f, device=self.device)
        self.i32 = torch.as_tensor(host_i, device=self.device)
        bp, fp, ip = self.bytes.data_ptr(), self.f64.data_ptr(), self.i32.data_ptr()
        self._layout = []
        reqs = []
        for sp, (s0, e0, o0), (p0, t0, f0, x0), (q0, c0) in zip(self.specs, byte_off, f64_off, i32_off):
            n, L, m = sp.n, sp.layers, sp.m
            reqs.append(anomps.MpsRequest(
                n, sp.chi, L, sp.precision, m, 0,
                fp + 8 * p0, bp + s0, bp + e0, fp + 8 * t0, fp + 8 * f0,
                (fp + 8 * x0) if trunc_err else 0, ip + 4 * q0, bp + o0, ip + 4 * c0))
            self._layout.append((o0, c0, x0))
        self.reqs = reqs
        self.order, self.plan = anomps.plan_mixed(reqs)
        self.table = anomps.request_table(reqs, self.order, self.device)
        self.queue = torch.zeros(anomps.MIXED_BUCKETS, dtype=torch.int32, device=self.device)
        self.max_layers = max((sp.layers for sp in self.specs), default=0)
        self.trunc_err = trunc_err
        self.n_req = N

    # ---- the path
    def init(self, stream=None):
        anomps.init_mixed(self.table, self.plan, stream)

    def step(self, stream=None):
        """One more layer for every request that still needs one."""
        anomps.apply_layer_mixed(self.table, self.plan, self.queue, stream)

    def measure(self, stream=None):
        anomps.pauli_pair_expect_mixed(self.table, self.plan, stream)

    def run(self, stream=None):
        self.init(stream)
        for _ in range(self.max_layers):
            self.step(stream)
        self.measure(stream)

    # ---- results (host copies, in spec order)
    def outputs(self):
        import torch
        out = []
        for sp, (o0, c0, x0) in zip(self.specs, self._layout):
            dt = torch.float64 if sp.precision == anomps.PREC_FP64 else torch.float32
            nbytes = sp.m * 15 * (8 if dt == torch.float64 else 4)
            out.append(self.bytes[o0:o0 + nbytes].view(dt).reshape(sp.m, 15))
        return [o.cpu().numpy() for o in out]

    def ctrl(self) -> np.ndarray:
        h = self.i32.cpu().numpy()
        return np.array([h[c0:c0 + 2] for (_, c0, _) in self._layout]).reshape(-1, 2)

    def trunc_errors(self):
        assert self.trunc_err
        h = self.f64.cpu().numpy()
        return [h[x0:x0 + sp.layers * (sp.n - 1)].reshape(sp.layers, sp.n - 1)
                for sp, (_, _, x0) in zip(self.specs, self._layout)]
