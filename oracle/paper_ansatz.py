"""The paper's own encoding circuit, simulated three ways in FP64 (oracle; test
infrastructure only).

§II-B: every pixel x_i in [0, 1] becomes the angle phi_i = 2 pi x_i - pi (Eq. (2)); the circuit
applies a Hadamard gate to every qubit, then R_Y(phi_i) to qubit i, then staggered
nearest-neighbour CNOTs, and this encoding-entangling layer is repeated L times.  The state
starts in |0...0>.  Readings taken where the text is brief:
* "staggered" = brickwork: CNOT(k, k+1) on every even bond k = 0, 2, 4, ... first, then on
  every odd bond k = 1, 3, 5, ...; control = the lower site.
* In the MPS the even and odd bonds are two left-to-right sweeps, each preceded by a
  right-canonical sweep (so every truncation sits at the orthogonality centre).  A bond
  without a gate in a sweep only moves the centre: its SVD keeps the old bond's rank, nothing
  is truncated.  A CNOT bond keeps at most min(chi, 2 D_old, rows, cols) singular values
  (a CNOT at most doubles the Schmidt rank across its bond).
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from . import gates, statevector
from . import mps as mps_mod

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def angle(x):
    """Eq. (2): phi = 2 pi x - pi."""
    return 2.0 * np.pi * np.asarray(x, dtype=np.float64) - np.pi


def bonds(n: int, parity: int):
    return range(parity, n - 1, 2)


# ------------------------------------------------------------------ statevector (n <= 20)
def sv_state(x, layers: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    psi = np.zeros([2] * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    phi = angle(x)
    for _ in range(layers):
        for k in range(n):
            psi = statevector._apply_1q(psi, H, k)
            psi = statevector._apply_1q(psi, gates.ry(phi[k]), k)
        for parity in (0, 1):
            for k in bonds(n, parity):
                psi = statevector._apply_cnot(psi, k, k + 1)
    return psi


def sv_features(x, layers: int, pairs) -> np.ndarray:
    return statevector.pauli_pair_features(sv_state(x, layers), pairs)


# ------------------------------------------------------------------ brute force (n <= 10)
def bf_state(x, layers: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    kron = lambda ops: reduce(np.kron, ops)
    u_h = kron([H] * n)
    u_ry = kron([gates.ry(p) for p in angle(x)])
    u_cx = np.eye(2 ** n, dtype=np.complex128)
    for parity in (0, 1):
        for k in bonds(n, parity):
            u_cx = kron([np.eye(2 ** k), gates.CNOT, np.eye(2 ** (n - k - 2))]) @ u_cx
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    for _ in range(layers):
        psi = u_cx @ (u_ry @ (u_h @ psi))
    return psi


def bf_features(x, layers: int, pairs) -> np.ndarray:
    from . import bruteforce
    psi = bf_state(x, layers)
    n = len(x)
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        for alpha in range(15):
            out[q, alpha] = np.vdot(psi, bruteforce.embedded_pauli(n, int(i), int(j), alpha) @ psi).real
    return out


# ------------------------------------------------------------------ MPS
def _canonicalise(m: mps_mod.MPS, site_gates) -> None:
    """Right-to-left LQ sweep; site_gates[k] (or None) applied to site k on the way."""
    a = m.tensors
    n = len(a)
    for k in range(n - 1, 0, -1):
        t = a[k] if site_gates is None else np.einsum("st,ltr->lsr", site_gates[k], a[k])
        dl, _, dr = t.shape
        q, r = np.linalg.qr(t.reshape(dl, 2 * dr).conj().T, mode="reduced")
        a[k] = q.conj().T.reshape(-1, 2, dr)
        a[k - 1] = np.einsum("lsc,cd->lsd", a[k - 1], r.conj().T)
    if site_gates is not None:
        a[0] = np.einsum("st,ltr->lsr", site_gates[0], a[0])


def _sweep(m: mps_mod.MPS, chi, parity: int, errs: np.ndarray, gaps: np.ndarray) -> None:
    """Left-to-right two-site sweep: CNOT on bonds k with k % 2 == parity, a pure centre move
    elsewhere."""
    a = m.tensors
    n = len(a)
    for k in range(n - 1):
        gate = (k % 2) == parity
        d_old = a[k].shape[2]
        theta2 = np.einsum("lsc,ctr->lstr", a[k], a[k + 1])
        if gate:
            theta2 = mps_mod.cnot_two_site(theta2)
        dl, dr = theta2.shape[0], theta2.shape[3]
        u, s, vh = np.linalg.svd(theta2.reshape(2 * dl, 2 * dr), full_matrices=False)
        bound = min(len(s), (2 if gate else 1) * d_old)
        if chi is None or not gate:
            d = min(bound, int(np.count_nonzero(s > mps_mod.EXACT_CUTOFF * s[0])))
        else:
            d = min(chi, bound)
        total = float(np.sum(s * s))
        if gate:
            errs[k] = float(np.sum(s[d:] ** 2)) / total
            gaps[k] = s[d - 1] - s[d] if d < len(s) else np.inf
        kept = s[:d] / np.linalg.norm(s[:d])
        a[k] = u[:, :d].reshape(dl, 2, d)
        a[k + 1] = (kept[:, None] * vh[:d]).reshape(d, 2, dr)


def mps_simulate(x, layers: int, chi=None) -> mps_mod.MPS:
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    m = mps_mod.MPS([np.array([1.0, 0.0], dtype=np.complex128).reshape(1, 2, 1) for _ in range(n)])
    site_gates = [gates.ry(p) @ H for p in angle(x)]
    for _ in range(layers):
        errs, gaps = np.zeros(n - 1), np.full(n - 1, np.inf)
        _canonicalise(m, site_gates)
        _sweep(m, chi, 0, errs, gaps)
        _canonicalise(m, None)
        _sweep(m, chi, 1, errs, gaps)
        m.trunc_err.append(errs)
        m.gaps.append(gaps)
    return m


def mps_features(x, layers: int, pairs, chi=None) -> np.ndarray:
    return mps_mod.pauli_pair_features(mps_simulate(x, layers, chi), pairs)


# ------------------------------------------------------------------ front door
def features(pixels, layers: int, pairs, chi=None) -> np.ndarray:
    """[B][m][15]: exact (statevector for n <= 20, untruncated MPS above) when chi is None,
    else the truncated MPS."""
    pixels = np.atleast_2d(pixels)
    n = pixels.shape[1]
    out = []
    for x in pixels:
        if chi is None and n <= statevector.MAX_QUBITS:
            out.append(sv_features(x, layers, pairs))
        else:
            out.append(mps_features(x, layers, pairs, chi))
    return np.stack(out)
