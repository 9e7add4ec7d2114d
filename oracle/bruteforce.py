"""Brute-force circuit unitary from Kronecker products (oracle; test infrastructure only).

A second, independent statevector path for tiny n (<= 10): the whole circuit is built as
a dense 2^n x 2^n matrix, and expectations use the embedded 2^n x 2^n Pauli operator.
It exists only to pin ``statevector`` (a wrong axis, gate order or CNOT direction in one
of the two would make them disagree).
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from . import gates


def _kron_all(ops):
    return reduce(np.kron, ops)


def layer_unitary(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    n = len(theta)
    u1 = _kron_all([gates.layer_gate(theta[k], phi[k]) for k in range(n)])
    ladder = np.eye(2 ** n, dtype=np.complex128)
    for k in range(n - 1):
        ck = _kron_all([np.eye(2 ** k), gates.CNOT, np.eye(2 ** (n - k - 2))])
        ladder = ck @ ladder  # CNOT(k, k+1) acts after the ones with smaller k
    return ladder @ u1


def state(x: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    n = len(x)
    if n > 10:
        raise ValueError("brute force limited to 10 qubits")
    psi = _kron_all([gates.encode_state(xk) for xk in x])
    for layer in range(len(theta)):
        psi = layer_unitary(theta[layer], phi[layer]) @ psi
    return psi


def embedded_pauli(n: int, i: int, j: int, alpha: int) -> np.ndarray:
    a, b = divmod(alpha + 1, 4)
    ops = [gates.I2] * n
    ops[i] = gates.PAULI[a]
    ops[j] = gates.PAULI[b]
    return _kron_all(ops)


def features(x, theta, phi, pairs) -> np.ndarray:
    psi = state(np.asarray(x, dtype=np.float64), theta, phi)
    n = len(x)
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        for alpha in range(15):
            out[q, alpha] = np.vdot(psi, embedded_pauli(n, int(i), int(j), alpha) @ psi).real
    return out
