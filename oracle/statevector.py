"""Plain statevector simulation (oracle; test infrastructure only).

This is the 2^n-amplitude backend that the paper compares against (§I, §III): exact, and
limited by memory.  Here it is used for n <= 20 as the exact reference of the circuit.

The state is a complex128 array of shape [2]*n with qubit 0 on axis 0 (the most
significant bit of a basis index), qubit k = pixel k of the row-major flattened image
(§II-B).
"""
from __future__ import annotations

import numpy as np

from . import gates

MAX_QUBITS = 20


def _apply_1q(psi: np.ndarray, u: np.ndarray, k: int) -> np.ndarray:
    out = np.tensordot(u, psi, axes=([1], [k]))
    return np.moveaxis(out, 0, k)


def _apply_cnot(psi: np.ndarray, c: int, t: int) -> np.ndarray:
    """CNOT(c, t): on the slice where qubit c is 1, swap the two values of qubit t."""
    n = psi.ndim
    out = psi.copy()
    idx1 = [slice(None)] * n
    idx1[c] = 1
    sub = psi[tuple(idx1)]  # qubit c removed: target axis shifts down if t > c
    tax = t - 1 if t > c else t
    out[tuple(idx1)] = np.flip(sub, axis=tax)
    return out


def product_state(x: np.ndarray) -> np.ndarray:
    """Angle-encoded product state: qubit k in R_Y(pi x_k)|0>."""
    n = len(x)
    psi = np.ones((), dtype=np.complex128)
    for k in range(n):
        psi = np.multiply.outer(psi, gates.encode_state(x[k]))
    return psi.reshape([2] * n)


def apply_layer(psi: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """One entangling layer: R_Y(theta_k) R_Z(phi_k) on every qubit, then CNOT(k, k+1)
    for k = 0, 1, ..., n-2 in that order."""
    n = psi.ndim
    for k in range(n):
        psi = _apply_1q(psi, gates.layer_gate(theta[k], phi[k]), k)
    for k in range(n - 1):
        psi = _apply_cnot(psi, k, k + 1)
    return psi


def simulate(x: np.ndarray, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """|psi(x)> after len(theta) layers; theta, phi are [L][n]."""
    n = len(x)
    if n > MAX_QUBITS:
        raise ValueError(f"statevector oracle limited to {MAX_QUBITS} qubits, got {n}")
    psi = product_state(np.asarray(x, dtype=np.float64))
    for layer in range(len(theta)):
        psi = apply_layer(psi, theta[layer], phi[layer])
    return psi


def pair_rdm(psi: np.ndarray, i: int, j: int) -> np.ndarray:
    """Two-site reduced density matrix rho_ij (4x4), rows/cols indexed s_i*2 + s_j:
    rho[(s,t),(s',t')] = sum_rest psi(s,t,rest) conj(psi(s',t',rest))."""
    m = np.moveaxis(psi, [i, j], [0, 1]).reshape(4, -1)
    return m @ m.conj().T


def pauli_pair_features(psi: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """[m][15] real expectations <P_a (x) P_b> = Re Tr(rho_ij (P_a (x) P_b)) (Eq. (4)-(5))."""
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        rho = pair_rdm(psi, int(i), int(j))
        for alpha in range(15):
            out[q, alpha] = np.trace(rho @ gates.pair_pauli(alpha)).real
    return out


def features(x, theta, phi, pairs) -> np.ndarray:
    """Exact Pauli-pair features of one image."""
    return pauli_pair_features(simulate(x, theta, phi), pairs)
