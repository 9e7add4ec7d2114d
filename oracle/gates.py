"""Gate matrices and the two-qubit Pauli basis (oracle; test infrastructure only).

Conventions (readings of §II-B / §II-C, where the paper gives no matrices):
* R_Y(t) = [[cos t/2, -sin t/2], [sin t/2, cos t/2]],  R_Z(t) = diag(e^{-it/2}, e^{it/2}).
* The single-qubit layer gate on qubit k is U = R_Y(theta_k) @ R_Z(phi_k) (R_Z acts first).
* CNOT(c, t) maps |c, t> -> |c, t XOR c>.
* Paulis are indexed I, X, Y, Z = 0, 1, 2, 3; a pair feature alpha' = 4a + b - 1 for
  (a, b) != (0, 0), with P_a acting on the lower site i and P_b on site j (Eq. (4)).
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = (I2, X, Y, Z)

# |c t> basis, c the more significant bit.
CNOT = np.array([[1, 0, 0, 0],
                 [0, 1, 0, 0],
                 [0, 0, 0, 1],
                 [0, 0, 1, 0]], dtype=np.complex128)


def ry(t: float) -> np.ndarray:
    c, s = np.cos(t / 2.0), np.sin(t / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(t: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def layer_gate(theta: float, phi: float) -> np.ndarray:
    """One-qubit gate of an entangling layer: R_Y(theta) R_Z(phi)."""
    return ry(theta) @ rz(phi)


def encode_state(x: float) -> np.ndarray:
    """Angle encoding of one pixel: R_Y(pi x)|0>."""
    return ry(np.pi * x) @ np.array([1.0, 0.0], dtype=np.complex128)


def pair_pauli(alpha: int) -> np.ndarray:
    """4x4 operator P_a (x) P_b for feature index alpha = 4a + b - 1 (alpha in 0..14)."""
    a, b = divmod(alpha + 1, 4)
    return np.kron(PAULI[a], PAULI[b])
