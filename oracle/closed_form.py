"""Closed-form Pauli-pair features (oracle; test infrastructure only).

* L = 0: the encoded state is a product state, so every pair expectation factorises into
  single-qubit Bloch components, r_k = (1, sin pi x_k, 0, cos pi x_k) for (I, X, Y, Z).
* L = 1: the CNOT ladder is a Clifford circuit C, so <psi|P|psi> = <phi|C^dag P C|phi> with
  |phi> the product state after the one-qubit gates.  C^dag P C is again a Pauli string up
  to a sign; it is found by conjugating P by CNOT(n-2, n-1) first and CNOT(0, 1) last (the
  reverse of the order in which the ladder acts).  The two-qubit conjugation table is
  derived numerically from the 4x4 CNOT matrix, and the expectation in the product state
  is the sign times the product of single-qubit Bloch components.  Valid for any n.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import gates


def bloch(v: np.ndarray) -> np.ndarray:
    """(1, <X>, <Y>, <Z>) of a normalised single-qubit state v."""
    return np.array([np.vdot(v, p @ v).real for p in gates.PAULI])


def l0_features(x: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    r = np.stack([np.ones_like(x), np.sin(np.pi * x), np.zeros_like(x), np.cos(np.pi * x)], 1)
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        for alpha in range(15):
            a, b = divmod(alpha + 1, 4)
            out[q, alpha] = r[i, a] * r[j, b]
    return out


def _cnot_table() -> dict:
    """(P_c, P_t) -> (sign, P_c', P_t') with CNOT (P_c (x) P_t) CNOT = sign P_c' (x) P_t'."""
    table = {}
    for a, b in itertools.product(range(4), repeat=2):
        conj = gates.CNOT @ np.kron(gates.PAULI[a], gates.PAULI[b]) @ gates.CNOT
        for c, d in itertools.product(range(4), repeat=2):
            ref = np.kron(gates.PAULI[c], gates.PAULI[d])
            for sign in (1, -1):
                if np.allclose(conj, sign * ref):
                    table[(a, b)] = (sign, c, d)
        assert (a, b) in table
    return table


_CNOT_TABLE = _cnot_table()


def heisenberg_ladder(string: list) -> tuple[int, list]:
    """C^dag P C for the ladder C = CNOT(n-2,n-1) ... CNOT(0,1); returns (sign, string)."""
    s = list(string)
    sign = 1
    for k in range(len(s) - 2, -1, -1):
        sg, s[k], s[k + 1] = _CNOT_TABLE[(s[k], s[k + 1])]
        sign *= sg
    return sign, s


def l1_features(x, theta, phi, pairs) -> np.ndarray:
    """Exact features after one layer, any number of qubits."""
    n = len(x)
    rvec = np.stack([bloch(gates.layer_gate(theta[0][k], phi[0][k]) @ gates.encode_state(x[k]))
                     for k in range(n)])
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        for alpha in range(15):
            a, b = divmod(alpha + 1, 4)
            string = [0] * n
            string[i], string[j] = a, b
            sign, img = heisenberg_ladder(string)
            val = float(sign)
            for k, pk in enumerate(img):
                if pk:
                    val *= rvec[k, pk]
            out[q, alpha] = val
    return out
