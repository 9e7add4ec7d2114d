"""Adaptive-observable readout (oracle; test infrastructure only).

§II-A: each observable H_q is a 4x4 Hermitian matrix on its pair, built from real
parameter sets A_q (real off-diagonal part), B_q (imaginary off-diagonal part) and D_q
(diagonal).  Reading of the layout (the paper gives none): basis |s_i s_j> with i the
lower site, H[j][j] = D[j] for j = 0..3, and for the six upper-triangle positions (j, k)
in row-major order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3): H[j][k] = A + iB, H[k][j] = A - iB.

Eq. (4): c_{q,alpha} = 2^{-2} Tr(H_q P_alpha) over the 16 two-qubit Paulis (alpha = 4a + b,
alpha = 0 the identity).  Eq. (5): <H_q> = sum_alpha c_{q,alpha} <P_alpha>, with <II> = 1.
Eq. (6): y = W q + b.
"""
from __future__ import annotations

import numpy as np

from . import gates

UPPER = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def hermitian(a_q: np.ndarray, b_q: np.ndarray, d_q: np.ndarray) -> np.ndarray:
    h = np.diag(d_q.astype(np.complex128))
    for idx, (j, k) in enumerate(UPPER):
        h[j, k] = a_q[idx] + 1j * b_q[idx]
        h[k, j] = a_q[idx] - 1j * b_q[idx]
    return h


def pauli16(alpha16: int) -> np.ndarray:
    a, b = divmod(alpha16, 4)
    return np.kron(gates.PAULI[a], gates.PAULI[b])


def coefficients(a: np.ndarray, b: np.ndarray, d: np.ndarray) -> np.ndarray:
    """[m][16] real Pauli coefficients c_{q,alpha} (Eq. (4))."""
    m = len(a)
    out = np.empty((m, 16))
    for q in range(m):
        h = hermitian(a[q], b[q], d[q])
        for al in range(16):
            out[q, al] = 0.25 * np.trace(h @ pauli16(al)).real
    return out


def features_from_paulis(coeff: np.ndarray, pauli: np.ndarray) -> np.ndarray:
    """q[b][q] = c_{q,0} + sum_{alpha'} c_{q,alpha'+1} <P_alpha'>  (Eq. (5)); pauli is
    [batch][m][15]."""
    return coeff[None, :, 0] + np.einsum("qa,bqa->bq", coeff[:, 1:], pauli)


def reconstruct(q: np.ndarray, w: np.ndarray, bias: np.ndarray) -> np.ndarray:
    """y[b] = W q[b] + bias (Eq. (6))."""
    return q @ w.T + bias[None, :]


def readout(pauli, a, b, d, w, bias) -> np.ndarray:
    return reconstruct(features_from_paulis(coefficients(a, b, d), pauli), w, bias)
