"""Matrix product state simulation in FP64 (oracle; test infrastructure only).

Follows §II-B: the state is the chain of Eq. (3), |psi> = sum_s A[0]^{s_0} ... A[n-1]^{s_{n-1}}
|s_0 ... s_{n-1}>, site tensors A[k] of shape (D_{k-1}, 2, D_k) with D_{-1} = D_{n-1} = 1.
One-qubit gates update one local tensor; a nearest-neighbour two-qubit gate contracts the
two neighbouring tensors, applies the gate and splits the result again by an SVD keeping at
most chi singular values (chi is the maximum virtual dimension).

Where the paper is silent the oracle takes these readings:
* Canonical form: before each layer's CNOT ladder the chain is brought to right-canonical
  form by a right-to-left sweep of LQ factorisations (the layer's one-qubit gates are
  applied during that sweep); the ladder then sweeps left to right, so every truncation
  happens at the orthogonality centre, where the singular values are the Schmidt values.
* Truncation: keep D = min(chi, rank bound) singular triplets, largest first; the kept
  singular values are rescaled to unit 2-norm; the discarded weight
  eps = sum_discarded sigma^2 / sum_all sigma^2 is recorded per bond.
* Untruncated mode (chi=None): drop only sigma <= 1e-13 sigma_max (numerical zeros).
* Expectations: explicit left/right environments and transfer-matrix propagation between
  the two sites of a pair; no canonical-form shortcut is used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import gates

EXACT_CUTOFF = 1e-13


@dataclass
class MPS:
    tensors: list
    trunc_err: list = field(default_factory=list)   # per layer: [n-1] discarded weights
    gaps: list = field(default_factory=list)        # per layer: [n-1] sigma_D - sigma_{D+1}
    spectra: list = field(default_factory=list)     # per layer: list of the n-1 full spectra

    @property
    def n(self) -> int:
        return len(self.tensors)

    def bond_dims(self) -> list:
        return [t.shape[2] for t in self.tensors[:-1]]


def product_mps(x: np.ndarray) -> MPS:
    """Angle-encoded product state as an MPS with all bond dimensions 1."""
    return MPS([gates.encode_state(xk).reshape(1, 2, 1) for xk in x])


def _apply_1q(a: np.ndarray, u: np.ndarray) -> np.ndarray:
    # A'[l, s, r] = sum_s' U[s, s'] A[l, s', r]
    return np.einsum("st,ltr->lsr", u, a)


def canonicalise_right(mps: MPS, theta: np.ndarray, phi: np.ndarray) -> None:
    """Apply the layer's one-qubit gates and bring sites n-1 .. 1 to right-canonical form."""
    a = mps.tensors
    n = len(a)
    for k in range(n - 1, 0, -1):
        t = _apply_1q(a[k], gates.layer_gate(theta[k], phi[k]))
        dl, _, dr = t.shape
        m = t.reshape(dl, 2 * dr)
        # LQ factorisation M = L Q from the QR factorisation of M^H.
        q, r = np.linalg.qr(m.conj().T, mode="reduced")
        lfac = r.conj().T
        a[k] = q.conj().T.reshape(-1, 2, dr)
        a[k - 1] = np.einsum("lsc,cd->lsd", a[k - 1], lfac)
    a[0] = _apply_1q(a[0], gates.layer_gate(theta[0], phi[0]))


def cnot_two_site(theta2: np.ndarray) -> np.ndarray:
    """CNOT with control = first site, target = second site on a two-site tensor
    Theta[l, s, t, r]: (s, t) -> (s, t XOR s)."""
    gated = theta2.copy()
    gated[:, 1, :, :] = theta2[:, 1, ::-1, :]
    return gated


def truncate(s: np.ndarray, chi: int | None):
    """Number kept, discarded weight, gap sigma_D - sigma_{D+1} and the kept singular
    values rescaled to unit 2-norm."""
    if chi is None:
        d = int(np.count_nonzero(s > EXACT_CUTOFF * s[0]))
    else:
        d = min(chi, len(s))
    err = float(np.sum(s[d:] ** 2)) / float(np.sum(s * s))
    gap = s[d - 1] - s[d] if d < len(s) else np.inf
    return d, err, gap, s[:d] / np.linalg.norm(s[:d])


def cnot_ladder(mps: MPS, chi: int | None) -> None:
    """CNOT(k, k+1) for k = 0..n-2, each as a two-site update with SVD truncation."""
    a = mps.tensors
    n = len(a)
    errs = np.zeros(n - 1)
    gaps = np.full(n - 1, np.inf)
    spectra = []
    for k in range(n - 1):
        theta2 = np.einsum("lsc,ctr->lstr", a[k], a[k + 1])
        gated = cnot_two_site(theta2)
        dl, dr = gated.shape[0], gated.shape[3]
        mat = gated.reshape(2 * dl, 2 * dr)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
        spectra.append(s)
        d, errs[k], gaps[k], kept = truncate(s, chi)
        a[k] = u[:, :d].reshape(dl, 2, d)
        a[k + 1] = (kept[:, None] * vh[:d]).reshape(d, 2, dr)
    mps.trunc_err.append(errs)
    mps.gaps.append(gaps)
    mps.spectra.append(spectra)


def apply_layer(mps: MPS, theta: np.ndarray, phi: np.ndarray, chi: int | None) -> None:
    canonicalise_right(mps, theta, phi)
    cnot_ladder(mps, chi)


def simulate(x, theta, phi, chi: int | None) -> MPS:
    mps = product_mps(np.asarray(x, dtype=np.float64))
    for layer in range(len(theta)):
        apply_layer(mps, theta[layer], phi[layer], chi)
    return mps


def left_envs(a: list) -> list:
    """L_k (ket index, bra index) = contraction of sites 0..k-1 with their conjugates."""
    envs = [np.ones((1, 1), dtype=np.complex128)]
    for t in a:
        envs.append(np.einsum("ab,asc,bsd->cd", envs[-1], t, t.conj(), optimize=True))
    return envs


def right_envs(a: list) -> list:
    """R_k (ket, bra) = contraction of sites k..n-1; R_n = 1."""
    n = len(a)
    envs = [None] * (n + 1)
    envs[n] = np.ones((1, 1), dtype=np.complex128)
    for k in range(n - 1, -1, -1):
        t = a[k]
        envs[k] = np.einsum("asc,cd,bsd->ab", t, envs[k + 1], t.conj(), optimize=True)
    return envs


def pair_rdm(a: list, lenv: list, renv: list, i: int, j: int) -> np.ndarray:
    """rho_ij (4x4, index s_i*2 + s_j): open with L_i and A[i], carry through the transfer
    matrices of sites i+1..j-1, close with A[j] and R_{j+1}."""
    f = np.einsum("ab,asc,bud->sucd", lenv[i], a[i], a[i].conj(), optimize=True)
    for k in range(i + 1, j):
        # transfer map of site k on every (s, u) block: F <- sum_x A_x^T F conj(A_x)
        f = sum(a[k][:, x, :].T @ f @ a[k][:, x, :].conj() for x in range(2))
    rho = np.einsum("sucd,ctb,dvf,bf->stuv", f, a[j], a[j].conj(), renv[j + 1], optimize=True)
    return rho.reshape(4, 4)


def pauli_pair_features(mps: MPS, pairs: np.ndarray) -> np.ndarray:
    a = mps.tensors
    lenv, renv = left_envs(a), right_envs(a)
    out = np.empty((len(pairs), 15))
    for q, (i, j) in enumerate(pairs):
        rho = pair_rdm(a, lenv, renv, int(i), int(j))
        for alpha in range(15):
            out[q, alpha] = np.trace(rho @ gates.pair_pauli(alpha)).real
    return out


def norm2(mps: MPS) -> float:
    return float(left_envs(mps.tensors)[-1][0, 0].real)


def features(x, theta, phi, pairs, chi: int | None = None) -> tuple[np.ndarray, MPS]:
    mps = simulate(x, theta, phi, chi)
    return pauli_pair_features(mps, pairs), mps


def to_statevector(mps: MPS) -> np.ndarray:
    """Contract the chain into a dense [2]*n array (small n only)."""
    psi = mps.tensors[0]
    for t in mps.tensors[1:]:
        psi = np.tensordot(psi, t, axes=([psi.ndim - 1], [0]))
    return psi.reshape([2] * mps.n)
