"""Front door of the oracle: Pauli-pair features for a batch (test infrastructure only).

``exact_features`` is the plain definition out[b][q][alpha] = <psi(x_b)| P_a^{(i_q)} P_b^{(j_q)}
|psi(x_b)> (Eq. (1), (4), (5)); it uses the statevector for n <= 20 and the untruncated MPS
otherwise.  ``truncated_features`` follows the MPS algorithm step by step with bond
dimension at most chi (§II-B) and is what a truncating simulator must reproduce.
"""
from __future__ import annotations

import numpy as np

from . import mps as mps_mod
from . import statevector


def exact_features(pixels, theta, phi, pairs) -> np.ndarray:
    pixels = np.atleast_2d(pixels)
    n = pixels.shape[1]
    out = []
    for x in pixels:
        if n <= statevector.MAX_QUBITS:
            out.append(statevector.features(x, theta, phi, pairs))
        else:
            out.append(mps_mod.features(x, theta, phi, pairs, chi=None)[0])
    return np.stack(out)


def truncated_features(pixels, theta, phi, pairs, chi: int):
    """Returns (features [B][m][15], trunc_err [B][L][n-1], gaps [B][L][n-1])."""
    pixels = np.atleast_2d(pixels)
    feats, errs, gaps = [], [], []
    for x in pixels:
        f, m = mps_mod.features(x, theta, phi, pairs, chi=chi)
        feats.append(f)
        errs.append(np.stack(m.trunc_err) if m.trunc_err else np.zeros((0, len(x) - 1)))
        gaps.append(np.stack(m.gaps) if m.gaps else np.zeros((0, len(x) - 1)))
    return np.stack(feats), np.stack(errs), np.stack(gaps)
