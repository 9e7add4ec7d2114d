"""Tolerances shared by the GPU parity tests.

Truncated complex64 results: the kept subspace of a truncated bond moves under a perturbation
eta of the two-site matrix by about eta / gap (Wedin's theorem), which changes the truncated
state by about eta * sigma_D / gap (the rotation mixes the directions of sigma_D and
sigma_D+1); first-order changes of successive truncations add.  eta is the complex64 rounding
the state has accumulated, about 16 * 2^-24 (exact cells at 49 qubits show errors of ~1e-6),
and an expectation moves by at most twice the state, so a truncated complex64 image is held to
    tol = max(1e-5, 32 * 2^-24 * kappa),  kappa = sum over truncated bonds of sigma_D / gap,
with sigma_D the smallest kept singular value and gap = sigma_D - sigma_D+1 in the oracle's
spectra.
"""
FP64_TOL = 1e-10
FP32_TOL = 1e-5
FP32_TRUNC_C = 32.0


def kappa(m, chi):
    """Sum of sigma_D / (sigma_D - sigma_D+1) over the truncated bonds of an oracle MPS run."""
    k = 0.0
    for layer in m.spectra:
        for s in layer:
            d = min(chi, len(s))
            if d < len(s):
                k += s[d - 1] / max(s[d - 1] - s[d], 1e-300)
    return k


def fp32_truncated_tol(m, chi):
    return max(FP32_TOL, FP32_TRUNC_C * 2.0 ** -24 * kappa(m, chi))
