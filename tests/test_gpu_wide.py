"""Parity of the wide-slot path (S = 32, 64, 128: one 256-lane workgroup per image, per-bond
matrices in an HBM workspace) with the CPU oracle, through the C-ABI.

Exact regime (chi >= 2^L) against the statevector on 4x4 images, where bonds reach 32, 64 and
128 at L = 5, 6, 7; the truncated regime against the oracle's truncated MPS step by step (and
the truncation bound against the exact result); a 7x7 image at L = 7, chi = 128 against the
untruncated oracle MPS; the paper's own circuit in a wide slot.  Tolerances as for the narrow
slots: FP64 1e-10, complex64 state with FP64 SVD 1e-5.
"""
import numpy as np
import pytest

from oracle import features as ofeat, paper_ansatz as opa
from paper_2607_10280_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def A():
    import torch  # noqa: F401
    from paper_2607_10280_amd import anomps
    anomps.lib()
    return anomps


def run(A, pixels, theta, phi, pairs, chi, prec, trunc=False):
    import torch
    print(f"[case] wide B={np.shape(pixels)[0]} n={np.shape(pixels)[1]} L={len(theta)} chi={chi} "
          f"prec={prec} slot={A.slot_dim(np.shape(pixels)[1], chi, len(theta))}", flush=True)
    res = A.extract_features(pixels, theta, phi, pairs, chi, prec, return_trunc_err=trunc)
    torch.cuda.synchronize()
    return tuple(r.cpu().numpy() for r in res)


@pytest.mark.parametrize("L,chi,prec", [(5, 32, 0), (6, 64, 0), (7, 128, 0), (6, 64, 1), (7, 128, 1)])
def test_exact_regime_4x4(A, L, chi, prec):
    p, n, B = 4, 16, 3
    assert A.slot_dim(n, chi, L) == chi
    x = inputs.blob_images(B, p, 400 + L)
    th, ph = inputs.layer_angles(L, n, 410 + L)
    pairs = np.concatenate([inputs.neighbour_pairs(p, True), np.array([[0, 15], [3, 12]], np.int32)])
    out, status = run(A, x, th, ph, pairs, chi, prec)
    ref = ofeat.exact_features(x, th, ph, pairs)
    assert np.all(status == 0)
    tol = FP64_TOL if prec == A.PREC_FP64 else FP32_TOL
    assert out.dtype == (np.float64 if prec == A.PREC_FP64 else np.float32)
    assert np.abs(out - ref).max() <= tol


@pytest.mark.parametrize("L,chi", [(6, 32), (7, 48), (7, 64)])
def test_truncated_regime_4x4(A, L, chi):
    """chi < 2^L in a wide slot: the GPU follows the truncated oracle; the discarded weights
    agree and bound the distance to the exact features."""
    p, n, B = 4, 16, 2
    x = inputs.uniform_pixels(B, n, 420 + L + chi)
    th, ph = inputs.layer_angles(L, n, 430 + L)
    pairs = inputs.neighbour_pairs(p)
    out, status, terr = run(A, x, th, ph, pairs, chi, A.PREC_FP64, trunc=True)
    ref, errs, gaps = ofeat.truncated_features(x, th, ph, pairs, chi)
    exact = ofeat.exact_features(x, th, ph, pairs)
    assert np.all(status == 0)
    assert errs.max() > 0
    np.testing.assert_allclose(terr, errs, atol=1e-12, rtol=1e-8)
    for b in range(B):
        bound = 2 * np.sum(np.sqrt(2 * errs[b]))
        assert np.abs(out[b] - exact[b]).max() <= bound + 1e-12
        if np.min(gaps[b]) > 1e-6:
            assert np.abs(out[b] - ref[b]).max() <= 1e-9, (b, np.min(gaps[b]))


def test_7x7_chi128_sampled(A):
    """49 qubits, L = 7, chi = 128 = 2^L (no truncation): one blob image against the oracle's
    untruncated MPS, complex64 state with FP64 SVD."""
    p, n, L = 7, 49, 7
    x = inputs.blob_images(1, p, 440)
    th, ph = inputs.layer_angles(L, n, 441)
    pairs = inputs.neighbour_pairs(p)
    out, status = run(A, x, th, ph, pairs, 128, A.PREC_FP32)
    print("[step] GPU done, oracle", flush=True)
    ref = ofeat.exact_features(x, th, ph, pairs)
    assert np.all(status == 0)
    assert np.abs(out - ref).max() <= FP32_TOL


def test_paper_circuit_wide(A):
    """The paper's encoding circuit (H, R_Y(2 pi x - pi), brickwork CNOTs) at L = 6 on a 4x4
    image: bonds reach 64, so the wide kernels run both layer programs' sweeps."""
    import torch
    p, n, L, B = 4, 16, 6, 2
    x = inputs.blob_images(B, p, 450)
    pairs = inputs.neighbour_pairs(p, True)
    print(f"[case] wide paper circuit n={n} L={L} chi=64", flush=True)
    out, status = A.paper_features(x, L, pairs, 64, A.PREC_FP64)
    torch.cuda.synchronize()
    out, status = out.cpu().numpy(), status.cpu().numpy()
    assert np.all(status == 0)
    for b in range(B):
        assert np.abs(out[b] - opa.sv_features(x[b], L, pairs)).max() <= FP64_TOL
