"""The allocation-free measurement (mps_pauli_pair_expect_noalloc) through the C-ABI: its
environments live in the library's fixed scratch array, so it must give exactly the results of
mps_pauli_pair_expect with a caller-owned environment buffer, on consecutive calls of different
sizes (the second smaller than the first), and reject batches that do not fit."""
import numpy as np
import pytest

from paper_2607_10280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch  # noqa: F401
    from paper_2607_10280_amd import anomps
    anomps.lib()
    return anomps


def _prepared(A, p, L, chi, B, prec, seed):
    import torch
    n = p * p
    x = inputs.blob_images(B, p, seed)
    th, ph = inputs.layer_angles(L, n, seed + 1)
    pairs = inputs.neighbour_pairs(p)
    b = A.new_batch(n, chi, L, B, prec)
    A.init_batch(b, torch.as_tensor(x, device="cuda").contiguous())
    if L:
        A.apply_layers(b, torch.as_tensor(th, device="cuda").contiguous(),
                       torch.as_tensor(ph, device="cuda").contiguous())
    return b, torch.as_tensor(pairs, device="cuda").contiguous()


def _both(A, b, pairs_d):
    import torch
    dt = torch.float64 if b.desc.precision == A.PREC_FP64 else torch.float32
    m = pairs_d.shape[0]
    ref = torch.full((b.desc.batch, m, 15), float("nan"), dtype=dt, device="cuda")
    A.pauli_pair_expect(b, pairs_d, ref)
    got = torch.full_like(ref, float("nan"))
    env = b.desc.env
    b.desc.env = 0  # the allocation-free call must not touch the caller's environment buffer
    try:
        A.pauli_pair_expect_noalloc(b, pairs_d, got)
    finally:
        b.desc.env = env
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_two_calls_second_smaller(A):
    cases = [(7, 4, 16, 96, A.PREC_FP32, 40), (4, 2, 4, 8, A.PREC_FP64, 50)]
    for p, L, chi, B, prec, seed in cases:
        print(f"[case] noalloc p={p} L={L} chi={chi} B={B} prec={prec}", flush=True)
        b, pairs_d = _prepared(A, p, L, chi, B, prec, seed)
        need = A.env_bytes(p * p, chi, L, B, prec)
        assert need <= A.NOALLOC_SCRATCH_BYTES
        ref, got = _both(A, b, pairs_d)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(ref, got), (p, L, chi, B, prec)


def test_noalloc_rejects_oversized_and_wide(A):
    import torch
    # 7x7, chi = 16, L = 4 at 1024 images: 210 MB of environments, beyond the 64 MiB scratch
    b = A.new_batch(49, 16, 4, 1024, A.PREC_FP32)
    out = torch.empty((1024, 84, 15), dtype=torch.float32, device="cuda")
    pairs_d = torch.as_tensor(inputs.neighbour_pairs(7), device="cuda").contiguous()
    with pytest.raises(A.MpsError) as e:
        A.pauli_pair_expect_noalloc(b, pairs_d, out)
    assert e.value.code == -2
    # slots above 16 are not served by the scratch
    w = A.new_batch(16, 32, 5, 1, A.PREC_FP32)
    o = torch.empty((1, 24, 15), dtype=torch.float32, device="cuda")
    pw = torch.as_tensor(inputs.neighbour_pairs(4), device="cuda").contiguous()
    with pytest.raises(A.MpsError) as e:
        A.pauli_pair_expect_noalloc(w, pw, o)
    assert e.value.code == -4
    torch.cuda.synchronize()
