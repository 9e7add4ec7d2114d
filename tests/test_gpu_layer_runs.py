"""mps_apply_layers (several layers per call) against one mps_apply_layer call per layer and the
oracle, through the C-ABI.  A run of exact layers goes through the two run kernels (the core
sites take every layer of the run on chip).  The arithmetic is the per-layer kernels', but the
compiler may contract a product and a sum into one FMA in one kernel and not in the other, so
FP64 agrees to a few ulps; in complex64 the run's intermediate tensors also stay in FP64.
"""
import numpy as np
import pytest

from oracle import features as ofeat
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


def both(A, x, th, ph, pairs, chi, prec):
    import torch
    print(f"[case] runs B={len(x)} n={x.shape[1]} L={len(th)} chi={chi} prec={prec}", flush=True)
    res = []
    for per_layer in (False, True):
        o, s, t = A.extract_features(x, th, ph, pairs, chi, prec, return_trunc_err=True,
                                     per_layer=per_layer)
        torch.cuda.synchronize()
        res.append((o.cpu().numpy(), s.cpu().numpy(), t.cpu().numpy()))
    return res


@pytest.mark.parametrize("p,L,chi", [(7, 4, 16), (4, 4, 16), (3, 3, 16), (5, 3, 8)])
def test_run_matches_per_layer_fp64(A, p, L, chi):
    n, B = p * p, 3
    x = inputs.blob_images(B, p, 600 + p)
    th, ph = inputs.layer_angles(L, n, 601 + L)
    pairs = inputs.neighbour_pairs(p)
    (o1, s1, t1), (o2, s2, t2) = both(A, x, th, ph, pairs, chi, A.PREC_FP64)
    assert np.all(s1 == 0) and np.all(s2 == 0)
    assert np.abs(o1 - o2).max() <= 1e-13
    assert np.all(t1 == 0.0) and np.all(t2 == 0.0)
    ref = ofeat.exact_features(x[:1], th, ph, pairs) if n <= 25 else None
    if ref is not None:
        assert np.abs(o1[:1] - ref).max() <= FP64_TOL


def test_run_matches_per_layer_complex64(A):
    p, L, chi, B = 7, 4, 16, 4
    n = p * p
    x = inputs.blob_images(B, p, 610)
    th, ph = inputs.layer_angles(L, n, 611)
    pairs = inputs.neighbour_pairs(p)
    (o1, s1, t1), (o2, s2, t2) = both(A, x, th, ph, pairs, chi, A.PREC_FP32)
    assert np.all(s1 == 0) and np.all(s2 == 0)
    assert np.abs(o1 - o2).max() <= 2e-6
    ref = ofeat.exact_features(x[:1], th, ph, pairs)
    assert np.abs(o1[:1] - ref).max() <= FP32_TOL


def test_run_then_truncating_layer(A):
    """chi = 8 at L = 4: the first three layers form a run, the fourth truncates and takes the
    canonical sweep + SVD ladder inside the same call; the discarded weights match the per-layer
    calls and the oracle's truncated MPS."""
    p, L, chi, B = 4, 4, 8, 2
    n = p * p
    x = inputs.uniform_pixels(B, n, 620)
    th, ph = inputs.layer_angles(L, n, 621)
    pairs = inputs.neighbour_pairs(p)
    (o1, s1, t1), (o2, s2, t2) = both(A, x, th, ph, pairs, chi, A.PREC_FP64)
    assert np.all(s1 == 0) and np.all(s2 == 0)
    assert np.abs(o1 - o2).max() <= 1e-12
    np.testing.assert_allclose(t1, t2, atol=1e-14, rtol=1e-10)
    assert np.all(t1[:, :3] == 0.0) and t1[:, 3].max() > 0
    ref, errs, gaps = ofeat.truncated_features(x, th, ph, pairs, chi)
    np.testing.assert_allclose(t1, errs, atol=1e-12, rtol=1e-8)
    for b in range(B):
        if np.min(gaps[b]) > 1e-6:
            assert np.abs(o1[b] - ref[b]).max() <= 1e-9


def test_run_argument_errors(A):
    import torch
    n, L = 16, 2
    b = A.new_batch(n, 16, L, 1, A.PREC_FP64)
    A.init_batch(b, torch.zeros((1, n), dtype=torch.float64, device="cuda"))
    th = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(A.MpsError) as e:
        A.apply_layers(b, th, th)          # 3 layers into a batch sized for 2
    assert e.value.code == -1
    A.apply_layers(b, th[:2], th[:2])
    with pytest.raises(A.MpsError):
        A.apply_layers(b, th[:1], th[:1])  # nothing left
    torch.cuda.synchronize()
    assert int(b.status.cpu()[0]) == 0


def test_run_inside_hip_graph(A):
    """init + mps_apply_layers (a run, so the ends go to the library's second stream) + the
    measurement captured as one HIP graph; three replays with eager work and synchronisations
    between them each equal the eager result bit for bit."""
    import torch
    p, L, chi, B = 7, 4, 16, 64
    n = p * p
    x = inputs.blob_images(B, p, 630)
    th, ph = inputs.layer_angles(L, n, 631)
    pairs = inputs.neighbour_pairs(p)
    print(f"[case] graph replay B={B} n={n} L={L} chi={chi}", flush=True)
    dev = "cuda"
    pix = torch.as_tensor(x, device=dev).contiguous()
    thd = torch.as_tensor(th, device=dev).contiguous()
    phd = torch.as_tensor(ph, device=dev).contiguous()
    pd = torch.as_tensor(pairs, device=dev).contiguous()
    b = A.new_batch(n, chi, L, B, A.PREC_FP32)
    out = torch.empty((B, len(pairs), 15), dtype=torch.float32, device=dev)

    def step():
        A.init_batch(b, pix)
        A.apply_layers(b, thd, phd)
        A.pauli_pair_expect(b, pd, out)

    step()
    torch.cuda.synchronize()
    eager = out.cpu().numpy().copy()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        step()
    for r in range(3):
        out.zero_()
        step()                       # eager work between the replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager)
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {r}"
    assert np.all(b.status.cpu().numpy() == 0)
