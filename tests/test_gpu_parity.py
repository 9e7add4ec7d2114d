"""Parity of the HIP path (through the C-ABI) with the CPU oracle, element by element.

Tolerances: FP64 batches 1e-10 absolute against the exact result (and against the truncated
oracle when chi < 2^L); FP32 batches (complex64 state, FP64 SVD) 1e-5 absolute.
"""
import numpy as np
import pytest

from oracle import closed_form, features as ofeat, readout as oread, mps as omps
from oracle import paper_ansatz as opa
from paper_2607_10280_amd import inputs
from tests.golden_cases import hand_derived_cases
from tests.tolerances import fp32_truncated_tol

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
    print(f"[case] B={np.shape(pixels)[0]} n={np.shape(pixels)[1]} L={len(theta)} chi={chi} "
          f"prec={prec} m={len(pairs)}", flush=True)
    res = A.extract_features(pixels, theta, phi, pairs, chi, prec, return_trunc_err=trunc)
    torch.cuda.synchronize()
    return tuple(r.cpu().numpy() for r in res)


# ------------------------------------------------------------------ tiny config (exact)
def test_tiny_config_fp64(A):
    p, n, B = 4, 16, 8
    x = inputs.uniform_pixels(B, n, 0)
    th, ph = inputs.layer_angles(1, n, 1)
    pairs = inputs.neighbour_pairs(p)
    out, status = run(A, x, th, ph, pairs, 4, A.PREC_FP64)
    ref = ofeat.exact_features(x, th, ph, pairs)
    assert out.dtype == np.float64 and out.shape == (B, 24, 15)
    assert np.all(status == 0)
    assert np.abs(out - ref).max() <= FP64_TOL


@pytest.mark.parametrize("case", hand_derived_cases(), ids=lambda c: c["name"])
def test_hand_derived(A, case):
    for chi in (2, 4):
        out, status = run(A, case["x"][None], case["theta"], case["phi"], case["pairs"], chi,
                          A.PREC_FP64)
        assert np.all(status == 0)
        np.testing.assert_allclose(out[0], case["expect"], atol=FP64_TOL)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4])
def test_exact_regime_fp64(A, L):
    p, n, B = 4, 16, 5
    x = inputs.uniform_pixels(B, n, 10 + L)
    th, ph = inputs.layer_angles(L, n, 20 + L)
    pairs = inputs.neighbour_pairs(p)
    out, status = run(A, x, th, ph, pairs, max(2 ** L, 2), A.PREC_FP64)
    ref = ofeat.exact_features(x, th, ph, pairs)
    assert np.all(status == 0)
    assert np.abs(out - ref).max() <= FP64_TOL


@pytest.mark.parametrize("L,chi", [(2, 2), (3, 2), (3, 4), (4, 4), (4, 8), (3, 3), (4, 5), (4, 6)])
def test_truncated_regime_fp64(A, L, chi):
    """chi < 2^L: the GPU follows the truncated oracle step by step; P5 bounds both."""
    p, n, B = 4, 16, 4
    x = inputs.uniform_pixels(B, n, 30 + L)
    th, ph = inputs.layer_angles(L, n, 40 + L)
    pairs = inputs.neighbour_pairs(p)
    out, status, terr = run(A, x, th, ph, pairs, chi, A.PREC_FP64, trunc=True)
    ref, errs, gaps = ofeat.truncated_features(x, th, ph, pairs, chi)
    exact = ofeat.exact_features(x, th, ph, pairs)
    assert np.all(status == 0)
    np.testing.assert_allclose(terr, errs, atol=1e-12, rtol=1e-8)
    for b in range(B):
        bound = 2 * np.sum(np.sqrt(2 * errs[b]))
        assert np.abs(out[b] - exact[b]).max() <= bound + 1e-12
        # a non-degenerate truncation is unique: element-wise parity
        if np.min(gaps[b]) > 1e-6:
            assert np.abs(out[b] - ref[b]).max() <= 1e-9, (b, np.min(gaps[b]))


@pytest.mark.parametrize("p", [7, 16])
def test_l1_closed_form_large(A, p):
    n, B = p * p, 3
    x = inputs.blob_images(B, p, 50 + p)
    th, ph = inputs.layer_angles(1, n, 60 + p)
    pairs = inputs.neighbour_pairs(p)
    ref = np.stack([closed_form.l1_features(x[b], th, ph, pairs) for b in range(B)])
    out64, st = run(A, x, th, ph, pairs, 16, A.PREC_FP64)
    assert np.all(st == 0) and np.abs(out64 - ref).max() <= FP64_TOL
    out32, st = run(A, x, th, ph, pairs, 16, A.PREC_FP32)
    assert out32.dtype == np.float32
    assert np.all(st == 0) and np.abs(out32 - ref).max() <= FP32_TOL


def test_l0_closed_form(A):
    p, n, B = 7, 49, 4
    x = inputs.blob_images(B, p, 70)
    pairs = inputs.neighbour_pairs(p)
    empty = np.zeros((0, n))
    out, st = run(A, x, empty, empty, pairs, 16, A.PREC_FP64)
    ref = np.stack([closed_form.l0_features(x[b], pairs) for b in range(B)])
    assert np.abs(out - ref).max() <= 1e-14


@pytest.mark.parametrize("L,chi", [(2, 4), (3, 8), (4, 16), (2, 2), (3, 2), (3, 4), (4, 2), (4, 4),
                                   (4, 8), (4, 12), (4, 6), (3, 5)])
def test_49q_grid_fp32(A, L, chi):
    """7x7 blob images, complex64 contractions with FP64 SVD: exact cells against the exact
    oracle at 1e-5; truncated cells against the truncated oracle element by element on every
    image at the gap-derived tolerance of tests/tolerances.py, the discarded weights, and the
    truncation bound
    |<P> - <P>_exact| <= 2 sum sqrt(2 eps) on every image."""
    p, n, B = 7, 49, 4
    x = inputs.blob_images(B, p, 80 + L)
    th, ph = inputs.layer_angles(L, n, 90 + L)
    pairs = inputs.neighbour_pairs(p)
    out, st, terr = run(A, x, th, ph, pairs, chi, A.PREC_FP32, trunc=True)
    assert np.all(st == 0)
    exact = ofeat.exact_features(x, th, ph, pairs)
    if chi >= 2 ** L:
        assert np.abs(out - exact).max() <= FP32_TOL
        return
    for b in range(B):
        m = omps.simulate(x[b], th, ph, chi)
        ref = omps.pauli_pair_features(m, pairs)
        errs = np.stack(m.trunc_err)
        tol = fp32_truncated_tol(m, chi)
        err = np.abs(out[b] - ref).max()
        print(f"[trunc] L={L} chi={chi} image {b}: max err {err:.2e}, tol {tol:.2e}", flush=True)
        assert err <= tol, (b, err, tol)
        bound = 2.0 * np.sum(np.sqrt(2.0 * errs))
        assert np.abs(out[b] - exact[b]).max() <= bound + FP32_TOL, b
        np.testing.assert_allclose(terr[b], errs, atol=1e-6, rtol=1e-3)


@pytest.mark.parametrize("prec", [0, 1])
def test_exact_layer_modes_agree(A, prec):
    """chi = 16 = 2^L keeps every singular value, so each layer is applied by default as the
    parity product operator site by site; the one-sweep QR split and the canonical sweep +
    Jacobi SVD ladder give the same features, all three match the oracle, and the two exact
    modes report zero discarded weight."""
    p, n, B, L, chi = 7, 49, 4, 4, 16
    x = inputs.blob_images(B, p, 500)
    th, ph = inputs.layer_angles(L, n, 501)
    pairs = inputs.neighbour_pairs(p)
    res = {}
    try:
        for mode in (A.EXACT_SVD, A.EXACT_QR, A.EXACT_MPO):
            A.set_exact_layers(mode)
            res[mode] = run(A, x, th, ph, pairs, chi, prec, trunc=True)
    finally:
        A.set_exact_layers(A.EXACT_MPO)
    ref = ofeat.exact_features(x[:2], th, ph, pairs)
    tol = FP64_TOL if prec == A.PREC_FP64 else FP32_TOL
    svd = res[A.EXACT_SVD][0]
    for mode, (out, status, terr) in res.items():
        assert np.all(status == 0), mode
        if mode == A.EXACT_SVD:
            assert terr.max() < 1e-20
        else:
            assert np.all(terr == 0.0), mode
        assert np.abs(out - svd).max() <= tol, mode
        assert np.abs(out[:2] - ref).max() <= tol, mode


# ------------------------------------------------------------------ edge cases
def test_edge_two_sites_and_long_range_pairs(A):
    # n = 2 (single bond), and a 7-site chain with all pairs (long-range propagation).
    x = np.array([[0.3, 0.8]])
    th, ph = inputs.layer_angles(2, 2, 100)
    pairs = np.array([[0, 1]], np.int32)
    out, st = run(A, x, th, ph, pairs, 2, A.PREC_FP64)
    assert np.abs(out - ofeat.exact_features(x, th, ph, pairs)).max() <= FP64_TOL
    n = 7
    x = inputs.uniform_pixels(3, n, 101)
    th, ph = inputs.layer_angles(3, n, 102)
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)][::-1], np.int32)
    out, st = run(A, x, th, ph, pairs, 8, A.PREC_FP64)
    assert np.abs(out - ofeat.exact_features(x, th, ph, pairs)).max() <= FP64_TOL


def test_edge_empty_pairs_and_ragged_batch(A):
    import torch
    n = 9
    x = inputs.uniform_pixels(7, n, 110)
    th, ph = inputs.layer_angles(2, n, 111)
    out, st = run(A, x, th, ph, np.zeros((0, 2), np.int32), 4, A.PREC_FP32)
    assert out.shape == (7, 0, 15) and np.all(st == 0)
    pairs = inputs.neighbour_pairs(3)
    out, st = run(A, x, th, ph, pairs, 4, A.PREC_FP64)
    assert np.abs(out - ofeat.exact_features(x, th, ph, pairs)).max() <= FP64_TOL
    torch.cuda.synchronize()


def test_edge_nonfinite_pixel_and_invalid_pair(A):
    import torch
    n = 9
    x = inputs.uniform_pixels(3, n, 120)
    x[1, 4] = np.nan
    th, ph = inputs.layer_angles(1, n, 121)
    pairs = inputs.neighbour_pairs(3)
    out, st = run(A, x, th, ph, pairs, 2, A.PREC_FP64)
    assert st[1] & A.IMG_NONFINITE and st[0] == 0 and st[2] == 0
    assert np.abs(out[[0, 2]] - ofeat.exact_features(x[[0, 2]], th, ph, pairs)).max() <= FP64_TOL
    # an invalid pair sent to the device (bypassing the host validator) gives NaN, others fine
    b = A.new_batch(n, 2, 1, 2, A.PREC_FP64)
    A.init_batch(b, torch.as_tensor(x[[0, 2]], device="cuda").contiguous())
    A.apply_layer(b, torch.as_tensor(th[0], device="cuda"), torch.as_tensor(ph[0], device="cuda"))
    bad = np.array([[0, 1], [5, 3], [2, 9], [1, 4]], np.int32)
    out = torch.empty((2, 4, 15), dtype=torch.float64, device="cuda")
    A.pauli_pair_expect(b, torch.as_tensor(bad, device="cuda"), out)
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[:, 1])) and np.all(np.isnan(o[:, 2]))
    ref = ofeat.exact_features(x[[0, 2]], th, ph, bad[[0, 3]])
    assert np.abs(o[:, [0, 3]] - ref).max() <= FP64_TOL
    with pytest.raises(A.MpsError):
        A.apply_layer(b, torch.as_tensor(th[0], device="cuda"), torch.as_tensor(ph[0], device="cuda"))


def test_determinism_and_batch_invariance(A):
    p, n = 7, 49
    x = inputs.blob_images(6, p, 130)
    th, ph = inputs.layer_angles(3, n, 131)
    pairs = inputs.neighbour_pairs(p)
    a, _ = run(A, x, th, ph, pairs, 8, A.PREC_FP32)
    b, _ = run(A, x, th, ph, pairs, 8, A.PREC_FP32)
    assert np.array_equal(a, b)
    alone, _ = run(A, x[3:4], th, ph, pairs, 8, A.PREC_FP32)
    assert np.array_equal(alone[0], a[3])


# ------------------------------------------------------------------ readout
@pytest.mark.parametrize("f64", [True, False])
def test_readout(A, f64):
    import torch
    p, n, B = 7, 49, 4
    x = inputs.blob_images(B, p, 140)
    th, ph = inputs.layer_angles(2, n, 141)
    pairs = inputs.neighbour_pairs(p)
    m = len(pairs)
    a, bb, d, w, bias = inputs.readout_params(m, 784, 142)
    bias = bias + np.linspace(-0.1, 0.1, 784)
    prec = A.PREC_FP64 if f64 else A.PREC_FP32
    out, _ = run(A, x, th, ph, pairs, 4, prec)
    dt = torch.float64 if f64 else torch.float32
    dev = "cuda"
    T = lambda v: torch.as_tensor(v, dtype=dt, device=dev).contiguous()
    coeff = torch.empty((m, 16), dtype=dt, device=dev)
    A.ano_coeffs(T(a), T(bb), T(d), coeff)
    y = torch.empty((B, 784), dtype=dt, device=dev)
    A.ano_readout(T(out), coeff, T(w), T(bias), y)
    torch.cuda.synchronize()
    ref_c = oread.coefficients(a, bb, d)
    ref_y = oread.readout(out.astype(np.float64), a, bb, d, w, bias)
    tol = 1e-12 if f64 else 1e-5
    assert np.abs(coeff.cpu().numpy() - ref_c).max() <= tol
    assert np.abs(y.cpu().numpy() - ref_y).max() <= tol * 10


@pytest.mark.parametrize("f64,B,m,out_dim", [(False, 37, 156, 784), (True, 37, 156, 784),
                                             (True, 3, 4096, 40), (False, 19, 1, 5)])
def test_readout_blocks(A, f64, B, m, out_dim):
    """The blocked readout on ragged image and output blocks, a block size cut down to fit LDS
    (156 observables in FP64), the one-image-per-workgroup form for very long feature vectors
    (4096, the largest, in FP64) and a single observable, against the oracle's readout."""
    import torch
    rng = np.random.default_rng(700 + m)
    pauli = rng.uniform(-1, 1, (B, m, 15))
    a, bb, d, w, bias = inputs.readout_params(m, out_dim, 701)
    dt = torch.float64 if f64 else torch.float32
    T = lambda v: torch.as_tensor(v, dtype=dt, device="cuda").contiguous()
    print(f"[case] readout f64={f64} B={B} m={m} out={out_dim}", flush=True)
    coeff = torch.empty((m, 16), dtype=dt, device="cuda")
    A.ano_coeffs(T(a), T(bb), T(d), coeff)
    y = torch.empty((B, out_dim), dtype=dt, device="cuda")
    pd = T(pauli)
    A.ano_readout(pd, coeff, T(w), T(bias), y)
    torch.cuda.synchronize()
    ref_y = oread.readout(pd.cpu().numpy().astype(np.float64), a, bb, d, w, bias)
    tol = 1e-11 if f64 else 2e-5
    assert np.abs(y.cpu().numpy() - ref_y).max() <= tol * max(1.0, np.abs(ref_y).max())


# ------------------------------------------------------------------ full-size workload
@pytest.mark.parametrize("mode", ["svd", "mpo"])
def test_headline_size_sampled(A, mode):
    """7x7, L=4, chi=16, batch 1024 (complex64 / FP64 SVD), in the benchmark's layer mode (the
    canonical sweep + Jacobi SVD ladder) and with the exact shortcut: sampled images against
    the exact oracle, invariants on every output."""
    p, n, B, L = 7, 49, 1024, 4
    x = inputs.blob_images(B, p, 2)
    th, ph = inputs.layer_angles(L, n, 3 + L)
    pairs = inputs.neighbour_pairs(p)
    try:
        A.set_exact_layers(A.EXACT_SVD if mode == "svd" else A.EXACT_MPO)
        out, st = run(A, x, th, ph, pairs, 16, A.PREC_FP32)
    finally:
        A.set_exact_layers(A.EXACT_MPO)
    assert np.all(st == 0)
    assert np.all(np.isfinite(out)) and np.abs(out).max() <= 1 + 1e-5
    assert np.all(np.sum(out.astype(np.float64) ** 2, axis=2) <= 3 + 1e-4)
    sample = [0, 1, 511, 1023]
    ref = ofeat.exact_features(x[sample], th, ph, pairs)
    assert np.abs(out[sample] - ref).max() <= FP32_TOL


# ------------------------------------------------------------------ split-BF16 contractions
# Each product term carries a relative error of at most ~3 * 2^-18 (two bf16 roundings and the
# dropped lo*lo term); an expectation passes through about 2n + 2p such contraction levels
# (environment sweep and pair transfers), which gives ~1e-3 for 7x7 and ~4e-3 for 16x16 if
# every level erred at the bound in the same direction.  The test bar is that linear bound.
SPLIT_TOL = {7: 2.0 ** -10, 16: 2.0 ** -8}


@pytest.mark.parametrize("p", [7, 16])
def test_split_bf16_contractions(A, p):
    n, B, L = p * p, 2, 4
    x = inputs.blob_images(B, p, 150 + p)
    th, ph = inputs.layer_angles(L, n, 151 + p)
    pairs = inputs.neighbour_pairs(p)
    out, st = run(A, x, th, ph, pairs, 16, A.PREC_SPLIT_BF16)
    f32, _ = run(A, x, th, ph, pairs, 16, A.PREC_FP32)
    assert np.all(st == 0) and out.dtype == np.float32
    ref = ofeat.exact_features(x, th, ph, pairs)
    err, err32 = np.abs(out - ref).max(), np.abs(f32 - ref).max()
    print(f"[split-bf16] p={p} max err {err:.3e} (fp32 {err32:.3e})", flush=True)
    assert err <= SPLIT_TOL[p]
    assert err > 0  # the variant really runs (a bit-exact match would mean the FP32 path ran)


@pytest.mark.parametrize("L,chi", [(1, 16), (2, 32), (2, 64)])
def test_precision_grid_256_qubits(A, L, chi):
    """16x16 images at shallow depth with a large bond limit: the bond rule caps every bond at
    2^L, so FP32 and split-BF16 run the same vector contractions and both meet the FP32 bar."""
    p = 16
    n = p * p
    x = inputs.blob_images(2, p, 180 + L)
    th, ph = inputs.layer_angles(L, n, 181 + L)
    pairs = inputs.neighbour_pairs(p)
    ref = ofeat.exact_features(x, th, ph, pairs)
    f32, st = run(A, x, th, ph, pairs, chi, A.PREC_FP32)
    split, st2 = run(A, x, th, ph, pairs, chi, A.PREC_SPLIT_BF16)
    assert A.slot_dim(n, chi, L) == 2 ** L
    assert np.all(st == 0) and np.all(st2 == 0)
    assert np.abs(f32 - ref).max() <= FP32_TOL
    assert np.array_equal(split, f32)


# ------------------------------------------------------------------ the paper's own circuit


def run_paper(A, pixels, L, pairs, chi, prec, trunc=False):
    import torch
    print(f"[case] paper circuit B={np.shape(pixels)[0]} n={np.shape(pixels)[1]} L={L} chi={chi} "
          f"prec={prec} m={len(pairs)}", flush=True)
    res = A.paper_features(pixels, L, pairs, chi, prec, return_trunc_err=trunc)
    torch.cuda.synchronize()
    return tuple(r.cpu().numpy() for r in res)


@pytest.mark.parametrize("x0,L,n", [(0.0, 1, 4), (0.0, 1, 5), (0.0, 2, 5), (0.75, 1, 5), (0.5, 3, 6)])
def test_paper_circuit_special_inputs(A, x0, L, n):
    """Inputs whose results are worked out by hand in the oracle's pins."""
    pairs = np.array([[i, j] for i in range(n) for j in range(i + 1, n)], dtype=np.int32)
    x = np.full((1, n), x0)
    out, st = run_paper(A, x, L, pairs, 8, A.PREC_FP64)
    assert st[0] == 0
    assert np.abs(out[0] - opa.sv_features(x[0], L, pairs)).max() <= 1e-12


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_paper_circuit_exact_fp64(A, L):
    p, n, B = 4, 16, 3
    x = inputs.blob_images(B, p, 160 + L)
    pairs = inputs.neighbour_pairs(p, diagonal=True)
    out, st = run_paper(A, x, L, pairs, 16, A.PREC_FP64)
    assert np.all(st == 0)
    assert np.abs(out - opa.features(x, L, pairs)).max() <= FP64_TOL


@pytest.mark.parametrize("L,chi", [(2, 2), (3, 2), (3, 3), (4, 4), (4, 6)])
def test_paper_circuit_truncated_fp64(A, L, chi):
    p, n, B = 4, 16, 3
    x = inputs.uniform_pixels(B, n, 170 + 10 * L + chi)
    pairs = inputs.neighbour_pairs(p, diagonal=True)
    out, st, te = run_paper(A, x, L, pairs, chi, A.PREC_FP64, trunc=True)
    assert np.all(st == 0)
    exact = opa.features(x, L, pairs)
    for b in range(B):
        m = opa.mps_simulate(x[b], L, chi)
        ref = omps.pauli_pair_features(m, pairs)
        errs = np.stack(m.trunc_err)
        bound = 2.0 * np.sum(np.sqrt(2.0 * errs))
        assert np.abs(out[b] - exact[b]).max() <= bound + 1e-9
        if np.min(np.stack(m.gaps)) > 1e-6:
            assert np.abs(out[b] - ref).max() <= FP64_TOL
            assert np.abs(te[b] - errs).max() <= 1e-10


def test_paper_circuit_49q_fp32(A):
    """7x7 with the paper's 156 neighbour pairs, L = 4, chi = 16, complex64 + FP64 SVD."""
    p, n, B, L = 7, 49, 2, 4
    x = inputs.blob_images(B, p, 180)
    pairs = inputs.neighbour_pairs(p, diagonal=True)
    assert len(pairs) == 156
    out, st = run_paper(A, x, L, pairs, 16, A.PREC_FP32)
    assert np.all(st == 0)
    assert np.abs(out - opa.features(x, L, pairs)).max() <= FP32_TOL
