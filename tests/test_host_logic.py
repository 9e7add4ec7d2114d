"""Host-side logic of the serving loop and the input generators (CPU only)."""
import numpy as np
import pytest

from paper_2607_10280_amd import inputs
from paper_2607_10280_amd.serving import ALIGN, ArenaAllocator


def test_arena_first_fit_and_coalescing():
    a = ArenaAllocator(10 * ALIGN)
    x = a.alloc(3 * ALIGN)
    y = a.alloc(2 * ALIGN + 1)       # rounded up to 3 blocks
    z = a.alloc(ALIGN)
    assert (x, y, z) == (0, 3 * ALIGN, 6 * ALIGN) and a.used == 7 * ALIGN
    assert a.alloc(4 * ALIGN) is None  # only 3 blocks left at the end
    a.release(y, 2 * ALIGN + 1)
    assert a.alloc(3 * ALIGN) == 3 * ALIGN  # the freed hole is reused first
    a.release(3 * ALIGN, 3 * ALIGN)
    a.release(x, 3 * ALIGN)
    a.release(z, ALIGN)
    assert a.free == [(0, 10 * ALIGN)] and a.used == 0  # everything coalesced back


def test_arena_random_alloc_free_never_overlaps():
    rng = np.random.Generator(np.random.PCG64(5))
    a = ArenaAllocator(200 * ALIGN)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            a.release(off, live.pop(off))
        else:
            n = int(rng.integers(1, 20 * ALIGN))
            off = a.alloc(n)
            if off is not None:
                live[off] = n
        spans = sorted((o, o + -(-n // ALIGN) * ALIGN) for o, n in live.items())
        assert all(s1[1] <= s2[0] for s1, s2 in zip(spans, spans[1:]))
        assert a.used == sum(e - s for s, e in spans)
        free = sum(ln for _, ln in a.free)
        assert free + a.used == a.size


def test_request_mix_and_arrivals_are_seeded():
    m1 = inputs.request_mix(50, [7, 8], [1, 2, 3], [2, 16], 9)
    m2 = inputs.request_mix(50, [7, 8], [1, 2, 3], [2, 16], 9)
    assert m1 == m2
    assert {q["p"] for q in m1} <= {7, 8} and {q["chi"] for q in m1} <= {2, 16}
    t = inputs.poisson_arrivals(20000, 500.0, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 500.0) < 15.0  # rate within ~3 sigma


@pytest.mark.parametrize("p", [2, 3, 7])
def test_diagonal_pairs(p):
    pr = inputs.neighbour_pairs(p, diagonal=True)
    assert len(pr) == 2 * p * (p - 1) + 2 * (p - 1) ** 2
    assert len({tuple(x) for x in pr}) == len(pr) and np.all(pr[:, 0] < pr[:, 1])
    for i, j in pr:  # grid neighbours (8-neighbourhood)
        ri, ci, rj, cj = i // p, i % p, j // p, j % p
        assert max(abs(ri - rj), abs(ci - cj)) == 1


def test_layers_that_keep_every_singular_value():
    """The exact-split policy's layer test: with chi >= 2^L every layer keeps min(rows, cols)
    singular values at every bond (so the closed-form dimensions are full rank), and a layer
    that reaches the chi cap in the middle of the chain does not."""
    from paper_2607_10280_amd import workload as w
    for n, chi, L in [(49, 16, 4), (16, 4, 2), (144, 16, 2), (256, 16, 2), (49, 128, 7)]:
        assert all(w.layer_keeps_all(n, chi, l) for l in range(L)), (n, chi, L)
    assert [w.layer_keeps_all(49, 8, l) for l in range(4)] == [True, True, True, False]
    assert [w.layer_keeps_all(49, 2, l) for l in range(3)] == [True, False, False]
    # a truncating layer's middle bond: D = chi < min(rows, cols)
    n, chi, l, k = 49, 8, 3, 20
    D = w.bond(n, chi, l + 1, k)
    assert D == 8 and min(2 * w.bond(n, chi, l + 1, k - 1), 2 * w.bond(n, chi, l, k + 1)) == 16
    # the exact paths are priced below the SVD path and read/write each tensor once
    f_mpo, f_qr, f_svd = (w.layer_flops(49, 16, 3, m) for m in ("mpo", "qr", "svd"))
    assert f_qr["svd_fp64"] == 0 and 0 < f_qr["total_fp64"] < f_svd["total_fp64"]
    assert 0 < f_mpo["total_fp64"] < f_qr["total_fp64"]
    assert w.layer_bytes(49, 16, 3, 4) == w.state_bytes(49, 16, 3, 4) + w.state_bytes(49, 16, 4, 4)


def test_exact_layer_before_truncation_priced_as_qr():
    """A layer that keeps every singular value but is followed by a truncating one is counted
    as the QR sweep (the library applies it so); the last layer of a batch and layers followed
    by exact ones keep the product-operator count."""
    from paper_2607_10280_amd import workload as w
    assert [w.next_truncates(49, 8, l, 4) for l in range(4)] == [False, False, True, False]
    assert [w.next_truncates(49, 64, l, 7) for l in range(7)] == [False] * 5 + [True, False]
    assert not any(w.next_truncates(49, 16, l, 4) for l in range(4))
    assert w.layer_flops(49, 8, 2, "mpo", n_layers=4) == w.layer_flops(49, 8, 2, "qr")
    assert w.layer_flops(49, 8, 1, "mpo", n_layers=4) == w.layer_flops(49, 8, 1, "mpo")
    assert w.layer_flops(49, 16, 3, "mpo", n_layers=4) == w.layer_flops(49, 16, 3, "mpo")


def test_product_operator_plan():
    """The site-by-site form of an exact layer applies exactly when the layer keeps every
    singular value; its reduced ends at 7x7, chi = 16 are the bonds whose rule dimension is
    the full left (2^(k+1)) or right (2^(n-k-1)) space."""
    from paper_2607_10280_amd import workload as w
    for n in range(2, 40):
        for chi in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 64, 128):
            for layer in range(8):
                assert (w.mpo_plan(n, chi, layer) is not None) == w.layer_keeps_all(n, chi, layer)
    assert [w.mpo_plan(49, 16, l) for l in range(4)] == [(-1, 48), (0, 47), (1, 46), (2, 45)]
    kl, kr = w.mpo_plan(49, 16, 3)
    assert all(w.bond(49, 16, 4, k) == 2 ** (k + 1) for k in range(kl + 1))
    assert all(w.bond(49, 16, 4, k) == 2 ** (49 - k - 1) for k in range(kr, 48))
    assert all(w.bond(49, 16, 4, k) == 2 * w.bond(49, 16, 3, k) for k in range(kl + 1, kr))
    # a short chain whose two reduced ends meet at one site
    assert w.mpo_plan(4, 16, 3) == (1, 2)
