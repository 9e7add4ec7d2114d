"""Pins of the oracle's version of the paper's own encoding circuit (§II-B, Eq. (2)): three
independent simulations agree, hand-derived special inputs give the values worked out below,
the MPS obeys the bond-dimension rule and the truncation bound, and planted mistakes are
caught.  CPU only."""
import numpy as np
import pytest

from oracle import paper_ansatz as pa
from paper_2607_10280_amd import inputs

ALL_PAIRS = lambda n: np.array([[i, j] for i in range(n) for j in range(i + 1, n)], dtype=np.int32)
# alpha = 4a + b - 1 with P_a on the lower site i, P_b on j
A_XI, A_ZI, A_IX, A_IZ, A_XX, A_ZZ = 3, 11, 0, 2, 4, 14


def single_site(feats, pairs, n, a_lower, a_upper):
    """<P_k> for every site k, read from the pair features (k as lower or upper site)."""
    out = np.zeros(n)
    for q, (i, j) in enumerate(pairs):
        out[i] = feats[q, a_lower]
        out[j] = feats[q, a_upper]
    return out


@pytest.mark.parametrize("n,L,seed", [(2, 1, 0), (3, 2, 1), (5, 3, 2), (6, 1, 3), (7, 2, 4)])
def test_statevector_vs_bruteforce(n, L, seed):
    x = inputs.uniform_pixels(1, n, 900 + seed)[0]
    pairs = ALL_PAIRS(n)
    assert np.abs(pa.sv_features(x, L, pairs) - pa.bf_features(x, L, pairs)).max() < 1e-13


@pytest.mark.parametrize("n,L", [(4, 1), (9, 2), (12, 3), (16, 2)])
def test_mps_vs_statevector(n, L):
    x = inputs.uniform_pixels(1, n, 910 + n)[0]
    pairs = inputs.neighbour_pairs(int(round(np.sqrt(n))), True) if int(np.sqrt(n)) ** 2 == n else ALL_PAIRS(n)
    assert np.abs(pa.mps_features(x, L, pairs) - pa.sv_features(x, L, pairs)).max() < 1e-12


# x = 0 gives phi = -pi (Eq. (2)); R_Y(-pi) H |0> = R_Y(-pi)|+> = |->.  A CNOT whose target is |->
# flips its control between |+> and |-> (phase kick-back); a target |+> changes nothing.
# n = 5, L = 1: even bonds (0,1), (2,3) turn sites 0 and 2 into |+>; odd bonds (1,2) (target
# |+>, nothing) and (3,4) (target |->, site 3 -> |+>).  Result |+ - + + ->, so <X_k> below.
# n = 4: (0,1), (2,3) then (1,2) with target |+>: |+ - + ->.
@pytest.mark.parametrize("n,expect_x", [(4, [1, -1, 1, -1]), (5, [1, -1, 1, 1, -1])])
def test_zero_image_one_layer(n, expect_x):
    pairs = ALL_PAIRS(n)
    f = pa.sv_features(np.zeros(n), 1, pairs)
    np.testing.assert_allclose(single_site(f, pairs, n, A_XI, A_IX), expect_x, atol=1e-12)
    np.testing.assert_allclose(single_site(f, pairs, n, A_ZI, A_IZ), 0.0, atol=1e-12)
    for q, (i, j) in enumerate(pairs):  # product state: pair values factorise
        assert abs(f[q, A_XX] - expect_x[i] * expect_x[j]) < 1e-12


# Second layer from |+ - + + ->: H gives |0 1 0 0 1>, R_Y(-pi) maps |0> -> -|1>, |1> -> |0>:
# bits 1 0 1 1 0; even CNOTs: b1 ^= b0 -> 1, b3 ^= b2 -> 0; odd: b2 ^= b1 -> 0, b4 ^= b3 -> 0.
# Basis state |1 1 0 0 0>: <Z_k> = (-1)^b_k.
def test_zero_image_two_layers():
    n = 5
    pairs = ALL_PAIRS(n)
    f = pa.sv_features(np.zeros(n), 2, pairs)
    np.testing.assert_allclose(single_site(f, pairs, n, A_ZI, A_IZ), [-1, -1, 1, 1, 1], atol=1e-12)
    np.testing.assert_allclose(single_site(f, pairs, n, A_XI, A_IX), 0.0, atol=1e-12)


# x = 3/4 gives phi = pi/2 and R_Y(pi/2)|+> = |1> (H first, then R_Y; the other order would give
# |0>).  Bits 1 1 1 1 1; even CNOTs: b1 -> 0, b3 -> 0; odd: b2 ^= b1 (0), b4 ^= b3 (0).  |1 0 1 0 1>.
def test_three_quarter_image_one_layer():
    n = 5
    pairs = ALL_PAIRS(n)
    f = pa.sv_features(np.full(n, 0.75), 1, pairs)
    np.testing.assert_allclose(single_site(f, pairs, n, A_ZI, A_IZ), [-1, 1, -1, 1, -1], atol=1e-12)


# x = 1/2 gives phi = 0: the layer is H followed by CNOTs.  |+...+> is left alone by every CNOT;
# H maps it back to |0...0>, also left alone.  Odd L: <X_k> = 1; even L: <Z_k> = 1.
@pytest.mark.parametrize("L", [1, 2, 3])
def test_half_image(L):
    n = 6
    pairs = ALL_PAIRS(n)
    f = pa.mps_features(np.full(n, 0.5), L, pairs)
    a = (A_XI, A_IX) if L % 2 else (A_ZI, A_IZ)
    np.testing.assert_allclose(single_site(f, pairs, n, *a), 1.0, atol=1e-12)


def test_bond_dimension_rule():
    """With chi given, the truncated MPS keeps min(chi, 2^l, 2^(k+1), 2^(n-k-1)) after l layers
    (the same closed form as the CNOT ladder) on generic inputs."""
    n = 12
    x = inputs.uniform_pixels(1, n, 920)[0]
    for chi in (3, 4, 8):
        for L in (1, 2, 3, 4):
            m = pa.mps_simulate(x, L, chi)
            expect = [min(chi, 2 ** L, 2 ** (k + 1), 2 ** (n - k - 1)) for k in range(n - 1)]
            assert m.bond_dims() == expect, (chi, L)


@pytest.mark.parametrize("chi", [2, 4])
def test_truncation_bound(chi):
    n, L = 16, 3
    x = inputs.blob_images(1, 4, 930)[0]
    pairs = inputs.neighbour_pairs(4, True)
    m = pa.mps_simulate(x, L, chi)
    from oracle import mps as omps
    got = omps.pauli_pair_features(m, pairs)
    exact = pa.sv_features(x, L, pairs)
    bound = 2.0 * np.sum(np.sqrt(2.0 * np.concatenate(m.trunc_err)))
    assert np.concatenate(m.trunc_err).max() > 0
    assert np.abs(got - exact).max() <= bound + 1e-12


# ------------------------------------------------------------------ planted mistakes
def test_mutation_angle_offset(monkeypatch):
    monkeypatch.setattr(pa, "angle", lambda x: 2.0 * np.pi * np.asarray(x, dtype=np.float64))
    with pytest.raises(AssertionError):
        test_zero_image_one_layer(5, [1, -1, 1, 1, -1])


def test_mutation_ladder_instead_of_brickwork(monkeypatch):
    monkeypatch.setattr(pa, "bonds", lambda n, parity: range(0, n - 1) if parity == 0 else range(0))
    with pytest.raises(AssertionError):
        test_zero_image_one_layer(5, [1, -1, 1, 1, -1])


def test_mutation_missing_hadamard(monkeypatch):
    monkeypatch.setattr(pa, "H", np.eye(2, dtype=np.complex128))
    with pytest.raises(AssertionError):
        test_three_quarter_image_one_layer()
