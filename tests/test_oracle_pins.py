"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Nothing here compares the oracle with itself: each test checks it against hand-derived
values (tests/golden), closed forms, an independent brute-force path, invariants, or the
truncation bound.  The mutation tests at the end plant plausible mistakes in the oracle
(on the CPU) and check that at least one pin catches each of them.
"""
import numpy as np
import pytest

from oracle import bruteforce, closed_form, features, gates, mps, readout, statevector
from paper_2607_10280_amd import inputs
from tests.golden_cases import hand_derived_cases

CASES = hand_derived_cases()


def all_pairs(n):
    return np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int32)


# ---------------------------------------------------------------- hand-derived values
@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_derived_statevector(case):
    got = statevector.features(case["x"], case["theta"], case["phi"], case["pairs"])
    np.testing.assert_allclose(got, case["expect"], atol=1e-14)


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_derived_mps(case):
    for chi in (None, 2, 4):
        got, _ = mps.features(case["x"], case["theta"], case["phi"], case["pairs"], chi)
        np.testing.assert_allclose(got, case["expect"], atol=1e-13)


def test_ghz_degenerate_spectrum():
    case = next(c for c in CASES if c["name"] == "ghz5")
    m = mps.simulate(case["x"], case["theta"], case["phi"], chi=None)
    for s in m.spectra[0]:
        np.testing.assert_allclose(s[:2], [2 ** -0.5, 2 ** -0.5], atol=1e-14)
        assert np.all(s[2:] < 1e-15)


# ---------------------------------------------------------------- brute force (P6)
@pytest.mark.parametrize("n,L,seed", [(2, 1, 0), (3, 2, 1), (5, 3, 2), (6, 2, 3), (7, 1, 4)])
def test_statevector_vs_bruteforce(n, L, seed):
    x = inputs.uniform_pixels(1, n, seed)[0]
    th, ph = inputs.layer_angles(L, n, seed + 100)
    pairs = all_pairs(n)
    np.testing.assert_allclose(statevector.features(x, th, ph, pairs),
                               bruteforce.features(x, th, ph, pairs), atol=1e-13)


# ---------------------------------------------------------------- closed forms (P1, P2)
@pytest.mark.parametrize("p", [2, 4, 7, 16])
def test_l0_closed_form(p):
    n = p * p
    x = inputs.uniform_pixels(1, n, 11)[0]
    pairs = inputs.neighbour_pairs(p)
    empty = np.zeros((0, n))
    ref = closed_form.l0_features(x, pairs)
    if n <= 16:
        np.testing.assert_allclose(statevector.features(x, empty, empty, pairs), ref, atol=1e-14)
    got, _ = mps.features(x, empty, empty, pairs, chi=None)
    np.testing.assert_allclose(got, ref, atol=1e-14)
    # <Z_i> = cos(pi x_i): the (Z, I) feature of every horizontal pair.
    np.testing.assert_allclose(ref[: p * (p - 1), 11], np.cos(np.pi * x[pairs[: p * (p - 1), 0]]),
                               atol=1e-15)


@pytest.mark.parametrize("n", [2, 5, 9, 16])
def test_l1_closed_form_vs_statevector(n):
    x = inputs.uniform_pixels(1, n, 21)[0]
    th, ph = inputs.layer_angles(1, n, 22)
    pairs = all_pairs(n)
    np.testing.assert_allclose(closed_form.l1_features(x, th, ph, pairs),
                               statevector.features(x, th, ph, pairs), atol=1e-13)


@pytest.mark.parametrize("p", [7, 16])
def test_l1_closed_form_vs_mps(p):
    n = p * p
    x = inputs.blob_images(1, p, 31)[0]
    th, ph = inputs.layer_angles(1, n, 32)
    pairs = inputs.neighbour_pairs(p)
    got, m = mps.features(x, th, ph, pairs, chi=None)
    assert max(m.bond_dims()) == 2
    np.testing.assert_allclose(got, closed_form.l1_features(x, th, ph, pairs), atol=1e-12)


# ---------------------------------------------------------------- MPS vs statevector
@pytest.mark.parametrize("n,L", [(4, 1), (9, 2), (12, 3), (16, 4)])
def test_mps_untruncated_vs_statevector(n, L):
    x = inputs.uniform_pixels(1, n, 41)[0]
    th, ph = inputs.layer_angles(L, n, 42)
    pairs = all_pairs(n) if n <= 9 else inputs.neighbour_pairs(int(round(n ** 0.5))) \
        if int(round(n ** 0.5)) ** 2 == n else all_pairs(n)[:60]
    ref = statevector.features(x, th, ph, pairs)
    got, m = mps.features(x, th, ph, pairs, chi=None)
    np.testing.assert_allclose(got, ref, atol=1e-12)
    assert max(m.bond_dims()) <= 2 ** L


# ---------------------------------------------------------------- exactness threshold (P7)
@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_exact_at_chi_2_pow_L(L):
    p, n = 4, 16
    x = inputs.uniform_pixels(1, n, 51)[0]
    th, ph = inputs.layer_angles(L, n, 52 + L)
    pairs = inputs.neighbour_pairs(p)
    ref = statevector.features(x, th, ph, pairs)
    got, m = mps.features(x, th, ph, pairs, chi=2 ** L)
    np.testing.assert_allclose(got, ref, atol=1e-12)
    assert np.max(np.array(m.trunc_err)) < 1e-24
    if L >= 2:
        _, m_small = mps.features(x, th, ph, pairs, chi=2 ** (L - 1))
        assert np.max(np.array(m_small.trunc_err)) > 1e-6


def test_bond_dims_rule():
    """Bond dimension after layer l: min(chi, 2^l, 2^{k+1}, 2^{n-k-1})."""
    n = 16
    x = inputs.uniform_pixels(1, n, 61)[0]
    th, ph = inputs.layer_angles(4, n, 62)
    for chi in (2, 4, 8, 16, 32):
        m = mps.product_mps(x)
        for layer in range(4):
            mps.apply_layer(m, th[layer], ph[layer], chi)
            want = [min(chi, 2 ** (layer + 1), 2 ** (k + 1), 2 ** (n - k - 1)) for k in range(n - 1)]
            assert m.bond_dims() == want


# ---------------------------------------------------------------- truncation bound (P5)
@pytest.mark.parametrize("chi", [2, 4, 8])
def test_truncation_bound(chi):
    n, L = 16, 4
    x = inputs.uniform_pixels(1, n, 71)[0]
    th, ph = inputs.layer_angles(L, n, 72)
    pairs = inputs.neighbour_pairs(4)
    exact_psi = statevector.simulate(x, th, ph)
    got, m = mps.features(x, th, ph, pairs, chi)
    eps = np.array(m.trunc_err)
    dist_bound = np.sum(np.sqrt(2 * eps))
    approx_psi = mps.to_statevector(m)
    dist = np.linalg.norm((approx_psi * np.exp(-1j * np.angle(np.vdot(approx_psi, exact_psi))) -
                           exact_psi).ravel())
    assert dist <= dist_bound + 1e-12
    err = np.abs(got - statevector.pauli_pair_features(exact_psi, pairs)).max()
    assert err <= 2 * dist_bound + 1e-12
    assert err > 1e-8   # genuinely truncated


def test_single_truncation_equals_fidelity_loss():
    """n=4, L=2, chi=2: only the middle bond of the second layer is truncated (4 -> 2), at the
    orthogonality centre, so its discarded weight equals 1 - |<psi|psi_t>|^2."""
    n = 4
    x = inputs.uniform_pixels(1, n, 81)[0]
    th, ph = inputs.layer_angles(2, n, 82)
    m = mps.simulate(x, th, ph, chi=2)
    eps = np.array(m.trunc_err)
    assert np.count_nonzero(eps > 1e-20) == 1 and eps[1, 1] > 1e-6
    exact = statevector.simulate(x, th, ph).ravel()
    approx = mps.to_statevector(m).ravel()
    np.testing.assert_allclose(1.0 - abs(np.vdot(exact, approx)) ** 2, eps[1, 1], rtol=1e-9)


# ---------------------------------------------------------------- invariants (P4)
def _rho_from_features(f):
    rho = 0.25 * np.kron(gates.I2, gates.I2)
    for alpha in range(15):
        rho = rho + 0.25 * f[alpha] * gates.pair_pauli(alpha)
    return rho


@pytest.mark.parametrize("chi", [None, 2, 8])
def test_invariants(chi):
    p, n, L = 5, 25, 3
    x = inputs.blob_images(1, p, 91)[0]
    th, ph = inputs.layer_angles(L, n, 92)
    pairs = inputs.neighbour_pairs(p)
    f, m = mps.features(x, th, ph, pairs, chi)
    assert np.all(np.abs(f) <= 1 + 1e-12)
    assert np.all(np.sum(f ** 2, axis=1) <= 3 + 1e-10)
    for q in range(len(pairs)):
        rho = _rho_from_features(f[q])
        assert np.allclose(rho, rho.conj().T)
        assert abs(np.trace(rho) - 1) < 1e-14
        assert np.linalg.eigvalsh(rho).min() > -1e-12
    # Single-site marginals <P_a (x) I> agree across all pairs sharing the lower site.
    marg = {}
    for q, (i, j) in enumerate(pairs):
        for site, vals in ((i, f[q, [3, 7, 11]]), (j, f[q, [0, 1, 2]])):
            marg.setdefault(int(site), []).append(vals)
    for vals in marg.values():
        assert np.ptp(np.array(vals), axis=0).max() < 1e-12
    assert abs(mps.norm2(m) - 1) < 1e-12
    for layer in m.spectra:   # singular values non-negative and sorted
        for s in layer:
            assert np.all(s >= 0) and np.all(np.diff(s) <= 0)
    rdm = mps.right_envs(m.tensors)
    assert abs(rdm[0][0, 0] - 1) < 1e-12


def test_canonical_forms():
    n = 12
    x = inputs.uniform_pixels(1, n, 101)[0]
    th, ph = inputs.layer_angles(3, n, 102)
    m = mps.simulate(x, th[:2], ph[:2], chi=None)
    mps.canonicalise_right(m, th[2], ph[2])
    for k in range(1, n):   # right-canonical: sum_s A^s A^{s dag} = I
        t = m.tensors[k]
        g = np.einsum("asb,csb->ac", t, t.conj())
        np.testing.assert_allclose(g, np.eye(t.shape[0]), atol=1e-13)
    mps.cnot_ladder(m, chi=None)
    for k in range(n - 1):  # left-canonical after the ladder: sum_s A^{s dag} A^s = I
        t = m.tensors[k]
        g = np.einsum("asb,asc->bc", t.conj(), t)
        np.testing.assert_allclose(g, np.eye(t.shape[2]), atol=1e-13)


# ---------------------------------------------------------------- readout (P8)
def test_readout_identity():
    """Sum_alpha c_alpha <P_alpha> = Tr(rho_ij H_q), rho from the statevector (Eq. (4)-(5))."""
    p, n = 3, 9
    x = inputs.uniform_pixels(1, n, 111)[0]
    th, ph = inputs.layer_angles(2, n, 112)
    pairs = inputs.neighbour_pairs(p)
    a, b, d, w, bias = inputs.readout_params(len(pairs), 7, 113)
    psi = statevector.simulate(x, th, ph)
    pauli = statevector.pauli_pair_features(psi, pairs)[None]
    coeff = readout.coefficients(a, b, d)
    q = readout.features_from_paulis(coeff, pauli)[0]
    for idx, (i, j) in enumerate(pairs):
        h = readout.hermitian(a[idx], b[idx], d[idx])
        assert np.allclose(h, h.conj().T)
        np.testing.assert_allclose(q[idx], np.trace(statevector.pair_rdm(psi, i, j) @ h).real,
                                   atol=1e-13)
    y = readout.readout(pauli, a, b, d, w, bias + 0.5)
    np.testing.assert_allclose(y[0], w @ q + 0.5, atol=1e-14)
    # Diagonal-only observable: c_II = mean(D), c_ZZ = (D0 - D1 - D2 + D3)/4.
    cd = readout.coefficients(np.zeros((1, 6)), np.zeros((1, 6)), np.array([[1.0, 2.0, 3.0, 4.0]]))
    assert abs(cd[0, 0] - 2.5) < 1e-15 and abs(cd[0, 15] - 0.0) < 1e-15
    assert abs(cd[0, 3] - (1 - 2 + 3 - 4) / 4) < 1e-15 and abs(cd[0, 12] - (1 + 2 - 3 - 4) / 4) < 1e-15


def test_exact_features_front_door():
    p = 4
    x = inputs.uniform_pixels(3, p * p, 121)
    th, ph = inputs.layer_angles(2, p * p, 122)
    pairs = inputs.neighbour_pairs(p)
    ex = features.exact_features(x, th, ph, pairs)
    tr, err, gaps = features.truncated_features(x, th, ph, pairs, chi=4)
    assert ex.shape == (3, 24, 15) and err.shape == (3, 2, 15)
    np.testing.assert_allclose(ex, tr, atol=1e-12)


# ---------------------------------------------------------------- planted mistakes
def _golden_error(fn):
    return max(np.abs(fn(c) - c["expect"]).max() for c in CASES)


def test_mutation_gate_order(monkeypatch):
    monkeypatch.setattr(gates, "layer_gate", lambda t, p: gates.rz(p) @ gates.ry(t))
    err = _golden_error(lambda c: statevector.features(c["x"], c["theta"], c["phi"], c["pairs"]))
    assert err > 0.5


def test_mutation_y_sign(monkeypatch):
    monkeypatch.setattr(gates, "PAULI", (gates.I2, gates.X, -gates.Y, gates.Z))
    err = _golden_error(lambda c: statevector.features(c["x"], c["theta"], c["phi"], c["pairs"]))
    assert err > 0.5


def test_mutation_pauli_site_order(monkeypatch):
    def swapped(alpha):
        a, b = divmod(alpha + 1, 4)
        return np.kron(gates.PAULI[b], gates.PAULI[a])
    monkeypatch.setattr(gates, "pair_pauli", swapped)
    err = _golden_error(lambda c: statevector.features(c["x"], c["theta"], c["phi"], c["pairs"]))
    assert err > 0.5


def test_mutation_rz_sign(monkeypatch):
    monkeypatch.setattr(gates, "rz", lambda t: np.diag([np.exp(0.5j * t), np.exp(-0.5j * t)]))
    err = _golden_error(lambda c: statevector.features(c["x"], c["theta"], c["phi"], c["pairs"]))
    assert err > 0.5


def test_mutation_statevector_cnot_direction(monkeypatch):
    orig = statevector._apply_cnot
    monkeypatch.setattr(statevector, "_apply_cnot", lambda psi, c, t: orig(psi, t, c))
    n = 5
    x = inputs.uniform_pixels(1, n, 131)[0]
    th, ph = inputs.layer_angles(2, n, 132)
    pairs = all_pairs(n)
    err = np.abs(statevector.features(x, th, ph, pairs) - bruteforce.features(x, th, ph, pairs)).max()
    assert err > 1e-2


def _mps_vs_sv_error():
    n = 9
    x = inputs.uniform_pixels(1, n, 141)[0]
    th, ph = inputs.layer_angles(2, n, 142)
    pairs = all_pairs(n)
    got, _ = mps.features(x, th, ph, pairs, chi=None)
    return np.abs(got - statevector.features(x, th, ph, pairs)).max()


def test_mutation_mps_cnot_on_wrong_branch(monkeypatch):
    def wrong(theta2):
        g = theta2.copy()
        g[:, 0, :, :] = theta2[:, 0, ::-1, :]
        return g
    monkeypatch.setattr(mps, "cnot_two_site", wrong)
    assert _mps_vs_sv_error() > 1e-2


def test_mutation_mps_missing_conjugate(monkeypatch):
    def bad_left(a):
        envs = [np.ones((1, 1), dtype=np.complex128)]
        for t in a:
            envs.append(np.einsum("ab,asc,bsd->cd", envs[-1], t, t))
        return envs
    monkeypatch.setattr(mps, "left_envs", bad_left)
    assert _mps_vs_sv_error() > 1e-2


def test_mutation_no_renormalisation(monkeypatch):
    orig = mps.truncate

    def no_renorm(s, chi):
        d, err, gap, kept = orig(s, chi)
        return d, err, gap, s[:d]
    monkeypatch.setattr(mps, "truncate", no_renorm)
    n = 16
    x = inputs.uniform_pixels(1, n, 151)[0]
    th, ph = inputs.layer_angles(3, n, 152)
    m = mps.simulate(x, th, ph, chi=2)
    assert abs(mps.norm2(m) - 1) > 1e-3


def test_mutation_ladder_order(monkeypatch):
    """Reversing the ladder order (CNOT(n-2,n-1) first) breaks the two-layer GHZ case."""
    def reversed_ladder(psi, theta, phi):
        n = psi.ndim
        for k in range(n):
            psi = statevector._apply_1q(psi, gates.layer_gate(theta[k], phi[k]), k)
        for k in range(n - 2, -1, -1):
            psi = statevector._apply_cnot(psi, k, k + 1)
        return psi
    monkeypatch.setattr(statevector, "apply_layer", reversed_ladder)
    err = _golden_error(lambda c: statevector.features(c["x"], c["theta"], c["phi"], c["pairs"]))
    assert err > 0.5
