"""Algorithmic work model of the feature-extraction path (flops and HBM bytes per image).

These are the counts a roofline is priced with: the operations the method needs at the bond
dimensions it actually uses, not what a particular kernel executes.

* A complex multiply-add (cMAC) is 8 real flops.
* SVD of an m x n complex matrix (m >= n; singular values, thin U and V) is priced with the
  R-SVD count of Golub & Van Loan (6 m n^2 + 20 n^3 real flops) times 4 for complex
  arithmetic; a one-sided Jacobi SVD typically executes 1.5-3x this many flops.
* Bond dimensions follow the rule D_k = min(chi, 2^layers, 2^(k+1), 2^(n-k-1)).
"""
from __future__ import annotations

CMAC = 8


def bond(n: int, chi: int, layers: int, k: int) -> int:
    if k < 0 or k >= n - 1:
        return 1
    return min(chi, 2 ** layers, 2 ** (k + 1), 2 ** (n - k - 1))


def svd_flops(m: int, n: int) -> float:
    if m < n:
        m, n = n, m
    return 4.0 * (6.0 * m * n * n + 20.0 * n ** 3)


def layer_keeps_all(n: int, chi: int, layer: int) -> bool:
    """True when every bond of the layer keeps all min(rows, cols) singular values."""
    return all(bond(n, chi, layer + 1, k) == min(2 * bond(n, chi, layer + 1, k - 1),
                                                 2 * bond(n, chi, layer, k + 1))
               for k in range(n - 1))


def mpo_plan(n: int, chi: int, layer: int):
    """Chain ends of a layer applied as the parity product operator: bonds 0..kl are reduced
    from the left (D_k = 2 D_{k-1} < 2 D_k^old), bonds kr..n-2 from the right
    (D_k = 2 D_{k+1} < 2 D_k^old), every bond between keeps D_k = 2 D_k^old.  None when the bond
    rule has another shape (exactly when the layer does not keep every singular value)."""
    do = lambda k: bond(n, chi, layer, k)
    dn = lambda k: bond(n, chi, layer + 1, k)
    kl = -1
    while kl + 1 <= n - 2 and dn(kl + 1) < 2 * do(kl + 1) and dn(kl + 1) == 2 * dn(kl):
        kl += 1
    kr = n - 1
    while kr - 1 > kl and dn(kr - 1) < 2 * do(kr - 1) and dn(kr - 1) == 2 * dn(kr):
        kr -= 1
    if any(dn(k) != 2 * do(k) for k in range(kl + 1, kr)):
        return None
    return kl, kr


def next_truncates(n: int, chi: int, layer: int, n_layers: int) -> bool:
    """True when layer `layer` + 1 exists and truncates.  The library then applies layer
    `layer` by the QR sweep even in mode "mpo" (the canonical gauge it leaves lets the
    truncating layer's Jacobi SVDs converge in fewer sweeps)."""
    return layer + 1 < n_layers and not layer_keeps_all(n, chi, layer + 1)


def householder_qr_flops(m: int, n: int) -> float:
    """Complex Householder QR of an m x n matrix (m >= n) with Q formed explicitly: each
    reflector costs a dot product and an update over the remaining columns and rows, once to
    reduce and once to form Q."""
    return CMAC * 4.0 * sum((n - j) * (m - j) for j in range(n))


def layer_flops(n: int, chi: int, layer: int, mode: str = "mpo", n_layers: int | None = None) -> dict:
    """Work of applying layer `layer` (0-based) to one image.  mode "mpo" (a layer that keeps
    every singular value, applied as the parity product operator): the gate on every old
    tensor, the left and right carries over the reduced chain ends and their product into the
    first full sites.  mode "qr" (such a layer in one sweep): gate the neighbour, then split
    each bond exactly -- through two Householder blocks of the centre when D = 2 D_old (no
    two-site matrix), else contract Theta' and split it by Householder QR (or not at all when D
    equals its row count).  Otherwise, and for mode "svd": canonical sweep (gate + LQ of each
    site's D_{k-1} x 2D_k matrix -- it needs only orthonormal rows, priced as Householder QR of
    the conjugate transpose with Q formed -- + absorbing L into the left neighbour), then the
    ladder (two-site contraction, SVD, U^H Theta' for the new centre).  With n_layers given,
    mode "mpo" counts a layer followed by a truncating one as mode "qr", as the library runs
    it."""
    if mode == "mpo" and n_layers is not None and next_truncates(n, chi, layer, n_layers):
        mode = "qr"
    d_old = lambda k: bond(n, chi, layer, k)
    d_new = lambda k: bond(n, chi, layer + 1, k)
    plan = mpo_plan(n, chi, layer) if mode == "mpo" else None
    if plan is not None:
        kl, kr = plan
        lm = lambda k: 1 if k == 0 else 2 * d_old(k - 1)
        gate = sum(CMAC * 4 * d_old(k - 1) * d_old(k) for k in range(n))
        carry = 0.0
        for k in range(kl + 1):          # C_k = C_{k-1} B[k] (one parity block per row)
            carry += CMAC * d_new(k) * d_old(k) * lm(k)
        for k in range(n - 1, kr, -1):   # R_k = B[k] R_{k+1}
            carry += CMAC * lm(k) * 2 * d_new(k) * d_old(k)
        carry += CMAC * d_new(kl) * 2 * d_old(kl + 1) * lm(kl + 1)   # C B at site kl+1
        carry += CMAC * d_new(kr - 1) * 2 * d_new(kr) * d_old(kr)    # (C) B R at site kr
        return {"qr_fp64": 0.0, "svd_fp64": 0.0, "other_fp64": gate + carry,
                "total_fp64": gate + carry}
    if mode in ("mpo", "qr") and layer_keeps_all(n, chi, layer):
        qr = other = 0.0
        other += CMAC * 4 * d_old(0)
        for k in range(n - 1):
            dl, dc, dr, d = d_new(k - 1), d_old(k), d_old(k + 1), d_new(k)
            rows, cols = 2 * dl, 2 * dr
            other += CMAC * 4 * dc * dr                      # gate on site k+1
            if d == 2 * dc and dl >= dc:
                # two Householder blocks of the centre (Dl x Dc each), then the centre
                # R (triangular) times the gated neighbour
                qr += 2 * householder_qr_flops(dl, dc)
                other += CMAC * d * cols * (dc + 1) / 2
            else:
                other += CMAC * rows * cols * dc             # two-site matrix
                if d != rows:
                    qr += householder_qr_flops(rows, cols)
        return {"qr_fp64": qr, "svd_fp64": 0.0, "other_fp64": other, "total_fp64": qr + other}
    svd = qr = other = 0.0
    for k in range(n - 1, 0, -1):
        # orthonormal rows of site k (D_{k-1} x 2 D_k): the LQ factorisation it needs, i.e.
        # Householder QR of its conjugate transpose with Q formed; L into site k-1
        dl, dr = d_old(k - 1), d_old(k)
        qr += householder_qr_flops(2 * dr, dl)
        other += CMAC * (4 * dl * dr + 2 * d_old(k - 2) * dl * dl)
    other += CMAC * 4 * d_old(0)
    for k in range(n - 1):
        dl, dc, dr, d = d_new(k - 1), d_old(k), d_old(k + 1), d_new(k)
        svd += svd_flops(2 * dl, 2 * dr)
        other += CMAC * (2 * dl * dc * 2 * dr + 2 * d * dl * dc + d * 2 * dr * 2 * dc)
    return {"qr_fp64": qr, "svd_fp64": svd, "other_fp64": other, "total_fp64": svd + qr + other}


def env_flops(n: int, chi: int, layers: int) -> float:
    d = lambda k: bond(n, chi, layers, k)
    total = 0
    for k in range(n):
        dl, dr = d(k - 1), d(k)
        total += 2 * dl * dr * dl + dr * dr * 2 * dl   # left sweep
        total += 2 * dr * dl * dr + dl * dl * 2 * dr   # right sweep
    return CMAC * float(total)


def pair_flops(n: int, chi: int, layers: int, pairs) -> float:
    """Open at i, carry through i+1..j-1 (shared by all partners of i), close at each j.  Only
    the blocks F^00 and F^01 of the open index are carried: F^11 = L_j - F^00 at the close,
    since the two diagonal blocks sum to the left environment."""
    d = lambda k: bond(n, chi, layers, k)
    by_start: dict = {}
    for i, j in pairs:
        by_start.setdefault(int(i), []).append(int(j))
    total = 0
    for i, js in by_start.items():
        dl, dc = d(i - 1), d(i)
        total += 2 * dl * dc * dl + 2 * dc * dc * dl
        for k in range(i + 1, max(js)):
            a, b = d(k - 1), d(k)
            total += 4 * a * b * a + 2 * b * b * 2 * a
        for j in js:
            dd, dj = d(j - 1), d(j)
            total += 2 * dj * dd * dj + 3 * dd * dd * dj + 16 * dd * dd
    return CMAC * float(total)


def state_bytes(n: int, chi: int, layers: int, real_bytes: int) -> int:
    """Bytes of one image's site tensors at the given number of layers (used corners only)."""
    return sum(bond(n, chi, layers, k - 1) * 2 * bond(n, chi, layers, k) * 2 * real_bytes
               for k in range(n))


def layer_bytes(n: int, chi: int, layer: int, real_bytes: int, mode: str = "mpo") -> int:
    """HBM traffic of one layer for one image: the canonical sweep reads and writes every
    tensor once, the ladder reads and writes every tensor once; a layer that keeps every
    singular value (modes "mpo" and "qr") reads the old tensors once and writes the new ones
    once."""
    if mode in ("mpo", "qr") and layer_keeps_all(n, chi, layer):
        return state_bytes(n, chi, layer, real_bytes) + state_bytes(n, chi, layer + 1, real_bytes)
    return 2 * state_bytes(n, chi, layer, real_bytes) + 2 * state_bytes(n, chi, layer + 1, real_bytes)
