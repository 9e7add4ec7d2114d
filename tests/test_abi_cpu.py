"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and its
host-only calls (sizes, bond-dimension rule, pair validation) behave as documented.  No
kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mps as omps
from paper_2607_10280_amd import anomps, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "anomps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mps_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(anomps.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(anomps.EXPORTS)


def test_bond_dim_rule_matches_oracle():
    x = inputs.uniform_pixels(1, 12, 3)[0]
    th, ph = inputs.layer_angles(4, 12, 4)
    for chi in (1, 2, 3, 4, 8, 16):
        m = omps.product_mps(x)
        for layer in range(4):
            omps.apply_layer(m, th[layer], ph[layer], chi)
            got = [anomps.bond_dim(12, chi, layer + 1, k) for k in range(11)]
            assert got == m.bond_dims(), (chi, layer)
    assert anomps.bond_dim(49, 16, 4, -1) == 1 and anomps.bond_dim(49, 16, 4, 48) == 1
    assert anomps.bond_dim(49, 16, 4, 49) == 0


def test_sizes():
    P = anomps.PREC_FP32
    assert anomps.slot_dim(49, 16, 4) == 16
    assert anomps.slot_dim(49, 16, 0) == 2
    assert anomps.slot_dim(256, 64, 2) == 4
    assert anomps.state_bytes(49, 16, 4, 1024, P) == 1024 * 49 * 2 * 16 * 16 * 2 * 4
    assert anomps.env_bytes(49, 16, 4, 1024, P) == 1024 * 2 * 50 * 16 * 16 * 2 * 4
    assert anomps.state_bytes(49, 16, 4, 2, anomps.PREC_FP64) == 2 * 49 * 2 * 256 * 2 * 8
    # over capacity: bond 256 is beyond this build (slots up to 128)
    assert anomps.state_bytes(49, 256, 8, 1, P) == 0
    assert "MPS_MAX_BOND" in anomps.lib().mps_last_error().decode()
    assert anomps.slot_dim(49, 128, 7) == 128 and anomps.slot_dim(16, 64, 6) == 64
    assert anomps.state_bytes(1, 4, 1, 1, P) == 0
    assert anomps.state_bytes(16, 4, 1, 1, 7) == 0


def test_wide_slot_sizes():
    """Slots beyond 16 append an FP64 workspace per image to the environment buffer: the larger of
    the layer's 12 S^2, both environment sides' 6 S^2 and four pair workgroups' 4 x 12 S^2
    complex128 elements, after the environments rounded up to 256 bytes."""
    for n, chi, L, B, P, real in [(49, 32, 5, 3, anomps.PREC_FP32, 4), (16, 64, 6, 2, anomps.PREC_FP64, 8),
                                  (49, 128, 7, 1, anomps.PREC_FP32, 4), (11, 32, 8, 5, anomps.PREC_FP32, 4)]:
        S = anomps.slot_dim(n, chi, L)
        assert S > 16
        env = B * 2 * (n + 1) * S * S * 2 * real
        env = (env + 255) // 256 * 256
        ws = -(-48 * S * S // 64) * 64 * 16
        assert anomps.env_bytes(n, chi, L, B, P) == env + B * ws
        assert anomps.state_bytes(n, chi, L, B, P) == B * n * 2 * S * S * 2 * real
    # narrow slots keep the plain environment size
    assert anomps.env_bytes(49, 16, 4, 2, anomps.PREC_FP32) == 2 * 2 * 50 * 16 * 16 * 2 * 4


def test_exact_layer_policy_arguments():
    anomps.set_exact_layers(anomps.EXACT_SVD)
    anomps.set_exact_layers(anomps.EXACT_QR)
    anomps.set_exact_layers(anomps.EXACT_MPO)
    for bad in (3, -1):
        with pytest.raises(anomps.MpsError) as e:
            anomps.set_exact_layers(bad)
        assert e.value.code == -1


def test_validate_pairs():
    anomps.validate_pairs(inputs.neighbour_pairs(7), 49)
    anomps.validate_pairs(np.zeros((0, 2), np.int32), 49)
    for bad in ([(3, 3)], [(4, 2)], [(0, 49)], [(-1, 2)]):
        with pytest.raises(anomps.MpsError) as e:
            anomps.validate_pairs(np.array(bad, np.int32), 49)
        assert e.value.code == -1
    many = np.array([(0, j) for j in range(1, 300)], np.int32)
    with pytest.raises(anomps.MpsError) as e:
        anomps.validate_pairs(many, 400)
    assert e.value.code == -2


def test_neighbour_pairs_layout():
    p = inputs.neighbour_pairs(7)
    assert p.shape == (84, 2)
    assert tuple(p[0]) == (0, 1) and tuple(p[41]) == (47, 48) and tuple(p[42]) == (0, 7)
    assert np.all(p[:42, 1] - p[:42, 0] == 1) and np.all(p[42:, 1] - p[42:, 0] == 7)
    assert inputs.neighbour_pairs(16).shape == (480, 2)


def _req(n, chi, L, prec, m=4, ptr=0x1000):
    return anomps.MpsRequest(n, chi, L, prec, m, 0, ptr, ptr, ptr, ptr, ptr, 0, ptr, ptr, ptr)


def test_plan_mixed_groups_buckets_and_orders_by_work():
    reqs = [_req(16, 4, 1, anomps.PREC_FP32), _req(49, 16, 4, anomps.PREC_FP32),
            _req(9, 2, 3, anomps.PREC_FP64), _req(36, 16, 2, anomps.PREC_FP32),
            _req(64, 16, 2, anomps.PREC_FP32), _req(49, 16, 3, anomps.PREC_FP64)]
    order, plan = anomps.plan_mixed(reqs)
    assert sorted(order) == list(range(len(reqs)))
    slot = lambda r: anomps.slot_dim(r.n_sites, r.chi, r.n_layers)
    bucket = lambda r: 4 * (r.precision == anomps.PREC_FP32) + int(np.log2(slot(r))) - 1
    seq = [bucket(reqs[i]) for i in order]
    assert seq == sorted(seq)
    assert plan.n_req == len(reqs)
    for k in range(anomps.MIXED_BUCKETS):
        members = [reqs[i] for i in order[plan.begin[k]:plan.begin[k] + plan.count[k]]]
        assert all(bucket(r) == k for r in members)
        if members:
            assert plan.max_sites[k] == max(r.n_sites for r in members)
    # within the S=4 FP32 bucket the 64-site request (more work) comes before the 36-site one
    b4 = [reqs[i].n_sites for i in order[plan.begin[5]:plan.begin[5] + plan.count[5]]]
    assert b4 == [64, 36]


def test_plan_mixed_rejects_bad_requests():
    with pytest.raises(anomps.MpsError) as e:
        anomps.plan_mixed([_req(16, 4, 1, anomps.PREC_FP32), _req(16, 4, 1, anomps.PREC_FP32, ptr=0)])
    assert e.value.code == -1 and "request 1" in str(e.value)
    with pytest.raises(anomps.MpsError) as e:
        anomps.plan_mixed([_req(16, 4, 1, anomps.PREC_SPLIT_BF16)])
    assert e.value.code == -4
    with pytest.raises(anomps.MpsError) as e:
        anomps.plan_mixed([_req(64, 32, 5, anomps.PREC_FP32)])
    assert e.value.code == -2 and "mixed-table limit" in str(e.value)
    order, plan = anomps.plan_mixed([])
    assert len(order) == 0 and plan.n_req == 0
