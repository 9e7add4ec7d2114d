"""The autotuner's launch schedules never change a result: every pair-kernel schedule (image
blocking of the launch order, cap on resident workgroups) and every mixed-table grid size gives
bit-identical features; the tuner picks one of its candidates and its JSON cache round-trips."""
import numpy as np
import pytest

from paper_2607_10280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch  # noqa: F401
    from paper_2607_10280_amd import anomps, autotune, mixed
    anomps.lib()
    return anomps, autotune, mixed


@pytest.mark.parametrize("B,prec", [(64, 1), (24, 1), (40, 0)])
def test_pair_schedules_bit_identical(A, B, prec):
    import torch
    anomps, autotune, _ = A
    p, n, L, chi = 7, 49, 4, 16
    x = inputs.blob_images(B, p, 600 + B)
    th, ph = inputs.layer_angles(L, n, 601)
    b = anomps.new_batch(n, chi, L, B, prec)
    anomps.init_batch(b, torch.as_tensor(x, device="cuda").contiguous())
    anomps.apply_layers(b, torch.as_tensor(th, device="cuda").contiguous(),
                        torch.as_tensor(ph, device="cuda").contiguous())
    pairs = torch.as_tensor(inputs.neighbour_pairs(p), device="cuda").contiguous()
    real = torch.float64 if prec == anomps.PREC_FP64 else torch.float32
    ref = None
    try:
        for cand in autotune.MEASURE_CANDIDATES + ((8, 4), (16, 0)):
            print(f"[case] B={B} prec={prec} schedule {cand}", flush=True)
            anomps.set_measure_tuning(*cand)
            out = torch.full((B, pairs.shape[0], 15), float("nan"), dtype=real, device="cuda")
            anomps.pauli_pair_expect(b, pairs, out)
            got = out.cpu().numpy()
            assert np.all(np.isfinite(got))
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), cand
    finally:
        anomps.set_measure_tuning(*anomps.DEFAULT_MEASURE_SCHEDULE)
    with pytest.raises(anomps.MpsError):
        anomps.set_measure_tuning(-8, 0)
    with pytest.raises(anomps.MpsError):
        anomps.set_measure_tuning(0, 2)


def test_tune_measure_and_cache(A, tmp_path):
    anomps, autotune, _ = A
    try:
        choice, ms, timings = autotune.tune_measure(49, 16, 4, 64, anomps.PREC_FP32,
                                                    candidates=((0, 0), (32, 0), (32, 12)),
                                                    repeats=1)
        assert choice in timings and ms == min(timings.values()) and ms > 0
        path = str(tmp_path / "tune.json")
        key = autotune.measure_key(49, 16, 4, 64, anomps.PREC_FP32)
        autotune.save_measure(key, choice, path)
        autotune.save({3: (2, 1.0, {})}, path)  # the mixed choices share the file
        assert autotune.load_measure(key, path) == tuple(choice)
        assert autotune.load_and_apply(path) == {3: 2}
        assert autotune.load_measure("measure/none", path) is None
    finally:
        anomps.set_measure_tuning(*anomps.DEFAULT_MEASURE_SCHEDULE)
        anomps.set_mixed_tuning(3, 0)


def test_mixed_grid_sizes_bit_identical(A):
    import torch
    anomps, autotune, mixed = A
    cases = [(6, 2, 16), (4, 3, 8), (7, 1, 16), (5, 2, 4), (8, 2, 16), (3, 2, 2)]
    specs = []
    for r, (p, L, chi) in enumerate(cases):
        n = p * p
        x = inputs.blob_images(1, p, 700 + r)[0]
        th, ph = inputs.layer_angles(L, n, 710 + r)
        specs.append(mixed.RequestSpec(x, th, ph, inputs.neighbour_pairs(p), chi, anomps.PREC_FP32))
    mr = mixed.MixedRequests(specs)
    ref = None
    try:
        for per_cu in (1, 2, 4, 0):
            for bucket in range(anomps.MIXED_BUCKETS):
                anomps.set_mixed_tuning(bucket, per_cu)
            mr.bytes.zero_()
            mr.run()
            torch.cuda.synchronize()
            got = mr.outputs()
            if ref is None:
                ref = got
            for r in range(len(specs)):
                assert np.array_equal(got[r], ref[r]), (per_cu, r)
    finally:
        for bucket in range(anomps.MIXED_BUCKETS):
            anomps.set_mixed_tuning(bucket, 0)
