"""Mixed request tables (persistent per-bucket launches) on the GPU: every request's result
equals the same image run alone through the batch calls (bit for bit: the same device code),
matches the oracle within the batch tolerances, and a HIP-graph replay of the whole sequence
reproduces the eager result."""
import numpy as np
import pytest

from oracle import features as ofeat
from paper_2607_10280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch  # noqa: F401
    from paper_2607_10280_amd import anomps, mixed
    anomps.lib()
    return anomps, mixed


def make_specs(mixed, anomps, cases, seed):
    """cases: list of (p, L, chi, precision)."""
    specs = []
    for r, (p, L, chi, prec) in enumerate(cases):
        n = p * p
        x = inputs.blob_images(1, p, seed + 17 * r)[0]
        th, ph = inputs.layer_angles(L, n, seed + 17 * r + 1)
        specs.append(mixed.RequestSpec(x, th, ph, inputs.neighbour_pairs(p), chi, prec))
    return specs


def alone(anomps, sp):
    import torch
    # one mps_apply_layer call per layer, the mixed table's own step structure
    res = anomps.extract_features(sp.pixels[None], sp.theta, sp.phi, sp.pairs, sp.chi, sp.precision,
                                  per_layer=True)
    torch.cuda.synchronize()
    return res[0].cpu().numpy()[0], int(res[1].cpu().numpy()[0])


CASES = [(4, 2, 4, 0), (6, 1, 16, 1), (7, 4, 16, 1), (3, 3, 2, 0), (5, 2, 16, 1), (7, 3, 8, 1),
         (4, 0, 4, 1), (8, 2, 16, 1), (2, 1, 2, 0), (6, 3, 5, 1), (7, 4, 16, 0), (5, 4, 3, 1)]


def test_mixed_equals_alone_and_oracle(M):
    import torch
    anomps, mixed = M
    specs = make_specs(mixed, anomps, CASES, 300)
    print(f"[case] mixed table of {len(specs)} requests", flush=True)
    mr = mixed.MixedRequests(specs)
    mr.run()
    torch.cuda.synchronize()
    outs, ctrl = mr.outputs(), mr.ctrl()
    for r, sp in enumerate(specs):
        assert ctrl[r][0] == sp.layers and ctrl[r][1] == 0
        ref_alone, st = alone(anomps, sp)
        assert st == 0
        assert np.array_equal(outs[r], ref_alone), f"request {r} differs from its batch-1 run"
    # oracle on requests in the exact regime (chi >= 2^L), small enough for the CPU
    for r in (0, 1, 4, 6, 8):
        sp = specs[r]
        ref = ofeat.truncated_features(sp.pixels[None], sp.theta, sp.phi, sp.pairs, sp.chi)[0][0]
        tol = 1e-10 if sp.precision == anomps.PREC_FP64 else 1e-5
        assert np.abs(outs[r] - ref).max() <= tol


def test_mixed_steps_skip_finished_requests(M):
    import torch
    anomps, mixed = M
    specs = make_specs(mixed, anomps, [(4, 1, 4, 1), (4, 3, 8, 1), (5, 2, 4, 0)], 400)
    mr = mixed.MixedRequests(specs)
    mr.init()
    for _ in range(5):  # more steps than any request needs: extra steps change nothing
        mr.step()
    mr.measure()
    torch.cuda.synchronize()
    assert np.array_equal(mr.ctrl()[:, 0], [1, 3, 2])
    for r, sp in enumerate(specs):
        assert np.array_equal(mr.outputs()[r], alone(anomps, sp)[0])


def test_mixed_graph_replay(M):
    """init + all layer steps + measurement captured once, replayed three times with eager work
    in between; every replay equals the eager run."""
    import torch
    anomps, mixed = M
    specs = make_specs(mixed, anomps, [(6, 2, 16, 1), (4, 2, 4, 0), (7, 1, 16, 1), (5, 3, 8, 1)], 500)
    mr = mixed.MixedRequests(specs)
    mr.run()
    torch.cuda.synchronize()
    eager = mr.outputs()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            mr.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        junk = torch.randn(1 << 16, device="cuda") * 2.0  # eager work between replays
        mr.bytes.zero_()
        g.replay()
        torch.cuda.synchronize()
        del junk
        got = mr.outputs()
        for r in range(len(specs)):
            assert np.array_equal(got[r], eager[r]), f"replay {rep} request {r}"
        assert np.array_equal(mr.ctrl()[:, 0], [sp.layers for sp in specs])


def test_mixed_nonfinite_pixel_flags_only_its_request(M):
    import torch
    anomps, mixed = M
    specs = make_specs(mixed, anomps, [(4, 2, 4, 1), (4, 2, 4, 1)], 600)
    specs[1].pixels = specs[1].pixels.copy()
    specs[1].pixels[5] = np.nan
    mr = mixed.MixedRequests(specs)
    mr.run()
    torch.cuda.synchronize()
    ctrl = mr.ctrl()
    assert ctrl[0][1] == 0 and ctrl[1][1] & anomps.IMG_NONFINITE
    assert np.array_equal(mr.outputs()[0], alone(anomps, specs[0])[0])
