"""The training step on cached features (mps_ano_train_step) against the oracle's step:
loss, updated parameters and Adam moments after several steps, FP64 and FP32."""
import numpy as np
import pytest

from oracle import train as otrain
from paper_2607_10280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("f64", [True, False])
def test_train_steps_match_oracle(f64):
    import torch
    from paper_2607_10280_amd import anomps
    rng = np.random.Generator(np.random.PCG64(70))
    nb, m, out = 37, 24, 53
    pauli = rng.uniform(-1, 1, size=(nb, m, 15))
    a, b, d, w, bias = inputs.readout_params(m, out, 71, w_std=0.2)
    bias = rng.uniform(-0.1, 0.1, size=out)
    target = rng.uniform(-1, 1, size=(nb, out))
    dt = torch.float64 if f64 else torch.float32
    T = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=dt, device="cuda")
    tr = anomps.AnoTrainer(T(a), T(b), T(d), T(w), T(bias), nb, lr_obs=0.02, lr_lin=0.01)
    params = (a, b, d, w, bias)
    state = [(np.zeros_like(p), np.zeros_like(p)) for p in params]
    tol = 1e-11 if f64 else 2e-5
    print(f"[case] train f64={f64} batch={nb} m={m} out={out}", flush=True)
    for step in range(1, 6):
        loss = tr.step(T(pauli), T(target))
        torch.cuda.synchronize()
        lref, params, state = otrain.train_step(pauli, params, state, target, step, 0.02, 0.01)
        assert abs(float(loss.item()) - lref) <= tol * max(1.0, lref)
        for got, ref in zip(tr.params, params):
            assert np.abs(got.cpu().numpy() - ref).max() <= tol
    mom = np.concatenate([s[0].reshape(-1) for s in state])
    assert np.abs(tr.mom.cpu().numpy() - mom).max() <= tol
