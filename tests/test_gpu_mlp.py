"""Rank-predictor kernels (FP32) against the FP64 oracle reference, through
the C ABI: forward pass, full-batch MSE gradient, one Adam step, training."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] - 0.25 * X[:, 2] * X[:, 3]).astype(np.float32)
    return X, t


@pytest.mark.parametrize("n", [1, 63, 64, 1000])
def test_forward_and_gradient_match_oracle(lib, n):
    import torch
    th = mlp.init(7).astype(np.float32)
    X, t = _data(n, 3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    w = dev(th)
    y = lib.mlp_forward(w, dev(X)).cpu().numpy()
    yo, _ = mlp.forward(th.astype(np.float64), X.astype(np.float64))
    assert np.allclose(y, yo, rtol=1e-4, atol=1e-4 * np.abs(yo).max())
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    g = torch.zeros_like(w)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lib.mlp_train_step(w, m, v, g, dev(X), dev(t), 1, 1e-3, loss)
    lo, go = mlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    gg = g.cpu().numpy()
    assert abs(float(loss.item()) - lo) <= 1e-4 * max(1.0, lo)
    assert np.linalg.norm(gg - go) <= 1e-4 * np.linalg.norm(go)
    # one Adam step from zero moments (closed form: lr * g / (|g| + eps))
    wo, _, _ = mlp.adam_step(th.astype(np.float64), gg.astype(np.float64), np.zeros(mlp.NPARAM),
                             np.zeros(mlp.NPARAM), 1, lr=1e-3)
    assert np.allclose(w.cpu().numpy(), wo, rtol=1e-5, atol=1e-6)


def test_training_is_deterministic_and_reduces_loss(lib):
    import torch
    X, t = _data(2000, 5)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Xd, td = dev(X), dev(t)
    finals = []
    for rep in range(2):
        w = dev(mlp.init(7).astype(np.float32))
        m, v, g = torch.zeros_like(w), torch.zeros_like(w), torch.zeros_like(w)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        lib.mlp_train_step(w, m, v, g, Xd, td, 1, 3e-3, loss)
        l0 = float(loss.item())
        for s in range(2, 301):
            lib.mlp_train_step(w, m, v, g, Xd, td, s, 3e-3, loss)
        assert float(loss.item()) < 0.2 * l0
        finals.append(w.cpu().numpy())
    assert np.array_equal(finals[0], finals[1])
