"""CPU pins of the scorer-side references: the FP64 MLP gradient against
central finite differences, the BF16 rounding against PyTorch's own
conversion, Adam against torch.optim.Adam, and the AUC against
scikit-learn."""
import numpy as np
import pytest
import torch

from oracle import metrics
from oracle import mlp as M


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.1, M.N_PARAMS) * scale
    return p


def test_parameter_count():
    assert M.N_PARAMS == 82689


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (37, M.IN))
    y = (rng.random(37) < 0.4).astype(np.float64)
    p = _params(2)
    g, _ = M.grad(p, X, y, bf=False)
    idx = np.concatenate([rng.choice(np.arange(M.W1.start, M.W1.stop), 25, replace=False),
                          rng.choice(np.arange(M.B1.start, M.B1.stop), 10, replace=False),
                          rng.choice(np.arange(M.W2.start, M.W2.stop), 25, replace=False),
                          rng.choice(np.arange(M.B2.start, M.B2.stop), 10, replace=False),
                          rng.choice(np.arange(M.W3.start, M.W3.stop), 10, replace=False), [M.B3.start]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.bce(M.forward(pp, X, False)[0], y) - M.bce(M.forward(pm, X, False)[0], y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 10, 20000), rng.normal(0, 1e-3, 2000), [0.0, -0.0, 1.0, 3.0, 1e-40]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_bf16_forward_close_to_fp64():
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (50, M.IN))
    p = _params(5)
    z1, _ = M.forward(p, X, True)
    z2, _ = M.forward(p, X, False)
    assert np.abs(z1 - z2).max() < 0.05 * max(1.0, np.abs(z2).max())


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.normal(0, 1, 50)
    gs = [rng.normal(0, 1, 50) for _ in range(5)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, 1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = M.adam(p, m, v, g, t, 1e-2)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_auc_matches_sklearn():
    from sklearn.metrics import roc_auc_score
    rng = np.random.default_rng(7)
    for ties in (False, True):
        s = rng.normal(0, 1, 3000)
        if ties:
            s = np.round(s, 1)
        y = rng.random(3000) < 0.3
        assert metrics.auc(s, y) == pytest.approx(roc_auc_score(y, s), abs=1e-12)
    assert metrics.auc([1, 2, 3, 4], [0, 0, 1, 1]) == 1.0
    assert metrics.auc([1, 1, 1, 1], [0, 1, 0, 1]) == 0.5
