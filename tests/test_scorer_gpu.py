"""GPU MLP kernels (BF16 MFMA) against the FP64 reference with the same
BF16 rounding points: forward logits, gradients (<= 1e-3 relative per
parameter block) and one Adam step."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu

BLOCKS = {"W1": M.W1, "b1": M.B1, "W2": M.W2, "b2": M.B2, "w3": M.W3, "b3": M.B3}


def _setup(rows, seed):
    import torch
    import paper_0908_3934_amd as gn
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (rows, M.IN)).astype(np.float32)
    y = (rng.random(rows) < 0.3).astype(np.float32)
    p = gn.Mlp.init_params(seed)
    net = gn.Mlp(p)
    return net, p, X, y, torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")


@pytest.mark.parametrize("rows", [1, 63, 777, 5000])
def test_forward_matches_reference(rows):
    import torch
    net, p, X, y, Xd, yd = _setup(rows, rows)
    z = net.forward(Xd).cpu().numpy().astype(np.float64)
    zr, _ = M.forward(p.astype(np.float64), X.astype(np.float64), bf=True)
    scale = max(1.0, np.abs(zr).max())
    assert np.abs(z - zr).max() <= 2e-3 * scale
    assert np.median(np.abs(z - zr)) <= 1e-4 * scale


@pytest.mark.parametrize("rows", [777, 9000])
def test_gradient_matches_reference(rows):
    import torch
    net, p, X, y, Xd, yd = _setup(rows, 10 + rows)
    g, loss = net.grad(Xd, yd)
    g = g.cpu().numpy().astype(np.float64)
    gr, lr = M.grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), bf=True)
    assert float(loss.cpu()) == pytest.approx(lr, rel=1e-4)
    for name, sl in BLOCKS.items():
        err = np.linalg.norm(g[sl] - gr[sl]) / max(np.linalg.norm(gr[sl]), 1e-12)
        assert err <= 1e-3, (name, err)


def test_adam_step_matches_reference():
    import torch
    net, p, X, y, Xd, yd = _setup(2048, 99)
    gr, _ = M.grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), bf=True)
    net.train_step(Xd, yd, 1e-3)
    p1 = net.get_params().astype(np.float64)
    pr, _, _ = M.adam(p.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), gr, 1, 1e-3)
    # the first Adam step moves each parameter by ~lr*sign(g): compare the moves
    step, step_r = p1 - p, pr - p
    big = np.abs(gr) > 1e-6
    assert np.mean(np.sign(step[big]) == np.sign(step_r[big])) > 0.99
    assert np.abs(step - step_r)[big].max() <= 2e-4


def test_training_reduces_loss():
    import torch
    import paper_0908_3934_amd as gn
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (8192, M.IN)).astype(np.float32)
    w = rng.normal(0, 1, M.IN)
    y = ((X @ w) > 0).astype(np.float32)               # a learnable rule
    Xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    net = gn.Mlp(gn.Mlp.init_params(1))
    _, l0 = net.grad(Xd, yd)
    for _ in range(200):
        net.train_step(Xd, yd, 2e-3)
    _, l1 = net.grad(Xd, yd)
    assert float(l1.cpu()) < 0.25 * float(l0.cpu())


@pytest.mark.parametrize("rows", [70001])
def test_forward_many_tiles_with_input_norm(rows):
    """Forward (one fused kernel) over many 32-row tiles per wave with a
    ragged last tile, under a non-trivial input standardisation."""
    import torch
    net, p, X, y, Xd, yd = _setup(rows, 4)
    rng = np.random.default_rng(8)
    shift = rng.normal(0, 0.5, M.IN).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, M.IN).astype(np.float32)
    net.set_input_norm(shift, scale)
    z = net.forward(Xd).cpu().numpy().astype(np.float64)
    zr, _ = M.forward(p.astype(np.float64), X.astype(np.float64), bf=True,
                      shift=shift.astype(np.float64), scale=scale.astype(np.float64))
    scale_z = max(1.0, np.abs(zr).max())
    assert np.abs(z - zr).max() <= 2e-3 * scale_z
    assert np.median(np.abs(z - zr)) <= 1e-4 * scale_z


def test_forward_after_training_steps():
    """Adam keeps every BF16 copy of the weights current, including the
    layout the fused forward kernel stages: logits after a few steps match
    the reference evaluated at the parameters read back."""
    import torch
    net, p, X, y, Xd, yd = _setup(3000, 21)
    for _ in range(3):
        net.train_step(Xd, yd, 1e-2)
    p1 = net.get_params().astype(np.float64)
    z = net.forward(Xd).cpu().numpy().astype(np.float64)
    zr, _ = M.forward(p1, X.astype(np.float64), bf=True)
    scale_z = max(1.0, np.abs(zr).max())
    assert np.abs(z - zr).max() <= 2e-3 * scale_z
