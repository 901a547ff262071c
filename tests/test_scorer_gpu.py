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
        # element by element, against the block's largest gradient
        bound = 1e-3 * np.abs(gr[sl]).max() + 1e-7
        worst = np.abs(g[sl] - gr[sl]).max()
        assert worst <= bound, (name, worst, bound, int(np.argmax(np.abs(g[sl] - gr[sl]))))


def test_adam_step_matches_reference():
    import torch
    net, p, X, y, Xd, yd = _setup(2048, 99)
    gr, _ = M.grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), bf=True)
    net.train_step(Xd, yd, 1e-3)
    p1 = net.get_params().astype(np.float64)
    pr, _, _ = M.adam(p.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), gr, 1, 1e-3)
    # the first Adam step moves each parameter by lr*g/(|g| + eps): compare the moves
    step, step_r = p1 - p, pr - p
    big = np.abs(gr) > 1e-6
    assert np.mean(np.sign(step[big]) == np.sign(step_r[big])) > 0.99
    assert np.abs(step - step_r)[big].max() <= 2e-4
    # where |g| >> eps the move is lr*sign(g) up to lr*eps/|g|, and the FP32
    # parameter is rounded once: element-wise bound
    clear = np.abs(gr) > 1e-4
    tol = 1e-3 * 1e-8 / np.abs(gr[clear]) + 2.0 * np.spacing(np.abs(p[clear]).astype(np.float32)) + 1e-9
    assert (np.abs(step - step_r)[clear] <= tol).all()


def test_two_adam_steps_match_reference():
    """Two optimizer steps on the same batch: bias correction of step 2 and
    the moments carried between calls, element by element against the FP64
    reference (gradient at the reference's own parameters)."""
    import torch
    net, p, X, y, Xd, yd = _setup(2048, 98)
    lr = 1e-3
    net.train_step(Xd, yd, lr)
    net.train_step(Xd, yd, lr)
    p2 = net.get_params().astype(np.float64)
    pr = p.astype(np.float64)
    m = np.zeros(M.N_PARAMS)
    v = np.zeros(M.N_PARAMS)
    gs = []
    for t in (1, 2):
        gr, _ = M.grad(pr, X.astype(np.float64), y.astype(np.float64), bf=True)
        gs.append(gr)
        pr, m, v = M.adam(pr, m, v, gr, t, lr)
    moved = np.abs(pr - p) > 1e-4
    assert moved.mean() > 0.5
    assert np.mean(np.sign(p2 - p)[moved] == np.sign(pr - p)[moved]) > 0.999
    # where both gradients are clear of the rounding noise and agree in sign,
    # the two-step move is well conditioned: element-wise bound
    g1, g2 = gs
    clear = (np.abs(g1) > 1e-2 * np.abs(g1).max()) & (np.abs(g2) > 1e-2 * np.abs(g2).max()) & \
        (np.sign(g1) == np.sign(g2))
    assert clear.sum() > 1000
    assert np.abs(p2 - pr)[clear].max() <= 0.05 * lr


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
