"""Cost-model network: the float64 oracle pinned by finite differences and
by torch's float64 autograd; the GPU forward/backward/Adam kernels checked
against the oracle."""
import numpy as np
import pytest

from oracle import mlp

F, W = 40, 64


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.num_params(F, W)) * scale


def rand_batch(seed, B=37):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, F))
    T = rng.standard_normal(B)
    return X, T


# ---------------------------------------------------------------- oracle pins
def test_num_params():
    assert mlp.num_params(F, W) == 6849


def test_forward_closed_form_tiny():
    """A hand-built network: W1 picks x0 into unit 0, ReLU, W2 copies unit 0,
    W3 doubles it, b3 = 1, so y = 2 * max(x0, 0) + 1."""
    p = np.zeros(mlp.num_params(F, W))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, F, W)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    W3[0, 0] = 2.0
    b3[0] = 1.0
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = np.zeros((3, F))
    X[:, 0] = [-1.0, 0.5, 3.0]
    assert np.allclose(mlp.forward(p, X, F, W), [1.0, 2.0, 7.0])


def test_gradient_central_differences():
    p = rand_params(1)
    X, T = rand_batch(2, B=9)
    _, g = mlp.loss_grad(p, X, T, F, W)
    rng = np.random.default_rng(3)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T, F, W) - mlp.loss(p - e, X, T, F, W)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p = rand_params(4)
    X, T = rand_batch(5)
    L, g = mlp.loss_grad(p, X, T, F, W)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    i = 0
    parts = []
    for shape in [(W, F), (W,), (W, W), (W,), (1, W), (1,)]:
        n = int(np.prod(shape))
        parts.append(pt[i:i + n].reshape(shape))
        i += n
    W1, b1, W2, b2, W3, b3 = parts
    x = torch.tensor(X, dtype=torch.float64)
    y = torch.relu(torch.relu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    lt = torch.mean((y[:, 0] - torch.tensor(T, dtype=torch.float64)) ** 2)
    lt.backward()
    assert abs(lt.item() - L) < 1e-12
    assert np.max(np.abs(pt.grad.numpy() - g)) < 1e-12


def test_adam_first_step_moves_by_lr():
    """Adam's first step moves every coordinate with a non-zero gradient by
    lr (up to eps): m_hat = g, v_hat = g^2."""
    p = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.1])
    p1, m, v = mlp.adam_step(p, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    assert np.allclose(p1, -0.01 * np.sign(g), atol=1e-9)


# ---------------------------------------------------------------- GPU kernels
@pytest.mark.gpu
def test_gpu_loss_grad_matches_oracle():
    import torch
    from paper_2602_09604_amd import sv
    m = sv.Mlp(seed=7)
    try:
        p = m.get_params().astype(np.float64)
        for B in (1, 37, 64, 200, 4096):
            X, T = rand_batch(B, B=B)
            L, g = m.loss_grad(torch.tensor(X, dtype=torch.float32, device="cuda"),
                               torch.tensor(T, dtype=torch.float32, device="cuda"))
            Lo, go = mlp.loss_grad(p, X.astype(np.float32), T.astype(np.float32), F, W)
            assert abs(L - Lo) <= 1e-4 * max(1.0, abs(Lo)), (B, L, Lo)
            rel = np.linalg.norm(g - go) / max(np.linalg.norm(go), 1e-30)
            assert rel <= 1e-4, (B, rel)
    finally:
        m.free()


@pytest.mark.gpu
def test_gpu_forward_and_adam_match_oracle():
    import torch
    from paper_2602_09604_amd import sv
    m = sv.Mlp(seed=11)
    try:
        p0 = m.get_params().astype(np.float64)
        X, T = rand_batch(12, B=300)
        xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        td = torch.tensor(T, dtype=torch.float32, device="cuda")
        y = m.forward(xd)
        yo = mlp.forward(p0, X.astype(np.float32), F, W)
        assert np.max(np.abs(y - yo)) <= 1e-4 * max(1.0, np.max(np.abs(yo)))
        # three Adam steps against the oracle's
        p, mo, vo = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        for t in range(1, 4):
            m.loss_grad(xd, td)
            m.adam_step(1e-3)
            _, g = mlp.loss_grad(p, X.astype(np.float32), T.astype(np.float32), F, W)
            p, mo, vo = mlp.adam_step(p, g, mo, vo, t, lr=1e-3)
        assert np.max(np.abs(m.get_params() - p)) < 1e-5
    finally:
        m.free()


@pytest.mark.gpu
def test_gpu_training_fits_a_smooth_target():
    import torch
    from paper_2602_09604_amd import sv
    rng = np.random.default_rng(0)
    X = (rng.random((2048, F)) < 0.3).astype(np.float32)
    T = (X[:, :10].sum(axis=1) * 0.3 - X[:, 20] + 0.1 * X[:, 30:].sum(axis=1)).astype(np.float32)
    m = sv.Mlp(seed=1)
    try:
        xd = torch.tensor(X, device="cuda")
        td = torch.tensor(T, device="cuda")
        l0, _ = m.loss_grad(xd, td)
        lf = m.train(xd, td, epochs=400, lr=3e-3)
        assert lf < 0.02 * l0, (l0, lf)
    finally:
        m.free()
