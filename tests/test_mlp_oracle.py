"""Pins the FP64 scheduler-network oracle: central finite differences, an
independent library implementation (torch CPU autograd and torch.optim.Adam),
and closed forms of Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def data(K, B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, mlp.N_IN))
    T = rng.normal(size=(B, K))
    M = (rng.random((B, K)) < 0.7).astype(float)
    M[0, 0] = 1.0
    return X, T, M


@pytest.mark.parametrize("K", [1, 3, 9])
def test_gradient_matches_central_differences(K):
    theta = mlp.init_params(K, seed=K)
    X, T, M = data(K, 17, seed=K + 1)
    Y, cache = mlp.forward(theta, X, K)
    g = mlp.backward(theta, cache, Y, T, M, K)
    rng = np.random.default_rng(5)
    idx = rng.choice(theta.size, size=min(300, theta.size), replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(mlp.forward(tp, X, K)[0], T, M) - mlp.loss(mlp.forward(tm, X, K)[0], T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_backward_and_adam_match_torch():
    torch = pytest.importorskip("torch")
    K = 5
    theta = mlp.init_params(K, seed=11)
    X, T, M = data(K, 23, seed=12)
    W1, b1, W2, b2, W3, b3 = [torch.tensor(p, dtype=torch.float64, requires_grad=True)
                              for p in mlp.unpack(theta, K)]
    net = lambda x: torch.relu(torch.relu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3  # noqa: E731
    Xt, Tt, Mt = (torch.tensor(a) for a in (X, T, M))
    Y = net(Xt)
    ours, _ = mlp.forward(theta, X, K)
    np.testing.assert_allclose(Y.detach().numpy(), ours, rtol=1e-13, atol=1e-13)
    L = (Mt * (Y - Tt) ** 2).sum() / Mt.sum()
    L.backward()
    g_t = np.concatenate([p.grad.numpy().ravel() for p in (W1, b1, W2, b2, W3, b3)])
    Yo, cache = mlp.forward(theta, X, K)
    np.testing.assert_allclose(mlp.backward(theta, cache, Yo, T, M, K), g_t, rtol=1e-12, atol=1e-14)
    # five Adam steps against torch.optim.Adam
    params = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in mlp.unpack(theta, K)]
    opt = torch.optim.Adam(params, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        opt.zero_grad()
        W1, b1, W2, b2, W3, b3 = params
        Yt = torch.relu(torch.relu(Xt @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
        ((Mt * (Yt - Tt) ** 2).sum() / Mt.sum()).backward()
        opt.step()
    ref = np.concatenate([p.detach().numpy().ravel() for p in params])
    ours, _ = mlp.train(theta, X, T, M, K, steps=5, lr=1e-2)
    np.testing.assert_allclose(ours, ref, rtol=1e-10, atol=1e-12)


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the update is lr * g / (|g| + eps)
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    theta, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    np.testing.assert_allclose(theta, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_fits_a_separable_target():
    """The network learns a target that depends on one input feature."""
    K = 2
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(256, mlp.N_IN))
    T = np.stack([X[:, 0], -X[:, 0]], axis=1)
    M = np.ones_like(T)
    theta, hist = mlp.train(mlp.init_params(K, seed=4), X, T, M, K, steps=400, lr=3e-3)
    assert hist[-1] < 0.02 * hist[0]
    Y, _ = mlp.forward(theta, X, K)
    assert np.mean(np.argmin(Y, 1) == np.argmin(T, 1)) > 0.95


def test_masked_entries_do_not_contribute():
    K = 3
    theta = mlp.init_params(K, seed=2)
    X, T, M = data(K, 9, seed=3)
    Y, cache = mlp.forward(theta, X, K)
    T2 = T.copy()
    T2[M == 0] += 1e6  # masked targets are irrelevant
    np.testing.assert_array_equal(mlp.backward(theta, cache, Y, T, M, K), mlp.backward(theta, cache, Y, T2, M, K))
    assert mlp.loss(Y, T, M) == mlp.loss(Y, T2, M)
