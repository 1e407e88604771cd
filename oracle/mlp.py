"""FP64 reference of the level scheduler's network. TEST INFRASTRUCTURE ONLY.

A multilayer perceptron 6 -> 64 -> 64 -> K with ReLU after the two hidden
layers and a linear output. Output k is the predicted log run time of
action k for the level described by the 6 input features; the scheduler
takes the arg-min. Training minimises the masked mean squared error on the
log times of the actions that were measured, with Adam (Kingma & Ba 2015,
Algorithm 1: beta1 = 0.9, beta2 = 0.999, epsilon = 1e-8, bias-corrected).

Parameter vector layout (shared with the GPU side through the C ABI):
  W1[64][6], b1[64], W2[64][64], b2[64], W3[K][64], b3[K]   (row-major)
"""
import numpy as np

N_IN, N_HID = 6, 64


def n_params(K):
    return N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + K * N_HID + K


def unpack(theta, K):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (n_params(K),)
    o = 0
    out = []
    for shape in ((N_HID, N_IN), (N_HID,), (N_HID, N_HID), (N_HID,), (K, N_HID), (K,)):
        size = int(np.prod(shape))
        out.append(theta[o:o + size].reshape(shape))
        o += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


def forward(theta, X, K):
    """Returns the outputs Y [B, K] and the activations needed by backward."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, K)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    Y = h2 @ W3.T + b3
    return Y, (X, z1, h1, z2, h2)


def loss(Y, T, M):
    """Masked mean squared error: sum of M*(Y-T)^2 over entries / sum of M."""
    M = np.asarray(M, np.float64)
    cnt = M.sum()
    return float((M * (Y - T) ** 2).sum() / cnt) if cnt > 0 else 0.0


def backward(theta, cache, Y, T, M, K):
    """Gradient of loss(Y, T, M) with respect to theta (chain rule, by hand)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, K)
    X, z1, h1, z2, h2 = cache
    M = np.asarray(M, np.float64)
    cnt = M.sum()
    dY = 2.0 * M * (Y - T) / cnt if cnt > 0 else np.zeros_like(Y)
    gW3 = dY.T @ h2
    gb3 = dY.sum(axis=0)
    dh2 = dY @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def train(theta, X, T, M, K, steps, lr):
    """Full-batch Adam for `steps` steps; returns (theta, loss history)."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        Y, cache = forward(theta, X, K)
        hist.append(loss(Y, T, M))
        g = backward(theta, cache, Y, T, M, K)
        theta, m, v = adam_step(theta, g, m, v, t, lr)
    return theta, hist


def init_params(K, seed):
    """He-style uniform initial weights from a seeded numpy generator (test inputs)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((N_IN, N_HID), (N_HID, N_HID), (N_HID, K)):
        bound = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)))
        parts.append(np.zeros(fan_out))
    return pack(parts)
