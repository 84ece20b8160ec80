"""Pins for oracle.mlp: gradients against central differences, Adam on a quadratic."""
import numpy as np

from oracle import mlp
from synth import splitmix64, uniform01


def _params(seed):
    u = 2 * uniform01(seed, 6337) - 1
    W1 = u[:2048].reshape(64, 32) * 0.3
    b1 = u[2048:2112] * 0.1
    W2 = u[2112:6208].reshape(64, 64) * 0.2
    b2 = u[6208:6272] * 0.1
    w3 = u[6272:6336] * 0.2
    b3 = float(u[6336])
    return [W1, b1, W2, b2, w3, b3]


def test_features():
    X = mlp.features(np.array([0b1011, 1 << 31], dtype=np.uint64))
    assert X.shape == (2, 32)
    assert list(np.nonzero(X[0])[0]) == [0, 1, 3] and list(np.nonzero(X[1])[0]) == [31]


def test_gradients_central_differences():
    P = _params(1)
    X = mlp.features(splitmix64(2, 16) & np.uint64(0xFFFFFFFF))
    tgt = uniform01(3, 16)
    G = mlp.gradients(P, X, tgt)
    h = 1e-6
    checked = 0
    for pi, p in enumerate(P):
        if np.isscalar(p):
            Pp = list(P); Pp[pi] = p + h
            Pm = list(P); Pm[pi] = p - h
            num = (mlp.loss(Pp, X, tgt) - mlp.loss(Pm, X, tgt)) / (2 * h)
            assert abs(num - G[pi]) < 1e-7
            checked += 1
            continue
        flat = p.reshape(-1)
        for j in range(0, flat.size, max(1, flat.size // 23)):
            Pp = [q.copy() if not np.isscalar(q) else q for q in P]
            Pm = [q.copy() if not np.isscalar(q) else q for q in P]
            Pp[pi].reshape(-1)[j] += h
            Pm[pi].reshape(-1)[j] -= h
            num = (mlp.loss(Pp, X, tgt) - mlp.loss(Pm, X, tgt)) / (2 * h)
            assert abs(num - G[pi].reshape(-1)[j]) < 1e-7 * max(1.0, abs(num))
            checked += 1
    assert checked > 100


def test_adam_minimises_quadratic():
    P = [np.array([3.0, -2.0])]
    m = [np.zeros(2)]
    v = [np.zeros(2)]
    for step in range(1, 3001):
        G = [2 * P[0]]
        P, m, v = mlp.adam_step(P, G, m, v, step, lr=0.01)
    assert np.abs(P[0]).max() < 1e-3
    # first step moves each coordinate by lr against the gradient sign
    P1, _, _ = mlp.adam_step([np.array([1.0, -1.0])], [np.array([5.0, -0.1])],
                             [np.zeros(2)], [np.zeros(2)], 1, lr=0.1)
    assert np.allclose(P1[0], [0.9, -0.9], atol=1e-6)
