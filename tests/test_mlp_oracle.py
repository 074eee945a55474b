"""Pins of the FP64 reference network: gradient against central finite
differences, ReLU and bias handling on a hand-sized case, Adam's first step."""
import numpy as np

from oracle.mlp_oracle import MLPRef


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    net = MLPRef(in_dim=5, hidden=7, layers=2, rank=3, out_dim=6)
    p = rng.standard_normal(net.nparam) * 0.5
    X = rng.standard_normal((4, 5))
    Zs = rng.standard_normal((4, 6))
    mu, sig = rng.standard_normal(5) * 0.1, 1 + rng.random(5)
    loss, g = net.loss_grad(p, X, Zs, mu, sig)
    h = 1e-6
    idx = rng.choice(net.nparam, 60, replace=False)
    for i in idx:
        e = np.zeros(net.nparam); e[i] = h
        fd = (net.loss(p + e, X, Zs, mu, sig) - net.loss(p - e, X, Zs, mu, sig)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert loss == net.loss(p, X, Zs, mu, sig)


def test_hand_case_relu_and_bias():
    # 1 input -> 1 hidden (ReLU) -> 1 rank -> 1 output, all weights known
    net = MLPRef(in_dim=1, hidden=1, layers=1, rank=1, out_dim=1)
    # W1=2, b1=-1, W2=3, b2=0.5, W3=-1, b3=4
    p = np.array([2.0, -1.0, 3.0, 0.5, -1.0, 4.0])
    X = np.array([[1.0], [0.25]])
    Z = net.forward(p, X, 0.0, 1.0)[-1]
    # x=1: h=relu(1)=1, a=3.5, z=0.5;  x=0.25: h=relu(-0.5)=0, a=0.5, z=3.5
    assert np.allclose(Z.ravel(), [0.5, 3.5])


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 0.0]); g = np.array([0.3, -5.0, 1e-3])
    q, m, v = MLPRef.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # after bias correction the first step is lr * g/|g| (up to eps)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-7)
