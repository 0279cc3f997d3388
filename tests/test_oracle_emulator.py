"""Pins of the oracle emulator: special cases that reduce to affine maps."""
import numpy as np

from oracle.emulator import activation, emulate, mlp


def tiny_net(rng, dims, beta=None, gamma=None):
    W = [rng.normal(size=(dims[l + 1], dims[l])) for l in range(len(dims) - 1)]
    b = [rng.normal(size=dims[l + 1]) for l in range(len(dims) - 1)]
    H = len(dims) - 2
    be = [np.full(dims[l + 1], beta) if beta is not None else rng.normal(size=dims[l + 1]) for l in range(H)]
    ga = [np.full(dims[l + 1], gamma) if gamma is not None else rng.normal(size=dims[l + 1]) for l in range(H)]
    return dict(W=W, b=b, beta=be, gamma=ga, in_shift=rng.normal(size=dims[0]),
                in_scale=rng.uniform(0.5, 2.0, size=dims[0]), out_mu=rng.normal(size=dims[-1]),
                out_sigma=rng.uniform(0.5, 2.0, size=dims[-1]))


def compose_affine(net, scales):
    """Collapse x -> (W_L diag(s_{L-1}) ... diag(s_1) W_1 x + ...) into (A, c)."""
    A = np.eye(net["W"][0].shape[1])
    c = np.zeros(net["W"][0].shape[1])
    for l, (W, b) in enumerate(zip(net["W"], net["b"])):
        A, c = W @ A, W @ c + b
        if l < len(scales):
            A, c = scales[l][:, None] * A, scales[l] * c
    return A, c


def test_identity_activation_is_affine():
    rng = np.random.default_rng(0)
    net = tiny_net(rng, (3, 5, 4, 2), gamma=1.0)
    A, c = compose_affine(net, [np.ones(5), np.ones(4)])
    th = rng.normal(size=(7, 3))
    x = (th - net["in_shift"]) / net["in_scale"]
    want = net["out_mu"] + net["out_sigma"] * (x @ A.T + c)
    np.testing.assert_allclose(emulate(th, net), want, rtol=1e-12, atol=1e-12)


def test_zero_beta_gate_is_constant():
    rng = np.random.default_rng(1)
    net = tiny_net(rng, (2, 3, 3, 2), beta=0.0)
    scales = [(g + (1 - g) * 0.5) for g in net["gamma"]]
    A, c = compose_affine(net, scales)
    x = rng.normal(size=(5, 2))
    np.testing.assert_allclose(mlp(x, net), x @ A.T + c, rtol=1e-12, atol=1e-12)


def test_activation_odd_part_closed_form():
    rng = np.random.default_rng(2)
    t, beta, gamma = rng.normal(size=50) * 3, rng.normal(size=50), rng.normal(size=50)
    lhs = activation(t, beta, gamma) + activation(-t, beta, gamma)
    np.testing.assert_allclose(lhs, (1 - gamma) * t * np.tanh(beta * t / 2), rtol=1e-12, atol=1e-14)
    # large positive beta t -> identity; large negative -> gamma t
    np.testing.assert_allclose(activation(np.array([50.0]), 2.0, 0.3), [50.0])
    np.testing.assert_allclose(activation(np.array([-50.0]), 2.0, 0.3), [-15.0])
