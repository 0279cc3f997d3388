"""Neural emulator: a fully connected network with a gated activation.

The paper replaces Boltzmann codes by CosmoPower-JAX networks (Sec. 2.2 and
2.4) that map cosmological parameters to spectra; it does not print the
architecture.  The form used here:

    x   = (theta_sel - in_shift) / in_scale
    h_l = f_l(W_l h_{l-1} + b_l),         l = 1 .. H
    y   = out_mu + out_sigma * (W_{H+1} h_H + b_{H+1})
    f_l(t) = (gamma_l + (1 - gamma_l) * sigmoid(beta_l * t)) * t   (per unit)

Pinned by: gamma = 1 (identity activation) and beta = 0 (constant gate), which
reduce the network to a composition of affine maps, and by the closed form
f(t) + f(-t) = (1 - gamma) t tanh(beta t / 2) of the activation.
"""
import numpy as np


def sigmoid(u):
    return 1.0 / (1.0 + np.exp(-u))


def activation(t, beta, gamma):
    """Gated activation f(t) = (gamma + (1 - gamma) sigmoid(beta t)) t, per unit."""
    return (gamma + (1.0 - gamma) * sigmoid(beta * t)) * t


def mlp(x, net):
    """Raw network output W_{H+1} h_H + b_{H+1} for inputs x [rows, n_in]."""
    h = x
    n_hidden = len(net["W"]) - 1
    for l in range(n_hidden):
        t = h @ net["W"][l].T + net["b"][l]
        h = activation(t, net["beta"][l], net["gamma"][l])
    return h @ net["W"][-1].T + net["b"][-1]


def emulate(inputs, net, out_mu=None):
    """Emulator prediction y = mu + sigma * mlp((inputs - shift) / scale).

    ``out_mu`` overrides ``net["out_mu"]`` (the shear emulator uses a
    per-redshift-node offset table).
    """
    x = (inputs - net["in_shift"]) / net["in_scale"]
    mu = net["out_mu"] if out_mu is None else out_mu
    return mu + net["out_sigma"] * mlp(x, net)
