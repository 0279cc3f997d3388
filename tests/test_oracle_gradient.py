"""Pins of the complex-step oracle gradient: central differences and exact zeros."""
import numpy as np

import workloads as W
from oracle.gradient import central_difference, loglike_grad


def check(model, theta, rel):
    logl, g = loglike_grad(theta, model)
    width = np.where(model["prior_kind"] == 0, model["prior_b"] - model["prior_a"], model["prior_b"])
    fd = central_difference(theta, model, 1e-5 * width)
    scale = np.max(np.abs(g), axis=1, keepdims=True)
    err = np.abs(g - fd) / scale
    assert np.all(err < rel), err.max()
    return g


def test_cmb_diag_gradient():
    m = W.load_model("cmb6")
    th = W.posterior_draws(m["theta_fid"], m["fisher_sigma"], 3)
    check(m, th, 1e-5)


def test_cmb_block_gradient():
    m = W.load_model("cmb4x2500")
    th = W.posterior_draws(m["theta_fid"], m["fisher_sigma"], 2)
    check(m, th, 1e-5)


def test_cmb_cv_gradient():
    m = W.load_model("cmbtt_cv")
    th = W.posterior_draws(m["theta_fid"], m["fisher_sigma"], 2)
    check(m, th, 1e-5)


def test_shear_gradient_and_extra_nuisance_zero():
    m = W.load_model("shear10")
    scale = np.minimum(m["fisher_sigma"], 0.1 * np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0))
    th = W.posterior_draws(m["theta_fid"], scale, 2)
    g = check(m, th, 1e-4)
    assert np.all(g[:, -15:] == 0.0)


def test_out_of_support_gradient_is_zero():
    m = W.load_model("cmb6")
    th = np.full((1, 6), 0.5)
    th[0, 2] = 1.5
    logl, g = loglike_grad(th, m)
    assert logl[0] == -np.inf and np.all(g == 0)
