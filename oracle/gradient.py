"""Gradient of the log-likelihood by the complex step (Squire & Trapp 1998).

d logL / d theta_k = Im logL(theta + i h e_k) / h with h = 1e-30, exact to
rounding because every operation of the oracle likelihoods is complex
analytic (interpolation indices and range masks use the real part only).
Out-of-support rows get logL = -inf and a zero gradient.

Pinned by: central finite differences, and by the exact zero gradient of the
extra nuisance parameters that do not enter the likelihood.
"""
import numpy as np

from .likelihood import loglike, loglike_raw

H_CS = 1e-30


def loglike_grad(theta, model):
    """(logL [B], grad [B, d]) at theta [B, d]."""
    theta = np.asarray(theta, dtype=np.float64)
    B, d = theta.shape
    logl = loglike(theta, model)
    grad = np.zeros((B, d))
    ok = np.isfinite(logl)
    if np.any(ok):
        th = theta[ok]
        for k in range(d):
            tc = th.astype(np.complex128)
            tc[:, k] += 1j * H_CS
            grad[ok, k] = loglike_raw(tc, model).imag / H_CS
    return logl, grad


def central_difference(theta, model, step):
    """Central finite differences with per-coordinate steps ``step`` [d]."""
    theta = np.asarray(theta, dtype=np.float64)
    B, d = theta.shape
    g = np.zeros((B, d))
    for k in range(d):
        tp, tm = theta.copy(), theta.copy()
        tp[:, k] += step[k]
        tm[:, k] -= step[k]
        g[:, k] = (loglike_raw(tp, model) - loglike_raw(tm, model)) / (2 * step[k])
    return g
