"""Prior transform and per-model log-likelihood dispatch.

Priors are the per-parameter uniform or Gaussian distributions of Table 1.
Nested sampling draws in the unit hypercube and maps u -> theta:
    uniform U(a, b):  theta = a + (b - a) u
    normal  N(mu, s): theta = mu + s sqrt(2) erfinv(2u - 1)
The evidence, Eq. (1), integrates L(theta) pi(theta) dtheta; in u the prior
is uniform, so Z = int L(T(u)) du.

Support convention: theta outside a uniform prior's [a, b] has logL = -inf
(the sampler relies on it); NaN theta gives NaN.

Pinned by: scipy.stats.norm.ppf / uniform quantiles for the transform; the
per-model likelihoods carry their own pins.
"""
import numpy as np
from scipy.special import erfinv

from . import cmb, shear

UNIFORM, NORMAL = 0, 1


def prior_transform(u, model):
    """u [B, d] in the unit cube -> theta [B, d]."""
    kind, a, b = model["prior_kind"], model["prior_a"], model["prior_b"]
    uni = a + (b - a) * u
    nrm = a + b * np.sqrt(2.0) * erfinv(2.0 * u - 1.0)
    return np.where(kind[None, :] == UNIFORM, uni, nrm)


def in_support(theta, model):
    """True where every uniform-prior coordinate lies in its [a, b]."""
    kind, a, b = model["prior_kind"], model["prior_a"], model["prior_b"]
    t = theta.real
    ok = (t >= a[None, :]) & (t <= b[None, :])
    ok = ok | (kind[None, :] != UNIFORM)
    return np.all(ok, axis=1)


def gauss_loglike(theta, model):
    """Diagonal Gaussian N(theta; mu, sigma^2) including its normalisation."""
    r = (theta - model["mu"][None, :]) / model["sigma"][None, :]
    d = theta.shape[1]
    return -0.5 * np.sum(r * r, axis=1) - np.sum(np.log(model["sigma"])) - 0.5 * d * np.log(2 * np.pi)


def loglike_raw(theta, model):
    """Log-likelihood of theta [B, d] with no support check."""
    kind = model["kind"]
    if kind == "cmb_diag":
        return cmb.loglike_diag(theta, model)
    if kind == "cmb_block":
        return cmb.loglike_block(theta, model)
    if kind == "cmb_cv":
        return cmb.loglike_cv(theta, model)
    if kind == "shear":
        return shear.loglike(theta, model)
    if kind == "gauss":
        return gauss_loglike(theta, model)
    raise ValueError(kind)


def loglike(theta, model, chunk=None):
    """Batched log-likelihood with the support convention; optional row chunking."""
    theta = np.asarray(theta)
    B = theta.shape[0]
    out = np.full(B, -np.inf, dtype=np.result_type(theta.dtype, np.float64))
    ok = in_support(theta, model) | np.any(np.isnan(theta.real), axis=1)
    idx = np.nonzero(ok)[0]
    step = chunk or max(1, idx.size)
    for s in range(0, idx.size, step):
        sel = idx[s:s + step]
        out[sel] = loglike_raw(theta[sel], model)
    return out


def loglike_u(u, model, chunk=None):
    """Log-likelihood on the unit hypercube (points outside it give -inf)."""
    u = np.asarray(u, dtype=np.float64)
    inside = np.all((u >= 0.0) & (u <= 1.0), axis=1)
    out = np.full(u.shape[0], -np.inf)
    if np.any(inside):
        out[inside] = loglike(prior_transform(u[inside], model), model, chunk=chunk)
    return out
