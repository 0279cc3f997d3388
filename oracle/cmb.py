"""CMB likelihoods: Gaussian forms and the cosmic-variance-limited TT likelihood
(Sec. 2.3-2.4 of the paper).

The paper's CMB analysis emulates C_l and evaluates them against mock data
(Sec. 2.4).  The workloads here use a Gaussian chi^2 of the emulated model
vector against a synthetic data vector:

* diagonal covariance (one emulator, raw outputs):
      logL = -1/2 sum_i ((d_i - m_i)/sigma_i)^2 - sum_i log sigma_i - n/2 log 2 pi
* block covariance (four emulators TT, TE, EE, phiphi; C = 10^y for TT, EE,
  phiphi and C = y for TE; data spectrum-major [TT | TE | EE | PP]): per
  multipole the residuals (TT, TE, EE) share a 3x3 covariance Sigma_l, PP is
  diagonal with sigma_pp,l:
      logL = -1/2 sum_l |L_l^{-1} r_l|^2 - 1/2 sum_l (r^pp_l / sigma_pp,l)^2
             - sum log diag(L_l) - sum log sigma_pp,l - n/2 log 2 pi,
  with L_l the lower Cholesky factor of Sigma_l.

Cosmic-variance-limited temperature likelihood (the paper's CMB analysis,
Sec. 2.4): with no noise, (2l+1) Ch_l / C_l follows a chi^2 distribution with
k = 2l+1 degrees of freedom, so the density of the observed Ch_l given the
emulated C_l = 10^y_l is p(Ch_l | C_l) = (k / C_l) f_k(k Ch_l / C_l), with
      log f_k(x) = (k/2 - 1) log x - x/2 - (k/2) log 2 - log Gamma(k/2),
and logL = sum_l log p(Ch_l | C_l) over l = l_min, l_min + 1, ...

Pinned by: scipy.stats.multivariate_normal.logpdf on the full covariance
(a library the oracle does not call) for small multipole ranges; for the
cosmic-variance form, scipy.stats.chi2.logpdf, the closed-form maximum at
C_l = Ch_l and the unit normalisation of p(Ch_l | C_l).
"""
import numpy as np
from scipy.special import gammaln

from .emulator import emulate

LOG2PI = np.log(2.0 * np.pi)


def model_vector(theta, model):
    """Concatenated model spectra [B, n] (spectrum-major)."""
    parts = []
    for net, is_log in zip(model["nets"], model["spec_log"]):
        y = emulate(theta, net)
        parts.append(10.0 ** y if is_log else y)
    return np.concatenate(parts, axis=1)


def loglike_diag(theta, model):
    """Diagonal-covariance Gaussian log-likelihood for a batch theta [B, d]."""
    m = model_vector(theta, model)
    r = (model["data"][None, :] - m) / model["sigma"][None, :]
    n = r.shape[1]
    chi2 = np.sum(r * r, axis=1)
    return -0.5 * chi2 - np.sum(np.log(model["sigma"])) - 0.5 * n * LOG2PI


def loglike_block(theta, model):
    """Per-multipole 3x3 block (TT, TE, EE) plus diagonal PP Gaussian log-likelihood."""
    m = model_vector(theta, model)
    n_ell = model["cov_blocks"].shape[0]
    r = model["data"][None, :] - m                      # [B, 4 n_ell]
    r3 = np.stack([r[:, 0:n_ell], r[:, n_ell:2 * n_ell], r[:, 2 * n_ell:3 * n_ell]], axis=2)
    L = np.linalg.cholesky(model["cov_blocks"])         # [n_ell, 3, 3]
    # whitened residual y_l = L_l^{-1} r_l for every walker and multipole
    y = np.linalg.solve(L[None, :, :, :], r3[..., None])[..., 0]
    rpp = r[:, 3 * n_ell:4 * n_ell] / model["sigma_pp"][None, :]
    chi2 = np.sum(y * y, axis=(1, 2)) + np.sum(rpp * rpp, axis=1)
    logdet_half = np.sum(np.log(np.diagonal(L, axis1=1, axis2=2))) + np.sum(np.log(model["sigma_pp"]))
    n = 4 * n_ell
    return -0.5 * chi2 - logdet_half - 0.5 * n * LOG2PI


def loglike_cv(theta, model):
    """Cosmic-variance-limited TT log-likelihood for a batch theta [B, d]."""
    C = 10.0 ** emulate(theta, model["nets"][0])          # [B, n_ell]
    ell = model["ell_min"] + np.arange(C.shape[1], dtype=np.float64)
    k = 2.0 * ell + 1.0
    x = k[None, :] * model["data"][None, :] / C
    log_f = (0.5 * k - 1.0) * np.log(x) - 0.5 * x - 0.5 * k * np.log(2.0) - gammaln(0.5 * k)
    return np.sum(np.log(k[None, :] / C) + log_f, axis=1)
