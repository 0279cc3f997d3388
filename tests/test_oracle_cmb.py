"""Pins of the Gaussian CMB-style likelihoods against scipy's multivariate normal."""
import numpy as np
from scipy.stats import multivariate_normal

import workloads as W
from oracle import cmb


def test_diag_matches_scipy():
    m = W.cmb_diag_structure(hidden=(8, 8), n_out=12)
    rng = np.random.default_rng(3)
    m["sigma"] = rng.uniform(0.01, 0.1, size=12)
    th = rng.uniform(size=(4, 6))
    m["data"] = cmb.model_vector(th[:1], m)[0] + m["sigma"] * rng.normal(size=12)
    got = cmb.loglike_diag(th, m)
    mv = cmb.model_vector(th, m)
    for b in range(4):
        want = multivariate_normal.logpdf(m["data"], mean=mv[b], cov=np.diag(m["sigma"] ** 2))
        np.testing.assert_allclose(got[b], want, rtol=1e-12)


def test_block_matches_scipy():
    m = W.cmb_block_structure(n_ell=5, hidden=(8, 8))
    rng = np.random.default_rng(4)
    th = rng.uniform(size=(3, 6))
    mv = cmb.model_vector(th, m)
    n = 5
    A = rng.normal(size=(n, 3, 3))
    blocks = A @ np.transpose(A, (0, 2, 1)) + 0.5 * np.eye(3)
    scale = np.abs(mv[0, :3 * n]).reshape(3, n).T          # [n, 3]
    blocks = blocks * scale[:, :, None] * scale[:, None, :]
    m["cov_blocks"] = blocks
    m["sigma_pp"] = 0.1 * np.abs(mv[0, 3 * n:])
    m["data"] = mv[0] * (1 + 0.05 * rng.normal(size=4 * n))
    full = np.zeros((4 * n, 4 * n))
    for l in range(n):
        idx = [l, n + l, 2 * n + l]
        full[np.ix_(idx, idx)] = blocks[l]
        full[3 * n + l, 3 * n + l] = m["sigma_pp"][l] ** 2
    got = cmb.loglike_block(th, m)
    # scipy's eigenvalue cut-off is absolute-scale sensitive: evaluate in units of
    # the marginal standard deviations and add back the Jacobian sum(log s)
    s = np.sqrt(np.diag(full))
    for b in range(3):
        want = multivariate_normal.logpdf(m["data"] / s, mean=mv[b] / s, cov=full / np.outer(s, s))
        np.testing.assert_allclose(got[b], want - np.sum(np.log(s)), rtol=1e-10)


def test_te_linear_other_spectra_exponentiated():
    m = W.cmb_block_structure(n_ell=4, hidden=(8,))
    th = np.full((1, 6), 0.4)
    mv = cmb.model_vector(th, m)[0]
    from oracle.emulator import emulate
    for s, is_log in enumerate(m["spec_log"]):
        y = emulate(th, m["nets"][s])[0]
        np.testing.assert_allclose(mv[4 * s:4 * s + 4], 10 ** y if is_log else y, rtol=1e-14)


# ------------------------------------------------------- cosmic-variance limit
def constant_cv_model(logc, data, ell_min):
    """CV model whose emulator returns log10 C = logc for every theta (zero last
    layer), so the likelihood is an explicit function of C_l."""
    import copy
    m = copy.deepcopy(W.structure("cmbtt_cv"))
    n = len(logc)
    net = m["nets"][0]
    net["W"][-1] = np.zeros((n, net["W"][-1].shape[1]))
    net["b"][-1] = np.zeros(n)
    net["out_mu"] = np.asarray(logc, dtype=np.float64)
    net["out_sigma"] = np.ones(n)
    m["data"] = np.asarray(data, dtype=np.float64)
    m["ell_min"] = ell_min
    return m


def test_cv_likelihood_is_the_chi2_density():
    from scipy import stats
    rng = np.random.default_rng(0)
    ell_min, n = 7, 40
    ell = ell_min + np.arange(n)
    k = 2.0 * ell + 1
    C = 10.0 ** rng.uniform(-10, -8, n)
    data = C * rng.chisquare(k) / k
    m = constant_cv_model(np.log10(C), data, ell_min)
    got = cmb.loglike_cv(np.full((2, 6), 0.5), m)
    want = np.sum(stats.chi2.logpdf(k * data / C, k) + np.log(k / C))
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_cv_likelihood_peaks_at_the_observed_spectrum():
    rng = np.random.default_rng(1)
    n = 30
    data = 10.0 ** rng.uniform(-10, -8, n)
    base = cmb.loglike_cv(np.full((1, 6), 0.5), constant_cv_model(np.log10(data), data, 2))[0]
    for j in (0, 11, 29):
        for dlog in (1e-3, -1e-3):
            logc = np.log10(data).copy()
            logc[j] += dlog
            assert cmb.loglike_cv(np.full((1, 6), 0.5), constant_cv_model(logc, data, 2))[0] < base


def test_cv_density_is_normalised():
    """Integral over the observed Ch_l of p(Ch_l | C_l) is 1 (single multipole)."""
    from scipy import integrate
    for ell in (2, 30, 400):
        C = 3e-9
        m = constant_cv_model([np.log10(C)], [C], ell)

        def p(ch):
            m["data"] = np.array([ch])
            return np.exp(cmb.loglike_cv(np.full((1, 6), 0.5), m)[0])
        total, _ = integrate.quad(p, 0.0, 20 * C, points=[C], limit=200)
        assert abs(total - 1.0) < 1e-8, (ell, total)
