"""Pins of the prior transform (Table 1) and the support convention."""
import numpy as np
from scipy.stats import norm

import workloads as W
from oracle.likelihood import in_support, loglike, prior_transform


def test_prior_transform_matches_scipy_quantiles():
    m = W.structure("shear10")
    u = np.random.default_rng(10).uniform(size=(50, m["d"]))
    th = prior_transform(u, m)
    for i in range(m["d"]):
        a, b = m["prior_a"][i], m["prior_b"][i]
        want = a + (b - a) * u[:, i] if m["prior_kind"][i] == 0 else norm.ppf(u[:, i], loc=a, scale=b)
        np.testing.assert_allclose(th[:, i], want, rtol=1e-12, atol=1e-14)


def test_support_convention():
    m = W.load_model("cmb6")
    th = np.full((4, 6), 0.5)
    th[1, 0] = -1e-9
    th[2, 5] = 1.0
    th[3, 3] = np.nan
    ll = loglike(th, m)
    assert np.isfinite(ll[0]) and ll[1] == -np.inf and np.isfinite(ll[2]) and np.isnan(ll[3])
    assert list(in_support(th[:3], m)) == [True, False, True]
