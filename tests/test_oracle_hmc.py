"""Pins of the HMC oracle (oracle/hmc.py) against closed forms and
invariants that do not come from the oracle itself."""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import hmc


def gaussian_target(mu, sig):
    mu, sig = np.asarray(mu, float), np.asarray(sig, float)

    def target(theta):
        r = (theta - mu) / sig
        return -0.5 * np.sum(r * r, axis=1), -(r / sig)
    return target


def test_leapfrog_matches_closed_form_on_a_gaussian():
    """One leapfrog step on U = x^2 / (2 s^2) with inverse mass m is the linear
    map A = K(eps/2) D(eps) K(eps/2), det A = 1, tr A = 2 - eps^2 m / s^2 =
    2 cos(phi); hence A^L = sin(L phi)/sin(phi) A - sin((L-1) phi)/sin(phi) I."""
    rng = np.random.default_rng(0)
    d, L, eps = 3, 17, 0.21
    mu, sig = rng.normal(size=d), np.array([0.7, 1.3, 2.0])
    minv = np.array([0.5, 1.0, 3.0])
    th0 = mu + rng.normal(size=(2, d))
    p0 = rng.normal(size=(2, d))
    target = gaussian_target(mu, sig)
    _, g0 = target(th0)
    th, p, _, _, left = hmc.leapfrog(th0, p0, g0, minv, eps, L, target)
    assert not left.any()
    for i in range(d):
        k = eps / 2 / sig[i] ** 2
        A = np.array([[1 - eps * minv[i] * k, eps * minv[i]],
                      [-k * (2 - eps * minv[i] * k), 1 - eps * minv[i] * k]])
        phi = np.arccos(1 - eps ** 2 * minv[i] / (2 * sig[i] ** 2))
        AL = (np.sin(L * phi) * A - np.sin((L - 1) * phi) * np.eye(2)) / np.sin(phi)
        want = AL @ np.stack([th0[:, i] - mu[i], p0[:, i]])
        np.testing.assert_allclose(th[:, i] - mu[i], want[0], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(p[:, i], want[1], rtol=1e-11, atol=1e-12)


def quartic_target(theta):
    s = np.sum(theta * theta, axis=1)
    return -0.25 * s * s + 0.3 * theta[:, 0], -(s[:, None] * theta) + np.array([0.3, 0.0])


def test_leapfrog_is_time_reversible():
    rng = np.random.default_rng(1)
    th0 = rng.normal(size=(4, 2))
    p0 = rng.normal(size=(4, 2))
    minv = np.array([0.8, 1.2])
    _, g0 = quartic_target(th0)
    th1, p1, _, g1, _ = hmc.leapfrog(th0, p0, g0, minv, 0.05, 40, quartic_target)
    th2, p2, _, _, _ = hmc.leapfrog(th1, -p1, g1, minv, 0.05, 40, quartic_target)
    np.testing.assert_allclose(th2, th0, rtol=0, atol=1e-10)
    np.testing.assert_allclose(-p2, p0, rtol=0, atol=1e-10)


def test_energy_error_is_second_order():
    rng = np.random.default_rng(2)
    th0 = rng.normal(size=(8, 2))
    p0 = rng.normal(size=(8, 2))
    minv = np.array([1.0, 1.0])
    errs = []
    for eps, L in ((0.1, 20), (0.05, 40)):
        lp0, g0 = quartic_target(th0)
        _, p1, lp1, _, _ = hmc.leapfrog(th0, p0, g0, minv, eps, L, quartic_target)
        dH = (hmc.kinetic(p1, minv) - lp1) - (hmc.kinetic(p0, minv) - lp0)
        errs.append(np.max(np.abs(dH)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_samples_of_a_gaussian_have_its_moments():
    mu, sig = np.array([0.5, -1.0]), np.array([1.0, 2.0])
    out = hmc.run(None, np.tile(mu, (8, 1)), sig ** 2, n_iter=1500, n_leapfrog=7, step=0.4, seed=11,
                  target=gaussian_target(mu, sig))
    x = out["samples"][200:].reshape(-1, 2)
    assert out["accept"].mean() > 0.8
    # generous bounds: the chains are correlated, N_eff is well below len(x)
    assert np.all(np.abs(x.mean(axis=0) - mu) < 0.15 * sig)
    np.testing.assert_allclose(x.std(axis=0), sig, rtol=0.1)


def test_tiny_steps_are_always_accepted():
    mu, sig = np.zeros(3), np.ones(3)
    out = hmc.run(None, np.random.default_rng(3).normal(size=(5, 3)), np.ones(3), n_iter=20, n_leapfrog=3,
                  step=1e-4, seed=5, target=gaussian_target(mu, sig))
    assert out["accept"].all()


def test_momenta_follow_the_mass_matrix():
    minv = np.array([0.25, 4.0])
    p = np.concatenate([hmc.momenta(9, np.arange(4000), t, minv) for t in range(3)])
    assert np.all(np.abs(p.mean(axis=0)) < 4 * np.sqrt(1 / minv / len(p)))
    np.testing.assert_allclose(p.var(axis=0), 1 / minv, rtol=0.05)


def test_log_prior_is_the_normal_density_up_to_a_constant():
    m = W.structure("shear10")
    rng = np.random.default_rng(4)
    th = W.prior_draws(m, 5, tag=8)
    th2 = th + 0.01 * rng.normal(size=th.shape)
    lp, gp = hmc.log_prior(th, m)
    lp2, _ = hmc.log_prior(th2, m)
    nrm = m["prior_kind"] == 1
    ref = stats.norm.logpdf(th2[:, nrm], m["prior_a"][nrm], m["prior_b"][nrm]).sum(axis=1) - \
        stats.norm.logpdf(th[:, nrm], m["prior_a"][nrm], m["prior_b"][nrm]).sum(axis=1)
    np.testing.assert_allclose(lp2 - lp, ref, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(gp[:, nrm], -(th[:, nrm] - m["prior_a"][nrm]) / m["prior_b"][nrm] ** 2, rtol=1e-13)
    assert np.all(gp[:, ~nrm] == 0.0)


def test_trajectory_leaving_the_support_is_rejected():
    m = W.load_model("cmb6")
    target = hmc.make_target(m)
    th0 = np.array([[0.02, 0.5, 0.5, 0.5, 0.5, 0.5]])
    lp0, g0 = target(th0)
    p0 = np.zeros((1, 6))
    p0[0, 0] = -10.0                                   # one drift of 0.05 * 10 leaves [0, 1]
    _, _, lp, _, left = hmc.leapfrog(th0, p0, g0, np.ones(6), 0.05, 3, target)
    assert left[0]
    # drifts of 10 |p| leave the unit box unless every |p_i| < 0.1: every trajectory is rejected
    out = hmc.run(m, np.tile(th0, (3, 1)), np.ones(6), n_iter=2, n_leapfrog=1, step=10.0, seed=1, target=target)
    assert out["left"].all() and not out["accept"].any()
    np.testing.assert_array_equal(out["theta"], np.tile(th0, (3, 1)))
