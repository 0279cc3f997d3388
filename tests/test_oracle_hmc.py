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


def test_reflection_keeps_chains_in_the_box():
    """cmb6 chains started 0.02 from the theta_0 = 0 wall with posterior-scale
    steps: the pull toward the mode carries unwalled trajectories beyond
    theta_0 = 1; with the walls they are reflected, none is rejected for it."""
    m = W.load_model("cmb6")
    target = hmc.make_target(m)
    th0 = np.tile(m["theta_fid"], (8, 1))
    th0[:, 0] = 0.02
    minv = np.full(6, 0.02 ** 2)
    lo, hi = hmc.box(m, 6)
    p0 = hmc.momenta(4, np.arange(8), 0, minv)
    _, g0 = target(th0)
    th, _, lp, _, left = hmc.leapfrog(th0, p0, g0, minv, 0.5, 6, target, lo, hi)
    free, _, _, _, _ = hmc.leapfrog(th0, p0, g0, minv, 0.5, 6, target)        # no walls
    assert np.any((free < 0) | (free > 1))                                  # unwalled trajectories leave the box ...
    assert not left.any() and np.all(np.isfinite(lp))                      # ... and is reflected, not rejected
    assert np.all((th >= 0.0) & (th <= 1.0))


def test_reflection_is_reversible_and_conserves_kinetic_energy():
    rng = np.random.default_rng(5)
    th0 = 0.2 * rng.normal(size=(4, 2))
    p0 = 3.0 * rng.normal(size=(4, 2))
    minv = np.array([0.8, 1.2])
    lo, hi = np.array([-0.4, -np.inf]), np.array([0.3, np.inf])
    th0[:, 0] = np.clip(th0[:, 0], -0.39, 0.29)
    flat = lambda th: (np.zeros(th.shape[0]), np.zeros_like(th))
    th1, p1, _, _, left = hmc.leapfrog(th0, p0, np.zeros_like(th0), minv, 0.2, 25, flat, lo, hi)
    assert not left.any()
    assert np.all((th1[:, 0] >= lo[0]) & (th1[:, 0] <= hi[0]))
    np.testing.assert_allclose(np.abs(p1), np.abs(p0), rtol=0, atol=0)     # flat target: only sign flips
    np.testing.assert_allclose(hmc.kinetic(p1, minv), hmc.kinetic(p0, minv), rtol=1e-15)
    _, g1 = quartic_target(th1)
    t1, q1, _, g1, _ = hmc.leapfrog(th0, p0, quartic_target(th0)[1], minv, 0.02, 60, quartic_target, lo, hi)
    t2, q2, _, _, _ = hmc.leapfrog(t1, -q1, g1, minv, 0.02, 60, quartic_target, lo, hi)
    np.testing.assert_allclose(t2, th0, rtol=0, atol=1e-9)
    np.testing.assert_allclose(-q2, p0, rtol=0, atol=1e-9)


def test_flat_target_in_a_box_gives_uniform_samples():
    """A flat log pi in [0, 1]^2: H is conserved exactly (reflections only flip
    momenta), every trajectory is accepted and the chains sample U(0, 1)^2."""
    flat = lambda th: (np.zeros(th.shape[0]), np.zeros_like(th))
    model = {"prior_kind": np.zeros(2, dtype=np.int32), "prior_a": np.zeros(2), "prior_b": np.ones(2)}
    out = hmc.run(model, np.full((16, 2), 0.5), np.ones(2), n_iter=400, n_leapfrog=5, step=0.37, seed=2,
                  target=flat)
    assert out["accept"].all()
    x = out["samples"][50:].reshape(-1, 2)
    assert np.all((x >= 0) & (x <= 1))
    assert np.all(np.abs(x.mean(axis=0) - 0.5) < 0.02)
    np.testing.assert_allclose(x.var(axis=0), 1 / 12, rtol=0.06)
