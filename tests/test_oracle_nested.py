"""Pins of the oracle nested sampler and evidence accumulator."""
import numpy as np
from scipy.special import ndtr
from scipy.stats import kstest

from oracle import nested


def gauss_box(mu, sigma):
    mu, sigma = np.asarray(mu), np.asarray(sigma)

    def loglike_u(u):
        r = (u - mu) / sigma
        return -0.5 * np.sum(r * r, axis=1) - np.sum(np.log(sigma)) - 0.5 * mu.size * np.log(2 * np.pi)

    logZ = np.sum(np.log(ndtr((1 - mu) / sigma) - ndtr(-mu / sigma)))
    return loglike_u, logZ


def test_accumulator_quadrature_limit():
    """L(X) = exp(-X/s) with exact volumes X_i = exp(-i/n): Z -> s (1 - exp(-1/s))."""
    s = 0.1
    exact = np.log(s * (1 - np.exp(-1 / s)))
    errs = []
    for n in (1000, 4000):
        i = np.arange(1, 40 * n + 1)
        logZ, H = nested.evidence(-np.exp(-i / n) / s, np.full(i.size, n))
        errs.append(abs(logZ - exact))
    assert errs[0] < 3e-3
    assert 3.0 < errs[0] / errs[1] < 5.0           # first-order quadrature error, O(1/n)


def test_gaussian_box_closed_form_evidence():
    loglike_u, logZ = gauss_box([0.1, 0.5, 0.8], [0.05, 0.1, 0.08])
    res = nested.run(loglike_u, 3, 300, 150, 15, seed=11, n_rep=200)
    assert abs(res["logZ"] - logZ) < 3 * res["sigma"], (res["logZ"], logZ, res["sigma"])
    assert 0.5 < res["sigma"] / res["sigma_skilling"] < 2.0
    assert res["n_stalls"] == 0


def test_zscore_calibration_over_seeds():
    loglike_u, logZ = gauss_box([0.3, 0.6], [0.05, 0.07])
    z = []
    for seed in range(20):
        res = nested.run(loglike_u, 2, 100, 50, 10, seed=100 + seed, n_rep=100)
        z.append((res["logZ"] - logZ) / res["sigma"])
    z = np.array(z)
    assert abs(z.mean()) < 0.75, z
    assert 0.5 < z.std() < 1.6, z


def test_single_and_half_deletion_agree():
    """Deleting k = n/2 points per iteration introduces no approximation (Sec. 2.2)."""
    loglike_u, logZ = gauss_box([0.4, 0.7], [0.06, 0.05])
    r1 = nested.run(loglike_u, 2, 60, 1, 10, seed=21, n_rep=100)
    r2 = nested.run(loglike_u, 2, 60, 30, 10, seed=22, n_rep=100)
    tol = 3 * np.hypot(r1["sigma"], r2["sigma"])
    assert abs(r1["logZ"] - r2["logZ"]) < tol
    assert abs(r1["logZ"] - logZ) < 3 * r1["sigma"]


def test_slice_draws_uniform_in_ball():
    """Hit-and-run slice steps under a ball constraint leave (r/R)^d ~ U(0,1)."""
    d, R, k = 3, 0.3, 2000
    c = np.full(d, 0.5)

    def loglike_u(u):
        return -np.sum((u - c) ** 2, axis=1)

    u0 = np.tile(c, (k, 1))
    L = 0.2 * np.eye(d)
    u, logl, ne, ns = nested.slice_step(loglike_u, u0, np.zeros(k), -R * R, L, 5 * d, seed=3, it=1)
    r = np.sqrt(np.sum((u - c) ** 2, axis=1))
    assert np.all(r < R)
    assert kstest((r / R) ** d, "uniform").pvalue > 1e-3
    dirs = (u - c) / r[:, None]
    assert np.all(np.abs(dirs.mean(axis=0)) < 0.1)
    assert np.all(ns == 0) and np.all(ne >= 5 * d)


def test_replicates_reproducible_and_centered():
    loglike_u, _ = gauss_box([0.5, 0.5], [0.1, 0.1])
    res = nested.run(loglike_u, 2, 80, 40, 10, seed=5, n_rep=0)
    reps = nested.evidence_replicates(res["dead_logl"], res["dead_n"], seed=5, n_rep=300)
    again = nested.evidence_replicates(res["dead_logl"], res["dead_n"], seed=5, n_rep=300, chunk=7)
    assert np.array_equal(reps, again)
    assert abs(reps.mean() - res["logZ"]) < 0.5 * reps.std() + 0.05


def brute_covariance(u):
    """Sample covariance (1/(n-1)) by explicit loops over points and entries."""
    n, d = u.shape
    mean = [sum(u[i][c] for i in range(n)) / n for c in range(d)]
    S = np.zeros((d, d))
    for a in range(d):
        for b in range(d):
            S[a, b] = sum((u[i][a] - mean[a]) * (u[i][b] - mean[b]) for i in range(n)) / (n - 1)
    return S


def test_direction_cholesky_brute_force():
    """L L^T = Sigma + 1e-12 tr(Sigma)/d I, Sigma with the 1/(n-1) normalisation;
    L lower-triangular with a positive diagonal."""
    rng = np.random.default_rng(17)
    for n, d in ((7, 3), (40, 6)):
        u = rng.uniform(size=(n, d)) * rng.uniform(0.1, 1.0, size=d)
        S = brute_covariance(u)
        L = nested.direction_cholesky(u)
        assert np.array_equal(L, np.tril(L)) and np.all(np.diag(L) > 0)
        want = S + 1e-12 * np.trace(S) / d * np.eye(d)
        np.testing.assert_allclose(L @ L.T, want, rtol=1e-12, atol=1e-15)
        # the 1/n normalisation differs by n/(n-1): far outside the tolerance
        assert np.max(np.abs(S * (n - 1) / n - S)) > 1e-3 * np.max(np.abs(S))


def test_direction_cholesky_jitter_on_a_singular_set():
    """d points in d dimensions have a singular covariance: the trace-scaled
    jitter alone makes it factorisable, and L L^T - Sigma is that jitter."""
    rng = np.random.default_rng(18)
    d = 4
    u = rng.uniform(size=(d, d))
    S = brute_covariance(u)
    assert np.min(np.linalg.eigvalsh(S)) < 1e-14 * np.trace(S)
    L = nested.direction_cholesky(u)
    jit = 1e-12 * np.trace(S) / d
    np.testing.assert_allclose(np.diag(L @ L.T - S), jit, rtol=1e-2)
    off = (L @ L.T - S)[~np.eye(d, dtype=bool)]
    assert np.max(np.abs(off)) < 1e-2 * jit


def test_run_takes_directions_from_the_live_set_before_deletion(monkeypatch):
    """Each iteration's direction covariance is that of all n live points,
    the k about to be replaced included (iteration 1: the initial draws)."""
    from oracle.philox import uniforms
    seen = []
    orig = nested.direction_cholesky

    def spy(u):
        seen.append(np.array(u, copy=True))
        return orig(u)

    monkeypatch.setattr(nested, "direction_cholesky", spy)
    loglike_u, _ = gauss_box([0.4, 0.6], [0.1, 0.1])
    nested.run(loglike_u, 2, 20, 10, 4, seed=31, max_iter=2, n_rep=0)
    assert len(seen) == 2
    init = uniforms(31, 0, np.arange(20), 0, 0, np.arange(2))
    assert seen[0].shape == (20, 2)
    np.testing.assert_array_equal(seen[0], init)
