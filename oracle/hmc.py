"""Hamiltonian Monte Carlo on the likelihood's gradient.  Test infrastructure:
the plain FP64 reference that the HIP sampler is checked against; nothing in
the product imports it.

The paper's likelihoods are differentiable (their gradients come from the
same emulator, Sec. 2.2), which lets a gradient-based sampler run beside
nested sampling on the same posterior.  This is the textbook HMC of Duane et
al. (1987) / Neal (2011): target

    log pi(theta) = logL(theta) + log prior(theta),

the prior of Table 1 (normal priors contribute -(theta - mu)^2 / (2 sigma^2),
uniform priors nothing inside their box; outside the support log pi = -inf),
momenta p ~ N(0, M) with a diagonal inverse mass m (M = diag(1/m)),
Hamiltonian H = -log pi(theta) + sum_i m_i p_i^2 / 2, and L leapfrog
(Stormer-Verlet) steps of size eps per trajectory:

    p <- p + eps/2 grad log pi(theta)
    repeat L times:  theta <- theta + eps m p;  reflect;
                     p <- p + h grad log pi(theta)
                     with h = eps, except h = eps/2 after the last drift,

then a Metropolis accept with probability min(1, exp(H0 - H1)).  Uniform-prior
coordinates are kept in their box by reflection (Neal 2011, Sec. 5.5.1): a
drift that ends beyond a wall b is mirrored to b - (theta - b) and that
momentum component changes sign, repeated until inside; reflection conserves
volume, kinetic energy and time reversibility, so the chain stays exact.  A
trajectory that still reaches log pi = -inf (or needs more than 64 bounces in
one drift) is rejected.

Random numbers (philox.py): stream 2 draws the momenta, z_i = Box-Muller of
draws 2i, 2i+1 of the sequence (chain, 0, iteration), p_i = z_i / sqrt(m_i);
stream 3 draws the accept uniform u, draw 0 of (chain, 0, iteration); accept
iff log u < H0 - H1.

Every update below is a separately rounded FP64 operation in the order
written, and every sum over parameters runs in parameter order, so that the
HIP sampler (same draws, same order, no contraction) replays a run.

Pinned by: the exact leapfrog map of a Gaussian target (a linear map known in
closed form), time reversibility of the integrator (also through
reflections), its O(eps^2) energy error, the moments of samples of a Gaussian
target, and uniform samples of a flat target in a box.
"""
import numpy as np

from .gradient import loglike_grad
from .philox import normals, uniforms

STREAM_MOMENTUM = 2
STREAM_ACCEPT = 3


def log_prior(theta, model):
    """(log prior [B], its gradient [B, d]) inside the support (normal
    priors only; uniform priors contribute 0), accumulated in parameter order."""
    theta = np.asarray(theta, dtype=np.float64)
    B, d = theta.shape
    lp = np.zeros(B)
    gp = np.zeros((B, d))
    for i in range(d):
        if model["prior_kind"][i] == 1:
            mu, sig = model["prior_a"][i], model["prior_b"][i]
            r = (theta[:, i] - mu) / sig
            lp = lp - 0.5 * (r * r)
            gp[:, i] = -(r / sig)
    return lp, gp


def make_target(model, grad_fn=None):
    """target(theta [B, d]) -> (log pi [B], grad log pi [B, d]); -inf and a zero
    gradient outside the support."""
    grad_fn = grad_fn or (lambda th: loglike_grad(th, model))

    def target(theta):
        logl, g = grad_fn(theta)
        lp, gp = log_prior(theta, model)
        logpi = logl + lp
        grad = g + gp
        bad = ~np.isfinite(logl)
        logpi[bad] = -np.inf
        grad[bad] = 0.0
        return logpi, grad
    return target


def kinetic(p, minv):
    """sum_i m_i p_i^2 / 2, accumulated in parameter order."""
    k = np.zeros(p.shape[0])
    for i in range(p.shape[1]):
        k = k + (minv[i] * p[:, i]) * p[:, i]
    return 0.5 * k


MAX_BOUNCES = 64


def reflect(theta, p, lo, hi):
    """Mirror coordinates beyond lo / hi back inside, flipping their momenta,
    one wall per pass; returns (theta, p, stuck [B])."""
    for _ in range(MAX_BOUNCES):
        up = theta > hi[None, :]
        dn = ~up & (theta < lo[None, :])
        if not (up.any() or dn.any()):
            break
        theta = np.where(up, hi[None, :] - (theta - hi[None, :]), theta)
        theta = np.where(dn, lo[None, :] - (theta - lo[None, :]), theta)
        p = np.where(up | dn, -p, p)
    stuck = np.any((theta > hi[None, :]) | (theta < lo[None, :]), axis=1)
    return theta, p, stuck


def box(model, d):
    """(lo, hi) walls of the uniform-prior coordinates; +-inf elsewhere."""
    if model is None:
        return np.full(d, -np.inf), np.full(d, np.inf)
    uni = np.asarray(model["prior_kind"]) == 0
    return (np.where(uni, model["prior_a"], -np.inf).astype(np.float64),
            np.where(uni, model["prior_b"], np.inf).astype(np.float64))


def leapfrog(theta, p, grad, minv, step, n_leapfrog, target, lo=None, hi=None):
    """L leapfrog steps from (theta, p) with grad = grad log pi(theta),
    reflecting at the walls lo / hi.  Returns (theta, p, log pi, grad, rejected [B])."""
    theta = np.array(theta, dtype=np.float64, copy=True)
    p = np.array(p, dtype=np.float64, copy=True)
    d = theta.shape[1]
    lo = np.full(d, -np.inf) if lo is None else lo
    hi = np.full(d, np.inf) if hi is None else hi
    half = 0.5 * step
    p = p + half * grad
    left = np.zeros(theta.shape[0], dtype=bool)
    logpi = None
    for l in range(n_leapfrog):
        theta = theta + step * (minv[None, :] * p)
        theta, p, stuck = reflect(theta, p, lo, hi)
        logpi, grad = target(theta)
        left |= stuck | ~np.isfinite(logpi)
        p = p + (half if l == n_leapfrog - 1 else step) * grad
    return theta, p, logpi, grad, left


def momenta(seed, chains, it, minv):
    d = minv.shape[0]
    U = uniforms(seed, STREAM_MOMENTUM, chains, 0, it, np.arange(2 * d))
    z = normals(U[:, 0::2], U[:, 1::2])
    return z / np.sqrt(minv)[None, :]


def run(model, theta0, minv, n_iter, n_leapfrog, step, seed, target=None):
    """C chains from theta0 [C, d] for n_iter trajectories.

    Returns dict(samples [n_iter, C, d], logp [n_iter, C], accept [n_iter, C],
    left [n_iter, C], theta [C, d]); samples[t] is the state after trajectory t.
    """
    target = target or make_target(model)
    theta = np.array(theta0, dtype=np.float64, copy=True)
    minv = np.asarray(minv, dtype=np.float64)
    C, d = theta.shape
    lo, hi = box(model, d)
    chains = np.arange(C)
    logpi, grad = target(theta)
    samples = np.zeros((n_iter, C, d))
    logp = np.zeros((n_iter, C))
    acc = np.zeros((n_iter, C), dtype=bool)
    lefts = np.zeros((n_iter, C), dtype=bool)
    for t in range(n_iter):
        p = momenta(seed, chains, t, minv)
        H0 = kinetic(p, minv) - logpi
        th1, p1, lp1, g1, left = leapfrog(theta, p, grad, minv, step, n_leapfrog, target, lo, hi)
        H1 = kinetic(p1, minv) - lp1
        u = uniforms(seed, STREAM_ACCEPT, chains, 0, t, [0])[:, 0]
        with np.errstate(invalid="ignore", divide="ignore"):
            ok = ~left & (np.log(u) < H0 - H1)
        theta[ok] = th1[ok]
        logpi[ok] = lp1[ok]
        grad[ok] = g1[ok]
        samples[t] = theta
        logp[t] = logpi
        acc[t] = ok
        lefts[t] = left
    return dict(samples=samples, logp=logp, accept=acc, left=lefts, theta=theta)
