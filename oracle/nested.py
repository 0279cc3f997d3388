"""Nested slice sampling with k-deletion and the evidence accumulator.

Nested sampling (Sec. 2.1 of the paper; Skilling 2006) keeps n live points,
repeatedly discards the lowest-likelihood ones and replaces them by draws from
the prior constrained to L > L*, accumulating the evidence of Eq. (1) as a sum
of likelihoods times shrinking prior volumes.  The parallel form (Sec. 2.2)
deletes the k lowest points at once and evolves k replacements together; the
constrained draws are made by slice sampling (Neal 2003), which the paper
adopts in the GPU-vectorised "nested slice sampling" form.  The paper does not
print that algorithm's internals; the steps below are textbook hit-and-run
slice sampling in the unit hypercube:

one iteration (iteration index it >= 1)
  1. order the live points by (logL, index); the k lowest die, with live
     counts n, n-1, ..., n-k+1 at death; L* = the largest dead logL.
  2. directions: Sigma = sample covariance of the n live u before deletion,
     L_S = chol(Sigma + 1e-12 tr(Sigma)/d I).
  3. spawn: walker w starts at survivor floor(U (n-k)) of the ordered
     survivors (draw 0 of step 0).
  4. walk: n_inner steps; each draws v = L_S zeta (zeta standard normal, draws
     0..2d-1 by Box-Muller), r (draw 2d), brackets t_L = -r, t_R = 1 - r,
     steps each end out by 1 while the end point is inside (at most 10 times
     per end), then shrinks: t ~ U(t_L, t_R) (draws 2d+1, ...); accept if
     inside, else move the end on t's side to t.  A bracket narrower than
     1e-12 (or 200 rejected shrinks) is a stall and keeps the point.
     "inside" means u in [0,1]^d and logL(u) > L*; points outside the cube
     cost no likelihood evaluation.
  5. the k walkers replace the k dead points (same slots).
  6. stop when the live evidence share log(X mean_live L) - log(Z_dead +
     X mean_live L) falls below log(frac_remain).
finally the live points die in ascending order with live counts n, ..., 1.

Evidence (Skilling): log X_i = -sum_{m <= i} 1/n_m, w_i = X_{i-1} - X_i,
log Z = logsumexp(logL_i + log w_i) in float64, H = sum p_i (logL_i - log Z).
Error: std of log Z over R replicate shrinkage sequences
log t_m = log(1 - U_m)/n_m (Philox stream 1), and sqrt(H/n) as a cross-check.

Pinned by: the closed-form evidence of a Gaussian likelihood in the unit box;
a brute-force covariance for the direction factor and a record of which
points run() hands it;
the exact quadrature limit for L(X) = exp(-X/s); uniformity of slice draws
inside a ball constraint; agreement of k = 1 and k = n/2 runs.
"""
import numpy as np
from scipy.special import logsumexp

from .philox import uniforms, normals

MAX_EXPAND = 10
MAX_SHRINK = 200
STALL_WIDTH = 1e-12


def direction_cholesky(u):
    """Lower Cholesky of the live-point covariance plus a trace-scaled jitter.

    Sigma = sum_i (u_i - mean)(u_i - mean)^T / (n - 1) over the rows given
    (the n live points before deletion, as run() passes them); returns L with
    L L^T = Sigma + 1e-12 tr(Sigma)/d I.  Pinned by an explicit double loop
    over points and entries and by a singular point set that only the jitter
    makes factorisable."""
    d = u.shape[1]
    S = np.cov(u, rowvar=False, ddof=1).reshape(d, d)
    return np.linalg.cholesky(S + 1e-12 * np.trace(S) / d * np.eye(d))


def slice_step(loglike_u, u, logl, logl_star, L_dir, n_inner, seed, it, walker_ids=None):
    """Advance walkers u [k, d] by n_inner slice steps under logL > logl_star.

    Returns (u, logl, n_evals [k], n_stalls [k]).  All walkers advance in
    lockstep rounds with one batched likelihood call per round; because every
    draw is addressed by (walker, step, draw), the result does not depend on
    that schedule.
    """
    u = np.array(u, dtype=np.float64, copy=True)
    logl = np.array(logl, dtype=np.float64, copy=True)
    k, d = u.shape
    wid = np.arange(k) if walker_ids is None else np.asarray(walker_ids)
    n_evals = np.zeros(k, dtype=np.int64)
    n_stall = np.zeros(k, dtype=np.int64)

    def inside(x, active):
        ok = np.zeros(k, dtype=bool)
        ll = np.full(k, -np.inf)
        box = active & np.all((x >= 0.0) & (x <= 1.0), axis=1)
        if np.any(box):
            ll[box] = loglike_u(x[box])
            n_evals[box] += 1
            ok[box] = ll[box] > logl_star
        return ok, ll

    for s in range(1, n_inner + 1):
        U = uniforms(seed, 0, wid, s, it, np.arange(2 * d + 1))
        zeta = normals(U[:, 0:2 * d:2], U[:, 1:2 * d:2])
        v = zeta @ L_dir.T
        r = U[:, 2 * d]
        tL, tR = -r, 1.0 - r
        for sign in (-1.0, 1.0):
            active = np.ones(k, dtype=bool)
            for _ in range(MAX_EXPAND):
                t = tL if sign < 0 else tR
                ok, _ = inside(u + t[:, None] * v, active)
                grow = active & ok
                if sign < 0:
                    tL = np.where(grow, tL - 1.0, tL)
                else:
                    tR = np.where(grow, tR + 1.0, tR)
                active = grow
                if not np.any(active):
                    break
        active = np.ones(k, dtype=bool)
        q = 2 * d + 1
        for _ in range(MAX_SHRINK):
            Uq = uniforms(seed, 0, wid, s, it, [q])[:, 0]
            q += 1
            t = tL + Uq * (tR - tL)
            x = u + t[:, None] * v
            ok, ll = inside(x, active)
            acc = active & ok
            u[acc] = x[acc]
            logl[acc] = ll[acc]
            rej = active & ~ok
            tL = np.where(rej & (t < 0.0), t, tL)
            tR = np.where(rej & (t >= 0.0), t, tR)
            stall = rej & (tR - tL < STALL_WIDTH)
            n_stall += stall
            active = rej & ~stall
            if not np.any(active):
                break
        n_stall += active
    return u, logl, n_evals, n_stall


def evidence(dead_logl, dead_n):
    """log Z and H from the expected shrinkage log X_i = -sum 1/n_m."""
    dead_logl = np.asarray(dead_logl, dtype=np.float64)
    inv = 1.0 / np.asarray(dead_n, dtype=np.float64)
    logX = -np.cumsum(inv)
    logX_prev = np.concatenate([[0.0], logX[:-1]])
    logw = logX_prev + np.log(-np.expm1(-inv))
    logZ = logsumexp(dead_logl + logw)
    p = np.exp(dead_logl + logw - logZ)
    finite = np.isfinite(dead_logl)
    H = np.sum(p[finite] * (dead_logl[finite] - logZ))
    return logZ, H


def evidence_replicates(dead_logl, dead_n, seed, n_rep=1000, chunk=16):
    """log Z of n_rep replicate shrinkage sequences log t_m = log(1 - U_m)/n_m."""
    dead_logl = np.asarray(dead_logl, dtype=np.float64)
    n = np.asarray(dead_n, dtype=np.float64)
    M = dead_logl.size
    out = np.empty(n_rep)
    for r0 in range(0, n_rep, chunk):
        reps = np.arange(r0, min(n_rep, r0 + chunk))
        U = uniforms(seed, 1, reps[:, None], 0, 0, np.arange(M))[:, 0, :]   # [R, M]
        logt = np.log1p(-U) / n[None, :]
        logX = np.cumsum(logt, axis=1)
        logX_prev = np.concatenate([np.zeros((reps.size, 1)), logX[:, :-1]], axis=1)
        logw = logX_prev + np.log(-np.expm1(logt))
        out[reps] = logsumexp(dead_logl[None, :] + logw, axis=1)
    return out


def run(loglike_u, d, n_live, n_delete, n_inner, seed, frac_remain=1e-3, max_iter=100000,
        n_rep=1000, callback=None):
    """Nested slice sampling; returns a dict with logZ, sigma, H and the dead points."""
    n, k = n_live, n_delete
    u = uniforms(seed, 0, np.arange(n), 0, 0, np.arange(d))
    logl = loglike_u(u)
    n_evals_total = n
    dead_logl, dead_n, dead_u = [], [], []
    logX, logZ = 0.0, -np.inf
    n_stalls = 0
    it = 0
    while it < max_iter:
        it += 1
        order = np.lexsort((np.arange(n), logl))
        dead, surv = order[:k], order[k:]
        lstar = logl[dead[-1]]
        for j, idx in enumerate(dead):
            nj = n - j
            logw = logX + np.log(-np.expm1(-1.0 / nj))
            logZ = np.logaddexp(logZ, logl[idx] + logw)
            logX -= 1.0 / nj
            dead_logl.append(logl[idx]); dead_n.append(nj); dead_u.append(u[idx].copy())
        L_dir = direction_cholesky(u)
        pick = np.floor(uniforms(seed, 0, np.arange(k), 0, it, [0])[:, 0] * (n - k)).astype(np.int64)
        start = surv[pick]
        nu, nl, ne, ns = slice_step(loglike_u, u[start], logl[start], lstar, L_dir, n_inner, seed, it)
        u[dead] = nu
        logl[dead] = nl
        n_evals_total += int(ne.sum())
        n_stalls += int(ns.sum())
        live_term = logsumexp(logl) - np.log(n) + logX
        if callback is not None:
            callback(it, lstar, logZ, live_term)
        if live_term - np.logaddexp(logZ, live_term) < np.log(frac_remain):
            break
    order = np.lexsort((np.arange(n), logl))
    for j, idx in enumerate(order):
        dead_logl.append(logl[idx]); dead_n.append(n - j); dead_u.append(u[idx].copy())
    logZ, H = evidence(dead_logl, dead_n)
    reps = evidence_replicates(dead_logl, dead_n, seed, n_rep=n_rep) if n_rep else np.array([logZ])
    return dict(logZ=logZ, sigma=float(np.std(reps)), sigma_skilling=float(np.sqrt(max(H, 0.0) / n)),
                H=H, n_iter=it, n_evals=n_evals_total, n_stalls=n_stalls,
                dead_logl=np.array(dead_logl), dead_n=np.array(dead_n), dead_u=np.array(dead_u))
