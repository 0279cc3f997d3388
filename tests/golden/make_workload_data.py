"""Write the synthetic data vectors and covariances of the named workloads.

Run:  python tests/golden/make_workload_data.py
Calls only ``oracle/`` (the FP64 reference) and ``workloads/`` (seeded draws).
The paper's trained emulators, Planck mock and LSST-like covariance are not
published; these files stand in for them (shapes from the paper's Sec. 2.3-2.4
and App. A).

cmb6        data = m(theta_fid) + sigma eps; one scalar sigma chosen so that the
            median Fisher error of the six parameters is 0.02.
cmb4x2500   per-multipole 3x3 covariance Sigma_l = D_l R_l D_l over (TT, TE, EE),
            D = sqrt(2/(2l+1)) |C_fid| (TE: sqrt(C_TT C_EE)), R_l a seeded
            correlation; PP diagonal sqrt(2/(2l+1)) C_pp; data = C_fid + noise.
cmbtt_cv    cosmic-variance-limited TT: data Ch_l = C_l(theta_fid) X_l / (2l+1),
            X_l ~ chi^2 with 2l+1 degrees of freedom (seeded).
shear*      Gaussian (Knox) covariance per multipole,
            Cov[(ij),(kl)] = (Ch_ik Ch_jl + Ch_il Ch_jk) / ((2l+1) dl f_sky),
            Ch = C + delta sigma_e^2 / n_bar  (sigma_e = 0.3, n_bar = 6 arcmin^-2
            per bin, f_sky = 0.35), plus (0.01)^2 C_fid C_fid^T; data = C_fid + L eps.
shear_cmp   as shear10 with the data made at a seeded (w0, wa) point; shared by
            the LCDM (37 parameters) and w0wa (39 parameters) models.
shear_paper the paper's shape: 10 bins, 1025 nodes, n_bar = 3 arcmin^-2 per bin
            (30 in total); data made with the full likelihood (emulator at
            every node) at theta_fid (LCDM values); shared by shear_full,
            shear_interp and their LCDM variants.
Every file also stores theta_fid and fisher_sigma (Fisher 1-sigma per
parameter; prior width for parameters the data do not constrain).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W                                   # noqa: E402
from oracle import cmb, shear                           # noqa: E402
from oracle.emulator import emulate                     # noqa: E402
from oracle.likelihood import loglike                   # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def jacobian_cs(fn, theta):
    """Complex-step Jacobian of a vector function at one point [n_out, d]."""
    d = theta.size
    cols = []
    for k in range(d):
        tc = theta.astype(np.complex128)[None, :]
        tc[0, k] += 1e-30j
        cols.append(fn(tc)[0].imag / 1e-30)
    return np.stack(cols, axis=1)


def fisher_sigma(J_white, model, active):
    F = J_white.T @ J_white
    for i in range(model["d"]):
        if model["prior_kind"][i] == W.NORMAL:
            F[i, i] += 1.0 / model["prior_b"][i] ** 2
    sig = np.empty(model["d"])
    idx = np.nonzero(active)[0]
    Fi = np.linalg.inv(F[np.ix_(idx, idx)])
    sig[idx] = np.sqrt(np.diag(Fi))
    for i in np.nonzero(~active)[0]:
        sig[i] = 0.1 * (model["prior_b"][i] - model["prior_a"][i])
    return sig


def make_cmb6():
    m = W.structure("cmb6")
    th = W.fiducial_cmb()
    mf = cmb.model_vector(th[None, :], m)[0]
    J = jacobian_cs(lambda t: cmb.model_vector(t, m), th)
    s_unit = np.sqrt(np.diag(np.linalg.inv(J.T @ J)))
    sigma = 0.02 / np.median(s_unit)
    data = mf + sigma * W.noise(mf.size, tag=1)
    fs = s_unit * sigma
    np.savez_compressed(os.path.join(OUT, "workload_cmb6.npz"), data=data,
                        sigma=np.full(mf.size, sigma), theta_fid=th, fisher_sigma=fs)
    m.update(data=data, sigma=np.full(mf.size, sigma))
    print("cmb6: sigma", sigma, "logL(fid)", loglike(th[None, :], m))


def make_cmb_cv():
    m = W.structure("cmbtt_cv")
    th = W.fiducial_cmb()
    net = m["nets"][0]
    y = emulate(th[None, :], net)[0]
    ell = m["ell_min"] + np.arange(y.size, dtype=np.float64)
    k = 2.0 * ell + 1.0
    data = 10.0 ** y * np.random.default_rng([W.NOISE_SEED, 400]).chisquare(k) / k
    # Fisher matrix of the cosmic-variance likelihood: sum_l (k/2) dlnC/dtheta_i dlnC/dtheta_j
    J = np.log(10.0) * jacobian_cs(lambda t: emulate(t, net), th)
    F = (J * (0.5 * k)[:, None]).T @ J
    fs = np.sqrt(np.diag(np.linalg.inv(F)))
    np.savez_compressed(os.path.join(OUT, "workload_cmbtt_cv.npz"), data=data, theta_fid=th, fisher_sigma=fs)
    m.update(data=data)
    print("cmbtt_cv: fisher sigma", fs, "logL(fid)", loglike(th[None, :], m))


def make_cmb_block():
    m = W.structure("cmb4x2500")
    th = W.fiducial_cmb()
    mf = cmb.model_vector(th[None, :], m)[0]
    n = m["ell"].size
    tt, te, ee, pp = (mf[i * n:(i + 1) * n] for i in range(4))
    f = np.sqrt(2.0 / (2.0 * m["ell"] + 1.0))
    D = np.stack([f * np.abs(tt), f * np.sqrt(np.abs(tt * ee)), f * np.abs(ee)], axis=1)
    A = W.correlation_factors(n)
    S = A @ np.transpose(A, (0, 2, 1)) + 3.0 * np.eye(3)[None]
    dn = np.sqrt(np.einsum("lii->li", S))
    R = S / (dn[:, :, None] * dn[:, None, :])
    blocks = D[:, :, None] * R * D[:, None, :]
    sigma_pp = f * np.abs(pp)
    eps = W.noise(4 * n, tag=2).reshape(4, n)
    Lb = np.linalg.cholesky(blocks)
    r3 = np.einsum("lij,jl->il", Lb, eps[:3])
    data = mf + np.concatenate([r3[0], r3[1], r3[2], sigma_pp * eps[3]])
    # Fisher: whiten the Jacobian block by block
    J = jacobian_cs(lambda t: cmb.model_vector(t, m), th)
    J3 = np.stack([J[0:n], J[n:2 * n], J[2 * n:3 * n]], axis=1)          # [n, 3, d]
    Jw = np.linalg.solve(Lb, J3).reshape(3 * n, -1)
    Jw = np.concatenate([Jw, J[3 * n:] / sigma_pp[:, None]], axis=0)
    fs = fisher_sigma(Jw, m, np.ones(6, dtype=bool))
    np.savez_compressed(os.path.join(OUT, "workload_cmb4x2500.npz"), data=data, cov_blocks=blocks,
                        sigma_pp=sigma_pp, theta_fid=th, fisher_sigma=fs)
    m.update(data=data, cov_blocks=blocks, sigma_pp=sigma_pp)
    print("cmb4x2500: logL(fid)", loglike(th[None, :], m), "fisher", fs)


def knox_cov(C, model):
    nb, ne = model["n_bins"], model["n_ell"]
    ell = shear.ell_grid(model)
    rho = (model["ell_max"] / model["ell_min"]) ** (1.0 / (ne - 1))
    dl = ell * (np.sqrt(rho) - 1.0 / np.sqrt(rho))
    n_sr = 30.0 / nb * (60.0 * 180.0 / np.pi) ** 2        # 30 arcmin^-2 over the bins
    noise = 0.3 ** 2 / n_sr
    prs = shear.pairs(nb)
    Cm = np.zeros((ne, nb, nb))
    for p, (i, j) in enumerate(prs):
        Cm[:, i, j] = Cm[:, j, i] = C[p * ne:(p + 1) * ne]
    Cm += noise * np.eye(nb)[None]
    npair = len(prs)
    cov = np.zeros((npair * ne, npair * ne))
    for b in range(ne):
        norm = (2 * ell[b] + 1) * dl[b] * 0.35
        for p, (i, j) in enumerate(prs):
            for q, (k, l) in enumerate(prs):
                cov[p * ne + b, q * ne + b] = (Cm[b, i, k] * Cm[b, j, l] + Cm[b, i, l] * Cm[b, j, k]) / norm
    cov += 1e-4 * np.outer(C, C)
    return cov


def make_shear(name, structure_name, w0wa=None, tag=3):
    m = W.structure(structure_name)
    th = m["theta_fid"].copy()
    if w0wa is not None:
        th[m["names"].index("w0")], th[m["names"].index("wa")] = w0wa
    C = shear.spectra(th[None, :], m)[0][0]
    cov = knox_cov(C, m)
    L = np.linalg.cholesky(cov)
    data = C + L @ W.noise(C.size, tag=tag)
    J = jacobian_cs(lambda t: shear.spectra(t, m)[0], th)
    Jw = np.linalg.solve(L, J)
    active = np.array([not n.startswith("xi") for n in m["names"]])
    fs = fisher_sigma(Jw, m, active)
    np.savez_compressed(os.path.join(OUT, f"workload_{name}.npz"), data=data, cov=cov,
                        theta_fid=th, fisher_sigma=fs)
    m.update(data=data, cov=cov)
    print(name, "logL(fid)", loglike(th[None, :], m), "fisher", np.round(fs, 4))


if __name__ == "__main__":
    make_cmb6()
    make_cmb_block()
    make_cmb_cv()
    make_shear("shear64", "shear64", tag=3)
    make_shear("shear10", "shear10", tag=4)
    make_shear("shear_cmp", "shear10", w0wa=W.w0wa_point(), tag=5)
    make_shear("shear_paper", "shear_full", tag=6)
