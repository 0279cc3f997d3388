"""Tomographic cosmic-shear likelihood, App. A of the paper (Eqs. A1-A4).

For every walker, on a grid of n_a scale factors evenly spaced from a = 1 to
a_min = 1/(1 + 5.02) (App. A, last paragraph):

1. Background (flat CPL dark energy, radiation neglected):
       E^2(a) = Om a^-3 + (1 - Om) a^{-3(1 + w0 + wa)} exp(-3 wa (1 - a)),
       Om = (omega_b + omega_cdm) / h^2,  c/H0 = 2997.92458 / h Mpc,
       chi(a) = int_a^1 (c/H0) / (a'^2 E(a')) da'   (Simpson per grid interval),
       J = d chi / d(-a) = (c/H0) / (a^2 E).
   Growth (the paper does not fix D; growth-index form, D(a=1) = 1):
       D(a) = exp(-int_a^1 Om(a')^0.55 da'/a'),  Om(a) = Om a^-3 / E^2.
2. Redshift distributions with photo-z shift n_i(z) -> n_i(z - Dz_i)
   (App. A, third item): Gaussians of mean zbar_i + Dz_i and width 0.1,
   zero at z = 0, normalised to unit integral over z by the trapezoid rule in a
   (dz = da / a^2).
3. Lensing window, Eq. (A3), split as
       W^g_i = 3/2 Om (H0/c)^2 (chi/a) [G0_i(chi) - chi G1_i(chi)],
       G0_i = int_chi^chiH n_i dchi',  G1_i = int_chi^chiH n_i / chi' dchi',
   both reverse cumulative trapezoids in a.
   NLA window, Eq. (A4), with n_i(chi) = n_i(z) (H0/c) E:
       W^I_i = -A_IA,i C1 rho_cr Om n_i(chi) / D,  C1 rho_cr = 5e-14 * 2.77536627e11.
4. Eq. (A1) sums four Limber integrals that all use P_dd, so the sum equals one
   Limber integral of the effective window W_i = W^g_i + W^I_i.
5. Matter power spectrum: the emulator gives log10 P at n_k log-spaced k and
   N_z redshift nodes; the table is carried to the z of every grid node in z,
   either ("cubic") by a not-a-knot cubic spline over nodes uniform on
   [0, z_max], or ("linear", App. B) by linear interpolation over nodes at
   scale factors evenly spaced from 1 to a_min.  With N_z = n_a the linear
   nodes are the integration nodes themselves, so the emulator is evaluated at
   every node (the paper's "full" likelihood); N_z about n_a / 10 is its
   interpolated likelihood.  A Catmull-Rom cubic in log10 k (linear ghost nodes
   at both ends) then evaluates it at k = (l + 1/2)/chi (Eq. A2).  P = 0
   outside [k_min, k_max] and at chi = 0.
6. Limber, Eq. (A2), trapezoid in a with the analytic Jacobian J, and the
   multiplicative bias (App. A, second item):
       C_ij(l) = (1 + m_i)(1 + m_j) sum_j q_j J_j W_i W_j / chi_j^2 P(k_lj, z_j).
7. Gaussian likelihood with a dense covariance (App. A, last paragraph):
       logL = -1/2 |L^{-1}(d - C)|^2 - sum log L_ii - n/2 log 2 pi.

Pinned by: the Einstein-de Sitter closed forms chi = 2 (c/H0)(1 - sqrt a),
D = a; scipy.integrate.quad distances for flat LCDM; Eqs. (A2)-(A4) integrated
directly in chi by adaptive quadrature for an EdS background and a power-law
P; exactness of the z-spline on cubics, of the linear z-interpolation on
lines, its one-sided error bound on concave tables, and the identity of the
N_z = n_a table with the emulator evaluated at every node; exactness of the
k-interpolation on quadratics; Limber integrals cut by the emulated k range
against quadrature over the chi range inside it; identical spectra for
identical bins; and
scipy.stats.multivariate_normal for the Gaussian.
"""
import numpy as np
from scipy.interpolate import CubicSpline

C_KM_S = 299792.458
C1_RHOCR = 5e-14 * 2.77536627e11
GROWTH_INDEX = 0.55
NZ_SIGMA = 0.1
LOG2PI = np.log(2.0 * np.pi)


# --------------------------------------------------------------------- grids
def a_grid(model):
    return np.linspace(1.0, model["a_min"], model["n_a"])


def linear_z(model):
    return model.get("z_interp", "cubic") == "linear"


def z_nodes(model):
    """Emulator redshift nodes: uniform in z ("cubic"), or at scale factors
    evenly spaced from 1 to a_min ("linear")."""
    if linear_z(model):
        return 1.0 / np.linspace(1.0, model["a_min"], model["n_z"]) - 1.0
    return np.linspace(0.0, 1.0 / model["a_min"] - 1.0, model["n_z"])


def ell_grid(model):
    return np.logspace(np.log10(model["ell_min"]), np.log10(model["ell_max"]), model["n_ell"])


def log10k_grid(model):
    return np.linspace(np.log10(model["k_min"]), np.log10(model["k_max"]), model["n_k"])


def trapezoid_weights(a):
    da = a[0] - a[1]
    q = np.full(a.size, da)
    q[0] = q[-1] = 0.5 * da
    return q


def pairs(nb):
    return [(i, j) for i in range(nb) for j in range(i, nb)]


# ------------------------------------------------------------ parameter map
def physical(theta, model):
    """Physical slots [B, 9 + 3 nb] from theta (fixed slots from model['pfix'])."""
    B = theta.shape[0]
    pidx, pfix = model["pidx"], model["pfix"]
    out = np.empty((B, pidx.size), dtype=theta.dtype)
    for s, ix in enumerate(pidx):
        out[:, s] = theta[:, ix] if ix >= 0 else pfix[s]
    return out


def unpack(phys, nb):
    cos = {k: phys[:, i:i + 1] for i, k in enumerate(
        ["omega_b", "omega_cdm", "h", "n_s", "lnAs", "w0", "wa", "c_min", "eta0"])}
    cos["A_IA"] = phys[:, 9:9 + nb]
    cos["Dz"] = phys[:, 9 + nb:9 + 2 * nb]
    cos["m"] = phys[:, 9 + 2 * nb:9 + 3 * nb]
    return cos


# --------------------------------------------------------------- background
def hubble_E(a, Om, w0, wa):
    E2 = Om * a ** -3.0 + (1.0 - Om) * a ** (-3.0 * (1.0 + w0 + wa)) * np.exp(-3.0 * wa * (1.0 - a))
    return np.sqrt(E2)


def background(a, Om, h, w0, wa):
    """chi [B, n_a], J = dchi/d(-a) [B, n_a], E [B, n_a], D [B, n_a].

    Om, h, w0, wa have shape [B, 1]; a is the descending grid.
    """
    c_H0 = C_KM_S / (100.0 * h)
    am = 0.5 * (a[:-1] + a[1:])
    da = a[:-1] - a[1:]

    def f(x):
        return c_H0 / (x * x * hubble_E(x, Om, w0, wa))

    def g(x):
        E = hubble_E(x, Om, w0, wa)
        return (Om * x ** -3.0 / (E * E)) ** GROWTH_INDEX / x

    fa, fm = f(a), f(am)
    inc = da / 6.0 * (fa[:, :-1] + 4.0 * fm + fa[:, 1:])
    zero = np.zeros((Om.shape[0], 1), dtype=inc.dtype)
    chi = np.concatenate([zero, np.cumsum(inc, axis=1)], axis=1)
    ga, gm = g(a), g(am)
    ginc = da / 6.0 * (ga[:, :-1] + 4.0 * gm + ga[:, 1:])
    lnD = np.concatenate([zero, -np.cumsum(ginc, axis=1)], axis=1)
    return chi, fa, hubble_E(a, Om, w0, wa), np.exp(lnD)


# --------------------------------------------------------------- n(z), windows
def redshift_distributions(a, zbar, Dz):
    """Normalised n_i(z_j) [B, nb, n_a]; zbar [nb], Dz [B, nb]."""
    z = 1.0 / a - 1.0
    mean = zbar[None, :, None] + Dz[:, :, None]
    n = np.exp(-((z[None, None, :] - mean) ** 2) / (2.0 * NZ_SIGMA ** 2))
    n[:, :, 0] = 0.0
    q = trapezoid_weights(a)
    norm = np.sum(q[None, None, :] * n / (a * a)[None, None, :], axis=2)
    return n / norm[:, :, None]


def reverse_cumtrapz(g, a):
    """G(j) = int_{a_min}^{a_j} g da by the trapezoid rule over nodes j..n_a-1."""
    da = a[0] - a[1]
    seg = 0.5 * da * (g[..., :-1] + g[..., 1:])
    rc = np.cumsum(seg[..., ::-1], axis=-1)[..., ::-1]
    return np.concatenate([rc, np.zeros(g.shape[:-1] + (1,), dtype=rc.dtype)], axis=-1)


def windows(a, n, chi, E, D, Om, h, A_IA):
    """Effective windows W_i = W^g_i + W^I_i [B, nb, n_a] (Eqs. A3, A4)."""
    H0_c = 100.0 * h / C_KM_S                                  # [B, 1]
    a2 = (a * a)[None, None, :]
    g0 = n / a2
    chi_safe = np.where(np.arange(a.size) == 0, 1.0, chi)       # chi_0 = 0
    g1 = n / (a2 * chi_safe[:, None, :])
    g1[:, :, 0] = 0.0                                            # n_i(0) = 0
    G0 = reverse_cumtrapz(g0, a)
    G1 = reverse_cumtrapz(g1, a)
    chi3 = chi[:, None, :]
    Wg = 1.5 * Om[:, :, None] * H0_c[:, :, None] ** 2 * (chi3 / a[None, None, :]) * (G0 - chi3 * G1)
    n_chi = n * H0_c[:, :, None] * E[:, None, :]
    WI = -A_IA[:, :, None] * C1_RHOCR * Om[:, :, None] * n_chi / D[:, None, :]
    return Wg + WI


# ------------------------------------------------------------ P(k, z) lookup
def emulator_table(cos, model):
    """log10 P at (z node, k mode): Y [B, N_z, n_k]."""
    from .emulator import emulate
    net = model["nets"][0]
    zn = z_nodes(model)
    B, Nz = cos["h"].shape[0], zn.size
    cols = [cos["omega_b"], cos["omega_cdm"], cos["h"], cos["n_s"], cos["lnAs"],
            cos["c_min"], cos["eta0"]]
    base = np.concatenate(cols, axis=1)                           # [B, 7]
    inp = np.concatenate([np.repeat(base, Nz, axis=0),
                          np.tile(zn, B)[:, None].astype(base.dtype)], axis=1)
    out_mu = np.tile(net["out_mu"], (B, 1))                       # [B*Nz, n_k]
    return emulate(inp, net, out_mu=out_mu).reshape(B, Nz, -1)


def interp_z(Y, model):
    """Y [B, N_z, n_k] at the nodes -> [B, n_a, n_k] at z_j = 1/a_j - 1: a
    not-a-knot cubic spline, or piecewise-linear interpolation, along z."""
    a = a_grid(model)
    zn = z_nodes(model)
    zj = np.minimum(1.0 / a - 1.0, zn[-1])
    if linear_z(model):
        out = np.empty((Y.shape[0], zj.size, Y.shape[2]), dtype=Y.dtype)
        for b in range(Y.shape[0]):
            for c in range(Y.shape[2]):
                out[b, :, c] = np.interp(zj, zn, Y[b, :, c])
        return out
    return CubicSpline(zn, Y, axis=1, bc_type="not-a-knot")(zj)


def interp_k(Yz, log10k, model):
    """Catmull-Rom in log10 k; Yz [B, n_a, n_k], log10k [B, n_ell, n_a] -> [B, n_ell, n_a]."""
    u0 = np.log10(model["k_min"])
    du = (np.log10(model["k_max"]) - u0) / (model["n_k"] - 1)
    nk = model["n_k"]
    s = (log10k - u0) / du
    i = np.clip(np.floor(s.real).astype(np.int64), 0, nk - 2)
    t = s - i
    ext = np.concatenate([2 * Yz[..., :1] - Yz[..., 1:2], Yz,
                          2 * Yz[..., -1:] - Yz[..., -2:-1]], axis=2)   # ghosts at both ends
    B, n_ell, n_a = log10k.shape
    bi = np.arange(B)[:, None, None]
    ji = np.arange(n_a)[None, None, :]
    pm1, p0, p1, p2 = (ext[bi, ji, i + 1 + o] for o in (-1, 0, 1, 2))
    m0 = 0.5 * (p1 - pm1)
    m1 = 0.5 * (p2 - p0)
    t2, t3 = t * t, t * t * t
    return (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + t) * m0 + (-2 * t3 + 3 * t2) * p1 + (t3 - t2) * m1


def power_at_limber_k(Y, chi, model):
    """P(k = (l + 1/2)/chi_j, z_j) [B, n_ell, n_a] from the node table Y;
    zero where k lies outside [k_min, k_max] and at chi = 0.  The zero rule is
    pinned by Limber integrals cut at both ends of the k range against direct
    quadrature over the chi range inside it."""
    ell = ell_grid(model)
    Yz = interp_z(Y, model)
    chi_safe = np.where(np.arange(chi.shape[1]) == 0, 1.0, chi)
    k = (ell[None, :, None] + 0.5) / chi_safe[:, None, :]
    inside = (k.real >= model["k_min"]) & (k.real <= model["k_max"])
    inside[:, :, 0] = False
    # points outside the emulated range are looked up at k_min and then zeroed
    log10k = np.where(inside, np.log10(k), np.log10(model["k_min"]))
    val = 10.0 ** interp_k(Yz, log10k, model)
    return np.where(inside, val, 0.0)


# ------------------------------------------------------------------ Limber
def limber(W, chi, J, P, m, a):
    """C [B, n_pairs * n_ell], pair-major with pairs (i <= j) in lexicographic order."""
    q = trapezoid_weights(a)
    chi_safe = np.where(np.arange(a.size) == 0, 1.0, chi)
    w = q[None, :] * J / (chi_safe * chi_safe)
    w[:, 0] = 0.0
    out = []
    for i, j in pairs(W.shape[1]):
        integrand = w[:, None, :] * W[:, i:i + 1, :] * W[:, j:j + 1, :] * P
        out.append((1.0 + m[:, i:i + 1]) * (1.0 + m[:, j:j + 1]) * np.sum(integrand, axis=2))
    return np.concatenate(out, axis=1)


def spectra(theta, model, Y=None):
    """Tomographic C_ij(l) [B, n_pairs * n_ell] and the intermediate stages."""
    nb = model["n_bins"]
    cos = unpack(physical(theta, model), nb)
    a = a_grid(model)
    Om = (cos["omega_b"] + cos["omega_cdm"]) / cos["h"] ** 2
    chi, J, E, D = background(a, Om, cos["h"], cos["w0"], cos["wa"])
    n = redshift_distributions(a, np.asarray(model["nz_mean"]), cos["Dz"])
    W = windows(a, n, chi, E, D, Om, cos["h"], cos["A_IA"])
    if Y is None:
        Y = emulator_table(cos, model)
    P = power_at_limber_k(Y, chi, model)
    C = limber(W, chi, J, P, cos["m"], a)
    return C, dict(chi=chi, J=J, E=E, D=D, n=n, W=W, Y=Y, P=P)


def gaussian_loglike(C, data, cov):
    """-1/2 |L^{-1}(d - C)|^2 - sum log L_ii - n/2 log 2 pi, L = chol(cov)."""
    from scipy.linalg import solve_triangular
    L = np.linalg.cholesky(cov)
    r = (data[None, :] - C).T
    y = solve_triangular(L, r, lower=True)
    chi2 = np.sum(y * y, axis=0)
    return -0.5 * chi2 - np.sum(np.log(np.diag(L))) - 0.5 * data.size * LOG2PI


def loglike(theta, model):
    C, _ = spectra(theta, model)
    return gaussian_loglike(C, model["data"], model["cov"])
