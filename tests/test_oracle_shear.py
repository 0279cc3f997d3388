"""Pins of the oracle cosmic-shear likelihood (App. A of the paper)."""
import numpy as np
import pytest
from scipy import integrate
from scipy.stats import multivariate_normal

import workloads as W
from oracle import shear

C_KM_S = 299792.458


def eds_theta(model, h=0.7, A_IA=(0.5, -1.0), Dz=(0.02, -0.03), m=(0.01, -0.02)):
    """theta with Om = 1 (omega_b + omega_cdm = h^2), w0 = -1, wa = 0."""
    th = np.zeros(model["d"])
    names = model["names"]
    vals = dict(omega_b=0.02, omega_cdm=h * h - 0.02, h=h, n_s=0.96, lnAs=3.0, w0=-1.0, wa=0.0,
                c_min=2.6, eta0=0.7)
    for k, v in vals.items():
        th[names.index(k)] = v
    for i in range(model["n_bins"]):
        th[names.index(f"A_IA_{i + 1}")] = A_IA[i]
        th[names.index(f"Dz_{i + 1}")] = Dz[i]
        th[names.index(f"m_{i + 1}")] = m[i]
    return th[None, :]


def test_eds_background_closed_form():
    a = np.linspace(1.0, 1 / 6.02, 256)
    h = np.array([[0.7]])
    chi, J, E, D = shear.background(a, np.array([[1.0]]), h, np.array([[-1.0]]), np.array([[0.0]]))
    c_H0 = C_KM_S / 70.0
    np.testing.assert_allclose(chi[0], 2 * c_H0 * (1 - np.sqrt(a)), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(D[0], a, rtol=1e-9)   # Simpson error O(da^4)
    np.testing.assert_allclose(J[0], c_H0 / np.sqrt(a), rtol=1e-14)
    np.testing.assert_allclose(E[0], a ** -1.5, rtol=1e-14)


def test_lcdm_distance_matches_quad():
    a = np.linspace(1.0, 1 / 6.02, 256)
    Om, h = 0.31, 0.68
    chi = shear.background(a, np.array([[Om]]), np.array([[h]]), np.array([[-1.0]]), np.array([[0.0]]))[0][0]
    c_H0 = C_KM_S / (100 * h)
    for j in (10, 100, 255):
        z = 1 / a[j] - 1
        ref = c_H0 * integrate.quad(lambda x: 1 / np.sqrt(Om * (1 + x) ** 3 + 1 - Om), 0, z,
                                    epsabs=0, epsrel=1e-13)[0]
        np.testing.assert_allclose(chi[j], ref, rtol=1e-9)


def test_cpl_dark_energy_density_matches_continuity_equation():
    w0, wa, Om = -0.8, 0.3, 0.3
    for a in (0.9, 0.5, 0.2):
        # rho_DE(a)/rho_DE(1) = exp(3 int_a^1 (1 + w(a'))/a' da'),  w = w0 + wa (1 - a)
        rho = np.exp(3 * integrate.quad(lambda x: (1 + w0 + wa * (1 - x)) / x, a, 1, epsrel=1e-13)[0])
        E2 = Om * a ** -3 + (1 - Om) * rho
        got = shear.hubble_E(np.array([a]), Om, w0, wa)[0]
        np.testing.assert_allclose(got ** 2, E2, rtol=1e-11)


def test_growth_index_close_to_exact_growing_mode():
    """Growth-index D(a) against the exact linear growth ODE for flat LCDM (< 0.5%)."""
    from scipy.integrate import solve_ivp
    Om = 0.3
    a = np.linspace(1.0, 1 / 6.02, 256)
    D = shear.background(a, np.array([[Om]]), np.array([[0.7]]), np.array([[-1.0]]), np.array([[0.0]]))[3][0]

    def E(x):
        return np.sqrt(Om * x ** -3 + 1 - Om)

    def rhs(x, y):
        e = E(x)
        dlnE = (-1.5 * Om * x ** -4) / (e * e)        # dE/da / E
        return [y[1], -(3 / x + dlnE) * y[1] + 1.5 * Om / (x ** 5 * e * e) * y[0]]

    a0 = 1e-3
    sol = solve_ivp(rhs, (a0, 1.0), [a0, 1.0], rtol=1e-11, atol=1e-14, dense_output=True)
    Dex = sol.sol(a[::-1])[0][::-1]
    Dex = Dex / sol.sol(1.0)[0]
    np.testing.assert_allclose(D, Dex, rtol=5e-3)


def test_z_spline_exact_on_cubics():
    m = W.shear_structure(n_z=10, n_bins=2, n_extra=0, hidden=(4,), n_k=7)
    zn = shear.z_nodes(m)
    rng = np.random.default_rng(6)
    c = rng.normal(size=(4, 7))
    Y = (c[0] + c[1] * zn[:, None] + c[2] * zn[:, None] ** 2 + c[3] * zn[:, None] ** 3)[None]
    z = 1 / shear.a_grid(m) - 1
    want = c[0] + c[1] * z[:, None] + c[2] * z[:, None] ** 2 + c[3] * z[:, None] ** 3
    np.testing.assert_allclose(shear.interp_z(Y, m)[0], want, rtol=1e-11, atol=1e-11)


def test_k_interpolation_exact_on_quadratics_and_lines():
    m = W.shear_structure(n_z=4, n_bins=2, n_extra=0, hidden=(4,), n_k=30, n_a=5)
    u = shear.log10k_grid(m)
    rng = np.random.default_rng(7)
    q = rng.normal(size=3)
    Yz = np.broadcast_to(q[0] + q[1] * u + q[2] * u ** 2, (1, 5, 30)).copy()
    du = u[1] - u[0]
    x = rng.uniform(u[1], u[-2], size=(1, 6, 5))             # interior intervals only
    np.testing.assert_allclose(shear.interp_k(Yz, x, m), q[0] + q[1] * x + q[2] * x ** 2, rtol=1e-11, atol=1e-11)
    Yl = np.broadcast_to(q[0] + q[1] * u, (1, 5, 30)).copy()
    x = rng.uniform(u[0], u[-1], size=(1, 6, 5))
    x[0, 0, :2] = [u[0], u[-1]]
    np.testing.assert_allclose(shear.interp_k(Yl, x, m), q[0] + q[1] * x, rtol=1e-12, atol=1e-12)
    assert du > 0


def direct_limber(model, theta, A, n_pk, pairs_ells, k_range=None):
    """Eqs. (A2)-(A4) integrated in chi by adaptive quadrature (EdS, P = A k^n).
    With k_range = (k_lo, k_hi), P is zero where (l + 1/2)/chi leaves it, so
    the integral runs over chi in [(l + 1/2)/k_hi, (l + 1/2)/k_lo] only."""
    cos = shear.unpack(shear.physical(theta, model), model["n_bins"])
    h = float(cos["h"][0, 0])
    c_H0 = C_KM_S / (100 * h)
    z_max = 1 / model["a_min"] - 1
    chi_of_z = lambda z: 2 * c_H0 * (1 - (1 + z) ** -0.5)
    chiH = chi_of_z(z_max)
    mu = np.asarray(model["nz_mean"]) + cos["Dz"][0]
    norm = [integrate.quad(lambda z: np.exp(-(z - mu_i) ** 2 / 0.02), 0, z_max, epsrel=1e-13)[0] for mu_i in mu]

    def n_z(i, z):
        return np.exp(-(z - mu[i]) ** 2 / 0.02) / norm[i]

    def window(i, chi):
        a = (1 - chi / (2 * c_H0)) ** 2
        z = 1 / a - 1
        G = integrate.quad(lambda zp: n_z(i, zp) * (1 - chi / chi_of_z(zp)), z, z_max,
                           epsabs=0, epsrel=1e-12, limit=200)[0]
        Wg = 1.5 / c_H0 ** 2 * chi / a * G
        WI = -cos["A_IA"][0, i] * shear.C1_RHOCR * n_z(i, z) * (1 + z) ** 1.5 / c_H0 / a
        return Wg + WI

    out = []
    for (i, j), ell in pairs_ells:
        f = lambda chi: window(i, chi) * window(j, chi) / chi ** 2 * A * ((ell + 0.5) / chi) ** n_pk
        lo, hi = 1e-6, chiH
        if k_range is not None:
            lo, hi = max(lo, (ell + 0.5) / k_range[1]), min(hi, (ell + 0.5) / k_range[0])
        val = integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-10, limit=400)[0] if hi > lo else 0.0
        out.append((1 + cos["m"][0, i]) * (1 + cos["m"][0, j]) * val)
    return np.array(out)


@pytest.mark.parametrize("n_a_list", [(256, 511, 1021)])
def test_windows_and_limber_match_direct_integration(n_a_list):
    A, n_pk = 2e3, -1.3
    errs = []
    cases = [((0, 0), 20.0), ((0, 1), 300.0), ((1, 1), 3000.0)]
    ref = None
    for n_a in n_a_list:
        m = W.shear_structure(n_z=6, n_bins=2, n_extra=0, hidden=(4,), n_a=n_a, n_k=200)
        m["nz_mean"] = np.array([1.0, 1.5])
        m["k_min"], m["k_max"] = 1e-6, 1e4
        th = eds_theta(m)
        u = shear.log10k_grid(m)
        Y = np.broadcast_to(np.log10(A) + n_pk * u, (1, m["n_z"], m["n_k"])).copy()
        C = shear.spectra(th, m, Y=Y)[0][0]
        ells = shear.ell_grid(m)
        got = []
        for (i, j), ell in cases:
            p = shear.pairs(2).index((i, j))
            b = int(np.argmin(np.abs(ells - ell)))
            got.append(C[p * m["n_ell"] + b])
        if ref is None:
            ell_used = [shear.ell_grid(m)[int(np.argmin(np.abs(shear.ell_grid(m) - e)))] for _, e in cases]
            ref = direct_limber(m, th, A, n_pk, [(c[0], e) for c, e in zip(cases, ell_used)])
        errs.append(np.abs(np.array(got) / ref - 1))
    errs = np.array(errs)
    assert np.all(errs[0] < 2e-4), errs
    ratio = errs[0] / errs[1]
    assert np.all((ratio > 3.0) & (ratio < 5.0)), (errs, ratio)


def test_limber_power_is_zero_outside_the_emulated_k_range():
    """P = 0 where k = (l + 1/2)/chi leaves [k_min, k_max]: with a range that
    cuts the chi integral at both ends (k_max at small chi for every l, k_min
    at large chi for the lowest l) the spectra equal the direct integral over
    the chi range inside and are far from the uncut integral; where the whole
    range lies outside (l = 3000 needs chi > chi_H for k <= k_max) the
    spectrum is exactly zero."""
    A, n_pk = 2e3, -1.3
    k_range = (0.03, 0.5)
    m = W.shear_structure(n_z=6, n_bins=2, n_extra=0, hidden=(4,), n_a=1021, n_k=200)
    m["nz_mean"] = np.array([1.0, 1.5])
    m["k_min"], m["k_max"] = k_range
    th = eds_theta(m)
    u = shear.log10k_grid(m)
    Y = np.broadcast_to(np.log10(A) + n_pk * u, (1, m["n_z"], m["n_k"])).copy()
    C = shear.spectra(th, m, Y=Y)[0][0]
    ells = shear.ell_grid(m)
    cases = [((0, 0), 0), ((0, 1), 12), ((1, 1), 15)]
    got = np.array([C[shear.pairs(2).index(pq) * m["n_ell"] + b] for pq, b in cases])
    pe = [(pq, ells[b]) for pq, b in cases]
    cut = direct_limber(m, th, A, n_pk, pe, k_range=k_range)
    uncut = direct_limber(m, th, A, n_pk, pe)
    # the cut is a step in the integrand: first-order trapezoid error (measured
    # 1.4e-3 at most on this grid)
    np.testing.assert_allclose(got, cut, rtol=5e-3)
    assert np.all(np.abs(uncut / cut - 1) > 0.3), uncut / cut
    top = C[shear.pairs(2).index((0, 1)) * m["n_ell"] + m["n_ell"] - 1]
    chi_H = 2 * C_KM_S / 70.0 * (1 - np.sqrt(m["a_min"]))
    assert ells[-1] + 0.5 > k_range[1] * chi_H and top == 0.0


def test_multiplicative_bias_and_photoz_shift():
    m = W.shear_structure(n_z=6, n_bins=2, n_extra=0, hidden=(4,), n_k=50)
    m["nz_mean"] = np.array([0.8, 1.2])
    th0 = eds_theta(m, m=(0.0, 0.0), Dz=(0.0, 0.0))
    Y = np.random.default_rng(8).normal(size=(1, 6, 50)) * 0.1 + 2
    C0 = shear.spectra(th0, m, Y=Y)[0][0].reshape(3, -1)
    th1 = eds_theta(m, m=(0.05, -0.1), Dz=(0.0, 0.0))
    C1 = shear.spectra(th1, m, Y=Y)[0][0].reshape(3, -1)
    np.testing.assert_allclose(C1[0], 1.05 ** 2 * C0[0], rtol=1e-13)
    np.testing.assert_allclose(C1[1], 1.05 * 0.9 * C0[1], rtol=1e-13)
    np.testing.assert_allclose(C1[2], 0.9 ** 2 * C0[2], rtol=1e-13)
    # photo-z shift: bin means moved by Dz equal a model with shifted nominal means
    th2 = eds_theta(m, m=(0.0, 0.0), Dz=(0.03, -0.02))
    C2 = shear.spectra(th2, m, Y=Y)[0][0]
    m2 = dict(m, nz_mean=np.array([0.83, 1.18]))
    np.testing.assert_allclose(C2, shear.spectra(th0, m2, Y=Y)[0][0], rtol=1e-12)


def test_dense_gaussian_matches_scipy():
    rng = np.random.default_rng(9)
    n = 12
    A = rng.normal(size=(n, n))
    s = 10 ** rng.uniform(-11, -9, size=n)
    cov = (A @ A.T + n * np.eye(n)) * np.outer(s, s)
    C = s * rng.normal(size=(3, n))
    data = s * rng.normal(size=n)
    got = shear.gaussian_loglike(C, data, cov)
    for b in range(3):
        want = multivariate_normal.logpdf(data / s, mean=C[b] / s, cov=cov / np.outer(s, s)) - np.sum(np.log(s))
        np.testing.assert_allclose(got[b], want, rtol=1e-11)


def test_extra_nuisances_do_not_enter():
    m = W.load_model("shear10")
    th = np.repeat(m["theta_fid"][None], 2, axis=0)
    th[1, -15:] = np.linspace(0.01, 0.99, 15)
    from oracle.likelihood import loglike
    ll = loglike(th, m)
    assert ll[0] == ll[1]


def small_linear(n_z, n_a=41, n_bins=2):
    return W.shear_structure(n_z=n_z, n_bins=n_bins, n_extra=0, hidden=(8,), n_k=30, n_a=n_a,
                             z_interp="linear")


def test_linear_z_full_grid_is_the_emulator_at_every_node():
    """N_z = n_a: the table carried to the integration nodes equals the emulator
    evaluated directly at z_j = (1 - a_j)/a_j of every node (App. B's full
    likelihood), built here from the a-grid without the node tables."""
    from oracle.emulator import emulate
    m = small_linear(n_z=41)
    th = W.posterior_draws(m["theta_fid"], np.full(m["d"], 0.01), 2, tag=40)
    cos = shear.unpack(shear.physical(th, m), m["n_bins"])
    Yz = shear.interp_z(shear.emulator_table(cos, m), m)
    a = 1.0 - np.arange(41) * ((1.0 - m["a_min"]) / 40.0)
    z = (1.0 - a) / a
    base = np.concatenate([cos[k] for k in ("omega_b", "omega_cdm", "h", "n_s", "lnAs", "c_min", "eta0")], axis=1)
    for b in range(2):
        inp = np.concatenate([np.repeat(base[b:b + 1], 41, axis=0), z[:, None]], axis=1)
        want = emulate(inp, m["nets"][0], out_mu=m["nets"][0]["out_mu"])
        np.testing.assert_allclose(Yz[b], want, rtol=1e-12, atol=1e-12)


def test_linear_z_exact_on_lines():
    m = small_linear(n_z=5)
    zn = shear.z_nodes(m)
    assert zn[0] == 0.0 and np.isclose(zn[-1], 5.02) and np.all(np.diff(1.0 / (1.0 + zn)) < 0)
    rng = np.random.default_rng(41)
    c = rng.normal(size=(2, 30))
    Y = (c[0] + c[1] * zn[:, None])[None]
    z = 1.0 / shear.a_grid(m) - 1.0
    np.testing.assert_allclose(shear.interp_z(Y, m)[0], c[0] + c[1] * z[:, None], rtol=1e-12, atol=1e-12)


def test_linear_z_error_on_concave_tables_is_one_sided_and_bounded():
    """For a concave f the chord lies below f: 0 <= f - interp <= h^2/8 max|f''|
    on every interval (h its width), equality at the nodes."""
    m = small_linear(n_z=9, n_a=101)
    zn = shear.z_nodes(m)
    f = lambda z: -2.0 * (0.22 * z + 0.02 * z ** 2) + np.log10(1.0 - z / 9.0)
    Y = np.broadcast_to(f(zn)[:, None], (1, 9, 30)).copy()
    z = np.minimum(1.0 / shear.a_grid(m) - 1.0, zn[-1])
    err = f(z) - shear.interp_z(Y, m)[0, :, 0]
    n = np.clip(np.searchsorted(zn, z, side="right") - 1, 0, 7)
    h = zn[n + 1] - zn[n]
    f2 = 0.08 + 1.0 / (np.log(10.0) * (9.0 - zn[n + 1]) ** 2)      # max |f''| on the interval
    assert np.all(err >= -1e-15)
    assert np.all(err <= h * h / 8.0 * f2 + 1e-15)
    assert err.max() > 1e-3                                      # the bias is really there
    assert abs(err[0]) < 1e-15 and abs(err[-1]) < 1e-14


def test_identical_bins_give_identical_spectra():
    """Ten bins with one n(z) and equal nuisances: all 55 spectra coincide
    (a wrong pair index, bin offset or window term would split them)."""
    m = W.shear_structure(n_z=6, n_bins=10, n_extra=0, hidden=(4,), n_a=64, n_k=40)
    m["nz_mean"] = np.full(10, 0.9)
    th = m["theta_fid"][None].copy()
    for i in range(1, 11):
        th[0, m["names"].index(f"A_IA_{i}")] = 0.5
        th[0, m["names"].index(f"Dz_{i}")] = 0.0
        th[0, m["names"].index(f"m_{i}")] = 0.01
    rng = np.random.default_rng(42)
    Y = rng.normal(size=(1, 6, 40)) * 0.05 + 2.0
    C = shear.spectra(th, m, Y=Y)[0][0].reshape(55, -1)
    assert C.shape == (55, m["n_ell"]) and np.all(C[0] != 0)
    np.testing.assert_allclose(C, np.broadcast_to(C[0], C.shape), rtol=1e-13)
    # one bin shifted: exactly the ten spectra involving it change
    th2 = th.copy()
    th2[0, m["names"].index("Dz_4")] = 0.05
    C2 = shear.spectra(th2, m, Y=Y)[0][0].reshape(55, -1)
    changed = np.any(C2 != C, axis=1)
    involve = np.array([3 in p for p in shear.pairs(10)])
    np.testing.assert_array_equal(changed, involve)


def test_paper_shaped_structures():
    for lcdm, d in ((False, 39), (True, 37)):
        for v in ("full", "interp"):
            m = W.shear_paper_structure(v, lcdm=lcdm)
            assert m["d"] == d and m["n_bins"] == 10 and m["n_a"] == 1025
            assert m["n_z"] == (1025 if v == "full" else 103) and m["z_interp"] == "linear"
            assert len(shear.pairs(10)) * m["n_ell"] == 1100
            assert m["nets"][0]["out_mu"].shape == (m["n_z"], 420)
