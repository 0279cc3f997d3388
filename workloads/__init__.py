"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module draws random numbers and states configuration scalars; it holds
none of the likelihood or sampler arithmetic.  Everything here stands in for
assets the paper used but did not publish (trained emulator weights, mock data
vectors and survey covariances, Sec. 2.3-2.4 and App. A): the emulator
weights are seeded random draws, and the data vectors / covariances are read
from ``tests/golden/workload_*.npz`` (written by
``tests/golden/make_workload_data.py``).

Parameter order of the cosmic-shear models (Table 1 of the paper, five
tomographic bins):
    [omega_b, omega_cdm, h, n_s, ln10^10 A_s, w0, wa, c_min, eta0,
     A_IA_1..5, Dz_1..5, m_1..5, xi_1..15]
The fifteen ``xi`` are extra nuisance parameters with a U(0,1) prior that do
not enter the likelihood (39 parameters in total).  The LCDM variant fixes
w0 = -1, wa = 0 and has 37 parameters.
"""
from __future__ import annotations

import os
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(os.path.dirname(HERE), "tests", "golden")

# prior kinds
UNIFORM, NORMAL = 0, 1

# ---------------------------------------------------------------- shear layout
# physical slots, in the order the likelihood consumes them
SHEAR_COSMO = ["omega_b", "omega_cdm", "h", "n_s", "lnAs", "w0", "wa", "c_min", "eta0"]
# Table 1 of the paper: (kind, a, b, fiducial); a,b = lo,hi (uniform) or mu,sigma (normal)
TABLE1 = {
    "omega_b": (UNIFORM, 0.01875, 0.02625, 0.02242),
    "omega_cdm": (UNIFORM, 0.05, 0.255, 0.11933),
    "h": (UNIFORM, 0.64, 0.982, 0.6766),
    "n_s": (UNIFORM, 0.84, 1.1, 0.9665),
    "lnAs": (UNIFORM, 1.61, 3.91, 3.047),
    "w0": (UNIFORM, -1.5, -0.5, -1.0),
    "wa": (UNIFORM, -0.5, 0.5, 0.0),
    "c_min": (UNIFORM, 2.0, 4.0, 2.6),
    "eta0": (UNIFORM, 0.5, 1.0, 0.7),
    "A_IA": (UNIFORM, -6.0, 6.0, None),   # fiducial 1 - 0.1 i
    "Dz": (NORMAL, 0.0, 0.01, 0.0),
    "m": (NORMAL, 0.01, 0.02, 0.01),
    "xi": (UNIFORM, 0.0, 1.0, 0.5),
}
# emulator inputs of the P(k,z) network: five cosmological, two baryonic, z
SHEAR_EMU_INPUTS = ["omega_b", "omega_cdm", "h", "n_s", "lnAs", "c_min", "eta0"]

# number of physical slots of the shear likelihood for nb bins
def shear_n_phys(nb: int) -> int:
    return 9 + 3 * nb


# --------------------------------------------------------------- RNG helpers
def _rng(seed: int, *tag: int) -> np.random.Generator:
    return np.random.default_rng([seed, *tag])


MODEL_SEED = 13307
NOISE_SEED = 1
THETA_SEED = 2


def draw_mlp(dims, seed, tag, kind):
    """Seeded MLP parameters: a list of (W [n_out, n_in], b, beta, gamma).

    kind "small":  W, b, beta, gamma ~ N(0, 0.1^2)
    kind "wide":   W ~ N(0, 1/fan_in), b ~ N(0, 0.01^2), beta ~ N(1, 0.1^2),
                   gamma ~ N(0.3, 0.1^2)
    beta/gamma exist for hidden layers only (the last layer is affine).
    """
    rng = _rng(seed, tag)
    layers = []
    L = len(dims) - 1
    for l in range(L):
        n_in, n_out = dims[l], dims[l + 1]
        if kind == "small":
            W = rng.normal(0.0, 0.1, size=(n_out, n_in))
            b = rng.normal(0.0, 0.1, size=n_out)
            beta = rng.normal(0.0, 0.1, size=n_out)
            gamma = rng.normal(0.0, 0.1, size=n_out)
        else:
            W = rng.normal(0.0, 1.0 / np.sqrt(n_in), size=(n_out, n_in))
            b = rng.normal(0.0, 0.01, size=n_out)
            beta = rng.normal(1.0, 0.1, size=n_out)
            gamma = rng.normal(0.3, 0.1, size=n_out)
        if l == L - 1:
            beta = np.zeros(0)
            gamma = np.zeros(0)
        layers.append((W, b, beta, gamma))
    return layers


def net_dict(layers, in_shift, in_scale, out_mu, out_sigma):
    return {
        "W": [l[0] for l in layers],
        "b": [l[1] for l in layers],
        "beta": [l[2] for l in layers[:-1]],
        "gamma": [l[3] for l in layers[:-1]],
        "in_shift": np.asarray(in_shift, dtype=np.float64),
        "in_scale": np.asarray(in_scale, dtype=np.float64),
        "out_mu": np.asarray(out_mu, dtype=np.float64),
        "out_sigma": np.asarray(out_sigma, dtype=np.float64),
    }


# -------------------------------------------------------------------- configs
def cmb_cv_structure(n_ell=2500, hidden=(512, 512, 512, 512), seed=MODEL_SEED):
    """Temperature spectrum emulator 6 -> 4x512 -> n_ell (log10 C_l at l = 2, 3, ...)
    for the cosmic-variance-limited likelihood; output baseline as the TT
    network of the four-spectrum workload, sigma_out = 0.1."""
    d = 6
    ell = np.arange(2, 2 + n_ell, dtype=np.float64)
    tt = 1e-9 * (ell / 100.0) ** -1.0 * np.exp(-((ell / 1500.0) ** 2))
    layers = draw_mlp((d, *hidden, n_ell), seed, 20, "wide")
    net = net_dict(layers, np.full(d, 0.5), np.full(d, 0.5), np.log10(tt), np.full(n_ell, 0.1))
    return {
        "kind": "cmb_cv",
        "d": d,
        "prior_kind": np.zeros(d, dtype=np.int32),
        "prior_a": np.zeros(d),
        "prior_b": np.ones(d),
        "nets": [net],
        "spec_log": [True],
        "ell_min": 2,
    }



def cmb_diag_structure(hidden=(128, 128, 128), n_out=200, seed=MODEL_SEED):
    """Small CMB-style emulator: 6 -> 3x128 -> 200, weights N(0, 0.1^2)."""
    d = 6
    layers = draw_mlp((d, *hidden, n_out), seed, 1, "small")
    net = net_dict(layers, np.full(d, 0.5), np.full(d, 0.5), np.zeros(n_out), np.ones(n_out))
    return {
        "kind": "cmb_diag",
        "d": d,
        "prior_kind": np.zeros(d, dtype=np.int32),
        "prior_a": np.zeros(d),
        "prior_b": np.ones(d),
        "nets": [net],
        "spec_log": [False],
    }


def cmb_block_structure(n_ell=2500, hidden=(512, 512, 512, 512), seed=MODEL_SEED):
    """Four CMB spectrum emulators (TT, TE, EE, phiphi), 6 -> 4x512 -> n_ell.

    Output baselines (synthetic stand-ins for trained output normalisation):
      log10 C^TT = log10[1e-9  (l/100)^-1 exp(-(l/1500)^2)]
      log10 C^EE = log10[1e-10 (l/100)^-0.5 exp(-(l/1800)^2)]
      log10 C^pp = log10[1e-7  (l/100)^-3]
      C^TE       = 0.5 sqrt(C^TT C^EE) cos(l/80)  (linear output)
    sigma_out = 0.1 for the log spectra, 0.1 sqrt(C^TT C^EE) for TE.
    """
    d = 6
    ell = np.arange(2, 2 + n_ell, dtype=np.float64)
    tt = 1e-9 * (ell / 100.0) ** -1.0 * np.exp(-((ell / 1500.0) ** 2))
    ee = 1e-10 * (ell / 100.0) ** -0.5 * np.exp(-((ell / 1800.0) ** 2))
    pp = 1e-7 * (ell / 100.0) ** -3.0
    te_scale = np.sqrt(tt * ee)
    mus = [np.log10(tt), 0.5 * te_scale * np.cos(ell / 80.0), np.log10(ee), np.log10(pp)]
    sigs = [np.full(n_ell, 0.1), 0.1 * te_scale, np.full(n_ell, 0.1), np.full(n_ell, 0.1)]
    nets = []
    for s in range(4):
        layers = draw_mlp((d, *hidden, n_ell), seed, 10 + s, "wide")
        nets.append(net_dict(layers, np.full(d, 0.5), np.full(d, 0.5), mus[s], sigs[s]))
    return {
        "kind": "cmb_block",
        "d": d,
        "prior_kind": np.zeros(d, dtype=np.int32),
        "prior_a": np.zeros(d),
        "prior_b": np.ones(d),
        "nets": nets,
        "spec_log": [True, False, True, True],
        "ell": ell,
    }


def shear_structure(n_z=64, n_bins=5, n_extra=15, lcdm=False, hidden=(512, 512, 512, 512),
                    n_a=256, n_k=420, n_ell=20, seed=MODEL_SEED, z_interp="cubic", growth="power"):
    """Cosmic-shear likelihood structure (App. A of the paper, synthetic emulator).

    Emulator: 8 inputs (5 cosmological, c_min, eta0, z) -> hidden -> n_k values
    of log10 P(k, z_n) at the z nodes (uniform on [0, z_max] for z_interp
    "cubic"; at scale factors evenly spaced from 1 to a_min for "linear").
    Output normalisation mu(k, z) = log10 P_base(k) + g(z),
    P_base(k) = 2e4 (k/0.02) / (1 + (k/0.02)^2)^1.75 Mpc^3, sigma_out = 0.1,
    g(z) = -2 log10(1 + z) ("power"), or the concave stand-in
    g(z) = -2 (0.15 z + 0.06 z^2) ("concave": P falls as D^2 with
    log10 D = -(0.15 z + 0.06 z^2), so linear interpolation in z underestimates
    it, as App. B describes for the emulated spectrum).
    """
    a_min = 1.0 / (1.0 + 5.02)
    z_max = 1.0 / a_min - 1.0
    k_min, k_max = 1e-5, 50.0
    names, pk, pa, pb, fid = [], [], [], [], []

    def add(name, key, fidv=None):
        kd, a, b, f = TABLE1[key]
        names.append(name); pk.append(kd); pa.append(a); pb.append(b)
        fid.append(f if fidv is None else fidv)

    cosmo = [c for c in SHEAR_COSMO if not (lcdm and c in ("w0", "wa"))]
    for c in cosmo:
        add(c, c)
    for i in range(1, n_bins + 1):
        add(f"A_IA_{i}", "A_IA", 1.0 - 0.1 * i)
    for i in range(1, n_bins + 1):
        add(f"Dz_{i}", "Dz")
    for i in range(1, n_bins + 1):
        add(f"m_{i}", "m")
    for i in range(1, n_extra + 1):
        add(f"xi_{i}", "xi")
    d = len(names)
    # map physical slots -> theta index (-1 = fixed)
    phys_names = SHEAR_COSMO + [f"A_IA_{i}" for i in range(1, n_bins + 1)] \
        + [f"Dz_{i}" for i in range(1, n_bins + 1)] + [f"m_{i}" for i in range(1, n_bins + 1)]
    pidx = np.array([names.index(p) if p in names else -1 for p in phys_names], dtype=np.int32)
    pfix = np.zeros(len(phys_names))
    pfix[SHEAR_COSMO.index("w0")] = -1.0
    pfix[SHEAR_COSMO.index("wa")] = 0.0
    # emulator input normalisation: prior midpoint / half width; z: z_max/2
    in_shift = [0.5 * (TABLE1[c][1] + TABLE1[c][2]) for c in SHEAR_EMU_INPUTS] + [0.5 * z_max]
    in_scale = [0.5 * (TABLE1[c][2] - TABLE1[c][1]) for c in SHEAR_EMU_INPUTS] + [0.5 * z_max]
    k = np.logspace(np.log10(k_min), np.log10(k_max), n_k)
    if z_interp == "linear":
        z_nodes = 1.0 / np.linspace(1.0, a_min, n_z) - 1.0
    else:
        z_nodes = np.linspace(0.0, z_max, n_z)
    p_base = 2e4 * (k / 0.02) / (1.0 + (k / 0.02) ** 2) ** 1.75
    if growth == "concave":
        gz = -2.0 * (0.15 * z_nodes + 0.06 * z_nodes ** 2)
    else:
        gz = -2.0 * np.log10(1.0 + z_nodes)
    out_mu = np.log10(p_base)[None, :] + gz[:, None]
    layers = draw_mlp((8, *hidden, n_k), seed, 30, "wide")
    net = net_dict(layers, in_shift, in_scale, out_mu, np.full(n_k, 0.1))
    return {
        "kind": "shear",
        "d": d,
        "names": names,
        "prior_kind": np.array(pk, dtype=np.int32),
        "prior_a": np.array(pa, dtype=np.float64),
        "prior_b": np.array(pb, dtype=np.float64),
        "theta_fid": np.array(fid, dtype=np.float64),
        "nets": [net],
        "pidx": pidx,
        "pfix": pfix,
        "n_bins": n_bins,
        "nz_mean": np.linspace(0.3, 1.5, n_bins) if n_bins == 5 else np.linspace(0.2, 2.0, n_bins),
        "nz_sigma": 0.1,
        "n_a": n_a,
        "a_min": a_min,
        "n_z": n_z,
        "k_min": k_min,
        "k_max": k_max,
        "n_k": n_k,
        "ell_min": 20.0,
        "ell_max": 3000.0,
        "n_ell": n_ell,
        "z_interp": z_interp,
    }


def shear_paper_structure(variant="full", lcdm=False):
    """The paper's shear analysis shape (App. A): 10 tomographic bins (55
    spectra x 20 multipoles), 3 nuisances per bin (37 / 39 parameters), 1025
    scale-factor nodes; "full" evaluates the emulator at every node, "interp"
    at 103 nodes (10x coarser) with linear interpolation in z (App. B)."""
    n_z = {"full": 1025, "interp": 103}[variant]
    return shear_structure(n_z=n_z, n_bins=10, n_extra=0, lcdm=lcdm, n_a=1025, z_interp="linear",
                           growth="concave")


def gauss_structure(d=6, mu=None, sigma=None):
    """Diagonal Gaussian likelihood on the unit box; its evidence has a closed form."""
    mu = np.full(d, 0.5) if mu is None else np.asarray(mu, dtype=np.float64)
    sigma = np.full(d, 0.05) if sigma is None else np.asarray(sigma, dtype=np.float64)
    return {
        "kind": "gauss",
        "d": d,
        "prior_kind": np.zeros(d, dtype=np.int32),
        "prior_a": np.zeros(d),
        "prior_b": np.ones(d),
        "mu": mu,
        "sigma": sigma,
    }


CONFIGS = {
    "cmb6": dict(builder="cmb_diag", n_live=100, n_delete=50, inner_per_dim=5, frac_remain=1e-3),
    "cmb4x2500": dict(builder="cmb_block", batches=(4096, 65536)),
    "shear64": dict(builder="shear", n_z=64, batch=4096),
    "shear10": dict(builder="shear", n_z=10, batches=(1024, 4096, 16384)),
    "shear_lcdm_vs_w0wa": dict(builder="shear", n_z=10, n_live=1000, n_delete=500),
}


def structure(name: str):
    """Model structure (weights, priors, grid scalars) of a named workload."""
    if name == "cmb6":
        return cmb_diag_structure()
    if name == "cmb4x2500":
        return cmb_block_structure()
    if name == "cmbtt_cv":
        return cmb_cv_structure()
    if name == "shear64":
        return shear_structure(n_z=64)
    if name == "shear10":
        return shear_structure(n_z=10)
    if name == "shear10_lcdm":
        return shear_structure(n_z=10, lcdm=True)
    if name == "shear_cmp_w0wa":
        return shear_structure(n_z=10)
    if name == "shear_cmp_lcdm":
        return shear_structure(n_z=10, lcdm=True)
    if name in ("shear_full", "shear_interp", "shear_full_lcdm", "shear_interp_lcdm"):
        return shear_paper_structure(name.split("_")[1], lcdm=name.endswith("_lcdm"))
    raise KeyError(name)


def load_model(name: str):
    """Structure plus the stored synthetic data vector and covariance."""
    m = structure(name)
    data_name = name
    if name.startswith("shear_cmp"):
        data_name = "shear_cmp"
    elif name.startswith("shear_full") or name.startswith("shear_interp"):
        data_name = "shear_paper"
    path = os.path.join(GOLDEN, f"workload_{data_name}.npz")
    with np.load(path, allow_pickle=False) as z:
        for key in z.files:
            if name.endswith("_lcdm") and key in ("theta_fid", "fisher_sigma"):
                continue       # stored for the 39-parameter model; LCDM keeps its own
            m[key] = z[key]
    return m


# ---------------------------------------------------------------- theta draws
def prior_draws(model, n: int, seed: int = THETA_SEED, tag: int = 0):
    """n seeded draws of theta from the prior (throughput workloads)."""
    rng = _rng(seed, 100 + tag)
    th = np.empty((n, model["d"]))
    for i in range(model["d"]):
        a, b = model["prior_a"][i], model["prior_b"][i]
        if model["prior_kind"][i] == UNIFORM:
            th[:, i] = rng.uniform(a, b, size=n)
        else:
            th[:, i] = rng.normal(a, b, size=n)
    return th


def posterior_draws(center, scale, n: int, seed: int = THETA_SEED, tag: int = 0):
    """Seeded Gaussian draws around a point (posterior-region tolerance tests)."""
    rng = _rng(seed, 200 + tag)
    center = np.asarray(center, dtype=np.float64)
    return center[None, :] + np.asarray(scale)[None, :] * rng.normal(size=(n, center.size))


def noise(n: int, seed: int = NOISE_SEED, tag: int = 0):
    return _rng(seed, 300 + tag).normal(size=n)


def fiducial_cmb(d=6, seed=MODEL_SEED):
    return _rng(seed, 400).uniform(0.3, 0.7, size=d)


def w0wa_point(seed=MODEL_SEED):
    r = _rng(seed, 500)
    return r.uniform(-1.2, -0.8), r.uniform(-0.3, 0.3)


def correlation_factors(n_blocks, seed=MODEL_SEED):
    """Seeded 3x3 factors A for the per-multipole correlation R = norm(A A^T + 3 I)."""
    return _rng(seed, 600).normal(size=(n_blocks, 3, 3))


def eval_budgets(n: int, lo=1, hi=25, seed=MODEL_SEED):
    """Seeded per-walker likelihood-evaluation budgets U{lo..hi} (ragged bench)."""
    return _rng(seed, 700).integers(lo, hi + 1, size=n).astype(np.int32)
