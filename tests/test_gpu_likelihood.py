"""Parity of the HIP batched likelihood (ns_loglike_batch) with the FP64 oracle.

Tolerances (stated per precision form):
* FP64: |dlogL| <= 1e-6 for walkers in the posterior region (theta_fid plus
  Fisher-scaled Gaussian draws); for prior draws, where chi^2 reaches 1e6+,
  |dlogL| <= 1e-12 |logL| + 1e-6.
* FP32 / BF16X3: |dlogL| <= 1e-2 on posterior-region walkers (the bar for the
  reduced-precision forms).
* BF16 (operands rounded to 8 bits of mantissa, FP32 accumulation): misses
  that bar on the CMB workloads (|dlogL| ~ 0.1-1) and on shear10 / shear64;
  those cases only report the measured error (the test is marked skipped with
  it: nothing is certified for that form there).  The paper-shaped shear pair
  meets the 1e-2 bar in BF16 and is held to it.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.likelihood import loglike as oracle_loglike

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def built():
    from paper_2509_13307_amd import _capi
    _capi.lib()
    return True


_models = {}


def gpu_model(name):
    from paper_2509_13307_amd import Model
    if name not in _models:
        _models[name] = (W.load_model(name), Model(W.load_model(name)))
    return _models[name]


def post_scale(m):
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    return np.minimum(m["fisher_sigma"], 0.1 * width)


def run_gpu(model, theta, prec="fp64"):
    t = torch.tensor(theta, dtype=torch.float64, device=DEV)
    out = model.loglike(t, precision=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_fp64(ref, got, label):
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), label
    d = np.abs(ref[fin] - got[fin])
    tol = 1e-12 * np.abs(ref[fin]) + 1e-6
    say(f"{label}: max|dlogL| = {d.max():.3e}  max rel = {(d / np.abs(ref[fin])).max():.3e}")
    assert np.all(d <= tol), (label, d.max())


@pytest.mark.parametrize("name,B", [("cmb6", 1000), ("cmb4x2500", 300), ("cmbtt_cv", 300), ("shear10", 24),
                                    ("shear64", 12), ("shear_full", 5), ("shear_interp", 9)])
def test_fp64_posterior_and_prior(built, name, B):
    say(f"case fp64 {name} B={B}")
    m, g = gpu_model(name)
    th_post = W.posterior_draws(m["theta_fid"], post_scale(m), B, tag=1)
    th_prior = W.prior_draws(m, B + 7, tag=1)
    for label, th in (("posterior", th_post), ("prior", th_prior)):
        ref = oracle_loglike(th, m, chunk=64)
        got = run_gpu(g, th)
        check_fp64(ref, got, f"{name} {label}")


@pytest.mark.parametrize("name,B,sample", [("cmb4x2500", 4096, 40), ("cmbtt_cv", 4096, 40), ("shear64", 4096, 6),
                                           ("shear10", 16384, 6), ("shear_interp", 4096, 4), ("shear_full", 512, 3)])
def test_fp64_full_size_sampled(built, name, B, sample):
    say(f"case fp64 full {name} B={B}")
    m, g = gpu_model(name)
    th = W.prior_draws(m, B, tag=2)
    th[: B // 2] = W.posterior_draws(m["theta_fid"], post_scale(m), B // 2, tag=2)
    got = run_gpu(g, th)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([[0, 1, 127, 128, B // 2 - 1, B // 2, B - 2, B - 1],
                                    rng.integers(0, B, size=sample)]))
    ref = oracle_loglike(th[idx], m, chunk=64)
    check_fp64(ref, got[idx], f"{name} full B={B}")


@pytest.mark.parametrize("name,B,sample", [("cmb4x2500", 4096, 40), ("cmbtt_cv", 4096, 40), ("shear10", 4096, 6),
                                           ("shear_interp", 4096, 4)])
def test_bf16x3_full_size_sampled(built, name, B, sample):
    """The headline form at the benchmark's batch and launch shape: posterior-
    region walkers, sampled rows (ends of the batch, block boundaries and random
    rows) against the FP64 oracle, |dlogL| <= 1e-2."""
    say(f"case bf16x3 full {name} B={B}")
    m, g = gpu_model(name)
    th = W.posterior_draws(m["theta_fid"], post_scale(m), B, tag=18)
    got = run_gpu(g, th, "bf16x3")
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([[0, 1, 31, 32, 63, 64, B // 2, B - 2, B - 1], rng.integers(0, B, size=sample)]))
    ref = oracle_loglike(th[idx], m, chunk=64)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got[idx]))
    d = np.abs(got[idx][fin] - ref[fin])
    say(f"{name} bf16x3 B={B}: |dlogL| max {d.max():.3e} over {fin.sum()} sampled walkers")
    assert d.max() <= 1e-2


def test_edge_cases(built):
    say("case edge cmb6")
    m, g = gpu_model("cmb6")
    th = np.tile(m["theta_fid"], (5, 1))
    th[1, 2] = -0.01          # outside U(0,1)
    th[2, 5] = 1.0            # on the boundary: inside
    th[3, 0] = np.nan         # NaN -> NaN
    got = run_gpu(g, th)
    ref = oracle_loglike(th, m)
    assert got[1] == -np.inf and np.isnan(got[3])
    np.testing.assert_allclose(got[[0, 2, 4]], ref[[0, 2, 4]], rtol=1e-13, atol=1e-7)
    one = run_gpu(g, th[:1])
    assert abs(one[0] - ref[0]) < 1e-7
    # B = 0 is a no-op
    out = g.loglike(torch.empty(0, 6, dtype=torch.float64, device=DEV))
    assert out.numel() == 0
    # leading dimension > d
    wide = np.concatenate([th, np.zeros((5, 3))], axis=1)
    t = torch.tensor(wide, dtype=torch.float64, device=DEV)
    got2 = g.loglike(t).cpu().numpy()
    np.testing.assert_array_equal(np.isnan(got2), np.isnan(got))
    np.testing.assert_allclose(got2[[0, 2, 4]], got[[0, 2, 4]], rtol=0, atol=0)


def test_batch_and_permutation_invariance(built):
    say("case invariance cmb4x2500")
    m, g = gpu_model("cmb4x2500")
    th = W.posterior_draws(m["theta_fid"], post_scale(m), 257, tag=3)
    full = run_gpu(g, th, "bf16")
    perm = np.random.default_rng(1).permutation(257)
    again = run_gpu(g, th[perm], "bf16")
    np.testing.assert_array_equal(again, full[perm])
    single = run_gpu(g, th[100:101], "bf16")
    assert single[0] == full[100]


# Workloads on which plain BF16 misses the |dlogL| <= 1e-2 bar: their cases
# report the error and are skipped; every other (workload, form) is held to it.
BF16_BELOW_BAR = {"cmb6", "cmb4x2500", "cmbtt_cv", "shear10", "shear64"}


@pytest.mark.parametrize("name", ["cmb6", "cmb4x2500", "cmbtt_cv", "shear10", "shear64", "shear_full",
                                  "shear_interp"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_reduced_precision_forms(built, name, prec):
    say(f"case {prec} {name}")
    m, g = gpu_model(name)
    B = {"shear_full": 12, "shear_interp": 32}.get(name, 64 if name.startswith("shear") else 256)
    th = W.posterior_draws(m["theta_fid"], post_scale(m), B, tag=4)
    ref = oracle_loglike(th, m, chunk=64)
    got = run_gpu(g, th, prec)
    fin = np.isfinite(ref)                 # draws beyond a uniform prior bound give -inf on both sides
    assert np.array_equal(fin, np.isfinite(got))
    assert fin.sum() >= B // 2
    d = np.abs(got[fin] - ref[fin])
    say(f"{name} {prec}: |dlogL| max {d.max():.3e} median {np.median(d):.3e} over {fin.sum()} walkers")
    if prec == "bf16" and name in BF16_BELOW_BAR:
        pytest.skip(f"plain BF16 is below the 1e-2 bar on {name}: measured |dlogL| max {d.max():.3e} "
                    f"(reported only)")
    assert d.max() <= 1e-2


@pytest.mark.parametrize("name,B", [("cmb6", 300), ("cmb4x2500", 333), ("cmbtt_cv", 333), ("cmbtt_cv", 3100),
                                    ("shear10", 70), ("shear64", 9), ("shear_interp", 5)])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_fused_mlp_matches_layer_by_layer(built, name, B, prec, monkeypatch):
    """The one-kernel emulator gives bitwise the layer-by-layer result, with
    the autotuned launch shape and with each candidate shape pinned (the
    chi^2 staged after it).  For the one-network CMB models the default path
    adds the chi^2 in the emulator's epilogue (the diagonal one always, the
    cosmic-variance one from 3072 rows): its logL is the same for every
    launch shape, bitwise, and within 1e-12 relative of the staged chi^2
    (the same terms summed in another order)."""
    say(f"case fused {prec} {name}")
    from paper_2509_13307_amd import Model
    m = W.load_model(name)
    th = torch.tensor(W.prior_draws(m, B, tag=5), device=DEV)

    def run(env):
        for k in ("NSMI_NO_FUSED_MLP", "NSMI_FUSED_CFG", "NSMI_NO_FUSED_CHI2"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = Model(m)
        out = g.loglike(th, prec).cpu().numpy()
        report = g.tuning_report()
        g.close()
        return out, report

    ref, _ = run({"NSMI_NO_FUSED_MLP": "1"})
    got, report = run({"NSMI_NO_FUSED_CHI2": "1"})
    say(f"{name} {prec}: tuned {report}")
    np.testing.assert_array_equal(got, ref)
    width = m["nets"][0]["W"][0].shape[0]          # hidden width: 128 or 512
    ncfg = 10 if prec == "bf16" or width == 128 else 8
    for c in range(ncfg):
        got, _ = run({"NSMI_FUSED_CFG": str(c), "NSMI_NO_FUSED_CHI2": "1"})
        np.testing.assert_array_equal(got, ref)
    if name != "cmb6" and not (name == "cmbtt_cv" and B >= 3072):   # chi^2 in the epilogue from 3072 rows
        return
    fchi, report = run({})
    say(f"{name} {prec}: chi^2 in the epilogue, tuned {report}; "
        f"max |fused - staged| {np.max(np.abs(fchi - ref)):.3e}")
    assert any("chi2" in k for k in report)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(fchi))
    np.testing.assert_allclose(fchi[fin], ref[fin], rtol=1e-12, atol=1e-9)
    for c in range(ncfg):
        got, _ = run({"NSMI_FUSED_CFG": str(c)})
        np.testing.assert_array_equal(got, fchi)


@pytest.mark.parametrize("name,prec,B", [("cmbtt_cv", "fp64", 16384), ("shear_cmp_lcdm", "fp64", 8192),
                                         ("shear_cmp_lcdm", "bf16x3", 8192)])
def test_logl_does_not_depend_on_the_batch(built, name, prec, B):
    """A walker's logL is the same, bitwise, in a batch of 96 and in a batch of
    B: the launch shapes that the batch size selects (FP64 GEMM tiles of 32 or
    64 rows, dense-chi^2 tiles of 32 or 64 walkers, the autotuned one-kernel
    emulator shape) all keep every sum in the same order.  At 96 walkers the
    small tiles run, at B the large ones."""
    say(f"case batch independence {name} {prec} B={B}")
    from paper_2509_13307_amd import Model
    m = W.load_model(name)
    g = Model(m)
    th = torch.tensor(W.prior_draws(m, B, tag=11), device=DEV)
    big = g.loglike(th, prec).cpu().numpy()
    small = g.loglike(th[:96].contiguous(), prec).cpu().numpy()
    g.close()
    say(f"  {int(np.isfinite(small).sum())} of 96 finite; max |small - big| "
        f"{np.nanmax(np.abs(small - big[:96])):.3e}")
    np.testing.assert_array_equal(small, big[:96])


def test_tuning_cache_round_trip(built, tmp_path, monkeypatch):
    """The autotuner's choices go to the on-disk cache; a new model on the same
    GPU architecture starts with them (no timing runs, same results), and
    entries of another architecture, another candidate table, an out-of-range
    candidate or a malformed line are ignored."""
    say("case tuning cache")
    from paper_2509_13307_amd import Model
    path = tmp_path / "tune.txt"
    for k in ("NSMI_NO_FUSED_MLP", "NSMI_FUSED_CFG", "NSMI_NO_AUTOTUNE"):
        monkeypatch.delenv(k, raising=False)
    monkeypatch.setenv("NSMI_TUNE_CACHE", str(path))
    m = W.load_model("cmb6")
    th = torch.tensor(W.prior_draws(m, 300, tag=5), device=DEV)
    g = Model(m)
    assert g.tuning_report() == {}
    ref = g.loglike(th, "bf16x3").cpu().numpy()
    rep = g.tuning_report()
    g.close()
    lines = path.read_text().splitlines()
    assert len(rep) >= 1 and len(lines) == len(rep)
    f = lines[0].split()
    assert len(f) == 8
    bogus = [" ".join(["gfx000:other"] + f[1:3] + ["999"] + f[4:]),          # another architecture
             " ".join(f[:1] + ["0"] + f[2:3] + ["998"] + f[4:]),            # another candidate table
             " ".join(f[:3] + ["997"] + f[4:7] + ["99"]),                   # candidate out of range
             "not a cache line"]
    with open(path, "a") as fh:
        fh.write("\n".join(bogus) + "\n")
    g2 = Model(m)
    assert g2.tuning_report() == rep                    # loaded at creation, before any launch
    got = g2.loglike(th, "bf16x3").cpu().numpy()
    g2.close()
    np.testing.assert_array_equal(got, ref)
    assert len(path.read_text().splitlines()) == len(lines) + len(bogus)   # nothing tuned again
    monkeypatch.setenv("NSMI_TUNE_CACHE", "off")
    g3 = Model(m)
    assert g3.tuning_report() == {}
    g3.close()


@pytest.mark.parametrize("n_z", [4, 5, 7])
def test_fp64_shear_few_redshift_nodes(built, n_z):
    """Shear likelihood with the smallest redshift-node tables the spline
    supports (no or one interior unknown in the z system), against the oracle."""
    say(f"case fp64 shear n_z={n_z}")
    from paper_2509_13307_amd import Model
    base = W.load_model("shear10")
    m = W.shear_structure(n_z=n_z)
    for key in ("data", "cov", "theta_fid", "fisher_sigma"):
        m[key] = base[key]
    g = Model(m)
    th = W.posterior_draws(m["theta_fid"], post_scale(m), 9, tag=6)
    ref = oracle_loglike(th, m, chunk=16)
    got = run_gpu(g, th)
    g.close()
    check_fp64(ref, got, f"shear n_z={n_z}")


SHEAR_GRIDS = [
    # n_a, n_bins, n_ell, z_interp, n_z: ragged node chunks, 1-10 bins, 1-32 multipoles;
    # cubic n_z of 12, 40 and 90 take each z-spline kernel shape (columns in
    # registers up to 16 or 64 nodes, staged in LDS beyond)
    (300, 3, 25, "linear", 31),
    (3, 1, 1, "linear", 2),
    (700, 7, 32, "cubic", 12),
    (257, 10, 4, "linear", 257),
    (200, 4, 10, "cubic", 40),
    (520, 2, 6, "cubic", 90),
]


@pytest.mark.parametrize("n_a,n_bins,n_ell,z_interp,n_z", SHEAR_GRIDS)
def test_shear_grid_shapes(built, n_a, n_bins, n_ell, z_interp, n_z):
    """Shear likelihoods on grids away from the workloads' (node counts that
    leave a partial chunk, the smallest grid, 7 and 10 bins, up to 32
    multipoles, both z modes) with a small emulator, against the oracle; the
    data are the oracle's spectra at theta_fid with 5% noise and a diagonal
    covariance."""
    say(f"case shear grid n_a={n_a} bins={n_bins} n_ell={n_ell} {z_interp} n_z={n_z}")
    from paper_2509_13307_amd import Model
    from oracle import shear as oshear
    m = W.shear_structure(n_z=n_z, n_bins=n_bins, n_extra=0, hidden=(64, 64), n_a=n_a, n_k=60, n_ell=n_ell,
                          z_interp=z_interp)
    C = oshear.spectra(m["theta_fid"][None], m)[0][0]
    sig = 0.05 * np.abs(C) + 1e-3 * np.abs(C).max()
    m["data"] = C + sig * np.random.default_rng(n_a).normal(size=C.size)
    m["cov"] = np.diag(sig ** 2)
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    th = W.posterior_draws(m["theta_fid"], 0.02 * width, 7, tag=9)
    th[:, 2] = np.clip(th[:, 2], 0.65, None)
    ref = oracle_loglike(th, m, chunk=8)
    g = Model(m)
    got = run_gpu(g, th)
    check_fp64(ref, got, f"shear grid n_a={n_a}")
    fin = np.isfinite(ref)
    for prec in ("fp32", "bf16x3"):
        d = np.abs(run_gpu(g, th, prec)[fin] - ref[fin])
        say(f"  {prec}: max |dlogL| {d.max():.3e}")
        assert d.max() <= 1e-2
    g.close()


def test_cv_model_validation(built):
    """The cosmic-variance model rejects a non-positive observed spectrum, a
    non-integer first multipole and an emulator that does not output log10 C_l."""
    say("case cv validation")
    from paper_2509_13307_amd import Model
    from paper_2509_13307_amd._capi import NSError
    base = W.load_model("cmbtt_cv")
    for key, val in (("data", np.where(np.arange(base["data"].size) == 7, 0.0, base["data"])),
                     ("ell_min", 2.5), ("spec_log", [False])):
        bad = dict(base)
        bad[key] = val
        with pytest.raises(NSError):
            Model(bad)


def test_cv_loglike_shifts_with_a_constant_offset(built):
    """Scaling every emulated C_l by 10^c (an output shift c in log10 C_l) changes
    logL by -sum_l (k_l/2)(ln 10 c + Ch_l/C_l (10^-c - 1)): checked on the GPU
    against that closed form evaluated with the oracle's spectra."""
    say("case cv offset")
    from paper_2509_13307_amd import Model
    from oracle.emulator import emulate
    m = W.load_model("cmbtt_cv")
    th = W.posterior_draws(m["theta_fid"], post_scale(m), 9, tag=12)
    c = 0.013
    shifted = dict(m)
    net = dict(m["nets"][0])
    net["out_mu"] = np.asarray(net["out_mu"]) + c
    shifted["nets"] = [net]
    g0, g1 = Model(m), Model(shifted)
    l0, l1 = run_gpu(g0, th), run_gpu(g1, th)
    g0.close()
    g1.close()
    C = 10.0 ** emulate(th, m["nets"][0])
    k = 2.0 * (m["ell_min"] + np.arange(C.shape[1])) + 1.0
    want = -np.sum(0.5 * k * (np.log(10.0) * c + m["data"] / C * (10.0 ** -c - 1.0)), axis=1)
    say(f"cv offset: max |d| {np.abs((l1 - l0) - want).max():.3e}")
    np.testing.assert_allclose(l1 - l0, want, rtol=1e-9, atol=1e-6)


def test_full_and_interpolated_shear_share_their_data(built):
    """App. B's pair on the same data: the GPU's logL difference interpolated -
    full matches the oracle's walker by walker, and the interpolated spectra
    (oracle) sit below the full ones almost everywhere (concave log10 P in z)."""
    say("case shear full vs interp")
    from oracle import shear as oshear
    mf, gf = gpu_model("shear_full")
    mi, gi = gpu_model("shear_interp")
    th = W.posterior_draws(mf["theta_fid"], post_scale(mf), 6, tag=13)
    th[:, 2] = np.maximum(th[:, 2], 0.65)
    d_gpu = run_gpu(gi, th) - run_gpu(gf, th)
    d_ref = oracle_loglike(th, mi) - oracle_loglike(th, mf)
    say(f"logL interp - full: gpu {np.round(d_gpu, 6)} oracle {np.round(d_ref, 6)}")
    np.testing.assert_allclose(d_gpu, d_ref, rtol=0, atol=2e-6)
    Cf = oshear.spectra(th[:1], mf)[0][0]
    Ci = oshear.spectra(th[:1], mi)[0][0]
    assert np.mean(Ci < Cf) > 0.95




def test_fp64_one_kernel_narrow_emulator_matches_layer_by_layer(built, monkeypatch):
    """The one-kernel FP64 forward of the narrow cmb6 network (with the
    diagonal chi^2 in the same launch) gives bitwise the layer-by-layer
    GEMMs plus the separate chi^2 kernel, and its theory vector bitwise the
    layer-by-layer outputs; a batch with a partial last row tile, prior draws
    outside the support and batch 1 included."""
    say("case fp64 one-kernel narrow cmb6")
    from paper_2509_13307_amd import Model
    m = W.load_model("cmb6")
    th = W.prior_draws(m, 333, tag=21)
    th[:80] = W.posterior_draws(m["theta_fid"], post_scale(m), 80, tag=21)
    th[5, 1] = 1.2                              # outside U(0,1): -inf
    t = torch.tensor(th, device=DEV)
    outs = []
    for env in ({}, {"NSMI_NO_FUSED_MLP": "1"}):
        monkeypatch.delenv("NSMI_NO_FUSED_MLP", raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = Model(m)
        outs.append((g.loglike(t).cpu().numpy(), g.theory(t).cpu().numpy(), g.loglike(t[:1]).cpu().numpy()))
        g.close()
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    assert outs[0][0][5] == -np.inf
    check_fp64(oracle_loglike(th, m, chunk=64), outs[0][0], "cmb6 one-kernel fp64")


def test_model_made_before_torch_opens_the_gpu():
    """A process whose first GPU call is the library's (a Model made before any
    torch tensor on the GPU) still has a working torch device afterwards."""
    import os
    import subprocess
    say("case Model before torch's first GPU call (child process)")
    code = ("import torch, workloads as W\n"
            "from paper_2509_13307_amd import Model\n"
            "g = Model(W.gauss_structure(d=3, mu=[0.1, 0.5, 0.8], sigma=[0.05, 0.1, 0.08]))\n"
            "th = torch.tensor([[0.1, 0.5, 0.8], [0.2, 0.4, 0.7]], dtype=torch.float64, device='cuda:0')\n"
            "print(repr(g.loglike(th, 'fp64').tolist()))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=100)
    say(r.stdout.strip(), r.stderr.strip()[-400:])
    assert r.returncode == 0
    from paper_2509_13307_amd import Model
    g = Model(W.gauss_structure(d=3, mu=[0.1, 0.5, 0.8], sigma=[0.05, 0.1, 0.08]))
    th = torch.tensor([[0.1, 0.5, 0.8], [0.2, 0.4, 0.7]], dtype=torch.float64, device=DEV)
    assert r.stdout.strip().splitlines()[-1] == repr(g.loglike(th, "fp64").tolist())
    g.close()
