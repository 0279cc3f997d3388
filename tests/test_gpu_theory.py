"""Element-by-element parity of the theory vector (ns_theory_batch) with the
FP64 oracle: the CMB spectra after the output transform (Sec. 2.4) and the
tomographic shear spectra after the multiplicative bias (Eqs. (A1)-(A4)),
entry by entry, at every workload shape.

Tolerances, per entry, with s the largest |C| of the same spectrum (CMB) or
of the same pair (shear) in that row, which sets the scale of entries that
cancel towards zero (C^TE, cross-bin spectra with intrinsic alignments):
* FP64: |dC| <= 1e-11 (|C| + s).  Every stage runs in FP64 and differs from
  the oracle only in the order of its sums (blocked GEMMs over K <= 512,
  chunked sums over <= 2048 scale-factor nodes, the 10^y and the spline
  weights), a few thousand roundings of 1.1e-16 at most: ~1e-13.
* BF16X3 and FP32: |dC| <= 3e-5 (|C| + s), about 2 x 2^-16.  A split-BF16
  product drops only the lo x lo term, at most 2^-16 of the product, FP32
  rounds at 2^-24, and both accumulate in FP32; over the layers of the
  emulator these errors average rather than add in one direction, so the
  output y and the spectra (10^y, or sums of 10^y in the shear case) stay
  within a small multiple of 2^-16 of their scale.  The 1e-2 logL bar of
  these forms is checked on the likelihood itself.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.cmb import model_vector as oracle_cmb_vector
from oracle.shear import spectra as oracle_shear_spectra

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_models = {}


def gpu_model(name):
    from paper_2509_13307_amd import Model
    if name not in _models:
        _models[name] = (W.load_model(name), Model(W.load_model(name)))
    return _models[name]


def post_scale(m):
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    return np.minimum(m["fisher_sigma"], 0.1 * width)


def oracle_theory(theta, m):
    if m["kind"] == "shear":
        out = []
        for i in range(0, theta.shape[0], 16):
            out.append(oracle_shear_spectra(theta[i:i + 16], m)[0])
        return np.concatenate(out, axis=0)
    return oracle_cmb_vector(theta, m)


def segments(m):
    """Lengths of the blocks that share a scale: one spectrum (CMB) or one
    tomographic pair (shear)."""
    if m["kind"] == "shear":
        return int(m["n_ell"])
    return int(np.asarray(m["data"]).size // len(m["nets"]))


def segment_scale(ref, seg):
    B, n = ref.shape
    s = np.abs(ref).reshape(B, n // seg, seg).max(axis=2, keepdims=True)
    return np.broadcast_to(s, (B, n // seg, seg)).reshape(B, n)


def check(ref, got, m, prec, label):
    assert ref.shape == got.shape, label
    assert np.all(np.isfinite(got)), label
    s = segment_scale(ref, segments(m))
    d = np.abs(got - ref)
    tol = (1e-11 if prec == "fp64" else 3e-5) * (np.abs(ref) + s)
    worst = (d / tol).max()
    say(f"{label}: max|dC|/(|C|+s) = {(d / (np.abs(ref) + s)).max():.3e}  worst/tol = {worst:.3f}")
    assert worst <= 1.0, (label, worst)


def run_theory(g, th, prec):
    t = torch.tensor(th, dtype=torch.float64, device=DEV)
    out = g.theory(t, precision=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = [("cmb6", 200), ("cmb4x2500", 37), ("cmbtt_cv", 37), ("shear10", 19), ("shear64", 7),
         ("shear_full", 3), ("shear_interp", 5)]


@pytest.mark.parametrize("name,B", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_theory_matches_oracle(name, B, prec):
    say(f"case theory {prec} {name} B={B}")
    m, g = gpu_model(name)
    th = W.posterior_draws(m["theta_fid"], post_scale(m), B, tag=21)
    if prec == "fp64":   # prior draws too: the whole support of the emulators
        th = np.concatenate([th, W.prior_draws(m, B // 2 + 1, tag=21)])
    got = run_theory(g, th, prec)
    check(oracle_theory(th, m), got, m, prec, f"{name} {prec} B={th.shape[0]}")


@pytest.mark.parametrize("name,B,sample", [("cmb4x2500", 4096, 12), ("cmbtt_cv", 4096, 12), ("shear10", 4096, 4),
                                           ("shear_interp", 4096, 3)])
def test_theory_full_batch_sampled(name, B, sample):
    """At the benchmark's batch (and so the launch shapes it times): rows at the
    ends of the batch, at workgroup-block boundaries and at random, in the
    headline split-BF16 form and in FP64."""
    m, g = gpu_model(name)
    th = W.posterior_draws(m["theta_fid"], post_scale(m), B, tag=22)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, 1, 31, 32, 63, 64, 127, 128, B - 2, B - 1],
                                    rng.integers(0, B, size=sample)]))
    ref = oracle_theory(th[idx], m)
    for prec in ("bf16x3", "fp64"):
        say(f"case theory full {prec} {name} B={B}")
        got = run_theory(g, th, prec)
        check(ref, got[idx], m, prec, f"{name} full {prec} B={B}")


def test_theory_row_stride_and_empty_batch():
    """ldo > n_data leaves the padding columns untouched; B = 0 is a no-op."""
    from paper_2509_13307_amd import _capi as C
    m, g = gpu_model("cmb4x2500")
    n = g.n_data
    th = torch.tensor(W.posterior_draws(m["theta_fid"], post_scale(m), 5, tag=23), dtype=torch.float64, device=DEV)
    ldo = n + 3
    out = torch.full((5, ldo), -7.0, dtype=torch.float64, device=DEV)
    C.check(C.lib().ns_theory_batch(g._h, ctypes.c_void_p(th.data_ptr()), th.stride(0), 5,
                                    ctypes.c_void_p(out.data_ptr()), ldo, C.PRECISIONS["fp64"], None))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[:, n:] == -7.0)
    np.testing.assert_array_equal(o[:, :n], g.theory(th).cpu().numpy())
    C.check(C.lib().ns_theory_batch(g._h, None, th.stride(0), 0, None, ldo, C.PRECISIONS["fp64"], None))
    assert C.lib().ns_theory_batch(g._h, ctypes.c_void_p(th.data_ptr()), th.stride(0), 5,
                                   ctypes.c_void_p(out.data_ptr()), n - 1, C.PRECISIONS["fp64"], None) == C.NS_E_SHAPE


def test_theory_consistent_with_loglike():
    """The FP64 theory vector fed to the oracle's Gaussian gives the library's
    own FP64 logL (the theory stage is the one the likelihood uses)."""
    from oracle.likelihood import in_support
    from oracle.shear import gaussian_loglike
    m, g = gpu_model("shear10")
    th = W.posterior_draws(m["theta_fid"], post_scale(m), 11, tag=24)
    t = torch.tensor(th, dtype=torch.float64, device=DEV)
    C = g.theory(t).cpu().numpy()
    ll = g.loglike(t).cpu().numpy()
    ok = in_support(th, m)
    assert ok.sum() >= 5 and np.all(ll[~ok] == -np.inf)
    ref = gaussian_loglike(C[ok], m["data"], m["cov"])
    say(f"shear10 theory->logL: max|d| = {np.abs(ref - ll[ok]).max():.3e}")
    assert np.abs(ref - ll[ok]).max() <= 1e-6
