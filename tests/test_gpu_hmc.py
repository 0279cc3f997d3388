"""HMC chains of ns_hmc (hand-written adjoint gradient) replayed by the FP64
oracle (oracle/hmc.py): same Philox draws, same update order.

Tolerances: positions agree to 1e-9 relative (the oracle's complex-step
gradient and the GPU adjoint differ at the 1e-13 level, and a trajectory
carries that difference through L steps); accept decisions and support exits
are identical.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hmc as ohmc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def start_points(m, C, scale, tag):
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    if "theta_fid" in m:
        sig = np.minimum(m["fisher_sigma"], 0.1 * width) * scale
        th = W.posterior_draws(m["theta_fid"], sig, C, tag=tag)
    else:
        th = np.tile(m["mu"], (C, 1)) + scale * m["sigma"] * np.random.default_rng(tag).normal(size=(C, m["d"]))
    lo = np.where(m["prior_kind"] == 0, m["prior_a"] + 1e-6 * width, -np.inf)
    hi = np.where(m["prior_kind"] == 0, m["prior_b"] - 1e-6 * width, np.inf)
    return np.clip(th, lo, hi)


def replay(m, C, n_iter, L, step, minv, seed, tag):
    from paper_2509_13307_amd import Model
    th0 = start_points(m, C, 0.5, tag)
    g = Model(m)
    s, lp, res, last = g.hmc(torch.tensor(th0, device=DEV), torch.tensor(minv), n_iter, L, step, seed=seed)
    g.close()
    ref = ohmc.run(m, th0, minv, n_iter, L, step, seed)
    s, lp = s.cpu().numpy(), lp.cpu().numpy()
    acc_gpu = res["n_accept"]
    say(f"accept gpu {acc_gpu} oracle {int(ref['accept'].sum())} of {C * n_iter}; left {res['n_left']} / "
        f"{int(ref['left'].sum())}; max |d theta| {np.max(np.abs(s - ref['samples'])):.3e}")
    assert acc_gpu == int(ref["accept"].sum())
    assert res["n_left"] == int(ref["left"].sum())
    np.testing.assert_allclose(s, ref["samples"], rtol=1e-9, atol=1e-12)
    fin = np.isfinite(ref["logp"])
    np.testing.assert_array_equal(fin, np.isfinite(lp))
    np.testing.assert_allclose(lp[fin], ref["logp"][fin], rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(last.cpu().numpy(), ref["theta"], rtol=1e-9, atol=1e-12)
    return res, ref


def test_hmc_replays_oracle_gauss():
    say("case hmc gauss")
    m = W.gauss_structure(d=3, mu=[0.3, 0.5, 0.7], sigma=[0.05, 0.1, 0.08])
    res, ref = replay(m, C=5, n_iter=12, L=8, step=0.3, minv=np.array([0.05, 0.1, 0.08]) ** 2, seed=3, tag=1)
    assert 0 < res["n_accept"] <= 60


def test_hmc_replays_oracle_cmb6():
    say("case hmc cmb6")
    m = W.load_model("cmb6")
    minv = np.minimum(m["fisher_sigma"], 0.1) ** 2
    res, ref = replay(m, C=3, n_iter=4, L=6, step=0.25, minv=minv, seed=5, tag=2)
    assert res["n_accept"] > 0


def test_hmc_replays_oracle_cmbtt_cv():
    say("case hmc cmbtt_cv")
    m = W.load_model("cmbtt_cv")
    minv = np.minimum(m["fisher_sigma"], 0.1) ** 2
    res, ref = replay(m, C=3, n_iter=3, L=5, step=0.25, minv=minv, seed=6, tag=6)
    assert res["n_accept"] > 0


def test_hmc_replays_oracle_shear10():
    say("case hmc shear10")
    m = W.load_model("shear10")
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    minv = np.minimum(m["fisher_sigma"], 0.1 * width) ** 2
    replay(m, C=2, n_iter=2, L=3, step=0.2, minv=minv, seed=7, tag=3)


def test_hmc_replays_oracle_linear_z_shear():
    """Shear with linear z-interpolation and two node chunks (small emulator,
    diagonal covariance): the chunked adjoint drives the chains."""
    say("case hmc shear linear z")
    from oracle import shear as oshear
    m = W.shear_structure(n_z=31, n_bins=3, n_extra=0, hidden=(64, 64), n_a=300, n_k=60, n_ell=25,
                          z_interp="linear")
    C = oshear.spectra(m["theta_fid"][None], m)[0][0]
    sig = 0.05 * np.abs(C) + 1e-3 * np.abs(C).max()
    m["data"] = C + sig * np.random.default_rng(300).normal(size=C.size)
    m["cov"] = np.diag(sig ** 2)
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    m["fisher_sigma"] = 0.005 * width
    res, _ = replay(m, C=2, n_iter=3, L=3, step=0.05, minv=(0.005 * width) ** 2, seed=8, tag=7)
    assert res["n_accept"] > 0


def test_hmc_reflects_at_the_walls():
    """A Gaussian centred 0.05 from the theta_0 = 0 wall: drifts cross the wall
    and are reflected; the oracle replays positions, accepts and rejections."""
    say("case hmc reflection")
    m = W.gauss_structure(d=2, mu=[0.05, 0.5], sigma=[0.1, 0.1])
    res, ref = replay(m, C=6, n_iter=10, L=6, step=0.8, minv=np.array([0.01, 0.01]), seed=4, tag=5)
    assert np.all((ref["samples"] >= 0) & (ref["samples"] <= 1))


def test_hmc_zero_iterations():
    say("case hmc zero iterations")
    from paper_2509_13307_amd import Model
    m = W.gauss_structure(d=2, mu=[0.5, 0.5], sigma=[0.1, 0.1])
    g = Model(m)
    th0 = torch.tensor([[0.5, 0.5], [0.4, 0.6]], dtype=torch.float64, device=DEV)
    s, lp, res, last = g.hmc(th0, torch.ones(2, dtype=torch.float64), 0, 4, 0.1)
    g.close()
    assert s.shape == (0, 2, 2) and res["n_accept"] == 0 and res["n_grad"] == 1
    assert torch.equal(last, th0)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_hmc_reduced_precision_gradient_runs(prec):
    """Reduced-precision gradients: not replayable draw for draw, but the chains
    stay finite and inside the support and accept most trajectories."""
    say(f"case hmc cmb6 {prec}")
    from paper_2509_13307_amd import Model
    m = W.load_model("cmb6")
    minv = np.minimum(m["fisher_sigma"], 0.1) ** 2
    th0 = start_points(m, 4, 0.5, 4)
    g = Model(m)
    s, lp, res, last = g.hmc(torch.tensor(th0, device=DEV), torch.tensor(minv), 20, 6, 0.25, seed=9,
                             precision=prec)
    g.close()
    s = s.cpu().numpy()
    say(f"{prec}: accept {res['n_accept']} of 80, left {res['n_left']}")
    assert np.all(np.isfinite(s)) and np.all((s >= 0) & (s <= 1))
    assert res["n_accept"] >= 40


def test_hmc_shear_is_bitwise_repeatable():
    """Two ns_hmc runs with the same seed on the shear likelihood give bitwise
    equal chains (deterministic adjoint: no float atomics)."""
    say("case hmc shear10 repeatable")
    from paper_2509_13307_amd import Model
    m = W.load_model("shear10")
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    minv = np.minimum(m["fisher_sigma"], 0.1 * width) ** 2
    th0 = torch.tensor(start_points(m, 4, 0.5, 9), device=DEV)
    g = Model(m)
    runs = [g.hmc(th0, torch.tensor(minv), 6, 5, 0.2, seed=11) for _ in range(2)]
    g.close()
    (s0, l0, r0, t0), (s1, l1, r1, t1) = runs
    say(f"accepted {r0['n_accept']} / {r1['n_accept']}")
    assert r0["n_accept"] == r1["n_accept"] and r0["n_left"] == r1["n_left"]
    assert torch.equal(s0, s1) and torch.equal(t0, t1)
    assert torch.equal(torch.nan_to_num(l0, neginf=-1e300), torch.nan_to_num(l1, neginf=-1e300))
