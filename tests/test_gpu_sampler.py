"""Parity of the HIP sampler (ns_prior_transform, ns_slice_step, ns_run) with
the oracle: both draw every random number from the same Philox4x64-10
sequences, so the GPU replays the oracle's trajectory up to FP64 rounding."""
import sys

import numpy as np
import pytest
import torch
from scipy.special import ndtr

import workloads as W
from oracle import nested
from oracle.likelihood import loglike_u, prior_transform
from oracle.philox import uniforms

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mk(desc):
    from paper_2509_13307_amd import Model
    return Model(desc)


def test_prior_transform_matches_oracle():
    say("case prior transform shear10")
    m = W.structure("shear10")
    u = np.random.default_rng(3).uniform(size=(333, m["d"]))
    g = mk(W.load_model("shear10"))
    th = g.prior_transform(torch.tensor(u, device=DEV)).cpu().numpy()
    np.testing.assert_allclose(th, prior_transform(u, m), rtol=1e-14, atol=1e-15)


def walkers_above(model, n, seed):
    d = model["d"]
    u = uniforms(seed, 0, np.arange(n), 0, 0, np.arange(d))
    ll = loglike_u(u, model)
    lstar = np.median(ll)
    keep = ll > lstar
    return u, ll, lstar, u[keep], ll[keep]


@pytest.mark.parametrize("name,k_live,n_inner", [("cmb6", 100, 6), ("shear10", 40, 2)])
def test_slice_step_replays_oracle(name, k_live, n_inner):
    say(f"case slice step {name}")
    m = W.load_model(name)
    u_all, _, lstar, u0, l0 = walkers_above(m, k_live, seed=9)
    L = nested.direction_cholesky(u_all)
    fn = lambda x: loglike_u(x, m)
    u_ref, l_ref, ne_ref, ns_ref = nested.slice_step(fn, u0, l0, lstar, L, n_inner, seed=9, it=4)
    g = mk(m)
    ut = torch.tensor(u0, device=DEV).contiguous()
    lt = torch.tensor(l0, device=DEV)
    ne, ns = g.slice_step(ut, lt, lstar, torch.tensor(L), n_inner, seed=9, it=4)
    torch.cuda.synchronize()
    say(f"{name}: evals {int(ne.sum())} vs oracle {int(ne_ref.sum())}")
    np.testing.assert_array_equal(ne.cpu().numpy(), ne_ref)
    np.testing.assert_array_equal(ns.cpu().numpy(), ns_ref)
    np.testing.assert_allclose(ut.cpu().numpy(), u_ref, rtol=0, atol=1e-10)
    np.testing.assert_allclose(lt.cpu().numpy(), l_ref, rtol=1e-12, atol=1e-7)
    assert np.all(lt.cpu().numpy() > lstar)


def test_ns_run_replays_oracle_gauss():
    say("case ns_run gauss")
    desc = W.gauss_structure(d=3, mu=[0.1, 0.5, 0.8], sigma=[0.05, 0.1, 0.08])
    ref = nested.run(lambda u: loglike_u(u, desc), 3, 200, 100, 15, seed=11, n_rep=200)
    g = mk(desc)
    res = g.run(200, 100, 15, seed=11, n_replicates=200, capacity=200000)
    say(f"gauss: gpu logZ {res['logz']:.10f} +- {res['sigma']:.4f} iters {res['n_iter']} | "
        f"oracle {ref['logZ']:.10f} +- {ref['sigma']:.4f} iters {ref['n_iter']}")
    assert res["n_iter"] == ref["n_iter"]
    assert res["n_evals"] == ref["n_evals"]
    assert abs(res["logz"] - ref["logZ"]) < 1e-8
    assert abs(res["sigma"] - ref["sigma"]) < 1e-8
    np.testing.assert_allclose(res["dead_logl"], ref["dead_logl"], rtol=1e-12, atol=1e-10)
    exact = np.sum(np.log(ndtr((1 - np.array([0.1, 0.5, 0.8])) / np.array([0.05, 0.1, 0.08]))
                          - ndtr(-np.array([0.1, 0.5, 0.8]) / np.array([0.05, 0.1, 0.08]))))
    assert abs(res["logz"] - exact) < 3 * res["sigma"]


def test_ns_run_replays_oracle_cmb6():
    say("case ns_run cmb6")
    m = W.load_model("cmb6")
    ref = nested.run(lambda u: loglike_u(u, m), 6, 100, 50, 30, seed=1, n_rep=100)
    g = mk(m)
    res = g.run(100, 50, 30, seed=1, n_replicates=100)
    say(f"cmb6: gpu logZ {res['logz']:.8f} +- {res['sigma']:.4f} iters {res['n_iter']} evals {res['n_evals']} "
        f"wall {res['wall_s']:.3f}s | oracle {ref['logZ']:.8f} iters {ref['n_iter']} evals {ref['n_evals']}")
    assert res["n_iter"] == ref["n_iter"]
    assert res["n_evals"] == ref["n_evals"]
    assert abs(res["logz"] - ref["logZ"]) < 1e-6
