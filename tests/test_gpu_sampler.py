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
    # a column view of a wider buffer: theta takes u's row stride, and the
    # guard column past the view is left alone
    wide = torch.full((u.shape[0], m["d"] + 5), 7.0, dtype=torch.float64, device=DEV)
    wide[:, :m["d"]] = torch.tensor(u, device=DEV)
    th2 = g.prior_transform(wide[:, :m["d"]])
    assert tuple(th2.shape) == (u.shape[0], m["d"])
    np.testing.assert_allclose(th2.cpu().numpy(), prior_transform(u, m), rtol=1e-14, atol=1e-15)
    assert bool((wide[:, m["d"]:] == 7.0).all())


def walkers_above(model, n, seed):
    d = model["d"]
    u = uniforms(seed, 0, np.arange(n), 0, 0, np.arange(d))
    ll = loglike_u(u, model)
    lstar = np.median(ll)
    keep = ll > lstar
    return u, ll, lstar, u[keep], ll[keep]


@pytest.mark.parametrize("spec", ["1", "3"])
@pytest.mark.parametrize("name,k_live,n_inner", [("cmb6", 100, 6), ("cmbtt_cv", 64, 3), ("shear10", 40, 2)])
def test_slice_step_replays_oracle(name, k_live, n_inner, spec, monkeypatch):
    """One proposal per walker and round, and three (speculative stepping-out
    and shrink chains): both replay the oracle's serial trajectories."""
    monkeypatch.setenv("NSMI_SPEC", spec)
    say(f"case slice step {name} spec {spec}")
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


def small_linear_shear():
    """Linear-z shear on two node chunks with a small emulator (fast oracle)."""
    from oracle import shear as oshear
    m = W.shear_structure(n_z=31, n_bins=3, n_extra=0, hidden=(64, 64), n_a=300, n_k=60, n_ell=25,
                          z_interp="linear")
    C = oshear.spectra(m["theta_fid"][None], m)[0][0]
    sig = 0.05 * np.abs(C) + 1e-3 * np.abs(C).max()
    m["data"] = C + sig * np.random.default_rng(300).normal(size=C.size)
    m["cov"] = np.diag(sig ** 2)
    return m


def test_slice_step_graph_replays_oracle_linear_z_shear(monkeypatch):
    """Enough rounds for the captured graphs (16 rounds per launch) on the
    chunked, linear-z shear likelihood: the oracle's trajectory is replayed,
    and turning the graphs off changes nothing."""
    say("case slice step shear linear z, graphs")
    m = small_linear_shear()
    u_all, _, lstar, u0, l0 = walkers_above(m, 48, seed=21)
    L = nested.direction_cholesky(u_all)
    fn = lambda x: loglike_u(x, m)
    u_ref, l_ref, ne_ref, ns_ref = nested.slice_step(fn, u0, l0, lstar, L, 10, seed=21, it=3)

    def run(env):
        monkeypatch.delenv("NSMI_NO_GRAPH", raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = mk(m)
        ut = torch.tensor(u0, device=DEV).contiguous()
        lt = torch.tensor(l0, device=DEV)
        ne, ns = g.slice_step(ut, lt, lstar, torch.tensor(L), 10, seed=21, it=3)
        torch.cuda.synchronize()
        out = ut.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), ns.cpu().numpy()
        g.close()
        return out

    got = run({})
    say(f"evals {int(got[2].sum())} vs oracle {int(ne_ref.sum())}, rounds >= {int(got[2].max())}")
    assert got[2].max() > 16
    np.testing.assert_array_equal(got[2], ne_ref)
    np.testing.assert_array_equal(got[3], ns_ref)
    np.testing.assert_allclose(got[0], u_ref, rtol=0, atol=1e-10)
    np.testing.assert_allclose(got[1], l_ref, rtol=1e-12, atol=1e-7)
    other = run({"NSMI_NO_GRAPH": "1"})
    for a, b in zip(got, other):
        np.testing.assert_array_equal(a, b)


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


@pytest.mark.parametrize("n_live,n_delete", [(300, 150), (1000, 500), (2400, 1200), (4096, 2048)])
def test_ns_run_replays_oracle_gauss_large(n_live, n_delete):
    """The configured (1000/500) and the sigma <= 0.1 (2400/1200) live-point
    counts, a count that is no power of two with fewer entries than its sort's
    padded width (300: 512 entries over two waves, one cross-wave stage) and
    the largest (4096: sixteen full waves, strides up to 2048 through LDS);
    the running evidence runs in blocks of ranks for k > 512."""
    say(f"case ns_run gauss {n_live}/{n_delete}")
    desc = W.gauss_structure(d=3, mu=[0.1, 0.5, 0.8], sigma=[0.05, 0.1, 0.08])
    ref = nested.run(lambda u: loglike_u(u, desc), 3, n_live, n_delete, 15, seed=11, n_rep=100)
    g = mk(desc)
    res = g.run(n_live, n_delete, 15, seed=11, n_replicates=100, capacity=400000)
    g.close()
    say(f"gauss {n_live}: gpu logZ {res['logz']:.10f} +- {res['sigma']:.4f} iters {res['n_iter']} "
        f"evals {res['n_evals']} | oracle {ref['logZ']:.10f} +- {ref['sigma']:.4f} iters {ref['n_iter']} "
        f"evals {ref['n_evals']}")
    assert res["n_iter"] == ref["n_iter"]
    assert res["n_evals"] == ref["n_evals"]
    assert res["n_dead"] == ref["dead_logl"].size
    np.testing.assert_array_equal(res["dead_n"], ref["dead_n"])
    np.testing.assert_allclose(res["dead_logl"], ref["dead_logl"], rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(res["dead_u"], ref["dead_u"], rtol=0, atol=1e-10)
    assert abs(res["logz"] - ref["logZ"]) < 1e-8
    assert abs(res["sigma"] - ref["sigma"]) < 1e-8


@pytest.mark.parametrize("name,n_all,n_inner,prec", [("cmb6", 2400, 4, "fp64"), ("cmb6", 2400, 4, "bf16x3"),
                                                     ("shear10", 2048, 1, "fp64")])
def test_slice_step_many_walkers_replays_oracle(name, n_all, n_inner, prec):
    """Ragged slice rounds over 1024-1200 walkers (the nested-sampling batch and
    the ragged benchmark's walker counts) replay the oracle's trajectories."""
    say(f"case slice step {name} {n_all // 2} walkers {prec}")
    m = W.load_model(name)
    u_all, ll_all, lstar, u0, l0 = walkers_above(m, n_all, seed=9)
    L = nested.direction_cholesky(u_all)
    g = mk(m)
    lg = l0
    if prec != "fp64":
        # threshold and start values in the form, as a run in that form has them
        th_all = g.prior_transform(torch.tensor(u_all, device=DEV).contiguous())
        lb = g.loglike(th_all.contiguous(), prec).cpu().numpy()
        lstar = np.median(lb)
        keep = lb > lstar
        u0, l0, lg = u_all[keep], ll_all[keep], lb[keep]
    fn = lambda x: loglike_u(x, m)
    u_ref, l_ref, ne_ref, ns_ref = nested.slice_step(fn, u0, l0, lstar, L, n_inner, seed=9, it=4)
    ut = torch.tensor(u0, device=DEV).contiguous()
    lt = torch.tensor(lg, device=DEV)
    ne, ns = g.slice_step(ut, lt, lstar, torch.tensor(L), n_inner, seed=9, it=4, precision=prec)
    torch.cuda.synchronize()
    g.close()
    ne, ns = ne.cpu().numpy(), ns.cpu().numpy()
    say(f"{name} {prec}: {u0.shape[0]} walkers, evals {int(ne.sum())} vs oracle {int(ne_ref.sum())}, "
        f"per walker {ne.min()}..{ne.max()}")
    if prec == "fp64":
        np.testing.assert_array_equal(ne, ne_ref)
        np.testing.assert_array_equal(ns, ns_ref)
        np.testing.assert_allclose(ut.cpu().numpy(), u_ref, rtol=0, atol=1e-10)
        np.testing.assert_allclose(lt.cpu().numpy(), l_ref, rtol=1e-12, atol=1e-7)
    else:
        # decisions at the threshold may differ where |dlogL| of the form
        # reaches L*: every walker ends inside the constraint, and nearly all
        # replay the FP64 trajectory
        same = np.all(np.abs(ut.cpu().numpy() - u_ref) <= 1e-10, axis=1)
        say(f"  {same.mean():.4f} of the walkers replay the FP64 oracle exactly")
        assert same.mean() > 0.95
    assert np.all(lt.cpu().numpy() > lstar)


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


def test_graph_replay_and_autotune_do_not_change_results(monkeypatch):
    """Captured-graph slice rounds and tuned BF16 tiles give bitwise the eager results."""
    say("case graph/autotune invariance")
    m = W.load_model("cmb6")
    u_all, _, lstar, u0, l0 = walkers_above(m, 100, seed=5)
    L = torch.tensor(nested.direction_cholesky(u_all))
    outs = []
    # layer-by-layer emulator, so that the tuned GEMM tiles are the ones exercised
    monkeypatch.setenv("NSMI_NO_FUSED_MLP", "1")
    for env in ({}, {"NSMI_NO_GRAPH": "1", "NSMI_NO_AUTOTUNE": "1"}):
        for k in ("NSMI_NO_GRAPH", "NSMI_NO_AUTOTUNE"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = mk(m)
        ut = torch.tensor(u0, device=DEV).contiguous()
        lt = torch.tensor(l0, device=DEV)
        ne, ns = g.slice_step(ut, lt, lstar, L, 8, seed=5, it=2, precision="bf16")
        th = torch.tensor(W.prior_draws(m, 300, tag=3), device=DEV)
        ll = g.loglike(th, "bf16")
        outs.append((ut.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), ll.cpu().numpy()))
        g.close()
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("name,n", [("cmb6", 100), ("shear10", 40)])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_fused_emulator_slice_step_matches_layer_by_layer(monkeypatch, name, n, prec):
    """Ragged slice rounds (device row count, compacted walkers) through the
    one-kernel emulator give bitwise the layer-by-layer results (chi^2 staged
    after the emulator).  With the chi^2 in the emulator's epilogue (cmb6)
    the logL differ in the last bits only (same terms, other summation
    order): for this seed no slice decision falls that close to a threshold,
    so the walk (positions, evaluation and stall counts) is the same and the
    logL agree to 1e-12."""
    say(f"case fused slice step {name} {prec}")
    m = W.load_model(name)
    u_all, _, lstar, u0, l0 = walkers_above(m, n, seed=6)
    L = torch.tensor(nested.direction_cholesky(u_all))
    outs = []
    for env in ({"NSMI_NO_FUSED_CHI2": "1"}, {"NSMI_NO_FUSED_MLP": "1"}, {}):
        for k in ("NSMI_NO_FUSED_MLP", "NSMI_NO_FUSED_CHI2"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = mk(m)
        ut = torch.tensor(u0, device=DEV).contiguous()
        lt = torch.tensor(l0, device=DEV)
        ne, ns = g.slice_step(ut, lt, lstar, L, 3, seed=6, it=4, precision=prec)
        outs.append((ut.cpu().numpy(), lt.cpu().numpy(), ne.cpu().numpy(), ns.cpu().numpy()))
        g.close()
    say(f"{name} {prec}: evals {outs[0][2].sum()} (min {outs[0][2].min()}, max {outs[0][2].max()})")
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    for i in (0, 2, 3):
        np.testing.assert_array_equal(outs[2][i], outs[1][i])
    np.testing.assert_allclose(outs[2][1], outs[1][1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_ns_run_resume_is_bitwise(tmp_path, prec):
    """A run cut short by max_iter (checkpoints every 3 iterations and at its
    end) and continued from the file gives bitwise the uninterrupted run."""
    say(f"case ns_run checkpoint/resume cmb6 {prec}")
    m = W.load_model("cmb6")
    g = mk(m)
    full = g.run(100, 50, 30, precision=prec, seed=4, n_replicates=100, capacity=100000)
    path = tmp_path / "run.ckpt"
    part = g.run(100, 50, 30, precision=prec, seed=4, n_replicates=100, capacity=100000, max_iter=7,
                 checkpoint_path=path, checkpoint_every=3)
    assert part["n_iter"] == 7 and path.exists()
    rest = g.run(100, 50, 30, precision=prec, seed=4, n_replicates=100, capacity=100000,
                 checkpoint_path=path, resume=True)
    # a checkpoint of other options is refused
    with pytest.raises(RuntimeError, match="other run options"):
        g.run(100, 50, 30, precision=prec, seed=5, n_replicates=100, checkpoint_path=path, resume=True)
    g.close()
    say(f"full: logZ {full['logz']!r} iters {full['n_iter']} evals {full['n_evals']}; resumed from "
        f"{rest['resumed_iter']}: logZ {rest['logz']!r} iters {rest['n_iter']} evals {rest['n_evals']}")
    assert rest["resumed_iter"] == 7
    for key in ("logz", "sigma", "h", "n_iter", "n_evals", "n_stalls", "n_dead"):
        assert rest[key] == full[key], key
    for key in ("dead_logl", "dead_n", "dead_u"):
        np.testing.assert_array_equal(rest[key], full[key])


@pytest.mark.parametrize("name,n_live,n_inner,prec", [("gauss", 2400, 15, "fp64"), ("cmb6", 100, 30, "fp64"),
                                                      ("cmbtt_cv", 200, 6, "bf16x3")])
def test_ns_run_does_not_depend_on_speculation(name, n_live, n_inner, prec):
    """Speculative proposals (1, 2 or 4 per bracket end and round) change the
    rounds a run takes, not its result: every output is bitwise equal."""
    say(f"case ns_run speculation {name}")
    m = W.gauss_structure(d=3, mu=[0.1, 0.5, 0.8], sigma=[0.05, 0.1, 0.08]) if name == "gauss" else W.load_model(name)
    g = mk(m)
    runs = [g.run(n_live, n_live // 2, n_inner, precision=prec, seed=8, n_replicates=50, capacity=400000,
                  speculate=sp, max_iter=12 if name == "cmbtt_cv" else 100000) for sp in (1, 2, 4)]
    g.close()
    for sp, r in zip((1, 2, 4), runs):
        say(f"  speculate {sp}: logZ {r['logz']!r} iters {r['n_iter']} evals {r['n_evals']} wall {r['wall_s']:.3f}s")
    for r in runs[1:]:
        for key in ("logz", "sigma", "h", "n_iter", "n_evals", "n_stalls", "n_dead"):
            assert r[key] == runs[0][key], key
        for key in ("dead_logl", "dead_n", "dead_u"):
            np.testing.assert_array_equal(r[key], runs[0][key])
