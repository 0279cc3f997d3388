"""ns_loglike_batch_noalloc -- the likelihood for callers that cannot allocate
device memory (its model vector lives in the library's per-GPU scratch array)
-- against the allocating ns_loglike_batch: bitwise equal logL on two calls in
a row, the second with a smaller batch; batches beyond the array's capacity
and forms outside its scope are refused before any launch."""
import sys

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,prec,B1,B2", [("cmb4x2500", "bf16x3", 1600, 333), ("cmbtt_cv", "bf16", 2048, 100),
                                             ("cmb6", "bf16x3", 4096, 77), ("cmb6", "fp64", 3000, 5)])
def test_noalloc_matches_allocating_entry_point(name, prec, B1, B2):
    say(f"case noalloc {name} {prec} B={B1},{B2}")
    from paper_2509_13307_amd import Model
    m = W.load_model(name)
    g = Model(m)
    for B in (B1, B2):
        th = torch.tensor(W.prior_draws(m, B, tag=B), device=DEV)
        ref = g.loglike(th, prec)
        out = torch.full((B,), 7.0, dtype=torch.float64, device=DEV)
        g.loglike_noalloc(th, out, prec)
        torch.cuda.synchronize()
        say(f"  B={B}: {int(torch.isfinite(out).sum())} finite, max |diff| "
            f"{float((out - ref).abs().nan_to_num(0.0).max()):.3e}")
        assert torch.equal(out, ref)
    g.close()


def test_noalloc_refuses_beyond_capacity_and_outside_scope():
    say("case noalloc limits")
    from paper_2509_13307_amd import Model
    m = W.load_model("cmb4x2500")
    g = Model(m)
    B = 1700                                   # the array holds 1658 rows of this model
    th = torch.tensor(W.prior_draws(m, B, tag=1), device=DEV)
    out = torch.full((B,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError, match="scratch"):
        g.loglike_noalloc(th, out, "bf16x3")
    with pytest.raises(RuntimeError, match="forms"):
        g.loglike_noalloc(th[:10], out[:10], "fp32")
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())            # nothing was launched
    g.close()
