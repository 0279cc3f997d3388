#!/usr/bin/env python3
"""Batched likelihood throughput and nested-sampling wall time on one MI355X.

Step: one ns_loglike_batch call over B = 4096 walkers of the four-spectrum CMB
emulator workload (6 parameters -> 4 networks 6-512-512-512-512-2500 ->
TT/TE/EE/PP at l = 2..2501, 3x3 block + diagonal Gaussian chi^2 over 10000
data), theta resident in HBM.  Every precision form is timed; `value` is the
BF16-MFMA form, the FP64 form is reported beside it.  The nested-sampling leg
times ns_run on the 6-parameter CMB emulator likelihood until sigma(log Z) <=
0.1.  The CPU baseline is the FP64 oracle on a bounded sample of the same
workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

MI355X_PEAK = {"bf16": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}   # dense TFLOP/s
HBM_PEAK_GBS = 8000.0


def gemm_flops(B, K, N):
    return 2.0 * B * K * N


def mlp_flops(net, rows):
    """Algorithmic FLOPs of one network over `rows` rows (2 per MAC, all layers)."""
    return sum(2.0 * rows * W.shape[0] * W.shape[1] for W in net["W"])


KERNEL_SOURCES = {"mlp_fused": ("paper_2509_13307_amd/csrc/mlp_fused.hip", "paper_2509_13307_amd/csrc/devutil.h")}


def measured_traffic(dom, B, workload):
    """HBM bytes per launch of kernel `dom` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the plain-copy calibration; None
    when no summary exists for this workload and batch or the kernel sources
    changed since it was taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"{dom}_hbm_bytes.json")
    key = next((k for k in KERNEL_SOURCES if dom.startswith(k)), None)
    if key is None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[key]:
        h.update(open(os.path.join(here, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest() or rec.get("batch") != B or rec.get("workload") != workload:
        return None
    return rec["fetch_kib"] * 1024 * rec["fetch_scale"] + rec["write_kib"] * 1024 * rec["write_scale"]


def measured_mfma_busy(dom, B, workload):
    """MFMA-busy fraction and clock of kernel `dom` from the committed
    rocprofv3 counter summary (SQ_VALU_MFMA_BUSY_CYCLES over the SIMDs' active
    cycles, GRBM_GUI_ACTIVE per XCD over the launch time); None when no summary
    exists for this workload and batch or the kernel sources changed since."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"{dom}_mfma_busy.json")
    key = next((k for k in KERNEL_SOURCES if dom.startswith(k)), None)
    if key is None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[key]:
        h.update(open(os.path.join(here, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest() or rec.get("batch") != B or rec.get("workload") != workload:
        return None
    return dict(frac=round(rec["mfma_busy_frac"], 4), clock_ghz=round(rec["clock_ghz"], 3),
                launch_us=round(rec["launch_s_median"] * 1e6, 2), source="profiles/" + os.path.basename(path))


def roofline_of(dom, avg_s, prec, m, B, workload):
    """Roofline entry of kernel `dom` from its average launch time: algorithmic
    work of one launch over the form's published MI355X peak."""
    net = m["nets"][0]
    n_nets = len(m["nets"])                       # networks of equal shape share one launch
    rows = B * int(m.get("n_z", 1))
    K_last, N_last = net["W"][-1].shape[1], net["W"][-1].shape[0]
    K_hid = net["W"][1].shape[1]
    issued = None
    if dom.startswith("mlp_fused"):
        work = n_nets * mlp_flops(net, rows)
        gemm = n_nets * sum(2.0 * rows * W.shape[0] * W.shape[1] for W in net["W"][1:])
        # MFMA instructions issued: 3 products per split-BF16 multiply
        issued = (3.0 if prec == "bf16x3" else 1.0) * gemm
        unit, bound = "TFLOP/s", "mfma"
    elif dom.endswith("_out"):
        work, unit, bound = n_nets * gemm_flops(rows, K_last, N_last), "TFLOP/s", "mfma"
    elif dom.endswith("_hidden"):
        work, unit, bound = n_nets * gemm_flops(rows, K_hid, K_hid), "TFLOP/s", "mfma"
    else:
        elem = 8 if prec == "fp64" else 4
        work, unit, bound = float(B) * m["data"].size * elem, "GB/s", "hbm"
    if unit == "TFLOP/s":
        achieved = work / avg_s / 1e12
        peak = MI355X_PEAK[prec]
    else:
        achieved = work / avg_s / 1e9
        peak = HBM_PEAK_GBS
    traffic = measured_traffic(dom, B, workload)
    r = dict(kernel=dom, bound=bound, achieved=round(achieved, 2), peak=peak, unit=unit,
             frac=round(achieved / peak, 4), traffic=traffic, avg_launch_us=round(avg_s * 1e6, 2),
             work_per_launch=work)
    if issued is not None:
        r["mfma_issued_frac"] = round(issued / avg_s / 1e12 / peak, 4)
        busy = measured_mfma_busy(dom, B, workload)
        if busy is not None:
            r["mfma_busy_profiled"] = busy
    return r


WORKLOAD_TEXT = {
    "cmb4x2500": "6 params -> 4 x (6-512-512-512-512-2500) emulators, 3x3 block + diagonal Gaussian over 10000 "
                 "data, prior-draw theta",
    "cmb6": "6 params -> 6-128-128-128-200 emulator, diagonal Gaussian over 200 data, prior-draw theta",
    "cmbtt_cv": "6 params -> 6-512-512-512-512-2500 TT emulator, cosmic-variance-limited likelihood, prior-draw theta",
    "shear10": "39 params, emulator 8-512-512-512-512-420 at 10 z nodes (cubic in z), 256 a-nodes, 5 bins, "
               "dense 300 x 300 chi^2, prior-draw theta",
    "shear64": "39 params, emulator 8-512-512-512-512-420 at 64 z nodes (cubic in z), 256 a-nodes, 5 bins, "
               "dense 300 x 300 chi^2, prior-draw theta",
    "shear_full": "39 params, emulator 8-512-512-512-512-420 at all 1025 a-nodes, 10 bins, dense 1100 x 1100 "
                  "chi^2, prior-draw theta",
    "shear_interp": "39 params, emulator 8-512-512-512-512-420 at 103 nodes (linear in z), 1025 a-nodes, 10 bins, "
                    "dense 1100 x 1100 chi^2, prior-draw theta",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="before each form's warmup steps, run that form's calls back to back (untimed) for this "
                         "long, so that the timed steps see the clocks of sustained work (0: off)")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--workload", default="cmb4x2500")
    ap.add_argument("--forms", default="bf16,bf16x3,fp32,fp64")
    ap.add_argument("--no-ns", action="store_true")
    ap.add_argument("--ns-only", action="store_true",
                    help="run only the nested-sampling leg (one JSON line), e.g. for a kernel trace of ns_run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-shear", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batch-scaling sweep")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the per-workload |dlogL| leg")
    ap.add_argument("--model-comparison", action="store_true",
                    help="only run the LCDM vs w0wa nested-sampling comparison and print its JSON")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain device copies of 256 MiB (reference for HBM byte counters)")
    ap.add_argument("--shear-paper", action="store_true",
                    help="only run the paper-shaped shear pair (full vs linear-z interpolated) and print its JSON")
    ap.add_argument("--sp-ns", default="",
                    help="with --shear-paper: comma list of precisions for the nested-sampling comparison")
    ap.add_argument("--mc-precision", default="bf16x3")
    ap.add_argument("--mc-live", type=int, default=1000)
    ap.add_argument("--mc-hmc-iter", type=int, default=400)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); runs on several GPUs "
              "are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2509_13307_amd import Model

    if args.calibrate_copy:
        n = 256 << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return

    if args.shear_paper:
        ns_precs = [p for p in args.sp_ns.split(",") if p]
        print(json.dumps(shear_paper(Model, W, torch, ns_precs, args.mc_live)), flush=True)
        return

    if args.ns_only:
        print(json.dumps({"ns": ns_leg(Model, W)}), flush=True)
        return

    if args.model_comparison:
        print(json.dumps(model_comparison(Model, W, args.mc_precision, args.mc_live, args.mc_hmc_iter)), flush=True)
        return

    dev = "cuda:0"
    B = args.batch
    m = W.load_model(args.workload)
    g = Model(m)
    theta_np = W.prior_draws(m, B, tag=7)
    theta = torch.tensor(theta_np, dtype=torch.float64, device=dev)
    logl = torch.empty(B, dtype=torch.float64, device=dev)
    forms = args.forms.split(",")
    res = {}
    traces = {}
    settle = {}
    for prec in forms:
        # the GPU's clocks fall within milliseconds of idling and take some
        # tens of milliseconds of steady work to come back; a sampler keeps the
        # GPU busy, so the timed steps follow a stretch of back-to-back calls
        g.loglike(theta, prec, out=logl)             # first call: autotuning of the form
        torch.cuda.synchronize()
        t_s, n_s = time.perf_counter(), 0
        while (time.perf_counter() - t_s) * 1e3 < args.settle_ms:
            for _ in range(8):
                g.loglike(theta, prec, out=logl)
            n_s += 8
            torch.cuda.synchronize()
        settle[prec] = dict(calls=n_s, ms=round((time.perf_counter() - t_s) * 1e3, 1))
        for _ in range(args.warmup):
            g.loglike(theta, prec, out=logl)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.loglike(theta, prec, out=logl)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        # same work with every kernel bracketed by HIP events on its stream
        g.trace(True)
        e0.record()
        for _ in range(args.steps):
            g.loglike(theta, prec, out=logl)
        e1.record()
        torch.cuda.synchronize()
        ms_traced = e0.elapsed_time(e1) / args.steps
        traces[prec] = g.trace_report()
        g.trace(False)
        res[prec] = dict(evals_per_s=B / (ms * 1e-3), ms_per_step=ms, ms_per_step_traced=ms_traced,
                         wall_s=wall, logl_finite=int(torch.isfinite(logl).sum().item()))
        print(f"# {prec}: {ms:.3f} ms/step, {B / (ms * 1e-3):.4g} evals/s", file=sys.stderr, flush=True)

    # headline: BF16-operand MFMA form that meets |dlogL| <= 1e-2 against the
    # FP64 oracle (split BF16, FP32 accumulation); plain BF16 is reported beside it
    head = "bf16x3" if "bf16x3" in res else forms[0]
    # dominant kernel of the headline form: largest total traced time
    tr = traces[head]
    dom = max(tr, key=lambda k: tr[k][1])
    n_launch, tot_ms = tr[dom]
    avg_s = tot_ms / n_launch * 1e-3
    roofline = roofline_of(dom, avg_s, head, m, B, args.workload)
    out = {
        "metric": "likelihood evals/sec @batch 4096 (BF16 vs FP64); NS wall time to logZ +/-0.1",
        "value": round(res[head]["evals_per_s"], 1),
        "unit": "likelihood evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[head]["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT.get(args.workload, '')}",
                   "batch": B, "parallelism": "single GPU"},
        "forms": {p: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()} for p, r in res.items()},
        "fp64_evals_per_s": round(res["fp64"]["evals_per_s"], 1) if "fp64" in res else None,
        "bf16_evals_per_s": round(res["bf16"]["evals_per_s"], 1) if "bf16" in res else None,
        "kernels": {p: {k: [n, round(t / n * 1e3, 2)] for k, (n, t) in tr_.items()} for p, tr_ in traces.items()},
        "roofline": roofline,
        "settle": dict(ms_requested=args.settle_ms, per_form=settle,
                       note="untimed back-to-back calls of each form before its warmup steps"),
        "bf16_tiles": g.tuning_report(),
    }
    if "fp64" in traces and head != "fp64":
        # the paper's own arithmetic: roofline of the FP64 form's dominant kernel
        tr64 = traces["fp64"]
        dom64 = max(tr64, key=lambda k: tr64[k][1])
        n64, t64 = tr64[dom64]
        out["roofline_fp64"] = roofline_of(dom64, t64 / n64 * 1e-3, "fp64", m, B, args.workload)

    # per-call distribution of the headline form: 50 calls, each between its own events
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for e0, e1 in evs:
        e0.record()
        g.loglike(theta, head, out=logl)
        e1.record()
    torch.cuda.synchronize()
    per = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    out["per_call_ms"] = {"form": head, "calls": 50, "median": round(float(np.median(per)), 4),
                          "p10": round(float(np.percentile(per, 10)), 4),
                          "p90": round(float(np.percentile(per, 90)), 4)}
    out["env"] = environment(torch)

    if not args.no_sweep:
        out["batch_scaling"] = batch_sweep(Model, W, torch, dev)

    if not args.no_ns:
        out["ns"] = ns_leg(Model, W)

    if not args.no_shear:
        out["shear"] = shear_leg(Model, W, torch, dev)

    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(Model, W, torch, dev)

    if not args.no_cpu:
        out["cpu_baseline"], out["accuracy"] = cpu_leg(m, g, forms, torch, dev)
        if not args.no_accuracy:
            out["accuracy"]["per_workload"] = accuracy_leg(Model, W, torch, dev)

    print(json.dumps(out), flush=True)


def accuracy_leg(Model, W, torch, dev):
    """max |dlogL| of every form against the FP64 oracle on posterior-region
    walkers (theta_fid plus Fisher-scaled Gaussian draws, capped at a tenth of
    a uniform prior's width), per workload; the bars are 1e-6 (FP64) and
    1e-2 (reduced forms)."""
    from oracle.likelihood import loglike as oracle_loglike
    plan = [("cmb6", 64), ("cmb4x2500", 64), ("cmbtt_cv", 64), ("shear10", 32), ("shear64", 32),
            ("shear_full", 16), ("shear_interp", 16)]
    out = {}
    for name, B in plan:
        m = W.load_model(name)
        g = Model(m)
        width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
        th = W.posterior_draws(m["theta_fid"], np.minimum(m["fisher_sigma"], 0.1 * width), B, tag=19)
        ref = oracle_loglike(th, m, chunk=64)
        fin = np.isfinite(ref)
        t = torch.tensor(th, dtype=torch.float64, device=dev)
        row = {"walkers": int(fin.sum())}
        for p in ("fp64", "fp32", "bf16x3", "bf16"):
            got = g.loglike(t, p).cpu().numpy()
            row[p] = float(np.max(np.abs(got[fin] - ref[fin])))
        row["meets_bar"] = {p: bool(row[p] <= (1e-6 if p == "fp64" else 1e-2)) for p in ("fp64", "fp32", "bf16x3", "bf16")}
        out[name] = row
        g.close()
        print(f"# accuracy {name}: {json.dumps(row)}", file=sys.stderr, flush=True)
    return out


def adjoint_leg(Model, W, torch, dev):
    """ns_loglike_grad_batch (logL and d logL / d theta by the hand-written
    adjoint) at batch 4096: gradients per second and the rate of the
    emulator's backward GEMMs (input gradients only: the multiply-adds of its
    forward GEMM layers once more), against the peak of their arithmetic
    (FP64 for the FP64 form; the reduced forms run the adjoint in FP32)."""
    B = 4096
    out = {}
    for name, precs in (("cmb4x2500", ("fp64", "bf16x3")), ("shear64", ("fp64",))):
        m = W.load_model(name)
        g = Model(m)
        th = torch.tensor(W.prior_draws(m, B, tag=22), dtype=torch.float64, device=dev)
        rows = B * int(m.get("n_z", 1))
        back_flops = sum(2.0 * rows * Wl.shape[0] * Wl.shape[1] for net in m["nets"] for Wl in net["W"][1:])
        for prec in precs:
            g.loglike_grad(th, prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3
            e0.record()
            for _ in range(reps):
                g.loglike_grad(th, prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            g.trace(True)
            g.loglike_grad(th, prec)
            tr = g.trace_report()
            g.trace(False)
            key = "adj_gemm_f64" if prec == "fp64" else "adj_gemm_f32"
            n_adj, t_adj = tr.get(key, (0, 0.0))
            peak = MI355X_PEAK["fp64" if prec == "fp64" else "fp32"]
            achieved = back_flops / (t_adj * 1e-3) / 1e12 if t_adj > 0 else None
            out[f"{name}_{prec}"] = dict(
                batch=B, ms_per_call=round(ms, 3), grads_per_s=round(B / (ms * 1e-3), 1),
                backward_gemm=dict(kernel=key, launches=n_adj, total_us=round(t_adj * 1e3, 1),
                                   work_flop=back_flops, achieved_tflops=None if achieved is None else round(achieved, 2),
                                   peak_tflops=peak, frac=None if achieved is None else round(achieved / peak, 4)),
                kernels_us={k: round(t / n * 1e3, 2) for k, (n, t) in tr.items()})
            print(f"# adjoint {name} {prec}: {json.dumps(out[f'{name}_{prec}'])}", file=sys.stderr, flush=True)
        g.close()
    return out


def environment(torch):
    """ROCm / device / host description and, when rocm-smi answers, clocks and power."""
    import platform
    import subprocess
    env = {"device": torch.cuda.get_device_name(0), "hip": torch.version.hip, "torch": torch.__version__}
    try:
        env["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        env["rocm"] = None
    try:
        import shutil
        smi = shutil.which("rocm-smi")
        # run the (Python) tool through this interpreter, not through its #! line
        r = subprocess.run([sys.executable, smi, "--showclocks", "--showpower", "--json"], capture_output=True,
                           text=True, timeout=30)
        env["rocm_smi"] = json.loads(r.stdout) if r.returncode == 0 else None
    except (OSError, subprocess.SubprocessError, ValueError, TypeError):
        env["rocm_smi"] = None
    env["host"] = platform.node()
    return env


def time_calls(g, th, prec, torch, warm=2, reps=5):
    """Mean ms per call of g.loglike over `reps` calls after `warm` (HIP events)."""
    for _ in range(warm):
        g.loglike(th, prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.loglike(th, prec)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_sweep(Model, W, torch, dev):
    """Likelihood time against batch size (the analogue of the paper's Fig. 1:
    time of a batched call relative to a call on one parameter set)."""
    plan = [("cmb4x2500", ("bf16x3", "fp64"), (1, 16, 64, 256, 1024, 4096, 16384, 65536)),
            ("shear_interp", ("bf16x3", "fp64"), (1, 16, 64, 256, 1024, 4096)),
            ("shear_full", ("bf16x3",), (1, 16, 64, 256, 1024))]
    out = {}
    for name, precs, batches in plan:
        m = W.load_model(name)
        g = Model(m)
        th_all = W.prior_draws(m, max(batches), tag=17)
        for prec in precs:
            rows = []
            t1 = None
            for B in batches:
                th = torch.tensor(th_all[:B], dtype=torch.float64, device=dev)
                ms = time_calls(g, th, prec, torch)
                t1 = ms if t1 is None else t1
                rows.append(dict(batch=B, ms_per_call=round(ms, 4), evals_per_s=round(B / (ms * 1e-3), 1),
                                 time_rel_single=round(ms / t1, 3)))
            out[f"{name}_{prec}"] = rows
            print(f"# sweep {name} {prec}: {json.dumps(rows)}", file=sys.stderr, flush=True)
        g.close()
    return out


def ns_leg(Model, W):
    """Nested slice sampling on the 6-parameter CMB emulator likelihood."""
    import torch
    m = W.load_model("cmb6")
    g = Model(m)
    torch.cuda.synchronize()
    out = {}
    # one untimed iteration per form and live-point count first: the
    # likelihood's launch shapes are tuned on first use (a one-time cost of a
    # model, kept out of the timed runs)
    for n, prec in ((100, "fp64"), (2400, "fp64"), (2400, "bf16x3")):
        g.run(n, n // 2, 30, precision=prec, seed=1, n_replicates=0, max_iter=1)
    r = g.run(100, 50, 30, precision="fp64", seed=1, n_replicates=1000)
    out["as_configured"] = dict(n_live=100, n_delete=50, logz=r["logz"], sigma=r["sigma"], wall_s=r["wall_s"],
                                n_iter=r["n_iter"], n_evals=r["n_evals"])
    for prec in ("fp64", "bf16x3"):
        r = g.run(2400, 1200, 30, precision=prec, seed=2, n_replicates=1000)
        out[f"to_sigma_0.1_{prec}"] = dict(n_live=2400, n_delete=1200, logz=r["logz"], sigma=r["sigma"],
                                           wall_s=r["wall_s"], n_iter=r["n_iter"], n_evals=r["n_evals"])
    g.close()
    # the paper's CMB analysis shape: cosmic-variance-limited TT likelihood of
    # one 6-512x4-2500 emulator, 1000 live points, 500 replaced per iteration
    m = W.load_model("cmbtt_cv")
    g = Model(m)
    for prec in ("fp64", "bf16x3"):
        g.run(1000, 500, 30, precision=prec, seed=3, n_replicates=0, max_iter=1)
        r = g.run(1000, 500, 30, precision=prec, seed=3, n_replicates=1000)
        out[f"cmbtt_cv_{prec}"] = dict(n_live=1000, n_delete=500, logz=r["logz"], sigma=r["sigma"],
                                       wall_s=r["wall_s"], n_iter=r["n_iter"], n_evals=r["n_evals"])
    g.close()
    print(f"# ns: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def ns_posterior(g, r, torch, dev):
    """Weighted posterior samples from the dead points of an ns_run: weight
    L_i (X_{i-1} - X_i) with log X_i = -sum_{j <= i} 1 / n_j (Eq. 1)."""
    n = r["dead_n"].astype(np.float64)
    logx = -np.cumsum(1.0 / n)
    x = np.exp(logx)
    xprev = np.concatenate([[1.0], x[:-1]])
    logw = r["dead_logl"] + np.log(xprev - x)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    th = g.prior_transform(torch.tensor(r["dead_u"], device=dev)).cpu().numpy()
    mean = w @ th
    std = np.sqrt(w @ (th - mean) ** 2)
    return th, w, mean, std


def model_comparison(Model, W, prec, n_live, hmc_iter=400, hmc_warmup=100):
    """Bayes factor of LCDM (37 parameters) against w0wa (39) on the same
    synthetic shear data (made at a seeded w0wa point): nested slice sampling
    with n_live live points, n_live/2 deleted per iteration, 5 d slice steps.
    Alongside, 4 HMC chains on the w0wa posterior with the FP64 adjoint
    gradient; their posterior means are compared with the nested-sampling
    posterior (difference in units of its standard deviation)."""
    import torch
    dev = "cuda:0"
    out = {"precision": prec, "n_live": n_live, "n_delete": n_live // 2}
    post = {}
    for name in ("shear_cmp_lcdm", "shear_cmp_w0wa"):
        m = W.load_model(name)
        g = Model(m)
        r = g.run(n_live, n_live // 2, 5 * m["d"], precision=prec, seed=7, n_replicates=1000, capacity=2000000)
        out[name] = {k: r[k] for k in ("logz", "sigma", "sigma_skilling", "h", "n_iter", "n_evals", "n_stalls",
                                       "n_dead", "wall_s")}
        out[name]["d"] = m["d"]
        print(f"# {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)
        if name == "shear_cmp_w0wa":
            th, w, mean, std = ns_posterior(g, r, torch, dev)
            post = dict(th=th, w=w, mean=mean, std=std, model=m, g=g)
        else:
            g.close()
    a, b = out["shear_cmp_lcdm"], out["shear_cmp_w0wa"]
    out["log_B01"] = a["logz"] - b["logz"]
    out["log_B01_sigma"] = float(np.hypot(a["sigma"], b["sigma"]))
    out["wall_s_total"] = a["wall_s"] + b["wall_s"]
    # HMC chains from four posterior draws, inverse mass = NS posterior variance
    m, g = post["model"], post["g"]
    rng = np.random.default_rng(3)
    start = post["th"][rng.choice(len(post["w"]), size=4, p=post["w"])]
    minv = torch.tensor(post["std"] ** 2)
    step, L = 0.1, 16
    cur = torch.tensor(start, device=dev)
    wall = 0.0
    rounds = 4
    for r in range(rounds):          # warmup: scale the step toward ~70% acceptance
        _, _, res, cur = g.hmc(cur, minv, hmc_warmup // rounds, L, step, seed=100 + r, keep_samples=False)
        wall += res["wall_s"]
        acc = res["n_accept"] / (4 * (hmc_warmup // rounds))
        step *= float(np.clip(np.exp(2.0 * (acc - 0.7)), 0.5, 2.0))
    s, lp, res, _ = g.hmc(cur, minv, hmc_iter, L, step, seed=11)
    wall += res["wall_s"]
    x = s.reshape(-1, m["d"]).cpu().numpy()
    z = (x.mean(axis=0) - post["mean"]) / post["std"]
    out["hmc"] = dict(chains=4, iterations=hmc_iter, warmup=hmc_warmup, n_leapfrog=L, step=round(step, 4),
                      precision="fp64", accept_rate=res["n_accept"] / (4 * hmc_iter), rejected_at_walls=res["n_left"],
                      wall_s=wall,
                      max_abs_mean_diff_in_ns_sigma=float(np.max(np.abs(z))),
                      rms_mean_diff_in_ns_sigma=float(np.sqrt(np.mean(z ** 2))),
                      mean_diff_in_ns_sigma=[round(float(v), 3) for v in z])
    print(f"# hmc: {json.dumps(out['hmc'])}", file=sys.stderr, flush=True)
    g.close()
    return out


def shear_paper(Model, W, torch, ns_precs, n_live):
    """The paper's shear pair (App. A, B): 10 bins, 1025 scale-factor nodes,
    the emulator at every node ("full") or at 103 nodes with linear
    interpolation in z ("interp").  Likelihood throughput at batch 512 and
    4096, the interpolation's logL offset over posterior draws, and
    optionally LCDM vs w0wa nested sampling on both (n_live live points,
    n_live / 2 replaced per iteration, 5 d slice steps)."""
    dev = "cuda:0"
    out = {}
    models = {}
    for name in ("shear_full", "shear_interp"):
        m = W.load_model(name)
        g = Model(m)
        models[name] = (m, g)
        res = {}
        for B in (512, 4096):
            th = torch.tensor(W.prior_draws(m, B, tag=14), dtype=torch.float64, device=dev)
            for prec in ("bf16x3", "fp64"):
                if name == "shear_full" and B == 4096 and prec == "fp64":
                    continue
                g.loglike(th, prec)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 3
                e0.record()
                for _ in range(reps):
                    g.loglike(th, prec)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                g.trace(True)
                g.loglike(th, prec)
                tr = g.trace_report()
                g.trace(False)
                res[f"b{B}_{prec}"] = dict(ms_per_step=round(ms, 3), evals_per_s=round(B / (ms * 1e-3), 1),
                                           kernels_us={k: round(t / n * 1e3, 2) for k, (n, t) in tr.items()})
            del th
        out[name] = res
        print(f"# {name}: {json.dumps(res)}", file=sys.stderr, flush=True)
    out["speedup_interp_over_full"] = {
        k: round(out["shear_full"][k]["ms_per_step"] / out["shear_interp"][k]["ms_per_step"], 2)
        for k in out["shear_full"] if k in out["shear_interp"]}
    # systematic offset of the interpolated likelihood over the posterior
    mf, gf = models["shear_full"]
    mi, gi = models["shear_interp"]
    width = np.where(mf["prior_kind"] == 0, mf["prior_b"] - mf["prior_a"], 1.0)
    th = W.posterior_draws(mf["theta_fid"], np.minimum(mf["fisher_sigma"], 0.1 * width), 512, tag=15)
    th = np.clip(th, mf["prior_a"] + 1e-9 * width, np.where(mf["prior_kind"] == 0, mf["prior_b"] - 1e-9 * width, np.inf))
    tt = torch.tensor(th, device=dev)
    lf, li = gf.loglike(tt).cpu().numpy(), gi.loglike(tt).cpu().numpy()
    dl = li - lf
    out["dlogL_interp_minus_full"] = dict(walkers=int(dl.size), mean=float(dl.mean()), std=float(dl.std()),
                                          min=float(dl.min()), max=float(dl.max()),
                                          logL_full_std=float(lf.std()))
    print(f"# dlogL: {json.dumps(out['dlogL_interp_minus_full'])}", file=sys.stderr, flush=True)
    # HMC on the same pair (the paper's gradient-sampler comparison): 60 chains,
    # FP64 adjoint gradients, 16 leapfrog steps, step adapted over 15 warmup
    # trajectories, then 20 timed trajectories
    hmc = {}
    for name in ("shear_full", "shear_interp"):
        m, g = models[name]
        sig = np.minimum(m["fisher_sigma"], 0.1 * width)
        th0 = W.posterior_draws(m["theta_fid"], 0.5 * sig, 60, tag=16)
        th0 = np.clip(th0, m["prior_a"] + 1e-6 * width,
                      np.where(m["prior_kind"] == 0, m["prior_b"] - 1e-6 * width, np.inf))
        cur = torch.tensor(th0, device=dev)
        minv = torch.tensor(sig ** 2)
        step, L, warm = 0.1, 16, 0.0
        for r in range(3):
            _, _, res, cur = g.hmc(cur, minv, 5, L, step, seed=200 + r, keep_samples=False)
            warm += res["wall_s"]
            step *= float(np.clip(np.exp(2.0 * (res["n_accept"] / 300.0 - 0.7)), 0.5, 2.0))
        _, _, res, cur = g.hmc(cur, minv, 20, L, step, seed=210, keep_samples=False)
        hmc[name] = dict(chains=60, n_leapfrog=L, iterations=20, step=round(step, 4),
                         accept_rate=res["n_accept"] / 1200.0, rejected_at_walls=res["n_left"],
                         wall_s=round(res["wall_s"], 3), s_per_trajectory=round(res["wall_s"] / 20, 4),
                         gradient_evals=int(res["n_grad"]) * 60, warmup_wall_s=round(warm, 3))
        print(f"# hmc {name}: {json.dumps(hmc[name])}", file=sys.stderr, flush=True)
    hmc["speedup_interp_over_full"] = round(hmc["shear_full"]["wall_s"] / hmc["shear_interp"]["wall_s"], 2)
    out["hmc_fp64"] = hmc
    for name in list(models):
        models[name][1].close()
    for prec in ns_precs:
        runs = {}
        for name in ("shear_full_lcdm", "shear_full", "shear_interp_lcdm", "shear_interp"):
            m = W.load_model(name)
            g = Model(m)
            r = g.run(n_live, n_live // 2, 5 * m["d"], precision=prec, seed=7, n_replicates=1000)
            runs[name] = {k: r[k] for k in ("logz", "sigma", "n_iter", "n_evals", "wall_s")}
            runs[name]["d"] = m["d"]
            print(f"# ns {prec} {name}: {json.dumps(runs[name])}", file=sys.stderr, flush=True)
            g.close()
        for v in ("full", "interp"):
            a, b = runs[f"shear_{v}_lcdm"], runs[f"shear_{v}"]
            runs[f"log_B01_{v}"] = a["logz"] - b["logz"]
            runs[f"log_B01_{v}_sigma"] = float(np.hypot(a["sigma"], b["sigma"]))
            runs[f"wall_s_{v}"] = a["wall_s"] + b["wall_s"]
        runs["ns_speedup_interp_over_full"] = runs["wall_s_full"] / runs["wall_s_interp"]
        out[f"ns_{prec}"] = runs
    return out


def to_unit_cube(theta, model):
    """Inverse prior transform (uniform: affine; normal: Gaussian CDF)."""
    from scipy.special import ndtr
    a, b = model["prior_a"][None, :], model["prior_b"][None, :]
    uni = (theta - a) / (b - a)
    nrm = ndtr((theta - a) / b)
    return np.where(model["prior_kind"][None, :] == 0, uni, nrm)


def shear_leg(Model, W, torch, dev):
    """Cosmic-shear likelihood throughput at batch 4096 (64 and 10 redshift
    nodes), the paper-shaped full / interpolated pair at batch 512, and ragged
    slice-step batches of 1024-16384 walkers on the 10-node likelihood, where
    walkers need different numbers of likelihood evaluations per step
    (compacted each round)."""
    out = {}
    for name in ("shear64", "shear10"):
        m = W.load_model(name)
        g = Model(m)
        th = torch.tensor(W.prior_draws(m, 4096, tag=12), dtype=torch.float64, device=dev)
        res = {}
        for prec in ("bf16", "bf16x3", "fp64"):
            g.loglike(th, prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                g.loglike(th, prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            g.trace(True)
            g.loglike(th, prec)
            tr = g.trace_report()
            g.trace(False)
            res[prec] = dict(ms_per_step=round(ms, 3), evals_per_s=round(4096 / (ms * 1e-3), 1),
                             kernels_us={k: round(t / n * 1e3, 2) for k, (n, t) in tr.items()})
        out[f"{name}_b4096"] = res
        print(f"# {name}: {json.dumps(res)}", file=sys.stderr, flush=True)
    # the paper's shear pair (10 bins, 1025 nodes): full vs linear-z interpolated
    # likelihood at the nested-sampling batch (512 walkers)
    pair = {}
    for name in ("shear_full", "shear_interp"):
        m = W.load_model(name)
        g = Model(m)
        th = torch.tensor(W.prior_draws(m, 512, tag=14), dtype=torch.float64, device=dev)
        for prec in ("bf16x3", "bf16"):
            g.loglike(th, prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                g.loglike(th, prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            pair[f"{name}_b512_{prec}"] = dict(ms_per_step=round(ms, 3), evals_per_s=round(512 / (ms * 1e-3), 1))
        g.close()
    for prec in ("bf16x3", "bf16"):
        pair[f"speedup_interp_over_full_{prec}"] = round(pair[f"shear_full_b512_{prec}"]["ms_per_step"] /
                                                         pair[f"shear_interp_b512_{prec}"]["ms_per_step"], 2)
    out["paper_shear_pair"] = pair
    print(f"# paper shear pair: {json.dumps(pair)}", file=sys.stderr, flush=True)
    m = W.load_model("shear10")
    g = Model(m)
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    scale = np.minimum(m["fisher_sigma"], 0.1 * width)
    rag = {}
    for k in (1024, 4096, 16384):
        th = W.posterior_draws(m["theta_fid"], scale, k, tag=13)
        th = np.clip(th, m["prior_a"] + 1e-9 * width, np.where(m["prior_kind"] == 0, m["prior_b"] - 1e-9 * width, np.inf))
        u = to_unit_cube(th, m)
        tt = torch.tensor(th, dtype=torch.float64, device=dev)
        for prec in ("bf16x3", "fp64"):
            ll = g.loglike(tt, prec).cpu().numpy()
            lstar = float(np.quantile(ll[np.isfinite(ll)], 0.05))
            keep = np.nonzero(ll > lstar)[0]
            uu = torch.tensor(u[keep], dtype=torch.float64, device=dev).contiguous()
            lt = torch.tensor(ll[keep], dtype=torch.float64, device=dev)
            L = torch.linalg.cholesky(torch.cov(uu.T) + 1e-12 * torch.eye(m["d"], device=dev, dtype=torch.float64))
            # one untimed step on copies: launch-shape tuning and graph set-up for this walker count
            g.slice_step(uu.clone(), lt.clone(), lstar, L, 2, seed=2, it=1, precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ne, ns = g.slice_step(uu, lt, lstar, L, 2, seed=3, it=1, precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nev = ne.cpu().numpy()
            rag[f"k{keep.size}_{prec}"] = dict(walkers=int(keep.size), n_inner=2, evals=int(nev.sum()),
                                                evals_per_walker_min=int(nev.min()), evals_per_walker_max=int(nev.max()),
                                                wall_s=round(dt, 4), evals_per_s=round(nev.sum() / dt, 1))
    out["ragged_slice_shear10"] = rag
    print(f"# ragged: {json.dumps(rag)}", file=sys.stderr, flush=True)
    return out


def cpu_leg(m, g, forms, torch, dev):
    """FP64 oracle on a bounded sample (about 10-30 s of host time) and the
    accuracy of every GPU form on the same sample."""
    from threadpoolctl import threadpool_info
    import workloads as W
    from oracle.likelihood import loglike as oracle_loglike
    width = np.where(m["prior_kind"] == 0, m["prior_b"] - m["prior_a"], 1.0)
    th = W.posterior_draws(m["theta_fid"], np.minimum(m["fisher_sigma"], 0.1 * width), 64, tag=9)
    t0 = time.perf_counter()
    n = 0
    ref = None
    while time.perf_counter() - t0 < 10.0:
        ref = oracle_loglike(th, m, chunk=64)
        n += th.shape[0]
    dt = time.perf_counter() - t0
    info = threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    cpu = dict(value=round(n / dt, 2), unit="likelihood evals/s", cores=threads, kind="oracle",
               sample=f"{n} FP64 oracle evaluations ({n // th.shape[0]} passes over 64 posterior-region "
                      f"walkers of the same workload) in {dt:.1f} s")
    # the same with one BLAS thread (about 5 s)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0, n1 = time.perf_counter(), 0
        while time.perf_counter() - t0 < 5.0:
            oracle_loglike(th[:16], m, chunk=16)
            n1 += 16
        cpu["value_1_thread"] = round(n1 / (time.perf_counter() - t0), 2)
    cpu["host_cpu"] = next((l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")),
                           None)
    cpu["nproc"] = os.cpu_count()
    cpu["blas"] = [{k: i.get(k) for k in ("internal_api", "version", "num_threads")} for i in info]
    # the oracle's nested sampler on the 6-parameter CMB workload, as configured
    from oracle import nested
    from oracle.likelihood import loglike_u
    m6 = W.load_model("cmb6")
    t0 = time.perf_counter()
    r6 = nested.run(lambda u: loglike_u(u, m6), 6, 100, 50, 30, seed=1, n_rep=100)
    cpu["ns_cmb6_oracle"] = dict(n_live=100, n_delete=50, logz=r6["logZ"], n_evals=int(r6["n_evals"]),
                                 wall_s=round(time.perf_counter() - t0, 2))
    acc = {}
    t = torch.tensor(th, dtype=torch.float64, device=dev)
    for p in forms:
        got = g.loglike(t, p).cpu().numpy()
        acc[p] = float(np.max(np.abs(got - ref)))
    return cpu, {"max_abs_dlogl_posterior_64": acc}


if __name__ == "__main__":
    main()
