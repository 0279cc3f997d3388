"""Python handle on a libnsmi model: marshals a model description into the C
ABI and calls its entry points on torch device tensors (torch provides device
memory and the current HIP stream; all arithmetic runs in the library)."""
import ctypes

import numpy as np
import torch

from . import _capi as C


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _on_device(t, device):
    return t.is_cuda and (t.device.index if t.device.index is not None else torch.cuda.current_device()) == device


def check_rows(t, d, device, name="theta"):
    """Rows handed to the library as a device pointer with a leading dimension:
    a float64 tensor on the model's device, [B, ld >= d], unit column stride."""
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 tensor")
    if not _on_device(t, device):
        raise TypeError(f"{name} must live on HIP device {device}")
    if t.dim() != 2 or t.shape[1] < d or t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < d):
        raise ValueError(f"{name} must be [B, ld >= d] with unit column stride")


def check_vector(t, n, dtype, device, name):
    """A contiguous length-n vector of `dtype` on `device` (a torch.device)."""
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype):
        raise TypeError(f"{name} must be a {dtype} tensor")
    if t.device != device:
        raise TypeError(f"{name} must live on {device}")
    if t.dim() != 1 or t.shape[0] != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous vector of length {n}")


class Model:
    """A likelihood model resident on one HIP device.

    ``desc`` is a dict with the fields of ``ns_model_desc`` (see include/ns.h):
    kind ("cmb_diag", "cmb_block", "cmb_cv", "shear", "gauss"), d, prior_kind/a/b, nets
    (each with W, b, beta, gamma, in_shift, in_scale, out_mu, out_sigma),
    spec_log, data, sigma / cov_blocks + sigma_pp / cov, the shear geometry,
    pidx/pfix, and mu/sigma for "gauss".
    """

    def __init__(self, desc, device=0):
        self._keep = []
        self.kind = desc["kind"]
        self.d = int(desc["d"])
        self.device = device
        self.n_data = 0
        D = C.ModelDesc()
        D.kind = C.KINDS[self.kind]
        D.d = self.d
        D.prior_kind = self._p(_i32(desc["prior_kind"]), C.c_int32_p)
        D.prior_a = self._p(_f64(desc["prior_a"]), C.c_double_p)
        D.prior_b = self._p(_f64(desc["prior_b"]), C.c_double_p)
        if self.kind == "gauss":
            D.mu = self._p(_f64(desc["mu"]), C.c_double_p)
            D.gsigma = self._p(_f64(desc["sigma"]), C.c_double_p)
        else:
            nets = desc["nets"]
            arr = (C.NetDesc * len(nets))()
            for i, net in enumerate(nets):
                arr[i] = self._net(net)
            self._keep.append(arr)
            D.n_nets = len(nets)
            D.nets = ctypes.cast(arr, ctypes.POINTER(C.NetDesc))
            data = _f64(desc["data"])
            D.n_data = data.size
            self.n_data = int(data.size)
            D.data = self._p(data, C.c_double_p)
            if self.kind in ("cmb_diag", "cmb_block", "cmb_cv"):
                D.spec_log = self._p(_i32([int(x) for x in desc["spec_log"]]), C.c_int32_p)
            if self.kind == "cmb_cv":
                D.ell_min = float(desc["ell_min"])
            if self.kind == "cmb_diag":
                D.sigma = self._p(_f64(desc["sigma"]), C.c_double_p)
            elif self.kind == "cmb_block":
                D.cov_blocks = self._p(_f64(desc["cov_blocks"]), C.c_double_p)
                D.sigma_pp = self._p(_f64(desc["sigma_pp"]), C.c_double_p)
            elif self.kind == "shear":
                D.cov = self._p(_f64(desc["cov"]), C.c_double_p)
                D.n_bins = int(desc["n_bins"])
                D.nz_mean = self._p(_f64(desc["nz_mean"]), C.c_double_p)
                D.nz_sigma = float(desc["nz_sigma"])
                D.n_a = int(desc["n_a"])
                D.a_min = float(desc["a_min"])
                D.n_z = int(desc["n_z"])
                D.k_min = float(desc["k_min"])
                D.k_max = float(desc["k_max"])
                D.n_k = int(desc["n_k"])
                D.ell_min = float(desc["ell_min"])
                D.ell_max = float(desc["ell_max"])
                D.n_ell = int(desc["n_ell"])
                D.z_interp = 1 if desc.get("z_interp", "cubic") == "linear" else 0
                D.pidx = self._p(_i32(desc["pidx"]), C.c_int32_p)
                D.pfix = self._p(_f64(desc["pfix"]), C.c_double_p)
        # torch ships its own HIP runtime: it has to open the GPU before the
        # library's runtime does, or torch finds no device afterwards.
        torch.cuda.init()
        h = ctypes.c_void_p()
        C.check(C.lib().ns_model_create(ctypes.byref(D), device, ctypes.byref(h)))
        self._h = h
        self._keep = []          # the library copied everything it needs

    def _p(self, a, typ):
        self._keep.append(a)
        return a.ctypes.data_as(typ)

    def _net(self, net):
        L = len(net["W"])
        nd = C.NetDesc()
        nd.n_layers = L
        dims = [net["W"][0].shape[1]] + [w.shape[0] for w in net["W"]]
        nd.dims = self._p(_i32(dims), C.c_int32_p)

        def plist(arrs, n):
            ps = (C.c_double_p * max(n, 1))()
            for i in range(n):
                ps[i] = self._p(_f64(arrs[i]), C.c_double_p)
            self._keep.append(ps)
            return ps

        nd.W = plist(net["W"], L)
        nd.b = plist(net["b"], L)
        nd.beta = plist(net["beta"], L - 1)
        nd.gamma = plist(net["gamma"], L - 1)
        nd.in_shift = self._p(_f64(net["in_shift"]), C.c_double_p)
        nd.in_scale = self._p(_f64(net["in_scale"]), C.c_double_p)
        nd.out_mu = self._p(_f64(net["out_mu"]), C.c_double_p)
        nd.out_sigma = self._p(_f64(net["out_sigma"]), C.c_double_p)
        return nd

    # ----------------------------------------------------------------- calls
    def _check_theta(self, theta, name="theta"):
        check_rows(theta, self.d, self.device, name)

    def loglike(self, theta, precision="fp64", out=None):
        """logL [B] (float64 device tensor) of theta [B, >= d]."""
        self._check_theta(theta)
        B = theta.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        else:
            check_vector(out, B, torch.float64, theta.device, "out")
        C.check(C.lib().ns_loglike_batch(self._h, _ptr(theta), theta.stride(0), B, _ptr(out),
                                         C.PRECISIONS[precision], _stream()))
        return out

    def loglike_noalloc(self, theta, out, precision="bf16x3"):
        """logL into `out` [B] by the allocation-free entry point
        (ns_loglike_batch_noalloc): the caller provides every buffer."""
        self._check_theta(theta)
        B = theta.shape[0]
        check_vector(out, B, torch.float64, theta.device, "out")
        C.check(C.lib().ns_loglike_batch_noalloc(self._h, _ptr(theta), theta.stride(0), B, _ptr(out),
                                                 C.PRECISIONS[precision], _stream()))
        return out

    def theory(self, theta, precision="fp64"):
        """Theory vector [B, n_data] (float64 device tensor) of theta [B, >= d]:
        the prediction the likelihood compares with the data, in data order."""
        self._check_theta(theta)
        B = theta.shape[0]
        out = torch.empty(B, self.n_data, dtype=torch.float64, device=theta.device)
        C.check(C.lib().ns_theory_batch(self._h, _ptr(theta), theta.stride(0), B, _ptr(out), self.n_data,
                                        C.PRECISIONS[precision], _stream()))
        return out

    def loglike_grad(self, theta, precision="fp64"):
        self._check_theta(theta)
        B = theta.shape[0]
        logl = torch.empty(B, dtype=torch.float64, device=theta.device)
        grad = torch.empty(B, self.d, dtype=torch.float64, device=theta.device)
        C.check(C.lib().ns_loglike_grad_batch(self._h, _ptr(theta), theta.stride(0), B, _ptr(logl), _ptr(grad),
                                              C.PRECISIONS[precision], _stream()))
        return logl, grad

    def prior_transform(self, u):
        """theta [B, d] of unit-cube points u [B, >= d].  The library reads u and
        writes theta with one leading dimension, so theta is allocated with
        u's row stride and its first d columns are returned."""
        self._check_theta(u, "u")
        B, ld = u.shape[0], u.stride(0)
        theta = torch.empty((B, ld), dtype=torch.float64, device=u.device)
        C.check(C.lib().ns_prior_transform(self._h, _ptr(u), _ptr(theta), ld, B, _stream()))
        return theta[:, :self.d]

    def slice_step(self, u, logl, logl_star, dir_chol, n_inner, seed, it, precision="fp64"):
        """In-place slice steps of walkers u [k, d], logl [k]; returns (n_evals, n_stalls)."""
        check_rows(u, self.d, self.device, "u")
        k = u.shape[0]
        if u.shape[1] != self.d or not u.is_contiguous():
            raise ValueError("u must be contiguous [k, d]")
        check_vector(logl, k, torch.float64, u.device, "logl")
        if tuple(dir_chol.shape) != (self.d, self.d):
            raise ValueError("dir_chol must be [d, d]")
        ne = torch.empty(k, dtype=torch.int32, device=u.device)
        ns = torch.empty(k, dtype=torch.int32, device=u.device)
        L = dir_chol.to(device=u.device, dtype=torch.float64).contiguous()
        C.check(C.lib().ns_slice_step(self._h, _ptr(u), _ptr(logl), _ptr(ne), _ptr(ns), k, float(logl_star),
                                      _ptr(L), int(n_inner), int(seed), int(it), C.PRECISIONS[precision],
                                      _stream()))
        return ne, ns

    def run(self, n_live, n_delete, n_inner, precision="fp64", frac_remain=1e-3, seed=1, max_iter=100000,
            n_replicates=1000, capacity=0, checkpoint_path=None, checkpoint_every=0, resume=False, speculate=0):
        """Nested slice sampling; returns a dict (logz, sigma, h, ..., and dead points if capacity > 0).
        With checkpoint_path the state is written every checkpoint_every
        iterations and when max_iter ends the run; resume=True continues from
        that file if it exists.  speculate: slice proposals per bracket end and
        round (1-4, 0 = the library's choice); the result does not depend on it."""
        path = None if checkpoint_path is None else str(checkpoint_path).encode()
        o = C.RunOpts(n_live, n_delete, n_inner, C.PRECISIONS[precision], frac_remain, seed, max_iter, n_replicates,
                      path, int(checkpoint_every), 1 if resume else 0, int(speculate))
        r = C.RunResult()
        dl = np.zeros(capacity)
        dn = np.zeros(capacity, dtype=np.int32)
        du = np.zeros((capacity, self.d))
        nullp = ctypes.c_void_p()
        args = (dl.ctypes.data_as(ctypes.c_void_p), dn.ctypes.data_as(ctypes.c_void_p),
                du.ctypes.data_as(ctypes.c_void_p)) if capacity else (nullp, nullp, nullp)
        C.check(C.lib().ns_run(self._h, ctypes.byref(o), ctypes.byref(r), *args, capacity, _stream()))
        out = {f: getattr(r, f) for f, _ in C.RunResult._fields_}
        if capacity:
            n = min(capacity, r.n_dead)
            out.update(dead_logl=dl[:n], dead_n=dn[:n], dead_u=du[:n])
        return out

    def hmc(self, theta0, inv_mass, n_iter, n_leapfrog, step, seed=1, precision="fp64", keep_samples=True):
        """Hamiltonian Monte Carlo chains from theta0 [chains, d] (device tensor);
        returns (samples [n_iter, chains, d], logp [n_iter, chains], result dict,
        last state)."""
        dev = torch.device("cuda", self.device)
        theta = theta0.to(device=dev, dtype=torch.float64).contiguous().clone()
        if theta.dim() != 2 or theta.shape[1] != self.d:
            raise ValueError("theta0 must be [chains, d]")
        n_ch, d = theta.shape
        if inv_mass.numel() != d:
            raise ValueError("inv_mass must hold d values")
        minv = inv_mass.to(device=theta.device, dtype=torch.float64).contiguous()
        samples = logp = None
        if keep_samples:
            samples = torch.empty((n_iter, n_ch, d), dtype=torch.float64, device=theta.device)
            logp = torch.empty((n_iter, n_ch), dtype=torch.float64, device=theta.device)
        o = C.HmcOpts(n_ch, n_iter, n_leapfrog, C.PRECISIONS[precision], step, seed)
        r = C.HmcResult()
        nullp = ctypes.c_void_p()
        C.check(C.lib().ns_hmc(self._h, ctypes.byref(o), _ptr(minv), _ptr(theta),
                               _ptr(samples) if keep_samples else nullp, _ptr(logp) if keep_samples else nullp,
                               ctypes.byref(r), _stream()))
        return samples, logp, {f: getattr(r, f) for f, _ in C.HmcResult._fields_}, theta

    def trace(self, enable=True):
        """Bracket every kernel launch with HIP events (see ns_trace_enable)."""
        C.check(C.lib().ns_trace_enable(self._h, 1 if enable else 0))

    def trace_report(self):
        """{kernel: (launches, total_ms)} since the last report."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        C.check(C.lib().ns_trace_report(self._h, buf, len(buf)))
        return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}

    def tuning_report(self):
        """{layer shape: tile configuration} chosen by the BF16 autotuner."""
        import json
        buf = ctypes.create_string_buffer(1 << 14)
        C.check(C.lib().ns_tuning_report(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None):
            C.check(C.lib().ns_model_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
