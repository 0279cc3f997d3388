// Hamiltonian Monte Carlo on the hand-written adjoint (gradient samplers
// beside nested sampling, Sec. 2.2): C chains, target
//   log pi = logL + log prior (normal priors -(theta - mu)^2 / 2 sigma^2,
//   uniform priors 0 inside their box, -inf outside the support),
// diagonal inverse mass m, L leapfrog steps of size eps per trajectory,
// Metropolis accept.  Uniform-prior coordinates are reflected at their walls
// (momentum sign flipped); a trajectory that still meets log pi = -inf is
// rejected.
//
// Per trajectory: hmc_start_kernel (momenta, H0, first half kick and drift),
// then per leapfrog step one batched gradient of logL and hmc_step_kernel
// (prior terms, support flag, kick, next drift), then hmc_accept_kernel.
// Random numbers: Philox stream 2 for the momenta (draws 2i, 2i+1 of
// (chain, 0, iteration) -> Box-Muller), stream 3 for the accept uniform.
// Every update is a separately rounded FP64 operation (no contraction) in a
// fixed order, sums over parameters in parameter order, so that a run can be
// replayed step for step by a plain FP64 implementation.
#include <chrono>

#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

constexpr uint64_t HMC_STREAM_MOMENTUM = 2, HMC_STREAM_ACCEPT = 3;

struct HmcState {
    double* th;  double* lp;  double* g;    // current state: theta [C x d], log pi [C], grad [C x d]
    double* th1; double* lp1; double* g1;   // trajectory point
    double* p;                              // momentum [C x d]
    double* h0;                             // H at the start of the trajectory [C]
    int* left;                              // trajectory left the support [C]
    int* n_acc; int* n_left;                // per-chain counters
};

// Mirrors x back into [lo, hi] (one wall per pass, at most 64 passes),
// flipping p at every wall (Neal 2011, Sec. 5.5.1); false if still outside.
__device__ __forceinline__ bool reflect(double& x, double& p, double lo, double hi) {
#pragma clang fp contract(off)
    for (int b = 0; b < 64; ++b) {
        if (x > hi) {
            x = hi - (x - hi);
            p = -p;
        } else if (x < lo) {
            x = lo - (x - lo);
            p = -p;
        } else {
            return true;
        }
    }
    return !(x > hi || x < lo);
}

// Adds the prior terms to (lp, g), which hold logL and its gradient at th.
__device__ __forceinline__ void add_prior(const double* th, double& lp, double* g, int d, const int* pk,
                                          const double* pa, const double* pb) {
#pragma clang fp contract(off)
    if (!isfinite(lp)) {
        lp = -INFINITY;
        for (int i = 0; i < d; ++i) g[i] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int i = 0; i < d; ++i) {
        if (pk[i] != NS_PRIOR_NORMAL) continue;
        const double r = (th[i] - pa[i]) / pb[i];
        acc = acc - 0.5 * (r * r);
        g[i] = g[i] + -(r / pb[i]);
    }
    lp = lp + acc;
}

__global__ void hmc_prior_kernel(HmcState S, int C, int d, const int* __restrict__ pk,
                                 const double* __restrict__ pa, const double* __restrict__ pb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    add_prior(S.th + (int64_t)c * d, S.lp[c], S.g + (int64_t)c * d, d, pk, pa, pb);
}

// Momenta, H0, first half kick and first drift.
__global__ void hmc_start_kernel(HmcState S, const double* __restrict__ minv, int C, int d, double step,
                                 uint64_t seed, uint64_t it, const int* __restrict__ pk,
                                 const double* __restrict__ pa, const double* __restrict__ pb) {
#pragma clang fp contract(off)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const double half = 0.5 * step;
    double k = 0.0;
    bool inside = true;
    for (int i = 0; i < d; ++i) {
        const double u1 = philox_uniform(seed, HMC_STREAM_MOMENTUM, (uint64_t)c, 0, it, 2 * i);
        const double u2 = philox_uniform(seed, HMC_STREAM_MOMENTUM, (uint64_t)c, 0, it, 2 * i + 1);
        const double z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
        const double p = z / sqrt(minv[i]);
        k = k + (minv[i] * p) * p;
        const int64_t e = (int64_t)c * d + i;
        double pk1 = p + half * S.g[e];
        double x = S.th[e] + step * (minv[i] * pk1);
        if (pk[i] == NS_PRIOR_UNIFORM) inside = reflect(x, pk1, pa[i], pb[i]) && inside;
        S.p[e] = pk1;
        S.th1[e] = x;
    }
    S.h0[c] = 0.5 * k - S.lp[c];
    S.left[c] = inside ? 0 : 1;
}

// After the gradient of logL at th1: prior terms, support flag, kick by h,
// and (unless last) the next drift.
__global__ void hmc_step_kernel(HmcState S, const double* __restrict__ minv, int C, int d, double step, double h,
                                int last, const int* __restrict__ pk, const double* __restrict__ pa,
                                const double* __restrict__ pb) {
#pragma clang fp contract(off)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int64_t o = (int64_t)c * d;
    add_prior(S.th1 + o, S.lp1[c], S.g1 + o, d, pk, pa, pb);
    bool inside = isfinite(S.lp1[c]);
    for (int i = 0; i < d; ++i) {
        double pn = S.p[o + i] + h * S.g1[o + i];
        if (!last) {
            double x = S.th1[o + i] + step * (minv[i] * pn);
            if (pk[i] == NS_PRIOR_UNIFORM) inside = reflect(x, pn, pa[i], pb[i]) && inside;
            S.th1[o + i] = x;
        }
        S.p[o + i] = pn;
    }
    if (!inside) S.left[c] = 1;
}

__global__ void hmc_accept_kernel(HmcState S, const double* __restrict__ minv, int C, int d, uint64_t seed,
                                  uint64_t it, double* __restrict__ samples, double* __restrict__ logp) {
#pragma clang fp contract(off)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int64_t o = (int64_t)c * d;
    double k = 0.0;
    for (int i = 0; i < d; ++i) k = k + (minv[i] * S.p[o + i]) * S.p[o + i];
    const double h1 = 0.5 * k - S.lp1[c];
    const double u = philox_uniform(seed, HMC_STREAM_ACCEPT, (uint64_t)c, 0, it, 0);
    const bool ok = !S.left[c] && (log(u) < S.h0[c] - h1);
    if (ok) {
        for (int i = 0; i < d; ++i) {
            S.th[o + i] = S.th1[o + i];
            S.g[o + i] = S.g1[o + i];
        }
        S.lp[c] = S.lp1[c];
        S.n_acc[c] += 1;
    }
    if (S.left[c]) S.n_left[c] += 1;
    if (samples)
        for (int i = 0; i < d; ++i) samples[(it * (uint64_t)C + c) * d + i] = S.th[o + i];
    if (logp) logp[it * (uint64_t)C + c] = S.lp[c];
}

void hmc_run(ns_model* m, const ns_hmc_opts* o, const double* minv, double* theta, double* samples, double* logp,
             ns_hmc_result* res, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int C = o->n_chains, d = m->d, L = o->n_leapfrog;
    const size_t nd = (size_t)C * d;
    // doubles: th, g, th1, g1, p (5 C d) + lp, lp1, h0 (3 C); ints: left, n_acc, n_left (3 C)
    m->ws_hmc.ensure((5 * nd + 3 * (size_t)C) * sizeof(double) + 3 * (size_t)C * sizeof(int));
    double* base = m->ws_hmc.as<double>();
    HmcState S;
    S.th = base; S.g = base + nd; S.th1 = base + 2 * nd; S.g1 = base + 3 * nd; S.p = base + 4 * nd;
    S.lp = base + 5 * nd; S.lp1 = S.lp + C; S.h0 = S.lp1 + C;
    S.left = reinterpret_cast<int*>(S.h0 + C); S.n_acc = S.left + C; S.n_left = S.n_acc + C;
    NS_HIP(hipMemcpyAsync(S.th, theta, nd * sizeof(double), hipMemcpyDeviceToDevice, s));
    NS_HIP(hipMemsetAsync(S.left, 0, 3 * (size_t)C * sizeof(int), s));
    const int* pk = m->prior_kind.as<int>();
    const double* pa = m->prior_a.as<double>();
    const double* pb = m->prior_b.as<double>();
    const dim3 grid((unsigned)((C + 63) / 64)), blk(64);
    loglike_grad_batch(m, S.th, d, C, S.lp, S.g, o->precision, s);
    hipLaunchKernelGGL(hmc_prior_kernel, grid, blk, 0, s, S, C, d, pk, pa, pb);
    NS_HIP(hipGetLastError());
    for (int64_t t = 0; t < o->n_iter; ++t) {
        hipLaunchKernelGGL(hmc_start_kernel, grid, blk, 0, s, S, minv, C, d, o->step, o->seed, (uint64_t)t, pk, pa,
                           pb);
        for (int l = 0; l < L; ++l) {
            loglike_grad_batch(m, S.th1, d, C, S.lp1, S.g1, o->precision, s);
            const bool last = l == L - 1;
            hipLaunchKernelGGL(hmc_step_kernel, grid, blk, 0, s, S, minv, C, d, o->step,
                               last ? 0.5 * o->step : o->step, (int)last, pk, pa, pb);
        }
        hipLaunchKernelGGL(hmc_accept_kernel, grid, blk, 0, s, S, minv, C, d, o->seed, (uint64_t)t, samples, logp);
        NS_HIP(hipGetLastError());
    }
    NS_HIP(hipMemcpyAsync(theta, S.th, nd * sizeof(double), hipMemcpyDeviceToDevice, s));
    std::vector<int> cnt(2 * (size_t)C);
    NS_HIP(hipMemcpyAsync(cnt.data(), S.n_acc, 2 * (size_t)C * sizeof(int), hipMemcpyDeviceToHost, s));
    NS_HIP(hipStreamSynchronize(s));
    res->n_accept = 0;
    res->n_left = 0;
    for (int c = 0; c < C; ++c) {
        res->n_accept += cnt[c];
        res->n_left += cnt[C + c];
    }
    res->n_grad = 1 + (int64_t)o->n_iter * L;
    res->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace nsmi
