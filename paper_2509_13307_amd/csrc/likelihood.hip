// Gaussian chi^2 stages of the CMB likelihoods (Gaussian forms of the
// emulated spectra of Sec. 2.3-2.4), the diagonal-Gaussian test likelihood, the prior transform
// (Table 1) and the per-kind dispatch of the batched likelihood.
//
// All chi^2 arithmetic is FP64 whatever the emulator precision: the model
// vector (FP32 or FP64) is widened before the residual is formed.
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

// ------------------------------------------------------------ diagonal chi^2
// One wave per walker; lanes stride over the n data points.
template <class T>
__global__ __launch_bounds__(256) void chi2_diag_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const T* __restrict__ mvec, int n,
    int64_t ldm, const double* __restrict__ data, const double* __restrict__ isig, double cst,
    double* __restrict__ logl, const int* __restrict__ count) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (count) B = min<int64_t>(B, *count);
    if (row >= B) return;
    const T* mv = mvec + row * ldm;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
        double r = (data[i] - (double)mv[i]) * isig[i];
        s = fma(r, r, s);
    }
    s = wave_sum(s);
    if (lane == 0) {
        const bool ok = in_support(theta + row * ld, d, pk, pa, pb);
        logl[row] = ok ? -0.5 * s + cst : -INFINITY;
    }
}

// ------------------------------------------------- 3x3 block + diagonal chi^2
// Model vector spectrum-major [TT | TE | EE | PP], spectrum k at column k sp
// (sp >= n_ell, padded for aligned rows).  Per multipole
// the residual (TT, TE, EE) is whitened with the precomputed inverse Cholesky
// factor (lower, 6 entries); PP is whitened by 1/sigma_pp.  A block of 256
// threads handles ROWS walkers so the per-multipole constants are read once.
template <class T, int ROWS>
__global__ __launch_bounds__(256) void chi2_block_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const T* __restrict__ mvec,
    int n_ell, int sp, const double* __restrict__ data, const double* __restrict__ linv,
    const double* __restrict__ isig_pp, double cst, double* __restrict__ logl,
    const int* __restrict__ count) {
    __shared__ double red[ROWS][4];
    if (count) B = min<int64_t>(B, *count);
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    if (r0 >= B) return;
    const int64_t n = 4 * (int64_t)sp;
    double s[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) s[r] = 0.0;
    for (int l = threadIdx.x; l < n_ell; l += blockDim.x) {
        const double* L = linv + 6 * (int64_t)l;
        const double l00 = L[0], l10 = L[1], l11 = L[2], l20 = L[3], l21 = L[4], l22 = L[5];
        const double dtt = data[l], dte = data[n_ell + l], dee = data[2 * n_ell + l], dpp = data[3 * n_ell + l];
        const double ip = isig_pp[l];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int64_t row = r0 + r;
            if (row >= B) break;
            const T* mv = mvec + row * n;
            const double rtt = dtt - (double)mv[l], rte = dte - (double)mv[sp + l];
            const double ree = dee - (double)mv[2 * sp + l], rpp = (dpp - (double)mv[3 * sp + l]) * ip;
            const double y0 = l00 * rtt;
            const double y1 = l10 * rtt + l11 * rte;
            const double y2 = l20 * rtt + l21 * rte + l22 * ree;
            s[r] += y0 * y0 + y1 * y1 + y2 * y2 + rpp * rpp;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        double v = wave_sum(s[r]);
        if (lane == 0) red[r][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < ROWS) {
        const int64_t row = r0 + threadIdx.x;
        if (row < B) {
            const double chi2 = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
            const bool ok = in_support(theta + row * ld, d, pk, pa, pb);
            logl[row] = ok ? -0.5 * chi2 + cst : -INFINITY;
        }
    }
}

// ----------------------------------------------- cosmic-variance-limited TT
// One workgroup (four waves) per walker; y = log10 C_l (emulator output), FP64
// accumulation: logL = c - sum_l (k_l/2) (ln 10 y_l + Ch_l 10^-y_l).  Each
// thread sums the multipoles l = t, t + 256, ...; the wave sums are added in
// wave order.  (One wave per walker left each lane a serial chain of ~40
// FP64 exponentials: 17-20 us per call at any batch.)
template <class T>
__global__ __launch_bounds__(256) void cv_loglike_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const T* __restrict__ y, int n, int64_t ldm,
    const double* __restrict__ data, const double* __restrict__ halfk, double cst, double* __restrict__ logl,
    const int* __restrict__ count) {
    __shared__ double red[4];
    const int64_t row = blockIdx.x;
    if (count) B = min<int64_t>(B, *count);
    if (row >= B) return;                                 // whole workgroups
    const T* yr = y + row * ldm;
    // support check, lane i of each wave for parameter i (d <= 64): vector
    // loads, in flight under the sum, tested after it
    const int si = min((int)(threadIdx.x & 63), d - 1);
    const int sk = pk[si];
    const double st = theta[row * ld + si], slo = pa[si], shi = pb[si];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double lc = 2.302585092994045684 * (double)yr[i];     // ln C_l
        s += halfk[i] * (lc + data[i] * exp(-lc));
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    const bool ok = __all(!((sk == NS_PRIOR_UNIFORM) & ((st < slo) | (st > shi))));
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = red[0] + red[1] + red[2] + red[3];
        logl[row] = ok ? cst - tot : -INFINITY;
    }
}

// ------------------------------------------------------------ Gaussian test
__global__ void gauss_kernel(const double* __restrict__ theta, int64_t ld, int64_t B, int d,
                             const int* __restrict__ pk, const double* __restrict__ pa,
                             const double* __restrict__ pb, const double* __restrict__ mu,
                             const double* __restrict__ isig, double cst, double* __restrict__ logl,
                             const int* __restrict__ count) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (count) B = min<int64_t>(B, *count);
    if (row >= B) return;
    const double* th = theta + row * ld;
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        const double r = (th[i] - mu[i]) * isig[i];
        s = fma(r, r, s);
    }
    logl[row] = in_support(th, d, pk, pa, pb) ? -0.5 * s + cst : -INFINITY;
}

// ------------------------------------------------------------ prior transform
__global__ void prior_transform_kernel(const double* __restrict__ u, double* __restrict__ theta,
                                       int64_t ld, int64_t B, int d, const int* __restrict__ pk,
                                       const double* __restrict__ pa, const double* __restrict__ pb,
                                       const int* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (count) B = min<int64_t>(B, *count);
    if (i >= B * d) return;
    const int64_t row = i / d;
    const int c = (int)(i % d);
    const double x = u[row * ld + c];
    theta[row * ld + c] = prior_map(x, pk[c], pa[c], pb[c]);
}

void prior_transform(ns_model* m, const double* u, double* theta, int64_t ld, int64_t B,
                     const int* count, hipStream_t s) {
    const int64_t n = B * m->d;
    if (n == 0) return;
    TraceScope ts(m, s, "prior_transform");
    hipLaunchKernelGGL(prior_transform_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u, theta,
                       ld, B, m->d, m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(),
                       count);
    NS_HIP(hipGetLastError());
}

void gauss_loglike(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl,
                   const int* count, hipStream_t s) {
    TraceScope ts(m, s, "gauss");
    hipLaunchKernelGGL(gauss_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, theta, ld, B, m->d,
                       m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(),
                       m->g_mu.as<double>(), m->g_isig.as<double>(), m->logl_const, logl, count);
    NS_HIP(hipGetLastError());
}

int64_t cmb_spec_stride(const ns_model* m) {
    const int64_t n = m->kind == NS_MODEL_CMB_BLOCK ? m->n_ell_cmb : m->n_data;
    return (n + 31) / 32 * 32;
}
int64_t cmb_row_stride(const ns_model* m) { return (int64_t)m->nets.size() * cmb_spec_stride(m); }

void cmb_chi2(ns_model* m, const double* theta, int64_t ld, int64_t B, const void* mvec, double* logl,
              int prec, const int* count, hipStream_t s) {
    const int* pk = m->prior_kind.as<int>();
    const double* pa = m->prior_a.as<double>();
    const double* pb = m->prior_b.as<double>();
    TraceScope ts(m, s, m->kind == NS_MODEL_CMB_DIAG ? "chi2_diag" : (m->kind == NS_MODEL_CMB_CV ? "cv_loglike"
                                                                                                 : "chi2_block"));
    if (m->kind == NS_MODEL_CMB_CV) {
        dim3 g((unsigned)B);
        if (prec == NS_FP64)
            hipLaunchKernelGGL(cv_loglike_kernel<double>, g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const double*)mvec, m->n_data, cmb_row_stride(m), m->data.as<double>(),
                               m->cv_halfk.as<double>(), m->logl_const, logl, count);
        else
            hipLaunchKernelGGL(cv_loglike_kernel<float>, g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const float*)mvec, m->n_data, cmb_row_stride(m), m->data.as<double>(),
                               m->cv_halfk.as<double>(), m->logl_const, logl, count);
    } else if (m->kind == NS_MODEL_CMB_DIAG) {
        dim3 g((unsigned)((B + 3) / 4));
        if (prec == NS_FP64)
            hipLaunchKernelGGL(chi2_diag_kernel<double>, g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const double*)mvec, m->n_data, cmb_row_stride(m), m->data.as<double>(),
                               m->inv_sigma.as<double>(), m->logl_const, logl, count);
        else
            hipLaunchKernelGGL(chi2_diag_kernel<float>, g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const float*)mvec, m->n_data, cmb_row_stride(m), m->data.as<double>(),
                               m->inv_sigma.as<double>(), m->logl_const, logl, count);
    } else {
        constexpr int R = 8;
        dim3 g((unsigned)((B + R - 1) / R));
        if (prec == NS_FP64)
            hipLaunchKernelGGL((chi2_block_kernel<double, R>), g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const double*)mvec, m->n_ell_cmb, cmb_spec_stride(m), m->data.as<double>(),
                               m->blk_linv.as<double>(), m->inv_sigma_pp.as<double>(), m->logl_const, logl, count);
        else
            hipLaunchKernelGGL((chi2_block_kernel<float, R>), g, dim3(256), 0, s, theta, ld, B, m->d, pk, pa, pb,
                               (const float*)mvec, m->n_ell_cmb, cmb_spec_stride(m), m->data.as<double>(),
                               m->blk_linv.as<double>(), m->inv_sigma_pp.as<double>(), m->logl_const, logl, count);
    }
    NS_HIP(hipGetLastError());
}

// Theory rows of the CMB kinds: spectrum g of walker b sits at columns
// b rs + g sp + i of the emulator output (T); out[b ldo + g nper + i] (double),
// the data order of the likelihood.  Grid-stride over B G nper elements.
template <class T>
__global__ __launch_bounds__(256) void theory_gather_kernel(const T* __restrict__ src, int64_t B, int G, int nper,
                                                            int64_t sp, int64_t rs, double* __restrict__ out,
                                                            int64_t ldo) {
    const int64_t n = (int64_t)G * nper, total = B * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / n, j = e - b * n;
        const int g = (int)(j / nper), i = (int)(j - (int64_t)g * nper);
        out[b * ldo + j] = (double)src[b * rs + g * sp + i];
    }
}

void theory_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* out, int64_t ldo, int prec,
                  hipStream_t s) {
    if (B == 0) return;
    NS_CHECK(m->kind != NS_MODEL_GAUSS, NS_E_UNSUPPORTED, "the Gaussian test model has no theory vector");
    const size_t elem = prec == NS_FP64 ? 8 : 4;
    if (m->kind == NS_MODEL_SHEAR) {
        const int n_k = m->nets[0]->dims.back();
        m->ws_out.ensure((size_t)B * m->n_z * n_k * elem);
        const int id0 = 0, no_log = 0;
        void* out0 = m->ws_out.p;
        emulator_forward(m, &id0, 1, theta, ld, B, &out0, n_k, &no_log, prec, nullptr, s);
        const double* Cv = shear_spectra_from_table(m, theta, ld, B, prec, nullptr, s);
        const size_t row = (size_t)m->n_data * sizeof(double);
        NS_HIP(hipMemcpy2DAsync(out, (size_t)ldo * sizeof(double), Cv, row, row, (size_t)B, hipMemcpyDeviceToDevice,
                                s));
        return;
    }
    // CMB kinds: the emulator with every output transform (C = 10^y where the
    // spectrum is emulated in log10), then a gather into data order
    const int64_t n = cmb_row_stride(m), sp = cmb_spec_stride(m);
    m->ws_out.ensure((size_t)B * n * elem);
    int ids[4];
    void* outs[4];
    const int G = (int)m->nets.size();
    for (int g = 0; g < G; ++g) {
        ids[g] = g;
        outs[g] = m->ws_out.as<char>() + g * sp * elem;
    }
    emulator_forward(m, ids, G, theta, ld, B, outs, n, m->spec_log.data(), prec, nullptr, s);
    const int nper = m->n_data / G;
    const int64_t total = B * m->n_data;
    const dim3 grid((unsigned)std::min<int64_t>((total + 255) / 256, 65536));
    if (prec == NS_FP64)
        hipLaunchKernelGGL(theory_gather_kernel<double>, grid, dim3(256), 0, s, m->ws_out.as<double>(), B, G, nper, sp,
                           n, out, ldo);
    else
        hipLaunchKernelGGL(theory_gather_kernel<float>, grid, dim3(256), 0, s, m->ws_out.as<float>(), B, G, nper, sp,
                           n, out, ldo);
    NS_HIP(hipGetLastError());
}

void loglike_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, int prec,
                   const int* count, hipStream_t s) {
    if (B == 0) return;
    if (m->kind == NS_MODEL_GAUSS) {
        gauss_loglike(m, theta, ld, B, logl, count, s);
        return;
    }
    const size_t elem = prec == NS_FP64 ? 8 : 4;
    if (m->kind == NS_MODEL_CMB_DIAG || m->kind == NS_MODEL_CMB_BLOCK || m->kind == NS_MODEL_CMB_CV) {
        // spectrum g at column g sp of rows of cmb_row_stride: 128-byte aligned
        // output lines for the emulator's stores
        const int64_t n = cmb_row_stride(m), sp = cmb_spec_stride(m);
        m->ws_out.ensure((size_t)B * n * elem);
        int ids[4];
        void* outs[4];
        const int G = (int)m->nets.size();
        for (int g = 0; g < G; ++g) {
            ids[g] = g;
            outs[g] = m->ws_out.as<char>() + g * sp * elem;
        }
        // narrow FP64 networks: emulator and diagonal chi^2 in one launch
        if (m->kind == NS_MODEL_CMB_DIAG && prec == NS_FP64 &&
            emulator_forward_f64_narrow(m, theta, ld, B, nullptr, 0, m->spec_log[0], logl, count, s))
            return;
        // one network in a BF16-operand form: the chi^2 in the emulator's epilogue
        if (emulator_chi2_fused(m, theta, ld, B, logl, prec, count, s)) return;
        // the cosmic-variance stage reads log10 C_l itself
        static const int raw[4] = {0, 0, 0, 0};
        emulator_forward(m, ids, G, theta, ld, B, outs, n, m->kind == NS_MODEL_CMB_CV ? raw : m->spec_log.data(),
                         prec, count, s);
        cmb_chi2(m, theta, ld, B, m->ws_out.p, logl, prec, count, s);
        return;
    }
    // shear: emulator table [B * n_z x n_k], then projection and chi^2
    const int n_k = m->nets[0]->dims.back();
    m->ws_out.ensure((size_t)B * m->n_z * n_k * elem);
    const int id0 = 0, no_log = 0;
    void* out0 = m->ws_out.p;
    emulator_forward(m, &id0, 1, theta, ld, B, &out0, n_k, &no_log, prec, count, s);
    shear_loglike_from_table(m, theta, ld, B, logl, prec, count, s);
}

}  // namespace nsmi
