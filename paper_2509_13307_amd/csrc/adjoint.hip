// Hand-written adjoint of the batched likelihood (input gradients only).
//
// logL = -1/2 |L^{-1}(d - C)|^2 + const, so d logL / dC = L^{-T} L^{-1} (d - C)
// (Cholesky whitening run backwards, FP64).  The CMB seed kernels apply the
// output transform's derivative (C = 10^y: dC/dy = C ln 10; y = mu + sigma o)
// to obtain d logL / d o for the raw network outputs o; emulator_backward
// carries it through the GEMM chain (transposed weights, f'(t) from the
// saved pre-activations) to the emulator inputs; grad_assemble_kernel maps
// input gradients back to theta (summing over networks and redshift rows)
// and adds the direct (non-emulator) part.  Rows outside the prior support
// get logL = -inf and a zero gradient.
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

// CMB seeds: model vector mvec [B x n] (T) -> logL and delta[g][row][n_pad]
// (T) for each of the G networks.  Diagonal: dlogL/dC_i = r_i / sigma_i^2.
// Block: per multipole g3 = Linv^T (Linv r3); PP: r / sigma_pp^2.
struct SeedNet {
    const double* sigma_out;   // [n_out]
    int is_log;
};

// ROWS walkers per workgroup: the data, whitening blocks and output scales of
// a multipole are loaded once for all of them (one walker per workgroup read
// them again for every walker).  Each walker's chi^2 is summed per thread over
// l = t, t + 256, ..., then over the waves in wave order.
template <class T, int ROWS>
__global__ __launch_bounds__(256) void cmb_seed_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const T* __restrict__ mvec, int kind, int n,
    int n_ell, const double* __restrict__ data, const double* __restrict__ isig, const double* __restrict__ linv,
    const double* __restrict__ isig_pp, double cst, SeedNet s0, SeedNet s1, SeedNet s2, SeedNet s3, int n_pad,
    size_t gstride, T* __restrict__ delta, double* __restrict__ logl) {
    __shared__ double red[ROWS][4];
    __shared__ int okr[ROWS];
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    if (r0 >= B) return;
    const int nr = (int)min<int64_t>(ROWS, B - r0);
    if (threadIdx.x < ROWS)
        okr[threadIdx.x] = threadIdx.x < nr && in_support(theta + (r0 + threadIdx.x) * ld, d, pk, pa, pb);
    __syncthreads();
    const SeedNet sn[4] = {s0, s1, s2, s3};
    double chi2[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) chi2[r] = 0.0;
    // d logL / d o of output i of network g for walker r from d logL / d C
    auto put = [&](int r, int g, int i, int64_t moff, double gc, double so) {
        const int64_t row = r0 + r;
        const double C = (double)mvec[row * (int64_t)n + moff];
        const double dv = gc * so * (sn[g].is_log ? C * 2.302585092994045684 : 1.0);
        delta[g * gstride + row * n_pad + i] = okr[r] ? (T)dv : T(0);
    };
    if (kind == NS_MODEL_CMB_DIAG) {
        for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
            if (i < n) {
                const double di = data[i], is = isig[i], so = sn[0].sigma_out[i];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    if (r >= nr) break;
                    const double rr = di - (double)mvec[(r0 + r) * (int64_t)n + i];
                    const double w = rr * is;
                    chi2[r] += w * w;
                    put(r, 0, i, i, w * is, so);
                }
            } else {
                for (int r = 0; r < nr; ++r) delta[(r0 + r) * n_pad + i] = T(0);
            }
        }
    } else {
        for (int l = threadIdx.x; l < n_pad; l += blockDim.x) {
            if (l < n_ell) {
                const double* Lq = linv + 6 * (int64_t)l;
                const double q0 = Lq[0], q1 = Lq[1], q2 = Lq[2], q3 = Lq[3], q4 = Lq[4], q5 = Lq[5];
                const double dtt = data[l], dte = data[n_ell + l], dee = data[2 * n_ell + l];
                const double dpp = data[3 * n_ell + l], ip = isig_pp[l];
                const double so0 = sn[0].sigma_out[l], so1 = sn[1].sigma_out[l], so2 = sn[2].sigma_out[l];
                const double so3 = sn[3].sigma_out[l];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    if (r >= nr) break;
                    const T* mv = mvec + (r0 + r) * (int64_t)n;
                    const double rtt = dtt - (double)mv[l], rte = dte - (double)mv[n_ell + l];
                    const double ree = dee - (double)mv[2 * n_ell + l];
                    const double rpp = dpp - (double)mv[3 * n_ell + l];
                    const double y0 = q0 * rtt, y1 = q1 * rtt + q2 * rte;
                    const double y2 = q3 * rtt + q4 * rte + q5 * ree;
                    const double wp = rpp * ip;
                    chi2[r] += y0 * y0 + y1 * y1 + y2 * y2 + wp * wp;
                    put(r, 0, l, l, q0 * y0 + q1 * y1 + q3 * y2, so0);
                    put(r, 1, l, n_ell + l, q2 * y1 + q4 * y2, so1);
                    put(r, 2, l, 2 * n_ell + l, q5 * y2, so2);
                    put(r, 3, l, 3 * n_ell + l, wp * ip, so3);
                }
            } else {
                for (int r = 0; r < nr; ++r)
                    for (int g = 0; g < 4; ++g) delta[g * gstride + (r0 + r) * n_pad + l] = T(0);
            }
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const double v = wave_sum(chi2[r]);
        if (lane == 0) red[r][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < nr) {
        const double c2 = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
        logl[r0 + threadIdx.x] = okr[threadIdx.x] ? -0.5 * c2 + cst : -INFINITY;
    }
}

constexpr int SEED_ROWS = 8;

// Cosmic-variance seeds: y = log10 C_l, logL = c - sum (k/2)(ln 10 y + Ch 10^-y),
// d logL / d y_l = -(k/2) ln 10 (1 - Ch_l / C_l); delta = that times sigma_out.
template <class T>
__global__ __launch_bounds__(256) void cv_seed_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const T* __restrict__ y, int n,
    const double* __restrict__ data, const double* __restrict__ halfk, const double* __restrict__ sigma_out,
    double cst, int n_pad, T* __restrict__ delta, double* __restrict__ logl) {
    __shared__ double red[4];
    const int64_t row = blockIdx.x;
    if (row >= B) return;
    const bool ok = in_support(theta + row * ld, d, pk, pa, pb);
    const T* yr = y + row * (int64_t)n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
        double dv = 0.0;
        if (i < n) {
            const double lc = 2.302585092994045684 * (double)yr[i];
            const double r = data[i] * exp(-lc);
            s += halfk[i] * (lc + r);
            dv = -halfk[i] * 2.302585092994045684 * (1.0 - r) * sigma_out[i];
        }
        delta[row * n_pad + i] = ok ? (T)dv : T(0);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = red[0] + red[1] + red[2] + red[3];
        logl[row] = ok ? cst - t : -INFINITY;
    }
}

// grad[w][c] = direct[w][c] + sum_g sum_z sum_k [src_k == c] gx[g][w rpw + z][k]; zero outside the support.
__global__ void grad_assemble_kernel(int64_t B, int d, int G, int rpw, int n_in, const int* __restrict__ src,
                                     const double* __restrict__ gx, const double* __restrict__ direct,
                                     const double* __restrict__ logl, double* __restrict__ grad) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * d) return;
    const int64_t w = e / d;
    const int c = (int)(e % d);
    double s = direct ? direct[e] : 0.0;
    const int64_t rows = B * rpw;
    for (int g = 0; g < G; ++g)
        for (int z = 0; z < rpw; ++z)
            for (int k = 0; k < n_in; ++k)
                if (src[k] == c) s += gx[((int64_t)g * rows + w * rpw + z) * n_in + k];
    grad[e] = logl[w] == -INFINITY ? 0.0 : s;
}

__global__ void gauss_grad_kernel(const double* __restrict__ theta, int64_t ld, int64_t B, int d,
                                  const int* __restrict__ pk, const double* __restrict__ pa,
                                  const double* __restrict__ pb, const double* __restrict__ mu,
                                  const double* __restrict__ isig, double cst, double* __restrict__ logl,
                                  double* __restrict__ grad) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= B) return;
    const double* th = theta + row * ld;
    const bool ok = in_support(th, d, pk, pa, pb);
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        const double r = (th[i] - mu[i]) * isig[i];
        s = fma(r, r, s);
        grad[row * d + i] = ok ? -r * isig[i] : 0.0;
    }
    logl[row] = ok ? -0.5 * s + cst : -INFINITY;
}

void loglike_grad_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, double* grad,
                        int prec, hipStream_t s) {
    if (B == 0) return;
    const int* pk = m->prior_kind.as<int>();
    const double* pa = m->prior_a.as<double>();
    const double* pb = m->prior_b.as<double>();
    if (m->kind == NS_MODEL_GAUSS) {
        TraceScope ts(m, s, "gauss_grad");
        hipLaunchKernelGGL(gauss_grad_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, theta, ld, B, m->d,
                           pk, pa, pb, m->g_mu.as<double>(), m->g_isig.as<double>(), m->logl_const, logl, grad);
        NS_HIP(hipGetLastError());
        return;
    }
    const bool f64 = prec == NS_FP64;
    const size_t elem = f64 ? 8 : 4;
    const int G = (int)m->nets.size();
    int ids[4] = {0, 1, 2, 3};
    const Net& net0 = *m->nets[0];
    const int L = net0.n_layers;
    const int rpw = net0.out_mu_rows;
    const int64_t rows = B * rpw;
    size_t max_w = 0;
    for (int l = 1; l < L; ++l) max_w = std::max(max_w, (size_t)net0.dims[l]);
    const int n_pad = net0.layers[L - 1]->n_pad;
    const size_t gstride = (size_t)rows * std::max(max_w, (size_t)n_pad);
    m->ws_gact[0].ensure(G * gstride * elem);
    m->ws_gact[1].ensure(G * gstride * elem);
    // reduced forms: forward in the requested form, adjoint in FP32
    const int bprec = f64 ? NS_FP64 : NS_FP32;
    if (m->kind == NS_MODEL_CMB_CV) {
        const int64_t n = m->n_data;
        m->ws_out.ensure((size_t)B * n * elem);
        void* outs[1] = {m->ws_out.p};
        const int raw[1] = {0};
        emulator_forward(m, ids, 1, theta, ld, B, outs, n, raw, prec, nullptr, s, true);
        {
            TraceScope ts(m, s, "adj_seed_cv");
            if (f64)
                hipLaunchKernelGGL(cv_seed_kernel<double>, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, m->d, pk,
                                   pa, pb, m->ws_out.as<double>(), (int)n, m->data.as<double>(),
                                   m->cv_halfk.as<double>(), m->nets[0]->out_sigma64.as<double>(), m->logl_const,
                                   n_pad, m->ws_gact[0].as<double>(), logl);
            else
                hipLaunchKernelGGL(cv_seed_kernel<float>, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, m->d, pk,
                                   pa, pb, m->ws_out.as<float>(), (int)n, m->data.as<double>(),
                                   m->cv_halfk.as<double>(), m->nets[0]->out_sigma64.as<double>(), m->logl_const,
                                   n_pad, m->ws_gact[0].as<float>(), logl);
            NS_HIP(hipGetLastError());
        }
        emulator_backward(m, ids, 1, B, bprec, s);
        TraceScope ts(m, s, "adj_assemble");
        grad_assemble(m, B, 1, rpw, nullptr, logl, grad, s);
        return;
    }
    if (m->kind == NS_MODEL_CMB_DIAG || m->kind == NS_MODEL_CMB_BLOCK) {
        const int64_t n = m->n_data;
        m->ws_out.ensure((size_t)B * n * elem);
        void* outs[4];
        int64_t off = 0;
        for (int g = 0; g < G; ++g) {
            outs[g] = m->ws_out.as<char>() + off * elem;
            off += m->nets[g]->dims.back();
        }
        emulator_forward(m, ids, G, theta, ld, B, outs, n, m->spec_log.data(), prec, nullptr, s, true);
        SeedNet sn[4] = {};
        for (int g = 0; g < G; ++g) sn[g] = SeedNet{m->nets[g]->out_sigma64.as<double>(), m->spec_log[g]};
        {
            TraceScope ts(m, s, "adj_seed_chi2");
            if (f64)
                hipLaunchKernelGGL((cmb_seed_kernel<double, SEED_ROWS>), dim3((unsigned)((B + SEED_ROWS - 1) / SEED_ROWS)),
                                   dim3(256), 0, s, theta, ld, B, m->d,
                                   pk, pa, pb, m->ws_out.as<double>(), m->kind, (int)n, m->n_ell_cmb,
                                   m->data.as<double>(), m->inv_sigma.as<double>(), m->blk_linv.as<double>(),
                                   m->inv_sigma_pp.as<double>(), m->logl_const, sn[0], sn[1], sn[2], sn[3], n_pad,
                                   gstride, m->ws_gact[0].as<double>(), logl);
            else
                hipLaunchKernelGGL((cmb_seed_kernel<float, SEED_ROWS>), dim3((unsigned)((B + SEED_ROWS - 1) / SEED_ROWS)),
                                   dim3(256), 0, s, theta, ld, B, m->d,
                                   pk, pa, pb, m->ws_out.as<float>(), m->kind, (int)n, m->n_ell_cmb,
                                   m->data.as<double>(), m->inv_sigma.as<double>(), m->blk_linv.as<double>(),
                                   m->inv_sigma_pp.as<double>(), m->logl_const, sn[0], sn[1], sn[2], sn[3], n_pad,
                                   gstride, m->ws_gact[0].as<float>(), logl);
            NS_HIP(hipGetLastError());
        }
        emulator_backward(m, ids, G, B, bprec, s);
        TraceScope ts(m, s, "adj_assemble");
        grad_assemble(m, B, G, rpw, nullptr, logl, grad, s);
        return;
    }
    shear_grad(m, theta, ld, B, logl, grad, prec, s);
}

void grad_assemble(ns_model* m, int64_t B, int G, int rpw, const double* direct, const double* logl, double* grad,
                   hipStream_t s) {
    hipLaunchKernelGGL(grad_assemble_kernel, dim3((unsigned)((B * m->d + 255) / 256)), dim3(256), 0, s, B, m->d, G,
                       rpw, m->nets[0]->dims[0], m->emu_src_d.as<int>(), m->ws_gx.as<double>(), direct, logl, grad);
    NS_HIP(hipGetLastError());
}

}  // namespace nsmi
