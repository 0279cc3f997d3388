// Adjoint of the cosmic-shear likelihood (App. A of the paper), input
// gradients only.
//
// Reverse mode runs from logL back to the emulator table:
//   dense chi^2:   g_C = L^{-T} L^{-1} (d - C)                                  (FP64)
//   Limber (A2):   C_pb = f_p sum_j W_a(j) W_b(j) P_bj wq_j,  f_p = (1+m_a)(1+m_b)
//                  -> g(P wq)_bj, g W_i(j), g wq_j, and g chi_j through k = (l+1/2)/chi_j
//   P lookup:      P = 10^{CR(t; Yhat_j(c))}, Yhat = spline along z of the table
//                  -> scatter into g Y, g M (second derivatives), then M = S(Y)
//                  is transposed (zspline_adjoint_kernel) -> g Y -> emulator backward.
// Forward mode covers the per-walker background and windows, which depend on
// few parameters: tangents of chi, J, E, D, n_i, W_i and wq in the directions
// (Om, h, w0, wa) and, per bin, (Dz_i, A_IA_i); the direct gradient is
//   sum_j [ sum_i gW_i(j) dW_i(j) + g wq_j dwq_j + g chi_j dchi_j ].
// Every Limber-adjoint term belongs to one a-node, so thread j owns node j.
#include "devutil.h"
#include "nsmi.h"
#include "shear_common.h"

namespace nsmi {

// ------------------------------------------------------- dense chi^2 adjoint
// 16 walkers per block: y = L^{-1}d - L^{-1}C, g_C = L^{-T} y, logL.
constexpr int DA_W = 16;
__global__ __launch_bounds__(256) void dense_chi2_adjoint_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const double* __restrict__ C, int n,
    const double* __restrict__ Linv, const double* __restrict__ LinvT, const double* __restrict__ wv, double cst,
    double* __restrict__ logl, double* __restrict__ gC) {
    extern __shared__ double sm[];
    double* Cs = sm;                   // [DA_W][n]
    double* Ys = sm + DA_W * n;        // [DA_W][n]
    __shared__ double red[DA_W][16];
    const int64_t w0 = (int64_t)blockIdx.x * DA_W;
    if (w0 >= B) return;
    for (int e = threadIdx.x; e < DA_W * n; e += 256) {
        const int64_t w = w0 + e / n;
        Cs[e] = w < B ? C[w * n + e % n] : 0.0;
    }
    __syncthreads();
    const int wk = threadIdx.x % DA_W, part = threadIdx.x / DA_W;
    double s = 0.0;
    for (int i = part; i < n; i += 256 / DA_W) {
        const double* Li = Linv + (int64_t)i * n;
        double acc = 0.0;
        for (int k = 0; k <= i; ++k) acc = fma(Li[k], Cs[wk * n + k], acc);
        const double y = wv[i] - acc;
        Ys[wk * n + i] = y;
        s = fma(y, y, s);
    }
    red[wk][part] = s;
    __syncthreads();
    const int64_t w = w0 + wk;
    bool ok = false;
    if (w < B) {
        ok = true;
        const double* th = theta + w * ld;
        for (int i = 0; i < d; ++i)
            if (pk[i] == NS_PRIOR_UNIFORM && (th[i] < pa[i] || th[i] > pb[i])) ok = false;
    }
    for (int k = part; k < n; k += 256 / DA_W) {
        const double* Lk = LinvT + (int64_t)k * n;     // row k of L^{-T}: entries i >= k
        double acc = 0.0;
        for (int i = k; i < n; ++i) acc = fma(Lk[i], Ys[wk * n + i], acc);
        if (w < B) gC[w * n + k] = ok ? acc : 0.0;
    }
    if (part == 0 && w < B) {
        double chi2 = 0.0;
        for (int p = 0; p < 256 / DA_W; ++p) chi2 += red[wk][p];
        logl[w] = ok ? -0.5 * chi2 + cst : -INFINITY;
    }
}

// ---------------------------------------------------- Limber + window adjoint
// One workgroup (256 threads, thread j = a-node j) per walker.
// Outputs: gY, gM [B x n_z x n_k] (accumulated, must start at zero) and the
// direct gradient gdir [B x d] (fully written).
template <class T>
__global__ __launch_bounds__(256) void limber_adjoint_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, ShearGeom G,
    const int* __restrict__ pidx, const double* __restrict__ pfix, const double* __restrict__ nz_mean,
    const double* __restrict__ agrid, const int* __restrict__ zidx, const double* __restrict__ zcoef,
    const double* __restrict__ ell, const T* __restrict__ Ytab, const T* __restrict__ Mtab,
    const double* __restrict__ Cv, const double* __restrict__ gC, double* __restrict__ gY,
    double* __restrict__ gM, double* __restrict__ gdir) {
    __shared__ double scan[20 * 256];
    __shared__ double Hs[64 * 55];          // G_pb f_p, pair-major
    __shared__ double red[32][4];
    __shared__ double node_chi[256];
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int na = G.n_a, nb = G.n_bins, ne = G.n_ell, npair = G.n_pairs;
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double ob = phys(0), oc = phys(1), h = phys(2), w0 = phys(5), wa = phys(6);
    const double Om = (ob + oc) / (h * h);
    const double cH0 = C_KM_S / (100.0 * h), H0c = 1.0 / cH0;
    const int nout = npair * ne;

    // H_pb = g_C[pb] (1 + m_a)(1 + m_b)
    for (int o = t; o < nout; o += 256) {
        const int p = o / ne;
        int a = 0, rem = p;
        while (rem >= nb - a) { rem -= nb - a; ++a; }
        const int bb = a + rem;
        Hs[o] = gC[w * nout + o] * (1.0 + phys(9 + 2 * nb + a)) * (1.0 + phys(9 + 2 * nb + bb));
    }

    // ---- background with tangents in (Om, h, w0, wa)
    struct EB { double E, dE[4]; };
    auto Eval = [&](double a) {
        EB r;
        const double X = pow(a, -3.0 * (1.0 + w0 + wa)) * exp(-3.0 * wa * (1.0 - a));
        r.E = sqrt(Om / (a * a * a) + (1.0 - Om) * X);
        const double la = log(a);
        r.dE[0] = (1.0 / (a * a * a) - X) / (2.0 * r.E);
        r.dE[1] = 0.0;
        r.dE[2] = (1.0 - Om) * X * (-3.0 * la) / (2.0 * r.E);
        r.dE[3] = (1.0 - Om) * X * (-3.0 * la - 3.0 * (1.0 - a)) / (2.0 * r.E);
        return r;
    };
    // f = cH0/(a^2 E), g = (Om a^-3/E^2)^0.55 / a, with tangents
    auto FG = [&](double a, double* f, double* df, double* g, double* dg) {
        const EB e = Eval(a);
        *f = cH0 / (a * a * e.E);
        *g = pow(Om / (a * a * a) / (e.E * e.E), GROWTH_INDEX) / a;
        for (int q = 0; q < 4; ++q) {
            df[q] = -*f * e.dE[q] / e.E;
            dg[q] = -2.0 * GROWTH_INDEX * *g * e.dE[q] / e.E;
        }
        df[1] += -*f / h;
        dg[0] += GROWTH_INDEX * *g / Om;
    };
    const bool node = t < na;
    const double a = node ? agrid[t] : 1.0;
    double fa = 0.0, dfa[4] = {0, 0, 0, 0}, ga, dga[4];
    FG(a, &fa, dfa, &ga, dga);
    const EB ea = Eval(a);
    double inc[10];
    for (int q = 0; q < 10; ++q) inc[q] = 0.0;
    if (node && t < na - 1) {
        const double a1 = agrid[t + 1], am = 0.5 * (a + a1);
        double fm, dfm[4], gm, dgm[4], f1, df1[4], g1, dg1[4];
        FG(am, &fm, dfm, &gm, dgm);
        FG(a1, &f1, df1, &g1, dg1);
        inc[0] = G.da / 6.0 * (fa + 4.0 * fm + f1);
        inc[1] = G.da / 6.0 * (ga + 4.0 * gm + g1);
        for (int q = 0; q < 4; ++q) {
            inc[2 + q] = G.da / 6.0 * (dfa[q] + 4.0 * dfm[q] + df1[q]);
            inc[6 + q] = G.da / 6.0 * (dga[q] + 4.0 * dgm[q] + dg1[q]);
        }
    }
    block_scan<10>(inc, scan, false);
    // exclusive values at node t
    for (int q = 0; q < 10; ++q) scan[q * 256 + t] = inc[q];
    __syncthreads();
    double bg[10];
    for (int q = 0; q < 10; ++q) bg[q] = (node && t > 0) ? scan[q * 256 + t - 1] : 0.0;
    __syncthreads();
    const double chi = bg[0], D = exp(-bg[1]);
    double dchi[4], dlnD[4];
    for (int q = 0; q < 4; ++q) { dchi[q] = bg[2 + q]; dlnD[q] = -bg[6 + q]; }
    node_chi[t] = chi;
    const double E = ea.E;
    const double qw = (t == 0 || t == na - 1) ? 0.5 * G.da : G.da;

    // ---- n_i(z) with Dz tangents, normalisation
    const double z = 1.0 / a - 1.0;
    double n[MAXB], dn[MAXB];
    for (int i = 0; i < nb; ++i) {
        const double mu = nz_mean[i] + phys(9 + nb + i);
        const double dz = z - mu;
        const double raw = (node && t > 0) ? exp(-dz * dz / (2.0 * G.nz_sigma * G.nz_sigma)) : 0.0;
        n[i] = raw;
        dn[i] = raw * dz / (G.nz_sigma * G.nz_sigma);
    }
    for (int i = 0; i < nb; ++i) {
        double v0 = wave_sum(node ? qw * n[i] / (a * a) : 0.0);
        double v1 = wave_sum(node ? qw * dn[i] / (a * a) : 0.0);
        if (lane == 0) { red[2 * i][wid] = v0; red[2 * i + 1][wid] = v1; }
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const double N = red[2 * i][0] + red[2 * i][1] + red[2 * i][2] + red[2 * i][3];
        const double dN = red[2 * i + 1][0] + red[2 * i + 1][1] + red[2 * i + 1][2] + red[2 * i + 1][3];
        n[i] /= N;
        dn[i] = dn[i] / N - n[i] * dN / N;
    }
    __syncthreads();

    // ---- reverse cumulative trapezoids G0, G1 and their tangents, 5 bins per pass
    // per bin: G0, G1, dG0/dDz, dG1/dDz, dG1/d(Om, h, w0, wa)
    double G0[MAXB], G1[MAXB], G0z[MAXB], G1z[MAXB], G1c[MAXB][4];
    const double a2 = a * a;
    for (int b0 = 0; b0 < nb; b0 += 5) {
        const int cnt = nb - b0 < 5 ? nb - b0 : 5;
        // integrands at this node: g0 = n/a^2, g1 = n/(a^2 chi), tangents
        double v[20];
        for (int q = 0; q < 20; ++q) v[q] = 0.0;
        for (int c = 0; c < cnt; ++c) {
            const int i = b0 + c;
            v[c] = node ? n[i] / a2 : 0.0;
            v[5 + c] = (node && t > 0) ? n[i] / (a2 * chi) : 0.0;
            v[10 + c] = node ? dn[i] / a2 : 0.0;
            v[15 + c] = (node && t > 0) ? dn[i] / (a2 * chi) : 0.0;
        }
        // segment [t, t+1] from the neighbour's integrand
        for (int q = 0; q < 20; ++q) scan[q * 256 + t] = v[q];
        __syncthreads();
        double sg[20];
        const bool has = node && t < na - 1;
        for (int q = 0; q < 20; ++q) sg[q] = has ? 0.5 * G.da * (v[q] + scan[q * 256 + t + 1]) : 0.0;
        __syncthreads();
        block_scan<20>(sg, scan, true);
        for (int c = 0; c < cnt; ++c) {
            G0[b0 + c] = sg[c];
            G1[b0 + c] = sg[5 + c];
            G0z[b0 + c] = sg[10 + c];
            G1z[b0 + c] = sg[15 + c];
        }
        // cosmological tangents of G1: integrand -n chi_dot / (a^2 chi^2)
        for (int q = 0; q < 20; ++q) v[q] = 0.0;
        for (int c = 0; c < cnt; ++c)
            for (int q = 0; q < 4; ++q)
                v[4 * c + q] = (node && t > 0) ? -n[b0 + c] * dchi[q] / (a2 * chi * chi) : 0.0;
        for (int q = 0; q < 20; ++q) scan[q * 256 + t] = v[q];
        __syncthreads();
        for (int q = 0; q < 20; ++q) sg[q] = has ? 0.5 * G.da * (v[q] + scan[q * 256 + t + 1]) : 0.0;
        __syncthreads();
        block_scan<20>(sg, scan, true);
        for (int c = 0; c < cnt; ++c)
            for (int q = 0; q < 4; ++q) G1c[b0 + c][q] = sg[4 * c + q];
    }

    // ---- windows and tangents: directions 0..3 = (Om, h, w0, wa), 4 = Dz_i, 5 = A_i
    double W[MAXB], dW[MAXB][6];
    const double pref = 1.5 * Om * H0c * H0c;
    const double dpref[4] = {pref / Om, 2.0 * pref / h, 0.0, 0.0};
    const double dlnE[4] = {ea.dE[0] / E, 0.0, ea.dE[2] / E, ea.dE[3] / E};
    for (int i = 0; i < nb; ++i) {
        const double Q = G0[i] - chi * G1[i];
        const double Wg = pref * chi / a * Q;
        const double A = phys(9 + i);
        const double base = C1_RHOCR * Om * H0c * E / D;     // W^I = -A n base
        const double WI = -A * n[i] * base;
        W[i] = node ? Wg + WI : 0.0;
        for (int q = 0; q < 4; ++q) {
            const double dQ = -dchi[q] * G1[i] - chi * G1c[i][q];
            const double dWg = dpref[q] * chi / a * Q + pref * dchi[q] / a * Q + pref * chi / a * dQ;
            double dlnbase = dlnE[q] - dlnD[q];
            if (q == 0) dlnbase += 1.0 / Om;
            if (q == 1) dlnbase += 1.0 / h;
            dW[i][q] = node ? dWg + WI * dlnbase : 0.0;
        }
        const double dQz = G0z[i] - chi * G1z[i];
        dW[i][4] = node ? pref * chi / a * dQz - A * dn[i] * base : 0.0;
        dW[i][5] = node ? -n[i] * base : 0.0;
    }
    // wq = q J / chi^2 and tangents
    double wq = 0.0, dwq[4] = {0, 0, 0, 0};
    if (node && t > 0) {
        wq = qw * fa / (chi * chi);
        for (int q = 0; q < 4; ++q) dwq[q] = wq * (dfa[q] / fa - 2.0 * dchi[q] / chi);
    }
    __syncthreads();

    // ---- Limber adjoint at node t, all multipoles
    double gW[MAXB];
    for (int i = 0; i < nb; ++i) gW[i] = 0.0;
    double gwq = 0.0, gchi = 0.0;
    if (node && t > 0) {
        const int nn = zidx[t];
        const double c0 = zcoef[4 * t], c1 = zcoef[4 * t + 1], c2 = zcoef[4 * t + 2], c3 = zcoef[4 * t + 3];
        const T* Yw = Ytab + w * (int64_t)G.n_z * G.n_k;
        const T* Mw = Mtab + w * (int64_t)G.n_z * G.n_k;
        double* gYw = gY + w * (int64_t)G.n_z * G.n_k;
        double* gMw = gM + w * (int64_t)G.n_z * G.n_k;
        for (int b = 0; b < ne; ++b) {
            const double k = (ell[b] + 0.5) / chi;
            if (!(k >= G.k_min && k <= G.k_max)) continue;
            const double s = (log10(k) - G.u0) / G.du;
            int i0 = (int)floor(s);
            i0 = i0 < 0 ? 0 : (i0 > G.n_k - 2 ? G.n_k - 2 : i0);
            const double tt = s - i0;
            auto Yz = [&](int col) {
                const int64_t o0 = (int64_t)nn * G.n_k + col, o1 = o0 + G.n_k;
                return c0 * (double)Yw[o0] + c1 * (double)Yw[o1] + c2 * (double)Mw[o0] + c3 * (double)Mw[o1];
            };
            const bool lo_ghost = i0 == 0, hi_ghost = i0 + 2 >= G.n_k;
            const double p0 = Yz(i0), p1 = Yz(i0 + 1);
            const double pm = lo_ghost ? 2.0 * p0 - p1 : Yz(i0 - 1);
            const double p2 = hi_ghost ? 2.0 * p1 - p0 : Yz(i0 + 2);
            const double m0 = 0.5 * (p1 - pm), m1 = 0.5 * (p2 - p0);
            const double t2 = tt * tt, t3 = t2 * tt;
            const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + tt, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
            const double lp = h00 * p0 + h10 * m0 + h01 * p1 + h11 * m1;
            const double dlp_dt = (6 * t2 - 6 * tt) * p0 + (3 * t2 - 4 * tt + 1) * m0 + (-6 * t2 + 6 * tt) * p1 +
                                  (3 * t2 - 2 * tt) * m1;
            const double P = exp(lp * LN10);
            const double Pw = P * wq;
            // gPw = sum_p H_pb W_a W_b; gW accumulation
            double gPw = 0.0;
            int p = 0;
            for (int ia = 0; ia < nb; ++ia)
                for (int ib = ia; ib < nb; ++ib, ++p) {
                    const double Hv = Hs[p * ne + b];
                    gPw += Hv * W[ia] * W[ib];
                    if (ia == ib) {
                        gW[ia] += 2.0 * Hv * Pw * W[ia];
                    } else {
                        gW[ia] += Hv * Pw * W[ib];
                        gW[ib] += Hv * Pw * W[ia];
                    }
                }
            gwq += gPw * P;
            const double gP = gPw * wq;
            gchi += gP * (-P * dlp_dt / (G.du * chi));
            const double glp = gP * P * LN10;
            // d lp / d (pm, p0, p1, p2), ghosts folded into the real columns
            double wm = -0.5 * h10, w0c = h00 - 0.5 * h11, w1c = h01 + 0.5 * h10, w2 = 0.5 * h11;
            if (lo_ghost) { w0c += 2.0 * wm; w1c -= wm; wm = 0.0; }
            if (hi_ghost) { w1c += 2.0 * w2; w0c -= w2; w2 = 0.0; }
            auto scatter = [&](int col, double wgt) {
                const double gy = glp * wgt;
                const int64_t o0 = (int64_t)nn * G.n_k + col, o1 = o0 + G.n_k;
                atomicAdd(&gYw[o0], c0 * gy);
                atomicAdd(&gYw[o1], c1 * gy);
                atomicAdd(&gMw[o0], c2 * gy);
                atomicAdd(&gMw[o1], c3 * gy);
            };
            if (!lo_ghost) scatter(i0 - 1, wm);
            scatter(i0, w0c);
            scatter(i0 + 1, w1c);
            if (!hi_ghost) scatter(i0 + 2, w2);
        }
    }

    // ---- direct gradient: reduce over nodes
    double acc[4 + 2 * MAXB];
    for (int q = 0; q < 4; ++q) {
        double v = gwq * dwq[q] + gchi * dchi[q];
        for (int i = 0; i < nb; ++i) v += gW[i] * dW[i][q];
        acc[q] = v;
    }
    for (int i = 0; i < nb; ++i) {
        acc[4 + i] = gW[i] * dW[i][4];
        acc[4 + nb + i] = gW[i] * dW[i][5];
    }
    const int nacc = 4 + 2 * nb;
    __syncthreads();
    for (int q = 0; q < nacc; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[q][wid] = v;
    }
    __syncthreads();
    if (t < d) gdir[w * d + t] = 0.0;
    __syncthreads();
    if (t == 0) {
        double tot[4 + 2 * MAXB];
        for (int q = 0; q < nacc; ++q) tot[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
        // (Om, h) -> (omega_b, omega_cdm, h)
        const double dOm = tot[0];
        auto add = [&](int slot, double v) { if (pidx[slot] >= 0) gdir[w * d + pidx[slot]] += v; };
        add(0, dOm / (h * h));
        add(1, dOm / (h * h));
        add(2, tot[1] - 2.0 * Om / h * dOm);
        add(5, tot[2]);
        add(6, tot[3]);
        for (int i = 0; i < nb; ++i) {
            add(9 + nb + i, tot[4 + i]);
            add(9 + i, tot[4 + nb + i]);
        }
        // multiplicative biases: dC_pb/dm_i = C_pb [(i==a) + (i==b)] / (1 + m_i)
        for (int i = 0; i < nb; ++i) {
            double v = 0.0;
            int p = 0;
            for (int ia = 0; ia < nb; ++ia)
                for (int ib = ia; ib < nb; ++ib, ++p) {
                    const int mult = (ia == i) + (ib == i);
                    if (!mult) continue;
                    for (int b = 0; b < ne; ++b)
                        v += gC[w * nout + p * ne + b] * Cv[w * nout + p * ne + b] * mult;
                }
            add(9 + 2 * nb + i, v / (1.0 + phys(9 + 2 * nb + i)));
        }
    }
}

// ------------------------------------------------------------ spline adjoint
// gY += S^T gM for the not-a-knot spline of each (walker, k) column, then
// delta_out[row = w n_z + n][c] = gY[n][c] sigma_out[c] (padded to n_pad).
template <class T>
__global__ __launch_bounds__(256) void zspline_adjoint_kernel(double* __restrict__ gY, double* __restrict__ gM,
                                                              int64_t B, int nz, int nk, double h,
                                                              const double* __restrict__ sigma_out, int n_pad,
                                                              T* __restrict__ delta) {
    __shared__ double cps[256];
    if (threadIdx.x == 0) {
        double c = 0.0;
        for (int n = 2; n <= nz - 3 && n < 256; ++n) {
            c = 1.0 / (4.0 - (n == 2 ? 0.0 : c));
            cps[n] = c;
        }
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= B * n_pad) return;
    const int64_t w = g / n_pad;
    const int c = (int)(g % n_pad);
    if (c >= nk) {
        for (int n = 0; n < nz; ++n) delta[(w * nz + n) * n_pad + c] = T(0);
        return;
    }
    double* gy = gY + w * nz * nk + c;
    double* gm = gM + w * nz * nk + c;
    auto Y = [&](int n) -> double& { return gy[(int64_t)n * nk]; };
    auto Mg = [&](int n) -> double& { return gm[(int64_t)n * nk]; };
    const double ih2 = 1.0 / (h * h);
    // M_0 = 2 M_1 - M_2 and M_{N-1} = 2 M_{N-2} - M_{N-3}: fold their adjoints
    // into the other nodes first (valid for every nz >= 4)
    const double g0 = Mg(0), gl = Mg(nz - 1);
    Mg(1) += 2.0 * g0;
    Mg(2) -= g0;
    Mg(nz - 2) += 2.0 * gl;
    Mg(nz - 3) -= gl;
    double gM1 = Mg(1);
    double gMb = Mg(nz - 2);
    if (nz > 4) {
        // interior (1,4,1) system is symmetric: g_rhs = T^{-1} gM_interior (same Thomas sweep)
        double dp = 0.0;
        for (int n = 2; n <= nz - 3; ++n) {
            dp = (Mg(n) - (n == 2 ? 0.0 : dp)) * cps[n];
            Mg(n) = dp;
        }
        double next = dp;
        for (int n = nz - 4; n >= 2; --n) {
            next = Mg(n) - cps[n] * next;
            Mg(n) = next;
        }
        // rhs_n = 6 d2Y_n / h^2 - [n == 2] M_1 - [n == nz-3] M_{N-2}
        gM1 -= Mg(2);
        gMb -= Mg(nz - 3);
        for (int n = 2; n <= nz - 3; ++n) {
            const double gr = 6.0 * ih2 * Mg(n);
            Y(n + 1) += gr;
            Y(n) -= 2.0 * gr;
            Y(n - 1) += gr;
        }
    }
    // M_1 = d2Y_1 / h^2, M_{N-2} = d2Y_{N-2} / h^2
    Y(2) += gM1 * ih2; Y(1) -= 2.0 * gM1 * ih2; Y(0) += gM1 * ih2;
    Y(nz - 1) += gMb * ih2; Y(nz - 2) -= 2.0 * gMb * ih2; Y(nz - 3) += gMb * ih2;
    const double sg = sigma_out[c];
    for (int n = 0; n < nz; ++n) delta[(w * nz + n) * n_pad + c] = (T)(Y(n) * sg);
}

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ------------------------------------------------------------------ driver
void shear_grad(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, double* grad, int prec,
                hipStream_t s) {
    NS_CHECK(!m->z_linear && m->n_a <= 256, NS_E_UNSUPPORTED,
             "the shear gradient covers the cubic z-spline on at most 256 nodes");
    const bool f64 = prec == NS_FP64;
    const size_t elem = f64 ? 8 : 4;
    const int nk = m->n_k, nz = m->n_z, n = m->n_data, d = m->d;
    const int64_t rows = B * nz;
    // forward: emulator table (with pre-activation saves), spline, spectra
    m->ws_out.ensure((size_t)B * nz * nk * elem);
    const int id0 = 0, no_log = 0;
    void* out0 = m->ws_out.p;
    emulator_forward(m, &id0, 1, theta, ld, B, &out0, nk, &no_log, prec, nullptr, s, true);
    shear_loglike_from_table(m, theta, ld, B, logl, prec, nullptr, s);
    const size_t mbytes = (size_t)B * nz * nk * elem;
    const void* Mtab = m->ws_aux.p;
    const double* Cv = reinterpret_cast<const double*>(m->ws_aux.as<char>() + mbytes);
    // adjoint scratch: gC [B n], gY, gM [B nz nk], gdir [B d]
    const size_t ntab = (size_t)B * nz * nk;
    m->ws_grad.ensure(((size_t)B * n + 2 * ntab + (size_t)B * d) * sizeof(double));
    double* gC = m->ws_grad.as<double>();
    double* gY = gC + (size_t)B * n;
    double* gM = gY + ntab;
    double* gdir = gM + ntab;
    {
        TraceScope ts(m, s, "adj_dense_chi2");
        const size_t sm = 2 * (size_t)DA_W * n * sizeof(double);
        NS_CHECK(sm <= 160 * 1024, NS_E_UNSUPPORTED, "data vector too long for the chi^2 adjoint");
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_adjoint_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sm));
        hipLaunchKernelGGL(dense_chi2_adjoint_kernel, dim3((unsigned)((B + DA_W - 1) / DA_W)), dim3(256), sm, s, theta,
                           ld, B, d, m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(), Cv, n,
                           m->cov_linv.as<double>(), m->cov_linvT.as<double>(), m->cov_w.as<double>(), m->logl_const,
                           logl, gC);
        NS_HIP(hipGetLastError());
    }
    {
        TraceScope ts(m, s, "adj_limber");
        hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, gY, (int64_t)(2 * ntab));
        const ShearGeom G = shear_geom(m);
        if (f64)
            hipLaunchKernelGGL(limber_adjoint_kernel<double>, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, d, G,
                               m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->nz_mean_d.as<double>(),
                               m->agrid_d.as<double>(), m->zsp_idx_d.as<int>(), m->zsp_coef_d.as<double>(),
                               m->ell_d.as<double>(), m->ws_out.as<double>(), (const double*)Mtab, Cv, gC, gY, gM, gdir);
        else
            hipLaunchKernelGGL(limber_adjoint_kernel<float>, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, d, G,
                               m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->nz_mean_d.as<double>(),
                               m->agrid_d.as<double>(), m->zsp_idx_d.as<int>(), m->zsp_coef_d.as<double>(),
                               m->ell_d.as<double>(), m->ws_out.as<float>(), (const float*)Mtab, Cv, gC, gY, gM, gdir);
        NS_HIP(hipGetLastError());
    }
    // spline adjoint -> delta for the emulator's raw outputs
    const Net& net = *m->nets[0];
    const int n_pad = net.layers[net.n_layers - 1]->n_pad;
    size_t max_w = 0;
    for (int l = 1; l < net.n_layers; ++l) max_w = std::max(max_w, (size_t)net.dims[l]);
    const size_t gstride = (size_t)rows * std::max(max_w, (size_t)n_pad);
    m->ws_gact[0].ensure(gstride * elem);
    m->ws_gact[1].ensure(gstride * elem);
    {
        TraceScope ts(m, s, "adj_zspline");
        const double hz = (1.0 / m->a_min - 1.0) / (nz - 1);
        const dim3 gz((unsigned)((B * n_pad + 255) / 256));
        if (f64)
            hipLaunchKernelGGL(zspline_adjoint_kernel<double>, gz, dim3(256), 0, s, gY, gM, B, nz, nk, hz,
                               net.out_sigma64.as<double>(), n_pad, m->ws_gact[0].as<double>());
        else
            hipLaunchKernelGGL(zspline_adjoint_kernel<float>, gz, dim3(256), 0, s, gY, gM, B, nz, nk, hz,
                               net.out_sigma64.as<double>(), n_pad, m->ws_gact[0].as<float>());
        NS_HIP(hipGetLastError());
    }
    emulator_backward(m, &id0, 1, B, f64 ? NS_FP64 : NS_FP32, s);
    TraceScope ts(m, s, "adj_assemble");
    grad_assemble(m, B, 1, nz, gdir, logl, grad, s);
}

}  // namespace nsmi
