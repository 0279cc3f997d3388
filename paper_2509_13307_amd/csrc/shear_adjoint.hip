// Adjoint of the cosmic-shear likelihood (App. A of the paper), input
// gradients only.
//
// Reverse mode runs from logL back to the emulator table:
//   dense chi^2:   g_C = L^{-T} L^{-1} (d - C)  (two FP64-MFMA GEMMs, shear.hip)
//   Limber (A2):   C_pb = f_p sum_j W_a(j) W_b(j) P_bj wq_j,  f_p = (1+m_a)(1+m_b)
//                  -> g(P wq)_bj, g W_i(j), g wq_j, and g chi_j through k = (l+1/2)/chi_j
//   P lookup:      P = 10^{CR(t; Yhat_j(c))}, Yhat = the table carried to z_j
//                  (cubic spline or linear in z) -> scatter into g Y (and g M, the
//                  spline second derivatives, whose map M = S(Y) is then
//                  transposed by zspline_adjoint_kernel) -> emulator backward.
// Forward mode covers the per-walker background and windows, which depend on
// few parameters: shear_tangent_kernel stores, per a-node, chi, wq, W_i and
// their tangents in the directions (Om, h, w0, wa) and, per bin, (Dz_i,
// A_IA,i); limber_adjoint_kernel contracts them into the direct gradient
//   sum_j [ sum_i gW_i(j) dW_i(j) + g wq_j dwq_j + g chi_j dchi_j ].
// Every Limber-adjoint term belongs to one a-node, so a thread owns a node
// (the a-grid is taken in chunks of 256 nodes).
//
// The scatter into g Y (and g M) is accumulated in 64-bit fixed point, so that
// its result does not depend on the order in which the nodes of a walker
// reach a table entry: limber_adjoint_kernel computes and stores every
// g log10 P_bj of the walker and their largest magnitude G; then
// limber_scatter_kernel adds each contribution c w g log10 P (|c w| < 2:
// spline and Catmull-Rom weights) rounded to the grid 2^(e - FX_BITS),
// G < 2^e, as integers: slab by slab (runs of z rows that fit in LDS, each
// taking the parts of the contributions that fall on its rows) with LDS
// atomics, then each row once as a double.  At most
// n_a n_ell <= 2^16 contributions reach one entry, so every partial sum stays
// below 2^(FX_BITS + 17) < 2^63; the grid step is below G 2^-44 (about
// 6e-14 G), well under the FP64 gradient's error against the complex step.
// The spline-curvature table g M takes contributions smaller by the factor
// max |c2|, |c3| <= 0.385 h^2 / 6 (h the z-node spacing) and has a grid finer
// by 2^mshift, mshift = floor(log2(6 / (0.385 h^2))).
#include "devutil.h"
#include "nsmi.h"
#include "shear_common.h"

namespace nsmi {

// ------------------------------------------------ background / window tangents
// Forward-mode tangents per node, one workgroup (256 threads) per walker,
// nodes in chunks of 256.  Directions 0..3 = (Om, h, w0, wa); per bin, Dz_i
// and A_IA,i.  Output record per node, structure of arrays
// tg[(w S + field) n_a + j], S = TG_FIXED + 7 n_bins:
constexpr int TG_CHI = 0, TG_DCHI = 1, TG_WQ = 5, TG_DWQ = 6, TG_LND = 10, TG_DLND = 11, TG_FIXED = 15;
// W_i at TG_FIXED + i, dW_i / d(Om, h, w0, wa)_q at TG_FIXED + nb + 4 i + q,
// dW_i / dDz_i at TG_FIXED + 5 nb + i, dW_i / dA_IA,i at TG_FIXED + 6 nb + i.
//   (a) forward pass: Simpson increments of chi, -ln D and their tangents,
//       prefix sums carried from chunk to chunk;
//   (b) n(z) normalisations N_i and dN_i / dDz_i;
//   (c) reverse pass (last chunk first), bins in groups of 5: reverse
//       cumulative trapezoids G0, G1 and their Dz tangents, then the
//       (Om, h, w0, wa) tangents of G1; windows and their tangents.
struct EB { double E, dE[4]; };

__global__ __launch_bounds__(256) void shear_tangent_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, ShearGeom G, const int* __restrict__ pidx,
    const double* __restrict__ pfix, const double* __restrict__ nz_mean, const double* __restrict__ agrid,
    double* __restrict__ tg) {
    __shared__ double buf[20 * 4];              // block_scan totals
    __shared__ double red[2 * MAXB][4];
    __shared__ double carry[10];                // forward prefix sums of the chunks before
    __shared__ double nrm[2 * MAXB];            // N_i, dN_i
    __shared__ double gcs[4][20];               // reverse sums of the chunks above, per (group, scan)
    __shared__ double bcs[4][20];               // ... and after this chunk (thread 0)
    __shared__ double gnx[4][20];               // integrands of the node above the chunk
    __shared__ double xw[4][20];                // wave-boundary exchange
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int na = G.n_a, nb = G.n_bins, nch = (na + 255) / 256;
    const int S = TG_FIXED + 7 * nb;
    auto rec = [&](int f, int j) -> double& { return tg[((int64_t)w * S + f) * na + j]; };
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double ob = phys(0), oc = phys(1), h = phys(2), w0 = phys(5), wa = phys(6);
    const double Om = (ob + oc) / (h * h);
    const double cH0 = C_KM_S / (100.0 * h), H0c = 1.0 / cH0;
    const double s2 = G.nz_sigma * G.nz_sigma;
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
    auto FG = [&](double a, double& f, double* df, double& g, double* dg) {
        const EB e = Eval(a);
        f = cH0 / (a * a * e.E);
        g = pow(Om / (a * a * a) / (e.E * e.E), GROWTH_INDEX) / a;
        for (int q = 0; q < 4; ++q) {
            df[q] = -f * e.dE[q] / e.E;
            dg[q] = -2.0 * GROWTH_INDEX * g * e.dE[q] / e.E;
        }
        df[1] += -f / h;
        dg[0] += GROWTH_INDEX * g / Om;
    };

    // (a) chi, ln D and tangents at every node
    if (t < 10) carry[t] = 0.0;
    if (t == 0) {
        rec(TG_CHI, 0) = rec(TG_LND, 0) = 0.0;
        for (int q = 0; q < 4; ++q) rec(TG_DCHI + q, 0) = rec(TG_DLND + q, 0) = 0.0;
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int j = c * 256 + t;
        double inc[10];
        for (int q = 0; q < 10; ++q) inc[q] = 0.0;
        if (j < na - 1) {
            const double a = agrid[j], a1 = agrid[j + 1], am = 0.5 * (a + a1);
            double fa, dfa[4], ga, dga[4], fm, dfm[4], gm, dgm[4], f1, df1[4], g1, dg1[4];
            FG(a, fa, dfa, ga, dga);
            FG(am, fm, dfm, gm, dgm);
            FG(a1, f1, df1, g1, dg1);
            inc[0] = G.da / 6.0 * (fa + 4.0 * fm + f1);
            inc[1] = G.da / 6.0 * (ga + 4.0 * gm + g1);
            for (int q = 0; q < 4; ++q) {
                inc[2 + q] = G.da / 6.0 * (dfa[q] + 4.0 * dfm[q] + df1[q]);
                inc[6 + q] = G.da / 6.0 * (dga[q] + 4.0 * dgm[q] + dg1[q]);
            }
        }
        block_scan<10>(inc, buf, false);
        if (j < na - 1) {                        // sums over intervals 0..j: values at node j + 1
            rec(TG_CHI, j + 1) = carry[0] + inc[0];
            rec(TG_LND, j + 1) = -(carry[1] + inc[1]);
            for (int q = 0; q < 4; ++q) {
                rec(TG_DCHI + q, j + 1) = carry[2 + q] + inc[2 + q];
                rec(TG_DLND + q, j + 1) = -(carry[6 + q] + inc[6 + q]);
            }
        }
        __syncthreads();
        if (t == 255)
            for (int q = 0; q < 10; ++q) carry[q] += inc[q];
    }

    // (b) normalisations of n_i(z) and their Dz tangents
    {
        double sn[MAXB], sd[MAXB];
        for (int i = 0; i < MAXB; ++i) sn[i] = sd[i] = 0.0;
        for (int c = 0; c < nch; ++c) {
            const int j = c * 256 + t;
            if (j <= 0 || j >= na) continue;
            const double a = agrid[j], z = 1.0 / a - 1.0;
            const double qw = j == na - 1 ? 0.5 * G.da : G.da;
            for (int i = 0; i < nb; ++i) {
                const double dz = z - (nz_mean[i] + phys(9 + nb + i));
                const double raw = exp(-dz * dz / (2.0 * s2));
                sn[i] += qw * raw / (a * a);
                sd[i] += qw * (raw * dz / s2) / (a * a);
            }
        }
        for (int i = 0; i < nb; ++i) {
            const double v0 = wave_sum(sn[i]), v1 = wave_sum(sd[i]);
            if (lane == 0) { red[2 * i][wid] = v0; red[2 * i + 1][wid] = v1; }
        }
        if (t < 80) { gcs[t / 20][t % 20] = 0.0; gnx[t / 20][t % 20] = 0.0; }
        __syncthreads();
        if (t < 2 * nb) nrm[t] = red[t][0] + red[t][1] + red[t][2] + red[t][3];
        __syncthreads();
    }

    // (c) reverse pass: G sums, windows and tangents
    const double pref = 1.5 * Om * H0c * H0c;
    const double dpref[4] = {pref / Om, 2.0 * pref / h, 0.0, 0.0};
    for (int c = nch - 1; c >= 0; --c) {
        const int j = c * 256 + t;
        const bool node = j < na, live = node && j > 0, has = node && j < na - 1;
        const double a = node ? agrid[j] : 1.0, a2 = a * a, z = 1.0 / a - 1.0;
        const double chi = node ? rec(TG_CHI, j) : 0.0;
        double dchi[4], dlnD[4];
        for (int q = 0; q < 4; ++q) {
            dchi[q] = node ? rec(TG_DCHI + q, j) : 0.0;
            dlnD[q] = node ? rec(TG_DLND + q, j) : 0.0;
        }
        const double D = exp(node ? rec(TG_LND, j) : 0.0);
        const EB ea = Eval(a);
        const double E = ea.E;
        const double dlnE[4] = {ea.dE[0] / E, 0.0, ea.dE[2] / E, ea.dE[3] / E};
        double fa, dfa[4], ga, dga[4];
        FG(a, fa, dfa, ga, dga);
        const double qw = (j == 0 || j == na - 1) ? 0.5 * G.da : G.da;
        if (node) {
            const double wq = live ? qw * fa / (chi * chi) : 0.0;
            rec(TG_WQ, j) = wq;
            for (int q = 0; q < 4; ++q) rec(TG_DWQ + q, j) = live ? wq * (dfa[q] / fa - 2.0 * dchi[q] / chi) : 0.0;
        }
        for (int grp = 0; grp * 5 < nb; ++grp) {
            const int b0 = 5 * grp, cnt = min(5, nb - b0);
            double n[5], dn[5];
            for (int cc = 0; cc < 5; ++cc) {
                n[cc] = dn[cc] = 0.0;
                if (cc >= cnt || !live) continue;
                const int i = b0 + cc;
                const double dz = z - (nz_mean[i] + phys(9 + nb + i));
                const double raw = exp(-dz * dz / (2.0 * s2));
                const double N = nrm[2 * i], dN = nrm[2 * i + 1];
                n[cc] = raw / N;
                dn[cc] = (raw * dz / s2) / N - n[cc] * dN / N;
            }
            double Gs[20], Gc[20];
            for (int sc = 0; sc < 2; ++sc) {
                const int slot = 2 * grp + sc;
                double v[20];
                for (int k = 0; k < 20; ++k) v[k] = 0.0;
                for (int cc = 0; cc < cnt; ++cc) {
                    if (sc == 0) {
                        v[cc] = node ? n[cc] / a2 : 0.0;
                        v[5 + cc] = live ? n[cc] / (a2 * chi) : 0.0;
                        v[10 + cc] = node ? dn[cc] / a2 : 0.0;
                        v[15 + cc] = live ? dn[cc] / (a2 * chi) : 0.0;
                    } else {
                        for (int q = 0; q < 4; ++q) v[4 * cc + q] = live ? -n[cc] * dchi[q] / (a2 * chi * chi) : 0.0;
                    }
                }
                if (lane == 0)
                    for (int k = 0; k < 20; ++k) xw[wid][k] = v[k];
                __syncthreads();
                double sg[20];
                for (int k = 0; k < 20; ++k) {
                    double nv = __shfl_down(v[k], 1, 64);
                    if (lane == 63) nv = wid < 3 ? xw[wid + 1][k] : gnx[slot][k];
                    sg[k] = has ? 0.5 * G.da * (v[k] + nv) : 0.0;
                }
                __syncthreads();
                if (t == 0)
                    for (int k = 0; k < 20; ++k) gnx[slot][k] = v[k];
                block_scan<20>(sg, buf, true);
                for (int k = 0; k < 20; ++k) sg[k] += gcs[slot][k];
                if (t == 0)
                    for (int k = 0; k < 20; ++k) bcs[slot][k] = sg[k];
                for (int k = 0; k < 20; ++k) {
                    if (sc == 0) Gs[k] = sg[k];
                    else Gc[k] = sg[k];
                }
            }
            if (node) {
                for (int cc = 0; cc < cnt; ++cc) {
                    const int i = b0 + cc;
                    const double G0 = Gs[cc], G1 = Gs[5 + cc], G0z = Gs[10 + cc], G1z = Gs[15 + cc];
                    const double Q = G0 - chi * G1;
                    const double Wg = pref * chi / a * Q;
                    const double A = phys(9 + i);
                    const double base = C1_RHOCR * Om * H0c * E / D;     // W^I = -A n base
                    const double WI = -A * n[cc] * base;
                    rec(TG_FIXED + i, j) = Wg + WI;
                    for (int q = 0; q < 4; ++q) {
                        const double dQ = -dchi[q] * G1 - chi * Gc[4 * cc + q];
                        const double dWg = dpref[q] * chi / a * Q + pref * dchi[q] / a * Q + pref * chi / a * dQ;
                        double dlnbase = dlnE[q] - dlnD[q];
                        if (q == 0) dlnbase += 1.0 / Om;
                        if (q == 1) dlnbase += 1.0 / h;
                        rec(TG_FIXED + nb + 4 * i + q, j) = dWg + WI * dlnbase;
                    }
                    rec(TG_FIXED + 5 * nb + i, j) = pref * chi / a * (G0z - chi * G1z) - A * dn[cc] * base;
                    rec(TG_FIXED + 6 * nb + i, j) = -n[cc] * base;
                }
            }
        }
        __syncthreads();
        if (t < 80) gcs[t / 20][t % 20] = bcs[t / 20][t % 20];
        __syncthreads();
    }
}

// --------------------------------------------------------- Limber adjoint
constexpr int FX_BITS = 45;

// log10 k of multipole b at comoving distance chi -> Catmull-Rom interval i0,
// its offset tt and the ghost flags at the ends of the k grid (one definition
// for both passes of the Limber adjoint)
struct KPos { int i0; double tt; bool lo_ghost, hi_ghost; };
__device__ __forceinline__ KPos k_position(double k, const ShearGeom& G) {
    const double s = (log10(k) - G.u0) / G.du;
    int i0 = (int)floor(s);
    i0 = i0 < 0 ? 0 : (i0 > G.n_k - 2 ? G.n_k - 2 : i0);
    return KPos{i0, s - i0, i0 == 0, i0 + 2 >= G.n_k};
}

// One workgroup (256 threads) per walker, thread = a-node j (chunks of 256):
// g(P wq), g W_i(j), g wq_j and g chi_j (through k = (l+1/2)/chi_j) from the
// Limber sums; g log10 P_bj goes to glp [B x n_ell x n_a] and the walker's
// fixed-point grid step to gstep [B] (limber_scatter_kernel then sums them
// into the tables g Y, g M); the node terms are contracted with the tangents
// of shear_tangent_kernel into the direct gradient gdir [B x d] (fully
// written).
template <class T, bool LINZ>
__global__ __launch_bounds__(256) void limber_adjoint_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, ShearGeom G,
    const int* __restrict__ pidx, const double* __restrict__ pfix, const int* __restrict__ zidx,
    const double* __restrict__ zcoef, const double* __restrict__ ell, const T* __restrict__ Ytab,
    const T* __restrict__ Mtab, const double* __restrict__ Cv, const double* __restrict__ gC,
    const double* __restrict__ tg, double* __restrict__ glp_buf, double* __restrict__ gstep,
    double* __restrict__ gdir) {
    __shared__ double Hs[55 * 32];          // G_pb f_p, pair-major
    __shared__ double red[4 + 2 * MAXB][4];
    __shared__ double gmx[4];
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int na = G.n_a, nb = G.n_bins, ne = G.n_ell, npair = G.n_pairs, nch = (na + 255) / 256;
    const int S = TG_FIXED + 7 * nb;
    auto rec = [&](int f, int j) { return tg[((int64_t)w * S + f) * na + j]; };
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double h = phys(2);
    const double Om = (phys(0) + phys(1)) / (h * h);
    const int nout = npair * ne;

    // H_pb = g_C[pb] (1 + m_a)(1 + m_b)
    for (int o = t; o < nout; o += 256) {
        const int p = o / ne;
        int a = 0, rem = p;
        while (rem >= nb - a) { rem -= nb - a; ++a; }
        const int bb = a + rem;
        Hs[o] = gC[w * nout + o] * (1.0 + phys(9 + 2 * nb + a)) * (1.0 + phys(9 + 2 * nb + bb));
    }
    __syncthreads();
    double acc[4 + 2 * MAXB];
    for (int q = 0; q < 4 + 2 * MAXB; ++q) acc[q] = 0.0;
    const T* Yw = Ytab + w * (int64_t)G.n_z * G.n_k;
    const T* Mw = LINZ ? Yw : Mtab + w * (int64_t)G.n_z * G.n_k;
    double* glw = glp_buf + w * (int64_t)ne * na;
    double gmax = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int j = c * 256 + t;
        if (j <= 0 || j >= na) continue;
        double W[MAXB], gW[MAXB];
        for (int i = 0; i < nb; ++i) {
            W[i] = rec(TG_FIXED + i, j);
            gW[i] = 0.0;
        }
        const double chi = rec(TG_CHI, j), wq = rec(TG_WQ, j);
        double gwq = 0.0, gchi = 0.0;
        const int nn = zidx[j];
        const double c0 = zcoef[4 * j], c1 = zcoef[4 * j + 1];
        const double c2 = LINZ ? 0.0 : zcoef[4 * j + 2], c3 = LINZ ? 0.0 : zcoef[4 * j + 3];
        for (int b = 0; b < ne; ++b) {
            const double k = (ell[b] + 0.5) / chi;
            if (!(k >= G.k_min && k <= G.k_max)) continue;
            const KPos kp = k_position(k, G);
            const int i0 = kp.i0;
            const double tt = kp.tt;
            // log10 P at z_j from rows nn, nn + 1 of Y (and of M for cubic z)
            auto zmix = [&](T ya, T yb, T ma, T mb) {
                if (LINZ) return c0 * (double)ya + c1 * (double)yb;
                return c0 * (double)ya + c1 * (double)yb + c2 * (double)ma + c3 * (double)mb;
            };
            auto Yz = [&](int col) {
                const int64_t o0 = (int64_t)nn * G.n_k + col, o1 = o0 + G.n_k;
                return zmix(Yw[o0], Yw[o1], LINZ ? T(0) : Mw[o0], LINZ ? T(0) : Mw[o1]);
            };
            const bool lo_ghost = kp.lo_ghost, hi_ghost = kp.hi_ghost;
            double pm, p0, p1, p2;
            if (!lo_ghost && !hi_ghost) {
                // columns i0 - 1 .. i0 + 2 of each row in one (element-aligned) vector load
                struct Q4 { T v[4]; };
                auto row4 = [&](const T* q) { Q4 r; __builtin_memcpy(&r, q, sizeof(r)); return r; };
                const int64_t o = (int64_t)nn * G.n_k + i0 - 1;
                const Q4 ya = row4(Yw + o), yb = row4(Yw + o + G.n_k);
                Q4 ma = {}, mb = {};
                if (!LINZ) {
                    ma = row4(Mw + o);
                    mb = row4(Mw + o + G.n_k);
                }
                pm = zmix(ya.v[0], yb.v[0], ma.v[0], mb.v[0]);
                p0 = zmix(ya.v[1], yb.v[1], ma.v[1], mb.v[1]);
                p1 = zmix(ya.v[2], yb.v[2], ma.v[2], mb.v[2]);
                p2 = zmix(ya.v[3], yb.v[3], ma.v[3], mb.v[3]);
            } else {
                p0 = Yz(i0);
                p1 = Yz(i0 + 1);
                pm = lo_ghost ? 2.0 * p0 - p1 : Yz(i0 - 1);
                p2 = hi_ghost ? 2.0 * p1 - p0 : Yz(i0 + 2);
            }
            const double m0 = 0.5 * (p1 - pm), m1 = 0.5 * (p2 - p0);
            const double t2 = tt * tt, t3 = t2 * tt;
            const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + tt, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
            const double lp = h00 * p0 + h10 * m0 + h01 * p1 + h11 * m1;
            const double dlp_dt = (6 * t2 - 6 * tt) * p0 + (3 * t2 - 4 * tt + 1) * m0 + (-6 * t2 + 6 * tt) * p1 +
                                  (3 * t2 - 2 * tt) * m1;
            const double P = exp(lp * LN10);
            const double Pw = P * wq;
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
            glw[(int64_t)b * na + j] = glp;
            gmax = fmax(gmax, fabs(glp));
        }
        // contract with the tangents of this node
        for (int q = 0; q < 4; ++q) {
            double v = gwq * rec(TG_DWQ + q, j) + gchi * rec(TG_DCHI + q, j);
            for (int i = 0; i < nb; ++i) v += gW[i] * rec(TG_FIXED + nb + 4 * i + q, j);
            acc[q] += v;
        }
        for (int i = 0; i < nb; ++i) {
            acc[4 + i] += gW[i] * rec(TG_FIXED + 5 * nb + i, j);
            acc[4 + nb + i] += gW[i] * rec(TG_FIXED + 6 * nb + i, j);
        }
    }

    // ---- direct gradient: reduce over nodes
    const int nacc = 4 + 2 * nb;
    for (int q = 0; q < nacc; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[q][wid] = v;
    }
    for (int k = t; k < d; k += 256) gdir[w * d + k] = 0.0;
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

    // ---- g Y (and g M) in fixed point: the walker's grid from its largest
    // |g log10 P| (a NaN anywhere makes the step NaN and skips the scatter)
    {
        const double v = wave_max(gmax);
        if (lane == 0) gmx[wid] = v;
    }
    __syncthreads();
    const double gm_all = fmax(fmax(gmx[0], gmx[1]), fmax(gmx[2], gmx[3]));
    const bool ok = !isnan(gmx[0] + gmx[1] + gmx[2] + gmx[3]) && gm_all <= 1.7e308;
    int e = 0;
    if (ok && gm_all > 0.0) (void)frexp(gm_all, &e);                  // gm_all < 2^e
    if (t == 0) gstep[w] = ok ? ldexp(1.0, e - FX_BITS) : NAN;
}

// Fixed-point scatter of g log10 P_bj (limber_adjoint_kernel's glp_buf and
// grid step gstep) into the tables gY (and gM for the cubic z-spline), one
// workgroup per walker.  Slab s = (first node, end node, first row, last row)
// of `slabs`: the z rows partitioned into runs, each with the nodes whose two
// rows meet it.  A slab adds the contributions of its nodes to its own rows
// only, as integers in LDS (atomics); every row's sum is then complete, and
// the slab writes its rows as doubles (integer x grid step, 2^-mshift finer
// for gM).  Every entry of the walker's tables is written.  A walker whose
// grid step is NaN (a non-finite gradient) gets NaN tables.
template <bool LINZ>
__global__ __launch_bounds__(256) void limber_scatter_kernel(
    int64_t B, ShearGeom G, const int* __restrict__ zidx, const double* __restrict__ zcoef,
    const double* __restrict__ ell, const double* __restrict__ tg, const double* __restrict__ glp_buf,
    const int4* __restrict__ slabs, int n_slabs, int rmax, const double* __restrict__ gstep, int mshift,
    double* __restrict__ gY, double* __restrict__ gM) {
    extern __shared__ unsigned long long sl[];          // [tables][rmax][n_k]
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x;
    const int na = G.n_a, ne = G.n_ell, nk = G.n_k, nz = G.n_z;
    const int S = TG_FIXED + 7 * G.n_bins;
    const double step = gstep[w];
    const bool ok = !isnan(step);
    const double scale = 1.0 / step, mscale = ldexp(scale, mshift);     // powers of two: exact
    const double mstep = ldexp(step, -mshift);
    const int tab = rmax * nk;
    double* gYw = gY + w * (int64_t)nz * nk;
    double* gMw = LINZ ? gYw : gM + w * (int64_t)nz * nk;
    const double* glw = glp_buf + w * (int64_t)ne * na;
    const double* chiw = tg + ((int64_t)w * S + TG_CHI) * na;
    auto fx_add = [&](unsigned long long* p, double v, double sc) {
        if (v != 0.0) atomicAdd(p, (unsigned long long)llrint(v * sc));
    };
    for (int s = 0; s < n_slabs; ++s) {
        const int4 sb = slabs[s];
        const int lo = sb.z, nr = sb.w - sb.z + 1, nj = sb.y - sb.x;
        for (int e = t; e < nr * nk; e += 256) {
            sl[e] = 0ull;
            if (!LINZ) sl[tab + e] = 0ull;
        }
        __syncthreads();
        if (ok)
            for (int it = t; it < nj * ne; it += 256) {
                const int j = sb.x + it % nj, b = it / nj;
                const double chi = chiw[j];
                const double k = (ell[b] + 0.5) / chi;
                if (!(k >= G.k_min && k <= G.k_max)) continue;
                const double glp = glw[(int64_t)b * na + j];
                if (glp == 0.0) continue;
                // the node's rows zi[j], zi[j] + 1 as rows of this slab (either may lie outside it)
                const int r0 = zidx[j] - lo, r1 = r0 + 1;
                const bool in0 = r0 >= 0, in1 = r1 < nr;
                const double c0 = zcoef[4 * j], c1 = zcoef[4 * j + 1];
                const double c2 = LINZ ? 0.0 : zcoef[4 * j + 2], c3 = LINZ ? 0.0 : zcoef[4 * j + 3];
                const KPos kp = k_position(k, G);
                const double tt = kp.tt, t2 = tt * tt, t3 = t2 * tt;
                const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + tt, h01 = -2 * t3 + 3 * t2,
                             h11 = t3 - t2;
                // d lp / d (pm, p0, p1, p2), ghosts folded into the real columns
                double wm = -0.5 * h10, w0c = h00 - 0.5 * h11, w1c = h01 + 0.5 * h10, w2 = 0.5 * h11;
                if (kp.lo_ghost) { w0c += 2.0 * wm; w1c -= wm; wm = 0.0; }
                if (kp.hi_ghost) { w1c += 2.0 * w2; w0c -= w2; w2 = 0.0; }
                auto scatter = [&](int col, double wgt) {
                    const double gy = glp * wgt;
                    if (in0) {
                        fx_add(&sl[r0 * nk + col], c0 * gy, scale);
                        if (!LINZ) fx_add(&sl[tab + r0 * nk + col], c2 * gy, mscale);
                    }
                    if (in1) {
                        fx_add(&sl[r1 * nk + col], c1 * gy, scale);
                        if (!LINZ) fx_add(&sl[tab + r1 * nk + col], c3 * gy, mscale);
                    }
                };
                if (!kp.lo_ghost) scatter(kp.i0 - 1, wm);
                scatter(kp.i0, w0c);
                scatter(kp.i0 + 1, w1c);
                if (!kp.hi_ghost) scatter(kp.i0 + 2, w2);
            }
        __syncthreads();
        const int64_t g0 = (int64_t)lo * nk;
        for (int e = t; e < nr * nk; e += 256) {
            gYw[g0 + e] = ok ? (double)(long long)sl[e] * step : NAN;
            if (!LINZ) gMw[g0 + e] = ok ? (double)(long long)sl[tab + e] * mstep : NAN;
        }
        __syncthreads();                                // LDS reused by the next slab
    }
}

// ------------------------------------------------------------ spline adjoint
// gY, gM (doubles, from limber_scatter_kernel): gY += S^T gM for the
// not-a-knot spline of each (walker, k) column, and
// delta_out[row = w n_z + n][c] = gY[n][c] sigma_out[c] (padded to n_pad).
template <class T>
__global__ __launch_bounds__(256) void zspline_adjoint_kernel(double* __restrict__ gY, double* __restrict__ gM,
                                                              int64_t B, int nz, int nk, double h,
                                                              const double* __restrict__ sigma_out, int n_pad,
                                                              T* __restrict__ delta, int linear) {
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
    if (linear) {                               // no spline: delta = g Y sigma_out
        const double sg = sigma_out[c];
        for (int n = 0; n < nz; ++n) delta[(w * nz + n) * n_pad + c] = (T)(gy[(int64_t)n * nk] * sg);
        return;
    }
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

// ------------------------------------------------------------------ driver
void shear_grad(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, double* grad, int prec,
                hipStream_t s) {
    const bool f64 = prec == NS_FP64, lin = m->z_linear;
    const size_t elem = f64 ? 8 : 4;
    const int nk = m->n_k, nz = m->n_z, n = m->n_data, d = m->d, na = m->n_a, nb = m->n_bins;
    const int64_t rows = B * nz;
    // forward: emulator table (with pre-activation saves), spline, spectra
    m->ws_out.ensure((size_t)B * nz * nk * elem);
    const int id0 = 0, no_log = 0;
    void* out0 = m->ws_out.p;
    emulator_forward(m, &id0, 1, theta, ld, B, &out0, nk, &no_log, prec, nullptr, s, true);
    shear_loglike_from_table(m, theta, ld, B, logl, prec, nullptr, s);
    const size_t mbytes = lin ? 0 : (size_t)B * nz * nk * elem;
    const void* Mtab = m->ws_aux.p;
    const double* Cv = reinterpret_cast<const double*>(m->ws_aux.as<char>() + mbytes);
    // adjoint scratch: gC, R [B n], chi^2 partial sums [n_ct B], gY (and gM) [B nz nk],
    // tangents [B S n_a], gdir [B d], g log10 P [B n_ell n_a], fixed-point grid [B]
    const size_t ntab = (size_t)B * nz * nk, n_ct = (n + 63) / 64;
    const size_t S = TG_FIXED + 7 * (size_t)nb;
    m->ws_grad.ensure(((size_t)B * (2 * n + n_ct) + (lin ? 1 : 2) * ntab + (size_t)B * S * na + (size_t)B * d +
                       (size_t)B * m->n_ell * na + (size_t)B) *
                      sizeof(double));
    double* gC = m->ws_grad.as<double>();
    double* R = gC + (size_t)B * n;
    double* part = R + (size_t)B * n;
    double* gY = part + (size_t)B * n_ct;
    double* gM = lin ? gY : gY + ntab;          // spline second derivatives: cubic z only
    double* tg = gY + (lin ? 1 : 2) * ntab;
    double* gdir = tg + (size_t)B * S * na;
    double* glp = gdir + (size_t)B * d;
    double* gstep = glp + (size_t)B * m->n_ell * na;
    // finer fixed-point grid of g M: its coefficients are at most 0.385 h^2 / 6
    const double hz = (1.0 / m->a_min - 1.0) / (nz - 1);
    const int mshift = lin ? 0 : std::max(0, std::min(40, (int)std::floor(std::log2(6.0 / (0.385 * hz * hz)))));
    {
        TraceScope ts(m, s, "adj_dense_chi2");
        dense_chi2_adjoint(m, theta, ld, B, Cv, R, part, logl, gC, s);
    }
    const ShearGeom G = shear_geom(m);
    {
        TraceScope ts(m, s, "adj_tangents");
        hipLaunchKernelGGL(shear_tangent_kernel, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, G,
                           m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->nz_mean_d.as<double>(),
                           m->agrid_d.as<double>(), tg);
        NS_HIP(hipGetLastError());
    }
    {
        TraceScope ts(m, s, "adj_limber");
        auto launch = [&](auto kern, const auto* Y) {
            hipLaunchKernelGGL(kern, dim3((unsigned)B), dim3(256), 0, s, theta, ld, B, d, G, m->pidx_d.as<int>(),
                               m->pfix_d.as<double>(), m->zsp_idx_d.as<int>(), m->zsp_coef_d.as<double>(),
                               m->ell_d.as<double>(), Y, (decltype(Y))Mtab, Cv, gC, tg, glp, gstep, gdir);
        };
        if (f64) {
            if (lin) launch(limber_adjoint_kernel<double, true>, m->ws_out.as<double>());
            else launch(limber_adjoint_kernel<double, false>, m->ws_out.as<double>());
        } else {
            if (lin) launch(limber_adjoint_kernel<float, true>, m->ws_out.as<float>());
            else launch(limber_adjoint_kernel<float, false>, m->ws_out.as<float>());
        }
        NS_HIP(hipGetLastError());
    }
    {
        TraceScope ts(m, s, "adj_limber_scatter");
        const size_t smem = (size_t)(lin ? 1 : 2) * m->lslab_rows * nk * sizeof(unsigned long long);
        const auto kern = lin ? limber_scatter_kernel<true> : limber_scatter_kernel<false>;
        if (smem > 64 * 1024)
            NS_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        hipLaunchKernelGGL(kern, dim3((unsigned)B), dim3(256), smem, s, B, G, m->zsp_idx_d.as<int>(),
                           m->zsp_coef_d.as<double>(), m->ell_d.as<double>(), tg, glp, m->lslab_d.as<int4>(),
                           m->n_lslab, m->lslab_rows, gstep, mshift, gY, gM);
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
        const dim3 gz((unsigned)((B * n_pad + 255) / 256));
        if (f64)
            hipLaunchKernelGGL(zspline_adjoint_kernel<double>, gz, dim3(256), 0, s, gY, gM, B, nz, nk, hz,
                               net.out_sigma64.as<double>(), n_pad, m->ws_gact[0].as<double>(), (int)lin);
        else
            hipLaunchKernelGGL(zspline_adjoint_kernel<float>, gz, dim3(256), 0, s, gY, gM, B, nz, nk, hz,
                               net.out_sigma64.as<double>(), n_pad, m->ws_gact[0].as<float>(), (int)lin);
        NS_HIP(hipGetLastError());
    }
    emulator_backward(m, &id0, 1, B, f64 ? NS_FP64 : NS_FP32, s);
    TraceScope ts(m, s, "adj_assemble");
    grad_assemble(m, B, 1, nz, gdir, logl, grad, s);
}

}  // namespace nsmi
