// Cosmic-shear likelihood stages after the emulator (App. A of the paper).
//
// zspline_kernel   second derivatives M_n(k) of the not-a-knot cubic spline of
//                  log10 P along the uniform z nodes, one thread per (walker, k):
//                  M_1 and M_{N-2} follow directly from the not-a-knot
//                  conditions on a uniform grid, the interior (1, 4, 1)
//                  system is solved by a Thomas sweep, M_0 and M_{N-1} are
//                  linear extrapolations.
// limber_kernel    one workgroup per walker, nodes in chunks of 256:
//                  (a) background on the a-grid: E(a), chi by per-interval
//                      Simpson, J = dchi/d(-a), growth D (growth index 0.55);
//                  (b) n_i(z) with photo-z shifts, normalised by the trapezoid
//                      rule; lensing window Eq. (A3) as (chi/a)(G0 - chi G1)
//                      with reverse cumulative trapezoids; NLA window Eq. (A4);
//                      effective window W = W^g + W^I (the four terms of Eq. (A1)
//                      share P_dd);
//                  (c) P(k = (l+1/2)/chi_j, z_j): spline or linear in z,
//                      Catmull-Rom in log10 k (linear ghost nodes), zero
//                      outside [k_min, k_max];
//                  (d) Limber sum Eq. (A2) by the trapezoid rule in a with the
//                      analytic Jacobian, times (1 + m_i)(1 + m_j).
//                  (a)-(b) are FP64; (c)-(d) run in the form's type T.
// dense_chi2_kernel  y = L^{-1} d - L^{-1} C with the host-factorised dense
//                  covariance, logL = -1/2 |y|^2 - sum log L_ii - n/2 log 2 pi
//                  (FP64; L^{-1} C on the FP64 MFMA).
#include "devutil.h"
#include "nsmi.h"
#include "shear_common.h"

namespace nsmi {

// -------------------------------------------------------------- z-spline
// One thread per (walker, k) column, one wave per block.  The column is first
// staged in LDS ([n_z][64] per wave; the loads are independent, so they are
// all in flight together), then the Thomas sweep of the (1, 4, 1) system runs
// from LDS, its forward values overwriting the staged y in place, and each
// second derivative is written to HBM once.
template <class T>
__global__ __launch_bounds__(64) void zspline_kernel(const T* __restrict__ Y, T* __restrict__ M, int64_t B,
                                                     int nz, int nk, double h, const int* __restrict__ count) {
    extern __shared__ __attribute__((aligned(16))) unsigned char zs_smem[];
    T* ys = reinterpret_cast<T*>(zs_smem);             // [nz][64]: y, then d' of the sweep
    // c'_n of the (1, 4, 1) Thomas sweep: data independent, tabulated once per block
    __shared__ T cps[256];
    if (threadIdx.x == 0) {
        T c = T(0);
        for (int n = 2; n <= nz - 3 && n < 256; ++n) {
            c = T(1) / (T(4) - (n == 2 ? T(0) : c));
            cps[n] = c;
        }
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (count) B = min<int64_t>(B, *count);
    if (g >= B * nk) return;
    const int t = threadIdx.x;
    const int64_t w = g / nk;
    const int c = (int)(g % nk);
    const T* y = Y + w * nz * nk + c;
    T* mm = M + w * nz * nk + c;
#pragma unroll 8
    for (int n = 0; n < nz; ++n) ys[n * 64 + t] = y[(int64_t)n * nk];
    const T ih2 = T(1.0 / (h * h));
    auto yv = [&](int n) { return ys[n * 64 + t]; };
    const T M1 = (yv(2) - T(2) * yv(1) + yv(0)) * ih2;
    const T Mb = (yv(nz - 1) - T(2) * yv(nz - 2) + yv(nz - 3)) * ih2;   // M_{N-2}
    T M2 = Mb, Mc = M1;                                 // n_z = 4: nodes 2 and n_z - 3 are N-2 and 1
    // interior unknowns n = 2 .. nz-3: M_{n-1} + 4 M_n + M_{n+1} = 6 d2Y_n / h^2
    if (nz > 4) {
        T dpv = T(0);
        T ym = yv(1), y0 = yv(2);
        for (int n = 2; n <= nz - 3; ++n) {
            const T yp = yv(n + 1);
            T rhs = T(6) * (yp - T(2) * y0 + ym) * ih2;
            if (n == 2) rhs -= M1;
            if (n == nz - 3) rhs -= Mb;
            dpv = (rhs - (n == 2 ? T(0) : dpv)) * cps[n];
            ys[n * 64 + t] = dpv;                       // y_n is held in y0 from here on
            ym = y0;
            y0 = yp;
        }
        T next = dpv;                                   // M_{nz-3} = d'_{nz-3}
        mm[(int64_t)(nz - 3) * nk] = next;
        Mc = next;
        for (int n = nz - 4; n >= 2; --n) {
            next = ys[n * 64 + t] - cps[n] * next;
            mm[(int64_t)n * nk] = next;
        }
        M2 = next;
    }
    mm[(int64_t)1 * nk] = M1;
    mm[(int64_t)(nz - 2) * nk] = Mb;
    mm[0] = T(2) * M1 - M2;
    mm[(int64_t)(nz - 1) * nk] = T(2) * Mb - Mc;
}

// One workgroup (256 threads) per walker.  The n_a nodes are taken in chunks
// of 256, one node per thread: a forward pass builds chi and -ln D (kept in
// LDS for every node) and the n(z) normalisations; a reverse pass, from the
// last chunk to the first, builds the windows (reverse cumulative sums carried
// from chunk to chunk), looks up P and adds each chunk's share of the Limber
// sums to per-thread accumulators.  LINZ: linear z-interpolation (no spline
// second derivatives).
constexpr int LB_SLOTS = 2;     // (pair, 4-ell group) items per thread
template <class T, bool LINZ>
__global__ __launch_bounds__(256) void limber_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, ShearGeom G,
    const int* __restrict__ pidx, const double* __restrict__ pfix, const double* __restrict__ nz_mean,
    const double* __restrict__ agrid, const int* __restrict__ zidx, const double* __restrict__ zcoef,
    const double* __restrict__ lell, const T* __restrict__ Ytab, const T* __restrict__ Mtab,
    double* __restrict__ Cout, const int* __restrict__ count) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (count) B = min<int64_t>(B, *count);
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int na = G.n_a, nb = G.n_bins;
    const int nch = (na + 255) / 256;
    const int nl4 = (G.n_ell + 3) & ~3;
    double* buf = reinterpret_cast<double*>(smem);                    // [2 MAXB][4] block_scan totals
    double* red = buf + 2 * MAXB * 4;                                 // [MAXB][4]
    double* bc = red + MAXB * 4;                                      // [2 MAXB] next carry (thread 0)
    double* gcs = bc + 2 * MAXB;                                      // [2 MAXB] sums over the chunks above
    double* mus = gcs + 2 * MAXB;                                     // [MAXB] n(z) means
    double* nrm = mus + MAXB;                                         // [MAXB] n(z) normalisations
    double* gnx = nrm + MAXB;                                         // [2 MAXB] g0, g1 of the node above the chunk
    double* xw = gnx + 2 * MAXB;                                      // [4][2 MAXB] wave-boundary exchange
    double* chis = xw + 4 * 2 * MAXB;                                 // [nch 256 + 1]
    double* lnDs = chis + nch * 256 + 1;                              // [nch 256 + 1]
    T* Wt = reinterpret_cast<T*>(lnDs + nch * 256 + 1);               // [nb][256]
    T* Pl = Wt + nb * 256;                                            // [256][nl4]

    // physical parameters
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double ob = phys(0), oc = phys(1), h = phys(2), w0 = phys(5), wa = phys(6);
    const double Om = (ob + oc) / (h * h);
    const double cH0 = C_KM_S / (100.0 * h), H0c = 1.0 / cH0;
    auto Efn = [&](double a) {
        return sqrt(Om / (a * a * a) + (1.0 - Om) * pow(a, -3.0 * (1.0 + w0 + wa)) * exp(-3.0 * wa * (1.0 - a)));
    };
    auto ffn = [&](double a) { return cH0 / (a * a * Efn(a)); };
    auto gfn = [&](double a) {
        const double E = Efn(a);
        return pow(Om / (a * a * a) / (E * E), GROWTH_INDEX) / a;
    };
    if (t < MAXB) mus[t] = t < nb ? nz_mean[t] + phys(9 + nb + t) : 0.0;
    __syncthreads();
    const double s2 = 2.0 * G.nz_sigma * G.nz_sigma;

    // (a) forward pass: Simpson increments of chi and -ln D on [a_j, a_{j+1}];
    // chis[j] / lnDs[j] = sums over intervals 0..j-1; n(z) normalisations
    double nsum[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) nsum[i] = 0.0;
    if (t == 0) chis[0] = lnDs[0] = 0.0;
    double carry0 = 0.0, carry1 = 0.0;
    for (int c = 0; c < nch; ++c) {
        const int j = c * 256 + t;
        const bool node = j < na;
        const double a = node ? agrid[j] : 1.0;
        double inc[2] = {0.0, 0.0};
        if (node && j < na - 1) {
            const double a1 = agrid[j + 1], am = 0.5 * (a + a1);
            inc[0] = G.da / 6.0 * (ffn(a) + 4.0 * ffn(am) + ffn(a1));
            inc[1] = G.da / 6.0 * (gfn(a) + 4.0 * gfn(am) + gfn(a1));
        }
        block_scan<2>(inc, buf, false);
        chis[j + 1] = carry0 + inc[0];
        lnDs[j + 1] = carry1 + inc[1];
        if (node && j > 0) {
            const double z = 1.0 / a - 1.0;
            const double q = j == na - 1 ? 0.5 * G.da : G.da;
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                if (i >= nb) continue;
                const double dz = z - mus[i];
                nsum[i] += q * exp(-dz * dz / s2) / (a * a);
            }
        }
        __syncthreads();
        carry0 = chis[c * 256 + 256];
        carry1 = lnDs[c * 256 + 256];
    }
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        if (i >= nb) continue;
        const double v = wave_sum(nsum[i]);
        if (lane == 0) red[i * 4 + wid] = v;
    }
    if (t < 2 * MAXB) gnx[t] = gcs[t] = 0.0;
    __syncthreads();
    if (t < MAXB) nrm[t] = t < nb ? red[t * 4] + red[t * 4 + 1] + red[t * 4 + 2] + red[t * 4 + 3] : 1.0;
    __syncthreads();

    // (d) bookkeeping: item = (pair p, group of 4 ell bins); each chunk's node
    // range is split into nseg segments whose partial sums are added in a
    // fixed order at the end
    const int ng = nl4 / 4, nitem = G.n_pairs * ng;
    const int nseg = nitem >= 256 ? 1 : 256 / nitem;
    const int len = (min(na, 256) + nseg - 1) / nseg;
    const int nout = G.n_pairs * G.n_ell;
    auto pair_of = [&](int p, int& bi, int& bj) {
        int rem = p;
        bi = 0;
        while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
        bj = bi + rem;
    };
    T acc[LB_SLOTS][4];
#pragma unroll
    for (int s = 0; s < LB_SLOTS; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[s][e] = T(0);

    // reverse pass over the chunks
    for (int c = nch - 1; c >= 0; --c) {
        const int j = c * 256 + t;
        const bool node = j < na;
        const double a = node ? agrid[j] : 1.0;
        const double Ea = node ? Efn(a) : 1.0;
        const double fa = cH0 / (a * a * Ea);
        const double chi = node ? chis[j] : 0.0;
        const double D = exp(-(node ? lnDs[j] : 0.0));
        const double z = 1.0 / a - 1.0;
        const double q = (j == 0 || j == na - 1) ? 0.5 * G.da : G.da;
        // (b) normalised n_i(z_j); integrands of G0, G1 at this node
        double nr[MAXB], g0[MAXB], g1[MAXB];
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            if (i >= nb) { nr[i] = g0[i] = g1[i] = 0.0; continue; }
            const double dz = z - mus[i];
            nr[i] = (node && j > 0) ? exp(-dz * dz / s2) : 0.0;
            nr[i] /= nrm[i];
            g0[i] = node ? nr[i] / (a * a) : 0.0;
            g1[i] = (node && j > 0) ? nr[i] / (a * a * chi) : 0.0;
        }
        // trapezoid segment [j, j+1]: node j+1 from the next lane, the next
        // wave (through LDS) or the chunk above (gnx)
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                xw[wid * 2 * MAXB + i] = g0[i];
                xw[wid * 2 * MAXB + MAXB + i] = g1[i];
            }
        __syncthreads();
        double seg[2 * MAXB];
        const bool has = node && j < na - 1;
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            double n0 = __shfl_down(g0[i], 1, 64), n1 = __shfl_down(g1[i], 1, 64);
            if (lane == 63) {
                const double* src = wid < 3 ? xw + (wid + 1) * 2 * MAXB : gnx;
                n0 = src[i];
                n1 = src[MAXB + i];
            }
            seg[i] = (has && i < nb) ? 0.5 * G.da * (g0[i] + n0) : 0.0;
            seg[MAXB + i] = (has && i < nb) ? 0.5 * G.da * (g1[i] + n1) : 0.0;
        }
        __syncthreads();
        if (t == 0)
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                gnx[i] = g0[i];
                gnx[MAXB + i] = g1[i];
            }
        block_scan<2 * MAXB>(seg, buf, true);      // sum over the chunk's segments m >= j
#pragma unroll
        for (int k = 0; k < 2 * MAXB; ++k) seg[k] += gcs[k];
        if (t == 0)
#pragma unroll
            for (int k = 0; k < 2 * MAXB; ++k) bc[k] = seg[k];
        const double pref = 1.5 * Om * H0c * H0c * chi / a;
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            if (i >= nb) continue;
            const double Wg = pref * (seg[i] - chi * seg[MAXB + i]);
            const double AIA = phys(9 + i);
            const double WI = -AIA * C1_RHOCR * Om * nr[i] * H0c * Ea / D;
            Wt[i * 256 + t] = node ? (T)(Wg + WI) : T(0);
        }

        // (c) P at the Limber wavenumbers for this node, node-major [256][nl4]
        // (ell contiguous); log10 k = log10(l + 1/2) - log10 chi_j
        {
            const bool live = node && j > 0;
            const double lchi = live ? log10(chi) : 0.0;
            const T wqj = (node && j > 0) ? (T)(q * fa / (chi * chi)) : T(0);
            const int n = live ? zidx[j] : 0;
            const int zc = live ? 4 * j : 0;
            const T c0 = (T)zcoef[zc], c1 = (T)zcoef[zc + 1];
            const T c2 = LINZ ? T(0) : (T)zcoef[zc + 2], c3 = LINZ ? T(0) : (T)zcoef[zc + 3];
            const T* y0 = Ytab + w * (int64_t)G.n_z * G.n_k + (int64_t)n * G.n_k;
            const T* m0p = LINZ ? y0 : Mtab + w * (int64_t)G.n_z * G.n_k + (int64_t)n * G.n_k;
            auto Yz = [&](int col) {
                if (LINZ) return c0 * y0[col] + c1 * y0[col + G.n_k];
                return c0 * y0[col] + c1 * y0[col + G.n_k] + c2 * m0p[col] + c3 * m0p[col + G.n_k];
            };
#pragma unroll 4
            for (int b = 0; b < nl4; ++b) {
                T P = T(0);
                const double lk = b < G.n_ell ? lell[b] - lchi : 0.0;
                if (live && b < G.n_ell && lk >= G.u0 && lk <= G.u1) {
                    const double sv = (lk - G.u0) / G.du;
                    int i0 = (int)floor(sv);
                    i0 = i0 < 0 ? 0 : (i0 > G.n_k - 2 ? G.n_k - 2 : i0);
                    const T tt = (T)(sv - i0);
                    const T p0 = Yz(i0), p1 = Yz(i0 + 1);
                    const T pm = i0 > 0 ? Yz(i0 - 1) : T(2) * p0 - p1;
                    const T p2 = i0 + 2 < G.n_k ? Yz(i0 + 2) : T(2) * p1 - p0;
                    const T mk0 = T(0.5) * (p1 - pm), mk1 = T(0.5) * (p2 - p0);
                    const T t2 = tt * tt, t3 = t2 * tt;
                    const T lp = (T(2) * t3 - T(3) * t2 + T(1)) * p0 + (t3 - T(2) * t2 + tt) * mk0 +
                                 (T(-2) * t3 + T(3) * t2) * p1 + (t3 - t2) * mk1;
                    P = exp10_of<T>(lp) * wqj;
                }
                Pl[t * nl4 + b] = P;
            }
        }
        __syncthreads();
        if (t == 0)
#pragma unroll
            for (int k = 0; k < 2 * MAXB; ++k) gcs[k] = bc[k];

        // (d) this chunk's share of the Limber sums
        const int jl1 = min(256, na - c * 256);
#pragma unroll
        for (int s = 0; s < LB_SLOTS; ++s) {
            const int it = t + 256 * s;
            if (it >= nitem * nseg) continue;
            const int item = it % nitem, sg = it / nitem;
            const int p = item / ng, gq = item % ng;
            int bi, bj;
            pair_of(p, bi, bj);
            const T* Wi = Wt + bi * 256;
            const T* Wj = Wt + bj * 256;
            const int j0 = max(c == 0 ? 1 : 0, sg * len), j1 = min(jl1, (sg + 1) * len);
            for (int jl = j0; jl < j1; ++jl) {
                const T A = Wi[jl] * Wj[jl];
                const T* Pj = Pl + jl * nl4 + 4 * gq;
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[s][e] += A * Pj[e];
            }
        }
        __syncthreads();
    }

    auto store = [&](int item, const T (&v)[4]) {
        const int p = item / ng, gq = item % ng;
        int bi, bj;
        pair_of(p, bi, bj);
        const double mi = phys(9 + 2 * nb + bi), mj = phys(9 + 2 * nb + bj);
        for (int e = 0; e < 4; ++e) {
            const int b = 4 * gq + e;
            if (b < G.n_ell) Cout[w * nout + p * G.n_ell + b] = (1.0 + mi) * (1.0 + mj) * (double)v[e];
        }
    };
    if (nseg == 1) {
#pragma unroll
        for (int s = 0; s < LB_SLOTS; ++s)
            if (t + 256 * s < nitem) store(t + 256 * s, acc[s]);
    } else {
        T* part = Pl;                                   // [nseg][nitem][4] (nseg nitem <= 256)
        if (t < nitem * nseg)
#pragma unroll
            for (int e = 0; e < 4; ++e) part[t * 4 + e] = acc[0][e];
        __syncthreads();
        for (int item = t; item < nitem; item += 256) {
            T v[4] = {T(0), T(0), T(0), T(0)};
            for (int sg = 0; sg < nseg; ++sg)
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] += part[(sg * nitem + item) * 4 + e];
            store(item, v);
        }
    }
}

// ---------------------------------------------------------------- dense chi^2
// Y = C L^{-T} for a block of 16 walkers on v_mfma_f64_16x16x4f64, then
// chi^2_b = sum_n (w_n - Y_bn)^2 with w = L^{-1} d.  The block's spectra sit
// in LDS (A operand); L^{-1} is read in fragment order (one coalesced 512-byte
// load per wave and MFMA), and the K steps above the diagonal, where L^{-1}
// vanishes, are skipped.  Wave w owns column tiles w, w + 4, ... (DM_CT per
// pass); row sums are reduced in a fixed order (deterministic).
constexpr int DM_W = 16;      // walkers per workgroup
constexpr int DM_CT = 5;      // column tiles per wave per pass
__global__ __launch_bounds__(256) void dense_chi2_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, int d, const int* __restrict__ pk,
    const double* __restrict__ pa, const double* __restrict__ pb, const double* __restrict__ C, int n,
    const double* __restrict__ Lf, const double* __restrict__ wv, double cst, double* __restrict__ logl,
    const int* __restrict__ count) {
    extern __shared__ double Cs[];                 // [DM_W][n16 + 2]
    __shared__ double red[4][DM_W];
    if (count) B = min<int64_t>(B, *count);
    const int64_t w0 = (int64_t)blockIdx.x * DM_W;
    if (w0 >= B) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n16 = (n + 15) & ~15, cs = n16 + 2;
    const int nt_all = n16 / 16, kc_all = n16 / 4;
    for (int e = tid; e < DM_W * n16; e += 256) {
        const int r = e / n16, k = e % n16;
        const int64_t w = w0 + r;
        Cs[r * cs + k] = (w < B && k < n) ? C[w * n + k] : 0.0;
    }
    __syncthreads();
    double srow[4] = {0.0, 0.0, 0.0, 0.0};          // rows (lane >> 4) + 4 r
    for (int t0 = wave; t0 < nt_all; t0 += 4 * DM_CT) {
        f64x4_t acc[DM_CT];
#pragma unroll
        for (int j = 0; j < DM_CT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[j][r] = 0.0;
        const int jmax = min(DM_CT - 1, (nt_all - 1 - t0) / 4);
        const int kmax = min(4 * (t0 + 4 * jmax) + 4, kc_all);
#pragma unroll 2
        for (int kc = 0; kc < kmax; ++kc) {
            const double a = Cs[(lane & 15) * cs + 4 * kc + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < DM_CT; ++j) {
                const int nt = t0 + 4 * j;
                if (j <= jmax && kc < 4 * nt + 4) {
                    const double b = Lf[((size_t)nt * kc_all + kc) * 64 + lane];
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < DM_CT; ++j) {
            const int col = 16 * (t0 + 4 * j) + (lane & 15);
            if (j > jmax || col >= n) continue;
            const double wn = wv[col];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double e = wn - acc[j][r];
                srow[r] = fma(e, e, srow[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) srow[r] += __shfl_xor(srow[r], o, 64);
    if ((lane & 15) == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave][(lane >> 4) + 4 * r] = srow[r];
    __syncthreads();
    if (tid < DM_W) {
        const int64_t w = w0 + tid;
        if (w < B) {
            const double chi2 = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
            bool ok = true;
            const double* th = theta + w * ld;
            for (int i = 0; i < d; ++i)
                if (pk[i] == NS_PRIOR_UNIFORM && (th[i] < pa[i] || th[i] > pb[i])) ok = false;
            logl[w] = ok ? -0.5 * chi2 + cst : -INFINITY;
        }
    }
}

ShearGeom shear_geom(const ns_model* m) {
    ShearGeom G;
    G.n_a = m->n_a; G.n_z = m->n_z; G.n_k = m->n_k; G.n_ell = m->n_ell; G.n_bins = m->n_bins;
    G.n_pairs = m->n_pairs;
    G.a_min = m->a_min; G.da = (1.0 - m->a_min) / (m->n_a - 1); G.zmax = 1.0 / m->a_min - 1.0;
    G.k_min = m->k_min; G.k_max = m->k_max; G.u0 = log10(m->k_min);
    G.du = (log10(m->k_max) - log10(m->k_min)) / (m->n_k - 1); G.nz_sigma = m->nz_sigma;
    G.u1 = log10(m->k_max);
    return G;
}

static size_t limber_smem(const ns_model* m, size_t elem) {
    const size_t nch = (m->n_a + 255) / 256;
    return (2 * MAXB * 4 + MAXB * 4 + 3 * 2 * MAXB + 2 * MAXB + 4 * 2 * MAXB + 2 * (nch * 256 + 1)) * sizeof(double) +
           (size_t)(m->n_bins + ((m->n_ell + 3) & ~3)) * 256 * elem;
}

template <bool LINZ>
static void launch_limber(ns_model* m, const double* theta, int64_t ld, int64_t B, int prec, const void* Mtab,
                          double* Cv, const int* count, size_t sm, hipStream_t s) {
    const ShearGeom G = shear_geom(m);
    if (prec == NS_FP64)
        hipLaunchKernelGGL((limber_kernel<double, LINZ>), dim3((unsigned)B), dim3(256), sm, s, theta, ld, B, G,
                           m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->nz_mean_d.as<double>(),
                           m->agrid_d.as<double>(), m->zsp_idx_d.as<int>(), m->zsp_coef_d.as<double>(),
                           m->lell_d.as<double>(), m->ws_out.as<double>(), (const double*)Mtab, Cv, count);
    else
        hipLaunchKernelGGL((limber_kernel<float, LINZ>), dim3((unsigned)B), dim3(256), sm, s, theta, ld, B, G,
                           m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->nz_mean_d.as<double>(),
                           m->agrid_d.as<double>(), m->zsp_idx_d.as<int>(), m->zsp_coef_d.as<double>(),
                           m->lell_d.as<double>(), m->ws_out.as<float>(), (const float*)Mtab, Cv, count);
    NS_HIP(hipGetLastError());
}

void shear_loglike_from_table(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl,
                              int prec, const int* count, hipStream_t s) {
    const int nk = m->n_k, nz = m->n_z;
    const size_t elem = prec == NS_FP64 ? 8 : 4;
    const int n = m->n_data;
    // aux: spline second derivatives [B x nz x nk] (cubic z only) then spectra [B x n] (double)
    const size_t mbytes = m->z_linear ? 0 : (size_t)B * nz * nk * elem;
    m->ws_aux.ensure(mbytes + (size_t)B * n * sizeof(double));
    void* Mtab = m->ws_aux.p;
    double* Cv = reinterpret_cast<double*>(m->ws_aux.as<char>() + mbytes);
    const double zmax = 1.0 / m->a_min - 1.0;
    const double hz = zmax / (nz - 1);
    if (!m->shear_attr_set) {   // once per model, outside any stream capture
        const void* fns[4] = {(const void*)limber_kernel<double, false>, (const void*)limber_kernel<float, false>,
                              (const void*)limber_kernel<double, true>, (const void*)limber_kernel<float, true>};
        for (const void* f : fns)
            NS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        NS_HIP(hipFuncSetAttribute((const void*)zspline_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   150 * 1024));
        NS_HIP(hipFuncSetAttribute((const void*)zspline_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   150 * 1024));
        m->shear_attr_set = true;
    }
    if (!m->z_linear) {
        const int64_t nthr = B * nk;
        dim3 gz((unsigned)((nthr + 63) / 64));
        TraceScope ts(m, s, "zspline");
        const size_t zsm = (size_t)nz * 64 * elem;
        if (prec == NS_FP64)
            hipLaunchKernelGGL(zspline_kernel<double>, gz, dim3(64), zsm, s, m->ws_out.as<double>(), (double*)Mtab,
                               B, nz, nk, hz, count);
        else
            hipLaunchKernelGGL(zspline_kernel<float>, gz, dim3(64), zsm, s, m->ws_out.as<float>(), (float*)Mtab, B,
                               nz, nk, hz, count);
        NS_HIP(hipGetLastError());
    }
    const size_t sm = limber_smem(m, elem);
    NS_CHECK(sm <= 160 * 1024, NS_E_UNSUPPORTED, "Limber stage needs more LDS than a workgroup has");
    {
        TraceScope ts(m, s, "limber");
        if (m->z_linear)
            launch_limber<true>(m, theta, ld, B, prec, Mtab, Cv, count, sm, s);
        else
            launch_limber<false>(m, theta, ld, B, prec, Mtab, Cv, count, sm, s);
    }
    const size_t sm2 = (size_t)DM_W * (((n + 15) & ~15) + 2) * sizeof(double);
    if (sm2 > 64 * 1024 && !m->chi2_attr_set) {
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)sm2));
        m->chi2_attr_set = true;
    }
    TraceScope ts(m, s, "dense_chi2");
    hipLaunchKernelGGL(dense_chi2_kernel, dim3((unsigned)((B + DM_W - 1) / DM_W)), dim3(256), sm2, s, theta, ld, B,
                       m->d, m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(), Cv, n,
                       m->cov_linv_frag.as<double>(), m->cov_w.as<double>(), m->logl_const, logl, count);
    NS_HIP(hipGetLastError());
}

}  // namespace nsmi
