// Cosmic-shear likelihood stages after the emulator (App. A of the paper).
//
// zspline_reg_kernel, zspline_kernel
//                  second derivatives M_n(k) of the not-a-knot cubic spline of
//                  log10 P along the uniform z nodes, one thread per (walker, k)
//                  (the column in registers for n_z <= 64, else in LDS):
//                  M_1 and M_{N-2} follow directly from the not-a-knot
//                  conditions on a uniform grid, the interior (1, 4, 1)
//                  system is solved by a Thomas sweep, M_0 and M_{N-1} are
//                  linear extrapolations.
// shear_windows_kernel  one workgroup per walker, one wave per bin for (b):
//                  (a) background on the a-grid: E(a), chi by per-interval
//                      Simpson, J = dchi/d(-a), growth D (growth index 0.55);
//                  (b) n_i(z) with photo-z shifts (normalised by the trapezoid
//                      rule); lensing window Eq. (A3) as (chi/a)(G0 - chi G1)
//                      with reverse cumulative trapezoids; NLA window Eq. (A4);
//                      effective window W = W^g + W^I (the four terms of Eq. (A1)
//                      share P_dd); all FP64.
// limber_sum_kernel  one workgroup per (walker, chunk of 256 nodes):
//                  (c) P(k = (l+1/2)/chi_j, z_j): spline or linear in z,
//                      Catmull-Rom in log10 k (linear ghost nodes), zero
//                      outside [k_min, k_max];
//                  (d) Limber sum Eq. (A2) by the trapezoid rule in a with the
//                      analytic Jacobian, times (1 + m_i)(1 + m_j);
//                  (c)-(d) run in the form's type T.
// dense_chi2_gemm_kernel, dense_chi2_finish_kernel
//                  y = L^{-1} d - L^{-1} C with the host-factorised dense
//                  covariance, logL = -1/2 |y|^2 - sum log L_ii - n/2 log 2 pi
//                  (FP64; L^{-1} C as a tiled GEMM on the FP64 MFMA).
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

// zspline_reg_kernel: the same sweep for n_z <= NZ with the column held in
// registers (one thread per (walker, k) column, 256 per workgroup): no LDS
// staging, so more waves per CU hide the serial sweep.  The loops run over
// the compile-time bound NZ with the run-time n_z as a guard, so the column
// stays in registers; every value is computed by the expressions of
// zspline_kernel in the same order.
template <class T, int NZ>
__global__ __launch_bounds__(256) void zspline_reg_kernel(const T* __restrict__ Y, T* __restrict__ M, int64_t B,
                                                          int nz, int nk, double h, const int* __restrict__ count) {
    __shared__ T cps[NZ];
    if (threadIdx.x == 0) {
        T c = T(0);
        for (int n = 2; n <= nz - 3; ++n) {
            c = T(1) / (T(4) - (n == 2 ? T(0) : c));
            cps[n] = c;
        }
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (count) B = min<int64_t>(B, *count);
    if (g >= B * nk) return;
    const int64_t w = g / nk;
    const int c = (int)(g % nk);
    const T* y = Y + w * nz * nk + c;
    T* mm = M + w * nz * nk + c;
    T v[NZ];                                            // y_n, then d'_n of the sweep
#pragma unroll
    for (int n = 0; n < NZ; ++n) v[n] = n < nz ? y[(int64_t)n * nk] : T(0);
    T yl0 = T(0), yl1 = T(0), yl2 = T(0);               // y at n_z - 1, n_z - 2, n_z - 3
#pragma unroll
    for (int n = 0; n < NZ; ++n) {
        if (n == nz - 1) yl0 = v[n];
        if (n == nz - 2) yl1 = v[n];
        if (n == nz - 3) yl2 = v[n];
    }
    const T ih2 = T(1.0 / (h * h));
    const T M1 = (v[2] - T(2) * v[1] + v[0]) * ih2;
    const T Mb = (yl0 - T(2) * yl1 + yl2) * ih2;       // M_{N-2}
    T M2 = Mb, Mc = M1;                                 // n_z = 4: nodes 2 and n_z - 3 are N-2 and 1
    if (nz > 4) {
        T dpv = T(0);
        T ym = v[1], y0 = v[2];
#pragma unroll
        for (int n = 2; n < NZ - 1; ++n) {
            if (n > nz - 3) continue;
            const T yp = v[n + 1];
            T rhs = T(6) * (yp - T(2) * y0 + ym) * ih2;
            if (n == 2) rhs -= M1;
            if (n == nz - 3) rhs -= Mb;
            dpv = (rhs - (n == 2 ? T(0) : dpv)) * cps[n];
            v[n] = dpv;                                 // y_n is held in y0 from here on
            ym = y0;
            y0 = yp;
        }
        T next = dpv;                                   // M_{nz-3} = d'_{nz-3}
        mm[(int64_t)(nz - 3) * nk] = next;
        Mc = next;
#pragma unroll
        for (int n = NZ - 1; n >= 2; --n) {
            if (n > nz - 4) continue;
            next = v[n] - cps[n] * next;
            mm[(int64_t)n * nk] = next;
        }
        M2 = next;
    }
    mm[(int64_t)1 * nk] = M1;
    mm[(int64_t)(nz - 2) * nk] = Mb;
    mm[0] = T(2) * M1 - M2;
    mm[(int64_t)(nz - 1) * nk] = T(2) * Mb - Mc;
}

// shear_windows_kernel: one workgroup (256 threads) per walker, in four
// phases over the n_a nodes.  Per-node values live in LDS in lane-major order:
// with k = ceil(n_a / 64), node j sits at (j mod k) 64 + j / k, so lane l of a
// wave that owns the consecutive nodes l k .. l k + k - 1 reads them without
// bank conflicts, and every running sum below is a serial pass over k nodes
// in registers plus one wave-wide scan of the 64 lane totals.
// (1) every thread: E(a), f = dchi/d(-a) = c / (H0 a^2 E) and the growth
//     integrand Om(a)^0.55 / a at its nodes, then at the midpoints of its
//     intervals, giving the Simpson increments of chi and of -ln D; powers of
//     a come from the model's ln a_j and ln a_mid tables (one exp each);
// (2) waves 0 and 1: exclusive prefix sums of the two increments, in place
//     (chi_j and -ln D_j);
// (3) every thread: the per-node factors of the windows; log10 chi_j out;
// (4) one wave per tomographic bin (bins i, i + 4, ...): unnormalised n_i(z_j),
//     the reverse cumulative trapezoids G0, G1 (a first pass for the lane
//     totals, a suffix scan over the lanes, a second pass that carries the
//     sums down the lane's nodes), and W_i = W^g_i + W^I_i
//     (Eqs. (A3), (A4)) times sqrt(q_j J_j / chi_j^2); the n_i normalisation
//     is summed on the way.
// The windows are linear in n_i, so the normalisations are applied to the
// spectra.  Output per walker: the scaled windows [nb][n_a] (the Limber
// integrand is the product of two of them and P), log10 chi_j [n_a] and the
// normalisations [nb].
template <class T, int KMAX>
__global__ __launch_bounds__(256, 2) void shear_windows_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, ShearGeom G,
    const int* __restrict__ pidx, const double* __restrict__ pfix, const double* __restrict__ nz_mean,
    const double* __restrict__ agrid, const double* __restrict__ lna, T* __restrict__ Wout,
    double* __restrict__ lchi_out, double* __restrict__ norm_out, const int* __restrict__ count) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (count) B = min<int64_t>(B, *count);
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    constexpr int NW = 4;                     // waves (blockDim 256)
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int na = G.n_a, nb = G.n_bins;
    const int k = (na + 63) >> 6, L = 64 * k;
    double* S0 = reinterpret_cast<double*>(smem);
    double* S1 = S0 + L;
    double* S2 = S1 + L;
    double* S3 = S2 + L;
    double* S4 = S3 + L;
    double* S5 = S4 + L;

    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double ob = phys(0), oc = phys(1), h = phys(2), w0 = phys(5), wa = phys(6);
    const double Om = (ob + oc) / (h * h);
    const double cH0 = C_KM_S / (100.0 * h), H0c = 1.0 / cH0;
    const double pde = -3.0 * (1.0 + w0 + wa);
    // E, f and the growth integrand at scale factor a (ln a given)
    auto bg = [&](double a, double la, double& E, double& f, double& g) {
        const double ia = 1.0 / a, ia2 = ia * ia, ia3 = ia2 * ia;
        const double E2 = Om * ia3 + (1.0 - Om) * exp(pde * la - 3.0 * wa * (1.0 - a));
        E = sqrt(E2);
        f = cH0 * ia2 / E;
        g = exp(GROWTH_INDEX * log(Om * ia3 / E2)) * ia;
    };

    // (1) S0 E_j, S1 f_j, S2 growth integrand; S3, S4 the Simpson increments
    // of the interval [j, j+1] (0 for the last node)
    // (threads walk the positions p = r 64 + l, node j = l k + r; at most
    // KMAX / 4 per thread, unrolled so that their exp / log chains overlap)
    constexpr int U = (KMAX + 3) / 4;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = t + 256 * u;
        const int j = (p & 63) * k + (p >> 6);
        if (p >= L || j >= na) continue;
        double E, f, g;
        bg(agrid[j], lna[j], E, f, g);
        S0[p] = E;
        S1[p] = f;
        S2[p] = g;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = t + 256 * u;
        const int r = p >> 6, j = (p & 63) * k + r;
        if (p >= L || j >= na) continue;
        double ic = 0.0, id = 0.0;
        if (j < na - 1) {
            double E, f, g;
            bg(0.5 * (agrid[j] + agrid[j + 1]), lna[na + j], E, f, g);
            const int p1 = r + 1 < k ? p + 64 : (p & 63) + 1;     // node j + 1
            ic = G.da / 6.0 * (S1[p] + 4.0 * f + S1[p1]);
            id = G.da / 6.0 * (S2[p] + 4.0 * g + S2[p1]);
        }
        S3[p] = ic;
        S4[p] = id;
    }
    __syncthreads();
    // (2) S3 <- chi_j, S4 <- -ln D_j (sums over the intervals below j)
    if (wid < 2) {
        double* X = wid == 0 ? S3 : S4;
        double run = 0.0;
        for (int r = 0; r < k; ++r)
            if (lane * k + r < na) {
                const double x = X[r * 64 + lane];
                X[r * 64 + lane] = run;
                run += x;
            }
        double inc = run;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        const double up = __shfl_up(inc, 1, 64), ex = lane > 0 ? up : 0.0;
        for (int r = 0; r < k; ++r)
            if (lane * k + r < na) X[r * 64 + lane] += ex;
    }
    __syncthreads();
    // (3) per-node factors, in place: S0 z_j, S1 1/a^2, S2 1/(a^2 chi),
    // S3 sw pref, S4 sw pref chi, S5 sw wI; sw = sqrt(q f / chi^2),
    // pref = (3/2) Om (H0/c)^2 chi / a, wI = -C1 rho_cr Om (H0/c) E / D
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = t + 256 * u;
        const int j = (p & 63) * k + (p >> 6);
        if (p >= L || j >= na) continue;
        const double a = agrid[j], E = S0[p], f = S1[p], chi = S3[p], D = exp(-S4[p]);
        const double ia = 1.0 / a, ia2 = ia * ia;
        const double q = (j == 0 || j == na - 1) ? 0.5 * G.da : G.da;
        const bool in = j > 0;
        const double sw = in ? sqrt(q * f / (chi * chi)) : 0.0;
        const double pref = 1.5 * Om * H0c * H0c * chi * ia;
        S0[p] = ia - 1.0;
        S1[p] = ia2;
        S2[p] = in ? ia2 / chi : 0.0;
        S3[p] = sw * pref;
        S4[p] = sw * pref * chi;
        S5[p] = -sw * C1_RHOCR * Om * H0c * E / D;
        lchi_out[w * na + j] = in ? log10(chi) : 0.0;
    }
    __syncthreads();
    // (4) one wave per bin; lane l owns nodes l k + r, r < k <= KMAX, its
    // n_i values held in registers between the two passes
    const double is2 = 1.0 / (2.0 * G.nz_sigma * G.nz_sigma), hda = 0.5 * G.da;
    const int j0 = lane * k;
    for (int i = wid; i < nb; i += NW) {
        const double mu = nz_mean[i] + phys(9 + nb + i), AIA = phys(9 + i);
        double nrv[KMAX];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) {      // unnormalised n_i(z_j), 0 at z = 0
            const int j = j0 + r;
            double v = 0.0;
            if (r < k && j > 0 && j < na) {
                const double dz = S0[r * 64 + lane] - mu;
                v = exp(-dz * dz * is2);
            }
            nrv[r] = v;
        }
        // integrands at the first node of the next lane
        const double f0 = j0 < na ? nrv[0] * S1[lane] : 0.0, f1 = j0 < na ? nrv[0] * S2[lane] : 0.0;
        double n0 = __shfl_down(f0, 1, 64), n1 = __shfl_down(f1, 1, 64);
        if (lane == 63) n0 = n1 = 0.0;
        // lane totals of the trapezoid segments [j, j+1], and the normalisation
        double tot0 = 0.0, tot1 = 0.0, nsum = 0.0, x0 = n0, x1 = n1;
#pragma unroll
        for (int r = KMAX - 1; r >= 0; --r) {
            const int j = j0 + r, p = r * 64 + lane;
            if (r >= k) continue;
            double g0 = 0.0, g1 = 0.0;
            if (j < na) {
                g0 = nrv[r] * S1[p];
                g1 = nrv[r] * S2[p];
                nsum += (j == na - 1 ? hda : G.da) * g0;
                if (j < na - 1) {
                    tot0 += hda * (g0 + x0);
                    tot1 += hda * (g1 + x1);
                }
            }
            x0 = g0;
            x1 = g1;
        }
        // sums over the nodes of the lanes above
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double y0 = __shfl_down(tot0, off, 64), y1 = __shfl_down(tot1, off, 64);
            if (lane + off < 64) {
                tot0 += y0;
                tot1 += y1;
            }
        }
        double c0 = __shfl_down(tot0, 1, 64), c1 = __shfl_down(tot1, 1, 64);
        if (lane == 63) c0 = c1 = 0.0;
        T* Wo = Wout + (w * nb + i) * na;
        x0 = n0;
        x1 = n1;
#pragma unroll
        for (int r = KMAX - 1; r >= 0; --r) {
            const int j = j0 + r, p = r * 64 + lane;
            if (r >= k || j >= na) continue;
            const double nr = nrv[r];
            const double g0 = nr * S1[p], g1 = nr * S2[p];
            if (j < na - 1) {
                c0 += hda * (g0 + x0);
                c1 += hda * (g1 + x1);
            }
            Wo[j] = (T)(S3[p] * c0 - S4[p] * c1 + AIA * S5[p] * nr);
            x0 = g0;
            x1 = g1;
        }
        const double v = wave_sum(nsum);
        if (lane == 0) norm_out[w * nb + i] = v;
    }
}

// limber_sum_kernel: one workgroup (256 threads) per (walker, chunk of 256
// nodes).  (c) thread = node: log10 P carried to z_j (cubic spline or linear
// in z), Catmull-Rom in log10 k at k = (l + 1/2)/chi_j, P = 10^(.), zero
// outside [k_min, k_max]; [256][LB] in LDS with the chunk's scaled windows.
// (d) thread = (pair, node segment): all LB multipoles of one pair in
// registers, C_ij(l) += W~_i W~_j P(l); the segments are added in a fixed
// order, times (1 + m_i)(1 + m_j) / (N_i N_j) with the n(z) normalisations N.
template <class T, bool LINZ, int LB>
__global__ __launch_bounds__(256) void limber_sum_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t B, ShearGeom G,
    const int* __restrict__ pidx, const double* __restrict__ pfix, const int* __restrict__ zidx,
    const double* __restrict__ zcoef, const double* __restrict__ lell, const T* __restrict__ Ytab,
    const T* __restrict__ Mtab, const T* __restrict__ Win, const double* __restrict__ lchi_in,
    const double* __restrict__ norm_in, double* __restrict__ Cout, double* __restrict__ part,
    const int* __restrict__ count) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    if (count) B = min<int64_t>(B, *count);
    const int64_t w = blockIdx.x;
    if (w >= B) return;
    const int t = threadIdx.x;
    const int na = G.n_a, nb = G.n_bins, npr = G.n_pairs, nl = G.n_ell;
    const int nch = (na + 255) / 256, c = blockIdx.y;    // this workgroup's chunk of nodes
    constexpr int WS = 257;                                           // padded row of the window table
    T* Ws = reinterpret_cast<T*>(smem);                               // [nb][WS]
    T* Pl = Ws + nb * WS;                                             // [256][LB]
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    auto pair_of = [&](int p, int& bi, int& bj) {
        int rem = p;
        bi = 0;
        while (rem >= nb - bi) { rem -= nb - bi; ++bi; }
        bj = bi + rem;
    };
    const int nseg = max(1, 256 / npr);
    const int len = (256 + nseg - 1) / nseg;
    const bool worker = t < npr * nseg;
    const int pw = t % npr, sg = t / npr;
    int bi = 0, bj = 0;
    if (worker) pair_of(pw, bi, bj);
    T acc[LB];
#pragma unroll
    for (int e = 0; e < LB; ++e) acc[e] = T(0);
    const int64_t tab = w * (int64_t)G.n_z * G.n_k;
    {
        const int j = c * 256 + t;
        const bool node = j < na;
        for (int i = 0; i < nb; ++i) Ws[i * WS + t] = node ? Win[(w * nb + i) * na + j] : T(0);
        const bool live = node && j > 0;
        const double lchi = live ? lchi_in[w * na + j] : 0.0;
        const int n = live ? zidx[j] : 0;
        const int zc = live ? 4 * j : 0;
        const T c0 = (T)zcoef[zc], c1 = (T)zcoef[zc + 1];
        const T c2 = LINZ ? T(0) : (T)zcoef[zc + 2], c3 = LINZ ? T(0) : (T)zcoef[zc + 3];
        const T* y0 = Ytab + tab + (int64_t)n * G.n_k;
        const T* m0p = LINZ ? y0 : Mtab + tab + (int64_t)n * G.n_k;
        // log10 P at z_j from rows n, n + 1 of Y (and of M for cubic z)
        auto zmix = [&](T ya, T yb, T ma, T mb) {
            if (LINZ) return c0 * ya + c1 * yb;
            return c0 * ya + c1 * yb + c2 * ma + c3 * mb;
        };
        auto Yz = [&](int col) {
            return zmix(y0[col], y0[col + G.n_k], LINZ ? T(0) : m0p[col], LINZ ? T(0) : m0p[col + G.n_k]);
        };
        // the four columns i0 - 1 .. i0 + 2 of one row in one load each (the
        // rows are only element-aligned; the target allows such vector loads)
        struct Q4 { T v[4]; };
        auto row4 = [&](const T* p) { Q4 q; __builtin_memcpy(&q, p, sizeof(q)); return q; };
#pragma unroll 4
        for (int b = 0; b < LB; ++b) {
            T P = T(0);
            const double lk = b < nl ? lell[b] - lchi : 0.0;
            if (live && b < nl && lk >= G.u0 && lk <= G.u1) {
                const double sv = (lk - G.u0) / G.du;
                int i0 = (int)floor(sv);
                i0 = i0 < 0 ? 0 : (i0 > G.n_k - 2 ? G.n_k - 2 : i0);
                const T tt = (T)(sv - i0);
                T pm, p0, p1, p2;
                if (i0 > 0 && i0 + 2 < G.n_k) {
                    const Q4 ya = row4(y0 + i0 - 1), yb = row4(y0 + G.n_k + i0 - 1);
                    Q4 ma = {}, mb = {};
                    if (!LINZ) {
                        ma = row4(m0p + i0 - 1);
                        mb = row4(m0p + G.n_k + i0 - 1);
                    }
                    pm = zmix(ya.v[0], yb.v[0], ma.v[0], mb.v[0]);
                    p0 = zmix(ya.v[1], yb.v[1], ma.v[1], mb.v[1]);
                    p1 = zmix(ya.v[2], yb.v[2], ma.v[2], mb.v[2]);
                    p2 = zmix(ya.v[3], yb.v[3], ma.v[3], mb.v[3]);
                } else {
                    p0 = Yz(i0);
                    p1 = Yz(i0 + 1);
                    pm = i0 > 0 ? Yz(i0 - 1) : T(2) * p0 - p1;
                    p2 = i0 + 2 < G.n_k ? Yz(i0 + 2) : T(2) * p1 - p0;
                }
                const T mk0 = T(0.5) * (p1 - pm), mk1 = T(0.5) * (p2 - p0);
                const T t2 = tt * tt, t3 = t2 * tt;
                const T lp = (T(2) * t3 - T(3) * t2 + T(1)) * p0 + (t3 - T(2) * t2 + tt) * mk0 +
                             (T(-2) * t3 + T(3) * t2) * p1 + (t3 - t2) * mk1;
                P = exp10_of<T>(lp);
            }
            Pl[t * LB + b] = P;
        }
        __syncthreads();
        if (worker) {
            const int j0 = sg * len, j1 = min(min(256, na - c * 256), (sg + 1) * len);
            const T* Wi = Ws + bi * WS;
            const T* Wj = Ws + bj * WS;
            for (int jl = j0; jl < j1; ++jl) {
                const T A = Wi[jl] * Wj[jl];
                const T* Pj = Pl + jl * LB;
#pragma unroll
                for (int e = 0; e < LB; ++e) acc[e] += A * Pj[e];
            }
        }
        __syncthreads();
    }
    // segments -> LDS (nseg npr <= 256 rows of LB), added in order; with
    // several chunks the chunk's sums go to `part` for limber_reduce_kernel
    if (worker)
#pragma unroll
        for (int e = 0; e < LB; ++e) Pl[(sg * npr + pw) * LB + e] = acc[e];
    __syncthreads();
    const int nout = npr * nl;
    for (int o = t; o < nout; o += 256) {
        const int p = o / nl, b = o % nl;
        T v = T(0);
        for (int s = 0; s < nseg; ++s) v += Pl[(s * npr + p) * LB + b];
        if (nch > 1) {
            part[(w * nch + c) * nout + o] = (double)v;
            continue;
        }
        int ci, cj;
        pair_of(p, ci, cj);
        const double mi = phys(9 + 2 * nb + ci), mj = phys(9 + 2 * nb + cj);
        Cout[w * nout + o] = (1.0 + mi) * (1.0 + mj) * (double)v / (norm_in[w * nb + ci] * norm_in[w * nb + cj]);
    }
}

// Sum of the node chunks' Limber partial sums in chunk order, times
// (1 + m_i)(1 + m_j) / (N_i N_j); one thread per (walker, spectrum, multipole).
__global__ void limber_reduce_kernel(const double* __restrict__ theta, int64_t ld, int64_t B, ShearGeom G,
                                     const int* __restrict__ pidx, const double* __restrict__ pfix,
                                     const double* __restrict__ norm_in, const double* __restrict__ part,
                                     double* __restrict__ Cout, const int* __restrict__ count) {
    if (count) B = min<int64_t>(B, *count);
    const int nb = G.n_bins, nl = G.n_ell, nout = G.n_pairs * nl, nch = (G.n_a + 255) / 256;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= B * nout) return;
    const int64_t w = g / nout;
    const int o = (int)(g % nout), p = o / nl;
    double v = 0.0;
    for (int c = 0; c < nch; ++c) v += part[(w * nch + c) * nout + o];
    int ci = 0, rem = p;
    while (rem >= nb - ci) { rem -= nb - ci; ++ci; }
    const int cj = ci + rem;
    auto phys = [&](int slot) { const int ix = pidx[slot]; return ix >= 0 ? theta[w * ld + ix] : pfix[slot]; };
    const double mi = phys(9 + 2 * nb + ci), mj = phys(9 + 2 * nb + cj);
    Cout[w * nout + o] = (1.0 + mi) * (1.0 + mj) * v / (norm_in[w * nb + ci] * norm_in[w * nb + cj]);
}

// ---------------------------------------------------------------- dense chi^2
// Y = C L^{-T} as a GEMM over (64-walker x 64-column) output tiles on
// v_mfma_f64_16x16x4f64: each wave owns a 32 x 32 quarter (2 x 2 MFMA
// tiles); K blocks of 32 are staged through LDS (double-buffered, the next
// block's global loads in flight during the current block's MFMAs).  L^{-T}
// is lower-triangular in (column, k), so a column tile stops at its own K
// range.  Each tile writes its walkers' partial sums of (w_n - Y_bn)^2 over its
// 64 columns, w = L^{-1} d; dense_chi2_finish_kernel adds the column tiles in
// a fixed order (deterministic).
// BM walkers per tile: 64 (four waves of 32 walkers x 32 columns), or 32 (four
// waves of 16 x 32) when the 64-walker grid has fewer than eight workgroups
// per CU: the column tiles of a triangular L^{-T} differ in length up to n / 64
// fold, and with few workgroups the longest ones run alone.  Both pair the
// same columns within a lane and reduce them in the same order, so a walker's
// chi^2 is the same for either.
// K blocks of KB = 32, or 64 when the 32-walker grid has no more workgroups
// than the GPU has CUs: there each K block costs a global-load latency that
// the MFMA work of a block does not cover, so half as many blocks (its 99 KB
// of LDS allow one workgroup per CU, which a larger grid would queue behind)
constexpr int DG_N = 64;
template <int BM, int KB>
constexpr size_t dg_smem() { return (2 * KB * BM + 2 * KB * DG_N + 2 * BM) * sizeof(double); }
// MODE 0: Y = C L^{-T} (Bm = L^{-T}, K range [0, 64 (ct + 1))), partial sums of
//         (w - Y)^2; with R != nullptr also the residuals R = w - Y.
// MODE 1: out = R L^{-1} (Bm = L^{-1} row-major, K range [64 ct, np)), the
//         chi^2 adjoint g_C = L^{-T} L^{-1} (d - C), written to `out`.
template <int MODE, int BM, int KB>
__global__ __launch_bounds__(256) void dense_chi2_gemm_kernel(const double* __restrict__ C, int64_t B, int n, int np,
                                                              const double* __restrict__ Lt,
                                                              const double* __restrict__ wv,
                                                              double* __restrict__ part, int64_t pstride,
                                                              double* __restrict__ R, const int* __restrict__ count) {
    extern __shared__ double dg_lds[];
    constexpr int TI = BM / 32;                        // 16-walker MFMA tiles per wave
    constexpr int LA = BM * KB / 256;                  // A elements per thread and K block
    constexpr int LB = KB * DG_N / 256;                // B elements per thread and K block
    constexpr int LQ = LA > LB ? LA : LB;
    auto As = reinterpret_cast<double (*)[KB][BM]>(dg_lds);                           // [2][k][walker]
    auto Bs = reinterpret_cast<double (*)[KB][DG_N]>(dg_lds + 2 * KB * BM);           // [2][k][column]
    auto red = reinterpret_cast<double (*)[BM]>(dg_lds + 2 * KB * (BM + DG_N));       // [2][walker]
    if (count) B = min<int64_t>(B, *count);
    const int64_t b0 = (int64_t)blockIdx.x * BM;
    if (b0 >= B) return;
    const int ct = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (BM / 2) * (wave >> 1), wc = 32 * (wave & 1);
    const int kbeg = MODE == 0 ? 0 : DG_N * ct;
    const int kend = MODE == 0 ? min(np, DG_N * (ct + 1)) : np;
    double ra[LA], rb[LB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < LQ; ++q) {
            const int e = tid + 256 * q;
            if (q < LA) {
                const int row = e / KB, k = e % KB;       // A: KB consecutive k of one walker
                const int64_t b = b0 + row;
                const int kk = k0 + k;
                ra[q] = (b < B && kk < n) ? C[b * n + kk] : 0.0;
            }
            if (q < LB) {
                const int kb = e >> 6, col = e & 63;      // B: one row of the column tile
                rb[q] = Lt[(size_t)(k0 + kb) * np + DG_N * ct + col];
            }
        }
    };
    auto sstore = [&](int bf) {
#pragma unroll
        for (int q = 0; q < LQ; ++q) {
            const int e = tid + 256 * q;
            if (q < LA) As[bf][e % KB][e / KB] = ra[q];
            if (q < LB) Bs[bf][e >> 6][e & 63] = rb[q];
        }
    };
    f64x4_t acc[TI][2];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
    gload(kbeg);
    sstore(0);
    __syncthreads();
    int bf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += KB) {
        const bool more = k0 + KB < kend;
        if (more) gload(k0 + KB);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            double a[TI], bv[2];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = As[bf][kk + (lane >> 4)][wr + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[bf][kk + (lane >> 4)][wc + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (more) sstore(bf ^ 1);
        __syncthreads();
        bf ^= 1;
    }
    // D row (lane >> 4) + 4 r, column lane & 15 of MFMA tile (i, j)
    if (MODE == 1) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t b = b0 + wr + 16 * i + (lane >> 4) + 4 * r;
                    const int col = DG_N * ct + wc + 16 * j + (lane & 15);
                    if (b < B && col < n) R[b * n + col] = acc[i][j][r];
                }
        return;
    }
    // (w_n - Y_bn)^2 summed over this wave's columns
    double srow[TI][4];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double sacc = 0.0;
            const int64_t b = b0 + wr + 16 * i + (lane >> 4) + 4 * r;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = DG_N * ct + wc + 16 * j + (lane & 15);
                if (col < n) {
                    const double e = wv[col] - acc[i][j][r];
                    sacc = fma(e, e, sacc);
                    if (R != nullptr && b < B) R[b * n + col] = e;
                }
            }
            srow[i][r] = sacc;
        }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) srow[i][r] += __shfl_xor(srow[i][r], o, 64);
    if ((lane & 15) == 0)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave & 1][wr + 16 * i + (lane >> 4) + 4 * r] = srow[i][r];
    __syncthreads();
    if (tid < BM && b0 + tid < B) part[(int64_t)ct * pstride + b0 + tid] = red[0][tid] + red[1][tid];
}

__global__ void dense_chi2_finish_kernel(const double* __restrict__ theta, int64_t ld, int64_t B, int d,
                                         const int* __restrict__ pk, const double* __restrict__ pa,
                                         const double* __restrict__ pb, const double* __restrict__ part,
                                         int64_t pstride, int n_ct, double cst, double* __restrict__ logl,
                                         const int* __restrict__ count) {
    if (count) B = min<int64_t>(B, *count);
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    SupportLoads sup;                                  // in flight with the partials
    support_load(sup, theta + w * ld, d, pk, pa, pb);
    // the column tiles' partials added in tile order, loaded eight at a time
    double chi2 = 0.0;
    for (int c0 = 0; c0 < n_ct; c0 += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = c0 + j < n_ct ? part[(int64_t)(c0 + j) * pstride + w] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (c0 + j < n_ct) chi2 += v[j];
    }
    logl[w] = support_test(sup, theta + w * ld, d, pk, pa, pb) ? -0.5 * chi2 + cst : -INFINITY;
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

static size_t windows_smem(const ns_model* m) { return 6 * 64 * (size_t)((m->n_a + 63) / 64) * sizeof(double); }

static int limber_lb(const ns_model* m) { return m->n_ell <= 20 ? 20 : 32; }

static size_t limber_sum_smem(const ns_model* m, size_t elem) {
    return ((size_t)m->n_bins * 257 + 256 * (size_t)limber_lb(m)) * elem;
}

template <class T, bool LINZ>
static void launch_limber_sum(ns_model* m, const ShearGeom& G, const double* theta, int64_t ld, int64_t B,
                              const void* Mtab, const T* Win, const double* lchi, const double* norm, double* Cv,
                              double* part, const int* count, size_t sm, hipStream_t s) {
    const int nch = (m->n_a + 255) / 256;
    auto kern = limber_lb(m) == 20 ? limber_sum_kernel<T, LINZ, 20> : limber_sum_kernel<T, LINZ, 32>;
    hipLaunchKernelGGL(kern, dim3((unsigned)B, (unsigned)nch), dim3(256), sm, s, theta, ld, B, G,
                       m->pidx_d.as<int>(), m->pfix_d.as<double>(), m->zsp_idx_d.as<int>(),
                       m->zsp_coef_d.as<double>(), m->lell_d.as<double>(), m->ws_out.as<T>(), (const T*)Mtab, Win,
                       lchi, norm, Cv, part, count);
    NS_HIP(hipGetLastError());
    if (nch > 1) {
        const int64_t n = B * m->n_data;
        hipLaunchKernelGGL(limber_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, ld, B, G,
                           m->pidx_d.as<int>(), m->pfix_d.as<double>(), norm, part, Cv, count);
        NS_HIP(hipGetLastError());
    }
}

template <class T>
static void launch_limber(ns_model* m, const double* theta, int64_t ld, int64_t B, const void* Mtab, double* Cv,
                          const int* count, hipStream_t s) {
    const ShearGeom G = shear_geom(m);
    const int na = m->n_a, nb = m->n_bins;
    // windows [B][nb][na] (T), log10 chi [B][na], normalisations [B][nb], and
    // the Limber sums of each node chunk [B][nch][n_data]
    const size_t nch = (na + 255) / 256;
    const size_t wbytes = ((size_t)B * nb * na * sizeof(T) + 7) / 8 * 8;
    m->ws_win.ensure(wbytes + (size_t)B * (na + nb + (nch > 1 ? nch * m->n_data : 0)) * sizeof(double));
    T* Win = m->ws_win.as<T>();
    double* lchi = reinterpret_cast<double*>(m->ws_win.as<char>() + wbytes);
    double* norm = lchi + (size_t)B * na;
    double* part = norm + (size_t)B * nb;
    const size_t sm1 = windows_smem(m), sm2 = limber_sum_smem(m, sizeof(T));
    NS_CHECK(sm1 <= 160 * 1024 && sm2 <= 160 * 1024, NS_E_UNSUPPORTED, "Limber stage needs more LDS than a workgroup has");
    {
        TraceScope ts(m, s, "shear_windows");
        // nodes per lane k = ceil(n_a / 64) <= 32, bounded by the kernel's KMAX
        const int k = (na + 63) / 64;
        auto kern = k <= 4 ? shear_windows_kernel<T, 4>
                           : (k <= 8 ? shear_windows_kernel<T, 8>
                                     : (k <= 20 ? shear_windows_kernel<T, 20> : shear_windows_kernel<T, 32>));
        hipLaunchKernelGGL(kern, dim3((unsigned)B), dim3(256), sm1, s, theta, ld, B, G, m->pidx_d.as<int>(),
                           m->pfix_d.as<double>(), m->nz_mean_d.as<double>(), m->agrid_d.as<double>(),
                           m->lna_d.as<double>(), Win, lchi, norm, count);
        NS_HIP(hipGetLastError());
    }
    TraceScope ts(m, s, "limber");
    if (m->z_linear)
        launch_limber_sum<T, true>(m, G, theta, ld, B, Mtab, Win, lchi, norm, Cv, part, count, sm2, s);
    else
        launch_limber_sum<T, false>(m, G, theta, ld, B, Mtab, Win, lchi, norm, Cv, part, count, sm2, s);
}

double* shear_spectra_from_table(ns_model* m, const double* theta, int64_t ld, int64_t B, int prec,
                                 const int* count, hipStream_t s) {
    const int nk = m->n_k, nz = m->n_z;
    const size_t elem = prec == NS_FP64 ? 8 : 4;
    const int n = m->n_data;
    // aux: spline second derivatives [B x nz x nk] (cubic z only) then spectra [B x n] (double)
    const size_t mbytes = m->z_linear ? 0 : (size_t)B * nz * nk * elem;
    const size_t n_ct_max = (n + 63) / 64;
    m->ws_aux.ensure(mbytes + (size_t)B * (n + n_ct_max) * sizeof(double));
    void* Mtab = m->ws_aux.p;
    double* Cv = reinterpret_cast<double*>(m->ws_aux.as<char>() + mbytes);
    const double zmax = 1.0 / m->a_min - 1.0;
    const double hz = zmax / (nz - 1);
    if (!m->shear_attr_set) {   // once per model, outside any stream capture
        const void* fns[] = {(const void*)shear_windows_kernel<double, 4>, (const void*)shear_windows_kernel<float, 4>,
                             (const void*)shear_windows_kernel<double, 8>, (const void*)shear_windows_kernel<float, 8>,
                             (const void*)shear_windows_kernel<double, 20>, (const void*)shear_windows_kernel<float, 20>,
                             (const void*)shear_windows_kernel<double, 32>, (const void*)shear_windows_kernel<float, 32>,
                             (const void*)limber_sum_kernel<double, false, 20>,
                             (const void*)limber_sum_kernel<double, false, 32>,
                             (const void*)limber_sum_kernel<double, true, 20>,
                             (const void*)limber_sum_kernel<double, true, 32>,
                             (const void*)limber_sum_kernel<float, false, 20>,
                             (const void*)limber_sum_kernel<float, false, 32>,
                             (const void*)limber_sum_kernel<float, true, 20>,
                             (const void*)limber_sum_kernel<float, true, 32>};
        for (const void* f : fns)
            NS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_gemm_kernel<0, 64, 32>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dg_smem<64, 32>()));
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_gemm_kernel<1, 64, 32>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dg_smem<64, 32>()));
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_gemm_kernel<0, 32, 64>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dg_smem<32, 64>()));
        NS_HIP(hipFuncSetAttribute((const void*)dense_chi2_gemm_kernel<1, 32, 64>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dg_smem<32, 64>()));
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
        const dim3 gr((unsigned)((nthr + 255) / 256));
        if (prec == NS_FP64) {
            if (nz <= 16)
                hipLaunchKernelGGL((zspline_reg_kernel<double, 16>), gr, dim3(256), 0, s, m->ws_out.as<double>(),
                                   (double*)Mtab, B, nz, nk, hz, count);
            else if (nz <= 64)
                hipLaunchKernelGGL((zspline_reg_kernel<double, 64>), gr, dim3(256), 0, s, m->ws_out.as<double>(),
                                   (double*)Mtab, B, nz, nk, hz, count);
            else
                hipLaunchKernelGGL(zspline_kernel<double>, gz, dim3(64), zsm, s, m->ws_out.as<double>(),
                                   (double*)Mtab, B, nz, nk, hz, count);
        } else {
            if (nz <= 16)
                hipLaunchKernelGGL((zspline_reg_kernel<float, 16>), gr, dim3(256), 0, s, m->ws_out.as<float>(),
                                   (float*)Mtab, B, nz, nk, hz, count);
            else if (nz <= 64)
                hipLaunchKernelGGL((zspline_reg_kernel<float, 64>), gr, dim3(256), 0, s, m->ws_out.as<float>(),
                                   (float*)Mtab, B, nz, nk, hz, count);
            else
                hipLaunchKernelGGL(zspline_kernel<float>, gz, dim3(64), zsm, s, m->ws_out.as<float>(), (float*)Mtab,
                                   B, nz, nk, hz, count);
        }
        NS_HIP(hipGetLastError());
    }
    if (prec == NS_FP64)
        launch_limber<double>(m, theta, ld, B, Mtab, Cv, count, s);
    else
        launch_limber<float>(m, theta, ld, B, Mtab, Cv, count, s);
    return Cv;
}

// One dense chi^2 GEMM launch of mode MODE over B walkers: 64-walker tiles, or
// 32-walker tiles when the 64-walker grid has fewer than eight workgroups per
// CU, with K blocks of 64 when that grid has at most one workgroup per CU
// (identical results; dense_chi2_gemm_kernel)
template <int MODE>
static void launch_dense_gemm(const ns_model* m, const double* C, int64_t B, int n, int np, int n_ct,
                              const double* Lm, const double* wv, double* part, double* R, const int* count,
                              hipStream_t s) {
    const int64_t cus = device_cus(m->device);
    const int64_t g64 = (B + 63) / 64 * n_ct, g32 = (B + 31) / 32 * n_ct;
    const dim3 grid32((unsigned)((B + 31) / 32), (unsigned)n_ct);
    if (g32 <= cus)
        hipLaunchKernelGGL((dense_chi2_gemm_kernel<MODE, 32, 64>), grid32, dim3(256), (dg_smem<32, 64>()), s, C, B, n,
                           np, Lm, wv, part, B, R, count);
    else if (g64 < 8 * cus)
        hipLaunchKernelGGL((dense_chi2_gemm_kernel<MODE, 32, 32>), grid32, dim3(256), (dg_smem<32, 32>()), s, C, B, n,
                           np, Lm, wv, part, B, R, count);
    else
        hipLaunchKernelGGL((dense_chi2_gemm_kernel<MODE, 64, 32>), dim3((unsigned)((B + 63) / 64), (unsigned)n_ct),
                           dim3(256), (dg_smem<64, 32>()), s, C, B, n, np, Lm, wv, part, B, R, count);
}

void shear_loglike_from_table(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl,
                              int prec, const int* count, hipStream_t s) {
    const int n = m->n_data;
    double* Cv = shear_spectra_from_table(m, theta, ld, B, prec, count, s);
    // chi^2 partial sums per 64-column tile: [n_ct x B] after the spectra
    const int np = (n + DG_N - 1) / DG_N * DG_N, n_ct = np / DG_N;
    double* part = Cv + (size_t)B * n;
    {
        TraceScope ts(m, s, "dense_chi2");
        launch_dense_gemm<0>(m, Cv, B, n, np, n_ct, m->cov_lt_pad.as<double>(), m->cov_w.as<double>(), part,
                             (double*)nullptr, count, s);
        NS_HIP(hipGetLastError());
        hipLaunchKernelGGL(dense_chi2_finish_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, theta, ld,
                           B, m->d, m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(), part, B,
                           n_ct, m->logl_const, logl, count);
        NS_HIP(hipGetLastError());
    }
}

// logL and its gradient with respect to the spectra C [B x n] of the dense
// Gaussian: R = w - L^{-1} C (scratch [B x n]), logL from the partial sums
// (part: [n_ct x B] scratch), g_C = L^{-T} R.
void dense_chi2_adjoint(ns_model* m, const double* theta, int64_t ld, int64_t B, const double* Cv, double* R,
                        double* part, double* logl, double* gC, hipStream_t s) {
    const int n = m->n_data;
    const int np = (n + DG_N - 1) / DG_N * DG_N, n_ct = np / DG_N;
    launch_dense_gemm<0>(m, Cv, B, n, np, n_ct, m->cov_lt_pad.as<double>(), m->cov_w.as<double>(), part, R,
                         (const int*)nullptr, s);
    NS_HIP(hipGetLastError());
    hipLaunchKernelGGL(dense_chi2_finish_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, theta, ld, B,
                       m->d, m->prior_kind.as<int>(), m->prior_a.as<double>(), m->prior_b.as<double>(), part, B, n_ct,
                       m->logl_const, logl, (const int*)nullptr);
    NS_HIP(hipGetLastError());
    launch_dense_gemm<1>(m, R, B, n, np, n_ct, m->cov_l_pad.as<double>(), (const double*)nullptr, (double*)nullptr,
                         gC, (const int*)nullptr, s);
    NS_HIP(hipGetLastError());
}

}  // namespace nsmi
