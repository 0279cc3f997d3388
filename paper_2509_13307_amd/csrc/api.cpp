// C ABI of libnsmi (declared in include/ns.h): argument validation, the model
// handle with its host-side FP64 preparation (covariance factorisations,
// grids, spline coefficients, weight conversions), and dispatch to the HIP
// kernels.  No exception crosses the ABI: every entry point maps failures to
// an ns_status and a thread-local message.
#include <cmath>
#include <cstring>
#include <exception>
#include <functional>
#include <string>
#include <vector>

#include "nsmi.h"

namespace nsmi {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void DevBuf::ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        throw Error{NS_E_NOMEM, std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e)};
    }
    bytes = n;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

Net::~Net() {
    for (Layer* l : layers) delete l;
}

static hipEvent_t pool_event(ns_model* m) {
    if (!m->trace_pool.empty()) {
        hipEvent_t e = m->trace_pool.back();
        m->trace_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    NS_HIP(hipEventCreate(&e));
    return e;
}

TraceScope::TraceScope(ns_model* m_, hipStream_t s_, const char* name) : m(m_), s(s_) {
    if (!m->trace || m->noalloc_call) return;
    ns_model::TraceRec r{name, pool_event(m), pool_event(m)};
    NS_HIP(hipEventRecord(r.e0, s));
    m->trace_recs.push_back(r);
    rec = (int)m->trace_recs.size() - 1;
}

TraceScope::~TraceScope() {
    if (rec >= 0) (void)hipEventRecord(m->trace_recs[rec].e1, s);
}

// ------------------------------------------------------------ host FP64 algebra
// Lower Cholesky factor of a symmetric n x n matrix (row-major); false if not SPD.
static bool cholesky(std::vector<double>& A, int n) {
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) s -= A[(size_t)j * n + p] * A[(size_t)j * n + p];
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        const double djj = std::sqrt(s);
        A[(size_t)j * n + j] = djj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) t -= A[(size_t)i * n + p] * A[(size_t)j * n + p];
            A[(size_t)i * n + j] = t / djj;
        }
        for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
    }
    return true;
}

// Inverse of a lower-triangular matrix (row-major) by column forward substitution.
static std::vector<double> lower_inverse(const std::vector<double>& L, int n) {
    std::vector<double> X((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        X[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
        for (int i = c + 1; i < n; ++i) {
            double s = 0.0;
            for (int p = c; p < i; ++p) s += L[(size_t)i * n + p] * X[(size_t)p * n + c];
            X[(size_t)i * n + c] = -s / L[(size_t)i * n + i];
        }
    }
    return X;
}

static void check_ptr(const void* p, const char* what) {
    if (!p) throw Error{NS_E_INVALID, std::string("null pointer: ") + what};
}

static Net* build_net(const ns_net_desc& nd, int mu_rows) {
    NS_CHECK(nd.n_layers >= 2, NS_E_SHAPE, "emulator needs >= 2 layers");
    check_ptr(nd.dims, "net.dims");
    check_ptr(nd.W, "net.W");
    check_ptr(nd.b, "net.b");
    check_ptr(nd.beta, "net.beta");
    check_ptr(nd.gamma, "net.gamma");
    check_ptr(nd.in_shift, "net.in_shift");
    check_ptr(nd.in_scale, "net.in_scale");
    check_ptr(nd.out_mu, "net.out_mu");
    check_ptr(nd.out_sigma, "net.out_sigma");
    Net* net = new Net();
    try {
        net->n_layers = nd.n_layers;
        net->dims.assign(nd.dims, nd.dims + nd.n_layers + 1);
        for (int v : net->dims) NS_CHECK(v >= 1, NS_E_SHAPE, "emulator layer width must be >= 1");
        NS_CHECK(net->dims[0] <= 16, NS_E_UNSUPPORTED, "emulator supports <= 16 inputs");
        for (int l = 1; l < nd.n_layers; ++l)
            NS_CHECK(net->dims[l] % 64 == 0, NS_E_UNSUPPORTED, "hidden widths must be multiples of 64 (MFMA tiles)");
        net->fused = fused_shape(net->dims);
        const int H = net->dims[1];
        const int n_out_net = net->dims.back();
        const size_t fcols = (size_t)(n_out_net + H - 1) / H * H;
        std::vector<bf16_t> fh, fl;
        std::vector<float> fv;
        if (net->fused) {
            fh.assign((size_t)(nd.n_layers - 2) * H * H + fcols * H, 0);
            fl.assign(fh.size(), 0);
            fv.assign((size_t)(nd.n_layers - 2) * 3 * H + n_out_net, 0.0f);
        }
        for (int l = 0; l < nd.n_layers; ++l) {
            Layer* ly = new Layer();
            net->layers.push_back(ly);
            const int K = net->dims[l], N = net->dims[l + 1];
            ly->n_in = K;
            ly->n_out = N;
            ly->hidden = l < nd.n_layers - 1;
            check_ptr(nd.W[l], "net.W[l]");
            check_ptr(nd.b[l], "net.b[l]");
            const size_t nw = (size_t)K * N;
            upload(ly->W64, nd.W[l], nw);
            upload(ly->b64, nd.b[l], (size_t)N);
            std::vector<float> wf(nw), bf(N);
            for (size_t i = 0; i < nw; ++i) wf[i] = (float)nd.W[l][i];
            for (int i = 0; i < N; ++i) bf[i] = (float)nd.b[l][i];
            upload(ly->W32, wf.data(), nw);
            upload(ly->b32, bf.data(), (size_t)N);
            std::vector<bf16_t> hi(nw), lo(nw);
            for (size_t i = 0; i < nw; ++i) {
                hi[i] = host_f2bf(wf[i]);
                lo[i] = host_f2bf(wf[i] - host_bf2f(hi[i]));
            }
            upload(ly->Whi, hi.data(), nw);
            upload(ly->Wlo, lo.data(), nw);
            if (net->fused && l >= 1) {
                // fragment order: block (kc, nt) of 64 lanes x 8 inputs at
                // (kc n_cols / 32 + nt) 512; lane q holds unit 32 nt + q % 32,
                // inputs 16 kc + 8 (q / 32) + i
                const int KC = K / 16;
                const size_t base = (size_t)(l - 1) * H * H;
                const int n_cols = ly->hidden ? H : (int)fcols;
                const int ntl = n_cols / 32;
                for (int nt = 0; nt < n_cols / 32; ++nt)
                    for (int kc = 0; kc < KC; ++kc)
                        for (int q = 0; q < 64; ++q) {
                            const int n = nt * 32 + q % 32;
                            if (n >= N) continue;
                            for (int i = 0; i < 8; ++i) {
                                const size_t src = (size_t)n * K + kc * 16 + 8 * (q / 32) + i;
                                const size_t dst = base + (((size_t)kc * ntl + nt) * 64 + q) * 8 + i;
                                fh[dst] = hi[src];
                                fl[dst] = lo[src];
                            }
                        }
                float* v = fv.data() + (size_t)(l - 1) * 3 * H;
                if (ly->hidden) {
                    check_ptr(nd.beta[l], "net.beta[l]");
                    check_ptr(nd.gamma[l], "net.gamma[l]");
                }
                for (int i = 0; i < N; ++i) {
                    v[i] = bf[i];
                    if (ly->hidden) {
                        v[H + i] = (float)nd.beta[l][i];
                        v[2 * H + i] = (float)nd.gamma[l][i];
                    }
                }
            }
            // transposed, zero-padded copies for the adjoint GEMMs
            ly->n_pad = (N + 63) / 64 * 64;
            std::vector<double> wt((size_t)K * ly->n_pad, 0.0);
            std::vector<float> wtf((size_t)K * ly->n_pad, 0.0f);
            for (int n = 0; n < N; ++n)
                for (int k = 0; k < K; ++k) {
                    wt[(size_t)k * ly->n_pad + n] = nd.W[l][(size_t)n * K + k];
                    wtf[(size_t)k * ly->n_pad + n] = (float)nd.W[l][(size_t)n * K + k];
                }
            upload(ly->WT64, wt.data(), wt.size());
            upload(ly->WT32, wtf.data(), wtf.size());
            if (ly->hidden) {
                check_ptr(nd.beta[l], "net.beta[l]");
                check_ptr(nd.gamma[l], "net.gamma[l]");
                upload(ly->beta64, nd.beta[l], (size_t)N);
                upload(ly->gamma64, nd.gamma[l], (size_t)N);
                std::vector<float> be(N), ga(N);
                for (int i = 0; i < N; ++i) { be[i] = (float)nd.beta[l][i]; ga[i] = (float)nd.gamma[l][i]; }
                upload(ly->beta32, be.data(), (size_t)N);
                upload(ly->gamma32, ga.data(), (size_t)N);
            }
        }
        net->narrow64 = narrow_f64_shape(net->dims);
        if (net->narrow64) {
            std::vector<double> f64;
            for (int l = 1; l < nd.n_layers; ++l) {
                const int K = net->dims[l], N = net->dims[l + 1], NT = (N + 15) / 16, K4 = K / 4;
                const size_t base = f64.size();
                f64.resize(base + (size_t)K4 * NT * 64, 0.0);
                for (int kq = 0; kq < K4; ++kq)
                    for (int nt = 0; nt < NT; ++nt)
                        for (int q = 0; q < 64; ++q) {
                            const int n = nt * 16 + q % 16, k = kq * 4 + q / 16;
                            if (n < N) f64[base + ((size_t)kq * NT + nt) * 64 + q] = nd.W[l][(size_t)n * K + k];
                        }
            }
            upload(net->Wf64, f64.data(), f64.size());
        }
        if (net->fused) {
            upload(net->Wf, fh.data(), fh.size());
            upload(net->Wfl, fl.data(), fl.size());
            upload(net->fvec, fv.data(), fv.size());
        }
        const int n_in = net->dims[0], n_out = net->dims.back();
        upload(net->in_shift, nd.in_shift, (size_t)n_in);
        upload(net->in_scale, nd.in_scale, (size_t)n_in);
        for (int i = 0; i < n_in; ++i) NS_CHECK(nd.in_scale[i] != 0.0, NS_E_INVALID, "in_scale must be non-zero");
        net->out_mu_rows = mu_rows;
        const size_t nmu = (size_t)mu_rows * n_out;
        upload(net->out_mu64, nd.out_mu, nmu);
        upload(net->out_sigma64, nd.out_sigma, (size_t)n_out);
        std::vector<float> muf(nmu), sgf(n_out);
        for (size_t i = 0; i < nmu; ++i) muf[i] = (float)nd.out_mu[i];
        for (int i = 0; i < n_out; ++i) sgf[i] = (float)nd.out_sigma[i];
        upload(net->out_mu32, muf.data(), nmu);
        upload(net->out_sigma32, sgf.data(), (size_t)n_out);
    } catch (...) {
        delete net;
        throw;
    }
    return net;
}

static void build_model(ns_model* m, const ns_model_desc* D) {
    const double LOG2PI = std::log(2.0 * M_PI);
    m->kind = D->kind;
    m->d = D->d;
    NS_CHECK(D->kind >= 0 && D->kind <= 4, NS_E_INVALID, "unknown model kind");
    NS_CHECK(D->d >= 1 && D->d <= 64, NS_E_SHAPE, "d must be in [1, 64]");
    check_ptr(D->prior_kind, "prior_kind");
    check_ptr(D->prior_a, "prior_a");
    check_ptr(D->prior_b, "prior_b");
    for (int i = 0; i < D->d; ++i) {
        NS_CHECK(D->prior_kind[i] == NS_PRIOR_UNIFORM || D->prior_kind[i] == NS_PRIOR_NORMAL, NS_E_INVALID,
                 "prior kind must be uniform or normal");
        if (D->prior_kind[i] == NS_PRIOR_UNIFORM)
            NS_CHECK(D->prior_a[i] < D->prior_b[i], NS_E_INVALID, "uniform prior needs a < b");
        else
            NS_CHECK(D->prior_b[i] > 0.0, NS_E_INVALID, "normal prior needs sigma > 0");
    }
    upload(m->prior_kind, D->prior_kind, (size_t)D->d);
    m->any_normal_prior = false;
    for (int i = 0; i < D->d; ++i) m->any_normal_prior = m->any_normal_prior || D->prior_kind[i] == NS_PRIOR_NORMAL;
    upload(m->prior_a, D->prior_a, (size_t)D->d);
    upload(m->prior_b, D->prior_b, (size_t)D->d);

    if (D->kind == NS_MODEL_GAUSS) {
        check_ptr(D->mu, "mu");
        check_ptr(D->gsigma, "gsigma");
        std::vector<double> is(D->d);
        double c = -0.5 * D->d * LOG2PI;
        for (int i = 0; i < D->d; ++i) {
            NS_CHECK(D->gsigma[i] > 0.0, NS_E_INVALID, "gsigma must be > 0");
            is[i] = 1.0 / D->gsigma[i];
            c -= std::log(D->gsigma[i]);
        }
        upload(m->g_mu, D->mu, (size_t)D->d);
        upload(m->g_isig, is.data(), (size_t)D->d);
        m->logl_const = c;
        return;
    }

    check_ptr(D->nets, "nets");
    check_ptr(D->data, "data");
    const int want_nets = D->kind == NS_MODEL_CMB_BLOCK ? 4 : 1;
    NS_CHECK(D->n_nets == want_nets, NS_E_SHAPE, "wrong number of emulator networks for this model kind");
    const int mu_rows = D->kind == NS_MODEL_SHEAR ? D->n_z : 1;
    NS_CHECK(mu_rows >= 1, NS_E_SHAPE, "n_z must be >= 1");
    for (int i = 0; i < D->n_nets; ++i) m->nets.push_back(build_net(D->nets[i], mu_rows));
    const int n_in = m->nets[0]->dims[0];
    for (auto* n : m->nets) NS_CHECK(n->dims[0] == n_in, NS_E_SHAPE, "networks must share their inputs");
    m->n_data = D->n_data;

    if (D->kind == NS_MODEL_CMB_DIAG || D->kind == NS_MODEL_CMB_BLOCK || D->kind == NS_MODEL_CMB_CV) {
        NS_CHECK(n_in <= D->d, NS_E_SHAPE, "CMB emulator inputs exceed d");
        m->emu_src.resize(n_in);
        for (int i = 0; i < n_in; ++i) m->emu_src[i] = i;
        m->emu_fix.assign(n_in, 0.0);
        check_ptr(D->spec_log, "spec_log");
        m->spec_log.assign(D->spec_log, D->spec_log + D->n_nets);
    }
    if (D->kind == NS_MODEL_CMB_CV) {
        const int n = D->n_data;
        NS_CHECK(n == m->nets[0]->dims.back(), NS_E_SHAPE, "n_data must equal the emulator outputs");
        NS_CHECK(m->spec_log[0] == 1, NS_E_INVALID, "the CMB_CV emulator must output log10 C_l (spec_log 1)");
        NS_CHECK(D->ell_min >= 0.0 && D->ell_min == std::floor(D->ell_min), NS_E_INVALID,
                 "ell_min must be a non-negative integer");
        // log p(Ch | C) = c_l - (k/2)(ln C + Ch/C), k = 2l+1, with
        // c_l = ln k + (k/2 - 1)(ln k + ln Ch) - (k/2) ln 2 - ln Gamma(k/2)
        std::vector<double> hk(n);
        double c = 0.0;
        for (int b = 0; b < n; ++b) {
            NS_CHECK(D->data[b] > 0.0, NS_E_INVALID, "observed spectrum must be > 0");
            const double k = 2.0 * (D->ell_min + b) + 1.0;
            hk[b] = 0.5 * k;
            c += std::log(k) + (0.5 * k - 1.0) * (std::log(k) + std::log(D->data[b])) - 0.5 * k * std::log(2.0) -
                 std::lgamma(0.5 * k);
        }
        upload(m->cv_halfk, hk.data(), hk.size());
        m->logl_const = c;
    } else if (D->kind == NS_MODEL_CMB_DIAG) {
        NS_CHECK(D->n_data == m->nets[0]->dims.back(), NS_E_SHAPE, "n_data must equal the emulator outputs");
        check_ptr(D->sigma, "sigma");
        std::vector<double> is(D->n_data);
        double c = -0.5 * D->n_data * LOG2PI;
        for (int i = 0; i < D->n_data; ++i) {
            NS_CHECK(D->sigma[i] > 0.0, NS_E_NOT_SPD, "sigma must be > 0");
            is[i] = 1.0 / D->sigma[i];
            c -= std::log(D->sigma[i]);
        }
        upload(m->inv_sigma, is.data(), is.size());
        m->logl_const = c;
    } else if (D->kind == NS_MODEL_CMB_BLOCK) {
        const int ne = m->nets[0]->dims.back();
        for (auto* n : m->nets) NS_CHECK(n->dims.back() == ne, NS_E_SHAPE, "all four spectra need n_ell outputs");
        NS_CHECK(D->n_data == 4 * ne, NS_E_SHAPE, "n_data must be 4 n_ell");
        check_ptr(D->cov_blocks, "cov_blocks");
        check_ptr(D->sigma_pp, "sigma_pp");
        m->n_ell_cmb = ne;
        std::vector<double> linv((size_t)ne * 6), isp(ne);
        double c = -0.5 * D->n_data * LOG2PI;
        for (int l = 0; l < ne; ++l) {
            std::vector<double> A(D->cov_blocks + (size_t)l * 9, D->cov_blocks + (size_t)l * 9 + 9);
            NS_CHECK(cholesky(A, 3), NS_E_NOT_SPD, "3x3 covariance block " + std::to_string(l) + " is not SPD");
            std::vector<double> X = lower_inverse(A, 3);
            linv[(size_t)l * 6 + 0] = X[0];
            linv[(size_t)l * 6 + 1] = X[3];
            linv[(size_t)l * 6 + 2] = X[4];
            linv[(size_t)l * 6 + 3] = X[6];
            linv[(size_t)l * 6 + 4] = X[7];
            linv[(size_t)l * 6 + 5] = X[8];
            c -= std::log(A[0]) + std::log(A[4]) + std::log(A[8]);
            NS_CHECK(D->sigma_pp[l] > 0.0, NS_E_NOT_SPD, "sigma_pp must be > 0");
            isp[l] = 1.0 / D->sigma_pp[l];
            c -= std::log(D->sigma_pp[l]);
        }
        upload(m->blk_linv, linv.data(), linv.size());
        upload(m->inv_sigma_pp, isp.data(), isp.size());
        m->logl_const = c;
    } else {
        // cosmic shear
        NS_CHECK(D->n_bins >= 1 && D->n_bins <= 10, NS_E_UNSUPPORTED, "n_bins must be in [1, 10]");
        NS_CHECK(D->z_interp == 0 || D->z_interp == 1, NS_E_INVALID, "z_interp must be 0 (cubic) or 1 (linear)");
        NS_CHECK(D->n_a >= 3 && D->n_a <= 2048, NS_E_UNSUPPORTED, "n_a must be in [3, 2048]");
        if (D->z_interp == 0)
            NS_CHECK(D->n_z >= 4 && D->n_z <= 256, NS_E_UNSUPPORTED, "n_z must be in [4, 256] (not-a-knot spline)");
        else
            NS_CHECK(D->n_z >= 2 && D->n_z <= D->n_a, NS_E_UNSUPPORTED, "n_z must be in [2, n_a] (linear z)");
        NS_CHECK(D->n_k >= 4, NS_E_SHAPE, "n_k must be >= 4");
        NS_CHECK(D->n_ell >= 1 && D->n_ell <= 32, NS_E_UNSUPPORTED, "n_ell must be in [1, 32]");
        NS_CHECK(D->a_min > 0.0 && D->a_min < 1.0, NS_E_INVALID, "a_min must be in (0, 1)");
        NS_CHECK(D->k_min > 0.0 && D->k_max > D->k_min, NS_E_INVALID, "need 0 < k_min < k_max");
        NS_CHECK(D->ell_min > 0.0 && D->ell_max >= D->ell_min, NS_E_INVALID, "need 0 < ell_min <= ell_max");
        NS_CHECK(D->nz_sigma > 0.0, NS_E_INVALID, "nz_sigma must be > 0");
        check_ptr(D->nz_mean, "nz_mean");
        check_ptr(D->pidx, "pidx");
        check_ptr(D->pfix, "pfix");
        check_ptr(D->cov, "cov");
        const int nb = D->n_bins;
        m->n_bins = nb; m->n_a = D->n_a; m->n_z = D->n_z; m->n_k = D->n_k; m->n_ell = D->n_ell;
        m->n_pairs = nb * (nb + 1) / 2;
        m->nz_sigma = D->nz_sigma; m->a_min = D->a_min; m->k_min = D->k_min; m->k_max = D->k_max;
        NS_CHECK(D->n_data == m->n_pairs * D->n_ell, NS_E_SHAPE, "n_data must be n_pairs * n_ell");
        NS_CHECK(D->n_data <= 1248, NS_E_UNSUPPORTED, "shear data vector longer than 1248");
        m->z_linear = D->z_interp == 1;
        NS_CHECK(n_in == 8, NS_E_SHAPE, "shear emulator takes 8 inputs");
        NS_CHECK(m->nets[0]->dims.back() == D->n_k, NS_E_SHAPE, "shear emulator must output n_k values");
        const int nphys = 9 + 3 * nb;
        m->pidx.assign(D->pidx, D->pidx + nphys);
        m->pfix.assign(D->pfix, D->pfix + nphys);
        for (int s = 0; s < nphys; ++s) NS_CHECK(m->pidx[s] >= -1 && m->pidx[s] < D->d, NS_E_SHAPE, "pidx out of range");
        upload(m->pidx_d, m->pidx.data(), m->pidx.size());
        upload(m->pfix_d, m->pfix.data(), m->pfix.size());
        upload(m->nz_mean_d, D->nz_mean, (size_t)nb);
        // emulator inputs: omega_b, omega_cdm, h, n_s, lnAs, c_min, eta0, z
        const int slots[7] = {0, 1, 2, 3, 4, 7, 8};
        m->emu_src.resize(8);
        m->emu_fix.assign(8, 0.0);
        for (int i = 0; i < 7; ++i) {
            m->emu_src[i] = m->pidx[slots[i]] >= 0 ? m->pidx[slots[i]] : SRC_FIXED;
            m->emu_fix[i] = m->pfix[slots[i]];
        }
        m->emu_src[7] = SRC_ZNODE;
        // grids
        const int na = D->n_a, nz = D->n_z;
        std::vector<double> a(na);
        const double step = (D->a_min - 1.0) / (na - 1);
        for (int j = 0; j < na; ++j) a[j] = 1.0 + j * step;
        a[na - 1] = D->a_min;
        upload(m->agrid_d, a.data(), a.size());
        std::vector<double> la(2 * (size_t)na, 0.0);
        for (int j = 0; j < na; ++j) la[j] = std::log(a[j]);
        for (int j = 0; j + 1 < na; ++j) la[na + j] = std::log(0.5 * (a[j] + a[j + 1]));
        upload(m->lna_d, la.data(), la.size());
        const double zmax = 1.0 / D->a_min - 1.0;
        const double hz = zmax / (nz - 1);
        std::vector<double> zn(nz);
        std::vector<int> zi(na);
        std::vector<double> zc((size_t)na * 4, 0.0);
        if (m->z_linear) {
            // nodes at scale factors evenly spaced from 1 to a_min, computed like
            // the a-grid (with n_z = n_a they are its nodes); linear weights in z
            std::vector<double> an(nz);
            const double stz = (D->a_min - 1.0) / (nz - 1);
            for (int n = 0; n < nz; ++n) an[n] = 1.0 + n * stz;
            an[nz - 1] = D->a_min;
            for (int n = 0; n < nz; ++n) zn[n] = 1.0 / an[n] - 1.0;
            int n = 0;
            for (int j = 0; j < na; ++j) {
                const double z = std::min(1.0 / a[j] - 1.0, zn[nz - 1]);
                while (n < nz - 2 && zn[n + 1] <= z) ++n;
                double t = (z - zn[n]) / (zn[n + 1] - zn[n]);
                t = std::min(1.0, std::max(0.0, t));
                zi[j] = n;
                zc[4 * j + 0] = 1.0 - t;
                zc[4 * j + 1] = t;
            }
        } else {
            for (int n = 0; n < nz; ++n) zn[n] = n * hz;
            zn[nz - 1] = zmax;
            for (int j = 0; j < na; ++j) {
                const double z = std::min(1.0 / a[j] - 1.0, zmax);
                int n = (int)std::floor(z / hz);
                n = std::max(0, std::min(n, nz - 2));
                const double t = (z - zn[n]) / hz, u = 1.0 - t;
                zi[j] = n;
                zc[4 * j + 0] = u;
                zc[4 * j + 1] = t;
                zc[4 * j + 2] = hz * hz / 6.0 * (u * u * u - u);
                zc[4 * j + 3] = hz * hz / 6.0 * (t * t * t - t);
            }
        }
        upload(m->znodes_d, zn.data(), zn.size());
        upload(m->zsp_idx_d, zi.data(), zi.size());
        upload(m->zsp_coef_d, zc.data(), zc.size());
        // Slabs of the Limber adjoint's scatter: the z rows cut into runs of at
        // most lslab_rows rows, the rows of the gradient tables one workgroup
        // holds in LDS (64 KiB; at least the two rows of one node), each with
        // the nodes (1 .. n_a - 1) whose rows zi[j], zi[j] + 1 meet it.  The
        // nodes' z only grows along the a-grid, so those nodes are a run.
        {
            const int tables = m->z_linear ? 1 : 2;
            const size_t row_bytes = (size_t)tables * D->n_k * sizeof(unsigned long long);
            const int rmax = std::max(2, (int)((64 * 1024) / row_bytes));
            for (int j = 2; j < na; ++j)
                NS_CHECK(zi[j] >= zi[j - 1], NS_E_INVALID, "z-spline intervals not monotone along the a-grid");
            std::vector<int> sl;
            int j0 = 1;
            for (int lo = 0; lo < nz; lo += rmax) {
                const int hi = std::min(nz - 1, lo + rmax - 1);
                while (j0 < na && zi[j0] + 1 < lo) ++j0;
                int j1 = j0;
                while (j1 < na && zi[j1] <= hi) ++j1;
                sl.insert(sl.end(), {j0, j1, lo, hi});
            }
            m->n_lslab = (int)(sl.size() / 4);
            m->lslab_rows = rmax;
            upload(m->lslab_d, sl.data(), sl.size());
        }
        std::vector<double> ell(D->n_ell);
        const double l0 = std::log10(D->ell_min), l1 = std::log10(D->ell_max);
        for (int b = 0; b < D->n_ell; ++b)
            ell[b] = std::pow(10.0, D->n_ell > 1 ? l0 + b * (l1 - l0) / (D->n_ell - 1) : l0);
        upload(m->ell_d, ell.data(), ell.size());
        std::vector<double> lell(D->n_ell);
        for (int b = 0; b < D->n_ell; ++b) lell[b] = std::log10(ell[b] + 0.5);
        upload(m->lell_d, lell.data(), lell.size());
        // dense covariance: L^{-1} and the whitened data
        const int n = D->n_data;
        std::vector<double> A(D->cov, D->cov + (size_t)n * n);
        NS_CHECK(cholesky(A, n), NS_E_NOT_SPD, "covariance is not SPD");
        std::vector<double> X = lower_inverse(A, n);
        std::vector<double> w(n, 0.0);
        double c = -0.5 * n * LOG2PI;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int p = 0; p <= i; ++p) s += X[(size_t)i * n + p] * D->data[p];
            w[i] = s;
            c -= std::log(A[(size_t)i * n + i]);
        }
        upload(m->cov_linv, X.data(), X.size());
        std::vector<double> XT((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) XT[(size_t)k * n + i] = X[(size_t)i * n + k];
        upload(m->cov_linvT, XT.data(), XT.size());
        const int np = (n + 63) / 64 * 64;
        std::vector<double> LP((size_t)np * np, 0.0);
        for (int k = 0; k < n; ++k)
            for (int i = 0; i < n; ++i) LP[(size_t)k * np + i] = X[(size_t)i * n + k];
        upload(m->cov_lt_pad, LP.data(), LP.size());
        std::fill(LP.begin(), LP.end(), 0.0);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) LP[(size_t)i * np + k] = X[(size_t)i * n + k];
        upload(m->cov_l_pad, LP.data(), LP.size());
        upload(m->cov_w, w.data(), w.size());
        m->logl_const = c;
    }
    upload(m->data, D->data, (size_t)D->n_data);
    upload(m->emu_src_d, m->emu_src.data(), m->emu_src.size());
    upload(m->emu_fix_d, m->emu_fix.data(), m->emu_fix.size());
    if (!m->znodes_d.p) {
        double z0 = 0.0;
        upload(m->znodes_d, &z0, 1);
    }
}

static int guard(const std::function<void()>& f) {
    try {
        f();
        g_last_error.clear();
        return NS_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return NS_E_NOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return NS_E_INVALID;
    } catch (...) {
        g_last_error = "unknown failure";
        return NS_E_INVALID;
    }
}

static void bind_device(const ns_model* m) {
    NS_HIP(hipSetDevice(m->device));
}

static void check_prec(int p) {
    NS_CHECK(p >= NS_FP64 && p <= NS_BF16X3, NS_E_INVALID, "unknown precision");
}

}  // namespace nsmi

ns_model::~ns_model() {
    for (auto* n : nets) delete n;
    for (auto& r : trace_recs) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    for (auto e : trace_pool) (void)hipEventDestroy(e);
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    if (graph_event) (void)hipEventDestroy(graph_event);
}

using namespace nsmi;

extern "C" {

ns_status ns_model_create(const ns_model_desc* desc, int32_t device, ns_model** out) {
    return (ns_status)guard([&] {
        check_ptr(desc, "desc");
        check_ptr(out, "out");
        *out = nullptr;
        int n = 0;
        NS_HIP(hipGetDeviceCount(&n));
        NS_CHECK(device >= 0 && device < n, NS_E_INVALID, "no such HIP device");
        NS_HIP(hipSetDevice(device));
        scratch_init(device);                   // address of the allocation-free path's array on this device
        ns_model* m = new ns_model();
        m->device = device;
        try {
            tune_cache_load(m);                 // launch shapes measured before on this GPU architecture
            build_model(m, desc);
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

ns_status ns_model_free(ns_model* model) {
    return (ns_status)guard([&] {
        if (!model) return;
        NS_HIP(hipSetDevice(model->device));
        NS_HIP(hipDeviceSynchronize());
        delete model;
    });
}

ns_status ns_model_dim(const ns_model* model, int32_t* d) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_ptr(d, "d");
        *d = model->d;
    });
}

ns_status ns_prior_transform(ns_model* model, const double* u, double* theta, int64_t ld, int64_t B,
                             void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        NS_CHECK(B >= 0, NS_E_SHAPE, "B must be >= 0");
        NS_CHECK(ld >= model->d, NS_E_SHAPE, "ld must be >= d");
        if (B == 0) return;
        check_ptr(u, "u");
        check_ptr(theta, "theta");
        bind_device(model);
        prior_transform(model, u, theta, ld, B, nullptr, (hipStream_t)stream);
    });
}

ns_status ns_loglike_batch(ns_model* model, const double* theta, int64_t ld, int64_t B, double* logl,
                           int32_t precision, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_prec(precision);
        NS_CHECK(B >= 0, NS_E_SHAPE, "B must be >= 0");
        NS_CHECK(ld >= model->d, NS_E_SHAPE, "ld must be >= d");
        NS_CHECK(B <= (int64_t)1 << 26, NS_E_SHAPE, "B too large");
        if (B == 0) return;
        check_ptr(theta, "theta");
        check_ptr(logl, "logl");
        bind_device(model);
        loglike_batch(model, theta, ld, B, logl, precision, nullptr, (hipStream_t)stream);
    });
}

ns_status ns_theory_batch(ns_model* model, const double* theta, int64_t ld, int64_t B, double* out, int64_t ldo,
                          int32_t precision, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_prec(precision);
        NS_CHECK(B >= 0, NS_E_SHAPE, "B must be >= 0");
        NS_CHECK(ld >= model->d, NS_E_SHAPE, "ld must be >= d");
        NS_CHECK(B <= (int64_t)1 << 24, NS_E_SHAPE, "B too large");
        NS_CHECK(model->kind != NS_MODEL_GAUSS, NS_E_UNSUPPORTED, "the Gaussian test model has no theory vector");
        NS_CHECK(ldo >= model->n_data, NS_E_SHAPE, "ldo must be >= n_data");
        if (B == 0) return;
        check_ptr(theta, "theta");
        check_ptr(out, "out");
        bind_device(model);
        theory_batch(model, theta, ld, B, out, ldo, precision, (hipStream_t)stream);
    });
}

ns_status ns_loglike_batch_noalloc(ns_model* model, const double* theta, int64_t ld, int64_t B, double* logl,
                                   int32_t precision, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_prec(precision);
        NS_CHECK(B >= 0 && ld >= model->d, NS_E_SHAPE, "B must be >= 0 and ld >= d");
        if (B > 0) {
            check_ptr(theta, "theta");
            check_ptr(logl, "logl");
        }
        bind_device(model);
        loglike_batch_noalloc(model, theta, ld, B, logl, precision, (hipStream_t)stream);
    });
}

ns_status ns_loglike_grad_batch(ns_model* model, const double* theta, int64_t ld, int64_t B, double* logl,
                                double* grad, int32_t precision, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_prec(precision);
        NS_CHECK(B >= 0, NS_E_SHAPE, "B must be >= 0");
        NS_CHECK(ld >= model->d, NS_E_SHAPE, "ld must be >= d");
        NS_CHECK(B <= (int64_t)1 << 24, NS_E_SHAPE, "B too large");
        if (B == 0) return;
        check_ptr(theta, "theta");
        check_ptr(logl, "logl");
        check_ptr(grad, "grad");
        bind_device(model);
        loglike_grad_batch(model, theta, ld, B, logl, grad, precision, (hipStream_t)stream);
    });
}

ns_status ns_slice_step(ns_model* model, double* u, double* logl, int32_t* n_evals, int32_t* n_stalls, int64_t k,
                        double logl_star, const double* dir_chol, int32_t n_inner, uint64_t seed, uint64_t iter,
                        int32_t precision, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_prec(precision);
        NS_CHECK(k >= 0 && k <= (1 << 24), NS_E_SHAPE, "k must be in [0, 2^24]");
        NS_CHECK(n_inner >= 0, NS_E_INVALID, "n_inner must be >= 0");
        if (k == 0 || n_inner == 0) return;
        check_ptr(u, "u");
        check_ptr(logl, "logl");
        check_ptr(n_evals, "n_evals");
        check_ptr(n_stalls, "n_stalls");
        check_ptr(dir_chol, "dir_chol");
        bind_device(model);
        slice_step_host_lstar(model, u, logl, n_evals, n_stalls, k, logl_star, dir_chol, n_inner, seed, iter,
                              precision, (hipStream_t)stream);
    });
}

ns_status ns_run(ns_model* model, const ns_run_opts* opts, ns_run_result* result, double* dead_logl,
                 int32_t* dead_n, double* dead_u, int64_t capacity, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_ptr(opts, "opts");
        check_ptr(result, "result");
        check_prec(opts->precision);
        NS_CHECK(capacity >= 0, NS_E_SHAPE, "capacity must be >= 0");
        bind_device(model);
        run(model, opts, result, dead_logl, dead_n, dead_u, capacity, (hipStream_t)stream);
    });
}

ns_status ns_hmc(ns_model* model, const ns_hmc_opts* opts, const double* inv_mass, double* theta,
                 double* samples, double* logp, ns_hmc_result* result, void* stream) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_ptr(opts, "opts");
        check_ptr(result, "result");
        check_prec(opts->precision);
        NS_CHECK(opts->n_chains >= 1 && opts->n_chains <= (1 << 20), NS_E_SHAPE, "n_chains must be in [1, 2^20]");
        NS_CHECK(opts->n_iter >= 0, NS_E_SHAPE, "n_iter must be >= 0");
        NS_CHECK(opts->n_leapfrog >= 1, NS_E_SHAPE, "n_leapfrog must be >= 1");
        NS_CHECK(opts->step > 0.0 && std::isfinite(opts->step), NS_E_INVALID, "step must be positive and finite");
        check_ptr(inv_mass, "inv_mass");
        check_ptr(theta, "theta");
        bind_device(model);
        hmc_run(model, opts, inv_mass, theta, samples, logp, result, (hipStream_t)stream);
    });
}

ns_status ns_trace_enable(ns_model* model, int32_t enable) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        bind_device(model);
        NS_HIP(hipDeviceSynchronize());
        for (auto& r : model->trace_recs) {
            model->trace_pool.push_back(r.e0);
            model->trace_pool.push_back(r.e1);
        }
        model->trace_recs.clear();
        model->trace = enable != 0;
    });
}

ns_status ns_trace_report(ns_model* model, char* buf, int64_t buf_len) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_ptr(buf, "buf");
        NS_CHECK(buf_len > 0, NS_E_SHAPE, "buf_len must be > 0");
        bind_device(model);
        NS_HIP(hipDeviceSynchronize());
        std::vector<std::string> names;
        std::vector<double> tot;
        std::vector<long> cnt;
        for (auto& r : model->trace_recs) {
            float ms = 0.f;
            NS_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
            size_t i = 0;
            while (i < names.size() && names[i] != r.name) ++i;
            if (i == names.size()) { names.push_back(r.name); tot.push_back(0.0); cnt.push_back(0); }
            tot[i] += ms;
            cnt[i] += 1;
            model->trace_pool.push_back(r.e0);
            model->trace_pool.push_back(r.e1);
        }
        model->trace_recs.clear();
        std::string js = "{";
        for (size_t i = 0; i < names.size(); ++i) {
            char tmp[256];
            snprintf(tmp, sizeof tmp, "%s\"%s\": [%ld, %.9g]", i ? ", " : "", names[i].c_str(), cnt[i], tot[i]);
            js += tmp;
        }
        js += "}";
        NS_CHECK((int64_t)js.size() < buf_len, NS_E_SHAPE, "trace report buffer too small");
        memcpy(buf, js.c_str(), js.size() + 1);
    });
}

ns_status ns_tuning_report(ns_model* model, char* buf, int64_t buf_len) {
    return (ns_status)guard([&] {
        check_ptr(model, "model");
        check_ptr(buf, "buf");
        const std::string js = bf16_tuning_report(model);
        NS_CHECK((int64_t)js.size() < buf_len, NS_E_SHAPE, "tuning report buffer too small");
        memcpy(buf, js.c_str(), js.size() + 1);
    });
}

const char* ns_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
