// Internal declarations of libnsmi: the model handle, workspaces and the
// kernel launchers shared by the translation units.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <bitset>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ns.h"

namespace nsmi {

// ----------------------------------------------------------------- errors
struct Error {
    ns_status code;
    std::string msg;
};
void set_error(const std::string& msg);

#define NS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::nsmi::Error{NS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define NS_CHECK(cond, code, text)                                                     \
    do {                                                                               \
        if (!(cond)) throw ::nsmi::Error{code, text};                                  \
    } while (0)

// --------------------------------------------------------- device buffers
// Owning device allocation; grows on demand (contents are not preserved).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void ensure(size_t n);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

template <class T>
T* upload(DevBuf& buf, const T* host, size_t n) {
    buf.ensure(n * sizeof(T));
    if (n) NS_HIP(hipMemcpy(buf.p, host, n * sizeof(T), hipMemcpyHostToDevice));
    return buf.as<T>();
}

// BF16 storage (round to nearest even from FP32)
typedef uint16_t bf16_t;
inline bf16_t host_f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
inline float host_bf2f(bf16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// ----------------------------------------------------------- emulator
// One layer's parameters in every storage form the kernels use.
struct Layer {
    int n_in = 0, n_out = 0;
    bool hidden = false;
    DevBuf W64, b64, beta64, gamma64;        // double
    DevBuf W32, b32, beta32, gamma32;        // float
    DevBuf Whi, Wlo;                         // bf16 hi / lo split of W
    int n_pad = 0;                           // n_out rounded up to 64
    DevBuf WT64, WT32;                       // W^T [n_in x n_pad], zero padded (adjoint)
};

struct Net {
    int n_layers = 0;
    std::vector<int> dims;
    std::vector<Layer*> layers;
    DevBuf in_shift, in_scale;               // double [dims[0]]
    DevBuf out_mu64, out_sigma64;            // double
    DevBuf out_mu32, out_sigma32;            // float
    int out_mu_rows = 1;                     // 1 (CMB) or n_z (shear)
    // One-kernel BF16 forward (networks that pass fused_shape): BF16 hi / lo
    // weights of GEMM layers 2..L in MFMA fragment order, one 1 KB block per
    // (16 inputs kc, 32 units nt) at (kc n_tiles + nt) 512 elements within the
    // layer, layer l (0-based) at element l H^2, output units zero padded to a
    // multiple of H; fvec holds b, beta, gamma of each hidden
    // GEMM layer (3H floats each) followed by the output bias.
    bool fused = false;
    DevBuf Wf, Wfl, fvec;
    // One-kernel FP64 forward (networks that pass narrow_f64_shape): weights
    // of GEMM layers 2..L in v_mfma_f64_16x16x4f64 fragment order, layer after
    // layer; block (kq, nt) of a layer with NT = ceil(N / 16) column tiles at
    // (kq NT + nt) 64, lane q holding W[16 nt + q % 16][4 kq + q / 16] (0 past N)
    bool narrow64 = false;
    DevBuf Wf64;
    ~Net();
};

// Emulator input source per input column: >= 0 theta column, -1 fixed value,
// -2 redshift node of the row.
enum { SRC_FIXED = -1, SRC_ZNODE = -2 };

}  // namespace nsmi

// ------------------------------------------------------------ model handle
struct ns_model {
    int kind = 0, d = 0, device = 0;
    nsmi::DevBuf prior_kind, prior_a, prior_b;
    bool any_normal_prior = false;   // some parameter has a normal prior (its map needs erfinv)
    std::vector<nsmi::Net*> nets;
    std::vector<int> spec_log;
    int n_data = 0;
    nsmi::DevBuf data;

    // emulator input mapping (length dims[0] of the first net)
    std::vector<int> emu_src;
    std::vector<double> emu_fix;
    nsmi::DevBuf emu_src_d, emu_fix_d, znodes_d;

    // CMB
    nsmi::DevBuf inv_sigma;          // diag: 1/sigma [n]
    nsmi::DevBuf blk_linv;           // block: [n_ell x 6] lower inverse (00,10,11,20,21,22)
    nsmi::DevBuf inv_sigma_pp;       // block: [n_ell]
    int n_ell_cmb = 0;
    double logl_const = 0.0;         // -sum log diag(L) - n/2 log 2pi
    nsmi::DevBuf cv_halfk;           // CMB_CV: (2l+1)/2 per multipole [n]

    // shear
    int n_bins = 0, n_a = 0, n_z = 0, n_k = 0, n_ell = 0, n_pairs = 0;
    double nz_sigma = 0.1, a_min = 0, k_min = 0, k_max = 0;
    std::vector<int> pidx;
    std::vector<double> pfix;
    nsmi::DevBuf pidx_d, pfix_d, nz_mean_d;
    nsmi::DevBuf agrid_d;            // a_j [n_a]
    nsmi::DevBuf lna_d;              // ln a_j [n_a], then ln of the interval midpoints [n_a - 1]
    nsmi::DevBuf zsp_idx_d;          // int [n_a]: spline interval of z_j
    nsmi::DevBuf lslab_d;            // int4 [n_lslab]: Limber-adjoint scatter slabs (first node, end node, first row, last row)
    int n_lslab = 0, lslab_rows = 0; // slab count, z rows held in LDS per slab
    nsmi::DevBuf zsp_coef_d;         // double [n_a x 4]: (1-t, t, h^2/6((1-t)^3-(1-t)), h^2/6(t^3-t));
                                     // linear z: (1-t, t, 0, 0)
    nsmi::DevBuf ws_win;             // shear windows [B][nb][n_a] (form type), log10 chi, n(z) normalisations
    bool z_linear = false;           // linear z-interpolation on nodes evenly spaced in a
    nsmi::DevBuf ell_d;              // double [n_ell]
    nsmi::DevBuf lell_d;             // double [n_ell]: log10(l + 1/2)
    nsmi::DevBuf cov_linv;           // double [n x n] lower-triangular inverse Cholesky factor
    nsmi::DevBuf cov_linvT;          // its transpose (row k holds column k), for the adjoint
    nsmi::DevBuf cov_lt_pad;         // L^{-T} row-major [np x np], np = n rounded up to 64, zero padded
    nsmi::DevBuf cov_l_pad;          // L^{-1} row-major [np x np], zero padded (chi^2 adjoint)
    nsmi::DevBuf cov_w;              // double [n]: L^{-1} d

    // GAUSS
    nsmi::DevBuf g_mu, g_isig;

    // workspaces (grow on demand)
    nsmi::DevBuf ws_act[2];          // hidden activations ping-pong
    nsmi::DevBuf ws_out;             // emulator outputs / model vectors
    nsmi::DevBuf ws_aux;             // stage outputs (spline M, spectra, ...)
    nsmi::DevBuf ws_theta;           // theta scratch for the sampler
    nsmi::DevBuf ws_logl;            // logL scratch for the sampler
    nsmi::DevBuf ws_slice;           // slice-sampler state
    nsmi::DevBuf ws_flag;            // small device counters/flags
    nsmi::DevBuf ws_grad;            // adjoint scratch
    nsmi::DevBuf ws_tsave;           // saved pre-activations [G x (L-1) x rows x width]
    nsmi::DevBuf ws_gact[2];         // adjoint activations ping-pong [G x rows x n_pad]
    nsmi::DevBuf ws_gx;              // input gradients [G x rows x n_in]
    nsmi::DevBuf ws_hmc;             // HMC chain state
    nsmi::DevBuf ws_chi;             // chi^2 tile partials of the one-kernel emulator [blocks x tiles x B]
    hipStream_t graph_stream = nullptr;  // stream the captured sampler graphs replay on
    hipEvent_t graph_event = nullptr;
    bool shear_attr_set = false;     // hipFuncSetAttribute done for the Limber kernels
    std::bitset<192> fused_attr_set;  // ... and per instance of the one-kernel emulator
    // BF16 tile / fused launch-shape choice per (kind, M, N, K, networks), measured at first use
    // or read from the on-disk cache (tune_path, entries of this GPU architecture only)
    std::map<std::tuple<int, int64_t, int, int, int>, int> tune;
    std::string arch;                // gcnArchName of the model's device
    std::string tune_path;           // on-disk tuning cache ("" when off)

    // per-kernel tracing: HIP events bracketing each launch on its stream
    bool trace = false;
    bool noalloc_call = false;       // inside ns_loglike_batch_noalloc: no tuning runs, no trace events
    struct TraceRec { const char* name; hipEvent_t e0, e1; };
    std::vector<TraceRec> trace_recs;
    std::vector<hipEvent_t> trace_pool;

    ~ns_model();
};

namespace nsmi {

// Records a HIP event pair around the launches in its scope when the model's
// tracing is on (see ns_trace_enable).
struct TraceScope {
    ns_model* m;
    hipStream_t s;
    int rec = -1;
    TraceScope(ns_model* m_, hipStream_t s_, const char* name);
    ~TraceScope();
};

// ---------------------------------------------------------- launchers
// Emulator: outputs of net `ni` for `rows` rows (rows = B, or B * n_z for shear).
// theta [B x ld] device; `count` optional device row count (rows beyond it skipped).
// Output written to `out` ([rows x ldo], double for NS_FP64 else float);
// is_log applies 10^y after the output transform.
// `nets` lists G <= 4 networks of identical shape that run in one grid; outs[g]
// and is_log[g] belong to nets[g].
// save_t keeps every hidden pre-activation in m->ws_tsave for the adjoint.
void emulator_forward(ns_model* m, const int* nets, int G, const double* theta, int64_t ld, int64_t B,
                      void* const* outs, int64_t ldo, const int* is_log, int prec, const int* count,
                      hipStream_t s, bool save_t = false);

// Network shapes the one-kernel BF16-operand forward supports: 3..8 layers,
// <= 16 inputs, every hidden width equal to 128 or 512.
bool fused_shape(const std::vector<int>& dims);
// Whole-network forward in one kernel for NS_BF16 / NS_BF16X3 (activations
// resident in LDS); returns false without launching when the form or the
// network shape does not fit it.
bool emulator_forward_fused(ns_model* m, const int* nets, int G, const double* theta, int64_t ld, int64_t B,
                            void* const* outs, int64_t ldo, const int* is_log, int prec, const int* count,
                            hipStream_t s);
// Emulator and chi^2 in one launch for the one-network CMB kinds (diagonal
// Gaussian, cosmic-variance TT) in the BF16-operand forms: logL [B] written;
// false (nothing launched) for other models or forms, or with
// NSMI_NO_FUSED_CHI2 or NSMI_NO_FUSED_MLP set.  `part` (chi2_fused_part_bytes)
// holds the tile partials of the launch shapes that split the output blocks;
// nullptr: the model's workspace.
bool emulator_chi2_fused(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, int prec,
                         const int* count, hipStream_t s, double* part = nullptr);
size_t chi2_fused_part_bytes(const ns_model* m, int64_t B);

// Adjoint of the emulator: from delta_out[g] ([rows x n_pad] FP64 for NS_FP64
// else FP32; derivative of logL w.r.t. the raw network outputs) back to the
// per-network, per-row input gradients gx [G x rows x n_in] (w.r.t. the
// un-normalised inputs).  Requires a preceding forward with save_t.
void emulator_backward(ns_model* m, const int* nets, int G, int64_t B, int prec, hipStream_t s);

// Batched log-likelihood and its gradient (hand-written adjoint).
void loglike_grad_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, double* grad,
                        int prec, hipStream_t s);
void shear_grad(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, double* grad, int prec,
                hipStream_t s);
// grad = direct (optional) + emulator input gradients in m->ws_gx mapped to theta; 0 where logl = -inf.
void grad_assemble(ns_model* m, int64_t B, int G, int rpw, const double* direct, const double* logl, double* grad,
                   hipStream_t s);

// CMB model vector layout of the batched likelihood: spectrum g of walker b at
// element b cmb_row_stride + g cmb_spec_stride (lengths rounded up to 32).
int64_t cmb_spec_stride(const ns_model* m);
int64_t cmb_row_stride(const ns_model* m);

// CMB chi^2 on model vectors (double or float per prec, the layout above) ->
// logL, with support mask.
void cmb_chi2(ns_model* m, const double* theta, int64_t ld, int64_t B, const void* mvec,
              double* logl, int prec, const int* count, hipStream_t s);

// Shear likelihood stages after the emulator table is in m->ws_out.
void dense_chi2_adjoint(ns_model* m, const double* theta, int64_t ld, int64_t B, const double* Cv, double* R,
                        double* part, double* logl, double* gC, hipStream_t s);
void shear_loglike_from_table(ns_model* m, const double* theta, int64_t ld, int64_t B,
                              double* logl, int prec, const int* count, hipStream_t s);
// The spectra C [B x n_data] (double, in m->ws_aux) without the chi^2.
double* shear_spectra_from_table(ns_model* m, const double* theta, int64_t ld, int64_t B, int prec,
                                 const int* count, hipStream_t s);

void gauss_loglike(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl,
                   const int* count, hipStream_t s);

// Full batched likelihood (dispatch by kind).
void loglike_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl,
                   int prec, const int* count, hipStream_t s);

// Theory vector of every walker, in data order, as double: out [B x ldo].
void theory_batch(ns_model* m, const double* theta, int64_t ld, int64_t B, double* out, int64_t ldo,
                  int prec, hipStream_t s);

void prior_transform(ns_model* m, const double* u, double* theta, int64_t ld, int64_t B,
                     const int* count, hipStream_t s);

// Parameter from its unit-cube coordinate x (the priors of Table 1): uniform
// on [a, b], or normal with mean a and standard deviation b.  Shared by the
// prior-transform kernel and the slice sampler, which maps its proposals as
// it writes them.
__device__ __forceinline__ double prior_map(double x, int kind, double a, double b) {
    return kind == NS_PRIOR_UNIFORM ? a + (b - a) * x : a + b * 1.4142135623730950488 * erfinv(2.0 * x - 1.0);
}

// theta outside a uniform prior's [a, b] -> false (NaN compares false: kept)
__device__ __forceinline__ bool in_support(const double* th, int d, const int* kind, const double* a,
                                           const double* b) {
    // parameters in groups of 8, every load of a group unconditional (places
    // past d repeat the last parameter, whose test is idempotent) and the
    // tests combined without short circuits: a group's loads are in flight
    // together instead of one parameter's after another's
    bool ok = true;
    for (int i0 = 0; i0 < d; i0 += 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = min(i0 + j, d - 1);
            const int k = kind[i];
            const double t = th[i], lo = a[i], hi = b[i];
            ok = ok & !((k == NS_PRIOR_UNIFORM) & ((t < lo) | (t > hi)));
        }
    }
    return ok;
}

// in_support in two halves, for a check whose loads should be in flight
// while other work runs: support_load issues the loads of the first eight
// parameters (places past d repeat the last one), support_test forms the
// same result from them and the remaining parameters.
struct SupportLoads {
    double t[8], lo[8], hi[8];
    int k[8];
};
__device__ __forceinline__ void support_load(SupportLoads& s, const double* th, int d, const int* kind,
                                             const double* a, const double* b) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = min(j, d - 1);
        s.k[j] = kind[i];
        s.t[j] = th[i];
        s.lo[j] = a[i];
        s.hi[j] = b[i];
    }
}
__device__ __forceinline__ bool support_test(const SupportLoads& s, const double* th, int d, const int* kind,
                                             const double* a, const double* b) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 8; ++j) ok = ok & !((s.k[j] == NS_PRIOR_UNIFORM) & ((s.t[j] < s.lo[j]) | (s.t[j] > s.hi[j])));
    return d > 8 ? ok & in_support(th + 8, d - 8, kind + 8, a + 8, b + 8) : ok;
}

// Networks the one-kernel FP64 forward supports: 3..8 layers, <= 16 inputs,
// every hidden width 128, <= 256 outputs.
bool narrow_f64_shape(const std::vector<int>& dims);
// Compute units of HIP device dev (queried once per device).
int device_cus(int dev);
// One-kernel FP64 forward of a model's single narrow network (rows = B,
// outputs [B x ldo] in out), or with logl != nullptr the diagonal-Gaussian
// logL of a CMB_DIAG model instead of the outputs; false without launching
// when the model does not fit it.
bool emulator_forward_f64_narrow(ns_model* m, const double* theta, int64_t ld, int64_t B, double* out,
                                 int64_t ldo, int is_log, double* logl, const int* count, hipStream_t s);

// Name of candidate c of the one-kernel forward (width 512 or 128, split form
// or not), and the number of candidates.
const char* fused_cfg_name(int h512, int x3, int c);
int fused_ncfg_of(int h512, int x3);

// JSON of the BF16 tile configurations the autotuner chose so far.
std::string bf16_tuning_report(const ns_model* m);

// Autotuner tables: candidates of tuning kind `kind` (0 BF16 hidden GEMM,
// 1 BF16 output GEMM, 2 + split + 2 wide + 4 chi^2 mode + 8 sampler rounds:
// one-kernel emulator) and their names.
int tune_ncfg(int kind);
const char* tune_cfg_name(int kind, int c);
// On-disk tuning cache: load the entries of the model's GPU architecture into
// m->tune (at creation), record a new choice in m->tune and the file.
void tune_cache_load(ns_model* m);
void tune_cache_store(ns_model* m, const std::tuple<int, int64_t, int, int, int>& key, int cfg);

// Slice steps for k walkers with the threshold in device memory (lstar_dev)
// or given on the host; synchronises s.
void slice_step(ns_model* m, double* u, double* logl, int* n_evals, int* n_stalls, int64_t k,
                const double* lstar_dev, const double* L, int n_inner, uint64_t seed, uint64_t iter, int prec,
                hipStream_t s);
void slice_step_host_lstar(ns_model* m, double* u, double* logl, int* n_evals, int* n_stalls, int64_t k,
                           double lstar, const double* L, int n_inner, uint64_t seed, uint64_t iter, int prec,
                           hipStream_t s);

// Hamiltonian Monte Carlo chains (synchronises s).
void hmc_run(ns_model* m, const ns_hmc_opts* o, const double* minv, double* theta, double* samples, double* logp,
             ns_hmc_result* res, hipStream_t s);

// Allocation-free likelihood: the scratch array's device address, taken once
// per device with that device current (at the first model created on it),
// and the batched CMB likelihood with its model vector in that array.
void scratch_init(int device);
size_t scratch_bytes();
void loglike_batch_noalloc(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, int prec,
                           hipStream_t s);

// Nested slice sampling to convergence.
void run(ns_model* m, const ns_run_opts* o, ns_run_result* res, double* dl_h, int* dn_h, double* du_h,
         int64_t cap, hipStream_t s);

}  // namespace nsmi
