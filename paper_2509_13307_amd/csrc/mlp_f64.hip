// Whole-network FP64 emulator forward in one kernel for narrow networks
// (every hidden width 128, at most 256 outputs), with the diagonal
// Gaussian chi^2 of Sec. 2.3 optionally evaluated in the same kernel: the
// nested sampler's rounds evaluate a few thousand walkers of the 6-parameter
// CMB emulator, where one launch per layer plus one for the chi^2 cost more
// than the arithmetic.
//
// One workgroup (four waves) owns 16 rows (one v_mfma_f64_16x16x4f64 row
// tile).  Layer 1 runs on the VALU; GEMM layers take their A operand from the
// activations in LDS and their B operand from weights stored at model
// creation in MFMA fragment order (per K step of 4 and 16-unit column tile,
// the 64 lanes' values contiguous: one coalesced 512-byte load).  Wave w owns
// column tiles w, w + 4, ...; every accumulator runs k = 0, 4, 8, ... as in
// the layer-by-layer FP64 GEMM, the epilogues are that path's expressions,
// and the chi^2 sums each row as the separate chi^2 kernel does (lane i takes
// data points i, i + 64, ...; then a wave sum), so both paths agree bitwise.
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

constexpr int MF_R = 16;            // rows per workgroup
constexpr int MF_MAXOUT = 256;      // outputs (16 column tiles: 4 per wave)
constexpr int MF_MAXHID = 6;        // hidden GEMM layers

struct F64Args {
    const double* W1; const double* b1; const double* be1; const double* ga1;   // layer 1 [H x n_in]
    const double* shift; const double* scale;
    const double* Wf;                                  // fragments of the GEMM layers, in layer order
    const double* bias[MF_MAXHID + 1];                 // GEMM layer l (hidden, then output)
    const double* beta[MF_MAXHID];
    const double* gamma[MF_MAXHID];
    const double* mu; const double* sigma;
    int n_in, n_hidden, N_out, is_log;
    double* out; int64_t ldo;                          // outputs, when no chi^2 is fused
    const double* data; const double* isig; double cst; double* logl;   // fused diagonal chi^2
    int d; const int* pk; const double* pa; const double* pb;
};

bool narrow_f64_shape(const std::vector<int>& dims) {
    const int L = (int)dims.size() - 1;
    if (L < 3 || L - 2 > MF_MAXHID || dims[0] > 16 || dims[L] > MF_MAXOUT) return false;
    const int H = dims[1];
    if (H != 128) return false;
    for (int l = 1; l < L; ++l)
        if (dims[l] != H) return false;
    return true;
}

// GEMM layer over the workgroup's 16 rows: wave w's column tiles w, w + 4,
// ... (TPW of them), K steps k = 0, 4, 8, ...; the B fragments run PF steps
// ahead in a register ring of 16 fragments (slot u feeds step kq, then is
// refilled with step kq + PF), about 1000 cycles of MFMA work, so the L2
// latency of the weights is not on each step's path.
template <int TPW, int K4, int LDA>
__device__ __forceinline__ void mf_layer_gemm(const double* __restrict__ act, const double* __restrict__ Wl, int NT,
                                              int wave, int lane, f64x4_t (&acc)[TPW]) {
    constexpr int MF_PF = 16 / TPW;
    static_assert(K4 % MF_PF == 0, "K steps must be a multiple of the prefetch depth");
    double bq[MF_PF][TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.0;
    // loads and MFMAs are unconditional (a branch around either makes the
    // compiler wait for every load in flight): tiles past NT recompute tile
    // NT - 1 and steps past the layer re-read its last step; neither result
    // is stored
    int ntc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) ntc[t] = min(wave + 4 * t, NT - 1);
    auto fetch = [&](int kq, double (&b)[TPW]) {
        kq = min(kq, K4 - 1);
#pragma unroll
        for (int t = 0; t < TPW; ++t) b[t] = Wl[((size_t)kq * NT + ntc[t]) * 64 + lane];
    };
#pragma unroll
    for (int u = 0; u < MF_PF; ++u) fetch(u, bq[u]);
    for (int kq0 = 0; kq0 < K4; kq0 += MF_PF) {
#pragma unroll
        for (int u = 0; u < MF_PF; ++u) {
            const int kq = kq0 + u;
            const double a = act[(lane & 15) * LDA + kq * 4 + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < TPW; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq[u][t], acc[t], 0, 0, 0);
            fetch(kq + MF_PF, bq[u]);
        }
    }
}

// One GEMM layer and its epilogue: hidden (bias, gated activation, back into
// act after a barrier) or output (transform; into ys or the output rows).
template <int TPW, int H, bool CHI2>
__device__ __forceinline__ void mf_layer(double* act, double* ys, const F64Args& A, const double* Wl, int l,
                                         bool hid, int NT, int64_t r0, int64_t nrows, int wave, int lane) {
    constexpr int LDA = H + 1, K4 = H / 4;
    f64x4_t acc[TPW];
    mf_layer_gemm<TPW, K4, LDA>(act, Wl, NT, wave, lane, acc);
    if (hid) {
        __syncthreads();                               // every wave done reading this layer's input
        const double* bb = A.bias[l];
        const double* be = A.beta[l];
        const double* ga = A.gamma[l];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int nt = wave + 4 * t;
            if (nt >= NT) continue;
            const int c = nt * 16 + (lane & 15);
            const double pb = bb[c], pbe = be[c], pga = ga[c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = (lane >> 4) + 4 * r;
                act[rr * LDA + c] = gated<double>(acc[t][r] + pb, pbe, pga);
            }
        }
        __syncthreads();                               // next layer's input complete
    } else {
        const double* bo = A.bias[l];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int nt = wave + 4 * t;
            if (nt >= NT) continue;
            const int c = nt * 16 + (lane & 15);
            if (c >= A.N_out) continue;
            const double pb = bo[c], ps = A.sigma[c], pm = A.mu[c];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = (lane >> 4) + 4 * r;
                double y = pm + ps * (acc[t][r] + pb);
                if (A.is_log) y = exp10_of<double>(y);
                if (CHI2) ys[rr * MF_MAXOUT + c] = y;
                else if (r0 + rr < nrows) A.out[(r0 + rr) * A.ldo + c] = y;
            }
        }
    }
}

template <int H, bool CHI2>
__global__ __launch_bounds__(256, 2) void mlp_f64_kernel(const double* __restrict__ theta, int64_t ld, int64_t rows,
                                                         const int* __restrict__ src, const double* __restrict__ fix,
                                                         F64Args A, const int* __restrict__ count) {
    constexpr int LDA = H + 1;                         // LDS row stride (doubles): conflict-free A reads
    constexpr int K4 = H / 4;                          // K steps of a GEMM layer
    __shared__ double act[MF_R * LDA];
    __shared__ double xs[MF_R][16];
    __shared__ double ys[CHI2 ? MF_R * MF_MAXOUT : 1];
    int64_t nrows = rows;
    if (count) nrows = min<int64_t>(rows, (int64_t)(*count));
    const int64_t r0 = (int64_t)blockIdx.x * MF_R;
    if (r0 >= nrows) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n_in = A.n_in, N_out = A.N_out;
    // chi^2 mode: whether each row's walker lies in the prior's support, found
    // now (the first threads, one row each) so that its loads overlap the
    // inputs' instead of closing the kernel
    __shared__ int okr[MF_R];
    if (CHI2 && tid < MF_R) {
        const int64_t row = r0 + tid;
        okr[tid] = row < nrows && in_support(theta + row * ld, A.d, A.pk, A.pa, A.pb);
    }
    for (int e = tid; e < MF_R * 16; e += 256) {
        const int rr = e / 16, k = e % 16;
        const int64_t r = r0 + rr;
        double v = 0.0;
        if (r < nrows && k < n_in) {
            const int s = src[k];
            const double t = s >= 0 ? theta[r * ld + s] : fix[k];
            v = (t - A.shift[k]) / A.scale[k];
        }
        xs[rr][k] = v;
    }
    __syncthreads();
    {
        // each thread's unit c for its rows tid / H, tid / H + 256 / H, ...,
        // all of them side by side (one row after the other would wait on
        // each row's exponential and division in turn)
        constexpr int RS = 256 / H, NR = MF_R / RS;
        const int c = tid % H, rr0 = tid / H;
        double w1[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) w1[k] = k < n_in ? A.W1[c * n_in + k] : 0.0;
        const double b1 = A.b1[c], be1 = A.be1[c], ga1 = A.ga1[c];
        double acc[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = b1;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < n_in)
#pragma unroll
                for (int j = 0; j < NR; ++j) acc[j] += w1[k] * xs[rr0 + j * RS][k];
#pragma unroll
        for (int j = 0; j < NR; ++j) act[(rr0 + j * RS) * LDA + c] = gated<double>(acc[j], be1, ga1);
    }
    __syncthreads();
    size_t foff = 0;
    for (int l = 0; l <= A.n_hidden; ++l) {
        const bool hid = l < A.n_hidden;
        const int NT = hid ? H / 16 : (N_out + 15) / 16;
        const double* Wl = A.Wf + foff;
        foff += (size_t)K4 * NT * 64;
        if (NT <= 4) mf_layer<1, H, CHI2>(act, ys, A, Wl, l, hid, NT, r0, nrows, wave, lane);
        else if (NT <= 8) mf_layer<2, H, CHI2>(act, ys, A, Wl, l, hid, NT, r0, nrows, wave, lane);
        else mf_layer<4, H, CHI2>(act, ys, A, Wl, l, hid, NT, r0, nrows, wave, lane);
    }
    if (CHI2) {
        // wave w sums rows w, w + 4, w + 8, w + 12, side by side (each row's
        // terms in the order of the staged chi^2 kernel, then a wave sum)
        __syncthreads();
        constexpr int RW = MF_R / 4;
        double s[RW];
#pragma unroll
        for (int j = 0; j < RW; ++j) s[j] = 0.0;
        for (int i = lane; i < N_out; i += 64) {
            const double di = A.data[i], wi = A.isig[i];
#pragma unroll
            for (int j = 0; j < RW; ++j) {
                const double r = (di - ys[(wave + 4 * j) * MF_MAXOUT + i]) * wi;
                s[j] = fma(r, r, s[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < RW; ++j) s[j] = wave_sum(s[j]);
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < RW; ++j) {
                const int rr = wave + 4 * j;
                if (r0 + rr < nrows) A.logl[r0 + rr] = okr[rr] ? -0.5 * s[j] + A.cst : -INFINITY;
            }
    }
}

// FP64 forward (and, for the diagonal CMB likelihood, logL) of a narrow
// single network in one launch; false without launching when the model does
// not fit it.  logl != nullptr fuses the chi^2 (outputs are then not stored).
bool emulator_forward_f64_narrow(ns_model* m, const double* theta, int64_t ld, int64_t B, double* out,
                                 int64_t ldo, int is_log, double* logl, const int* count, hipStream_t s) {
    if (m->nets.size() != 1 || !m->nets[0]->narrow64 || m->nets[0]->out_mu_rows != 1) return false;
    if (getenv("NSMI_NO_FUSED_MLP") != nullptr) return false;
    const Net& net = *m->nets[0];
    const int L = net.n_layers, H = net.dims[1];
    F64Args A{};
    const Layer& l1 = *net.layers[0];
    A.W1 = l1.W64.as<double>(); A.b1 = l1.b64.as<double>();
    A.be1 = l1.beta64.as<double>(); A.ga1 = l1.gamma64.as<double>();
    A.shift = net.in_shift.as<double>(); A.scale = net.in_scale.as<double>();
    A.Wf = net.Wf64.as<double>();
    for (int l = 1; l < L; ++l) {
        const Layer& ly = *net.layers[l];
        A.bias[l - 1] = ly.b64.as<double>();
        if (l < L - 1) {
            A.beta[l - 1] = ly.beta64.as<double>();
            A.gamma[l - 1] = ly.gamma64.as<double>();
        }
    }
    A.mu = net.out_mu64.as<double>(); A.sigma = net.out_sigma64.as<double>();
    A.n_in = net.dims[0]; A.n_hidden = L - 2; A.N_out = net.dims[L]; A.is_log = is_log;
    A.out = out; A.ldo = ldo;
    if (logl) {
        A.data = m->data.as<double>(); A.isig = m->inv_sigma.as<double>(); A.cst = m->logl_const; A.logl = logl;
        A.d = m->d; A.pk = m->prior_kind.as<int>(); A.pa = m->prior_a.as<double>(); A.pb = m->prior_b.as<double>();
    }
    TraceScope ts(m, s, logl ? "mlp_f64_chi2" : "mlp_f64");
    const dim3 grid((unsigned)((B + MF_R - 1) / MF_R));
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, theta, ld, B, m->emu_src_d.as<int>(),
                           m->emu_fix_d.as<double>(), A, count);
    };
    (void)H;
    if (logl) go(mlp_f64_kernel<128, true>);
    else go(mlp_f64_kernel<128, false>);
    NS_HIP(hipGetLastError());
    return true;
}

}  // namespace nsmi
