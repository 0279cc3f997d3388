// Emulator MLP forward on gfx950 (Sec. 2.2 and 2.4 of the paper: neural
// emulators replace Boltzmann codes; the network form is CosmoPower-like):
//   x = (inputs - shift)/scale,  h_l = f_l(W_l h_{l-1} + b_l),
//   y = mu + sigma * (W_L h_{L-1} + b_L),  f(t) = (gamma + (1-gamma) sigmoid(beta t)) t.
//
// Layer 1 (6-8 inputs) runs on the VALU in FP32/FP64 so that theta is never
// quantised.  Layers 2..L are GEMMs  Y[M x N] = epi(X[M x K] W^T), W stored
// [N x K] (both operands K-contiguous), on MFMA:
//   NS_BF16   v_mfma_f32_32x32x16_bf16, activations stored in BF16
//   NS_BF16X3 the same MFMA on hi/lo BF16 splits of both operands
//             (hi*hi + hi*lo + lo*hi), activations stored in FP32
//   NS_FP32   v_mfma_f32_32x32x2f32
//   NS_FP64   LDS-tiled VALU FMA in double
// The epilogue applies bias + gated activation (hidden layers) or the output
// transform mu + sigma * (.), optionally 10^y (output layer).
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

// ------------------------------------------------------------------ layer 1
template <class T, class OutT> __device__ __forceinline__ OutT cvt_out(T v);
template <> __device__ __forceinline__ double cvt_out<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt_out<float, float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t cvt_out<float, uint16_t>(float v) { return f2bf(v); }

template <class T, class OutT, int ROWS>
__global__ __launch_bounds__(256) void first_layer_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t rows, int rows_per_walker,
    const int* __restrict__ src, const double* __restrict__ fix, const double* __restrict__ znodes,
    const double* __restrict__ shift, const double* __restrict__ scale, int n_in,
    const T* __restrict__ W, const T* __restrict__ b, const T* __restrict__ beta,
    const T* __restrict__ gamma, int n_out, OutT* __restrict__ out, int64_t ldo,
    const int* __restrict__ count) {
    __shared__ T xs[ROWS][16];
    int64_t nrows = rows;
    if (count) nrows = min<int64_t>(rows, (int64_t)(*count) * rows_per_walker);
    const int64_t r0 = (int64_t)blockIdx.x * ROWS;
    if (r0 >= nrows) return;
    if (threadIdx.x < ROWS * n_in) {
        int rr = threadIdx.x / n_in, k = threadIdx.x % n_in;
        int64_t r = r0 + rr;
        double v = 0.0;
        if (r < nrows) {
            int64_t w = r / rows_per_walker;
            int zi = (int)(r % rows_per_walker);
            int s = src[k];
            v = s >= 0 ? theta[w * ld + s] : (s == SRC_ZNODE ? znodes[zi] : fix[k]);
            v = (v - shift[k]) / scale[k];
        }
        xs[rr][k] = (T)v;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n_out; c += blockDim.x) {
        T wrow[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) wrow[k] = k < n_in ? W[(int64_t)c * n_in + k] : T(0);
        const T bc = b[c], be = beta[c], ga = gamma[c];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            int64_t r = r0 + rr;
            if (r >= nrows) break;
            T acc = bc;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < n_in) acc += wrow[k] * xs[rr][k];
            out[r * ldo + c] = cvt_out<T, OutT>(gated<T>(acc, be, ga));
        }
    }
}

// ------------------------------------------------------------------ epilogues
// Hidden layer: bias + gated activation, store as OutT.
template <class T, class OutT> struct EpiHidden {
    const T* b; const T* beta; const T* gamma;
    OutT* out; int64_t ldo;
    struct Col { T b, be, ga; };
    __device__ __forceinline__ Col col(int c) const { return Col{b[c], beta[c], gamma[c]}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col& p, T acc) const {
        out[r * ldo + c] = cvt_out<T, OutT>(gated<T>(acc + p.b, p.be, p.ga));
    }
};

// Output layer: y = mu[row % mu_rows][c] + sigma[c] (acc + b[c]); 10^y if log.
template <class T> struct EpiOut {
    const T* b; const T* mu; const T* sigma;
    T* out; int64_t ldo; int mu_rows; int n_out; int is_log;
    struct Col { T b, s; int c; };
    __device__ __forceinline__ Col col(int c) const { return Col{b[c], sigma[c], c}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col& p, T acc) const {
        int zr = mu_rows > 1 ? (int)(r % mu_rows) : 0;
        T y = mu[(int64_t)zr * n_out + c] + p.s * (acc + p.b);
        if (is_log) y = exp(y * T(2.302585092994045684));
        out[r * ldo + c] = y;
    }
};

// ------------------------------------------------- MFMA GEMM, BF16 operands
// WG tile 128 x 128, four waves in 2 x 2, each wave 64 x 64 = 2 x 2 tiles of
// 32 x 32; BK = 64 staged through LDS (row stride BK + 8 avoids bank conflicts).
// AMODE 0: A is BF16.  AMODE 1: A is FP32, split into hi + lo BF16 (BF16X3).
constexpr int GB_M = 128, GB_N = 128, GB_K = 64, GB_LDS = GB_K + 8;

template <int AMODE, class Epi>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(
    const void* __restrict__ Aptr, int64_t lda, const uint16_t* __restrict__ Whi,
    const uint16_t* __restrict__ Wlo, int64_t M, int N, int K, Epi epi,
    const int* __restrict__ count, int rows_per_count) {
    __shared__ __attribute__((aligned(16))) uint16_t As[GB_M * GB_LDS];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GB_N * GB_LDS];
    __shared__ __attribute__((aligned(16))) uint16_t Al[AMODE ? GB_M * GB_LDS : 8];
    __shared__ __attribute__((aligned(16))) uint16_t Bl[AMODE ? GB_N * GB_LDS : 8];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)blockIdx.y * GB_M;
    const int n0 = blockIdx.x * GB_N;
    if (m0 >= M) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    for (int k0 = 0; k0 < K; k0 += GB_K) {
        // stage A and B tiles: 128 rows x 64 k = 1024 chunks of 8 elements
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + it * 256;
            const int row = c >> 3, kc = (c & 7) * 8;
            const int64_t gr = m0 + row;
            uint4 hi = make_uint4(0, 0, 0, 0), lo = make_uint4(0, 0, 0, 0);
            if (gr < M) {
                if (AMODE == 0) {
                    hi = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(Aptr) + gr * lda + k0 + kc);
                } else {
                    const float* ap = static_cast<const float*>(Aptr) + gr * lda + k0 + kc;
                    float4 f0 = *reinterpret_cast<const float4*>(ap);
                    float4 f1 = *reinterpret_cast<const float4*>(ap + 4);
                    float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
                    uint16_t h[8], l[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        h[e] = f2bf(f[e]);
                        l[e] = f2bf(f[e] - bf2f(h[e]));
                    }
                    hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
                    lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
                }
            }
            *reinterpret_cast<uint4*>(&As[row * GB_LDS + kc]) = hi;
            if (AMODE) *reinterpret_cast<uint4*>(&Al[row * GB_LDS + kc]) = lo;
            const int gn = n0 + row;
            uint4 wh = make_uint4(0, 0, 0, 0), wl = make_uint4(0, 0, 0, 0);
            if (gn < N) {
                wh = *reinterpret_cast<const uint4*>(Whi + (int64_t)gn * K + k0 + kc);
                if (AMODE) wl = *reinterpret_cast<const uint4*>(Wlo + (int64_t)gn * K + k0 + kc);
            }
            *reinterpret_cast<uint4*>(&Bs[row * GB_LDS + kc]) = wh;
            if (AMODE) *reinterpret_cast<uint4*>(&Bl[row * GB_LDS + kc]) = wl;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GB_K; kk += 16) {
            const int koff = kk + (lane >> 5) * 8;
            bf16x8_t a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8_t*>(&As[(wr * 64 + i * 32 + (lane & 31)) * GB_LDS + koff]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8_t*>(&Bs[(wc * 64 + j * 32 + (lane & 31)) * GB_LDS + koff]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (AMODE) {
                bf16x8_t al[2], bl[2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    al[i] = *reinterpret_cast<const bf16x8_t*>(&Al[(wr * 64 + i * 32 + (lane & 31)) * GB_LDS + koff]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    bl[j] = *reinterpret_cast<const bf16x8_t*>(&Bl[(wc * 64 + j * 32 + (lane & 31)) * GB_LDS + koff]);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], b[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }
    // epilogue: lane owns column (lane & 31) of each 32 x 32 tile
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = n0 + wc * 64 + j * 32 + (lane & 31);
        if (c >= N) continue;
        const auto p = epi.col(c);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wr * 64 + i * 32 + (lane >> 5) * 4 + (r >> 2) * 8 + (r & 3);
                if (row < M) epi.store(row, c, p, acc[i][j][r]);
            }
    }
}

// ------------------------------------------------------ MFMA GEMM, FP32
// Same WG tiling; v_mfma_f32_32x32x2f32, BK = 32, LDS row stride 33 floats.
constexpr int GF_K = 32, GF_LDS = GF_K + 1;

template <class Epi>
__global__ __launch_bounds__(256) void gemm_f32_kernel(
    const float* __restrict__ A, int64_t lda, const float* __restrict__ W, int64_t M, int N, int K,
    Epi epi, const int* __restrict__ count, int rows_per_count) {
    __shared__ float As[GB_M * GF_LDS];
    __shared__ float Bs[GB_N * GF_LDS];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)blockIdx.y * GB_M;
    const int n0 = blockIdx.x * GB_N;
    if (m0 >= M) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    f32x16_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    for (int k0 = 0; k0 < K; k0 += GF_K) {
        // 128 rows x 32 k = 1024 float4 chunks
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + it * 256;
            const int row = c >> 3, kc = (c & 7) * 4;
            const int64_t gr = m0 + row;
            float4 av = make_float4(0.f, 0.f, 0.f, 0.f), wv = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gr < M) av = *reinterpret_cast<const float4*>(A + gr * lda + k0 + kc);
            const int gn = n0 + row;
            if (gn < N) wv = *reinterpret_cast<const float4*>(W + (int64_t)gn * K + k0 + kc);
            float* ad = &As[row * GF_LDS + kc];
            ad[0] = av.x; ad[1] = av.y; ad[2] = av.z; ad[3] = av.w;
            float* bd = &Bs[row * GF_LDS + kc];
            bd[0] = wv.x; bd[1] = wv.y; bd[2] = wv.z; bd[3] = wv.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GF_K; kk += 2) {
            const int koff = kk + (lane >> 5);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[(wr * 64 + i * 32 + (lane & 31)) * GF_LDS + koff];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[(wc * 64 + j * 32 + (lane & 31)) * GF_LDS + koff];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int c = n0 + wc * 64 + j * 32 + (lane & 31);
        if (c >= N) continue;
        const auto p = epi.col(c);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wr * 64 + i * 32 + (lane >> 5) * 4 + (r >> 2) * 8 + (r & 3);
                if (row < M) epi.store(row, c, p, acc[i][j][r]);
            }
    }
}

// ------------------------------------------------------ VALU GEMM, FP64
// WG tile 64 x 64, BK = 16, 256 threads with a 4 x 4 register tile each
// (rows ty + 16 i, columns tx + 16 j).
constexpr int GD_M = 64, GD_N = 64, GD_K = 16;

template <class Epi>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    const double* __restrict__ A, int64_t lda, const double* __restrict__ W, int64_t M, int N,
    int K, Epi epi, const int* __restrict__ count, int rows_per_count) {
    __shared__ double As[GD_K][GD_M + 1];
    __shared__ double Bs[GD_K][GD_N + 1];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)blockIdx.y * GD_M;
    const int n0 = blockIdx.x * GD_N;
    if (m0 >= M) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += GD_K) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + it * 256;          // 64 rows x 16 k
            const int row = c >> 4, kk = c & 15;
            const int64_t gr = m0 + row;
            As[kk][row] = (gr < M && k0 + kk < K) ? A[gr * lda + k0 + kk] : 0.0;
            const int gn = n0 + row;
            Bs[kk][row] = (gn < N && k0 + kk < K) ? W[(int64_t)gn * K + k0 + kk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GD_K; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = n0 + tx + 16 * j;
        if (c >= N) continue;
        const auto p = epi.col(c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = m0 + ty + 16 * i;
            if (row < M) epi.store(row, c, p, acc[i][j]);
        }
    }
}

// ------------------------------------------------------------------ driver
static inline dim3 grid2(int64_t M, int N, int bm, int bn) {
    return dim3((unsigned)((N + bn - 1) / bn), (unsigned)((M + bm - 1) / bm));
}

void emulator_forward(ns_model* m, int ni, const double* theta, int64_t ld, int64_t B, void* out,
                      int64_t ldo, int is_log, int prec, const int* count, hipStream_t s) {
    Net& net = *m->nets[ni];
    const int L = net.n_layers;
    const int rpw = net.out_mu_rows;                 // rows per walker
    const int64_t rows = B * rpw;
    const int n_in = net.dims[0];
    NS_CHECK(n_in <= 16, NS_E_UNSUPPORTED, "emulator with more than 16 inputs");
    const int h1 = net.dims[1];
    const size_t act_elem = prec == NS_FP64 ? 8 : (prec == NS_BF16 ? 2 : 4);
    size_t max_w = 0;
    for (int l = 1; l < L; ++l) max_w = std::max(max_w, (size_t)net.dims[l]);
    m->ws_act[0].ensure((size_t)rows * max_w * act_elem);
    m->ws_act[1].ensure((size_t)rows * max_w * act_elem);
    Layer& l1 = *net.layers[0];
    const int rows_blk = 4;
    dim3 g1((unsigned)((rows + rows_blk - 1) / rows_blk));
    const int* src = m->emu_src_d.as<int>();
    const double* fix = m->emu_fix_d.as<double>();
    const double* zn = m->znodes_d.as<double>();
    {
    TraceScope ts(m, s, "emu_first_layer");
    if (prec == NS_FP64) {
        hipLaunchKernelGGL((first_layer_kernel<double, double, 4>), g1, dim3(256), 0, s, theta, ld, rows, rpw,
                           src, fix, zn, net.in_shift.as<double>(), net.in_scale.as<double>(), n_in,
                           l1.W64.as<double>(), l1.b64.as<double>(), l1.beta64.as<double>(), l1.gamma64.as<double>(),
                           h1, m->ws_act[0].as<double>(), (int64_t)h1, count);
    } else if (prec == NS_BF16) {
        hipLaunchKernelGGL((first_layer_kernel<float, uint16_t, 4>), g1, dim3(256), 0, s, theta, ld, rows, rpw,
                           src, fix, zn, net.in_shift.as<double>(), net.in_scale.as<double>(), n_in,
                           l1.W32.as<float>(), l1.b32.as<float>(), l1.beta32.as<float>(), l1.gamma32.as<float>(),
                           h1, m->ws_act[0].as<uint16_t>(), (int64_t)h1, count);
    } else {
        hipLaunchKernelGGL((first_layer_kernel<float, float, 4>), g1, dim3(256), 0, s, theta, ld, rows, rpw,
                           src, fix, zn, net.in_shift.as<double>(), net.in_scale.as<double>(), n_in,
                           l1.W32.as<float>(), l1.b32.as<float>(), l1.beta32.as<float>(), l1.gamma32.as<float>(),
                           h1, m->ws_act[0].as<float>(), (int64_t)h1, count);
    }
    NS_HIP(hipGetLastError());
    }
    int cur = 0;
    for (int l = 1; l < L; ++l) {
        Layer& ly = *net.layers[l];
        const int K = ly.n_in, N = ly.n_out;
        const bool last = (l == L - 1);
        void* A = m->ws_act[cur].p;
        void* dst = last ? out : m->ws_act[cur ^ 1].p;
        static const char* names[4][2] = {{"gemm_f64_hidden", "gemm_f64_out"}, {"gemm_f32_hidden", "gemm_f32_out"},
                                          {"gemm_bf16_hidden", "gemm_bf16_out"},
                                          {"gemm_bf16x3_hidden", "gemm_bf16x3_out"}};
        TraceScope ts(m, s, names[prec][last ? 1 : 0]);
        if (prec == NS_FP64) {
            dim3 g = grid2(rows, N, GD_M, GD_N);
            if (!last) {
                EpiHidden<double, double> e{ly.b64.as<double>(), ly.beta64.as<double>(), ly.gamma64.as<double>(),
                                           (double*)dst, (int64_t)N};
                hipLaunchKernelGGL((gemm_f64_kernel<EpiHidden<double, double>>), g, dim3(256), 0, s,
                                   (const double*)A, (int64_t)K, ly.W64.as<double>(), rows, N, K, e, count, rpw);
            } else {
                EpiOut<double> e{ly.b64.as<double>(), net.out_mu64.as<double>(), net.out_sigma64.as<double>(),
                                 (double*)dst, last ? ldo : (int64_t)N, net.out_mu_rows, N, is_log};
                hipLaunchKernelGGL(gemm_f64_kernel<EpiOut<double>>, g, dim3(256), 0, s,
                                   (const double*)A, (int64_t)K, ly.W64.as<double>(), rows, N, K, e, count, rpw);
            }
        } else if (prec == NS_FP32) {
            NS_CHECK(K % GF_K == 0, NS_E_UNSUPPORTED, "FP32 MFMA layers need K % 32 == 0");
            dim3 g = grid2(rows, N, GB_M, GB_N);
            if (!last) {
                EpiHidden<float, float> e{ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(),
                                         (float*)dst, (int64_t)N};
                hipLaunchKernelGGL((gemm_f32_kernel<EpiHidden<float, float>>), g, dim3(256), 0, s,
                                   (const float*)A, (int64_t)K, ly.W32.as<float>(), rows, N, K, e, count, rpw);
            } else {
                EpiOut<float> e{ly.b32.as<float>(), net.out_mu32.as<float>(), net.out_sigma32.as<float>(),
                                (float*)dst, last ? ldo : (int64_t)N, net.out_mu_rows, N, is_log};
                hipLaunchKernelGGL(gemm_f32_kernel<EpiOut<float>>, g, dim3(256), 0, s,
                                   (const float*)A, (int64_t)K, ly.W32.as<float>(), rows, N, K, e, count, rpw);
            }
        } else {
            NS_CHECK(K % GB_K == 0, NS_E_UNSUPPORTED, "BF16 MFMA layers need K % 64 == 0");
            dim3 g = grid2(rows, N, GB_M, GB_N);
            const bool x3 = prec == NS_BF16X3;
            if (!last) {
                if (x3) {
                    EpiHidden<float, float> e{ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(),
                                             (float*)dst, (int64_t)N};
                    hipLaunchKernelGGL((gemm_bf16_kernel<1, EpiHidden<float, float>>), g, dim3(256), 0, s, A,
                                       (int64_t)K, ly.Whi.as<uint16_t>(), ly.Wlo.as<uint16_t>(), rows, N, K, e, count, rpw);
                } else {
                    EpiHidden<float, uint16_t> e{ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(),
                                                (uint16_t*)dst, (int64_t)N};
                    hipLaunchKernelGGL((gemm_bf16_kernel<0, EpiHidden<float, uint16_t>>), g, dim3(256), 0, s, A,
                                       (int64_t)K, ly.Whi.as<uint16_t>(), ly.Wlo.as<uint16_t>(), rows, N, K, e, count, rpw);
                }
            } else {
                EpiOut<float> e{ly.b32.as<float>(), net.out_mu32.as<float>(), net.out_sigma32.as<float>(),
                                (float*)dst, last ? ldo : (int64_t)N, net.out_mu_rows, N, is_log};
                if (x3)
                    hipLaunchKernelGGL((gemm_bf16_kernel<1, EpiOut<float>>), g, dim3(256), 0, s, A, (int64_t)K,
                                       ly.Whi.as<uint16_t>(), ly.Wlo.as<uint16_t>(), rows, N, K, e, count, rpw);
                else
                    hipLaunchKernelGGL((gemm_bf16_kernel<0, EpiOut<float>>), g, dim3(256), 0, s, A, (int64_t)K,
                                       ly.Whi.as<uint16_t>(), ly.Wlo.as<uint16_t>(), rows, N, K, e, count, rpw);
            }
        }
        NS_HIP(hipGetLastError());
        cur ^= 1;
    }
}

}  // namespace nsmi
