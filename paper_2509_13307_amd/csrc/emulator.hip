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
//   NS_FP64   v_mfma_f64_16x16x4f64
// The epilogue applies bias + gated activation (hidden layers) or the output
// transform mu + sigma * (.), optionally 10^y (output layer).
//
// Networks with identical shapes (the four CMB spectra) run in one grid,
// blockIdx.z selecting the network, so a 4096-walker layer fills the chip.
#include "devutil.h"
#include "gemm_bf16.h"
#include "nsmi.h"

namespace nsmi {

constexpr int MAXG = 4;

// ------------------------------------------------------------------ layer 1
template <class T, class OutT> __device__ __forceinline__ OutT cvt_out(T v);
template <> __device__ __forceinline__ double cvt_out<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt_out<float, float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t cvt_out<float, uint16_t>(float v) { return f2bf(v); }

template <class T, class OutT> struct FirstArgs {
    const T* W[MAXG];
    const T* b[MAXG];
    const T* beta[MAXG];
    const T* gamma[MAXG];
    const double* shift[MAXG];
    const double* scale[MAXG];
    OutT* out[MAXG];
    T* tsave[MAXG];
};

// One workgroup per block of FL_ROWS rows.  The normalised inputs of the
// block are computed once per row into LDS; thread t owns CPT consecutive
// units (its CPT x n_in weights held in registers) for every
// (256 / (n_out / CPT))-th row of the block.  Each unit's sum runs in input
// order starting from the bias, whatever the thread mapping.
constexpr int FL_ROWS = 16;                  // small blocks: short serial chains per thread

template <class T, class OutT, int NI, int CPT>
__global__ __launch_bounds__(256) void first_layer_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t rows, int rows_per_walker,
    const int* __restrict__ src, const double* __restrict__ fix, const double* __restrict__ znodes, int n_in,
    int n_out, FirstArgs<T, OutT> P, const int* __restrict__ count) {
    __shared__ T xs[FL_ROWS][NI];
    const int g = blockIdx.z;
    int64_t nrows = rows;
    if (count) nrows = min<int64_t>(rows, (int64_t)(*count) * rows_per_walker);
    const int64_t r0 = (int64_t)blockIdx.x * FL_ROWS;
    if (r0 >= nrows) return;
    const int tid = threadIdx.x;
    const int groups = n_out / CPT;
    const int rpi = 256 / groups;                      // rows per pass of the workgroup
    // this thread's CPT units: weights requested before the barrier, so that
    // they arrive with the inputs
    const int c0 = (tid % groups) * CPT;
    T wr[CPT][NI], bb[CPT], be[CPT], ga[CPT];
    const T* W = P.W[g];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        bb[j] = P.b[g][c0 + j];
        be[j] = P.beta[g][c0 + j];
        ga[j] = P.gamma[g][c0 + j];
#pragma unroll
        for (int k = 0; k < NI; ++k) wr[j][k] = k < n_in ? W[(c0 + j) * n_in + k] : T(0);
    }
    for (int e = tid; e < FL_ROWS * NI; e += 256) {
        const int rr = e / NI, k = e % NI;
        const int64_t r = r0 + rr;
        T v = T(0);
        if (k < n_in && r < nrows) {
            const int64_t w = r / rows_per_walker;
            const int zi = (int)(r % rows_per_walker);
            const int s = src[k];
            const double t = s >= 0 ? theta[w * ld + s] : (s == SRC_ZNODE ? znodes[zi] : fix[k]);
            v = (T)((t - P.shift[g][k]) / P.scale[g][k]);
        }
        xs[rr][k] = v;
    }
    __syncthreads();
    if (tid >= groups * rpi) return;
    // the thread's rows tid / groups, + rpi, ..., FR at a time with their CPT
    // units side by side (the FP64 activations' exponentials and divisions of
    // one row after another would each wait on the last; in FP32, with twice
    // the units per thread, more rows at a time cost occupancy instead)
    constexpr int FR = sizeof(T) == 8 ? 4 : 1;
    for (int rr0 = tid / groups; rr0 < FL_ROWS; rr0 += FR * rpi) {
        T acc[FR][CPT];
#pragma unroll
        for (int q = 0; q < FR; ++q)
#pragma unroll
            for (int j = 0; j < CPT; ++j) acc[q][j] = bb[j];
#pragma unroll
        for (int k = 0; k < NI; ++k)
            if (k < n_in)
#pragma unroll
                for (int q = 0; q < FR; ++q) {
                    const int rr = min(rr0 + q * rpi, FL_ROWS - 1);
                    const T x = xs[rr][k];
#pragma unroll
                    for (int j = 0; j < CPT; ++j) acc[q][j] += wr[j][k] * x;
                }
#pragma unroll
        for (int q = 0; q < FR; ++q) {
            const int rr = rr0 + q * rpi;
            const int64_t r = r0 + rr;
            if (rr >= FL_ROWS || r >= nrows) break;
            OutT* out = P.out[g] + r * n_out + c0;
            T* ts = P.tsave[g] ? P.tsave[g] + r * n_out + c0 : nullptr;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                if (ts) ts[j] = acc[q][j];
                out[j] = cvt_out<T, OutT>(gated<T>(acc[q][j], be[j], ga[j]));
            }
        }
    }
}

// ------------------------------------------------------------------ epilogues
// Hidden layer: bias + gated activation, store as OutT; optionally keep the
// pre-activation t (for the adjoint) in tsave.
template <class T, class OutT> struct EpiHidden {
    const T* b; const T* beta; const T* gamma;
    OutT* out; int64_t ldo;
    T* tsave = nullptr;
    struct Col { T b, be, ga; };
    __device__ __forceinline__ Col col(int c) const { return Col{b[c], beta[c], gamma[c]}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col& p, T acc) const {
        const T t = acc + p.b;
        if (tsave) tsave[r * ldo + c] = t;
        out[r * ldo + c] = cvt_out<T, OutT>(gated<T>(t, p.be, p.ga));
    }
};

// Adjoint of a hidden layer: delta_{l-1} = (delta_l W_l) * f'(t_{l-1}),
// f'(t) = gamma + (1 - gamma) [s + beta t s (1 - s)], s = sigmoid(beta t).
template <class T> struct EpiBack {
    const T* tsave; const T* beta; const T* gamma;
    T* out; int64_t ldo;
    struct Col { T be, ga; };
    __device__ __forceinline__ Col col(int c) const { return Col{beta[c], gamma[c]}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col& p, T acc) const {
        const T t = tsave[r * ldo + c];
        const T s = sigmoid<T>(p.be * t);
        out[r * ldo + c] = acc * (p.ga + (T(1) - p.ga) * (s + p.be * t * s * (T(1) - s)));
    }
};

// Adjoint of the first layer: plain store of delta_1 W_1 restricted to inputs.
template <class T> struct EpiPlain {
    T* out; int64_t ldo;
    struct Col { int c; };
    __device__ __forceinline__ Col col(int c) const { return Col{c}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col&, T acc) const { out[r * ldo + c] = acc; }
};

// Output layer: y = mu[row % mu_rows][c] + sigma[c] (acc + b[c]); 10^y if log.
template <class T> struct EpiOut {
    const T* b; const T* mu; const T* sigma;
    T* out; int64_t ldo; int mu_rows; int n_out; int is_log;
    struct Col { T b, s, mu0; int c; };
    __device__ __forceinline__ Col col(int c) const { return Col{b[c], sigma[c], mu[c], c}; }
    __device__ __forceinline__ void store(int64_t r, int c, const Col& p, T acc) const {
        const T m = mu_rows > 1 ? mu[(int64_t)(r % mu_rows) * n_out + c] : p.mu0;
        T y = m + p.s * (acc + p.b);
        if (is_log) y = exp10_of<T>(y);
        out[r * ldo + c] = y;
    }
};


// ------------------------------------------------- MFMA GEMM, BF16 operands
// WG tile 128 x 128, four waves in 2 x 2, each wave 64 x 64 = 2 x 2 tiles of
// 32 x 32; BK = 64 staged through LDS (row stride BK + 8 avoids bank conflicts).
// The next K tile is fetched into registers while the current one feeds the
// MFMAs.  AMODE 0: A is BF16, LDS double buffered.  AMODE 1: A is FP32, split
// into hi + lo BF16 (BF16X3), single LDS buffer (four operand planes).
constexpr int GB_M = 128, GB_N = 128, GB_K = 64, GB_LDS = GB_K + 8;
constexpr int GB_TILE = GB_M * GB_LDS;   // elements of one operand tile in LDS

template <int AMODE>
struct Bf16Stage {
    uint4 a[4], al[AMODE ? 4 : 1], b[4], bl[AMODE ? 4 : 1];
};

template <int AMODE>
__device__ __forceinline__ void bf16_fetch(Bf16Stage<AMODE>& st, const void* Aptr, int64_t lda,
                                           const uint16_t* Whi, const uint16_t* Wlo, int64_t m0, int n0, int64_t M,
                                           int N, int K, int k0, int tid) {
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
                const float4 f0 = *reinterpret_cast<const float4*>(ap);
                const float4 f1 = *reinterpret_cast<const float4*>(ap + 4);
                const float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
                uint32_t h[8], l[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint16_t hb = f2bf(f[e]);
                    h[e] = hb;
                    l[e] = bf16_lo(f[e], hb);
                }
                hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
                lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
            }
        }
        st.a[it] = hi;
        if (AMODE) st.al[it] = lo;
        const int gn = n0 + row;
        uint4 wh = make_uint4(0, 0, 0, 0), wl = make_uint4(0, 0, 0, 0);
        if (gn < N) {
            wh = *reinterpret_cast<const uint4*>(Whi + (int64_t)gn * K + k0 + kc);
            if (AMODE) wl = *reinterpret_cast<const uint4*>(Wlo + (int64_t)gn * K + k0 + kc);
        }
        st.b[it] = wh;
        if (AMODE) st.bl[it] = wl;
    }
}

template <int AMODE>
__device__ __forceinline__ void bf16_stash(const Bf16Stage<AMODE>& st, uint16_t* As, uint16_t* Bs, uint16_t* Al,
                                           uint16_t* Bl, int tid) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int c = tid + it * 256;
        const int off = (c >> 3) * GB_LDS + (c & 7) * 8;
        *reinterpret_cast<uint4*>(&As[off]) = st.a[it];
        *reinterpret_cast<uint4*>(&Bs[off]) = st.b[it];
        if (AMODE) {
            *reinterpret_cast<uint4*>(&Al[off]) = st.al[it];
            *reinterpret_cast<uint4*>(&Bl[off]) = st.bl[it];
        }
    }
}

template <int AMODE>
__device__ __forceinline__ void bf16_mfma_tile(f32x16_t (&acc)[2][2], const uint16_t* As, const uint16_t* Bs,
                                               const uint16_t* Al, const uint16_t* Bl, int lane, int wr, int wc) {
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
}

template <int AMODE, class Epi>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(Group<Epi> G, int64_t lda, int64_t M, int N, int K,
                                                        const int* __restrict__ count, int rows_per_count) {
    // AMODE 0: two buffers of (A, B); AMODE 1: one buffer of (A hi, B hi, A lo, B lo)
    __shared__ __attribute__((aligned(16))) uint16_t lds[4 * GB_TILE];
    const TileId tile = xcd_tile();
    const int g = tile.g;
    const void* Aptr = G.A[g];
    const uint16_t* Whi = static_cast<const uint16_t*>(G.W[g]);
    const uint16_t* Wlo = static_cast<const uint16_t*>(G.Wl[g]);
    const Epi& epi = G.epi[g];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)tile.ty * GB_M;
    const int n0 = tile.tx * GB_N;
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

    Bf16Stage<AMODE> st;
    const int nk = K / GB_K;
    bf16_fetch<AMODE>(st, Aptr, lda, Whi, Wlo, m0, n0, M, N, K, 0, tid);
    if (AMODE == 0) {
        bf16_stash<AMODE>(st, lds, lds + GB_TILE, nullptr, nullptr, tid);
        __syncthreads();
        for (int t = 0; t < nk; ++t) {
            uint16_t* cur = lds + (t & 1) * 2 * GB_TILE;
            uint16_t* nxt = lds + ((t + 1) & 1) * 2 * GB_TILE;
            if (t + 1 < nk) bf16_fetch<AMODE>(st, Aptr, lda, Whi, Wlo, m0, n0, M, N, K, (t + 1) * GB_K, tid);
            bf16_mfma_tile<AMODE>(acc, cur, cur + GB_TILE, nullptr, nullptr, lane, wr, wc);
            if (t + 1 < nk) bf16_stash<AMODE>(st, nxt, nxt + GB_TILE, nullptr, nullptr, tid);
            __syncthreads();
        }
    } else {
        for (int t = 0; t < nk; ++t) {
            bf16_stash<AMODE>(st, lds, lds + GB_TILE, lds + 2 * GB_TILE, lds + 3 * GB_TILE, tid);
            __syncthreads();
            if (t + 1 < nk) bf16_fetch<AMODE>(st, Aptr, lda, Whi, Wlo, m0, n0, M, N, K, (t + 1) * GB_K, tid);
            bf16_mfma_tile<AMODE>(acc, lds, lds + GB_TILE, lds + 2 * GB_TILE, lds + 3 * GB_TILE, lane, wr, wc);
            __syncthreads();
        }
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
__global__ __launch_bounds__(256) void gemm_f32_kernel(Group<Epi> G, int64_t lda, int64_t M, int N, int K,
                                                       const int* __restrict__ count, int rows_per_count) {
    __shared__ float As[GB_M * GF_LDS];
    __shared__ float Bs[GB_N * GF_LDS];
    const int g = blockIdx.z;
    const float* A = static_cast<const float*>(G.A[g]);
    const float* W = static_cast<const float*>(G.W[g]);
    const Epi& epi = G.epi[g];
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

    // 128 rows x 32 k = 1024 float4 chunks per operand; the next K block is
    // fetched into registers while the current one feeds the MFMAs
    float4 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + it * 256;
            const int row = c >> 3, kc = (c & 7) * 4;
            const int64_t gr = m0 + row;
            ra[it] = make_float4(0.f, 0.f, 0.f, 0.f);
            rb[it] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gr < M) ra[it] = *reinterpret_cast<const float4*>(A + gr * lda + k0 + kc);
            const int gn = n0 + row;
            if (gn < N) rb[it] = *reinterpret_cast<const float4*>(W + (int64_t)gn * K + k0 + kc);
        }
    };
    gload(0);
    for (int k0 = 0; k0 < K; k0 += GF_K) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + it * 256;
            const int row = c >> 3, kc = (c & 7) * 4;
            float* ad = &As[row * GF_LDS + kc];
            ad[0] = ra[it].x; ad[1] = ra[it].y; ad[2] = ra[it].z; ad[3] = ra[it].w;
            float* bd = &Bs[row * GF_LDS + kc];
            bd[0] = rb[it].x; bd[1] = rb[it].y; bd[2] = rb[it].z; bd[3] = rb[it].w;
        }
        __syncthreads();
        if (k0 + GF_K < K) gload(k0 + GF_K);
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

// ------------------------------------------------------ MFMA GEMM, FP64
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// register r of lane l returns D[l / 16 + 4 r][l % 16].
// WG tile BM x 64 (BM = 64: four waves in 2 x 2, each 32 x 32 = 2 x 2 tiles of
// 16 x 16; BM = 32, for grids too small to fill the GPU: four waves in 1 x 4,
// each 32 x 16); BK = 32, LDS row stride 33 doubles.  The next K block's tiles
// are fetched into registers while the current one feeds the MFMAs (the K
// order of every accumulator is the same for both tiles: k = 0, 4, 8, ...).
// Bounded to 128 registers so that four waves share each SIMD (left free the
// compiler takes 164 and three fit; four hide the barrier and LDS latency
// better, 4-7% faster).
constexpr int GD_M = 64, GD_N = 64, GD_K = 32, GD_LDS = GD_K + 1;

template <class Epi, int BM>
__global__ __launch_bounds__(256, 4) void gemm_f64_kernel(Group<Epi> G, int64_t lda, int64_t M, int N, int K,
                                                       const int* __restrict__ count, int rows_per_count) {
    constexpr int WN = 4 / (BM / 32);                  // waves across N
    constexpr int TN = GD_N / 16 / WN;                 // 16-wide tiles per wave across N
    constexpr int LA = BM * GD_K / 256;                // A elements per thread and K block
    __shared__ double As[BM * GD_LDS];
    __shared__ double Bs[GD_N * GD_LDS];
    const int g = blockIdx.z;
    const double* A = static_cast<const double*>(G.A[g]);
    const double* W = static_cast<const double*>(G.W[g]);
    const Epi& epi = G.epi[g];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)blockIdx.y * BM;
    const int n0 = blockIdx.x * GD_N;
    if (m0 >= M) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WN, wc = wave % WN;
    f64x4_t acc[2][TN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
    double ra[LA], rb[8];
    auto gload = [&](int k0) {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int c = tid + it * 256;          // rows x 32 k
            const int row = c >> 5, kk = c & 31;
            if (it < LA) {
                const int64_t gr = m0 + row;
                ra[it] = (gr < M && k0 + kk < K) ? A[gr * lda + k0 + kk] : 0.0;
            }
            const int gn = n0 + row;
            rb[it] = (gn < N && k0 + kk < K) ? W[(int64_t)gn * K + k0 + kk] : 0.0;
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int c = tid + it * 256;
            if (it < LA) As[(c >> 5) * GD_LDS + (c & 31)] = ra[it];
            Bs[(c >> 5) * GD_LDS + (c & 31)] = rb[it];
        }
    };
    gload(0);
    for (int k0 = 0; k0 < K; k0 += GD_K) {
        sstore();
        __syncthreads();
        if (k0 + GD_K < K) gload(k0 + GD_K);
#pragma unroll
        for (int kq = 0; kq < GD_K; kq += 4) {
            const int koff = kq + (lane >> 4);
            double a[2], b[TN];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[(wr * 32 + i * 16 + (lane & 15)) * GD_LDS + koff];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[(wc * 16 * TN + j * 16 + (lane & 15)) * GD_LDS + koff];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int c = n0 + wc * 16 * TN + j * 16 + (lane & 15);
        if (c >= N) continue;
        const auto p = epi.col(c);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
                if (row < M) epi.store(row, c, p, acc[i][j][r]);
            }
    }
}

// ------------------------------------------------------ BF16 tile autotuner
// Candidate tile configurations of gemm_bf16_t.  All of them accumulate each
// output over K in the same order, so the choice never changes a result; the
// fastest one for a (layer kind, M, N, K, networks) key is measured on the
// device at first use (outside stream capture) and kept in the model.
template <class Epi>
using Bf16Launch = void (*)(const Group<Epi>&, int64_t, int, int, int, const int*, int, hipStream_t);

template <int BM, int BN, int BK, int WM, int WN, int NB, class Epi>
static void bf16_launch(const Group<Epi>& P, int64_t M, int N, int K, int G, const int* count, int rpw,
                        hipStream_t s) {
    const dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)G);
    hipLaunchKernelGGL((gemm_bf16_t<BM, BN, BK, WM, WN, NB, Epi>), grid, dim3(64 * WM * WN), 0, s, P, (int64_t)K, M,
                       N, K, count, rpw);
}

static const char* const BF16_CFG_NAMES[] = {"128x128x64 waves 2x2 lds x1", "128x128x64 waves 2x2 lds x2",
                                            "128x128x64 waves 4x2 lds x2", "128x128x32 waves 2x2 lds x2"};
constexpr int BF16_NCFG = 4;

template <class Epi>
static Bf16Launch<Epi> bf16_candidate(int i) {
    switch (i) {
        case 0: return bf16_launch<128, 128, 64, 2, 2, 1, Epi>;
        case 1: return bf16_launch<128, 128, 64, 2, 2, 2, Epi>;
        case 2: return bf16_launch<128, 128, 64, 4, 2, 2, Epi>;
        default: return bf16_launch<128, 128, 32, 2, 2, 2, Epi>;
    }
}

template <class Epi>
static void launch_bf16_tuned(ns_model* m, int kind, const Group<Epi>& P, int64_t M, int N, int K, int G,
                              const int* count, int rpw, hipStream_t s) {
    const auto key = std::make_tuple(kind, M, N, K, G);
    auto it = m->tune.find(key);
    int best = 0;
    if (it != m->tune.end()) {
        best = it->second;
    } else {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        NS_HIP(hipStreamIsCapturing(s, &cs));
        if (cs == hipStreamCaptureStatusNone && !m->trace && getenv("NSMI_NO_AUTOTUNE") == nullptr) {
            hipEvent_t e0, e1;
            NS_HIP(hipEventCreate(&e0));
            NS_HIP(hipEventCreate(&e1));
            float best_ms = 1e30f;
            for (int c = 0; c < BF16_NCFG; ++c) {
                const auto fn = bf16_candidate<Epi>(c);
                fn(P, M, N, K, G, count, rpw, s);
                NS_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 3; ++r) fn(P, M, N, K, G, count, rpw, s);
                NS_HIP(hipEventRecord(e1, s));
                NS_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                NS_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) { best_ms = ms; best = c; }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            tune_cache_store(m, key, best);
        }
    }
    bf16_candidate<Epi>(best)(P, M, N, K, G, count, rpw, s);
}

// kinds 2 .. 17: one-kernel forward, 2 + split + 2 wide + 4 chi^2 mode + 8
// rounds of the sampler (rows a device count below the launch's maximum)
int tune_ncfg(int kind) { return kind < 2 ? BF16_NCFG : fused_ncfg_of(((kind - 2) >> 1) & 1, (kind - 2) & 1); }
const char* tune_cfg_name(int kind, int c) {
    return kind < 2 ? BF16_CFG_NAMES[c] : fused_cfg_name(((kind - 2) >> 1) & 1, (kind - 2) & 1, c);
}

std::string bf16_tuning_report(const ns_model* m) {
    std::string js = "{";
    bool first = true;
    for (const auto& kv : m->tune) {
        char tmp[256];
        const int kind = std::get<0>(kv.first);
        static const char* kinds[18] = {
            "bf16_hidden", "bf16_out", "fused_bf16", "fused_bf16x3", "fused_bf16", "fused_bf16x3",
            "fused_chi2_bf16", "fused_chi2_bf16x3", "fused_chi2_bf16", "fused_chi2_bf16x3",
            "fused_bf16 rounds", "fused_bf16x3 rounds", "fused_bf16 rounds", "fused_bf16x3 rounds",
            "fused_chi2_bf16 rounds", "fused_chi2_bf16x3 rounds", "fused_chi2_bf16 rounds", "fused_chi2_bf16x3 rounds"};
        const char* cfg = tune_cfg_name(kind, kv.second);
        snprintf(tmp, sizeof tmp, "%s\"%s M=%lld N=%d K=%d networks=%d\": \"%s\"", first ? "" : ", ", kinds[kind],
                 (long long)std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                 std::get<4>(kv.first), cfg);
        js += tmp;
        first = false;
    }
    return js + "}";
}

// ------------------------------------------------------------------ driver
static inline dim3 grid3(int64_t M, int N, int bm, int bn, int G) {
    return dim3((unsigned)((N + bn - 1) / bn), (unsigned)((M + bm - 1) / bm), (unsigned)G);
}

// Compute units of device dev (queried once per device).
int device_cus(int dev) {
    static int cus[64] = {0};
    if (dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// One FP64 GEMM launch: 64-row tiles, or 32-row tiles when the 64-row grid
// has fewer than eight workgroups per CU (a sampler round's few thousand
// rows: twice the workgroups fill the CUs more evenly); the two give
// identical results (gemm_f64_kernel).
template <class Epi>
static void launch_gemm_f64(const ns_model* m, const Group<Epi>& P, int64_t lda, int64_t rows, int N, int K, int G,
                            const int* count, int rpw, hipStream_t s) {
    const dim3 gr = grid3(rows, N, GD_M, GD_N, G);
    if ((int64_t)gr.x * gr.y * gr.z < 8 * (int64_t)device_cus(m->device))
        hipLaunchKernelGGL((gemm_f64_kernel<Epi, 32>), grid3(rows, N, 32, GD_N, G), dim3(256), 0, s, P, lda, rows, N,
                           K, count, rpw);
    else
        hipLaunchKernelGGL((gemm_f64_kernel<Epi, 64>), gr, dim3(256), 0, s, P, lda, rows, N, K, count, rpw);
}

template <class T, class OutT>
static void launch_first(ns_model* m, const int* nets, int G, const double* theta, int64_t ld, int64_t rows,
                         int rpw, OutT* act0, size_t act_stride, T* tsave, size_t save_stride, const int* count,
                         hipStream_t s) {
    FirstArgs<T, OutT> P{};
    const Net& n0 = *m->nets[nets[0]];
    for (int g = 0; g < G; ++g) {
        const Net& net = *m->nets[nets[g]];
        const Layer& l1 = *net.layers[0];
        if (sizeof(T) == 8) {
            P.W[g] = (const T*)l1.W64.p; P.b[g] = (const T*)l1.b64.p;
            P.beta[g] = (const T*)l1.beta64.p; P.gamma[g] = (const T*)l1.gamma64.p;
        } else {
            P.W[g] = (const T*)l1.W32.p; P.b[g] = (const T*)l1.b32.p;
            P.beta[g] = (const T*)l1.beta32.p; P.gamma[g] = (const T*)l1.gamma32.p;
        }
        P.shift[g] = net.in_shift.as<double>();
        P.scale[g] = net.in_scale.as<double>();
        P.out[g] = act0 + g * act_stride;
        P.tsave[g] = tsave ? tsave + g * save_stride : nullptr;
    }
    const int n_out = n0.dims[1], n_in = n0.dims[0];
    constexpr int CPT = sizeof(T) == 8 ? 4 : 8;
    NS_CHECK(n_out % CPT == 0 && n_out / CPT <= 256, NS_E_UNSUPPORTED,
             "first hidden width must be a multiple of 8 and at most 1024");
    dim3 g1((unsigned)((rows + FL_ROWS - 1) / FL_ROWS), 1, (unsigned)G);
    if (n_in <= 8)
        hipLaunchKernelGGL((first_layer_kernel<T, OutT, 8, CPT>), g1, dim3(256), 0, s, theta, ld, rows, rpw,
                           m->emu_src_d.as<int>(), m->emu_fix_d.as<double>(), m->znodes_d.as<double>(), n_in, n_out,
                           P, count);
    else
        hipLaunchKernelGGL((first_layer_kernel<T, OutT, 16, CPT>), g1, dim3(256), 0, s, theta, ld, rows, rpw,
                           m->emu_src_d.as<int>(), m->emu_fix_d.as<double>(), m->znodes_d.as<double>(), n_in, n_out,
                           P, count);
}

void emulator_forward(ns_model* m, const int* nets, int G, const double* theta, int64_t ld, int64_t B,
                      void* const* outs, int64_t ldo, const int* is_log, int prec, const int* count,
                      hipStream_t s, bool save_t) {
    NS_CHECK(G >= 1 && G <= MAXG, NS_E_UNSUPPORTED, "at most 4 networks per launch");
    const Net& net0 = *m->nets[nets[0]];
    for (int g = 1; g < G; ++g)
        NS_CHECK(m->nets[nets[g]]->dims == net0.dims, NS_E_SHAPE, "grouped networks must share their shapes");
    const int L = net0.n_layers;
    const int rpw = net0.out_mu_rows;                 // rows per walker
    const int64_t rows = B * rpw;
    NS_CHECK(net0.dims[0] <= 16, NS_E_UNSUPPORTED, "emulator with more than 16 inputs");
    if (!save_t && getenv("NSMI_NO_FUSED_MLP") == nullptr &&
        emulator_forward_fused(m, nets, G, theta, ld, B, outs, ldo, is_log, prec, count, s))
        return;
    if (!save_t && prec == NS_FP64 && G == 1 && nets[0] == 0 &&
        emulator_forward_f64_narrow(m, theta, ld, B, static_cast<double*>(outs[0]), ldo, is_log[0], nullptr, count,
                                    s))
        return;
    const size_t act_elem = prec == NS_FP64 ? 8 : (prec == NS_BF16 ? 2 : 4);
    size_t max_w = 0;
    for (int l = 1; l < L; ++l) max_w = std::max(max_w, (size_t)net0.dims[l]);
    const size_t act_stride = (size_t)rows * max_w;      // elements per network
    m->ws_act[0].ensure(G * act_stride * act_elem);
    m->ws_act[1].ensure(G * act_stride * act_elem);
    // pre-activation saves for the adjoint: slot (g, l-1) holds t of hidden layer l
    const size_t tsz = prec == NS_FP64 ? 8 : 4;
    const size_t save_stride = (size_t)(L - 1) * act_stride;   // elements per network
    if (save_t) m->ws_tsave.ensure(G * save_stride * tsz);
    char* tbase = save_t ? m->ws_tsave.as<char>() : nullptr;
    auto tslot = [&](int g, int slot) -> void* {
        return tbase ? (void*)(tbase + ((size_t)g * save_stride + (size_t)slot * act_stride) * tsz) : nullptr;
    };
    {
        TraceScope ts(m, s, "emu_first_layer");
        if (prec == NS_FP64)
            launch_first<double, double>(m, nets, G, theta, ld, rows, rpw, m->ws_act[0].as<double>(), act_stride,
                                         (double*)tslot(0, 0), save_stride, count, s);
        else if (prec == NS_BF16)
            launch_first<float, uint16_t>(m, nets, G, theta, ld, rows, rpw, m->ws_act[0].as<uint16_t>(),
                                          act_stride, (float*)tslot(0, 0), save_stride, count, s);
        else
            launch_first<float, float>(m, nets, G, theta, ld, rows, rpw, m->ws_act[0].as<float>(), act_stride,
                                       (float*)tslot(0, 0), save_stride, count, s);
        NS_HIP(hipGetLastError());
    }
    int cur = 0;
    for (int l = 1; l < L; ++l) {
        const int K = net0.dims[l], N = net0.dims[l + 1];
        const bool last = (l == L - 1);
        static const char* names[4][2] = {{"gemm_f64_hidden", "gemm_f64_out"}, {"gemm_f32_hidden", "gemm_f32_out"},
                                          {"gemm_bf16_hidden", "gemm_bf16_out"},
                                          {"gemm_bf16x3_hidden", "gemm_bf16x3_out"}};
        TraceScope ts(m, s, names[prec][last ? 1 : 0]);
        char* A0 = m->ws_act[cur].as<char>();
        char* D0 = m->ws_act[cur ^ 1].as<char>();
        auto A_of = [&](int g) { return (const void*)(A0 + g * act_stride * act_elem); };
        auto D_of = [&](int g) { return last ? outs[g] : (void*)(D0 + g * act_stride * act_elem); };
        if (prec == NS_FP64) {
            if (!last) {
                Group<EpiHidden<double, double>> P{};
                for (int g = 0; g < G; ++g) {
                    const Layer& ly = *m->nets[nets[g]]->layers[l];
                    P.A[g] = A_of(g); P.W[g] = ly.W64.p;
                    P.epi[g] = {ly.b64.as<double>(), ly.beta64.as<double>(), ly.gamma64.as<double>(),
                                (double*)D_of(g), (int64_t)N, (double*)tslot(g, l)};
                }
                launch_gemm_f64(m, P, (int64_t)K, rows, N, K, G, count, rpw, s);
            } else {
                Group<EpiOut<double>> P{};
                for (int g = 0; g < G; ++g) {
                    const Net& net = *m->nets[nets[g]];
                    const Layer& ly = *net.layers[l];
                    P.A[g] = A_of(g); P.W[g] = ly.W64.p;
                    P.epi[g] = {ly.b64.as<double>(), net.out_mu64.as<double>(), net.out_sigma64.as<double>(),
                                (double*)D_of(g), ldo, net.out_mu_rows, N, is_log[g]};
                }
                launch_gemm_f64(m, P, (int64_t)K, rows, N, K, G, count, rpw, s);
            }
        } else if (prec == NS_FP32) {
            NS_CHECK(K % GF_K == 0, NS_E_UNSUPPORTED, "FP32 MFMA layers need K % 32 == 0");
            const dim3 gr = grid3(rows, N, GB_M, GB_N, G);
            if (!last) {
                Group<EpiHidden<float, float>> P{};
                for (int g = 0; g < G; ++g) {
                    const Layer& ly = *m->nets[nets[g]]->layers[l];
                    P.A[g] = A_of(g); P.W[g] = ly.W32.p;
                    P.epi[g] = {ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(), (float*)D_of(g),
                                (int64_t)N, (float*)tslot(g, l)};
                }
                hipLaunchKernelGGL((gemm_f32_kernel<EpiHidden<float, float>>), gr, dim3(256), 0, s, P, (int64_t)K,
                                   rows, N, K, count, rpw);
            } else {
                Group<EpiOut<float>> P{};
                for (int g = 0; g < G; ++g) {
                    const Net& net = *m->nets[nets[g]];
                    const Layer& ly = *net.layers[l];
                    P.A[g] = A_of(g); P.W[g] = ly.W32.p;
                    P.epi[g] = {ly.b32.as<float>(), net.out_mu32.as<float>(), net.out_sigma32.as<float>(),
                                (float*)D_of(g), ldo, net.out_mu_rows, N, is_log[g]};
                }
                hipLaunchKernelGGL((gemm_f32_kernel<EpiOut<float>>), gr, dim3(256), 0, s, P, (int64_t)K, rows, N, K,
                                   count, rpw);
            }
        } else {
            NS_CHECK(K % GB_K == 0, NS_E_UNSUPPORTED, "BF16 MFMA layers need K % 64 == 0");
            const dim3 gr = grid3(rows, N, GB_M, GB_N, G);
            const bool x3 = prec == NS_BF16X3;
            if (!last) {
                if (x3) {
                    Group<EpiHidden<float, float>> P{};
                    for (int g = 0; g < G; ++g) {
                        const Layer& ly = *m->nets[nets[g]]->layers[l];
                        P.A[g] = A_of(g); P.W[g] = ly.Whi.p; P.Wl[g] = ly.Wlo.p;
                        P.epi[g] = {ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(),
                                    (float*)D_of(g), (int64_t)N, (float*)tslot(g, l)};
                    }
                    hipLaunchKernelGGL((gemm_bf16_kernel<1, EpiHidden<float, float>>), gr, dim3(256), 0, s, P,
                                       (int64_t)K, rows, N, K, count, rpw);
                } else {
                    Group<EpiHidden<float, uint16_t>> P{};
                    for (int g = 0; g < G; ++g) {
                        const Layer& ly = *m->nets[nets[g]]->layers[l];
                        P.A[g] = A_of(g); P.W[g] = ly.Whi.p; P.Wl[g] = ly.Wlo.p;
                        P.epi[g] = {ly.b32.as<float>(), ly.beta32.as<float>(), ly.gamma32.as<float>(),
                                    (uint16_t*)D_of(g), (int64_t)N, (float*)tslot(g, l)};
                    }
                    launch_bf16_tuned(m, 0, P, rows, N, K, G, count, rpw, s);
                }
            } else {
                Group<EpiOut<float>> P{};
                for (int g = 0; g < G; ++g) {
                    const Net& net = *m->nets[nets[g]];
                    const Layer& ly = *net.layers[l];
                    P.A[g] = A_of(g); P.W[g] = ly.Whi.p; P.Wl[g] = ly.Wlo.p;
                    P.epi[g] = {ly.b32.as<float>(), net.out_mu32.as<float>(), net.out_sigma32.as<float>(),
                                (float*)D_of(g), ldo, net.out_mu_rows, N, is_log[g]};
                }
                if (x3)
                    hipLaunchKernelGGL((gemm_bf16_kernel<1, EpiOut<float>>), gr, dim3(256), 0, s, P, (int64_t)K,
                                       rows, N, K, count, rpw);
                else
                    launch_bf16_tuned(m, 1, P, rows, N, K, G, count, rpw, s);
            }
        }
        NS_HIP(hipGetLastError());
        cur ^= 1;
    }
}

// ----------------------------------------------------------------- adjoint
// gx[g][r][k] = sum_n delta_1[g][r][n] W_1[n][k] / scale[k]: one wave per row.
template <class T>
__global__ __launch_bounds__(256) void first_layer_back_kernel(const T* __restrict__ delta, int64_t rows,
                                                               int n1, int n_in, FirstArgs<T, T> P, size_t dstride,
                                                               double* __restrict__ gx, const int* __restrict__ count,
                                                               int rpw) {
    const int g = blockIdx.z;
    int64_t nrows = rows;
    if (count) nrows = min<int64_t>(rows, (int64_t)(*count) * rpw);
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= nrows) return;
    const T* dr = delta + g * dstride + r * n1;
    const T* W = P.W[g];
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int n = lane; n < n1; n += 64) {
        const double dv = (double)dr[n];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < n_in) acc[k] = fma(dv, (double)W[(int64_t)n * n_in + k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < n_in) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) gx[((int64_t)g * rows + r) * n_in + k] = v / P.scale[g][k];
        }
    }
}

template <class T>
static void backward_impl(ns_model* m, const int* nets, int G, int64_t B, const int* count, hipStream_t s) {
    const bool f64 = sizeof(T) == 8;
    const Net& net0 = *m->nets[nets[0]];
    const int L = net0.n_layers;
    const int rpw = net0.out_mu_rows;
    const int64_t rows = B * rpw;
    size_t max_w = 0;
    for (int l = 1; l < L; ++l) max_w = std::max(max_w, (size_t)net0.dims[l]);
    const size_t act_stride = (size_t)rows * max_w;
    const size_t save_stride = (size_t)(L - 1) * act_stride;
    const size_t gstride = (size_t)rows * std::max(max_w, (size_t)net0.layers[L - 1]->n_pad);
    char* tbase = m->ws_tsave.as<char>();
    auto tslot = [&](int g, int slot) {
        return (const T*)(tbase + ((size_t)g * save_stride + (size_t)slot * act_stride) * sizeof(T));
    };
    int cur = 0;
    for (int l = L - 1; l >= 1; --l) {
        const int Kred = net0.layers[l]->n_pad, Nout = net0.dims[l];
        TraceScope ts(m, s, f64 ? "adj_gemm_f64" : "adj_gemm_f32");
        Group<EpiBack<T>> P{};
        for (int g = 0; g < G; ++g) {
            const Net& net = *m->nets[nets[g]];
            const Layer& ly = *net.layers[l];
            const Layer& lb = *net.layers[l - 1];
            P.A[g] = m->ws_gact[cur].as<T>() + g * gstride;
            P.W[g] = f64 ? ly.WT64.p : ly.WT32.p;
            P.epi[g] = {tslot(g, l - 1), (const T*)(f64 ? lb.beta64.p : lb.beta32.p),
                        (const T*)(f64 ? lb.gamma64.p : lb.gamma32.p), m->ws_gact[cur ^ 1].as<T>() + g * gstride,
                        (int64_t)Nout};
        }
        if constexpr (sizeof(T) == 8)
            launch_gemm_f64(m, P, (int64_t)Kred, rows, Nout, Kred, G, count, rpw, s);
        else
            hipLaunchKernelGGL((gemm_f32_kernel<EpiBack<T>>), grid3(rows, Nout, GB_M, GB_N, G), dim3(256), 0, s, P,
                               (int64_t)Kred, rows, Nout, Kred, count, rpw);
        NS_HIP(hipGetLastError());
        cur ^= 1;
    }
    FirstArgs<T, T> P{};
    for (int g = 0; g < G; ++g) {
        const Net& net = *m->nets[nets[g]];
        const Layer& l1 = *net.layers[0];
        P.W[g] = (const T*)(f64 ? l1.W64.p : l1.W32.p);
        P.scale[g] = net.in_scale.as<double>();
    }
    const int n_in = net0.dims[0];
    m->ws_gx.ensure((size_t)G * rows * n_in * sizeof(double));
    TraceScope ts(m, s, "adj_first_layer");
    hipLaunchKernelGGL(first_layer_back_kernel<T>, dim3((unsigned)((rows + 3) / 4), 1, (unsigned)G), dim3(256), 0, s,
                       m->ws_gact[cur].as<T>(), rows, net0.dims[1], n_in, P, gstride, m->ws_gx.as<double>(), count,
                       rpw);
    NS_HIP(hipGetLastError());
}

void emulator_backward(ns_model* m, const int* nets, int G, int64_t B, int prec, hipStream_t s) {
    if (prec == NS_FP64)
        backward_impl<double>(m, nets, G, B, nullptr, s);
    else
        backward_impl<float>(m, nets, G, B, nullptr, s);
}

}  // namespace nsmi
