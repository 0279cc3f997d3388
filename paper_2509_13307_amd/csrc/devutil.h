// Device-side helpers shared by the kernels of libnsmi (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsmi {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4_t;

// round-to-nearest-even float -> bf16 bits
// FP32 -> BF16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Low BF16 part of the split v = hi + lo, hi = f2bf(v): lo = f2bf(v - hi) with
// the subtraction kept apart from whatever product produced v (a fused
// multiply-subtract would see the unrounded product instead of v).
__device__ __forceinline__ uint16_t bf16_lo(float v, uint16_t hi) {
#pragma clang fp contract(off)
    return f2bf(v - bf2f(hi));
}

template <class T> __device__ __forceinline__ T sigmoid(T u) { return T(1) / (T(1) + exp(-u)); }
// FP32: hardware exp2 and reciprocal (about 1 ulp each)
template <> __device__ __forceinline__ float sigmoid<float>(float u) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u * -1.44269504088896341f));
}
// 10^y (output transform of log10-emulated spectra)
template <class T> __device__ __forceinline__ T exp10_of(T y) { return exp(y * T(2.302585092994045684)); }
// FP32: 10^y = 2^(p_hi + p_lo) with p_hi = fl(y log2 10) and p_lo its rounding
// residual (plus the residual of log2 10 itself), so that the argument
// rounding (up to |y log2 10| 2^-24) does not reach the result; then
// 2^p_lo = 1 + p_lo ln 2 to first order (|p_lo| < 1e-5)
template <> __device__ __forceinline__ float exp10_of<float>(float y) {
    const float c_hi = 3.321928024291992f, c_lo = 7.059536955011936e-08f;
    const float p_hi = y * c_hi;
    const float p_lo = fmaf(y, c_hi, -p_hi) + y * c_lo;
    return __builtin_amdgcn_exp2f(p_hi) * fmaf(p_lo, 0.6931471824645996f, 1.0f);
}

// gated activation (gamma + (1 - gamma) sigmoid(beta t)) t
template <class T> __device__ __forceinline__ T gated(T t, T beta, T gamma) {
    return (gamma + (T(1) - gamma) * sigmoid<T>(beta * t)) * t;
}

// ----------------------------------------------------------- reductions
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <class T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// block-wide sum; `red` is LDS scratch of >= blockDim.x/64 elements
template <class T> __device__ T block_sum(T v, T* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = T(0);
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------- Philox4x64-10
struct u64x4 { uint64_t x[4]; };

__device__ __forceinline__ u64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    u64x4 o;
    o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}

__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// draw q of the sequence (c1, c2, c3) under key (seed, stream): word q mod 4
// of Philox block q / 4 (picked by selects, not by a run-time array index,
// which would put the block in scratch memory)
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t stream, uint64_t c1,
                                                 uint64_t c2, uint64_t c3, uint64_t q) {
    const u64x4 b = philox4x64(q >> 2, c1, c2, c3, seed, stream);
    const int r = (int)(q & 3);
    return u01(r == 0 ? b.x[0] : r == 1 ? b.x[1] : r == 2 ? b.x[2] : b.x[3]);
}

// draws q and q + 1 (q even) of the sequence: one Philox block
__device__ __forceinline__ void philox_uniform_pair(uint64_t seed, uint64_t stream, uint64_t c1, uint64_t c2,
                                                    uint64_t c3, uint64_t q, double& a, double& b) {
    const u64x4 x = philox4x64(q >> 2, c1, c2, c3, seed, stream);
    const bool hi = (q & 2) != 0;
    a = u01(hi ? x.x[2] : x.x[0]);
    b = u01(hi ? x.x[3] : x.x[1]);
}

}  // namespace nsmi
