// BF16 MFMA GEMM template for gfx950:  Y[M x N] = epi(X[M x K] W^T),
// X [M x K] BF16 row-major (lda), W [N x K] BF16 row-major (K-contiguous).
//
// Workgroup tile BM x BN from WM x WN waves; each wave owns a
// (BM/WM) x (BN/WN) block of v_mfma_f32_32x32x16_bf16 tiles.  K advances in
// steps of BK staged through LDS (row stride BK + 8 elements: conflict-free
// 16-byte reads).  The next K step is fetched into registers while the
// current one feeds the MFMAs; NBUF = 2 double-buffers the LDS (one barrier
// per step), NBUF = 1 trades that barrier for half the LDS and so more
// resident workgroups.  Tiles are remapped so that the 8 XCDs each receive a
// contiguous run of tiles (shared activation rows stay in one XCD's L2).
//
// Lane layout of v_mfma_f32_32x32x16_bf16 (checked on the device): lane l
// supplies A[l % 32][8 (l / 32) + i] and B[8 (l / 32) + i][l % 32], i < 8;
// accumulator register r of lane l holds D[4 (l / 32) + 8 (r / 4) + r % 4][l % 32].
#pragma once

#include "devutil.h"

namespace nsmi {

struct TileId { int g, ty, tx; };
__device__ __forceinline__ TileId xcd_tile() {
    const int nx = gridDim.x, ny = gridDim.y;
    const int total = nx * ny * gridDim.z;
    int i = (blockIdx.z * ny + blockIdx.y) * nx + blockIdx.x;
    if ((total & 7) == 0) i = (i & 7) * (total >> 3) + (i >> 3);
    TileId t;
    t.tx = i % nx;
    t.ty = (i / nx) % ny;
    t.g = i / (nx * ny);
    return t;
}

// Per-launch operands: up to 4 networks of equal shape (blockIdx.z selects).
template <class Epi> struct Group {
    const void* A[4];
    const void* W[4];
    const void* Wl[4];
    Epi epi[4];
};

template <int BM, int BN, int BK, int WM, int WN, int NBUF>
struct Bf16Tile {
    static constexpr int NT = 64 * WM * WN;             // threads per workgroup
    static constexpr int LDSK = BK + 8;                 // LDS row stride (elements)
    static constexpr int TI = BM / WM / 32, TJ = BN / WN / 32;
    static constexpr int CA = BM * BK / 8 / NT;         // 16-byte chunks per thread, A
    static constexpr int CB = BN * BK / 8 / NT;         // 16-byte chunks per thread, B
    static constexpr int STAGE = (BM + BN) * LDSK;      // elements per LDS stage
    static constexpr int LDS_BYTES = NBUF * STAGE * 2;
    static_assert(BM % (32 * WM) == 0 && BN % (32 * WN) == 0, "wave tiles must be multiples of 32");
    static_assert((BM * BK / 8) % NT == 0 && (BN * BK / 8) % NT == 0, "stage must split evenly");
    static_assert(BK % 16 == 0, "BK must be a multiple of 16");
};

template <int BM, int BN, int BK, int WM, int WN, int NBUF, class Epi>
__global__ __launch_bounds__(64 * WM * WN) void gemm_bf16_t(Group<Epi> G, int64_t lda, int64_t M, int N, int K,
                                                            const int* __restrict__ count, int rows_per_count) {
    using T = Bf16Tile<BM, BN, BK, WM, WN, NBUF>;
    constexpr int LDSK = T::LDSK, TI = T::TI, TJ = T::TJ, CA = T::CA, CB = T::CB;
    constexpr int KC = BK / 8;                          // 16-byte chunks per row per stage
    __shared__ __attribute__((aligned(16))) uint16_t lds[NBUF * T::STAGE];
    const TileId tile = xcd_tile();
    const int g = tile.g;
    const uint16_t* A = static_cast<const uint16_t*>(G.A[g]);
    const uint16_t* W = static_cast<const uint16_t*>(G.W[g]);
    const Epi& epi = G.epi[g];
    if (count) M = min<int64_t>(M, (int64_t)(*count) * rows_per_count);
    const int64_t m0 = (int64_t)tile.ty * BM;
    const int n0 = tile.tx * BN;
    if (m0 >= M) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / WN, wc = wave % WN;

    f32x16_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    uint4 ra[CA], rb[CB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int it = 0; it < CA; ++it) {
            const int c = tid + it * T::NT;
            const int row = c / KC, kc = (c % KC) * 8;
            const int64_t gr = m0 + row;
            ra[it] = gr < M ? *reinterpret_cast<const uint4*>(A + gr * lda + k0 + kc) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int it = 0; it < CB; ++it) {
            const int c = tid + it * T::NT;
            const int row = c / KC, kc = (c % KC) * 8;
            const int gn = n0 + row;
            rb[it] = gn < N ? *reinterpret_cast<const uint4*>(W + (int64_t)gn * K + k0 + kc) : make_uint4(0, 0, 0, 0);
        }
    };
    auto stash = [&](uint16_t* st) {
#pragma unroll
        for (int it = 0; it < CA; ++it) {
            const int c = tid + it * T::NT;
            *reinterpret_cast<uint4*>(&st[(c / KC) * LDSK + (c % KC) * 8]) = ra[it];
        }
#pragma unroll
        for (int it = 0; it < CB; ++it) {
            const int c = tid + it * T::NT;
            *reinterpret_cast<uint4*>(&st[(BM + c / KC) * LDSK + (c % KC) * 8]) = rb[it];
        }
    };
    auto compute = [&](const uint16_t* st) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int koff = kk + (lane >> 5) * 8;
            bf16x8_t a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i)
                a[i] = *reinterpret_cast<const bf16x8_t*>(
                    &st[(wr * (BM / WM) + i * 32 + (lane & 31)) * LDSK + koff]);
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                b[j] = *reinterpret_cast<const bf16x8_t*>(
                    &st[(BM + wc * (BN / WN) + j * 32 + (lane & 31)) * LDSK + koff]);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };

    const int nk = K / BK;
    fetch(0);
    if (NBUF == 2) {
        stash(lds);
        __syncthreads();
        for (int t = 0; t < nk; ++t) {
            uint16_t* cur = lds + (t & 1) * T::STAGE;
            uint16_t* nxt = lds + ((t + 1) & 1) * T::STAGE;
            if (t + 1 < nk) fetch((t + 1) * BK);
            compute(cur);
            if (t + 1 < nk) stash(nxt);
            __syncthreads();
        }
    } else {
        for (int t = 0; t < nk; ++t) {
            stash(lds);
            __syncthreads();
            if (t + 1 < nk) fetch((t + 1) * BK);
            compute(lds);
            __syncthreads();
        }
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
        const int c = n0 + wc * (BN / WN) + j * 32 + (lane & 31);
        if (c >= N) continue;
        const auto p = epi.col(c);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wr * (BM / WM) + i * 32 + (lane >> 5) * 4 + (r >> 2) * 8 + (r & 3);
                if (row < M) epi.store(row, c, p, acc[i][j][r]);
            }
    }
}

}  // namespace nsmi
