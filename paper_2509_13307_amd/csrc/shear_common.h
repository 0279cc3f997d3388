// Constants and block-level helpers shared by the cosmic-shear forward and
// adjoint kernels (App. A of the paper).
#pragma once

#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

constexpr double C_KM_S = 299792.458;                 // speed of light [km/s]
constexpr double C1_RHOCR = 5e-14 * 2.77536627e11;    // C1 rho_cr of the NLA model (Eq. A4)
constexpr double GROWTH_INDEX = 0.55;
constexpr double LN10 = 2.302585092994045684;
constexpr int MAXB = 10;                              // tomographic bins supported by the kernels

struct ShearGeom {
    int n_a, n_z, n_k, n_ell, n_bins, n_pairs;
    double a_min, da, zmax, k_min, k_max, u0, du, nz_sigma;
    double u1;        // log10 k_max
};

ShearGeom shear_geom(const ns_model* m);

// Inclusive prefix sum over the block (blockDim = 256) of NV per-thread values;
// reverse = true sums from the last thread down.  Each wave scans with
// shuffles, then adds the totals of the waves before it (buf: NV x 4 doubles).
template <int NV>
__device__ void block_scan(double (&v)[NV], double* buf, bool reverse) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double y = reverse ? __shfl_down(x, off, 64) : __shfl_up(x, off, 64);
            if (reverse ? lane + off < 64 : lane >= off) x += y;
        }
        v[q] = x;
    }
    if (lane == (reverse ? 0 : 63))
#pragma unroll
        for (int q = 0; q < NV; ++q) buf[q * 4 + wid] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double pre = 0.0;
        for (int k = 0; k < 4; ++k)
            if (reverse ? k > wid : k < wid) pre += buf[q * 4 + k];
        v[q] += pre;
    }
    __syncthreads();
}

}  // namespace nsmi
