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
};

ShearGeom shear_geom(const ns_model* m);

// Inclusive prefix sum over the block (blockDim = 256) of NV per-thread values;
// reverse = true sums from the last thread down.  buf holds NV x 256 doubles.
template <int NV>
__device__ void block_scan(double (&v)[NV], double* buf, bool reverse) {
    const int t = threadIdx.x;
    const int src = reverse ? 255 - t : t;
#pragma unroll
    for (int q = 0; q < NV; ++q) buf[q * 256 + src] = v[q];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        double add[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) add[q] = src >= off ? buf[q * 256 + src - off] : 0.0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NV; ++q) buf[q * 256 + src] += add[q];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = buf[q * 256 + src];
    __syncthreads();
}

}  // namespace nsmi
