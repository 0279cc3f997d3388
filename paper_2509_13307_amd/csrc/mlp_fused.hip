// Whole-network emulator forward in one kernel for the BF16-operand forms
// (NS_BF16 and the split form NS_BF16X3), Sec. 2.2 and 2.4 of the paper.
//
// One workgroup owns a block of R = 32 RT rows of one network.  The block's
// activations stay in LDS (BF16; hi and lo planes for the split form) from
// the first layer to the output layer.  Weights are never staged: each GEMM
// layer's weights are stored at model creation in MFMA fragment order (one
// 1 KB block per 32 output units x 16 inputs, lane l holding the 8 inputs
// 8 (l / 32) .. + 7 of unit l % 32; the blocks of one K step of a layer are
// contiguous, so the waves of all workgroups, which reach a K step together,
// spread their requests over the L2 channels), so a wave fetches the B operand of one
// v_mfma_f32_32x32x16_bf16 with a single coalesced 16-byte-per-lane load
// straight into registers, P K-steps ahead of its use.  No weight element is
// used by two waves of a workgroup, so LDS staging would bring no reuse.
//
// Wave w of NW = H / 64 owns output units [64 w, 64 w + 64) of each H-wide
// column block: 2 column tiles x RT row tiles of 32 x 32.  Layer 1
// (n_in <= 16 inputs) runs on the VALU in FP32.  Every output sees exactly
// the arithmetic of the layer-by-layer path (same K order, same per-
// accumulator MFMA sequence hi*hi, hi*lo, lo*hi, same epilogues), so both
// paths give identical results.  The split residual v - hi is an explicitly
// rounded subtraction: contracted with the activation's last multiply it
// would see the unrounded product, which the stored FP32 value of the
// layer-by-layer path does not.
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

constexpr int FM_MAXHID = 6;   // hidden GEMM layers supported
constexpr int FM_SLACK = 64;   // bytes behind the activation planes (read-ahead past a layer's last K step)

struct FusedNet {
    const float* W1; const float* b1; const float* be1; const float* ga1;   // first layer (FP32)
    const double* shift; const double* scale;
    const uint16_t* Wf;    // fragment-ordered BF16 hi weights of GEMM layers 2..L, layer l at l H^2
    const uint16_t* Wfl;   // ... lo parts (split form)
    const float* vec;      // hidden layer l: b, beta, gamma at l 3H + {0, H, 2H}; output bias after them
    const float* mu; const float* sigma;
    float* out; int is_log;
};

struct FusedArgs {
    FusedNet net[4];
    int n_hidden;        // hidden GEMM layers (network layers - 2)
    int n_in, N_out, mu_rows;
    int64_t ldo;
    int qg;              // output-block groups (grid z): each runs the hidden layers, then its share of the
                         // output layer's H-wide column blocks
    // chi^2 in the output epilogue instead of stored outputs (one network):
    // chi = 1 diagonal Gaussian, 2 cosmic-variance TT (see chi2_term)
    int chi;
    const double* cdata; const double* cw;  // data vector and inverse sigma (1) or (2l+1)/2 (2)
    double cst;                             // logL constant
    double* logl;                           // [rows] (one output group) ...
    double* part;                           // ... or [n_cb][H/32][rows] tile partials (several groups)
    const double* theta_s; int64_t ld_s; int d;   // support check of each walker
    const int* pk; const double* pa; const double* pb;
};

// One chi^2 term of output c with model value y (the FP32 output the store
// path would write): diagonal Gaussian ((data - y) / sigma)^2, or the
// cosmic-variance TT term (2l+1)/2 (ln C + data / C) with C = 10^y (Sec. 2.4
// of the paper); the same expressions as the staged kernels chi2_diag_kernel
// and cv_loglike_kernel.
__device__ __forceinline__ double chi2_term(int chi, double y, double data, double w) {
    if (chi == 1) {
        const double r = (data - y) * w;
        return r * r;
    }
    const double lc = 2.302585092994045684 * y;
    return w * (lc + data * exp(-lc));
}

// Sum of v[0..7] over the 32 lanes of each half wave, one row per value:
// afterwards lane l (l % 4 == 0) holds the sum for value (l & 31) >> 2.
// Partial sums of lanes c and c ^ m are added for m = 16, 8, 4, 2, 1 in this
// order, so every row's sum is the same tree over its 32 columns wherever
// the row sits.
__device__ __forceinline__ double tile_row_sums(const double (&v)[8], int lane) {
    // scalars and value selects (a select of two array elements can become a
    // select of their addresses, which keeps the array out of registers)
    double a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3], a4 = v[4], a5 = v[5], a6 = v[6], a7 = v[7];
    bool up = lane & 16;                                // 8 values -> 4
    double s0 = up ? a0 : a4, s1 = up ? a1 : a5, s2 = up ? a2 : a6, s3 = up ? a3 : a7;
    double k0 = up ? a4 : a0, k1 = up ? a5 : a1, k2 = up ? a6 : a2, k3 = up ? a7 : a3;
    a0 = k0 + __shfl_xor(s0, 16, 64);
    a1 = k1 + __shfl_xor(s1, 16, 64);
    a2 = k2 + __shfl_xor(s2, 16, 64);
    a3 = k3 + __shfl_xor(s3, 16, 64);
    up = lane & 8;                                      // 4 -> 2
    s0 = up ? a0 : a2; s1 = up ? a1 : a3;
    k0 = up ? a2 : a0; k1 = up ? a3 : a1;
    a0 = k0 + __shfl_xor(s0, 8, 64);
    a1 = k1 + __shfl_xor(s1, 8, 64);
    up = lane & 4;                                      // 2 -> 1
    s0 = up ? a0 : a1;
    k0 = up ? a1 : a0;
    a0 = k0 + __shfl_xor(s0, 4, 64);
    const double x = a0 + __shfl_xor(a0, 2, 64);
    return x + __shfl_xor(x, 1, 64);
}

bool fused_shape(const std::vector<int>& dims) {
    const int L = (int)dims.size() - 1;
    if (L < 3 || L - 2 > FM_MAXHID || dims[0] > 16) return false;
    const int H = dims[1];
    if (H != 128 && H != 512) return false;
    for (int l = 1; l < L; ++l)
        if (dims[l] != H) return false;
    return true;
}

template <int H, int RT, bool X3, int P, int CT, bool CHI>
__global__ __launch_bounds__(2 * H / CT) void mlp_fused_kernel(
    const double* __restrict__ theta, int64_t ld, int64_t rows, int rows_per_walker, const int* __restrict__ src,
    const double* __restrict__ fix, const double* __restrict__ znodes, FusedArgs A, const int* __restrict__ count) {
    constexpr int WC = 32 * CT;            // output units per wave and column block
    constexpr int NT = 64 * (H / WC);      // threads: one wave per WC units
    constexpr int R = 32 * RT;             // rows per workgroup
    constexpr int HS = H + 8;              // LDS row stride of an activation plane (elements)
    constexpr int KC = H / 16;             // K steps of one GEMM layer
    static_assert(KC % P == 0 && P % 2 == 0, "prefetch depth must be even and divide the K steps");
    static_assert(NT % H == 0, "threads must be a multiple of the hidden width");
    extern __shared__ __attribute__((aligned(16))) uint16_t fm_lds[];
    // [R][HS] hi (or only) plane, then the lo plane (split form), then
    // FM_SLACK bytes that the read-ahead of a layer's last K step may touch
    uint16_t* hs = fm_lds;
    uint16_t* hl = fm_lds + R * HS;
    // chi^2 mode: [R][H / 32] row sums per 32-unit tile, behind the slack
    constexpr int NTILE = H / 32;
    double* csl = reinterpret_cast<double*>(fm_lds + (X3 ? 2 : 1) * R * HS + FM_SLACK / 2);
    __shared__ float xs[R][16];
    __shared__ int zrow[R];                // redshift-node index of each row (row mod mu_rows)
    __shared__ int rowo[R];                // output offset of each row (row ldo), -1 beyond the live rows

    // Only the row blocks below the live row count (a device-side count in
    // the sampler's rounds) carry work: the first nlb G qg workgroups in
    // launch order take them, the rest leave at once.  Launch order deals
    // workgroups round-robin to the 8 XCDs, so the live ones span every XCD
    // however few they are; within them the order is XCD-aware, each XCD
    // receiving a contiguous run of (output group, network, row block).
    int64_t nrows = rows;
    if (count) nrows = min<int64_t>(rows, (int64_t)(*count) * rows_per_walker);
    const int nlb = (int)((nrows + R - 1) / R);            // live row blocks per network
    const int live = nlb * gridDim.y * gridDim.z;
    int lin = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (lin >= live) return;
    if ((live & 7) == 0) lin = (lin & 7) * (live >> 3) + (lin >> 3);
    const int g = (lin / nlb) % gridDim.y, rb = lin % nlb, q = lin / (nlb * gridDim.y);
    const FusedNet N = A.net[g];           // by value: the fields live in scalar registers
    const int64_t r0 = (int64_t)rb * R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_in = A.n_in, n_hidden = A.n_hidden, N_out = A.N_out;
    const int nvalid = (int)min<int64_t>(R, nrows - r0);   // live rows of this block
    // output group q takes the column blocks [ob0, ob0 + nob); its segments
    // are the hidden layers, then those blocks (v -> real segment seg_of(v))
    const int ncb = (N_out + H - 1) / H;
    const int per = (ncb + A.qg - 1) / A.qg, ob0 = q * per;
    const int nob = min(ncb, ob0 + per) - ob0;
    if (nob <= 0) return;
    const int nseg = n_hidden + nob;
    if (tid < R) {
        zrow[tid] = A.mu_rows > 1 ? (int)((r0 + tid) % A.mu_rows) : 0;
        rowo[tid] = tid < nvalid ? tid * (int)A.ldo : -1;
    }
    if (CHI)
        for (int e = tid; e < R * NTILE; e += NT) csl[e] = 0.0;
    // layer-1 weights of this thread's unit (see first_layer), requested
    // before the barrier so that they arrive with the inputs
    const int c1 = tid % H;
    float w1[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w1[k] = k < n_in ? N.W1[c1 * n_in + k] : 0.0f;
    const float b1 = N.b1[c1], be1 = N.be1[c1], ga1 = N.ga1[c1];
    // chi^2 mode, one output group: whether the row's walker lies in the
    // prior's support (the first threads, one row each), while the last
    // threads bring in the inputs below
    bool row_ok = true;
    if (CHI && A.qg == 1 && tid < nvalid)
        row_ok = in_support(A.theta_s + (r0 + tid) / rows_per_walker * A.ld_s, A.d, A.pk, A.pa, A.pb);

    // ---- layer-1 inputs (normalised parameters) into LDS, element e by
    // thread NT - 1 - e
    for (int e = NT - 1 - tid; e < R * n_in; e += NT) {
        const int rr = e / n_in, k = e % n_in;
        const int64_t r = r0 + rr;
        float v = 0.0f;
        if (r < nrows) {
            const int64_t w = r / rows_per_walker;
            const int zi = (int)(r % rows_per_walker);
            const int s = src[k];
            const double t = s >= 0 ? theta[w * ld + s] : (s == SRC_ZNODE ? znodes[zi] : fix[k]);
            v = (float)((t - N.shift[k]) / N.scale[k]);
        }
        xs[rr][k] = v;
    }

    // ---- layer 1 (FP32 VALU, the arithmetic of the layer-by-layer path).  NT
    // is a multiple of H: each thread keeps one unit c (weights in registers)
    // for rows tid / H, tid / H + NT / H, ..., FU of them at a time, so that
    // their LDS reads, sums and activations overlap (one row after the other
    // would wait on each row's reads and exp in turn)
    auto first_layer = [&]() {
        constexpr int RS = NT / H, NR = R / RS, FU = NR < 8 ? NR : 8;
        static_assert(R % RS == 0 && NR % FU == 0, "rows per thread");
        const int c = c1, rr0 = tid / H;
        for (int j0 = 0; j0 < NR; j0 += FU) {
            float acc[FU];
#pragma unroll
            for (int j = 0; j < FU; ++j) acc[j] = b1;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < n_in)
#pragma unroll
                    for (int j = 0; j < FU; ++j) acc[j] += w1[k] * xs[rr0 + (j0 + j) * RS][k];
#pragma unroll
            for (int j = 0; j < FU; ++j) {
                const int rr = rr0 + (j0 + j) * RS;
                const float v = gated<float>(acc[j], be1, ga1);
                const uint16_t hi = f2bf(v);
                hs[rr * HS + c] = hi;
                if (X3) hl[rr * HS + c] = bf16_lo(v, hi);
            }
        }
    };

    // ---- GEMM stages: hidden layers, then the output layer's H-wide column
    // blocks; stage s = (segment s / KC, K step s % KC).  Loads and MFMAs are
    // unconditional within the live segments (stages past the end re-read the
    // last one, the partly live last tile computes on valid addresses and
    // stores its live units only), so the weight prefetch stays in flight
    // across segments, epilogues and barriers.
    auto seg_of = [&](int v) { return v < n_hidden ? v : v + ob0; };
    // fragment block (kc, nt) of a layer with nt_l 32-unit tiles sits at
    // (kc nt_l + nt) 512 elements: one K step of a layer is contiguous.  The
    // wave's fragments of K step 0 of segment v start at the (wave-uniform)
    // element offset seg_frag(v); successive K steps lie `stride` apart, and
    // lane l reads elements 8 l .. 8 l + 7 of each 512-element block.
    const int nt_out = ncb * H / 32;
    auto seg_frag = [&](int v, int& stride) -> size_t {
        const int seg = seg_of(v);
        const bool hid = seg < n_hidden;
        int nb = (hid ? 0 : (seg - n_hidden) * H) + wave * WC;
        if (!hid && nb >= N_out) nb = 0;
        stride = (hid ? H / 32 : nt_out) * 512;
        return (size_t)min(seg, n_hidden) * H * H + (size_t)(nb / 32) * 512;
    };
    const unsigned lane8 = (unsigned)lane * 8u;
    bf16x8_t rh[P][CT], rl[P][CT];
    auto fetch = [&](size_t off, bf16x8_t (&bh)[CT], bf16x8_t (&bl)[CT]) {
        const uint16_t* wh = N.Wf + off;
        const uint16_t* wl = N.Wfl + off;
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            bh[j] = *reinterpret_cast<const bf16x8_t*>(wh + j * 512 + lane8);
            if (X3) bl[j] = *reinterpret_cast<const bf16x8_t*>(wl + j * 512 + lane8);
        }
    };
    f32x16_t acc[RT][CT];
    auto zero_acc = [&]() {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    };
    zero_acc();
    // segment state of this wave: v, its fragments (cur, scur), the next
    // segment's (nxt, snext) and the epilogue vectors of v
    int v = 0, scur = 0, snext = 0;
    size_t cur = seg_frag(0, scur), nxt = 0;
    // the first stages' weights, requested behind layer 1 (in flight across
    // it they would hold registers that layer 1 needs)
    auto prefetch = [&]() {
#pragma unroll
        for (int u = 0; u < P; ++u) fetch(cur + (size_t)u * scur, rh[u], rl[u]);
    };

    // A operands (activation fragments) of one K step, double-buffered: the
    // LDS reads of step kc + 1 are issued before the MFMAs of step kc.  The
    // read-ahead past the end of a run of K steps is discarded (the next run
    // reads its first step again); past a layer's last step it lands in the
    // next row's first elements or, for the last row, in the slack behind the
    // planes.
    // Element offsets of this lane's A rows, one per row tile and plane.  The
    // empty asm makes them opaque: folded into each read, the lo plane's
    // offset (beyond the 64 KiB immediate range of an LDS read) would need a
    // register per K step, which the compiler precomputes and spills.
    int aoff[RT][2];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        aoff[i][0] = i * 32 * HS + (lane & 31) * HS + (lane >> 5) * 8;
        aoff[i][1] = aoff[i][0] + R * HS;
        asm volatile("" : "+v"(aoff[i][0]), "+v"(aoff[i][1]));
    }
    bf16x8_t ah[2][RT], al[2][RT];
    auto read_a = [&](int kc, bf16x8_t (&xh)[RT], bf16x8_t (&xl)[RT]) {
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            xh[i] = *reinterpret_cast<const bf16x8_t*>(&fm_lds[aoff[i][0] + kc * 16]);
            if (X3) xl[i] = *reinterpret_cast<const bf16x8_t*>(&fm_lds[aoff[i][1] + kc * 16]);
        }
    };
    float e0[CT], e1[CT], e2[CT];
    double cd[CT], cv[CT];                 // chi^2 mode: data and weight of the wave's output units
    // start of segment v: the next segment's fragments (the stage P steps past
    // the last K step is in the next segment, or, after the last segment, the
    // last stage again) and the epilogue vectors, loaded while the K steps run
    auto seg_begin = [&]() {
        snext = 0;
        nxt = v + 1 < nseg ? seg_frag(v + 1, snext) : cur + (size_t)(KC - 1) * scur;
        const int seg = seg_of(v);
        const bool hid = seg < n_hidden;
        const int nb = (hid ? 0 : (seg - n_hidden) * H) + wave * WC;
        const float* vb = N.vec + (size_t)seg * 3 * H;             // hidden: b, beta, gamma
        const float* bo = N.vec + (size_t)n_hidden * 3 * H;        // output: bias
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int c = nb + j * 32 + (lane & 31);
            if (hid) {
                e0[j] = vb[c]; e1[j] = vb[H + c]; e2[j] = vb[2 * H + c];
            } else {
                const int cc = min(c, N_out - 1);
                e0[j] = bo[cc]; e1[j] = N.sigma[cc]; e2[j] = N.mu[cc];
                if (CHI) { cd[j] = A.cdata[cc]; cv[j] = A.cw[cc]; }
            }
        }
    };
    // K steps [k0, k1) of segment v
    auto ksteps = [&](int k0, int k1) {
        read_a(k0, ah[0], al[0]);
        for (int kc0 = k0; kc0 < k1; kc0 += P) {
            const bool last = kc0 + P >= KC;
            const size_t fb = last ? nxt : cur + (size_t)(kc0 + P) * scur;
            const int fs = last ? snext : scur;
#pragma unroll
            for (int u = 0; u < P; ++u) {
                // slot u feeds this step's MFMAs first and is then refilled with
                // the stage P steps ahead: no register copies, loads stay in flight
                const int kc = kc0 + u;
                const bf16x8_t (&bh)[CT] = rh[u];
                const bf16x8_t (&bl)[CT] = rl[u];
                // k0 and P are even, so kc and u have the same parity
                read_a(kc + 1, ah[(u + 1) & 1], al[(u + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
                const bf16x8_t (&xh)[RT] = ah[u & 1];
                const bf16x8_t (&xl)[RT] = al[u & 1];
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int j = 0; j < CT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bh[j], acc[i][j], 0, 0, 0);
                if (X3) {
#pragma unroll
                    for (int i = 0; i < RT; ++i)
#pragma unroll
                        for (int j = 0; j < CT; ++j) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bl[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[i], bh[j], acc[i][j], 0, 0, 0);
                        }
                }
                fetch(fb + (size_t)u * fs, rh[u], rl[u]);
                // keep the refill right behind the MFMAs that read the slot:
                // left to itself the scheduler sinks these loads to the end of
                // the unrolled steps, next to their first use, and the
                // prefetch distance collapses to a few instructions
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto seg_end = [&]() {
        cur = nxt;
        scur = snext;
        ++v;
        zero_acc();
    };
    // epilogue of hidden segment v: gated activation of this wave's units, the
    // BF16 (hi, lo) split into LDS
    auto hidden_epi = [&]() {
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int c = wave * WC + j * 32 + (lane & 31);
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = i * 32 + (lane >> 5) * 4 + (r >> 2) * 8 + (r & 3);
                    const float v = gated<float>(acc[i][j][r] + e0[j], e1[j], e2[j]);
                    const uint16_t hi = f2bf(v);
                    hs[row * HS + c] = hi;
                    if (X3) hl[row * HS + c] = bf16_lo(v, hi);
                }
        }
    };
    // epilogue of output segment v (units nb + ...): mean + sigma y, 10^ for
    // log-emulated outputs, stored to the live rows
    // chi^2 mode: per 32-unit tile, the row sums of the terms (tile_row_sums)
    // are added to the tile's LDS slot of the row, block after block
    auto chi_epi = [&](int nb) {
        const bool is_log = N.is_log;
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int c = nb + j * 32 + (lane & 31);
            const bool live_c = c < N_out;
            const float bb = e0[j], sg = e1[j], mu0 = e2[j];
            const double dat = cd[j], cw = cv[j];
            const int tile = (wave * WC + j * 32) / 32;
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int hf = 0; hf < 2; ++hf) {                // accumulator rows r = 8 hf .. 8 hf + 7
                    // the eight terms side by side: one uniform branch per
                    // kind of term, and the dead units' terms (computed on
                    // the last unit's data) dropped by a select, so that the
                    // exponentials and FP64 products of the rows overlap
                    float y[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) y[k] = mu0 + sg * (acc[i][j][8 * hf + k] + bb);
                    if (is_log)
#pragma unroll
                        for (int k = 0; k < 8; ++k) y[k] = exp10_of<float>(y[k]);
                    double v[8];
                    if (A.chi == 1) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) v[k] = chi2_term(1, (double)y[k], dat, cw);
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) v[k] = chi2_term(2, (double)y[k], dat, cw);
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = live_c ? v[k] : 0.0;
                    const double sum = tile_row_sums(v, lane);
                    if ((lane & 3) == 0) {
                        const int rr = 8 * hf + ((lane & 31) >> 2);
                        const int row = i * 32 + (lane >> 5) * 4 + (rr >> 2) * 8 + (rr & 3);
                        csl[row * NTILE + tile] += sum;
                    }
                }
        }
    };
    auto output_epi = [&](int nb) {
        const bool zdep = A.mu_rows > 1, is_log = N.is_log;
        // every row of the block live and one mean row: row addresses are
        // wave-uniform, the lane adds its column and its 4-row group
        const bool plain = nvalid == R && !zdep;
        const int64_t ldo = A.ldo;
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int c = nb + j * 32 + (lane & 31);
            if (c >= N_out) continue;
            const float bb = e0[j], sg = e1[j], mu0 = e2[j];
            if (plain) {
                const unsigned lofs = (unsigned)((lane >> 5) * 4 * ldo + c);
                float* ob = N.out + r0 * ldo;
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        float* rowp = ob + (int64_t)(i * 32 + (r >> 2) * 8 + (r & 3)) * ldo;
                        float y = mu0 + sg * (acc[i][j][r] + bb);
                        if (is_log) y = exp10_of<float>(y);
                        rowp[lofs] = y;
                    }
            } else {
                float* ob = N.out + r0 * ldo + c;
                // row offsets come from LDS: kept in registers they would hold
                // 64-bit addresses live across the whole stage loop.  The lane's
                // first row is opaque to the compiler, so that the reads use one
                // base register and immediate offsets instead of an address per
                // row that it would precompute and spill.
                int lr0 = (lane >> 5) * 4;
                asm volatile("" : "+v"(lr0));
#pragma unroll
                for (int i = 0; i < RT; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int lr = lr0 + i * 32 + (r >> 2) * 8 + (r & 3);
                        const int ro = rowo[lr];
                        if (ro < 0) continue;
                        const float m = zdep ? N.mu[zrow[lr] * N_out + c] : mu0;
                        float y = m + sg * (acc[i][j][r] + bb);
                        if (is_log) y = exp10_of<float>(y);
                        ob[ro] = y;
                    }
            }
        }
        // drain this segment's stores here (vmcnt(0) only), so that the next
        // K-step run starts with nothing but the weight prefetch in flight and
        // its waits can count just those loads
        __builtin_amdgcn_s_waitcnt(0x0F70);
    };
    // output unit base of segment v for this wave; a wave whose units of an
    // output block all lie past N_out has none in the later blocks either
    auto out_nb = [&]() { return (seg_of(v) - n_hidden) * H + wave * WC; };

    __syncthreads();
    first_layer();
    prefetch();
    __syncthreads();
    for (; v < n_hidden; ) {
        seg_begin();
        ksteps(0, KC);
        __syncthreads();                                   // every wave done reading this layer's input
        hidden_epi();
        __syncthreads();                                   // next layer's input complete
        seg_end();
    }
    // output column blocks: no barriers, the waves run free
    for (; v < nseg; ) {
        const int nb = out_nb();
        if (nb >= N_out) break;
        seg_begin();
        ksteps(0, KC);
        if (CHI) chi_epi(nb);
        else output_epi(nb);
        seg_end();
    }
    if (!CHI) return;
    // chi^2 mode: every wave's tile sums are in LDS; per row, tiles in order
    // (one output group: logL), or each tile's sum as a partial of its block
    __syncthreads();
    for (int t = tid; t < R * NTILE; t += NT) {
        const int rr = t / NTILE, tile = t % NTILE;
        if (rr >= nvalid || A.qg == 1) continue;
        A.part[((int64_t)ob0 * NTILE + tile) * nrows + r0 + rr] = csl[t];
    }
    if (A.qg == 1 && tid < nvalid) {
        double sum = csl[tid * NTILE];
        for (int tile = 1; tile < NTILE; ++tile) sum += csl[tid * NTILE + tile];
        A.logl[r0 + tid] = !row_ok ? -INFINITY : (A.chi == 1 ? -0.5 * sum + A.cst : A.cst - sum);
    }
}

// Several output groups: logL of each row from the tile partials of every
// output block, tiles outer and blocks inner, in the order of one group's
// LDS slots (each slot adds its tile's block sums in block order, then the
// tiles are summed), so the value does not depend on the launch shape.
__global__ __launch_bounds__(256) void chi2_fused_finish_kernel(const double* __restrict__ part, int nblk,
                                                                int ntile, int64_t rows, FusedArgs A,
                                                                const int* __restrict__ count) {
    int64_t nr = rows;
    if (count) nr = min<int64_t>(rows, (int64_t)(*count));
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double sum = 0.0;
    for (int tile = 0; tile < ntile; ++tile) {
        double ts = part[(int64_t)tile * nr + r];
        for (int b = 1; b < nblk; ++b) ts += part[((int64_t)b * ntile + tile) * nr + r];
        sum = tile == 0 ? ts : sum + ts;
    }
    const bool ok = in_support(A.theta_s + r * A.ld_s, A.d, A.pk, A.pa, A.pb);
    A.logl[r] = !ok ? -INFINITY : (A.chi == 1 ? -0.5 * sum + A.cst : A.cst - sum);
}

template <int H, int RT, bool X3, int P, int CT, bool CHI>
static void launch_fused(ns_model* m, const FusedArgs& A, const double* theta, int64_t ld, int64_t rows, int rpw,
                         int G, const int* count, hipStream_t s) {
    constexpr int R = 32 * RT;
    constexpr int NT = 64 * (H / (32 * CT));
    const size_t base = (size_t)(X3 ? 2 : 1) * R * (H + 8) * sizeof(uint16_t) + FM_SLACK;
    const size_t slots = (size_t)R * (H / 32) * sizeof(double);     // chi^2 mode's row sums
    const size_t smem = base + (CHI ? slots : 0);
    const auto kern = mlp_fused_kernel<H, RT, X3, P, CT, CHI>;
    const int rtc = RT == 2 ? 0 : (RT == 1 ? 1 : 2);
    const int bit = ((((int)CHI * 3 + rtc) * 2 + (H == 512)) * 2 + X3) * 8 + (CT == 1) * 4 +
                    (P == 2 ? 0 : (P == 4 ? 1 : 2));
    if (smem > 64 * 1024 && !m->fused_attr_set[bit]) {
        NS_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        m->fused_attr_set[bit] = true;
    }
    const dim3 grid((unsigned)((rows + R - 1) / R), (unsigned)G, (unsigned)A.qg);
    hipLaunchKernelGGL(kern, grid, dim3(NT), smem, s, theta, ld, rows, rpw, m->emu_src_d.as<int>(),
                       m->emu_fix_d.as<double>(), m->znodes_d.as<double>(), A, count);
}

// Candidate launch shapes: 64-row blocks with waves of 32 or 64 output units
// and 2-8 K steps of weight prefetch, 32-row blocks (twice the workgroups for
// small batches of one network) and, for plain BF16 (one activation plane),
// 128-row blocks (half the weight traffic per row); and, for small batches,
// shapes whose workgroups each take one of the output layer's H-wide column
// blocks after running the hidden layers themselves ("output blocks split"):
// more workgroups and a shorter serial chain per workgroup, at the price of
// the hidden layers computed once per column block.  All candidates give
// identical results.
using FusedLaunch = void (*)(ns_model*, const FusedArgs&, const double*, int64_t, int64_t, int, int, const int*,
                             hipStream_t);
struct FusedCfg { FusedLaunch fn, fn_chi; const char* name; bool split_out; };
template <int H, int RT, bool X3, int P, int CT>
constexpr FusedCfg fcfg(const char* name, bool split_out = false) {
    return {launch_fused<H, RT, X3, P, CT, false>, launch_fused<H, RT, X3, P, CT, true>, name, split_out};
}
constexpr int FUSED_NCFG = 10;                    // table width; the split form at width 512 has 8 candidates
static int fused_ncfg(int h512, int x3) { return x3 && h512 ? 8 : 10; }
static const FusedCfg FUSED_CFGS[2][2][FUSED_NCFG] = {
    {   // H = 128
        {fcfg<128, 2, false, 4, 2>("fused 2 waves x 64 units, prefetch 4"),
         fcfg<128, 2, false, 8, 2>("fused 2 waves x 64 units, prefetch 8"),
         fcfg<128, 2, false, 4, 1>("fused 4 waves x 32 units, prefetch 4"),
         fcfg<128, 2, false, 8, 1>("fused 4 waves x 32 units, prefetch 8"),
         fcfg<128, 1, false, 4, 1>("fused 4 waves x 32 units, 32 rows, prefetch 4"),
         fcfg<128, 1, false, 8, 1>("fused 4 waves x 32 units, 32 rows, prefetch 8"),
         fcfg<128, 4, false, 4, 1>("fused 4 waves x 32 units, 128 rows, prefetch 4"),
         fcfg<128, 4, false, 4, 2>("fused 2 waves x 64 units, 128 rows, prefetch 4"),
         fcfg<128, 1, false, 4, 1>("fused 4 waves x 32 units, 32 rows, prefetch 4, output blocks split", true),
         fcfg<128, 1, false, 8, 1>("fused 4 waves x 32 units, 32 rows, prefetch 8, output blocks split", true)},
        {fcfg<128, 2, true, 2, 2>("fused split 2 waves x 64 units, prefetch 2"),
         fcfg<128, 2, true, 4, 2>("fused split 2 waves x 64 units, prefetch 4"),
         fcfg<128, 2, true, 2, 1>("fused split 4 waves x 32 units, prefetch 2"),
         fcfg<128, 2, true, 4, 1>("fused split 4 waves x 32 units, prefetch 4"),
         fcfg<128, 1, true, 2, 1>("fused split 4 waves x 32 units, 32 rows, prefetch 2"),
         fcfg<128, 1, true, 4, 1>("fused split 4 waves x 32 units, 32 rows, prefetch 4"),
         fcfg<128, 1, true, 8, 1>("fused split 4 waves x 32 units, 32 rows, prefetch 8"),
         fcfg<128, 2, true, 8, 1>("fused split 4 waves x 32 units, prefetch 8"),
         fcfg<128, 1, true, 2, 1>("fused split 4 waves x 32 units, 32 rows, prefetch 2, output blocks split", true),
         fcfg<128, 1, true, 8, 1>("fused split 4 waves x 32 units, 32 rows, prefetch 8, output blocks split", true)},
    },
    {   // H = 512
        {fcfg<512, 2, false, 4, 2>("fused 8 waves x 64 units, prefetch 4"),
         fcfg<512, 2, false, 8, 2>("fused 8 waves x 64 units, prefetch 8"),
         fcfg<512, 2, false, 4, 1>("fused 16 waves x 32 units, prefetch 4"),
         fcfg<512, 2, false, 8, 1>("fused 16 waves x 32 units, prefetch 8"),
         fcfg<512, 1, false, 4, 1>("fused 16 waves x 32 units, 32 rows, prefetch 4"),
         fcfg<512, 1, false, 8, 1>("fused 16 waves x 32 units, 32 rows, prefetch 8"),
         fcfg<512, 4, false, 4, 1>("fused 16 waves x 32 units, 128 rows, prefetch 4"),
         fcfg<512, 4, false, 4, 2>("fused 8 waves x 64 units, 128 rows, prefetch 4"),
         fcfg<512, 1, false, 4, 1>("fused 16 waves x 32 units, 32 rows, prefetch 4, output blocks split", true),
         fcfg<512, 1, false, 8, 1>("fused 16 waves x 32 units, 32 rows, prefetch 8, output blocks split", true)},
        {fcfg<512, 2, true, 2, 2>("fused split 8 waves x 64 units, prefetch 2"),
         fcfg<512, 2, true, 4, 2>("fused split 8 waves x 64 units, prefetch 4"),
         fcfg<512, 2, true, 2, 1>("fused split 16 waves x 32 units, prefetch 2"),
         fcfg<512, 2, true, 4, 1>("fused split 16 waves x 32 units, prefetch 4"),
         fcfg<512, 1, true, 2, 1>("fused split 16 waves x 32 units, 32 rows, prefetch 2"),
         fcfg<512, 1, true, 4, 1>("fused split 16 waves x 32 units, 32 rows, prefetch 4"),
         fcfg<512, 1, true, 2, 1>("fused split 16 waves x 32 units, 32 rows, prefetch 2, output blocks split", true),
         fcfg<512, 1, true, 4, 1>("fused split 16 waves x 32 units, 32 rows, prefetch 4, output blocks split", true)},
    },
};

const char* fused_cfg_name(int h512, int x3, int c) { return FUSED_CFGS[h512][x3][c].name; }
int fused_ncfg_of(int h512, int x3) { return fused_ncfg(h512, x3); }

// Returns false (and launches nothing) when the networks have no fragment-
// ordered weights (shape outside fused_shape) or the form is not BF16-operand.
// Shared by the store and chi^2 modes: the one-kernel arguments of networks
// nets[0..G) (outputs and flags filled in by the caller).
static FusedArgs fused_args(ns_model* m, const int* nets, int G) {
    const Net& n0 = *m->nets[nets[0]];
    const int L = n0.n_layers;
    FusedArgs A{};
    A.n_hidden = L - 2;
    A.n_in = n0.dims[0];
    A.N_out = n0.dims[L];
    A.mu_rows = n0.out_mu_rows;
    A.qg = 1;
    for (int g = 0; g < G; ++g) {
        const Net& net = *m->nets[nets[g]];
        FusedNet& F = A.net[g];
        const Layer& l1 = *net.layers[0];
        F.W1 = l1.W32.as<float>(); F.b1 = l1.b32.as<float>(); F.be1 = l1.beta32.as<float>(); F.ga1 = l1.gamma32.as<float>();
        F.shift = net.in_shift.as<double>();
        F.scale = net.in_scale.as<double>();
        F.Wf = net.Wf.as<uint16_t>();
        F.Wfl = net.Wfl.as<uint16_t>();
        F.vec = net.fvec.as<float>();
        F.mu = net.out_mu32.as<float>(); F.sigma = net.out_sigma32.as<float>();
    }
    return A;
}

// Launch shape (measured once per (form, mode, rows, outputs, width, networks)
// outside stream capture and tracing, or pinned / read from the cache), then
// the launch; in chi^2 mode with the output blocks split over workgroups, the
// finishing sum of the tile partials.
static void fused_run(ns_model* m, const FusedArgs& A, int H, bool x3, int G, const double* theta, int64_t ld,
                      int64_t B, const int* count, hipStream_t s) {
    const Net& n0 = *m->nets[0];
    const int rpw = n0.out_mu_rows;
    const int64_t rows = B * rpw;
    const int h512 = H == 512;
    const FusedCfg* cfgs = FUSED_CFGS[h512][x3];
    const int ncb = (A.N_out + H - 1) / H;
    // candidate c with its output-block grouping, on `nr` rows given on the
    // host (tuning) or on the launch's rows and device count
    auto run_rows = [&](int c, int64_t nr, const int* cnt) {
        FusedArgs Ac = A;
        Ac.qg = cfgs[c].split_out ? ncb : 1;
        (Ac.chi ? cfgs[c].fn_chi : cfgs[c].fn)(m, Ac, theta, ld, nr, rpw, G, cnt, s);
        if (Ac.chi && Ac.qg > 1)
            hipLaunchKernelGGL(chi2_fused_finish_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s,
                               (const double*)Ac.part, ncb, H / 32, nr, Ac, cnt);
    };
    auto run = [&](int c) { run_rows(c, rows, count); };
    // a sampler round's launch (rows a device count) is tuned apart from an
    // exact batch of the same maximum: the initial live points and the rounds
    // of 2 x speculation x k walkers can share one row count
    const auto key = std::make_tuple(2 + (int)x3 + 2 * h512 + (A.chi ? 4 : 0) + (count ? 8 : 0), rows, A.N_out, H, G);
    int best = 0;
    auto it = m->tune.find(key);
    const char* forced = getenv("NSMI_FUSED_CFG");      // pin one candidate (tests of every shape)
    if (forced != nullptr) {
        best = std::min(std::max(atoi(forced), 0), fused_ncfg(h512, x3) - 1);
    } else if (it != m->tune.end()) {
        best = it->second;
    } else {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        NS_HIP(hipStreamIsCapturing(s, &cs));
        if (cs == hipStreamCaptureStatusNone && !m->trace && !m->noalloc_call && getenv("NSMI_NO_AUTOTUNE") == nullptr) {
            hipEvent_t e0, e1;
            NS_HIP(hipEventCreate(&e0));
            NS_HIP(hipEventCreate(&e1));
            // two interleaved passes over the candidates, the faster pass counts
            // (clock and cache state drift between candidates of one pass).  A
            // launch whose live rows are a device count (the sampler's rounds,
            // whose batches vary from round to round below the maximum `rows`)
            // is timed at an eighth, a quarter and half of `rows` and ranked by
            // the sum: the maximum needs every walker to propose its full
            // speculation at both bracket ends, and most rounds carry a few
            // tenths of it (cosmic shear, 500 walkers: 2 600 of 10 000 rows
            // on average, where 32-row tiles take 57 us per call and the
            // 64-row tiles that win at the maximum 83 us).
            const int ncfg = fused_ncfg(h512, x3);
            const int64_t sizes[3] = {std::max<int64_t>(rpw, rows / 8 / rpw * rpw),
                                      std::max<int64_t>(rpw, rows / 4 / rpw * rpw),
                                      std::max<int64_t>(rpw, rows / 2 / rpw * rpw)};
            const int nsz = count ? 3 : 1;
            float tot_ms[FUSED_NCFG];
            for (int c = 0; c < ncfg; ++c) tot_ms[c] = 0.f;
            for (int z = 0; z < nsz; ++z) {
                const int64_t nr = count ? sizes[z] : rows;
                float best_ms[FUSED_NCFG];
                for (int c = 0; c < ncfg; ++c) best_ms[c] = 1e30f;
                for (int pass = 0; pass < 2; ++pass)
                    for (int c = 0; c < ncfg; ++c) {
                        run_rows(c, nr, nullptr);
                        NS_HIP(hipEventRecord(e0, s));
                        for (int r = 0; r < 4; ++r) run_rows(c, nr, nullptr);
                        NS_HIP(hipEventRecord(e1, s));
                        NS_HIP(hipEventSynchronize(e1));
                        float ms = 0.f;
                        NS_HIP(hipEventElapsedTime(&ms, e0, e1));
                        best_ms[c] = std::min(best_ms[c], ms);
                    }
                for (int c = 0; c < ncfg; ++c) tot_ms[c] += best_ms[c];
            }
            for (int c = 1; c < ncfg; ++c)
                if (tot_ms[c] < tot_ms[best]) best = c;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            tune_cache_store(m, key, best);
        }
    }
    TraceScope ts(m, s, A.chi ? (x3 ? "mlp_fused_chi2_bf16x3" : "mlp_fused_chi2_bf16")
                              : (x3 ? "mlp_fused_bf16x3" : "mlp_fused_bf16"));
    run(best);
    NS_HIP(hipGetLastError());
}

// Returns false (and launches nothing) when the networks have no fragment-
// ordered weights (shape outside fused_shape) or the form is not BF16-operand.
bool emulator_forward_fused(ns_model* m, const int* nets, int G, const double* theta, int64_t ld, int64_t B,
                            void* const* outs, int64_t ldo, const int* is_log, int prec, const int* count,
                            hipStream_t s) {
    if (prec != NS_BF16 && prec != NS_BF16X3) return false;
    const Net& n0 = *m->nets[nets[0]];
    if (!n0.fused) return false;
    FusedArgs A = fused_args(m, nets, G);
    A.ldo = ldo;
    for (int g = 0; g < G; ++g) {
        A.net[g].out = static_cast<float*>(outs[g]);
        A.net[g].is_log = is_log[g];
    }
    fused_run(m, A, n0.dims[1], prec == NS_BF16X3, G, theta, ld, B, count, s);
    return true;
}

size_t chi2_fused_part_bytes(const ns_model* m, int64_t B) {
    const Net& n0 = *m->nets[0];
    const int H = n0.dims[1], ncb = (n0.dims[n0.n_layers] + H - 1) / H;
    return (size_t)ncb * (H / 32) * std::max<int64_t>(B, 1) * sizeof(double);
}

bool emulator_chi2_fused(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, int prec,
                         const int* count, hipStream_t s, double* part) {
    if (prec != NS_BF16 && prec != NS_BF16X3) return false;
    if (m->kind != NS_MODEL_CMB_DIAG && m->kind != NS_MODEL_CMB_CV) return false;
    if (m->nets.size() != 1 || !m->nets[0]->fused || m->nets[0]->out_mu_rows != 1) return false;
    // staged chi^2 (tests compare the two), or the layer-by-layer forward
    if (getenv("NSMI_NO_FUSED_CHI2") != nullptr || getenv("NSMI_NO_FUSED_MLP") != nullptr) return false;
    // The cosmic-variance terms take an FP64 exp each, which in the epilogue
    // lengthens every workgroup's serial path by about 10 us, against a staged
    // kernel that spreads them over the whole GPU in 10 us (1 000 rows) to
    // 20 us (4 096 rows): fused only from FUSED_CV_MIN_ROWS rows (measured:
    // 4 096 rows 104 instead of 111 us, 1 000 rows 79 instead of 66 us).  A
    // fixed rule, not a timing, so that which sum a batch gets (they differ
    // in the last bits) does not depend on the machine.
    constexpr int64_t FUSED_CV_MIN_ROWS = 3072;
    if (m->kind == NS_MODEL_CMB_CV && B < FUSED_CV_MIN_ROWS) return false;
    const int id0 = 0;
    const Net& n0 = *m->nets[0];
    const int H = n0.dims[1];
    FusedArgs A = fused_args(m, &id0, 1);
    const bool cv = m->kind == NS_MODEL_CMB_CV;
    A.net[0].out = nullptr;
    A.net[0].is_log = cv ? 0 : m->spec_log[0];             // the cosmic-variance terms take log10 C_l
    A.chi = cv ? 2 : 1;
    A.cdata = m->data.as<double>();
    A.cw = cv ? m->cv_halfk.as<double>() : m->inv_sigma.as<double>();
    A.cst = m->logl_const;
    A.logl = logl;
    if (!part) {
        m->ws_chi.ensure(chi2_fused_part_bytes(m, B));
        part = m->ws_chi.as<double>();
    }
    A.part = part;
    A.theta_s = theta;
    A.ld_s = ld;
    A.d = m->d;
    A.pk = m->prior_kind.as<int>();
    A.pa = m->prior_a.as<double>();
    A.pb = m->prior_b.as<double>();
    fused_run(m, A, H, prec == NS_BF16X3, 1, theta, ld, B, count, s);
    return true;
}

}  // namespace nsmi
