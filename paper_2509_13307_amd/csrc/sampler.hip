// Nested slice sampling on the device (Sec. 2.1-2.2 of the paper; slice
// sampling after Neal 2003, as adopted by the paper's GPU nested sampler).
//
// Slice step.  Each walker runs a hit-and-run slice state machine in the unit
// cube.  Per step s = 1..n_inner it draws a direction v = L zeta (zeta by
// Box-Muller from Philox draws 0..2d-1) and an offset r (draw 2d), brackets
// [t_L, t_R] = [-r, 1-r], steps each end out while it is inside the constraint
// (at most 10 times per end; the two ends in the same rounds, since they are
// independent), then shrinks with draws 2d+1, 2d+2, ... until a
// point inside is found (accept), the bracket is narrower than 1e-12 or 200
// shrinks were rejected (stall: the point is kept).  "Inside" means
// u in [0,1]^d and logL(T(u)) > L*; proposals outside the cube cost no
// likelihood evaluation.
//
// The walkers advance in rounds: slice_advance_kernel applies the previous
// round's likelihood values and runs every walker forward until it needs a
// new evaluation, appending that proposal (in the cube and mapped through the
// prior) to a compacted batch; the batched likelihood then runs on the
// compacted rows only.  The batch size and the count of unfinished walkers
// live in two counter pairs used by rounds of alternating parity, so each
// round's advance clears the pair of the next round and no separate reset
// launch is needed.  Every random number is addressed by (walker, step,
// draw), so the result does not depend on the order of the compacted rows.
//
// Nested-sampling bookkeeping (k-deletion, the running evidence) runs in
// single-workgroup kernels; the host only polls a termination flag.  The
// final log Z, H and the replicate log Z for the error bar (FP64) are
// parallel over the dead points: prefix sums of the log-shrinkages, then a
// max-shifted sum of exponentials.
#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

enum { ST_NEWSTEP = 0, ST_OUT = 1, ST_SHRINK = 3, ST_DONE = 4 };
constexpr int MAX_EXPAND = 10;
constexpr int MAX_SHRINK = 200;
constexpr double STALL_WIDTH = 1e-12;
constexpr int MAX_DIM = 64;

struct SliceState {
    double* u;        // [k x d] walker positions (caller buffer)
    double* logl;     // [k]
    double* v;        // [k x d] current direction
    double* tl;       // [k]
    double* tr;       // [k]
    double* tp;       // [k] t of the pending proposal
    int* st;          // [k] phase
    int* step;        // [k] current step (1-based)
    int* q;           // [k] next draw index
    int* ne;          // [k] left-end expansions (stepping out; -1 once that end is final) /
                      //     rejected shrinks
    int* ne2;         // [k] right-end expansions (stepping out; -1 once final)
    int* pend;        // [k] compact slot of the pending (left-end or shrink) proposal, -1 none
    int* pend2;       // [k] compact slot of the pending right-end proposal, -1 none
    int* n_evals;     // [k]
    int* n_stalls;    // [k]
    double* xc;       // [2k x d] compacted proposals (unit cube)
    int* cidx;        // [2k] walker of each compact slot
    double* llc;      // [2k] likelihood of each compact slot
    int* ccount;      // [2] compact batch size of the rounds of even / odd parity
    int* active;      // [2] walkers not done after the advance of such a round
};

__global__ void slice_init_kernel(SliceState S, int64_t k) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w == 0) {
        S.ccount[0] = S.ccount[1] = 0;
        S.active[0] = S.active[1] = 0;
    }
    if (w >= k) return;
    S.st[w] = ST_NEWSTEP;
    S.step[w] = 0;
    S.pend[w] = -1;
    S.pend2[w] = -1;
    S.n_evals[w] = 0;
    S.n_stalls[w] = 0;
}

// One wave per walker, lane i = coordinate i (d <= 64).  The walker's phase
// state is uniform across the wave and kept in registers; the direction draw
// (lane i: Box-Muller of draws 2i, 2i+1), the product with L (lane i sums row
// i in column order, as a serial loop would) and the proposal are spread over
// the lanes, so every value is bitwise that of one thread per walker.
__global__ __launch_bounds__(256) void slice_advance_kernel(SliceState S, int64_t k, int d,
                                                            const double* __restrict__ lstar_p,
                                                            const double* __restrict__ L, int n_inner,
                                                            uint64_t seed, uint64_t iter, int par,
                                                            const int* __restrict__ pk, const double* __restrict__ pa,
                                                            const double* __restrict__ pb,
                                                            double* __restrict__ thc) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    // the counters of the other parity were last read by the previous round's
    // likelihood, which has finished: clear them for the next round
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.ccount[par ^ 1] = 0;
        S.active[par ^ 1] = 0;
    }
    // the walker's state is requested first (the idle waves of the last block
    // read walker k - 1 and leave after the barrier); the direction factor
    // goes to LDS meanwhile, so that the row products of a new direction
    // read LDS instead of waiting on one global load per column
    const int64_t wr = w < k ? w : k - 1;
    const bool act = lane < d;
    const double lstar = *lstar_p;
    int st = S.st[wr], step = S.step[wr], q = S.q[wr], ne = S.ne[wr], pend = S.pend[wr];
    int ne2 = S.ne2[wr], pend2 = S.pend2[wr];
    int nev = S.n_evals[wr], nst = S.n_stalls[wr];
    double tl = S.tl[wr], tr = S.tr[wr], tp = S.tp[wr], logl = S.logl[wr];
    double ui = act ? S.u[wr * d + lane] : 0.0, vi = act ? S.v[wr * d + lane] : 0.0;
    __shared__ double Ls[MAX_DIM * MAX_DIM];
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) Ls[e] = L[e];
    __syncthreads();
    if (w >= k) return;                                   // whole waves
    bool moved = false;
    // outcome of a shrink proposal at t = tp
    auto shrink = [&](bool inside, double ll) {
        if (inside) {
            ui = __dadd_rn(ui, __dmul_rn(tp, vi));
            logl = ll;
            moved = true;
            st = ST_NEWSTEP;
        } else {
            if (tp < 0.0) tl = tp; else tr = tp;
            ne += 1;
            if (tr - tl < STALL_WIDTH || ne >= MAX_SHRINK) {
                nst += 1;
                st = ST_NEWSTEP;
            }
        }
    };
    // the point at t along the direction: its compact slot, or -1 outside the
    // unit cube (no evaluation: outside the constraint)
    auto propose = [&](double t) -> int {
        const double xi = __dadd_rn(ui, __dmul_rn(t, vi));
        const bool inbox = __ballot(act && !((xi >= 0.0) && (xi <= 1.0))) == 0;
        if (!inbox) return -1;
        int slot = 0;
        if (lane == 0) slot = atomicAdd(S.ccount + par, 1);
        slot = __shfl(slot, 0, 64);
        if (act) {
            S.xc[(int64_t)slot * d + lane] = xi;
            thc[(int64_t)slot * d + lane] = prior_map(xi, pk[lane], pa[lane], pb[lane]);
        }
        if (lane == 0) S.cidx[slot] = (int)w;
        return slot;
    };
    // last round's evaluations
    if (st == ST_OUT) {
        if (pend >= 0) {
            const double ll = S.llc[pend];
            pend = -1;
            nev += 1;
            if (ll > lstar) { tl -= 1.0; ne += 1; } else ne = -1;
        }
        if (pend2 >= 0) {
            const double ll = S.llc[pend2];
            pend2 = -1;
            nev += 1;
            if (ll > lstar) { tr += 1.0; ne2 += 1; } else ne2 = -1;
        }
    } else if (pend >= 0) {
        const double ll = S.llc[pend];
        pend = -1;
        nev += 1;
        shrink(ll > lstar, ll);
    }
    while (true) {
        if (st == ST_DONE) break;
        if (st == ST_NEWSTEP) {
            if (step >= n_inner) { st = ST_DONE; break; }
            const int s = ++step;
            double z = 0.0;
            if (act) {
                const double u1 = philox_uniform(seed, 0, (uint64_t)w, (uint64_t)s, iter, 2 * lane);
                const double u2 = philox_uniform(seed, 0, (uint64_t)w, (uint64_t)s, iter, 2 * lane + 1);
                z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
            }
            double acc = 0.0;
            for (int j = 0; j < d; ++j) {
                const double zj = __shfl(z, j, 64);
                if (act && j <= lane) acc = __dadd_rn(acc, __dmul_rn(Ls[lane * d + j], zj));
            }
            vi = act ? acc : 0.0;
            const double r = philox_uniform(seed, 0, (uint64_t)w, (uint64_t)s, iter, 2 * d);
            tl = -r;
            tr = 1.0 - r;
            q = 2 * d + 1;
            ne = 0;
            ne2 = 0;
            st = ST_OUT;
            continue;
        }
        if (st == ST_OUT) {
            // both ends step out at once, each proposing its current end until
            // that point is outside the slice or the cube or it has expanded
            // MAX_EXPAND times; the ends do not interact, so the evaluations
            // and the final bracket are those of stepping out one end after
            // the other
            if (ne >= 0) {
                if (ne >= MAX_EXPAND) ne = -1;
                else if ((pend = propose(tl)) < 0) ne = -1;
            }
            if (ne2 >= 0) {
                if (ne2 >= MAX_EXPAND) ne2 = -1;
                else if ((pend2 = propose(tr)) < 0) ne2 = -1;
            }
            if (pend >= 0 || pend2 >= 0) break;
            st = ST_SHRINK;
            ne = 0;
            continue;
        }
        const int qq = q++;
        const double U = philox_uniform(seed, 0, (uint64_t)w, (uint64_t)step, iter, (uint64_t)qq);
        tp = __dadd_rn(tl, __dmul_rn(U, __dsub_rn(tr, tl)));
        if ((pend = propose(tp)) < 0) {
            shrink(false, -INFINITY);
            continue;
        }
        break;
    }
    if (act) {
        if (moved) S.u[w * d + lane] = ui;
        S.v[w * d + lane] = vi;
    }
    if (lane == 0) {
        S.st[w] = st; S.step[w] = step; S.q[w] = q; S.ne[w] = ne; S.pend[w] = pend;
        S.ne2[w] = ne2; S.pend2[w] = pend2;
        S.n_evals[w] = nev; S.n_stalls[w] = nst;
        S.tl[w] = tl; S.tr[w] = tr; S.tp[w] = tp; S.logl[w] = logl;
        if (st != ST_DONE) atomicAdd(S.active + par, 1);
    }
}

// ------------------------------------------------------------- NS kernels
struct NSState {
    double logx;      // log X after the deaths recorded so far
    double logz;      // running log Z of the dead points
    double lstar;     // current threshold
    double live_term; // log(X mean_live L)
    int64_t n_dead;
    int64_t n_evals;
    int64_t n_stalls;
    int stop;
};

__device__ __forceinline__ double logaddexp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = fmax(a, b);
    return m + log1p(exp(-fabs(a - b)));
}

// Bitonic sort of (logl, index) for n <= 4096 in one workgroup of 1024 threads;
// then the k lowest die: dead-point records and the running evidence (FP64).
__global__ __launch_bounds__(1024) void ns_select_kernel(const double* __restrict__ logl,
                                                         const double* __restrict__ u, int n, int k, int d,
                                                         int* __restrict__ order, NSState* __restrict__ S,
                                                         double* __restrict__ dead_logl, int* __restrict__ dead_n,
                                                         double* __restrict__ dead_u, int64_t dead_cap,
                                                         int record) {
    __shared__ double key[4096];
    __shared__ int idx[4096];
    int N2 = 1;
    while (N2 < n) N2 <<= 1;
    for (int i = threadIdx.x; i < N2; i += blockDim.x) {
        key[i] = i < n ? logl[i] : INFINITY;
        idx[i] = i < n ? i : 0x7fffffff;
    }
    __syncthreads();
    for (int size = 2; size <= N2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < N2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const double ki = key[i], kj = key[j];
                    const int ii = idx[i], ij = idx[j];
                    // (logl, index) lexicographic; NaN sorts after +inf
                    const bool gt = (ki > kj) || (ki == kj && ii > ij) || (isnan(ki) && !isnan(kj));
                    if (gt == up) {
                        key[i] = kj; key[j] = ki;
                        idx[i] = ij; idx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) order[i] = idx[i];
    __syncthreads();
    if (!record) return;
    const int64_t base = S->n_dead;
    for (int e = threadIdx.x; e < k * d; e += blockDim.x) {
        const int j = e / d, c = e % d;
        if (base + j < dead_cap) dead_u[(base + j) * d + c] = u[(int64_t)idx[j] * d + c];
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x)
        if (base + j < dead_cap) {
            dead_logl[base + j] = key[j];
            dead_n[base + j] = n - j;
        }
    // The running log Z is the serial chain of log-additions in death order
    // (the stopping rule reads it).  Its per-death terms 1/n_j and
    // log(1 - e^{-1/n_j}) depend on the rank only: the workgroup tabulates
    // them for a block of ranks, then one thread runs the chain over the block.
    constexpr int QB = 512;
    __shared__ double qinv[QB], qlog[QB];
    double logx = S->logx, logz = S->logz;
    for (int j0 = 0; j0 < k; j0 += QB) {
        __syncthreads();
        for (int j = j0 + threadIdx.x; j < min(k, j0 + QB); j += blockDim.x) {
            const double inv = 1.0 / (double)(n - j);
            qinv[j - j0] = inv;
            qlog[j - j0] = log(-expm1(-inv));
        }
        __syncthreads();
        if (threadIdx.x == 0)
#pragma unroll 8
            for (int j = j0; j < min(k, j0 + QB); ++j) {
                const double logw = logx + qlog[j - j0];
                logz = logaddexp(logz, key[j] + logw);
                logx -= qinv[j - j0];
            }
    }
    if (threadIdx.x == 0) {
        S->logx = logx;
        S->logz = logz;
        S->lstar = key[k - 1];
        S->n_dead = base + k;
    }
}

// Live-point covariance (1/(n-1)), trace jitter, Cholesky (lower, row-major).
// The live points pass through LDS in chunks of whole points (coalesced
// loads); each mean and each covariance entry is still one thread's sum over
// the points in index order.
__global__ __launch_bounds__(256) void ns_dircov_kernel(const double* __restrict__ u, int n, int d,
                                                        double* __restrict__ L) {
    constexpr int STAGE = 3072;                            // doubles of staged points
    constexpr int EPT = MAX_DIM * MAX_DIM / 256;           // covariance entries per thread at most
    __shared__ double mean[MAX_DIM];
    __shared__ double S[MAX_DIM * MAX_DIM];
    __shared__ double X[STAGE];
    const int pc = STAGE / d;                              // points per chunk
    auto stage = [&](int i0, int i1) {
        __syncthreads();
        for (int e = threadIdx.x; e < (i1 - i0) * d; e += blockDim.x) X[e] = u[(int64_t)i0 * d + e];
        __syncthreads();
    };
    double s = 0.0;
    for (int i0 = 0; i0 < n; i0 += pc) {
        const int i1 = min(n, i0 + pc);
        stage(i0, i1);
        if (threadIdx.x < d)
            for (int i = i0; i < i1; ++i) s += X[(i - i0) * d + threadIdx.x];
    }
    if (threadIdx.x < d) mean[threadIdx.x] = s / n;
    double acc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) acc[q] = 0.0;
    for (int i0 = 0; i0 < n; i0 += pc) {
        const int i1 = min(n, i0 + pc);
        stage(i0, i1);                                     // its first barrier also publishes mean
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e >= d * d) break;
            const int a = e / d, b = e % d;
            if (b > a) continue;
            const double ma = mean[a], mb = mean[b];
            for (int i = i0; i < i1; ++i) acc[q] += (X[(i - i0) * d + a] - ma) * (X[(i - i0) * d + b] - mb);
        }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e >= d * d) break;
        const int a = e / d, b = e % d;
        if (b > a) continue;
        S[a * d + b] = S[b * d + a] = acc[q] / (n - 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int a = 0; a < d; ++a) tr += S[a * d + a];
        const double jit = 1e-12 * tr / d;
        for (int a = 0; a < d; ++a) S[a * d + a] += jit;
        for (int j = 0; j < d; ++j) {
            double s = S[j * d + j];
            for (int p = 0; p < j; ++p) s -= S[j * d + p] * S[j * d + p];
            const double djj = sqrt(fmax(s, 0.0));
            S[j * d + j] = djj;
            for (int i = j + 1; i < d; ++i) {
                double t = S[i * d + j];
                for (int p = 0; p < j; ++p) t -= S[i * d + p] * S[j * d + p];
                S[i * d + j] = djj > 0.0 ? t / djj : 0.0;
            }
        }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) L[a * d + b] = b <= a ? S[a * d + b] : 0.0;
    }
}

// Walker w starts at survivor floor(U (n-k)) (draw 0 of step 0).
__global__ void ns_spawn_kernel(const double* __restrict__ u, const double* __restrict__ logl,
                                const int* __restrict__ order, int n, int k, int d, uint64_t seed,
                                uint64_t iter, double* __restrict__ wu, double* __restrict__ wl) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= k) return;
    const double U = philox_uniform(seed, 0, (uint64_t)w, 0, iter, 0);
    int pick = (int)floor(U * (double)(n - k));
    pick = pick > n - k - 1 ? n - k - 1 : pick;
    const int src = order[k + pick];
    for (int c = 0; c < d; ++c) wu[(int64_t)w * d + c] = u[(int64_t)src * d + c];
    wl[w] = logl[src];
}

__global__ void ns_replace_kernel(double* __restrict__ u, double* __restrict__ logl,
                                  const int* __restrict__ order, int k, int d, const double* __restrict__ wu,
                                  const double* __restrict__ wl) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= k) return;
    const int dst = order[w];
    for (int c = 0; c < d; ++c) u[(int64_t)dst * d + c] = wu[(int64_t)w * d + c];
    logl[dst] = wl[w];
}

// live term log(X mean_live L) and the stopping rule
__global__ __launch_bounds__(256) void ns_term_kernel(const double* __restrict__ logl, int n,
                                                      NSState* __restrict__ S, double log_frac) {
    __shared__ double red[4];
    double m = -INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, logl[i]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += exp(logl[i] - mx);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = red[0] + red[1] + red[2] + red[3];
        const double live = mx + log(tot) - log((double)n) + S->logx;
        S->live_term = live;
        S->stop = (live - logaddexp(S->logz, live)) < log_frac ? 1 : 0;
    }
}

// initial live points: u[i][c] = draw c of (walker i, step 0, iteration 0)
__global__ void ns_init_kernel(double* __restrict__ u, int n, int d, uint64_t seed, NSState* S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) {
        S->logx = 0.0; S->logz = -INFINITY; S->lstar = -INFINITY; S->live_term = 0.0;
        S->n_dead = 0; S->n_evals = n; S->n_stalls = 0; S->stop = 0;
    }
    if (e >= (int64_t)n * d) return;
    const int i = (int)(e / d), c = (int)(e % d);
    u[e] = philox_uniform(seed, 0, (uint64_t)i, 0, 0, (uint64_t)c);
}

// final: live points die in ascending order with counts n, n-1, ..., 1
__global__ void ns_final_kernel(const double* __restrict__ logl, const double* __restrict__ u,
                                const int* __restrict__ order, int n, int d, NSState* __restrict__ S,
                                double* __restrict__ dead_logl, int* __restrict__ dead_n,
                                double* __restrict__ dead_u, int64_t dead_cap) {
    const int64_t base = S->n_dead;
    for (int e = threadIdx.x; e < n * d; e += blockDim.x) {
        const int j = e / d, c = e % d;
        if (base + j < dead_cap) dead_u[(base + j) * d + c] = u[(int64_t)order[j] * d + c];
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (base + j < dead_cap) {
            dead_logl[base + j] = logl[order[j]];
            dead_n[base + j] = n - j;
        }
    __syncthreads();
    if (threadIdx.x == 0) S->n_dead = base + n;
}

// Exclusive prefix sum of one value per thread over a workgroup of NT threads
// (NT a multiple of 64, at most 1024): shuffle scans within the waves, then
// the totals of the waves before (buf: NT / 64 doubles).
template <int NT>
__device__ double block_exclusive_sum(double x, double* buf) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    const double up = __shfl_up(inc, 1, 64);
    __syncthreads();
    if (lane == 63) buf[wid] = inc;
    __syncthreads();
    double pre = 0.0;
    for (int w = 0; w < wid; ++w) pre += buf[w];
    return pre + (lane > 0 ? up : 0.0);
}

// workgroup-wide maximum (buf: blockDim / 64 doubles)
__device__ double block_max(double v, double* buf) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) buf[wid] = v;
    __syncthreads();
    double r = buf[0];
    for (int w = 1; w < nw; ++w) r = fmax(r, buf[w]);
    return r;
}

// log Z and H from the expected shrinkage log X_i = -sum_{m<i} 1/n_m (Eq. (1)
// with the mean log-shrinkage per death), FP64, one workgroup of 1024
// threads.  Thread t walks the contiguous run [t c, t c + c) of the M dead
// points, c = ceil(M / 1024): the runs' sums of 1/n_m are scanned across the
// workgroup to give log X at the start of each run, then
// log Z = mx + log sum_i exp(L_i + log w_i - mx) with
// log w_i = log X_{i-1} + log(1 - e^{-1/n_i}) and mx the largest term, and
// H = sum_i p_i (L_i - log Z) over the finite L_i, p_i = e^{L_i + log w_i - log Z}.
// out[0] = log Z, out[1] = H.
__global__ __launch_bounds__(1024) void ns_evidence_kernel(const double* __restrict__ dl,
                                                           const int* __restrict__ dn, int64_t M,
                                                           double* __restrict__ out) {
    __shared__ double buf[16];
    const int64_t c = (M + 1023) / 1024;
    const int64_t i0 = min<int64_t>(M, (int64_t)threadIdx.x * c), i1 = min<int64_t>(M, i0 + c);
    double s = 0.0;
    for (int64_t i = i0; i < i1; ++i) s += 1.0 / dn[i];
    const double x0 = -block_exclusive_sum<1024>(s, buf);
    // L_i + log w_i, advancing log X past point i
    auto term = [&](int64_t i, double& logx) {
        const double inv = 1.0 / dn[i];
        const double v = dl[i] + (logx + log(-expm1(-inv)));
        logx -= inv;
        return v;
    };
    double logx = x0, mx = -INFINITY;
    for (int64_t i = i0; i < i1; ++i) mx = fmax(mx, term(i, logx));
    mx = block_max(mx, buf);
    logx = x0;
    double se = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double v = term(i, logx);
        if (v > -INFINITY) se += exp(v - mx);
    }
    se = block_sum(se, buf);
    const double logz = mx > -INFINITY ? mx + log(se) : -INFINITY;
    logx = x0;
    double h = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double v = term(i, logx);
        if (isfinite(dl[i])) h += exp(v - logz) * (dl[i] - logz);
    }
    h = block_sum(h, buf);
    if (threadIdx.x == 0) {
        out[0] = logz;
        out[1] = h;
    }
}

// log Z of replicate shrinkage sequences log t_m = log(1 - U_m)/n_m (draw m
// of replicate r, stream 1), one workgroup of 256 threads per replicate.
// Thread t takes the run [t c, t c + c) of the dead points (c a multiple of 4:
// one Philox block per 4 draws); the runs' sums of log t are scanned for
// log X at the start of each run, then each thread keeps a running
// (max, sum of exp) of L_m + log X_{m-1} + log(1 - t_m) and the pairs are
// combined over the workgroup.
__global__ __launch_bounds__(256) void ns_replicates_kernel(const double* __restrict__ dl,
                                                            const int* __restrict__ dn, int64_t M, int R,
                                                            uint64_t seed, double* __restrict__ out) {
    __shared__ double buf[4];
    const int r = blockIdx.x;
    if (r >= R) return;                                   // whole workgroups
    const int64_t c = ((M + 255) / 256 + 3) / 4 * 4;
    const int64_t i0 = min<int64_t>(M, (int64_t)threadIdx.x * c), i1 = min<int64_t>(M, i0 + c);
    auto draws = [&](int64_t m) { return philox4x64((uint64_t)(m >> 2), (uint64_t)r, 0, 0, seed, 1); };
    double s = 0.0;
    for (int64_t m = i0; m < i1; m += 4) {
        const u64x4 b = draws(m);
        for (int e = 0; e < 4 && m + e < i1; ++e) s += log1p(-u01(b.x[e])) / (double)dn[m + e];
    }
    double logx = block_exclusive_sum<256>(s, buf);
    double mx = -INFINITY, se = 0.0;
    for (int64_t m = i0; m < i1; m += 4) {
        const u64x4 b = draws(m);
        for (int e = 0; e < 4 && m + e < i1; ++e) {
            const double lt = log1p(-u01(b.x[e])) / (double)dn[m + e];
            const double v = dl[m + e] + (logx + log(-expm1(lt)));
            logx += lt;
            if (v > mx) {
                se = (mx > -INFINITY ? se * exp(mx - v) : 0.0) + 1.0;
                mx = v;
            } else if (v > -INFINITY) {
                se += exp(v - mx);
            }
        }
    }
    const double gm = block_max(mx, buf);
    const double sc = block_sum(mx > -INFINITY ? se * exp(mx - gm) : 0.0, buf);
    if (threadIdx.x == 0) out[r] = gm > -INFINITY ? gm + log(sc) : -INFINITY;
}

// ------------------------------------------------------------------ host side
__global__ void set_scalar_kernel(double* p, double v) {
    if (threadIdx.x == 0) *p = v;
}

// add the per-walker evaluation and stall counts of one slice step to the run totals
__global__ __launch_bounds__(256) void ns_count_kernel(const int* __restrict__ ne, const int* __restrict__ ns,
                                                       int k, NSState* __restrict__ S) {
    __shared__ long long red[2][4];
    long long a = 0, b = 0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) { a += ne[i]; b += ns[i]; }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = a; red[1][threadIdx.x >> 6] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        S->n_evals += red[0][0] + red[0][1] + red[0][2] + red[0][3];
        S->n_stalls += red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

static SliceState carve_slice(ns_model* m, int64_t k, int d, double* u, double* logl, int* ne, int* ns) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t bytes = al(k * d * 8) * 3 + al(k * 8) * 5 + al(k * 4) * 9 + al(8) * 2;
    m->ws_slice.ensure(bytes);
    char* p = m->ws_slice.as<char>();
    SliceState S;
    S.u = u; S.logl = logl; S.n_evals = ne; S.n_stalls = ns;
    S.v = (double*)p; p += al(k * d * 8);
    S.xc = (double*)p; p += al(2 * k * d * 8);
    S.tl = (double*)p; p += al(k * 8);
    S.tr = (double*)p; p += al(k * 8);
    S.tp = (double*)p; p += al(k * 8);
    S.llc = (double*)p; p += al(2 * k * 8);
    S.st = (int*)p; p += al(k * 4);
    S.step = (int*)p; p += al(k * 4);
    S.q = (int*)p; p += al(k * 4);
    S.ne = (int*)p; p += al(k * 4);
    S.ne2 = (int*)p; p += al(k * 4);
    S.pend = (int*)p; p += al(k * 4);
    S.pend2 = (int*)p; p += al(k * 4);
    S.cidx = (int*)p; p += al(2 * k * 4);
    S.ccount = (int*)p; p += al(8);
    S.active = (int*)p; p += al(8);
    return S;
}

// host flag buffer: pinned, one per model
static int* host_flag(ns_model* m) {
    if (!m->host_pinned) NS_HIP(hipHostMalloc(&m->host_pinned, 256, hipHostMallocDefault));
    return static_cast<int*>(m->host_pinned);
}

void slice_step(ns_model* m, double* u, double* logl, int* n_evals, int* n_stalls, int64_t k,
                const double* lstar_dev, const double* L, int n_inner, uint64_t seed, uint64_t iter, int prec,
                hipStream_t s) {
    const int d = m->d;
    NS_CHECK(d <= MAX_DIM, NS_E_UNSUPPORTED, "slice sampler supports d <= 64");
    if (k == 0) return;
    SliceState S = carve_slice(m, k, d, u, logl, n_evals, n_stalls);
    // up to two proposals per walker and round (both ends while stepping out)
    m->ws_theta.ensure((size_t)2 * k * d * sizeof(double));
    double* thc = m->ws_theta.as<double>();
    int* flag = host_flag(m);
    const dim3 gw((unsigned)((k + 255) / 256));
    hipLaunchKernelGGL(slice_init_kernel, gw, dim3(256), 0, s, S, k);
    NS_HIP(hipGetLastError());
    const int chunk = 16;                     // even: every chunk starts at parity 0
    const int64_t max_rounds = (int64_t)n_inner * (2 * MAX_EXPAND + MAX_SHRINK + 4) + 8;
    int64_t rounds = 0;
    auto rounds_chunk = [&](hipStream_t st) {
        for (int c = 0; c < chunk; ++c) {
            // round c uses the counters of parity c & 1 (cleared by the round before)
            const int par = c & 1;
            {
                TraceScope ts(m, st, "slice_advance");
                hipLaunchKernelGGL(slice_advance_kernel, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, st, S, k, d,
                                   lstar_dev, L, n_inner, seed, iter, par, m->prior_kind.as<int>(),
                                   m->prior_a.as<double>(), m->prior_b.as<double>(), thc);
            }
            loglike_batch(m, thc, d, 2 * k, S.llc, prec, S.ccount + par, st);
        }
        NS_HIP(hipGetLastError());
    };
    // First chunk eagerly on the caller's stream (sizes every workspace); the
    // following chunks replay one captured graph of `chunk` rounds on the
    // model's own stream, which is ordered after the caller's work.
    const bool graphs = !m->trace && getenv("NSMI_NO_GRAPH") == nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t run = s;
    while (true) {
        if (rounds == 0 || !graphs) {
            rounds_chunk(run);
        } else {
            if (!exec) {
                if (!m->graph_stream) NS_HIP(hipStreamCreateWithFlags(&m->graph_stream, hipStreamNonBlocking));
                if (!m->graph_event) NS_HIP(hipEventCreateWithFlags(&m->graph_event, hipEventDisableTiming));
                NS_HIP(hipEventRecord(m->graph_event, s));
                NS_HIP(hipStreamWaitEvent(m->graph_stream, m->graph_event, 0));
                run = m->graph_stream;
                hipGraph_t graph;
                NS_HIP(hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal));
                rounds_chunk(run);
                NS_HIP(hipStreamEndCapture(run, &graph));
                const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                NS_HIP(ie);
            }
            NS_HIP(hipGraphLaunch(exec, run));
        }
        rounds += chunk;
        NS_HIP(hipMemcpyAsync(flag, S.active + ((chunk - 1) & 1), sizeof(int), hipMemcpyDeviceToHost, run));
        NS_HIP(hipStreamSynchronize(run));
        if (*flag == 0) break;
        if (rounds >= max_rounds) {
            if (exec) (void)hipGraphExecDestroy(exec);
            throw Error{NS_E_INVALID, "slice sampler did not terminate"};
        }
    }
    if (exec) NS_HIP(hipGraphExecDestroy(exec));
}

void slice_step_host_lstar(ns_model* m, double* u, double* logl, int* n_evals, int* n_stalls, int64_t k,
                           double lstar, const double* L, int n_inner, uint64_t seed, uint64_t iter, int prec,
                           hipStream_t s) {
    m->ws_flag.ensure(256);
    double* lp = m->ws_flag.as<double>();
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, s, lp, lstar);
    NS_HIP(hipGetLastError());
    slice_step(m, u, logl, n_evals, n_stalls, k, lp, L, n_inner, seed, iter, prec, s);
}

void run(ns_model* m, const ns_run_opts* o, ns_run_result* res, double* dl_h, int* dn_h, double* du_h,
         int64_t cap, hipStream_t s) {
    const int n = o->n_live, k = o->n_delete, d = m->d;
    NS_CHECK(n >= 2 && n <= 4096, NS_E_INVALID, "n_live must be in [2, 4096]");
    NS_CHECK(k >= 1 && k < n, NS_E_INVALID, "n_delete must be in [1, n_live)");
    NS_CHECK(o->n_inner >= 1, NS_E_INVALID, "n_inner must be >= 1");
    NS_CHECK(d <= MAX_DIM, NS_E_UNSUPPORTED, "nested sampling supports d <= 64");
    NS_CHECK(o->frac_remain > 0.0 && o->frac_remain < 1.0, NS_E_INVALID, "frac_remain must be in (0, 1)");
    NS_CHECK(o->max_iter >= 1, NS_E_INVALID, "max_iter must be >= 1");
    NS_CHECK(o->n_replicates >= 0, NS_E_INVALID, "n_replicates must be >= 0");
    hipEvent_t ev0, ev1;
    NS_HIP(hipEventCreate(&ev0));
    NS_HIP(hipEventCreate(&ev1));
    NS_HIP(hipEventRecord(ev0, s));
    DevBuf live_u, live_l, order, wu, wl, wne, wns, L, state, th, dl, dn, du, ev;
    live_u.ensure((size_t)n * d * 8);
    live_l.ensure((size_t)n * 8);
    order.ensure((size_t)n * 4);
    wu.ensure((size_t)k * d * 8);
    wl.ensure((size_t)k * 8);
    wne.ensure((size_t)k * 4);
    wns.ensure((size_t)k * 4);
    L.ensure((size_t)d * d * 8);
    state.ensure(sizeof(NSState));
    th.ensure((size_t)n * d * 8);
    int64_t dcap = std::max<int64_t>(4 * (int64_t)n, 1024);
    dl.ensure(dcap * 8); dn.ensure(dcap * 4); du.ensure(dcap * d * 8);
    NSState* S = state.as<NSState>();
    NSState hs;
    hipLaunchKernelGGL(ns_init_kernel, dim3((unsigned)(((int64_t)n * d + 255) / 256)), dim3(256), 0, s,
                       live_u.as<double>(), n, d, o->seed, S);
    NS_HIP(hipGetLastError());
    prior_transform(m, live_u.as<double>(), th.as<double>(), d, n, nullptr, s);
    loglike_batch(m, th.as<double>(), d, n, live_l.as<double>(), o->precision, nullptr, s);
    const double log_frac = log(o->frac_remain);
    int64_t it = 0;
    int64_t n_dead = 0;
    const double* lstar_dev = reinterpret_cast<const double*>(reinterpret_cast<const char*>(S) + offsetof(NSState, lstar));
    while (it < o->max_iter) {
        ++it;
        if (n_dead + k + n > dcap) {
            const int64_t ncap = std::max<int64_t>(2 * dcap, n_dead + k + n);
            DevBuf dl2, dn2, du2;
            dl2.ensure(ncap * 8); dn2.ensure(ncap * 4); du2.ensure(ncap * d * 8);
            NS_HIP(hipMemcpyAsync(dl2.p, dl.p, n_dead * 8, hipMemcpyDeviceToDevice, s));
            NS_HIP(hipMemcpyAsync(dn2.p, dn.p, n_dead * 4, hipMemcpyDeviceToDevice, s));
            NS_HIP(hipMemcpyAsync(du2.p, du.p, n_dead * d * 8, hipMemcpyDeviceToDevice, s));
            NS_HIP(hipStreamSynchronize(s));
            std::swap(dl.p, dl2.p); std::swap(dl.bytes, dl2.bytes);
            std::swap(dn.p, dn2.p); std::swap(dn.bytes, dn2.bytes);
            std::swap(du.p, du2.p); std::swap(du.bytes, du2.bytes);
            dcap = ncap;
        }
        hipLaunchKernelGGL(ns_select_kernel, dim3(1), dim3(1024), 0, s, live_l.as<double>(), live_u.as<double>(), n,
                           k, d, order.as<int>(), S, dl.as<double>(), dn.as<int>(), du.as<double>(), dcap, 1);
        hipLaunchKernelGGL(ns_dircov_kernel, dim3(1), dim3(256), 0, s, live_u.as<double>(), n, d, L.as<double>());
        hipLaunchKernelGGL(ns_spawn_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, live_u.as<double>(),
                           live_l.as<double>(), order.as<int>(), n, k, d, o->seed, (uint64_t)it, wu.as<double>(),
                           wl.as<double>());
        NS_HIP(hipGetLastError());
        slice_step(m, wu.as<double>(), wl.as<double>(), wne.as<int>(), wns.as<int>(), k, lstar_dev, L.as<double>(),
                   o->n_inner, o->seed, (uint64_t)it, o->precision, s);
        hipLaunchKernelGGL(ns_count_kernel, dim3(1), dim3(256), 0, s, wne.as<int>(), wns.as<int>(), k, S);
        hipLaunchKernelGGL(ns_replace_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s,
                           live_u.as<double>(), live_l.as<double>(), order.as<int>(), k, d, wu.as<double>(),
                           wl.as<double>());
        hipLaunchKernelGGL(ns_term_kernel, dim3(1), dim3(256), 0, s, live_l.as<double>(), n, S, log_frac);
        NS_HIP(hipGetLastError());
        NS_HIP(hipMemcpyAsync(&hs, S, sizeof(NSState), hipMemcpyDeviceToHost, s));
        NS_HIP(hipStreamSynchronize(s));
        n_dead = hs.n_dead;
        if (hs.stop) break;
    }
    // final: live points in ascending order
    hipLaunchKernelGGL(ns_select_kernel, dim3(1), dim3(1024), 0, s, live_l.as<double>(), live_u.as<double>(), n, k,
                       d, order.as<int>(), S, dl.as<double>(), dn.as<int>(), du.as<double>(), dcap, 0);
    hipLaunchKernelGGL(ns_final_kernel, dim3(1), dim3(256), 0, s, live_l.as<double>(), live_u.as<double>(),
                       order.as<int>(), n, d, S, dl.as<double>(), dn.as<int>(), du.as<double>(), dcap);
    const int64_t M = n_dead + n;
    const int R = o->n_replicates;
    ev.ensure((size_t)(2 + std::max(R, 1)) * 8);
    hipLaunchKernelGGL(ns_evidence_kernel, dim3(1), dim3(1024), 0, s, dl.as<double>(), dn.as<int>(), M, ev.as<double>());
    if (R > 0)
        hipLaunchKernelGGL(ns_replicates_kernel, dim3((unsigned)R), dim3(256), 0, s, dl.as<double>(),
                           dn.as<int>(), M, R, o->seed, ev.as<double>() + 2);
    NS_HIP(hipGetLastError());
    std::vector<double> evh(2 + std::max(R, 1));
    NS_HIP(hipMemcpyAsync(evh.data(), ev.p, evh.size() * 8, hipMemcpyDeviceToHost, s));
    NS_HIP(hipMemcpyAsync(&hs, S, sizeof(NSState), hipMemcpyDeviceToHost, s));
    NS_HIP(hipEventRecord(ev1, s));
    NS_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NS_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    const int64_t ncopy = std::min<int64_t>(M, cap);
    if (dl_h && ncopy > 0) NS_HIP(hipMemcpy(dl_h, dl.p, ncopy * 8, hipMemcpyDeviceToHost));
    if (dn_h && ncopy > 0) NS_HIP(hipMemcpy(dn_h, dn.p, ncopy * 4, hipMemcpyDeviceToHost));
    if (du_h && ncopy > 0) NS_HIP(hipMemcpy(du_h, du.p, ncopy * d * 8, hipMemcpyDeviceToHost));
    res->logz = evh[0];
    res->h = evh[1];
    double mean = 0.0, var = 0.0;
    for (int r = 0; r < R; ++r) mean += evh[2 + r];
    if (R > 0) mean /= R;
    for (int r = 0; r < R; ++r) var += (evh[2 + r] - mean) * (evh[2 + r] - mean);
    res->sigma = R > 0 ? sqrt(var / R) : 0.0;
    res->sigma_skilling = sqrt(std::max(evh[1], 0.0) / n);
    res->n_iter = it;
    res->n_evals = hs.n_evals;
    res->n_stalls = hs.n_stalls;
    res->n_dead = M;
    res->wall_s = ms * 1e-3;
}

}  // namespace nsmi
