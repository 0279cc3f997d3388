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
// compacted rows only.  Round c uses counter slot c mod 3 (batch size and
// unfinished walkers): it reads slot c-1 (all walkers finished there: the
// round returns at once, and so does the likelihood on its empty batch),
// fills slot c and clears slot c+1 for the next round, so a fixed sequence of
// rounds can be replayed without host work in between.  Every random number
// is addressed by (walker, step, draw), so the result does not depend on the
// order of the compacted rows.
//
// A nested-sampling run is driven from the device: one captured graph of 24
// rounds with a control kernel before every 8th round, launched again and
// again.  The control kernel (one workgroup) finishes an iteration once its
// walkers have all stopped (replacement, live term, stopping rule) and begins
// the next one (selection of the k lowest, dead records, running evidence,
// direction factor, spawn of the walkers); between those points it does
// nothing.  The host keeps one graph launch ahead and reads a small control
// block after each, so it only acts at checkpoints, buffer growth and the end.
// The final log Z, H and the replicate log Z for the error bar (FP64) are
// parallel over the dead points: prefix sums of the log-shrinkages, then a
// max-shifted sum of exponentials.
#include <cstdio>
#include <memory>

#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

enum { ST_NEWSTEP = 0, ST_OUT = 1, ST_SHRINK = 3, ST_DONE = 4 };
constexpr int MAX_EXPAND = 10;
constexpr int MAX_SHRINK = 200;
constexpr double STALL_WIDTH = 1e-12;
constexpr int MAX_DIM = 64;

constexpr int MAX_SPEC = 4;      // speculative proposals per bracket end and round

struct SliceState {
    double* u;        // [k x d] walker positions (caller buffer)
    double* logl;     // [k]
    double* v;        // [k x d] current direction
    double* tl;       // [k]
    double* tr;       // [k]
    int* st;          // [k] phase
    int* step;        // [k] current step (1-based)
    int* q;           // [k] next draw index
    int* ne;          // [k] left-end expansions (stepping out; -1 once that end is final) /
                      //     rejected shrinks
    int* ne2;         // [k] right-end expansions (stepping out; -1 once final)
    int* pend;        // [k] first compact slot of the pending proposals, -1 none
    int* npl;         // [k] pending left-end (or shrink) proposals, in slots pend ..
    int* npr;         // [k] pending right-end proposals, in the slots after those
    int* n_evals;     // [k]
    int* n_stalls;    // [k]
    double* xc;       // [2 spec k x d] compacted proposals (unit cube)
    int* cidx;        // [2 spec k] walker of each compact slot
    double* llc;      // [2 spec k] likelihood of each compact slot
    int* ccount;      // [3] compact batch size of the rounds of slot c mod 3
    int* active;      // [3] walkers not done after the advance of such a round
};

// Walkers at their first step; counters for a first round in slot 0 (slot 2,
// "the round before", marked unfinished); the walk's iteration index.
__global__ void slice_init_kernel(SliceState S, int64_t k, int64_t* iter_p, uint64_t iter) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w == 0) {
        S.ccount[0] = S.ccount[1] = S.ccount[2] = 0;
        S.active[0] = S.active[1] = 0;
        S.active[2] = 1;
        *iter_p = (int64_t)iter;
    }
    if (w >= k) return;
    S.st[w] = ST_NEWSTEP;
    S.step[w] = 0;
    S.pend[w] = -1;
    S.npl[w] = 0;
    S.npr[w] = 0;
    S.n_evals[w] = 0;
    S.n_stalls[w] = 0;
}

// A group of GS lanes per walker (GS the power of two >= d, at least 8, so a
// wave carries 64 / GS walkers), lane i of the group = coordinate i.  The
// walker's phase state is uniform across its group and kept in registers;
// the direction draw (lane i: Box-Muller of draws 2i, 2i+1), the product with
// L (lane i sums row i in column order, as a serial loop would) and the
// proposals are spread over the group's lanes, so every value is bitwise that
// of one thread per walker.
//
// Speculation (spec proposals per bracket end and round): the stepping-out
// points t_L, t_L - 1, ... of an end, and the shrink points that follow one
// another if each is rejected (the next bracket, hence the next point, is
// known from the sign of t before any evaluation), are all fixed in advance;
// a walker proposes up to spec of them at once and applies the results in
// the serial algorithm's order, so every decision, draw and counted
// evaluation is that algorithm's (results past the deciding one are not
// used).  spec = 1 is the plain one-proposal-per-round walk.  Proposals are
// written after the state machine has run, with compact slots taken by one
// atomic per wave.  NORMAL: some prior is normal (its map needs erfinv, whose
// FP64 form alone takes more than half the registers; without it the kernel
// fits three waves per SIMD instead of one).
template <int GS, bool NORMAL>
__global__ __launch_bounds__(256) void slice_advance_kernel(SliceState S, int64_t k, int d,
                                                            const double* __restrict__ lstar_p,
                                                            const double* __restrict__ L, int n_inner,
                                                            uint64_t seed, const int64_t* __restrict__ iter_p,
                                                            int round, int spec,
                                                            const int* __restrict__ pk, const double* __restrict__ pa,
                                                            const double* __restrict__ pb,
                                                            double* __restrict__ thc) {
    constexpr int WPW = 64 / GS;
    const int lane = threadIdx.x & 63, lg = lane & (GS - 1), gb = lane - lg;
    const int64_t w = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * WPW + lane / GS;
    const int slot = round % 3, prev = (round + 2) % 3, next = (round + 1) % 3;
    // slot c+1 was last read by round c-1, which has finished: clear it for
    // the next round; if no walker was left after the round before, there is
    // nothing to do (this round's slot is already clear)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.ccount[next] = 0;
        S.active[next] = 0;
    }
    // the walker's state is requested first, together with the flag that says
    // whether the round has work (groups past the last walker read walker
    // k - 1 and take no part); the direction factor goes to LDS meanwhile, so
    // that the row products of a new direction read LDS instead of waiting on
    // one global load per column
    const bool live = w < k;
    const int64_t wr = live ? w : k - 1;
    const bool act = lg < d;
    const int busy_prev = S.active[prev];
    const uint64_t iter = (uint64_t)*iter_p;
    const double lstar = *lstar_p;
    int st = S.st[wr], step = S.step[wr], q = S.q[wr], ne = S.ne[wr], ne2 = S.ne2[wr];
    int pend = S.pend[wr], npl = S.npl[wr], npr = S.npr[wr];
    int nev = S.n_evals[wr], nst = S.n_stalls[wr];
    double tl = S.tl[wr], tr = S.tr[wr], logl = S.logl[wr];
    double ui = act ? S.u[wr * d + lg] : 0.0, vi = act ? S.v[wr * d + lg] : 0.0;
    if (busy_prev == 0) return;
    __shared__ double Ls[MAX_DIM * MAX_DIM];
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) Ls[e] = L[e];
    if (!live) {                        // walker k - 1's state was read: none of it is this group's
        st = ST_DONE;
        pend = -1;
        npl = npr = 0;
    }
    // last round's results for this walker (at most 2 spec <= GS of them):
    // lane i of the group loads result i, all in one load
    static_assert(GS >= 2 * MAX_SPEC, "a group holds a walker's pending results");
    const double llv = (pend >= 0 && lg < npl + npr) ? S.llc[pend + lg] : 0.0;
    auto ll_at = [&](int i) { return __shfl(llv, gb + i, 64); };
    // This round's random numbers, one Philox4x64 block per lane of the
    // group, computed once for the whole wave (instead of on each state's
    // path in turn) and kept in LDS (pw: the block of the thread's lane, as
    // uniforms): lanes [0, nd) hold blocks 0 .. nd - 1 of step s0 + 1 (s0 the
    // walker's step at the start of the round), whose draws 0 .. 2d are the
    // next direction's Box-Muller pairs and offset; lanes [nd, GS) hold the
    // blocks of step s0 from draw q's block on, the shrink draws that follow.
    // A draw outside these comes from draw()'s own batches.
    __shared__ double pw[256][4];
    const int nd = (2 * d + 4) >> 2;
    // q is only meaningful once the walker has begun a step (a walker between
    // steps has none; the initial state leaves it unset)
    const int qs = (st == ST_OUT || st == ST_SHRINK) ? q : 0;
    const int step0 = step, qb0 = (qs >> 2) << 2, qend0 = qb0 + 4 * (GS - nd);
    const int wl0 = threadIdx.x - lane + gb;        // this group's lane 0 in pw
    {
        const bool dlane = lg < nd;
        const u64x4 b = philox4x64(dlane ? (uint64_t)lg : (uint64_t)((qs >> 2) + lg - nd), (uint64_t)w,
                                   (uint64_t)(dlane ? step + 1 : step), iter, seed, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) pw[threadIdx.x][j] = u01(b.x[j]);
    }
    __syncthreads();
    const uint64_t gmask = GS == 64 ? ~0ull : (((1ull << GS) - 1) << gb);
    bool moved = false;
    // lane i of the group: row i of L z (L lower triangular), summed over
    // j = 0 .. i in order; the z_j come from the group's lanes four shuffles
    // at a time
    auto lz = [&](double z) {
        double acc = 0.0;
        int j = 0;
        for (; j + 4 <= d; j += 4) {
            double zq[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) zq[t] = __shfl(z, gb + j + t, 64);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (act && j + t <= lg) acc = __dadd_rn(acc, __dmul_rn(Ls[lg * d + j + t], zq[t]));
        }
        for (; j < d; ++j) {
            const double zj = __shfl(z, gb + j, 64);
            if (act && j <= lg) acc = __dadd_rn(acc, __dmul_rn(Ls[lg * d + j], zj));
        }
        return act ? acc : 0.0;
    };
    // the direction of step s0 + 1, v' = L z (z by Box-Muller from the draws
    // above), and its offset r', formed once for the wave here rather than on
    // the path of the walkers that begin a step this round
    double vnext = 0.0;
    {
        double z = 0.0;
        if (act) {
            const double u1 = pw[wl0 + (lg >> 1)][2 * (lg & 1)], u2 = pw[wl0 + (lg >> 1)][2 * (lg & 1) + 1];
            z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
        }
        vnext = lz(z);
    }
    const double rnext = pw[wl0 + (d >> 1)][2 * (d & 1)];
    // the point at t along the direction lies in the unit cube (outside it
    // needs no evaluation: it is outside the constraint)
    auto inbox = [&](double t) {
        const double xi = __dadd_rn(ui, __dmul_rn(t, vi));
        return (__ballot(act && !((xi >= 0.0) && (xi <= 1.0))) & gmask) == 0;
    };
    // draws of the current step: the precomputed ones, else GS at a time
    // (lane i of the group computes draw qb + i; a draw outside the batch
    // starts a new one at that draw)
    double ub = 0.0;
    int qb = -(1 << 30);
    auto draw = [&](int qq) {
        if (step == step0 && qq >= qb0 && qq < qend0) {
            const int o = qq - qb0;
            return pw[wl0 + nd + (o >> 2)][o & 3];
        }
        if (qq < qb || qq >= qb + GS) {
            qb = qq;
            ub = philox_uniform(seed, 0, (uint64_t)w, (uint64_t)step, iter, (uint64_t)(qq + lg));
        }
        return __shfl(ub, gb + (qq - qb), 64);
    };
    // shrink point from the bracket and draw qq
    auto shrink_point = [&](double a, double b, int qq) {
        const double U = draw(qq);
        return __dadd_rn(a, __dmul_rn(U, __dsub_rn(b, a)));
    };
    // last round's evaluations, in the serial order
    if (pend >= 0) {
        if (st == ST_OUT) {
            for (int i = 0; i < npl; ++i) {            // left end at t_L, t_L - 1, ...
                const double ll = ll_at(i);
                nev += 1;
                if (ll > lstar) { tl -= 1.0; ne += 1; } else { ne = -1; break; }
            }
            for (int i = 0; i < npr; ++i) {            // right end at t_R, t_R + 1, ...
                const double ll = ll_at(npl + i);
                nev += 1;
                if (ll > lstar) { tr += 1.0; ne2 += 1; } else { ne2 = -1; break; }
            }
        } else {
            // the shrink chain again from its start: points outside the cube are
            // rejected without evaluation, the evaluated ones take their results
            int kk = 0;
            while (true) {
                const double t = shrink_point(tl, tr, q);
                ++q;
                if (inbox(t)) {
                    const double ll = ll_at(kk);
                    ++kk;
                    nev += 1;
                    if (ll > lstar) {
                        ui = __dadd_rn(ui, __dmul_rn(t, vi));
                        logl = ll;
                        moved = true;
                        st = ST_NEWSTEP;
                        break;
                    }
                }
                if (t < 0.0) tl = t; else tr = t;
                ne += 1;
                if (tr - tl < STALL_WIDTH || ne >= MAX_SHRINK) {
                    nst += 1;
                    st = ST_NEWSTEP;
                    break;
                }
                if (kk == npl) break;
            }
        }
        pend = -1;
        npl = npr = 0;
    }
    double tq[2 * MAX_SPEC];            // this round's proposals: npl left-end / shrink points, then npr right-end
    while (true) {
        if (st == ST_DONE) break;
        if (st == ST_NEWSTEP) {
            if (step >= n_inner) { st = ST_DONE; break; }
            const int s = ++step;
            qb = -(1 << 30);                // the draws of the step before are gone
            double r;
            if (s == step0 + 1) {
                vi = vnext;
                r = rnext;
            } else {
                // a second new step in one round: lane i < d draws the pair
                // 2i, 2i + 1 for Box-Muller, lane d (when the group has one
                // more lane) the pair 2d, 2d + 1, whose first member is r
                double z = 0.0, u1 = 0.0, u2 = 0.0;
                if (lg <= d) philox_uniform_pair(seed, 0, (uint64_t)w, (uint64_t)s, iter, 2 * (uint64_t)lg, u1, u2);
                r = d < GS ? __shfl(u1, gb + d, 64)
                           : philox_uniform(seed, 0, (uint64_t)w, (uint64_t)s, iter, 2 * (uint64_t)d);
                if (act) z = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
                vi = lz(z);
            }
            tl = -r;
            tr = 1.0 - r;
            q = 2 * d + 1;
            ne = 0;
            ne2 = 0;
            st = ST_OUT;
            continue;
        }
        if (st == ST_OUT) {
            // both ends step out at once, each proposing its next points until
            // one is outside the cube or the end has expanded MAX_EXPAND times;
            // the ends do not interact, so the evaluations and the final
            // bracket are those of stepping out one end after the other
            if (ne >= 0) {
                double t = tl;
                while (npl < spec && ne + npl < MAX_EXPAND) {
                    if (npl > 0) t -= 1.0;
                    if (!inbox(t)) break;
                    tq[npl++] = t;
                }
                if (npl == 0) ne = -1;
            }
            if (ne2 >= 0) {
                double t = tr;
                while (npr < spec && ne2 + npr < MAX_EXPAND) {
                    if (npr > 0) t += 1.0;
                    if (!inbox(t)) break;
                    tq[npl + npr++] = t;
                }
                if (npr == 0) ne2 = -1;
            }
            if (npl + npr > 0) break;
            st = ST_SHRINK;
            ne = 0;
            continue;
        }
        // shrink: the next spec points in the cube, each on the bracket the
        // rejections before it leave; the state stays at the chain's start
        double ca = tl, cb = tr;
        int cne = ne, cq = q;
        bool stall = false;
        while (npl < spec) {
            const double t = shrink_point(ca, cb, cq);
            ++cq;
            if (inbox(t)) tq[npl++] = t;
            if (t < 0.0) ca = t; else cb = t;
            ++cne;
            if (cb - ca < STALL_WIDTH || cne >= MAX_SHRINK) { stall = true; break; }
        }
        if (npl > 0) break;
        // the bracket collapsed with no point in the cube: the step stalls now
        (void)stall;
        tl = ca; tr = cb; ne = cne; q = cq;
        nst += 1;
        st = ST_NEWSTEP;
    }
    // compact slots: exclusive prefix of the walkers' proposal counts over the
    // wave (group leaders hold them), one atomic for the wave
    const int nmine = npl + npr;
    const int nemit = (lg == 0) ? nmine : 0;
    int inc = nemit;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    const int total = __shfl(inc, 63, 64);
    int base = 0;
    if (lane == 0 && total > 0) base = atomicAdd(S.ccount + slot, total);
    base = __shfl(base, 0, 64) + __shfl(inc - nemit, gb, 64);
#pragma unroll 1
    for (int e = 0; e < nmine; ++e) {
        const int cs = base + e;
        const double xi = __dadd_rn(ui, __dmul_rn(tq[e], vi));
        if (act) {
            S.xc[(int64_t)cs * d + lg] = xi;
            thc[(int64_t)cs * d + lg] = NORMAL ? prior_map(xi, pk[lg], pa[lg], pb[lg]) : pa[lg] + (pb[lg] - pa[lg]) * xi;
        }
        if (lg == 0) S.cidx[cs] = (int)w;
    }
    if (nmine > 0) pend = base;
    if (live) {
        if (act) {
            if (moved) S.u[w * d + lg] = ui;
            S.v[w * d + lg] = vi;
        }
        if (lg == 0) {
            S.st[w] = st; S.step[w] = step; S.q[w] = q; S.ne[w] = ne; S.ne2[w] = ne2;
            S.pend[w] = pend; S.npl[w] = npl; S.npr[w] = npr;
            S.n_evals[w] = nev; S.n_stalls[w] = nst;
            S.tl[w] = tl; S.tr[w] = tr; S.logl[w] = logl;
        }
    }
    // unfinished walkers: one atomic for the wave
    const uint64_t busy = __ballot(live && lg == 0 && st != ST_DONE);
    if (lane == 0 && busy) atomicAdd(S.active + slot, (int)__popcll(busy));
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

// Control block of a run (device memory): where the device-driven iteration
// stands and why it stopped, read by the host after each graph launch.
struct NSCtl {
    int64_t it;          // iteration of the walkers (1-based); between iterations the last finished one
    int64_t max_iter;
    int64_t ckpt_every;  // > 0: pause after iterations that are multiples of it
    int need_begin;      // the next control point begins iteration it + 1
    int walking;         // the walkers of iteration it are stepping
    int pause;           // stopped at an iteration boundary for a checkpoint
    int grow;            // stopped at an iteration boundary: dead-point storage too small
    int done;            // 1: stopping rule met, 2: max_iter reached
    int pad;
};

// Dead-point storage of a run (device memory, so that it can grow between
// launches of a captured graph).
struct DeadBuf {
    double* dl;       // [cap] logL
    int* dn;          // [cap] live points at death
    double* du;       // [cap x d] unit-cube position
    int64_t cap;
};

__device__ __forceinline__ double logaddexp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = fmax(a, b);
    return m + log1p(exp(-fabs(a - b)));
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

// Integer image of a double that orders as the doubles do, with -0 as +0
// and every NaN after +inf.
__device__ inline uint64_t order_bits(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x == 0.0 ? 0.0 : x);
    return isnan(x) ? ~0ull : ((b >> 63) ? ~b : (b | 0x8000000000000000ull));
}

// (a, ia) comes before (b, ib) in the order of (logL, index)
__device__ inline bool before(uint64_t a, int ia, uint64_t b, int ib) {
    return (a < b) | ((a == b) & (ia < ib));
}

// Sort of the live points by (logl, index) -- NaN after +inf, ties by index --
// for n <= 4096 by one workgroup of at least N2 / 4 threads: a bitonic network
// over N2 = max(256, n rounded up to a power of two) entries, the padding
// after every point.  Entry e = 256 w + 4 lane + r lives in register r of that
// lane of wave w: strides 1 and 2 compare registers of one lane, strides 4 to
// 128 lanes of one wave (shuffles), larger strides go through LDS.  On return
// key[j] is the logl of the j-th point in that order and idx[j] its index,
// j < n (key: N2 doubles of LDS, idx: N2 ints).
__device__ void sort_live(const double* __restrict__ logl, int n, double* key, int* idx) {
    int N2 = 256;
    while (N2 < n) N2 <<= 1;
    uint64_t* kb = reinterpret_cast<uint64_t*>(key);
    const int lane = threadIdx.x & 63;
    const int e0 = (threadIdx.x >> 6) * 256 + lane * 4;
    const bool act = e0 < N2;                          // wave-uniform
    uint64_t k[4];
    int x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = e0 + r;
        k[r] = e < n ? order_bits(logl[e]) : ~0ull;
        x[r] = e < n ? e : 0x7fffffff;
    }
    // the entry of register a goes first (ascending) or last, of a < b
    auto regs = [&](int a, int b, bool up) {
        if (before(k[b], x[b], k[a], x[a]) == up) {
            const uint64_t tk = k[a]; k[a] = k[b]; k[b] = tk;
            const int tx = x[a]; x[a] = x[b]; x[b] = tx;
        }
    };
    for (int S = 2; S <= N2; S <<= 1) {
        if (S >= 512) {
            __syncthreads();                           // the last loads from LDS are done
            if (act)
#pragma unroll
                for (int r = 0; r < 4; ++r) { kb[e0 + r] = k[r]; idx[e0 + r] = x[r]; }
            __syncthreads();
            for (int s = S >> 1; s >= 256; s >>= 1) {
                for (int p = threadIdx.x; p < (N2 >> 1); p += blockDim.x) {
                    const int a = ((p & ~(s - 1)) << 1) | (p & (s - 1)), b = a + s;
                    const uint64_t ka = kb[a], kbb = kb[b];
                    const int ia = idx[a], ib = idx[b];
                    if (before(kbb, ib, ka, ia) == ((a & S) == 0)) {
                        kb[a] = kbb; kb[b] = ka;
                        idx[a] = ib; idx[b] = ia;
                    }
                }
                __syncthreads();
            }
            if (act)
#pragma unroll
                for (int r = 0; r < 4; ++r) { k[r] = kb[e0 + r]; x[r] = idx[e0 + r]; }
        }
        if (!act) continue;
        const bool up = (e0 & S) == 0;                 // for S >= 4 the same for the four registers
        for (int s = S >= 256 ? 128 : S >> 1; s >= 4; s >>= 1) {
            const int m = s >> 2;
            const int src = (lane ^ m) << 2;
            const bool keep_first = ((lane & m) == 0) == up;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int plo = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)k[r]);
                const int phi = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(k[r] >> 32));
                const int px = __builtin_amdgcn_ds_bpermute(src, x[r]);
                const uint64_t pk = ((uint64_t)(uint32_t)phi << 32) | (uint32_t)plo;
                if (before(pk, px, k[r], x[r]) == keep_first) { k[r] = pk; x[r] = px; }
            }
        }
        if (S >= 4) { regs(0, 2, up); regs(1, 3, up); regs(0, 1, up); regs(2, 3, up); }
        else { regs(0, 1, true); regs(2, 3, false); }
    }
    __syncthreads();                                   // the last loads from LDS are done
    if (act)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (e0 + r < n) { idx[e0 + r] = x[r]; key[e0 + r] = logl[x[r]]; }
    __syncthreads();
}

constexpr int CTL_NT = 1024;
constexpr int CTL_LDS = 4096 + 2080 + MAX_DIM;   // doubles: sort keys + indices, or dircov's regions

// Direction factor by one workgroup of CTL_NT threads: live-point covariance
// (1/(n-1)), trace jitter 1e-12 tr/d, lower Cholesky factor L (row-major).
// Each mean and each covariance entry is a sum over the points split into a
// fixed number of strided parts (part p takes points p, p + P, ..., in index
// order), and the parts are added in order.  lds: CTL_LDS doubles.
__device__ void dircov_block(const double* __restrict__ u, int n, int d, double* __restrict__ L, double* lds) {
    constexpr int NT = CTL_NT, STAGE = 4096;
    double* X = lds;                                   // staged points, then the covariance [d x d]
    double* P = lds + STAGE;                           // partial sums (<= 2080)
    double* mean = P + 2080;                           // [d]
    const int t = threadIdx.x;
    {
        const int spm = NT / d, c = t % d, sp = t / d;
        double s = 0.0;
        if (sp < spm)
            for (int i = sp; i < n; i += spm) s += u[(int64_t)i * d + c];
        __syncthreads();
        if (sp < spm) P[sp * d + c] = s;
        __syncthreads();
        if (t < d) {
            double m = 0.0;
            for (int q = 0; q < spm; ++q) m += P[q * d + t];
            mean[t] = m / n;
        }
        __syncthreads();
    }
    const int ne = d * (d + 1) / 2;
    const int spc = ne <= NT ? NT / ne : 1;            // parts per entry
    constexpr int EPT = (MAX_DIM * (MAX_DIM + 1) / 2 + NT - 1) / NT;
    int ea[EPT], eb[EPT], sp = 0;
    double acc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        int e = -1;
        if (ne <= NT) {
            if (q == 0 && t < spc * ne) { e = t % ne; sp = t / ne; }
        } else if (t + NT * q < ne) {
            e = t + NT * q;
        }
        int a = 0;
        if (e >= 0)
            while ((a + 1) * (a + 2) / 2 <= e) ++a;
        ea[q] = e >= 0 ? a : -1;
        eb[q] = e >= 0 ? e - a * (a + 1) / 2 : 0;
        acc[q] = 0.0;
    }
    const int pc = STAGE / d;                          // points per staged chunk
    for (int i0 = 0; i0 < n; i0 += pc) {
        const int i1 = min(n, i0 + pc);
        __syncthreads();
        for (int x = t; x < (i1 - i0) * d; x += NT) X[x] = u[(int64_t)i0 * d + x];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            if (ea[q] < 0) continue;
            const int a = ea[q], b = eb[q];
            const double ma = mean[a], mb = mean[b];
            const int first = i0 + (((sp - i0) % spc) + spc) % spc;
            for (int i = first; i < i1; i += spc) acc[q] += (X[(i - i0) * d + a] - ma) * (X[(i - i0) * d + b] - mb);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q)
        if (ea[q] >= 0) P[ne <= NT ? sp * ne + (ea[q] * (ea[q] + 1) / 2 + eb[q]) : t + NT * q] = acc[q];
    __syncthreads();
    for (int e = t; e < ne; e += NT) {
        double v = 0.0;
        for (int q = 0; q < spc; ++q) v += P[q * ne + e];
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= e) ++a;
        const int b = e - a * (a + 1) / 2;
        X[a * d + b] = X[b * d + a] = v / (n - 1);
    }
    __syncthreads();
    // Cholesky by the first wave, lane i for row i (d <= 64), one column at a
    // time: entry (i, j) subtracts L_ip L_jp for p = 0 .. j-1 in that order.
    if (t < 64) {
        double tr = 0.0;
        for (int a = 0; a < d; ++a) tr += X[a * d + a];
        const double jit = 1e-12 * tr / d;
        const int i = t;
        if (i < d) X[i * d + i] += jit;
        for (int j = 0; j < d; ++j) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // column j - 1 is in LDS for every lane
            __builtin_amdgcn_wave_barrier();
            double v = 0.0;
            if (i >= j && i < d) {
                v = X[i * d + j];
                for (int p = 0; p < j; ++p) v -= X[i * d + p] * X[j * d + p];
            }
            const double djj = sqrt(fmax(__shfl(v, j, 64), 0.0));
            if (i == j) X[j * d + j] = djj;
            else if (i > j && i < d) X[i * d + j] = djj > 0.0 ? v / djj : 0.0;
        }
    }
    __syncthreads();
    for (int e = t; e < d * d; e += NT) {
        const int a = e / d, b = e - a * d;
        L[e] = b <= a ? X[e] : 0.0;
    }
}

// Control point of a run, placed before slice round `round` of the graph (one
// workgroup of CTL_NT threads).
//  Finish: if iteration `it` is walking and no walker was left after the
//   round before, add the walkers' evaluation and stall counts, put the
//   walkers in the dead points' slots, compute the live term
//   log(X mean_live L) and the stopping rule, and decide: done (rule or
//   max_iter), grow (dead storage cannot take k more), pause (checkpoint
//   due) or begin the next iteration.
//  Begin (iteration it + 1): order the live points by (logL, index); the k
//   lowest die with live counts n, ..., n-k+1 (dead records; log X shrinks
//   by 1/n_j per death; running log Z += the log-sum-exp of
//   logL_j + log X_{j-1} + log(1 - e^{-1/n_j}), each term formed as a serial
//   chain would form it); L* = the largest dead logL; walker w starts at
//   survivor floor(U (n-k)) (draw 0 of step 0 of the iteration); the
//   direction factor from the live points before the deletion.
// Between those points it returns at once.
__global__ __launch_bounds__(CTL_NT) void ns_control_kernel(NSCtl* __restrict__ ctl, NSState* __restrict__ S,
                                                            const DeadBuf* __restrict__ db, SliceState W,
                                                            double* __restrict__ live_u, double* __restrict__ live_l,
                                                            int* __restrict__ order, double* __restrict__ L, int n,
                                                            int k, int d, uint64_t seed, double log_frac, int round) {
    __shared__ double lds[CTL_LDS];
    __shared__ double red[CTL_NT / 64];
    __shared__ double s_logx;
    __shared__ int s_begin;
    const int t = threadIdx.x;
    const int prev = (round + 2) % 3;
    const int64_t it0 = ctl->it;
    const int walking = ctl->walking, need_begin = ctl->need_begin;
    const int left = W.active[prev];
    __syncthreads();                                  // every thread has read ctl before it changes
    int begin = need_begin;
    if (walking && left == 0) {
        long long a = 0, b = 0;
        for (int w = t; w < k; w += CTL_NT) {
            a += W.n_evals[w];
            b += W.n_stalls[w];
        }
        a = wave_sum(a);
        b = wave_sum(b);
        for (int e = t; e < k * d; e += CTL_NT) {
            const int w = e / d, c = e - w * d;
            live_u[(int64_t)order[w] * d + c] = W.u[e];
        }
        for (int w = t; w < k; w += CTL_NT) live_l[order[w]] = W.logl[w];
        __syncthreads();
        double mx = -INFINITY;
        for (int i = t; i < n; i += CTL_NT) mx = fmax(mx, live_l[i]);
        mx = block_max(mx, red);
        double se = 0.0;
        for (int i = t; i < n; i += CTL_NT) se += exp(live_l[i] - mx);
        se = block_sum(se, red);
        __shared__ long long cnt[2][CTL_NT / 64];
        if ((t & 63) == 0) {
            cnt[0][t >> 6] = a;
            cnt[1][t >> 6] = b;
        }
        __syncthreads();
        if (t == 0) {
            long long ta = 0, tb = 0;
            for (int q = 0; q < CTL_NT / 64; ++q) {
                ta += cnt[0][q];
                tb += cnt[1][q];
            }
            S->n_evals += ta;
            S->n_stalls += tb;
            const double live = mx + log(se) - log((double)n) + S->logx;
            S->live_term = live;
            S->stop = (live - logaddexp(S->logz, live)) < log_frac ? 1 : 0;
            ctl->walking = 0;
            int nb = 0;
            if (S->stop) ctl->done = 1;
            else if (it0 >= ctl->max_iter) ctl->done = 2;
            else if (S->n_dead + k > db->cap) ctl->grow = 1;
            else if (ctl->ckpt_every > 0 && it0 % ctl->ckpt_every == 0) ctl->pause = 1;
            else nb = 1;
            s_begin = nb;
        }
        __syncthreads();
        begin = s_begin;
    }
    if (!begin) return;

    const int64_t it1 = it0 + 1;
    double* key = lds;
    int* idx = reinterpret_cast<int*>(lds + 4096);
    sort_live(live_l, n, key, idx);
    const DeadBuf D = *db;
    const int64_t base = S->n_dead;
    const double logx0 = S->logx, logz0 = S->logz;
    for (int e = t; e < k * d; e += CTL_NT) {
        const int j = e / d, c = e - j * d;
        D.du[(base + j) * d + c] = live_u[(int64_t)idx[j] * d + c];
    }
    for (int j = t; j < k; j += CTL_NT) {
        D.dl[base + j] = key[j];
        D.dn[base + j] = n - j;
    }
    // running evidence: thread t takes ranks [4t, 4t + 4) (k < 4096)
    constexpr int RPT = 4;
    const int j0 = min(k, t * RPT), j1 = min(k, j0 + RPT);
    double sinv = 0.0;
    for (int j = j0; j < j1; ++j) sinv += 1.0 / (double)(n - j);
    double lx = logx0 - block_exclusive_sum<CTL_NT>(sinv, red);
    double v[RPT], mloc = -INFINITY;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        v[r] = -INFINITY;
        const int j = j0 + r;
        if (j < j1) {
            const double inv = 1.0 / (double)(n - j);
            v[r] = key[j] + (lx + log(-expm1(-inv)));
            lx -= inv;
            mloc = fmax(mloc, v[r]);
        }
    }
    if (j0 < j1 && j1 == k) s_logx = lx;               // log X after the k deaths
    const double mall = block_max(mloc, red);
    double se = 0.0;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
        if (v[r] > -INFINITY) se += exp(v[r] - mall);
    se = block_sum(se, red);
    if (t == 0) {
        S->logz = logaddexp(logz0, mall > -INFINITY ? mall + log(se) : -INFINITY);
        S->logx = s_logx;
        S->lstar = key[k - 1];
        S->n_dead = base + k;
    }
    for (int i = t; i < n; i += CTL_NT) order[i] = idx[i];
    // spawn: survivor floor(U (n - k)), U = draw 0 of (walker, step 0, iteration it + 1);
    // the source index waits in W.pend until the copy
    for (int w = t; w < k; w += CTL_NT) {
        const double U = philox_uniform(seed, 0, (uint64_t)w, 0, (uint64_t)it1, 0);
        int pick = (int)floor(U * (double)(n - k));
        pick = pick > n - k - 1 ? n - k - 1 : pick;
        W.pend[w] = idx[k + pick];
        W.logl[w] = key[k + pick];
    }
    __syncthreads();
    for (int e = t; e < k * d; e += CTL_NT) {
        const int w = e / d, c = e - w * d;
        W.u[e] = live_u[(int64_t)W.pend[w] * d + c];
    }
    __syncthreads();
    for (int w = t; w < k; w += CTL_NT) {
        W.st[w] = ST_NEWSTEP;
        W.step[w] = 0;
        W.pend[w] = -1;
        W.npl[w] = 0;
        W.npr[w] = 0;
        W.n_evals[w] = 0;
        W.n_stalls[w] = 0;
    }
    dircov_block(live_u, n, d, L, lds);                // its first barrier ends the sort's use of lds
    if (t == 0) {
        W.active[prev] = 1;                            // the next round runs
        ctl->it = it1;
        ctl->walking = 1;
        ctl->need_begin = 0;
    }
}

// order of the live points by (logL, index), one workgroup
__global__ __launch_bounds__(CTL_NT) void ns_sort_kernel(const double* __restrict__ logl, int n,
                                                         int* __restrict__ order) {
    __shared__ double key[4096];
    __shared__ int idx[4096];
    sort_live(logl, n, key, idx);
    for (int i = threadIdx.x; i < n; i += blockDim.x) order[i] = idx[i];
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

__global__ void zero_ints_kernel(int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

static SliceState carve_slice(ns_model* m, int64_t k, int d, int spec, double* u, double* logl, int* ne, int* ns,
                              int64_t** iter_p) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int64_t kc = 2 * (int64_t)spec * k;          // compact slots
    const size_t bytes = al(k * d * 8) + al(kc * d * 8) + al(k * 8) * 2 + al(kc * 8) + al(k * 4) * 8 +
                         al(kc * 4) + al(16) * 3;
    m->ws_slice.ensure(bytes);
    char* p = m->ws_slice.as<char>();
    SliceState S;
    S.u = u; S.logl = logl; S.n_evals = ne; S.n_stalls = ns;
    S.v = (double*)p; p += al(k * d * 8);
    S.xc = (double*)p; p += al(kc * d * 8);
    S.tl = (double*)p; p += al(k * 8);
    S.tr = (double*)p; p += al(k * 8);
    S.llc = (double*)p; p += al(kc * 8);
    S.st = (int*)p; p += al(k * 4);
    S.step = (int*)p; p += al(k * 4);
    S.q = (int*)p; p += al(k * 4);
    S.ne = (int*)p; p += al(k * 4);
    S.ne2 = (int*)p; p += al(k * 4);
    S.pend = (int*)p; p += al(k * 4);
    S.npl = (int*)p; p += al(k * 4);
    S.npr = (int*)p; p += al(k * 4);
    S.cidx = (int*)p; p += al(kc * 4);
    S.ccount = (int*)p; p += al(16);
    S.active = (int*)p; p += al(16);
    if (iter_p) *iter_p = (int64_t*)p;
    return S;
}

// Owning handles for the graph objects and pinned host memory of one call, so
// that every error path ends a capture and releases what it made.
struct Capture {
    hipStream_t s = nullptr;
    bool on = false;
    void begin(hipStream_t st) {
        s = st;
        NS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        on = true;
    }
    hipGraph_t end() {
        hipGraph_t g = nullptr;
        on = false;
        NS_HIP(hipStreamEndCapture(s, &g));
        return g;
    }
    ~Capture() {
        if (on) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
        }
    }
};
struct GraphExec {
    hipGraphExec_t e = nullptr;
    ~GraphExec() {
        if (e) (void)hipGraphExecDestroy(e);
    }
};
struct PinnedHost {
    void* p = nullptr;
    explicit PinnedHost(size_t n) { NS_HIP(hipHostMalloc(&p, n, hipHostMallocDefault)); }
    ~PinnedHost() {
        if (p) (void)hipHostFree(p);
    }
};
struct EventPair {
    hipEvent_t e[2] = {nullptr, nullptr};
    explicit EventPair(unsigned flags) {
        NS_HIP(hipEventCreateWithFlags(&e[0], flags));
        NS_HIP(hipEventCreateWithFlags(&e[1], flags));
    }
    ~EventPair() {
        for (auto x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Capture the launches of `body` on stream st into an executable graph.
template <class F>
static void capture_graph(hipStream_t st, GraphExec& ge, F&& body) {
    Capture cap;
    cap.begin(st);
    body(st);
    hipGraph_t g = cap.end();
    const hipError_t ie = hipGraphInstantiate(&ge.e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NS_HIP(ie);
}

// the model's own stream for captured graphs (capture needs a stream other
// than the null stream), ordered after the caller's stream s
static hipStream_t graph_stream_after(ns_model* m, hipStream_t s) {
    if (!m->graph_stream) NS_HIP(hipStreamCreateWithFlags(&m->graph_stream, hipStreamNonBlocking));
    if (!m->graph_event) NS_HIP(hipEventCreateWithFlags(&m->graph_event, hipEventDisableTiming));
    NS_HIP(hipEventRecord(m->graph_event, s));
    NS_HIP(hipStreamWaitEvent(m->graph_stream, m->graph_event, 0));
    return m->graph_stream;
}

static bool graphs_enabled(const ns_model* m) { return !m->trace && getenv("NSMI_NO_GRAPH") == nullptr; }

constexpr int GRAPH_ROUNDS = 24;      // slice rounds per captured graph (a multiple of 3)
constexpr int CTL_EVERY = 8;          // rounds between control points of a nested-sampling graph

static void advance_round(ns_model* m, const SliceState& S, int64_t k, int spec, const double* lstar_dev,
                          const double* L, int n_inner, uint64_t seed, const int64_t* iter_p, int round, int prec,
                          hipStream_t st) {
    const int d = m->d;
    double* thc = m->ws_theta.as<double>();
    {
        TraceScope ts(m, st, "slice_advance");
        auto launch = [&](auto kern, int gs) {
            const int64_t per_block = 4 * (64 / gs);
            hipLaunchKernelGGL(kern, dim3((unsigned)((k + per_block - 1) / per_block)), dim3(256), 0, st, S, k, d,
                               lstar_dev, L, n_inner, seed, iter_p, round, spec, m->prior_kind.as<int>(),
                               m->prior_a.as<double>(), m->prior_b.as<double>(), thc);
        };
        if (m->any_normal_prior) {
            if (d <= 8) launch(slice_advance_kernel<8, true>, 8);
            else if (d <= 16) launch(slice_advance_kernel<16, true>, 16);
            else if (d <= 32) launch(slice_advance_kernel<32, true>, 32);
            else launch(slice_advance_kernel<64, true>, 64);
        } else {
            if (d <= 8) launch(slice_advance_kernel<8, false>, 8);
            else if (d <= 16) launch(slice_advance_kernel<16, false>, 16);
            else if (d <= 32) launch(slice_advance_kernel<32, false>, 32);
            else launch(slice_advance_kernel<64, false>, 64);
        }
    }
    loglike_batch(m, thc, d, 2 * spec * k, S.llc, prec, S.ccount + round % 3, st);
}

// Speculative proposals per bracket end and round (1 .. MAX_SPEC): the
// request, else NSMI_SPEC, else the library's choice -- 2 for the CMB and
// test likelihoods while a round stays within 8192 rows (two proposals per end
// take the rounds per iteration from about 140 to 90 on the CMB workloads,
// more take them to about 75 while the batches, hence the likelihood's cost,
// grow), 1 for the shear likelihood (its cost grows with the rows from small
// batches on).
static int slice_spec(const ns_model* m, int64_t k, int requested) {
    int spec = requested;
    if (spec <= 0) {
        const char* e = getenv("NSMI_SPEC");
        spec = e ? atoi(e) : 0;
    }
    if (spec <= 0) spec = (m->kind == NS_MODEL_SHEAR || 4 * k > 8192) ? 1 : 2;
    return std::min(std::max(spec, 1), MAX_SPEC);
}

void slice_step(ns_model* m, double* u, double* logl, int* n_evals, int* n_stalls, int64_t k,
                const double* lstar_dev, const double* L, int n_inner, uint64_t seed, uint64_t iter, int prec,
                hipStream_t s) {
    const int d = m->d;
    NS_CHECK(d <= MAX_DIM, NS_E_UNSUPPORTED, "slice sampler supports d <= 64");
    if (k == 0) return;
    int64_t* iter_p = nullptr;
    const int spec = slice_spec(m, k, 0);
    SliceState S = carve_slice(m, k, d, spec, u, logl, n_evals, n_stalls, &iter_p);
    // up to 2 spec proposals per walker and round (both ends while stepping out)
    m->ws_theta.ensure((size_t)2 * spec * k * d * sizeof(double));
    PinnedHost flag(64);
    int* hflag = static_cast<int*>(flag.p);
    hipLaunchKernelGGL(slice_init_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, S, k, iter_p, iter);
    NS_HIP(hipGetLastError());
    const int64_t max_rounds = (int64_t)n_inner * (2 * MAX_EXPAND + MAX_SHRINK + 4) + 8;
    auto chunk = [&](hipStream_t st) {
        for (int c = 0; c < GRAPH_ROUNDS; ++c)
            advance_round(m, S, k, spec, lstar_dev, L, n_inner, seed, iter_p, c, prec, st);
        NS_HIP(hipGetLastError());
    };
    // first chunk eagerly on the caller's stream (sizes every workspace, tunes
    // launch shapes); the following chunks replay one captured graph on the
    // model's own stream, ordered after the caller's work
    GraphExec ge;
    hipStream_t run = s;
    int64_t rounds = 0;
    while (true) {
        if (rounds == 0 || !graphs_enabled(m)) {
            chunk(run);
        } else {
            if (!ge.e) {
                run = graph_stream_after(m, s);
                capture_graph(run, ge, chunk);
            }
            NS_HIP(hipGraphLaunch(ge.e, run));
        }
        rounds += GRAPH_ROUNDS;
        NS_HIP(hipMemcpyAsync(hflag, S.active + (GRAPH_ROUNDS - 1) % 3, sizeof(int), hipMemcpyDeviceToHost, run));
        NS_HIP(hipStreamSynchronize(run));
        if (*hflag == 0) break;
        NS_CHECK(rounds < max_rounds, NS_E_INVALID, "slice sampler did not terminate");
    }
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

// ------------------------------------------------------------ checkpoints
// File layout (native byte order): CkptHeader, then live u [n x d] and live
// logL [n] (double), dead logL [n_dead] (double), dead live counts [n_dead]
// (int32), dead u [n_dead x d] (double).
struct CkptHeader {
    char magic[8];                // "NSMICKP1"
    int32_t kind, d, n_data, n_live, n_delete, n_inner, precision, stop;
    uint64_t seed;
    double frac_remain;
    int64_t it, n_dead, n_evals, n_stalls;
    double logx, logz, lstar, live_term;
};

static void write_checkpoint(const char* path, const CkptHeader& h, const std::vector<double>& lu,
                             const std::vector<double>& ll, const std::vector<double>& dl,
                             const std::vector<int>& dn, const std::vector<double>& du) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    NS_CHECK(f != nullptr, NS_E_INVALID, std::string("cannot write checkpoint ") + tmp);
    bool ok = fwrite(&h, sizeof(h), 1, f) == 1;
    auto put = [&](const void* p, size_t bytes) {
        if (bytes) ok = ok && fwrite(p, 1, bytes, f) == bytes;
    };
    put(lu.data(), lu.size() * 8);
    put(ll.data(), ll.size() * 8);
    put(dl.data(), dl.size() * 8);
    put(dn.data(), dn.size() * 4);
    put(du.data(), du.size() * 8);
    ok = (fclose(f) == 0) && ok;
    NS_CHECK(ok, NS_E_INVALID, std::string("short write of checkpoint ") + tmp);
    NS_CHECK(rename(tmp.c_str(), path) == 0, NS_E_INVALID, std::string("cannot rename checkpoint to ") + path);
}

static bool read_checkpoint(const char* path, CkptHeader& h, std::vector<double>& lu, std::vector<double>& ll,
                            std::vector<double>& dl, std::vector<int>& dn, std::vector<double>& du) {
    FILE* f = fopen(path, "rb");
    if (!f) return false;
    std::unique_ptr<FILE, int (*)(FILE*)> guard(f, fclose);
    NS_CHECK(fread(&h, sizeof(h), 1, f) == 1 && memcmp(h.magic, "NSMICKP1", 8) == 0, NS_E_INVALID,
             std::string("not a checkpoint of this library: ") + path);
    NS_CHECK(h.d >= 1 && h.d <= MAX_DIM && h.n_live >= 2 && h.n_live <= 4096 && h.n_dead >= 0 &&
                 h.n_dead <= ((int64_t)1 << 40),
             NS_E_INVALID, std::string("corrupt checkpoint header: ") + path);
    lu.resize((size_t)h.n_live * h.d);
    ll.resize(h.n_live);
    dl.resize(h.n_dead);
    dn.resize(h.n_dead);
    du.resize((size_t)h.n_dead * h.d);
    bool ok = true;
    auto get = [&](void* p, size_t bytes) {
        if (bytes) ok = ok && fread(p, 1, bytes, f) == bytes;
    };
    get(lu.data(), lu.size() * 8);
    get(ll.data(), ll.size() * 8);
    get(dl.data(), dl.size() * 8);
    get(dn.data(), dn.size() * 4);
    get(du.data(), du.size() * 8);
    NS_CHECK(ok, NS_E_INVALID, std::string("truncated checkpoint: ") + path);
    return true;
}

// ------------------------------------------------------------------- ns_run
struct RunSnap {
    NSCtl ctl;
    NSState st;
};

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
    NS_CHECK(o->checkpoint_every >= 0, NS_E_INVALID, "checkpoint_every must be >= 0");
    NS_CHECK(o->resume == 0 || o->resume == 1, NS_E_INVALID, "resume must be 0 or 1");
    NS_CHECK(o->speculate >= 0 && o->speculate <= MAX_SPEC, NS_E_INVALID, "speculate must be in [0, 4]");
    const char* ckpt = (o->checkpoint_path && o->checkpoint_path[0]) ? o->checkpoint_path : nullptr;
    NS_CHECK(ckpt || (o->checkpoint_every == 0 && o->resume == 0), NS_E_INVALID,
             "checkpoint_every and resume need a checkpoint_path");
    EventPair tev(hipEventDefault);
    NS_HIP(hipEventRecord(tev.e[0], s));
    DevBuf live_u, live_l, order, wu, wl, wne, wns, L, snapd, dbuf, th, ev;
    DevBuf dl, dn, du;
    live_u.ensure((size_t)n * d * 8);
    live_l.ensure((size_t)n * 8);
    order.ensure((size_t)n * 4);
    wu.ensure((size_t)k * d * 8);
    wl.ensure((size_t)k * 8);
    wne.ensure((size_t)k * 4);
    wns.ensure((size_t)k * 4);
    L.ensure((size_t)d * d * 8);
    snapd.ensure(sizeof(RunSnap));                    // control and state side by side: one copy reads both
    dbuf.ensure(sizeof(DeadBuf));
    th.ensure((size_t)n * d * 8);
    NSState* S = &snapd.as<RunSnap>()->st;
    NSCtl* ctl = &snapd.as<RunSnap>()->ctl;
    int64_t dcap = 0;
    // (re)allocate the dead-point storage for at least `need` points, keeping the first n_keep
    auto grow_dead = [&](int64_t need, int64_t n_keep, hipStream_t st) {
        if (need <= dcap) return;
        const int64_t ncap = std::max<int64_t>(std::max<int64_t>(2 * dcap, need), 1024);
        DevBuf dl2, dn2, du2;
        dl2.ensure(ncap * 8);
        dn2.ensure(ncap * 4);
        du2.ensure(ncap * d * 8);
        if (n_keep > 0) {
            NS_HIP(hipMemcpyAsync(dl2.p, dl.p, n_keep * 8, hipMemcpyDeviceToDevice, st));
            NS_HIP(hipMemcpyAsync(dn2.p, dn.p, n_keep * 4, hipMemcpyDeviceToDevice, st));
            NS_HIP(hipMemcpyAsync(du2.p, du.p, n_keep * d * 8, hipMemcpyDeviceToDevice, st));
        }
        NS_HIP(hipStreamSynchronize(st));
        std::swap(dl.p, dl2.p); std::swap(dl.bytes, dl2.bytes);
        std::swap(dn.p, dn2.p); std::swap(dn.bytes, dn2.bytes);
        std::swap(du.p, du2.p); std::swap(du.bytes, du2.bytes);
        dcap = ncap;
        const DeadBuf hb{dl.as<double>(), dn.as<int>(), du.as<double>(), dcap};
        NS_HIP(hipMemcpy(dbuf.p, &hb, sizeof(hb), hipMemcpyHostToDevice));
    };

    // ---- start: fresh live points, or the state of a checkpoint
    CkptHeader hdr{};
    std::vector<double> c_lu, c_ll, c_dl, c_du;
    std::vector<int> c_dn;
    bool resumed = false;
    if (ckpt && o->resume && read_checkpoint(ckpt, hdr, c_lu, c_ll, c_dl, c_dn, c_du)) {
        NS_CHECK(hdr.kind == m->kind && hdr.d == d && hdr.n_data == m->n_data && hdr.n_live == n &&
                     hdr.n_delete == k && hdr.n_inner == o->n_inner && hdr.precision == o->precision &&
                     hdr.seed == o->seed && hdr.frac_remain == o->frac_remain,
                 NS_E_INVALID, std::string("checkpoint ") + ckpt + " belongs to another model or other run options");
        resumed = true;
    }
    NSCtl hc{};
    hc.max_iter = o->max_iter;
    hc.ckpt_every = ckpt ? o->checkpoint_every : 0;
    if (resumed) {
        grow_dead(std::max<int64_t>(4 * (int64_t)n, hdr.n_dead + k + n), 0, s);
        NS_HIP(hipMemcpy(live_u.p, c_lu.data(), c_lu.size() * 8, hipMemcpyHostToDevice));
        NS_HIP(hipMemcpy(live_l.p, c_ll.data(), c_ll.size() * 8, hipMemcpyHostToDevice));
        if (hdr.n_dead > 0) {
            NS_HIP(hipMemcpy(dl.p, c_dl.data(), c_dl.size() * 8, hipMemcpyHostToDevice));
            NS_HIP(hipMemcpy(dn.p, c_dn.data(), c_dn.size() * 4, hipMemcpyHostToDevice));
            NS_HIP(hipMemcpy(du.p, c_du.data(), c_du.size() * 8, hipMemcpyHostToDevice));
        }
        NSState hs{hdr.logx, hdr.logz, hdr.lstar, hdr.live_term, hdr.n_dead, hdr.n_evals, hdr.n_stalls, hdr.stop};
        NS_HIP(hipMemcpy(S, &hs, sizeof(hs), hipMemcpyHostToDevice));
        hc.it = hdr.it;
        hc.need_begin = hdr.stop ? 0 : 1;
        hc.done = hdr.stop ? 1 : (hdr.it >= o->max_iter ? 2 : 0);
        if (hc.done) hc.need_begin = 0;
    } else {
        grow_dead(std::max<int64_t>(4 * (int64_t)n, 1024), 0, s);
        hipLaunchKernelGGL(ns_init_kernel, dim3((unsigned)(((int64_t)n * d + 255) / 256)), dim3(256), 0, s,
                           live_u.as<double>(), n, d, o->seed, S);
        NS_HIP(hipGetLastError());
        prior_transform(m, live_u.as<double>(), th.as<double>(), d, n, nullptr, s);
        loglike_batch(m, th.as<double>(), d, n, live_l.as<double>(), o->precision, nullptr, s);
        hc.it = 0;
        hc.need_begin = 1;
    }
    NS_HIP(hipMemcpyAsync(ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s));
    NS_HIP(hipStreamSynchronize(s));

    // ---- the device-driven iteration
    int64_t* iter_unused = nullptr;
    const int spec = slice_spec(m, k, o->speculate);
    SliceState W = carve_slice(m, k, d, spec, wu.as<double>(), wl.as<double>(), wne.as<int>(), wns.as<int>(),
                               &iter_unused);
    m->ws_theta.ensure((size_t)2 * spec * k * d * sizeof(double));
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, W.ccount, 3);
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, W.active, 3);
    NS_HIP(hipGetLastError());
    const double log_frac = log(o->frac_remain);
    const double* lstar_dev = reinterpret_cast<const double*>(reinterpret_cast<const char*>(S) + offsetof(NSState, lstar));
    const int64_t* it_dev = reinterpret_cast<const int64_t*>(reinterpret_cast<const char*>(ctl) + offsetof(NSCtl, it));
    auto block = [&](hipStream_t st) {
        for (int c = 0; c < GRAPH_ROUNDS; ++c) {
            if (c % CTL_EVERY == 0) {
                TraceScope ts(m, st, "ns_control");
                hipLaunchKernelGGL(ns_control_kernel, dim3(1), dim3(CTL_NT), 0, st, ctl, S, dbuf.as<DeadBuf>(), W,
                                   live_u.as<double>(), live_l.as<double>(), order.as<int>(), L.as<double>(), n, k,
                                   d, o->seed, log_frac, c);
            }
            advance_round(m, W, k, spec, lstar_dev, L.as<double>(), o->n_inner, o->seed, it_dev, c, o->precision, st);
        }
        NS_HIP(hipGetLastError());
    };
    hipStream_t st = graphs_enabled(m) ? graph_stream_after(m, s) : s;
    PinnedHost pin(2 * sizeof(RunSnap));
    RunSnap* snap = static_cast<RunSnap*>(pin.p);
    EventPair sev(hipEventDisableTiming);
    GraphExec ge;
    auto launch = [&]() {
        if (ge.e) NS_HIP(hipGraphLaunch(ge.e, st));
        else block(st);
    };
    auto snapshot = [&](int i) {
        NS_HIP(hipMemcpyAsync(&snap[i], snapd.p, sizeof(RunSnap), hipMemcpyDeviceToHost, st));
        NS_HIP(hipEventRecord(sev.e[i], st));
    };
    // the first launch runs eagerly: it sizes every workspace and tunes the
    // likelihood's launch shapes before anything is captured
    block(st);
    snapshot(0);
    NS_HIP(hipEventSynchronize(sev.e[0]));
    if (graphs_enabled(m)) capture_graph(st, ge, block);
    const int64_t max_graphs_per_iter =
        ((int64_t)o->n_inner * (2 * MAX_EXPAND + MAX_SHRINK + 4) + 8) / GRAPH_ROUNDS + 3;
    int64_t last_it = -1, same_it = 0;
    int cur = 0;
    RunSnap h = snap[0];
    auto write_ckpt = [&](const RunSnap& hs) {
        CkptHeader w{};
        memcpy(w.magic, "NSMICKP1", 8);
        w.kind = m->kind; w.d = d; w.n_data = m->n_data; w.n_live = n; w.n_delete = k;
        w.n_inner = o->n_inner; w.precision = o->precision; w.stop = hs.st.stop;
        w.seed = o->seed; w.frac_remain = o->frac_remain;
        w.it = hs.ctl.it; w.n_dead = hs.st.n_dead; w.n_evals = hs.st.n_evals; w.n_stalls = hs.st.n_stalls;
        w.logx = hs.st.logx; w.logz = hs.st.logz; w.lstar = hs.st.lstar; w.live_term = hs.st.live_term;
        std::vector<double> lu((size_t)n * d), ll(n), dlv(hs.st.n_dead), duv((size_t)hs.st.n_dead * d);
        std::vector<int> dnv(hs.st.n_dead);
        NS_HIP(hipMemcpy(lu.data(), live_u.p, lu.size() * 8, hipMemcpyDeviceToHost));
        NS_HIP(hipMemcpy(ll.data(), live_l.p, ll.size() * 8, hipMemcpyDeviceToHost));
        if (hs.st.n_dead > 0) {
            NS_HIP(hipMemcpy(dlv.data(), dl.p, dlv.size() * 8, hipMemcpyDeviceToHost));
            NS_HIP(hipMemcpy(dnv.data(), dn.p, dnv.size() * 4, hipMemcpyDeviceToHost));
            NS_HIP(hipMemcpy(duv.data(), du.p, duv.size() * 8, hipMemcpyDeviceToHost));
        }
        write_checkpoint(ckpt, w, lu, ll, dlv, dnv, duv);
    };
    while (true) {
        if (!h.ctl.done && !h.ctl.pause && !h.ctl.grow) {
            // one launch in flight beyond the state being read
            launch();
            snapshot(cur ^ 1);
            NS_HIP(hipEventSynchronize(sev.e[cur]));
            h = snap[cur];
            cur ^= 1;
            if (!(h.ctl.done || h.ctl.pause || h.ctl.grow)) {
                if (h.ctl.it == last_it && h.ctl.walking) {
                    NS_CHECK(++same_it <= max_graphs_per_iter, NS_E_INVALID, "slice sampler did not terminate");
                } else {
                    last_it = h.ctl.it;
                    same_it = 0;
                }
                continue;
            }
            // the launch in flight started nothing new: wait for it
            NS_HIP(hipEventSynchronize(sev.e[cur]));
            h = snap[cur];
        }
        if (h.ctl.done) break;
        if (h.ctl.pause) {
            write_ckpt(h);
            h.ctl.pause = 0;
        }
        if (h.ctl.grow) {
            grow_dead(h.st.n_dead + k + n, h.st.n_dead, st);
            h.ctl.grow = 0;
        }
        h.ctl.need_begin = 1;
        NS_HIP(hipMemcpy(ctl, &h.ctl, sizeof(NSCtl), hipMemcpyHostToDevice));
        launch();
        snapshot(cur);
        NS_HIP(hipEventSynchronize(sev.e[cur]));
        h = snap[cur];
    }
    NS_HIP(hipStreamSynchronize(st));
    if (ckpt && h.ctl.done == 2) write_ckpt(h);        // a run ended by max_iter can be continued

    // ---- final: live points in ascending order, then log Z, H and the replicates
    int64_t n_dead = h.st.n_dead;
    grow_dead(n_dead + n, n_dead, st);
    hipLaunchKernelGGL(ns_sort_kernel, dim3(1), dim3(CTL_NT), 0, st, live_l.as<double>(), n, order.as<int>());
    hipLaunchKernelGGL(ns_final_kernel, dim3(1), dim3(256), 0, st, live_l.as<double>(), live_u.as<double>(),
                       order.as<int>(), n, d, S, dl.as<double>(), dn.as<int>(), du.as<double>(), dcap);
    const int64_t M = n_dead + n;
    const int R = o->n_replicates;
    ev.ensure((size_t)(2 + std::max(R, 1)) * 8);
    hipLaunchKernelGGL(ns_evidence_kernel, dim3(1), dim3(1024), 0, st, dl.as<double>(), dn.as<int>(), M,
                       ev.as<double>());
    if (R > 0)
        hipLaunchKernelGGL(ns_replicates_kernel, dim3((unsigned)R), dim3(256), 0, st, dl.as<double>(),
                           dn.as<int>(), M, R, o->seed, ev.as<double>() + 2);
    NS_HIP(hipGetLastError());
    std::vector<double> evh(2 + std::max(R, 1));
    NS_HIP(hipMemcpyAsync(evh.data(), ev.p, evh.size() * 8, hipMemcpyDeviceToHost, st));
    NS_HIP(hipStreamSynchronize(st));
    NS_HIP(hipEventRecord(tev.e[1], s));
    NS_HIP(hipEventSynchronize(tev.e[1]));
    float ms = 0.f;
    NS_HIP(hipEventElapsedTime(&ms, tev.e[0], tev.e[1]));
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
    res->n_iter = h.ctl.it;
    res->n_evals = h.st.n_evals;
    res->n_stalls = h.st.n_stalls;
    res->n_dead = M;
    res->wall_s = ms * 1e-3;
    res->resumed_iter = resumed ? hdr.it : 0;
}

}  // namespace nsmi
