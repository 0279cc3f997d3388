/*
 * ns.h -- C ABI of the MI355X batched-likelihood and nested-slice-sampling
 * library (libnsmi.so).
 *
 * The library evaluates, for thousands of walkers at once, the log-likelihoods
 * of the paper "High-Dimensional Bayesian Model Comparison in Cosmology with
 * GPU-accelerated Nested Sampling and Neural Emulators" (Lovick et al.,
 * arXiv:2509.13307) and runs nested slice sampling on them:
 *
 *   - neural-emulator likelihoods of CMB spectra (Sec. 2.3-2.4): the
 *     cosmic-variance-limited TT likelihood of Sec. 2.4 and Gaussian chi^2
 *     forms of the same emulators,
 *   - the tomographic cosmic-shear likelihood of Sec. 2.5 and App. A:
 *     emulated P(k, z) (on every redshift node, or on a coarser grid
 *     interpolated in z as in App. B),
 *     extended Limber projection Eq. (A2) with lensing and intrinsic-alignment
 *     windows Eqs. (A3)-(A4), summed as in Eq. (A1), multiplicative shear bias
 *     and photo-z shifts, and a dense-covariance Gaussian,
 *   - nested sampling with k-deletion (Sec. 2.1-2.2) and the evidence of
 *     Eq. (1), from which Bayes factors follow by Eq. (2).
 *
 * Conventions shared by every entry point
 *   - Every function returns ns_status: 0 on success, a negative code on
 *     failure.  No function throws or aborts across the ABI; the message of
 *     the last failure on the calling thread is returned by ns_last_error().
 *   - Pointers marked "device" are HIP device memory on the model's device;
 *     "host" pointers are ordinary CPU memory.  The caller owns every buffer
 *     it passes and keeps it alive until the work queued on `stream` that
 *     uses it has completed; the library never frees or retains caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Arguments are validated before any launch; a rejected call queues
 *     nothing.
 *   - Parameters theta are in physical units, row-major [B x ld], ld >= d.
 *     A theta outside a uniform prior's [a, b] has logL = -inf and gradient 0
 *     (not an error: the sampler relies on it).  A NaN theta gives NaN.
 *   - Calls on one model must not overlap in time unless they are queued on
 *     the same stream (the model's workspaces are shared).  Different models
 *     are independent.
 */
#ifndef NS_H
#define NS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NS_OK = 0,
    NS_E_INVALID = -1,     /* null pointer, bad enum, bad scalar argument     */
    NS_E_SHAPE = -2,       /* inconsistent sizes                              */
    NS_E_HIP = -3,         /* a HIP runtime call failed                       */
    NS_E_NOMEM = -4,       /* device or host allocation failed                */
    NS_E_NOT_SPD = -5,     /* covariance not symmetric positive definite      */
    NS_E_UNSUPPORTED = -6  /* valid request this build does not implement     */
} ns_status;
/* A slice step whose bracket collapses without finding a point inside the
 * constraint keeps its walker where it was and is counted (n_stalls of
 * ns_slice_step, ns_run_result.n_stalls); it is not an error, so there is no
 * stall status code. */

/* Arithmetic of the emulator and projection stages.  The final Gaussian
 * chi^2 (Cholesky whitening, reductions) and all sampler bookkeeping are FP64
 * in every form. */
typedef enum {
    NS_FP64 = 0,   /* everything in double                                   */
    NS_FP32 = 1,   /* emulator and Limber stages in float                    */
    NS_BF16 = 2,   /* hidden and output layers on BF16 MFMA, FP32 accumulate;
                      first layer, output transform and Limber in FP32       */
    NS_BF16X3 = 3  /* as NS_BF16 with weights and activations split into
                      hi + lo BF16 parts, three MFMA products per tile       */
} ns_precision;

typedef enum {
    NS_MODEL_CMB_DIAG = 0,   /* one emulator, Gaussian with diagonal covariance */
    NS_MODEL_CMB_BLOCK = 1,  /* TT, TE, EE, PP emulators; 3x3 block + diagonal  */
    NS_MODEL_SHEAR = 2,      /* cosmic shear, Sec. 2.5 and App. A               */
    NS_MODEL_GAUSS = 3,      /* diagonal Gaussian in theta (closed-form evidence) */
    NS_MODEL_CMB_CV = 4      /* TT emulator, cosmic-variance-limited likelihood:
                                (2l+1) Ch_l / C_l ~ chi^2 with 2l+1 d.o.f. (Sec. 2.4) */
} ns_model_kind;

enum { NS_PRIOR_UNIFORM = 0, NS_PRIOR_NORMAL = 1 };

/* One emulator network (Sec. 2.2, 2.4 and 2.5: CosmoPower-style MLP):
 *   x   = (inputs - in_shift) / in_scale
 *   h_l = f_l(W_l h_{l-1} + b_l),  f_l(t) = (gamma_l + (1 - gamma_l) sigmoid(beta_l t)) t
 *   y   = out_mu + out_sigma * (W_L h_{L-1} + b_L)
 * All arrays are host memory, copied at ns_model_create. */
typedef struct ns_net_desc {
    int32_t n_layers;             /* L >= 2 affine layers (L-1 hidden)         */
    const int32_t* dims;          /* [L+1]: dims[0] inputs ... dims[L] outputs  */
    const double* const* W;       /* [L] row-major [dims[l+1] x dims[l]]        */
    const double* const* b;       /* [L] [dims[l+1]]                            */
    const double* const* beta;    /* [L-1] [dims[l+1]]                          */
    const double* const* gamma;   /* [L-1] [dims[l+1]]                          */
    const double* in_shift;       /* [dims[0]]                                  */
    const double* in_scale;       /* [dims[0]]                                  */
    const double* out_mu;         /* [dims[L]] (CMB) or [n_z x dims[L]] (shear) */
    const double* out_sigma;      /* [dims[L]]                                  */
} ns_net_desc;

/* Model description (host memory; copied at creation, may be freed after). */
typedef struct ns_model_desc {
    int32_t kind;                 /* ns_model_kind                              */
    int32_t d;                    /* sampled parameters                         */
    const int32_t* prior_kind;    /* [d] NS_PRIOR_*                             */
    const double* prior_a;        /* [d] uniform lower bound / normal mean      */
    const double* prior_b;        /* [d] uniform upper bound / normal sigma     */

    int32_t n_nets;               /* CMB_DIAG 1, CMB_BLOCK 4, SHEAR 1, GAUSS 0,
                                     CMB_CV 1 (outputs log10 C_l, spec_log 1)   */
    const ns_net_desc* nets;
    const int32_t* spec_log;      /* CMB: [n_nets], 1 -> C = 10^y, 0 -> C = y    */

    int32_t n_data;               /* data vector length                         */
    const double* data;           /* [n_data]; CMB_CV: observed Ch_l > 0 at
                                     l = ell_min, ell_min + 1, ...               */
    const double* sigma;          /* CMB_DIAG: [n_data] standard deviations     */
    const double* cov_blocks;     /* CMB_BLOCK: [n_ell x 3 x 3] (TT, TE, EE)    */
    const double* sigma_pp;       /* CMB_BLOCK: [n_ell]                         */
    const double* cov;            /* SHEAR: [n_data x n_data] row-major,
                                     n_data = n_pairs n_ell <= 1248              */

    /* SHEAR geometry (App. A) */
    int32_t n_bins;               /* tomographic bins (<= 10)                   */
    const double* nz_mean;        /* [n_bins] Gaussian n(z) means               */
    double nz_sigma;              /* Gaussian n(z) width                        */
    int32_t n_a;                  /* scale-factor nodes, a = 1 .. a_min (<= 2048) */
    double a_min;
    int32_t n_z;                  /* emulator redshift nodes (see z_interp)     */
    double k_min, k_max;          /* emulated k range [1/Mpc], log-spaced       */
    int32_t n_k;
    double ell_min, ell_max;      /* SHEAR: log-spaced multipoles; CMB_CV:
                                     ell_min = first multipole (integer >= 0)    */
    int32_t n_ell;                /* SHEAR: <= 32                               */
    const int32_t* pidx;          /* [9 + 3 n_bins] theta index per physical slot
                                     (omega_b, omega_cdm, h, n_s, lnAs, w0, wa,
                                      c_min, eta0, A_IA.., Dz.., m..), -1 = fixed */
    const double* pfix;           /* [9 + 3 n_bins] values of fixed slots       */

    /* GAUSS */
    const double* mu;             /* [d]                                        */
    const double* gsigma;         /* [d]                                        */

    /* SHEAR: how the emulated log10 P reaches the z of every a-node (App. B).
     * 0: not-a-knot cubic spline over n_z nodes uniform on [0, 1/a_min - 1]
     *    (4 <= n_z <= 256);
     * 1: linear in z over n_z nodes at scale factors evenly spaced from 1 to
     *    a_min (2 <= n_z <= n_a); n_z = n_a puts a node on every a-node (the
     *    paper's full likelihood), n_z ~ n_a / 10 is its interpolated one. */
    int32_t z_interp;
} ns_model_desc;

typedef struct ns_model ns_model; /* opaque, library-owned */

/* Create a model on HIP device `device`: the likelihood L(theta) and prior
 * pi(theta) of the evidence integral Eq. (1) -- priors of Table 1, emulator
 * networks (Sec. 2.2), the CMB likelihoods (Sec. 2.3-2.4) or the cosmic-shear
 * likelihood (Sec. 2.5, App. A-B).  Copies weights, data and grids to the
 * device and factorises the covariance in FP64 on the host.  *out receives a
 * library-owned handle (release with ns_model_free).
 * Errors: NS_E_INVALID / NS_E_SHAPE for bad descriptions, NS_E_NOT_SPD when a
 * covariance (block) has no Cholesky factor, NS_E_HIP / NS_E_NOMEM. */
ns_status ns_model_create(const ns_model_desc* desc, int32_t device, ns_model** out);

/* Release a model and its device memory (synchronises the device). NULL is a no-op. */
ns_status ns_model_free(ns_model* model);

/* Number of sampled parameters of a model. */
ns_status ns_model_dim(const ns_model* model, int32_t* d);

/* Prior transform (Table 1): u in the unit cube -> theta.
 *   uniform U(a, b): a + (b - a) u;   normal N(mu, s): mu + s sqrt(2) erfinv(2u - 1)
 * u, theta: device [B x ld] row-major (may alias).  Asynchronous on stream. */
ns_status ns_prior_transform(ns_model* model, const double* u, double* theta, int64_t ld,
                             int64_t B, void* stream);

/* Batched log-likelihood logL(theta_b), b < B: the likelihood of Eq. (1)
 * evaluated for many parameter points at once, which Sec. 2.2 names the
 * bottleneck of the parallel sampler (emulator -> [Limber projection Eqs.
 * (A1)-(A4) + nuisances] -> Gaussian chi^2, or the cosmic-variance sum of
 * Sec. 2.4).  All constants are included (logL is a normalised density of the
 * data), so log Z from it is a normalised evidence.
 * theta: device [B x ld] (caller-owned, read only); logl: device [B]
 * (caller-owned, written).  Asynchronous on stream.
 * B = 0 is a no-op.  NS_E_UNSUPPORTED for precisions a model kind lacks. */
ns_status ns_loglike_batch(ns_model* model, const double* theta, int64_t ld, int64_t B,
                           double* logl, int32_t precision, void* stream);

/* ns_loglike_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same results, bitwise, with the
 * emulator's model vector in a library-owned device array of 64 MiB per GPU
 * (set up when the first model is created on that GPU and held until the
 * process ends) instead of the model's grow-on-demand workspace; no
 * allocation, no launch-shape tuning runs (the shape tuned by an earlier
 * ns_loglike_batch call of the same batch size, else the first candidate) and
 * no trace events.
 * Covers the CMB model kinds in the NS_BF16 / NS_BF16X3 forms of one-kernel
 * emulator networks (hidden widths 128 or 512), and NS_FP64 on a narrow
 * CMB_DIAG model (hidden width 128: emulator and chi^2 in one kernel, no
 * scratch); NS_E_UNSUPPORTED otherwise.  The array holds the model vectors of
 * at most 64 MiB / (4 x row length) walkers (1 658 for the four-spectrum
 * 2 x 2500-multipole model); larger B is NS_E_SHAPE, nothing launched.
 * All calls on one GPU share the array: calls that overlap in time on one GPU
 * (any models, any streams) race and must be ordered by the caller.
 * theta: device [B x ld]; logl: device [B]; both caller-owned.  Asynchronous
 * on stream. */
ns_status ns_loglike_batch_noalloc(ns_model* model, const double* theta, int64_t ld, int64_t B,
                                   double* logl, int32_t precision, void* stream);

/* Theory vector of every walker: the prediction the likelihood compares with
 * the data, in the data's order, after every stage before the chi^2 (or the
 * cosmic-variance sum), by the same kernels as ns_loglike_batch.
 *   CMB_DIAG: the emulator outputs y (Sec. 2.3); CMB_BLOCK: C^TT | C^TE |
 *   C^EE | C^pp, each n_ell long, C = 10^y where spec_log is 1; CMB_CV:
 *   C^TT_l = 10^y; SHEAR: C_ij(l_b) after the multiplicative bias
 *   (Eqs. (A1)-(A4)), pairs i <= j in lexicographic order, then l_b.
 * theta: device [B x ld]; out: device [B x ldo] double, ldo >= n_data; both
 * caller-owned.  Rows of theta outside the prior support are computed all the
 * same (the support test belongs to the likelihood).  Asynchronous on stream.
 * NS_E_UNSUPPORTED for GAUSS; NS_E_SHAPE for ldo < n_data or B > 2^24;
 * B = 0 is a no-op. */
ns_status ns_theory_batch(ns_model* model, const double* theta, int64_t ld, int64_t B,
                          double* out, int64_t ldo, int32_t precision, void* stream);

/* As ns_loglike_batch, plus grad: device [B x d] (caller-owned, written),
 * d logL / d theta by the hand-written adjoint of every stage (input
 * gradients only): the gradients that Sec. 2.2 notes an automatically
 * differentiable likelihood makes available to gradient-based samplers
 * (Sec. 4.2).  Rows outside the prior support get logL = -inf and grad = 0.
 * FP64 form: every stage in double; the reduced forms run the forward pass in
 * their form and the adjoint in FP32.  Deterministic: repeated calls give
 * bitwise equal results.  Asynchronous on stream. */
ns_status ns_loglike_grad_batch(ns_model* model, const double* theta, int64_t ld, int64_t B,
                                double* logl, double* grad, int32_t precision, void* stream);

/* n_inner hit-and-run slice steps (Sec. 2.1; Neal 2003) for k walkers in the
 * unit cube under the hard constraint logL(T(u)) > logl_star:
 *   u:        device [k x d] in/out (start points must satisfy the constraint)
 *   logl:     device [k] in/out
 *   n_evals:  device [k] out, likelihood evaluations per walker
 *   n_stalls: device [k] out, steps that kept their point (bracket collapsed)
 *   dir_chol: device [d x d] lower-triangular factor of the direction
 *             covariance (row-major)
 * Random numbers: Philox4x64-10, key (seed, 0), counter (q/4, walker, step,
 * iter), word q mod 4, U = (w >> 11) 2^-53; per step s (1..n_inner): draws
 * 0..2d-1 give d Box-Muller normals, draw 2d the bracket offset, then one
 * draw per shrink.  Step-out at most 10 per end, stall when the bracket is
 * narrower than 1e-12 or after 200 shrinks.
 * The walkers advance in rounds of one batched likelihood call.  A walker may
 * propose several of its next points in one round: the stepping-out points
 * of an end and the chain of shrink points that follow one another if each
 * is rejected are fixed before any evaluation, so the results are applied in
 * the serial order and u, logl, n_evals and n_stalls are exactly those of
 * one proposal at a time (evaluations past the deciding one are not counted).
 * The number per end and round is the library's choice (environment
 * NSMI_SPEC = 1..4 sets it).
 * Synchronises `stream` (the host polls a completion flag). */
ns_status ns_slice_step(ns_model* model, double* u, double* logl, int32_t* n_evals,
                        int32_t* n_stalls, int64_t k, double logl_star, const double* dir_chol,
                        int32_t n_inner, uint64_t seed, uint64_t iter, int32_t precision,
                        void* stream);

typedef struct ns_run_opts {
    int32_t n_live;          /* live points n (2 .. 4096)                       */
    int32_t n_delete;        /* k deleted and evolved in parallel per iteration */
    int32_t n_inner;         /* slice steps per walker per iteration            */
    int32_t precision;       /* ns_precision of the likelihood                  */
    double frac_remain;      /* stop when the live share of Z falls below this  */
    uint64_t seed;
    int32_t max_iter;
    int32_t n_replicates;    /* shrinkage replicates for sigma(log Z)           */
    const char* checkpoint_path; /* host, NUL-terminated file name, or NULL    */
    int32_t checkpoint_every;    /* > 0: write the run's state after every
                                    iteration that is a multiple of this       */
    int32_t resume;              /* 1: continue from checkpoint_path if that
                                    file exists (else start afresh)            */
    int32_t speculate;           /* slice proposals per bracket end and round,
                                    1..4 (0: the library's choice); any value
                                    gives the same result, see ns_slice_step   */
} ns_run_opts;

typedef struct ns_run_result {
    double logz;             /* log Z, Eq. (1), FP64 logsumexp                  */
    double sigma;            /* std of log Z over shrinkage replicates          */
    double sigma_skilling;   /* sqrt(H / n)                                     */
    double h;                /* information H                                   */
    int64_t n_iter;
    int64_t n_evals;
    int64_t n_stalls;
    int64_t n_dead;
    double wall_s;           /* wall time of this call                          */
    int64_t resumed_iter;    /* iteration the run continued from (0: fresh)     */
} ns_run_result;

/* Nested slice sampling to convergence (Sec. 2.1-2.2): k-deletion, slice
 * steps with live-covariance directions, FP64 evidence accumulation.
 * Optional outputs (host, may be NULL): dead_logl [capacity], dead_n
 * [capacity], dead_u [capacity x d]; if the run produces more than `capacity`
 * dead points only the first `capacity` are written (result->n_dead has the
 * total).  Synchronous.
 * Checkpoints: with checkpoint_path set, the state at the end of an iteration
 * (live points, dead points, evidence accumulators, iteration index) is
 * written to that file after every checkpoint_every-th iteration and when
 * max_iter ends the run (written to "<path>.tmp", then renamed).  A call with
 * resume = 1 and the same model and options (n_live, n_delete, n_inner,
 * precision, seed, frac_remain; max_iter may grow) continues from the file:
 * every random number is addressed by (seed, iteration, walker, step, draw)
 * and every reduction has a fixed order, so the continued run gives bitwise
 * the result of an uninterrupted one.  NS_E_INVALID if the file is not a
 * checkpoint of this library or belongs to other options. */
ns_status ns_run(ns_model* model, const ns_run_opts* opts, ns_run_result* result,
                 double* dead_logl, int32_t* dead_n, double* dead_u, int64_t capacity,
                 void* stream);

typedef struct ns_hmc_opts {
    int32_t n_chains;        /* C >= 1 chains advanced together                */
    int32_t n_iter;          /* trajectories per chain (>= 0)                  */
    int32_t n_leapfrog;      /* L >= 1 leapfrog steps per trajectory           */
    int32_t precision;       /* ns_precision of the likelihood and its gradient */
    double step;             /* leapfrog step eps > 0                          */
    uint64_t seed;
} ns_hmc_opts;

typedef struct ns_hmc_result {
    int64_t n_accept;        /* accepted trajectories over all chains          */
    int64_t n_left;          /* trajectories rejected for leaving the support  */
    int64_t n_grad;          /* gradient evaluations per chain                 */
    double wall_s;
} ns_hmc_result;

/* Hamiltonian Monte Carlo on the same posterior, with the gradient of
 * ns_loglike_grad_batch (gradients of the emulated likelihood, Sec. 2.2;
 * Duane et al. 1987, Neal 2011): target log pi = logL + log prior (normal
 * priors -(theta - mu)^2 / (2 sigma^2), uniform priors 0 inside their box,
 * -inf outside the support), momenta p ~ N(0, diag(1 / inv_mass)),
 * H = -log pi + sum_i inv_mass_i p_i^2 / 2, L leapfrog steps of size step,
 * Metropolis accept with probability min(1, exp(H0 - H1)).  A drift that
 * crosses a wall of a uniform prior is mirrored back (x -> b - (x - b), that
 * momentum component negated; Neal 2011, Sec. 5.5.1), at most 64 walls per
 * drift; a trajectory that still meets log pi = -inf is rejected
 * (result->n_left).
 *   inv_mass: device [d], > 0
 *   theta:    device [C x d] in: start points, out: last state
 *   samples:  device [n_iter x C x d] or NULL: state after each trajectory
 *   logp:     device [n_iter x C] or NULL: log pi of those states
 * Random numbers: Philox4x64-10 as for ns_slice_step, key (seed, 2) for the
 * momenta (draws 2i, 2i+1 of (chain, 0, iteration) -> Box-Muller normal z_i,
 * p_i = z_i / sqrt(inv_mass_i)) and key (seed, 3) for the accept uniform u
 * (draw 0 of (chain, 0, iteration); accept iff log u < H0 - H1).  Every update
 * is a separately rounded FP64 operation, sums run in parameter order.
 * NS_E_INVALID / NS_E_SHAPE for bad options; synchronises `stream`. */
ns_status ns_hmc(ns_model* model, const ns_hmc_opts* opts, const double* inv_mass, double* theta,
                 double* samples, double* logp, ns_hmc_result* result, void* stream);

/* Kernel tracing (instrumentation, no paper passage): while enabled, every
 * kernel the library launches for `model` is bracketed by a pair of HIP
 * events recorded on its launch stream.  Enabling or disabling synchronises
 * the device and discards pending records. */
ns_status ns_trace_enable(ns_model* model, int32_t enable);

/* Synchronise the device and write the traced kernels since the last report
 * as JSON {"kernel": [launches, total_ms], ...} into buf (host, buf_len bytes,
 * NUL-terminated; NS_E_SHAPE if it does not fit).  Clears the records. */
ns_status ns_trace_report(ns_model* model, char* buf, int64_t buf_len);

/* Launch shapes the library's autotuner has chosen for this model so far
 * (measured or read from the on-disk cache): BF16 GEMM tiles of the
 * layer-by-layer path and launch shapes of the one-kernel BF16 / BF16X3
 * emulator forward, as JSON {"<kind> M=.. N=.. K=.. networks=..": "<shape>"}
 * (host buf, NUL-terminated; NS_E_SHAPE if it does not fit).  Every
 * candidate accumulates in the same order, so the choice never changes a
 * result.  Environment: NSMI_NO_AUTOTUNE keeps the first candidate;
 * NSMI_FUSED_CFG=c pins candidate c (0-9 at hidden width 128 and for BF16 at
 * 512, 0-7 for BF16X3 at 512) of the one-kernel forward; NSMI_NO_FUSED_MLP
 * selects the layer-by-layer forward; NSMI_NO_FUSED_CHI2 stages the chi^2 of
 * the one-network CMB models after the one-kernel forward instead of adding
 * it in the forward's epilogue (results equal to 1e-12 relative: the same
 * terms summed in another order); NSMI_TUNE_CACHE names the on-disk
 * cache of choices ("off": none; default $XDG_CACHE_HOME/nsmi/tune.txt or
 * $HOME/.cache/nsmi/tune.txt), read by ns_model_create for the device's GPU
 * architecture and appended to on every new choice. */
ns_status ns_tuning_report(ns_model* model, char* buf, int64_t buf_len);

/* Message of the last failed call on this thread ("" if none). */
const char* ns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NS_H */
