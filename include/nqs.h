/*
 * nqs.h -- C interface of libnqs, the MI355X (gfx950) library for
 * mixed-precision Metropolis-Hastings sampling of neural quantum states.
 *
 * The operations follow "Neural Quantum States in Mixed Precision"
 * (arXiv 2601.20782):
 *   nqs_downcast       FP64 master -> reduced-precision sampling copy
 *                      (two-copy scheme, Sec. IV.B; formats of App. A, Table A)
 *   nqs_sample         Metropolis-Hastings sampling of pi = |psi|^2 / sum |psi|^2
 *                      (Sec. II, Eq. eq:loss; acceptance Sec. III.A; single-flip
 *                      proposal App. C Eq. eq:app:local_prop; exchange move App. E)
 *   nqs_sample_noisy   the same sampler on log pi + zeta(x), zeta fixed per x
 *                      (Sec. IV.A, Eq. eq:pert_chain)
 *   nqs_local_energy   eps(x) = sum_{x'} H(x,x') psi(x')/psi(x)
 *                      (App. I.1, Eq. eq:local_energies; TFIM Eq. eq:TFIM; Heisenberg App. E)
 *   nqs_energy_stats   FP64 mean / variance / error bar of the local energies (Eq. eq:loss)
 *   nqs_logpsi_grad    O_k(x) = d log psi(x) / d theta_k (App. I.1, Eq. eq:forces)
 *   nqs_forces         F = E[O eps] - E[O] E[eps] (Eq. eq:forces), FP64
 *   nqs_logpsi_grad_cols  a column block of O (same equation)
 *   nqs_gram           S = E[Obar^T Obar] (Eq. eq:smat) or its sample-space twin
 *                      T = Obar Obar^T / n, FP32 matrix cores
 *   nqs_sample_gram    T accumulated over column blocks of O, so that O is
 *                      never held whole (large networks)
 *   nqs_sample_gram_factored  the same T from the per-layer factors of O, FP64
 *   nqs_sr_solve / nqs_sr_update  the stochastic-reconfiguration step in
 *                      sample space: (T + shift) y = eps - mean eps, then
 *                      master -= lr O^T (y - mean y) / n (App. I.2)
 *   nqs_sr_solve_mixed the same solve preconditioned by a Cholesky factor
 *                      computed in a reduced format, refined in FP64 (Sec. V)
 *
 * Conventions (every entry point):
 *   - All array arguments are DEVICE pointers unless marked "host".  The
 *     caller allocates and owns every buffer; the library owns only the model
 *     handle (its reduced-precision weight copies and lookup tables) and a
 *     per-device workspace it grows on demand.
 *   - Calls are stream ordered and asynchronous: `stream` is a hipStream_t
 *     (NULL = the default stream).  Argument validation happens on the host
 *     before any launch; a rejected call launches nothing.
 *   - Spins are int8 +1 (up) / -1 (down); configurations are row-major
 *     [sample][site]; site i = x*L + y on an L x L lattice.
 *   - Errors are status codes; nqs_last_error() returns a thread-local message
 *     describing the last non-OK status.  Faults inside kernels surface at the
 *     caller's next synchronisation of `stream`.
 *   - Results depend only on (parameters, configuration, seed, step offset,
 *     global chain id) and, for the RBM samplers, on the lanes per chain G,
 *     which fixes the FP32 summation order of the log-ratio.  Chains per
 *     workgroup and the placement of lookup tables never change a result.
 */
#ifndef NQS_H
#define NQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NQS_OK = 0,
    NQS_EINVAL = 1,        /* bad argument (shape, null pointer, out-of-range value) */
    NQS_ENOMEM = 2,        /* device allocation failed */
    NQS_EDEVICE = 3,       /* a HIP call failed */
    NQS_EUNSUPPORTED = 4,  /* valid but not implemented combination */
    NQS_ENUMERIC = 5       /* non-finite parameters */
} nqs_status;

typedef enum { NQS_F64 = 0, NQS_F32 = 1, NQS_F16 = 2, NQS_BF16 = 3, NQS_FP8_E4M3 = 4 } nqs_dtype;
typedef enum { NQS_RBM = 0, NQS_FFNN = 1, NQS_RESCNN = 2, NQS_CRBM = 3 } nqs_arch;
typedef enum { NQS_MOVE_FLIP = 0, NQS_MOVE_EXCHANGE = 1 } nqs_move;
typedef enum { NQS_TFIM = 0, NQS_HEISENBERG = 1 } nqs_ham_kind;

#define NQS_MAX_LAYERS 8

/* Network description.
 * RBM (App. G, real parameters): log psi = a.s + sum_{j<M} log cosh((W s + b)_j),
 *   widths[0] = M, parameter vector [a(N), b(M), W(M x N, row-major)].
 * FFNN: h_l = ReLU(W_l h_{l-1} + b_l) for l < n_layers, log psi = sum log cosh(z_last),
 *   parameter vector [W_1 (w1 x N), b_1, W_2 (w2 x w1), b_2, ...].  Its FP8 E4M3
 *   copy scales each W_l and b_l by amax/448 and each hidden-layer output h_l
 *   by 2^ceil(log2(B_l/448)) before rounding it to E4M3, with B_l a bound on
 *   |h_l| over every configuration (B_0 = 1, B_l = max_k sum_i |W_l[k,i]|
 *   B_{l-1} + |b_l[k]| on the rounded weights); it samples on the batched-GEMM
 *   path (lanes_per_chain is ignored) and gives local energies.
 * RESCNN (App. H): residual convolutional network on the periodic lat_L x lat_L
 *   lattice (lat_dim = 2, n_visible = lat_L^2), widths[0] = F filters,
 *   n_layers = R residual blocks:  h0 = Conv(s);  h += Conv(phi(Conv(phi(LN h))));
 *   log psi = sum over sites and channels of LN(h_R).  Conv: 3x3 cross-
 *   correlation, circular padding, bias; LN: per site over channels, scale and
 *   shift, eps 1e-6; phi: GELU (tanh form).  Parameter vector [W0 (F x 9), b0],
 *   per block [gamma, beta, W1 (F x F x 9), b1, W2 (F x F x 9), b2], then
 *   [gamma_f, beta_f]; W[o][c][k], k = 3 (dx+1) + (dy+1) for the input site
 *   (x+dx, y+dy), site i = x L + y.  Sampling (single flips), TFIM local
 *   energies on its lattice, log psi and log-derivatives (nqs_logpsi_grad, its
 *   VJP, nqs_sample_gram with O formed whole, nqs_sr_update); no FP8 copy, no
 *   factored T, no column blocks of O.
 * CRBM: the RBM with complex a, b, W (widths[0] = M, n_layers = 1); |psi|^2 =
 *   exp(2 Re log psi) is sampled.  Parameter vector of 2 (N + M + M N) reals:
 *   the real parts in the RBM order, then the imaginary parts; a format rounds
 *   both parts.  Sampling (single flips), TFIM local energies (nqs_local_energy
 *   gives the real part, nqs_local_energy_complex both), log-derivatives
 *   (nqs_logpsi_grad: O_k = d log psi / d p_k with respect to the complex
 *   parameters p_k, log psi being holomorphic in them: s_i, tanh theta_j,
 *   tanh theta_j s_i; stored as [n][2P'] reals, Re O then Im O, P' = N + M + MN;
 *   logpsi = Re log psi; no vector-Jacobian product), the complex T of
 *   nqs_gram mode 3 and the SR step of nqs_sr_solve_complex / nqs_sr_update.
 * marshall = 1 multiplies psi by (-1)^{#up spins on sublattice A}, A = {(x+y) even}
 *   (lat_dim = 2) or {i even} (lat_dim = 1), on an L = lat_L lattice. */
typedef struct {
    int32_t arch;                     /* nqs_arch */
    int32_t n_visible;                /* N */
    int32_t n_layers;                 /* RBM: 1 */
    int32_t widths[NQS_MAX_LAYERS];
    int32_t marshall;
    int32_t lat_dim, lat_L;
} nqs_model_desc;

/* Hamiltonian on a dim-dimensional periodic (pbc = 1) or open lattice of side L (L >= 3 when periodic):
 *   NQS_TFIM:       H = J sum_<ij> sz_i sz_j + h sum_i sx_i           (Eq. eq:TFIM)
 *   NQS_HEISENBERG: H = J sum_<ij> sigma_i . sigma_j (Pauli matrices)  (App. E) */
typedef struct {
    int32_t kind;                     /* nqs_ham_kind */
    int32_t dim, L, pbc;
    double J, h;
} nqs_ham_desc;

/* Sampling configuration (Sec. III.A).
 * Each proposal consumes one Philox4x32-10 block (Salmon et al., SC'11) with
 * key = seed and counter = (step, global chain id, instance_id << 8 | 0): site
 * i = floor(r0*N/2^32); exchange partner j = floor(r1*(N-1)/2^32), j += (j >= i);
 * u = (r2 >> 8) * 2^-24.  Accept iff u < exp(min(Delta, 0)), Delta =
 * 2 (log|psi(s')| - log|psi(s)|), computed in FP32 from the `dtype` copy.
 * A sweep is sweep_size proposals (0 => N); after n_burnin sweeps one sample
 * per chain per sweep is written.  `step` runs from step_offset, so a run can
 * be resumed bit-exactly by passing the previous chain_state with
 * init_chains = 0 and step_offset advanced by the proposals already made.
 * init_chains = 1 draws the start states from the init stream (counter tag 1):
 * flip moves take spin i from bit i%32 of word i/32; exchange moves shuffle
 * N/2 up and N/2 down spins by Fisher-Yates. */
typedef struct {
    int64_t n_chains;
    int32_t n_sweeps, n_burnin, sweep_size;
    int32_t move;                     /* nqs_move */
    int32_t dtype;                    /* sampling copy: NQS_F32 / NQS_F16 / NQS_BF16, or NQS_FP8_E4M3 for an RBM or FFNN */
    int32_t init_chains;
    uint64_t seed, step_offset;
    uint32_t instance_id;
    int64_t chain_id_offset;          /* global id of chain 0 (for splitting chains across devices) */
    int32_t lanes_per_chain;          /* RBM: 0 = a fixed function of (N, M), 16, 32 or 64 lanes per chain
                                         (raised until the model fits), or NQS_LANES_TUNED = the measured
                                         choice (see nqs_sample_plan).
                                         Dense network: 0 = automatic, -1 = the batched-GEMM path
                                         (a full forward pass of every proposal; the path taken
                                         anyway for depth != 2 or wide first layers) */
    int32_t refresh_sweeps;           /* recompute the incremental state every k sweeps (0 => 1) */
} nqs_sample_cfg;

#define NQS_LANES_TUNED (-2)

/* Optional per-proposal decision trace of the first n_chains_traced chains
 * (device buffers of n_chains_traced x total-proposals entries, row-major),
 * used to replay every decision against the CPU reference. */
typedef struct {
    int32_t n_chains_traced;
    int32_t *site;                    /* i | (j << 16); j = 0xFFFF for single flips */
    uint32_t *ubits;                  /* r2 >> 8 */
    float *delta;                     /* Delta in FP32 as computed by the kernel */
    uint8_t *accepted;                /* 1 = accepted */
} nqs_trace;

typedef struct nqs_model nqs_model;   /* opaque, library-owned */

/* Create a model from a HOST FP64 parameter vector (copied to the device as
 * the FP64 master).  Returns NQS_ENUMERIC for non-finite parameters. */
nqs_status nqs_model_create(const nqs_model_desc *desc, const double *host_params, int64_t n_params,
                            nqs_model **out);
/* Replace the FP64 master from a HOST vector; reduced-precision copies are rebuilt on next use. */
nqs_status nqs_model_set_params(nqs_model *m, const double *host_params, int64_t n_params);
/* Replace the FP64 master from a DEVICE vector (stream ordered); copies are rebuilt on `stream`. */
nqs_status nqs_model_set_params_device(nqs_model *m, const double *dev_params, int64_t n_params, void *stream);
nqs_status nqs_model_destroy(nqs_model *m);
/* Build the `dtype` sampling copy from the FP64 master now (the downcast of
 * the two-copy scheme, Sec. IV.B), instead of lazily at the next call that
 * needs it.  Synchronises `stream` once to read back the weight range. */
nqs_status nqs_model_prepare(nqs_model *m, int32_t dtype, void *stream);
int64_t nqs_model_num_params(const nqs_model *m);

/* Downcast (Sec. IV.B two-copy scheme, App. A): round every FP64 value of
 * `src` to `dtype` with round-to-nearest-even in ONE rounding, and write the
 * rounded values, widened back to FP32 (exact), to dst[n].  For
 * NQS_FP8_E4M3 a per-tensor scale = amax/448 (FP32) is applied first
 * (value = q * scale, q an OCP E4M3 code) and written to scale_out[0]
 * (device, may be NULL otherwise). */
nqs_status nqs_downcast(const double *src, int64_t n, int32_t dtype, float *dst, float *scale_out, void *stream);

/* Metropolis-Hastings sampling (see nqs_sample_cfg).
 *   chain_state [n_chains][N]   in/out (ignored on input when init_chains = 1)
 *   samples     [n_sweeps][n_chains][N] out (may be NULL)
 *   logpsi      [n_sweeps][n_chains]   out, log|psi| of each sample in the sampling precision (may be NULL)
 *   n_accepted  [n_chains] out, accepted proposals over all sweeps incl. burn-in (may be NULL)
 *   trace       host struct with device buffers, or NULL */
nqs_status nqs_sample(nqs_model *m, const nqs_sample_cfg *cfg, int8_t *chain_state, int8_t *samples,
                      float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, void *stream);

/* Run-time detectors of a sampling call (the RBM single-flip sampler):
 *   - proposals whose log-ratio Delta is NaN or infinite (such a proposal is
 *     rejected, as the acceptance test of Sec. III.A is false for it): non-
 *     finite parameters or an overflow in the network's arithmetic;
 *   - the longest run of sweeps in which a chain accepted nothing (the loss
 *     of ergodicity that Sec. IV.A describes when the perturbation grows);
 *   - the drift of the incremental state: the largest difference between
 *     log|psi| carried by the accepted log-ratios since the previous refresh
 *     and log|psi| recomputed from theta = W s + b at the refresh (Eq.
 *     eq:pert_chain needs the perturbation to be a fixed function of the
 *     configuration, which a drifting incremental state would break).
 * Per-chain device arrays (each may be NULL; the library then keeps them in
 * its workspace), the host summary filled in when the call returns. */
typedef struct {
    int32_t stuck_after;              /* in: a chain counts as stuck after this many sweeps without an accepted
                                         move (0 => 10) */
    uint64_t *nonfinite;              /* [n_chains] device out: proposals with a non-finite Delta */
    uint32_t *longest_stuck;          /* [n_chains] device out: longest run of sweeps without an accepted move */
    float *drift;                     /* [n_chains] device out: largest |log psi drift| at a refresh */
    uint64_t total_nonfinite;         /* host out */
    int64_t chains_stuck;             /* host out: chains whose longest_stuck >= stuck_after */
    float max_drift;                  /* host out */
} nqs_sample_diag;

/* nqs_sample with the run-time detectors above (RBM, single flips; the traced
 * kernel, so slower than nqs_sample); samples, log psi, acceptances, traces and
 * results equal nqs_sample's.  Synchronises `stream`; returns NQS_ENUMERIC
 * (outputs written) when any Delta was not finite, NQS_EUNSUPPORTED for other
 * networks or moves. */
nqs_status nqs_sample_checked(nqs_model *m, const nqs_sample_cfg *cfg, int8_t *chain_state, int8_t *samples,
                              float *logpsi, uint64_t *n_accepted, const nqs_trace *trace, nqs_sample_diag *diag,
                              void *stream);

/* Launch plan of the RBM sampler (single flips) for this model, cfg.dtype and
 * cfg.n_chains: lanes per chain G, hidden units per lane K = ceil(M/G),
 * chains per workgroup, and whether the (cosh 2W, sinh 2W) table sits in LDS.
 * With cfg->lanes_per_chain = NQS_LANES_TUNED the plan is measured: every
 * valid G in {16, 32, 64}, both table placements and two chains-per-workgroup
 * counts are timed on a short burn-in from fresh states in scratch memory (no
 * caller buffer is touched; `stream` is synchronised), and the fastest is kept
 * for the life of the process, keyed by (device, N, M, dtype, n_chains).
 * nqs_sample with NQS_LANES_TUNED then uses it, so its results equal those of
 * a call with lanes_per_chain = plan->lanes_per_chain.  Any other
 * lanes_per_chain gives the fixed rule's plan without running anything.
 * NQS_EUNSUPPORTED for other networks. */
typedef struct {
    int32_t lanes_per_chain;
    int32_t units_per_lane;
    int32_t chains_per_block;
    int32_t table_in_lds;
    int32_t tuned;                    /* 1: measured */
    float tuned_ms;                   /* the chosen candidate's time on the tuning burn-in (0 for the rule) */
} nqs_launch_plan;
nqs_status nqs_sample_plan(nqs_model *m, const nqs_sample_cfg *cfg, nqs_launch_plan *plan, void *stream);

/* One sampling job of a batch: a model, its configuration and its buffers
 * (same meaning as the arguments of nqs_sample; trace may be NULL). */
typedef struct {
    nqs_model *model;
    nqs_sample_cfg cfg;
    int8_t *chain_state;
    int8_t *samples;
    float *logpsi;
    uint64_t *n_accepted;
    const nqs_trace *trace;
} nqs_sample_job;

/* Sample many independent instances (RBM, single flips) of uneven sizes.
 *   mode 0: one persistent launch; work items of 256 / G chains are sorted by
 *           decreasing cost and taken from a shared counter.
 *   mode 1: one launch per job, in order, on `stream`.
 * Each instance runs at its own lanes per chain G: cfg.lanes_per_chain = 32
 * or 64 as given (32 serves M <= 256, 64 serves M <= 1024), 0 for 32 when
 * M <= 256 and 64 above, NQS_LANES_TUNED for a measured choice made for the
 * whole batch: the persistent launch is timed on a short burn-in from fresh
 * states in scratch memory with the tuned instances at 32 lanes, at 64, and
 * at each one's single-launch choice (nqs_sample_plan restricted to 32/64),
 * and the fastest assignment is kept for the life of the process, keyed by
 * the batch's (N, M, dtype, n_chains, request) list.  Both modes produce
 * identical results, equal to nqs_sample of each job at its G; traced chains
 * record their decisions.  The batch descriptors are staged in the library
 * workspace; the call synchronises `stream` once before launching (and while
 * tuning). */
nqs_status nqs_sample_batched(const nqs_sample_job *jobs, int32_t n_jobs, int32_t mode, void *stream);

/* Metropolis-Hastings sampling of the noisy target of Sec. IV.A:
 *   log pi~(x) = log pi(x) + zeta(x),  zeta(x) = noise_sigma * g(x),
 * g(x) a standard normal held fixed per configuration: Philox4x32-10 with the
 * configuration's four 32-bit words as counter (spin i up = bit i % 32 of word
 * i / 32, sites >= N zero) and noise_seed as key; then Box-Muller on the first
 * two outputs, u1 = ((r0 >> 8) + 1) 2^-24, u2 = (r1 >> 8) 2^-24,
 * g = sqrt(-2 ln u1) cos(2 pi u2).  (The paper's log psi~ = log psi + zeta/2.)
 * The proposal stream, arguments and outputs are those of nqs_sample; logpsi
 * is the noiseless log|psi|.  RBM with single flips, N <= 128, the ratio table
 * in LDS; noise_sigma = 0 is nqs_sample.  For studying how a perturbation of
 * log pi biases expectation values and acceptance (Eq. eq:pert_chain). */
nqs_status nqs_sample_noisy(nqs_model *m, const nqs_sample_cfg *cfg, double noise_sigma, uint64_t noise_seed,
                            int8_t *chain_state, int8_t *samples, float *logpsi, uint64_t *n_accepted, void *stream);

/* Local energies eps[n_samples] (FP64 sums of FP32 amplitude ratios computed
 * from the `eval_dtype` copy of the parameters: NQS_F32 by default). */
nqs_status nqs_local_energy(nqs_model *m, const nqs_ham_desc *ham, const int8_t *samples, int64_t n_samples,
                            int32_t eval_dtype, double *eloc, void *stream);

/* Complex local energies of a complex RBM (TFIM): eloc_re[n], eloc_im[n]
 * (FP64 sums of FP32 complex flip ratios).  For the other networks, eloc_re
 * as nqs_local_energy and eloc_im zero. */
nqs_status nqs_local_energy_complex(nqs_model *m, const nqs_ham_desc *ham, const int8_t *samples, int64_t n_samples,
                                   int32_t eval_dtype, double *eloc_re, double *eloc_im, void *stream);

/* stats[4] (device, FP64): mean, unbiased variance, standard error of the
 * per-chain means, n.  eloc is laid out [sweep][chain] with n_chains chains;
 * the error bar needs n % n_chains == 0 and n_chains >= 2 (else NaN). */
nqs_status nqs_energy_stats(const double *eloc, int64_t n, int64_t n_chains, double *stats, void *stream);

/* nqs_energy_stats for callers that cannot allocate (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same results, with their scratch (512 block partials and the n_chains chain
 * means, FP64) in a fixed device array of 131072 doubles (1 MiB) per GPU, held
 * until the process ends; nothing is allocated.  NQS_EINVAL when the error bar
 * would need more than 130560 chain means (n % n_chains == 0 and n_chains >= 2
 * with n_chains > 130560).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race, so the
 * caller serialises them.  No part of the array needs to start at zero. */
nqs_status nqs_energy_stats_noalloc(const double *eloc, int64_t n, int64_t n_chains, double *stats, void *stream);

/* Log-amplitudes and log-derivatives from the FP32 copy.
 *   logpsi  [n] out (may be NULL)
 *   O       [n][P] out, row-major (may be NULL)
 *   vjp_in  [n] with vjp_out [P]: vjp_out = sum_k vjp_in[k] O[k][:] (both NULL to skip) */
nqs_status nqs_logpsi_grad(nqs_model *m, const int8_t *samples, int64_t n, float *logpsi, float *O,
                           const float *vjp_in, float *vjp_out, void *stream);

/* Columns [p0, p1) of O (Eq. eq:forces, the log-derivatives): O[n][p1 - p0],
 * row-major, O[k][p - p0] = d log psi(x_k) / d theta_p, FP32 copy.  The
 * parameter order is the one of nqs_logpsi_grad.  NQS_EINVAL unless
 * 0 <= p0 < p1 <= P. */
nqs_status nqs_logpsi_grad_cols(nqs_model *m, const int8_t *samples, int64_t n, int64_t p0, int64_t p1, float *O,
                                void *stream);

/* F[P] = mean_k O[k] eps[k] - mean_k O[k] * mean_k eps[k] and Omean[P]
 * (both FP64; Omean may be NULL). */
nqs_status nqs_forces(const float *O, const double *eloc, int64_t n, int64_t P, double *F, double *Omean,
                      void *stream);

/* Centred Gram matrix on FP32 matrix cores, Obar = O - mean over samples:
 *   mode 0: S[P][P] = Obar^T Obar / n      (Eq. eq:smat)
 *   mode 1: T[n][n] = Obar Obar^T / n      (same non-zero spectrum)
 *   mode 2: T[n][n] += Obar Obar^T / n     (O a column block; summing the
 *           blocks of all parameters gives the T of mode 1)
 *   mode 3: a complex network's O[n][2P'] (Re O, then Im O): T = Obar Obar^H / n,
 *           the sample-space twin of S_nm = E[O_n* O_m] - E[O_n*] E[O_m]
 *           (Eq. eq:smat), written as the real matrix out[2n][2n] =
 *           [[Re T, -Im T], [Im T, Re T]] (the Gram matrix of the rows
 *           [Re Obar, -Im Obar] and [Im Obar, Re Obar], divided by n); P even;
 *           2n x P floats of library workspace
 * `out` is FP32, row-major; in mode 2 it must hold the sum so far. */
nqs_status nqs_gram(const float *O, int64_t n, int64_t P, int32_t mode, float *out, void *stream);

/* T[n][n] = Obar Obar^T / n of the samples (Eq. eq:smat taken in sample
 * space), without ever holding all of O: the parameters are walked in column
 * blocks of `chunk_params` (0 = automatic, blocks of at most 1 GiB), each block
 * of O is formed in the library workspace and its T accumulated on the matrix
 * cores.  A dense network's blocks are expanded from per-sample layer inputs
 * and deltas (computed once, n x (sum of widths) floats each), an RBM's are
 * recomputed from the samples.  Block values equal the columns of
 * nqs_logpsi_grad bit for bit.  T is overwritten.  Blocks are summed in
 * parameter order, so the result does not depend on timing but does depend
 * on chunk_params through FP32 rounding.  n is at most 1,048,560. */
nqs_status nqs_sample_gram(nqs_model *m, const int8_t *samples, int64_t n, int64_t chunk_params, float *T,
                           void *stream);

/* The same T[n][n] evaluated from the factors of O instead of O itself.  Each
 * layer's O is an outer product per sample (dense layer l: delta_l x a_{l-1}
 * plus delta_l for the bias; RBM: tanh(theta) x s plus tanh(theta) and s), so
 *   O_k . O_l = sum_layers (U_k.U_l + c)(V_k.V_l + 1) - c
 * needs Gram matrices of the per-sample factors (a few thousand values)
 * rather than of all P parameters, and the centring is exact algebra with the
 * means of O.  Factors are FP32 (as in nqs_logpsi_grad); means, centring and
 * the contraction (FP64 matrix cores) are FP64; T is rounded to FP32 once.
 * Workspace: n x (sum of factor widths) floats plus the mean matrices
 * (about P doubles) and a few n-vectors.  T is overwritten; deterministic. */
nqs_status nqs_sample_gram_factored(nqs_model *m, const int8_t *samples, int64_t n, float *T, void *stream);

/* Stochastic-reconfiguration step in sample space (App. I.2, Eq. eq:smat;
 * forces of Eq. eq:forces).  The direction delta of (S + shift) delta = F,
 * S = Obar^T Obar / n, F = Obar^T (eps - mean eps) / n, equals Obar^T y / n
 * with (T + shift) y = eps - mean eps, T = Obar Obar^T / n (push-through
 * identity; S and T share their non-zero spectrum).
 *
 * nqs_sr_solve: y[n] (FP64, device) from T[n][n] (FP32, e.g. from
 *   nqs_sample_gram_factored) and eloc[n] (FP64), by Jacobi-preconditioned
 *   conjugate gradients in FP64 until ||r|| <= tol ||b|| or max_iter
 *   iterations.  shift >= 0 (T is singular along the constant vector, which
 *   the centred right-hand side avoids).  Synchronises `stream`; *iters and
 *   *rel_resid (host pointers, may be NULL) report the iteration count and
 *   ||r|| / ||b|| (0 when b = 0).  The residual is read every 8 iterations, so
 *   the count is a multiple of 8 (or max_iter) and up to 7 iterations may run
 *   past the one that first met tol.  Deterministic.
 * nqs_sr_update: master[P] (FP64, device, the caller's parameter vector) -=
 *   lr * delta, delta = O^T (y - mean y) / n through the FP32 copy's
 *   log-derivatives of `samples` (the n samples T was formed from).  The
 *   model's own copies are not touched: pass `master` to
 *   nqs_model_set_params_device for the next step.  For the complex RBM,
 *   y[2n] = (Re z, Im z) from nqs_sr_solve_complex and delta =
 *   O^H (z - mean z) / n, complex: master's real parts move by lr Re delta and
 *   its imaginary parts by lr Im delta (Eq. eq:sr_step with complex S, F).
 * nqs_sr_solve_complex: the complex system (T + shift) z = eps - mean eps of a
 *   complex network, T2[2n][2n] its real embedding from nqs_gram mode 3,
 *   eloc_re / eloc_im[n] the complex local energies (FP64); y2[2n] = (Re z,
 *   Im z), the two halves of the right-hand side centred separately (in a
 *   buffer of library workspace), then the same Jacobi conjugate gradients as
 *   nqs_sr_solve on 2n unknowns.  Together with nqs_sr_update this gives the
 *   parameter-space direction (S + shift) delta = F of Eqs. eq:smat and
 *   eq:forces (the push-through identity). */
nqs_status nqs_sr_solve(const float *T, const double *eloc, int64_t n, double shift, double tol, int32_t max_iter,
                        double *y, int32_t *iters, double *rel_resid, void *stream);
nqs_status nqs_sr_solve_complex(const float *T2, const double *eloc_re, const double *eloc_im, int64_t n, double shift,
                                double tol, int32_t max_iter, double *y2, int32_t *iters, double *rel_resid,
                                void *stream);
nqs_status nqs_sr_update(nqs_model *m, const int8_t *samples, int64_t n, const double *y, double lr, double *master,
                         void *stream);

/* The same y[n] by mixed precision (Sec. V points to mixed-precision
 * iterative solvers for the preconditioning step; App. I.2 on why its
 * accuracy matters: errors are amplified by the condition number of S).
 * T + shift is factorised L L^T in `factor_dtype` (NQS_F32, NQS_BF16 or
 * NQS_F16: the operands of the blocked trailing updates and of the inverse's
 * products are rounded to the format on the matrix cores, with FP32
 * accumulation; diagonal blocks and panels FP32), L^{-1} is formed the same
 * way, and conjugate gradients in FP64 preconditioned by L^{-T} L^{-1} run
 * until ||r|| <= tol ||b|| or max_iter iterations.  The preconditioner is
 * symmetric positive definite whatever the rounding, so the result is the
 * FP64 solution; the format sets the iteration count.  A pivot not larger than
 * the format's unit round-off times its original diagonal entry (T + shift
 * not positive definite at that precision) is replaced by that entry and
 * counted in *n_pivots_fixed (host pointer, may be NULL).  If a BF16/FP16
 * factorisation replaces more than n / 8 pivots, or its preconditioned
 * residual is not a positive finite number (the factor's inverse overflowed),
 * the solve is redone with an FP32 factor, and failing that with the Jacobi
 * preconditioner of nqs_sr_solve; *factor_used (host, may be NULL) reports
 * the factor format that produced y, or -1 for Jacobi.  n <= 65536;
 * workspace 2 np^2 floats, np = n rounded up to 64.  Synchronises `stream`;
 * *iters, *rel_resid as for nqs_sr_solve, for the attempt that produced y.
 * Deterministic. */
nqs_status nqs_sr_solve_mixed(const float *T, const double *eloc, int64_t n, double shift, int32_t factor_dtype,
                              double tol, int32_t max_iter, double *y, int32_t *iters, double *rel_resid,
                              int64_t *n_pivots_fixed, int32_t *factor_used, void *stream);

const char *nqs_last_error(void);
const char *nqs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
