/*
 * tvmc.h -- C ABI of the MI355X (gfx950) implementation of trajectory-unravelled
 * time-dependent variational Monte Carlo (otVMC).
 *
 * Method: Apostoli, D'Alberto, Genoni, Bertaina, Galli, "Unraveling Open Quantum Dynamics
 * with Time-Dependent Variational Monte Carlo".  Each trajectory carries complex variational
 * parameters theta (M of them) and follows the otVMC equations (Eq. 8):
 *     sum_k' S_kk' dtheta_k' = -i F_k dt + sum_n N^n_k o dW_n,
 * with O_k = d log psi / d theta_k, E_eff = (H_eff^Strat psi)(x)/psi(x) (Eq. 5),
 * B^n = (L_n psi)(x)/psi(x), S = <O* O> - <O*><O>, F = <O* E_eff> - <O*><E_eff>,
 * N^n = <O* B^n> - <O*><B^n>, all estimated from Metropolis samples of |psi|^2.  The
 * increment is D = -i F dt + sum_n N^n dW_n (paragraph after Eq. 9), the solve is
 * (S + eps I) delta = D, and the Stratonovich predictor-correctors of App. C advance theta.
 *
 * Conventions (hbar = 1):
 *   H = sum_{i<j} J_ij sz_i sz_j + hx sum_i sx_i        (the LITF Hamiltonian, Eq. 10, with
 *       the couplings and field passed in: the paper's sign is J_ij < 0, hx = -h)
 *   L_n = sqrt(rate_n) * op_n(site_n), op in {sigma^-, sigma^+, sigma^z}   (Eq. 1)
 *   configuration sigma_i = +-1 (sz eigenvalues), packed into W = ceil(N / 64) 64-bit words:
 *   bit i % 64 of word i / 64 set <=> sigma_i = +1; bits at and above N are zero.
 *
 * Parameter layout theta (interleaved re, im doubles):
 *   Jastrow (Eq. 12): [a_0..a_{N-1}, eta_01, eta_02, .., eta_0,N-1, eta_12, .., eta_N-2,N-1]
 *   LJPHd   (the partially inhomogeneous Jastrow of the LITF section, open chain):
 *            [a_0..a_{N-1}, eta_jk for k - j <= d in the Jastrow order, eta_(d+1) .. eta_(N-1)],
 *            the last block shared by every pair at that distance; d = N-1 is the Jastrow
 *            layout itself and d = 0 the homogeneous LJH (2N - 1 parameters)
 *   RBM     (Eq. 11): [a_0..a_{N-1}, b_0..b_{N'-1}, w_00, w_01, .., w_0,N'-1, w_10, ..]
 *
 * Ownership: every host pointer passed in is read during the call and may be freed after it.
 * The device workspace is allocated by the caller (size from tvmc_workspace_size), must stay
 * alive and untouched until tvmc_destroy, and is never freed by the library.  The library
 * allocates no device memory.  Work is enqueued asynchronously on the caller's HIP stream;
 * getters and tvmc_synchronize block on that stream.  No call throws or aborts: failures are
 * reported as tvmc_status, with a message from tvmc_last_error.
 */
#ifndef TVMC_H
#define TVMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tvmc_ctx tvmc_ctx;

typedef enum {
    TVMC_OK = 0,
    TVMC_E_INVAL = 1,        /* bad argument or unsupported size */
    TVMC_E_NOMEM = 2,        /* workspace too small */
    TVMC_E_DEVICE = 3,       /* a HIP runtime call failed */
    TVMC_E_NUMERIC = 4,      /* non-positive pivot or non-finite update in some trajectory */
    TVMC_E_STATE = 5,        /* stage calls out of order */
    TVMC_E_UNSUPPORTED = 6
} tvmc_status;

enum { TVMC_JUMP_SIGMA_MINUS = 0, TVMC_JUMP_SIGMA_PLUS = 1, TVMC_JUMP_SIGMA_Z = 2 };
enum { TVMC_ANSATZ_JASTROW = 0, TVMC_ANSATZ_RBM = 1, TVMC_ANSATZ_LJPH = 2 };
enum { TVMC_SCHEME_HEUN = 0, TVMC_SCHEME_MIDPOINT = 1 };
/* FP64: S accumulated with FP64 vector FMAs.  MFMA: for the Jastrow ansaetze S is accumulated on
 * int8 matrix cores (every O_k is +-1, or an LJPHd distance sum, |O| <= N-d-1, fed as itself up to
 * N = 128 and as its half, |h| <= (N-d)/2, beyond), exactly, so both give the same S bit for bit;
 * the int8 form refuses n_samples times that bound squared >= 2^31 (TVMC_E_INVAL); for the RBM it
 * is the three-term BF16 split with FP32 accumulation.  Solve and theta stay FP64 in both. */
enum { TVMC_PREC_FP64 = 0, TVMC_PREC_MFMA = 1 };

/* One Lindblad problem (Eq. 1 with the Hamiltonian of Eq. 10), shared by all trajectories of a
 * context (see tvmc_init_batch for one problem per trajectory). */
typedef struct {
    int32_t n_sites;              /* N, 1..192 (the learned proposal and the SNR solve: 1..64) */
    const double *J;              /* host, N*N row-major, symmetric, zero diagonal */
    double hx;
    int32_t n_jumps;              /* 0..256 */
    const int32_t *jump_kind;     /* host, n_jumps entries of TVMC_JUMP_* */
    const int32_t *jump_site;     /* host, n_jumps entries in [0, N) */
    const double *jump_rate;      /* host, n_jumps entries >= 0 */
} tvmc_problem;

typedef struct {
    int32_t kind;                 /* TVMC_ANSATZ_JASTROW, TVMC_ANSATZ_RBM or TVMC_ANSATZ_LJPH */
    int32_t n_hidden;             /* RBM hidden units N', 1..256 (ignored otherwise) */
    int32_t range;                /* LJPHd: d in [0, N-1] (ignored otherwise); solved in parameter space
                                     (a shared eta's O_k is an integer sum, |O_k| <= N-1) */
} tvmc_ansatz;

typedef struct {
    int32_t n_traj;               /* trajectories integrated together (grid dimension) */
    int32_t traj_offset;          /* id of the first trajectory: selects its random streams */
    int32_t n_samples;            /* Metropolis samples per evaluation, multiple of n_chains */
    int32_t n_chains;             /* Markov chains per trajectory, multiple of 8 or < 8 */
    int32_t burn_sweeps;          /* sweeps (N proposals each) before recording, per evaluation */
    int32_t thin_sweeps;          /* sweeps between recorded samples */
    int32_t init_sweeps;          /* extra burn-in at the very first evaluation */
    int32_t scheme;               /* TVMC_SCHEME_* (App. C) */
    double dt;
    double diag_shift;            /* eps of (S + eps I) */
    int32_t precision;            /* TVMC_PREC_* */
    int32_t obs_every;            /* record moments at steps that are multiples of this (0: never) */
    int32_t n_obs_max;            /* capacity of the moment history */
    uint64_t seed;                /* Philox4x32-10 key */
    /* learned proposal (either ansatz): a masked autoregressive network per trajectory, trained
     * on the trajectory's own samples, proposes one independent Metropolis-Hastings move at the
     * start of every sweep; single-spin flips remain the fallback */
    int32_t proposal;             /* TVMC_PROPOSAL_* */
    int32_t ar_hidden;            /* hidden units of the network, 1..256, ar_hidden * N <= 8192 */
    int32_t ar_train_every;       /* train at steps that are multiples of this (0: only on request) */
    int32_t ar_train_iters;       /* Adam steps per training */
    double ar_lr;                 /* Adam learning rate */
    int32_t solver;               /* TVMC_SOLVER_*: how the regularised system is solved */
    int32_t unravelling;          /* TVMC_SSE_*: which stochastic Schroedinger equation is unravelled */
    int32_t regulariser;          /* TVMC_REG_*: how (S + eps I) delta = D is regularised */
    double snr_tau;               /* TVMC_REG_SNR: the SNR threshold (the paper uses 4) */
    int32_t use_graph;            /* 1: tvmc_sde_step runs plain steps (no moments, no training, timing
                                     off, step >= 1) by replaying one captured HIP graph of a step;
                                     the results are the same bits as the eager launches; needs a
                                     stream other than the default one */
    int32_t sampler_chains;       /* Markov chains per sampler workgroup (one wavefront each): 0 picks
                                     the largest of 8, 4, 2, 1 dividing n_chains (16 when it divides
                                     for the RBM with N' <= 128 and for the Jastrow ansaetze with
                                     N > 64); else 1, 2, 4, 8 or 16 (RBM with N' <= 128 only),
                                     dividing n_chains.  A launch shape only: the samples are the
                                     same bits for every value */
} tvmc_config;

/* SHIFT: the Cholesky solve of (S + eps I) delta = D.  SNR: the regulariser the paper names in
 * the text after Eq. 9: D in the eigenbasis of S + eps I (S + eps I = V diag(lam) V^T), each
 * component rho_k = (V^T D)_k kept with weight 1 / (1 + (tau / SNR_k)^6), where SNR_k =
 * |rho_k| sqrt(N_s) / sqrt(<|q_k|^2> - |rho_k|^2) over the per-sample contributions
 * q_k(x) = u_k(x) (G(x) - <G>), u_k(x) = sum_l V_lk (O_l(x) - <O_l>), G(x) = -i dt E_eff(x)
 * + sum_n B^n(x) dW_n; delta = sum_k V_k keep_k rho_k / lam_k, eigenvalues below 1e-14 of the
 * largest dropped.  Parameter space, M <= 2176; eps may be 0.  For the RBM's complex Hermitian S
 * the rotations carry the phase of A_pq and V is unitary (rho = V^H D, u_k = sum_l V_lk (O_l -
 * <O_l>), q_k = conj(u_k) (G - <G>)).  The eigen-decomposition (parallel Jacobi) overwrites S: after tvmc_sr_solve, TVMC_Q_S
 * holds diag(lam) up to rounding, and TVMC_Q_EIG the pairs (lam_k, SNR_k). */
enum { TVMC_REG_SHIFT = 0, TVMC_REG_SNR = 1 };

/* NONLINEAR: the norm-preserving SSE of Eq. 2 (Stratonovich form Eqs. 4-5).  LINEAR: the linear
 * SSE of App. B: E_eff becomes the local value of H - (i/2) sum_n (L_n^dag L_n + L_n^2) (no
 * <L + L^dag> drive, so F^lin = F - i sum_n <L_n + L_n^dag> N^n), and every trajectory also
 * carries log Q, Q = e^{phi + phi*} <psi_theta|psi_theta>, integrated by the step's own scheme
 * from dQ = Q (2 Im<E_eff^lin> dt + 2 sum_n Re<B^n> o dW_n); trajectory averages are then
 * weighted, (1/N_T) sum_j <A>_j Q_j.  log Q starts at 0 (Q = 1). */
enum { TVMC_SSE_NONLINEAR = 0, TVMC_SSE_LINEAR = 1 };

enum { TVMC_PROPOSAL_FLIP = 0, TVMC_PROPOSAL_LEARNED = 1 };
/* FP64 Cholesky of S + eps I: one workgroup per trajectory (one launch per solve), or several
 * workgroups per trajectory (a few launches per 64-column panel), which fills the device when
 * the batch has fewer trajectories than compute units; AUTO picks by batch size. */
enum { TVMC_SOLVER_AUTO = 0, TVMC_SOLVER_ONE_GROUP = 1, TVMC_SOLVER_MULTI_GROUP = 2 };
/* Sample space: the same increment through the push-through identity
 * (A^H A + eps I)^-1 A^H = A^H (A A^H + eps I)^-1 with A = (O - <O>) / sqrt(N_s), i.e. an
 * N_s x N_s system T u = G - <G> and delta = A^H u / sqrt(N_s); AUTO takes it when M > N_s.
 * TVMC_Q_S then returns T + eps I (N_s x N_s, lower triangle). */
enum { TVMC_SOLVER_SAMPLE_SPACE = 3 };

/* Quantities readable with tvmc_get (per trajectory unless noted). */
enum {
    TVMC_Q_THETA = 0,       /* double[2M] current theta */
    TVMC_Q_THETA_EVAL = 1,  /* double[2M] theta of the current evaluation */
    TVMC_Q_DELTA0 = 2,      /* double[2M] predictor increment */
    TVMC_Q_DELTA1 = 3,      /* double[2M] corrector increment */
    TVMC_Q_SAMPLES = 4,     /* uint64[n_samples][W] packed configurations of the last sampling */
    TVMC_Q_ELOC = 5,        /* double[2 n_samples] local energy of H */
    TVMC_Q_S = 6,           /* double[M*M] S + eps I, lower triangle valid (before the solve, which
                               factorises it in place); for the RBM complex, double[2 M*M] interleaved */
    TVMC_Q_D = 7,           /* double[2M] D */
    TVMC_Q_OBAR = 8,        /* <O_k>: double[M] for the Jastrow ansatz (real), double[2M] for the RBM */
    TVMC_Q_BMEAN = 9,       /* double[2 n_jumps] <B^n> */
    TVMC_Q_DW = 10,         /* double[n_jumps] Wiener increments of the current step */
    TVMC_Q_ACCEPTS = 11,    /* uint32[n_chains] accepted proposals in the last sampling */
    TVMC_Q_CHAINS = 12,     /* uint64[n_chains][W] chain configurations (settable) */
    TVMC_Q_MOMENTS = 13,    /* double[9] moments (mx,my,mz,sxx,syy,szz,sxy,sxz,syz) */
    TVMC_Q_OBS_HIST = 14,   /* double[n_obs_max*9] moment history; traj selects the trajectory */
    TVMC_Q_AR_PARAMS = 15,  /* float[P] network parameters W1 [H][N] | b1 [H] | W2 [N][H] | b2 [N],
                               P = 2 N H + N + H (settable) */
    TVMC_Q_AR_GRAD = 16,    /* float[P] gradient of the mean negative log-likelihood */
    TVMC_Q_AR_LOGQ = 17,    /* float[n_samples] log q of the last samples */
    TVMC_Q_AR_LOSS = 18,    /* double[1] mean negative log-likelihood */
    TVMC_Q_AR_ACCEPTS = 19, /* uint32[n_chains] accepted learned proposals in the last sampling */
    TVMC_Q_LOGNORM = 20,    /* double[1] log Q of the linear SSE at the current step (0 for the nonlinear SSE) */
    TVMC_Q_LOGNORM_HIST = 21, /* double[n_obs_max] log Q at the times of the moment history */
    TVMC_Q_EIG = 22,          /* double[2M] (lam_k, SNR_k) of the last SNR solve, in the solver's order */
    TVMC_Q_AR_LOGQ_BF16 = 23  /* float[n_samples] log q of the last samples under the BF16 network the
                                 sampler's acceptance test uses (computed by the get, on its stream) */
};

/* Bytes of device workspace needed for this problem, ansatz and configuration. */
tvmc_status tvmc_workspace_size(const tvmc_problem *problem, const tvmc_ansatz *ansatz,
                                const tvmc_config *config, size_t *bytes);

/* Create a context: copies the problem into the workspace, sets theta = theta0 (host,
 * interleaved, M complex values shared by every trajectory; NULL = all zeros, the +x coherent
 * state of the Jastrow ansatz) and draws the initial chain configurations uniformly.
 * stream: a hipStream_t (NULL = default stream). */
tvmc_status tvmc_init(const tvmc_problem *problem, const tvmc_ansatz *ansatz, const tvmc_config *config,
                      const double *theta0, void *d_workspace, size_t workspace_bytes, void *stream,
                      tvmc_ctx **out);

/* Batches with one problem per trajectory (n_problems = n_traj; 1 means shared): the problems
 * must share N, hx and the jump channels (kind and site); J and the rates may differ.  Used
 * for uneven batches (one context per system size, each on its own stream). */
tvmc_status tvmc_workspace_size_batch(const tvmc_problem *problems, int32_t n_problems, const tvmc_ansatz *ansatz,
                                      const tvmc_config *config, size_t *bytes);
tvmc_status tvmc_init_batch(const tvmc_problem *problems, int32_t n_problems, const tvmc_ansatz *ansatz,
                            const tvmc_config *config, const double *theta0, void *d_workspace,
                            size_t workspace_bytes, void *stream, tvmc_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): tvmc_init with the library's own static workspace in
 * place of a caller-allocated one.  The workspace is a device array of tvmc_static_workspace_bytes
 * bytes (64 MiB) that every device loading the library holds until the process ends; a problem
 * needing more (tvmc_workspace_size) returns TVMC_E_NOMEM.  One problem shared by every
 * trajectory; the context works on the current device and runs every solve on `stream` (no side
 * streams or events are created).  No device memory is allocated.  A device's static workspace
 * serves one live context at a time: a second tvmc_init_static on that device returns
 * TVMC_E_STATE until the first is destroyed (contexts on one device would otherwise overwrite
 * each other's state).  It keeps the last context's contents; tvmc_init_static clears or writes
 * everything a run reads before it is read, as tvmc_init does. */
tvmc_status tvmc_static_workspace_bytes(size_t *bytes);
tvmc_status tvmc_init_static(const tvmc_problem *problem, const tvmc_ansatz *ansatz, const tvmc_config *config,
                             const double *theta0, void *stream, tvmc_ctx **out);

/* Metropolis sampling of |psi|^2 at the current evaluation point (text after Eq. 9); at the
 * predictor stage it also draws the step's Wiener increments.  Requires the stage to be ready. */
tvmc_status tvmc_sample(tvmc_ctx *ctx);
/* Local estimators, <B^n>, D and S + eps I (definitions after Eq. 8).  Requires tvmc_sample. */
tvmc_status tvmc_estimate(tvmc_ctx *ctx);
/* Regularised solve (S + eps I) delta = D in FP64 (Cholesky).  Requires tvmc_estimate. */
tvmc_status tvmc_sr_solve(tvmc_ctx *ctx);
/* Predictor-corrector update of App. C for the current stage.  Requires tvmc_sr_solve. */
tvmc_status tvmc_update(tvmc_ctx *ctx);
/* n_steps full steps (noise, predictor, corrector); records moments every obs_every steps
 * from the predictor samples.  Requires the predictor stage to be ready. */
tvmc_status tvmc_sde_step(tvmc_ctx *ctx, int32_t n_steps);
/* Train the learned proposal on the last samples (needs TVMC_PROPOSAL_LEARNED): n_iters Adam
 * steps, each on log q, the loss and the gradient of the current parameters; n_iters = 0 only
 * evaluates log q, the loss and the gradient.  Requires samples at the current point. */
tvmc_status tvmc_train_proposal(tvmc_ctx *ctx, int32_t n_iters);
/* Moments of the collective spin from the last samples (observables paragraph of the LITF
 * section); copies double[n_traj][9] to moments_out when it is not NULL. */
tvmc_status tvmc_observables(tvmc_ctx *ctx, double *moments_out);
/* Trajectory average (Eq. 3) of the last moments: out[0..2] = M, out[3..11] = C (row-major),
 * out[12] = xi^2 (Wineland, minimum over the plane orthogonal to M).  For the linear SSE the
 * average is App. B's weighted one, each trajectory's moments times its Q at the time they were
 * taken, divided by N_T. */
tvmc_status tvmc_ensemble(tvmc_ctx *ctx, double *out);
/* The same average for history record `slot` of the moments (slot < 0: the last moments), and,
 * when loo_xi2 is not NULL, a jackknife over the trajectories: loo_xi2[t] (n_traj doubles) is
 * xi^2 of the average with trajectory t left out (n_traj >= 2).  A record not yet taken returns
 * TVMC_E_INVAL. */
tvmc_status tvmc_ensemble_at(tvmc_ctx *ctx, int32_t slot, double *out, double *loo_xi2);
/* Copy a quantity (TVMC_Q_*) of one trajectory to host memory of at least `bytes` bytes. */
tvmc_status tvmc_get(tvmc_ctx *ctx, int32_t what, int32_t traj, void *host_out, size_t bytes);
/* Overwrite theta (TVMC_Q_THETA) or the chain configurations (TVMC_Q_CHAINS) of a trajectory. */
tvmc_status tvmc_set(tvmc_ctx *ctx, int32_t what, int32_t traj, const void *host_in, size_t bytes);
/* Checkpoint at a step boundary (stage 0, before tvmc_sample): everything a later step reads --
 * theta, the chain configurations, the step counter that keys the Philox streams, the moment
 * and log Q histories and the last moments, log Q, the learned proposal's parameters and Adam
 * state -- as one host blob of tvmc_state_size bytes.  Loading it into a context created with
 * the same problem, ansatz and configuration continues the run bit for bit.  Saving off a step
 * boundary returns TVMC_E_STATE; a blob of another shape returns TVMC_E_INVAL. */
tvmc_status tvmc_state_size(const tvmc_ctx *ctx, size_t *bytes);
tvmc_status tvmc_save_state(tvmc_ctx *ctx, void *host_out, size_t bytes);
tvmc_status tvmc_load_state(tvmc_ctx *ctx, const void *host_in, size_t bytes);
/* Current step index and stage (0 predictor, 1 corrector). */
tvmc_status tvmc_position(const tvmc_ctx *ctx, int32_t *step, int32_t *stage);
/* Wait for the stream and report TVMC_E_NUMERIC if any trajectory failed. */
tvmc_status tvmc_synchronize(tvmc_ctx *ctx);
/* Average duration in milliseconds of the last n launches of the named kernel group
 * ("sample", "estimate", "sbuild", "solve", "update"), measured with HIP events on the
 * context's stream when timing was enabled with tvmc_set_timing. */
tvmc_status tvmc_set_timing(tvmc_ctx *ctx, int32_t enable);
tvmc_status tvmc_timing(tvmc_ctx *ctx, const char *group, double *avg_ms, int32_t *count);
const char *tvmc_last_error(const tvmc_ctx *ctx);
tvmc_status tvmc_destroy(tvmc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
