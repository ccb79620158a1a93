/*
 * mc_cl.h -- C-ABI of the MI355X (gfx950) Monte Carlo closed-loop library.
 *
 * Method: Kaysfeld, Zanon, Joergensen, "Performance Quantification of a
 * Nonlinear Model Predictive Controller by Parallel Monte Carlo Simulations
 * of a Closed-loop System" (arXiv 2212.02197).  Every sample integrates the
 * stochastic continuous-discrete CSTR (CDS section, eq. (CDS); Model section,
 * eq. (CSTR)) by Euler-Maruyama sub-steps, runs the CD-EKF (NMPC section,
 * eq. (predictionEquations) and eq. (Josph)), applies either the NMPC (OCP of
 * eq. (OPC_general) by single-shooting SQP: QP subproblem, Armijo line search
 * eq. (Armijo), damped BFGS, scaled KKT test eq. (convergence)) or the PI law
 * eq. (PI), and accumulates its cost eq. (Phi).
 *
 * Conventions
 *  - All arithmetic is FP64.  Units: L, s, K, mol; plant flow F in L/s; NMPC
 *    decision inputs u in mL/min (Results section: 0 <= u <= 1000 mL/min).
 *  - Functions return an int status: MC_CL_OK (0) or a negative MC_CL_E*.
 *  - Per-sample numerical events (SQP iteration cap, line-search cap, BFGS
 *    reset, non-finite state) are data in the outputs, never errors.
 *  - Device pointers are HIP device addresses on the context's device; host
 *    pointers are ordinary CPU memory.  The library never frees caller memory.
 *  - Thread safety: one context must not be used from two threads at once;
 *    different contexts are independent.
 */
#ifndef MC_CL_H
#define MC_CL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_CL_ABI_VERSION 6u
#define MC_CL_SPMAX 8        /* setpoint schedule levels                        */
#define MC_CL_NMAX 64        /* largest NMPC horizon                            */
#define MC_CL_NHIST 202      /* histogram: underflow, 200 bins, overflow        */

enum {
    MC_CL_OK = 0,
    MC_CL_EINVAL = -1,       /* bad argument / parameter out of its domain      */
    MC_CL_EHIP = -2,         /* HIP runtime error (text kept for strerror)      */
    MC_CL_ENOMEM = -3,       /* device allocation failed                        */
    MC_CL_ESTATE = -4,       /* call out of order (costs before run, ...)       */
    MC_CL_EUNSUPPORTED = -5  /* valid request the library does not handle      */
};

/* Per-sample counter rows of mc_cl_outputs.counters ([MC_CL_NCNT][S]).      */
enum {
    MC_CL_CNT_KIND = 0,      /* 0 NMPC, 1 PI                                    */
    MC_CL_CNT_N,             /* horizon                                         */
    MC_CL_CNT_L,             /* closed-loop intervals                           */
    MC_CL_CNT_OCP,           /* OCPs solved (= L for NMPC; Table I)             */
    MC_CL_CNT_OCP_FAIL,      /* OCPs that hit the SQP iteration cap             */
    MC_CL_CNT_SQP_ITER,      /* SQP iterations (QP solves)                      */
    MC_CL_CNT_IPM_ITER,      /* interior-point iterations                       */
    MC_CL_CNT_LS_TRIALS,     /* shooting evaluations of the objective           */
    MC_CL_CNT_LS_CAP,        /* line searches that hit the backtrack cap        */
    MC_CL_CNT_BFGS_SKIP,     /* BFGS updates skipped (kappa <= eps_m)           */
    MC_CL_CNT_BFGS_RESET,    /* W reset to I after a non-positive pivot         */
    MC_CL_CNT_IPM_CAP,       /* QPs that hit the interior-point iteration cap   */
    MC_CL_CNT_NONFINITE,     /* 1 if a non-finite state appeared; an NMPC
                                sample whose plant output stops being finite
                                ends its closed loop there (Phi is NaN, no
                                further OCP is solved)                       */
    MC_CL_CNT_GRAD,          /* objective-gradient evaluations                  */
    MC_CL_CNT_AS_ITER,       /* active-set QP iterations (linear solves)        */
    MC_CL_NCNT
};

/*
 * Campaign parameters.  The caller owns it; mc_cl_create copies it.
 * Set struct_size = sizeof(mc_cl_params) and abi_version = MC_CL_ABI_VERSION.
 */
typedef struct {
    uint32_t struct_size, abi_version;
    /* plant, eq. (CSTR): V (L), k0 (L/(mol s)), Ea/R (K), beta (K L/mol),
     * inlet concentrations (mol/L) and temperature (K)                      */
    double V, k0, EaR, beta, cAin, cBin, cTin;
    double sigma[3];          /* diffusion diag(sigma_A, sigma_B, sigma_T)    */
    double Rmeas;             /* measurement variance of y = c_T + v (K^2)    */
    double Ts;                /* sampling time (s)                            */
    int32_t Ns;               /* Euler-Maruyama sub-steps per interval        */
    int32_t L;                /* closed-loop intervals N-bar (Phi has L+1)    */
    /* setpoint zbar(t_i), t_i = i Ts: level sp_z[j] from interval sp_i[j]
     * (sp_i[0] = 0, increasing), periodic with sp_period intervals if > 0;
     * optional per-sample step zbar *= (1 + sign sp_step_rel) from interval
     * istep ~ U{sp_step_lo..sp_step_hi}, sign a fair coin                    */
    int32_t n_sp, sp_period;
    int32_t sp_i[MC_CL_SPMAX];
    double sp_z[MC_CL_SPMAX];
    double sp_step_rel;
    int32_t sp_step_lo, sp_step_hi;
    /* NMPC: horizon N (1..64), RK4 steps per interval Nc, output weight Qz,
     * input bounds (mL/min)                                                  */
    int32_t N, Nc;
    double Qz, umin, umax;
    /* SQP: KKT tolerance, Armijo c1, backtracking factor                     */
    double sqp_eps, ls_c1, ls_beta;
    int32_t sqp_max_iter, ls_max_bt;
    int32_t grad_mode;        /* 0 forward sensitivities, 1 adjoint           */
    int32_t ipm_max_iter;     /* interior-point iteration cap of the QP       */
    /* PI, eq. (PI); flow in L/s, clip bounds pi_umin..pi_umax                */
    double kP, kI, kaw, pi_umin, pi_umax;
    /* CD-EKF initial covariance P_{-1|-1}; initial-state mode:
     * x0_mode 0: n0 = C_in V, x-hat = c_T,in V (Results section)
     * x0_mode 1: n0 = n_ss(zbar(0)) (1 + x0_rel_std xi), x-hat = n_ss,T      */
    double P0, x0_rel_std;
    int32_t x0_mode;
    int32_t kind_split;       /* >= 0: ids < split are NMPC, others PI         */
    int32_t default_kind;     /* kind when kind_split < 0 (0 NMPC, 1 PI)       */
    int32_t run_ekf_for_pi;   /* run the estimator for PI samples too          */
    /* Monte Carlo                                                            */
    uint64_t seed;            /* Philox key                                    */
    int64_t noise_mod;        /* noise id = sample id mod noise_mod (0: id)    */
    int64_t n_samples;        /* S >= 1                                        */
    int64_t sample_id_offset; /* first sample id (chunking, subsets)           */
    int32_t n_horizon_choices;/* > 0: N ~ U{horizon_choices[0..n-1]} per sample */
    int32_t horizon_choices[4];
    int32_t L_lo, L_hi;       /* L_lo < L_hi: L ~ U{L_lo..L_hi} per sample      */
    double kin_lognorm_sigma; /* > 0: plant k0, Ea/R times exp(sigma xi)        */
    int32_t hess_warm;        /* 1: OCP i+1 starts from OCP i's W shifted       */
    int32_t want_grad;        /* PI: keep checkpoints for mc_cl_grad            */
    double noise_scale;       /* 1 stochastic, 0 deterministic run             */
    int32_t ckpt_interval;    /* PI reverse pass: intervals per checkpoint (0 = auto) */
    /* NMPC samples per wavefront, used exactly; 0 = auto: a cost model's
     * choice, evened out over the resident wavefronts (made as small as the
     * same number of rounds allows; by at most an eighth when the groups
     * take several rounds)                                                  */
    int32_t samples_per_wave;
    /* QP solver and Hessian form: 0 primal-dual interior point on the
     * BFGS matrix W (the paper's method family); 1 primal-dual active set on
     * W warm-started from the SQP multipliers, with the interior-point method
     * as fallback when the active set has not settled after 8 factorisations;
     * 2 (default) the same active-set iteration on H = W^-1 kept by the
     * inverse BFGS update, whose QP with |A| active bounds costs one H g
     * product and an |A| x |A| solve; sets not settled after 8 full updates
     * continue with least-index single changes (at most 64), and only then
     * fall back to the interior point on H^-1.
     * All return the QP's unique minimiser; the SQP iterates are the same up
     * to rounding.                                                          */
    int32_t qp_solver;
    /* > 0: mc_cl_run processes the campaign in ceil(S / chunk_samples)
     * chunks, each a contiguous range of every horizon class's wavefront
     * groups and of the PI samples, by replaying one captured HIP graph of
     * the chunk step (the NMPC and PI launches) per chunk with the chunk
     * index kept on the device; 0: one launch per kernel.  Results are
     * bitwise the same either way.  Trajectory outputs need chunk_samples =
     * 0 (EUNSUPPORTED otherwise).                                           */
    int32_t chunk_samples;
    /* > 0: plan the launches for this many compute units (at most the
     * device's), for runs on a stream limited to them (mc_cl_stream_create);
     * 0: all of the device's compute units.                                 */
    int32_t cu_limit;
    /* Model of the estimator and the NMPC's OCP: 1 (the paper's case study)
     * the one-state model x = n_T closed by the reaction invariants; 3 the
     * three-state eq. (CSTR) drift with the nominal kinetics, x = (n_A, n_B,
     * n_T), a 3x3 CD-EKF (eq. (predictionEquations), eq. (Josph)) with
     * P_0 = P0 I and x-hat_0 = C_in V (x0_mode 0) or the model's steady
     * state at zbar(0) (x0_mode 1).  Other values: EINVAL; 3 with
     * grad_mode 0: EUNSUPPORTED (forward sensitivities are one-state only). */
    int32_t model_nx;
    /* Optional per-sample arrays, host memory of n_samples entries each,
     * copied by mc_cl_create (NULL: the rules above).  Column s of every
     * output is the sample these arrays give at index s.
     *   sample_ids: global sample id (0 .. 2^32 - 2) that keys the sample's
     *     noise and scenario draws and the kind_split test; default
     *     sample_id_offset + s.  Ids may repeat or come in any order
     *     (strided subsets of a campaign).
     *   kind: 0 NMPC, 1 PI, in place of kind_split / default_kind.
     *   horizon: N (1..64), in place of N and horizon_choices.
     *   lengths: L (0 .. 2^24), in place of L and L_lo..L_hi.
     * EINVAL for a value outside its range.                                 */
    const int64_t *sample_ids;
    const uint8_t *kind;
    const int32_t *horizon;
    const int32_t *lengths;
    /* Discretisation of the NMPC's OCP: 0 single shooting (the inputs are
     * the decision variables; the settings above); 1 direct multiple
     * shooting, eq. (OCP_NLP), the paper's own NLP: states and inputs are
     * decision variables, the structured QP eq. (QP-subproblem) is solved by
     * a Riccati-recursion primal-dual interior point, the line search uses
     * Powell's l1 merit, the Hessian is the block damped BFGS from W^[0] = I
     * at every OCP (hess_warm, qp_solver, grad_mode and samples_per_wave do
     * not apply; 64 samples per wavefront).  1 needs model_nx = 1
     * (EUNSUPPORTED otherwise) and umin < umax (EINVAL).                    */
    int32_t nlp_form;
    /* Optional caller-owned device workspace (NULL: the library allocates).
     * When given, every device buffer of the context is carved from it, in
     * order, 256-byte aligned; workspace_size must be at least what
     * mc_cl_workspace_size reports for the same parameters (ENOMEM
     * otherwise), the pointer 256-byte aligned (EINVAL otherwise).  It must
     * stay valid until mc_cl_destroy; the library never frees it.
     * mc_cl_tune may need more (its trial shapes grow the workspaces):
     * ENOMEM when the rest does not hold them.                              */
    void *workspace;
    size_t workspace_size;
    /* NMPC horizon classes of an unchunked run on the whole device: 0 one
     * launch after another on the caller's stream (default); 1 on the
     * caller's stream and two library-owned side streams forked from it and
     * joined back into it by events.  The results are bitwise the same.
     * Measured on c3 (three classes): 9.89 s one after another, 10.34 s
     * concurrent.                                                           */
    int32_t class_streams;
} mc_cl_params;

/* Optional outputs of mc_cl_run; every pointer may be NULL.  All are device
 * pointers on the context's device, written asynchronously on the stream.
 * Layout is structure-of-arrays over samples, sample s at column s.         */
typedef struct {
    double *phi;              /* [S] eq. (Phi)                                 */
    int32_t *counters;        /* [MC_CL_NCNT][S]                               */
    uint64_t *ashash;         /* [S] FNV-1a-64 over (i, active-set bitmask) of
                                 every OCP; bit k set if u_k is within 1e-6 of
                                 a bound at the implemented solution           */
    /* Trajectories, row i = interval i, with T = the largest entry of
     * lengths[] when given, else L_hi if L_lo < L_hi (drawn lengths), else L:
     * every sample's own length is at most T.  Row i
     * of a sample's column is written for i <= its L (z) or i < its L (u,
     * x-hat); later rows of that column are left as they were.              */
    double *traj_z;           /* [T+1][S] output z = c_T (K)                   */
    double *traj_u;           /* [T][S] implemented flow (L/s)                 */
    double *traj_xhat;        /* [T][S] filtered estimate x-hat_{i|i} (its n_T
                                 entry with the three-state model)             */
} mc_cl_outputs;

/* Campaign statistics (per controller: index 0 NMPC, 1 PI), over the
 * samples whose Phi is finite (a diverged closed loop, see
 * MC_CL_CNT_NONFINITE, is left out and counted in totals).                  */
typedef struct {
    int64_t count[2];
    double mean[2];           /* mean Phi                                      */
    double var[2];            /* sample variance of Phi (divisor count - 1)    */
    int64_t hist[2][MC_CL_NHIST]; /* log10 Phi in 200 bins on [-4, 4),
                                     [0] underflow, [201] overflow             */
    int64_t totals[MC_CL_NCNT];   /* column sums of the counters               */
    double flops_algorithmic; /* FP64 work of the campaign by the per-routine
                                 table times the counters                      */
    double flops_by_kind[2];  /* the same split by controller (NMPC, PI)      */
    size_t workspace_bytes;   /* device memory the context holds               */
} mc_cl_stats;

typedef struct mc_cl_ctx mc_cl_ctx;   /* opaque, library-owned                */

/* Validate parameters, pick the launch plan, allocate device workspaces on
 * the current HIP device.  EINVAL on out-of-domain parameters (non-finite
 * values, V <= 0, N outside 1..64, umin > umax, S < 1, ...), ENOMEM,
 * EHIP.  *out is set only on MC_CL_OK.                                       */
int mc_cl_create(const mc_cl_params *p, mc_cl_ctx **out);

/* Run the campaign asynchronously on hip_stream (a hipStream_t; NULL = the
 * null stream): every sample's closed loop, then the Phi statistics.  Results
 * stay in the context; `o` (may be NULL) names extra device outputs.  With
 * several horizon classes, no chunking, no cu_limit and class_streams = 1,
 * the classes' kernels run concurrently on two library-owned streams forked
 * from hip_stream and joined back into it by events (same results as one
 * after another).
 * EUNSUPPORTED if trajectories are requested of a chunked run.             */
int mc_cl_run(mc_cl_ctx *c, void *hip_stream, const mc_cl_outputs *o);

/* Wait for the last run, then copy Phi ([S], host, may be NULL) and the
 * statistics (host, may be NULL).  ESTATE before any run.                   */
int mc_cl_costs(mc_cl_ctx *c, double *phi_host, mc_cl_stats *st);

/* PI samples only: gradient of mean Phi over the PI samples w.r.t.
 * theta = (Kc, tau_i), kP = Kc, kI = Kc / tau_i, by the reverse pass through
 * the whole closed loop from plant-state checkpoints (noise held fixed).
 * g (host, 2 doubles) receives d mean Phi / d theta after the stream is
 * synchronised; per_sample (device, [2][S], may be NULL) receives each
 * sample's dPhi/dtheta (0 for NMPC samples).  ESTATE without a previous run
 * with want_grad = 1 or with no PI sample.                                  */
int mc_cl_grad(mc_cl_ctx *c, void *hip_stream, double g[2], double *per_sample);

/* Release the context and its device memory (waits for its work).          */
void mc_cl_destroy(mc_cl_ctx *c);

/* Static text for a status code (for MC_CL_EHIP: the last HIP error text).  */
const char *mc_cl_strerror(int status);

/* Version of the ABI this library implements.                              */
uint32_t mc_cl_abi_version(void);

/* Diagnostics.
 * mc_cl_kernel_ms: device time (ms, HIP events on the run's stream) of the
 * last run's NMPC kernels (all classes, fork to join) [0], PI kernel [1],
 * statistics [2] and of the last
 * mc_cl_grad reverse pass [3]; waits for the run.  ESTATE before a run.
 * For a chunked run (chunk_samples > 0) [0] spans every graph replay, NMPC
 * and PI kernels together, and [1] is -1.                                   
 * mc_cl_plan: launch plan of the NMPC horizon classes, 5 ints per class
 * {NMAX, samples, samples per wavefront, work groups, resident wavefronts};
 * with the multiple-shooting NLP a work group is one sample, taken by an
 * NMAX-lane segment (64 / NMAX per wavefront).  Returns the number of
 * classes written (<= max_classes).                                         */
int mc_cl_kernel_ms(mc_cl_ctx *c, float ms[4]);
int mc_cl_plan(mc_cl_ctx *c, int32_t *out, int max_classes);

/* Measured launch-shape tuning (the batching runtime).  For every NMPC
 * horizon class, times the campaign's own samples cut to their first
 * `trial_intervals` closed-loop intervals at each candidate number of
 * samples per wavefront (at most 4, 8, 16, 32, 64, each evened out over the
 * resident wavefronts as for samples_per_wave = 0) and keeps the fastest
 * (spw[] reports the value used); for a
 * campaign with want_grad and PI samples, times the PI forward pass with
 * checkpoints plus the reverse pass at each candidate checkpoint interval
 * C (2, 5, 10, 25, 50; those above the longest sample's L skipped,
 * time -1) and keeps the fastest; for a campaign with PI samples, times
 * the PI pass (with the reverse pass at the chosen C when the gradient is
 * wanted) with 1, 2 and 4 lanes per sample and keeps the fastest (without
 * tuning the library takes the most lanes that keep the PI launch at one
 * wavefront per SIMD).  Phi, the counters and the gradient are bitwise the
 * same for every launch shape and lane count; C moves the gradient by
 * rounding only (each segment is recomputed from its checkpoint).  Synchronises `hip_stream`; the trial launches overwrite the last
 * run's results, so mc_cl_costs / mc_cl_grad need a new mc_cl_run.  The
 * workspaces grow to the largest candidate tried.  EINVAL for a null
 * argument or trial_intervals < 1; ENOMEM, EHIP.                           */
#define MC_CL_TUNE_NSPW 5
#define MC_CL_TUNE_NCK 5
#define MC_CL_TUNE_NPIK 3
typedef struct {
    int32_t n_classes;
    int32_t nmax[3];                      /* NMAX of each horizon class      */
    int32_t spw[3];                       /* chosen samples per wavefront    */
    float nmpc_ms[3][MC_CL_TUNE_NSPW];    /* trial time per candidate        */
    int32_t ckpt_interval;                /* chosen C (0: no PI gradient)    */
    float grad_ms[MC_CL_TUNE_NCK];        /* trial time per candidate C      */
    int32_t pi_lanes;                     /* chosen lanes per PI sample (0:
                                             no PI samples)                  */
    float pi_ms[MC_CL_TUNE_NPIK];         /* trial time at 1, 2, 4 lanes     */
} mc_cl_tune_result;
int mc_cl_tune(mc_cl_ctx *c, void *hip_stream, int32_t trial_intervals, mc_cl_tune_result *r);

/* Device bytes mc_cl_create needs for these parameters (their workspace
 * fields are ignored), for a caller-passed workspace.  Plans the campaign
 * on the current device as mc_cl_create does (allocating and releasing its
 * buffers).  Errors as mc_cl_create.                                        */
int mc_cl_workspace_size(const mc_cl_params *p, size_t *bytes);

/* Allocation-free run, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Runs the campaign `p` describes on hip_stream with the same
 * kernels as mc_cl_create + mc_cl_run and the same results (the launch shape
 * differs; Phi, the counters and the hashes do not depend on it), but
 * allocates nothing: the per-sample lists, the work queues and the NMPC
 * workspaces live in a library-owned device array of
 * MC_CL_STATIC_SCRATCH_BYTES per device (taken when the library is loaded
 * on the device, held until the process ends).
 * Outputs: o->phi ([S], device) is required; o->counters and o->ashash are
 * optional device outputs as for mc_cl_run; trajectories, want_grad,
 * chunking, the per-sample arrays and nlp_form 1 are EUNSUPPORTED; the
 * workspace fields are ignored.  No statistics are
 * formed.  Synchronises hip_stream once (after planning), then returns with
 * the campaign's kernels queued on it.
 * EINVAL for invalid parameters or outputs, or when the campaign needs more
 * than the array: about 96 bytes per sample (88 when the caller takes the
 * counters, 80 with the hashes too) plus one wavefront slot of one sample
 * (about 0.5 MB at N > 32).  Every call on a device shares that device's
 * array and overwrites the last call's contents: calls that overlap on one
 * device (two streams, two threads) race and must not be made.            */
#define MC_CL_STATIC_SCRATCH_BYTES (64u << 20)
int mc_cl_run_static(const mc_cl_params *p, void *hip_stream, const mc_cl_outputs *o);

/* A HIP stream on the current device whose kernels run on its first n_cu
 * compute units only (a CU-masked stream; n_cu <= 0 or >= the device's
 * count: all), for throughput against compute units (the GPU analogue of
 * the Parallel scalability study).  Pair it with mc_cl_params.cu_limit =
 * n_cu.  *stream receives the hipStream_t, owned by the caller and released
 * with mc_cl_stream_destroy.  EINVAL for a null argument; EHIP.            */
int mc_cl_stream_create(int32_t n_cu, void **stream);
int mc_cl_stream_destroy(void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MC_CL_H */
