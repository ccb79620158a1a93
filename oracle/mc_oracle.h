/*
 * mc_oracle.h -- plain FP64 CPU oracle for the Monte Carlo closed-loop CSTR
 * (Kaysfeld, Zanon, Joergensen, "Performance Quantification of a Nonlinear
 * Model Predictive Controller by Parallel Monte Carlo Simulations of a
 * Closed-loop System", arXiv 2212.02197).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product path
 * (paper_2212_02197_amd + libmc_cl.so) never calls it; the two share no code.
 *
 * Every routine follows the paper's equations in its own order and notation,
 * with no blocking, fusion or reordering.  Readings where the paper is silent
 * are listed at the definition that takes them.
 */
#ifndef MC_ORACLE_H
#define MC_ORACLE_H
#include <stdint.h>

#define OC_NMAX 64          /* largest NMPC horizon the oracle accepts      */
#define OC_SPMAX 8          /* largest number of setpoint schedule levels    */

/* Everything a campaign needs.  All FP64; units: L, s, K, mol.               */
typedef struct {
    /* plant model, eq. (CSTR) of the Model section                           */
    double V, k0, EaR, beta, cAin, cBin, cTin;
    double sigma[3];        /* diag(sigma_A, sigma_B, sigma_T)              */
    double Rmeas;           /* measurement variance R (K^2)                  */
    /* simulation, Results section: Ts, Ns                                   */
    double Ts;
    int32_t Ns, L;          /* EM sub-steps per interval; intervals (N-bar)  */
    /* setpoint: piecewise constant in the interval index i (t_i = i Ts)     */
    int32_t n_sp, sp_period;        /* sp_period 0 = hold last level        */
    int32_t sp_i[OC_SPMAX];
    double  sp_z[OC_SPMAX];
    double  sp_step_rel;            /* 0 = no per-sample step               */
    int32_t sp_step_lo, sp_step_hi; /* step interval ~ U{lo..hi}            */
    /* NMPC: horizon, RK4 steps, weight, bounds (mL/min)                     */
    int32_t N, Nc;
    double Qz, umin, umax;
    double sqp_eps, ls_c1, ls_beta;
    int32_t sqp_max_iter, ls_max_bt, grad_mode;  /* 0 fwd-sens, 1 adjoint  */
    int32_t ipm_max_iter;
    int32_t want_grad;              /* PI samples: tangent dPhi/d(Kc, tau_i) */
    /* PI, eq. (PI); flow in L/s                                             */
    double kP, kI, kaw, pi_umin, pi_umax;
    /* EKF / initial state                                                   */
    double P0, x0_rel_std;
    int32_t x0_mode;                /* 0 inlet C_in V, 1 steady state*(1+std xi) */
    int32_t kind_split;             /* ids < split: NMPC, else PI            */
    int32_t default_kind;           /* used when kind_split < 0: 0 NMPC 1 PI */
    int32_t run_ekf_for_pi;
    /* Monte Carlo                                                           */
    uint64_t seed;
    int64_t noise_mod;              /* noise id = sample id mod this (0: id) */
    int32_t n_horizon_choices;      /* >0: N ~ U{horizon_choices}            */
    int32_t horizon_choices[4];
    int32_t L_lo, L_hi;             /* L_lo < L_hi: L ~ U{L_lo..L_hi}         */
    double kin_lognorm_sigma;       /* >0: plant k0, EaR * exp(sigma xi)      */
    int32_t hess_warm;              /* 1: shifted previous W, 0: W = I per OCP */
    int32_t model_nx;               /* estimator and OCP model: 1 the one-state
                                       model (the paper's), 3 the three-state
                                       eq. (CSTR) model                      */
    double noise_scale;             /* 1 stochastic; 0 deterministic run (the
                                       filter keeps its R and sigma)         */
    int32_t nlp_form;               /* OCP discretisation: 0 single shooting,
                                       1 multiple shooting, eq. (OCP_NLP)
                                       (one-state model; mc_oracle_ms.c)     */
} oc_params;

/* Per-sample result.                                                        */
typedef struct {
    double phi;                 /* eq. (Phi)                                 */
    double dphi[2];             /* PI: dPhi/d(Kc, tau_i) (tangent), else 0   */
    uint64_t ashash;            /* FNV-1a over (i, active-set bitmask)       */
    int32_t kind, N, L, n_ocp;
    int32_t n_ocp_fail;         /* SQP iteration cap hits                    */
    int32_t sqp_iter, ipm_iter, ls_trials, ls_cap, bfgs_skip, bfgs_reset;
    int32_t ipm_cap, nonfinite, grad_evals;
} oc_sample_out;

#ifdef __cplusplus
extern "C" {
#endif
/* building blocks, exported so the tests can pin each one */
void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void oc_normal_pair(uint64_t seed, uint32_t block, uint32_t step, uint32_t id,
                    uint32_t tag, double out[4]);  /* xi0, xi1, u1, u2       */
void oc_f3(const oc_params *p, double k0, double EaR, const double n[3], double F, double out[3]);
void oc_f3_jac(const oc_params *p, double k0, double EaR, const double n[3], double F,
               double J[9], double fF[3]);
void oc_f1(const oc_params *p, double x, double F, double out[3]); /* f, df/dx, df/dF */
void oc_steady_state(const oc_params *p, double T, double *F_ss, double n_ss[3]);
double oc_setpoint(const oc_params *p, int32_t i, int32_t istep, double sign);
void oc_em_step(const oc_params *p, double k0, double EaR, double n[3], double F,
                const double xi[3]);
void oc_ekf_predict(const oc_params *p, double *x, double *P, double F);
void oc_ekf_update(const oc_params *p, double *x, double *P, double y);
double oc_ocp_shoot(const oc_params *p, int32_t N, double x0, const double *u,
                    const double *zbar, double *xs);
void oc_ocp_grad_adjoint(const oc_params *p, int32_t N, const double *u,
                         const double *zbar, const double *xs, double *grad);
void oc_ocp_grad_fwd(const oc_params *p, int32_t N, double x0, const double *u,
                     const double *zbar, double *grad);
void oc_ekf3_predict(const oc_params *p, double x[3], double P[9], double F);
void oc_ekf3_update(const oc_params *p, double x[3], double P[9], double y);
double oc_ocp3_shoot(const oc_params *p, int32_t N, const double x0[3], const double *u,
                     const double *zbar, double *xs);
void oc_ocp3_grad_adjoint(const oc_params *p, int32_t N, const double *u,
                          const double *zbar, const double *xs, double *grad);
void oc_ocp3_grad_fwd(const oc_params *p, int32_t N, const double x0[3], const double *u,
                      const double *zbar, double *grad);
int  oc_box_qp(int32_t N, const double *W, const double *g, const double *lo,
               const double *hi, int32_t max_iter, double *d, double *nl, double *nu,
               int32_t *iters);
int  oc_bfgs_update(int32_t N, double *W, const double *s, const double *y);
int  oc_sqp(const oc_params *p, int32_t N, const double *x0, const double *zbar, double *u,
            double *pil, double *piu, double *W, int32_t reset_W, oc_sample_out *cnt);
void oc_run_sample(const oc_params *p, int64_t sample_id, oc_sample_out *out,
                   double *traj_z, double *traj_u, double *traj_xhat);
/* As oc_run_sample, with caller-given {kind, N, L} (ov, -1 = the draw; or
 * NULL), also recording the PI integral state after interval i's update
 * (traj_I[i], PI samples; may be NULL).                                     */
void oc_run_sample_ext(const oc_params *p, int64_t sample_id, const int32_t *ov,
                       oc_sample_out *out, double *traj_z, double *traj_u, double *traj_xhat,
                       double *traj_I);
/* The per-sample scenario draws: iv = {kind, N, L, step interval},
 * dv = {step sign, plant k0, plant Ea/R}.                                   */
void oc_scenario(const oc_params *p, int64_t sample_id, int32_t iv[4], double dv[3]);
void oc_run(const oc_params *p, const int64_t *ids, int64_t n, int32_t nthreads,
            oc_sample_out *out);
/* As oc_run with caller-given per-sample {kind, N, L} (ov: [3][n], row 0
 * kind, 1 horizon, 2 length of task t at column t; -1 keeps the draw).     */
void oc_run_ov(const oc_params *p, const int64_t *ids, const int32_t *ov, int64_t n,
               int32_t nthreads, oc_sample_out *out);
void oc_stats(const double *phi, int64_t n, double *mean, double *var,
              int64_t *hist /* 202 */);
/* multiple shooting (mc_oracle_ms.c)                                        */
void oc_ms_interval(const oc_params *p, double x, double u, double out[3]);
int  oc_ms_qp(const oc_params *p, int32_t N, const double *W, const double *gf,
              const double *A, const double *B, const double *c, const double *u,
              double *dxi, double *mu, double *nl, double *nu, int32_t *iters);
int  oc_ms_sqp(const oc_params *p, int32_t N, double x0, const double *zbar, double *u,
               double *x, oc_sample_out *cnt);
#ifdef __cplusplus
}
#endif
#endif
