/*
 * mc_oracle.c -- plain, slow, FP64 CPU oracle of the Monte Carlo closed-loop
 * CSTR of arXiv 2212.02197.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  It shares no code, header, table or constant
 * with the HIP library; both receive the same parameter values as inputs and
 * each draws its own noise from the published Philox4x32-10 definition.
 *
 * Order of one closed-loop interval (Results section, "Closed-loop simulation",
 * and the CDS section): cost term, measurement, CD-EKF prediction and
 * filtering, controller (NMPC by single-shooting SQP, or the PI law of
 * eq. (PI)), then Euler-Maruyama sub-steps of the three-state SDE eq. (CSTR).
 *
 * Built with gcc -O2 (no -ffast-math, no FMA contraction target).
 */
#include "mc_oracle.h"
#include <math.h>
#include <float.h>
#include <string.h>
#include <stdlib.h>
#include <pthread.h>

#define ML_MIN_PER_L_S 60000.0   /* 1 L/s = 60000 mL/min (unit conversion) */

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of the 4x32 S-box on the counter,
 * the key bumped by the Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Two standard normals by Box-Muller from one Philox block.
 * counter = (block, step, id, tag), key = (seed lo, seed hi).
 * u1 = (m1 + 1) 2^-53 in (0, 1], u2 = m2 2^-53 in [0, 1), m = top 53 bits of
 * the 64-bit word formed by two outputs.  out = {xi0, xi1, u1, u2}.          */
void oc_normal_pair(uint64_t seed, uint32_t block, uint32_t step, uint32_t id,
                    uint32_t tag, double out[4])
{
    uint32_t ctr[4] = {block, step, id, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oc_philox4x32_10(ctr, key, r);
    uint64_t m1 = ((((uint64_t)r[0]) << 32) | r[1]) >> 11;
    uint64_t m2 = ((((uint64_t)r[2]) << 32) | r[3]) >> 11;
    double u1 = ((double)(m1 + 1)) * 0x1p-53;
    double u2 = ((double)m2) * 0x1p-53;
    double rho = sqrt(-2.0 * log(u1));
    double ang = 6.283185307179586 * u2;
    out[0] = rho * cos(ang);
    out[1] = rho * sin(ang);
    out[2] = u1;
    out[3] = u2;
}

/* Noise tags of the counter's last word. */
enum { TAG_PROCESS = 0, TAG_MEAS = 1, TAG_X0 = 2, TAG_KIN = 3, TAG_SCEN = 4 };

/* ------------------------------------------------------------------------
 * Model section, eq. (CSTR): dn = (C_in F - c F + R V) dt + F sigma dw,
 * c = n / V, R = S^T r(c), r = k(c_T) c_A c_B, k = k0 exp(-(Ea/R)/c_T),
 * S = [-1, -2, beta] for the three-state model.
 * ---------------------------------------------------------------------- */
void oc_f3(const oc_params *p, double k0, double EaR, const double n[3], double F,
           double out[3])
{
    double cA = n[0] / p->V, cB = n[1] / p->V, cT = n[2] / p->V;
    double r = k0 * exp(-EaR / cT) * cA * cB;
    out[0] = p->cAin * F - cA * F + (-1.0) * r * p->V;
    out[1] = p->cBin * F - cB * F + (-2.0) * r * p->V;
    out[2] = p->cTin * F - cT * F + p->beta * r * p->V;
}

/* Jacobian of f3 w.r.t. n (row-major 3x3) and its derivative w.r.t. F.    */
void oc_f3_jac(const oc_params *p, double k0, double EaR, const double n[3], double F,
               double J[9], double fF[3])
{
    double V = p->V;
    double cA = n[0] / V, cB = n[1] / V, cT = n[2] / V;
    double k = k0 * exp(-EaR / cT);
    /* dr/dc = (k cB, k cA, k EaR/cT^2 cA cB); dc/dn = 1/V; R V = S r V     */
    double dr_dn[3] = { k * cB / V, k * cA / V, k * (EaR / (cT * cT)) * cA * cB / V };
    double S[3] = { -1.0, -2.0, p->beta };
    int a, b;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b)
            J[3 * a + b] = (a == b ? -F / V : 0.0) + S[a] * dr_dn[b] * V;
    fF[0] = p->cAin - cA;
    fF[1] = p->cBin - cB;
    fF[2] = p->cTin - cT;
}

/* One-state model (C_in = [c_T,in], S = [beta], sigma = [sigma_T]) with the
 * state x = n_T = c_T V.  The concentrations the rate needs are closed by the
 * reaction invariants of S = [-1, -2, beta]:
 *   c_A = c_A,in + (c_T,in - c_T)/beta,  c_B = c_B,in + 2 (c_T,in - c_T)/beta.
 * out = {f1, df1/dx, df1/dF}.                                               */
void oc_f1(const oc_params *p, double x, double F, double out[3])
{
    double V = p->V, beta = p->beta;
    double cT = x / V;
    double cA = p->cAin + (p->cTin - cT) / beta;
    double cB = p->cBin + 2.0 * (p->cTin - cT) / beta;
    double k = p->k0 * exp(-p->EaR / cT);
    double r = k * cA * cB;
    /* dr/dc_T = k (Ea/R)/c_T^2 c_A c_B + k (dcA/dcT c_B + c_A dcB/dcT)      */
    double dr = k * (p->EaR / (cT * cT)) * cA * cB
              + k * ((-1.0 / beta) * cB + cA * (-2.0 / beta));
    out[0] = (p->cTin - cT) * F + beta * r * V;
    out[1] = -F / V + beta * dr;          /* d/dx = (1/V) d/dc_T            */
    out[2] = p->cTin - cT;
}

/* Steady state of the one-state model at temperature T:
 * 0 = (c_T,in - T) F + beta r(T) V  =>  F_ss = beta r V / (T - c_T,in);
 * n_ss = (c_A(T), c_B(T), T) V from the reaction invariants.                */
void oc_steady_state(const oc_params *p, double T, double *F_ss, double n_ss[3])
{
    double cA = p->cAin + (p->cTin - T) / p->beta;
    double cB = p->cBin + 2.0 * (p->cTin - T) / p->beta;
    double r = p->k0 * exp(-p->EaR / T) * cA * cB;
    *F_ss = p->beta * r * p->V / (T - p->cTin);
    n_ss[0] = cA * p->V;
    n_ss[1] = cB * p->V;
    n_ss[2] = T * p->V;
}

/* Setpoint z-bar(t_i): piecewise constant in the interval index, optionally
 * periodic, times (1 + sign rel) from the sample's step interval on.       */
double oc_setpoint(const oc_params *p, int32_t i, int32_t istep, double sign)
{
    int32_t ii = p->sp_period > 0 ? i % p->sp_period : i;
    double z = p->sp_z[0];
    int j;
    for (j = 1; j < p->n_sp; ++j)
        if (ii >= p->sp_i[j]) z = p->sp_z[j];
    if (p->sp_step_rel != 0.0 && i >= istep) z = z * (1.0 + sign * p->sp_step_rel);
    return z;
}

/* Euler-Maruyama sub-step of eq. (CSTR): n <- n + h f3 + F sigma sqrt(h) xi,
 * h = Ts/Ns, dw ~ N(0, I h).                                                */
void oc_em_step(const oc_params *p, double k0, double EaR, double n[3], double F,
                const double xi[3])
{
    double h = p->Ts / (double)p->Ns;
    double f[3];
    int a;
    oc_f3(p, k0, EaR, n, F, f);
    for (a = 0; a < 3; ++a)
        n[a] = n[a] + h * f[a] + F * p->sigma[a] * sqrt(h) * xi[a];
}

/* ------------------------------------------------------------------------
 * CD-EKF, NMPC section "State estimator".
 * Prediction, eq. (predictionEquations): dx/dt = f, dP/dt = A P + P A^T +
 * sigma sigma^T over one sampling interval with the previous input held.
 * The integrator is not stated; classical RK4 with Nc steps (the OCP's
 * integrator) on the joint (x, P) system, A evaluated at each stage.        */
void oc_ekf_predict(const oc_params *p, double *x, double *P, double F)
{
    double h = p->Ts / (double)p->Nc;
    double q = (F * p->sigma[2]) * (F * p->sigma[2]);
    double X = *x, PP = *P;
    int c;
    for (c = 0; c < p->Nc; ++c) {
        double f[3], k1x, k1P, k2x, k2P, k3x, k3P, k4x, k4P;
        oc_f1(p, X, F, f);
        k1x = f[0]; k1P = 2.0 * f[1] * PP + q;
        oc_f1(p, X + 0.5 * h * k1x, F, f);
        k2x = f[0]; k2P = 2.0 * f[1] * (PP + 0.5 * h * k1P) + q;
        oc_f1(p, X + 0.5 * h * k2x, F, f);
        k3x = f[0]; k3P = 2.0 * f[1] * (PP + 0.5 * h * k2P) + q;
        oc_f1(p, X + h * k3x, F, f);
        k4x = f[0]; k4P = 2.0 * f[1] * (PP + h * k3P) + q;
        X = X + h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        PP = PP + h / 6.0 * (k1P + 2.0 * k2P + 2.0 * k3P + k4P);
    }
    *x = X;
    *P = PP;
}

/* Filtering with the Joseph-form covariance, eq. (Josph); g(x) = x / V
 * (the measured temperature), so C = 1/V.                                   */
void oc_ekf_update(const oc_params *p, double *x, double *P, double y)
{
    double C = 1.0 / p->V;
    double yhat = *x / p->V;
    double e = y - yhat;
    double Re = p->Rmeas + C * (*P) * C;
    double K = (*P) * C / Re;
    double IKC = 1.0 - K * C;
    *x = *x + K * e;
    *P = IKC * (*P) * IKC + K * p->Rmeas * K;
}

/* ------------------------------------------------------------------------
 * OCP of eq. (OPC_general) discretised by single shooting: u in mL/min are
 * the only decision variables, x_0 = x-hat_{i|i}, x_{k+1} = RK4^Nc(x_k,
 * u_k), objective phi = sum_{k=1..N} Qz (z_k - zbar_k)^2 Ts with z = x / V
 * (Results section).  zbar[k-1] is the setpoint at t_{i+k}.
 * xs (may be NULL) receives the state at the start of every RK4 step
 * (N*Nc values) and x_N last.                                               */
double oc_ocp_shoot(const oc_params *p, int32_t N, double x0, const double *u,
                    const double *zbar, double *xs)
{
    double h = p->Ts / (double)p->Nc;
    double x = x0, phi = 0.0;
    int k, c;
    for (k = 0; k < N; ++k) {
        double F = u[k] / ML_MIN_PER_L_S;
        for (c = 0; c < p->Nc; ++c) {
            double f[3], k1, k2, k3, k4;
            if (xs) xs[k * p->Nc + c] = x;
            oc_f1(p, x, F, f); k1 = f[0];
            oc_f1(p, x + 0.5 * h * k1, F, f); k2 = f[0];
            oc_f1(p, x + 0.5 * h * k2, F, f); k3 = f[0];
            oc_f1(p, x + h * k3, F, f); k4 = f[0];
            x = x + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
        }
        {
            double ez = x / p->V - zbar[k];
            phi += p->Qz * ez * ez * p->Ts;
        }
    }
    if (xs) xs[N * p->Nc] = x;
    return phi;
}

/* Gradient of phi by the discrete adjoint of the RK4 shooting integrator:
 * lambda runs backwards through every RK4 step; the stage derivatives are
 * those of the forward step, recomputed from the stored step-start state.  */
void oc_ocp_grad_adjoint(const oc_params *p, int32_t N, const double *u,
                         const double *zbar, const double *xs, double *grad)
{
    double h = p->Ts / (double)p->Nc;
    double lam = 0.0;
    int k, c;
    for (k = N - 1; k >= 0; --k) {
        double F = u[k] / ML_MIN_PER_L_S;
        double Fbar = 0.0;
        /* d phi / d x_{k+1} from the stage cost at t_{i+k+1}                */
        {
            double xk1 = xs[(k + 1) * p->Nc];
            double ez = xk1 / p->V - zbar[k];
            lam += p->Qz * 2.0 * ez * (1.0 / p->V) * p->Ts;
        }
        for (c = p->Nc - 1; c >= 0; --c) {
            double x = xs[k * p->Nc + c];
            double f1s[3], f2s[3], f3s[3], f4s[3];
            double kb1, kb2, kb3, kb4, xb;
            oc_f1(p, x, F, f1s);
            oc_f1(p, x + 0.5 * h * f1s[0], F, f2s);
            oc_f1(p, x + 0.5 * h * f2s[0], F, f3s);
            oc_f1(p, x + h * f3s[0], F, f4s);
            /* x+ = x + h/6 (k1 + 2 k2 + 2 k3 + k4)                           */
            xb = lam;
            kb1 = lam * h / 6.0;
            kb2 = lam * h / 3.0;
            kb3 = lam * h / 3.0;
            kb4 = lam * h / 6.0;
            /* k4 = f(x + h k3)                                              */
            xb += kb4 * f4s[1];
            kb3 += kb4 * f4s[1] * h;
            Fbar += kb4 * f4s[2];
            /* k3 = f(x + h/2 k2)                                            */
            xb += kb3 * f3s[1];
            kb2 += kb3 * f3s[1] * 0.5 * h;
            Fbar += kb3 * f3s[2];
            /* k2 = f(x + h/2 k1)                                            */
            xb += kb2 * f2s[1];
            kb1 += kb2 * f2s[1] * 0.5 * h;
            Fbar += kb2 * f2s[2];
            /* k1 = f(x)                                                     */
            xb += kb1 * f1s[1];
            Fbar += kb1 * f1s[2];
            lam = xb;
        }
        grad[k] = Fbar / ML_MIN_PER_L_S;
    }
}

/* Gradient of phi by forward sensitivities: the tangent-linear RK4 carries
 * dx/du_j for every j < k+1 through each step; dphi/du_j accumulates the
 * stage-cost derivative times the sensitivity at each t_{i+k}.              */
void oc_ocp_grad_fwd(const oc_params *p, int32_t N, double x0, const double *u,
                     const double *zbar, double *grad)
{
    double h = p->Ts / (double)p->Nc;
    double S[OC_NMAX];
    double x = x0;
    int k, c, j;
    for (j = 0; j < N; ++j) { S[j] = 0.0; grad[j] = 0.0; }
    for (k = 0; k < N; ++k) {
        double F = u[k] / ML_MIN_PER_L_S;
        double dF = 1.0 / ML_MIN_PER_L_S;      /* dF/du_k                      */
        for (c = 0; c < p->Nc; ++c) {
            double f1s[3], f2s[3], f3s[3], f4s[3];
            oc_f1(p, x, F, f1s);
            oc_f1(p, x + 0.5 * h * f1s[0], F, f2s);
            oc_f1(p, x + 0.5 * h * f2s[0], F, f3s);
            oc_f1(p, x + h * f3s[0], F, f4s);
            for (j = 0; j <= k; ++j) {
                double src = (j == k) ? dF : 0.0;
                double d1 = f1s[1] * S[j] + f1s[2] * src;
                double d2 = f2s[1] * (S[j] + 0.5 * h * d1) + f2s[2] * src;
                double d3 = f3s[1] * (S[j] + 0.5 * h * d2) + f3s[2] * src;
                double d4 = f4s[1] * (S[j] + h * d3) + f4s[2] * src;
                S[j] = S[j] + h / 6.0 * (d1 + 2.0 * d2 + 2.0 * d3 + d4);
            }
            x = x + h / 6.0 * (f1s[0] + 2.0 * f2s[0] + 2.0 * f3s[0] + f4s[0]);
        }
        {
            double ez = x / p->V - zbar[k];
            double dphidx = p->Qz * 2.0 * ez * (1.0 / p->V) * p->Ts;
            for (j = 0; j <= k; ++j) grad[j] += dphidx * S[j];
        }
    }
}

/* ------------------------------------------------------------------------
 * Three-state model for the estimator and the OCP: the plant's eq. (CSTR)
 * drift with the nominal kinetics (k0, Ea/R), state x = n = (n_A, n_B, n_T),
 * output z = n_T / V.  The paper's case study uses the one-state model for
 * both; this is the same CD-EKF and OCP at n_x = 3 (no model-plant mismatch
 * apart from the noise and sampled kinetics).
 * ---------------------------------------------------------------------- */

/* A P + P A^T + Q, Q = diag(q), all row-major 3x3.                          */
static void lyap3_rhs(const double A[9], const double P[9], const double q[3], double out[9])
{
    int a, b, c;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double t = (a == b) ? q[a] : 0.0;
            for (c = 0; c < 3; ++c) t += A[3 * a + c] * P[3 * c + b] + P[3 * a + c] * A[3 * b + c];
            out[3 * a + b] = t;
        }
}

/* CD-EKF prediction, eq. (predictionEquations) at n_x = 3: dx/dt = f3(x, F),
 * dP/dt = A P + P A^T + F^2 diag(sigma_A^2, sigma_B^2, sigma_T^2) (the
 * diffusion F sigma of eq. (CSTR)), A = df3/dx; classical RK4 with Nc steps
 * on the joint (x, P) system, A evaluated at each stage.                    */
void oc_ekf3_predict(const oc_params *p, double x[3], double P[9], double F)
{
    double h = p->Ts / (double)p->Nc;
    double q[3];
    int a, e, c;
    for (a = 0; a < 3; ++a) q[a] = (F * p->sigma[a]) * (F * p->sigma[a]);
    for (c = 0; c < p->Nc; ++c) {
        double kx[4][3], kP[4][9], xs[3], Ps[9], J[9], fF[3];
        int st;
        static const double a_st[4] = {0.0, 0.5, 0.5, 1.0};
        for (st = 0; st < 4; ++st) {
            for (a = 0; a < 3; ++a) xs[a] = x[a] + (st ? a_st[st] * h * kx[st - 1][a] : 0.0);
            for (e = 0; e < 9; ++e) Ps[e] = P[e] + (st ? a_st[st] * h * kP[st - 1][e] : 0.0);
            oc_f3(p, p->k0, p->EaR, xs, F, kx[st]);
            oc_f3_jac(p, p->k0, p->EaR, xs, F, J, fF);
            lyap3_rhs(J, Ps, q, kP[st]);
        }
        for (a = 0; a < 3; ++a)
            x[a] = x[a] + h / 6.0 * (kx[0][a] + 2.0 * kx[1][a] + 2.0 * kx[2][a] + kx[3][a]);
        for (e = 0; e < 9; ++e)
            P[e] = P[e] + h / 6.0 * (kP[0][e] + 2.0 * kP[1][e] + 2.0 * kP[2][e] + kP[3][e]);
    }
}

/* Filtering, eq. (Josph), with g(x) = n_T / V: C = [0, 0, 1/V],
 * R_e = R + C P C^T, K = P C^T / R_e, x += K (y - C x),
 * P = (I - K C) P (I - K C)^T + K R K^T.                                    */
void oc_ekf3_update(const oc_params *p, double x[3], double P[9], double y)
{
    double C[3] = {0.0, 0.0, 1.0 / p->V};
    double PC[3], K[3], IKC[9], T[9], Re, e;
    int a, b, c;
    e = y - (C[0] * x[0] + C[1] * x[1] + C[2] * x[2]);
    for (a = 0; a < 3; ++a) PC[a] = P[3 * a + 0] * C[0] + P[3 * a + 1] * C[1] + P[3 * a + 2] * C[2];
    Re = p->Rmeas + C[0] * PC[0] + C[1] * PC[1] + C[2] * PC[2];
    for (a = 0; a < 3; ++a) K[a] = PC[a] / Re;
    for (a = 0; a < 3; ++a) x[a] = x[a] + K[a] * e;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) IKC[3 * a + b] = (a == b ? 1.0 : 0.0) - K[a] * C[b];
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double t = 0.0;
            for (c = 0; c < 3; ++c) t += IKC[3 * a + c] * P[3 * c + b];
            T[3 * a + b] = t;
        }
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double t = K[a] * p->Rmeas * K[b];
            for (c = 0; c < 3; ++c) t += T[3 * a + c] * IKC[3 * b + c];
            P[3 * a + b] = t;
        }
}

/* Single shooting of the OCP with the three-state model: x_{k+1} =
 * RK4^Nc(x_k, u_k), phi = sum_k Qz (n_T,k+1 / V - zbar_k)^2 Ts.
 * xs (may be NULL) receives the state at the start of every RK4 step
 * (3 values each, step k Nc + c at xs[3 (k Nc + c)]) and x_N last.          */
double oc_ocp3_shoot(const oc_params *p, int32_t N, const double x0[3], const double *u,
                     const double *zbar, double *xs)
{
    double h = p->Ts / (double)p->Nc;
    double x[3] = {x0[0], x0[1], x0[2]}, phi = 0.0;
    int k, c, a;
    for (k = 0; k < N; ++k) {
        double F = u[k] / ML_MIN_PER_L_S;
        for (c = 0; c < p->Nc; ++c) {
            double k1[3], k2[3], k3[3], k4[3], t[3];
            if (xs) for (a = 0; a < 3; ++a) xs[3 * (k * p->Nc + c) + a] = x[a];
            oc_f3(p, p->k0, p->EaR, x, F, k1);
            for (a = 0; a < 3; ++a) t[a] = x[a] + 0.5 * h * k1[a];
            oc_f3(p, p->k0, p->EaR, t, F, k2);
            for (a = 0; a < 3; ++a) t[a] = x[a] + 0.5 * h * k2[a];
            oc_f3(p, p->k0, p->EaR, t, F, k3);
            for (a = 0; a < 3; ++a) t[a] = x[a] + h * k3[a];
            oc_f3(p, p->k0, p->EaR, t, F, k4);
            for (a = 0; a < 3; ++a) x[a] = x[a] + h / 6.0 * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
        }
        {
            double ez = x[2] / p->V - zbar[k];
            phi += p->Qz * ez * ez * p->Ts;
        }
    }
    if (xs) for (a = 0; a < 3; ++a) xs[3 * N * p->Nc + a] = x[a];
    return phi;
}

/* y = M^T v for row-major 3x3 M.                                            */
static void mtv3(const double M[9], const double v[3], double y[3])
{
    int a;
    for (a = 0; a < 3; ++a) y[a] = M[a] * v[0] + M[3 + a] * v[1] + M[6 + a] * v[2];
}

/* y = M v for row-major 3x3 M.                                              */
static void mv3(const double M[9], const double v[3], double y[3])
{
    int a;
    for (a = 0; a < 3; ++a) y[a] = M[3 * a] * v[0] + M[3 * a + 1] * v[1] + M[3 * a + 2] * v[2];
}

/* Gradient of the three-state phi by the discrete adjoint of the RK4
 * shooting: the adjoint vector runs backwards through every RK4 step, each
 * stage contributing J_s^T of its adjoint; stage states recomputed from
 * the stored step-start states.                                             */
void oc_ocp3_grad_adjoint(const oc_params *p, int32_t N, const double *u,
                          const double *zbar, const double *xs, double *grad)
{
    double h = p->Ts / (double)p->Nc;
    double lam[3] = {0.0, 0.0, 0.0};
    int k, c, a;
    for (k = N - 1; k >= 0; --k) {
        double F = u[k] / ML_MIN_PER_L_S;
        double Fbar = 0.0;
        {
            double ez = xs[3 * (k + 1) * p->Nc + 2] / p->V - zbar[k];
            lam[2] += p->Qz * 2.0 * ez * (1.0 / p->V) * p->Ts;
        }
        for (c = p->Nc - 1; c >= 0; --c) {
            const double *x = xs + 3 * (k * p->Nc + c);
            double st[4][3], kk[4][3], J[4][9], fF[4][3];
            double kb[4][3], xb[3], sb[3];
            static const double a_st[4] = {0.0, 0.5, 0.5, 1.0};
            int s;
            for (s = 0; s < 4; ++s) {
                for (a = 0; a < 3; ++a) st[s][a] = x[a] + (s ? a_st[s] * h * kk[s - 1][a] : 0.0);
                oc_f3(p, p->k0, p->EaR, st[s], F, kk[s]);
                oc_f3_jac(p, p->k0, p->EaR, st[s], F, J[s], fF[s]);
            }
            /* x+ = x + h/6 (k1 + 2 k2 + 2 k3 + k4)                           */
            for (a = 0; a < 3; ++a) {
                xb[a] = lam[a];
                kb[0][a] = lam[a] * h / 6.0;
                kb[1][a] = lam[a] * h / 3.0;
                kb[2][a] = lam[a] * h / 3.0;
                kb[3][a] = lam[a] * h / 6.0;
            }
            /* k_s = f(x + a_s h k_{s-1}), from the last stage back           */
            for (s = 3; s >= 0; --s) {
                mtv3(J[s], kb[s], sb);
                for (a = 0; a < 3; ++a) {
                    xb[a] += sb[a];
                    if (s > 0) kb[s - 1][a] += a_st[s] * h * sb[a];
                }
                Fbar += fF[s][0] * kb[s][0] + fF[s][1] * kb[s][1] + fF[s][2] * kb[s][2];
            }
            for (a = 0; a < 3; ++a) lam[a] = xb[a];
        }
        grad[k] = Fbar / ML_MIN_PER_L_S;
    }
}

/* Gradient of the three-state phi by forward sensitivities: the tangent
 * dx/du_j (3 values) of every j <= k is carried through each RK4 step with
 * the stage Jacobians.                                                      */
void oc_ocp3_grad_fwd(const oc_params *p, int32_t N, const double x0[3], const double *u,
                      const double *zbar, double *grad)
{
    double h = p->Ts / (double)p->Nc;
    double S[OC_NMAX][3];
    double x[3] = {x0[0], x0[1], x0[2]};
    int k, c, j, a, s;
    static const double a_st[4] = {0.0, 0.5, 0.5, 1.0};
    for (j = 0; j < N; ++j) { S[j][0] = S[j][1] = S[j][2] = 0.0; grad[j] = 0.0; }
    for (k = 0; k < N; ++k) {
        double F = u[k] / ML_MIN_PER_L_S;
        double dF = 1.0 / ML_MIN_PER_L_S;
        for (c = 0; c < p->Nc; ++c) {
            double st[4][3], kk[4][3], J[4][9], fF[4][3];
            for (s = 0; s < 4; ++s) {
                for (a = 0; a < 3; ++a) st[s][a] = x[a] + (s ? a_st[s] * h * kk[s - 1][a] : 0.0);
                oc_f3(p, p->k0, p->EaR, st[s], F, kk[s]);
                oc_f3_jac(p, p->k0, p->EaR, st[s], F, J[s], fF[s]);
            }
            for (j = 0; j <= k; ++j) {
                double src = (j == k) ? dF : 0.0;
                double d[4][3], t[3], Jt[3];
                for (s = 0; s < 4; ++s) {
                    for (a = 0; a < 3; ++a) t[a] = S[j][a] + (s ? a_st[s] * h * d[s - 1][a] : 0.0);
                    mv3(J[s], t, Jt);
                    for (a = 0; a < 3; ++a) d[s][a] = Jt[a] + fF[s][a] * src;
                }
                for (a = 0; a < 3; ++a)
                    S[j][a] = S[j][a] + h / 6.0 * (d[0][a] + 2.0 * d[1][a] + 2.0 * d[2][a] + d[3][a]);
            }
            for (a = 0; a < 3; ++a)
                x[a] = x[a] + h / 6.0 * (kk[0][a] + 2.0 * kk[1][a] + 2.0 * kk[2][a] + kk[3][a]);
        }
        {
            double ez = x[2] / p->V - zbar[k];
            double dphidx = p->Qz * 2.0 * ez * (1.0 / p->V) * p->Ts;
            for (j = 0; j <= k; ++j) grad[j] += dphidx * S[j][2];
        }
    }
}

/* ------------------------------------------------------------------------
 * Box-constrained QP subproblem of the SQP section (single shooting: no
 * equality constraints, bounds on the input step):
 *   min 1/2 d^T W d + g^T d   s.t.  lo <= d <= hi.
 * The paper solves its QP with a primal-dual interior-point method (Riccati
 * based for the multiple-shooting structure).  Here the same family in dense
 * form: Mehrotra predictor-corrector with slacks s_l = d - lo, s_u = hi - d,
 * multipliers nu_l, nu_u >= 0, and the Newton matrix W + diag(nu_l/s_l +
 * nu_u/s_u) factored by Cholesky; separate primal and dual step lengths
 * (fraction to the boundary 0.995), which keeps the iteration from cycling on
 * inputs whose curvature is tiny.  Start: d strictly inside the box, 1e-2 of
 * its width from the nearer bound, nu = 1.  Stop: stationarity residual
 * <= 1e-12 (1 + |g| + |Wd|), bound residuals <= 1e-12 (1 + |lo| + |hi|),
 * mean complementarity <= 1e-14 (1 + |g|) (infinity norms).
 * Returns 0 converged, 1 iteration cap, -1 non-positive pivot (W not
 * positive definite).                                                       */
static int chol_factor(int N, const double *M, double *Lf)
{
    int i, j, k;
    for (j = 0; j < N; ++j) {
        double s = M[j * N + j];
        for (k = 0; k < j; ++k) s -= Lf[j * N + k] * Lf[j * N + k];
        if (!(s > 0.0)) return -1;
        Lf[j * N + j] = sqrt(s);
        for (i = j + 1; i < N; ++i) {
            double t = M[i * N + j];
            for (k = 0; k < j; ++k) t -= Lf[i * N + k] * Lf[j * N + k];
            Lf[i * N + j] = t / Lf[j * N + j];
        }
    }
    return 0;
}

static void chol_solve(int N, const double *Lf, const double *b, double *x)
{
    double y[OC_NMAX];
    int i, k;
    for (i = 0; i < N; ++i) {
        double t = b[i];
        for (k = 0; k < i; ++k) t -= Lf[i * N + k] * y[k];
        y[i] = t / Lf[i * N + i];
    }
    for (i = N - 1; i >= 0; --i) {
        double t = y[i];
        for (k = i + 1; k < N; ++k) t -= Lf[k * N + i] * x[k];
        x[i] = t / Lf[i * N + i];
    }
}

/* largest a in (0, 1] with v + a dv >= 0 for every component               */
static double max_step(int N, const double *v, const double *dv, double a)
{
    int i;
    for (i = 0; i < N; ++i)
        if (dv[i] < 0.0) {
            double t = -v[i] / dv[i];
            if (t < a) a = t;
        }
    return a;
}

static int ipm_core(int32_t N, const double *W, const double *g, const double *lo,
                    const double *hi, int32_t max_iter, double *d, double *nl, double *nu,
                    int32_t *iters)
{
    double sl[OC_NMAX], su[OC_NMAX], Wd[OC_NMAX], rL[OC_NMAX], rU[OC_NMAX];
    double rhs[OC_NMAX], dd_a[OC_NMAX], dsl_a[OC_NMAX], dsu_a[OC_NMAX];
    double dnl_a[OC_NMAX], dnu_a[OC_NMAX], dd[OC_NMAX], dsl[OC_NMAX], dsu[OC_NMAX];
    double dnl[OC_NMAX], dnu[OC_NMAX];
    double M[OC_NMAX * OC_NMAX], Lf[OC_NMAX * OC_NMAX];
    double gnorm = 0.0, bnorm = 0.0;
    int i, j, it;

    /* strictly interior start                                              */
    for (i = 0; i < N; ++i) {
        double delta = 1e-2 * (hi[i] - lo[i]);
        double di = 0.0;
        if (di < lo[i] + delta) di = lo[i] + delta;
        if (di > hi[i] - delta) di = hi[i] - delta;
        d[i] = di;
        sl[i] = d[i] - lo[i];
        su[i] = hi[i] - d[i];
        nl[i] = 1.0;
        nu[i] = 1.0;
        if (fabs(g[i]) > gnorm) gnorm = fabs(g[i]);
        if (fabs(lo[i]) > bnorm) bnorm = fabs(lo[i]);
        if (fabs(hi[i]) > bnorm) bnorm = fabs(hi[i]);
    }
    for (it = 0;; ++it) {
        double rSn = 0.0, Wdn = 0.0, rPn = 0.0, mu = 0.0, mu_a = 0.0;
        double ap_aff, ad_aff, ap, ad, sigma;
        for (i = 0; i < N; ++i) {
            double t = 0.0;
            for (j = 0; j < N; ++j) t += W[i * N + j] * d[j];
            Wd[i] = t;
            rL[i] = d[i] - sl[i] - lo[i];
            rU[i] = hi[i] - d[i] - su[i];
            {
                double rs = Wd[i] + g[i] - nl[i] + nu[i];
                if (fabs(rs) > rSn) rSn = fabs(rs);
            }
            if (fabs(Wd[i]) > Wdn) Wdn = fabs(Wd[i]);
            if (fabs(rL[i]) > rPn) rPn = fabs(rL[i]);
            if (fabs(rU[i]) > rPn) rPn = fabs(rU[i]);
            mu += sl[i] * nl[i] + su[i] * nu[i];
        }
        mu = mu / (2.0 * N);
        if (rSn <= 1e-12 * (1.0 + gnorm + Wdn) && rPn <= 1e-12 * (1.0 + bnorm)
            && mu <= 1e-14 * (1.0 + gnorm)) {
            *iters = it;
            return 0;
        }
        if (it == max_iter) { *iters = it; return 1; }
        /* Newton matrix and its Cholesky factor                            */
        for (i = 0; i < N; ++i)
            for (j = 0; j < N; ++j)
                M[i * N + j] = W[i * N + j] + (i == j ? nl[i] / sl[i] + nu[i] / su[i] : 0.0);
        if (chol_factor(N, M, Lf) != 0) { *iters = it; return -1; }
        /* predictor (affine scaling) direction                              */
        for (i = 0; i < N; ++i)
            rhs[i] = -(Wd[i] + g[i]) - nl[i] * rL[i] / sl[i] + nu[i] * rU[i] / su[i];
        chol_solve(N, Lf, rhs, dd_a);
        for (i = 0; i < N; ++i) {
            dsl_a[i] = dd_a[i] + rL[i];
            dsu_a[i] = -dd_a[i] + rU[i];
            dnl_a[i] = -nl[i] - nl[i] / sl[i] * dsl_a[i];
            dnu_a[i] = -nu[i] - nu[i] / su[i] * dsu_a[i];
        }
        /* separate primal and dual step lengths                             */
        ap_aff = max_step(N, su, dsu_a, max_step(N, sl, dsl_a, 1.0));
        ad_aff = max_step(N, nu, dnu_a, max_step(N, nl, dnl_a, 1.0));
        for (i = 0; i < N; ++i)
            mu_a += (sl[i] + ap_aff * dsl_a[i]) * (nl[i] + ad_aff * dnl_a[i])
                  + (su[i] + ap_aff * dsu_a[i]) * (nu[i] + ad_aff * dnu_a[i]);
        mu_a = mu_a / (2.0 * N);
        sigma = (mu_a / mu) * (mu_a / mu) * (mu_a / mu);
        /* corrector (centering + second-order) direction                   */
        for (i = 0; i < N; ++i) {
            double cl = dsl_a[i] * dnl_a[i];
            double cu = dsu_a[i] * dnu_a[i];
            rhs[i] = -(Wd[i] + g[i]) + (sigma * mu - cl - nl[i] * rL[i]) / sl[i]
                                     - (sigma * mu - cu - nu[i] * rU[i]) / su[i];
        }
        chol_solve(N, Lf, rhs, dd);
        for (i = 0; i < N; ++i) {
            double cl = dsl_a[i] * dnl_a[i];
            double cu = dsu_a[i] * dnu_a[i];
            dsl[i] = dd[i] + rL[i];
            dsu[i] = -dd[i] + rU[i];
            dnl[i] = (sigma * mu - cl - nl[i] * dsl[i]) / sl[i] - nl[i];
            dnu[i] = (sigma * mu - cu - nu[i] * dsu[i]) / su[i] - nu[i];
        }
        ap = 0.995 * max_step(N, su, dsu, max_step(N, sl, dsl, 1.0));
        ad = 0.995 * max_step(N, nu, dnu, max_step(N, nl, dnl, 1.0));
        if (ap > 1.0) ap = 1.0;
        if (ad > 1.0) ad = 1.0;
        for (i = 0; i < N; ++i) {
            d[i] += ap * dd[i];
            sl[i] += ap * dsl[i];
            su[i] += ap * dsu[i];
            nl[i] += ad * dnl[i];
            nu[i] += ad * dnu[i];
        }
    }
}

/* The QP is solved in Jacobi-scaled variables d = D dt, D = diag(W)^-1/2,
 * so the scaled Hessian has a unit diagonal: DWD dt + Dg with bounds lo/D,
 * hi/D; multipliers map back as nu = nu_t / D.  The minimiser is the same;
 * only the interior-point path is preconditioned.                          */
int oc_box_qp(int32_t N, const double *W, const double *g, const double *lo,
              const double *hi, int32_t max_iter, double *d, double *nl, double *nu,
              int32_t *iters)
{
    double Dg[OC_NMAX], Ws[OC_NMAX * OC_NMAX], gs[OC_NMAX], los[OC_NMAX], his[OC_NMAX];
    int i, j, st;
    for (i = 0; i < N; ++i) {
        if (!(W[i * N + i] > 0.0)) { *iters = 0; return -1; }
        Dg[i] = 1.0 / sqrt(W[i * N + i]);
    }
    for (i = 0; i < N; ++i) {
        for (j = 0; j < N; ++j) Ws[i * N + j] = Dg[i] * W[i * N + j] * Dg[j];
        gs[i] = Dg[i] * g[i];
        los[i] = lo[i] / Dg[i];
        his[i] = hi[i] / Dg[i];
    }
    st = ipm_core(N, Ws, gs, los, his, max_iter, d, nl, nu, iters);
    for (i = 0; i < N; ++i) {
        d[i] = Dg[i] * d[i];
        nl[i] = nl[i] / Dg[i];
        nu[i] = nu[i] / Dg[i];
    }
    return st;
}

/* Damped BFGS update of the SQP section ("Block BFGS update"), one dense
 * block (single shooting): theta rule 0.2 / 0.8, r = theta y + (1-theta) W s,
 * update only when min(s^T W s, s^T r) exceeds the machine precision.
 * Returns 1 updated, 0 skipped.                                             */
int oc_bfgs_update(int32_t N, double *W, const double *s, const double *y)
{
    double Ws[OC_NMAX], r[OC_NMAX];
    double sWs = 0.0, sy = 0.0, sr = 0.0, theta;
    int i, j;
    for (i = 0; i < N; ++i) {
        double t = 0.0;
        for (j = 0; j < N; ++j) t += W[i * N + j] * s[j];
        Ws[i] = t;
    }
    for (i = 0; i < N; ++i) { sWs += s[i] * Ws[i]; sy += s[i] * y[i]; }
    if (sy >= 0.2 * sWs) theta = 1.0;
    else theta = 0.8 * sWs / (sWs - sy);
    for (i = 0; i < N; ++i) r[i] = theta * y[i] + (1.0 - theta) * Ws[i];
    for (i = 0; i < N; ++i) sr += s[i] * r[i];
    {
        double kappa = sWs < sr ? sWs : sr;
        if (!(kappa > DBL_EPSILON)) return 0;
    }
    for (i = 0; i < N; ++i)
        for (j = 0; j < N; ++j)
            W[i * N + j] = W[i * N + j] - Ws[i] * Ws[j] / sWs + r[i] * r[j] / sr;
    return 1;
}

/* The OCP's objective and gradient for the model p->model_nx selects
 * (x0: 1 or 3 values).                                                      */
static double ocp_shoot(const oc_params *p, int32_t N, const double *x0, const double *u,
                        const double *zbar, double *xs)
{
    if (p->model_nx == 3) return oc_ocp3_shoot(p, N, x0, u, zbar, xs);
    return oc_ocp_shoot(p, N, x0[0], u, zbar, xs);
}

static void ocp_grad(const oc_params *p, int32_t N, const double *x0, const double *u,
                     const double *zbar, const double *xs, double *g)
{
    if (p->model_nx == 3) {
        if (p->grad_mode == 1) oc_ocp3_grad_adjoint(p, N, u, zbar, xs, g);
        else oc_ocp3_grad_fwd(p, N, x0, u, zbar, g);
        return;
    }
    if (p->grad_mode == 1) oc_ocp_grad_adjoint(p, N, u, zbar, xs, g);
    else oc_ocp_grad_fwd(p, N, x0[0], u, zbar, g);
}

/* ------------------------------------------------------------------------
 * SQP of the SQP section specialised to m_e = 0, m_l = m_u = N:
 * QP subproblem -> backtracking line search on the merit (which reduces to
 * f when there are no equality constraints) with the Armijo condition
 * eq. (Armijo), c1 = 1e-4, beta = 0.5 -> damped BFGS.  Convergence by the
 * scaled KKT test eq. (convergence) with s_max = 100.  W^[0] = I; W reset to
 * I when the QP reports indefiniteness.  On the iteration cap the last
 * iterate is kept.  x0: the OCP's initial state (1 or 3 values, model_nx).
 * u: in = warm start, out = last iterate.  Returns 1 if converged.          */
int oc_sqp(const oc_params *p, int32_t N, const double *x0, const double *zbar, double *u,
           double *pil, double *piu, double *W, int32_t reset_W, oc_sample_out *cnt)
{
    static const double smax = 100.0;
    double g[OC_NMAX], gn[OC_NMAX], lo[OC_NMAX], hi[OC_NMAX], d[OC_NMAX];
    double nl[OC_NMAX], nu[OC_NMAX], ut[OC_NMAX], s[OC_NMAX], yv[OC_NMAX];
    size_t nxs = (size_t)(N * p->Nc + 1) * (p->model_nx == 3 ? 3 : 1);
    double *xs = (double *)malloc(sizeof(double) * nxs);
    double *xt = (double *)malloc(sizeof(double) * nxs);
    double f;
    int i, j, l, converged = 0;

    for (i = 0; i < N; ++i) {
        if (u[i] < p->umin) u[i] = p->umin;
        if (u[i] > p->umax) u[i] = p->umax;
        pil[i] = 0.0;
        piu[i] = 0.0;
        if (reset_W)
            for (j = 0; j < N; ++j) W[i * N + j] = (i == j) ? 1.0 : 0.0;
    }
    f = ocp_shoot(p, N, x0, u, zbar, xs);
    ocp_grad(p, N, x0, u, zbar, xs, g);
    cnt->grad_evals++;
    cnt->ls_trials++;

    for (l = 0;; ++l) {
        double s1 = 0.0, sd, kkt = 0.0, D = 0.0, alpha;
        int st, it, bt, bad = 0;
        for (i = 0; i < N; ++i) s1 += fabs(pil[i]) + fabs(piu[i]);
        sd = (s1 / (2.0 * N) > smax ? s1 / (2.0 * N) : smax) / smax;
        for (i = 0; i < N; ++i) {
            double t = fabs(g[i] - pil[i] + piu[i]) / sd;
            if (t != t) bad = 1;
            if (t > kkt) kkt = t;
        }
        if (!bad && kkt <= p->sqp_eps) { converged = 1; break; }
        if (l == p->sqp_max_iter) break;

        for (i = 0; i < N; ++i) { lo[i] = p->umin - u[i]; hi[i] = p->umax - u[i]; }
        st = 0;
        for (i = 0; i < N; ++i) if (!(W[i * N + i] > 0.0)) st = -1;
        if (st == 0) {
            st = oc_box_qp(N, W, g, lo, hi, p->ipm_max_iter, d, nl, nu, &it);
            cnt->ipm_iter += it;
        }
        if (st == -1) {
            cnt->bfgs_reset++;
            for (i = 0; i < N; ++i)
                for (j = 0; j < N; ++j) W[i * N + j] = (i == j) ? 1.0 : 0.0;
            st = oc_box_qp(N, W, g, lo, hi, p->ipm_max_iter, d, nl, nu, &it);
            cnt->ipm_iter += it;
        }
        if (st == 1) cnt->ipm_cap++;
        cnt->sqp_iter++;

        for (i = 0; i < N; ++i) D += g[i] * d[i];
        alpha = 1.0;
        for (bt = 0;; ++bt) {
            double ft;
            for (i = 0; i < N; ++i) ut[i] = u[i] + alpha * d[i];
            ft = ocp_shoot(p, N, x0, ut, zbar, xt);
            cnt->ls_trials++;
            /* a predicted decrease below the merit's resolution cannot be
             * tested in floating point: the full step is taken             */
            if (bt == 0 && -D <= 64.0 * DBL_EPSILON * (1.0 + fabs(f))) { f = ft; break; }
            if (ft <= f + p->ls_c1 * alpha * D) { f = ft; break; }
            if (bt == p->ls_max_bt) { cnt->ls_cap++; f = ft; break; }
            alpha = p->ls_beta * alpha;
        }
        for (i = 0; i < N; ++i) {
            s[i] = ut[i] - u[i];
            u[i] = ut[i];
            pil[i] = pil[i] + alpha * (nl[i] - pil[i]);
            piu[i] = piu[i] + alpha * (nu[i] - piu[i]);
        }
        { double *tmp = xs; xs = xt; xt = tmp; }
        ocp_grad(p, N, x0, u, zbar, xs, gn);
        cnt->grad_evals++;
        for (i = 0; i < N; ++i) { yv[i] = gn[i] - g[i]; g[i] = gn[i]; }
        if (!oc_bfgs_update(N, W, s, yv)) cnt->bfgs_skip++;
    }
    free(xs);
    free(xt);
    return converged;
}

/* ------------------------------------------------------------------------
 * One closed-loop Monte Carlo sample.                                       */
typedef struct {
    int64_t noise_id;
    int32_t kind, N, L, istep;
    double sign, k0, EaR;
    double n0[3], xhat0, ubar;      /* ubar in L/s */
    double xhat3[3];                /* three-state estimator's x-hat_0      */
} oc_setup;

static uint32_t id32(int64_t id) { return (uint32_t)id; }

/* ov (or NULL): caller-given {kind, N, L} of the sample, -1 = the draw.   */
static void sample_setup(const oc_params *p, int64_t sample_id, const int32_t *ov, oc_setup *su)
{
    double nr[4];
    double Fss, nss[3];
    su->noise_id = p->noise_mod > 0 ? sample_id % p->noise_mod : sample_id;
    if (p->kind_split >= 0) su->kind = sample_id < p->kind_split ? 0 : 1;
    else su->kind = p->default_kind;
    su->N = p->N;
    su->L = p->L;
    if (p->n_horizon_choices > 0) {
        int idx;
        oc_normal_pair(p->seed, 0, 0, id32(su->noise_id), TAG_SCEN, nr);
        idx = (int)floor(nr[3] * p->n_horizon_choices);
        su->N = p->horizon_choices[idx];
    }
    if (p->L_lo < p->L_hi) {
        oc_normal_pair(p->seed, 1, 0, id32(su->noise_id), TAG_SCEN, nr);
        su->L = p->L_lo + (int32_t)floor(nr[3] * (double)(p->L_hi - p->L_lo + 1));
    }
    if (ov) {
        if (ov[0] >= 0) su->kind = ov[0];
        if (ov[1] >= 0) su->N = ov[1];
        if (ov[2] >= 0) su->L = ov[2];
    }
    su->istep = 0;
    su->sign = 0.0;
    if (p->sp_step_rel != 0.0) {
        oc_normal_pair(p->seed, 2, 0, id32(su->noise_id), TAG_SCEN, nr);
        su->istep = p->sp_step_lo
                  + (int32_t)floor(nr[3] * (double)(p->sp_step_hi - p->sp_step_lo + 1));
        oc_normal_pair(p->seed, 3, 0, id32(su->noise_id), TAG_SCEN, nr);
        su->sign = nr[3] < 0.5 ? 1.0 : -1.0;
    }
    su->k0 = p->k0;
    su->EaR = p->EaR;
    if (p->kin_lognorm_sigma > 0.0) {
        oc_normal_pair(p->seed, 0, 0, id32(su->noise_id), TAG_KIN, nr);
        su->k0 = p->k0 * exp(p->kin_lognorm_sigma * nr[0]);
        su->EaR = p->EaR * exp(p->kin_lognorm_sigma * nr[1]);
    }
    {
        double z0 = oc_setpoint(p, 0, su->istep, su->sign);
        oc_steady_state(p, z0, &Fss, nss);
        su->ubar = Fss;
        if (p->x0_mode == 0) {
            su->n0[0] = p->cAin * p->V;
            su->n0[1] = p->cBin * p->V;
            su->n0[2] = p->cTin * p->V;
            su->xhat0 = p->cTin * p->V;
            su->xhat3[0] = su->n0[0];
            su->xhat3[1] = su->n0[1];
            su->xhat3[2] = su->n0[2];
        } else {
            double nb[4];
            oc_normal_pair(p->seed, 0, 0, id32(su->noise_id), TAG_X0, nr);
            oc_normal_pair(p->seed, 1, 0, id32(su->noise_id), TAG_X0, nb);
            su->n0[0] = nss[0] * (1.0 + p->x0_rel_std * nr[0]);
            su->n0[1] = nss[1] * (1.0 + p->x0_rel_std * nr[1]);
            su->n0[2] = nss[2] * (1.0 + p->x0_rel_std * nb[0]);
            su->xhat0 = nss[2];
            su->xhat3[0] = nss[0];
            su->xhat3[1] = nss[1];
            su->xhat3[2] = nss[2];
        }
    }
}

static uint64_t fnv1a_bytes(uint64_t h, const unsigned char *b, int n)
{
    int i;
    for (i = 0; i < n; ++i) { h ^= (uint64_t)b[i]; h *= 1099511628211ull; }
    return h;
}

void oc_scenario(const oc_params *p, int64_t sample_id, int32_t iv[4], double dv[3])
{
    oc_setup su;
    sample_setup(p, sample_id, NULL, &su);
    iv[0] = su.kind;
    iv[1] = su.N;
    iv[2] = su.L;
    iv[3] = su.istep;
    dv[0] = su.sign;
    dv[1] = su.k0;
    dv[2] = su.EaR;
}

void oc_run_sample(const oc_params *p, int64_t sample_id, oc_sample_out *out,
                   double *traj_z, double *traj_u, double *traj_xhat)
{
    oc_run_sample_ext(p, sample_id, NULL, out, traj_z, traj_u, traj_xhat, NULL);
}

void oc_run_sample_ext(const oc_params *p, int64_t sample_id, const int32_t *ov,
                       oc_sample_out *out, double *traj_z, double *traj_u, double *traj_xhat,
                       double *traj_I)
{
    oc_setup su;
    double n[3], xhat, P, Fprev, Ihat = 0.0, phiacc = 0.0;
    double xh3[3], P3[9];            /* three-state estimator (model_nx 3)   */
    double ws[OC_NMAX], u[OC_NMAX], zb[OC_NMAX], pil[OC_NMAX], piu[OC_NMAX];
    double Wh[OC_NMAX * OC_NMAX];
    /* PI tangent w.r.t. theta = (Kc, tau_i) with kP = Kc, kI = Kc / tau_i:
     * dn[a][b] = dn_a/dtheta_b, dI[b] = dIhat/dtheta_b                       */
    double dn[3][2], dI[2] = {0.0, 0.0}, dphi[2] = {0.0, 0.0}, dF[2] = {0.0, 0.0};
    double dkP[2] = {1.0, 0.0}, dkI[2];
    double sqrtR = sqrt(p->Rmeas);
    double h = p->Ts / (double)p->Ns;
    int tangent;
    uint64_t hsh = 14695981039346656037ull;
    int i, j, k, a, b;

    memset(out, 0, sizeof(*out));
    sample_setup(p, sample_id, ov, &su);
    tangent = p->want_grad && su.kind == 1;
    {
        double Kc = p->kP, taui = p->kP / p->kI;
        dkI[0] = 1.0 / taui;
        dkI[1] = -Kc / (taui * taui);
    }
    for (a = 0; a < 3; ++a) { n[a] = su.n0[a]; dn[a][0] = 0.0; dn[a][1] = 0.0; }
    xhat = su.xhat0;
    P = p->P0;
    /* three-state estimator: x-hat_0 as the one-state reading, P_0 = P0 I   */
    for (a = 0; a < 3; ++a) {
        xh3[a] = su.xhat3[a];
        for (b = 0; b < 3; ++b) P3[3 * a + b] = (a == b) ? p->P0 : 0.0;
    }
    Fprev = su.ubar;
    for (k = 0; k < su.N; ++k) ws[k] = su.ubar * ML_MIN_PER_L_S;
    out->kind = su.kind;
    out->N = su.N;
    out->L = su.L;

    for (i = 0;; ++i) {
        double z = n[2] / p->V;
        double zb_i = oc_setpoint(p, i, su.istep, su.sign);
        double y, F, xi[4];
        /* cost term of eq. (Phi) on the true output z = c_T                 */
        phiacc += (z - zb_i) * (z - zb_i);
        if (traj_z) traj_z[i] = z;
        if (tangent)
            for (b = 0; b < 2; ++b) dphi[b] += 2.0 * (z - zb_i) * dn[2][b] / p->V;
        if (i == su.L) break;
        if (su.kind == 0 && !isfinite(z)) {
            /* the plant diverged: Phi is not a number and no further OCP
             * is solved                                                     */
            out->nonfinite = 1;
            break;
        }
        /* measurement y_i = c_T(t_i) + v_i, v ~ N(0, R)                     */
        oc_normal_pair(p->seed, 0, (uint32_t)i, id32(su.noise_id), TAG_MEAS, xi);
        y = z + p->noise_scale * sqrtR * xi[0];
        if ((su.kind == 0 || p->run_ekf_for_pi) && p->model_nx == 3) {
            oc_ekf3_predict(p, xh3, P3, Fprev);
            oc_ekf3_update(p, xh3, P3, y);
            xhat = xh3[2];
            for (a = 0; a < 9; ++a)
                if (!isfinite(P3[a])) out->nonfinite = 1;
            if (!isfinite(xh3[0]) || !isfinite(xh3[1])) out->nonfinite = 1;
        } else if (su.kind == 0 || p->run_ekf_for_pi) {
            oc_ekf_predict(p, &xhat, &P, Fprev);
            oc_ekf_update(p, &xhat, &P, y);
        }
        if (traj_xhat) traj_xhat[i] = xhat;
        if (!isfinite(xhat) || !isfinite(P)) out->nonfinite = 1;
        if (su.kind == 0) {
            /* NMPC: OCP from x-hat_{i|i} with the preview zbar(t_{i+1..i+N});
             * only the first input is implemented (receding horizon)         */
            uint64_t mask = 0;
            unsigned char buf[12];
            for (k = 0; k < su.N; ++k) {
                zb[k] = oc_setpoint(p, i + 1 + k, su.istep, su.sign);
                u[k] = ws[k];
            }
            if (p->nlp_form == 1) {
                /* the paper's multiple-shooting NLP, W^[0] = I at every OCP */
                double xms[OC_NMAX + 1];
                if (!oc_ms_sqp(p, su.N, xhat, zb, u, xms, out)) out->n_ocp_fail++;
            } else if (!oc_sqp(p, su.N, p->model_nx == 3 ? xh3 : &xhat, zb, u, pil, piu, Wh,
                               i == 0 || !p->hess_warm, out)) {
                out->n_ocp_fail++;
            }
            out->n_ocp++;
            for (k = 0; k < su.N; ++k)
                if (u[k] <= p->umin + 1e-6 || u[k] >= p->umax - 1e-6) mask |= (1ull << k);
            for (j = 0; j < 4; ++j) buf[j] = (unsigned char)(((uint32_t)i) >> (8 * j));
            for (j = 0; j < 8; ++j) buf[4 + j] = (unsigned char)(mask >> (8 * j));
            hsh = fnv1a_bytes(hsh, buf, 12);
            F = u[0] / ML_MIN_PER_L_S;
            for (k = 0; k + 1 < su.N; ++k) ws[k] = u[k + 1];
            ws[su.N - 1] = u[su.N - 1];
            if (p->hess_warm && p->nlp_form == 0) {
                /* shifted Hessian: drop u_0's row/column, repeat the last
                 * diagonal entry with no coupling                            */
                int r, c2;
                double last = Wh[(su.N - 1) * su.N + (su.N - 1)];
                for (r = 0; r + 1 < su.N; ++r)
                    for (c2 = 0; c2 + 1 < su.N; ++c2)
                        Wh[r * su.N + c2] = Wh[(r + 1) * su.N + (c2 + 1)];
                for (c2 = 0; c2 < su.N; ++c2) {
                    Wh[(su.N - 1) * su.N + c2] = 0.0;
                    Wh[c2 * su.N + (su.N - 1)] = 0.0;
                }
                Wh[(su.N - 1) * su.N + (su.N - 1)] = last;
            }
        } else {
            /* PI with clipping and anti-windup, eq. (PI); e uses y, not x-hat */
            double e = zb_i - y;
            double Pk = p->kP * e;
            double Ik = Ihat + p->Ts * p->kI * e;
            double uh = su.ubar + Pk + Ik;
            double uk = uh;
            int inside = (uh > p->pi_umin && uh < p->pi_umax);
            if (uk > p->pi_umax) uk = p->pi_umax;
            if (uk < p->pi_umin) uk = p->pi_umin;
            if (tangent) {
                for (b = 0; b < 2; ++b) {
                    double de = -dn[2][b] / p->V;
                    double dP = dkP[b] * e + p->kP * de;
                    double dIk = dI[b] + p->Ts * (dkI[b] * e + p->kI * de);
                    double duh = dP + dIk;
                    dF[b] = inside ? duh : 0.0;
                    dI[b] = dIk + p->Ts * p->kaw * (duh - dF[b]);
                }
            }
            Ihat = Ik + p->Ts * p->kaw * (uh - uk);
            if (traj_I) traj_I[i] = Ihat;
            F = uk;
        }
        if (traj_u) traj_u[i] = F;
        /* plant: Ns Euler-Maruyama sub-steps with the input held (ZOH)      */
        for (j = 0; j < p->Ns; ++j) {
            double x0[4], x1[4], w[3];
            oc_normal_pair(p->seed, 0, (uint32_t)(i * p->Ns + j), id32(su.noise_id),
                           TAG_PROCESS, x0);
            oc_normal_pair(p->seed, 1, (uint32_t)(i * p->Ns + j), id32(su.noise_id),
                           TAG_PROCESS, x1);
            w[0] = p->noise_scale * x0[0];
            w[1] = p->noise_scale * x0[1];
            w[2] = p->noise_scale * x1[0];
            if (tangent) {
                /* dn+ = dn + h (J dn + f_F dF) + dF sigma sqrt(h) xi        */
                double J[9], fF[3];
                oc_f3_jac(p, su.k0, su.EaR, n, F, J, fF);
                for (b = 0; b < 2; ++b) {
                    double dnew[3];
                    for (a = 0; a < 3; ++a) {
                        double Jd = J[3 * a + 0] * dn[0][b] + J[3 * a + 1] * dn[1][b]
                                  + J[3 * a + 2] * dn[2][b];
                        dnew[a] = dn[a][b] + h * (Jd + fF[a] * dF[b])
                                + dF[b] * p->sigma[a] * sqrt(h) * w[a];
                    }
                    for (a = 0; a < 3; ++a) dn[a][b] = dnew[a];
                }
            }
            oc_em_step(p, su.k0, su.EaR, n, F, w);
        }
        Fprev = F;
    }
    if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) out->nonfinite = 1;
    out->phi = phiacc / (double)(su.L + 1);
    out->dphi[0] = dphi[0] / (double)(su.L + 1);
    out->dphi[1] = dphi[1] / (double)(su.L + 1);
    out->ashash = hsh;
}

/* ------------------------------------------------------------------------
 * Thread pool over sample ids (one sample per task, no shared mutable state
 * beyond the task counter).                                                 */
typedef struct {
    const oc_params *p;
    const int64_t *ids;
    const int32_t *ov;        /* [3][n] {kind, N, L} per task, -1 = drawn, or NULL */
    int64_t n;
    oc_sample_out *out;
    int64_t next;
    pthread_mutex_t mu;
} oc_pool;

static void *oc_worker(void *arg)
{
    oc_pool *pool = (oc_pool *)arg;
    for (;;) {
        int64_t t;
        pthread_mutex_lock(&pool->mu);
        t = pool->next++;
        pthread_mutex_unlock(&pool->mu);
        if (t >= pool->n) break;
        if (pool->ov) {
            int32_t ov[3] = {pool->ov[t], pool->ov[pool->n + t], pool->ov[2 * pool->n + t]};
            oc_run_sample_ext(pool->p, pool->ids[t], ov, &pool->out[t], NULL, NULL, NULL, NULL);
        } else {
            oc_run_sample(pool->p, pool->ids[t], &pool->out[t], NULL, NULL, NULL);
        }
    }
    return NULL;
}

void oc_run(const oc_params *p, const int64_t *ids, int64_t n, int32_t nthreads,
            oc_sample_out *out)
{
    oc_run_ov(p, ids, NULL, n, nthreads, out);
}

void oc_run_ov(const oc_params *p, const int64_t *ids, const int32_t *ov, int64_t n,
               int32_t nthreads, oc_sample_out *out)
{
    oc_pool pool;
    pthread_t th[256];
    int t;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pool.p = p; pool.ids = ids; pool.ov = ov; pool.n = n; pool.out = out; pool.next = 0;
    pthread_mutex_init(&pool.mu, NULL);
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, oc_worker, &pool);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&pool.mu);
}

/* ------------------------------------------------------------------------
 * Distribution of Phi, eq. (Phi) over the samples whose Phi is finite (a
 * diverged closed loop has none): mean, sample variance
 * (divisor n-1), both with Neumaier-compensated sums; histogram of log10 Phi
 * in 200 equal bins on [-4, 4), left-closed, hist[0] = underflow, hist[201]
 * = overflow.                                                               */
static void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

void oc_stats(const double *phi, int64_t n, double *mean, double *var, int64_t *hist)
{
    double s = 0.0, c = 0.0, m, s2 = 0.0, c2 = 0.0;
    int64_t i, nf = 0;
    for (i = 0; i < 202; ++i) hist[i] = 0;
    for (i = 0; i < n; ++i)
        if (isfinite(phi[i])) { neumaier_add(&s, &c, phi[i]); nf++; }
    m = nf > 0 ? (s + c) / (double)nf : 0.0;
    for (i = 0; i < n; ++i)
        if (isfinite(phi[i])) neumaier_add(&s2, &c2, (phi[i] - m) * (phi[i] - m));
    *mean = m;
    *var = nf > 1 ? (s2 + c2) / (double)(nf - 1) : 0.0;
    for (i = 0; i < n; ++i) {
        double v;
        if (!isfinite(phi[i])) continue;
        v = log10(phi[i]);
        if (!(v >= -4.0)) hist[0]++;
        else if (v >= 4.0) hist[201]++;
        else {
            int64_t b = (int64_t)floor((v + 4.0) / 8.0 * 200.0);
            if (b > 199) b = 199;
            hist[1 + b]++;
        }
    }
}
