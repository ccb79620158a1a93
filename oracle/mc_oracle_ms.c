/*
 * mc_oracle_ms.c -- TEST INFRASTRUCTURE ONLY (part of the CPU oracle, see
 * mc_oracle.c).  The paper's own NLP formulation of the OCP: direct multiple
 * shooting, eq. (OCP_NLP), solved by the SQP of the Sequential Quadratic
 * Programming section -- structured QP subproblem eq. (QP-subproblem),
 * backtracking line search on Powell's l1 merit with its sigma update
 * (Line-search, eq. (Armijo)), block damped BFGS with W^[0] = I (Block BFGS
 * update) and the scaled KKT test eq. (convergence) with the constraint
 * residual test.  One-state model (the paper's case study).
 *
 * Plain and slow on purpose: dense matrices, no structure exploited.  The
 * structured QP has a unique minimiser (block-diagonal W positive definite),
 * so it is computed here by eliminating the state steps through the linear
 * dynamics (condensing) and solving the remaining box QP in the input steps
 * with the oracle's dense interior point (oc_box_qp); the state steps and
 * the equality multipliers follow by back substitution.  The paper's
 * solver reaches the same point by a Riccati-recursion interior point.
 *
 * Decision vector xi = [u_0, x_1, u_1, x_2, ..., u_{N-1}, x_N] (2N values;
 * u_k at 2k, x_k at 2k-1); x_0 = x-hat_{i|i} is a parameter.  Constraints
 * c_k = F(x_k, u_k) - x_{k+1} = 0, k = 0..N-1, with F = RK4^Nc of the
 * one-state model over one sampling interval (u in mL/min).  Lagrangian
 * L = f - lambda^T c - pi_l^T (u - u_min) - pi_u^T (u_max - u), f = phi of
 * the Regulator section (stage costs on x_1..x_N only).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "mc_oracle.h"

#define ML_MIN_PER_L_S 60000.0

/* One interval: out = {F(x, u), dF/dx, dF/du} by the tangent-linear RK4
 * (the exact derivatives of the discrete map), u in mL/min.               */
void oc_ms_interval(const oc_params *p, double x, double u, double out[3])
{
    double h = p->Ts / (double)p->Nc;
    double F = u / ML_MIN_PER_L_S, dF = 1.0 / ML_MIN_PER_L_S;
    double X = x, SX = 1.0, SU = 0.0;
    int c;
    for (c = 0; c < p->Nc; ++c) {
        double f1s[3], f2s[3], f3s[3], f4s[3];
        double X2, X3, X4, a1, a2, a3, a4, b1, b2, b3, b4;
        oc_f1(p, X, F, f1s);
        a1 = f1s[1] * SX;
        b1 = f1s[1] * SU + f1s[2] * dF;
        X2 = X + 0.5 * h * f1s[0];
        oc_f1(p, X2, F, f2s);
        a2 = f2s[1] * (SX + 0.5 * h * a1);
        b2 = f2s[1] * (SU + 0.5 * h * b1) + f2s[2] * dF;
        X3 = X + 0.5 * h * f2s[0];
        oc_f1(p, X3, F, f3s);
        a3 = f3s[1] * (SX + 0.5 * h * a2);
        b3 = f3s[1] * (SU + 0.5 * h * b2) + f3s[2] * dF;
        X4 = X + h * f3s[0];
        oc_f1(p, X4, F, f4s);
        a4 = f4s[1] * (SX + h * a3);
        b4 = f4s[1] * (SU + h * b3) + f4s[2] * dF;
        X = X + h / 6.0 * (f1s[0] + 2.0 * f2s[0] + 2.0 * f3s[0] + f4s[0]);
        SX = SX + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
        SU = SU + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4);
    }
    out[0] = X;
    out[1] = SX;
    out[2] = SU;
}

/* f = sum_{k=1..N} Qz Ts (x_k / V - zbar_k)^2, zbar_k = zbar[k-1].         */
static double ms_f(const oc_params *p, int32_t N, const double *x, const double *zbar)
{
    double f = 0.0;
    int k;
    for (k = 1; k <= N; ++k) {
        double e = x[k] / p->V - zbar[k - 1];
        f += p->Qz * p->Ts * e * e;
    }
    return f;
}

/* df/dx_k, k = 1..N (fx[k]; fx[0] unused).                                 */
static void ms_fx(const oc_params *p, int32_t N, const double *x, const double *zbar, double *fx)
{
    int k;
    fx[0] = 0.0;
    for (k = 1; k <= N; ++k)
        fx[k] = 2.0 * p->Qz * p->Ts * (x[k] / p->V - zbar[k - 1]) / p->V;
}

/* Interval maps at (x, u): Fv, A, B per k = 0..N-1, and c_k = F_k - x_{k+1}. */
static void ms_eval(const oc_params *p, int32_t N, const double *x, const double *u,
                    double *Fv, double *A, double *B, double *c)
{
    int k;
    for (k = 0; k < N; ++k) {
        double o[3];
        oc_ms_interval(p, x[k], u[k], o);
        Fv[k] = o[0];
        A[k] = o[1];
        B[k] = o[2];
        c[k] = o[0] - x[k + 1];
    }
}

/* grad_xi L in xi order (2N values).                                       */
static void ms_gradL(int32_t N, const double *fx, const double *A, const double *B,
                     const double *lam, const double *pil, const double *piu, double *gL)
{
    int k;
    for (k = 0; k < N; ++k) gL[2 * k] = -lam[k] * B[k] - pil[k] + piu[k];
    for (k = 1; k < N; ++k) gL[2 * k - 1] = fx[k] - lam[k] * A[k] + lam[k - 1];
    gL[2 * N - 1] = fx[N] + lam[N - 1];
}

/* Block structure of the Lagrangian Hessian (Block BFGS update): block 0 is
 * {u_0}, block k = 1..N-1 is {x_k, u_k}, block N is {x_N}.  first/size give
 * the block's first xi index and its size.                                 */
static void ms_block(int32_t N, int b, int *first, int *size)
{
    if (b == 0) { *first = 0; *size = 1; }
    else if (b == N) { *first = 2 * N - 1; *size = 1; }
    else { *first = 2 * b - 1; *size = 2; }
}

/* The damped BFGS update of one block of the dense W (n = 2N); returns 1
 * updated, 0 skipped (kappa <= eps_m).                                     */
static int ms_bfgs_block(int n, double *W, int f0, int m, const double *s, const double *y)
{
    double Ws[2], r[2], sWs = 0.0, sy = 0.0, sr = 0.0, theta, kappa;
    int i, j;
    for (i = 0; i < m; ++i) {
        double t = 0.0;
        for (j = 0; j < m; ++j) t += W[(f0 + i) * n + (f0 + j)] * s[f0 + j];
        Ws[i] = t;
    }
    for (i = 0; i < m; ++i) { sWs += s[f0 + i] * Ws[i]; sy += s[f0 + i] * y[f0 + i]; }
    theta = (sy >= 0.2 * sWs) ? 1.0 : 0.8 * sWs / (sWs - sy);
    for (i = 0; i < m; ++i) r[i] = theta * y[f0 + i] + (1.0 - theta) * Ws[i];
    for (i = 0; i < m; ++i) sr += s[f0 + i] * r[i];
    kappa = sWs < sr ? sWs : sr;
    if (!(kappa > DBL_EPSILON)) return 0;
    for (i = 0; i < m; ++i)
        for (j = 0; j < m; ++j)
            W[(f0 + i) * n + (f0 + j)] += -Ws[i] * Ws[j] / sWs + r[i] * r[j] / sr;
    return 1;
}

/* Every block positive definite (1x1: w > 0; 2x2: w11 > 0, det > 0).       */
static int ms_blocks_pd(int32_t N, const double *W)
{
    int n = 2 * N, b;
    for (b = 0; b <= N; ++b) {
        int f0, m;
        ms_block(N, b, &f0, &m);
        if (!(W[f0 * n + f0] > 0.0)) return 0;
        if (m == 2) {
            double det = W[f0 * n + f0] * W[(f0 + 1) * n + f0 + 1]
                       - W[f0 * n + f0 + 1] * W[(f0 + 1) * n + f0];
            if (!(det > 0.0)) return 0;
        }
    }
    return 1;
}

static void ms_identity(int n, double *W)
{
    int i, j;
    for (i = 0; i < n; ++i)
        for (j = 0; j < n; ++j) W[i * n + j] = (i == j) ? 1.0 : 0.0;
}

/* Structured QP, eq. (QP-subproblem):
 *   min 1/2 dxi^T W dxi + gf^T dxi
 *   s.t. dx_{k+1} = A_k dx_k + B_k du_k + c_k (dx_0 = 0),
 *        umin - u_k <= du_k <= umax - u_k,
 * with gf = grad f in xi order.  Condensed: dxi = T du + t, the box QP
 * min 1/2 du^T (T^T W T) du + (T^T (W t + gf))^T du by oc_box_qp, then dxi
 * and the multipliers mu (equalities) from the stationarity conditions in
 * dx_N, ..., dx_1.  Returns oc_box_qp's status (-1: not positive definite). */
int oc_ms_qp(const oc_params *p, int32_t N, const double *W, const double *gf,
             const double *A, const double *B, const double *c, const double *u,
             double *dxi, double *mu, double *nl, double *nu, int32_t *iters)
{
    int n = 2 * N, i, j, k, st;
    double *T = (double *)calloc((size_t)n * N, sizeof(double));
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *H = (double *)calloc((size_t)N * N, sizeof(double));
    double *WT = (double *)calloc((size_t)n * N, sizeof(double));
    double *h = (double *)calloc((size_t)N, sizeof(double));
    double *Wt = (double *)calloc((size_t)n, sizeof(double));
    double *Wd = (double *)calloc((size_t)n, sizeof(double));
    double lo[OC_NMAX] = {0.0}, hi[OC_NMAX] = {0.0}, du[OC_NMAX];
    for (i = 0; i < N; ++i) {
        lo[i] = p->umin - u[i];
        hi[i] = p->umax - u[i];
    }
    /* dxi = T du + t: du_k = du_k; dx_{k+1} = A_k dx_k + B_k du_k + c_k     */
    for (k = 0; k < N; ++k) T[(2 * k) * N + k] = 1.0;
    for (k = 0; k < N; ++k) {
        int row = 2 * (k + 1) - 1;       /* x_{k+1}                          */
        int prev = 2 * k - 1;            /* x_k (none for k = 0)             */
        for (j = 0; j < N; ++j) {
            double v = (prev >= 0 ? A[k] * T[prev * N + j] : 0.0) + (j == k ? B[k] : 0.0);
            T[row * N + j] = v;
        }
        t[row] = (prev >= 0 ? A[k] * t[prev] : 0.0) + c[k];
    }
    for (i = 0; i < n; ++i) {
        for (j = 0; j < N; ++j) {
            double s = 0.0;
            for (k = 0; k < n; ++k) s += W[i * n + k] * T[k * N + j];
            WT[i * N + j] = s;
        }
        {
            double s = 0.0;
            for (k = 0; k < n; ++k) s += W[i * n + k] * t[k];
            Wt[i] = s;
        }
    }
    for (i = 0; i < N; ++i) {
        for (j = 0; j < N; ++j) {
            double s = 0.0;
            for (k = 0; k < n; ++k) s += T[k * N + i] * WT[k * N + j];
            H[i * N + j] = s;
        }
        {
            double s = 0.0;
            for (k = 0; k < n; ++k) s += T[k * N + i] * (Wt[k] + gf[k]);
            h[i] = s;
        }
    }
    /* the condensed Hessian is symmetric up to rounding: use its mean     */
    for (i = 0; i < N; ++i)
        for (j = 0; j < i; ++j) {
            double m = 0.5 * (H[i * N + j] + H[j * N + i]);
            H[i * N + j] = m;
            H[j * N + i] = m;
        }
    st = oc_box_qp(N, H, h, lo, hi, p->ipm_max_iter, du, nl, nu, iters);
    if (st != -1) {
        for (i = 0; i < n; ++i) {
            double s = t[i];
            for (j = 0; j < N; ++j) s += T[i * N + j] * du[j];
            dxi[i] = s;
        }
        for (i = 0; i < n; ++i) {
            double s = 0.0;
            for (k = 0; k < n; ++k) s += W[i * n + k] * dxi[k];
            Wd[i] = s;
        }
        /* stationarity in dx_N: (W dxi)_xN + gf_xN + mu_{N-1} = 0; in dx_k
         * (k < N): (W dxi)_xk + gf_xk - mu_k A_k + mu_{k-1} = 0             */
        mu[N - 1] = -(Wd[2 * N - 1] + gf[2 * N - 1]);
        for (k = N - 1; k >= 1; --k)
            mu[k - 1] = -(Wd[2 * k - 1] + gf[2 * k - 1] - mu[k] * A[k]);
    }
    free(T); free(t); free(H); free(WT); free(h); free(Wt); free(Wd);
    return st;
}

/* The SQP on eq. (OCP_NLP).  u (in: warm start, out: last iterate; N
 * values), x (out: states x_1..x_N at x[1..N]; x[0] = x0), all multipliers
 * start at 0 and W^[0] = I.  The initial states follow the initial inputs
 * through the model (a feasible start, c = 0).  Returns 1 if converged.    */
int oc_ms_sqp(const oc_params *p, int32_t N, double x0, const double *zbar, double *u,
              double *x, oc_sample_out *cnt)
{
    static const double smax = 100.0;
    int n = 2 * N, i, k, l, converged = 0, first = 1;
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *gL = (double *)malloc(sizeof(double) * n), *gLn = (double *)malloc(sizeof(double) * n);
    double *gf = (double *)malloc(sizeof(double) * n), *dxi = (double *)malloc(sizeof(double) * n);
    double *s = (double *)malloc(sizeof(double) * n), *yv = (double *)malloc(sizeof(double) * n);
    double Fv[OC_NMAX], A[OC_NMAX], B[OC_NMAX], c[OC_NMAX], fx[OC_NMAX + 1];
    double Ft[OC_NMAX], At[OC_NMAX], Bt[OC_NMAX], ct[OC_NMAX], fxt[OC_NMAX + 1];
    double xt[OC_NMAX + 1], ut[OC_NMAX];
    double lam[OC_NMAX], pil[OC_NMAX], piu[OC_NMAX], mu[OC_NMAX], nl[OC_NMAX], nu[OC_NMAX];
    double sig[OC_NMAX];
    double f;

    ms_identity(n, W);
    x[0] = x0;
    for (k = 0; k < N; ++k) {
        double o[3];
        if (u[k] < p->umin) u[k] = p->umin;
        if (u[k] > p->umax) u[k] = p->umax;
        oc_ms_interval(p, x[k], u[k], o);
        x[k + 1] = o[0];
        lam[k] = pil[k] = piu[k] = 0.0;
        sig[k] = 0.0;
    }
    ms_eval(p, N, x, u, Fv, A, B, c);
    ms_fx(p, N, x, zbar, fx);
    f = ms_f(p, N, x, zbar);
    cnt->ls_trials++;
    cnt->grad_evals++;

    for (l = 0;; ++l) {
        double s1 = 0.0, sd, kkt = 0.0, cmax = 0.0, D, T0, alpha;
        int st, it, bt, bad = 0;
        ms_gradL(N, fx, A, B, lam, pil, piu, gL);
        for (k = 0; k < N; ++k) s1 += fabs(lam[k]) + fabs(pil[k]) + fabs(piu[k]);
        sd = (s1 / (3.0 * N) > smax ? s1 / (3.0 * N) : smax) / smax;
        for (i = 0; i < n; ++i) {
            double tv = fabs(gL[i]) / sd;
            if (tv != tv) bad = 1;
            if (tv > kkt) kkt = tv;
        }
        for (k = 0; k < N; ++k) {
            if (c[k] != c[k]) bad = 1;
            if (fabs(c[k]) > cmax) cmax = fabs(c[k]);
        }
        if (!bad && kkt <= p->sqp_eps && cmax <= p->sqp_eps) { converged = 1; break; }
        if (l == p->sqp_max_iter) break;

        /* gradient of f in xi order                                        */
        for (k = 0; k < N; ++k) gf[2 * k] = 0.0;
        for (k = 1; k <= N; ++k) gf[2 * k - 1] = fx[k];
        st = ms_blocks_pd(N, W) ? 0 : -1;
        if (st == 0) {
            st = oc_ms_qp(p, N, W, gf, A, B, c, u, dxi, mu, nl, nu, &it);
            cnt->ipm_iter += it;
        }
        if (st == -1) {
            cnt->bfgs_reset++;
            ms_identity(n, W);
            st = oc_ms_qp(p, N, W, gf, A, B, c, u, dxi, mu, nl, nu, &it);
            cnt->ipm_iter += it;
        }
        if (st == 1) cnt->ipm_cap++;
        cnt->sqp_iter++;

        /* Powell's l1 merit: sigma = |mu| at the first iteration, then
         * sigma_i = max(|mu_i|, (sigma_i + |mu_i|) / 2)                    */
        for (k = 0; k < N; ++k) {
            double am = fabs(mu[k]);
            if (first) sig[k] = am;
            else sig[k] = am > 0.5 * (sig[k] + am) ? am : 0.5 * (sig[k] + am);
        }
        first = 0;
        T0 = f;
        D = 0.0;
        for (k = 0; k < N; ++k) T0 += sig[k] * fabs(c[k]);
        for (i = 0; i < n; ++i) D += gf[i] * dxi[i];
        for (k = 0; k < N; ++k) D -= sig[k] * fabs(c[k]);
        alpha = 1.0;
        for (bt = 0;; ++bt) {
            double Tt;
            xt[0] = x0;
            for (k = 0; k < N; ++k) ut[k] = u[k] + alpha * dxi[2 * k];
            for (k = 1; k <= N; ++k) xt[k] = x[k] + alpha * dxi[2 * k - 1];
            ms_eval(p, N, xt, ut, Ft, At, Bt, ct);
            Tt = ms_f(p, N, xt, zbar);
            for (k = 0; k < N; ++k) Tt += sig[k] * fabs(ct[k]);
            cnt->ls_trials++;
            /* a predicted decrease below the merit's resolution cannot be
             * tested in floating point: the full step is taken             */
            if (bt == 0 && -D <= 64.0 * DBL_EPSILON * (1.0 + fabs(T0))) break;
            if (Tt <= T0 + p->ls_c1 * alpha * D) break;
            if (bt == p->ls_max_bt) { cnt->ls_cap++; break; }
            alpha = p->ls_beta * alpha;
        }
        /* step: xi, lambda, pi <- + alpha (delta)                          */
        for (k = 0; k < N; ++k) {
            s[2 * k] = ut[k] - u[k];
            lam[k] = lam[k] + alpha * (mu[k] - lam[k]);
            pil[k] = pil[k] + alpha * (nl[k] - pil[k]);
            piu[k] = piu[k] + alpha * (nu[k] - piu[k]);
        }
        for (k = 1; k <= N; ++k) s[2 * k - 1] = xt[k] - x[k];
        /* y = grad L(xi+, lambda+, pi+) - grad L(xi, lambda+, pi+)          */
        ms_gradL(N, fx, A, B, lam, pil, piu, gL);
        ms_fx(p, N, xt, zbar, fxt);
        ms_gradL(N, fxt, At, Bt, lam, pil, piu, gLn);
        for (i = 0; i < n; ++i) yv[i] = gLn[i] - gL[i];
        for (k = 0; k < N; ++k) {
            u[k] = ut[k];
            Fv[k] = Ft[k];
            A[k] = At[k];
            B[k] = Bt[k];
            c[k] = ct[k];
        }
        for (k = 1; k <= N; ++k) { x[k] = xt[k]; fx[k] = fxt[k]; }
        f = ms_f(p, N, x, zbar);
        cnt->grad_evals++;
        /* block damped BFGS                                                */
        {
            int b, skipped = 0;
            for (b = 0; b <= N; ++b) {
                int f0, m;
                ms_block(N, b, &f0, &m);
                if (!ms_bfgs_block(n, W, f0, m, s, yv)) skipped++;
            }
            if (skipped == N + 1) cnt->bfgs_skip++;
        }
    }
    free(W); free(gL); free(gLn); free(gf); free(dxi); free(s); free(yv);
    return converged;
}
