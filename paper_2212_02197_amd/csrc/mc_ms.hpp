// mc_ms.hpp -- the paper's NLP formulation of the NMPC's OCP on gfx950:
// direct multiple shooting, eq. (OCP_NLP), solved by the SQP of the
// Sequential Quadratic Programming section with
//   * the structured QP subproblem, eq. (QP-subproblem), solved by a
//     Mehrotra predictor-corrector primal-dual interior point whose Newton
//     systems are solved by a Riccati recursion over the stages (the
//     paper's solver family, Implementation / QP subproblem);
//   * the backtracking line search on Powell's l1 merit with its sigma
//     update, eq. (Armijo) (Line-search);
//   * the block damped BFGS update from W^[0] = I with a full reset on an
//     indefinite block (Block BFGS update);
//   * the scaled KKT test with the constraint residual test, eq.
//     (convergence).
// One-state model (the paper's case study), scalar per stage: every stage
// quantity is a scalar and the 2x2 Hessian blocks are three numbers, so the
// whole SQP runs one sample per lane with no cooperative work.  The stage
// arrays of a wavefront's 64 samples live in a per-wave-slot workspace,
// array a, stage k, lane l at ((a * NMAX + k) * 64 + l): each stage access of
// the wave is one coalesced 512-byte row.
//
// Decision vector xi = [u_0, x_1, u_1, ..., u_{N-1}, x_N]; x_0 = x-hat_{i|i}.
// Constraints c_k = F(x_k, u_k) - x_{k+1} (F: RK4 with Nc steps over Ts,
// u in mL/min); Lagrangian L = f - lambda^T c - pi_l^T (u - u_min)
// - pi_u^T (u_max - u); f = phi of the Regulator section, stage costs on
// x_1..x_N.
#pragma once
#include "mc_kernels.hpp"

namespace mccl {

// Stage arrays.  Index k = 0..N-1 throughout; the state entries of stage k
// are those of x_{k+1} (X, FX, WXX, DX, P, PV: the state after interval k).
enum : int {
    M_U = 0,   // u_k
    M_X,       // x_{k+1}
    M_LAM,     // lambda_k (constraint k)
    M_PIL, M_PIU,
    M_A, M_B,  // dF/dx, dF/du of interval k at (x_k, u_k)
    M_C,       // c_k
    M_FX,      // df/dx_{k+1}
    M_WXX,     // Hessian block entry of x_{k+1}
    M_WXU,     // off-diagonal entry of block {x_k, u_k} (k >= 1)
    M_WUU,     // entry of u_k
    M_SIG,     // merit weight sigma_k
    M_DU, M_DX, M_MU, M_NL, M_NU,      // QP primal (du_k, dx_{k+1}) and dual
    M_K, M_HI, M_P, M_KF, M_PV,        // Riccati: K_k, 1/H_uu,k, P_{k+1}, k_k, p_{k+1}
    M_DUA,     // predictor (affine) du_k
    M_COUNT
};

struct MsWork {
    const int64_t* pos;
    int64_t n_pos;
    int n_groups;
    int* queue;
    const int* qhi;
    double* ws;          // per slot: M_COUNT * NMAX * 64
    int64_t stride;
};

// Stage-array accessor of one lane.
template <int NMAX>
struct MsArr {
    double* base;   // slot base + lane
    __device__ __forceinline__ double& operator()(int a, int k) const {
        return base[((a * NMAX) + k) * 64];
    }
};

// One sampling interval of the one-state model, RK4 with Nc steps: returns
// F(x, u); with kDeriv also A = dF/dx, B = dF/du (u in mL/min) by the
// tangent-linear RK4, the exact derivatives of the discrete map.
template <bool kDeriv>
__device__ __forceinline__ double ms_interval(const DevParams& p, double x, double u, double& A,
                                              double& B) {
    const double h = p.Ts / (double)p.Nc;
    const double F = u / kMlMinPerLs;
    const double dF = 1.0 / kMlMinPerLs;
    double X = x, SX = 1.0, SU = 0.0;
    #pragma unroll 1
    for (int c = 0; c < p.Nc; ++c) {
        double a1 = 0, a2 = 0, a3 = 0, a4 = 0, f1 = 0, f2 = 0, f3 = 0, f4 = 0;
        const double k1 = model_f1<kDeriv>(p, X, F, a1, f1);
        const double k2 = model_f1<kDeriv>(p, X + 0.5 * h * k1, F, a2, f2);
        const double k3 = model_f1<kDeriv>(p, X + 0.5 * h * k2, F, a3, f3);
        const double k4 = model_f1<kDeriv>(p, X + h * k3, F, a4, f4);
        if (kDeriv) {
            const double d1x = a1 * SX, d1u = a1 * SU + f1 * dF;
            const double d2x = a2 * (SX + 0.5 * h * d1x), d2u = a2 * (SU + 0.5 * h * d1u) + f2 * dF;
            const double d3x = a3 * (SX + 0.5 * h * d2x), d3u = a3 * (SU + 0.5 * h * d2u) + f3 * dF;
            const double d4x = a4 * (SX + h * d3x), d4u = a4 * (SU + h * d3u) + f4 * dF;
            SX = SX + h / 6.0 * (d1x + 2.0 * d2x + 2.0 * d3x + d4x);
            SU = SU + h / 6.0 * (d1u + 2.0 * d2u + 2.0 * d3u + d4u);
        }
        X = X + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    }
    A = SX;
    B = SU;
    return X;
}

// Damped BFGS update of a 1x1 block w (Block BFGS update); returns 1 if
// applied, 0 if skipped (kappa <= eps_m).
__device__ __forceinline__ int ms_bfgs1(double& w, double s, double y) {
    const double Ws = w * s, sWs = s * Ws, sy = s * y;
    const double theta = (sy >= 0.2 * sWs) ? 1.0 : 0.8 * sWs / (sWs - sy);
    const double r = theta * y + (1.0 - theta) * Ws;
    const double sr = s * r;
    const double kappa = sWs < sr ? sWs : sr;
    if (!(kappa > 0x1p-52)) return 0;
    w = w - Ws * Ws / sWs + r * r / sr;
    return 1;
}

// The same for a 2x2 block [a b; b c] with s = (s1, s2), y = (y1, y2).
__device__ __forceinline__ int ms_bfgs2(double& a, double& b, double& c, double s1, double s2,
                                        double y1, double y2) {
    const double w1 = a * s1 + b * s2, w2 = b * s1 + c * s2;
    const double sWs = s1 * w1 + s2 * w2, sy = s1 * y1 + s2 * y2;
    const double theta = (sy >= 0.2 * sWs) ? 1.0 : 0.8 * sWs / (sWs - sy);
    const double r1 = theta * y1 + (1.0 - theta) * w1, r2 = theta * y2 + (1.0 - theta) * w2;
    const double sr = s1 * r1 + s2 * r2;
    const double kappa = sWs < sr ? sWs : sr;
    if (!(kappa > 0x1p-52)) return 0;
    a = a - w1 * w1 / sWs + r1 * r1 / sr;
    b = b - w1 * w2 / sWs + r1 * r2 / sr;
    c = c - w2 * w2 / sWs + r2 * r2 / sr;
    return 1;
}

// Structured QP, eq. (QP-subproblem), at the current SQP iterate:
//   min 1/2 dxi^T W dxi + sum_k fx_k dx_{k+1}
//   s.t. dx_{k+1} = A_k dx_k + B_k du_k + c_k (dx_0 = 0),
//        u_min - u_k <= du_k <= u_max - u_k,
// by a Mehrotra predictor-corrector primal-dual interior point: slacks
// t_l = du - lo, t_u = hi - du kept positive, bound multipliers nu > 0,
// fraction to the boundary 0.995 with separate primal and dual step
// lengths.  Each Newton system is the equality-constrained stage QP with
// R~_k = W_uu,k + nu_l/t_l + nu_u/t_u, solved by the backward Riccati
// recursion (factor K_k, 1/H_uu,k, P_{k+1} once per iteration, shared by
// predictor and corrector) and a forward sweep; the equality multipliers
// follow as mu_k = -(P_{k+1} dx_{k+1} + p_{k+1}).  Start strictly inside the
// box, 1e-2 of its width from the nearer bound, nu = 1, the states from the
// dynamics.  Stop: stationarity residual <= 1e-12 (1 + |fx| + |W dxi|) and
// mean complementarity <= 1e-14 (1 + |fx|) (infinity norms), or ipm_max_iter
// iterations.  Returns 0 converged, 1 iteration cap, -1 an H_uu <= 0 (W not
// positive definite).  Results in DU, DX, MU, NL, NU.
// The stage arrays arrive as separate restrict-qualified pointers (element
// k at [k * 64]): no store of one sweep can alias another array's load,
// so the unrolled sweeps issue the loads of several stages together.
__device__ __forceinline__ int ms_qp_body(const DevParams& p, int N, int& iters,
                                         const double* __restrict__ gU,
                                         const double* __restrict__ gA,
                                         const double* __restrict__ gB,
                                         const double* __restrict__ gC,
                                         const double* __restrict__ gFX,
                                         const double* __restrict__ gWXX,
                                         const double* __restrict__ gWXU,
                                         const double* __restrict__ gWUU,
                                         double* __restrict__ gDU,
                                         double* __restrict__ gDX,
                                         double* __restrict__ gMU,
                                         double* __restrict__ gNL,
                                         double* __restrict__ gNU,
                                         double* __restrict__ gK,
                                         double* __restrict__ gHI,
                                         double* __restrict__ gP,
                                         double* __restrict__ gKF,
                                         double* __restrict__ gPV,
                                         double* __restrict__ gDUA) {
    double gsc = 0.0;
    {
        double dx = 0.0;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
            const double dl = 1e-2 * (hi - lo);
            double du = 0.0;
            if (du < lo + dl) du = lo + dl;
            if (du > hi - dl) du = hi - dl;
            gDU[(k) * 64] = du;
            gNL[(k) * 64] = 1.0;
            gNU[(k) * 64] = 1.0;
            gMU[(k) * 64] = 0.0;
            dx = gA[(k) * 64] * dx + gB[(k) * 64] * du + gC[(k) * 64];
            gDX[(k) * 64] = dx;
            gsc = fmax(gsc, fabs(gFX[(k) * 64]));
        }
    }
    const double inv2N = 1.0 / (2.0 * N);
    #pragma unroll 1
    for (int it = 0;; ++it) {
        // backward sweep: residuals of the current point, their norms, the
        // Riccati factors and the predictor's vectors (complementarity
        // target 0)
        double Pn = gWXX[(N - 1) * 64];
        double rxN = gWXX[(N - 1) * 64] * gDX[(N - 1) * 64] + gFX[(N - 1) * 64] + gMU[(N - 1) * 64];
        double pn = rxN;
        double rmax = fabs(rxN), wd = fabs(gWXX[(N - 1) * 64] * gDX[(N - 1) * 64]), comp = 0.0;
        #pragma unroll 4
        for (int k = N - 1; k >= 0; --k) {
            const double A = gA[(k) * 64], B = gB[(k) * 64];
            const double du = gDU[(k) * 64], nl = gNL[(k) * 64], nu = gNU[(k) * 64], mu = gMU[(k) * 64];
            const double dxk = k >= 1 ? gDX[(k - 1) * 64] : 0.0;
            const double wuu = gWUU[(k) * 64], wxu = k >= 1 ? gWXU[(k) * 64] : 0.0;
            const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
            const double tl = du - lo, tu = hi - du;
            const double wdu = wuu * du + wxu * dxk;
            const double ru = wdu - mu * B - nl + nu;
            comp += tl * nl + tu * nu;
            const double Rt = wuu + nl / tl + nu / tu;
            const double rt = ru + nl - nu;
            const double e = pn;
            const double Huu = Rt + B * B * Pn;
            if (!(Huu > 0.0)) { iters = it; return -1; }
            const double hinv = 1.0 / Huu;
            const double kf = -(rt + B * e) * hinv;
            gHI[(k) * 64] = hinv;
            gKF[(k) * 64] = kf;
            gP[(k) * 64] = Pn;
            gPV[(k) * 64] = pn;
            rmax = fmax(rmax, fabs(ru));
            wd = fmax(wd, fabs(wdu));
            if (k >= 1) {
                const double wxx = gWXX[(k - 1) * 64];
                const double wdx = wxx * dxk + wxu * du;
                const double rx = wdx + gFX[(k - 1) * 64] - mu * A + gMU[(k - 1) * 64];
                const double Hux = wxu + B * Pn * A;
                const double K = -Hux * hinv;
                gK[(k) * 64] = K;
                Pn = wxx + A * A * Pn + Hux * K;
                pn = rx + A * e + Hux * kf;
                rmax = fmax(rmax, fabs(rx));
                wd = fmax(wd, fabs(wdx));
            }
        }
        const double muc = comp * inv2N;
        if (rmax <= 1e-12 * (1.0 + gsc + wd) && muc <= 1e-14 * (1.0 + gsc)) { iters = it; return 0; }
        if (it == p.ipm_max_iter) { iters = it; return 1; }
        // forward predictor: affine step and its lengths
        double apr = 1.0, adr = 1.0;
        {
            double dx = 0.0;
            #pragma unroll 4
            for (int k = 0; k < N; ++k) {
                const double dua = (k >= 1 ? gK[(k) * 64] * dx : 0.0) + gKF[(k) * 64];
                gDUA[(k) * 64] = dua;
                const double du = gDU[(k) * 64], nl = gNL[(k) * 64], nu = gNU[(k) * 64];
                const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
                const double tl = du - lo, tu = hi - du;
                const double dnl = -nl - nl * dua / tl, dnu = -nu + nu * dua / tu;
                if (dua < 0.0) apr = fmin(apr, -tl / dua);
                if (dua > 0.0) apr = fmin(apr, tu / dua);
                if (dnl < 0.0) adr = fmin(adr, -nl / dnl);
                if (dnu < 0.0) adr = fmin(adr, -nu / dnu);
                dx = gA[(k) * 64] * dx + gB[(k) * 64] * dua;
            }
        }
        double maff = 0.0;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            const double dua = gDUA[(k) * 64];
            const double du = gDU[(k) * 64], nl = gNL[(k) * 64], nu = gNU[(k) * 64];
            const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
            const double tl = du - lo, tu = hi - du;
            const double dnl = -nl - nl * dua / tl, dnu = -nu + nu * dua / tu;
            maff += (tl + apr * dua) * (nl + adr * dnl) + (tu - apr * dua) * (nu + adr * dnu);
        }
        maff *= inv2N;
        const double ratio = muc > 0.0 ? maff / muc : 0.0;
        const double smu = ratio * ratio * ratio * muc;   // sigma mu
        // backward corrector: the Riccati vectors with the centred,
        // second-order-corrected complementarity targets
        pn = rxN;
        #pragma unroll 4
        for (int k = N - 1; k >= 0; --k) {
            const double A = gA[(k) * 64], B = gB[(k) * 64];
            const double du = gDU[(k) * 64], nl = gNL[(k) * 64], nu = gNU[(k) * 64], mu = gMU[(k) * 64];
            const double dxk = k >= 1 ? gDX[(k - 1) * 64] : 0.0;
            const double wuu = gWUU[(k) * 64], wxu = k >= 1 ? gWXU[(k) * 64] : 0.0;
            const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
            const double tl = du - lo, tu = hi - du;
            const double ru = wuu * du + wxu * dxk - mu * B - nl + nu;
            const double dua = gDUA[(k) * 64];
            const double dnla = -nl - nl * dua / tl, dnua = -nu + nu * dua / tu;
            const double taul = smu - dua * dnla, tauu = smu + dua * dnua;
            const double rt = ru + nl - taul / tl - nu + tauu / tu;
            const double Pn1 = gP[(k) * 64];
            const double e = pn;
            const double kf = -(rt + B * e) * gHI[(k) * 64];
            gKF[(k) * 64] = kf;
            gPV[(k) * 64] = pn;
            if (k >= 1) {
                const double wxx = gWXX[(k - 1) * 64];
                const double rx = wxx * dxk + wxu * du + gFX[(k - 1) * 64] - mu * A + gMU[(k - 1) * 64];
                const double Hux = wxu + B * Pn1 * A;
                pn = rx + A * e + Hux * kf;
            }
        }
        // forward corrector, twice: step lengths, then the update with the
        // direction recomputed (the same arithmetic, so the same values)
        double ap = 1.0, ad = 1.0;
        #pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            double dx = 0.0;
            #pragma unroll 4
            for (int k = 0; k < N; ++k) {
                const double A = gA[(k) * 64], B = gB[(k) * 64];
                const double ddu = (k >= 1 ? gK[(k) * 64] * dx : 0.0) + gKF[(k) * 64];
                const double ddx = A * dx + B * ddu;
                const double dmu = -(gP[(k) * 64] * ddx + gPV[(k) * 64]);
                const double du = gDU[(k) * 64], nl = gNL[(k) * 64], nu = gNU[(k) * 64];
                const double lo = p.umin - gU[(k) * 64], hi = p.umax - gU[(k) * 64];
                const double tl = du - lo, tu = hi - du;
                const double dua = gDUA[(k) * 64];
                const double dnla = -nl - nl * dua / tl, dnua = -nu + nu * dua / tu;
                const double taul = smu - dua * dnla, tauu = smu + dua * dnua;
                const double dnl = (-tl * nl + taul - nl * ddu) / tl;
                const double dnu = (-tu * nu + tauu + nu * ddu) / tu;
                if (pass == 0) {
                    if (ddu < 0.0) ap = fmin(ap, -tl / ddu);
                    if (ddu > 0.0) ap = fmin(ap, tu / ddu);
                    if (dnl < 0.0) ad = fmin(ad, -nl / dnl);
                    if (dnu < 0.0) ad = fmin(ad, -nu / dnu);
                } else {
                    gDU[(k) * 64] = du + ap * ddu;
                    gDX[(k) * 64] = gDX[(k) * 64] + ap * ddx;
                    gMU[(k) * 64] = gMU[(k) * 64] + ad * dmu;
                    gNL[(k) * 64] = nl + ad * dnl;
                    gNU[(k) * 64] = nu + ad * dnu;
                }
                dx = ddx;
            }
            if (pass == 0) {
                ap = fmin(1.0, 0.995 * ap);
                ad = fmin(1.0, 0.995 * ad);
            }
        }
    }
}

template <int NMAX>
__device__ int ms_qp(const DevParams& p, const MsArr<NMAX>& a, int N, int& iters) {
    auto g = [&](int m) { return &a(m, 0); };
    return ms_qp_body(p, N, iters, g(M_U), g(M_A), g(M_B), g(M_C), g(M_FX), g(M_WXX), g(M_WXU), g(M_WUU), g(M_DU), g(M_DX), g(M_MU), g(M_NL), g(M_NU), g(M_K), g(M_HI), g(M_P), g(M_KF), g(M_PV), g(M_DUA));
}

// Merit of the trial point xi + alpha dxi: f + sigma^T |c| (value-only
// intervals).
template <int NMAX>
__device__ double ms_trial(const DevParams& p, const MsArr<NMAX>& a, int N, double x0, int i0,
                           int istep, double sign, double alpha) {
    double xk = x0, T = 0.0, dA, dB;
    #pragma unroll 1
    for (int k = 0; k < N; ++k) {
        const double xn = a(M_X, k) + alpha * a(M_DX, k);
        const double u = a(M_U, k) + alpha * a(M_DU, k);
        const double F = ms_interval<false>(p, xk, u, dA, dB);
        const double ez = xn / p.V - setpoint(p, i0 + 1 + k, istep, sign);
        T += a(M_SIG, k) * fabs(F - xn) + p.Qz * p.Ts * ez * ez;
        xk = xn;
    }
    return T;
}

// The SQP of one OCP from x-hat (x0) with the warm-started inputs in M_U;
// returns true if the KKT test passed (else the last iterate stands).
template <int NMAX>
__device__ bool ms_sqp(const DevParams& p, const MsArr<NMAX>& a, int N, double x0, int i0,
                       int istep, double sign, int (&cnt)[C_NCNT]) {
    const double smax = 100.0;
    const double cst = 2.0 * p.Qz * p.Ts / p.V;
    double f = 0.0;
    {
        // feasible start: the states follow the inputs; W^[0] = I
        double xk = x0;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            double u = a(M_U, k);
            if (u < p.umin) u = p.umin;
            if (u > p.umax) u = p.umax;
            a(M_U, k) = u;
            double A, B;
            const double F = ms_interval<true>(p, xk, u, A, B);
            a(M_A, k) = A;
            a(M_B, k) = B;
            a(M_X, k) = F;
            a(M_C, k) = 0.0;
            const double ez = F / p.V - setpoint(p, i0 + 1 + k, istep, sign);
            a(M_FX, k) = cst * ez;
            f += p.Qz * p.Ts * ez * ez;
            a(M_WXX, k) = 1.0;
            a(M_WXU, k) = 0.0;
            a(M_WUU, k) = 1.0;
            a(M_LAM, k) = 0.0;
            a(M_PIL, k) = 0.0;
            a(M_PIU, k) = 0.0;
            a(M_SIG, k) = 0.0;
            xk = F;
        }
    }
    cnt[C_LS]++;
    cnt[C_GRAD]++;
    bool first = true;
    #pragma unroll 1
    for (int l = 0;; ++l) {
        // eq. (convergence): |grad L / s_d|_inf <= eps and |c|_inf <= eps
        double s1 = 0.0, gmax = 0.0, cmax = 0.0;
        bool bad = false;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            const double lam = a(M_LAM, k), pl = a(M_PIL, k), pu = a(M_PIU, k);
            s1 += fabs(lam) + fabs(pl) + fabs(pu);
            const double gu = -lam * a(M_B, k) - pl + pu;
            const double gx = a(M_FX, k) + lam - (k + 1 < N ? a(M_LAM, k + 1) * a(M_A, k + 1) : 0.0);
            const double c = a(M_C, k);
            bad = bad || !(gu == gu) || !(gx == gx) || !(c == c);
            gmax = fmax(gmax, fmax(fabs(gu), fabs(gx)));
            cmax = fmax(cmax, fabs(c));
        }
        const double sd = fmax(smax, s1 / (3.0 * N)) / smax;
        if (!bad && gmax / sd <= p.sqp_eps && cmax <= p.sqp_eps) return true;
        if (l == p.sqp_max_iter) return false;
        // QP; an indefinite block (or H_uu <= 0 in the recursion) resets W
        bool pd = true;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            const double wuu = a(M_WUU, k), wxx = a(M_WXX, k);
            pd = pd && wuu > 0.0 && wxx > 0.0;
            if (k >= 1) {
                const double wx = a(M_WXX, k - 1), wxu = a(M_WXU, k);
                pd = pd && (wx * wuu - wxu * wxu > 0.0);
            }
        }
        int it = 0, st = pd ? ms_qp<NMAX>(p, a, N, it) : -1;
        cnt[C_IPM] += it;
        if (st == -1) {
            cnt[C_RESET]++;
            #pragma unroll 4
            for (int k = 0; k < N; ++k) {
                a(M_WXX, k) = 1.0;
                a(M_WXU, k) = 0.0;
                a(M_WUU, k) = 1.0;
            }
            st = ms_qp<NMAX>(p, a, N, it);
            cnt[C_IPM] += it;
        }
        if (st == 1) cnt[C_IPMCAP]++;
        cnt[C_SQP]++;
        // Powell's l1 merit: sigma = |mu| first, then max(|mu|, (sigma + |mu|)/2)
        double T0 = f, D = 0.0;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            const double am = fabs(a(M_MU, k));
            const double sg = first ? am : fmax(am, 0.5 * (a(M_SIG, k) + am));
            a(M_SIG, k) = sg;
            const double ac = fabs(a(M_C, k));
            T0 += sg * ac;
            D += a(M_FX, k) * a(M_DX, k) - sg * ac;
        }
        first = false;
        double alpha = 1.0;
        #pragma unroll 1
        for (int bt = 0;; ++bt) {
            const double Tt = ms_trial<NMAX>(p, a, N, x0, i0, istep, sign, alpha);
            cnt[C_LS]++;
            // a predicted decrease below the merit's resolution cannot be
            // tested in floating point: the full step is taken
            if (bt == 0 && -D <= 64.0 * 0x1p-52 * (1.0 + fabs(T0))) break;
            if (Tt <= T0 + p.ls_c1 * alpha * D) break;
            if (bt == p.ls_max_bt) { cnt[C_LSCAP]++; break; }
            alpha = p.ls_beta * alpha;
        }
        // the step, the new interval derivatives, and the block BFGS with
        // y = grad L(xi+, lambda+, pi+) - grad L(xi, lambda+, pi+)
        f = 0.0;
        int applied = 0;
        double xn = x0;              // x_k after the step
        double fxo_k = 0.0, fxn_k = 0.0, sx_k = 0.0;   // df/dx_k old / new, alpha dx_k
        #pragma unroll 1
        for (int k = 0; k < N; ++k) {
            const double Ao = a(M_A, k), Bo = a(M_B, k);
            const double su = alpha * a(M_DU, k);
            const double un = a(M_U, k) + su;
            const double sxn = alpha * a(M_DX, k);
            const double xk1 = a(M_X, k) + sxn;
            double An, Bn;
            const double F = ms_interval<true>(p, xn, un, An, Bn);
            const double lam = a(M_LAM, k) + alpha * (a(M_MU, k) - a(M_LAM, k));
            a(M_LAM, k) = lam;
            a(M_PIL, k) = a(M_PIL, k) + alpha * (a(M_NL, k) - a(M_PIL, k));
            a(M_PIU, k) = a(M_PIU, k) + alpha * (a(M_NU, k) - a(M_PIU, k));
            const double ez = xk1 / p.V - setpoint(p, i0 + 1 + k, istep, sign);
            const double fx_old = a(M_FX, k), fx_new = cst * ez;
            f += p.Qz * p.Ts * ez * ez;
            if (k == 0) {
                double w = a(M_WUU, 0);
                applied += ms_bfgs1(w, su, -lam * (Bn - Bo));
                a(M_WUU, 0) = w;
            } else {
                double wa = a(M_WXX, k - 1), wb = a(M_WXU, k), wc = a(M_WUU, k);
                applied += ms_bfgs2(wa, wb, wc, sx_k, su, fxn_k - fxo_k - lam * (An - Ao),
                                    -lam * (Bn - Bo));
                a(M_WXX, k - 1) = wa;
                a(M_WXU, k) = wb;
                a(M_WUU, k) = wc;
            }
            a(M_U, k) = un;
            a(M_X, k) = xk1;
            a(M_A, k) = An;
            a(M_B, k) = Bn;
            a(M_C, k) = F - xk1;
            a(M_FX, k) = fx_new;
            xn = xk1;
            fxo_k = fx_old;
            fxn_k = fx_new;
            sx_k = sxn;
        }
        {
            double w = a(M_WXX, N - 1);
            applied += ms_bfgs1(w, sx_k, fxn_k - fxo_k);
            a(M_WXX, N - 1) = w;
        }
        if (applied == 0) cnt[C_SKIP]++;
        cnt[C_GRAD]++;
    }
}

// Algorithmic FP64 work of a multiple-shooting NMPC sample from its counters
// (each +, -, *, / counts 1, an FMA 2):
//   interval value 73 Nc (4 model evaluations of 14 + the RK4 combination)
//   per stage of a trial; interval with derivatives 142 Nc + 4 (model with
//   its derivatives 26 each, the tangent stages 30, the combinations 8);
//   per SQP iteration the KKT test 10 N, the positive-definiteness test
//   4 N, the merit set-up 8 N, the accepted step with the block BFGS
//   60 N besides its intervals; per interior-point iteration 130 N (the
//   six stage sweeps of the predictor-corrector); the QP set-up 12 N.
__device__ __forceinline__ double ms_sample_flops(const DevParams& p, int N, int L,
                                                  const int (&c)[C_NCNT]) {
    const double Ns = p.Ns, Nc = p.Nc, n = N, l = L;
    double fl = 3.0 * (l + 1.0) + l * (8.0 + 52.0 * Ns) + l * (142.0 * Nc + 12.0);
    const double ivd = (142.0 * Nc + 4.0) * n;
    fl += (double)c[C_GRAD] * ivd;                            // start + accepted steps
    fl += (double)(c[C_LS] - c[C_GRAD]) * (73.0 * Nc + 12.0) * n;   // trials
    fl += (double)c[C_SQP] * (10.0 + 4.0 + 8.0 + 60.0 + 12.0) * n;
    fl += (double)c[C_IPM] * 130.0 * n;
    return fl;
}

// Persistent NMPC kernel of the multiple-shooting formulation: one sample
// per lane, 64 per wavefront, groups taken from the work queue.  The
// closed loop per interval is that of nmpc_kernel (cost, measurement, CD-EKF,
// OCP, first input applied, Ns Euler-Maruyama sub-steps); the OCP starts
// from the previous solution shifted by one interval with W^[0] = I.
template <int NMAX>
__global__ __launch_bounds__(64) void nmpc_ms_kernel(DevParams p, MsWork wk, Outs out) {
    const int lane = threadIdx.x;
    const MsArr<NMAX> a{wk.ws + (int64_t)blockIdx.x * wk.stride + lane};
    const double sqrtR = sqrt(p.Rmeas);
    const double h = p.Ts / (double)p.Ns;
    const double sqh = sqrt(h);
    const int g_hi = wk.qhi ? *wk.qhi : wk.n_groups;
    for (;;) {
        int grp = 0;
        if (lane == 0) grp = atomicAdd(wk.queue, 1);
        grp = __shfl(grp, 0, 64);
        if (grp >= g_hi) break;
        const int64_t idx = (int64_t)grp * 64 + lane;
        const bool has = idx < wk.n_pos;
        const int64_t pos = has ? wk.pos[idx] : 0;
        const Setup su = sample_setup(p, pos);
        const int N = has ? su.N : 1;
        const int L = has ? su.L : -1;
        int cnt[C_NCNT];
#pragma unroll
        for (int c = 0; c < C_NCNT; ++c) cnt[c] = 0;
        double n[3] = {su.n0[0], su.n0[1], su.n0[2]};
        double xhat = su.xhat0, P = p.P0, Fprev = su.ubar, phiacc = 0.0;
        uint64_t hsh = 14695981039346656037ull;
        if (has)
            #pragma unroll 1
            for (int k = 0; k < N; ++k) a(M_U, k) = su.ubar * kMlMinPerLs;
        const int Lmax = wave_max_i(L);
        int Lrun = L;   // cut short when the plant state stops being finite
        for (int i = 0; i <= Lmax; ++i) {
            const bool live = has && i <= Lrun;
            const bool step = live && i < Lrun;
            if (!live) continue;
            const double z = n[2] / p.V;
            const double zb = setpoint(p, i, su.istep, su.sign);
            phiacc += (z - zb) * (z - zb);
            if (out.tz) out.tz[(int64_t)i * out.S + pos] = z;
            if (!isfinite(z)) {
                // the plant diverged (Phi is not a number): no more OCPs
                cnt[C_NONFIN] = 1;
                Lrun = i;
                continue;
            }
            if (!step) continue;
            const double y = z + p.noise_scale * sqrtR *
                                     normal_first(p.seed, 0, (uint32_t)i, su.nid, kTagMeas);
            ekf_predict(p, xhat, P, Fprev);
            ekf_update(p, xhat, P, y);
            if (!isfinite(P) || !isfinite(xhat)) cnt[C_NONFIN] = 1;
            if (out.tx) out.tx[(int64_t)i * out.S + pos] = xhat;
            const bool conv = ms_sqp<NMAX>(p, a, N, xhat, i, su.istep, su.sign, cnt);
            cnt[C_OCP]++;
            if (!conv) cnt[C_OCP_FAIL]++;
            uint64_t mask = 0;
            #pragma unroll 4
            for (int k = 0; k < N; ++k) {
                const double v = a(M_U, k);
                if (v <= p.umin + 1e-6 || v >= p.umax - 1e-6) mask |= (1ull << k);
            }
            hsh = fnv1a_step(hsh, (uint32_t)i, mask);
            const double F = a(M_U, 0) / kMlMinPerLs;
            #pragma unroll 4
            for (int k = 0; k + 1 < N; ++k) a(M_U, k) = a(M_U, k + 1);
            if (out.tu) out.tu[(int64_t)i * out.S + pos] = F;
            #pragma unroll 1
            for (int j = 0; j < p.Ns; ++j) {
                double xi[3];
                process_noise(p, (uint32_t)(i * p.Ns + j), su.nid, xi);
                em_step(p, su.k0, su.EaR, n, F, h, sqh, xi);
            }
            Fprev = F;
        }
        if (has) {
            if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) cnt[C_NONFIN] = 1;
            out.phi[pos] = phiacc / (double)(L + 1);
            out.hash[pos] = hsh;
            cnt[C_KIND] = 0;
            cnt[C_N] = N;
            cnt[C_L] = L;
            out.flops[pos] = ms_sample_flops(p, N, L, cnt);
#pragma unroll
            for (int c = 0; c < C_NCNT; ++c) out.cnt[(int64_t)c * out.S + pos] = cnt[c];
        }
    }
}

}  // namespace mccl
