// mc_coop.hpp -- wavefront-cooperative dense algebra of the SQP for gfx950:
// the box-constrained QP subproblem (primal-dual interior point with a
// Cholesky-factored Newton matrix) and the damped BFGS update, one sample at
// a time on all 64 lanes.
//
// Layout: lane i owns variable i.  The sample's W lives in global memory,
// element (j, i) at W[j * NMAX + i], and is staged whole into LDS (Wl, same
// layout) at the start of each cooperative visit by direct global-to-LDS
// loads; W is symmetric, so lane i reading "column i" reads its own row and
// the LDS reads are bank-conflict free.  The
// Newton matrix is held in registers as each lane's full symmetric row
// Lx[0..NMAX); after the factorisation lane i holds row i of L (j < i), L_ii
// (j = i) and column i of L (j > i), so both triangular solves are
// column-oriented with the pivot value broadcast by readlane.  Lanes >= N pad
// the matrix with an identity block.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

namespace mccl {

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Stage the sample's W (NMAX x NMAX doubles, 16-byte aligned) into LDS with
// direct global-to-LDS loads: 1 KB per instruction, no registers involved,
// all in flight together, one wait.
template <int NMAX>
__device__ __forceinline__ void coop_stage(const double* __restrict__ Wg, double* Wl, int lane) {
    static_assert((NMAX * NMAX) % 128 == 0, "W must fill whole 1 KB rows");
    __builtin_amdgcn_s_waitcnt(0x0F70);   // earlier stores to W have landed
#pragma unroll
    for (int q = 0; q < NMAX * NMAX / 128; ++q)
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1)))*)(Wg + q * 128 + 2 * lane),
            (void __attribute__((address_space(3)))*)(Wl + q * 128), 16, 0, 0);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
}

// 1/sqrt(a) and sqrt(a) from the hardware reciprocal square root refined by
// two Newton steps (quadratic convergence to full FP64 precision).
__device__ __forceinline__ void rsqrt_newton(double a, double& inv, double& root) {
    double y = __builtin_amdgcn_rsq(a);
    y = y * (1.5 - 0.5 * a * y * y);
    y = y * (1.5 - 0.5 * a * y * y);
    inv = y;
    root = a * y;
}

// In-register right-looking Cholesky of the symmetric matrix whose row
// `lane` is Lx.  Column k is broadcast with readlane (no LDS round trip);
// column k+1 is updated first so the next pivot and its inverse square
// root are ready while the rest of the rank-1 update proceeds.  Returns
// false on a non-positive pivot (the sweep then finishes on unit pivots,
// branch-free, and the caller discards the factor).
template <int NMAX>
__device__ __forceinline__ bool coop_cholesky(double (&Lx)[NMAX], int lane, double& myinv) {
    myinv = 1.0;
    bool ok = true;
    double piv = readlane_d(Lx[0], 0);
    ok = ok && (piv > 0.0);
    piv = (piv > 0.0) ? piv : 1.0;
    double inv, rl;
    rsqrt_newton(piv, inv, rl);
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        const double lik = (lane > k) ? Lx[k] * inv : 0.0;
        myinv = (lane == k) ? inv : myinv;
        Lx[k] = (lane > k) ? lik : ((lane == k) ? rl : Lx[k]);
        double ninv = 1.0, nrl = 1.0;
        if (k + 1 < NMAX) {
            Lx[k + 1] = fma(-lik, readlane_d(lik, k + 1), Lx[k + 1]);
            double pn = readlane_d(Lx[k + 1], k + 1);
            ok = ok && (pn > 0.0);
            pn = (pn > 0.0) ? pn : 1.0;
            rsqrt_newton(pn, ninv, nrl);
        }
#pragma unroll
        for (int j = k + 2; j < NMAX; ++j) Lx[j] = fma(-lik, readlane_d(lik, j), Lx[j]);
        inv = ninv;
        rl = nrl;
    }
    // lane i's column part (j > i) still holds L[j][i] * L_ii: scale it
#pragma unroll
    for (int j = 0; j < NMAX; ++j) Lx[j] = (j > lane) ? Lx[j] * myinv : Lx[j];
    return ok;
}

// Solve L L^T x = r; lane i holds r_i on entry and x_i on return.
template <int NMAX>
__device__ __forceinline__ double coop_solve(const double (&Lx)[NMAX], int lane, double myinv,
                                             double r) {
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        const double yk = readlane_d(r * myinv, k);
        r = (lane == k) ? yk : ((lane > k) ? fma(-Lx[k], yk, r) : r);
    }
#pragma unroll
    for (int k = NMAX - 1; k >= 0; --k) {
        const double xk = readlane_d(r * myinv, k);
        r = (lane == k) ? xk : ((lane < k) ? fma(-Lx[k], xk, r) : r);
    }
    return r;
}

__device__ __forceinline__ double step_ratio(double v, double dv) {
    return dv < 0.0 ? -v / dv : 1.0;
}

struct QPResult {
    int status;   // 0 converged, 1 iteration cap, 2 active set unsettled, -1 not pos. definite
    int iters;
};

// Jacobi scaling of the staged W in place: Wt = D W D, D = diag(W)^-1/2, so
// Wt has a unit diagonal.  Returns false (wave-uniform) if a diagonal entry
// of W is not positive.  Lane i < N receives D_ii in Dg (1 elsewhere).  The
// product W_ij (D_i D_j) is symmetric in (i, j), so Wt stays exactly
// symmetric.
template <int NMAX>
__device__ __forceinline__ bool coop_scale(double* Wl, int N, int lane, double& Dg) {
    const bool act = lane < N;
    const int lc = lane < NMAX ? lane : NMAX - 1;
    double wii = Wl[lc * NMAX + lc];
    if (!act) wii = 1.0;
    if (__ballot(!(wii > 0.0))) return false;
    Dg = act ? 1.0 / sqrt(wii) : 1.0;
    double col[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) col[j] = Wl[j * NMAX + lc];
    __syncthreads();
    if (act) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (j < N) Wl[j * NMAX + lane] = col[j] * (Dg * readlane_d(Dg, j));
    }
    __syncthreads();
    return true;
}

// Box QP  min 1/2 d'Wd + g'd,  umin - u <= d <= umax - u  (the QP subproblem
// of the SQP section with bounds only), solved in the Jacobi-scaled variables
// d = D dt of coop_scale (Wt in LDS) by the Mehrotra predictor-corrector
// primal-dual interior-point method with separate primal and dual step
// lengths.  Lane i < N passes g_i, u_i, D_ii and receives d_i, nu_l,i, nu_u,i.
template <int NMAX>
__device__ __forceinline__ QPResult coop_box_qp(const double* Wt, int N, int lane, double Dg,
                                                double g, double u, double umin, double umax,
                                                int max_iter, double& d_out, double& nl_out,
                                                double& nu_out) {
    const bool act = lane < N;
    const int lc = lane < NMAX ? lane : NMAX - 1;
    QPResult res{0, 0};
    const double gs = act ? Dg * g : 0.0;
    const double lo = act ? (umin - u) / Dg : -1.0;
    const double hi = act ? (umax - u) / Dg : 1.0;
    double d = 0.0;
    {
        const double delta = 1e-2 * (hi - lo);
        if (d < lo + delta) d = lo + delta;
        if (d > hi - delta) d = hi - delta;
    }
    double sl = d - lo, su = hi - d;
    double nl = act ? 1.0 : 0.0, nu = act ? 1.0 : 0.0;
    if (!act) { d = 0.0; sl = 1.0; su = 1.0; }
    const double gnorm = wave_max(fabs(gs));
    const double bnorm = wave_max(act ? fmax(fabs(lo), fabs(hi)) : 0.0);
    const double inv2N = 1.0 / (2.0 * N);
    double Lx[NMAX];
    for (int it = 0;; ++it) {
        const double diag = act ? nl / sl + nu / su : 1.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) Lx[j] = Wt[j * NMAX + lc];
        double Wd = 0.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const double wt = (j < N && act) ? Lx[j] : 0.0;
            Wd = fma(wt, readlane_d(d, j), Wd);
            Lx[j] = (j == lane) ? wt + diag : wt;
        }
        const double rS = act ? Wd + gs - nl + nu : 0.0;
        const double rL = act ? d - sl - lo : 0.0;
        const double rU = act ? hi - d - su : 0.0;
        const double mu = wave_sum(act ? sl * nl + su * nu : 0.0) * inv2N;
        const double rSn = wave_max(fabs(rS));
        const double Wdn = wave_max(fabs(Wd));
        const double rPn = wave_max(fmax(fabs(rL), fabs(rU)));
        if (rSn <= 1e-12 * (1.0 + gnorm + Wdn) && rPn <= 1e-12 * (1.0 + bnorm) &&
            mu <= 1e-14 * (1.0 + gnorm)) {
            res.status = 0;
            res.iters = it;
            break;
        }
        if (it == max_iter) {
            res.status = 1;
            res.iters = it;
            break;
        }
        double myinv;
        if (!coop_cholesky<NMAX>(Lx, lane, myinv)) {
            res.status = -1;
            res.iters = it;
            return res;
        }
        // predictor
        double rhs = act ? -(Wd + gs) - nl * rL / sl + nu * rU / su : 0.0;
        const double dda = coop_solve<NMAX>(Lx, lane, myinv, rhs);
        const double dsla = dda + rL, dsua = -dda + rU;
        const double dnla = act ? -nl - nl / sl * dsla : 0.0;
        const double dnua = act ? -nu - nu / su * dsua : 0.0;
        const double apa = act ? fmin(fmin(step_ratio(sl, dsla), step_ratio(su, dsua)), 1.0) : 1.0;
        const double ada = act ? fmin(fmin(step_ratio(nl, dnla), step_ratio(nu, dnua)), 1.0) : 1.0;
        const double ap_aff = wave_min(apa), ad_aff = wave_min(ada);
        const double mu_a = wave_sum(act ? (sl + ap_aff * dsla) * (nl + ad_aff * dnla) +
                                               (su + ap_aff * dsua) * (nu + ad_aff * dnua)
                                         : 0.0) * inv2N;
        const double ratio = mu_a / mu;
        const double sigma = ratio * ratio * ratio;
        // corrector
        const double cl = dsla * dnla, cu = dsua * dnua;
        rhs = act ? -(Wd + gs) + (sigma * mu - cl - nl * rL) / sl - (sigma * mu - cu - nu * rU) / su
                  : 0.0;
        const double dd = coop_solve<NMAX>(Lx, lane, myinv, rhs);
        const double dsl = dd + rL, dsu = -dd + rU;
        const double dnl = act ? (sigma * mu - cl - nl * dsl) / sl - nl : 0.0;
        const double dnu = act ? (sigma * mu - cu - nu * dsu) / su - nu : 0.0;
        const double apc = act ? fmin(fmin(step_ratio(sl, dsl), step_ratio(su, dsu)), 1.0) : 1.0;
        const double adc = act ? fmin(fmin(step_ratio(nl, dnl), step_ratio(nu, dnu)), 1.0) : 1.0;
        double ap = 0.995 * wave_min(apc), ad = 0.995 * wave_min(adc);
        if (ap > 1.0) ap = 1.0;
        if (ad > 1.0) ad = 1.0;
        if (act) {
            d += ap * dd;
            sl += ap * dsl;
            su += ap * dsu;
            nl += ad * dnl;
            nu += ad * dnu;
        }
    }
    d_out = Dg * d;
    nl_out = nl / Dg;
    nu_out = nu / Dg;
    return res;
}

// Box QP by the primal-dual active-set method (a semismooth Newton method,
// Hintermueller, Ito and Kunisch, SIAM J. Optim. 13, 2003) in the same
// scaled variables.  From (d, lam) the predicted sets are
// A_lo = {lam + (lo - d) > 0}, A_hi = {lam + (hi - d) < 0} and the free rest
// I; the next iterate puts d_A on its bounds, solves
// W_II d_I = -(g + W_IA d_A)_I and sets lam_I = 0, lam_A = (W d + g)_A.  When
// the sets repeat the iterate meets the KKT conditions exactly (to
// rounding).  Warm start: d = 0 and lam = the SQP's current bound multiplier
// estimate pi_l - pi_u, so an unchanged active set costs one factorisation.
// status 2 = sets still changing after max_iter factorisations (the caller
// falls back to the interior-point method).
template <int NMAX>
__device__ __forceinline__ QPResult coop_box_qp_as(const double* Wt, int N, int lane, double Dg,
                                                   double g, double u, double lam0, double umin,
                                                   double umax, int max_iter, double& d_out,
                                                   double& nl_out, double& nu_out) {
    const bool act = lane < N;
    const int lc = lane < NMAX ? lane : NMAX - 1;
    QPResult res{0, 0};
    const double gs = act ? Dg * g : 0.0;
    const double lo = act ? (umin - u) / Dg : -1.0;
    const double hi = act ? (umax - u) / Dg : 1.0;
    double d = 0.0, lam = act ? Dg * lam0 : 0.0;
    int prev = -1, st = 0;
    for (int it = 0;; ++it) {
        st = 0;
        if (act) {
            if (lam + (lo - d) > 0.0) st = 1;
            else if (lam + (hi - d) < 0.0) st = 2;
        }
        if (it > 0 && !__ballot(st != prev)) {
            res.status = 0;
            res.iters = it;
            break;
        }
        if (it == max_iter) {
            res.status = 2;
            res.iters = it;
            break;
        }
        prev = st;
        const bool fr = act && st == 0;
        const uint64_t fmask = __ballot(fr);
        const double dA = st == 1 ? lo : (st == 2 ? hi : 0.0);
        double Lx[NMAX];
#pragma unroll
        for (int j = 0; j < NMAX; ++j) Lx[j] = Wt[j * NMAX + lc];
        double wa = 0.0;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const bool jfree = (fmask >> j) & 1ull;
            const double wt = (j < N && act) ? Lx[j] : 0.0;
            wa = jfree ? wa : fma(wt, readlane_d(dA, j), wa);
            Lx[j] = (j == lane) ? (fr ? wt : 1.0) : ((fr && jfree) ? wt : 0.0);
        }
        const double rhs = fr ? -(gs + wa) : dA;
        double myinv;
        if (!coop_cholesky<NMAX>(Lx, lane, myinv)) {
            res.status = -1;
            res.iters = it + 1;
            return res;
        }
        d = coop_solve<NMAX>(Lx, lane, myinv, rhs);
        if (!fr) d = dA;
        // multipliers of the active bounds: lam_A = (Wt d + g)_A
        const uint64_t amask = __ballot(act && !fr);
        if (amask) {
#pragma unroll
            for (int j = 0; j < NMAX; ++j) Lx[j] = Wt[j * NMAX + lc];
            double Wd = 0.0;
#pragma unroll
            for (int j = 0; j < NMAX; ++j)
                Wd = fma((j < N && act) ? Lx[j] : 0.0, readlane_d(d, j), Wd);
            lam = (act && !fr) ? Wd + gs : 0.0;
        } else {
            lam = 0.0;
        }
    }
    // active inputs land exactly on their bounds
    d_out = st == 1 ? umin - u : (st == 2 ? umax - u : Dg * d);
    nl_out = lam > 0.0 ? lam / Dg : 0.0;
    nu_out = lam < 0.0 ? -lam / Dg : 0.0;
    return res;
}

// Damped BFGS (SQP section, "Block BFGS update") on the sample's dense W:
// theta rule 0.2 / 0.8, r = theta y + (1 - theta) W s, skipped when
// min(s'Ws, s'r) <= machine epsilon.  Lane i < N passes s_i, y_i.  Wl is the
// staged LDS copy (updated in place), Wg the global W (updated columns are
// written back).  lds: 3 x 64 doubles.  Returns 1 if W was updated.
template <int NMAX>
__device__ __forceinline__ int coop_bfgs(double* Wl, double* __restrict__ Wg, int N, int lane,
                                         double s, double y) {
    const bool act = lane < N;
    const int lc = lane < NMAX ? lane : NMAX - 1;
    if (!act) { s = 0.0; y = 0.0; }
    double col[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) col[j] = Wl[j * NMAX + lc];
    double Ws = 0.0;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) Ws = fma((j < N && act) ? col[j] : 0.0, readlane_d(s, j), Ws);
    const double sWs = wave_sum(act ? s * Ws : 0.0);
    const double sy = wave_sum(act ? s * y : 0.0);
    const double theta = (sy >= 0.2 * sWs) ? 1.0 : 0.8 * sWs / (sWs - sy);
    const double r = theta * y + (1.0 - theta) * Ws;
    const double sr = wave_sum(act ? s * r : 0.0);
    const double kappa = sWs < sr ? sWs : sr;
    if (!(kappa > DBL_EPSILON)) return 0;
    const double Wsa = act ? Ws : 0.0, ra = act ? r : 0.0;
    if (act) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            if (j < N) {
                const double t1 = readlane_d(Wsa, j) * Ws;
                const double t2 = readlane_d(ra, j) * r;
                const double w = (col[j] - t1 / sWs) + t2 / sr;
                Wl[j * NMAX + lane] = w;
                Wg[j * NMAX + lane] = w;
            }
        }
    }
    __syncthreads();
    return 1;
}

// W <- I on the sample's N x N block, in global memory and (when Wl is
// given) in its staged LDS copy.
template <int NMAX>
__device__ __forceinline__ void coop_identity(double* Wl, double* __restrict__ Wg, int N, int lane) {
    if (lane < N) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (j < N) {
                const double v = (j == lane) ? 1.0 : 0.0;
                Wg[j * NMAX + lane] = v;
                if (Wl) Wl[j * NMAX + lane] = v;
            }
    }
    __syncthreads();
}

// Shift for the next OCP, from the staged copy Wl into global Wg:
// W'[i][j] = W[i+1][j+1] (i, j < N-1), last row and column zero except
// W'[N-1][N-1] = W[N-1][N-1].
template <int NMAX>
__device__ __forceinline__ void coop_shift(const double* Wl, double* __restrict__ Wg, int N,
                                           int lane) {
    const double last = Wl[(N - 1) * NMAX + (N - 1)];
    if (lane < N) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            if (j < N) {
                double w = 0.0;
                if (lane < N - 1 && j < N - 1) w = Wl[(j + 1) * NMAX + (lane + 1)];
                if (lane == N - 1 && j == N - 1) w = last;
                Wg[j * NMAX + lane] = w;
            }
        }
    }
    __syncthreads();
}

}  // namespace mccl
