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

typedef __attribute__((address_space(3))) double lds_double;

// Wave-uniform copies of values that arrive in VGPRs (function arguments).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double uni_d(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Wavefront reductions by DPP lane shuffles (VALU only, no LDS round
// trip): pairs, quads, 8-lane and 16-lane rows, then the row broadcasts
// 15 and 31 fold the four rows into lane 63, whose value is returned to
// every lane.  The order of the operations is fixed, so the result is
// deterministic and the same on all lanes.  `id` is the operation's
// identity (what a lane outside the selected rows contributes).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double old, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK,
                                               0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK,
                                               0xf, false);
    return __hiloint2double(hi, lo);
}
// v moved by a DPP control on every row and bank, lanes without a source
// reading 0 (bound_ctrl): no earlier value of the destination survives, so
// none has to be set up (quad permutations and row rotations have a source
// on every lane).
template <int CTRL>
__device__ __forceinline__ double dpp_z(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, double id, Op op) {
    v = op(v, dpp_z<0xB1>(v));    // quad_perm [1,0,3,2]
    v = op(v, dpp_z<0x4E>(v));    // quad_perm [2,3,0,1]
    v = op(v, dpp_z<0x124>(v));   // row_ror:4
    v = op(v, dpp_z<0x128>(v));   // row_ror:8
    v = op(v, dpp_d<0x142, 0xa>(id, v));   // row_bcast:15 into rows 1, 3
    v = op(v, dpp_d<0x143, 0xc>(id, v));   // row_bcast:31 into rows 2, 3
    return readlane_d(v, 63);
}
__device__ __forceinline__ double wave_sum(double v) {
    return wave_reduce(v, 0.0, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_max(double v) {
    return wave_reduce(v, -__builtin_inf(), [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double wave_min(double v) {
    return wave_reduce(v, __builtin_inf(), [](double a, double b) { return fmin(a, b); });
}

// Stage the sample's W (NMAX x NMAX doubles, 16-byte aligned) into LDS with
// direct global-to-LDS loads: 1 KB per instruction, no registers involved,
// all in flight together.  The matrices (32 KB per sample, a wavefront's
// next visit reads another sample's) are loaded and written back
// non-temporal, so that their stream does not evict the lane tiles, which a
// wavefront reads again in every SQP iteration, from the caches.  coop_stage_issue waits for this wave's earlier
// stores (to W among them) and issues the loads; coop_stage_wait waits for
// every load in flight (other loads issued in between complete with them).
template <int NMAX>
__device__ __forceinline__ void coop_stage_issue(const double* __restrict__ Wg, double* Wl, int lane) {
    static_assert((NMAX * NMAX) % 128 == 0, "W must fill whole 1 KB rows");
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): earlier stores to W have landed
#pragma unroll
    for (int q = 0; q < NMAX * NMAX / 128; ++q)
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1)))*)(Wg + q * 128 + 2 * lane),
            (void __attribute__((address_space(3)))*)(Wl + q * 128), 16, 0, 2 /* nt */);
}
__device__ __forceinline__ void coop_stage_wait() {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
}
template <int NMAX>
__device__ __forceinline__ void coop_stage(const double* __restrict__ Wg, double* Wl, int lane) {
    coop_stage_issue<NMAX>(Wg, Wl, lane);
    coop_stage_wait();
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
                __builtin_nontemporal_store(w, &Wg[j * NMAX + lane]);
            }
        }
    }
    __syncthreads();
    return 1;
}

// W <- I (equally H <- I) in global memory and (when Wl is given) in its
// staged LDS copy.  The whole NMAX x NMAX block is written: entries beyond
// the sample's N x N block are never read unmasked.
template <int NMAX>
__device__ __forceinline__ void coop_identity(double* Wl, double* __restrict__ Wg, int N, int lane) {
    (void)N;
    if (lane < NMAX) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
            const double v = (j == lane) ? 1.0 : 0.0;
            __builtin_nontemporal_store(v, &Wg[j * NMAX + lane]);
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
                __builtin_nontemporal_store(w, &Wg[j * NMAX + lane]);
            }
        }
    }
    __syncthreads();
}


// ---------------------------------------------------------------------------
// Inverse-Hessian form.  The sample keeps H = W^-1 (same layout as W, in
// global memory, staged to LDS per visit) and diag(W).  With H the QP of a
// fixed active set A needs no factorisation of W: from W d + g - lam = 0
// (lam_i > 0 on a lower bound, < 0 on an upper bound, 0 on free inputs),
// d = -H g + H[:, A] lam_A and d_A on its bounds give
// H_AA lam_A = d_A + (H g)_A, an |A| x |A| system.  The BFGS update of W
// maps to the product form of the inverse update, and W d = lam - g from
// the QP supplies W s for the damping.  Mathematically the iterates are
// those of the W form; the work per SQP iteration is O(N^2 + |A|^3).

// Rows of the sample's NMAX x NMAX block that a loop visits: N rounded up
// to a multiple of 8.  Outside its N x N block the block holds the
// identity (written whole at every reset; updates and shifts touch only
// the N x N block), so for lanes < N the extra rows are zero, and the
// vectors broadcast across them are zero on lanes >= N.
template <int NMAX>
__device__ __forceinline__ int rows8(int N) {
    const int r = (N + 7) & ~7;
    return r < NMAX ? r : NMAX;
}

// The staging buffer is followed by two vectors of NMAX doubles, through
// which a value of every lane is broadcast to all lanes: each lane writes
// its element, and a read of one address by every lane returns it to all
// (an LDS broadcast, one instruction for two doubles, against four
// v_readlane per two doubles).
template <int NMAX>
__device__ __forceinline__ double* lds_vec(double* Hl, int k) {
    return Hl + NMAX * NMAX + k * NMAX;
}
template <int NMAX>
__device__ __forceinline__ const double* lds_vec(const double* Hl, int k) {
    return Hl + NMAX * NMAX + k * NMAX;
}

// (H x)_i on lane i < N from the staged H (lane i reads its column, H
// symmetric); x_j, broadcast from lane j through the first LDS vector, must
// be 0 on lanes >= N; the result is 0 on lanes >= N.  Eight rows per step,
// four partial sums.
template <int NMAX>
__device__ __forceinline__ double coop_matvec(const double* Hl, int N, int lane, double x) {
    const int lc = lane < NMAX ? lane : NMAX - 1;
    const int R = rows8<NMAX>(N);
    double* const xl = lds_vec<NMAX>((double*)Hl, 0);
    __syncthreads();   // earlier readers of the vector are done
    if (lane < NMAX) xl[lane] = x;
    __syncthreads();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    #pragma unroll 2
    for (int j = 0; j < R; j += 8) {
        double h[8], xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) h[q] = Hl[(j + q) * NMAX + lc];
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[q] = xl[j + q];
        a0 = fma(h[0], xv[0], a0);
        a1 = fma(h[1], xv[1], a1);
        a2 = fma(h[2], xv[2], a2);
        a3 = fma(h[3], xv[3], a3);
        a0 = fma(h[4], xv[4], a0);
        a1 = fma(h[5], xv[5], a1);
        a2 = fma(h[6], xv[6], a2);
        a3 = fma(h[7], xv[7], a3);
    }
    const double acc = (a0 + a1) + (a2 + a3);
    return lane < N ? acc : 0.0;
}

// Damped BFGS of the SQP section in inverse form.  Lane i < N passes s_i,
// y_i, v_i = (W s)_i and diag(W)_ii (updated in place).  theta rule 0.2 /
// 0.8, r = theta y + (1 - theta) W s, skipped when min(s'Ws, s'r) <= eps_m;
// otherwise, with rho = 1 / s'r,
//   H+ = (I - rho s r') H (I - rho r s') + rho s s'
//      = H - rho (s (Hr)' + (Hr) s') + (rho^2 r'Hr + rho) s s',
// the exact inverse of W - Ws (Ws)'/s'Ws + r r'/s'r, and
//   diag(W+)_ii = W_ii - v_i^2 / s'Ws + r_i^2 / s'r.
// The staged copy Hl and the global H are both updated.  Returns 1 if
// updated; fl receives the FP64 work.
template <int NMAX>
__device__ __forceinline__ int coop_bfgs_h(double* Hl, double* __restrict__ Hg, int N, int lane,
                                           double s, double y, double v, double& wd, double& fl) {
    const bool act = lane < N;
    if (!act) { s = 0.0; y = 0.0; v = 0.0; }
    const double n = N;
    const double sWs = wave_sum(s * v);
    const double sy = wave_sum(s * y);
    const double theta = (sy >= 0.2 * sWs) ? 1.0 : 0.8 * sWs / (sWs - sy);
    const double r = act ? theta * y + (1.0 - theta) * v : 0.0;
    const double sr = wave_sum(s * r);
    const double kappa = sWs < sr ? sWs : sr;
    fl += 9.0 * n;
    if (!(kappa > DBL_EPSILON)) return 0;
    const double Hr = coop_matvec<NMAX>(Hl, N, lane, r);
    const double rHr = wave_sum(r * Hr);
    const double rho = 1.0 / sr;
    const double c = rho * rho * rHr + rho;
    const double a1 = c * s - rho * Hr;   // multiplies s_j
    const double a2 = -rho * s;           // multiplies (Hr)_j
    __syncthreads();   // every lane has read H and the broadcast vector for Hr
    double* const sl = lds_vec<NMAX>(Hl, 0);
    double* const hrl = lds_vec<NMAX>(Hl, 1);
    if (lane < NMAX) {
        sl[lane] = s;
        hrl[lane] = Hr;
    }
    __syncthreads();
    if (act) {
        // rows N..R-1 see s_j = (Hr)_j = 0 and are written back unchanged
        const int R = rows8<NMAX>(N);
        #pragma unroll 1
        for (int j = 0; j < R; j += 8) {
            double t[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) t[q] = Hl[(j + q) * NMAX + lane];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                t[q] = fma(a2, hrl[j + q], fma(a1, sl[j + q], t[q]));
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                Hl[(j + q) * NMAX + lane] = t[q];
                __builtin_nontemporal_store(t[q], &Hg[(j + q) * NMAX + lane]);
            }
        }
    }
    if (act) wd = (wd - v * v / sWs) + r * r / sr;
    __syncthreads();
    fl += 6.0 * n * n + 14.0 * n;
    return 1;
}

// H_AA x = b_A for the active set `amask` (m = |A| <= MM bits), with the
// system compressed onto lanes 0..m-1: lane k holds row k of H_AA, gathered
// from the staged H.  Lane i in A passes b_i and receives x for its
// variable in `lam`; xc (lane k) is the compressed solution.  Returns
// false on a non-positive pivot.
template <int NMAX, int MM>
__device__ __forceinline__ bool coop_active_solve(const double* Hl, uint64_t amask, int m, int lane,
                                                  double b, double& lam, double& xc) {
    int myvar = 0;
    {
        uint64_t mm = amask;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const int a = mm ? __ffsll((unsigned long long)mm) - 1 : 0;
            mm &= mm - 1;
            myvar = (lane == k) ? a : myvar;
        }
    }
    const bool row = lane < m;
    double Lx[MM];
    {
        uint64_t mm = amask;
#pragma unroll
        for (int jj = 0; jj < MM; ++jj) {
            const int a = mm ? __ffsll((unsigned long long)mm) - 1 : 0;
            mm &= mm - 1;
            const double h = Hl[a * NMAX + myvar];
            Lx[jj] = (row && jj < m) ? h : ((jj == lane) ? 1.0 : 0.0);
        }
    }
    const double bk = __shfl(b, myvar, 64);
    double myinv;
    const bool ok = coop_cholesky<MM>(Lx, lane, myinv);
    xc = coop_solve<MM>(Lx, lane, myinv, row ? bk : 0.0);
    const int rank = __popcll(amask & ((1ull << lane) - 1ull));
    const double xl = __shfl(xc, rank < 64 ? rank : 0, 64);
    lam = ((amask >> lane) & 1ull) ? xl : 0.0;
    return ok;
}

struct SolveOut {
    double lam, xc;
    int ok;
};

// The same as a separate function (not inlined): the factor's registers and
// the unrolled code stay out of the QP loop, whose register allocation
// would otherwise hoist the identity padding out of the loop and spill it.
template <int NMAX, int MM>
__device__ __noinline__ SolveOut coop_active_solve_far(lds_double* Hl3, uint64_t amask, int m,
                                                       double b) {
    SolveOut o{0.0, 0.0, 0};
    o.ok = coop_active_solve<NMAX, MM>((const double*)Hl3, uni_u64(amask), uni(m), (int)threadIdx.x,
                                       b, o.lam, o.xc);
    return o;
}

// Box QP  min 1/2 d'Wd + g'd,  umin - u <= d <= umax - u  by the
// primal-dual active-set iteration in inverse form.  The set prediction
// uses lam + W_ii (bound - d), the rule of the Jacobi-scaled variables of
// coop_box_qp_as written back in the original ones.  Lane i < N passes
// g_i, u_i, the multiplier estimate lam0_i = pi_l,i - pi_u,i and W_ii;
// it receives d_i, nu_l,i, nu_u,i and (W d)_i = lam_i - g_i.  After
// max_iter full set updates without settling, each further iteration
// changes only the lowest-index variable whose predicted status differs
// (least-index principal pivoting, finite for a positive definite H), for
// at most flip_iter iterations: on QPs of c1 closed loops this settled
// every set the full updates left cycling within 5-10 iterations on
// average, where the interior-point fallback costs an inversion of H and
// about a dozen factorisations.  Status 2: sets still changing after both
// phases; -1: H_AA not positive definite.
template <int NMAX>
__device__ __forceinline__ QPResult coop_box_qp_h(const double* Hl, lds_double* Hl3, int N, int lane, double wd, double g, double u,
                                                  double lam0, double umin, double umax,
                                                  int max_iter, double& d_out, double& nl_out,
                                                  double& nu_out, double& Wd_out, double& fl,
                                                  int flip_iter = 64) {
    const bool act = lane < N;
    const int lc = lane < NMAX ? lane : NMAX - 1;
    const double n = N;
    QPResult res{0, 0};
    const double lo = act ? umin - u : -1.0;
    const double hi = act ? umax - u : 1.0;
    const double hg = coop_matvec<NMAX>(Hl, N, lane, act ? g : 0.0);
    fl += 2.0 * n * n;
    double d = 0.0, lam = act ? lam0 : 0.0;
    int prev = -1, st = 0;
    for (int it = 0;; ++it) {
        st = 0;
        if (act) {
            if (lam + wd * (lo - d) > 0.0) st = 1;
            else if (lam + wd * (hi - d) < 0.0) st = 2;
        }
        if (it > 0 && !__ballot(st != prev)) {
            res.iters = it;
            break;
        }
        if (it == max_iter + flip_iter) {
            res.status = 2;
            res.iters = it;
            break;
        }
        if (it >= max_iter) {
            // single flip: only the lowest-index change is taken
            const uint64_t diff = __ballot(st != prev);
            const int f = __ffsll((unsigned long long)diff) - 1;
            st = lane == f ? st : prev;
        }
        prev = st;
        const uint64_t amask = __ballot(st != 0);
        const int m = __popcll(amask);
        const double dA = st == 1 ? lo : (st == 2 ? hi : 0.0);
        double acc = -hg;
        lam = 0.0;
        if (m > 0) {
            const double b = dA + hg;
            double xc = 0.0;
            bool ok;
            SolveOut so{0.0, 0.0, 0};
            if (m <= 8) {
                so = coop_active_solve_far<NMAX, 8>(Hl3, amask, m, b);
            } else if (m <= 16 || NMAX <= 16) {
                so = coop_active_solve_far<NMAX, 16>(Hl3, amask, m, b);
            } else if constexpr (NMAX > 16) {
                if constexpr (NMAX > 32) {
                    so = m > 32 ? coop_active_solve_far<NMAX, 64>(Hl3, amask, m, b)
                                : coop_active_solve_far<NMAX, 32>(Hl3, amask, m, b);
                } else {
                    so = coop_active_solve_far<NMAX, 32>(Hl3, amask, m, b);
                }
            }
            ok = so.ok;
            lam = so.lam;
            xc = so.xc;
            if (!ok) {
                res.status = -1;
                res.iters = it + 1;
                return res;
            }
            // d_I = -(H g)_I + H_IA lam_A, lam_A broadcast from the
            // compressed solution through the first LDS vector
            double* const xl = lds_vec<NMAX>((double*)Hl, 0);
            __syncthreads();
            if (lane < NMAX) xl[lane] = xc;
            __syncthreads();
            uint64_t mm = amask;
            #pragma unroll 1
            for (int k = 0; k < m; ++k) {
                const int a = __ffsll((unsigned long long)mm) - 1;
                mm &= mm - 1;
                acc = fma(Hl[a * NMAX + lc], xl[k], acc);
            }
            const double mf = m;
            fl += mf * mf * mf / 3.0 + 2.0 * mf * mf + 2.0 * n * mf;
        }
        fl += 6.0 * n;
        d = act ? (st ? dA : acc) : 0.0;
    }
    d_out = st == 1 ? lo : (st == 2 ? hi : d);
    nl_out = lam > 0.0 ? lam : 0.0;
    nu_out = lam < 0.0 ? -lam : 0.0;
    Wd_out = act ? lam - g : 0.0;
    return res;
}

// W = H^-1 into Wl (the staged buffer, overwriting H): Cholesky of H, then
// one solve per column.  For the rare QPs the active-set iteration leaves
// unsettled, which go to the interior-point method on W.  Returns false if
// H is not positive definite.
template <int NMAX>
__device__ __forceinline__ bool coop_invert(double* Hl, int N, int lane, double& fl) {
    const int lc = lane < NMAX ? lane : NMAX - 1;
    double Lx[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        const double h = Hl[j * NMAX + lc];
        Lx[j] = lane < N ? ((j < N) ? h : 0.0) : ((j == lane) ? 1.0 : 0.0);
    }
    __syncthreads();
    double myinv;
    if (!coop_cholesky<NMAX>(Lx, lane, myinv)) return false;
    #pragma unroll 1
    for (int j = 0; j < N; ++j) {
        const double x = coop_solve<NMAX>(Lx, lane, myinv, lane == j ? 1.0 : 0.0);
        if (lane < N) Hl[j * NMAX + lane] = x;
    }
    __syncthreads();
    const double n = N;
    fl += n * n * n / 3.0 + 2.0 * n * n * n;
    return true;
}

// Shift of H for the next OCP.  The W form drops u_0's row and column and
// repeats the last diagonal entry uncoupled; in inverse form the leading
// block becomes the inverse of W[1:, 1:], i.e. the Schur complement
// H[1:, 1:] - H[1:, 0] H[0, 1:] / H_00, and the last diagonal entry
// 1 / W_{N-1,N-1}.  From the staged copy Hl into global Hg.
template <int NMAX>
__device__ __forceinline__ void coop_shift_h(const double* Hl, double* __restrict__ Hg, int N,
                                             int lane, double wlast, double& fl) {
    const double inv_e = 1.0 / Hl[0];
    const int li = lane + 1 < NMAX ? lane + 1 : NMAX - 1;
    const double fi = (lane + 1 < N) ? Hl[li] : 0.0;   // H_0,i+1
    const double hlast = 1.0 / wlast;
    if (lane < N) {
        #pragma unroll 4
        for (int j = 0; j < N; ++j) {
            const int jr = j + 1 < NMAX ? j + 1 : NMAX - 1;
            const double p = readlane_d(fi, j) * fi;
            double w = Hl[jr * NMAX + li] - p * inv_e;
            if (!(lane < N - 1 && j < N - 1)) w = (lane == N - 1 && j == N - 1) ? hlast : 0.0;
            __builtin_nontemporal_store(w, &Hg[j * NMAX + lane]);
        }
    }
    __syncthreads();
    const double n = N;
    fl += 3.0 * n * n;
}

}  // namespace mccl
