// mc_kernels.hpp -- closed-loop kernels of the Monte Carlo CSTR campaign
// (arXiv 2212.02197) for gfx950.
//
//  * pi_kernel: one sample per group of K lanes (K = 1, 2 or 4), the whole
//    closed loop in registers.
//  * nmpc_kernel: persistent; each 64-lane wavefront pulls groups of `spw`
//    samples from a device work queue and runs their closed loops.  Scalar
//    serial work (plant, estimator, RK4 shooting, gradient, line search, KKT
//    test) runs one sample per lane; the dense QP and BFGS steps of the
//    samples still iterating run on the whole wavefront, one sample at a
//    time (ballot over the active lanes).
//  * pi_reverse_kernel: reverse pass of the PI closed loop from plant-state
//    checkpoints for dPhi/d(Kc, tau_i).
//  * stats kernels: deterministic fixed-order reductions of Phi.
#pragma once
#include "mc_coop.hpp"
#include "mc_dev.hpp"

// Wavefronts per SIMD the NMPC kernel is built for.  At NMAX = 64 the
// kernel needs its 512 registers per lane whatever is asked (one wave per
// SIMD), but asking for two makes the register allocator spill about 100
// registers instead of about 600 (c1: 5.71 s against 6.09 s per campaign).
// At NMAX 16 and 32 the request does give two waves per SIMD, with more
// spills, and that is slower (c4: 11.98 s against 10.09 s): one.
#ifndef MC_NMPC_WAVES_PER_EU_64
#define MC_NMPC_WAVES_PER_EU_64 2
#endif
#ifndef MC_NMPC_WAVES_PER_EU
#define MC_NMPC_WAVES_PER_EU 1
#endif

namespace mccl {

// Counter rows (match MC_CL_CNT_* of the C-ABI header).
enum : int {
    C_KIND = 0, C_N, C_L, C_OCP, C_OCP_FAIL, C_SQP, C_IPM, C_LS, C_LSCAP, C_SKIP, C_RESET,
    C_IPMCAP, C_NONFIN, C_GRAD, C_AS, C_NCNT
};

struct Outs {
    double* phi;       // [S]
    double* flops;     // [S] algorithmic FP64 work of the sample
    int32_t* cnt;      // [C_NCNT][S]
    uint64_t* hash;    // [S]
    double* tz;        // [L+1][S] or null
    double* tu;        // [L][S] or null
    double* tx;        // [L][S] or null
    int64_t S;
};

// Lane-tiled per-sample vectors of the SQP (element k of lane l's sample at
// base[v * NMAX * 64 + te(k) + l * kTB], the blocked layout of mc_dev.hpp).
// V_WD: diag(W) and V_V: W d, then W s after the line search (inverse form).
enum : int { V_U = 0, V_G, V_D, V_PIL, V_PIU, V_NL, V_NU, V_S, V_Y, V_WD, V_V, V_COUNT };

struct NmpcWork {
    const int64_t* pos;  // sample positions, grouped by spw
    int64_t n_pos;
    int spw;
    int n_groups;
    int* queue;          // next group; starts at the chunk's first group
    const int* qhi;      // end of the chunk's groups (device), or null: n_groups
    double* tiles;       // per slot: V_COUNT * NMAX * 64
    double* xs;          // per slot: 3 NMAX * 64 (interval derivatives of the shooting)
    double* W;           // per slot: spw * NMAX * NMAX
    int64_t tile_stride, xs_stride, w_stride;
};

__device__ __forceinline__ uint64_t fnv1a_step(uint64_t h, uint32_t i, uint64_t mask) {
#pragma unroll
    for (int j = 0; j < 4; ++j) { h ^= (uint64_t)((i >> (8 * j)) & 0xffu); h *= 1099511628211ull; }
#pragma unroll
    for (int j = 0; j < 8; ++j) { h ^= (mask >> (8 * j)) & 0xffull; h *= 1099511628211ull; }
    return h;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Algorithmic FP64 work of one sample from its counters (each +, -, *, /,
// sqrt, exp, log, sin, cos counts 1; an FMA counts 2; Philox is integer):
//   cost term 3, measurement 8, EM sub-step with its noise 52, PI law 10,
//   EKF interval 142 Nc + 12, shooting 73 N Nc + 9 N per trial,
//   adjoint gradient 78 N Nc + 9 N (the stage derivatives and interval
//   Jacobians, counted once per gradient although the shooting pass records
//   them at every trial, and the reverse sweep),
//   forward-sensitivity gradient 117 N Nc + 13 Nc N (N+1) + N (N+1) + 6 N,
//   interior-point iteration N^3/3 + 7 N^2 + 60 N,
//   active-set iteration N^3/3 + 6 N^2 + 10 N,
//   BFGS 2 N^2 + 9 N per attempt + 6 N^2 per applied update,
//   SQP bookkeeping 16 N per iteration.
// The inverse form (qp_solver 2) accumulates its QP, BFGS and shift work in
// `coop` as it runs (it depends on the active-set sizes): H g 2 N^2 per QP,
// per active-set solve m^3/3 + 2 m^2 + 2 N m + 6 N, BFGS 6 N^2 + 23 N per
// applied update (9 N if skipped), shift 3 N^2, inversion for the
// interior-point fallback 7 N^3 / 3; interior-point iterations as above.
// With the three-state model (nx = 3; model evaluation 21, its Jacobian 16
// more): EKF interval 490 Nc + 80, shooting 126 N Nc + 9 N per trial,
// adjoint gradient 520 N Nc + 28 N (the interval tangents carried through
// the RK4 stages and the reverse sweep with A_k^T).
__device__ __forceinline__ double sample_flops(const DevParams& p, int kind, int N, int L,
                                               const int (&c)[C_NCNT], int gmode, double coop,
                                               int nx) {
    const double Ns = p.Ns, Nc = p.Nc, n = N, l = L;
    double fl = 3.0 * (l + 1.0) + l * (8.0 + 52.0 * Ns);
    if (kind == 0 || p.run_ekf_for_pi) fl += l * (nx == 3 ? 490.0 * Nc + 80.0 : 142.0 * Nc + 12.0);
    if (kind == 1) return fl + 10.0 * l;
    const double shoot = nx == 3 ? 126.0 * n * Nc + 9.0 * n : 73.0 * n * Nc + 9.0 * n;
    const double grad = gmode == 1 ? (nx == 3 ? 520.0 * n * Nc + 28.0 * n : 78.0 * n * Nc + 9.0 * n)
                                   : 117.0 * n * Nc + 13.0 * Nc * n * (n + 1.0) + n * (n + 1.0) + 6.0 * n;
    const double ipm = n * n * n / 3.0 + 7.0 * n * n + 60.0 * n;
    const double asi = n * n * n / 3.0 + 6.0 * n * n + 10.0 * n;
    fl += (double)c[C_LS] * shoot + (double)c[C_GRAD] * grad + (double)c[C_IPM] * ipm;
    if (p.qp_solver == 2) return fl + coop + (double)c[C_SQP] * 16.0 * n;
    fl += (double)c[C_AS] * asi;
    fl += (double)c[C_SQP] * (2.0 * n * n + 9.0 * n + 16.0 * n) + (double)(c[C_SQP] - c[C_SKIP]) * 6.0 * n * n;
    return fl;
}

// ---------------------------------------------------------------------------
// Cooperative visits.  Each is a separate (not inlined) function so that its
// register allocation is its own: the closed loop's per-lane state stays
// out of the dense phase and the rarely taken paths stay out of the hot one.
// Arguments arrive in VGPRs; the wave-uniform ones are re-established as
// such with readfirstlane.  The staging buffer is passed as an LDS pointer.

// Counter deltas and FP64 work of one visit (wave-uniform).
struct VisitOut {
    double fl;
    int skip, reset, ipm, as, sqp, ipmcap;
    double gd;   // g'd of the QP step (the line search's directional derivative)
};

// H (or W) <- I in global memory and the staged copy: the rare reset after
// a non-positive pivot, out of line so that the identity's constants are
// not hoisted into the common path.
template <int NMAX>
__device__ __noinline__ void coop_reset(double* Ws, lds_double* Wl3) {
    coop_identity<NMAX>((double*)Wl3, Ws, NMAX, (int)threadIdx.x);
}

// Interior-point fallback of the inverse form on W = H^-1 (rare).
struct FallbackOut {
    double d, nl, nu, fl;
    int status, iters;
};
template <int NMAX>
__device__ __noinline__ FallbackOut coop_ipm_fallback(lds_double* Hl3, int N, double g, double u,
                                                      double umin, double umax, int max_iter) {
    double* Wl = (double*)Hl3;
    N = uni(N);
    const int lane = threadIdx.x;
    FallbackOut o{0.0, 0.0, 0.0, 0.0, -1, 0};
    double Dg = 1.0;
    if (coop_invert<NMAX>(Wl, N, lane, o.fl) && coop_scale<NMAX>(Wl, N, lane, Dg)) {
        const QPResult r = coop_box_qp<NMAX>(Wl, N, lane, Dg, g, u, uni_d(umin), uni_d(umax),
                                             uni(max_iter), o.d, o.nl, o.nu);
        o.status = r.status;
        o.iters = r.iters;
    }
    return o;
}

// Inverse-form visit of sample s: stage H, the pending BFGS update, then
// the QP if the sample is still iterating (flag 2), or the Hessian shift for
// the next OCP if its SQP has just ended (flag 4, with the update).  A QP
// whose active set has not settled goes to the interior-point method on
// W = H^-1; H_AA or W not positive definite resets H = I (and diag W = 1)
// once.
template <int NMAX>
__device__ __forceinline__ VisitOut coop_visit_h(double* TB, double* Ws, lds_double* Wl3, int Ns_, int s,
                                              int flags, double umin, double umax, int ipm_max_iter) {
    double* const Wl = (double*)Wl3;
    const int lane = threadIdx.x;
    Ns_ = uni(Ns_);
    s = uni(s);
    flags = uni(flags);
    umin = uni_d(umin);
    umax = uni_d(umax);
    VisitOut vo{0.0, 0, 0, 0, 0, 0, 0, 0.0};
    const bool in = lane < Ns_;
    double* const wdp = TB + V_WD * NMAX * 64 + te(lane) + s * kTB;
    // the sample's vectors (column s of the lane tiles) are loaded while H
    // is being staged
    coop_stage_issue<NMAX>(Ws, Wl, lane);
    const int lt = in ? lane : 0;
    const double* const tcol = TB + te(lt) + s * kTB;
    double wd = tcol[V_WD * NMAX * 64], si = tcol[V_S * NMAX * 64], yi = tcol[V_Y * NMAX * 64];
    double vi = tcol[V_V * NMAX * 64], gi = tcol[V_G * NMAX * 64], ui = tcol[V_U * NMAX * 64];
    double li = tcol[V_PIL * NMAX * 64] - tcol[V_PIU * NMAX * 64];
    coop_stage_wait();
    if (!in) { wd = 1.0; si = yi = vi = gi = ui = li = 0.0; }
    if (flags & 1) {
        const int upd = coop_bfgs_h<NMAX>(Wl, Ws, Ns_, lane, si, yi, vi, wd, vo.fl);
        if (!upd) vo.skip = 1;
        if (upd && in) *wdp = wd;
    }
    if (flags & 4) {
        // the shift of coop_visit_shift, on the H just updated and staged
        const double wlast = readlane_d(wd, Ns_ - 1);
        coop_shift_h<NMAX>(Wl, Ws, Ns_, lane, wlast, vo.fl);
    }
    if (flags & 2) {
        double d = 0.0, nl = 0.0, nu = 0.0, wdd = 0.0;
        QPResult r{0, 0};
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (attempt == 1) {
                vo.reset++;
                coop_reset<NMAX>(Ws, Wl3);
                wd = 1.0;
                if (in) *wdp = 1.0;
            }
            if (__ballot(in && !(wd > 0.0))) {
                r.status = -1;
                continue;
            }
            r = coop_box_qp_h<NMAX>(Wl, Wl3, Ns_, lane, wd, gi, ui, li, umin, umax, 8, d, nl, nu, wdd,
                                    vo.fl);
            vo.as += r.iters;
            if (r.status == 2) {
                const FallbackOut fb = coop_ipm_fallback<NMAX>(Wl3, Ns_, gi, ui, umin, umax, ipm_max_iter);
                vo.fl += fb.fl;
                vo.ipm += fb.iters;
                r.status = fb.status;
                r.iters = fb.iters;
                d = fb.d;
                nl = fb.nl;
                nu = fb.nu;
                wdd = in ? (nl - nu) - gi : 0.0;
            }
            if (r.status != -1) break;
        }
        vo.sqp = 1;
        if (r.status == 1) vo.ipmcap = 1;
        vo.gd = wave_sum(in ? gi * d : 0.0);
        if (in) {
            TB[V_D * NMAX * 64 + te(lane) + s * kTB] = d;
            TB[V_NL * NMAX * 64 + te(lane) + s * kTB] = nl;
            TB[V_NU * NMAX * 64 + te(lane) + s * kTB] = nu;
            TB[V_V * NMAX * 64 + te(lane) + s * kTB] = wdd;
        }
    }
    __syncthreads();
    return vo;
}

// W-form visit (qp_solver 0: interior point, 1: active set with the
// interior-point method as fallback) of sample s: stage W, the pending
// BFGS update, then the QP.  A non-positive pivot or diagonal (W not
// positive definite) resets W = I and solves again.
template <int NMAX>
__device__ __noinline__ VisitOut coop_visit_w(double* TB, double* Ws, lds_double* Wl3, int Ns_, int s,
                                              int flags, double umin, double umax, int ipm_max_iter,
                                              int qp_solver) {
    double* const Wl = (double*)Wl3;
    const int lane = threadIdx.x;
    Ns_ = uni(Ns_);
    s = uni(s);
    flags = uni(flags);
    qp_solver = uni(qp_solver);
    ipm_max_iter = uni(ipm_max_iter);
    umin = uni_d(umin);
    umax = uni_d(umax);
    VisitOut vo{0.0, 0, 0, 0, 0, 0, 0, 0.0};
    const bool in = lane < Ns_;
    coop_stage<NMAX>(Ws, Wl, lane);
    if (flags & 1) {
        const double si = in ? TB[V_S * NMAX * 64 + te(lane) + s * kTB] : 0.0;
        const double yi = in ? TB[V_Y * NMAX * 64 + te(lane) + s * kTB] : 0.0;
        if (!coop_bfgs<NMAX>(Wl, Ws, Ns_, lane, si, yi)) vo.skip = 1;
    }
    if (flags & 2) {
        const double gi = in ? TB[V_G * NMAX * 64 + te(lane) + s * kTB] : 0.0;
        const double ui = in ? TB[V_U * NMAX * 64 + te(lane) + s * kTB] : 0.0;
        const double li = in ? TB[V_PIL * NMAX * 64 + te(lane) + s * kTB] - TB[V_PIU * NMAX * 64 + te(lane) + s * kTB]
                             : 0.0;
        double d = 0.0, nl = 0.0, nu = 0.0, Dg = 1.0;
        QPResult r{0, 0};
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (attempt == 1) {
                vo.reset++;
                coop_reset<NMAX>(Ws, Wl3);
            }
            if (!coop_scale<NMAX>(Wl, Ns_, lane, Dg)) {
                r.status = -1;
                continue;
            }
            r.status = 2;
            if (qp_solver == 1) {
                r = coop_box_qp_as<NMAX>(Wl, Ns_, lane, Dg, gi, ui, li, umin, umax, 8, d, nl, nu);
                vo.as += r.iters;
            }
            if (r.status == 2) {
                r = coop_box_qp<NMAX>(Wl, Ns_, lane, Dg, gi, ui, umin, umax, ipm_max_iter, d, nl, nu);
                vo.ipm += r.iters;
            }
            if (r.status != -1) break;
        }
        vo.sqp = 1;
        if (r.status == 1) vo.ipmcap = 1;
        vo.gd = wave_sum(in ? gi * d : 0.0);
        if (in) {
            TB[V_D * NMAX * 64 + te(lane) + s * kTB] = d;
            TB[V_NL * NMAX * 64 + te(lane) + s * kTB] = nl;
            TB[V_NU * NMAX * 64 + te(lane) + s * kTB] = nu;
        }
    }
    __syncthreads();
    return vo;
}

// Hessian shift for the next OCP (W or inverse form) of sample s; returns
// the FP64 work.
template <int NMAX>
__device__ __noinline__ double coop_visit_shift(double* TB, double* Ws, lds_double* Wl3, int Ns_,
                                                int s, int inverse) {
    double* const Wl = (double*)Wl3;
    const int lane = threadIdx.x;
    Ns_ = uni(Ns_);
    s = uni(s);
    inverse = uni(inverse);
    coop_stage<NMAX>(Ws, Wl, lane);
    double fl = 0.0;
    if (inverse) {
        const double wlast = TB[V_WD * NMAX * 64 + te(Ns_ - 1) + s * kTB];
        coop_shift_h<NMAX>(Wl, Ws, Ns_, lane, wlast, fl);
    } else {
        coop_shift<NMAX>(Wl, Ws, Ns_, lane);
    }
    return fl;
}

// One backward pass over a lane's sample (lane-offset tiles, element k at
// [te(k)]): the discrete adjoint of the RK4 shooting over the interval
// derivatives ocp_shoot recorded, lambda_k = A_k (lambda_{k+1} + c_k) and
// g_k = dphi/du_k = B_k (lambda_{k+1} + c_k) backwards from lambda_N = 0,
// fused with, when kUpdate, the step of the
// accepted line search (u += alpha d, s = alpha d, pi += alpha (nu - pi),
// v = alpha v, y = g_new - g_old) and with the sums of the next KKT test,
// so that an SQP iteration reads each tile once.  The tiles of 8 intervals
// are loaded together ahead of their use.
template <bool kUpdate>
__device__ __forceinline__ KktSums adjoint_pass(int N, double alpha, const double* rec, double* U,
                                                const double* Dv, double* PIL, double* PIU,
                                                const double* NLv, const double* NUv, double* Sv,
                                                double* Vv, double* G, double* Y) {
    constexpr int kB = 8;
    double lam = 0.0;
    KktSums r{0.0, 0.0, false};
#pragma unroll 1
    for (int top = N - 1; top >= 0; top -= kB) {
        double A[kB], Bv[kB], Cc[kB], G0[kB], u[kB], dv[kB], pl[kB], pu[kB], nl[kB], nu[kB],
            vv[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = top - j >= 0 ? top - j : 0;
            const double* const rr = rec + (int64_t)(3 * k) * kTile;
            A[j] = rr[0];
            Bv[j] = rr[kTile];
            Cc[j] = rr[2 * kTile];
            if (kUpdate) {
                G0[j] = G[te(k)];
                u[j] = U[te(k)];
                dv[j] = Dv[te(k)];
                pl[j] = PIL[te(k)];
                pu[j] = PIU[te(k)];
                nl[j] = NLv[te(k)];
                nu[j] = NUv[te(k)];
                vv[j] = Vv[te(k)];
            }
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = top - j;
            if (k >= 0) {
                lam += Cc[j];
                const double gk = Bv[j] * lam;
                lam = A[j] * lam;
                double p_l = 0.0, p_u = 0.0;
                if (kUpdate) {
                    const double un = u[j] + alpha * dv[j];
                    Sv[te(k)] = un - u[j];
                    U[te(k)] = un;
                    p_l = pl[j] + alpha * (nl[j] - pl[j]);
                    p_u = pu[j] + alpha * (nu[j] - pu[j]);
                    PIL[te(k)] = p_l;
                    PIU[te(k)] = p_u;
                    Vv[te(k)] = alpha * vv[j];
                    Y[te(k)] = gk - G0[j];
                }
                G[te(k)] = gk;
                kkt_add(r, gk, p_l, p_u);
            }
        }
    }
    return r;
}

// adjoint_pass for the three-state record (ocp_shoot3): mu = lambda_{k+1} +
// c_k e_T, g_k = B_k . mu, lambda_k = A_k^T mu; the same fused step update
// and KKT sums.  The records of 4 intervals are loaded together.
template <bool kUpdate>
__device__ __forceinline__ KktSums adjoint_pass3(int N, double alpha, const double* rec, double* U,
                                                 const double* Dv, double* PIL, double* PIU,
                                                 const double* NLv, const double* NUv, double* Sv,
                                                 double* Vv, double* G, double* Y) {
    constexpr int kB = 4;
    double l0 = 0.0, l1 = 0.0, l2 = 0.0;
    KktSums r{0.0, 0.0, false};
#pragma unroll 1
    for (int top = N - 1; top >= 0; top -= kB) {
        double R[kB][13], G0[kB], u[kB], dv[kB], pl[kB], pu[kB], nl[kB], nu[kB], vv[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = top - j >= 0 ? top - j : 0;
            const double* const rr = rec + (int64_t)(13 * k) * kTile;
#pragma unroll
            for (int e = 0; e < 13; ++e) R[j][e] = rr[e * kTile];
            if (kUpdate) {
                G0[j] = G[te(k)];
                u[j] = U[te(k)];
                dv[j] = Dv[te(k)];
                pl[j] = PIL[te(k)];
                pu[j] = PIU[te(k)];
                nl[j] = NLv[te(k)];
                nu[j] = NUv[te(k)];
                vv[j] = Vv[te(k)];
            }
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            const int k = top - j;
            if (k >= 0) {
                const double m0 = l0, m1 = l1, m2 = l2 + R[j][12];
                const double gk = R[j][9] * m0 + R[j][10] * m1 + R[j][11] * m2;
                l0 = R[j][0] * m0 + R[j][3] * m1 + R[j][6] * m2;
                l1 = R[j][1] * m0 + R[j][4] * m1 + R[j][7] * m2;
                l2 = R[j][2] * m0 + R[j][5] * m1 + R[j][8] * m2;
                double p_l = 0.0, p_u = 0.0;
                if (kUpdate) {
                    const double un = u[j] + alpha * dv[j];
                    Sv[te(k)] = un - u[j];
                    U[te(k)] = un;
                    p_l = pl[j] + alpha * (nl[j] - pl[j]);
                    p_u = pu[j] + alpha * (nu[j] - pu[j]);
                    PIL[te(k)] = p_l;
                    PIU[te(k)] = p_u;
                    Vv[te(k)] = alpha * vv[j];
                    Y[te(k)] = gk - G0[j];
                }
                G[te(k)] = gk;
                kkt_add(r, gk, p_l, p_u);
            }
        }
    }
    return r;
}

// The shooting pass and the gradient pass of the estimator's model.
template <int NX, bool kRec>
__device__ __forceinline__ double shoot_nx(const DevParams& p, int N, const double (&x0)[NX],
                                           int i0, int istep, double sign, const double* u,
                                           const double* d, double alpha, bool use_d,
                                           double* rec) {
    if constexpr (NX == 3)
        return ocp_shoot3<kRec>(p, N, x0, i0, istep, sign, u, d, alpha, use_d, rec);
    else
        return ocp_shoot<kRec>(p, N, x0[0], i0, istep, sign, u, d, alpha, use_d, rec);
}

template <int NX, bool kUpdate>
__device__ __forceinline__ KktSums adjoint_nx(int N, double alpha, const double* rec, double* U,
                                              const double* Dv, double* PIL, double* PIU,
                                              const double* NLv, const double* NUv, double* Sv,
                                              double* Vv, double* G, double* Y) {
    if constexpr (NX == 3)
        return adjoint_pass3<kUpdate>(N, alpha, rec, U, Dv, PIL, PIU, NLv, NUv, Sv, Vv, G, Y);
    else
        return adjoint_pass<kUpdate>(N, alpha, rec, U, Dv, PIL, PIU, NLv, NUv, Sv, Vv, G, Y);
}

// One SQP solve (SQP section, single shooting) for every lane with `live`;
// returns per lane whether it converged.  u (V_U) holds the warm start on
// entry and the last iterate on return.
template <int NMAX, int GMODE, int NX>
__device__ __forceinline__ bool sqp_group(const DevParams& p, bool live, int N, int i, const Setup& su,
                          const double (&xhat)[NX], int lane, double* TB, double* XS, double* Wslot,
                          double* Wl, int (&cnt)[C_NCNT], double& qfl, bool pair_ls,
                          bool& shifted) {
    double* const U = TB + (V_U * NMAX) * 64 + lane * kTB;
    double* const G = TB + (V_G * NMAX) * 64 + lane * kTB;
    double* const Dv = TB + (V_D * NMAX) * 64 + lane * kTB;
    double* const PIL = TB + (V_PIL * NMAX) * 64 + lane * kTB;
    double* const PIU = TB + (V_PIU * NMAX) * 64 + lane * kTB;
    double* const NLv = TB + (V_NL * NMAX) * 64 + lane * kTB;
    double* const NUv = TB + (V_NU * NMAX) * 64 + lane * kTB;
    double* const Sv = TB + (V_S * NMAX) * 64 + lane * kTB;
    double* const Yv = TB + (V_Y * NMAX) * 64 + lane * kTB;
    double* const WDv = TB + (V_WD * NMAX) * 64 + lane * kTB;
    double* const Vv = TB + (V_V * NMAX) * 64 + lane * kTB;
    double* const Xs = XS + lane;
    static constexpr double smax = 100.0;
    static_assert(GMODE == 1 || NX == 1, "forward sensitivities: one-state model only");
    static_assert(NMAX % kTB == 0, "lane tiles hold whole blocks");

    double f = 0.0;
    if (live) {
        const bool fresh = i == 0 || !p.hess_warm;
        #pragma unroll 4
        for (int k = 0; k < N; ++k) {
            double v = U[te(k)];
            if (v < p.umin) v = p.umin;
            if (v > p.umax) v = p.umax;
            U[te(k)] = v;
            PIL[te(k)] = 0.0;
            PIU[te(k)] = 0.0;
            if (fresh) WDv[te(k)] = 1.0;
        }
    }
    // W = I for the first OCP (and every OCP without the warm start)
    {
        uint64_t m = __ballot(live && (i == 0 || !p.hess_warm));
        while (m) {
            const int s = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int Ns_ = __builtin_amdgcn_readlane(N, s);
            coop_identity<NMAX>(nullptr, Wslot + (int64_t)s * NMAX * NMAX, Ns_, lane);
        }
    }
    KktSums ks{0.0, 0.0, false};   // sums of the next KKT test
    double Dl = 0.0;               // g'd of the last QP step
    if (live) {
        f = shoot_nx<NX, GMODE == 1>(p, N, xhat, i, su.istep, su.sign, U, Dv, 0.0, false, Xs);
        cnt[C_LS]++;
        if constexpr (GMODE == 1)
            ks = adjoint_nx<NX, false>(N, 0.0, Xs, U, Dv, PIL, PIU, NLv, NUv, Sv, Vv, G, Yv);
        else
            ks = ocp_grad_fwd<NMAX>(p, N, xhat[0], i, su.istep, su.sign, U, G, nullptr, Dv, PIL, PIU);
        cnt[C_GRAD]++;
    }
    bool active = live, pending = false, converged = false;
    int l = 0;
    for (;;) {
        // scaled KKT test, eq. (convergence), on the lanes still iterating
        if (active) {
            // from the sums the gradient pass left (dividing the largest
            // |grad L|_k by sd > 0 selects the same maximum as dividing each)
            const double sd = (ks.s1 / (2.0 * N) > smax ? ks.s1 / (2.0 * N) : smax) / smax;
            const double kkt = ks.rmax / sd;
            const bool bad = ks.bad || (kkt != kkt);
            if (!bad && kkt <= p.sqp_eps) { converged = true; active = false; }
            else if (l == p.sqp_max_iter) { active = false; }
        }
        // wavefront-cooperative phase: pending BFGS updates, then QPs
        const uint64_t mp = __ballot(pending);
        const uint64_t ma = __ballot(active);
        uint64_t m = mp | ma;
        while (m) {
            const int s = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int Ns_ = __builtin_amdgcn_readlane(N, s);
            double* Ws = Wslot + (int64_t)s * NMAX * NMAX;
            // a pending update without a QP is the OCP's last visit: in
            // inverse form the Hessian shift for the next OCP joins it
            const bool last = ((mp >> s) & 1ull) && !((ma >> s) & 1ull) && p.hess_warm &&
                              p.qp_solver == 2;
            const int flags = (int)((mp >> s) & 1ull) | ((int)((ma >> s) & 1ull) << 1) |
                              (last ? 4 : 0);
            if (last && lane == s) shifted = true;
            const VisitOut vo =
                p.qp_solver == 2
                    ? coop_visit_h<NMAX>(TB, Ws, (lds_double*)Wl, Ns_, s, flags, p.umin, p.umax,
                                         p.ipm_max_iter)
                    : coop_visit_w<NMAX>(TB, Ws, (lds_double*)Wl, Ns_, s, flags, p.umin, p.umax,
                                         p.ipm_max_iter, p.qp_solver);
            if (lane == s) {
                Dl = vo.gd;
                qfl += vo.fl;
                cnt[C_SKIP] += vo.skip;
                cnt[C_RESET] += vo.reset;
                cnt[C_IPM] += vo.ipm;
                cnt[C_AS] += vo.as;
                cnt[C_SQP] += vo.sqp;
                cnt[C_IPMCAP] += vo.ipmcap;
            }
        }
        pending = false;
        if (ma == 0) break;
        // backtracking line search, eq. (Armijo), one sample per lane
        const double D = active ? Dl : 0.0;
        double alpha = 1.0;
        bool searching = active;
        int bt = 0;
        int rec_off = 0;   // column offset of the accepted trial's shooting record
        if (pair_ls) {
            // At most 32 samples per wavefront: lane l + 32, idle in the lane
            // phases, evaluates the trial after lane l's (step beta alpha,
            // its record in its own column) in the same pass, so a wavefront
            // whose lanes backtrack once pays one shooting pass, not two.
            // Lane l takes the first acceptable of the two in order, which
            // is the step, objective and counts of the serial search.
            const int src = lane & 31;
            const bool partner = lane >= 32;
            const int Np = __shfl(N, src, 64);
            double xp[NX];
#pragma unroll
            for (int a = 0; a < NX; ++a) xp[a] = __shfl(xhat[a], src, 64);
            const int isp = __shfl(su.istep, src, 64);
            const double sgp = __shfl(su.sign, src, 64);
            double* const Up = TB + (V_U * NMAX) * 64 + src * kTB;
            double* const Dp = TB + (V_D * NMAX) * 64 + src * kTB;
            for (;;) {
                const bool s_on = __shfl(searching ? 1 : 0, src, 64) != 0;
                if (!__ballot(s_on)) break;
                const int bt_o = __shfl(bt, src, 64);
                const double a_o = __shfl(alpha, src, 64);
                const int my_bt = partner ? bt_o + 1 : bt_o;
                const double my_a = partner ? p.ls_beta * a_o : a_o;
                double ft = 0.0;
                if (s_on && my_bt <= p.ls_max_bt)
                    ft = shoot_nx<NX, GMODE == 1>(p, Np, xp, i, isp, sgp, Up, Dp, my_a, true, Xs);
                const double ft2 = __shfl(ft, (lane + 32) & 63, 64);
                if (!partner && searching) {
                    cnt[C_LS]++;
                    bool accept = false;
                    if (bt == 0 && -D <= 64.0 * DBL_EPSILON * (1.0 + fabs(f))) accept = true;
                    else if (ft <= f + p.ls_c1 * alpha * D) accept = true;
                    else if (bt == p.ls_max_bt) { cnt[C_LSCAP]++; accept = true; }
                    if (accept) {
                        searching = false;
                        f = ft;
                        rec_off = 0;
                    } else {
                        // the partner's trial: bt + 1 <= ls_max_bt here
                        alpha = p.ls_beta * alpha;
                        ++bt;
                        cnt[C_LS]++;
                        if (ft2 <= f + p.ls_c1 * alpha * D) accept = true;
                        else if (bt == p.ls_max_bt) { cnt[C_LSCAP]++; accept = true; }
                        if (accept) {
                            searching = false;
                            f = ft2;
                            rec_off = 32;
                        } else {
                            alpha = p.ls_beta * alpha;
                            ++bt;
                        }
                    }
                }
            }
        } else {
            while (__ballot(searching)) {
                if (searching) {
                    const double ft =
                        shoot_nx<NX, GMODE == 1>(p, N, xhat, i, su.istep, su.sign, U, Dv, alpha, true, Xs);
                    cnt[C_LS]++;
                    bool accept = false;
                    if (bt == 0 && -D <= 64.0 * DBL_EPSILON * (1.0 + fabs(f))) accept = true;
                    else if (ft <= f + p.ls_c1 * alpha * D) accept = true;
                    else if (bt == p.ls_max_bt) { cnt[C_LSCAP]++; accept = true; }
                    if (accept) { searching = false; f = ft; }
                    else { alpha = p.ls_beta * alpha; ++bt; }
                }
            }
        }
        if (active) {
            if constexpr (GMODE == 1) {
                ks = adjoint_nx<NX, true>(N, alpha, Xs + rec_off, U, Dv, PIL, PIU, NLv, NUv, Sv, Vv, G,
                                          Yv);
            } else {
                #pragma unroll 4
                for (int k = 0; k < N; ++k) {
                    const double uo = U[te(k)];
                    const double un = uo + alpha * Dv[te(k)];
                    Sv[te(k)] = un - uo;
                    U[te(k)] = un;
                    PIL[te(k)] = PIL[te(k)] + alpha * (NLv[te(k)] - PIL[te(k)]);
                    PIU[te(k)] = PIU[te(k)] + alpha * (NUv[te(k)] - PIU[te(k)]);
                    Vv[te(k)] = alpha * Vv[te(k)];
                }
                ks = ocp_grad_fwd<NMAX>(p, N, xhat[0], i, su.istep, su.sign, U, G, Yv, Dv, PIL, PIU);
            }
            cnt[C_GRAD]++;
            pending = true;
            ++l;
        }
    }
    return converged;
}

template <int NMAX, int GMODE, int NX>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NMAX == 64 ? MC_NMPC_WAVES_PER_EU_64 : MC_NMPC_WAVES_PER_EU))) void nmpc_kernel(DevParams p, NmpcWork wk, Outs out) {
    // staged W (or H) of one sample, then two broadcast vectors (lds_vec)
    __shared__ __attribute__((aligned(16))) double Wl[NMAX * NMAX + 2 * NMAX];
    const int lane = threadIdx.x;
    double* const TB = wk.tiles + (int64_t)blockIdx.x * wk.tile_stride;
    double* const XS = wk.xs + (int64_t)blockIdx.x * wk.xs_stride;
    double* const Wslot = wk.W + (int64_t)blockIdx.x * wk.w_stride;
    double* const U = TB + (V_U * NMAX) * 64 + lane * kTB;
    const double sqrtR = sqrt(p.Rmeas);
    const double h = p.Ts / (double)p.Ns;
    const double sqh = sqrt(h);

    const int g_hi = wk.qhi ? *wk.qhi : wk.n_groups;
    for (;;) {
        int grp = 0;
        if (lane == 0) grp = atomicAdd(wk.queue, 1);
        grp = __shfl(grp, 0, 64);
        if (grp >= g_hi) break;
        const int64_t idx = (int64_t)grp * wk.spw + lane;
        const bool has = lane < wk.spw && idx < wk.n_pos;
        const int64_t pos = has ? wk.pos[idx] : 0;
        Setup su = sample_setup(pos);
        const int N = has ? su.N : 1;
        const int L = has ? su.L : -1;
        int cnt[C_NCNT];
#pragma unroll
        for (int c = 0; c < C_NCNT; ++c) cnt[c] = 0;
        double qfl = 0.0;   // inverse-form QP / BFGS / shift work of this lane's sample
        double n[3] = {su.n0[0], su.n0[1], su.n0[2]};
        // estimator state: x-hat (NX values) and P (1, or the 6 entries of
        // the symmetric 3x3 with P_0 = P0 I)
        double xhat[NX], P[NX == 3 ? 6 : 1];
        if constexpr (NX == 3) {
            if (p.x0_mode == 0) {
                xhat[0] = p.cAin * p.V;
                xhat[1] = p.cBin * p.V;
                xhat[2] = p.cTin * p.V;
            } else {
                // the model's steady state at zbar(0), as for the one-state filter
                const double T = setpoint(p, 0, su.istep, su.sign);
                xhat[0] = (p.cAin + (p.cTin - T) / p.beta) * p.V;
                xhat[1] = (p.cBin + 2.0 * (p.cTin - T) / p.beta) * p.V;
                xhat[2] = T * p.V;
            }
            P[0] = p.P0; P[1] = 0.0; P[2] = 0.0; P[3] = p.P0; P[4] = 0.0; P[5] = p.P0;
        } else {
            xhat[0] = su.xhat0;
            P[0] = p.P0;
        }
        double Fprev = su.ubar, phiacc = 0.0;
        uint64_t hsh = 14695981039346656037ull;
        if (has)
            #pragma unroll 1
            for (int k = 0; k < N; ++k) U[te(k)] = su.ubar * kMlMinPerLs;
        const int Lmax = wave_max_i(L);
        int Lrun = L;   // cut short when the plant state stops being finite
        for (int i = 0; i <= Lmax; ++i) {
            const bool live = has && i <= Lrun;
            bool step = live && i < Lrun;
            double z = 0.0;
            if (live) {
                z = n[2] / p.V;
                const double zb = setpoint(p, i, su.istep, su.sign);
                phiacc += (z - zb) * (z - zb);
                if (out.tz) out.tz[(int64_t)i * out.S + pos] = z;
                if (!isfinite(z)) {
                    // the plant diverged (Phi is not a number): no more OCPs
                    cnt[C_NONFIN] = 1;
                    Lrun = i;
                    step = false;
                }
            }
            if (step) {
                const double y = z + p.noise_scale * sqrtR *
                                         normal_first(p.seed, 0, (uint32_t)i, su.nid, kTagMeas);
                bool fin = true;
                if constexpr (NX == 3) {
                    ekf3_predict(p, xhat, P, Fprev);
                    ekf3_update(p, xhat, P, y);
#pragma unroll
                    for (int e = 0; e < 6; ++e) fin = fin && isfinite(P[e]);
                } else {
                    ekf_predict(p, xhat[0], P[0], Fprev);
                    ekf_update(p, xhat[0], P[0], y);
                    fin = isfinite(P[0]);
                }
#pragma unroll
                for (int a = 0; a < NX; ++a) fin = fin && isfinite(xhat[a]);
                if (out.tx) out.tx[(int64_t)i * out.S + pos] = xhat[NX - 1];
                if (!fin) cnt[C_NONFIN] = 1;
            }
            bool shifted = false;
            const bool conv = sqp_group<NMAX, GMODE, NX>(p, step, N, i, su, xhat, lane, TB, XS, Wslot,
                                                     Wl, cnt, qfl, wk.spw <= 32, shifted);
            if (p.hess_warm) {
                // samples whose last visit did not shift (no pending update)
                uint64_t m = __ballot(step && !shifted);
                while (m) {
                    const int s = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    const int Ns_ = __builtin_amdgcn_readlane(N, s);
                    double* Ws = Wslot + (int64_t)s * NMAX * NMAX;
                    const double fl =
                        coop_visit_shift<NMAX>(TB, Ws, (lds_double*)Wl, Ns_, s, p.qp_solver == 2);
                    if (lane == s) qfl += fl;
                }
            }
            if (step) {
                cnt[C_OCP]++;
                if (!conv) cnt[C_OCP_FAIL]++;
                uint64_t mask = 0;
                #pragma unroll 4
                for (int k = 0; k < N; ++k) {
                    const double v = U[te(k)];
                    if (v <= p.umin + 1e-6 || v >= p.umax - 1e-6) mask |= (1ull << k);
                }
                hsh = fnv1a_step(hsh, (uint32_t)i, mask);
                const double F = U[0] / kMlMinPerLs;
                double* const WDv = TB + (V_WD * NMAX) * 64 + lane * kTB;
                #pragma unroll 4
                for (int k = 0; k + 1 < N; ++k) {
                    U[te(k)] = U[te(k + 1)];
                    WDv[te(k)] = WDv[te(k + 1)];
                }
                if (out.tu) out.tu[(int64_t)i * out.S + pos] = F;
                #pragma unroll 1
                for (int j = 0; j < p.Ns; ++j) {
                    double xi[3];
                    process_noise(p, (uint32_t)(i * p.Ns + j), su.nid, xi);
                    em_step(p, su.k0, su.EaR, n, F, h, sqh, xi);
                }
                Fprev = F;
            }
        }
        if (has) {
            if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) cnt[C_NONFIN] = 1;
            out.phi[pos] = phiacc / (double)(L + 1);
            out.hash[pos] = hsh;
            cnt[C_KIND] = 0;
            cnt[C_N] = N;
            cnt[C_L] = L;
            out.flops[pos] = sample_flops(p, 0, N, L, cnt, GMODE, qfl, NX);
#pragma unroll
            for (int c = 0; c < C_NCNT; ++c) out.cnt[(int64_t)c * out.S + pos] = cnt[c];
        }
    }
}

// K lanes per PI sample.  A PI closed loop is one serial chain, so a launch
// with fewer wavefronts than SIMDs takes one chain's time, and most of a
// sub-step's instructions draw its noise (Philox, Box-Muller), which does
// not depend on the state.  The K lanes of a group draw the noise of K
// sub-steps at once, lane r that of sub-step j0 + r, and then all of them
// integrate the K sub-steps in turn, each taking a sub-step's normals from
// the lane that drew them by a DPP quad broadcast.  The lanes of a group
// compute the same values in the same order, so they hold the same state
// bit for bit (the results do not depend on K) and write the same outputs
// to the same addresses; every lane reads back only what it wrote itself.
template <int K, int RR>
__device__ __forceinline__ double group_bcast(double v) {
    static_assert((K == 1 || K == 2 || K == 4) && RR < K, "groups of 1, 2 or 4 lanes");
    if constexpr (K == 1) return v;
    else if constexpr (K == 2) return dpp_z<RR | RR << 2 | (2 + RR) << 4 | (2 + RR) << 6>(v);
    else return dpp_z<RR * 0x55>(v);   // quad_perm [RR, RR, RR, RR]
}
// The value that lane q of the group holds, on the whole group (q the same
// on every lane): a group draws per-interval noise for K intervals at once,
// lane q that of the q-th.
template <int K>
__device__ __forceinline__ double group_pick(double v, int q) {
    if constexpr (K == 1) return v;
    else if constexpr (K == 2) return q == 0 ? group_bcast<2, 0>(v) : group_bcast<2, 1>(v);
    else {
        const double v0 = group_bcast<4, 0>(v), v1 = group_bcast<4, 1>(v);
        const double v2 = group_bcast<4, 2>(v), v3 = group_bcast<4, 3>(v);
        return q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : v3));
    }
}
template <int K, int RR, class Step>
__device__ __forceinline__ void pi_group_steps(int j0, int Ns, const double (&own)[3], Step& step) {
    if constexpr (RR < K) {
        // j0 and Ns are the same on every lane: the broadcast runs on the
        // whole group
        if (j0 + RR < Ns) {
            const double xi[3] = {group_bcast<K, RR>(own[0]), group_bcast<K, RR>(own[1]),
                                  group_bcast<K, RR>(own[2])};
            step(j0 + RR, xi);
        }
        pi_group_steps<K, RR + 1>(j0, Ns, own, step);
    }
}
// The Ns Euler-Maruyama sub-steps of interval i, K at a time; step(j, xi)
// takes sub-step j with its noise.  A lane whose sub-step index passes Ns
// draws a noise value nobody uses.
template <int K, class Step>
__device__ __forceinline__ void pi_substeps(const DevParams& p, const Setup& su, int i, Step step) {
    const int r = (int)threadIdx.x & (K - 1);
    #pragma unroll 1
    for (int j0 = 0; j0 < p.Ns; j0 += K) {
        double own[3];
        process_noise(p, (uint32_t)(i * p.Ns + j0 + r), su.nid, own);
        pi_group_steps<K, 0>(j0, p.Ns, own, step);
    }
}
// The reverse sweep's counterpart: sub-steps j0, j0 - 1, ..., j0 - K + 1
// (those >= 0) in turn, each with the M values lane r = j0 - j formed.
template <int K, int RR, int M, class Step>
__device__ __forceinline__ void pi_group_back(int j0, const double (&own)[M], Step& step) {
    if constexpr (RR < K) {
        if (j0 - RR >= 0) {   // the same on every lane
            double v[M];
#pragma unroll
            for (int q = 0; q < M; ++q) v[q] = group_bcast<K, RR>(own[q]);
            step(v);
        }
        pi_group_back<K, RR + 1>(j0, own, step);
    }
}

// PI closed loop, eq. (PI), one sample per group of K lanes (sample t on
// lanes [K t, K (t + 1)) of the launch).  With ck != null the plant state
// (n, I-hat) at the start of every interval i = 0, C, 2C, ... is kept for
// the reverse pass: ck[((i / C) * 4 + f) * npi + t].  With ctl != null the
// launch covers the PI samples [c ppc, (c + 1) ppc) of chunk c = *ctl.
template <int K>
__global__ __launch_bounds__(64) void pi_kernel(DevParams p, const int64_t* pos_list, int64_t npi,
                                                Outs out, double* ck, const int* ctl, int64_t ppc) {
    int64_t t1 = npi, t = ((int64_t)blockIdx.x * 64 + threadIdx.x) / K;
    if (ctl) {
        const int64_t t0 = (int64_t)(*ctl) * ppc;
        t += t0;
        t1 = t0 + ppc < npi ? t0 + ppc : npi;
    }
    if (t >= t1) return;
    const int64_t pos = pos_list[t];
    const Setup su = sample_setup(pos);
    const double sqrtR = sqrt(p.Rmeas);
    const double h = p.Ts / (double)p.Ns;
    const double sqh = sqrt(h);
    double n[3] = {su.n0[0], su.n0[1], su.n0[2]};
    double xhat = su.xhat0, P = p.P0, Fprev = su.ubar, Ihat = 0.0, phiacc = 0.0;
    // the three-state estimator, when the model is selected (x-hat_0 and
    // P_0 = P0 I as in the NMPC kernel)
    double x3[3] = {0.0, 0.0, 0.0}, P3[6] = {p.P0, 0.0, 0.0, p.P0, 0.0, p.P0};
    if (p.model_nx == 3) {
        if (p.x0_mode == 0) {
            x3[0] = p.cAin * p.V; x3[1] = p.cBin * p.V; x3[2] = p.cTin * p.V;
        } else {
            const double T = setpoint(p, 0, su.istep, su.sign);
            x3[0] = (p.cAin + (p.cTin - T) / p.beta) * p.V;
            x3[1] = (p.cBin + 2.0 * (p.cTin - T) / p.beta) * p.V;
            x3[2] = T * p.V;
        }
    }
    int nonfin = 0;
    double meas = 0.0;   // measurement noise drawn for the group (below)
    for (int i = 0;; ++i) {
        const double z = n[2] / p.V;
        const double zb = setpoint(p, i, su.istep, su.sign);
        phiacc += (z - zb) * (z - zb);
        if (out.tz) out.tz[(int64_t)i * out.S + pos] = z;
        if (i == su.L) break;
        if (ck && p.ckpt_C > 0 && i % p.ckpt_C == 0) {
            const int64_t b = (int64_t)(i / p.ckpt_C) * 4;
            ck[(b + 0) * npi + t] = n[0];
            ck[(b + 1) * npi + t] = n[1];
            ck[(b + 2) * npi + t] = n[2];
            ck[(b + 3) * npi + t] = Ihat;
        }
        // the measurement noise of intervals i .. i + K - 1, lane r that of
        // i + r (i is the same on every lane still running)
        if ((i & (K - 1)) == 0)
            meas = normal_first(p.seed, 0, (uint32_t)(i + ((int)threadIdx.x & (K - 1))), su.nid,
                                kTagMeas);
        const double y = z + p.noise_scale * sqrtR * group_pick<K>(meas, i & (K - 1));
        if (p.run_ekf_for_pi && p.model_nx == 3) {
            ekf3_predict(p, x3, P3, Fprev);
            ekf3_update(p, x3, P3, y);
            xhat = x3[2];
            bool fin = isfinite(x3[0]) && isfinite(x3[1]) && isfinite(x3[2]);
#pragma unroll
            for (int e = 0; e < 6; ++e) fin = fin && isfinite(P3[e]);
            if (!fin) nonfin = 1;
        } else if (p.run_ekf_for_pi) {
            ekf_predict(p, xhat, P, Fprev);
            ekf_update(p, xhat, P, y);
            if (!isfinite(xhat) || !isfinite(P)) nonfin = 1;
        }
        if (out.tx) out.tx[(int64_t)i * out.S + pos] = xhat;
        const double e = zb - y;
        const double Ik = Ihat + p.Ts * p.kI * e;
        const double uh = su.ubar + p.kP * e + Ik;
        double uk = uh;
        if (uk > p.pi_umax) uk = p.pi_umax;
        if (uk < p.pi_umin) uk = p.pi_umin;
        Ihat = Ik + p.Ts * p.kaw * (uh - uk);
        const double F = uk;
        if (out.tu) out.tu[(int64_t)i * out.S + pos] = F;
        auto step = [&](int, const double (&xi)[3]) { em_step(p, su.k0, su.EaR, n, F, h, sqh, xi); };
        pi_substeps<K>(p, su, i, step);
        Fprev = F;
    }
    if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) nonfin = 1;
    out.phi[pos] = phiacc / (double)(su.L + 1);
    out.hash[pos] = 14695981039346656037ull;
    const int vals[C_NCNT] = {1, su.N, su.L, 0, 0, 0, 0, 0, 0, 0, 0, 0, nonfin, 0, 0};
    out.flops[pos] = sample_flops(p, 1, su.N, su.L, vals, 1, 0.0, p.model_nx);
#pragma unroll
    for (int c = 0; c < C_NCNT; ++c) out.cnt[(int64_t)c * out.S + pos] = vals[c];
}

// Reverse pass of the PI closed loop (pathwise, noise held fixed) from the
// checkpoints: each segment of C intervals is recomputed forward with its
// per-sub-step states and noise taped (tape[(step * 6 + f) * npi + t]),
// then swept backwards.  (Drawing the noise again in the reverse sweep
// instead of taping it halves the tape but adds two Philox blocks and a
// Box-Muller pair to each sample's serial chain: with one lane per sample,
// c2's reverse pass took 48.9 ms that way against 35.1 ms taped.)  Writes dPhi/dkP and dPhi/dkI
// per sample.  A sample takes K lanes as in pi_kernel: the recomputation
// draws the noise of K sub-steps at once, and the K lanes tape, sweep and
// write the same values.
template <int K>
__global__ __launch_bounds__(64) void pi_reverse_kernel(DevParams p, const int64_t* pos_list,
                                                        int64_t npi, const double* ck,
                                                        double* tape, double* iv_tape,
                                                        double* gk /* [2][npi] */) {
    const int64_t t = ((int64_t)blockIdx.x * 64 + threadIdx.x) / K;
    if (t >= npi) return;
    const int64_t pos = pos_list[t];
    const Setup su = sample_setup(pos);
    const double sqrtR = sqrt(p.Rmeas);
    const double h = p.Ts / (double)p.Ns;
    const double sqh = sqrt(h);
    const double iV = 1.0 / p.V;
    const int L = su.L, C = p.ckpt_C;
    const double wL = 1.0 / (double)(L + 1);
    // the final cost term z_L
    double nb[3] = {0.0, 0.0, 0.0};
    double Ib = 0.0, gkP = 0.0, gkI = 0.0;
    const int nseg = (L + C - 1) / C;
    // start: need z_L, i.e. the state after the last segment; recomputed in
    // the last segment's forward sweep.
    bool have_final = false;
    for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int i0 = sgi * C;
        const int i1 = min(i0 + C, L);
        double n[3] = {ck[((int64_t)sgi * 4 + 0) * npi + t], ck[((int64_t)sgi * 4 + 1) * npi + t],
                       ck[((int64_t)sgi * 4 + 2) * npi + t]};
        double Ihat = ck[((int64_t)sgi * 4 + 3) * npi + t];
        // forward recompute of the segment, taping
        double meas = 0.0;
        #pragma unroll 1
        for (int i = i0; i < i1; ++i) {
            const int li = i - i0;
            const double z = n[2] * iV;
            // the measurement noise of K intervals at once, as in pi_kernel
            if ((li & (K - 1)) == 0)
                meas = normal_first(p.seed, 0, (uint32_t)(i + ((int)threadIdx.x & (K - 1))), su.nid,
                                    kTagMeas);
            const double xm = p.noise_scale * sqrtR * group_pick<K>(meas, li & (K - 1));
            iv_tape[((int64_t)li * 5 + 0) * npi + t] = n[0];
            iv_tape[((int64_t)li * 5 + 1) * npi + t] = n[1];
            iv_tape[((int64_t)li * 5 + 2) * npi + t] = n[2];
            iv_tape[((int64_t)li * 5 + 3) * npi + t] = Ihat;
            iv_tape[((int64_t)li * 5 + 4) * npi + t] = xm;
            const double zb = setpoint(p, i, su.istep, su.sign);
            const double e = zb - (z + xm);
            const double Ik = Ihat + p.Ts * p.kI * e;
            const double uh = su.ubar + p.kP * e + Ik;
            double uk = uh;
            if (uk > p.pi_umax) uk = p.pi_umax;
            if (uk < p.pi_umin) uk = p.pi_umin;
            Ihat = Ik + p.Ts * p.kaw * (uh - uk);
            auto step = [&](int j, const double (&xi)[3]) {
                const int64_t st = (int64_t)li * p.Ns + j;
                tape[(st * 6 + 0) * npi + t] = n[0];
                tape[(st * 6 + 1) * npi + t] = n[1];
                tape[(st * 6 + 2) * npi + t] = n[2];
                tape[(st * 6 + 3) * npi + t] = xi[0];
                tape[(st * 6 + 4) * npi + t] = xi[1];
                tape[(st * 6 + 5) * npi + t] = xi[2];
                em_step(p, su.k0, su.EaR, n, uk, h, sqh, xi);
            };
            pi_substeps<K>(p, su, i, step);
        }
        if (!have_final) {
            // cost term of the last sample point t_L
            const double zL = n[2] * iV;
            nb[2] = 2.0 * (zL - setpoint(p, L, su.istep, su.sign)) * wL * iV;
            have_final = true;
        }
        // reverse sweep over the segment
        #pragma unroll 1
        for (int i = i1 - 1; i >= i0; --i) {
            const int li = i - i0;
            const double n0 = iv_tape[((int64_t)li * 5 + 0) * npi + t];
            const double n1 = iv_tape[((int64_t)li * 5 + 1) * npi + t];
            const double n2 = iv_tape[((int64_t)li * 5 + 2) * npi + t];
            const double Ih0 = iv_tape[((int64_t)li * 5 + 3) * npi + t];
            const double xm = iv_tape[((int64_t)li * 5 + 4) * npi + t];
            const double z = n2 * iV;
            const double zb = setpoint(p, i, su.istep, su.sign);
            const double e = zb - (z + xm);
            const double Ik = Ih0 + p.Ts * p.kI * e;
            const double uh = su.ubar + p.kP * e + Ik;
            double uk = uh;
            if (uk > p.pi_umax) uk = p.pi_umax;
            if (uk < p.pi_umin) uk = p.pi_umin;
            const bool inside = (uh > p.pi_umin && uh < p.pi_umax);
            // plant: Ns Euler-Maruyama sub-steps backwards, K at a time: lane
            // r reads the tape of sub-step j0 - r and forms its values that
            // do not depend on the adjoint (the rate's derivatives and the
            // input sensitivity), all K at once; the K lanes then apply the
            // sub-steps' transposed Jacobians in turn
            double Fb = 0.0;
            auto back = [&](const double (&cf)[6]) {
                // J^T nb with J = -F/V I + S dr^T V
                const double Snb = -nb[0] - 2.0 * nb[1] + p.beta * nb[2];
                const double m0 = nb[0] + h * (-uk * iV * nb[0] + cf[0] * Snb);
                const double m1 = nb[1] + h * (-uk * iV * nb[1] + cf[1] * Snb);
                const double m2 = nb[2] + h * (-uk * iV * nb[2] + cf[2] * Snb);
                Fb += nb[0] * cf[3] + nb[1] * cf[4] + nb[2] * cf[5];
                nb[0] = m0; nb[1] = m1; nb[2] = m2;
            };
            const int r = (int)threadIdx.x & (K - 1);
            #pragma unroll 1
            for (int j0 = p.Ns - 1; j0 >= 0; j0 -= K) {
                // a lane past sub-step 0 reads sub-step 0's tape; what it
                // forms is not used
                const int j = j0 - r >= 0 ? j0 - r : 0;
                const int64_t st = (int64_t)li * p.Ns + j;
                const double a0 = tape[(st * 6 + 0) * npi + t];
                const double a1 = tape[(st * 6 + 1) * npi + t];
                const double a2 = tape[(st * 6 + 2) * npi + t];
                const double x0 = tape[(st * 6 + 3) * npi + t];
                const double x1 = tape[(st * 6 + 4) * npi + t];
                const double x2 = tape[(st * 6 + 5) * npi + t];
                const double cA = a0 * iV, cB = a1 * iV, cT = a2 * iV;
                const double k = su.k0 * exp(-su.EaR / cT);
                // dr/dn = (k cB, k cA, k EaR/cT^2 cA cB) / V, times V for the
                // rows of S r V; dn+/dF = h (C_in - c) + sigma sqrt(h) xi
                const double cf[6] = {k * cB * iV * p.V, k * cA * iV * p.V,
                                      k * (su.EaR / (cT * cT)) * cA * cB * iV * p.V,
                                      h * (p.cAin - cA) + p.sig[0] * sqh * x0,
                                      h * (p.cBin - cB) + p.sig[1] * sqh * x1,
                                      h * (p.cTin - cT) + p.sig[2] * sqh * x2};
                pi_group_back<K, 0>(j0, cf, back);
            }
            // PI law backwards: I-hat_i = I + Ts kaw (uh - u)
            const double ub = Fb - Ib * p.Ts * p.kaw;
            const double uhb = Ib * p.Ts * p.kaw + (inside ? ub : 0.0);
            const double Ikb = uhb + Ib;
            gkI += Ikb * p.Ts * e;
            gkP += uhb * e;
            const double eb = Ikb * p.Ts * p.kI + uhb * p.kP;
            Ib = Ikb;
            // e = zb - y, y = z + v, cost (z - zb)^2 / (L + 1)
            const double zbar_ = -eb + 2.0 * (z - zb) * wL;
            nb[2] += zbar_ * iV;
        }
    }
    gk[t] = gkP;
    gk[npi + t] = gkI;
}

// ------------------------------------------------------------ statistics ---
// Deterministic reductions: a single 1024-thread block, thread t takes
// elements t, t + 1024, ... in order, then a fixed binary tree in LDS.
__global__ __launch_bounds__(1024) void stats_kernel(const double* phi, const int32_t* cnt,
                                                     int64_t S, const double* flops_per,
                                                     double* out /* see host */,
                                                     unsigned long long* hist,
                                                     long long* totals) {
    __shared__ double sh[1024];
    __shared__ double sh2[1024];
    const int t = threadIdx.x;
    const int32_t* kind = cnt;  // row C_KIND
    double mean[2];
    long long count[2] = {0, 0};
    for (int c = 0; c < 2; ++c) {
        double a = 0.0;
        long long k = 0;
        for (int64_t s = t; s < S; s += 1024)
            if (kind[s] == c && isfinite(phi[s])) { a += phi[s]; ++k; }
        sh[t] = a;
        sh2[t] = (double)k;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) { sh[t] += sh[t + w]; sh2[t] += sh2[t + w]; }
            __syncthreads();
        }
        count[c] = (long long)sh2[0];
        mean[c] = count[c] > 0 ? sh[0] / (double)count[c] : 0.0;
        __syncthreads();
    }
    for (int c = 0; c < 2; ++c) {
        double a = 0.0;
        for (int64_t s = t; s < S; s += 1024)
            if (kind[s] == c && isfinite(phi[s])) {
                const double dlt = phi[s] - mean[c];
                a += dlt * dlt;
                const double v = log10(phi[s]);
                int b;
                if (!(v >= -4.0)) b = 0;
                else if (v >= 4.0) b = 201;
                else {
                    b = (int)floor((v + 4.0) / 8.0 * 200.0);
                    if (b > 199) b = 199;
                    b += 1;
                }
                atomicAdd(&hist[c * 202 + b], 1ull);
            }
        sh[t] = a;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) {
            out[c * 3 + 0] = (double)count[c];
            out[c * 3 + 1] = mean[c];
            out[c * 3 + 2] = count[c] > 1 ? sh[0] / (double)(count[c] - 1) : 0.0;
        }
        __syncthreads();
    }
    // counter totals (integers: any order) and algorithmic flops (fixed tree)
    for (int r = 0; r < C_NCNT; ++r) {
        long long a = 0;
        for (int64_t s = t; s < S; s += 1024) a += cnt[(int64_t)r * S + s];
        atomicAdd((unsigned long long*)&totals[r], (unsigned long long)a);
    }
    double fl[2] = {0.0, 0.0};
    for (int64_t s = t; s < S; s += 1024) {
        const int k = cnt[s];
        fl[k == 0 ? 0 : 1] += flops_per[s];
    }
    for (int c = 0; c < 2; ++c) {
        sh[t] = fl[c];
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) out[6 + c] = sh[0];
        __syncthreads();
    }
}

// Sum of per-sample gradients over the PI samples (fixed tree, one block).
__global__ __launch_bounds__(1024) void grad_reduce_kernel(const double* gk, int64_t npi,
                                                           double* out) {
    __shared__ double sh[1024];
    const int t = threadIdx.x;
    for (int c = 0; c < 2; ++c) {
        double a = 0.0;
        for (int64_t s = t; s < npi; s += 1024) a += gk[c * npi + s];
        sh[t] = a;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) sh[t] += sh[t + w];
            __syncthreads();
        }
        if (t == 0) out[c] = sh[0];
        __syncthreads();
    }
}

}  // namespace mccl
