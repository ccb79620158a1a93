// mc_dev.hpp -- device building blocks of the Monte Carlo closed-loop CSTR
// (arXiv 2212.02197) for gfx950: counter-based noise, plant and model right-
// hand sides, CD-EKF, PI law, RK4 single shooting with adjoint and forward-
// sensitivity gradients.  One sample per lane; FP64 throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mccl {

constexpr double kMlMinPerLs = 60000.0;   // 1 L/s = 60000 mL/min
constexpr int kSpMax = 8;
constexpr int kTile = 64;                  // lanes per wavefront (CDNA)

// Lane tiles (the SQP's per-sample vectors of a wavefront's samples): in the
// block of one vector, element k of the sample on lane l sits at
//   (k / 16) * 1024 + l * 16 + k % 16,
// so each lane's sixteen consecutive elements fill one 128-byte cache line.
// A cooperative visit then reads one sample's vector in 4 lines instead of
// 64 (the visits' memory traffic was dominated by such column reads), and
// the one-sample-per-lane phases, which walk k, read sixteen consecutive
// elements from the same lines.  A lane's pointer into a vector is
// block + l * kTB; element k is at offset te(k).  NMAX is a multiple of kTB.
constexpr int kTB = 16;
__device__ __forceinline__ int te(int k) {
    return (int)(((unsigned)k / kTB) * (kTB * kTile) + ((unsigned)k % kTB));
}

// Parameters as the kernels see them (passed by value as a kernel argument).
struct DevParams {
    double V, k0, EaR, beta, cAin, cBin, cTin;
    double sig[3];
    double Rmeas, Ts;
    int Ns, L;
    int n_sp, sp_period;
    int sp_i[kSpMax];
    double sp_z[kSpMax];
    double sp_step_rel;
    int sp_step_lo, sp_step_hi;
    int N, Nc;
    double Qz, umin, umax;
    double sqp_eps, ls_c1, ls_beta;
    int sqp_max_iter, ls_max_bt, grad_mode, ipm_max_iter;
    double kP, kI, kaw, pi_umin, pi_umax;
    double P0, x0_rel_std;
    int x0_mode, kind_split, default_kind, run_ekf_for_pi;
    uint64_t seed;
    int64_t noise_mod, n_samples, id_offset;
    int n_hc;
    int hc[4];
    int L_lo, L_hi;
    double kin_sigma;
    int hess_warm, want_grad;
    double noise_scale;
    int ckpt_C, qp_solver;
    int L_cap;           // closed-loop intervals are cut at L_cap (trial launches)
    int model_nx;        // estimator / OCP model: 1 one-state closure, 3 three-state
    // caller-given per-sample arrays (device copies, indexed by the sample's
    // column), or null: sample id, kind, horizon, length
    const int64_t* ids;
    const uint8_t* kind_ov;
    const int32_t* N_ov;
    const int32_t* L_ov;
    int nlp_form;        // OCP discretisation: 0 single shooting, 1 multiple shooting
};

// Noise streams: the counter's last word.
enum : uint32_t { kTagProcess = 0, kTagMeas = 1, kTagX0 = 2, kTagKin = 3, kTagScen = 4 };

// ---------------------------------------------------------------- Philox ---
// Philox4x32-10 (Salmon et al., SC'11): counter (block, step, id, tag),
// key (seed lo, seed hi).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

struct Uniform2 { double u1, u2; };

// Two 53-bit uniforms from one block: u1 in (0, 1], u2 in [0, 1).
__device__ __forceinline__ Uniform2 philox_uniforms(uint64_t seed, uint32_t block, uint32_t step,
                                                     uint32_t id, uint32_t tag) {
    uint32_t c[4] = {block, step, id, tag};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t m1 = ((((uint64_t)c[0]) << 32) | c[1]) >> 11;
    const uint64_t m2 = ((((uint64_t)c[2]) << 32) | c[3]) >> 11;
    Uniform2 r;
    r.u1 = (double)(m1 + 1) * 0x1p-53;
    r.u2 = (double)m2 * 0x1p-53;
    return r;
}

// Box-Muller: xi0 = rho cos(2 pi u2), xi1 = rho sin(2 pi u2).
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t block, uint32_t step,
                                            uint32_t id, uint32_t tag, double& xi0, double& xi1) {
    const Uniform2 u = philox_uniforms(seed, block, step, id, tag);
    const double rho = sqrt(-2.0 * log(u.u1));
    double s, c;
    sincos(6.283185307179586 * u.u2, &s, &c);
    xi0 = rho * c;
    xi1 = rho * s;
}

__device__ __forceinline__ double normal_first(uint64_t seed, uint32_t block, uint32_t step,
                                               uint32_t id, uint32_t tag) {
    const Uniform2 u = philox_uniforms(seed, block, step, id, tag);
    return sqrt(-2.0 * log(u.u1)) * cos(6.283185307179586 * u.u2);
}

// ------------------------------------------------------- fast FP64 math ---
// 1/a for positive normal a: the hardware reciprocal estimate refined by two
// Newton steps (each doubles the number of correct bits), within 1 ulp of the
// correctly rounded quotient; half the instructions of an IEEE division,
// which the model's rate expression needs at every RK4 stage.
__device__ __forceinline__ double rcp_pos(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

// -------------------------------------------------------------- the model ---
// Three-state plant drift, eq. (CSTR): C_in F - c F + S r V, S = [-1,-2,beta].
__device__ __forceinline__ void plant_f3(const DevParams& p, double k0, double EaR,
                                         const double n[3], double F, double f[3]) {
    const double iV = 1.0 / p.V;
    const double cA = n[0] * iV, cB = n[1] * iV, cT = n[2] * iV;
    const double rV = k0 * exp(-EaR * rcp_pos(cT)) * cA * cB * p.V;
    f[0] = (p.cAin - cA) * F - rV;
    f[1] = (p.cBin - cB) * F - 2.0 * rV;
    f[2] = (p.cTin - cT) * F + p.beta * rV;
}

// One-state model x = n_T with the reaction-invariant closure; returns
// f1 and (optionally) df1/dx, df1/dF.
template <bool kDeriv>
__device__ __forceinline__ double model_f1(const DevParams& p, double x, double F,
                                           double& fx, double& fF) {
    const double iV = 1.0 / p.V;
    const double cT = x * iV;
    const double dT = p.cTin - cT;
    const double ib = 1.0 / p.beta;
    const double cA = p.cAin + dT * ib;
    const double cB = p.cBin + 2.0 * dT * ib;
    const double icT = rcp_pos(cT);
    const double k = p.k0 * exp(-p.EaR * icT);
    const double r = k * cA * cB;
    if (kDeriv) {
        const double dr = r * (p.EaR * icT * icT) - k * ib * (cB + 2.0 * cA);
        fx = -F * iV + p.beta * dr;
        fF = dT;
    }
    return dT * F + p.beta * r * p.V;
}

__device__ __forceinline__ double model_f1(const DevParams& p, double x, double F) {
    double a, b;
    return model_f1<false>(p, x, F, a, b);
}

// Euler-Maruyama sub-step n += h f3 + F sigma sqrt(h) xi.
__device__ __forceinline__ void em_step(const DevParams& p, double k0, double EaR, double n[3],
                                        double F, double h, double sqh, const double xi[3]) {
    double f[3];
    plant_f3(p, k0, EaR, n, F, f);
#pragma unroll
    for (int a = 0; a < 3; ++a) n[a] = n[a] + h * f[a] + F * p.sig[a] * sqh * xi[a];
}

// The three process-noise normals of sub-step `step` (blocks 0 and 1).
__device__ __forceinline__ void process_noise(const DevParams& p, uint32_t step, uint32_t id,
                                              double xi[3]) {
    normal_pair(p.seed, 0, step, id, kTagProcess, xi[0], xi[1]);
    xi[2] = normal_first(p.seed, 1, step, id, kTagProcess);
    const double s = p.noise_scale;
    xi[0] *= s; xi[1] *= s; xi[2] *= s;
}

// ------------------------------------------------------------- setpoint ---
__device__ __forceinline__ double setpoint(const DevParams& p, int i, int istep, double sign) {
    const int ii = p.sp_period > 0 ? i % p.sp_period : i;
    double z = p.sp_z[0];
    for (int j = 1; j < p.n_sp; ++j)
        if (ii >= p.sp_i[j]) z = p.sp_z[j];
    if (p.sp_step_rel != 0.0 && i >= istep) z = z * (1.0 + sign * p.sp_step_rel);
    return z;
}

// ---------------------------------------------------------------- CD-EKF ---
// Prediction over one sampling interval, RK4 with Nc steps on (x, P).
__device__ __forceinline__ void ekf_predict(const DevParams& p, double& x, double& P, double F) {
    const double h = p.Ts / (double)p.Nc;
    const double q = (F * p.sig[2]) * (F * p.sig[2]);
    double X = x, PP = P;
    #pragma unroll 1
    for (int c = 0; c < p.Nc; ++c) {
        double a1, a2, a3, a4, b;
        const double k1x = model_f1<true>(p, X, F, a1, b);
        const double k1P = 2.0 * a1 * PP + q;
        const double k2x = model_f1<true>(p, X + 0.5 * h * k1x, F, a2, b);
        const double k2P = 2.0 * a2 * (PP + 0.5 * h * k1P) + q;
        const double k3x = model_f1<true>(p, X + 0.5 * h * k2x, F, a3, b);
        const double k3P = 2.0 * a3 * (PP + 0.5 * h * k2P) + q;
        const double k4x = model_f1<true>(p, X + h * k3x, F, a4, b);
        const double k4P = 2.0 * a4 * (PP + h * k3P) + q;
        X = X + h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        PP = PP + h / 6.0 * (k1P + 2.0 * k2P + 2.0 * k3P + k4P);
    }
    x = X;
    P = PP;
}

// Filtering with the Joseph-form covariance, C = 1/V.
__device__ __forceinline__ void ekf_update(const DevParams& p, double& x, double& P, double y) {
    const double C = 1.0 / p.V;
    const double e = y - x * C;
    const double Re = p.Rmeas + C * P * C;
    const double K = P * C / Re;
    const double IKC = 1.0 - K * C;
    x = x + K * e;
    P = IKC * P * IKC + K * p.Rmeas * K;
}

// ------------------------------------------------ three-state model ---
// Estimator / OCP model at n_x = 3: eq. (CSTR)'s drift with the nominal
// kinetics; with kDeriv also J = df/dn (row-major) and df/dF.
template <bool kDeriv>
__device__ __forceinline__ void model_f3(const DevParams& p, const double n[3], double F,
                                         double f[3], double J[9], double fF[3]) {
    const double iV = 1.0 / p.V;
    const double cA = n[0] * iV, cB = n[1] * iV, cT = n[2] * iV;
    const double icT = rcp_pos(cT);
    const double k = p.k0 * exp(-p.EaR * icT);
    const double rV = k * cA * cB * p.V;
    const double eA = p.cAin - cA, eB = p.cBin - cB, eT = p.cTin - cT;
    f[0] = eA * F - rV;
    f[1] = eB * F - 2.0 * rV;
    f[2] = eT * F + p.beta * rV;
    if (kDeriv) {
        // d(r V)/dn = (k c_B, k c_A, r V (Ea/R) / (c_T^2 V))
        const double g0 = k * cB, g1 = k * cA, g2 = rV * p.EaR * icT * icT * iV;
        const double dg = -F * iV;
        J[0] = dg - g0;       J[1] = -g1;               J[2] = -g2;
        J[3] = -2.0 * g0;     J[4] = dg - 2.0 * g1;     J[5] = -2.0 * g2;
        J[6] = p.beta * g0;   J[7] = p.beta * g1;       J[8] = dg + p.beta * g2;
        fF[0] = eA;
        fF[1] = eB;
        fF[2] = eT;
    }
}

// Symmetric 3x3 stored as (00, 01, 02, 11, 12, 22).
__device__ __forceinline__ double sym3(const double P[6], int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return P[lo == 0 ? hi : (lo == 1 ? 2 + hi : 5)];
}

// o = J P + P J^T + diag(q) for symmetric P (= M + M^T + diag(q), M = J P).
__device__ __forceinline__ void lyap3(const double J[9], const double P[6], const double q[3],
                                      double o[6]) {
    double M[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            M[3 * a + b] = J[3 * a] * sym3(P, 0, b) + J[3 * a + 1] * sym3(P, 1, b) +
                           J[3 * a + 2] * sym3(P, 2, b);
    o[0] = 2.0 * M[0] + q[0];
    o[1] = M[1] + M[3];
    o[2] = M[2] + M[6];
    o[3] = 2.0 * M[4] + q[1];
    o[4] = M[5] + M[7];
    o[5] = 2.0 * M[8] + q[2];
}

// CD-EKF prediction at n_x = 3, eq. (predictionEquations): RK4 with Nc steps
// on (x, P), dP/dt = J P + P J^T + F^2 diag(sigma^2), J at every stage.
__device__ __forceinline__ void ekf3_predict(const DevParams& p, double x[3], double P[6],
                                             double F) {
    const double h = p.Ts / (double)p.Nc;
    const double h6 = h / 6.0;
    const double q[3] = {(F * p.sig[0]) * (F * p.sig[0]), (F * p.sig[1]) * (F * p.sig[1]),
                         (F * p.sig[2]) * (F * p.sig[2])};
#pragma unroll 1
    for (int c = 0; c < p.Nc; ++c) {
        double kx[3], kP[6], J[9], fF[3], ax[3], aP[6];
        model_f3<true>(p, x, F, kx, J, fF);
        lyap3(J, P, q, kP);
#pragma unroll
        for (int a = 0; a < 3; ++a) ax[a] = kx[a];
#pragma unroll
        for (int e = 0; e < 6; ++e) aP[e] = kP[e];
#pragma unroll
        for (int st = 1; st < 4; ++st) {
            const double cs = st == 3 ? h : 0.5 * h;
            const double w = st == 3 ? 1.0 : 2.0;
            double sx[3], sP[6];
#pragma unroll
            for (int a = 0; a < 3; ++a) sx[a] = x[a] + cs * kx[a];
#pragma unroll
            for (int e = 0; e < 6; ++e) sP[e] = P[e] + cs * kP[e];
            model_f3<true>(p, sx, F, kx, J, fF);
            lyap3(J, sP, q, kP);
#pragma unroll
            for (int a = 0; a < 3; ++a) ax[a] += w * kx[a];
#pragma unroll
            for (int e = 0; e < 6; ++e) aP[e] += w * kP[e];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] += h6 * ax[a];
#pragma unroll
        for (int e = 0; e < 6; ++e) P[e] += h6 * aP[e];
    }
}

// Filtering with the Joseph form, eq. (Josph), C = [0, 0, 1/V]:
// K = P C^T / (R + C P C^T), x += K (y - C x),
// P = (I - K C) P (I - K C)^T + K R K^T.
__device__ __forceinline__ void ekf3_update(const DevParams& p, double x[3], double P[6],
                                            double y) {
    const double C = 1.0 / p.V;
    const double e = y - x[2] * C;
    const double pc[3] = {P[2] * C, P[4] * C, P[5] * C};
    const double iRe = 1.0 / (p.Rmeas + C * pc[2]);
    const double K[3] = {pc[0] * iRe, pc[1] * iRe, pc[2] * iRe};
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] += K[a] * e;
    // T = (I - K C) P: T_ab = P_ab - K_a C P_2b
    double T[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) T[3 * a + b] = sym3(P, a, b) - K[a] * pc[b];
    // P_ab = T_ab - T_a2 C K_b + R K_a K_b
    const double R = p.Rmeas;
    P[0] = T[0] - T[2] * C * K[0] + R * K[0] * K[0];
    P[1] = T[1] - T[2] * C * K[1] + R * K[0] * K[1];
    P[2] = T[2] - T[2] * C * K[2] + R * K[0] * K[2];
    P[3] = T[4] - T[5] * C * K[1] + R * K[1] * K[1];
    P[4] = T[5] - T[5] * C * K[2] + R * K[1] * K[2];
    P[5] = T[8] - T[8] * C * K[2] + R * K[2] * K[2];
}

// --------------------------------------------------------- sample set-up ---
struct Setup {
    uint32_t nid;       // noise id
    int kind, N, L, istep;
    double sign, k0, EaR;
    double n0[3], xhat0, ubar;  // ubar in L/s
};

// Not inlined: it runs once per sample, and keeping its many loop-invariant
// constants out of the persistent kernel's register allocation leaves that
// allocation to the closed loop.
// Set-up of the sample in column `col`: its global id (caller-given or
// id_offset + col), noise id, kind, horizon and length (caller-given or
// drawn), scenario, kinetics and initial state.
//
// Every kernel of the library takes its DevParams as its first argument;
// the set-up reads them in place from the kernel's argument segment
// (constant memory, scalar loads), so no copy of the parameters is made in
// per-lane scratch memory and the kernels keep reading theirs from the
// argument segment too.
typedef const __attribute__((address_space(4))) char* KernargPtr;
__device__ __forceinline__ KernargPtr kernel_args() {
    return (KernargPtr)__builtin_amdgcn_kernarg_segment_ptr();
}
__device__ __noinline__ Setup sample_setup_k(KernargPtr args, int64_t col) {
    const DevParams& p = *(const DevParams*)args;
    Setup s;
    const int64_t sid = p.ids ? p.ids[col] : p.id_offset + col;
    const int64_t nid = p.noise_mod > 0 ? sid % p.noise_mod : sid;
    s.nid = (uint32_t)nid;
    s.kind = p.kind_split >= 0 ? (sid < p.kind_split ? 0 : 1) : p.default_kind;
    s.N = p.N;
    s.L = p.L;
    if (p.n_hc > 0) {
        const double u = philox_uniforms(p.seed, 0, 0, s.nid, kTagScen).u2;
        s.N = p.hc[(int)floor(u * p.n_hc)];
    }
    if (p.L_lo < p.L_hi) {
        const double u = philox_uniforms(p.seed, 1, 0, s.nid, kTagScen).u2;
        s.L = p.L_lo + (int)floor(u * (double)(p.L_hi - p.L_lo + 1));
    }
    if (p.kind_ov) s.kind = p.kind_ov[col];
    if (p.N_ov) s.N = p.N_ov[col];
    if (p.L_ov) s.L = p.L_ov[col];
    if (s.L > p.L_cap) s.L = p.L_cap;
    s.istep = 0;
    s.sign = 0.0;
    if (p.sp_step_rel != 0.0) {
        const double u = philox_uniforms(p.seed, 2, 0, s.nid, kTagScen).u2;
        s.istep = p.sp_step_lo + (int)floor(u * (double)(p.sp_step_hi - p.sp_step_lo + 1));
        const double v = philox_uniforms(p.seed, 3, 0, s.nid, kTagScen).u2;
        s.sign = v < 0.5 ? 1.0 : -1.0;
    }
    s.k0 = p.k0;
    s.EaR = p.EaR;
    if (p.kin_sigma > 0.0) {
        double a, b;
        normal_pair(p.seed, 0, 0, s.nid, kTagKin, a, b);
        s.k0 = p.k0 * exp(p.kin_sigma * a);
        s.EaR = p.EaR * exp(p.kin_sigma * b);
    }
    // steady state of the one-state model at zbar(0)
    const double T = setpoint(p, 0, s.istep, s.sign);
    const double cA = p.cAin + (p.cTin - T) / p.beta;
    const double cB = p.cBin + 2.0 * (p.cTin - T) / p.beta;
    const double r = p.k0 * exp(-p.EaR / T) * cA * cB;
    s.ubar = p.beta * r * p.V / (T - p.cTin);
    if (p.x0_mode == 0) {
        s.n0[0] = p.cAin * p.V;
        s.n0[1] = p.cBin * p.V;
        s.n0[2] = p.cTin * p.V;
        s.xhat0 = p.cTin * p.V;
    } else {
        double a, b;
        normal_pair(p.seed, 0, 0, s.nid, kTagX0, a, b);
        const double c = normal_first(p.seed, 1, 0, s.nid, kTagX0);
        s.n0[0] = cA * p.V * (1.0 + p.x0_rel_std * a);
        s.n0[1] = cB * p.V * (1.0 + p.x0_rel_std * b);
        s.n0[2] = T * p.V * (1.0 + p.x0_rel_std * c);
        s.xhat0 = T * p.V;
    }
    return s;
}
__device__ __forceinline__ Setup sample_setup(int64_t col) {
    return sample_setup_k(kernel_args(), col);
}

// ---------------------------------------------------- single shooting ---
// Lane-tiled vectors: element k of the lane's sample at t[te(k)].
// Objective of the OCP at u + alpha d (d ignored when use_d is false).
//
// With kRec the pass also records, for every control interval k, what the
// adjoint sweep needs, so that the sweep evaluates no model function and
// reads 3 values per interval instead of a per-step tape:
//   rec[(3 k + 0) kTile] = A_k = dx_{k+1}/dx_k,
//   rec[(3 k + 1) kTile] = B_k = dx_{k+1}/du_k (per mL/min),
//   rec[(3 k + 2) kTile] = c_k = d(stage cost at x_{k+1})/dx_{k+1}.
// A_k and B_k are the derivatives of the interval's RK4^{Nc} map, carried
// forward through the stages with df1/dx and df1/dF (which share f1's
// exponential and division); they sit beside the state recursion, not on it.
template <bool kRec>
__device__ __forceinline__ double ocp_shoot(const DevParams& p, int N, double x0, int i0,
                                            int istep, double sign, const double* u,
                                            const double* d, double alpha, bool use_d,
                                            double* rec) {
    const double h = p.Ts / (double)p.Nc;
    const double h2 = 0.5 * h, h6 = h / 6.0;
    const double iV = 1.0 / p.V;
    double x = x0, phi = 0.0;
    double un = u[0], dn = use_d ? d[0] : 0.0;   // interval k's input, loaded one interval ahead
#pragma unroll 1
    for (int k = 0; k < N; ++k) {
        double uk = un;
        if (use_d) uk = uk + alpha * dn;
        if (k + 1 < N) {
            un = u[te(k + 1)];
            if (use_d) dn = d[te(k + 1)];
        }
        const double F = uk / kMlMinPerLs;
        double A = 1.0, B = 0.0;
#pragma unroll 1
        for (int c = 0; c < p.Nc; ++c) {
            if (kRec) {
                double a0, a1, a2, a3, b0, b1, b2, b3;
                const double k1 = model_f1<true>(p, x, F, a0, b0);
                const double k2 = model_f1<true>(p, x + h2 * k1, F, a1, b1);
                const double k3 = model_f1<true>(p, x + h2 * k2, F, a2, b2);
                const double k4 = model_f1<true>(p, x + h * k3, F, a3, b3);
                // derivatives of the step's stages w.r.t. its start state
                const double t2 = a1 * (1.0 + h2 * a0);
                const double t3 = a2 * (1.0 + h2 * t2);
                const double t4 = a3 * (1.0 + h * t3);
                const double Am = 1.0 + h6 * (a0 + 2.0 * t2 + 2.0 * t3 + t4);
                // ... and w.r.t. F
                const double s2 = b1 + a1 * h2 * b0;
                const double s3 = b2 + a2 * h2 * s2;
                const double s4 = b3 + a3 * h * s3;
                const double Bm = h6 * (b0 + 2.0 * s2 + 2.0 * s3 + s4);
                B = Am * B + Bm;
                A = Am * A;
                x = x + h6 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
            } else {
                const double k1 = model_f1(p, x, F);
                const double k2 = model_f1(p, x + h2 * k1, F);
                const double k3 = model_f1(p, x + h2 * k2, F);
                const double k4 = model_f1(p, x + h * k3, F);
                x = x + h6 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
            }
        }
        const double ez = x * iV - setpoint(p, i0 + 1 + k, istep, sign);
        phi += p.Qz * ez * ez * p.Ts;
        if (kRec) {
            double* const r = rec + (int64_t)(3 * k) * kTile;
            r[0] = A;
            r[kTile] = B / kMlMinPerLs;
            r[2 * kTile] = p.Qz * 2.0 * ez * iV * p.Ts;
        }
    }
    return phi;
}

// Record width of one control interval: the one-state model keeps
// (A_k, B_k, c_k), the three-state model A_k (3x3, row-major), B_k (3) and
// the one non-zero entry of c_k (the stage cost depends on n_T only).
template <int NX>
constexpr int rec_width() { return NX == 3 ? 13 : 3; }

// ocp_shoot with the three-state model from x0 (3 values).  With kRec, for
// every interval k the record rec[(13 k + j) kTile] holds
//   j = 0..8:  A_k = dx_{k+1}/dx_k (row-major),
//   j = 9..11: B_k = dx_{k+1}/du_k (per mL/min),
//   j = 12:    c_k = d(stage cost at x_{k+1})/dn_{T,k+1}.
// The tangents of x_k and of F are carried through every RK4 stage beside
// the state (J_s times the stage's tangent), the form of the forward pass.
template <bool kRec>
__device__ __forceinline__ double ocp_shoot3(const DevParams& p, int N, const double (&x0)[3],
                                             int i0, int istep, double sign, const double* u,
                                             const double* d, double alpha, bool use_d,
                                             double* rec) {
    const double h = p.Ts / (double)p.Nc;
    const double h2 = 0.5 * h, h6 = h / 6.0;
    const double iV = 1.0 / p.V;
    double x[3] = {x0[0], x0[1], x0[2]};
    double phi = 0.0;
    double un = u[0], dn = use_d ? d[0] : 0.0;
#pragma unroll 1
    for (int k = 0; k < N; ++k) {
        double uk = un;
        if (use_d) uk = uk + alpha * dn;
        if (k + 1 < N) {
            un = u[te(k + 1)];
            if (use_d) dn = d[te(k + 1)];
        }
        const double F = uk / kMlMinPerLs;
        double A[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
        double B[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
        for (int c = 0; c < p.Nc; ++c) {
            if (kRec) {
                double kx[3], J[9], fF[3], ax[3], aA[9], aB[3], dA[9], dB[3];
                model_f3<true>(p, x, F, kx, J, fF);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        dA[3 * a + b] = J[3 * a] * A[b] + J[3 * a + 1] * A[3 + b] +
                                        J[3 * a + 2] * A[6 + b];
                    dB[a] = J[3 * a] * B[0] + J[3 * a + 1] * B[1] + J[3 * a + 2] * B[2] + fF[a];
                    ax[a] = kx[a];
                    aB[a] = dB[a];
                }
#pragma unroll
                for (int e = 0; e < 9; ++e) aA[e] = dA[e];
#pragma unroll
                for (int st = 1; st < 4; ++st) {
                    const double cs = st == 3 ? h : h2;
                    const double w = st == 3 ? 1.0 : 2.0;
                    double sx[3], sA[9], sB[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        sx[a] = x[a] + cs * kx[a];
                        sB[a] = B[a] + cs * dB[a];
                    }
#pragma unroll
                    for (int e = 0; e < 9; ++e) sA[e] = A[e] + cs * dA[e];
                    model_f3<true>(p, sx, F, kx, J, fF);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
#pragma unroll
                        for (int b = 0; b < 3; ++b)
                            dA[3 * a + b] = J[3 * a] * sA[b] + J[3 * a + 1] * sA[3 + b] +
                                            J[3 * a + 2] * sA[6 + b];
                        dB[a] = J[3 * a] * sB[0] + J[3 * a + 1] * sB[1] + J[3 * a + 2] * sB[2] +
                                fF[a];
                        ax[a] += w * kx[a];
                        aB[a] += w * dB[a];
                    }
#pragma unroll
                    for (int e = 0; e < 9; ++e) aA[e] += w * dA[e];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    x[a] += h6 * ax[a];
                    B[a] += h6 * aB[a];
                }
#pragma unroll
                for (int e = 0; e < 9; ++e) A[e] += h6 * aA[e];
            } else {
                double kx[3], ax[3], sx[3], J[9], fF[3];
                model_f3<false>(p, x, F, kx, J, fF);
#pragma unroll
                for (int a = 0; a < 3; ++a) ax[a] = kx[a];
#pragma unroll
                for (int st = 1; st < 4; ++st) {
                    const double cs = st == 3 ? h : h2;
                    const double w = st == 3 ? 1.0 : 2.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) sx[a] = x[a] + cs * kx[a];
                    model_f3<false>(p, sx, F, kx, J, fF);
#pragma unroll
                    for (int a = 0; a < 3; ++a) ax[a] += w * kx[a];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) x[a] += h6 * ax[a];
            }
        }
        const double ez = x[2] * iV - setpoint(p, i0 + 1 + k, istep, sign);
        phi += p.Qz * ez * ez * p.Ts;
        if (kRec) {
            double* const r = rec + (int64_t)(13 * k) * kTile;
#pragma unroll
            for (int e = 0; e < 9; ++e) r[e * kTile] = A[e];
#pragma unroll
            for (int a = 0; a < 3; ++a) r[(9 + a) * kTile] = B[a] / kMlMinPerLs;
            r[12 * kTile] = p.Qz * 2.0 * ez * iV * p.Ts;
        }
    }
    return phi;
}

// The sums of the scaled KKT test, eq. (convergence), over a lane's sample:
// s1 = sum |pi_l| + |pi_u| and rmax = max |g - pi_l + pi_u| (bad: NaN seen).
struct KktSums {
    double s1, rmax;
    bool bad;
};
__device__ __forceinline__ void kkt_add(KktSums& r, double g, double pl, double pu) {
    r.s1 += fabs(pl) + fabs(pu);
    const double v = fabs(g - pl + pu);
    r.bad |= (v != v);
    r.rmax = v > r.rmax ? v : r.rmax;
}

// Plain forward sensitivities S_j = dx/du_j: the state is integrated again
// from x0 with the inputs u, and the tangents of every u_j, j <= k, are
// carried through each RK4 step with the stage derivatives (NMAX register
// slots, unrolled); dphi/du_j accumulates in the lane tile `acc` (element j
// at acc[te(j)]).  Returns the sums of the next KKT test with the
// multipliers pil, piu.
template <int NMAX>
__device__ __forceinline__ KktSums ocp_grad_fwd(const DevParams& p, int N, double x0, int i0,
                                                int istep, double sign, const double* u,
                                                double* g, double* y, double* acc,
                                                const double* pil, const double* piu) {
    const double h = p.Ts / (double)p.Nc;
    const double h2 = 0.5 * h, h6 = h / 6.0;
    const double iV = 1.0 / p.V;
    const double dF = 1.0 / kMlMinPerLs;
    double S[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) S[j] = 0.0;
#pragma unroll 1
    for (int j = 0; j < N; ++j) acc[te(j)] = 0.0;
    double x = x0;
#pragma unroll 1
    for (int k = 0; k < N; ++k) {
        const double F = u[te(k)] / kMlMinPerLs;
#pragma unroll 1
        for (int c = 0; c < p.Nc; ++c) {
            double a[4], b[4];
            const double k1 = model_f1<true>(p, x, F, a[0], b[0]);
            const double k2 = model_f1<true>(p, x + h2 * k1, F, a[1], b[1]);
            const double k3 = model_f1<true>(p, x + h2 * k2, F, a[2], b[2]);
            const double k4 = model_f1<true>(p, x + h * k3, F, a[3], b[3]);
            x = x + h6 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
#pragma unroll
            for (int j = 0; j < NMAX; ++j) {
                if (j <= k) {
                    const double src = (j == k) ? dF : 0.0;
                    const double d1 = a[0] * S[j] + b[0] * src;
                    const double d2 = a[1] * (S[j] + h2 * d1) + b[1] * src;
                    const double d3 = a[2] * (S[j] + h2 * d2) + b[2] * src;
                    const double d4 = a[3] * (S[j] + h * d3) + b[3] * src;
                    S[j] = S[j] + h6 * (d1 + 2.0 * d2 + 2.0 * d3 + d4);
                }
            }
        }
        const double ez = x * iV - setpoint(p, i0 + 1 + k, istep, sign);
        const double dphidx = p.Qz * 2.0 * ez * iV * p.Ts;
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (j <= k) acc[te(j)] += dphidx * S[j];
    }
    KktSums r{0.0, 0.0, false};
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
        const double gj = acc[te(j)];
        if (y) y[te(j)] = gj - g[te(j)];
        g[te(j)] = gj;
        kkt_add(r, gj, pil[te(j)], piu[te(j)]);
    }
    return r;
}

}  // namespace mccl
