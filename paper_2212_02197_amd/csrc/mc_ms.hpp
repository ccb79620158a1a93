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
// One-state model (the paper's case study).
//
// Layout: one sample per segment of G lanes, stage k on the segment's lane k
// (G = 16, 32 or 64 by horizon class: four, two or one sample per
// wavefront; see Seg below).  Every stage quantity of the NLP and of the QP
// is one register per lane, so the SQP runs without any workspace in
// memory:
//   * the interval maps (values and tangents), the stage costs, the
//     gradient of the Lagrangian, the block BFGS updates and the
//     interior point's element-wise steps run on all stages at once, with
//     a stage's neighbours fetched by lane shifts;
//   * the stage recursions of the Riccati solve are parallel prefix scans
//     over the segment's lanes (log2 G steps): the scalar Riccati
//     recursion of the factor P_k is a linear-fractional map of P_{k+1},
//     composed as 2x2 matrices, and the recursions of the Riccati vector
//     and of the forward state steps are affine maps;
//   * sums and maxima over the stages are segment reductions.
// Only the feasible start of each OCP, where the states follow the inputs
// through the model, runs the stages one after another.
//
// Decision vector xi = [u_0, x_1, u_1, ..., u_{N-1}, x_N]; x_0 = x-hat_{i|i}.
// Constraints c_k = F(x_k, u_k) - x_{k+1} (F: RK4 with Nc steps over Ts,
// u in mL/min); Lagrangian L = f - lambda^T c - pi_l^T (u - u_min)
// - pi_u^T (u_max - u); f = phi of the Regulator section, stage costs on
// x_1..x_N.  Lane k holds u_k and the state after interval k, x_{k+1}
// (value, multiplier of c_k, df/dx_{k+1}, its Hessian entry W_{x_{k+1}}),
// and of the Hessian block {x_k, u_k} the entries W_{x_k u_k}, W_{u_k u_k}.
#pragma once
#include "mc_kernels.hpp"

#ifndef MC_MS_WAVES_PER_EU
#define MC_MS_WAVES_PER_EU 2   // wavefronts per SIMD the kernel is built for
#endif

namespace mccl {

struct MsWork {
    const int64_t* pos;  // sample positions, one per group
    int64_t n_pos;
    int n_groups;
    int* queue;          // next group; starts at the chunk's first group
    const int* qhi;      // end of the chunk's groups (device), or null: n_groups
};

// --------------------------------------------------------- lane shifts ---
// Data-parallel primitives (DPP) move values between lanes inside the VALU,
// with no LDS round trip.  Every lane must be active: none of these sits
// inside a lane condition.
// v of lane l - 1 (lane 0: `fill`, or 0) and of lane l + 1 (lanes >= n - 1:
// `fill`): the wavefront shifts by one lane.
__device__ __forceinline__ double lane_prev(double v) {
    return dpp_z<0x138>(v);   // wave_shr:1
}
__device__ __forceinline__ double lane_prev(double v, double fill) {
    return dpp_d<0x138, 0xf>(fill, v);
}
__device__ __forceinline__ double lane_next(double v, double fill, int n) {
    const double w = dpp_z<0x130>(v);   // wave_shl:1
    return (int)threadIdx.x + 1 < n ? w : fill;
}
// A row shift by d (CTRL) of v: lanes without a source in the row read 1.0
// when ONE is set, else 0.  The low words, and the high word for 0, take
// bound_ctrl (a lane without a source writes 0); the high word of 1.0 is
// preset in the destination, which a lane without a source leaves as it is,
// so no lane mask and no select is needed.
template <int CTRL, bool ONE>
__device__ __forceinline__ double dpp_row(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = ONE ? __builtin_amdgcn_update_dpp(0x3ff00000, __double2hiint(v), CTRL, 0xf, 0xf, false)
                       : __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Inclusive scans over the 64 lanes of the wavefront of maps composed by
// `after(f, g)` = f o g (lanes past a sample's stages carry the identity, so
// a scan over all lanes is exact for any horizon).  Prefix: lane k ends with
// f_k o f_{k-1} o ... o f_0; suffix: lane k ends with f_k o f_{k+1} o ....
// Within each 16-lane row the scan takes row shifts by 1, 2, 4 and 8
// (lanes without a source in the row compose with the identity).  Across
// rows, a prefix takes the row broadcasts of lanes 15 and 31; a suffix
// reads the row totals (lanes 16, 32, 48) and composes each row with the
// totals of the rows after it.
template <class T>
struct DppOps;
template <class T, class After>
__device__ __forceinline__ T scan_prefix(T f, T id, After after) {
    f = after(f, DppOps<T>::template row<0x111>(f));      // row_shr:1
    f = after(f, DppOps<T>::template row<0x112>(f));
    f = after(f, DppOps<T>::template row<0x114>(f));
    f = after(f, DppOps<T>::template row<0x118>(f));
    f = after(f, DppOps<T>::template mov<0x142, 0xa>(id, f));   // row_bcast:15
    f = after(f, DppOps<T>::template mov<0x143, 0xc>(id, f));   // row_bcast:31
    return f;
}
template <class T, class After>
__device__ __forceinline__ T scan_suffix(T f, T id, After after) {
    f = after(f, DppOps<T>::template row<0x101>(f));      // row_shl:1
    f = after(f, DppOps<T>::template row<0x102>(f));
    f = after(f, DppOps<T>::template row<0x104>(f));
    f = after(f, DppOps<T>::template row<0x108>(f));
    {
        const int row = threadIdx.x >> 4;
        const T t1 = DppOps<T>::readlane(f, 16), t3 = DppOps<T>::readlane(f, 48);
        const T s2 = after(DppOps<T>::readlane(f, 32), t3);   // rows 2..3
        f = after(f, row == 0 ? after(t1, s2) : row == 1 ? s2 : row == 2 ? t3 : id);
    }
    return f;
}

// Affine maps x -> a x + b.
struct Aff {
    double a, b;
};
template <>
struct DppOps<Aff> {
    template <int CTRL, int ROWMASK>
    __device__ static __forceinline__ Aff mov(Aff old, Aff v) {
        return Aff{dpp_d<CTRL, ROWMASK>(old.a, v.a), dpp_d<CTRL, ROWMASK>(old.b, v.b)};
    }
    template <int CTRL>
    __device__ static __forceinline__ Aff row(Aff v) {
        return Aff{dpp_row<CTRL, true>(v.a), dpp_row<CTRL, false>(v.b)};
    }
    __device__ static __forceinline__ Aff readlane(Aff v, int l) {
        return Aff{readlane_d(v.a, l), readlane_d(v.b, l)};
    }
};
__device__ __forceinline__ Aff aff_after(Aff f, Aff g) {
    return Aff{f.a * g.a, fma(f.a, g.b, f.b)};
}

// Linear-fractional maps P -> (m00 P + m01) / (m10 P + m11) as 2x2
// matrices; a map is unchanged by a scale factor, so each matrix is
// rescaled by a power of two (exact) to keep its entries near 1.
struct Mob {
    double m00, m01, m10, m11;
};
__device__ __forceinline__ Mob mob_norm(Mob m) {
    const double mx = fmax(fmax(fabs(m.m00), fabs(m.m01)), fmax(fabs(m.m10), fabs(m.m11)));
    int e = 0;
    (void)frexp(mx, &e);
    if (!(mx > 0.0) || !isfinite(mx)) e = 0;
    return Mob{ldexp(m.m00, -e), ldexp(m.m01, -e), ldexp(m.m10, -e), ldexp(m.m11, -e)};
}
template <>
struct DppOps<Mob> {
    template <int CTRL, int ROWMASK>
    __device__ static __forceinline__ Mob mov(Mob old, Mob v) {
        return Mob{dpp_d<CTRL, ROWMASK>(old.m00, v.m00), dpp_d<CTRL, ROWMASK>(old.m01, v.m01),
                   dpp_d<CTRL, ROWMASK>(old.m10, v.m10), dpp_d<CTRL, ROWMASK>(old.m11, v.m11)};
    }
    template <int CTRL>
    __device__ static __forceinline__ Mob row(Mob v) {
        return Mob{dpp_row<CTRL, true>(v.m00), dpp_row<CTRL, false>(v.m01),
                   dpp_row<CTRL, false>(v.m10), dpp_row<CTRL, true>(v.m11)};
    }
    __device__ static __forceinline__ Mob readlane(Mob v, int l) {
        return Mob{readlane_d(v.m00, l), readlane_d(v.m01, l), readlane_d(v.m10, l), readlane_d(v.m11, l)};
    }
};
// m o g as the matrix product m g (applied to a vector, g acts first).  A
// product of k rescaled matrices (largest entry below 1) has entries below
// 2^(k-1), so the scans rescale only the row totals (16 maps) and the
// compositions across rows stay far inside the FP64 range.  Rescaling by a
// power of two is exact and the map is unchanged by it, so where it happens
// does not change P.
__device__ __forceinline__ Mob mob_mul(Mob m, Mob g) {
    return Mob{fma(m.m00, g.m00, m.m01 * g.m10), fma(m.m00, g.m01, m.m01 * g.m11),
               fma(m.m10, g.m00, m.m11 * g.m10), fma(m.m10, g.m01, m.m11 * g.m11)};
}
__device__ __forceinline__ Mob mob_after(Mob m, Mob g) {
    return mob_norm(mob_mul(m, g));
}
__device__ __forceinline__ Mob mob_after_raw(Mob m, Mob g) {
    return mob_mul(m, g);
}
// Suffix scan: lane k ends with M_k M_{k+1} ....
__device__ __forceinline__ Mob scan_mob_suffix(Mob m) {
    const Mob id{1.0, 0.0, 0.0, 1.0};
    m = mob_after_raw(m, DppOps<Mob>::row<0x101>(m));      // row_shl:1
    m = mob_after_raw(m, DppOps<Mob>::row<0x102>(m));
    m = mob_after_raw(m, DppOps<Mob>::row<0x104>(m));
    m = mob_after(m, DppOps<Mob>::row<0x108>(m));
    const int row = threadIdx.x >> 4;
    const Mob t1 = DppOps<Mob>::readlane(m, 16), t3 = DppOps<Mob>::readlane(m, 48);
    const Mob s2 = mob_after_raw(DppOps<Mob>::readlane(m, 32), t3);
    return mob_after_raw(m, row == 0 ? mob_after_raw(t1, s2) : row == 1 ? s2 : row == 2 ? t3 : id);
}

// ------------------------------------------------------------ segments ---
// A wavefront holds 64 / G samples, sample j on the segment of lanes
// [jG, (j + 1)G), stage k of a sample on lane jG + k (G = 16, 32 or 64:
// horizons up to 16 take a 16-lane row each, up to 32 two rows).  Every
// lane shift, broadcast, reduction and scan below stays inside a segment,
// so a segment whose lanes are inactive (its sample done, or at another
// point of its control flow) never feeds another segment.
template <int G>
struct Seg {
    static_assert(G == 16 || G == 32 || G == 64, "segments of 16, 32 or 64 lanes");
    __device__ static __forceinline__ int k() { return (int)threadIdx.x & (G - 1); }
    __device__ static __forceinline__ int base() { return (int)threadIdx.x & (64 - G); }
    // v of stage k - 1 (stage 0: 0, or `fill`); of stage k + 1 (stages
    // >= n - 1: `fill`)
    __device__ static __forceinline__ double prev(double v) {
        if constexpr (G == 16) {
            return dpp_z<0x111>(v);   // row_shr:1: a row is a segment
        } else {
            const double w = dpp_z<0x138>(v);   // wave_shr:1
            if constexpr (G == 64) return w;
            else return k() == 0 ? 0.0 : w;
        }
    }
    __device__ static __forceinline__ double prev(double v, double fill) {
        if constexpr (G == 16) {
            return dpp_d<0x111, 0xf>(fill, v);
        } else {
            const double w = dpp_d<0x138, 0xf>(fill, v);
            if constexpr (G == 64) return w;
            else return k() == 0 ? fill : w;
        }
    }
    __device__ static __forceinline__ double next(double v, double fill, int n) {
        const double w = G == 16 ? dpp_z<0x101>(v) : dpp_z<0x130>(v);   // row_shl:1 / wave_shl:1
        return k() + 1 < n ? w : fill;
    }
    // v of stage j of this segment (j the same on the whole segment; at
    // G = 64 the same on the whole wavefront)
    __device__ static __forceinline__ double bcast(double v, int j) {
        if constexpr (G == 64) return readlane_d(v, j);
        else return __shfl(v, base() + j, 64);
    }
    // sum, maximum, minimum over the segment, in every lane of it: rows by
    // DPP, the two rows of a 32-lane segment by the gfx950 row-pair swap
    template <typename Op>
    __device__ static __forceinline__ double fold(double v, Op op) {
        v = op(v, dpp_z<0xB1>(v));    // quad_perm [1,0,3,2]
        v = op(v, dpp_z<0x4E>(v));    // quad_perm [2,3,0,1]
        v = op(v, dpp_z<0x124>(v));   // row_ror:4
        v = op(v, dpp_z<0x128>(v));   // row_ror:8
        if constexpr (G == 32) {
            const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
            const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
            v = op(__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1]));
        }
        return v;
    }
    __device__ static __forceinline__ double sum(double v) {
        if constexpr (G == 64) return wave_sum(v);
        else return fold(v, [](double a, double b) { return a + b; });
    }
    __device__ static __forceinline__ double max(double v) {
        if constexpr (G == 64) return wave_max(v);
        else return fold(v, [](double a, double b) { return fmax(a, b); });
    }
    __device__ static __forceinline__ double min(double v) {
        if constexpr (G == 64) return wave_min(v);
        else return fold(v, [](double a, double b) { return fmin(a, b); });
    }
    // some lane of the segment has c
    __device__ static __forceinline__ bool any(bool c) {
        const uint64_t m = __ballot(c);
        if constexpr (G == 64) return m != 0;
        else return ((m >> base()) & ((1ull << G) - 1)) != 0;
    }
    // the bit mask of lanes k < n of the segment with c (bit k)
    __device__ static __forceinline__ uint64_t mask(bool c) {
        const uint64_t m = __ballot(c);
        if constexpr (G == 64) return m;
        else return (m >> base()) & ((1ull << G) - 1);
    }
    // inclusive prefix / suffix scans of affine maps inside the segment
    __device__ static __forceinline__ Aff scan_prefix_aff(Aff f) {
        const Aff id{1.0, 0.0};
        if constexpr (G == 64) return scan_prefix(f, id, aff_after);
        f = aff_after(f, DppOps<Aff>::row<0x111>(f));
        f = aff_after(f, DppOps<Aff>::row<0x112>(f));
        f = aff_after(f, DppOps<Aff>::row<0x114>(f));
        f = aff_after(f, DppOps<Aff>::row<0x118>(f));
        if constexpr (G == 32) f = aff_after(f, DppOps<Aff>::mov<0x142, 0xa>(id, f));   // row_bcast:15
        return f;
    }
    template <class T, class After>
    __device__ static __forceinline__ T suffix_rows(T f, T id, After after) {
        f = after(f, DppOps<T>::template row<0x101>(f));
        f = after(f, DppOps<T>::template row<0x102>(f));
        f = after(f, DppOps<T>::template row<0x104>(f));
        f = after(f, DppOps<T>::template row<0x108>(f));
        if constexpr (G == 32) {
            // row 0 composes with row 1's total (lane 16), row 2 with row 3's (lane 48)
            const int row = threadIdx.x >> 4;
            const T t1 = DppOps<T>::readlane(f, 16), t3 = DppOps<T>::readlane(f, 48);
            f = after(f, row == 0 ? t1 : row == 2 ? t3 : id);
        }
        return f;
    }
    __device__ static __forceinline__ Aff scan_suffix_aff(Aff f) {
        if constexpr (G == 64) return scan_suffix(f, Aff{1.0, 0.0}, aff_after);
        else return suffix_rows(f, Aff{1.0, 0.0}, aff_after);
    }
    __device__ static __forceinline__ Mob scan_suffix_mob(Mob m) {
        if constexpr (G == 64) return scan_mob_suffix(m);
        if constexpr (G == 16) {
            m = mob_after_raw(m, DppOps<Mob>::row<0x101>(m));
            m = mob_after_raw(m, DppOps<Mob>::row<0x102>(m));
            m = mob_after_raw(m, DppOps<Mob>::row<0x104>(m));
            return mob_after_raw(m, DppOps<Mob>::row<0x108>(m));
        } else {
            m = mob_after_raw(m, DppOps<Mob>::row<0x101>(m));
            m = mob_after_raw(m, DppOps<Mob>::row<0x102>(m));
            m = mob_after_raw(m, DppOps<Mob>::row<0x104>(m));
            m = mob_after(m, DppOps<Mob>::row<0x108>(m));
            // row 0 composes with row 1's total (lane 16), row 2 with row 3's (lane 48)
            const int row = threadIdx.x >> 4;
            const Mob t1 = DppOps<Mob>::readlane(m, 16), t3 = DppOps<Mob>::readlane(m, 48);
            return mob_after_raw(m, row == 0 ? t1 : row == 2 ? t3 : Mob{1.0, 0.0, 0.0, 1.0});
        }
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

// 1/a for finite nonzero a: the hardware estimate and two Newton steps
// (each doubles the correct bits; within an ulp or two of the quotient).
// Where a may be 0 or infinite the interior point divides instead.
__device__ __forceinline__ double rcp_nr(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

// Structured QP, eq. (QP-subproblem), at the current SQP iterate:
//   min 1/2 dxi^T W dxi + sum_k fx_k dx_{k+1}
//   s.t. dx_{k+1} = A_k dx_k + B_k du_k + c_k (dx_0 = 0),
//        u_min - u_k <= du_k <= u_max - u_k,
// by a Mehrotra predictor-corrector primal-dual interior point: slacks
// t_l = du - lo, t_u = hi - du kept positive, bound multipliers nu > 0,
// fraction to the boundary 0.995 with separate primal and dual step
// lengths.  Each Newton system is the equality-constrained stage QP with
// R~_k = W_uu,k + nu_l/t_l + nu_u/t_u, solved by the Riccati recursion:
// backwards P_N = W_{x_N}, H_uu,k = R~_k + B_k^2 P_{k+1},
// H_ux,k = W_{x_k u_k} + B_k P_{k+1} A_k, K_k = -H_ux,k / H_uu,k,
// P_k = W_{x_k} + A_k^2 P_{k+1} + H_ux,k K_k (the factor, shared by
// predictor and corrector), the vector p_k = r_x,k + (A_k + B_k K_k) p_{k+1}
// + K_k r~_u,k and k_k = -(r~_u,k + B_k p_{k+1}) / H_uu,k; forwards
// du_k = K_k dx_k + k_k, dx_{k+1} = A_k dx_k + B_k du_k; the equality
// multipliers follow as mu_k = -(P_{k+1} dx_{k+1} + p_{k+1}).  Eliminating
// H_ux and H_uu, P_k = (alpha_k P_{k+1} + beta_k) / (B_k^2 P_{k+1} + R~_k)
// with alpha_k = W_{x_k} B_k^2 + A_k^2 R~_k - 2 W_{x_k u_k} A_k B_k and
// beta_k = W_{x_k} R~_k - W_{x_k u_k}^2 (both >= 0 for a positive definite
// block), which the lanes compose by a scan (each map divided by R~_k).  Start strictly inside the
// box, 1e-2 of its width from the nearer bound, nu = 1, the states from
// the dynamics.  Stop: stationarity residual <= 1e-12 (1 + |fx| + |W dxi|)
// and mean complementarity <= 1e-14 (1 + |fx|) (infinity norms), or
// ipm_max_iter iterations.  Returns 0 converged, 1 iteration cap, -1 an
// H_uu <= 0 (W not positive definite).  Lane k (k < N) passes its stage's
// data and receives du_k, dx_{k+1}, mu_k and the bound multipliers; lanes
// k >= N pass u = (u_min + u_max)/2, A = B = c = df/dx = 0 (no stage).
struct MsStage {
    double U, A, B, C, FX, WXX, WXU, WUU;
};
struct MsQpOut {
    double du, dx, mu, nl, nu;
};

template <int G>
__device__ __forceinline__ int ms_qp_lanes(const DevParams& p, int N, MsStage s,
                                        MsQpOut& o, int& iters) {
    using S = Seg<G>;
    const int lane = S::k();   // the stage of this lane
    const bool act = lane < N;
    const bool hasx = act && lane >= 1;   // the stage has a state x_k in the NLP
    const double lo = p.umin - s.U, hi = p.umax - s.U;
    const double wxu = lane >= 1 ? s.WXU : 0.0;
    const double wxp = S::prev(s.WXX);    // W_{x_k}
    const double fxp = S::prev(s.FX);     // df/dx_k
    const double PN = S::bcast(s.WXX, N - 1);  // W_{x_N}
    const double fxN = S::bcast(s.FX, N - 1);
    double du, nl = 1.0, nu = 1.0, mu = 0.0, dx;
    {
        const double dl = 1e-2 * (hi - lo);
        du = 0.0;
        if (du < lo + dl) du = lo + dl;
        if (du > hi - dl) du = hi - dl;
        double a = act ? s.A : 1.0, b = act ? fma(s.B, du, s.C) : 0.0;
        {
            const Aff r = S::scan_prefix_aff(Aff{a, b});
            a = r.a;
            b = r.b;
        }
        dx = b;   // dx_{k+1}; dx_0 = 0
    }
    const double gsc = S::max(act ? fabs(s.FX) : 0.0);
    const double inv2N = 1.0 / (2.0 * N);
    #pragma unroll 1
    for (int it = 0;; ++it) {
        // residuals of the current point
        const double dxk = S::prev(dx);   // dx_k (dx_0 = 0)
        const double mup = S::prev(mu);   // mu_{k-1}
        const double tl = du - lo, tu = hi - du;
        const double itl = 1.0 / tl, itu = 1.0 / tu;   // IEEE: a zero slack gives infinity
        const double wdu = s.WUU * du + wxu * dxk;
        const double ru = wdu - mu * s.B - nl + nu;
        const double Rt = s.WUU + nl * itl + nu * itu;
        const double rt = ru + nl - nu;
        const double wdx = wxp * dxk + wxu * du;
        const double rx = wdx + fxp - mu * s.A + mup;
        const double dxN = S::bcast(dx, N - 1), muN = S::bcast(mu, N - 1);
        const double rxN = PN * dxN + fxN + muN;
        const double comp = S::sum(act ? tl * nl + tu * nu : 0.0);
        // the stopping test reads the residuals alone: it comes before the
        // factorisation, which a converged or capped iterate does not need.
        // It needs both its parts, so the residual maxima are taken only
        // once the complementarity part holds (which it does in the last
        // iterations only; its sum is the same on the whole segment)
        const double muc = comp * inv2N;
        if (muc <= 1e-14 * (1.0 + gsc)) {
            double rl = act ? fabs(ru) : 0.0, wl = act ? fabs(wdu) : 0.0;
            if (hasx) {
                rl = fmax(rl, fabs(rx));
                wl = fmax(wl, fabs(wdx));
            }
            const double rmax = fmax(fabs(rxN), S::max(rl));
            const double wd = fmax(fabs(PN * dxN), S::max(wl));
            if (rmax <= 1e-12 * (1.0 + gsc + wd)) {
                iters = it;
                o = MsQpOut{du, dx, mu, nl, nu};
                return 0;
            }
        }
        if (it == p.ipm_max_iter) {
            iters = it;
            o = MsQpOut{du, dx, mu, nl, nu};
            return 1;
        }
        // Riccati factor: lane k composes the maps of stages k+1..N-1
        // (divided by R~_k: a slack that has reached 0 in floating point makes
        // R~_k infinite, and the map tends to P -> A_k^2 P + W_{x_k})
        Mob m{1.0, 0.0, 0.0, 1.0};
        if (hasx) {
            const double rR = 1.0 / Rt;
            m = Mob{fma(s.A, s.A, (wxp * s.B * s.B - 2.0 * wxu * s.A * s.B) * rR), fma(-wxu * wxu, rR, wxp),
                    s.B * s.B * rR, 1.0};
        }
        m = Mob{S::next(m.m00, 1.0, N), S::next(m.m01, 0.0, N), S::next(m.m10, 0.0, N),
                S::next(m.m11, 1.0, N)};
        m = S::scan_suffix_mob(mob_norm(m));
        const double Pn = (m.m00 * PN + m.m01) * rcp_nr(m.m10 * PN + m.m11);   // P_{k+1}
        const double Huu = Rt + s.B * s.B * Pn;
        if (S::any(act && !(Huu > 0.0))) {
            iters = it;
            return -1;
        }
        const double hinv = 1.0 / Huu;
        const double K = -(wxu + s.B * Pn * s.A) * hinv;   // K_0 is not used
        const double g = lane >= 1 ? fma(s.B, K, s.A) : 0.0;   // closed-loop gain of stage k
        // predictor's Riccati vector: lane k composes p-maps of stages k+1..N-1
        double va = hasx ? g : 1.0, vb = hasx ? fma(K, rt, rx) : 0.0;
        va = S::next(va, 1.0, N);
        vb = S::next(vb, 0.0, N);
        {
            const Aff r = S::scan_suffix_aff(Aff{va, vb});
            va = r.a;
            vb = r.b;
        }
        const double e = fma(va, rxN, vb);      // p_{k+1}
        const double kf = -(rt + s.B * e) * hinv;
        // forward predictor: affine step and its lengths
        double fa = act ? g : 1.0, fb = act ? s.B * kf : 0.0;
        {
            const Aff r = S::scan_prefix_aff(Aff{fa, fb});
            fa = r.a;
            fb = r.b;
        }
        // (lane shifts run on the whole wavefront, outside any lane condition)
        const double dxa = S::prev(fb);    // affine dx_k
        const double dua = (lane >= 1 ? K * dxa : 0.0) + kf;
        const double dnla = -nl - nl * dua * itl, dnua = -nu + nu * dua * itu;
        double apl = 1.0, adl = 1.0;
        if (act) {
            const double q = rcp_nr(dua);
            if (dua < 0.0) apl = fmin(apl, -tl * q);
            if (dua > 0.0) apl = fmin(apl, tu * q);
            if (dnla < 0.0) adl = fmin(adl, -nl * rcp_nr(dnla));
            if (dnua < 0.0) adl = fmin(adl, -nu * rcp_nr(dnua));
        }
        const double apr = S::min(apl), adr = S::min(adl);
        const double maff =
            S::sum(act ? (tl + apr * dua) * (nl + adr * dnla) + (tu - apr * dua) * (nu + adr * dnua)
                         : 0.0) * inv2N;
        const double ratio = muc > 0.0 ? maff / muc : 0.0;
        const double smu = ratio * ratio * ratio * muc;   // sigma mu
        // corrector: the centred, second-order-corrected complementarity
        // targets in the Riccati vector, then the forward steps
        const double taul = smu - dua * dnla, tauu = smu + dua * dnua;
        const double rt2 = ru + nl - taul * itl - nu + tauu * itu;
        double ca = hasx ? g : 1.0, cb = hasx ? fma(K, rt2, rx) : 0.0;
        ca = S::next(ca, 1.0, N);
        cb = S::next(cb, 0.0, N);
        {
            const Aff r = S::scan_suffix_aff(Aff{ca, cb});
            ca = r.a;
            cb = r.b;
        }
        const double e2 = fma(ca, rxN, cb);     // p_{k+1}
        const double kf2 = -(rt2 + s.B * e2) * hinv;
        double ga = act ? g : 1.0, gb = act ? s.B * kf2 : 0.0;
        {
            const Aff r = S::scan_prefix_aff(Aff{ga, gb});
            ga = r.a;
            gb = r.b;
        }
        const double ddx = gb;                  // dx_{k+1} step
        const double ddxk = S::prev(gb);
        const double ddu = (lane >= 1 ? K * ddxk : 0.0) + kf2;
        const double dmu = -(Pn * ddx + e2);
        const double dnl = fma(taul - nl * ddu, itl, -nl);
        const double dnu = fma(tauu + nu * ddu, itu, -nu);
        double apl2 = 1.0, adl2 = 1.0;
        if (act) {
            const double q = rcp_nr(ddu);
            if (ddu < 0.0) apl2 = fmin(apl2, -tl * q);
            if (ddu > 0.0) apl2 = fmin(apl2, tu * q);
            if (dnl < 0.0) adl2 = fmin(adl2, -nl * rcp_nr(dnl));
            if (dnu < 0.0) adl2 = fmin(adl2, -nu * rcp_nr(dnu));
        }
        const double ap = fmin(1.0, 0.995 * S::min(apl2));
        const double ad = fmin(1.0, 0.995 * S::min(adl2));
        if (act) {
            du = du + ap * ddu;
            dx = dx + ap * ddx;
            mu = mu + ad * dmu;
            nl = nl + ad * dnl;
            nu = nu + ad * dnu;
        }
    }
}

// SQP state of one OCP, stage k on lane k.
struct MsNlp {
    double U, X, LAM, PIL, PIU, A, B, C, FX, WXX, WXU, WUU, SIG;
};

// The SQP of one OCP from x-hat (x0) with the warm-started inputs in U;
// returns true if the KKT test passed (else the last iterate stands).
template <int G>
__device__ __forceinline__ bool ms_sqp_lanes(const DevParams& p, int N, double x0,
                                             int i0, int istep, double sign, double& Uio,
                                             int (&cnt)[C_NCNT]) {
    using S = Seg<G>;
    const int lane = S::k();   // the stage of this lane
    const bool act = lane < N;
    const double smax = 100.0;
    const double cst = 2.0 * p.Qz * p.Ts / p.V;
    const double qt = p.Qz * p.Ts;
    const double zb = setpoint(p, i0 + 1 + lane, istep, sign);   // zbar of x_{k+1}
    MsNlp v;
    v.U = act ? Uio : 0.5 * (p.umin + p.umax);   // lanes past the stages: inside the box
    if (v.U < p.umin) v.U = p.umin;
    if (v.U > p.umax) v.U = p.umax;
    {
        // feasible start: the states follow the inputs, one stage after another
        double xk = x0, X = 0.0;
        #pragma unroll 1
        for (int k = 0; k < N; ++k) {
            double dA, dB;
            xk = ms_interval<false>(p, xk, S::bcast(v.U, k), dA, dB);
            if (lane == k) X = xk;
        }
        v.X = X;
    }
    // interval tangents at (x_k, u_k), all stages at once
    {
        const double F = ms_interval<true>(p, S::prev(v.X, x0), v.U, v.A, v.B);
        v.C = F - v.X;
    }
    double f;
    {
        const double ez = v.X / p.V - zb;
        v.FX = cst * ez;
        f = S::sum(act ? qt * ez * ez : 0.0);
    }
    if (!act) v.A = v.B = v.C = v.FX = 0.0;
    v.WXX = 1.0;
    v.WXU = 0.0;
    v.WUU = 1.0;
    v.LAM = v.PIL = v.PIU = v.SIG = 0.0;
    cnt[C_LS]++;
    cnt[C_GRAD]++;
    bool first = true;
    #pragma unroll 1
    for (int l = 0;; ++l) {
        // eq. (convergence): |grad L / s_d|_inf <= eps and |c|_inf <= eps
        const double s1 = S::sum(act ? fabs(v.LAM) + fabs(v.PIL) + fabs(v.PIU) : 0.0);
        const double gu = -v.LAM * v.B - v.PIL + v.PIU;
        const double gx = v.FX + v.LAM - S::next(v.LAM * v.A, 0.0, N);
        const bool bad = S::any(act && (!(gu == gu) || !(gx == gx) || !(v.C == v.C)));
        const double gmax = S::max(act ? fmax(fabs(gu), fabs(gx)) : 0.0);
        const double cmax = S::max(act ? fabs(v.C) : 0.0);
        const double sd = fmax(smax, s1 / (3.0 * N)) / smax;
        if (!bad && gmax / sd <= p.sqp_eps && cmax <= p.sqp_eps) {
            Uio = v.U;
            return true;
        }
        if (l == p.sqp_max_iter) {
            Uio = v.U;
            return false;
        }
        // QP; an indefinite block (or H_uu <= 0 in the recursion) resets W
        bool reset;
        {
            const double wxp = S::prev(v.WXX, 1.0);
            const bool pdl = v.WUU > 0.0 && v.WXX > 0.0 && (lane == 0 || wxp * v.WUU - v.WXU * v.WXU > 0.0);
            reset = S::any(act && !pdl);
        }
        MsQpOut q{0.0, 0.0, 0.0, 0.0, 0.0};
        int st;
        #pragma unroll 1
        for (;;) {
            if (reset) {
                cnt[C_RESET]++;
                v.WXX = 1.0;
                v.WXU = 0.0;
                v.WUU = 1.0;
            }
            int it = 0;
            st = ms_qp_lanes<G>(p, N, MsStage{v.U, v.A, v.B, v.C, v.FX, v.WXX, v.WXU, v.WUU}, q, it);
            cnt[C_IPM] += it;
            if (st != -1 || reset) break;
            reset = true;
        }
        if (st == 1) cnt[C_IPMCAP]++;
        cnt[C_SQP]++;
        // Powell's l1 merit: sigma = |mu| first, then max(|mu|, (sigma + |mu|)/2)
        {
            const double am = fabs(q.mu);
            v.SIG = first ? am : fmax(am, 0.5 * (v.SIG + am));
        }
        first = false;
        const double ac = fabs(v.C);
        const double T0 = f + S::sum(act ? v.SIG * ac : 0.0);
        const double D = S::sum(act ? v.FX * q.dx - v.SIG * ac : 0.0);
        double alpha = 1.0;
        #pragma unroll 1
        for (int bt = 0;; ++bt) {
            // merit of the trial point xi + alpha dxi: f + sigma^T |c|
            const double xn = v.X + alpha * q.dx;
            const double u = v.U + alpha * q.du;
            double dA, dB;
            const double F = ms_interval<false>(p, S::prev(xn, x0), u, dA, dB);
            const double ez = xn / p.V - zb;
            const double Tt = S::sum(act ? v.SIG * fabs(F - xn) + qt * ez * ez : 0.0);
            cnt[C_LS]++;
            // a predicted decrease below the merit's resolution cannot be
            // tested in floating point: the full step is taken
            if (bt == 0 && -D <= 64.0 * 0x1p-52 * (1.0 + fabs(T0))) break;
            if (Tt <= T0 + p.ls_c1 * alpha * D) break;
            if (bt == p.ls_max_bt) {
                cnt[C_LSCAP]++;
                break;
            }
            alpha = p.ls_beta * alpha;
        }
        // the step, the new interval tangents, and the block BFGS with
        // y = grad L(xi+, lambda+, pi+) - grad L(xi, lambda+, pi+)
        const double su = alpha * q.du;
        const double un = v.U + su;
        const double sx = alpha * q.dx;           // step of x_{k+1}
        const double xk1 = v.X + sx;
        double An, Bn;
        const double F = ms_interval<true>(p, S::prev(xk1, x0), un, An, Bn);
        const double lam = v.LAM + alpha * (q.mu - v.LAM);
        v.LAM = lam;
        v.PIL = v.PIL + alpha * (q.nl - v.PIL);
        v.PIU = v.PIU + alpha * (q.nu - v.PIU);
        const double ez = xk1 / p.V - zb;
        const double fxn = cst * ez;
        f = S::sum(act ? qt * ez * ez : 0.0);
        // block k = {x_k, u_k} on lane k (block 0 = {u_0}); block N = {x_N}
        // on lane N - 1; W_{x_k} comes from lane k - 1 and goes back to it
        double wa = S::prev(v.WXX, 1.0);
        const double sxk = S::prev(sx);
        const double dfx = S::prev(fxn - v.FX);   // change of df/dx_k
        int applied = 0;
        if (lane == 0) {
            applied = ms_bfgs1(v.WUU, su, -lam * (Bn - v.B));
        } else if (act) {
            applied = ms_bfgs2(wa, v.WXU, v.WUU, sxk, su, dfx - lam * (An - v.A), -lam * (Bn - v.B));
        }
        double wN = v.WXX;
        if (lane == N - 1) applied |= ms_bfgs1(wN, sx, fxn - v.FX);
        const double wnext = S::next(wa, 0.0, N);
        if (act) v.WXX = lane == N - 1 ? wN : wnext;
        if (!S::any(act && applied)) cnt[C_SKIP]++;
        if (act) {
            v.U = un;
            v.X = xk1;
            v.A = An;
            v.B = Bn;
            v.C = F - xk1;
            v.FX = fxn;
        }
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


// NMPC kernel of the multiple-shooting formulation: a wavefront (64-lane
// workgroup) holds 64 / G samples, one per G-lane segment, each segment
// taking its next sample from the work queue as soon as its current one
// ends.  The closed loop per interval is that of nmpc_kernel (cost,
// measurement, CD-EKF, OCP, first input applied, Ns Euler-Maruyama
// sub-steps); the plant and the estimator are the same on every lane of a
// segment, the OCP runs a stage per lane.  The segments step their own
// intervals together: one pass of the loop is one control interval of each
// segment's sample.  Each OCP starts from the previous solution shifted by
// one interval with W^[0] = I.
template <int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MC_MS_WAVES_PER_EU))) void nmpc_ms_kernel(DevParams p, MsWork wk, Outs out) {
    using S = Seg<G>;
    const int kid = S::k();
    const double sqrtR = sqrt(p.Rmeas);
    const double h = p.Ts / (double)p.Ns;
    const double sqh = sqrt(h);
    const int g_hi = wk.qhi ? *wk.qhi : wk.n_groups;
    bool busy = false, drained = false;
    int64_t pos = 0;
    Setup su{};
    int N = 1, L = 0, i = 0;
    int cnt[C_NCNT];
    double n[3] = {0.0, 0.0, 0.0};
    double xhat = 0.0, P = 0.0, Fprev = 0.0, phiacc = 0.0, U = 0.0;
    uint64_t hsh = 0;
    #pragma unroll 1
    for (;;) {
        // a segment without a sample takes the next one (lane k = 0 of the
        // segment draws from the queue)
        if (!busy && !drained) {
            int grp = 0;
            if (kid == 0) grp = atomicAdd(wk.queue, 1);
            grp = G == 64 ? uni(__shfl(grp, 0, 64)) : __shfl(grp, S::base(), 64);
            if (grp >= g_hi) {
                drained = true;
            } else {
                busy = true;
                pos = wk.pos[grp];
                su = sample_setup(pos);
                N = G == 64 ? uni(su.N) : su.N;
                L = G == 64 ? uni(su.L) : su.L;
                i = 0;
#pragma unroll
                for (int c = 0; c < C_NCNT; ++c) cnt[c] = 0;
                n[0] = su.n0[0];
                n[1] = su.n0[1];
                n[2] = su.n0[2];
                xhat = su.xhat0;
                P = p.P0;
                Fprev = su.ubar;
                phiacc = 0.0;
                hsh = 14695981039346656037ull;
                U = su.ubar * kMlMinPerLs;   // u_k of the warm start on lane k
            }
        }
        if (__ballot(busy) == 0) break;
        if (busy) {
            // control interval i of this segment's sample
            const double z = n[2] / p.V;
            const double zb = setpoint(p, i, su.istep, su.sign);
            phiacc += (z - zb) * (z - zb);
            if (out.tz && kid == 0) out.tz[(int64_t)i * out.S + pos] = z;
            bool done = false;
            // (at G = 64 every lane holds the same sample: the branch is
            // made wavefront-uniform for the compiler, as are N and L)
            bool zbad = !isfinite(z);
            if constexpr (G == 64) zbad = uni(zbad ? 1 : 0) != 0;
            if (zbad) {
                // the plant diverged (Phi is not a number): no more OCPs
                cnt[C_NONFIN] = 1;
                done = true;
            } else if (i == L) {
                done = true;
            } else {
                const double y = z + p.noise_scale * sqrtR *
                                         normal_first(p.seed, 0, (uint32_t)i, su.nid, kTagMeas);
                ekf_predict(p, xhat, P, Fprev);
                ekf_update(p, xhat, P, y);
                if (!isfinite(P) || !isfinite(xhat)) cnt[C_NONFIN] = 1;
                if (out.tx && kid == 0) out.tx[(int64_t)i * out.S + pos] = xhat;
                const bool conv = ms_sqp_lanes<G>(p, N, xhat, i, su.istep, su.sign, U, cnt);
                cnt[C_OCP]++;
                if (!conv) cnt[C_OCP_FAIL]++;
                const uint64_t mask = S::mask(kid < N && (U <= p.umin + 1e-6 || U >= p.umax - 1e-6));
                hsh = fnv1a_step(hsh, (uint32_t)i, mask);
                const double F = S::bcast(U, 0) / kMlMinPerLs;
                U = S::next(U, U, N);   // shift: u_k <- u_{k+1}, the last one kept
                if (out.tu && kid == 0) out.tu[(int64_t)i * out.S + pos] = F;
                // the plant runs alike on every lane of the segment: lane k
                // draws the noise of sub-step j0 + k, and each sub-step takes
                // its normals from the lane that drew them (a lane past the
                // last sub-step draws a value nobody uses)
                #pragma unroll 1
                for (int j0 = 0; j0 < p.Ns; j0 += G) {
                    double own[3];
                    process_noise(p, (uint32_t)(i * p.Ns + j0 + kid), su.nid, own);
                    const int jn = p.Ns - j0 < G ? p.Ns - j0 : G;
                    #pragma unroll 1
                    for (int j = 0; j < jn; ++j) {
                        const double xi[3] = {S::bcast(own[0], j), S::bcast(own[1], j),
                                              S::bcast(own[2], j)};
                        em_step(p, su.k0, su.EaR, n, F, h, sqh, xi);
                    }
                }
                Fprev = F;
                ++i;
            }
            if (done) {
                if (!isfinite(n[0]) || !isfinite(n[1]) || !isfinite(n[2])) cnt[C_NONFIN] = 1;
                if (kid == 0) {
                    out.phi[pos] = phiacc / (double)(L + 1);
                    out.hash[pos] = hsh;
                    cnt[C_KIND] = 0;
                    cnt[C_N] = N;
                    cnt[C_L] = L;
                    out.flops[pos] = ms_sample_flops(p, N, L, cnt);
#pragma unroll
                    for (int c = 0; c < C_NCNT; ++c) out.cnt[(int64_t)c * out.S + pos] = cnt[c];
                }
                busy = false;
            }
        }
    }
}

}  // namespace mccl
