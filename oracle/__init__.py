"""ctypes binding of the FP64 CPU oracle (oracle/mc_oracle.c).

TEST INFRASTRUCTURE ONLY.  tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this; the product package never does.
It shares no code with the HIP path and imports nothing from it: callers hand
it plain workload dicts.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libmc_oracle.so")
_SRC = os.path.join(_HERE, "mc_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "mc_oracle_ms.c")]
SPMAX = 8
NMAX = 64


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            [os.path.getmtime(f) for f in _SRCS] + [os.path.getmtime(os.path.join(_HERE, "mc_oracle.h"))]):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, *_SRCS, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("V", C.c_double), ("k0", C.c_double), ("EaR", C.c_double), ("beta", C.c_double),
        ("cAin", C.c_double), ("cBin", C.c_double), ("cTin", C.c_double),
        ("sigma", C.c_double * 3), ("Rmeas", C.c_double),
        ("Ts", C.c_double), ("Ns", C.c_int32), ("L", C.c_int32),
        ("n_sp", C.c_int32), ("sp_period", C.c_int32),
        ("sp_i", C.c_int32 * SPMAX), ("sp_z", C.c_double * SPMAX),
        ("sp_step_rel", C.c_double), ("sp_step_lo", C.c_int32), ("sp_step_hi", C.c_int32),
        ("N", C.c_int32), ("Nc", C.c_int32),
        ("Qz", C.c_double), ("umin", C.c_double), ("umax", C.c_double),
        ("sqp_eps", C.c_double), ("ls_c1", C.c_double), ("ls_beta", C.c_double),
        ("sqp_max_iter", C.c_int32), ("ls_max_bt", C.c_int32), ("grad_mode", C.c_int32),
        ("ipm_max_iter", C.c_int32), ("want_grad", C.c_int32),
        ("kP", C.c_double), ("kI", C.c_double), ("kaw", C.c_double),
        ("pi_umin", C.c_double), ("pi_umax", C.c_double),
        ("P0", C.c_double), ("x0_rel_std", C.c_double),
        ("x0_mode", C.c_int32), ("kind_split", C.c_int32), ("default_kind", C.c_int32),
        ("run_ekf_for_pi", C.c_int32),
        ("seed", C.c_uint64), ("noise_mod", C.c_int64),
        ("n_horizon_choices", C.c_int32), ("horizon_choices", C.c_int32 * 4),
        ("L_lo", C.c_int32), ("L_hi", C.c_int32),
        ("kin_lognorm_sigma", C.c_double),
        ("hess_warm", C.c_int32), ("model_nx", C.c_int32), ("noise_scale", C.c_double),
        ("nlp_form", C.c_int32),
    ]


class SampleOut(C.Structure):
    _fields_ = [
        ("phi", C.c_double), ("dphi", C.c_double * 2), ("ashash", C.c_uint64),
        ("kind", C.c_int32), ("N", C.c_int32), ("L", C.c_int32), ("n_ocp", C.c_int32),
        ("n_ocp_fail", C.c_int32), ("sqp_iter", C.c_int32), ("ipm_iter", C.c_int32),
        ("ls_trials", C.c_int32), ("ls_cap", C.c_int32), ("bfgs_skip", C.c_int32),
        ("bfgs_reset", C.c_int32), ("ipm_cap", C.c_int32), ("nonfinite", C.c_int32),
        ("grad_evals", C.c_int32),
    ]


OUT_FIELDS = [f for f, _ in SampleOut._fields_]

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i32, i64, u32, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        P = C.POINTER
        pd = P(d)
        sig = {
            "oc_philox4x32_10": (None, [P(u32), P(u32), P(u32)]),
            "oc_normal_pair": (None, [u64, u32, u32, u32, u32, pd]),
            "oc_f3": (None, [P(Params), d, d, pd, d, pd]),
            "oc_f3_jac": (None, [P(Params), d, d, pd, d, pd, pd]),
            "oc_f1": (None, [P(Params), d, d, pd]),
            "oc_steady_state": (None, [P(Params), d, pd, pd]),
            "oc_setpoint": (d, [P(Params), i32, i32, d]),
            "oc_em_step": (None, [P(Params), d, d, pd, d, pd]),
            "oc_ekf_predict": (None, [P(Params), pd, pd, d]),
            "oc_ekf_update": (None, [P(Params), pd, pd, d]),
            "oc_ocp_shoot": (d, [P(Params), i32, d, pd, pd, pd]),
            "oc_ocp_grad_adjoint": (None, [P(Params), i32, pd, pd, pd, pd]),
            "oc_ocp_grad_fwd": (None, [P(Params), i32, d, pd, pd, pd]),
            "oc_ekf3_predict": (None, [P(Params), pd, pd, d]),
            "oc_ekf3_update": (None, [P(Params), pd, pd, d]),
            "oc_ocp3_shoot": (d, [P(Params), i32, pd, pd, pd, pd]),
            "oc_ocp3_grad_adjoint": (None, [P(Params), i32, pd, pd, pd, pd]),
            "oc_ocp3_grad_fwd": (None, [P(Params), i32, pd, pd, pd, pd]),
            "oc_box_qp": (C.c_int, [i32, pd, pd, pd, pd, i32, pd, pd, pd, P(i32)]),
            "oc_bfgs_update": (C.c_int, [i32, pd, pd, pd]),
            "oc_sqp": (C.c_int, [P(Params), i32, pd, pd, pd, pd, pd, pd, i32, P(SampleOut)]),
            "oc_run_sample": (None, [P(Params), i64, P(SampleOut), pd, pd, pd]),
            "oc_run_sample_ext": (None, [P(Params), i64, P(i32), P(SampleOut), pd, pd, pd, pd]),
            "oc_run_ov": (None, [P(Params), P(i64), P(i32), i64, i32, P(SampleOut)]),
            "oc_scenario": (None, [P(Params), i64, P(i32), pd]),
            "oc_run": (None, [P(Params), P(i64), i64, i32, P(SampleOut)]),
            "oc_stats": (None, [pd, i64, pd, pd, P(i64)]),
            "oc_ms_interval": (None, [P(Params), d, d, pd]),
            "oc_ms_qp": (C.c_int, [P(Params), i32, pd, pd, pd, pd, pd, pd, pd, pd, pd, pd, P(i32)]),
            "oc_ms_sqp": (C.c_int, [P(Params), i32, d, pd, pd, pd, P(SampleOut)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def params(cfg: dict) -> Params:
    """Fill the oracle's own parameter struct from a workload dict."""
    p = Params()
    for key in ("V", "k0", "EaR", "beta", "cAin", "cBin", "cTin", "Rmeas", "Ts", "Ns", "L",
                "sp_period", "sp_step_rel", "sp_step_lo", "sp_step_hi", "N", "Nc", "Qz",
                "umin", "umax", "sqp_eps", "ls_c1", "ls_beta", "sqp_max_iter", "ls_max_bt",
                "grad_mode", "ipm_max_iter", "want_grad", "kP", "kI", "kaw", "pi_umin",
                "pi_umax", "P0", "x0_rel_std", "x0_mode", "kind_split", "default_kind",
                "run_ekf_for_pi", "seed", "noise_mod", "L_lo", "L_hi", "kin_lognorm_sigma",
                "hess_warm", "noise_scale"):
        setattr(p, key, cfg[key])
    p.model_nx = cfg.get("model_nx", 1)
    assert p.model_nx in (1, 3)
    p.nlp_form = cfg.get("nlp_form", 0)
    assert p.nlp_form in (0, 1) and (p.nlp_form == 0 or p.model_nx == 1)
    for a in range(3):
        p.sigma[a] = cfg["sigma"][a]
    sp_i, sp_z = cfg["sp_i"], cfg["sp_z"]
    assert 1 <= len(sp_i) == len(sp_z) <= SPMAX
    p.n_sp = len(sp_i)
    for j in range(len(sp_i)):
        p.sp_i[j] = sp_i[j]
        p.sp_z[j] = sp_z[j]
    hc = cfg["horizon_choices"]
    p.n_horizon_choices = len(hc)
    for j, v in enumerate(hc):
        p.horizon_choices[j] = v
    return p


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().oc_philox4x32_10(c, k, o)
    return list(o)


def normal_pair(seed, block, step, sid, tag):
    o = np.zeros(4)
    lib().oc_normal_pair(seed, block, step, sid, tag, _dp(o))
    return o


def f3(cfg, n, F, k0=None, EaR=None):
    p = params(cfg)
    o = np.zeros(3)
    n = np.ascontiguousarray(n, dtype=np.float64)
    lib().oc_f3(C.byref(p), cfg["k0"] if k0 is None else k0,
                cfg["EaR"] if EaR is None else EaR, _dp(n), F, _dp(o))
    return o


def f3_jac(cfg, n, F):
    p = params(cfg)
    J = np.zeros(9)
    fF = np.zeros(3)
    n = np.ascontiguousarray(n, dtype=np.float64)
    lib().oc_f3_jac(C.byref(p), cfg["k0"], cfg["EaR"], _dp(n), F, _dp(J), _dp(fF))
    return J.reshape(3, 3), fF


def f1(cfg, x, F):
    p = params(cfg)
    o = np.zeros(3)
    lib().oc_f1(C.byref(p), x, F, _dp(o))
    return o


def steady_state(cfg, T):
    p = params(cfg)
    F = C.c_double()
    n = np.zeros(3)
    lib().oc_steady_state(C.byref(p), T, C.byref(F), _dp(n))
    return F.value, n


def setpoint(cfg, i, istep=0, sign=0.0):
    return lib().oc_setpoint(C.byref(params(cfg)), i, istep, sign)


def em_step(cfg, n, F, xi, k0=None, EaR=None):
    p = params(cfg)
    n = np.array(n, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    lib().oc_em_step(C.byref(p), cfg["k0"] if k0 is None else k0,
                     cfg["EaR"] if EaR is None else EaR, _dp(n), F, _dp(xi))
    return n


def ekf_predict(cfg, x, P, F):
    p = params(cfg)
    xx, PP = C.c_double(x), C.c_double(P)
    lib().oc_ekf_predict(C.byref(p), C.byref(xx), C.byref(PP), F)
    return xx.value, PP.value


def ekf_update(cfg, x, P, y):
    p = params(cfg)
    xx, PP = C.c_double(x), C.c_double(P)
    lib().oc_ekf_update(C.byref(p), C.byref(xx), C.byref(PP), y)
    return xx.value, PP.value


def ekf3_predict(cfg, x, P, F):
    """Three-state prediction: x (3,), P (3, 3) -> new (x, P)."""
    p = params(cfg)
    xx = np.array(x, dtype=np.float64).reshape(3)
    PP = np.array(P, dtype=np.float64).reshape(9)
    lib().oc_ekf3_predict(C.byref(p), _dp(xx), _dp(PP), F)
    return xx, PP.reshape(3, 3)


def ekf3_update(cfg, x, P, y):
    p = params(cfg)
    xx = np.array(x, dtype=np.float64).reshape(3)
    PP = np.array(P, dtype=np.float64).reshape(9)
    lib().oc_ekf3_update(C.byref(p), _dp(xx), _dp(PP), y)
    return xx, PP.reshape(3, 3)


def ocp_shoot(cfg, x0, u, zbar, want_xs=False):
    """OCP objective from x0 (a scalar: one-state model; 3 values: three-state
    model).  xs: the RK4 step-start states (3 per step for the three-state
    model)."""
    p = params(cfg)
    u = np.ascontiguousarray(u, dtype=np.float64)
    zbar = np.ascontiguousarray(zbar, dtype=np.float64)
    N = len(u)
    if np.ndim(x0) == 0:
        xs = np.zeros(N * cfg["Nc"] + 1)
        phi = lib().oc_ocp_shoot(C.byref(p), N, float(x0), _dp(u), _dp(zbar), _dp(xs))
    else:
        xv = np.ascontiguousarray(x0, dtype=np.float64).reshape(3)
        xs = np.zeros(3 * (N * cfg["Nc"] + 1))
        phi = lib().oc_ocp3_shoot(C.byref(p), N, _dp(xv), _dp(u), _dp(zbar), _dp(xs))
        xs = xs.reshape(-1, 3)
    return (phi, xs) if want_xs else phi


def ocp_grad(cfg, x0, u, zbar, mode):
    p = params(cfg)
    u = np.ascontiguousarray(u, dtype=np.float64)
    zbar = np.ascontiguousarray(zbar, dtype=np.float64)
    N = len(u)
    g = np.zeros(N)
    three = np.ndim(x0) > 0
    if mode == "adjoint":
        _, xs = ocp_shoot(cfg, x0, u, zbar, want_xs=True)
        xs = np.ascontiguousarray(xs.reshape(-1))
        fn = lib().oc_ocp3_grad_adjoint if three else lib().oc_ocp_grad_adjoint
        fn(C.byref(p), N, _dp(u), _dp(zbar), _dp(xs), _dp(g))
    elif three:
        xv = np.ascontiguousarray(x0, dtype=np.float64).reshape(3)
        lib().oc_ocp3_grad_fwd(C.byref(p), N, _dp(xv), _dp(u), _dp(zbar), _dp(g))
    else:
        lib().oc_ocp_grad_fwd(C.byref(p), N, x0, _dp(u), _dp(zbar), _dp(g))
    return g


def box_qp(W, g, lo, hi, max_iter=50):
    W = np.ascontiguousarray(W, dtype=np.float64)
    g, lo, hi = (np.ascontiguousarray(v, dtype=np.float64) for v in (g, lo, hi))
    N = len(g)
    d, nl, nu = np.zeros(N), np.zeros(N), np.zeros(N)
    it = C.c_int32()
    st = lib().oc_box_qp(N, _dp(W), _dp(g), _dp(lo), _dp(hi), max_iter, _dp(d), _dp(nl),
                         _dp(nu), C.byref(it))
    return st, d, nl, nu, it.value


def bfgs_update(W, s, y):
    W = np.array(W, dtype=np.float64)
    s, y = (np.ascontiguousarray(v, dtype=np.float64) for v in (s, y))
    upd = lib().oc_bfgs_update(len(s), _dp(W), _dp(s), _dp(y))
    return W, bool(upd)


def sqp(cfg, x0, zbar, u0):
    """One SQP solve; x0 a scalar (one-state model) or 3 values (three-state
    model, which cfg["model_nx"] must select)."""
    p = params(cfg)
    xv = np.array(np.atleast_1d(x0), dtype=np.float64)
    assert len(xv) == (3 if p.model_nx == 3 else 1)
    zbar = np.ascontiguousarray(zbar, dtype=np.float64)
    u = np.array(u0, dtype=np.float64)
    N = len(u)
    pil, piu = np.zeros(N), np.zeros(N)
    cnt = SampleOut()
    W = np.zeros(N * N)
    conv = lib().oc_sqp(C.byref(p), N, _dp(xv), _dp(zbar), _dp(u), _dp(pil), _dp(piu), _dp(W), 1,
                        C.byref(cnt))
    return bool(conv), u, pil, piu, {f: getattr(cnt, f) for f in OUT_FIELDS[4:]}


def run_sample(cfg, sid, traj=False):
    """One closed-loop sample; returns the result dict (+ trajectories:
    z, u, x-hat and, for PI samples, the integral state I-hat after each
    interval's update)."""
    p = params(cfg)
    o = SampleOut()
    Lmax = max(cfg["L"], cfg["L_hi"]) + 1
    tz, tu, tx, ti = np.zeros(Lmax), np.zeros(Lmax), np.zeros(Lmax), np.zeros(Lmax)
    if traj:
        lib().oc_run_sample_ext(C.byref(p), sid, None, C.byref(o), _dp(tz), _dp(tu), _dp(tx),
                                _dp(ti))
    else:
        lib().oc_run_sample(C.byref(p), sid, C.byref(o), None, None, None)
    res = _out_dict(o)
    if traj:
        L = o.L
        res["z"], res["u"], res["xhat"], res["Ihat"] = tz[:L + 1], tu[:L], tx[:L], ti[:L]
    return res


def scenario(cfg, sid):
    """Per-sample scenario draws: dict(kind, N, L, istep, sign, k0, EaR)."""
    p = params(cfg)
    iv = (C.c_int32 * 4)()
    dv = np.zeros(3)
    lib().oc_scenario(C.byref(p), sid, iv, _dp(dv))
    return dict(kind=iv[0], N=iv[1], L=iv[2], istep=iv[3], sign=dv[0], k0=dv[1], EaR=dv[2])


def _out_dict(o):
    r = {f: getattr(o, f) for f in OUT_FIELDS}
    r["dphi"] = (o.dphi[0], o.dphi[1])
    return r


def run(cfg, ids=None, nthreads=None, kind=None, horizon=None, lengths=None):
    """Closed loop for the given sample ids on a thread pool.  kind, horizon
    and lengths (optional, aligned with ids) replace the per-sample rules.
    Returns a dict of numpy arrays, one entry per field of SampleOut."""
    if ids is None:
        ids = np.arange(cfg["n_samples"], dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = len(ids)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    p = params(cfg)
    outs = (SampleOut * n)()
    if kind is None and horizon is None and lengths is None:
        lib().oc_run(C.byref(p), ids.ctypes.data_as(C.POINTER(C.c_int64)), n, nthreads, outs)
    else:
        ov = np.full((3, n), -1, dtype=np.int32)
        for row, a in enumerate((kind, horizon, lengths)):
            if a is not None:
                ov[row] = np.asarray(a, dtype=np.int32)
        lib().oc_run_ov(C.byref(p), ids.ctypes.data_as(C.POINTER(C.c_int64)),
                        ov.ctypes.data_as(C.POINTER(C.c_int32)), n, nthreads, outs)
    arr = np.frombuffer(outs, dtype=np.dtype({
        "names": OUT_FIELDS,
        "formats": ["f8", ("f8", 2), "u8"] + ["i4"] * 14,
        "offsets": [getattr(SampleOut, f).offset for f in OUT_FIELDS],
        "itemsize": C.sizeof(SampleOut)}))
    res = {f: np.array(arr[f]) for f in OUT_FIELDS}
    res["ids"] = ids
    return res


def stats(phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    m, v = C.c_double(), C.c_double()
    hist = np.zeros(202, dtype=np.int64)
    lib().oc_stats(_dp(phi), len(phi), C.byref(m), C.byref(v),
                   hist.ctypes.data_as(C.POINTER(C.c_int64)))
    return m.value, v.value, hist


def ms_interval(cfg, x, u):
    """One sampling interval of the one-state model: (F, dF/dx, dF/du)."""
    o = np.zeros(3)
    lib().oc_ms_interval(C.byref(params(cfg)), x, u, _dp(o))
    return tuple(o)


def ms_qp(cfg, W, gf, A, B, c, u):
    """The structured QP of the multiple-shooting SQP (condensed, dense):
    returns (status, dxi, mu, nu_l, nu_u, iterations)."""
    N = len(u)
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (W, gf, A, B, c, u)]
    dxi, mu, nl, nu = np.zeros(2 * N), np.zeros(N), np.zeros(N), np.zeros(N)
    it = C.c_int32()
    st = lib().oc_ms_qp(C.byref(params(cfg)), N, *[_dp(a) for a in arr], _dp(dxi), _dp(mu),
                        _dp(nl), _dp(nu), C.byref(it))
    return st, dxi, mu, nl, nu, it.value


def ms_sqp(cfg, x0, zbar, u0):
    """One multiple-shooting SQP solve (W^[0] = I): (converged, u, x, counters)."""
    p = params(cfg)
    zbar = np.ascontiguousarray(zbar, dtype=np.float64)
    u = np.array(u0, dtype=np.float64)
    x = np.zeros(len(u) + 1)
    cnt = SampleOut()
    conv = lib().oc_ms_sqp(C.byref(p), len(u), float(x0), _dp(zbar), _dp(u), _dp(x), C.byref(cnt))
    return bool(conv), u, x, {f: getattr(cnt, f) for f in OUT_FIELDS[4:]}
