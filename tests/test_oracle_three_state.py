"""Pins of the oracle's three-state estimator and OCP (the CD-EKF and the
single-shooting OCP of the NMPC section at n_x = 3, with eq. (CSTR)'s drift).

As for the one-state pins, none re-types an oracle formula: each compares
with a closed form, an independent ODE solver, finite differences of the
oracle's own maps, an algebraic identity of the Kalman filter or an
independent optimiser.  CPU only.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_2212_02197_amd import workloads as W

CFG = W.c1_paper_scale(model_nx=3)


def _spd(rng, scale):
    a = rng.standard_normal((3, 3)) * scale
    return a @ a.T + np.diag(scale ** 2 * np.ones(3))


# ------------------------------------------------------------- estimator ---
def test_ekf3_prediction_closed_form_linear_model(oracle):
    # k0 = 0: dn/dt = (C_in - n/V) F and dP/dt = -2F/V P + F^2 diag(sigma^2)
    # solve in closed form element by element (off-diagonal entries decay
    # without a source); the RK4 prediction converges to them at fourth order.
    V, F, t = CFG["V"], 0.012, CFG["Ts"]
    sig = np.array(CFG["sigma"])
    Cin = np.array([CFG["cAin"], CFG["cBin"], CFG["cTin"]]) * V
    x0 = np.array([0.3, 0.5, 300.0]) * V
    P0 = _spd(np.random.default_rng(3), 0.05)
    a = F / V
    xc = Cin + (x0 - Cin) * math.exp(-a * t)
    Pc = P0 * math.exp(-2 * a * t) + np.diag(F * sig ** 2 * V * (1 - math.exp(-2 * a * t)) / 2)
    eP = []
    for Nc in (5, 10, 20):
        x, P = oracle.ekf3_predict(dict(CFG, k0=0.0, Nc=Nc), x0, P0, F)
        np.testing.assert_allclose(x, xc, rtol=1e-9)
        eP.append(np.abs(P - Pc).max() / np.abs(Pc).max())
    assert eP[0] < 1e-7
    assert eP[0] / eP[1] == pytest.approx(16, rel=0.1)
    assert eP[1] / eP[2] == pytest.approx(16, rel=0.1)


def test_ekf3_covariance_is_transported_by_the_state_transition(oracle):
    # Without process noise dP/dt = A P + P A^T is solved by Phi P0 Phi^T,
    # Phi = dx(Ts)/dx(0).  Phi from central differences of the predicted
    # mean; the reaction couples all three states, so A is full and not
    # symmetric (a transposed product fails this).
    cfg = dict(CFG, sigma=[0.0, 0.0, 0.0], Nc=40)
    F, nss = oracle.steady_state(cfg, 320.0)
    x0 = nss * np.array([1.02, 0.97, 1.004])
    P0 = _spd(np.random.default_rng(5), 0.2)
    Phi = np.zeros((3, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = 1e-6 * x0[b]
        xp, _ = oracle.ekf3_predict(cfg, x0 + e, np.zeros((3, 3)), F)
        xm, _ = oracle.ekf3_predict(cfg, x0 - e, np.zeros((3, 3)), F)
        Phi[:, b] = (xp - xm) / (2 * e[b])
    assert np.abs(Phi - np.diag(np.diag(Phi))).max() > 1e-3 * np.abs(Phi).max()
    _, P = oracle.ekf3_predict(cfg, x0, P0, F)
    ref = Phi @ P0 @ Phi.T
    np.testing.assert_allclose(P, ref, rtol=0, atol=2e-7 * np.abs(ref).max())
    np.testing.assert_allclose(P, P.T, rtol=0, atol=1e-14 * np.abs(P).max())


def test_ekf3_noise_term_is_additive_and_quadratic_in_the_flow(oracle):
    # P(Ts) is affine in the noise covariance F^2 diag(sigma^2) for a fixed
    # mean path: scaling sigma by s scales the noise part of P by s^2.
    F, nss = oracle.steady_state(CFG, 320.0)
    x0 = nss * np.array([1.01, 0.99, 1.002])
    P0 = _spd(np.random.default_rng(7), 0.1)
    base = oracle.ekf3_predict(dict(CFG, sigma=[0.0, 0.0, 0.0]), x0, P0, F)[1]
    one = oracle.ekf3_predict(CFG, x0, P0, F)[1] - base
    three = oracle.ekf3_predict(dict(CFG, sigma=[3 * s for s in CFG["sigma"]]), x0, P0, F)[1] - base
    np.testing.assert_allclose(three, 9 * one, rtol=1e-9, atol=1e-12 * np.abs(one).max())
    assert np.all(np.linalg.eigvalsh(one) > 0)


def test_ekf3_joseph_form_equals_standard_form(oracle):
    # eq. (Josph) with the optimal gain: (I-KC)P(I-KC)^T + K R K^T =
    # P - P C^T C P / (C P C^T + R), and x += K (y - C x).
    rng = np.random.default_rng(11)
    V, R = CFG["V"], CFG["Rmeas"]
    C = np.array([0.0, 0.0, 1.0 / V])
    for scale in (1e-3, 0.1, 3.0):
        P = _spd(rng, scale)
        x = np.array([0.4, 0.6, 320.0]) * V
        y = 321.3
        xn, Pn = oracle.ekf3_update(CFG, x, P, y)
        S = C @ P @ C + R
        K = P @ C / S
        np.testing.assert_allclose(Pn, P - np.outer(P @ C, P @ C) / S, rtol=1e-11,
                                   atol=1e-13 * np.abs(P).max())
        np.testing.assert_allclose(xn, x + K * (y - C @ x), rtol=1e-14)
        assert np.all(np.linalg.eigvalsh(Pn) > -1e-14 * np.abs(P).max())


# ------------------------------------------------------------------ OCP ---
def _f3_numpy(cfg, n, F):
    # eq. (CSTR) drift written out in NumPy for the ODE reference
    V = cfg["V"]
    c = n / V
    r = cfg["k0"] * np.exp(-cfg["EaR"] / c[2]) * c[0] * c[1]
    S = np.array([-1.0, -2.0, cfg["beta"]])
    Cin = np.array([cfg["cAin"], cfg["cBin"], cfg["cTin"]])
    return Cin * F - c * F + S * r * V


def test_ocp3_shooting_is_fourth_order(oracle):
    cfg = dict(CFG)
    F, nss = oracle.steady_state(cfg, 320.0)
    x0 = nss * np.array([1.01, 0.99, 1.005])
    N = 4
    u = np.full(N, F * 60000 * 1.1)
    sol = integrate.solve_ivp(lambda t, n: _f3_numpy(cfg, n, u[0] / 60000.0),
                              (0, N * cfg["Ts"]), x0, method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    errs = []
    for Nc in (2, 4, 8):
        cfg["Nc"] = Nc
        _, xs = oracle.ocp_shoot(cfg, x0, u, np.full(N, 320.0), want_xs=True)
        errs.append(np.abs(xs[-1] - ref).max())
    assert errs[0] / errs[1] == pytest.approx(16, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(16, rel=0.15)


def test_ocp3_objective_definition(oracle):
    cfg = dict(CFG, Qz=2.5, Ts=0.7)
    N = 6
    u = np.linspace(400, 700, N)
    zb = np.linspace(318, 324, N)
    F, nss = oracle.steady_state(cfg, 320.0)
    phi, xs = oracle.ocp_shoot(cfg, nss, u, zb, want_xs=True)
    xk = xs[cfg["Nc"]::cfg["Nc"], 2]
    assert len(xk) == N
    assert phi == pytest.approx(np.sum(cfg["Qz"] * (xk / cfg["V"] - zb) ** 2 * cfg["Ts"]),
                                rel=1e-13)


@pytest.mark.parametrize("N", [1, 5, 20, 60])
def test_ocp3_gradient_adjoint_equals_tangent_and_fd(oracle, N):
    rng = np.random.default_rng(100 + N)
    F, nss = oracle.steady_state(CFG, 320.0)
    x0 = nss * (1 + 0.005 * rng.standard_normal(3))
    u = np.clip(F * 60000 + 150 * rng.standard_normal(N), 10, 990)
    zb = 320.0 + 5 * rng.standard_normal(N)
    ga = oracle.ocp_grad(CFG, x0, u, zb, "adjoint")
    gf = oracle.ocp_grad(CFG, x0, u, zb, "fwd")
    scale = np.abs(ga).max()
    np.testing.assert_allclose(ga, gf, rtol=0, atol=1e-12 * scale)
    gd = np.zeros(N)
    for j in range(N):
        h = 1e-6 * u[j]
        e = np.zeros(N)
        e[j] = h
        gd[j] = (oracle.ocp_shoot(CFG, x0, u + e, zb) - oracle.ocp_shoot(CFG, x0, u - e, zb)) / (2 * h)
    np.testing.assert_allclose(ga, gd, rtol=0, atol=1e-6 * scale)


def test_ocp3_on_the_invariant_manifold_matches_the_one_state_ocp(oracle):
    # From a state on the reaction-invariant manifold the three-state
    # trajectory stays on it, where f3's temperature row is f1: both OCPs
    # then have the same objective and gradient (up to rounding).
    cfg1 = W.c1_paper_scale()
    F, nss = oracle.steady_state(CFG, 325.0)
    rng = np.random.default_rng(2)
    u = np.clip(F * 60000 + 100 * rng.standard_normal(12), 10, 990)
    zb = 320.0 + 3 * rng.standard_normal(12)
    f3v = oracle.ocp_shoot(CFG, nss, u, zb)
    f1v = oracle.ocp_shoot(cfg1, nss[2], u, zb)
    assert f3v == pytest.approx(f1v, rel=1e-9)
    g3 = oracle.ocp_grad(CFG, nss, u, zb, "adjoint")
    g1 = oracle.ocp_grad(cfg1, nss[2], u, zb, "adjoint")
    np.testing.assert_allclose(g3, g1, rtol=0, atol=1e-8 * np.abs(g1).max())


def test_sqp3_against_scipy_lbfgsb(oracle):
    cfg = W.make(N=8, sqp_eps=1e-9, sqp_max_iter=400, model_nx=3)
    F, nss = oracle.steady_state(cfg, 320.0)
    for xf, z0 in (((1.0, 1.0, 1.004), 320.0), ((0.98, 1.01, 1.0), 326.0),
                   ((1.02, 0.99, 0.985), 315.0)):
        x0 = nss * np.array(xf)
        zb = np.full(8, z0)
        conv, u, pil, piu, cnt = oracle.sqp(cfg, x0, zb, np.full(8, F * 60000))
        assert conv
        res = optimize.minimize(lambda v: oracle.ocp_shoot(cfg, x0, v, zb),
                                np.full(8, F * 60000),
                                jac=lambda v: oracle.ocp_grad(cfg, x0, v, zb, "adjoint"),
                                bounds=[(0, 1000)] * 8, method="L-BFGS-B",
                                options=dict(ftol=1e-16, gtol=1e-11, maxiter=5000))
        f_sqp = oracle.ocp_shoot(cfg, x0, u, zb)
        assert f_sqp <= res.fun * (1 + 1e-9) + 1e-12
        np.testing.assert_allclose(u, res.x, rtol=0, atol=0.05)


# ----------------------------------------------------------- closed loop ---
def test_three_state_noise_free_closed_loop_settles(oracle):
    # The three-state NMPC holds each level of the schedule (Results
    # section); with no noise and no kinetic perturbation its model matches
    # the plant up to the integrators, so the filter's n_T stays on the
    # plant's.
    N = 20
    cfg = W.c1_paper_scale(kind_split=-1, default_kind=0, N=N, Ns=10, noise_scale=0.0,
                           model_nx=3)
    r = oracle.run_sample(cfg, 0, traj=True)
    z = r["z"]
    for i_end, zb in ((199 - N, 320.0), (399 - N, 335.0), (600, 300.0)):
        assert abs(z[i_end] - zb) < 1e-3, (i_end, z[i_end])
    assert r["n_ocp"] == 600 and r["nonfinite"] == 0
    assert np.abs(r["xhat"] / cfg["V"] - z[:-1]).max() < 0.05


def test_three_state_stochastic_sample_runs_its_ocps(oracle):
    cfg = W.c1_paper_scale(model_nx=3, L=40, N=20)
    r = oracle.run(cfg, ids=np.array([0, 1, 30000]), nthreads=3)
    assert r["n_ocp"].tolist() == [40, 40, 0]
    assert r["nonfinite"].tolist() == [0, 0, 0]
    assert np.all(r["n_ocp_fail"] == 0)
