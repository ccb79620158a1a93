"""The multiple-shooting kernel solves the structured QP's Riccati recursion
(paper: Sequential Quadratic Programming, the QP subproblem solved by a
Riccati-recursion interior point) with parallel scans over the stages
instead of a stage-by-stage sweep.  These CPU tests pin that reformulation
in plain numpy (FP64), independently of the HIP code:

* one backward step of the factor, P_k = W_x + A^2 P - H_ux^2 / H_uu with
  H_uu = R + B^2 P and H_ux = W_xu + B P A, equals the linear-fractional map
  P -> (alpha P + beta) / (B^2 P + R) with alpha = W_x B^2 + A^2 R - 2 W_xu A B
  and beta = W_x R - W_xu^2, divided through by R (also for R = infinity,
  where the serial step gives W_x + A^2 P);
* suffix products of those 2x2 maps, rescaled by powers of two, reproduce
  every P_k of the serial recursion;
* the Riccati vector and the forward state steps are affine maps whose
  prefix/suffix compositions reproduce the serial recursions;
* an interior point built on these scans (the kernel's algorithm) reaches the
  oracle's dense condensed QP solution.
"""
import numpy as np
import pytest

import oracle
from paper_2212_02197_amd import workloads as W


def serial_factor(PN, A, B, R, wx, wxu):
    """P_{k+1} for k = 0..N-1 by the serial backward step (stage k >= 1)."""
    N = len(A)
    P = np.zeros(N)
    Pc = PN
    for k in range(N - 1, -1, -1):
        P[k] = Pc
        if k >= 1:
            Huu = R[k] + B[k] ** 2 * Pc
            Hux = wxu[k] + B[k] * Pc * A[k]
            Pc = wx[k] + A[k] ** 2 * Pc - Hux * Hux / Huu
    return P


def mobius(A, B, R, wx, wxu):
    rR = 1.0 / R
    return np.stack([A * A + (wx * B * B - 2.0 * wxu * A * B) * rR, wx - wxu * wxu * rR, B * B * rR,
                     np.ones_like(A)])


def rescale(m):
    mx = np.max(np.abs(m), axis=0)
    e = np.frexp(mx)[1]
    return np.ldexp(m, -e[None, :])


def suffix_scan_mob(m):
    """Hillis-Steele inclusive suffix scan of 2x2 maps (lane k: M_k M_{k+1} ...)."""
    n = m.shape[1]
    d = 1
    while d < n:
        p = np.concatenate([m[:, d:], np.tile(np.array([[1.0], [0.0], [0.0], [1.0]]), (1, d))], axis=1)
        m = rescale(np.stack([m[0] * p[0] + m[1] * p[2], m[0] * p[1] + m[1] * p[3],
                              m[2] * p[0] + m[3] * p[2], m[2] * p[1] + m[3] * p[3]]))
        d <<= 1
    return m


def random_stages(rng, N):
    A = rng.uniform(0.5, 1.2, N)
    B = rng.uniform(-1e-2, 1e-2, N) * 10.0 ** rng.uniform(-2, 1, N)
    wx = np.exp(rng.normal(0, 1.5, N))
    R = np.exp(rng.normal(0, 2, N))
    wxu = rng.uniform(-0.95, 0.95, N) * np.sqrt(wx * R)
    return A, B, R, wx, wxu


def test_one_step_is_linear_fractional():
    rng = np.random.default_rng(11)
    for _ in range(200):
        A, B, R, wx, wxu = [v[0] for v in random_stages(rng, 1)]
        P = np.exp(rng.normal(0, 3))
        Huu = R + B * B * P
        ser = wx + A * A * P - (wxu + B * P * A) ** 2 / Huu
        m = mobius(np.array([A]), np.array([B]), np.array([R]), np.array([wx]), np.array([wxu]))[:, 0]
        mob = (m[0] * P + m[1]) / (m[2] * P + m[3])
        assert mob == pytest.approx(ser, rel=1e-11)
        # a positive definite block gives non-negative map entries
        assert (wx * B * B + A * A * R - 2 * wxu * A * B) >= -1e-12 * (wx * B * B + A * A * R)
        assert wx * R - wxu * wxu > 0


def test_infinite_input_curvature_limit():
    # a slack that is exactly 0 in floating point makes R infinite: the
    # serial step tends to W_x + A^2 P, and so does the map divided by R
    A, B, wx, wxu, P = 0.98, -2.3e-4, 1167.0, 3.3, 2284.4
    with np.errstate(divide="ignore", invalid="ignore"):
        m = mobius(np.array([A]), np.array([B]), np.array([np.inf]), np.array([wx]), np.array([wxu]))[:, 0]
    assert np.all(np.isfinite(m))
    assert (m[0] * P + m[1]) / (m[2] * P + m[3]) == pytest.approx(wx + A * A * P, rel=1e-15)


@pytest.mark.parametrize("N", [1, 2, 5, 16, 17, 33, 60, 64])
def test_factor_scan_matches_serial(N):
    rng = np.random.default_rng(N)
    A, B, R, wx, wxu = random_stages(rng, N)
    PN = np.exp(rng.normal(0, 1))
    ref = serial_factor(PN, A, B, R, wx, wxu)
    m = mobius(A, B, R, wx, wxu)
    m[:, 0] = [1.0, 0.0, 0.0, 1.0]            # stage 0 has no state x_0
    # lane k starts with the map of stage k + 1 (identity past the stages)
    sh = np.concatenate([m[:, 1:], np.array([[1.0], [0.0], [0.0], [1.0]])], axis=1)
    t = suffix_scan_mob(rescale(sh))
    P = (t[0] * PN + t[1]) / (t[2] * PN + t[3])
    np.testing.assert_allclose(P, ref, rtol=1e-12)


def suffix_scan_aff(a, b):
    n = len(a)
    d = 1
    while d < n:
        a2 = np.concatenate([a[d:], np.ones(d)])
        b2 = np.concatenate([b[d:], np.zeros(d)])
        a, b = a * a2, a * b2 + b
        d <<= 1
    return a, b


def prefix_scan_aff(a, b):
    n = len(a)
    d = 1
    while d < n:
        a2 = np.concatenate([np.ones(d), a[:-d]])
        b2 = np.concatenate([np.zeros(d), b[:-d]])
        a, b = a * a2, a * b2 + b
        d <<= 1
    return a, b


@pytest.mark.parametrize("N", [1, 3, 16, 40, 64])
def test_affine_recursions_match_serial(N):
    rng = np.random.default_rng(100 + N)
    g = rng.uniform(0.8, 1.05, N)
    h = rng.normal(0, 1, N)
    rN = rng.normal()
    # backward: p_k = g_k p_{k+1} + h_k (k >= 1), p_N = rN; lane k needs p_{k+1}
    p = np.zeros(N)
    pc = rN
    for k in range(N - 1, -1, -1):
        p[k] = pc
        if k >= 1:
            pc = g[k] * pc + h[k]
    a = np.concatenate([g[1:], [1.0]])
    b = np.concatenate([h[1:], [0.0]])
    a, b = suffix_scan_aff(a, b)
    np.testing.assert_allclose(a * rN + b, p, rtol=1e-12, atol=1e-12 * np.abs(p).max())
    # forward: x_{k+1} = g_k x_k + h_k, x_0 = 0
    x = np.zeros(N)
    xc = 0.0
    for k in range(N):
        xc = g[k] * xc + h[k]
        x[k] = xc
    a, b = prefix_scan_aff(g.copy(), h.copy())
    np.testing.assert_allclose(b, x, rtol=1e-12, atol=1e-12 * np.abs(x).max())


def scan_ipm(cfg, N, U, A, B, C, FX, WXX, WXU, WUU, maxit):
    """The kernel's interior point (stage k at index k), with the three
    stage recursions as scans."""
    lo, hi = cfg["umin"] - U, cfg["umax"] - U
    k1 = np.arange(N) >= 1
    wxu = np.where(k1, WXU, 0.0)
    wxp = np.concatenate([[0.0], WXX[:-1]])
    fxp = np.concatenate([[0.0], FX[:-1]])
    PN, fxN = WXX[-1], FX[-1]
    prev = lambda v: np.concatenate([[0.0], v[:-1]])
    nxt = lambda v, f: np.concatenate([v[1:], [f]])
    dl = 1e-2 * (hi - lo)
    du = np.minimum(np.maximum(0.0, lo + dl), hi - dl)
    nl, nu, mu = np.ones(N), np.ones(N), np.zeros(N)
    dx = prefix_scan_aff(A.copy(), B * du + C)[1]
    gsc = np.abs(FX).max()
    for it in range(maxit + 1):
        dxk, mup = prev(dx), prev(mu)
        tl, tu = du - lo, hi - du
        wdu = WUU * du + wxu * dxk
        ru = wdu - mu * B - nl + nu
        Rt = WUU + nl / tl + nu / tu
        rt = ru + nl - nu
        wdx = wxp * dxk + wxu * du
        rx = wdx + fxp - mu * A + mup
        rxN = PN * dx[-1] + fxN + mu[-1]
        rmax = max(abs(rxN), np.abs(ru).max(), np.abs(rx[1:]).max(initial=0.0))
        wd = max(abs(PN * dx[-1]), np.abs(wdu).max(), np.abs(wdx[1:]).max(initial=0.0))
        comp = np.sum(tl * nl + tu * nu)
        muc = comp / (2.0 * N)
        if rmax <= 1e-12 * (1 + gsc + wd) and muc <= 1e-14 * (1 + gsc):
            return du, dx, mu
        m = mobius(A, B, Rt, wxp, wxu)
        m[:, 0] = [1.0, 0.0, 0.0, 1.0]
        sh = np.concatenate([m[:, 1:], np.array([[1.0], [0.0], [0.0], [1.0]])], axis=1)
        t = suffix_scan_mob(rescale(sh))
        Pn = (t[0] * PN + t[1]) / (t[2] * PN + t[3])
        Huu = Rt + B * B * Pn
        assert np.all(Huu > 0)
        hinv = 1.0 / Huu
        K = -(wxu + B * Pn * A) * hinv
        g = np.where(k1, B * K + A, 0.0)
        va, vb = suffix_scan_aff(nxt(g, 1.0), nxt(K * rt + rx, 0.0))
        e = va * rxN + vb
        kf = -(rt + B * e) * hinv
        fb = prefix_scan_aff(g.copy(), B * kf)[1]
        dua = K * prev(fb) + kf
        dnla, dnua = -nl - nl * dua / tl, -nu + nu * dua / tu
        with np.errstate(divide="ignore"):
            apr = min(1.0, np.min(np.where(dua < 0, -tl / dua, np.where(dua > 0, tu / dua, 1.0))))
            adr = min(1.0, np.min(np.where(dnla < 0, -nl / dnla, 1.0)), np.min(np.where(dnua < 0, -nu / dnua, 1.0)))
        maff = np.sum((tl + apr * dua) * (nl + adr * dnla) + (tu - apr * dua) * (nu + adr * dnua)) / (2.0 * N)
        smu = (maff / muc) ** 3 * muc
        taul, tauu = smu - dua * dnla, smu + dua * dnua
        rt2 = ru + nl - taul / tl - nu + tauu / tu
        ca, cb = suffix_scan_aff(nxt(g, 1.0), nxt(K * rt2 + rx, 0.0))
        e2 = ca * rxN + cb
        kf2 = -(rt2 + B * e2) * hinv
        ddx = prefix_scan_aff(g.copy(), B * kf2)[1]
        ddu = K * prev(ddx) + kf2
        dmu = -(Pn * ddx + e2)
        dnl, dnu = (-tl * nl + taul - nl * ddu) / tl, (-tu * nu + tauu + nu * ddu) / tu
        with np.errstate(divide="ignore"):
            ap = min(1.0, 0.995 * np.min(np.where(ddu < 0, -tl / ddu, np.where(ddu > 0, tu / ddu, 1.0))))
            ad = min(1.0, 0.995 * min(np.min(np.where(dnl < 0, -nl / dnl, 1.0)), np.min(np.where(dnu < 0, -nu / dnu, 1.0))))
        du, dx, mu, nl, nu = du + ap * ddu, dx + ap * ddx, mu + ad * dmu, nl + ad * dnl, nu + ad * dnu
    raise AssertionError("interior point did not converge")


@pytest.mark.parametrize("N", [1, 2, 10, 25, 60])
def test_scan_interior_point_reaches_the_oracle_qp(N):
    cfg = W.c1_paper_scale()
    rng = np.random.default_rng(7 * N)
    U = rng.uniform(cfg["umin"], cfg["umax"], N)
    A, B, _, WXX, _ = random_stages(rng, N)
    C = rng.normal(0, 1e-2, N)
    FX = rng.normal(0, 1, N) * 10.0 ** rng.uniform(-3, 1)
    WUU = np.exp(rng.normal(0, 2, N))
    WXU = np.zeros(N)
    for k in range(1, N):
        WXU[k] = rng.uniform(-0.9, 0.9) * np.sqrt(WXX[k - 1] * WUU[k])
    n = 2 * N
    Wd = np.zeros((n, n))
    gf = np.zeros(n)
    for k in range(N):
        Wd[2 * k, 2 * k] = WUU[k]
        Wd[2 * k + 1, 2 * k + 1] = WXX[k]
        gf[2 * k + 1] = FX[k]
        if k >= 1:
            Wd[2 * k - 1, 2 * k] = Wd[2 * k, 2 * k - 1] = WXU[k]
    st, dxi, mu, _, _, _ = oracle.ms_qp(cfg, Wd, gf, A, B, C, U)
    assert st == 0
    du, dx, mu2 = scan_ipm(cfg, N, U, A, B, C, FX, WXX, WXU, WUU, cfg["ipm_max_iter"])
    sc = np.abs(dxi).max()
    np.testing.assert_allclose(du, dxi[0::2], rtol=0, atol=1e-9 * sc)
    np.testing.assert_allclose(dx, dxi[1::2], rtol=0, atol=1e-9 * sc)
    np.testing.assert_allclose(mu2, mu, rtol=0, atol=1e-9 * np.abs(mu).max())
