"""Seeded synthetic workload recipes for the Monte Carlo closed-loop CSTR.

Plain parameter data only: no arithmetic of the method lives here, so both the
HIP library and the CPU oracle can be fed from the same recipe.  Every noise
draw is made inside each side from (seed, sample id, step, tag) by Philox.

Sources of the values (arXiv 2212.02197):
  * Results section, "Closed-loop simulation": t0 = 0, tf = 600 s, Ts = 1 s,
    Ns = 20, N = 60, Nc = 5 RK4 steps, Qz = 1, x-hat_{-1|-1} = c_T,in V,
    P_{-1|-1} = 1e-6, 0 <= u <= 1000 mL/min, kP = -1e-3, kI = -1e-4, kaw = -1e-1,
    x0 = C_in V.
  * SQP section: c1 = 1e-4, beta = 0.5, s_max = 100; max 100 iterations
    (Results section, Table I discussion).
  * The paper defers the CSTR parameters to its reference on the adiabatic
    CSTR; the values below are that literature's (V = 0.105 L, k0 = e^24.6,
    Ea/R = 8500 K, beta = 560 / 4.186, c_A,in = 0.8, c_B,in = 1.2 mol/L,
    c_T,in = 273.65 K) and are project defaults, as are the noise levels, the
    setpoint schedule (the figure is missing) and the SQP tolerance.
"""
from __future__ import annotations

import copy

# Model and controller defaults (see the module docstring for provenance).
BASE = dict(
    V=0.105,
    k0=48266327438.62814,          # e^24.6  (L/(mol s))
    EaR=8500.0,                    # K
    beta=133.77926421404683,       # 560 / 4.186  (K L / mol)
    cAin=0.8, cBin=1.2, cTin=273.65,
    sigma=(0.01, 0.02, 5.0),       # diffusion diag(sigma_A, sigma_B, sigma_T)
    Rmeas=0.01,                    # K^2
    Ts=1.0, Ns=20, L=600,
    sp_i=(0, 200, 400), sp_z=(320.0, 335.0, 300.0), sp_period=0,
    sp_step_rel=0.0, sp_step_lo=0, sp_step_hi=0,
    N=60, Nc=5, Qz=1.0, umin=0.0, umax=1000.0,
    sqp_eps=1e-6, ls_c1=1e-4, ls_beta=0.5,
    sqp_max_iter=100, ls_max_bt=40, grad_mode=1, ipm_max_iter=50,
    want_grad=0,
    kP=-1e-3, kI=-1e-4, kaw=-1e-1, pi_umin=0.0, pi_umax=1.0 / 60.0,
    P0=1e-6, x0_rel_std=0.01, x0_mode=0,
    kind_split=-1, default_kind=0, run_ekf_for_pi=1,
    seed=0, noise_mod=0,
    horizon_choices=(), L_lo=0, L_hi=0,
    kin_lognorm_sigma=0.0,
    hess_warm=1,
    noise_scale=1.0,
    n_samples=1,
    sample_id_offset=0,            # first sample id (chunks, subsets)
    ckpt_interval=0,               # PI reverse pass checkpoint spacing (0: library default)
    samples_per_wave=0,            # NMPC lanes per wavefront (0: library plan)
    qp_solver=2,                   # 2 inverse form, 1 active set on W, 0 interior point on W
    chunk_samples=0,               # > 0: chunked run, one captured graph replay per chunk
    cu_limit=0,                    # > 0: plan for this many compute units (CU-masked stream)
    model_nx=1,                    # NMPC/EKF model: 1 the paper's one-state, 3 the three-state
    nlp_form=0,                    # OCP: 0 single shooting, 1 multiple shooting (the paper's NLP)
    class_streams=0,               # 1: NMPC horizon classes on concurrent streams
    # optional per-sample arrays of n_samples entries (None: the rules above)
    sample_ids=None,               # global sample ids (strided subsets, any order)
    kind=None,                     # 0 NMPC, 1 PI
    horizon=None,                  # N per sample
    lengths=None,                  # L per sample
)


def make(**over):
    """A copy of BASE with overrides."""
    cfg = copy.deepcopy(BASE)
    for k, v in over.items():
        if k not in cfg:
            raise KeyError(f"unknown workload key {k!r}")
        cfg[k] = v
    return cfg


def c0_small_nmpc(**over):
    """64 NMPC samples, 20 intervals, N = 10, Ns = 10, seed 0, steady-state
    start perturbed by (1 + 0.01 xi) per component, setpoint 320 K."""
    cfg = make(n_samples=64, L=20, Ns=10, N=10, seed=0, x0_mode=1,
               sp_i=(0,), sp_z=(320.0,), default_kind=0)
    cfg.update(over)
    return cfg


def c1_paper_scale(**over):
    """30,000 NMPC + 30,000 PI samples on shared noise (seed 1), L = 600,
    Ns = 20, N = 60, inlet start, 320 / 335 / 300 K schedule."""
    cfg = make(n_samples=60000, L=600, Ns=20, N=60, seed=1, x0_mode=0,
               kind_split=30000, noise_mod=30000)
    cfg.update(over)
    return cfg


def c2_pi_adjoint(**over):
    """10,000 PI samples, 2,000 intervals, Ns = 10, seed 2, schedule repeated
    every 600 intervals, inlet start; gradient w.r.t. (Kc, tau_i)."""
    cfg = make(n_samples=10000, L=2000, Ns=10, seed=2, x0_mode=0,
               sp_period=600, default_kind=1, want_grad=1)
    cfg.update(over)
    return cfg


def c3_uneven(**over):
    """100,000 NMPC samples, N ~ U{10, 25, 50}, L ~ U{100..400}, Ns = 10,
    plant kinetics perturbed by lognormal factors (sigma 0.05), steady-state
    start as c0, seed 3, adjoint-gradient SQP."""
    cfg = make(n_samples=100000, Ns=10, N=50, seed=3, x0_mode=1,
               horizon_choices=(10, 25, 50), L_lo=100, L_hi=400, L=400,
               kin_lognorm_sigma=0.05, default_kind=0, grad_mode=1)
    cfg.update(over)
    return cfg


def c4_mixed(**over):
    """1,000,000 samples: ids < 500,000 NMPC (N = 25), the rest PI on shared
    noise; L = 300, Ns = 10, 320 K with a +-10 % step at U{50..250}; seed 4."""
    cfg = make(n_samples=1000000, L=300, Ns=10, N=25, seed=4, x0_mode=1,
               sp_i=(0,), sp_z=(320.0,), sp_step_rel=0.1, sp_step_lo=50,
               sp_step_hi=250, kind_split=500000, noise_mod=500000)
    cfg.update(over)
    return cfg


CONFIGS = {
    "c0": c0_small_nmpc,
    "c1": c1_paper_scale,
    "c2": c2_pi_adjoint,
    "c3": c3_uneven,
    "c4": c4_mixed,
}
