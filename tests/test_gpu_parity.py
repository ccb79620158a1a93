"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Tolerances: per-sample Phi relative 1e-9 for PI and 1e-6 for NMPC; mean and
variance of each controller's Phi relative 1e-8; integer outputs (kind,
horizon, length, OCP counts, histogram) exact; every sample whose active-set
signature differs from the oracle's is a "flip" and fails the comparison.

NMPC cases run the SQP at the KKT tolerance EPS = 1e-10: at the throughput
default (1e-6, the NMPC per-sample bar itself) two roundings of the same
iteration can stop one SQP iteration apart.  At 1e-10 the oracle's two
mathematically equal gradient orders agree within 1e-8 on every sample of
these cases, except on c3 with its plant-model mismatch (see
test_c3_uneven_sampled).  Sizes: small cases span several wavefront groups
and a ragged tail; paper-scale configurations run strided subsets of their
sample ids (the sample_ids array) at full shape, in the launch shape the
benchmark uses.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a HIP device", allow_module_level=True)

import oracle  # noqa: E402
from paper_2212_02197_amd import binding, workloads as W  # noqa: E402

NTHREADS = min(16, len(os.sched_getaffinity(0)))
EPS = 1e-10


def gpu_run(cfg, traj=False):
    camp = binding.Campaign(cfg)
    camp.run(trajectories=traj)
    phi, stats = camp.costs()
    ps = camp.per_sample()
    tr = None
    if traj:
        tr = {k: v.cpu().numpy() for k, v in camp.traj.items()}
    camp.close()
    return phi, stats, ps, tr


def sample_ids(cfg):
    if cfg.get("sample_ids") is not None:
        return np.asarray(cfg["sample_ids"], dtype=np.int64)
    return np.arange(cfg["n_samples"], dtype=np.int64) + cfg.get("sample_id_offset", 0)


def oracle_run(cfg, ids=None):
    if ids is None:
        ids = sample_ids(cfg)
    return oracle.run(cfg, ids=np.asarray(ids, dtype=np.int64), nthreads=NTHREADS,
                      kind=cfg.get("kind"), horizon=cfg.get("horizon"),
                      lengths=cfg.get("lengths"))


def compare(phi_g, ps_g, ref, sel=None, tag=""):
    """Element-wise comparison at the bar: every NMPC sample within 1e-6,
    every PI sample within 1e-9, flipped or not.  Flips (an input within
    1e-6 mL/min of a bound in one run and not in the other at some OCP) are
    listed with their Phi errors.  Returns the max rel error per kind."""
    if sel is None:
        sel = np.arange(len(ref["phi"]))
    pg = phi_g[sel]
    kind = ref["kind"]
    # a diverged closed loop (Phi NaN) must diverge on both sides
    np.testing.assert_array_equal(np.isfinite(pg), np.isfinite(ref["phi"]), err_msg=tag)
    np.testing.assert_array_equal(ps_g["nonfinite"][sel], ref["nonfinite"], err_msg=tag)
    fin = np.isfinite(pg)
    rel = np.where(fin, np.abs(pg - ref["phi"]) / np.abs(np.where(fin, ref["phi"], 1.0)), 0.0)
    flips = np.nonzero(ps_g["ashash"][sel] != ref["ashash"])[0]
    for f in ("kind", "N", "L", "n_ocp"):
        np.testing.assert_array_equal(ps_g[f][sel], ref[f], err_msg=f"{tag} {f}")
    out = {}
    for k, tol in ((0, 1e-6), (1, 1e-9)):
        m = kind == k
        if not m.any():
            continue
        bad = np.nonzero(m & (rel > tol))[0]
        out[k] = float(rel[m].max())
        print(f"{tag} kind {k}: n={m.sum()} max rel {rel[m].max():.3e} flips {len(flips)} "
              f"above the bar {len(bad)}", flush=True)
        assert len(bad) == 0, (tag, k, bad[:5], rel[bad[:5]])
    # counters that rounding may move by one iteration are reported, not
    # compared; resets of W are rare events and must agree in total
    for f in ("n_ocp_fail", "sqp_iter", "ls_trials", "ls_cap", "bfgs_skip", "bfgs_reset"):
        d = ps_g[f][sel].astype(np.int64) - ref[f]
        print(f"{tag} counter {f}: gpu {ps_g[f][sel].sum()} oracle {ref[f].sum()} "
              f"max |diff| {np.abs(d).max()}", flush=True)
    # (a diverged sample's OCP on non-finite data takes other paths on each side)
    ok = ref["nonfinite"] == 0
    assert ps_g["bfgs_reset"][sel][ok].sum() == ref["bfgs_reset"][ok].sum(), tag
    for j in flips:
        print(f"{tag} flip: sample {j} kind {kind[j]} Phi rel {rel[j]:.2e}", flush=True)
    assert len(flips) <= max(1, len(sel) // 50), (tag, flips[:10])
    return out


def check_stats(stats, ref, kinds=(0, 1), hist=True):
    """Mean and variance of each controller's Phi within 1e-8 relative of the
    oracle's exact sums; histogram counts exact."""
    for k in kinds:
        m = ref["kind"] == k
        mo, vo, ho = oracle.stats(ref["phi"][m])
        assert stats["count"][k] == (m & np.isfinite(ref["phi"])).sum()
        print(f"stats kind {k}: n={m.sum()} mean {stats['mean'][k]:.12g} rel "
              f"{abs(stats['mean'][k] - mo) / mo:.2e} var rel "
              f"{abs(stats['var'][k] - vo) / vo:.2e}", flush=True)
        assert stats["mean"][k] == pytest.approx(mo, rel=1e-8)
        assert stats["var"][k] == pytest.approx(vo, rel=1e-8)
        if hist:
            np.testing.assert_array_equal(stats["hist"][k], ho)


def test_c0_small_nmpc_full():
    # two wavefronts of 32 samples (the automatic plan of so small a campaign
    # would give each sample a wavefront of its own): cooperative visits over
    # many samples and the paired line search
    cfg = W.c0_small_nmpc(samples_per_wave=32, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="c0")
    check_stats(stats, ref, kinds=(0,))


def test_c0_forward_sensitivity_mode():
    cfg = W.c0_small_nmpc(grad_mode=0, n_samples=40, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="c0-fwd")


def test_c1_pi_half_sampled():
    # paper-scale PI half: 640 strided ids of the 30,000 PI samples, full
    # L = 600, Ns = 20
    ids = 30000 + np.arange(0, 30000, 46)[:640]
    cfg = W.c1_paper_scale(n_samples=len(ids), sample_ids=ids)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="c1-pi")
    check_stats(stats, ref, kinds=(1,))


def test_c1_nmpc_production_shape():
    # paper-scale NMPC (N = 60, Nc = 5, L = 600, Ns = 20) on 256 strided ids
    # of the 30,000, in the benchmark's launch shape: 30 samples per
    # wavefront (NMAX 64, multi-sample cooperative visits, the paired line
    # search), 8 full wavefronts and a ragged ninth of 16
    ids = np.arange(0, 30000, 117)[:256]
    cfg = W.c1_paper_scale(n_samples=len(ids), sample_ids=ids, samples_per_wave=30,
                           sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert ps["n_ocp"].tolist() == [600] * len(ids)
    compare(phi, ps, ref, tag="c1-nmpc")
    check_stats(stats, ref, kinds=(0,))


def test_deterministic_runs_and_trajectories():
    # The KKT test stops the SQP once the scaled stationarity residual is
    # below eps; near that threshold two roundings of the same iteration can
    # stop one step apart, which moves the applied input by about eps
    # relative.  The element-wise trajectory comparison therefore runs at
    # eps = 1e-9, where that step is far below the 1e-5 tolerance on u.
    cfg = W.c1_paper_scale(n_samples=2, kind_split=1, noise_mod=1, noise_scale=0.0, N=20,
                           Ns=10, sqp_eps=1e-9)
    phi, stats, ps, tr = gpu_run(cfg, traj=True)
    for s in range(2):
        r = oracle.run_sample(cfg, s, traj=True)
        assert phi[s] == pytest.approx(r["phi"], rel=1e-6 if s == 0 else 1e-9)
        np.testing.assert_allclose(tr["z"][:, s], r["z"], rtol=1e-6 if s == 0 else 1e-9)
        np.testing.assert_allclose(tr["u"][:, s], r["u"], rtol=1e-5 if s == 0 else 1e-9,
                                   atol=1e-12)
    assert phi[0] < phi[1]  # NMPC beats PI in the deterministic case


def test_c3_uneven_sampled():
    # Uneven batch at full shape: N ~ U{10, 25, 50}, L ~ U{100..400}, plant
    # kinetics perturbed by lognormal factors (sigma 0.05), 128 strided ids.
    # The plant-model mismatch leaves some closed loops bang-bang between the
    # input bounds, where a rounding difference grows from interval to
    # interval: on those the oracle's two gradient orders (equal up to
    # rounding) themselves end more than 1e-6 apart, so Phi is not determined
    # at the per-sample bar by the inputs.  Determined samples (the two
    # orders within 1e-7, a tenth of the bar, same active sets) must meet the
    # bar.  On each rounding-sensitive sample the oracle follows itself
    # (outputs z within 1e-8) up to an interval t; up to there the GPU's z
    # must stay within 1e-6 of the oracle's.  Its error on the whole closed
    # loop is listed.
    ids = np.arange(0, 100000, 773)[:128]
    cfg = W.c3_uneven(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS)
    phi, stats, ps, tr = gpu_run(cfg, traj=True)
    ref = oracle_run(cfg)
    alt = oracle_run(dict(cfg, grad_mode=0))
    for f in ("kind", "N", "L", "n_ocp"):
        np.testing.assert_array_equal(ps[f], ref[f], err_msg=f)
    assert set(ps["N"].tolist()) == {10, 25, 50}
    rel_self = np.abs(alt["phi"] - ref["phi"]) / ref["phi"]
    det = (rel_self <= 1e-7) & (alt["ashash"] == ref["ashash"])
    g = np.nonzero(det)[0]
    print(f"c3: {det.sum()} of {len(det)} samples determined at 1e-7", flush=True)
    assert det.sum() >= 3 * len(det) // 4
    compare(phi, ps, {k: v[g] for k, v in ref.items() if k != "ids"}, sel=g, tag="c3 determined")
    rel = np.abs(phi - ref["phi"]) / ref["phi"]
    for j in np.nonzero(~det)[0]:
        cs = dict(cfg, sample_ids=None, n_samples=1)
        ra = oracle.run_sample(cs, int(ids[j]), traj=True)
        rb = oracle.run_sample(dict(cs, grad_mode=0), int(ids[j]), traj=True)
        L = int(ref["L"][j])
        z_g = tr["z"][:L + 1, j]
        dz = np.abs(ra["z"] - rb["z"]) > 1e-8 * np.abs(ra["z"])
        t = int(np.argmax(dz)) if dz.any() else L
        ez = np.abs(z_g[:t + 1] - ra["z"][:t + 1]) / ra["z"][:t + 1]
        print(f"c3 rounding-sensitive id {ids[j]} N {ref['N'][j]} L {L}: oracle follows itself "
              f"to interval {t}; there gpu z rel {ez.max():.2e}; whole loop gpu/oracle Phi rel "
              f"{rel[j]:.2e}, oracle/oracle {rel_self[j]:.2e}", flush=True)
        assert ez.max() <= 1e-6, ids[j]
    m, v, _ = oracle.stats(ref["phi"][g])
    m_g, v_g, _ = oracle.stats(phi[g])
    assert m_g == pytest.approx(m, rel=1e-8) and v_g == pytest.approx(v, rel=1e-8)


def test_diverged_plant_ends_the_closed_loop():
    # c3 id 1937 draws E_a/R = 6978 K (a -3.9 sigma kinetic factor): its plant
    # reacts about 100 times faster than the model and the Euler-Maruyama
    # sub-step diverges in the first interval.  Both sides stop that closed
    # loop when the plant output is no longer finite (Phi NaN, the
    # non-finite flag set, no further OCPs), and the statistics leave it out.
    ids = np.array([1936, 1937, 1938, 1939])
    cfg = W.c3_uneven(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert np.isnan(phi[1]) and ps["nonfinite"][1] == 1 and ps["n_ocp"][1] < ps["L"][1]
    compare(phi, ps, ref, tag="diverged plant")
    check_stats(stats, ref, kinds=(0,))
    assert stats["count"][0] == 3


def test_c3_all_horizon_classes_without_mismatch():
    # c3's horizons and ragged lengths at full shape with the nominal plant
    # kinetics (no model-plant mismatch): every sample at the bar
    ids = np.arange(5, 100000, 769)[:128]
    cfg = W.c3_uneven(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS, kin_lognorm_sigma=0.0)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert set(ps["N"].tolist()) == {10, 25, 50}
    assert len(set(ps["L"].tolist())) > 60
    compare(phi, ps, ref, tag="c3 nominal kinetics")
    check_stats(stats, ref, kinds=(0,))


def test_c4_mixed_strided_pairs():
    # c4's two halves: 128 strided NMPC ids (N = 25) and the PI samples that
    # share their noise ids, L = 300, +-10 % setpoint step
    nm = np.arange(11, 500000, 3901)[:128]
    ids = np.concatenate([nm, nm + 500000])
    cfg = W.c4_mixed(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert ps["kind"].tolist() == [0] * 128 + [1] * 128
    compare(phi, ps, ref, tag="c4")
    check_stats(stats, ref)


def test_c4_mixed_across_the_split():
    # ids 499,990 .. 500,009: ten NMPC (N = 25) then ten PI on shared noise ids
    cfg = W.c4_mixed(n_samples=20, sample_id_offset=499990, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="c4 split")
    assert ps["kind"].tolist() == [0] * 10 + [1] * 10


def test_caller_given_kind_horizon_and_length():
    # per-sample arrays in place of the campaign's rules: a PI sample among
    # NMPC ones, horizons of all three classes, lengths 0..13, repeated ids
    ids = np.array([3, 3, 17, 40, 41, 99, 5, 8])
    kind = np.array([0, 1, 0, 0, 1, 0, 0, 1], dtype=np.uint8)
    hor = np.array([10, 10, 20, 50, 7, 64, 1, 33], dtype=np.int32)
    lens = np.array([7, 7, 13, 0, 9, 4, 11, 2], dtype=np.int32)
    cfg = W.c0_small_nmpc(n_samples=len(ids), sample_ids=ids, kind=kind, horizon=hor,
                          lengths=lens, sqp_eps=EPS)
    phi, stats, ps, tr = gpu_run(cfg, traj=True)
    ref = oracle_run(cfg)
    np.testing.assert_array_equal(ps["kind"], kind)
    np.testing.assert_array_equal(ps["N"][kind == 0], hor[kind == 0])
    np.testing.assert_array_equal(ps["L"], lens)
    compare(phi, ps, ref, tag="caller arrays")
    assert tr["z"].shape == (lens.max() + 1, len(ids))
    for j in range(len(ids)):
        r = oracle.run_sample(dict(cfg, sample_ids=None, kind_split=-1,
                                   default_kind=int(kind[j]), N=int(hor[j]), L=int(lens[j]),
                                   n_samples=1), int(ids[j]), traj=True)
        np.testing.assert_allclose(tr["z"][:lens[j] + 1, j], r["z"],
                                   rtol=1e-6 if kind[j] == 0 else 1e-9)


def test_caller_workspace_matches_library_allocation():
    # every device buffer carved from one caller tensor sized by
    # mc_cl_workspace_size: bitwise the results of the library's own
    # allocations (three horizon classes, PI samples with the reverse pass);
    # a workspace one byte short is refused
    cfg = W.c3_uneven(n_samples=120, sample_id_offset=40, L_lo=6, L_hi=15, kind_split=130,
                      want_grad=1, sqp_eps=EPS)
    phi0, _, ps0, _ = gpu_run(cfg)
    camp = binding.Campaign(cfg)
    camp.run()
    g0, _ = camp.grad()
    camp.close()
    nbytes = binding.workspace_size(cfg)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    camp = binding.Campaign(cfg, workspace=ws)
    camp.run()
    phi, st = camp.costs()
    ps = camp.per_sample()
    g, _ = camp.grad()
    camp.close()
    print("caller workspace bytes", nbytes, "context reports", st["workspace_bytes"], flush=True)
    assert st["workspace_bytes"] == nbytes
    np.testing.assert_array_equal(phi, phi0)
    np.testing.assert_array_equal(ps["ashash"], ps0["ashash"])
    assert g == g0
    small = torch.empty(nbytes - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.McClError, match="ENOMEM"):
        binding.Campaign(cfg, workspace=small)


def test_pi_gradient_against_oracle_tangent():
    cfg = W.c2_pi_adjoint(n_samples=96, L=2000)
    camp = binding.Campaign(cfg)
    camp.run()
    phi, stats = camp.costs()
    g, ps = camp.grad(per_sample=True)
    gs = ps.cpu().numpy()
    camp.close()
    ref = oracle_run(cfg)
    rel = np.abs(phi - ref["phi"]) / ref["phi"]
    assert rel.max() <= 1e-9
    dref = ref["dphi"]
    for b in range(2):
        err = np.abs(gs[b] - dref[:, b])
        scale = np.abs(dref[:, b]).max()
        print("grad", b, "max abs err / scale %.3e" % (err.max() / scale), flush=True)
        assert err.max() <= 1e-9 * scale
    mean_ref = dref.mean(axis=0)
    assert g[0] == pytest.approx(mean_ref[0], rel=1e-9)
    assert g[1] == pytest.approx(mean_ref[1], rel=1e-9)


def test_pi_lanes_per_sample_do_not_change_results():
    # a PI campaign gives each sample 4, 2 or 1 lanes, the most that keep its
    # wavefronts at one per SIMD; planning for fewer compute units forces
    # each width on the same 640 samples (all CUs: 4 lanes, 40 wavefronts;
    # 8 CUs, 32 SIMDs: 2 lanes; 4 CUs, 16 SIMDs: 1 lane).  Costs,
    # trajectories and gradients are bitwise the same.
    cfg = W.c2_pi_adjoint(n_samples=640, L=60)
    runs = []
    for cu in (0, 8, 4):
        camp = binding.Campaign(dict(cfg, cu_limit=cu))
        camp.run(trajectories=True)
        phi, _ = camp.costs()
        g, gs = camp.grad(per_sample=True)
        tr = {k: v.cpu().numpy() for k, v in camp.traj.items()}
        runs.append((phi, np.asarray(g), gs.cpu().numpy(), tr))
        camp.close()
    phi0, g0, gs0, tr0 = runs[0]
    for phi, g, gs, tr in runs[1:]:
        np.testing.assert_array_equal(phi, phi0)
        np.testing.assert_array_equal(g, g0)
        np.testing.assert_array_equal(gs, gs0)
        for k in tr0:
            np.testing.assert_array_equal(tr[k], tr0[k], err_msg=k)
    ref = oracle_run(cfg)
    assert (np.abs(phi0 - ref["phi"]) / ref["phi"]).max() <= 1e-9


def test_launch_shape_does_not_change_results():
    cfg = W.c0_small_nmpc(n_samples=50, L=8)
    outs = []
    for spw in (8, 16, 64):
        phi, stats, ps, _ = gpu_run(dict(cfg, samples_per_wave=spw))
        outs.append((phi, ps["ashash"], ps["sqp_iter"]))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
        np.testing.assert_array_equal(o[2], outs[0][2])


def test_repeat_runs_are_bitwise_identical():
    cfg = W.c0_small_nmpc(n_samples=20, L=6, kind_split=10, noise_mod=10)
    camp = binding.Campaign(cfg)
    camp.run()
    a, _ = camp.costs()
    camp.run()
    b, _ = camp.costs()
    camp.close()
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("over", [dict(n_samples=1), dict(L=0), dict(N=1), dict(sqp_max_iter=1),
                                  dict(sqp_max_iter=0), dict(n_samples=65, L=3),
                                  dict(hess_warm=0, L=4)])
def test_edge_cases(over):
    cfg = W.c0_small_nmpc(**dict(dict(n_samples=5, L=5, sqp_eps=EPS), **over))
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag=f"edge {over}")
    if over.get("sqp_max_iter") is not None:
        # capped OCPs keep their last iterate; the failure counts agree
        np.testing.assert_array_equal(ps["n_ocp_fail"], ref["n_ocp_fail"])
        assert ps["n_ocp_fail"].sum() > 0


@pytest.mark.parametrize("qp", [0, 1])
def test_w_form_qp_solvers(qp):
    # the QP on the BFGS matrix W itself: interior point (0) and active set
    # with interior-point fallback (1); same closed loops as the default
    cfg = W.c0_small_nmpc(n_samples=24, qp_solver=qp, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag=f"qp_solver {qp}")


def test_mixed_horizons_share_wave_slots():
    # N ~ U{20, 30}: one NMAX class, so a wavefront's matrix slots are reused
    # by samples of both horizons (entries outside a sample's N x N block
    # must not leak into its QP); several groups and a ragged tail
    cfg = W.c0_small_nmpc(n_samples=70, L=12, horizon_choices=(20, 30), samples_per_wave=8,
                          sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert set(ps["N"].tolist()) == {20, 30}
    compare(phi, ps, ref, tag="mixed N")


def test_pi_autograd_function():
    # d mean Phi / d(Kc, tau_i) through torch.autograd over the library's
    # checkpointed reverse pass, against the mean of the oracle's pathwise
    # tangents d Phi_s / d(Kc, tau_i) and a central difference of the GPU
    # forward pass (relative step 1e-6)
    cfg = W.c2_pi_adjoint(n_samples=64, L=300, ckpt_interval=25)
    Kc, taui = cfg["kP"], cfg["kP"] / cfg["kI"]
    theta = torch.tensor([Kc, taui], dtype=torch.float64, device="cuda", requires_grad=True)
    phi = binding.pi_closed_loop(theta, cfg)
    loss = phi.mean()
    loss.backward()
    g = theta.grad.cpu().numpy()
    ref = oracle_run(cfg)
    g_ref = ref["dphi"].mean(axis=0)
    np.testing.assert_allclose(g, g_ref, rtol=1e-9)
    assert float(loss) == pytest.approx(ref["phi"].mean(), rel=1e-9)
    # theta on the host: the gradient comes back on the host
    th_cpu = theta.detach().cpu().requires_grad_(True)
    binding.pi_closed_loop(th_cpu, cfg).mean().backward()
    assert th_cpu.grad.device.type == "cpu"
    np.testing.assert_allclose(th_cpu.grad.numpy(), g, rtol=1e-12)
    for b in range(2):
        h = 1e-6 * abs(float(theta[b]))
        vals = []
        for sgn in (1, -1):
            th = theta.detach().clone()
            th[b] += sgn * h
            vals.append(float(binding.pi_closed_loop(th, cfg).mean()))
        fd = (vals[0] - vals[1]) / (2 * h)
        print("autograd", b, g[b], "central difference", fd, flush=True)
        assert g[b] == pytest.approx(fd, rel=1e-4, abs=1e-6 * abs(g).max())


def test_chunked_graph_run_matches_single_launch():
    # c4's mix (NMPC N = 25 below the split, PI above, +-10 % setpoint step)
    # in 5 chunks, each one replay of the captured chunk step: bitwise the
    # single-launch results, on every replay, and the oracle's on a sample
    cfg = W.c4_mixed(n_samples=600, kind_split=300, noise_mod=300, L=12, sp_step_lo=3,
                     sp_step_hi=9, sqp_eps=EPS)
    phi1, st1, ps1, _ = gpu_run(cfg)
    camp = binding.Campaign(dict(cfg, chunk_samples=130))
    outs = []
    for rep in range(3):
        camp.run()
        phi, st = camp.costs()
        ps = camp.per_sample()
        outs.append((phi, ps))
        torch.cuda.synchronize()
    camp.close()
    for phi, ps in outs:
        np.testing.assert_array_equal(phi, phi1)
        np.testing.assert_array_equal(ps["ashash"], ps1["ashash"])
        for f in binding.CNT_NAMES:
            np.testing.assert_array_equal(ps[f], ps1[f], err_msg=f)
    ids = np.arange(0, 600, 37)
    ref = oracle_run(cfg, ids=ids)
    compare(phi1, ps1, ref, sel=ids, tag="c4 chunked")


def test_concurrent_horizon_classes_match_sequential_launches():
    # three horizon classes (N 10 / 25 / 50) with ragged lengths: with
    # class_streams an unchunked run on the whole device launches them on
    # concurrent streams; by default one after another on the caller's
    # stream.  Bitwise the same results.
    cfg = W.c3_uneven(n_samples=90, sample_id_offset=7000, L_lo=15, L_hi=40, samples_per_wave=8)
    phi_c, _, ps_c, _ = gpu_run(dict(cfg, class_streams=1))
    phi_s, _, ps_s, _ = gpu_run(cfg)
    assert set(ps_c["N"].tolist()) == {10, 25, 50}
    np.testing.assert_array_equal(phi_c, phi_s)
    np.testing.assert_array_equal(ps_c["ashash"], ps_s["ashash"])
    for f in binding.CNT_NAMES:
        np.testing.assert_array_equal(ps_c[f], ps_s[f], err_msg=f)


def test_three_state_chunked_graph_run_matches_single_launch():
    cfg = W.c0_small_nmpc(n_samples=96, L=10, model_nx=3, samples_per_wave=16)
    phi1, _, ps1, _ = gpu_run(cfg)
    camp = binding.Campaign(dict(cfg, chunk_samples=40))
    for rep in range(2):
        camp.run()
        phi, _ = camp.costs()
        ps = camp.per_sample()
        np.testing.assert_array_equal(phi, phi1)
        np.testing.assert_array_equal(ps["sqp_iter"], ps1["sqp_iter"])
    camp.close()


def test_tune_keeps_results_and_picks_a_candidate():
    cfg = W.c0_small_nmpc(n_samples=300, L=10, kind_split=200, noise_mod=200)
    phi0, _, ps0, _ = gpu_run(cfg)
    camp = binding.Campaign(dict(cfg, want_grad=1))
    res = camp.tune(trial_intervals=3)
    print("tune", res, flush=True)
    # each candidate is a cap evened out over the resident wavefronts
    assert 1 <= res["classes"][0]["spw"] <= max(binding.TUNE_SPW)
    assert all(v > 0 for v in res["classes"][0]["trial_ms"].values())
    assert res["ckpt_interval"] in binding.TUNE_CKPT
    # lanes per PI sample: the 100 PI samples timed at 1, 2 and 4 lanes
    assert res["pi_lanes"] in binding.TUNE_PI_LANES
    assert all(v > 0 for v in res["pi_trial_ms"].values())
    assert camp.plan()[0]["spw"] == res["classes"][0]["spw"]
    camp.run()
    phi, st = camp.costs()
    ps = camp.per_sample()
    g, _ = camp.grad()
    camp.close()
    np.testing.assert_array_equal(phi, phi0)
    np.testing.assert_array_equal(ps["ashash"], ps0["ashash"])
    # the checkpoint interval moves the gradient by rounding only (each
    # segment is recomputed from its checkpoint by the reverse kernel's own
    # code, whose rounding may differ from the forward kernel's)
    camp = binding.Campaign(dict(cfg, want_grad=1, ckpt_interval=3))
    camp.run()
    camp.costs()
    g3, _ = camp.grad()
    camp.close()
    assert g[0] == pytest.approx(g3[0], rel=1e-12)
    assert g[1] == pytest.approx(g3[1], rel=1e-12)


def test_cu_limited_stream_matches_full_device():
    # planning for 16 compute units and running on a stream limited to them
    # changes the launch shape only: results bitwise equal, and the oracle's
    cfg = W.c0_small_nmpc(n_samples=70, L=6, sqp_eps=EPS)
    phi0, _, ps0, _ = gpu_run(cfg)
    cs = binding.CuStream(16)
    camp = binding.Campaign(dict(cfg, cu_limit=16))
    camp.run(stream=cs.stream)
    phi, _ = camp.costs()
    ps = camp.per_sample()
    camp.close()
    cs.close()
    np.testing.assert_array_equal(phi, phi0)
    np.testing.assert_array_equal(ps["ashash"], ps0["ashash"])
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="cu16")


# ------------------------------------------------------ three-state model ---
# The estimator and the OCP on the three-state eq. (CSTR) model (model_nx 3):
# same tolerances as the one-state cases.

def test_three_state_c0_full():
    # 64 NMPC samples, N = 10 (the 16-wide horizon class), perturbed
    # steady-state starts; the model matches the plant apart from the noise
    cfg = W.c0_small_nmpc(model_nx=3, samples_per_wave=16, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="c0-3state")
    check_stats(stats, ref, kinds=(0,))


def test_three_state_all_horizon_classes_and_pi_estimator():
    # horizons 10 / 25 / 50 (all three kernel classes) with ragged lengths,
    # then PI samples that run the three-state filter for their estimates
    cfg = W.c3_uneven(n_samples=30, sample_id_offset=5000, model_nx=3, kin_lognorm_sigma=0.0,
                      L_lo=20, L_hi=45, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    for f in ("kind", "N", "L", "n_ocp"):
        np.testing.assert_array_equal(ps[f], ref[f], err_msg=f)
    assert set(ps["N"].tolist()) == {10, 25, 50}
    compare(phi, ps, ref, tag="3state classes")


def test_three_state_trajectories_and_estimates():
    # stochastic closed loops, element by element: z, u and the filter's n_T
    # estimate (NMPC sample 0, PI sample 1 with the three-state filter)
    cfg = W.c1_paper_scale(n_samples=2, kind_split=1, noise_mod=1, N=20, Ns=10, L=60,
                           sqp_eps=1e-9, model_nx=3)
    phi, stats, ps, tr = gpu_run(cfg, traj=True)
    for s in range(2):
        r = oracle.run_sample(cfg, s, traj=True)
        tol = 1e-6 if s == 0 else 1e-9
        assert phi[s] == pytest.approx(r["phi"], rel=tol)
        np.testing.assert_allclose(tr["z"][:, s], r["z"], rtol=tol)
        np.testing.assert_allclose(tr["xhat"][:, s], r["xhat"], rtol=tol)
        np.testing.assert_allclose(tr["u"][:, s], r["u"], rtol=1e-5 if s == 0 else 1e-9,
                                   atol=1e-12)


def test_three_state_paired_line_search_is_the_serial_one():
    # at most 32 samples per wavefront the line search evaluates two trial
    # steps per pass on paired lanes; 64 per wavefront is the serial search
    cfg = W.c0_small_nmpc(n_samples=40, L=8, model_nx=3)
    outs = []
    for spw in (16, 64):
        phi, stats, ps, _ = gpu_run(dict(cfg, samples_per_wave=spw))
        outs.append((phi, ps["ashash"], ps["sqp_iter"], ps["ls_trials"]))
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("over", [dict(n_samples=1), dict(L=0), dict(N=1), dict(sqp_max_iter=1),
                                  dict(n_samples=65, L=3)])
def test_three_state_edge_cases(over):
    cfg = W.c0_small_nmpc(**dict(dict(n_samples=5, L=5, model_nx=3, sqp_eps=EPS), **over))
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag=f"3state edge {over}")


# ------------------------------------------------- multiple shooting (NLP) ---
# The paper's NLP formulation (nlp_form 1): states and inputs as decision
# variables, the structured QP by a Riccati-recursion interior point, Powell's
# l1 merit, the block BFGS from W^[0] = I at every OCP.  Same bar.

def test_multiple_shooting_c0_full():
    cfg = W.c0_small_nmpc(nlp_form=1, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="ms c0")
    check_stats(stats, ref, kinds=(0,))
    print("ms c0: OCP fails gpu", ps["n_ocp_fail"].sum(), "oracle", ref["n_ocp_fail"].sum(),
          "SQP iterations per OCP gpu", ps["sqp_iter"].sum() / ps["n_ocp"].sum(), flush=True)


def test_multiple_shooting_paper_horizon_strided():
    # N = 60, Nc = 5, Ns = 20 on 64 strided c1 NMPC ids (one wavefront),
    # the first 80 intervals (inlet start-up and the first setpoint)
    ids = np.arange(0, 30000, 469)[:64]
    cfg = W.c1_paper_scale(n_samples=len(ids), sample_ids=ids, L=80, nlp_form=1, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag="ms c1")
    check_stats(stats, ref, kinds=(0,))


def test_multiple_shooting_paper_scale_full_length():
    # the benchmark's multiple-shooting workload at full shape: N = 60, 600
    # intervals with both setpoint changes, 16 strided c1 NMPC ids
    ids = np.arange(3, 30000, 1873)[:16]
    cfg = W.c1_paper_scale(n_samples=len(ids), sample_ids=ids, nlp_form=1, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert (ps["L"] == 600).all() and (ps["kind"] == 0).all()
    compare(phi, ps, ref, tag="ms c1 full length")
    check_stats(stats, ref, kinds=(0,))


def test_multiple_shooting_c4_mixed_strided_pairs():
    # c4's shape on the paper's NLP: N = 25 (32-lane segments, two samples
    # per wavefront), L = 300 with the +-10 % setpoint step, NMPC ids and
    # the PI samples that share their noise ids.  KKT tolerance 1e-8: the
    # block BFGS restarts from I at every OCP and gains about one decade of
    # the KKT measure per 12 iterations here, so at 1e-10 a quarter of these
    # OCPs run to the 100-iteration cap (1.5 % at 1e-8, the cap rate of the
    # single-shooting c4 case at 1e-10)
    nm = np.arange(29, 500000, 7817)[:32]
    ids = np.concatenate([nm, nm + 500000])
    cfg = W.c4_mixed(n_samples=len(ids), sample_ids=ids, sqp_eps=1e-8, nlp_form=1)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert ps["kind"].tolist() == [0] * 32 + [1] * 32
    compare(phi, ps, ref, tag="ms c4")
    check_stats(stats, ref)


def test_multiple_shooting_mixed_classes_and_pi():
    # horizons of all three kernel classes with ragged lengths, then PI
    # samples (which do not solve OCPs)
    cfg = W.c3_uneven(n_samples=90, sample_id_offset=300, L_lo=10, L_hi=30, nlp_form=1,
                      kin_lognorm_sigma=0.0, kind_split=370, sqp_eps=EPS)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert set(ps["N"][ps["kind"] == 0].tolist()) == {10, 25, 50}
    assert (ps["kind"] == 1).sum() == 20
    compare(phi, ps, ref, tag="ms classes")


def test_multiple_shooting_trajectories_and_single_shooting():
    # element-wise z and u of a noise-free closed loop against the oracle; the
    # single-shooting path reaches the same inputs (each OCP has one
    # minimiser), so its trajectory agrees within the SQP tolerance's effect
    cfg = W.c1_paper_scale(n_samples=1, kind_split=-1, default_kind=0, noise_scale=0.0, N=20,
                           Ns=10, L=60, nlp_form=1, sqp_eps=EPS)
    phi, stats, ps, tr = gpu_run(cfg, traj=True)
    r = oracle.run_sample(cfg, 0, traj=True)
    np.testing.assert_allclose(tr["z"][:, 0], r["z"], rtol=1e-9)
    np.testing.assert_allclose(tr["u"][:, 0], r["u"], rtol=1e-6, atol=1e-12)
    phi_s, _, ps_s, tr_s = gpu_run(dict(cfg, nlp_form=0, sqp_max_iter=3000), traj=True)
    np.testing.assert_allclose(tr_s["z"][:, 0], tr["z"][:, 0], rtol=1e-8)
    assert ps["n_ocp_fail"][0] == 0


def test_multiple_shooting_chunked_and_concurrent_classes():
    # the segmented kernel under chunked graph replays (each chunk a range
    # of every class's queue) and with the classes on concurrent streams:
    # bitwise the single sequential launch, on every replay.  Nominal plant
    # kinetics: with c3's plant-model mismatch one of these 90 samples takes
    # a W reset the oracle does not (Phi within 8.5e-9), a rounding-sensitive
    # block near indefiniteness, which is not what this test is about
    cfg = W.c3_uneven(n_samples=90, sample_id_offset=7000, L_lo=15, L_hi=40, nlp_form=1, sqp_eps=EPS,
                      kin_lognorm_sigma=0.0)
    phi1, _, ps1, _ = gpu_run(cfg)
    assert set(ps1["N"].tolist()) == {10, 25, 50}
    runs = [gpu_run(dict(cfg, class_streams=1))[::2]]
    camp = binding.Campaign(dict(cfg, chunk_samples=25))
    for rep in range(2):
        camp.run()
        phi, _ = camp.costs()
        runs.append((phi, camp.per_sample()))
        torch.cuda.synchronize()
    camp.close()
    for phi, ps in runs:
        np.testing.assert_array_equal(phi, phi1)
        np.testing.assert_array_equal(ps["ashash"], ps1["ashash"])
        for f in binding.CNT_NAMES:
            np.testing.assert_array_equal(ps[f], ps1[f], err_msg=f)
    ref = oracle_run(cfg)
    compare(phi1, ps1, ref, tag="ms chunked classes")


def test_multiple_shooting_c3_shape_all_segment_widths():
    # c3's horizons (16-, 32- and 64-lane segments: four, two and one sample
    # per wavefront) and ragged lengths 100..400 at full shape, nominal plant
    # kinetics; segments refill from the queue at different intervals
    ids = np.arange(5, 100000, 769)[:96]
    cfg = W.c3_uneven(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS, kin_lognorm_sigma=0.0,
                      nlp_form=1)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert set(ps["N"].tolist()) == {10, 25, 50}
    assert len(set(ps["L"].tolist())) > 50
    compare(phi, ps, ref, tag="ms c3 nominal kinetics")
    check_stats(stats, ref, kinds=(0,))


def test_multiple_shooting_diverged_plant_stays_in_its_segment():
    # the diverging c3 sample of test_diverged_plant_ends_the_closed_loop
    # (id 1937, N = 10) on the paper's NLP: its 16-lane segment shares a
    # wavefront with the segments of the two other N = 10 samples, which
    # must not see its non-finite values; the closed loop stops on both
    # sides alike
    ids = np.array([1936, 1937, 1938, 1939])
    cfg = W.c3_uneven(n_samples=len(ids), sample_ids=ids, sqp_eps=EPS, nlp_form=1)
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    assert ps["N"].tolist() == [10, 10, 10, 25]
    assert np.isnan(phi[1]) and ps["nonfinite"][1] == 1 and ps["n_ocp"][1] < ps["L"][1]
    compare(phi, ps, ref, tag="ms diverged plant")
    check_stats(stats, ref, kinds=(0,))
    assert stats["count"][0] == 3


@pytest.mark.parametrize("over", [dict(n_samples=1), dict(L=0), dict(N=1), dict(sqp_max_iter=1),
                                  dict(sqp_max_iter=0), dict(n_samples=65, L=3)])
def test_multiple_shooting_edge_cases(over):
    cfg = W.c0_small_nmpc(**dict(dict(n_samples=5, L=5, sqp_eps=EPS, nlp_form=1), **over))
    phi, stats, ps, _ = gpu_run(cfg)
    ref = oracle_run(cfg)
    compare(phi, ps, ref, tag=f"ms edge {over}")
    if over.get("sqp_max_iter") is not None:
        np.testing.assert_array_equal(ps["n_ocp_fail"], ref["n_ocp_fail"])
