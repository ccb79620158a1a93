"""Benchmark: closed-loop Monte Carlo of the stochastic CSTR on one MI355X.

One step = one whole campaign of the paper-scale workload (30,000 NMPC +
30,000 PI closed loops on shared Philox noise, L = 600, Ns = 20, N = 60,
Nc = 5, FP64): every sample's plant, estimator and controller, then the Phi
statistics.  Inputs are seeded and synthetic; nothing crosses PCIe inside the
timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X: 256 CU x 128 FP64 FLOP/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--samples", type=int, default=0, help="override n_samples (development)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the adjoint-vs-plain comparison")
    ap.add_argument("--plain-samples", type=int, default=3000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the planned launch shape (skip the measured tuning)")
    ap.add_argument("--tune-intervals", type=int, default=6)
    ap.add_argument("--cu-scaling", action="store_true",
                    help="also measure NMPC throughput against compute units (CU-masked streams)")
    ap.add_argument("--model-nx", type=int, default=1, choices=(1, 3),
                    help="estimator / OCP model: 1 the paper's one-state model, 3 the three-state model")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--plain-configs", default="c0,c1,c3,c4",
                    help="configs of the adjoint-vs-plain comparison (subsets, equal eps)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the eps = 1e-8, Hessian-start and multiple-shooting side runs")
    ap.add_argument("--nlp-form", type=int, default=0, choices=(0, 1),
                    help="OCP discretisation: 0 single shooting, 1 the paper's multiple shooting")
    ap.add_argument("--eps", type=float, default=0.0, help="SQP KKT tolerance (0: the recipe's)")
    ap.add_argument("--ckpt", type=int, default=0,
                    help="PI reverse pass: intervals per checkpoint (0: the tuner's choice)")
    return ap.parse_args()


def kernel_source_sha256(multiple_shooting=False):
    """Hash of the kernel sources (csrc/*.hpp, csrc/*.hip sorted by name).
    The single-shooting and PI kernels do not depend on mc_ms.hpp (the
    multiple-shooting kernel), so their hash leaves it out unless asked."""
    import glob
    import hashlib
    d = os.path.join(ROOT, "paper_2212_02197_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(d, "*.hpp")) + glob.glob(os.path.join(d, "*.hip"))):
        if not multiple_shooting and os.path.basename(f) == "mc_ms.hpp":
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per NMPC launch from the committed counter summary, or None
    when the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "nmpc_kernel_c1_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and parts[0] in ("source_sha256", "traffic_bytes_per_launch"):
                vals[parts[0]] = parts[1]
    if vals.get("source_sha256") != kernel_source_sha256() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def host_cpu():
    """Host CPU model name and logical CPU counts (all, and this process's)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(cfg, seconds):
    """The oracle, as it stands, on the host cores: NMPC closed loops of the
    same workload, sample ids 0, 1, ... until about `seconds` of wall time.
    Threads: the CPUs this process may use, at most 16 (one GPU's share of a
    GPU host)."""
    import numpy as np

    import oracle
    model, n_all, n_aff = host_cpu()
    cores = min(16, n_aff)
    n_nmpc = cfg["kind_split"] if cfg["kind_split"] >= 0 else cfg["n_samples"]
    done, wall, batch, start = 0, 0.0, cores, 0
    while wall < seconds and start < n_nmpc:
        ids = np.arange(start, min(start + batch, n_nmpc), dtype=np.int64)
        t0 = time.perf_counter()
        oracle.run(cfg, ids=ids, nthreads=cores)
        wall += time.perf_counter() - t0
        done += len(ids)
        start += len(ids)
        log(f"cpu baseline: {done} samples, {wall:.1f} s")
    return dict(value=done / wall, unit="NMPC closed-loop sims/s", cores=cores, kind="oracle",
                sample=f"NMPC sample ids 0..{done - 1} of the same workload ({done} closed loops, "
                       f"{wall:.1f} s wall on {cores} threads; linear in the sample count, the "
                       f"samples being independent)",
                host_cpu_model=model, host_logical_cpus=n_all, cpus_available=n_aff)


def describe(cfg, name):
    """The workload in words, with the per-sample draws where there are any."""
    N = ("N~U{" + ",".join(str(v) for v in cfg["horizon_choices"]) + "}"
         if cfg["horizon_choices"] else f"N={cfg['N']}")
    L = (f"L~U{{{cfg['L_lo']}..{cfg['L_hi']}}}" if cfg["L_lo"] < cfg["L_hi"] else f"L={cfg['L']}")
    extra = []
    if cfg["kin_lognorm_sigma"] > 0:
        extra.append(f"plant kinetics x lognormal(sigma {cfg['kin_lognorm_sigma']})")
    if cfg["sp_step_rel"] != 0:
        extra.append(f"setpoint step +-{cfg['sp_step_rel']:.0%} at U{{{cfg['sp_step_lo']}.."
                     f"{cfg['sp_step_hi']}}}")
    if cfg.get("nlp_form", 0) == 1:
        extra.append("multiple-shooting NLP")
    if cfg.get("model_nx", 1) == 3:
        extra.append("three-state estimator and OCP model")
    return (f"{name}: {N}, {L}, Ns={cfg['Ns']}, Nc={cfg['Nc']}, seed={cfg['seed']}, "
            f"SQP eps={cfg['sqp_eps']}, {'adjoint' if cfg['grad_mode'] == 1 else 'forward-sensitivity'}"
            f" gradient" + "".join(", " + e for e in extra))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU; --gpus above 1 is not supported "
              "(samples are independent: a multi-GPU campaign shards sample ids)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2212_02197_amd import binding, workloads
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", 0)))
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)   # reads and writes n * 8 bytes
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read and written")
        del a, b
    cfg = workloads.CONFIGS[args.config](model_nx=args.model_nx, nlp_form=args.nlp_form)
    if args.eps > 0:
        cfg["sqp_eps"] = args.eps
    if args.ckpt > 0:
        cfg["ckpt_interval"] = args.ckpt
    if args.samples:
        cfg["n_samples"] = args.samples
        if cfg["kind_split"] >= 0:
            cfg["kind_split"] = args.samples // 2
            cfg["noise_mod"] = args.samples // 2
    S = cfg["n_samples"]
    camp = binding.Campaign(cfg)
    log(f"campaign {args.config}: {S} samples, launch plan {camp.plan()}")
    tuning = None
    if not args.no_tune:
        # measured launch shape, chosen before (outside) the timed region
        tuning = camp.tune(trial_intervals=args.tune_intervals)
        log(f"tuned launch shape: {tuning}; plan {camp.plan()}")
    for w in range(args.warmup):
        camp.run()
        camp.costs()
        log(f"warmup step {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        camp.run()
        if args.steps > 1:
            torch.cuda.synchronize()
            log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed region: {(t1 - t0) * 1000.0 / args.steps:.1f} ms per step")
    phi, stats = camp.costs()
    ms_kernels = camp.kernel_ms()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    # samples per controller (all of them: a diverged closed loop counts as
    # simulated, though the Phi statistics leave it out)
    n_pi = stats["totals"]["kind"]
    n_nmpc = S - n_pi
    value = n_nmpc / (ms_per_step / 1000.0) if n_nmpc else S / (ms_per_step / 1000.0)
    tot = stats["totals"]
    plan = camp.plan()
    # dominant kernel: the NMPC closed loop.  Algorithmic FP64 work of its
    # samples (per-sample table x counters, summed on the device) over its
    # duration from HIP events on the launch stream (last timed step).
    nmpc_flops = stats["flops_by_kind"][0]
    nmpc_ms = ms_kernels[0]
    roofline = None
    # a chunked run's event spans mix the NMPC and PI kernels (ms[1] = -1):
    # no per-kernel rate is derived from them
    per_kernel = ms_kernels[1] >= 0
    if n_nmpc and nmpc_ms > 0 and per_kernel:
        achieved = nmpc_flops / (nmpc_ms / 1000.0) / 1e12
        standard = (args.config == "c1" and not args.samples and args.model_nx == 1
                    and args.nlp_form == 0 and args.eps == 0)
        traffic = measured_traffic() if standard else None
        roofline = dict(bound="alu", achieved=round(achieved, 4),
                        peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5),
                        traffic=traffic)
        if traffic:
            # what the committed counters show besides the algorithmic rate
            roofline["hbm_frac_measured"] = round(traffic / (nmpc_ms / 1000.0) / (HBM_PEAK_GBS * 1e9), 4)
    camp_flops = stats["flops_algorithmic"]
    pi_grad = None
    if cfg.get("want_grad") and n_pi and per_kernel:
        # the PI reverse pass (checkpointed adjoint through the closed loop)
        # after the timed forward step: d mean Phi / d(Kc, tau_i)
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        g, _ = camp.grad()
        torch.cuda.synchronize()
        tg1 = time.perf_counter()
        ms_grad = camp.kernel_ms()[3]
        pi_grad = dict(samples=n_pi, forward_ms=round(ms_kernels[1], 3),
                       reverse_ms=round(ms_grad, 3), wall_ms=round((tg1 - tg0) * 1000.0, 3),
                       samples_per_s=round(n_pi / ((ms_kernels[1] + ms_grad) / 1000.0), 3),
                       dmeanphi_dKc=g[0], dmeanphi_dtaui=g[1],
                       ckpt_interval=(tuning or {}).get("ckpt_interval") or cfg.get("ckpt_interval"))
        log(f"PI gradient: forward {ms_kernels[1]:.1f} ms, reverse {ms_grad:.1f} ms")
    camp.close()

    plain = None
    if not args.no_plain and n_nmpc and args.model_nx == 1 and args.nlp_form == 0:
        plain = {}
        for name in [c for c in args.plain_configs.split(",") if c]:
            n = {"c0": 64, "c1": args.plain_samples, "c3": 2000, "c4": 5000}.get(name, 2000)
            pc = workloads.CONFIGS[name]()
            if args.eps > 0:
                pc["sqp_eps"] = args.eps
            plain[name] = adjoint_vs_plain(pc, n)
            log(f"adjoint vs plain {name} done")

    extras = None
    if not args.no_extras and args.config == "c1" and not args.samples and args.model_nx == 1 \
            and args.nlp_form == 0 and args.eps == 0:
        extras = side_runs(cfg)

    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, args.cpu_seconds)
    scaling = cu_scaling(cfg) if args.cu_scaling else None

    out = {
        "metric": "NMPC CSTR closed-loop sims/sec on 1 GPU; % FP64 peak; adjoint vs plain SQP",
        "value": round(value, 3),
        "unit": "NMPC closed-loop sims/s" if n_nmpc else "PI closed-loop sims/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{S} samples ({n_nmpc} NMPC + {n_pi} PI), "
                               + describe(cfg, args.config),
                   "samples": S, "nmpc_samples": n_nmpc, "pi_samples": n_pi},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "all_sims_per_s": round(S / (ms_per_step / 1000.0), 3),
        "kernel_ms": {"nmpc": round(ms_kernels[0], 3), "pi": round(ms_kernels[1], 3),
                      "stats": round(ms_kernels[2], 3)},
        "ocp": {"total": tot["n_ocp"], "failed": tot["n_ocp_fail"],
                "sqp_iter_per_ocp": round(tot["sqp_iter"] / max(1, tot["n_ocp"]), 3),
                "ipm_iter_per_sqp": round(tot["ipm_iter"] / max(1, tot["sqp_iter"]), 3)},
        "phi": {"mean_nmpc": stats["mean"][0], "var_nmpc": stats["var"][0],
                "mean_pi": stats["mean"][1], "var_pi": stats["var"][1]},
        "launch_plan": plan,
        "launch_tuning": tuning,
        "cu_scaling": scaling,
        "pi_gradient": pi_grad,
        "adjoint_vs_plain": plain,
        "side_runs": extras,
        "algorithmic_gflop_per_step": round(camp_flops / 1e9, 3),
    }
    print(json.dumps(out))


def cu_scaling(cfg, samples=32768, L=20, spw=32):
    """Fixed work (the first L intervals of `samples` NMPC closed loops of the
    workload, 32 per wavefront) on streams limited to the first k compute
    units: the GPU analogue of the paper's speed-up against CPU cores."""
    import torch

    from paper_2212_02197_amd import binding
    total = torch.cuda.get_device_properties(0).multi_processor_count
    ks = [k for k in (8, 16, 32, 64, 128, 256) if k <= total]
    rows = []
    for k in ks:
        cs = binding.CuStream(k)
        c = dict(cfg, n_samples=samples, kind_split=-1, default_kind=0, noise_mod=0, L=L,
                 cu_limit=k, samples_per_wave=spw)
        camp = binding.Campaign(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        camp.run(stream=cs.stream)
        camp.costs()
        dt = time.perf_counter() - t0
        rows.append(dict(cus=k, sims_per_s=round(samples / dt, 3), ms=round(dt * 1000.0, 1),
                         waves=camp.plan()[0]["slots"]))
        camp.close()
        cs.close()
        log(f"cu scaling: {k} CUs, {samples} samples x {L} intervals in {dt:.2f} s")
    k0, r0 = rows[0]["cus"], rows[0]["sims_per_s"]
    for r in rows:
        r["speedup"] = round(r["sims_per_s"] / r0, 3)
        r["efficiency"] = round(r["speedup"] / (r["cus"] / k0), 3)
    return dict(samples=samples, intervals=L, samples_per_wave=spw, rows=rows)


def nmpc_subset_run(cfg, n, stride=1, **over):
    """One timed run of n NMPC sample ids (0, stride, 2 stride, ...) of the
    workload; returns rate, kernel time and the OCP statistics."""
    import numpy as np
    import torch

    from paper_2212_02197_amd import binding
    n_nm = cfg["kind_split"] if cfg["kind_split"] >= 0 else cfg["n_samples"]
    ids = np.arange(0, n_nm, stride, dtype=np.int64)[:n]
    c = dict(cfg, n_samples=len(ids), sample_ids=ids, kind_split=-1, default_kind=0,
             noise_mod=cfg["noise_mod"], **over)
    camp = binding.Campaign(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    camp.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    phi, st = camp.costs()
    tot = st["totals"]
    out = dict(samples=len(ids), id_stride=stride, sims_per_s=round(len(ids) / dt, 3),
               nmpc_kernel_ms=round(camp.kernel_ms()[0], 3), ocp_total=tot["n_ocp"],
               ocp_failed=tot["n_ocp_fail"],
               sqp_iter_per_ocp=round(tot["sqp_iter"] / max(1, tot["n_ocp"]), 3),
               mean_phi=st["mean"][0])
    camp.close()
    return out, phi


def side_runs(cfg):
    """Paper-scale side measurements: the whole campaign's NMPC half at
    eps = 1e-8, and with the paper's multiple-shooting NLP; the paper's
    W^[0] = I at every OCP with single shooting and with the
    multiple-shooting NLP, on strided NMPC subsets beside the default single
    shooting with the shifted Hessian; a Monte Carlo tuning sweep."""
    import numpy as np
    import torch

    from paper_2212_02197_amd import binding
    res = {}
    c8 = dict(cfg, sqp_eps=1e-8)
    camp = binding.Campaign(c8)
    camp.run()
    camp.costs()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    camp.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, st = camp.costs()
    tot = st["totals"]
    n_nm = c8["n_samples"] - tot["kind"]
    res["eps_1e-8"] = dict(nmpc_sims_per_s=round(n_nm / dt, 3), ms_per_step=round(dt * 1e3, 3),
                           nmpc_kernel_ms=round(camp.kernel_ms()[0], 3), ocp_total=tot["n_ocp"],
                           ocp_failed=tot["n_ocp_fail"],
                           sqp_iter_per_ocp=round(tot["sqp_iter"] / max(1, tot["n_ocp"]), 3))
    camp.close()
    log(f"eps 1e-8: {res['eps_1e-8']}")
    # the paper's own NLP (multiple shooting, W^[0] = I) on the whole campaign
    cm = dict(cfg, nlp_form=1)
    camp = binding.Campaign(cm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    camp.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, st = camp.costs()
    tot = st["totals"]
    n_nm = cm["n_samples"] - tot["kind"]
    km = camp.kernel_ms()[0]
    tf = st["flops_by_kind"][0] / km / 1e9
    res["multiple_shooting_full"] = dict(
        nmpc_sims_per_s=round(n_nm / dt, 3), ms_per_step=round(dt * 1e3, 3),
        nmpc_kernel_ms=round(km, 3), ocp_total=tot["n_ocp"], ocp_failed=tot["n_ocp_fail"],
        sqp_iter_per_ocp=round(tot["sqp_iter"] / max(1, tot["n_ocp"]), 3),
        ipm_iter_per_sqp=round(tot["ipm_iter"] / max(1, tot["sqp_iter"]), 3),
        mean_phi_nmpc=st["mean"][0], algorithmic_tflops=round(tf, 4), frac_fp64_peak=round(tf / 78.6, 5))
    camp.close()
    log(f"multiple shooting, whole campaign: {res['multiple_shooting_full']}")
    n, stride = 1024, 29
    base, phi0 = nmpc_subset_run(cfg, n, stride)
    lit, phi1 = nmpc_subset_run(cfg, n, stride, hess_warm=0)
    ms, phi2 = nmpc_subset_run(cfg, n, stride, nlp_form=1)
    for r, ph in ((lit, phi1), (ms, phi2)):
        r["max_rel_phi_diff_vs_default"] = float(np.max(np.abs(ph - phi0) / phi0))
    res["hessian_start"] = dict(
        single_shooting_shifted_W=base, single_shooting_W0_identity=lit,
        multiple_shooting_W0_identity=ms,
        paper_table_I="424 of 18,000,000 OCPs (0.0024 %) reach the 100-iteration cap")
    log(f"hessian start: {res['hessian_start']}")
    # Monte Carlo tuning of the NMPC's input back-off on the same subset
    from paper_2212_02197_amd import tuning
    ids = np.arange(0, 30000, stride, dtype=np.int64)[:n]
    sub = dict(cfg, n_samples=len(ids), sample_ids=ids, kind_split=-1, default_kind=0)
    t0 = time.perf_counter()
    sw = tuning.sweep(sub, "backoff", (0.0, 50.0, 100.0, 200.0))
    g = tuning.crn_gradient(sub, "backoff", 100.0, 10.0)
    res["tuning_backoff"] = dict(samples=len(ids), candidates=sw,
                                 gradient_at_100=dict((k, g[k]) for k in ("gradient", "stderr", "step")),
                                 wall_s=round(time.perf_counter() - t0, 3))
    log(f"tuning: {res['tuning_backoff']}")
    return res


def adjoint_vs_plain(cfg, n):
    """Same NMPC samples (ids 0..n-1) solved with the adjoint gradient and
    with plain forward sensitivities at equal KKT tolerance."""
    import numpy as np
    import torch

    from paper_2212_02197_amd import binding
    res = {}
    phis = {}
    for mode, name in ((1, "adjoint"), (0, "plain")):
        c = dict(cfg, n_samples=n, kind_split=-1, default_kind=0, noise_mod=0, grad_mode=mode)
        camp = binding.Campaign(c)
        camp.run()
        camp.costs()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        camp.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        phi, st = camp.costs()
        ps = camp.per_sample()
        phis[name] = (phi, ps["ashash"])
        res[name] = dict(sims_per_s=round(n / dt, 3), nmpc_kernel_ms=round(camp.kernel_ms()[0], 3),
                         sqp_iter_per_ocp=round(st["totals"]["sqp_iter"] / st["totals"]["n_ocp"], 3))
        camp.close()
        log(f"{name} gradient: {n} NMPC samples in {dt:.2f} s")
    fin = np.isfinite(phis["adjoint"][0]) & np.isfinite(phis["plain"][0])
    rel = np.abs(phis["adjoint"][0][fin] - phis["plain"][0][fin]) / np.abs(phis["plain"][0][fin])
    res["samples"] = n
    res["diverged_samples"] = int((~fin).sum())
    res["speedup_adjoint_over_plain"] = round(res["adjoint"]["sims_per_s"] / res["plain"]["sims_per_s"], 4)
    res["max_rel_phi_diff"] = float(rel.max()) if rel.size else 0.0
    res["active_set_flips"] = int((phis["adjoint"][1] != phis["plain"][1]).sum())
    return res


if __name__ == "__main__":
    main()
