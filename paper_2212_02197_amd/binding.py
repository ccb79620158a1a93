"""ctypes binding of libmc_cl.so (include/mc_cl.h): argument marshalling only.

Every step of the method runs in the HIP library.  PyTorch provides device
memory and streams: output tensors are allocated with torch on the current
device and their data pointers handed to the C-ABI.  There is no CPU fallback:
if the library is missing, `lib()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmc_cl.so")

SPMAX, NMAX, NHIST = 8, 64, 202
CNT_NAMES = ["kind", "N", "L", "n_ocp", "n_ocp_fail", "sqp_iter", "ipm_iter", "ls_trials",
             "ls_cap", "bfgs_skip", "bfgs_reset", "ipm_cap", "nonfinite", "grad_evals",
             "as_iter"]
NCNT = len(CNT_NAMES)
STATUS = {0: "MC_CL_OK", -1: "MC_CL_EINVAL", -2: "MC_CL_EHIP", -3: "MC_CL_ENOMEM",
          -4: "MC_CL_ESTATE", -5: "MC_CL_EUNSUPPORTED"}
ABI_VERSION = 6


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("abi_version", C.c_uint32),
        ("V", C.c_double), ("k0", C.c_double), ("EaR", C.c_double), ("beta", C.c_double),
        ("cAin", C.c_double), ("cBin", C.c_double), ("cTin", C.c_double),
        ("sigma", C.c_double * 3), ("Rmeas", C.c_double), ("Ts", C.c_double),
        ("Ns", C.c_int32), ("L", C.c_int32),
        ("n_sp", C.c_int32), ("sp_period", C.c_int32),
        ("sp_i", C.c_int32 * SPMAX), ("sp_z", C.c_double * SPMAX),
        ("sp_step_rel", C.c_double), ("sp_step_lo", C.c_int32), ("sp_step_hi", C.c_int32),
        ("N", C.c_int32), ("Nc", C.c_int32),
        ("Qz", C.c_double), ("umin", C.c_double), ("umax", C.c_double),
        ("sqp_eps", C.c_double), ("ls_c1", C.c_double), ("ls_beta", C.c_double),
        ("sqp_max_iter", C.c_int32), ("ls_max_bt", C.c_int32),
        ("grad_mode", C.c_int32), ("ipm_max_iter", C.c_int32),
        ("kP", C.c_double), ("kI", C.c_double), ("kaw", C.c_double),
        ("pi_umin", C.c_double), ("pi_umax", C.c_double),
        ("P0", C.c_double), ("x0_rel_std", C.c_double),
        ("x0_mode", C.c_int32), ("kind_split", C.c_int32), ("default_kind", C.c_int32),
        ("run_ekf_for_pi", C.c_int32),
        ("seed", C.c_uint64), ("noise_mod", C.c_int64), ("n_samples", C.c_int64),
        ("sample_id_offset", C.c_int64),
        ("n_horizon_choices", C.c_int32), ("horizon_choices", C.c_int32 * 4),
        ("L_lo", C.c_int32), ("L_hi", C.c_int32),
        ("kin_lognorm_sigma", C.c_double),
        ("hess_warm", C.c_int32), ("want_grad", C.c_int32),
        ("noise_scale", C.c_double),
        ("ckpt_interval", C.c_int32), ("samples_per_wave", C.c_int32),
        ("qp_solver", C.c_int32), ("chunk_samples", C.c_int32),
        ("cu_limit", C.c_int32), ("model_nx", C.c_int32),
        ("sample_ids", C.c_void_p), ("kind", C.c_void_p), ("horizon", C.c_void_p),
        ("lengths", C.c_void_p), ("nlp_form", C.c_int32),
        ("workspace", C.c_void_p), ("workspace_size", C.c_size_t),
        ("class_streams", C.c_int32),
    ]


class Outputs(C.Structure):
    _fields_ = [("phi", C.c_void_p), ("counters", C.c_void_p), ("ashash", C.c_void_p),
                ("traj_z", C.c_void_p), ("traj_u", C.c_void_p), ("traj_xhat", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("count", C.c_int64 * 2), ("mean", C.c_double * 2), ("var", C.c_double * 2),
                ("hist", (C.c_int64 * NHIST) * 2), ("totals", C.c_int64 * NCNT),
                ("flops_algorithmic", C.c_double), ("flops_by_kind", C.c_double * 2),
                ("workspace_bytes", C.c_size_t)]


TUNE_SPW = (4, 8, 16, 32, 64)
TUNE_CKPT = (2, 5, 10, 25, 50)
TUNE_PI_LANES = (1, 2, 4)


class TuneResult(C.Structure):
    _fields_ = [("n_classes", C.c_int32), ("nmax", C.c_int32 * 3), ("spw", C.c_int32 * 3),
                ("nmpc_ms", (C.c_float * len(TUNE_SPW)) * 3), ("ckpt_interval", C.c_int32),
                ("grad_ms", C.c_float * len(TUNE_CKPT)), ("pi_lanes", C.c_int32),
                ("pi_ms", C.c_float * len(TUNE_PI_LANES))]


EXPORTS = ["mc_cl_create", "mc_cl_run", "mc_cl_costs", "mc_cl_grad", "mc_cl_destroy",
           "mc_cl_strerror", "mc_cl_abi_version", "mc_cl_kernel_ms", "mc_cl_plan",
           "mc_cl_tune", "mc_cl_stream_create", "mc_cl_stream_destroy", "mc_cl_workspace_size",
           "mc_cl_run_static"]
STATIC_SCRATCH_BYTES = 64 << 20

_lib = None


class McClError(RuntimeError):
    pass


def lib():
    """Load the in-tree HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise McClError(f"{LIB_PATH} is missing: build it with paper_2212_02197_amd.build")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mc_cl_create.restype = C.c_int
        L.mc_cl_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
        L.mc_cl_run.restype = C.c_int
        L.mc_cl_run.argtypes = [vp, vp, C.POINTER(Outputs)]
        L.mc_cl_costs.restype = C.c_int
        L.mc_cl_costs.argtypes = [vp, vp, C.POINTER(Stats)]
        L.mc_cl_grad.restype = C.c_int
        L.mc_cl_grad.argtypes = [vp, vp, C.POINTER(C.c_double), vp]
        L.mc_cl_destroy.restype = None
        L.mc_cl_destroy.argtypes = [vp]
        L.mc_cl_strerror.restype = C.c_char_p
        L.mc_cl_strerror.argtypes = [C.c_int]
        L.mc_cl_abi_version.restype = C.c_uint32
        L.mc_cl_abi_version.argtypes = []
        L.mc_cl_kernel_ms.restype = C.c_int
        L.mc_cl_kernel_ms.argtypes = [vp, C.POINTER(C.c_float)]
        L.mc_cl_plan.restype = C.c_int
        L.mc_cl_plan.argtypes = [vp, C.POINTER(C.c_int32), C.c_int]
        L.mc_cl_tune.restype = C.c_int
        L.mc_cl_tune.argtypes = [vp, vp, C.c_int32, C.POINTER(TuneResult)]
        L.mc_cl_stream_create.restype = C.c_int
        L.mc_cl_stream_create.argtypes = [C.c_int32, C.POINTER(vp)]
        L.mc_cl_stream_destroy.restype = C.c_int
        L.mc_cl_stream_destroy.argtypes = [vp]
        L.mc_cl_workspace_size.restype = C.c_int
        L.mc_cl_workspace_size.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t)]
        L.mc_cl_run_static.restype = C.c_int
        L.mc_cl_run_static.argtypes = [C.POINTER(Params), vp, C.POINTER(Outputs)]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().mc_cl_strerror(rc).decode()
        raise McClError(f"{what}: {STATUS.get(rc, rc)} ({msg})")


# per-sample arrays of the workload dict: key -> numpy dtype of the C array
PER_SAMPLE = {"sample_ids": "int64", "kind": "uint8", "horizon": "int32", "lengths": "int32"}


def per_sample_arrays(cfg: dict) -> dict:
    """Contiguous host copies of the workload's per-sample arrays (those
    not None), of the C types mc_cl_params names."""
    import numpy as np
    out = {}
    for key, dt in PER_SAMPLE.items():
        a = cfg.get(key)
        if a is not None:
            a = np.ascontiguousarray(a, dtype=dt)
            if a.shape != (int(cfg["n_samples"]),):
                raise ValueError(f"{key} must have n_samples entries")
            out[key] = a
    return out


def params(cfg: dict, arrays: dict = None) -> Params:
    """mc_cl_params from a workload dict (see workloads.py); `arrays` from
    per_sample_arrays(cfg) must stay alive while the struct is used."""
    p = Params()
    p.struct_size = C.sizeof(Params)
    p.abi_version = ABI_VERSION
    for key in ("V", "k0", "EaR", "beta", "cAin", "cBin", "cTin", "Rmeas", "Ts", "Ns", "L",
                "sp_period", "sp_step_rel", "sp_step_lo", "sp_step_hi", "N", "Nc", "Qz",
                "umin", "umax", "sqp_eps", "ls_c1", "ls_beta", "sqp_max_iter", "ls_max_bt",
                "grad_mode", "ipm_max_iter", "kP", "kI", "kaw", "pi_umin", "pi_umax", "P0",
                "x0_rel_std", "x0_mode", "kind_split", "default_kind", "run_ekf_for_pi", "seed",
                "noise_mod", "n_samples", "L_lo", "L_hi", "kin_lognorm_sigma", "hess_warm",
                "want_grad", "noise_scale"):
        setattr(p, key, cfg[key])
    p.sample_id_offset = cfg.get("sample_id_offset", 0)
    p.ckpt_interval = cfg.get("ckpt_interval", 0)
    p.samples_per_wave = cfg.get("samples_per_wave", 0)
    p.qp_solver = cfg.get("qp_solver", 2)
    p.chunk_samples = cfg.get("chunk_samples", 0)
    p.cu_limit = cfg.get("cu_limit", 0)
    p.model_nx = cfg.get("model_nx", 1)
    p.nlp_form = cfg.get("nlp_form", 0)
    p.class_streams = cfg.get("class_streams", 0)
    for a in range(3):
        p.sigma[a] = cfg["sigma"][a]
    sp_i, sp_z = cfg["sp_i"], cfg["sp_z"]
    if not 1 <= len(sp_i) == len(sp_z) <= SPMAX:
        raise ValueError("setpoint schedule must have 1..8 levels")
    p.n_sp = len(sp_i)
    for j in range(len(sp_i)):
        p.sp_i[j] = sp_i[j]
        p.sp_z[j] = sp_z[j]
    hc = cfg["horizon_choices"]
    p.n_horizon_choices = len(hc)
    for j, v in enumerate(hc):
        p.horizon_choices[j] = v
    for key, a in (arrays or {}).items():
        setattr(p, key, a.ctypes.data)
    return p


class Campaign:
    """One mc_cl context: create on the current device, run on a torch stream,
    read costs, statistics and the PI gradient."""

    def __init__(self, cfg: dict, workspace=None):
        """workspace: optional torch uint8 tensor on the device, at least
        workspace_size(cfg) bytes, that the context's buffers are carved
        from (kept referenced by the campaign)."""
        import torch
        self.torch = torch
        self.cfg = dict(cfg)
        self.S = int(cfg["n_samples"])
        arrays = per_sample_arrays(self.cfg)
        self.p = params(self.cfg, arrays)
        self.workspace = workspace
        if workspace is not None:
            self.p.workspace = workspace.data_ptr()
            self.p.workspace_size = workspace.numel() * workspace.element_size()
        h = C.c_void_p()
        _check(lib().mc_cl_create(C.byref(self.p), C.byref(h)), "mc_cl_create")
        self.h = h
        dev = torch.device("cuda", torch.cuda.current_device())
        self.phi = torch.empty(self.S, dtype=torch.float64, device=dev)
        self.counters = torch.empty((NCNT, self.S), dtype=torch.int32, device=dev)
        self.ashash = torch.empty(self.S, dtype=torch.int64, device=dev)
        self.traj = None

    def close(self):
        if getattr(self, "h", None):
            lib().mc_cl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, stream=None, trajectories: bool = False):
        """mc_cl_run on `stream` (torch.cuda.Stream; default: current stream)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream()
        o = Outputs(self.phi.data_ptr(), self.counters.data_ptr(), self.ashash.data_ptr(),
                    None, None, None)
        if trajectories:
            # rows for the longest possible sample (mc_cl_outputs: T)
            c = self.cfg
            if c.get("lengths") is not None:
                L = int(max(c["lengths"]))
            else:
                L = int(c["L_hi"] if c["L_lo"] < c["L_hi"] else c["L"])
            dev = self.phi.device
            self.traj = dict(z=torch.empty((L + 1, self.S), dtype=torch.float64, device=dev),
                             u=torch.empty((L, self.S), dtype=torch.float64, device=dev),
                             xhat=torch.empty((L, self.S), dtype=torch.float64, device=dev))
            o.traj_z = self.traj["z"].data_ptr()
            o.traj_u = self.traj["u"].data_ptr()
            o.traj_xhat = self.traj["xhat"].data_ptr()
        _check(lib().mc_cl_run(self.h, C.c_void_p(st.cuda_stream), C.byref(o)), "mc_cl_run")

    def costs(self):
        """Wait for the run; return (phi numpy array, stats dict)."""
        import numpy as np
        st = Stats()
        phi = np.empty(self.S, dtype=np.float64)
        _check(lib().mc_cl_costs(self.h, phi.ctypes.data_as(C.c_void_p), C.byref(st)),
               "mc_cl_costs")
        stats = dict(count=list(st.count), mean=list(st.mean), var=list(st.var),
                     hist=[np.array(list(st.hist[k]), dtype=np.int64) for k in range(2)],
                     totals={n: int(st.totals[i]) for i, n in enumerate(CNT_NAMES)},
                     flops_algorithmic=float(st.flops_algorithmic),
                     flops_by_kind=[float(st.flops_by_kind[0]), float(st.flops_by_kind[1])],
                     workspace_bytes=int(st.workspace_bytes))
        return phi, stats

    def per_sample(self):
        """Counters and hashes of the last run as numpy arrays (synchronises)."""
        self.torch.cuda.synchronize()
        cnt = self.counters.cpu().numpy()
        out = {n: cnt[i] for i, n in enumerate(CNT_NAMES)}
        out["ashash"] = self.ashash.cpu().numpy().view("u8")
        out["phi"] = self.phi.cpu().numpy()
        return out

    def grad(self, stream=None, per_sample: bool = False):
        """mc_cl_grad: d mean Phi (PI samples) / d(Kc, tau_i)."""
        torch = self.torch
        st = stream if stream is not None else torch.cuda.current_stream()
        g = (C.c_double * 2)()
        ps = None
        if per_sample:
            ps = torch.empty((2, self.S), dtype=torch.float64, device=self.phi.device)
        _check(lib().mc_cl_grad(self.h, C.c_void_p(st.cuda_stream), g,
                                None if ps is None else C.c_void_p(ps.data_ptr())), "mc_cl_grad")
        return (g[0], g[1]), ps

    def kernel_ms(self):
        ms = (C.c_float * 4)()
        _check(lib().mc_cl_kernel_ms(self.h, ms), "mc_cl_kernel_ms")
        return list(ms)

    def tune(self, trial_intervals: int = 6, stream=None):
        """mc_cl_tune: measured samples-per-wavefront (and PI checkpoint
        interval and lanes-per-sample) choice; returns the trial times and
        the choice."""
        st = stream if stream is not None else self.torch.cuda.current_stream()
        r = TuneResult()
        _check(lib().mc_cl_tune(self.h, C.c_void_p(st.cuda_stream), int(trial_intervals),
                                C.byref(r)), "mc_cl_tune")
        n = r.n_classes
        return dict(
            classes=[dict(nmax=r.nmax[k], spw=r.spw[k],
                          trial_ms={s: round(float(r.nmpc_ms[k][j]), 3)
                                    for j, s in enumerate(TUNE_SPW)}) for k in range(n)],
            ckpt_interval=r.ckpt_interval,
            grad_trial_ms={c: round(float(r.grad_ms[j]), 3) for j, c in enumerate(TUNE_CKPT)},
            pi_lanes=r.pi_lanes,
            pi_trial_ms={k: round(float(r.pi_ms[j]), 3) for j, k in enumerate(TUNE_PI_LANES)})

    def plan(self):
        buf = (C.c_int32 * 15)()
        n = lib().mc_cl_plan(self.h, buf, 3)
        return [dict(nmax=buf[5 * k], count=buf[5 * k + 1], spw=buf[5 * k + 2],
                     groups=buf[5 * k + 3], slots=buf[5 * k + 4]) for k in range(n)]


def workspace_size(cfg: dict) -> int:
    """mc_cl_workspace_size: device bytes a campaign of cfg needs."""
    arrays = per_sample_arrays(cfg)
    p = params(cfg, arrays)
    b = C.c_size_t()
    _check(lib().mc_cl_workspace_size(C.byref(p), C.byref(b)), "mc_cl_workspace_size")
    return int(b.value)


def run_static(cfg: dict, phi, counters=None, ashash=None, stream=None):
    """mc_cl_run_static: the campaign with no device allocation by the
    library, into caller tensors phi ([S] float64), counters ([NCNT, S]
    int32) and ashash ([S] int64) on the current device (the last two may be
    None).  Queued on `stream` (default: the current stream)."""
    import torch
    arrays = per_sample_arrays(cfg)
    p = params(cfg, arrays)
    st = stream if stream is not None else torch.cuda.current_stream()
    o = Outputs(phi.data_ptr(), None if counters is None else counters.data_ptr(),
                None if ashash is None else ashash.data_ptr(), None, None, None)
    _check(lib().mc_cl_run_static(C.byref(p), C.c_void_p(st.cuda_stream), C.byref(o)),
           "mc_cl_run_static")


def _pi_closed_loop_function():
    import torch

    class PIClosedLoop(torch.autograd.Function):
        """Per-sample closed-loop cost Phi as a differentiable function of the PI
        tuning theta = (Kc, tau_i), with kP = Kc and kI = Kc / tau_i (eq. (PI)).

        forward runs the campaign on the HIP path with plant-state checkpoints
        every `ckpt_interval` intervals (mc_cl_run with want_grad); backward
        runs the reverse pass over those checkpoints (mc_cl_grad) and returns
        sum_s grad_s dPhi_s/dtheta.  NMPC samples of a mixed campaign carry no
        gradient.  theta: float64 tensor of shape (2,); returns Phi, shape (S,),
        on the current device.
        """

        @staticmethod
        def forward(ctx, theta, cfg):
            Kc, taui = float(theta[0]), float(theta[1])
            camp = Campaign(dict(cfg, kP=Kc, kI=Kc / taui, want_grad=1))
            camp.run()
            ctx.camp = camp
            ctx.theta_device = theta.device
            return camp.phi.clone()

        @staticmethod
        def backward(ctx, gout):
            camp = ctx.camp
            _, ps = camp.grad(per_sample=True)
            camp.close()
            ctx.camp = None
            g = ps @ gout.to(device=ps.device, dtype=ps.dtype)
            return g.to(ctx.theta_device), None

    return PIClosedLoop


_PI_FN = None


def pi_closed_loop(theta, cfg):
    """Phi per sample at the PI tuning theta = (Kc, tau_i); differentiable in
    theta through the library's reverse pass (see PIClosedLoop)."""
    global _PI_FN
    if _PI_FN is None:
        _PI_FN = _pi_closed_loop_function()
    return _PI_FN.apply(theta, cfg)


class CuStream:
    """A stream limited to the first n_cu compute units (mc_cl_stream_create),
    as a torch external stream; close() releases it."""

    def __init__(self, n_cu: int):
        import torch
        h = C.c_void_p()
        _check(lib().mc_cl_stream_create(int(n_cu), C.byref(h)), "mc_cl_stream_create")
        self.h = h
        self.stream = torch.cuda.ExternalStream(h.value)

    def close(self):
        if getattr(self, "h", None):
            lib().mc_cl_stream_destroy(self.h)
            self.h = None
