"""The C-ABI library loads, exports every function include/mc_cl.h declares,
and its parameter/struct layout matches the header (checked with gcc's own
sizeof/offsetof).  CPU only: no compute call reaches the GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2212_02197_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mc_cl.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2212_02197_amd import build
    build.ensure_built()
    return binding.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mc_cl_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mc_cl_create", "mc_cl_run", "mc_cl_costs", "mc_cl_grad", "mc_cl_destroy",
              "mc_cl_strerror", "mc_cl_abi_version"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(mc_cl_\w+)", out))
    for f in declared_functions():
        assert f in exported, f
    for f in binding.EXPORTS:
        assert f in exported, f


def _c_layout(struct, fields):
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "mc_cl.h"', "int main(void){",
            f'printf("%zu\\n", sizeof({struct}));']
    for f in fields:
        prog.append(f'printf("%zu\\n", offsetof({struct}, {f}));')
    prog.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write("\n".join(prog))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    return vals[0], vals[1:]


@pytest.mark.parametrize("cstruct,pystruct", [("mc_cl_params", binding.Params),
                                              ("mc_cl_outputs", binding.Outputs),
                                              ("mc_cl_stats", binding.Stats),
                                              ("mc_cl_tune_result", binding.TuneResult)])
def test_struct_layout_matches_header(cstruct, pystruct):
    fields = [f for f, _ in pystruct._fields_]
    size, offs = _c_layout(cstruct, fields)
    assert size == C.sizeof(pystruct)
    for f, o in zip(fields, offs):
        assert getattr(pystruct, f).offset == o, f


def test_abi_version_and_strerror(lib):
    assert lib.mc_cl_abi_version() == binding.ABI_VERSION
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.mc_cl_strerror(code)


def _create(cfg, **over):
    cfg = dict(cfg, **over)
    arrays = binding.per_sample_arrays(cfg)
    p = binding.params(cfg, arrays)
    h = C.c_void_p()
    return binding.lib().mc_cl_create(C.byref(p), C.byref(h))


@pytest.mark.parametrize("over", [dict(kind=[0, 2, 1, 0]), dict(horizon=[10, 0, 10, 10]),
                                  dict(horizon=[10, 65, 10, 10]), dict(lengths=[5, -1, 5, 5]),
                                  dict(lengths=[5, (1 << 24) + 1, 5, 5]),
                                  dict(sample_ids=[0, -3, 1, 2]),
                                  dict(sample_ids=[0, 1, 2, (1 << 32) - 1])])
def test_invalid_per_sample_arrays_are_rejected(lib, over):
    from paper_2212_02197_amd import workloads
    assert _create(workloads.c0_small_nmpc(n_samples=4), **over) == -1


@pytest.mark.parametrize("over", [dict(V=0.0), dict(N=0), dict(N=65), dict(umin=5.0, umax=1.0),
                                  dict(n_samples=0), dict(Ns=0), dict(k0=float("nan")),
                                  dict(Ts=-1.0), dict(grad_mode=2), dict(P0=0.0),
                                  dict(sp_z=(250.0,), sp_i=(0,)), dict(kP=0.0),
                                  dict(chunk_samples=-1), dict(cu_limit=-1), dict(model_nx=2),
                                  dict(model_nx=0)])
def test_invalid_parameters_are_rejected_before_any_device_call(lib, over):
    from paper_2212_02197_amd import workloads
    assert _create(workloads.c0_small_nmpc(), **over) == -1


def test_caller_workspace_is_checked_before_any_device_call(lib):
    from paper_2212_02197_amd import workloads
    cfg = workloads.c0_small_nmpc(n_samples=4)
    p = binding.params(cfg)
    h = C.c_void_p()
    p.workspace = 0x1000 + 8          # not 256-byte aligned
    p.workspace_size = 1 << 20
    assert lib.mc_cl_create(C.byref(p), C.byref(h)) == -1
    p.workspace = 0x1000
    p.workspace_size = 0
    assert lib.mc_cl_create(C.byref(p), C.byref(h)) == -1
    b = C.c_size_t()
    assert lib.mc_cl_workspace_size(None, C.byref(b)) == -1


def test_multiple_shooting_parameters_are_checked(lib):
    from paper_2212_02197_amd import workloads
    unsupported = [k for k, v in binding.STATUS.items() if v == "MC_CL_EUNSUPPORTED"][0]
    cfg = workloads.c0_small_nmpc()
    assert _create(cfg, nlp_form=2) == -1
    assert _create(cfg, nlp_form=1, umin=5.0, umax=5.0) == -1
    assert _create(cfg, nlp_form=1, model_nx=3) == unsupported


def test_three_state_model_needs_the_adjoint_gradient(lib):
    from paper_2212_02197_amd import workloads
    unsupported = [k for k, v in binding.STATUS.items() if v == "MC_CL_EUNSUPPORTED"][0]
    assert _create(workloads.c0_small_nmpc(), model_nx=3, grad_mode=0) == unsupported


def test_struct_size_and_version_are_checked(lib):
    from paper_2212_02197_amd import workloads
    p = binding.params(workloads.c0_small_nmpc())
    p.struct_size = 8
    h = C.c_void_p()
    assert lib.mc_cl_create(C.byref(p), C.byref(h)) == -1
    p = binding.params(workloads.c0_small_nmpc())
    p.abi_version = 99
    assert lib.mc_cl_create(C.byref(p), C.byref(h)) == -1


def test_calls_on_null_context_fail_cleanly(lib):
    st = binding.Stats()
    assert lib.mc_cl_costs(None, None, C.byref(st)) == -1
    g = (C.c_double * 2)()
    assert lib.mc_cl_grad(None, None, g, None) == -1
    assert lib.mc_cl_run(None, None, None) == -1


def test_tune_rejects_bad_arguments(lib):
    r = binding.TuneResult()
    assert lib.mc_cl_tune(None, None, 6, C.byref(r)) == -1


def test_stream_helpers_reject_null(lib):
    assert lib.mc_cl_stream_create(4, None) == -1
    assert lib.mc_cl_stream_destroy(None) == -1


def test_static_run_rejects_before_any_device_call(lib):
    # mc_cl_run_static checks its arguments and the campaign's size against
    # the scratch array before it touches the device
    from paper_2212_02197_amd import workloads
    phi = (C.c_double * 4)()

    def call(cfg, **o):
        arrays = binding.per_sample_arrays(cfg)
        p = binding.params(cfg, arrays)
        out = binding.Outputs(C.cast(phi, C.c_void_p).value, None, None, None, None, None)
        for k, v in o.items():
            setattr(out, k, v)
        return lib.mc_cl_run_static(C.byref(p), None, C.byref(out))

    cfg = workloads.c0_small_nmpc(n_samples=4)
    assert lib.mc_cl_run_static(C.byref(binding.params(cfg)), None, None) == -1
    assert call(cfg, phi=None) == -1
    assert call(dict(cfg, N=0)) == -1
    assert call(cfg, traj_z=1234) == -5
    assert call(dict(cfg, want_grad=1)) == -5
    assert call(dict(cfg, chunk_samples=2)) == -5
    assert call(dict(cfg, lengths=[1, 2, 3, 4])) == -5
    # about 96 bytes per sample: a million samples exceed the 64 MiB array
    assert binding.STATIC_SCRATCH_BYTES == 64 << 20
    assert call(workloads.c4_mixed()) == -1
