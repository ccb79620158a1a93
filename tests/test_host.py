"""Host-side behaviour that needs no GPU: the product path fails loudly when
its native library is missing (there is no CPU fallback), bench.py refuses
runs on more than one GPU before touching a device, and every workload
recipe marshals into the C-ABI parameter struct."""
import os
import subprocess
import sys

import pytest

from paper_2212_02197_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_raises_when_the_library_is_missing():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2212_02197_amd import binding\n"
            "binding.LIB_PATH = '/nonexistent/libmc_cl.so'\n"
            "try:\n"
            "    binding.lib()\n"
            "except binding.McClError as e:\n"
            "    print('raised', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(1)\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "is missing" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("name", sorted(workloads.CONFIGS))
@pytest.mark.parametrize("nx", [1, 3])
def test_workloads_marshal_into_the_abi_struct(name, nx):
    cfg = workloads.CONFIGS[name](model_nx=nx)
    p = binding.params(cfg)
    assert p.struct_size == binding.C.sizeof(binding.Params)
    assert p.abi_version == binding.ABI_VERSION
    assert p.model_nx == nx
    assert p.n_samples == cfg["n_samples"]
    assert p.N == cfg["N"] and p.Nc == cfg["Nc"] and p.L == cfg["L"]
    assert list(p.sigma) == list(cfg["sigma"])


def test_unknown_workload_keys_are_rejected():
    with pytest.raises(KeyError):
        workloads.make(no_such_key=1)
